"""Parity of the 3f-model HIP step (two CH lattices, phi0 evolving) with the
FP64 3f oracle (run on an MI355X).

Element-by-element comparison of phi0, phi1, u, p and the raw populations of
all three lattices on the same seeded inputs, on boxes that span several
64 x 32 strip tiles with ragged tails, with walls, closed boxes and periodic
axes, with and without the extra mass flux S (unequal densities), unequal
pairwise tensions, a body force, a gauge and the scale factor d0 = 0.4."""
import sys

import numpy as np
import pytest

from paper_2311_05091_amd import geometry3f as G3F

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _oracle3f(orc, sp, steps):
    p = orc.make_params3f(sp.nx, sp.ny, periodic_x=sp.periodic_x, periodic_y=sp.periodic_y, d0=sp.d0, D=sp.D,
                          sigma01=sp.sigma01, sigma02=sp.sigma02, sigma12=sp.sigma12, rho=sp.rho, mu=sp.mu,
                          M_cst=sp.M_cst, M_deg=sp.M_deg, tau_phi=sp.tau_phi, s_phi=sp.s_phi, s_g=sp.s_g,
                          Fb=sp.Fb, rho_gauge=sp.rho_gauge)
    s = orc.Sim3F(p, sp.phi0, sp.phi1)
    s.step(steps)
    return s


def _gpu3f(specs, precision, steps, fill=None):
    from paper_2311_05091_amd.lbm3f import Context3F
    ctx = Context3F(precision=precision)
    for sp in specs:
        ctx.add_domain(sp)
    ctx.finalize(fill=fill)
    ctx.step(steps)
    return ctx


TENS = dict(sigma01=0.012, sigma02=0.008, sigma12=0.01)
RATIO = dict(rho=(2.0, 3.0, 1.0), mu=(0.2, 0.3, 0.1))
CASES = [
    ("lens_equal_tensions", lambda: G3F.drop_on_interface(nx=70, ny=41, R0=10.0, cx=30.3, cy=20.7), 80),
    ("unequal_tensions_S_force_ragged", lambda: G3F.drop_on_interface(
        nx=131, ny=37, R0=9.0, cx=50.2, cy=17.9, Fb=(2e-6, -1e-6), **TENS, **RATIO), 60),
    ("periodic_gauge_d0_04", lambda: G3F.with_params3f(G3F.drop_on_interface(
        nx=67, ny=45, R0=11.0, cx=33.1, cy=22.4, **TENS, **RATIO), periodic_y=1, d0=0.4, rho_gauge=0.3), 60),
    ("closed_box", lambda: G3F.with_params3f(G3F.drop_on_interface(
        nx=50, ny=40, R0=8.0, cx=24.6, cy=19.3, **RATIO), periodic_x=0), 60),
]


def _compare3f(ctx, sim, did=0, tol=1e-11, pop_tol=1e-12):
    g = ctx.moments(did)
    o = sim.moments()
    for name, a, b in zip(("phi0", "phi1", "ux", "uy", "p"), g, o):
        assert np.isfinite(a).all(), name
        err = np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)
        assert err <= tol, (name, err)
    f0o, f1o, go, _ = sim.get_state()
    f0g, f1g, gg = ctx.populations(did)
    for name, a, b, floor in (("f0", f0g, f0o, 1.0), ("f1", f1g, f1o, 1.0), ("g", gg, go, 1e-3)):
        assert np.abs(a - b).max() <= pop_tol * max(floor, np.abs(b).max()), name


@pytest.mark.parametrize("name,factory,steps", CASES, ids=[c[0] for c in CASES])
def test_fp64_parity_3f(orc, name, factory, steps):
    sp = factory()
    _say("3f fp64 parity", name, sp.nx, sp.ny, steps)
    ctx = _gpu3f([sp], 64, steps)
    sim = _oracle3f(orc, sp, steps)
    _compare3f(ctx, sim)
    ctx.close()


def test_batch_of_3f_domains_equals_single_runs():
    """Domains stepped together (with and without S, different sizes) equal
    the same domains stepped alone, bit for bit, in both precisions; arenas
    filled with zeros or NaN bytes before initialisation give the same bits."""
    specs = [CASES[0][1](), CASES[1][1](), CASES[3][1]()]
    _say("3f batch")
    for prec in (32, 64):
        ctx = _gpu3f(specs, prec, 30, fill=0xFF)
        for i, sp in enumerate(specs):
            one = _gpu3f([sp], prec, 30, fill=0x00)
            a, b = ctx.populations(i), one.populations(0)
            for k in range(3):
                assert np.isfinite(a[k]).all() and np.array_equal(a[k], b[k]), (prec, i, k)
            one.close()
        ctx.close()


def test_fp32_3f_against_fp64_oracle(orc):
    """FP32 storage (gauge 0) against the FP64 oracle after 200 steps of the
    unequal-tension case with S: relative L2 of phi0 and phi1 below 1e-5, of u
    below 1e-2 (u ~ 1e-4 is formed from populations of order one)."""
    sp = CASES[1][1]()
    _say("3f fp32")
    ctx = _gpu3f([sp], 32, 200)
    sim = _oracle3f(orc, sp, 200)
    g, o = ctx.moments(0), sim.moments()
    rl = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    e0, e1 = rl(g[0], o[0]), rl(g[1], o[1])
    eu = rl(np.stack(g[2:4]), np.stack(o[2:4]))
    print("3f FP32 vs FP64 oracle after 200 steps: rel L2 phi0 %.3e, phi1 %.3e, u %.3e" % (e0, e1, eu), flush=True)
    assert e0 < 1e-5 and e1 < 1e-5 and eu < 1e-2
    ctx.close()


def test_3f_phase_masses_conserved_gpu():
    sp = CASES[1][1]()
    _say("3f mass")
    for prec, tol in ((64, 1e-12), (32, 2e-6)):
        ctx = _gpu3f([sp], prec, 0)
        m0 = ctx.mass(0)
        assert np.allclose(m0, [sp.phi0.sum(), sp.phi1.sum()], rtol=1e-6)
        ctx.step(300)
        m = ctx.mass(0)
        assert np.all(np.abs(m - m0) <= tol * m0), (prec, m - m0)
        ctx.close()
