"""Open ends (non-equilibrium extrapolation at an inlet and an outlet, Sec. 4)
and flow rates (Sec. 4.6) of the HIP library against the FP64 oracle (run on
an MI355X): element-by-element parity on ragged channels with a solid disk
and a droplet at density ratio 10, under a pressure drop or a velocity inlet
that injects fluid 1, with every kernel family; open and closed domains in
one batch; flow rates; and the stratified two-fluid channel relaxed to its
steady state against the momentum equation, which gives the relative
permeabilities."""
import sys

import numpy as np
import pytest

from paper_2311_05091_amd import geometry as G
from _util import gpu_context, oracle_run

pytestmark = pytest.mark.gpu

RATIO10 = dict(rho=(1.0, 1.0, 0.1), mu=(0.15, 0.15, 0.015))


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _pressure_channel():
    sp = G.solid_disk_box(n=131, ny=37, Rs=7.0, R0=9.0, periodic_y=0, **RATIO10)
    return G.with_params(sp, periodic_x=0, open_x=1, inlet_type=0, p_in=2e-4, p_out=0.0)


def _velocity_inlet():
    sp = G.solid_disk_box(n=70, ny=29, Rs=5.0, R0=6.0, periodic_y=0)
    return G.with_params(sp, periodic_x=0, open_x=1, inlet_type=1, u_in=2e-3, p_out=0.0, phi1_in=1.0, d0=0.4)


def _compare(ctx, sim, did=0, tol=1e-11, pop_tol=1e-12):
    g = ctx.moments(did)
    o = sim.moments()
    for name, a, b in zip(("phi1", "ux", "uy", "p"), g, o):
        assert np.isfinite(a).all(), name
        err = np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)
        assert err <= tol, (name, err)
    fo, go, _ = sim.get_state()
    fg, gg = ctx.populations(did)
    assert np.abs(fg - fo).max() <= pop_tol * max(1.0, np.abs(fo).max())
    assert np.abs(gg - go).max() <= pop_tol * max(1e-3, np.abs(go).max())


@pytest.mark.parametrize("code", [1, 9, 17, 21, 23])
@pytest.mark.parametrize("case", ["pressure", "velocity"])
def test_open_ends_fp64_parity(orc, case, code):
    sp = _pressure_channel() if case == "pressure" else _velocity_inlet()
    _say("open", case, "tile", code)
    ctx = gpu_context([sp], precision=64, tile=code)
    ctx.step(300)
    sim = oracle_run(orc, sp, 300)
    _compare(ctx, sim)
    q = ctx.flow_rates(0)
    qo = sim.flow_rates()
    assert np.abs(q - qo).max() <= 1e-11 * np.abs(qo).max(), (q, qo)
    ctx.close()


def test_open_and_closed_domains_in_one_batch():
    """An open channel and closed boxes stepped together equal the same
    domains stepped alone, bit for bit (FP32 and FP64)."""
    specs = [_pressure_channel(), G.solid_disk_box(n=67, ny=23, Rs=5.0, R0=6.0, periodic_y=0), _velocity_inlet()]
    _say("open batch")
    for prec in (32, 64):
        ctx = gpu_context(specs, precision=prec, tile=9)
        ctx.step(120)
        for i, sp in enumerate(specs):
            one = gpu_context([sp], precision=prec, tile=9)
            one.step(120)
            a, b = ctx.populations(i), one.populations(0)
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), (prec, i)
            one.close()
        ctx.close()


def _layered_flow_bvp(phi1_y, mu1, mu2, Gf, ref=16):
    ny = len(phi1_y)
    n = ny * ref
    h = ny / n
    yf = -0.5 + h * np.arange(n + 1)
    yn = np.arange(ny, dtype=float)
    ph = np.interp(yf, yn, phi1_y)
    mu = mu1 * ph + mu2 * (1 - ph)
    mh = 0.5 * (mu[1:] + mu[:-1])
    A = np.zeros((n - 1, n - 1))
    for k in range(n - 1):
        A[k, k] = -(mh[k] + mh[k + 1]) / h ** 2
        if k > 0:
            A[k, k - 1] = mh[k] / h ** 2
        if k < n - 2:
            A[k, k + 1] = mh[k + 1] / h ** 2
    u = np.zeros(n + 1)
    u[1:-1] = np.linalg.solve(A, -Gf * np.ones(n - 1))
    return np.interp(yn, yf, u)


@pytest.mark.parametrize("prec", [32, 64])
def test_stratified_channel_flow_rates_and_relative_permeability(prec):
    """Two fluids in layers (viscosity ratio 5) under a uniform drive in a
    periodic channel, relaxed to steady flow on the GPU: each phase's rate
    matches the steady momentum equation with the simulated diffuse viscosity
    within 1%; K_p = rate / (G H^3 / (12 mu_p))."""
    ny, a, mu1, mu2, Gf, nx = 64, 24.0, 0.3, 0.06, 1e-6, 64
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    phi1 = 0.5 - 0.5 * np.tanh(2 * (y - (a - 0.5)) / 4.0)
    sp = G.DomainSpec(nx=nx, ny=ny, phi0=np.zeros((ny, nx)), phi1=phi1, periodic_x=1, periodic_y=0,
                      mu=(mu1, mu1, mu2), Fb=(Gf, 0.0), theta_deg=90.0, M_deg=0.01)
    _say("layers", prec)
    ctx = gpu_context([sp], precision=prec)
    ctx.step(40000)
    q = ctx.flow_rates(0)
    phi, ux, uy, p = ctx.moments(0)
    u_ode = _layered_flow_bvp(phi[:, 0], mu1, mu2, Gf)
    q1 = nx * float(np.sum(phi[:, 0] * u_ode))
    q2 = nx * float(np.sum((1 - phi[:, 0]) * u_ode))
    assert abs(q[1] - q1) <= 0.01 * q1 and abs(q[2] - q2) <= 0.01 * q2, (q, q1, q2)
    kp1 = q[1] / nx / (Gf * ny ** 3 / (12 * mu1))
    kp2 = q[2] / nx / (Gf * ny ** 3 / (12 * mu2))
    print("K_p: fluid 1 %.4f, fluid 2 %.4f" % (kp1, kp2), flush=True)
    assert 0 < kp2 < 1 and kp1 > 0
    ctx.close()
