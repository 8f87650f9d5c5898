"""Pins of the 3f-model oracle (three fluids, phi0 and phi1 each on a CH
lattice; Sec. 2.1, Sec. 3, Sec. 4, Sec. 4.1).

* Both phase masses are conserved (every CH lattice conserves its zeroth
  moment; streaming and bounce-back only move populations).
* Exchanging the labels of phases 0 and 1 (their fields, densities,
  viscosities, and sigma02 <-> sigma12) exchanges phi0 and phi1 of the
  solution and leaves u and p unchanged: the model treats both evolved
  phases alike, so any term written for one phase only (the extra mass flux
  S, the mobility f, eta_p, mubar_p) breaks it.
* A drop of phase 0 in phase 2 (no phase 1) obeys the Laplace law
  dp = sigma02 / R (R = 14; within 1% measured, 3% asserted): with phi1 = 0, mubar1
  vanishes identically and the model is a two-phase CH with tension (gamma0 + gamma2)/2 = sigma02
  (Sec. 2.1); unequal pairwise tensions make a mix-up of them show.
* A drop of phase 0 on a flat interface between phases 1 and 2 relaxes to a
  lens of two circular arcs whose corner angle inside phase 0 follows
  Neumann's triangle of the three tensions (120 degrees for equal tensions,
  the 3f case of Sec. 4.1; measured 121.5 and 123.4 against 120.0 and 124.2).
"""
import math

import numpy as np

TENS = dict(sigma01=0.012, sigma02=0.008, sigma12=0.01)


def _grid(nx, ny):
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    return x, y


def _drop_on_interface(nx, ny, R0, D, cx=None, cy=None):
    x, y = _grid(nx, ny)
    cx = nx / 2 - 0.5 if cx is None else cx
    cy = ny / 2 - 0.5 if cy is None else cy
    phi0 = 0.5 + 0.5 * np.tanh((R0 - np.hypot(x - cx, y - cy)) / (D / 2))
    phi1 = (1 - phi0) * (0.5 - 0.5 * np.tanh(2 * (y - cy) / D))
    return phi0, phi1


def test_3f_phase_masses_conserved(orc):
    phi0, phi1 = _drop_on_interface(48, 40, 9.0, 4.0, cx=20.3, cy=18.7)
    p = orc.make_params3f(48, 40, D=4.0, rho=(2.0, 3.0, 1.0), mu=(0.2, 0.3, 0.1), Fb=(2e-6, -1e-6), **TENS)
    s = orc.Sim3F(p, phi0, phi1)
    m0 = s.mass()
    assert np.allclose(m0, [phi0.sum(), phi1.sum()], rtol=1e-12)
    s.step(400)
    m = s.mass()
    assert np.all(np.abs(m - m0) <= 1e-12 * m0), m - m0
    out = s.moments()
    assert all(np.isfinite(a).all() for a in out)


def test_3f_exchanging_phases_0_and_1(orc):
    nx, ny = 48, 40
    phi0, phi1 = _drop_on_interface(nx, ny, 9.0, 4.0, cx=20.3, cy=18.7)
    kw = dict(D=4.0, M_deg=0.01, Fb=(2e-6, -1e-6))
    pa = orc.make_params3f(nx, ny, rho=(2.0, 3.0, 1.0), mu=(0.2, 0.3, 0.1), **TENS, **kw)
    pb = orc.make_params3f(nx, ny, rho=(3.0, 2.0, 1.0), mu=(0.3, 0.2, 0.1), sigma01=TENS["sigma01"],
                           sigma02=TENS["sigma12"], sigma12=TENS["sigma02"], **kw)
    a = orc.Sim3F(pa, phi0, phi1)
    b = orc.Sim3F(pb, phi1, phi0)
    a.step(300)
    b.step(300)
    ma, mb = a.moments(), b.moments()
    pairs = [(ma[0], mb[1]), (ma[1], mb[0]), (ma[2], mb[2]), (ma[3], mb[3]), (ma[4], mb[4])]
    for k, (u, v) in enumerate(pairs):
        assert np.abs(u - v).max() <= 1e-10 * max(np.abs(u).max(), 1e-12), (k, np.abs(u - v).max())
    # the flow is not trivial: phase 0 has moved
    assert np.abs(ma[0] - phi0).max() > 1e-3


def test_3f_laplace_law_for_phase_0_in_phase_2(orc):
    n = 96
    x, y = _grid(n, n)
    r = np.hypot(x - n / 2 + 0.5, y - n / 2 + 0.5)
    for R0 in (14.0,):
        phi0 = 0.5 + 0.5 * np.tanh((R0 - r) / 2.0)
        phi1 = np.zeros_like(phi0)
        p = orc.make_params3f(n, n, periodic_y=1, D=4.0, **TENS)
        s = orc.Sim3F(p, phi0, phi1)
        s.step(2000)
        # the pressure jump oscillates by about 10% with the box's slowly damped
        # acoustic modes: its mean over 4000 steps is compared
        ratio = []
        for _ in range(40):
            s.step(100)
            f0, f1, ux, uy, pr = s.moments()
            R = math.sqrt(f0.sum() / math.pi)
            ratio.append((pr[r < R - 6].mean() - pr[r > R + 10].mean()) * R / TENS["sigma02"])
        assert np.abs(f1).max() < 1e-12
        assert abs(np.mean(ratio) - 1.0) <= 0.03, (R0, np.mean(ratio))


def _lens_angles(f0, cy, D):
    """Angles (degrees) between the interface line y = cy and the circles fitted
    to the upper and lower arcs of phase 0 (points more than D from the line)."""
    from paper_2311_05091_amd import measure as Me
    out = []
    for side in (+1, -1):
        P = Me.interface_points(f0, mask=lambda X, Y: side * (Y - cy) > D)
        xc, yc, R = Me.fit_circle(P)
        out.append(math.degrees(math.acos(max(-1.0, min(1.0, side * (cy - yc) / R)))))
    return out


def test_3f_lens_corner_angles_follow_neumann_triangle(orc):
    """A drop of phase 0 on the flat interface between phases 1 (below) and 2
    relaxes to a lens whose corner angle inside phase 0 is fixed by the three
    tensions: cos(a0) = (s12^2 - s01^2 - s02^2) / (2 s01 s02) (120 deg for equal
    tensions, where both caps meet the line at 60 deg; 124.2 deg for
    s01, s02, s12 = 0.012, 0.008, 0.01)."""
    nx, ny = 128, 96
    cy = ny / 2 - 0.5
    phi0, phi1 = _drop_on_interface(nx, ny, 16.0, 4.0)
    for s01, s02, s12 in ((0.01, 0.01, 0.01), (0.012, 0.008, 0.01)):
        p = orc.make_params3f(nx, ny, D=4.0, sigma01=s01, sigma02=s02, sigma12=s12, M_deg=0.01)
        s = orc.Sim3F(p, phi0, phi1)
        s.step(4000)
        up, low = _lens_angles(s.moments()[0], cy, 4.0)
        a0 = math.degrees(math.acos((s12 ** 2 - s01 ** 2 - s02 ** 2) / (2 * s01 * s02)))
        assert abs(up + low - a0) <= 2.0, (s01, s02, s12, up, low, a0)
        if s01 == s02:
            assert abs(up - 60.0) <= 2.0 and abs(low - 60.0) <= 2.0, (up, low)
