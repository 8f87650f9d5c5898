"""Pins of the oracle's open boundaries (non-equilibrium extrapolation at an
inlet x = 0 and an outlet x = nx - 1, Sec. 4; reading R27) and of the flow
rates behind the relative permeability K_p (Sec. 4.6).

* Pressure-driven channel between half-way walls: the pressure falls
  linearly from p_in at the inlet node to p_out at the outlet node, so the
  interior gradient is (p_in - p_out)/(nx - 1), and the velocity is the
  Poiseuille parabola of that gradient.
* Velocity inlet: the steady volume flux is the same through every column,
  the mean velocity is the imposed u_in (within the 2% the plug inlet loses
  at the no-slip corners), and the profile is parabolic.
* One fluid at rest between equal inlet and outlet pressures stays at rest.
* Stratified co-current flow of two fluids driven by a uniform force in a
  periodic channel (the periodic form of a pressure drop): the flow rate of
  each phase, sum phi_p u_x, matches the steady momentum equation
  d/dy(mu(y) du/dy) = -G solved by finite differences with the simulated
  diffuse viscosity mu(y) = sum_p mu_p phi_p(y), and the sharp two-layer
  solution within the O(D/H) interface width.  K_p is these rates over the
  single-phase rate G H^3/(12 mu_p).
"""
import numpy as np

from paper_2311_05091_amd import geometry as G
from tests._util import oracle_params

MU = 0.15


def _channel(nx, ny, **kw):
    return G.DomainSpec(nx=nx, ny=ny, phi0=np.zeros((ny, nx)), phi1=np.zeros((ny, nx)), periodic_x=0, periodic_y=0,
                        mu=(MU, MU, MU), open_x=1, **kw)


def _run(orc, sp, steps):
    s = orc.Sim(oracle_params(orc, sp), sp.phi0, sp.phi1)
    s.step(steps)
    return s


def test_pressure_driven_channel_is_poiseuille(orc):
    nx, ny, p_in = 80, 33, 1e-4
    s = _run(orc, _channel(nx, ny, inlet_type=0, p_in=p_in, p_out=0.0), 8000)
    phi, ux, uy, p = s.moments()
    grad = (p_in - 0.0) / (nx - 1)
    interior = p[:, 2:nx - 2]
    fit = np.polyfit(np.arange(2, nx - 2), interior[ny // 2], 1)
    assert abs(-fit[0] - grad) <= 1e-3 * grad, (fit[0], grad)
    y = np.arange(ny) + 0.5            # distance from the half-way wall below
    ana = grad / (2 * MU) * y * (ny - y)
    for c in (5, nx // 2, nx - 6):
        assert np.abs(ux[:, c] - ana).max() <= 2e-3 * ana.max(), c
    flux = ux[:, 1:nx - 1].sum(axis=0)
    assert np.ptp(flux) <= 1e-6 * flux.mean()
    # the entrance regions adjust over a few columns; away from them the flow is parallel
    assert np.abs(uy[:, 10:nx - 10]).max() <= 1e-3 * ana.max(), np.abs(uy[:, 10:nx - 10]).max() / ana.max()


def test_velocity_inlet_conserves_flux(orc):
    nx, ny, u_in = 80, 33, 0.01
    s = _run(orc, _channel(nx, ny, inlet_type=1, u_in=u_in, p_out=0.0), 8000)
    phi, ux, uy, p = s.moments()
    # beside the inlet node the imposed plug profile still adjusts (2e-4 more flux in column 1);
    # along the channel the flux varies by about 1e-4: the scheme is weakly compressible and the
    # pressure falls by 2e-3 c_s^2 from inlet to outlet
    flux = ux[:, 2:nx - 1].sum(axis=0)
    assert np.ptp(flux) <= 5e-4 * flux.mean()
    umean = ux[:, nx // 2].mean()
    assert abs(umean - u_in) <= 0.03 * u_in, umean
    y = np.arange(ny) + 0.5
    ana = 6 * umean * y * (ny - y) / ny ** 2
    assert np.abs(ux[:, nx // 2] - ana).max() <= 2e-3 * ana.max()


def test_equal_pressures_keep_fluid_at_rest(orc):
    """One fluid at rest between equal inlet and outlet pressures, with a
    non-zero gauge in lambda_0 (which the extrapolation must cancel): the
    state stays at rest to rounding."""
    sp = _channel(40, 24, inlet_type=0, p_in=0.0, p_out=0.0, rho_gauge=0.7)
    s = _run(orc, sp, 400)
    phi, ux, uy, p = s.moments()
    assert np.abs(ux).max() < 1e-15 and np.abs(uy).max() < 1e-15, (np.abs(ux).max(), np.abs(uy).max())
    assert np.abs(p[:, 1:-1]).max() < 1e-15


def _layered_flow_bvp(phi1_y, mu1, mu2, Gf, ref=16):
    """d/dy(mu(y) du/dy) = -G on the channel [-1/2, ny - 1/2] with u = 0 at
    both half-way walls; mu(y) = mu1 phi1 + mu2 (1 - phi1), phi1 linearly
    interpolated between nodes.  Returns u and phi1 on the nodes."""
    ny = len(phi1_y)
    n = ny * ref
    h = ny / n
    yf = -0.5 + h * np.arange(n + 1)                  # fine grid, walls at both ends
    yn = np.arange(ny, dtype=float)
    ph = np.interp(yf, yn, phi1_y)
    mu = mu1 * ph + mu2 * (1 - ph)
    mh = 0.5 * (mu[1:] + mu[:-1])                     # face viscosities
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


def test_stratified_two_phase_flow_rates_and_kp(orc):
    ny, a, mu1, mu2, Gf = 64, 24.0, 0.3, 0.06, 1e-6
    nx = 4
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    phi1 = 0.5 - 0.5 * np.tanh(2 * (y - (a - 0.5)) / 4.0)    # fluid 1 below y = a (walls at -1/2, ny - 1/2)
    sp = G.DomainSpec(nx=nx, ny=ny, phi0=np.zeros((ny, nx)), phi1=phi1, periodic_x=1, periodic_y=0,
                      mu=(mu1, mu1, mu2), Fb=(Gf, 0.0), theta_deg=90.0, M_deg=0.01)
    s = orc.Sim(oracle_params(orc, sp), sp.phi0, sp.phi1)
    s.step(40000)
    q = s.flow_rates()
    phi, ux, uy, p = s.moments()
    assert abs(q[0] - ux.sum()) <= 1e-12 * abs(q[0])
    assert abs(q[1] + q[2] - q[0]) <= 1e-10 * abs(q[0])
    # against the steady momentum equation with the simulated diffuse viscosity
    u_ode = _layered_flow_bvp(phi[:, 0], mu1, mu2, Gf)
    assert np.abs(ux[:, 0] - u_ode).max() <= 0.01 * u_ode.max(), np.abs(ux[:, 0] - u_ode).max() / u_ode.max()
    q1_ode = nx * float(np.sum(phi[:, 0] * u_ode))
    q2_ode = nx * float(np.sum((1 - phi[:, 0]) * u_ode))
    assert abs(q[1] - q1_ode) <= 0.01 * q1_ode and abs(q[2] - q2_ode) <= 0.01 * q2_ode
    # sharp two-layer solution: mu1 u1' = mu2 u2' = C - G y at the interface y = a
    H, ya = float(ny), a
    # u1 = -G y^2/(2 mu1) + C y/mu1 ; u2 = -G (y^2 - H^2)/(2 mu2) + C (y - H)/mu2 ; continuity at ya
    C = (Gf * ya ** 2 / (2 * mu1) - Gf * (ya ** 2 - H ** 2) / (2 * mu2)) / (ya / mu1 - (ya - H) / mu2)
    Q1 = -Gf * ya ** 3 / (6 * mu1) + C * ya ** 2 / (2 * mu1)
    Q2 = (-Gf * ((H ** 3 - ya ** 3) / 3 - H ** 2 * (H - ya)) / (2 * mu2)
          + C * ((H ** 2 - ya ** 2) / 2 - H * (H - ya)) / mu2)
    assert abs(q[1] / nx - Q1) <= 0.05 * Q1 and abs(q[2] / nx - Q2) <= 0.05 * Q2, (q[1] / nx, Q1, q[2] / nx, Q2)
    # relative permeabilities against the single-phase rates G H^3/(12 mu_p)
    kp1 = q[1] / nx / (Gf * H ** 3 / (12 * mu1))
    kp2 = q[2] / nx / (Gf * H ** 3 / (12 * mu2))
    assert abs(kp1 - Q1 / (Gf * H ** 3 / (12 * mu1))) <= 0.05 * kp1 and 0 < kp2 < 1
