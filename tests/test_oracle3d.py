"""Pins of the three-dimensional (D3Q15) oracle against what the paper and the
mathematics fix: the lattice algebra of Appendix A (weights, the weighted
orthogonality of the Hermite matrix H = N_H M0, the lower-triangular
relaxation matrix), the moments the equilibria and sources of Sec. 3 are
designed to have, the inversion of g^eq by the 3D pressure formula, and the
physics of the full step (exact phase-mass conservation, plane Poiseuille
flow and shear-wave decay for the two viscosity relations, the linearised CH
decay rate, the Laplace law of a sphere, and Galilean consistency of a
translating interface at density ratio 10).

Mobility: the explicit scheme is stable on D3Q15 only for M_cst + M_deg up
to about 0.005 (D = 4): the 15-point Laplacian of the checkerboard mode is
-9.33 (-5.33 for the 9-point one in 2D), and the fastest CH mode decays at
about M (3D/4) lap^2 per step; 0.006 blows up within 100 steps, 0.005 and
below do not.  The 3D runs use 0.004."""
import math

import numpy as np
import pytest

D0S = [0.5, 0.4, 1.0 / 3.0]


@pytest.fixture(scope="module")
def O(orc):
    return orc


def test_weights(O):
    c = O.velocities3()
    for d0 in D0S:
        w = O.weights3(d0)
        assert abs(w.sum() - 1) < 1e-15
        assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), d0 * np.eye(3), atol=1e-15)
        assert abs(np.sum(w * c[:, 0] ** 2 * c[:, 1] ** 2) - d0 * d0) < 1e-15
        assert np.allclose(np.einsum("i,ia->a", w, c), 0.0)
    # d0 = 1/3: the standard D3Q15 weights
    assert np.allclose(O.weights3(1 / 3)[[0, 1, 7]], [2 / 9, 1 / 9, 1 / 72])
    # d0 = 1/2 leaves no weight on the rest velocity
    assert abs(O.weights3(0.5)[0]) < 1e-16


@pytest.mark.parametrize("d0", D0S)
def test_hermite_matrix_is_weight_orthogonal(O, d0):
    """H = N_H M0 (App. A, c = 1): rows orthogonal under sum_i w_i; norms of
    the zeroth to second order rows are 1, c_s^2, c_s^2 (1 - c_s^2)... """
    H = O.N3(d0) @ O.M0_3()
    w = O.weights3(d0)
    G = H @ np.diag(w) @ H.T
    assert np.abs(G - np.diag(np.diag(G))).max() < 1e-14
    cs2 = d0
    n = np.diag(G)
    assert abs(n[0] - 1) < 1e-14 and np.allclose(n[1:4], cs2)
    assert np.allclose(n[4:7], cs2 - cs2 ** 2)          # sum w (cx^2 - cs2)^2 = cs2 (1 - cs2)
    assert np.allclose(n[7:10], cs2 ** 2)               # sum w cx^2 cy^2
    assert np.allclose(n[10:13], cs2 ** 2 * (1 - cs2))  # sum w cx^2 (cy^2 - cs2)^2 on D3Q15
    # a change of any entry of N_H breaks the orthogonality (rows 4-6, 10-12, 14)
    for r, col in ((4, 0), (10, 1), (14, 0), (14, 4)):
        N = O.N3(d0)
        N[r, col] *= 1.1
        Hb = N @ O.M0_3()
        Gb = Hb @ np.diag(w) @ Hb.T
        if d0 == 0.5 and r == 14:
            continue   # w0 = 0 at d0 = 1/2: row 14 is then zero on the weighted lattice
        assert np.abs(Gb - np.diag(np.diag(Gb))).max() > 1e-6


def test_relaxation_matrix_lower_triangular(O):
    K = np.array([1.0, 1.2, 1.2, 1.2, 0.9, 0.9, 0.9, 1.3, 1.3, 1.3, 1.1, 1.1, 1.1, 1.1, 0.8])
    S = O.relaxation_matrix3(0.5, K)
    assert np.abs(np.triu(S, 1)).max() < 1e-15
    assert np.allclose(np.diag(S), K)
    assert np.allclose(O.relaxation_matrix3(0.4, np.full(15, 1.3)), 1.3 * np.eye(15))


def test_collision_reduces_to_bgk_and_conserves(O):
    rng = np.random.default_rng(1)
    f, feq, R = rng.normal(size=15), rng.normal(size=15), rng.normal(size=15)
    s = 1.25
    out = O.collide3(0.5, np.full(15, s), f, feq, R)
    assert np.allclose(out, f - s * (f - feq) + (1 - s / 2) * R, atol=1e-13)
    K = np.array([1.0, 1.2, 1.2, 1.2, 0.9, 0.9, 0.9, 1.3, 1.3, 1.3, 1.1, 1.1, 1.1, 1.1, 0.8])
    feq[:] = f + 0.01 * rng.normal(size=15)
    feq += (f.sum() - feq.sum()) / 15      # same zeroth moment
    out = O.collide3(0.5, K, f, feq, np.zeros(15))
    assert abs(out.sum() - f.sum()) < 1e-13


@pytest.mark.parametrize("d0", [0.5, 0.4])
def test_equilibrium_and_source_moments(O, d0):
    """f^eq: sum = phi, sum c = phi u, sum cc = c_s^2 eta mubar I; g^eq: sum =
    gauge, sum c = rho u, sum cc = P I + rho uu - (Su + uS)/2; F_i: sum = Q,
    sum c = G, sum cc = c_s^2 Q I + M2F (Sec. 3)."""
    c = O.velocities3()
    cc = np.einsum("ia,ib->iab", c, c)
    phi, emu, A = 0.7, 0.013, np.array([0.01, -0.02, 0.005])
    fe = O.feq3(d0, phi, emu, A)
    assert abs(fe.sum() - phi) < 1e-15
    assert np.allclose(c.T @ fe, A, atol=1e-16)
    assert np.allclose(np.einsum("i,iab->ab", fe, cc), d0 * emu * np.eye(3), atol=1e-16)
    gauge, P, rho = 0.3, 0.02, 0.8
    u, S = np.array([0.03, -0.01, 0.02]), np.array([1e-3, 2e-3, -5e-4])
    ge = O.geq3(d0, gauge, P, rho, u, S)
    assert abs(ge.sum() - gauge) < 1e-15
    assert np.allclose(c.T @ ge, rho * u, atol=1e-16)
    Pi = P * np.eye(3) + rho * np.outer(u, u) - 0.5 * (np.outer(S, u) + np.outer(u, S))
    assert np.allclose(np.einsum("i,iab->ab", ge, cc), Pi, atol=1e-16)
    Q, G = 0.004, np.array([1e-3, -2e-3, 3e-3])
    M2 = np.array([1e-3, 2e-3, -1e-3, 5e-4, -7e-4, 3e-4])
    Fp = O.Fpop3(d0, Q, G, M2)
    Mt = np.array([[M2[0], M2[3], M2[5]], [M2[3], M2[1], M2[4]], [M2[5], M2[4], M2[2]]])
    assert abs(Fp.sum() - Q) < 1e-16
    assert np.allclose(c.T @ Fp, G, atol=1e-16)
    assert np.allclose(np.einsum("i,iab->ab", Fp, cc), d0 * Q * np.eye(3) + Mt, atol=1e-16)


@pytest.mark.parametrize("d0", [0.5, 0.4, 1.0 / 3.0])
def test_pressure_inverts_equilibrium(O, d0):
    """With u.grad(rho) = 0 and a steady B the 3D pressure formula returns the
    P of g^eq exactly (any gauge)."""
    u, S = np.array([0.03, -0.01, 0.02]), np.array([1e-3, 2e-3, -5e-4])
    rho, P = 0.9, 0.0123
    B = float(np.dot(rho * u - S, u))
    for gauge in (0.0, 1.0):
        g = O.geq3(d0, gauge, P, rho, u, S)
        assert abs(O.pressure3(d0, 1.0, 1.1, g, 0.0, B, B) - P) < 1e-15


def _sim3(O, nx, ny, nz, phi0, phi1, **kw):
    return O.Sim3(O.make_params3(nx, ny, nz, **kw), phi0, phi1)


def test_mass_conservation_3d(O):
    """Sum of phi1 is invariant to rounding, with walls in z, density ratio 10
    (S active) and a solid sphere."""
    n = 14
    z, y, x = np.mgrid[0:n, 0:n, 0:n].astype(float)
    r0 = np.sqrt((x - 4.5) ** 2 + (y - 6.5) ** 2 + (z - 6.5) ** 2)
    phi0 = 0.5 - 0.5 * np.tanh((r0 - 3.0) / 2.0)
    r1 = np.sqrt((x - 9.0) ** 2 + (y - 6.5) ** 2 + (z - 7.0) ** 2)
    phi1 = (1 - phi0) * (0.5 + 0.5 * np.tanh((4.0 - r1) / 2.0))
    s = _sim3(O, n, n, n, phi0, phi1, periodic=(1, 1, 0), d0=0.4, rho=(1.0, 1.0, 0.1), mu=(0.15, 0.15, 0.015),
              Fb=(1e-5, 0.0, 0.0))
    m0 = s.mass()
    assert abs(m0 - phi1.sum()) < 1e-12 * m0
    s.step(150)
    ph, ux, uy, uz, p = s.moments()
    assert np.isfinite(ph).all() and np.abs(ux).max() > 0
    assert abs(s.mass() - m0) < 1e-12 * m0


def test_poiseuille_between_plates_3d(O):
    """Body-force flow between half-way bounce-back plates at z = -1/2 and
    nz - 1/2: u_x = F/(2 mu)(z + 1/2)(nz - 1/2 - z)."""
    nz, F, mu = 12, 1e-6, 0.15
    ones = np.ones((nz, 2, 2))
    s = _sim3(O, 2, 2, nz, 0 * ones, ones, periodic=(1, 1, 0), theta_deg=90.0, mu=(mu, mu, mu),
              Fb=(F, 0.0, 0.0))
    s.step(8000)
    ph, ux, uy, uz, p = s.moments()
    zz = np.arange(nz)
    uth = F / (2 * mu) * (zz + 0.5) * (nz - 0.5 - zz)
    assert np.abs(ux[:, 0, 0] - uth).max() < 3e-3 * uth.max()
    assert np.abs(uy).max() < 1e-6 * uth.max() and np.abs(uz).max() < 1e-6 * uth.max()


def _shear_rate3(O, diag, n=24, nu=0.15, U=1e-4, T=200):
    z, y, x = np.mgrid[0:n, 0:n, 0:n].astype(float)
    if diag:
        # velocity along (1, 1, 0)/sqrt2 varying along (1, -1, 0): relaxed through the
        # normal-stress moments (s2a)
        ph = 2 * np.pi * (x - y) / n
        ux0 = U / math.sqrt(2) * np.sin(ph)
        uy0 = ux0.copy()
        uz0 = 0 * ux0
        kk = 2 * (2 * np.pi / n) ** 2
    else:
        ph = 2 * np.pi * z / n
        ux0 = U * np.sin(ph)
        uy0 = 0 * ux0
        uz0 = 0 * ux0
        kk = (2 * np.pi / n) ** 2
    ones = np.ones((n, n, n))
    s = _sim3(O, n, n, n, 0 * ones, ones, periodic=(1, 1, 1), theta_deg=90.0, mu=(nu, nu, nu))
    f, g, lag = s.get_state()
    for k in range(n):
        for j in range(n):
            for i in range(n):
                u = (ux0[k, j, i], uy0[k, j, i], uz0[k, j, i])
                g[:, k, j, i] = O.geq3(0.5, 0.0, 0.0, 1.0, u, (0, 0, 0))
                f[:, k, j, i] = O.feq3(0.5, 1.0, 0.0, u)
    s.set_state(f, g, None)
    amp = []
    for _ in range(2):
        ux = s.moments()[1]
        amp.append(np.sum(ux * np.sin(ph)))
        s.step(T)
    return -math.log(amp[1] / amp[0]) / T, nu * kk


def test_shear_wave_axis_3d(O):
    lam, th = _shear_rate3(O, diag=False)
    assert abs(lam / th - 1) < 1e-2


def test_shear_wave_diagonal_3d(O):
    lam, th = _shear_rate3(O, diag=True)
    assert abs(lam / th - 1) < 1.5e-2


@pytest.mark.parametrize("Mc,Md,pbar", [(0.004, 0.0, 0.1), (0.0, 0.005, 0.85), (0.001, 0.004, 0.85)])
def test_linear_ch_decay_rate_3d(O, Mc, Md, pbar):
    """phi1 = pbar + eps cos(kx), phi0 = 0: linearised CH decay rate
    M k^2 [(12/D) g'(pbar) + (3D/4) k^2], k^2 the second-difference symbol."""
    nx, D = 48, 4.0
    x = np.arange(nx)
    k = 2 * np.pi / nx
    phi1 = np.tile(pbar + 1e-6 * np.cos(k * x), (2, 2, 1))
    s = _sim3(O, nx, 2, 2, np.zeros((2, 2, nx)), phi1, periodic=(1, 1, 1), D=D, theta_deg=90.0, M_cst=Mc,
              M_deg=Md)
    # at these mobilities the mode decays by ~1% per 1000 steps: a long window
    # after the initial transient
    s.step(2000)
    t, loga = [], []
    for j in range(12):
        ph = s.moments()[0]
        t.append(s.steps)
        loga.append(math.log(abs(np.fft.rfft(ph[0, 0] - ph[0, 0].mean())[1])))
        s.step(1000)
    lam = -np.polyfit(t, loga, 1)[0]
    gp = 1 - 6 * pbar + 6 * pbar ** 2
    kk = 4 * math.sin(k / 2) ** 2
    lam_th = (Mc + Md * pbar * (1 - pbar)) * kk * (12 / D * gp + 0.75 * D * kk)
    assert abs(lam / lam_th - 1) < 0.04


def test_laplace_law_sphere(O):
    """A free spherical droplet: p_in - p_out = 2 sigma12/R with both principal
    curvatures (the 1-2 tension is sigma12).  The diffuse interface adds an
    O(D/R) excess that shrinks with R (measured: 1.18 at R = 7, 1.14 at R = 8,
    1.11 at R = 9 on D = 4, converged in time); a tension off by a factor of 2
    or a single curvature would give 2 or 0.5."""
    n, R, D, sig = 28, 8.0, 4.0, 0.01
    z, y, x = np.mgrid[0:n, 0:n, 0:n].astype(float)
    c = n / 2 - 0.5
    r = np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2)
    phi1 = 0.5 + 0.5 * np.tanh((R - r) / (D / 2))
    s = _sim3(O, n, n, n, np.zeros_like(phi1), phi1, periodic=(1, 1, 1), theta_deg=90.0, M_cst=0.004, M_deg=0.0,
              sigma12=sig, D=D)
    s.step(1000)
    ph, ux, uy, uz, p = s.moments()
    dp = p[r < R - D].mean() - p[r > R + D].mean()
    Rf = (3 * ph.sum() / (4 * np.pi)) ** (1 / 3)   # radius of the sphere of the same volume
    ratio = dp / (2 * sig / Rf)
    print("3D Laplace ratio", ratio)
    assert 1.0 < ratio < 1.2


def test_translating_interface_3d_density_ratio_10(O):
    """Flat interfaces moving normal to themselves at density ratio 10 on the
    D3Q15 lattice with d0 = 0.4 (where the 3D constants K = 1 - 2 d0 and H
    of the pressure are non-zero): the velocity defect of the moving run
    against the resting one converges at second order in D (see the 2D
    Galilean pins)."""
    U = 0.025
    defects = []
    for D in (4.0, 8.0):
        n = int(16 * D)
        x = np.arange(n, dtype=float)[None, None, :].repeat(2, 0).repeat(2, 1)
        wi = 0.7 * D
        phi1 = 0.5 * (np.tanh((x - n / 4) / (wi / 2)) - np.tanh((x - 3 * n / 4) / (wi / 2)))
        rho = phi1 + 0.1 * (1 - phi1)
        p = O.make_params3(n, 2, 2, periodic=(1, 1, 1), d0=0.4, D=D, theta_deg=90.0, rho=(1.0, 1.0, 0.1),
                           mu=(0.15, 0.15, 0.015), M_cst=0.0, M_deg=0.004)
        steps = int(40 * D / 4)
        res = []
        for vel in (0.0, U):
            s = O.Sim3(p, np.zeros_like(phi1), phi1)
            f, g, lag = s.get_state()
            mub, gm = s.aux()
            eta = s.derived()["eta"]
            for k in range(2):
                for j in range(2):
                    for i in range(n):
                        f[:, k, j, i] = O.feq3(0.4, phi1[k, j, i], eta * mub[k, j, i], (phi1[k, j, i] * vel, 0, 0))
                        g[:, k, j, i] = O.geq3(0.4, 0.0, 0.0, rho[k, j, i], (vel, 0, 0), (0, 0, 0))
            lag[:] = 0
            lag[0] = phi1 * vel
            lag[3] = rho * vel * vel
            s.set_state(f, g, lag)
            s.step(steps)
            res.append(s.moments()[1])
        shift = int(round(U * steps))
        defects.append(np.abs(res[1] - U - np.roll(res[0], shift, axis=2)).max() / U)
    print("3D normal translation defect", defects)
    assert defects[1] < 0.1
    assert defects[0] / defects[1] > 3.0


def test_tangential_flow_along_relaxing_interface_3d(O):
    """Uniform flow U = 0.02 along z, parallel to flat interfaces normal to x
    that relax from twice their equilibrium width at density ratio 10 (S_x u_z
    != 0): momentum is carried with the mass flux rho u - S only if the S part
    of the flux rho uu - (Su + uS)/2 and F_c = -curl(S x u)/2 are right.  The
    defect of the moving run against the resting one converges at second order
    in D (see the 2D pin; a flipped or missing F_c breaks the order)."""
    U = 0.02
    defects = []
    for D in (4.0, 8.0):
        n = int(16 * D)
        x = np.arange(n, dtype=float)[None, None, :].repeat(2, 0).repeat(2, 1)
        wi = 2.0 * D
        phi1 = 0.5 * (np.tanh((x - n / 4) / (wi / 2)) - np.tanh((x - 3 * n / 4) / (wi / 2)))
        rho = phi1 + 0.1 * (1 - phi1)
        Mc = 0.004
        p = O.make_params3(n, 2, 2, periodic=(1, 1, 1), d0=0.4, D=D, theta_deg=90.0, rho=(1.0, 1.0, 0.1),
                           mu=(0.15, 0.15, 0.015), M_cst=Mc, M_deg=0.0)
        steps = int(20 * D / 4)
        res = []
        for vel in (0.0, U):
            s = O.Sim3(p, np.zeros_like(phi1), phi1)
            f, g, lag = s.get_state()
            mub, gm = s.aux()
            d = s.derived()
            S = 0.9 * Mc / d["gamma"][1] * gm          # (rho1 - rho2) M grad(mubar1)/gamma1
            u = np.array([0.0, 0.0, vel])
            for k in range(2):
                for j in range(2):
                    for i in range(n):
                        Sl = S[:, k, j, i]
                        f[:, k, j, i] = O.feq3(0.4, phi1[k, j, i], d["eta"] * mub[k, j, i], phi1[k, j, i] * u)
                        g[:, k, j, i] = O.geq3(0.4, 0.0, 0.0, rho[k, j, i], u, Sl)
            lag[:] = 0
            lag[2] = phi1 * vel                                   # phi1 u
            lag[3] = (rho * vel - S[2]) * vel                     # (rho u - S).u
            lag[6] = S[2] * vel                                   # C_zz
            lag[8] = 0.5 * S[1] * vel                             # C_yz
            lag[9] = 0.5 * S[0] * vel                             # C_xz
            lag[10] = S[1] * vel                                  # psi = S x u: (S_y u_z, -S_x u_z, 0)
            lag[11] = -S[0] * vel
            s.set_state(f, g, lag)
            s.step(steps)
            res.append(s.moments()[3])
        defects.append(np.abs(res[1] - U - res[0]).max() / U)
    order = math.log2(defects[0] / defects[1])
    print("3D tangential defect", defects, "order", order)
    assert defects[1] < 0.01
    assert order > 2.0
