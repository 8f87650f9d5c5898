"""Pins of the oracle's lattice algebra and pointwise physics.

Each check compares the oracle with something the paper or plain mathematics
fixes independently of the oracle's own code: moment identities the
equilibria are designed to satisfy (Sec. 3), the weighted orthogonality of
the Hermite basis H = N M0 (Sec. 4, App. A), the textbook D2Q9 weights at
d0 = 1/3 (Sec. 3), the BGK special case of the MRT collision, trigonometric
closed forms of the spreading factor and Young's law (Sec. 2.2), and the
Lagrange-multiplier property of mubar (Sec. 2.1).
"""
import math

import numpy as np
import pytest

rng = np.random.default_rng(20231109)


def _lat(orc):
    cx, cy = orc.velocities()
    return cx.astype(float), cy.astype(float)


@pytest.mark.parametrize("d0", [1.0 / 3.0, 0.5, 0.4, 0.6])
def test_weights_moments(orc, d0):
    w = orc.weights(d0)
    cx, cy = _lat(orc)
    assert abs(w.sum() - 1.0) < 1e-15
    assert abs(np.sum(w * cx)) < 1e-15 and abs(np.sum(w * cy)) < 1e-15
    # second-order isotropy: sum w c_a c_b = c_s^2 delta_ab, c_s^2 = d0
    assert abs(np.sum(w * cx * cx) - d0) < 1e-15
    assert abs(np.sum(w * cy * cy) - d0) < 1e-15
    assert abs(np.sum(w * cx * cy)) < 1e-15
    # fourth order: sum w cx^2 cy^2 = c_s^4
    assert abs(np.sum(w * cx ** 2 * cy ** 2) - d0 ** 2) < 1e-15


def test_textbook_weights_at_one_third(orc):
    """d0 = 1/3 reduces to the usual D2Q9 (Sec. 3): 4/9, 1/9, 1/36."""
    w = orc.weights(1.0 / 3.0)
    np.testing.assert_allclose(w, [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, rtol=0, atol=1e-15)


def test_velocity_order_matches_M0_rows(orc):
    cx, cy = _lat(orc)
    M0 = orc.M0()
    np.testing.assert_array_equal(M0[1], cx)
    np.testing.assert_array_equal(M0[2], cy)
    # the opposite of each velocity is in the set (needed by bounce-back)
    pairs = {(int(a), int(b)) for a, b in zip(cx, cy)}
    assert all((-a, -b) in pairs for a, b in pairs)


def test_inverse(orc):
    M0 = orc.M0()
    np.testing.assert_allclose(M0 @ orc.inverse9(M0), np.eye(9), atol=1e-14)
    A = rng.normal(size=(9, 9))
    np.testing.assert_allclose(A @ orc.inverse9(A), np.eye(9), atol=1e-12)


@pytest.mark.parametrize("d0", [1.0 / 3.0, 0.5, 0.4])
def test_hermite_basis_orthogonal(orc, d0):
    """H = N M0 is orthogonal under the weights (Sec. 4, App. A), with norms
    1, c2, c2, c2(1-c2), c2(1-c2), c2^2, c2^2(1-c2), c2^2(1-c2), (c2(1-c2))^2."""
    c2 = d0
    H = orc.N(c2) @ orc.M0()
    G = H @ np.diag(orc.weights(d0)) @ H.T
    q = c2 * (1 - c2)
    expect = np.diag([1, c2, c2, q, q, c2 * c2, c2 * q, c2 * q, q * q])
    np.testing.assert_allclose(G, expect, atol=1e-15)


def test_relaxation_matrix_lower_triangular(orc):
    """S = N^-1 K N is lower triangular with the rates on the diagonal (Sec. 4)."""
    K = rng.uniform(0.5, 1.9, 9)
    S = orc.relaxation_matrix(0.5, K)
    assert np.abs(np.triu(S, 1)).max() == 0.0
    np.testing.assert_allclose(np.diag(S), K, atol=1e-15)
    # for equal rates S is a multiple of the identity
    S1 = orc.relaxation_matrix(0.5, np.full(9, 1.3))
    np.testing.assert_allclose(S1, 1.3 * np.eye(9), atol=1e-15)


def test_collision_reduces_to_bgk(orc):
    """All rates equal s: Lambda = s I, so f* = f - s (f - feq) + (1 - s/2) R."""
    for s in (0.7, 1.0, 1.6):
        f, feq, R = rng.normal(size=(3, 9))
        out = orc.collide(0.5, np.full(9, s), f, feq, R)
        np.testing.assert_allclose(out, f - s * (f - feq) + (1 - s / 2) * R, atol=1e-14)


def test_collision_conserves_phi(orc):
    """Row 0 of S only holds s0 and sum R_i = 0, so sum f* = sum f when sum feq = sum f."""
    K = rng.uniform(0.5, 1.9, 9)
    f = rng.normal(size=9)
    phi = f.sum()
    feq = orc.feq(0.5, phi, 0.3, 0.01, -0.02)
    R = orc.Rpop(0.5, 1e-3, 2e-3, 0.7, 0.1, -0.2)
    out = orc.collide(0.5, K, f, feq, R)
    assert abs(out.sum() - phi) < 1e-14


@pytest.mark.parametrize("d0", [0.5, 1.0 / 3.0])
def test_feq_moments(orc, d0):
    """sum feq = phi, sum c feq = phi u, sum c c feq = c_s^2 eta mubar I (Sec. 3)."""
    cx, cy = _lat(orc)
    phi, emu, Ax, Ay = 0.37, 0.21, 0.013, -0.027
    f = orc.feq(d0, phi, emu, Ax, Ay)
    assert abs(f.sum() - phi) < 1e-15
    assert abs(np.sum(cx * f) - Ax) < 1e-15 and abs(np.sum(cy * f) - Ay) < 1e-15
    assert abs(np.sum(cx * cx * f) - d0 * emu) < 1e-15
    assert abs(np.sum(cy * cy * f) - d0 * emu) < 1e-15
    assert abs(np.sum(cx * cy * f)) < 1e-15


@pytest.mark.parametrize("d0", [0.5, 1.0 / 3.0])
def test_Rpop_moments(orc, d0):
    """sum R = 0, sum c R = d_t(phi u) + a eta c_s^2 grad(mubar) (Sec. 3)."""
    cx, cy = _lat(orc)
    dAx, dAy, a, gx, gy = 1e-3, -2e-3, 0.8, 0.05, -0.07
    R = orc.Rpop(d0, dAx, dAy, a, gx, gy)
    assert abs(R.sum()) < 1e-16
    assert abs(np.sum(cx * R) - (dAx + a * d0 * gx)) < 1e-15
    assert abs(np.sum(cy * R) - (dAy + a * d0 * gy)) < 1e-15
    assert abs(np.sum(cx * cx * R)) < 1e-16 and abs(np.sum(cx * cy * R)) < 1e-16


@pytest.mark.parametrize("d0", [0.5, 1.0 / 3.0])
def test_geq_moments(orc, d0):
    """sum geq = rho_0 gauge, sum c geq = rho u, sum c c geq = P I + rho u u - (Su + uS)/2."""
    cx, cy = _lat(orc)
    gauge, P, rho, ux, uy, Sx, Sy = 0.7, 1.3e-3, 1.4, 0.021, -0.013, 2e-3, -1e-3
    g = orc.geq(d0, gauge, P, rho, ux, uy, Sx, Sy)
    assert abs(g.sum() - gauge) < 1e-15
    assert abs(np.sum(cx * g) - rho * ux) < 1e-15
    assert abs(np.sum(cy * g) - rho * uy) < 1e-15
    assert abs(np.sum(cx * cx * g) - (P + rho * ux * ux - Sx * ux)) < 1e-15
    assert abs(np.sum(cy * cy * g) - (P + rho * uy * uy - Sy * uy)) < 1e-15
    assert abs(np.sum(cx * cy * g) - (rho * ux * uy - 0.5 * (Sx * uy + ux * Sy))) < 1e-15


@pytest.mark.parametrize("d0", [0.5, 1.0 / 3.0])
def test_Fpop_moments(orc, d0):
    """sum F = u.grad(rho), sum c F = F + phi0 rho f, second moments c_s^2 Q I + M2F (Sec. 3)."""
    cx, cy = _lat(orc)
    Q, Gx, Gy, Mxx, Myy, Mxy = 1e-4, 2e-3, -3e-3, 4e-5, -5e-5, 6e-5
    F = orc.Fpop(d0, Q, Gx, Gy, Mxx, Myy, Mxy)
    assert abs(F.sum() - Q) < 1e-16
    assert abs(np.sum(cx * F) - Gx) < 1e-16 and abs(np.sum(cy * F) - Gy) < 1e-16
    assert abs(np.sum(cx * cx * F) - (d0 * Q + Mxx)) < 1e-16
    assert abs(np.sum(cy * cy * F) - (d0 * Q + Myy)) < 1e-16
    assert abs(np.sum(cx * cy * F) - Mxy) < 1e-16


@pytest.mark.parametrize("d0", [0.5, 1.0 / 3.0, 0.45])
def test_pressure_inverts_equilibrium(orc, d0):
    """With g = geq(P), no density gradient and a steady (rho u - S).u, the
    pressure formula of Sec. 3 returns P, whatever the gauge."""
    for gauge in (0.0, 1.0):
        P, rho, ux, uy, Sx, Sy = 2.3e-3, 1.2, 0.03, -0.02, 1e-3, 3e-3
        g = orc.geq(d0, gauge, P, rho, ux, uy, Sx, Sy)
        B = (rho * ux - Sx) * ux + (rho * uy - Sy) * uy
        p = orc.pressure(d0, 1.0, 0.9, g, 0.0, B, B)
        assert abs(p - P) < 1e-15


def test_visc_rate_relation(orc):
    """(1/s - 1/2) c = mu/(rho (1 - phi0)) (Sec. 3) for both factors."""
    for cfac in (0.5, 0.25):
        for (mu, rho, phi0) in ((0.15, 1.0, 0.0), (0.015, 0.1, 0.3), (0.2, 2.0, 0.9)):
            s = orc.visc_rate(mu, rho, phi0, cfac)
            assert abs((1.0 / s - 0.5) * cfac - mu / (rho * (1.0 - phi0))) < 1e-14
    assert orc.visc_rate(0.15, 1.0, 1.0, 0.5) == 0.0


# ---------------------------------------------------------------------------
# Spreading parameters (Sec. 2.2)
# ---------------------------------------------------------------------------
THETAS = [30, 45, 60, 75, 90, 105, 120, 135, 150]


@pytest.mark.parametrize("kappa", [0.0, 0.8, 0.25])
@pytest.mark.parametrize("theta_deg", THETAS)
def test_spreading_factor_closed_form(orc, theta_deg, kappa):
    """1 - 2 sin^2 x = cos 2x: k = 9/(1+kappa) cos((pi/2) cos theta) below 90 deg,
    9/(1+kappa) (2 - cos((pi/2) cos theta)) above (sgn(0) is irrelevant: sin 0 = 0)."""
    th = math.radians(theta_deg)
    c = math.cos(0.5 * math.pi * math.cos(th))
    expect = 9.0 / (1.0 + kappa) * (c if theta_deg <= 90 else 2.0 - c)
    assert abs(orc.spreading_factor(th, kappa) - expect) < 1e-13


@pytest.mark.parametrize("theta_deg", THETAS)
def test_gamma_and_youngs_law(orc, theta_deg):
    """gamma_p from sigma_pq with sigma01 = k sigma12 and Young's law sigma02 =
    sigma01 + sigma12 cos theta equals the printed gamma_p(theta) of Sec. 2.2."""
    th = math.radians(theta_deg)
    s12 = 0.01
    p = orc.make_params(8, 8, theta_deg=theta_deg, sigma12=s12)
    d = orc.derive(p)
    k = d["k"]
    ct = math.cos(th)
    np.testing.assert_allclose(d["gamma"], [(2 * k + ct - 1) * s12, (1 - ct) * s12, (1 + ct) * s12],
                               rtol=1e-13)
    assert abs(d["sigma02"] - d["sigma01"] - s12 * ct) < 1e-15
    # pairwise sums recover the tensions
    g = d["gamma"]
    assert abs(0.5 * (g[1] + g[2]) - s12) < 1e-15
    assert abs(0.5 * (g[0] + g[1]) - d["sigma01"]) < 1e-15
    assert abs(3.0 / d["gammaT"] - sum(1.0 / x for x in g)) < 1e-9


def test_eta_from_relaxation(orc):
    """(M_cst + M_deg)/gamma_1 = (1/s1 - 1/2) eta c_s^2 (Sec. 3)."""
    p = orc.make_params(8, 8, theta_deg=60, sigma12=0.01, M_cst=0.002, M_deg=0.01, tau_phi=0.8)
    d = orc.derive(p)
    lhs = (0.002 + 0.01) / d["gamma"][1]
    assert abs(lhs - (0.8 - 0.5) * d["eta"] * 0.5) < 1e-12 * lhs


# ---------------------------------------------------------------------------
# Chemical potentials (Sec. 2.1)
# ---------------------------------------------------------------------------
def test_lagrange_multiplier_property(orc):
    """sum_p mubar_p / gamma_p = 0: the multiplier keeps phi0 + phi1 + phi2 = 1."""
    gam = [0.12, 0.005, 0.015]
    for _ in range(20):
        phi0, phi1 = rng.uniform(0, 0.5, 2)
        lap0, lap1 = rng.normal(scale=0.05, size=2)
        mu, mub = orc.chemical_potentials(gam, 4.0, phi0, phi1, lap0, lap1)
        assert abs(sum(m / g for m, g in zip(mub, gam))) < 1e-13 * max(1.0, np.abs(mub).max() / 0.005)


def test_binary_reduction(orc):
    """phi0 = 0 everywhere: mu2 = -(gamma2/gamma1) mu1 and mubar1 = mu1 exactly (binary CH)."""
    gam = [0.12, 0.005, 0.015]
    for _ in range(20):
        phi1 = rng.uniform(-0.1, 1.1)
        lap1 = rng.normal(scale=0.05)
        mu, mub = orc.chemical_potentials(gam, 4.0, 0.0, phi1, 0.0, lap1)
        assert abs(mu[0]) < 1e-18
        assert abs(mu[2] + gam[2] / gam[1] * mu[1]) < 1e-15
        assert abs(mub[1] - mu[1]) < 1e-15


def test_tanh_profile_zero_potential(orc):
    """phi = 1/2 + 1/2 tanh(2x/D) balances the bulk and gradient terms: with the
    exact second derivative the chemical potential vanishes (Sec. 2.1)."""
    D = 4.0
    gam = [0.12, 0.005, 0.015]
    for x in np.linspace(-6, 6, 25):
        t = math.tanh(2 * x / D)
        phi = 0.5 + 0.5 * t
        lap = -(4.0 / D ** 2) * t * (1 - t * t)  # d^2/dx^2 of the profile
        mu, _ = orc.chemical_potentials(gam, D, 0.0, phi, 0.0, lap)
        assert abs(mu[1]) < 1e-16
