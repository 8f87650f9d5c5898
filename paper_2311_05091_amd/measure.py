"""Measurements on phase fields: interface fit, contact angle, Laplace jump,
and the closed-form droplet shapes the paper compares against.

Pure numpy/scipy post-processing of fields read back from the library; none
of the step arithmetic lives here.
"""
from __future__ import annotations

import math

import numpy as np


# ---------------------------------------------------------------------------
# Closed forms (Sec. 4.2 and 4.3)
# ---------------------------------------------------------------------------
def cap_radius(theta_rad: float, R0: float) -> float:
    """Radius of a circular cap of contact angle theta whose area equals a
    semicircle of radius R0 (Sec. 4.2): R = R0 sqrt((pi/2)/(theta - sin cos))."""
    return R0 * math.sqrt((math.pi / 2.0) / (theta_rad - math.sin(theta_rad) * math.cos(theta_rad)))


def cap_height(theta_rad: float, R0: float) -> float:
    """Height H = R (1 - cos theta) of that cap (Sec. 4.2)."""
    return cap_radius(theta_rad, R0) * (1.0 - math.cos(theta_rad))


def cap_radius_from_area(theta_rad: float, area: float) -> float:
    """Radius of a cap of contact angle theta and given area: A = R^2 (theta - sin cos)."""
    return math.sqrt(area / (theta_rad - math.sin(theta_rad) * math.cos(theta_rad)))


def cylinder_lens(theta_rad: float, Rs: float, S0: float):
    """Equilibrium droplet on a cylinder of radius Rs with area S0 (Sec. 4.3).

    The droplet is a circle of radius r whose centre lies k_s = sqrt(r^2 + Rs^2
    - 2 r Rs cos theta) from the cylinder centre; its area outside the cylinder
    (circle minus the circle-circle lens) equals S0.  Returns (r, k_s, H_max)
    with H_max = r + k_s measured from the cylinder centre.  The square inside
    the last square root of the printed area formula is restored (the lens
    geometry requires it).
    """
    def area(r):
        ks = math.sqrt(r * r + Rs * Rs - 2.0 * r * Rs * math.cos(theta_rad))
        a1 = (ks * ks + r * r - Rs * Rs) / (2.0 * ks * r)
        a2 = (ks * ks - r * r + Rs * Rs) / (2.0 * ks * Rs)
        a1 = min(1.0, max(-1.0, a1))
        a2 = min(1.0, max(-1.0, a2))
        h = (ks * ks - r * r + Rs * Rs) / (2.0 * ks)
        return (math.pi * r * r - r * r * math.acos(a1) - Rs * Rs * math.acos(a2)
                + ks * math.sqrt(max(0.0, Rs * Rs - h * h)))

    lo, hi = 1e-6 * Rs, 1e3 * Rs
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if area(mid) < S0:
            lo = mid
        else:
            hi = mid
    r = 0.5 * (lo + hi)
    ks = math.sqrt(r * r + Rs * Rs - 2.0 * r * Rs * math.cos(theta_rad))
    return r, ks, r + ks


# ---------------------------------------------------------------------------
# Interface extraction and circle fit
# ---------------------------------------------------------------------------
def interface_points(phi: np.ndarray, level: float = 0.5, mask=None):
    """Sub-cell points where phi crosses `level` along grid rows and columns.

    `mask(x, y)` (vectorised) selects which points to keep.
    """
    pts = []
    ny, nx = phi.shape
    a = phi - level
    # along x
    s = a[:, :-1] * a[:, 1:]
    jy, jx = np.nonzero(s < 0)
    t = a[jy, jx] / (a[jy, jx] - a[jy, jx + 1])
    pts.append(np.stack([jx + t, jy.astype(float)], 1))
    # along y
    s = a[:-1, :] * a[1:, :]
    jy, jx = np.nonzero(s < 0)
    t = a[jy, jx] / (a[jy, jx] - a[jy + 1, jx])
    pts.append(np.stack([jx.astype(float), jy + t], 1))
    P = np.concatenate(pts, 0)
    if mask is not None and len(P):
        P = P[mask(P[:, 0], P[:, 1])]
    return P


def fit_circle(P: np.ndarray):
    """Algebraic (Kasa) circle fit refined by Gauss-Newton on geometric distance."""
    x, y = P[:, 0], P[:, 1]
    A = np.stack([x, y, np.ones_like(x)], 1)
    b = x * x + y * y
    c = np.linalg.lstsq(A, b, rcond=None)[0]
    xc, yc = c[0] / 2.0, c[1] / 2.0
    R = math.sqrt(c[2] + xc * xc + yc * yc)
    for _ in range(50):
        dx, dy = x - xc, y - yc
        d = np.sqrt(dx * dx + dy * dy)
        res = d - R
        J = np.stack([-dx / d, -dy / d, -np.ones_like(d)], 1)
        step = np.linalg.lstsq(J, -res, rcond=None)[0]
        xc, yc, R = xc + step[0], yc + step[1], R + step[2]
        if np.abs(step).max() < 1e-12:
            break
    return float(xc), float(yc), float(R)


def droplet_on_flat_wall(phi1: np.ndarray, y_wall: float, D: float, x_period=None):
    """Contact angle and height of a droplet resting on a flat wall at y = y_wall.

    The circle is fitted to the phi1 = 1/2 contour above y_wall + D (the
    diffuse triple-line region is excluded, Sec. 4.2).  cos(theta) =
    (y_wall - y_c)/R.  Returns dict(theta_deg, R, xc, yc, height).
    """
    ny, nx = phi1.shape
    # centre the droplet column-wise so that periodic wrap does not split it
    col = phi1.sum(0)
    shift = 0
    if x_period:
        shift = nx // 2 - int(np.argmax(np.convolve(col, np.ones(9), "same")))
        phi1 = np.roll(phi1, shift, axis=1)
    P = interface_points(phi1, 0.5, mask=lambda x, y: y > y_wall + D)
    xc, yc, R = fit_circle(P)
    c = (y_wall - yc) / R
    c = min(1.0, max(-1.0, c))
    theta = math.degrees(math.acos(c))
    return {"theta_deg": theta, "R": R, "xc": xc - shift, "yc": yc,
            "height": yc + R - y_wall, "npts": int(len(P))}


def droplet_on_cylinder(phi1: np.ndarray, centre, Rs: float, D: float):
    """Contact angle of a droplet on a cylinder (centre, radius Rs).

    Fits a circle to the phi1 = 1/2 contour farther than Rs + D from the
    cylinder centre; inverts k_s^2 = r^2 + Rs^2 - 2 r Rs cos(theta) (Sec. 4.3).
    """
    cx, cy = centre
    P = interface_points(phi1, 0.5, mask=lambda x, y: np.hypot(x - cx, y - cy) > Rs + D)
    xc, yc, r = fit_circle(P)
    ks = math.hypot(xc - cx, yc - cy)
    c = (r * r + Rs * Rs - ks * ks) / (2.0 * r * Rs)
    c = min(1.0, max(-1.0, c))
    return {"theta_deg": math.degrees(math.acos(c)), "r": r, "ks": ks, "H_max": r + ks,
            "xc": xc, "yc": yc}


def laplace_jump(p: np.ndarray, phi1: np.ndarray, centre, R: float, D: float):
    """Pressure inside minus outside a circular droplet, averaged away from the
    interface (inside: distance < R - 2D; outside: distance > R + 2D)."""
    ny, nx = p.shape
    y, x = np.mgrid[0:ny, 0:nx]
    d = np.hypot(x - centre[0], y - centre[1])
    inside = d < R - 2.0 * D
    outside = d > R + 2.0 * D
    return float(p[inside].mean() - p[outside].mean())


def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    """||a - b||_2 / ||b||_2 (0 when both are zero)."""
    nb = float(np.linalg.norm(np.asarray(b, dtype=np.float64).ravel()))
    na = float(np.linalg.norm((np.asarray(a, dtype=np.float64) - b).ravel()))
    return na / nb if nb > 0 else na
