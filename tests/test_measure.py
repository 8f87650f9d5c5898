"""Closed forms of Sec. 4.2 and 4.3 and the interface measurements."""
import math
import os

import numpy as np
import pytest

from paper_2311_05091_amd import measure as Me

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table1_flat_wall_heights.txt")


def _table1():
    rows = [l.split() for l in open(GOLD) if l.strip() and not l.startswith("#")]
    return [(float(a), float(b), float(c)) for a, b, c in rows]


def test_table1_closed_form():
    """H/R0 = (1 - cos t) sqrt((pi/2)/(t - sin t cos t)) reproduces the Table 1
    row labelled "Numerical" to its 4 printed digits (the labels look swapped)."""
    for th, _, num in _table1():
        h = Me.cap_height(math.radians(th), 1.0)
        assert abs(h - num) <= 6e-5, (th, h, num)


def test_table1_relative_errors_consistent():
    """The printed relative errors are |analytical - numerical|/numerical-row
    differences of the two rows (within the 2-digit rounding)."""
    errs = [2.72, 0.72, 0.15, 0.16, 0.0, 0.48, 0.04, 0.25, 0.03]
    for (th, a, n), e in zip(_table1(), errs):
        assert abs(100 * abs(a - n) / n - e) < 0.03 or abs(100 * abs(a - n) / a - e) < 0.03


def test_cap_area_consistent():
    for th in (30, 60, 90, 120, 150):
        t = math.radians(th)
        R = Me.cap_radius(t, 50.0)
        assert abs(R * R * (t - math.sin(t) * math.cos(t)) - math.pi * 50.0 ** 2 / 2) < 1e-9
        assert abs(Me.cap_radius_from_area(t, math.pi * 50.0 ** 2 / 2) - R) < 1e-12


def test_cylinder_lens_limits():
    """theta = 90 deg on a cylinder: the circles meet at right angles, k_s^2 = r^2 + Rs^2;
    the droplet area outside the cylinder is the circle minus the lens."""
    Rs = 150.0
    S0 = math.pi * 120.0 ** 2
    r, ks, H = Me.cylinder_lens(math.radians(90.0), Rs, S0)
    assert abs(ks * ks - (r * r + Rs * Rs)) < 1e-6 * ks * ks
    # brute-force area of {|x - c| < r} minus {|x| < Rs} on a fine grid
    h = 0.5
    xs = np.arange(-400, 400, h) + h / 2
    X, Y = np.meshgrid(xs, xs)
    inside = (X ** 2 + (Y - ks) ** 2 < r * r) & (X ** 2 + Y ** 2 >= Rs * Rs)
    assert abs(inside.sum() * h * h / S0 - 1) < 2e-3
    # larger contact angle -> the droplet sits higher
    H30 = Me.cylinder_lens(math.radians(30.0), Rs, S0)[2]
    H150 = Me.cylinder_lens(math.radians(150.0), Rs, S0)[2]
    assert H30 < H < H150


def test_circle_fit_exact():
    t = np.linspace(0, 2 * np.pi, 50, endpoint=False)
    P = np.stack([3.0 + 7.5 * np.cos(t), -2.0 + 7.5 * np.sin(t)], 1)
    xc, yc, R = Me.fit_circle(P)
    assert abs(xc - 3) < 1e-10 and abs(yc + 2) < 1e-10 and abs(R - 7.5) < 1e-10


def test_contact_angle_of_synthetic_cap():
    """A sharp-ish cap with a known angle is measured within 1 degree."""
    ny, nx = 80, 160
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    yw, R, th = 7.5, 30.0, math.radians(60.0)
    yc = yw - R * math.cos(th)
    phi = 0.5 + 0.5 * np.tanh((R - np.hypot(x - 80, y - yc)) / 2.0)
    phi[y < yw] = 0.0
    m = Me.droplet_on_flat_wall(phi, yw, 4.0)
    assert abs(m["theta_deg"] - 60.0) < 1.0
