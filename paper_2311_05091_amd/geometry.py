"""Seeded synthetic inputs: solid fields, initial phase fields and parameters.

This module holds no step arithmetic of the method: it only builds the
initial diffuse-interface fields of the paper's test problems (tanh
profiles, Sec. 4.1-4.3) and the synthetic geometries that stand in for the
paper's porous medium and for a batched sweep, plus the raw physical
parameters of each workload.  Both the GPU library and the CPU oracle take
their inputs from here.

Arrays are float64, shape [ny, nx], x fastest.  Node (i, j) sits at
(x, y) = (i, j); walls (non-periodic axes) sit half-way outside the first
and last node.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np


@dataclasses.dataclass
class DomainSpec:
    """Raw inputs of one domain (physical parameters and initial fields)."""
    nx: int
    ny: int
    phi0: np.ndarray
    phi1: np.ndarray
    periodic_x: int = 1
    periodic_y: int = 0
    d0: float = 0.5
    D: float = 4.0
    sigma12: float = 0.01
    theta_deg: float = 60.0
    kappa: float = 0.0
    rho: tuple = (1.0, 1.0, 1.0)
    mu: tuple = (0.15, 0.15, 0.15)
    M_cst: float = 0.0
    M_deg: float = 0.01
    tau_phi: float = 0.8
    s_phi: tuple = (1.0, 1.0, 1.0, 1.0)
    s_g: tuple = (1.0, 1.0, 1.0, 1.0)
    Fb: tuple = (0.0, 0.0)
    u_wall: tuple = (0.0, 0.0)
    omega_wall: float = 0.0
    wall_center: tuple = (0.0, 0.0)
    rho_gauge: float = 0.0
    open_x: int = 0          # 1: inlet at x = 0, outlet at x = nx - 1 (needs periodic_x = 0)
    inlet_type: int = 0      # 0: pressure p_in, 1: velocity (u_in, 0)
    p_in: float = 0.0
    u_in: float = 0.0
    p_out: float = 0.0
    phi1_in: float = 0.0     # phase-1 share of the fluid entering at the inlet
    name: str = ""

    def param_dict(self) -> dict:
        d = dataclasses.asdict(self)
        for k in ("phi0", "phi1", "name"):
            d.pop(k)
        return d


def _tanh_step(s, width):
    """1/2 + 1/2 tanh(s / (width/2)): 0 -> 1 across a layer of the given width."""
    return 0.5 + 0.5 * np.tanh(s / (0.5 * width))


def _grid(nx, ny):
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    return x, y


# ---------------------------------------------------------------------------
# Paper test problems
# ---------------------------------------------------------------------------
def flat_wall_droplet(nx=128, ny=64, wall_rows=8, R0=25.0, D=4.0, theta_deg=60.0,
                      sigma12=0.01, tau=0.8, name="flat_wall_droplet") -> DomainSpec:
    """Semicircular droplet on a flat diffuse wall (Sec. 4.2 initial fields).

    The solid occupies the bottom ``wall_rows`` rows: phi0 = 1/2 - 1/2 tanh(2(y - y_w)/D)
    with y_w = wall_rows - 1/2; the droplet is centred on the wall at x = nx/2 - 1/2.
    Density and viscosity ratios 1; tau sets the kinematic viscosity
    nu = (tau - 1/2) c_s^2 with c_s^2 = 1/2.
    """
    x, y = _grid(nx, ny)
    yw = wall_rows - 0.5
    xc = nx / 2.0 - 0.5
    phi0 = 0.5 - 0.5 * np.tanh(2.0 * (y - yw) / D)
    r = np.hypot(x - xc, y - yw)
    phi1 = (1.0 - phi0) * _tanh_step(R0 - r, D)
    nu = (tau - 0.5) * 0.5
    return DomainSpec(nx=nx, ny=ny, phi0=phi0, phi1=phi1, periodic_x=1, periodic_y=0,
                      D=D, sigma12=sigma12, theta_deg=theta_deg, kappa=0.0,
                      rho=(1.0, 1.0, 1.0), mu=(nu, nu, nu), name=name)


def cylinder_droplet(n=1024, Rs=150.0, R0=120.0, D=4.0, theta_deg=60.0, sigma12=0.01,
                     rho_ratio=10.0, mu_ratio=10.0, tau=0.8, centre=None,
                     name="cylinder_droplet") -> DomainSpec:
    """Droplet resting tangent on top of a diffuse solid cylinder (Sec. 4.3 fields).

    kappa = R0/Rs (Sec. 4.3).  Fluid 1 is the droplet: rho1/rho2 = rho_ratio,
    mu1/mu2 = mu_ratio, rho1 = 1, nu1 = (tau - 1/2)/2.
    """
    x, y = _grid(n, n)
    cx, cy = centre if centre is not None else (n / 2.0 - 0.5, 350.0 * n / 1024.0)
    phi0 = _tanh_step(Rs - np.hypot(x - cx, y - cy), D)
    dy = cy + Rs + R0
    phi1 = (1.0 - phi0) * _tanh_step(R0 - np.hypot(x - cx, y - dy), D)
    mu1 = (tau - 0.5) * 0.5
    return DomainSpec(nx=n, ny=n, phi0=phi0, phi1=phi1, periodic_x=1, periodic_y=0,
                      D=D, sigma12=sigma12, theta_deg=theta_deg, kappa=R0 / Rs,
                      rho=(1.0, 1.0, 1.0 / rho_ratio), mu=(mu1, mu1, mu1 / mu_ratio),
                      name=name)


def free_droplet(n=96, R=20.0, D=4.0, sigma12=0.01, theta_deg=90.0, tau=0.8,
                 name="free_droplet") -> DomainSpec:
    """Circular droplet of fluid 1 in fluid 2, no solid, periodic box."""
    x, y = _grid(n, n)
    c = n / 2.0 - 0.5
    phi0 = np.zeros((n, n))
    phi1 = _tanh_step(R - np.hypot(x - c, y - c), D)
    nu = (tau - 0.5) * 0.5
    return DomainSpec(nx=n, ny=n, phi0=phi0, phi1=phi1, periodic_x=1, periodic_y=1,
                      D=D, sigma12=sigma12, theta_deg=theta_deg, mu=(nu, nu, nu), name=name)


def solid_disk_box(n=16, Rs=3.0, R0=4.0, D=4.0, theta_deg=60.0, rho=(1.0, 1.0, 1.0),
                   mu=(0.15, 0.15, 0.15), periodic_y=1, ny=None,
                   name="solid_disk_box") -> DomainSpec:
    """Small box with a diffuse solid disk and a droplet next to it (parity cases)."""
    ny = n if ny is None else ny
    x, y = _grid(n, ny)
    phi0 = _tanh_step(Rs - np.hypot(x - 0.3 * n, y - 0.4 * ny), D)
    phi1 = (1.0 - phi0) * _tanh_step(R0 - np.hypot(x - 0.62 * n, y - 0.55 * ny), D)
    return DomainSpec(nx=n, ny=ny, phi0=phi0, phi1=phi1, periodic_x=1, periodic_y=periodic_y,
                      D=D, theta_deg=theta_deg, rho=rho, mu=mu, name=name)


# ---------------------------------------------------------------------------
# Synthetic porous medium (stands in for the paper's micro-CT sandpack)
# ---------------------------------------------------------------------------
def random_circles(nx, ny, rmin, rmax, porosity, seed, wall_gap=4.0, pair_gap=2.0,
                   keep_clear_x=0.0, max_tries=2_000_000):
    """Random sequential addition of non-overlapping circles, periodic in x.

    Radii are uniform in [rmin, rmax]; centres keep ``wall_gap`` cells (plus the
    radius) from the y walls, pairs keep r_a + r_b + pair_gap apart, and no
    circle reaches into x < keep_clear_x.  Stops when the solid area fraction
    reaches 1 - porosity.
    """
    rng = np.random.default_rng(seed)
    target = (1.0 - porosity) * nx * ny
    cell = 2.0 * rmax + pair_gap
    gx, gy = int(math.ceil(nx / cell)), int(math.ceil(ny / cell))
    buckets = {}
    circles = []
    area = 0.0
    tries = 0
    while area < target and tries < max_tries:
        tries += 1
        r = rng.uniform(rmin, rmax)
        cx = rng.uniform(0.0, nx)
        cy = rng.uniform(r + wall_gap, ny - r - wall_gap)
        if keep_clear_x > 0.0 and (cx - r < keep_clear_x + 2.0 or cx + r > nx - 2.0):
            continue
        bx, by = int(cx / cell) % gx, int(cy / cell)
        ok = True
        for ddx in (-1, 0, 1):
            for ddy in (-1, 0, 1):
                for (ox, oy, orr) in buckets.get(((bx + ddx) % gx, by + ddy), ()):
                    dx = abs(cx - ox)
                    dx = min(dx, nx - dx)
                    if dx * dx + (cy - oy) ** 2 < (r + orr + pair_gap) ** 2:
                        ok = False
                        break
                if not ok:
                    break
            if not ok:
                break
        if not ok:
            continue
        buckets.setdefault((bx, by), []).append((cx, cy, r))
        circles.append((cx, cy, r))
        area += math.pi * r * r
    return circles


def render_circles(nx, ny, circles, width):
    """phi0 = max over circles of 1/2 + 1/2 tanh((r - d)/(width/2)), x-periodic."""
    phi0 = np.zeros((ny, nx))
    pad = int(math.ceil(2.5 * width)) + 1
    for (cx, cy, r) in circles:
        x0 = int(math.floor(cx - r - pad))
        x1 = int(math.ceil(cx + r + pad))
        y0 = max(0, int(math.floor(cy - r - pad)))
        y1 = min(ny, int(math.ceil(cy + r + pad)))
        xs = np.arange(x0, x1)
        ys = np.arange(y0, y1)
        X, Y = np.meshgrid(xs, ys)
        val = _tanh_step(r - np.hypot(X - cx, Y - cy), width)
        cols = np.mod(xs, nx)
        sub = phi0[y0:y1][:, cols]
        phi0[y0:y1, cols] = np.maximum(sub, val)
    return phi0


def porous_medium(nx=4096, ny=2048, rmin=8.0, rmax=24.0, porosity=0.6, width=3.0,
                  inlet=256, seed=3, theta_deg=45.0, sigma12=0.01, body_force=1e-6,
                  mu_ratio=5.0, tau=0.8, name="porous_displacement") -> DomainSpec:
    """Synthetic 2D porous medium for the displacement workload.

    Circles fill the region x >= inlet; the obstacle-free slab x < inlet starts
    as wetting fluid 1 with a tanh front, the rest as fluid 2.  A body force
    drives the flow along +x.  Periodic in x, walls in y.
    """
    circles = random_circles(nx, ny, rmin, rmax, porosity * 1.0, seed, keep_clear_x=inlet)
    phi0 = render_circles(nx, ny, circles, width)
    x, _ = _grid(nx, ny)
    front = _tanh_step(inlet - 0.5 - x, width)
    phi1 = (1.0 - phi0) * front
    mu1 = (tau - 0.5) * 0.5
    return DomainSpec(nx=nx, ny=ny, phi0=phi0, phi1=phi1, periodic_x=1, periodic_y=0,
                      D=width, sigma12=sigma12, theta_deg=theta_deg, kappa=0.0,
                      rho=(1.0, 1.0, 1.0), mu=(mu1, mu1, mu1 / mu_ratio),
                      Fb=(body_force, 0.0), name=name)


def solid_fraction(phi0: np.ndarray) -> float:
    """Share of nodes inside the solid (phi0 > 1/2); porosity is 1 minus this."""
    return float(np.mean(phi0 > 0.5))


# ---------------------------------------------------------------------------
# Batched sweep: droplets on random rough walls
# ---------------------------------------------------------------------------
def rough_wall_droplet(s, seed, theta_deg=None, D=4.0, sigma12=0.01, tau=0.8,
                       base=24.0, n_modes=3, amp_max=4.0, max_mode=3,
                       name=None) -> DomainSpec:
    """Droplet of radius 0.2 s on a random rough wall h(x) = base + sum of sinusoids.

    h(x) = base + sum_k a_k sin(2 pi n_k x / s + p_k), a_k ~ U[0, amp_max] (so the
    amplitude is at most 12 cells), n_k ~ U{1..max_mode}, p_k ~ U[0, 2 pi); contact
    angle ~ U[30, 150] deg unless given.  The solid field is a tanh of the
    first-order normal distance (y - h)/sqrt(1 + h'^2), so the diffuse wall keeps
    the width D normal to the surface also where the wall is steep.
    Periodic in x (the wall is s-periodic), walls in y.
    """
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.0, amp_max, n_modes)
    nk = rng.integers(1, max_mode + 1, n_modes)
    ph = rng.uniform(0.0, 2.0 * math.pi, n_modes)
    th = rng.uniform(30.0, 150.0) if theta_deg is None else theta_deg
    x, y = _grid(s, s)
    k = 2.0 * math.pi * nk / s
    h = base + sum(a[i] * np.sin(k[i] * x + ph[i]) for i in range(n_modes))
    dh = sum(a[i] * k[i] * np.cos(k[i] * x + ph[i]) for i in range(n_modes))
    dist = (y - h) / np.sqrt(1.0 + dh * dh)
    phi0 = 0.5 - 0.5 * np.tanh(2.0 * dist / D)
    R0 = 0.2 * s
    xc = s / 2.0
    hc = base + sum(a[i] * math.sin(k[i] * xc + ph[i]) for i in range(n_modes))
    phi1 = (1.0 - phi0) * _tanh_step(R0 - np.hypot(x - xc, y - hc), D)
    nu = (tau - 0.5) * 0.5
    return DomainSpec(nx=s, ny=s, phi0=phi0, phi1=phi1, periodic_x=1, periodic_y=0,
                      D=D, sigma12=sigma12, theta_deg=float(th), kappa=0.0,
                      rho=(1.0, 1.0, 1.0), mu=(nu, nu, nu),
                      name=name or "rough_wall_%d" % seed)


def batched_sweep(n_domains=512, smin=128, smax=512, seed0=4000, **kw) -> List[DomainSpec]:
    """Independent rough-wall droplets with side lengths uniform in [smin, smax]."""
    out = []
    for i in range(n_domains):
        rng = np.random.default_rng(seed0 + i)
        s = int(rng.integers(smin, smax + 1))
        out.append(rough_wall_droplet(s, seed0 + i + 10_000_000, **kw))
    return out


def held_out_set(n_domains=1024, s=256, seed0=500000, **kw) -> List[DomainSpec]:
    """Held-out rough-wall droplets at a fixed side (no resampling needed)."""
    return [rough_wall_droplet(s, seed0 + j, **kw) for j in range(n_domains)]


def saturate_core(phi0: np.ndarray, phi1: np.ndarray, eps: float):
    """phi0 rounded up to exactly 1 where 1 - phi0 < eps (a solid core as FP32
    storage rounds it), and phi1 = (1 - phi0) x front recomputed with the same
    front; works for 2D and 3D arrays."""
    front = phi1 / np.maximum(1.0 - phi0, 1e-300)
    p0 = np.where(1.0 - phi0 < eps, 1.0, phi0)
    return p0, (1.0 - p0) * front


def with_params(spec: DomainSpec, **changes) -> DomainSpec:
    return dataclasses.replace(spec, **changes)


def default_workload(name: str, small: Optional[bool] = False) -> DomainSpec:
    """Named workloads used by the benchmark and the tests."""
    if name == "flat_wall_droplet":
        return flat_wall_droplet()
    if name == "porous_displacement":
        return porous_medium() if not small else porous_medium(nx=512, ny=256, seed=3, inlet=64)
    if name == "cylinder_droplet":
        return cylinder_droplet()
    raise KeyError(name)
