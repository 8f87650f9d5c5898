"""Seeded synthetic inputs of the 3D (D3Q15) workloads: solid fields, initial
phase fields and raw parameters.  No step arithmetic of the method lives here;
both the GPU library and the CPU oracle take their inputs from this module.

Arrays are float64 of shape [nz, ny, nx], x fastest; node (i, j, k) sits at
(x, y, z) = (i, j, k).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class DomainSpec3:
    nx: int
    ny: int
    nz: int
    phi0: np.ndarray
    phi1: np.ndarray
    periodic: tuple = (1, 1, 0)
    d0: float = 0.4
    D: float = 4.0
    sigma12: float = 0.01
    theta_deg: float = 60.0
    kappa: float = 0.0
    rho: tuple = (1.0, 1.0, 1.0)
    mu: tuple = (0.15, 0.15, 0.15)
    M_cst: float = 0.0
    M_deg: float = 0.004
    tau_phi: float = 0.8
    s_phi: tuple = (1.0, 1.0, 1.0, 1.0)
    s_g: tuple = (1.0, 1.0, 0.5, 0.5)
    Fb: tuple = (0.0, 0.0, 0.0)
    u_wall: tuple = (0.0, 0.0, 0.0)
    rho_gauge: float = 0.0
    name: str = ""


def _grid(nx, ny, nz):
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx].astype(np.float64)
    return x, y, z


def sphere_box(nx=24, ny=20, nz=22, Rs=4.0, R0=5.0, periodic=(1, 1, 0), D=4.0, **kw) -> DomainSpec3:
    """A diffuse solid sphere of radius Rs and a droplet of fluid 1 of radius R0
    touching it, in fluid 2."""
    x, y, z = _grid(nx, ny, nz)
    cs = (nx * 0.3, ny * 0.5, nz * 0.5)
    rs = np.sqrt((x - cs[0]) ** 2 + (y - cs[1]) ** 2 + (z - cs[2]) ** 2)
    phi0 = 0.5 - 0.5 * np.tanh(2 * (rs - Rs) / D)
    cd = (cs[0] + Rs + R0 * 0.8, cs[1], cs[2])
    rd = np.sqrt((x - cd[0]) ** 2 + (y - cd[1]) ** 2 + (z - cd[2]) ** 2)
    phi1 = (1 - phi0) * (0.5 + 0.5 * np.tanh(2 * (R0 - rd) / D))
    return DomainSpec3(nx=nx, ny=ny, nz=nz, phi0=phi0, phi1=phi1, periodic=periodic, D=D, name="sphere_box", **kw)


def porous_spheres(n=128, porosity=0.7, rmin=6.0, rmax=14.0, seed=5, D=3.0, inlet=16, **kw) -> DomainSpec3:
    """Random sequential addition of non-overlapping solid spheres (radius
    U[rmin, rmax], centre gap >= ra + rb + 2, periodic in x and y, >= 3 cells
    from the z walls) until the spheres fill 1 - porosity of the box or 200000
    placements have been tried (at n = 256 the packing jams first, at a solid
    share of 0.235);
    an obstacle-free slab x < inlet starts filled with wetting fluid 1.  A 3D
    stand-in for the paper's porous medium (Sec. 4.6), whose CT sample is not
    available: only its role as a large 3D throughput workload."""
    rng = np.random.default_rng(seed)
    nx = ny = nz = n
    x, y, z = _grid(nx, ny, nz)
    centres = []
    target = (1 - porosity) * nx * ny * nz
    vol = 0.0
    tries = 0
    while vol < target and tries < 200000:
        tries += 1
        r = rng.uniform(rmin, rmax)
        c = (rng.uniform(inlet + r, nx), rng.uniform(0, ny), rng.uniform(r + 3, nz - r - 3))
        ok = True
        for (cx, cy, cz, cr) in centres:
            dx = min(abs(c[0] - cx), nx - abs(c[0] - cx))
            dy = min(abs(c[1] - cy), ny - abs(c[1] - cy))
            if math.sqrt(dx * dx + dy * dy + (c[2] - cz) ** 2) < r + cr + 2:
                ok = False
                break
        if ok:
            centres.append((c[0], c[1], c[2], r))
            vol += 4.0 / 3.0 * math.pi * r ** 3
    phi0 = np.zeros((nz, ny, nx))
    for (cx, cy, cz, r) in centres:
        # the sphere's bounding box (periodic in x and y) with a margin of 2 D
        m = r + 2 * D
        ix = np.arange(int(math.floor(cx - m)), int(math.ceil(cx + m)) + 1)
        iy = np.arange(int(math.floor(cy - m)), int(math.ceil(cy + m)) + 1)
        iz = np.arange(max(0, int(math.floor(cz - m))), min(nz, int(math.ceil(cz + m)) + 1))
        Z, Y, X = np.meshgrid(iz, iy, ix, indexing="ij")
        d = np.sqrt((X - cx) ** 2 + (Y - cy) ** 2 + (Z - cz) ** 2)
        val = 0.5 - 0.5 * np.tanh(2 * (d - r) / D)
        sub = np.ix_(iz, iy % ny, ix % nx)
        phi0[sub] = np.maximum(phi0[sub], val)
    front = 0.5 - 0.5 * np.tanh(2 * (x - inlet) / D)
    phi1 = (1 - phi0) * front
    return DomainSpec3(nx=nx, ny=ny, nz=nz, phi0=phi0, phi1=phi1, periodic=(1, 1, 0), D=D, theta_deg=45.0,
                       mu=(0.15, 0.15, 0.03), Fb=(1e-6, 0.0, 0.0), name="porous_spheres_%d" % n, **kw)


def with_params3(spec: DomainSpec3, **changes) -> DomainSpec3:
    return dataclasses.replace(spec, **changes)
