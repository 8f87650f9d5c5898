"""Seeded synthetic inputs of the 3f model (three fluids, phi0 and phi1 both
evolving): initial phase fields and raw parameters.  No step arithmetic of
the method lives here; the GPU library and the CPU oracle take their inputs
from this module.  Arrays are float64 [ny, nx], x fastest; node (i, j) sits
at (x, y) = (i, j).
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class DomainSpec3F:
    nx: int
    ny: int
    phi0: np.ndarray
    phi1: np.ndarray
    periodic_x: int = 1
    periodic_y: int = 0
    d0: float = 0.5
    D: float = 4.0
    sigma01: float = 0.01
    sigma02: float = 0.01
    sigma12: float = 0.01
    rho: tuple = (1.0, 1.0, 1.0)
    mu: tuple = (0.15, 0.15, 0.15)
    M_cst: float = 0.0
    M_deg: float = 0.01
    tau_phi: float = 0.8
    s_phi: tuple = (1.0, 1.0, 1.0, 1.0)
    s_g: tuple = (1.0, 1.0, 1.0, 1.0)
    Fb: tuple = (0.0, 0.0)
    rho_gauge: float = 0.0
    name: str = ""


def drop_on_interface(nx=128, ny=96, R0=16.0, D=4.0, cx=None, cy=None, **kw) -> DomainSpec3F:
    """A drop of phase 0 (radius R0) on the flat interface y = cy between a
    layer of phase 1 below and phase 2 above (the set-up of Sec. 4.1)."""
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    cx = nx / 2 - 0.5 if cx is None else cx
    cy = ny / 2 - 0.5 if cy is None else cy
    phi0 = 0.5 + 0.5 * np.tanh((R0 - np.hypot(x - cx, y - cy)) / (D / 2))
    phi1 = (1 - phi0) * (0.5 - 0.5 * np.tanh(2 * (y - cy) / D))
    return DomainSpec3F(nx=nx, ny=ny, phi0=phi0, phi1=phi1, D=D, name="drop_on_interface", **kw)


def drops_in_layers(n=1024, n_drops=48, rmin=12.0, rmax=40.0, D=4.0, seed=11, **kw) -> DomainSpec3F:
    """Random non-overlapping drops of phase 0 (radius U[rmin, rmax], numpy
    PCG64) in a periodic box of horizontal layers of phases 1 and 2 (four
    layers): a large 3f throughput workload."""
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    phi0 = np.zeros((n, n))
    centres = []
    tries = 0
    while len(centres) < n_drops and tries < 100000:
        tries += 1
        r = rng.uniform(rmin, rmax)
        c = rng.uniform(0, n, size=2)
        ok = True
        for (px, py, pr) in centres:
            dx = min(abs(c[0] - px), n - abs(c[0] - px))
            dy = min(abs(c[1] - py), n - abs(c[1] - py))
            if np.hypot(dx, dy) < r + pr + 2 * D:
                ok = False
                break
        if ok:
            centres.append((c[0], c[1], r))
    for (px, py, r) in centres:
        # the drop's bounding box with a margin of 3 D, wrapped periodically
        m = r + 3 * D
        ix = np.arange(int(np.floor(px - m)), int(np.ceil(px + m)) + 1)
        iy = np.arange(int(np.floor(py - m)), int(np.ceil(py + m)) + 1)
        Y, X = np.meshgrid(iy, ix, indexing="ij")
        val = 0.5 + 0.5 * np.tanh((r - np.hypot(X - px, Y - py)) / (D / 2))
        sub = np.ix_(iy % n, ix % n)
        phi0[sub] = np.maximum(phi0[sub], val)
    layers = 0.5 + 0.5 * np.tanh((n / 8 - np.abs(((y + n / 8) % (n / 2)) - n / 4)) * 2 / D)
    phi1 = (1 - phi0) * layers
    return DomainSpec3F(nx=n, ny=n, phi0=phi0, phi1=phi1, periodic_x=1, periodic_y=1, D=D,
                        name="drops_in_layers_%d" % n, **kw)


def with_params3f(spec: DomainSpec3F, **changes) -> DomainSpec3F:
    return dataclasses.replace(spec, **changes)
