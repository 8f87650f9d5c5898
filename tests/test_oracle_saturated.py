"""Pins of reading R11 / R11': the s2a term of the pressure constant H at a
saturated solid node.

The NS rate s2a follows from the effective viscosity mu/(1 - phi0) (Sec. 3)
and is zero where phi0 = 1; the 2D and 3D constants H then hold a term
(2 - 4 d0)/s2a or K (3 - 7 d0)/s2a with no finite value (d0 != 1/2).  The
oracle takes the term as zero there: the node's second-order NS moments do
not relax, so the equilibrium pressure does not enter them.

The pins: a solid whose core is rounded to phi0 = 1 exactly (as FP32
storage rounds it, 1 - phi0 < 2^-25) at d0 = 0.4 and density ratio 10 stays
finite, and the flow in the fluid differs from that around the same solid
left unsaturated by no more than the change eps made to phi0 itself.  Taking
the term as infinite (the formula as printed) makes every field NaN within a
step; any other finite choice that disturbed the fluid would show up as a
difference above eps.
"""
import numpy as np

from paper_2311_05091_amd import geometry as G
from paper_2311_05091_amd import geometry3d as G3
from tests._util import oracle_params

EPS = 1e-4
RATIO10 = dict(rho=(1.0, 1.0, 0.1), mu=(0.15, 0.15, 0.015))


def _check(unsat, sat, p0):
    fluid = p0 < 0.5
    for k, (a, b) in enumerate(zip(sat, unsat)):
        assert np.isfinite(a).all(), k
        assert np.abs(a - b)[fluid].max() <= EPS, (k, np.abs(a - b)[fluid].max())


def test_saturated_core_2d(orc):
    sp = G.with_params(G.solid_disk_box(n=48, Rs=14.0, R0=8.0, D=4.0, **RATIO10), d0=0.4)
    p0, p1 = G.saturate_core(sp.phi0, sp.phi1, EPS)
    assert (p0 == 1.0).sum() >= 20
    p = oracle_params(orc, sp)
    out = []
    for a, b in ((sp.phi0, sp.phi1), (p0, p1)):
        s = orc.Sim(p, a, b)
        s.step(400)
        out.append(s.moments())
    _check(out[0], out[1], p0)


def test_saturated_core_3d(orc):
    sp = G3.sphere_box(nx=40, ny=32, nz=32, Rs=9.0, R0=6.0, D=3.0, **RATIO10)
    p0, p1 = G.saturate_core(sp.phi0, sp.phi1, EPS)
    assert (p0 == 1.0).sum() >= 20
    p = orc.make_params3(sp.nx, sp.ny, sp.nz, periodic=sp.periodic, d0=sp.d0, D=sp.D, sigma12=sp.sigma12,
                         theta_deg=sp.theta_deg, rho=sp.rho, mu=sp.mu, M_deg=sp.M_deg, tau_phi=sp.tau_phi,
                         s_phi=sp.s_phi, s_g=sp.s_g)
    out = []
    for a, b in ((sp.phi0, sp.phi1), (p0, p1)):
        s = orc.Sim3(p, a, b)
        s.step(200)
        out.append(s.moments())
    _check(out[0], out[1], p0)
