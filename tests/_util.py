"""Shared test helpers: run one DomainSpec on the oracle and on the HIP library."""
import numpy as np


def oracle_params(orc, sp, **kw):
    d = dict(periodic_x=sp.periodic_x, periodic_y=sp.periodic_y, d0=sp.d0, D=sp.D,
             sigma12=sp.sigma12, theta_deg=sp.theta_deg, kappa=sp.kappa, rho=sp.rho, mu=sp.mu,
             M_cst=sp.M_cst, M_deg=sp.M_deg, tau_phi=sp.tau_phi, s_phi=sp.s_phi, s_g=sp.s_g,
             Fb=sp.Fb, u_wall=sp.u_wall, omega_wall=sp.omega_wall,
             wall_center=sp.wall_center, rho_gauge=sp.rho_gauge, open_x=sp.open_x, inlet_type=sp.inlet_type,
             p_in=sp.p_in, u_in=sp.u_in, p_out=sp.p_out, phi1_in=sp.phi1_in)
    d.update(kw)
    return orc.make_params(sp.nx, sp.ny, **d)


def oracle_run(orc, sp, steps):
    s = orc.Sim(oracle_params(orc, sp), sp.phi0, sp.phi1)
    s.step(steps)
    return s


def gpu_context(specs, precision=64, tile=None):
    from paper_2311_05091_amd.lbm import Context
    ctx = Context(precision=precision)
    for sp in specs:
        ctx.add_domain(sp)
    ctx.finalize()
    if tile:
        ctx.set_tile(tile)
    return ctx


def rel_l2(a, b):
    nb = np.linalg.norm(np.ravel(b))
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / (nb if nb > 0 else 1.0)


def header_functions(path):
    """Names of the functions declared in a C header (int/void/const char* returns)."""
    import re
    src = open(path).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(\w+)\s*\(", src, flags=re.M)))
