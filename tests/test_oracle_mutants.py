"""The oracle's pins catch plausible mistakes in the terms they pin.

Each case plants one mistake in a copy of oracle/tpf_oracle.c or
oracle/tpf_oracle3d.c (a text
substitution: a dropped term, a flipped sign, a wrong factor), compiles it with
gcc into a temporary library and runs the pin that must catch it, in a
subprocess that loads the mutant (TPF_ORACLE_LIB).  The pin must fail.  A
control case runs the same harness on the unchanged source, whose pins must
pass.  Everything here runs on the CPU; the GPU library is not involved.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "tpf_oracle.c")
SRC3 = os.path.join(ROOT, "oracle", "tpf_oracle3d.c")
SRC3F = os.path.join(ROOT, "oracle", "tpf_oracle3f.c")
NORMAL = "tests/test_oracle_consistency.py::test_translating_interface_density_ratio_10"
TANGENT = "tests/test_oracle_consistency.py::test_tangential_flow_along_relaxing_interface"
CHANNEL = "tests/test_oracle_solid.py::test_diffuse_channel_momentum_balance"
SLIDE = "tests/test_oracle_solid.py::test_sliding_solid_adds_its_velocity"
SPIN = "tests/test_oracle_solid.py::test_spinning_cavity_rigid_rotation"
NORMAL3 = "tests/test_oracle3d.py::test_translating_interface_3d_density_ratio_10"
TANGENT3 = "tests/test_oracle3d.py::test_tangential_flow_along_relaxing_interface_3d"
LAPLACE3 = "tests/test_oracle3d.py::test_laplace_law_sphere"
POIS_OPEN = "tests/test_oracle_open.py::test_pressure_driven_channel_is_poiseuille"
VEL_OPEN = "tests/test_oracle_open.py::test_velocity_inlet_conserves_flux"
LAYERS = "tests/test_oracle_open.py::test_stratified_two_phase_flow_rates_and_kp"
RELABEL3F = "tests/test_oracle_3f.py::test_3f_exchanging_phases_0_and_1"
LAPLACE3F = "tests/test_oracle_3f.py::test_3f_laplace_law_for_phase_0_in_phase_2"
LENS3F = "tests/test_oracle_3f.py::test_3f_lens_corner_angles_follow_neumann_triangle"

# name, original text (must occur exactly once), replacement, pin that must fail
MUTANTS = [
    ("pressure_no_u_grad_rho", "(sum + (0.5 + H) * u_grad_rho", "(sum + 0.0 * u_grad_rho", NORMAL),
    ("pressure_H_sign", "(sum + (0.5 + H) * u_grad_rho", "(sum + (0.5 - H) * u_grad_rho", NORMAL),
    ("pressure_omega0_sign", "- w[0] * B / (1.0 - cs2)", "+ w[0] * B / (1.0 - cs2)", NORMAL),
    ("M2F_no_density_gradient", "+ 2.0 * cs2 * ux * drx + (1.0 - 3.0 * cs2) * Q;", "+ (1.0 - 3.0 * cs2) * Q;",
     NORMAL),
    ("M2F_no_isotropic_Q", "+ 2.0 * cs2 * ux * drx + (1.0 - 3.0 * cs2) * Q;", "+ 2.0 * cs2 * ux * drx;", NORMAL),
    ("Fpop_no_Q", "F[i] = w[i] * (Q + (CX[i]", "F[i] = w[i] * (0.0 * Q + (CX[i]", NORMAL),
    ("Fc_sign", "double Fcx = -0.5 * dpsiy, Fcy = 0.5 * dpsix;", "double Fcx = 0.5 * dpsiy, Fcy = -0.5 * dpsix;",
     TANGENT),
    ("Fc_dropped", "double Fcx = -0.5 * dpsiy, Fcy = 0.5 * dpsix;", "double Fcx = 0.0 * dpsiy, Fcy = 0.0 * dpsix;",
     TANGENT),
    ("geq_no_S_in_shear_flux", "double Pixy = rho * ux * uy - 0.5 * (Sx * uy + ux * Sy);",
     "double Pixy = rho * ux * uy;", TANGENT),
    ("S_sign", "double Sx = (rho1 - rho2) * Mob / d->gamma[1] * gmx;",
     "double Sx = -(rho1 - rho2) * Mob / d->gamma[1] * gmx;", TANGENT),
    ("penalty_full_correction", "double ux = usx + 0.5 * phi0 * fsx", "double ux = usx + 1.0 * phi0 * fsx", CHANNEL),
    ("penalty_force_doubled", "double Gx = Fx + phi0 * rho * fsx", "double Gx = Fx + 2.0 * phi0 * rho * fsx",
     CHANNEL),
    ("viscosity_without_solid_factor", "return (1.0 - phi0) / (mu_v / (rho * cfac) + 0.5 * (1.0 - phi0));",
     "return 1.0 / (mu_v / (rho * cfac) + 0.5);", CHANNEL),
    ("wall_velocity_sign", "double uwx = P->u_wall[0] - P->omega_wall", "double uwx = -P->u_wall[0] - P->omega_wall",
     SLIDE),
    ("wall_velocity_half", "double fsx = uwx - usx", "double fsx = 0.5 * uwx - usx", SLIDE),
    ("rotation_sign", "double uwy = P->u_wall[1] + P->omega_wall", "double uwy = P->u_wall[1] - P->omega_wall", SPIN),
    ("open_g_equilibrium_only", "s->gpost[(size_t)i * n + ib] = geb[i] + s->gpost[(size_t)i * n + in] - gen[i];",
     "s->gpost[(size_t)i * n + ib] = geb[i];", POIS_OPEN),
    ("open_inlet_pressure_from_neighbour", "if (P->inlet_type == 0) { pb = P->p_in;",
     "if (P->inlet_type == 0) { pb = pn;", POIS_OPEN),
    ("open_inlet_velocity_from_neighbour", "else { pb = pn; uxb = P->u_in; uyb = 0.0; }",
     "else { pb = pn; uxb = uxn; uyb = uyn; }", VEL_OPEN),
    ("flow_rate_phase1_unweighted", "b += p1 * ux;", "b += ux;", LAYERS),
]

# mistakes planted in the three-dimensional oracle
_FC3 = ("F[0] += -0.5 * (dpz[1] - dpy[2]);\n                F[1] += -0.5 * (dpx[2] - dpz[0]);\n"
        "                F[2] += -0.5 * (dpy[0] - dpx[1]);")
MUTANTS3 = [
    ("3d_Fc_sign", _FC3, _FC3.replace("-0.5", "0.5"), TANGENT3),
    ("3d_geq_no_S_in_shear_flux", "Pi[5] = rho * u[0] * u[2] - 0.5 * (S[0] * u[2] + u[0] * S[2]);",
     "Pi[5] = rho * u[0] * u[2];", TANGENT3),
    ("3d_S_sign", "S[k] = (rho1 - rho2) * Mob / s->gamma[1] * gm[k];",
     "S[k] = -(rho1 - rho2) * Mob / s->gamma[1] * gm[k];", TANGENT3),
    ("3d_pressure_K_of_2d", "double K = 1.0 - 2.0 * d0;", "double K = 1.0 - d0;", NORMAL3),
    ("3d_pressure_H_of_2d", "double cH = K * (3.0 - 7.0 * d0);", "double cH = K * (2.0 - 4.0 * d0);", NORMAL3),
    ("3d_stencil_weights", "orc3_weights(1.0 / 3.0, s->ws);", "orc3_weights(0.5, s->ws);", LAPLACE3),
]


def _run_pin(tmp_path, name, src_text, pin, src3_text=None, src3f_text=None):
    c = tmp_path / (name + ".c")
    c3 = tmp_path / (name + "_3d.c")
    c3f = tmp_path / (name + "_3f.c")
    so = tmp_path / (name + ".so")
    c.write_text(src_text)
    c3.write_text(src3_text if src3_text is not None else open(SRC3).read())
    c3f.write_text(src3f_text if src3f_text is not None else open(SRC3F).read())
    subprocess.check_call(["gcc", "-std=gnu11", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", str(so), str(c),
                           str(c3), str(c3f), "-lm"])
    env = dict(os.environ, TPF_ORACLE_LIB=str(so), OMP_NUM_THREADS=str(_THREADS))
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", pin],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)


# The planted mistakes are independent: all of them are compiled and their
# pins run once per module, _WORKERS at a time with _THREADS OpenMP threads
# each; every test item then checks its own result.
_WORKERS, _THREADS = 4, 2


def _cases():
    src, src3, src3f = open(SRC).read(), open(SRC3).read(), open(SRC3F).read()
    out = {"control": (src, NORMAL, None, None)}
    for name, orig, repl, pin in MUTANTS:
        out[name] = (src.replace(orig, repl), pin, None, None)
    for name, orig, repl, pin in MUTANTS3:
        out[name] = (src, pin, src3.replace(orig, repl), None)
    for name, orig, repl, pin in MUTANTS3F:
        out[name] = (src, pin, None, src3f.replace(orig, repl))
    return out


@pytest.fixture(scope="module")
def pin_results(tmp_path_factory):
    from concurrent.futures import ThreadPoolExecutor
    d = tmp_path_factory.mktemp("mutants")
    cases = _cases()
    with ThreadPoolExecutor(max_workers=_WORKERS) as ex:
        futs = {name: ex.submit(_run_pin, d, name, c[0], c[1], c[2], c[3]) for name, c in cases.items()}
        return {name: f.result() for name, f in futs.items()}


def test_unchanged_oracle_passes_through_the_harness(pin_results):
    r = pin_results["control"]
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("name,orig,repl,pin", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_fails_its_pin(pin_results, name, orig, repl, pin):
    assert open(SRC).read().count(orig) == 1, "mutation site changed: " + orig
    r = pin_results[name]
    assert r.returncode == 1 and " failed" in r.stdout, (name, r.stdout[-1500:])


@pytest.mark.parametrize("name,orig,repl,pin", MUTANTS3, ids=[m[0] for m in MUTANTS3])
def test_mutant_3d_fails_its_pin(pin_results, name, orig, repl, pin):
    assert open(SRC3).read().count(orig) == 1, "mutation site changed: " + orig
    r = pin_results[name]
    assert r.returncode == 1 and " failed" in r.stdout, (name, r.stdout[-1500:])


# mistakes planted in the 3f-model oracle
MUTANTS3F = [
    ("3f_S_phase1_only", "Mob * ((r0 - r2) * gm0x / s->gamma[0] + (r1 - r2) * gm1x / s->gamma[1])",
     "Mob * ((r1 - r2) * gm1x / s->gamma[1])", RELABEL3F),
    ("3f_mobility_of_2f1s", "double fdeg = (1.0 - phi0) * (1.0 - phi1) * (1.0 - phi2);",
     "double fdeg = phi1 * (1.0 - phi1) * (1.0 - phi0);", RELABEL3F),
    ("3f_eta_of_phase1", "eta[p] = (P->M_cst + P->M_deg) / (gamma[p] *", "eta[p] = (P->M_cst + P->M_deg) / (gamma[1] *",
     RELABEL3F),
    ("3f_viscosity_with_solid_factor", "double s2a = orc_visc_rate(mu_v, rho, 0.0,", "double s2a = orc_visc_rate(mu_v, rho, phi0,",
     RELABEL3F),
    ("3f_gamma2_tensions_swapped", "gamma[2] = P->sigma02 + P->sigma12 - P->sigma01;",
     "gamma[2] = P->sigma01 + P->sigma12 - P->sigma02;", LAPLACE3F),
    ("3f_gamma0_tensions_swapped", "gamma[0] = P->sigma01 + P->sigma02 - P->sigma12;",
     "gamma[0] = P->sigma01 + P->sigma12 - P->sigma02;", LENS3F),
]


@pytest.mark.parametrize("name,orig,repl,pin", MUTANTS3F, ids=[m[0] for m in MUTANTS3F])
def test_mutant_3f_fails_its_pin(pin_results, name, orig, repl, pin):
    assert open(SRC3F).read().count(orig) == 1, "mutation site changed: " + orig
    r = pin_results[name]
    assert r.returncode == 1 and " failed" in r.stdout, (name, r.stdout[-1500:])
