"""Plain FP64 CPU oracle of the coupled ternary phase-field LB step.

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module; the product package
never does.  The arithmetic lives in ``tpf_oracle.c`` (plain C, OpenMP over
rows); this file only compiles it with gcc and marshals numpy arrays through
ctypes.  It shares no code with the GPU library.

Method: Zhan, Chai & Shi, arXiv 2311.05091 -- Sec. 2 (model), Sec. 3 (LB
schemes), Sec. 4 (Hermite-moment collision, boundary conditions, 2f1s
mobility) and Appendix A (D2Q9 matrices).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tpf_oracle.c")
_SRC3 = os.path.join(_HERE, "tpf_oracle3d.c")
_SRC3F = os.path.join(_HERE, "tpf_oracle3f.c")
_LIB_PATH = os.path.join(_HERE, "libtpf_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-std=gnu11", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, _SRC3, _SRC3F, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Params(C.Structure):
    """Domain parameters, field for field the oracle's own ``orc_params``."""
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("periodic_x", C.c_int32), ("periodic_y", C.c_int32),
        ("d0", C.c_double), ("D", C.c_double), ("sigma12", C.c_double),
        ("theta", C.c_double), ("kappa", C.c_double),
        ("rho", C.c_double * 3), ("mu", C.c_double * 3),
        ("M_cst", C.c_double), ("M_deg", C.c_double), ("tau_phi", C.c_double),
        ("s_phi", C.c_double * 4), ("s_g", C.c_double * 4),
        ("Fb", C.c_double * 2), ("u_wall", C.c_double * 2),
        ("omega_wall", C.c_double), ("wall_center", C.c_double * 2),
        ("rho_gauge", C.c_double),
        ("open_x", C.c_int32), ("inlet_type", C.c_int32),
        ("p_in", C.c_double), ("u_in", C.c_double), ("p_out", C.c_double), ("phi1_in", C.c_double),
    ]


class Derived(C.Structure):
    _fields_ = [
        ("k", C.c_double), ("sigma01", C.c_double), ("sigma02", C.c_double),
        ("gamma", C.c_double * 3), ("gammaT", C.c_double), ("eta", C.c_double),
        ("cs2", C.c_double), ("w", C.c_double * 9), ("Kp", C.c_double),
    ]


class Params3F(C.Structure):
    """Parameters of a 3f-model domain, field for field ``orc3f_params``."""
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("periodic_x", C.c_int32), ("periodic_y", C.c_int32),
        ("d0", C.c_double), ("D", C.c_double),
        ("sigma01", C.c_double), ("sigma02", C.c_double), ("sigma12", C.c_double),
        ("rho", C.c_double * 3), ("mu", C.c_double * 3),
        ("M_cst", C.c_double), ("M_deg", C.c_double), ("tau_phi", C.c_double),
        ("s_phi", C.c_double * 4), ("s_g", C.c_double * 4),
        ("Fb", C.c_double * 2), ("rho_gauge", C.c_double),
    ]


class Params3(C.Structure):
    """Parameters of a 3D domain, field for field the oracle's ``orc3_params``."""
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("periodic", C.c_int32 * 3),
        ("d0", C.c_double), ("D", C.c_double), ("sigma12", C.c_double),
        ("theta", C.c_double), ("kappa", C.c_double),
        ("rho", C.c_double * 3), ("mu", C.c_double * 3),
        ("M_cst", C.c_double), ("M_deg", C.c_double), ("tau_phi", C.c_double),
        ("s_phi", C.c_double * 4), ("s_g", C.c_double * 4),
        ("Fb", C.c_double * 3), ("u_wall", C.c_double * 3),
        ("rho_gauge", C.c_double),
    ]


_D = C.POINTER(C.c_double)


def _lib_handle():
    global _lib
    if _lib is None:
        path = os.environ.get("TPF_ORACLE_LIB", _LIB_PATH)
        if path == _LIB_PATH and not os.path.exists(_LIB_PATH):
            build(force=True)
        lib = C.CDLL(path)
        lib.orc_create.restype = C.c_void_p
        lib.orc_create.argtypes = [C.POINTER(Params), _D, _D]
        lib.orc_free.argtypes = [C.c_void_p]
        lib.orc_step.argtypes = [C.c_void_p, C.c_int64]
        lib.orc_moments.argtypes = [C.c_void_p, _D, _D, _D, _D]
        lib.orc_aux.argtypes = [C.c_void_p, _D, _D, _D]
        lib.orc_flow_rates.argtypes = [C.c_void_p, _D]
        lib.orc_mass.restype = C.c_double
        lib.orc_mass.argtypes = [C.c_void_p]
        lib.orc_step_count.restype = C.c_int64
        lib.orc_step_count.argtypes = [C.c_void_p]
        lib.orc_get_state.argtypes = [C.c_void_p, _D, _D, _D]
        lib.orc_set_state.argtypes = [C.c_void_p, _D, _D, _D]
        lib.orc_get_derived.argtypes = [C.c_void_p, C.POINTER(Derived)]
        lib.orc_derive.restype = C.c_int
        lib.orc_derive.argtypes = [C.POINTER(Params), C.POINTER(Derived)]
        lib.orc_spreading_factor.restype = C.c_double
        lib.orc_spreading_factor.argtypes = [C.c_double, C.c_double]
        lib.orc_weights.argtypes = [C.c_double, _D]
        lib.orc_velocities.argtypes = [C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        lib.orc_M0.argtypes = [_D]
        lib.orc_N.argtypes = [C.c_double, _D]
        lib.orc_inverse9.restype = C.c_int
        lib.orc_inverse9.argtypes = [_D, _D]
        lib.orc_relaxation_matrix.argtypes = [C.c_double, _D, _D]
        lib.orc_collide.argtypes = [C.c_double, _D, _D, _D, _D, _D]
        lib.orc_chemical_potentials.argtypes = [_D, C.c_double, C.c_double, C.c_double,
                                                C.c_double, C.c_double, _D, _D]
        lib.orc_feq.argtypes = [C.c_double] * 5 + [_D]
        lib.orc_Rpop.argtypes = [C.c_double] * 6 + [_D]
        lib.orc_geq.argtypes = [C.c_double] * 8 + [_D]
        lib.orc_Fpop.argtypes = [C.c_double] * 7 + [_D]
        lib.orc_pressure.restype = C.c_double
        lib.orc_pressure.argtypes = [C.c_double, C.c_double, C.c_double, _D,
                                     C.c_double, C.c_double, C.c_double]
        lib.orc_visc_rate.restype = C.c_double
        lib.orc_visc_rate.argtypes = [C.c_double] * 4
        lib.orc_num_threads.restype = C.c_int
        if hasattr(lib, "orc3f_create"):
            lib.orc3f_create.restype = C.c_void_p
            lib.orc3f_create.argtypes = [C.POINTER(Params3F), _D, _D]
            lib.orc3f_free.argtypes = [C.c_void_p]
            lib.orc3f_step.argtypes = [C.c_void_p, C.c_int64]
            lib.orc3f_moments.argtypes = [C.c_void_p, _D, _D, _D, _D, _D]
            lib.orc3f_mass.argtypes = [C.c_void_p, _D]
            lib.orc3f_get_state.argtypes = [C.c_void_p, _D, _D, _D, _D]
            lib.orc3f_step_count.restype = C.c_int64
            lib.orc3f_step_count.argtypes = [C.c_void_p]
            lib.orc3f_derive.restype = C.c_int
            lib.orc3f_derive.argtypes = [C.POINTER(Params3F), _D, _D, _D]
        if hasattr(lib, "orc3_create"):
            lib.orc3_create.restype = C.c_void_p
            lib.orc3_create.argtypes = [C.POINTER(Params3), _D, _D]
            lib.orc3_free.argtypes = [C.c_void_p]
            lib.orc3_step.argtypes = [C.c_void_p, C.c_int64]
            lib.orc3_moments.argtypes = [C.c_void_p, _D, _D, _D, _D, _D]
            lib.orc3_aux.argtypes = [C.c_void_p, _D, _D]
            lib.orc3_mass.restype = C.c_double
            lib.orc3_mass.argtypes = [C.c_void_p]
            lib.orc3_step_count.restype = C.c_int64
            lib.orc3_step_count.argtypes = [C.c_void_p]
            lib.orc3_get_state.argtypes = [C.c_void_p, _D, _D, _D]
            lib.orc3_set_state.argtypes = [C.c_void_p, _D, _D, _D]
            lib.orc3_derived.argtypes = [C.c_void_p, _D, _D, _D]
            lib.orc3_weights.argtypes = [C.c_double, _D]
            lib.orc3_velocities.argtypes = [C.POINTER(C.c_int32)]
            lib.orc3_M0.argtypes = [_D]
            lib.orc3_N.argtypes = [C.c_double, _D]
            lib.orc3_inverse.restype = C.c_int
            lib.orc3_inverse.argtypes = [C.c_int, _D, _D]
            lib.orc3_relaxation_matrix.argtypes = [C.c_double, _D, _D]
            lib.orc3_collide.argtypes = [C.c_double, _D, _D, _D, _D, _D]
            lib.orc3_feq.argtypes = [C.c_double, C.c_double, C.c_double, _D, _D]
            lib.orc3_Rpop.argtypes = [C.c_double, _D, C.c_double, _D, _D]
            lib.orc3_geq.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, _D, _D, _D]
            lib.orc3_Fpop.argtypes = [C.c_double, C.c_double, _D, _D, _D]
            lib.orc3_pressure.restype = C.c_double
            lib.orc3_pressure.argtypes = [C.c_double, C.c_double, C.c_double, _D, C.c_double, C.c_double,
                                          C.c_double]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def _arr(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if n is not None:
        assert a.size == n
    return a


# ---------------------------------------------------------------------------
# Parameters
# ---------------------------------------------------------------------------
def make_params(nx, ny, *, periodic_x=1, periodic_y=0, d0=0.5, D=4.0, sigma12=0.01,
                theta_deg=60.0, kappa=0.0, rho=(1.0, 1.0, 1.0), mu=(0.15, 0.15, 0.15),
                M_cst=0.0, M_deg=0.1, tau_phi=0.8, s_phi=(1.0, 1.0, 1.0, 1.0),
                s_g=(1.0, 1.0, 1.0, 1.0), Fb=(0.0, 0.0), u_wall=(0.0, 0.0),
                omega_wall=0.0, wall_center=(0.0, 0.0), rho_gauge=0.0, open_x=0, inlet_type=0,
                p_in=0.0, u_in=0.0, p_out=0.0, phi1_in=0.0) -> Params:
    p = Params()
    p.nx, p.ny, p.periodic_x, p.periodic_y = nx, ny, periodic_x, periodic_y
    p.d0, p.D, p.sigma12 = d0, D, sigma12
    p.theta, p.kappa = math.radians(theta_deg), kappa
    p.rho[:] = list(rho)
    p.mu[:] = list(mu)
    p.M_cst, p.M_deg, p.tau_phi = M_cst, M_deg, tau_phi
    p.s_phi[:] = list(s_phi)
    p.s_g[:] = list(s_g)
    p.Fb[:] = list(Fb)
    p.u_wall[:] = list(u_wall)
    p.omega_wall = omega_wall
    p.wall_center[:] = list(wall_center)
    p.rho_gauge = rho_gauge
    p.open_x, p.inlet_type = open_x, inlet_type
    p.p_in, p.u_in, p.p_out, p.phi1_in = p_in, u_in, p_out, phi1_in
    return p


def derive(p: Params) -> dict:
    d = Derived()
    rc = _lib_handle().orc_derive(C.byref(p), C.byref(d))
    return {"ok": rc == 0, "k": d.k, "sigma01": d.sigma01, "sigma02": d.sigma02,
            "gamma": list(d.gamma), "gammaT": d.gammaT, "eta": d.eta, "cs2": d.cs2,
            "w": list(d.w), "Kp": d.Kp}


def spreading_factor(theta_rad: float, kappa: float) -> float:
    return _lib_handle().orc_spreading_factor(theta_rad, kappa)


# ---------------------------------------------------------------------------
# Lattice algebra and pointwise physics
# ---------------------------------------------------------------------------
def weights(d0: float) -> np.ndarray:
    w = np.zeros(9)
    _lib_handle().orc_weights(d0, _ptr(w))
    return w


def velocities():
    cx = (C.c_int32 * 9)()
    cy = (C.c_int32 * 9)()
    _lib_handle().orc_velocities(cx, cy)
    return np.array(cx[:]), np.array(cy[:])


def M0() -> np.ndarray:
    m = np.zeros(81)
    _lib_handle().orc_M0(_ptr(m))
    return m.reshape(9, 9)


def N(cs2: float) -> np.ndarray:
    m = np.zeros(81)
    _lib_handle().orc_N(cs2, _ptr(m))
    return m.reshape(9, 9)


def inverse9(a) -> np.ndarray:
    a = _arr(a).reshape(81).copy()
    out = np.zeros(81)
    rc = _lib_handle().orc_inverse9(_ptr(a), _ptr(out))
    assert rc == 0
    return out.reshape(9, 9)


def relaxation_matrix(cs2: float, Kdiag) -> np.ndarray:
    k = _arr(Kdiag, 9)
    out = np.zeros(81)
    _lib_handle().orc_relaxation_matrix(cs2, _ptr(k), _ptr(out))
    return out.reshape(9, 9)


def collide(cs2, Kdiag, f, feq, R) -> np.ndarray:
    out = np.zeros(9)
    _lib_handle().orc_collide(cs2, _ptr(_arr(Kdiag, 9)), _ptr(_arr(f, 9)), _ptr(_arr(feq, 9)),
                              _ptr(_arr(R, 9)), _ptr(out))
    return out


def chemical_potentials(gamma, D, phi0, phi1, lap0, lap1):
    g = _arr(gamma, 3)
    mu = np.zeros(3)
    mub = np.zeros(3)
    _lib_handle().orc_chemical_potentials(_ptr(g), D, phi0, phi1, lap0, lap1, _ptr(mu), _ptr(mub))
    return mu, mub


def feq(d0, phi, eta_mub, Ax, Ay):
    out = np.zeros(9)
    _lib_handle().orc_feq(d0, phi, eta_mub, Ax, Ay, _ptr(out))
    return out


def Rpop(d0, dAx, dAy, a, eta_gx, eta_gy):
    out = np.zeros(9)
    _lib_handle().orc_Rpop(d0, dAx, dAy, a, eta_gx, eta_gy, _ptr(out))
    return out


def geq(d0, rho_gauge, P, rho, ux, uy, Sx, Sy):
    out = np.zeros(9)
    _lib_handle().orc_geq(d0, rho_gauge, P, rho, ux, uy, Sx, Sy, _ptr(out))
    return out


def Fpop(d0, Q, Gx, Gy, Mxx, Myy, Mxy):
    out = np.zeros(9)
    _lib_handle().orc_Fpop(d0, Q, Gx, Gy, Mxx, Myy, Mxy, _ptr(out))
    return out


def pressure(d0, s0, s2a, g, u_grad_rho, B, B_prev):
    return _lib_handle().orc_pressure(d0, s0, s2a, _ptr(_arr(g, 9)), u_grad_rho, B, B_prev)


def visc_rate(mu_v, rho, phi0, cfac):
    return _lib_handle().orc_visc_rate(mu_v, rho, phi0, cfac)


def num_threads() -> int:
    return _lib_handle().orc_num_threads()


# ---------------------------------------------------------------------------
# Simulation
# ---------------------------------------------------------------------------
class Sim:
    """One domain advanced by the oracle.  Arrays are [ny, nx], x fastest."""

    def __init__(self, params: Params, phi0, phi1):
        self.params = params
        self.nx, self.ny = params.nx, params.ny
        n = self.nx * self.ny
        self._phi0 = _arr(phi0, n)
        self._phi1 = _arr(phi1, n)
        self._h = _lib_handle().orc_create(C.byref(params), _ptr(self._phi0), _ptr(self._phi1))
        if not self._h:
            raise ValueError("oracle rejected the parameters")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _lib_handle().orc_free(h)
            self._h = None

    def step(self, nsteps: int = 1):
        _lib_handle().orc_step(self._h, int(nsteps))

    @property
    def steps(self) -> int:
        return _lib_handle().orc_step_count(self._h)

    def moments(self):
        shape = (self.ny, self.nx)
        phi1, ux, uy, p = (np.zeros(shape) for _ in range(4))
        _lib_handle().orc_moments(self._h, _ptr(phi1), _ptr(ux), _ptr(uy), _ptr(p))
        return phi1, ux, uy, p

    def aux(self):
        shape = (self.ny, self.nx)
        mub, gmx, gmy = (np.zeros(shape) for _ in range(3))
        _lib_handle().orc_aux(self._h, _ptr(mub), _ptr(gmx), _ptr(gmy))
        return mub, gmx, gmy

    def mass(self) -> float:
        return _lib_handle().orc_mass(self._h)

    def flow_rates(self):
        """Sums over phi0 <= 1/2 of u_x, phi1 u_x, phi2 u_x (current level)."""
        q = np.zeros(3)
        _lib_handle().orc_flow_rates(self._h, _ptr(q))
        return q

    def get_state(self):
        n = self.nx * self.ny
        f = np.zeros((9, self.ny, self.nx))
        g = np.zeros((9, self.ny, self.nx))
        lag = np.zeros((7, self.ny, self.nx))
        _lib_handle().orc_get_state(self._h, _ptr(f), _ptr(g), _ptr(lag))
        assert f.size == 9 * n
        return f, g, lag

    def set_state(self, f=None, g=None, lag=None):
        n = self.nx * self.ny
        null = C.cast(None, _D)
        fa = _arr(f, 9 * n) if f is not None else None
        ga = _arr(g, 9 * n) if g is not None else None
        la = _arr(lag, 7 * n) if lag is not None else None
        _lib_handle().orc_set_state(self._h,
                                    _ptr(fa) if fa is not None else null,
                                    _ptr(ga) if ga is not None else null,
                                    _ptr(la) if la is not None else null)

    def derived(self) -> dict:
        d = Derived()
        _lib_handle().orc_get_derived(self._h, C.byref(d))
        return {"k": d.k, "gamma": list(d.gamma), "gammaT": d.gammaT, "eta": d.eta,
                "cs2": d.cs2, "w": list(d.w), "Kp": d.Kp}


# ---------------------------------------------------------------------------
# Three-dimensional (D3Q15) oracle
# ---------------------------------------------------------------------------
def make_params3(nx, ny, nz, *, periodic=(1, 1, 0), d0=0.5, D=4.0, sigma12=0.01, theta_deg=60.0,
                 kappa=0.0, rho=(1.0, 1.0, 1.0), mu=(0.15, 0.15, 0.15), M_cst=0.0, M_deg=0.004,
                 tau_phi=0.8, s_phi=(1.0, 1.0, 1.0, 1.0), s_g=(1.0, 1.0, 1.0, 1.0), Fb=(0.0, 0.0, 0.0),
                 u_wall=(0.0, 0.0, 0.0), rho_gauge=0.0) -> Params3:
    """3D parameters; the defaults are plain values for the pins (the 3D
    workloads pass NS s3 = s4 = 1/2 and d0 = 0.4 explicitly)."""
    p = Params3()
    p.nx, p.ny, p.nz = nx, ny, nz
    p.periodic[:] = list(periodic)
    p.d0, p.D, p.sigma12 = d0, D, sigma12
    p.theta, p.kappa = math.radians(theta_deg), kappa
    p.rho[:] = list(rho)
    p.mu[:] = list(mu)
    p.M_cst, p.M_deg, p.tau_phi = M_cst, M_deg, tau_phi
    p.s_phi[:] = list(s_phi)
    p.s_g[:] = list(s_g)
    p.Fb[:] = list(Fb)
    p.u_wall[:] = list(u_wall)
    p.rho_gauge = rho_gauge
    return p


def weights3(d0):
    w = np.zeros(15)
    _lib_handle().orc3_weights(d0, _ptr(w))
    return w


def velocities3():
    c = (C.c_int32 * 45)()
    _lib_handle().orc3_velocities(c)
    return np.array(list(c)).reshape(15, 3)


def M0_3():
    m = np.zeros((15, 15))
    _lib_handle().orc3_M0(_ptr(m))
    return m


def N3(cs2):
    m = np.zeros((15, 15))
    _lib_handle().orc3_N(cs2, _ptr(m))
    return m


def relaxation_matrix3(cs2, Kdiag):
    S = np.zeros((15, 15))
    _lib_handle().orc3_relaxation_matrix(cs2, _ptr(_arr(Kdiag, 15)), _ptr(S))
    return S


def collide3(cs2, Kdiag, f, feq, R):
    out = np.zeros(15)
    _lib_handle().orc3_collide(cs2, _ptr(_arr(Kdiag, 15)), _ptr(_arr(f, 15)), _ptr(_arr(feq, 15)),
                               _ptr(_arr(R, 15)), _ptr(out))
    return out


def feq3(d0, phi, eta_mub, A):
    out = np.zeros(15)
    _lib_handle().orc3_feq(d0, phi, eta_mub, _ptr(_arr(A, 3)), _ptr(out))
    return out


def Rpop3(d0, dA, a, eta_g):
    out = np.zeros(15)
    _lib_handle().orc3_Rpop(d0, _ptr(_arr(dA, 3)), a, _ptr(_arr(eta_g, 3)), _ptr(out))
    return out


def geq3(d0, gauge, P, rho, u, S):
    out = np.zeros(15)
    _lib_handle().orc3_geq(d0, gauge, P, rho, _ptr(_arr(u, 3)), _ptr(_arr(S, 3)), _ptr(out))
    return out


def Fpop3(d0, Q, G, M2):
    """M2 = (xx, yy, zz, xy, yz, xz)."""
    out = np.zeros(15)
    _lib_handle().orc3_Fpop(d0, Q, _ptr(_arr(G, 3)), _ptr(_arr(M2, 6)), _ptr(out))
    return out


def pressure3(d0, s0, s2a, g, Q, B, B_prev):
    return _lib_handle().orc3_pressure(d0, s0, s2a, _ptr(_arr(g, 15)), Q, B, B_prev)


class Sim3:
    """One 3D domain advanced by the oracle.  Arrays are [nz, ny, nx], x fastest."""

    NLAG = 13  # phi1 u (3), (rho u - S).u, sym(S u) (xx, yy, zz, xy, yz, xz), S x u (3)

    def __init__(self, params: Params3, phi0, phi1):
        self.params = params
        self.shape = (params.nz, params.ny, params.nx)
        n = params.nx * params.ny * params.nz
        self._phi0 = _arr(phi0, n)
        self._phi1 = _arr(phi1, n)
        self._h = _lib_handle().orc3_create(C.byref(params), _ptr(self._phi0), _ptr(self._phi1))
        if not self._h:
            raise ValueError("oracle rejected the parameters")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _lib_handle().orc3_free(h)
            self._h = None

    def step(self, nsteps: int = 1):
        _lib_handle().orc3_step(self._h, int(nsteps))

    @property
    def steps(self) -> int:
        return _lib_handle().orc3_step_count(self._h)

    def moments(self):
        out = [np.zeros(self.shape) for _ in range(5)]
        _lib_handle().orc3_moments(self._h, *[_ptr(a) for a in out])
        return tuple(out)  # phi1, ux, uy, uz, p

    def aux(self):
        mub = np.zeros(self.shape)
        gm = np.zeros((3,) + self.shape)
        _lib_handle().orc3_aux(self._h, _ptr(mub), _ptr(gm))
        return mub, gm

    def mass(self) -> float:
        return _lib_handle().orc3_mass(self._h)

    def get_state(self):
        f = np.zeros((15,) + self.shape)
        g = np.zeros((15,) + self.shape)
        lag = np.zeros((self.NLAG,) + self.shape)
        _lib_handle().orc3_get_state(self._h, _ptr(f), _ptr(g), _ptr(lag))
        return f, g, lag

    def set_state(self, f=None, g=None, lag=None):
        n = int(np.prod(self.shape))
        null = C.cast(None, _D)
        fa = _arr(f, 15 * n) if f is not None else None
        ga = _arr(g, 15 * n) if g is not None else None
        la = _arr(lag, self.NLAG * n) if lag is not None else None
        _lib_handle().orc3_set_state(self._h, _ptr(fa) if fa is not None else null,
                                     _ptr(ga) if ga is not None else null, _ptr(la) if la is not None else null)

    def derived(self) -> dict:
        k, eta = C.c_double(), C.c_double()
        g = np.zeros(3)
        _lib_handle().orc3_derived(self._h, C.byref(k), _ptr(g), C.byref(eta))
        return {"k": k.value, "gamma": list(g), "eta": eta.value}


def make_params3f(nx, ny, *, periodic_x=1, periodic_y=0, d0=0.5, D=4.0, sigma01=0.01, sigma02=0.01,
                  sigma12=0.01, rho=(1.0, 1.0, 1.0), mu=(0.15, 0.15, 0.15), M_cst=0.0, M_deg=0.01, tau_phi=0.8,
                  s_phi=(1.0, 1.0, 1.0, 1.0), s_g=(1.0, 1.0, 1.0, 1.0), Fb=(0.0, 0.0), rho_gauge=0.0) -> Params3F:
    """Parameters of the 3f model (three fluids, phi0 evolving)."""
    p = Params3F()
    p.nx, p.ny, p.periodic_x, p.periodic_y = nx, ny, periodic_x, periodic_y
    p.d0, p.D = d0, D
    p.sigma01, p.sigma02, p.sigma12 = sigma01, sigma02, sigma12
    p.rho[:] = list(rho)
    p.mu[:] = list(mu)
    p.M_cst, p.M_deg, p.tau_phi = M_cst, M_deg, tau_phi
    p.s_phi[:] = list(s_phi)
    p.s_g[:] = list(s_g)
    p.Fb[:] = list(Fb)
    p.rho_gauge = rho_gauge
    return p


def derive3f(p: Params3F):
    """(gamma[3], gammaT, eta[2]) of the 3f model, or None if a gamma_p <= 0."""
    g, gT, eta = np.zeros(3), C.c_double(), np.zeros(2)
    rc = _lib_handle().orc3f_derive(C.byref(p), _ptr(g), C.byref(gT), _ptr(eta))
    return None if rc else (g, gT.value, eta)


class Sim3F:
    """One 2D domain of the 3f model advanced by the oracle; arrays [ny, nx]."""

    NLAG = 9  # phi0 u, phi1 u, (rho u - S).u, sym(S u) (xx, yy, xy), psi

    def __init__(self, params: Params3F, phi0, phi1):
        self.params = params
        self.shape = (params.ny, params.nx)
        n = params.nx * params.ny
        self._phi0 = _arr(phi0, n)
        self._phi1 = _arr(phi1, n)
        self._h = _lib_handle().orc3f_create(C.byref(params), _ptr(self._phi0), _ptr(self._phi1))
        if not self._h:
            raise ValueError("oracle rejected the parameters")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _lib_handle().orc3f_free(h)
            self._h = None

    def step(self, nsteps: int = 1):
        _lib_handle().orc3f_step(self._h, int(nsteps))

    @property
    def steps(self) -> int:
        return _lib_handle().orc3f_step_count(self._h)

    def moments(self):
        out = [np.zeros(self.shape) for _ in range(5)]
        _lib_handle().orc3f_moments(self._h, *[_ptr(a) for a in out])
        return tuple(out)  # phi0, phi1, ux, uy, p

    def mass(self):
        m = np.zeros(2)
        _lib_handle().orc3f_mass(self._h, _ptr(m))
        return m

    def get_state(self):
        f0 = np.zeros((9,) + self.shape)
        f1 = np.zeros((9,) + self.shape)
        g = np.zeros((9,) + self.shape)
        lag = np.zeros((self.NLAG,) + self.shape)
        _lib_handle().orc3f_get_state(self._h, _ptr(f0), _ptr(f1), _ptr(g), _ptr(lag))
        return f0, f1, g, lag
