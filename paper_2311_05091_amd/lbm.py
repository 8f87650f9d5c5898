"""Python binding of the C ABI in include/tpf.h (argument marshalling only).

Every step of the method runs in the HIP library ``libtpf.so``; this module
loads it with ctypes, converts numpy arrays, and hands over device memory
(a torch tensor used as the arena) and the current torch stream.  It raises
when the library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional, Sequence

import numpy as np

from .geometry import DomainSpec

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libtpf.so")

TPF_OK, TPF_EINVAL, TPF_EDEVICE, TPF_ENAN, TPF_EBUDGET, TPF_ESTATE, TPF_EIO = 0, -1, -2, -3, -4, -5, -6


class TpfError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__("%s: %s (%d)" % (what, strerror(status), status))
        self.status = status


class DomainParams(C.Structure):
    """Mirror of tpf_domain_params."""
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


_lib = None
_D = C.POINTER(C.c_double)


def init_torch_device():
    """Initialises torch's HIP runtime (when a GPU is present) before a HIP
    library of this package is loaded.  torch carries its own HIP runtime; a
    library loaded into the process before torch has initialised the device
    finds no device once torch has (measured: tpf_create then reports zero
    devices), while the other order works."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()
_I32 = C.POINTER(C.c_int32)
_I64 = C.POINTER(C.c_int64)


def library() -> C.CDLL:
    """Loads libtpf.so (built by ``paper_2311_05091_amd.build``); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("HIP library %s is not built; run paper_2311_05091_amd/build.py "
                           "(there is no CPU fallback)" % LIB_PATH)
    init_torch_device()
    lib = C.CDLL(LIB_PATH)
    V = C.c_void_p
    sig = {
        "tpf_default_params": (None, [C.POINTER(DomainParams), C.c_int32, C.c_int32]),
        "tpf_create": (C.c_int, [C.POINTER(V), C.c_int32, V]),
        "tpf_add_domain": (C.c_int, [V, C.POINTER(DomainParams), _D, _D, _I32]),
        "tpf_arena_bytes": (C.c_int, [V, C.POINTER(C.c_uint64)]),
        "tpf_finalize": (C.c_int, [V, V, C.c_uint64]),
        "tpf_step": (C.c_int, [V, C.c_int64]),
        "tpf_run_to_residual": (C.c_int, [V, C.c_double, C.c_int32, C.c_int64, _I64]),
        "tpf_read_moments": (C.c_int, [V, C.c_int32, _D, _D, _D, _D]),
        "tpf_read_diag": (C.c_int, [V, C.c_int32, _D, _D, _I32, _I64]),
        "tpf_flow_rates": (C.c_int, [V, C.c_int32, _D]),
        "tpf_set_phi1": (C.c_int, [V, C.c_int32, _D]),
        "tpf_set_active": (C.c_int, [V, C.c_int32, C.c_int32]),
        "tpf_get_populations": (C.c_int, [V, C.c_int32, _D, _D]),
        "tpf_save": (C.c_int, [V, C.c_char_p]),
        "tpf_load": (C.c_int, [V, C.c_char_p]),
        "tpf_set_tile": (C.c_int, [V, C.c_int32]),
        "tpf_get_tile": (C.c_int, [V, _I32, _I32, _I32]),
        "tpf_tile_codes": (C.c_int, [_I32, _I32, _I32, _I32]),
        "tpf_autotune": (C.c_int, [V, C.c_int32, _D]),
        "tpf_size_class": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_char_p, C.c_int32]),
        "tpf_autotune_classes": (C.c_int, [V, C.c_int32, C.c_char_p, _I32]),
        "tpf_domain_tile": (C.c_int, [V, C.c_int32, _I32]),
        "tpf_set_launch_mode": (C.c_int, [V, C.c_int32]),
        "tpf_bytes_per_node": (C.c_int, [V, C.c_int32, _D]),
        "tpf_num_domains": (C.c_int, [V, _I32]),
        "tpf_domain_size": (C.c_int, [V, C.c_int32, _I32, _I32]),
        "tpf_derived": (C.c_int, [V, C.c_int32, _D, _D, _D, _D]),
        "tpf_kernel_timing": (C.c_int, [V, C.c_int32, _D, _I64]),
        "tpf_copy_bandwidth": (C.c_int, [V, V, C.c_uint64, C.c_int32, C.c_int32, V, _D]),
        "tpf_strerror": (C.c_char_p, [C.c_int32]),
        "tpf_destroy": (None, [V]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


EXPORTED = ("tpf_default_params", "tpf_create", "tpf_add_domain", "tpf_arena_bytes", "tpf_finalize",
            "tpf_step", "tpf_run_to_residual", "tpf_read_moments", "tpf_flow_rates", "tpf_read_diag", "tpf_set_phi1",
            "tpf_set_active",
            "tpf_get_populations", "tpf_save", "tpf_load", "tpf_set_tile", "tpf_get_tile",
            "tpf_tile_codes", "tpf_autotune", "tpf_size_class", "tpf_autotune_classes", "tpf_domain_tile",
            "tpf_set_launch_mode", "tpf_bytes_per_node",
            "tpf_num_domains", "tpf_domain_size", "tpf_derived", "tpf_kernel_timing",
            "tpf_copy_bandwidth", "tpf_strerror", "tpf_destroy")


def copy_bandwidth(nbytes: int = 1 << 30, nontemporal: bool = True, reps: int = 20) -> float:
    """HBM bandwidth (bytes read + written per second) of the library's device
    copy of nbytes between two torch device buffers (tpf_copy_bandwidth)."""
    import torch
    lib = library()
    a = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda")
    b = torch.zeros_like(a)
    ms = C.c_double()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    _check(lib.tpf_copy_bandwidth(C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), nbytes,
                                  1 if nontemporal else 0, reps, stream, C.byref(ms)), "tpf_copy_bandwidth")
    if not torch.equal(a, b):
        raise RuntimeError("tpf_copy_bandwidth: copy mismatch")
    return 2.0 * nbytes / (ms.value * 1e-3)


def strerror(status: int) -> str:
    try:
        return library().tpf_strerror(int(status)).decode()
    except Exception:  # library not loadable
        return "status %d" % status


def _check(rc: int, what: str, ok=(TPF_OK,)):
    if rc not in ok:
        raise TpfError(rc, what)
    return rc


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_D)


def params_from_spec(spec: DomainSpec) -> DomainParams:
    p = DomainParams()
    p.nx, p.ny = spec.nx, spec.ny
    p.periodic_x, p.periodic_y = int(spec.periodic_x), int(spec.periodic_y)
    p.d0, p.D, p.sigma12 = spec.d0, spec.D, spec.sigma12
    p.theta, p.kappa = math.radians(spec.theta_deg), spec.kappa
    p.rho[:] = list(spec.rho)
    p.mu[:] = list(spec.mu)
    p.M_cst, p.M_deg, p.tau_phi = spec.M_cst, spec.M_deg, spec.tau_phi
    p.s_phi[:] = list(spec.s_phi)
    p.s_g[:] = list(spec.s_g)
    p.Fb[:] = list(spec.Fb)
    p.u_wall[:] = list(spec.u_wall)
    p.omega_wall = spec.omega_wall
    p.wall_center[:] = list(spec.wall_center)
    p.rho_gauge = spec.rho_gauge
    p.open_x, p.inlet_type = int(spec.open_x), int(spec.inlet_type)
    p.p_in, p.u_in, p.p_out, p.phi1_in = spec.p_in, spec.u_in, spec.p_out, spec.phi1_in
    return p


def size_class(precision: int, nx: int, ny: int, has_s: bool) -> str:
    """The autotuner's size class of a domain (host only)."""
    buf = C.create_string_buffer(64)
    _check(library().tpf_size_class(precision, nx, ny, 1 if has_s else 0, buf, 64), "tpf_size_class")
    return buf.value.decode()


def tile_codes():
    lib = library()
    n = C.c_int32()
    lib.tpf_tile_codes(C.byref(n), None, None, None)
    codes = (C.c_int32 * n.value)()
    tx = (C.c_int32 * n.value)()
    ty = (C.c_int32 * n.value)()
    lib.tpf_tile_codes(C.byref(n), codes, tx, ty)
    return [(codes[i], tx[i], ty[i]) for i in range(n.value)]


class Context:
    """A set of domains advanced together on one GPU.

    precision: 32 or 64.  Device memory is one torch uint8 tensor handed to
    the library as its arena; work goes to the current torch stream.
    """

    def __init__(self, precision: int = 64, device: str = "cuda:0", use_torch_arena: bool = True):
        import torch
        self._torch = torch
        self.lib = library()
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self._h = C.c_void_p()
        _check(self.lib.tpf_create(C.byref(self._h), int(precision), C.c_void_p(self.stream.cuda_stream)),
               "tpf_create")
        self.precision = precision
        self.use_torch_arena = use_torch_arena
        self._arena = None
        self.specs = []

    # -- set-up ------------------------------------------------------------
    def add_domain(self, spec: DomainSpec) -> int:
        p = params_from_spec(spec)
        phi0 = np.ascontiguousarray(spec.phi0, dtype=np.float64)
        phi1 = np.ascontiguousarray(spec.phi1, dtype=np.float64)
        assert phi0.shape == (spec.ny, spec.nx) and phi1.shape == (spec.ny, spec.nx)
        did = C.c_int32()
        _check(self.lib.tpf_add_domain(self._h, C.byref(p), _dptr(phi0), _dptr(phi1), C.byref(did)),
               "tpf_add_domain")
        self.specs.append(spec)
        return did.value

    def finalize(self, fill: Optional[int] = None):
        """Binds the arena and initialises the domains.  fill: byte value the
        arena is set to first (tests use it to show that no step reads memory
        that initialisation did not write)."""
        nbytes = C.c_uint64()
        _check(self.lib.tpf_arena_bytes(self._h, C.byref(nbytes)), "tpf_arena_bytes")
        if self.use_torch_arena:
            self._arena = self._torch.empty(int(nbytes.value), dtype=self._torch.uint8, device=self.device)
            if fill is not None:
                self._arena.fill_(int(fill))
            ptr = C.c_void_p(self._arena.data_ptr())
        else:
            ptr = C.c_void_p(None)
        _check(self.lib.tpf_finalize(self._h, ptr, nbytes.value), "tpf_finalize")
        return self

    @property
    def arena_bytes(self) -> int:
        return 0 if self._arena is None else self._arena.numel()

    # -- stepping ------------------------------------------------------------
    def step(self, nsteps: int = 1):
        _check(self.lib.tpf_step(self._h, int(nsteps)), "tpf_step")

    def run_to_residual(self, tol: float, check_every: int = 100, max_steps: int = 10 ** 6):
        n = len(self.specs)
        out = (C.c_int64 * n)()
        rc = self.lib.tpf_run_to_residual(self._h, float(tol), int(check_every), int(max_steps), out)
        _check(rc, "tpf_run_to_residual", ok=(TPF_OK, TPF_EBUDGET, TPF_ENAN))
        return rc, np.array(out[:], dtype=np.int64)

    # -- read-out ------------------------------------------------------------
    def moments(self, did: int = 0):
        s = self.specs[did]
        out = [np.empty((s.ny, s.nx)) for _ in range(4)]
        _check(self.lib.tpf_read_moments(self._h, did, *[_dptr(a) for a in out]), "tpf_read_moments")
        return tuple(out)

    def flow_rates(self, did: int = 0) -> np.ndarray:
        """Sums over phi0 <= 1/2 of u_x, phi1 u_x, phi2 u_x (tpf_flow_rates)."""
        q = np.zeros(3)
        _check(self.lib.tpf_flow_rates(self._h, did, _dptr(q)), "tpf_flow_rates")
        return q

    def diag(self, did: int = 0) -> dict:
        m, r = C.c_double(), C.c_double()
        st, n = C.c_int32(), C.c_int64()
        _check(self.lib.tpf_read_diag(self._h, did, C.byref(m), C.byref(r), C.byref(st), C.byref(n)),
               "tpf_read_diag")
        return {"mass": m.value, "residual": r.value, "status": st.value, "steps": n.value}

    def populations(self, did: int = 0):
        s = self.specs[did]
        f = np.empty((9, s.ny, s.nx))
        g = np.empty((9, s.ny, s.nx))
        _check(self.lib.tpf_get_populations(self._h, did, _dptr(f), _dptr(g)), "tpf_get_populations")
        return f, g

    def set_active(self, did: int, active: bool):
        """Leaves the domain out of (False) or back in (True) the following steps."""
        _check(self.lib.tpf_set_active(self._h, int(did), 1 if active else 0), "tpf_set_active")

    def set_phi1(self, did: int, phi1: np.ndarray):
        a = np.ascontiguousarray(phi1, dtype=np.float64)
        _check(self.lib.tpf_set_phi1(self._h, did, _dptr(a)), "tpf_set_phi1")

    def save(self, path: str):
        _check(self.lib.tpf_save(self._h, path.encode()), "tpf_save")

    def load(self, path: str):
        _check(self.lib.tpf_load(self._h, path.encode()), "tpf_load")

    # -- tuning and measurement ----------------------------------------------
    def set_tile(self, code: int):
        _check(self.lib.tpf_set_tile(self._h, int(code)), "tpf_set_tile")

    def set_launch_mode(self, mode: int):
        """0: one launch per step; 1: persistent launches (strip and strip-group
        tiles; the residual checks of run_to_residual run inside them);
        2: one launch per step, tile shape chosen from the live work."""
        _check(self.lib.tpf_set_launch_mode(self._h, int(mode)), "tpf_set_launch_mode")

    def tile(self):
        c, x, y = C.c_int32(), C.c_int32(), C.c_int32()
        _check(self.lib.tpf_get_tile(self._h, C.byref(c), C.byref(x), C.byref(y)), "tpf_get_tile")
        return c.value, x.value, y.value

    def autotune(self, steps: int = 20) -> float:
        ms = C.c_double()
        _check(self.lib.tpf_autotune(self._h, int(steps), C.byref(ms)), "tpf_autotune")
        return ms.value

    def autotune_classes(self, steps: int = 20, cache_path: Optional[str] = None) -> int:
        """Per-size-class tile choice (timed, or read from the JSON cache);
        returns the number of classes that were timed."""
        n = C.c_int32()
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(self.lib.tpf_autotune_classes(self._h, int(steps), path, C.byref(n)), "tpf_autotune_classes")
        return n.value

    def domain_tile(self, did: int) -> int:
        c = C.c_int32()
        _check(self.lib.tpf_domain_tile(self._h, int(did), C.byref(c)), "tpf_domain_tile")
        return c.value

    def bytes_per_node(self, did: int = 0) -> float:
        b = C.c_double()
        _check(self.lib.tpf_bytes_per_node(self._h, did, C.byref(b)), "tpf_bytes_per_node")
        return b.value

    def derived(self, did: int = 0) -> dict:
        k, gT, eta = C.c_double(), C.c_double(), C.c_double()
        g = (C.c_double * 3)()
        _check(self.lib.tpf_derived(self._h, did, C.byref(k), g, C.byref(gT), C.byref(eta)), "tpf_derived")
        return {"k": k.value, "gamma": list(g), "gammaT": gT.value, "eta": eta.value}

    def kernel_timing(self, enable: bool):
        ms, n = C.c_double(), C.c_int64()
        _check(self.lib.tpf_kernel_timing(self._h, 1 if enable else 0, C.byref(ms), C.byref(n)),
               "tpf_kernel_timing")
        return ms.value, n.value

    def close(self):
        if self._h:
            self.lib.tpf_destroy(self._h)
            self._h = C.c_void_p()
        self._arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
