"""Python binding of the 3D C ABI in include/tpf3.h (argument marshalling only).

Every step runs in ``libtpf.so``; this module converts numpy arrays, hands the
library a torch tensor as its device arena and the current torch stream, and
raises when the library is missing (no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

from .geometry3d import DomainSpec3
from .lbm import TpfError, library, strerror  # noqa: F401  (TpfError re-exported)

_D = C.POINTER(C.c_double)
_I32 = C.POINTER(C.c_int32)
_I64 = C.POINTER(C.c_int64)


class DomainParams3(C.Structure):
    """Mirror of tpf3_domain_params."""
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


EXPORTED3 = ("tpf3_default_params", "tpf3_create", "tpf3_add_domain", "tpf3_arena_bytes", "tpf3_finalize",
             "tpf3_step", "tpf3_read_moments", "tpf3_read_mass", "tpf3_get_populations", "tpf3_set_tile",
             "tpf3_get_tile", "tpf3_bytes_per_node", "tpf3_kernel_timing", "tpf3_destroy")

_bound = False


def library3() -> C.CDLL:
    """libtpf.so with the 3D entry points' signatures set."""
    global _bound
    lib = library()
    if _bound:
        return lib
    V = C.c_void_p
    sig = {
        "tpf3_default_params": (None, [C.POINTER(DomainParams3), C.c_int32, C.c_int32, C.c_int32]),
        "tpf3_create": (C.c_int, [C.POINTER(V), C.c_int32, V]),
        "tpf3_add_domain": (C.c_int, [V, C.POINTER(DomainParams3), _D, _D, _I32]),
        "tpf3_arena_bytes": (C.c_int, [V, C.POINTER(C.c_uint64)]),
        "tpf3_finalize": (C.c_int, [V, V, C.c_uint64]),
        "tpf3_step": (C.c_int, [V, C.c_int64]),
        "tpf3_read_moments": (C.c_int, [V, C.c_int32, _D, _D, _D, _D, _D]),
        "tpf3_read_mass": (C.c_int, [V, C.c_int32, _D]),
        "tpf3_get_populations": (C.c_int, [V, C.c_int32, _D, _D]),
        "tpf3_set_tile": (C.c_int, [V, C.c_int32]),
        "tpf3_get_tile": (C.c_int, [V, _I32, _I32, _I32]),
        "tpf3_bytes_per_node": (C.c_int, [V, C.c_int32, _D]),
        "tpf3_kernel_timing": (C.c_int, [V, C.c_int32, _D, _I64]),
        "tpf3_destroy": (None, [V]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _bound = True
    return lib


def _check(rc: int, what: str):
    if rc != 0:
        raise TpfError(rc, what)


def params_from_spec3(s: DomainSpec3) -> DomainParams3:
    p = DomainParams3()
    p.nx, p.ny, p.nz = s.nx, s.ny, s.nz
    p.periodic[:] = [int(v) for v in s.periodic]
    p.d0, p.D, p.sigma12 = s.d0, s.D, s.sigma12
    p.theta, p.kappa = math.radians(s.theta_deg), s.kappa
    p.rho[:] = list(s.rho)
    p.mu[:] = list(s.mu)
    p.M_cst, p.M_deg, p.tau_phi = s.M_cst, s.M_deg, s.tau_phi
    p.s_phi[:] = list(s.s_phi)
    p.s_g[:] = list(s.s_g)
    p.Fb[:] = list(s.Fb)
    p.u_wall[:] = list(s.u_wall)
    p.rho_gauge = s.rho_gauge
    return p


class Context3:
    """3D domains advanced together on one GPU (precision 32 or 64); device
    memory is one torch uint8 tensor used as the library's arena."""

    def __init__(self, precision: int = 64, device: str = "cuda:0"):
        import torch
        self._torch = torch
        self.lib = library3()
        torch.cuda.set_device(torch.device(device))
        self.stream = torch.cuda.current_stream()
        self._h = C.c_void_p()
        _check(self.lib.tpf3_create(C.byref(self._h), precision, C.c_void_p(self.stream.cuda_stream)), "tpf3_create")
        self.precision = precision
        self.shapes = []
        self._arena = None

    def add_domain(self, spec: DomainSpec3) -> int:
        p = params_from_spec3(spec)
        phi0 = np.ascontiguousarray(spec.phi0, dtype=np.float64)
        phi1 = np.ascontiguousarray(spec.phi1, dtype=np.float64)
        assert phi0.shape == (spec.nz, spec.ny, spec.nx) and phi1.shape == phi0.shape
        did = C.c_int32()
        _check(self.lib.tpf3_add_domain(self._h, C.byref(p), phi0.ctypes.data_as(_D), phi1.ctypes.data_as(_D),
                                        C.byref(did)), "tpf3_add_domain")
        self.shapes.append((spec.nz, spec.ny, spec.nx))
        return did.value

    def finalize(self):
        nb = C.c_uint64()
        _check(self.lib.tpf3_arena_bytes(self._h, C.byref(nb)), "tpf3_arena_bytes")
        self._arena = self._torch.empty(int(nb.value) + 256, dtype=self._torch.uint8, device="cuda")
        base = self._arena.data_ptr()
        aligned = (base + 255) // 256 * 256
        _check(self.lib.tpf3_finalize(self._h, C.c_void_p(aligned), nb.value), "tpf3_finalize")

    def step(self, n: int):
        _check(self.lib.tpf3_step(self._h, int(n)), "tpf3_step")

    def moments(self, did: int = 0):
        shape = self.shapes[did]
        out = [np.zeros(shape) for _ in range(5)]
        _check(self.lib.tpf3_read_moments(self._h, did, *[a.ctypes.data_as(_D) for a in out]), "tpf3_read_moments")
        return tuple(out)   # phi1, ux, uy, uz, p

    def mass(self, did: int = 0) -> float:
        m = C.c_double()
        _check(self.lib.tpf3_read_mass(self._h, did, C.byref(m)), "tpf3_read_mass")
        return m.value

    def populations(self, did: int = 0):
        shape = (15,) + self.shapes[did]
        f, g = np.zeros(shape), np.zeros(shape)
        _check(self.lib.tpf3_get_populations(self._h, did, f.ctypes.data_as(_D), g.ctypes.data_as(_D)),
               "tpf3_get_populations")
        return f, g

    def set_tile(self, ty: int):
        _check(self.lib.tpf3_set_tile(self._h, int(ty)), "tpf3_set_tile")

    def tile(self):
        tx, ty, tz = C.c_int32(), C.c_int32(), C.c_int32()
        _check(self.lib.tpf3_get_tile(self._h, C.byref(tx), C.byref(ty), C.byref(tz)), "tpf3_get_tile")
        return tx.value, ty.value, tz.value

    def bytes_per_node(self, did: int = 0) -> float:
        b = C.c_double()
        _check(self.lib.tpf3_bytes_per_node(self._h, did, C.byref(b)), "tpf3_bytes_per_node")
        return b.value

    def kernel_timing(self, enable: bool):
        ms, n = C.c_double(), C.c_int64()
        _check(self.lib.tpf3_kernel_timing(self._h, 1 if enable else 0, C.byref(ms), C.byref(n)),
               "tpf3_kernel_timing")
        return ms.value, n.value

    def close(self):
        if self._h:
            self._torch.cuda.synchronize()
            self.lib.tpf3_destroy(self._h)
            self._h = C.c_void_p()
        self._arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
