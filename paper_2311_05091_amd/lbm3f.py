"""Python binding of the 3f-model C ABI in include/tpf3f.h (argument
marshalling only).

Every step runs in ``libtpf.so``; this module converts numpy arrays, hands the
library a torch tensor as its device arena and the current torch stream, and
raises when the library is missing (no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from .geometry3f import DomainSpec3F
from .lbm import TpfError, library  # noqa: F401  (TpfError re-exported)

_D = C.POINTER(C.c_double)
_I32 = C.POINTER(C.c_int32)
_I64 = C.POINTER(C.c_int64)


class DomainParams3F(C.Structure):
    """Mirror of tpf3f_domain_params."""
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


EXPORTED3F = ("tpf3f_default_params", "tpf3f_create", "tpf3f_add_domain", "tpf3f_arena_bytes", "tpf3f_finalize",
              "tpf3f_step", "tpf3f_read_moments", "tpf3f_read_mass", "tpf3f_get_populations",
              "tpf3f_bytes_per_node", "tpf3f_kernel_timing", "tpf3f_destroy")

_bound = False


def library3f() -> C.CDLL:
    """libtpf.so with the 3f entry points' signatures set."""
    global _bound
    lib = library()
    if _bound:
        return lib
    V = C.c_void_p
    sig = {
        "tpf3f_default_params": (None, [C.POINTER(DomainParams3F), C.c_int32, C.c_int32]),
        "tpf3f_create": (C.c_int, [C.POINTER(V), C.c_int32, V]),
        "tpf3f_add_domain": (C.c_int, [V, C.POINTER(DomainParams3F), _D, _D, _I32]),
        "tpf3f_arena_bytes": (C.c_int, [V, C.POINTER(C.c_uint64)]),
        "tpf3f_finalize": (C.c_int, [V, V, C.c_uint64]),
        "tpf3f_step": (C.c_int, [V, C.c_int64]),
        "tpf3f_read_moments": (C.c_int, [V, C.c_int32, _D, _D, _D, _D, _D]),
        "tpf3f_read_mass": (C.c_int, [V, C.c_int32, _D]),
        "tpf3f_get_populations": (C.c_int, [V, C.c_int32, _D, _D, _D]),
        "tpf3f_bytes_per_node": (C.c_int, [V, C.c_int32, _D]),
        "tpf3f_kernel_timing": (C.c_int, [V, C.c_int32, _D, _I64]),
        "tpf3f_destroy": (None, [V]),
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


def params_from_spec3f(s: DomainSpec3F) -> DomainParams3F:
    p = DomainParams3F()
    p.nx, p.ny, p.periodic_x, p.periodic_y = s.nx, s.ny, int(s.periodic_x), int(s.periodic_y)
    p.d0, p.D = s.d0, s.D
    p.sigma01, p.sigma02, p.sigma12 = s.sigma01, s.sigma02, s.sigma12
    p.rho[:] = list(s.rho)
    p.mu[:] = list(s.mu)
    p.M_cst, p.M_deg, p.tau_phi = s.M_cst, s.M_deg, s.tau_phi
    p.s_phi[:] = list(s.s_phi)
    p.s_g[:] = list(s.s_g)
    p.Fb[:] = list(s.Fb)
    p.rho_gauge = s.rho_gauge
    return p


class Context3F:
    """3f-model domains advanced together on one GPU (precision 32 or 64);
    device memory is one torch uint8 tensor used as the library's arena."""

    def __init__(self, precision: int = 64, device: str = "cuda:0"):
        import torch
        self._torch = torch
        self.lib = library3f()
        torch.cuda.set_device(torch.device(device))
        self.stream = torch.cuda.current_stream()
        self._h = C.c_void_p()
        _check(self.lib.tpf3f_create(C.byref(self._h), precision, C.c_void_p(self.stream.cuda_stream)),
               "tpf3f_create")
        self.precision = precision
        self.shapes = []
        self._arena = None

    def add_domain(self, spec: DomainSpec3F) -> int:
        p = params_from_spec3f(spec)
        phi0 = np.ascontiguousarray(spec.phi0, dtype=np.float64)
        phi1 = np.ascontiguousarray(spec.phi1, dtype=np.float64)
        assert phi0.shape == (spec.ny, spec.nx) and phi1.shape == phi0.shape
        did = C.c_int32()
        _check(self.lib.tpf3f_add_domain(self._h, C.byref(p), phi0.ctypes.data_as(_D), phi1.ctypes.data_as(_D),
                                         C.byref(did)), "tpf3f_add_domain")
        self.shapes.append((spec.ny, spec.nx))
        return did.value

    def finalize(self, fill: Optional[int] = None):
        nb = C.c_uint64()
        _check(self.lib.tpf3f_arena_bytes(self._h, C.byref(nb)), "tpf3f_arena_bytes")
        self._arena = self._torch.empty(int(nb.value) + 256, dtype=self._torch.uint8, device="cuda")
        if fill is not None:
            self._arena.fill_(int(fill))
        aligned = (self._arena.data_ptr() + 255) // 256 * 256
        _check(self.lib.tpf3f_finalize(self._h, C.c_void_p(aligned), nb.value), "tpf3f_finalize")

    def step(self, n: int):
        _check(self.lib.tpf3f_step(self._h, int(n)), "tpf3f_step")

    def moments(self, did: int = 0):
        out = [np.zeros(self.shapes[did]) for _ in range(5)]
        _check(self.lib.tpf3f_read_moments(self._h, did, *[a.ctypes.data_as(_D) for a in out]), "tpf3f_read_moments")
        return tuple(out)   # phi0, phi1, ux, uy, p

    def mass(self, did: int = 0):
        m = np.zeros(2)
        _check(self.lib.tpf3f_read_mass(self._h, did, m.ctypes.data_as(_D)), "tpf3f_read_mass")
        return m

    def populations(self, did: int = 0):
        shape = (9,) + self.shapes[did]
        f0, f1, g = np.zeros(shape), np.zeros(shape), np.zeros(shape)
        _check(self.lib.tpf3f_get_populations(self._h, did, f0.ctypes.data_as(_D), f1.ctypes.data_as(_D),
                                              g.ctypes.data_as(_D)), "tpf3f_get_populations")
        return f0, f1, g

    def bytes_per_node(self, did: int = 0) -> float:
        b = C.c_double()
        _check(self.lib.tpf3f_bytes_per_node(self._h, did, C.byref(b)), "tpf3f_bytes_per_node")
        return b.value

    def kernel_timing(self, enable: bool):
        ms, n = C.c_double(), C.c_int64()
        _check(self.lib.tpf3f_kernel_timing(self._h, 1 if enable else 0, C.byref(ms), C.byref(n)),
               "tpf3f_kernel_timing")
        return ms.value, n.value

    def close(self):
        if self._h:
            self._torch.cuda.synchronize()
            self.lib.tpf3f_destroy(self._h)
            self._h = C.c_void_p()
        self._arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
