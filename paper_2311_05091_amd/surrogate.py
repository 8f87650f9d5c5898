"""Learned warm start: a convolutional encoder-decoder that predicts the
equilibrium phase field phi1 of a droplet from the solid field phi0, the
contact angle and the droplet volume.  The lattice Boltzmann library then
relaxes from the prediction; the plain initial condition stays the fallback.

The network runs entirely in the HIP kernels of ``libtpf_nn.so`` (bf16
activations on the matrix cores, FP32 accumulation, FP32 master weights and
Adam).  This module only wires the layers together and marshals pointers;
torch tensors serve as device buffers.

Architecture (4 levels, 32-64-128-256 channels, input 256 x 256):
  encoder level l: [pool 2x2] conv3x3+ReLU -> conv3x3+ReLU  (skip_l)
  decoder level l: up 2x -> conv3x3+ReLU -> concat skip_l -> 2 x conv3x3+ReLU
  head: 1x1 conv -> sigmoid.
Input channels (padded to 32): phi0, (theta - 90 deg)/60 deg, droplet volume
(10 x sum(phi1)/area), and the plain initial phi1 (which places the droplet).
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
NN_LIB_PATH = os.path.join(_PKG, "libtpf_nn.so")
RES = 256
IN_CH = 32
IN_USED = 4
_nn = None

V = C.c_void_p
I32 = C.c_int32
I64 = C.c_int64
F32 = C.c_float


def nnlib() -> C.CDLL:
    """Loads libtpf_nn.so; raises if it has not been built (no CPU fallback)."""
    global _nn
    if _nn is not None:
        return _nn
    if not os.path.exists(NN_LIB_PATH):
        raise RuntimeError("HIP library %s is not built; run paper_2311_05091_amd/build.py" % NN_LIB_PATH)
    from .lbm import init_torch_device
    init_torch_device()
    lib = C.CDLL(NN_LIB_PATH)
    sig = {
        "tpfnn_mfma_selftest": [V, V, V, V],
        "tpfnn_conv3x3_fwd": [V, I32, I32, I32, I32, V, V, I32, I32, V, V],
        "tpfnn_weight_flip": [V, I32, I32, V, V],
        "tpfnn_conv3x3_wgrad": [V, V, I32, I32, I32, I32, I32, V, V, V, C.c_size_t, V],
        "tpfnn_relu_bwd": [V, V, I64, V],
        "tpfnn_avgpool2_fwd": [V, I32, I32, I32, I32, V, V],
        "tpfnn_avgpool2_bwd": [V, I32, I32, I32, I32, V, V],
        "tpfnn_upsample2_fwd": [V, I32, I32, I32, I32, V, V],
        "tpfnn_upsample2_bwd": [V, I32, I32, I32, I32, V, V],
        "tpfnn_concat": [V, I32, V, I32, I64, V, V],
        "tpfnn_split": [V, I32, I32, I64, V, V, V],
        "tpfnn_add_inplace": [V, V, I64, V],
        "tpfnn_head": [V, I64, I32, V, V, V, V, V, V, V, V, V, C.c_size_t, V],
        "tpfnn_head_noalloc": [V, I64, I32, V, V, V, V, V, V, V, V, V],
        "tpfnn_adam": [V, V, V, V, V, I64, F32, F32, F32, F32, I32, V],
        "tpfnn_to_bf16": [V, V, I64, V],
        "tpfnn_from_bf16": [V, V, I64, V],
        "tpfnn_resample": [V, I32, I32, I32, V, I32, I32, V],
        "tpfnn_pack_input": [V, V, V, V, I32, I32, I32, V, V],
        "tpfnn_mass_project": [V, V, I64, C.c_double, V, V, V],
        "tpfnn_mass_project_batch": [V, V, C.c_int32, I64, V, V, V, V],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.restype = C.c_int
        fn.argtypes = args
    for name, args in {"tpfnn_wgrad_workspace": [I32, I32, I32, I32, I32],
                       "tpfnn_head_workspace": [I64, I32]}.items():
        fn = getattr(lib, name)
        fn.restype = C.c_size_t
        fn.argtypes = args
    _nn = lib
    return lib


EXPORTED_NN = ("tpfnn_mfma_selftest", "tpfnn_conv3x3_fwd", "tpfnn_weight_flip", "tpfnn_wgrad_workspace",
               "tpfnn_conv3x3_wgrad", "tpfnn_relu_bwd", "tpfnn_avgpool2_fwd", "tpfnn_avgpool2_bwd",
               "tpfnn_upsample2_fwd", "tpfnn_upsample2_bwd", "tpfnn_concat", "tpfnn_split",
               "tpfnn_add_inplace", "tpfnn_head_workspace", "tpfnn_head", "tpfnn_head_noalloc", "tpfnn_adam",
               "tpfnn_to_bf16", "tpfnn_from_bf16", "tpfnn_resample", "tpfnn_pack_input", "tpfnn_mass_project",
               "tpfnn_mass_project_batch")


def _ck(rc, what):
    if rc != 0:
        raise RuntimeError("%s failed with status %d" % (what, rc))


def _p(t):
    return V(t.data_ptr())


def layer_table(widths=(32, 64, 128, 256)) -> List[Tuple[str, int, int]]:
    """(name, Cin, Cout) of every 3x3 convolution, in forward order."""
    L = len(widths)
    out = []
    for l in range(L):
        cin = IN_CH if l == 0 else widths[l - 1]
        out.append(("e%da" % l, cin, widths[l]))
        out.append(("e%db" % l, widths[l], widths[l]))
    for l in range(L - 2, -1, -1):
        out.append(("d%du" % l, widths[l + 1], widths[l]))
        out.append(("d%da" % l, 2 * widths[l], widths[l]))
        out.append(("d%db" % l, widths[l], widths[l]))
    return out


def init_params(widths=(32, 64, 128, 256), seed=0) -> Dict[str, Tuple[np.ndarray, np.ndarray]]:
    """He-normal weights [Cout,3,3,Cin] (input channels beyond the ones used are zero), zero biases."""
    rng = np.random.default_rng(seed)
    params = {}
    for name, cin, cout in layer_table(widths):
        fan = 9 * (IN_USED if name == "e0a" else cin)
        w = rng.normal(0.0, math.sqrt(2.0 / fan), (cout, 3, 3, cin))
        if name == "e0a":
            w[..., IN_USED:] = 0.0
        params[name] = (w, np.zeros(cout))
    params["head"] = (rng.normal(0.0, math.sqrt(1.0 / widths[0]), widths[0]), np.zeros(1))
    return params


class UNet:
    """Encoder-decoder on the BF16 matrix cores, trained with Adam."""

    def __init__(self, widths=(32, 64, 128, 256), seed=0, device="cuda:0", params=None):
        import torch
        self.torch = torch
        self.lib = nnlib()
        self.dev = torch.device(device)
        self.widths = tuple(widths)
        self.layers = layer_table(self.widths)
        self.stream = V(torch.cuda.current_stream(self.dev).cuda_stream)
        params = params if params is not None else init_params(self.widths, seed)
        f32 = dict(dtype=torch.float32, device=self.dev)
        self.w, self.b, self.wb, self.wt = {}, {}, {}, {}
        self.gw, self.gb, self.m, self.v = {}, {}, {}, {}
        for name, cin, cout in self.layers:
            w, b = params[name]
            self.w[name] = torch.tensor(np.asarray(w, np.float32).ravel(), **f32)
            self.b[name] = torch.tensor(np.asarray(b, np.float32), **f32)
            self.wb[name] = torch.empty(self.w[name].numel(), dtype=torch.bfloat16, device=self.dev)
            self.wt[name] = torch.empty_like(self.wb[name])
            _ck(self.lib.tpfnn_to_bf16(_p(self.w[name]), _p(self.wb[name]), self.w[name].numel(), self.stream),
                "to_bf16")
        wh, bh = params["head"]
        self.w["head"] = torch.tensor(np.asarray(wh, np.float32), **f32)
        self.b["head"] = torch.tensor(np.asarray(bh, np.float32), **f32)
        for k in self.w:
            self.gw[k] = torch.zeros_like(self.w[k])
            self.gb[k] = torch.zeros_like(self.b[k])
            self.m[k] = (torch.zeros_like(self.w[k]), torch.zeros_like(self.b[k]))
            self.v[k] = (torch.zeros_like(self.w[k]), torch.zeros_like(self.b[k]))
        self.t = 0
        self._bufN = None

    # ------------------------------------------------------------------
    def params_numpy(self) -> Dict[str, Tuple[np.ndarray, np.ndarray]]:
        out = {}
        for name, cin, cout in self.layers:
            out[name] = (self.w[name].cpu().numpy().astype(np.float64).reshape(cout, 3, 3, cin),
                         self.b[name].cpu().numpy().astype(np.float64))
        out["head"] = (self.w["head"].cpu().numpy().astype(np.float64),
                       self.b["head"].cpu().numpy().astype(np.float64))
        return out

    def n_params(self) -> int:
        return int(sum(self.w[k].numel() + self.b[k].numel() for k in self.w))

    def flops_per_sample(self) -> float:
        """Multiply-adds x 2 of the forward pass at 256 x 256."""
        tot = 0.0
        for name, cin, cout in self.layers:
            lvl = int(name[1])
            res = RES >> lvl
            tot += 2.0 * 9 * cin * cout * res * res
        return tot

    def _alloc(self, N):
        if self._bufN == N:
            return
        torch = self.torch
        bf = dict(dtype=torch.bfloat16, device=self.dev)
        self.act, self.grad = {}, {}
        W = self.widths
        L = len(W)
        shape = {}
        for l in range(L):
            r = RES >> l
            shape["e%da" % l] = (r, W[l])
            shape["e%db" % l] = (r, W[l])
            if l > 0:
                shape["p%d" % l] = (r, W[l - 1])
        for l in range(L - 1):
            r = RES >> l
            shape["u%d" % l] = (r, W[l + 1])
            shape["d%du" % l] = (r, W[l])
            shape["c%d" % l] = (r, 2 * W[l])
            shape["d%da" % l] = (r, W[l])
            shape["d%db" % l] = (r, W[l])
            shape["skipg%d" % l] = (r, W[l])
        shape["in"] = (RES, IN_CH)
        self.shape = shape
        for k, (r, c) in shape.items():
            self.act[k] = torch.empty(N * r * r * c, **bf)
            self.grad[k] = torch.empty(N * r * r * c, **bf)
        self.pred = torch.empty(N * RES * RES, dtype=torch.float32, device=self.dev)
        self.loss = torch.zeros(1, dtype=torch.float64, device=self.dev)
        ws = 0
        for name, cin, cout in self.layers:
            r = RES >> int(name[1])
            ws = max(ws, self.lib.tpfnn_wgrad_workspace(N, r, r, cin, cout))
        ws = max(ws, self.lib.tpfnn_head_workspace(N * RES * RES, W[0]))
        self.work = torch.empty(int(ws), dtype=torch.uint8, device=self.dev)
        self._bufN = N

    # ------------------------------------------------------------------
    def _conv(self, name, x, y, N, r):
        cin = cout = None
        for n_, ci, co in self.layers:
            if n_ == name:
                cin, cout = ci, co
        _ck(self.lib.tpfnn_conv3x3_fwd(_p(x), N, r, r, cin, _p(self.wb[name]), _p(self.b[name]), cout, 1,
                                       _p(y), self.stream), "conv " + name)

    def pack(self, phi0: np.ndarray, theta_deg: np.ndarray, vol: np.ndarray, phi1_init: Optional[np.ndarray] = None):
        """Builds the bf16 network input from [N,256,256] phi0, [N] angles, [N] volumes
        and the [N,256,256] plain initial phi1 (zero channel when None)."""
        torch = self.torch
        N = phi0.shape[0]
        self._alloc(N)
        t0 = torch.tensor(np.ascontiguousarray(phi0, np.float32), device=self.dev)
        t1 = None if phi1_init is None else torch.tensor(np.ascontiguousarray(phi1_init, np.float32),
                                                          device=self.dev)
        th = torch.tensor(np.asarray(theta_deg, np.float32), device=self.dev)
        vv = torch.tensor(np.asarray(vol, np.float32), device=self.dev)
        _ck(self.lib.tpfnn_pack_input(_p(t0), _p(t1) if t1 is not None else None, _p(th), _p(vv), N, RES, RES,
                                      _p(self.act["in"]), self.stream), "pack_input")
        # the inputs are read by the kernel queued above: keep them alive until it ran
        self._pack_keep = (t0, t1, th, vv)
        return N

    def forward(self, N):
        """Runs the network on self.act['in'] (N samples); returns the FP32 prediction tensor."""
        a = self.act
        L = len(self.widths)
        W = self.widths
        h = a["in"]
        for l in range(L):
            r = RES >> l
            if l > 0:
                _ck(self.lib.tpfnn_avgpool2_fwd(_p(h), N, 2 * r, 2 * r, W[l - 1], _p(a["p%d" % l]), self.stream),
                    "pool")
                h = a["p%d" % l]
            self._conv("e%da" % l, h, a["e%da" % l], N, r)
            self._conv("e%db" % l, a["e%da" % l], a["e%db" % l], N, r)
            h = a["e%db" % l]
        for l in range(L - 2, -1, -1):
            r = RES >> l
            _ck(self.lib.tpfnn_upsample2_fwd(_p(h), N, r // 2, r // 2, W[l + 1], _p(a["u%d" % l]), self.stream),
                "up")
            self._conv("d%du" % l, a["u%d" % l], a["d%du" % l], N, r)
            _ck(self.lib.tpfnn_concat(_p(a["d%du" % l]), W[l], _p(a["e%db" % l]), W[l], N * r * r,
                                      _p(a["c%d" % l]), self.stream), "concat")
            self._conv("d%da" % l, a["c%d" % l], a["d%da" % l], N, r)
            self._conv("d%db" % l, a["d%da" % l], a["d%db" % l], N, r)
            h = a["d%db" % l]
        self._last = h
        _ck(self.lib.tpfnn_head(_p(h), N * RES * RES, W[0], _p(self.w["head"]), _p(self.b["head"]),
                                _p(self.pred), None, None, None, None, None, None, 0, self.stream), "head")
        return self.pred

    def _conv_bwd(self, name, x, y, gy, gx, N, r):
        """gy: gradient of the ReLU output y (modified in place); gx may be None."""
        cin = cout = None
        for n_, ci, co in self.layers:
            if n_ == name:
                cin, cout = ci, co
        lib, st = self.lib, self.stream
        _ck(lib.tpfnn_relu_bwd(_p(y), _p(gy), y.numel(), st), "relu_bwd")
        _ck(lib.tpfnn_conv3x3_wgrad(_p(x), _p(gy), N, r, r, cin, cout, _p(self.gw[name]), _p(self.gb[name]),
                                    _p(self.work), self.work.numel(), st), "wgrad " + name)
        if gx is not None:
            _ck(lib.tpfnn_weight_flip(_p(self.wb[name]), cout, cin, _p(self.wt[name]), st), "flip")
            _ck(lib.tpfnn_conv3x3_fwd(_p(gy), N, r, r, cout, _p(self.wt[name]), None, cin, 0, _p(gx), st),
                "dgrad " + name)

    def loss_and_grads(self, N, target):
        """Head loss against target (FP32 tensor [N*256*256]) and all gradients."""
        a, g = self.act, self.grad
        W = self.widths
        L = len(W)
        lib, st = self.lib, self.stream
        _ck(lib.tpfnn_head(_p(self._last), N * RES * RES, W[0], _p(self.w["head"]), _p(self.b["head"]),
                           _p(self.pred), _p(target), _p(g["d0b"]), _p(self.gw["head"]), _p(self.gb["head"]),
                           _p(self.loss), _p(self.work), self.work.numel(), st), "head")
        for l in range(0, L - 1):
            r = RES >> l
            self._conv_bwd("d%db" % l, a["d%da" % l], a["d%db" % l], g["d%db" % l], g["d%da" % l], N, r)
            self._conv_bwd("d%da" % l, a["c%d" % l], a["d%da" % l], g["d%da" % l], g["c%d" % l], N, r)
            _ck(lib.tpfnn_split(_p(g["c%d" % l]), W[l], W[l], N * r * r, _p(g["d%du" % l]), _p(g["skipg%d" % l]),
                                st), "split")
            self._conv_bwd("d%du" % l, a["u%d" % l], a["d%du" % l], g["d%du" % l], g["u%d" % l], N, r)
            nxt = "e%db" % (L - 1) if l == L - 2 else "d%db" % (l + 1)
            _ck(lib.tpfnn_upsample2_bwd(_p(g["u%d" % l]), N, r // 2, r // 2, W[l + 1], _p(g[nxt]), st), "up_bwd")
        for l in range(L - 1, -1, -1):
            r = RES >> l
            if l < L - 1:
                _ck(lib.tpfnn_add_inplace(_p(g["e%db" % l]), _p(g["skipg%d" % l]), g["e%db" % l].numel(), st),
                    "add")
            self._conv_bwd("e%db" % l, a["e%da" % l], a["e%db" % l], g["e%db" % l], g["e%da" % l], N, r)
            xin = a["in"] if l == 0 else a["p%d" % l]
            gin = None if l == 0 else g["p%d" % l]
            self._conv_bwd("e%da" % l, xin, a["e%da" % l], g["e%da" % l], gin, N, r)
            if l > 0:
                _ck(lib.tpfnn_avgpool2_bwd(_p(g["p%d" % l]), N, 2 * r, 2 * r, W[l - 1], _p(g["e%db" % (l - 1)]), st),
                    "pool_bwd")
        return self.loss

    def adam_step(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        lib, st = self.lib, self.stream
        for k in self.w:
            wb = self.wb.get(k)
            _ck(lib.tpfnn_adam(_p(self.w[k]), _p(self.m[k][0]), _p(self.v[k][0]), _p(self.gw[k]),
                               _p(wb) if wb is not None else None, self.w[k].numel(), lr, b1, b2, eps, self.t, st),
                "adam")
            _ck(lib.tpfnn_adam(_p(self.b[k]), _p(self.m[k][1]), _p(self.v[k][1]), _p(self.gb[k]), None,
                               self.b[k].numel(), lr, b1, b2, eps, self.t, st), "adam")

    def train_step(self, N, target, lr=1e-3):
        self.forward(N)
        loss = self.loss_and_grads(N, target)
        self.adam_step(lr)
        return loss

    def predict(self, phi0, theta_deg, vol, phi1_init=None) -> np.ndarray:
        """[N,256,256] prediction of phi1 (numpy float32)."""
        return self.predict_device(phi0, theta_deg, vol, phi1_init).cpu().numpy()

    def predict_device(self, phi0, theta_deg, vol, phi1_init=None):
        """[N,256,256] prediction of phi1 left on the device: a view of the
        network's output buffer, valid until its next forward pass (work
        queued on the same stream before that pass reads it in order)."""
        N = self.pack(phi0, theta_deg, vol, phi1_init)
        return self.forward(N).reshape(N, RES, RES)


# ---------------------------------------------------------------------------
# Data: resampling between domain grids and the 256 x 256 network grid
# ---------------------------------------------------------------------------
def resample(fields: np.ndarray, dh: int, dw: int, device="cuda:0") -> np.ndarray:
    """Bilinear resampling of [N,sh,sw] float fields on the GPU (corner-aligned)."""
    import torch
    lib = nnlib()
    src = torch.tensor(np.ascontiguousarray(fields, np.float32), device=device)
    N, sh, sw = fields.shape
    dst = torch.empty(N * dh * dw, dtype=torch.float32, device=device)
    st = V(torch.cuda.current_stream(torch.device(device)).cuda_stream)
    _ck(lib.tpfnn_resample(_p(src), N, sh, sw, _p(dst), dh, dw, st), "resample")
    return dst.reshape(N, dh, dw).cpu().numpy()


def volume_feature(phi1: np.ndarray) -> float:
    """Droplet size input: 10 x (sum of phi1)/(number of nodes)."""
    return 10.0 * float(np.sum(phi1)) / phi1.size


def warm_start_field(pred256: np.ndarray, phi0: np.ndarray, target_mass: float, device="cuda:0") -> np.ndarray:
    """Maps a 256 x 256 prediction to a domain on the GPU: bilinear resampling
    to its grid, then the mass projection phi1 = sigmoid(logit(p) + c)(1 - phi0)
    with the shift c that gives sum(phi1) = the droplet's mass.  Raises
    ValueError when the prediction is not finite or the mass is out of reach."""
    import torch
    lib = nnlib()
    ny, nx = phi0.shape
    if not np.isfinite(pred256).all():
        raise ValueError("non-finite prediction")
    dev = torch.device(device)
    st = V(torch.cuda.current_stream(dev).cuda_stream)
    src = torch.tensor(np.ascontiguousarray(pred256, np.float32), device=dev)
    p = torch.empty(ny * nx, dtype=torch.float32, device=dev)
    _ck(lib.tpfnn_resample(_p(src), 1, pred256.shape[0], pred256.shape[1], _p(p), ny, nx, st), "resample")
    t0 = torch.tensor(np.ascontiguousarray(phi0, np.float32).ravel(), device=dev)
    out = torch.empty(ny * nx, dtype=torch.float64, device=dev)
    info = torch.empty(2, dtype=torch.float64, device=dev)
    _ck(lib.tpfnn_mass_project(_p(p), _p(t0), ny * nx, float(target_mass), _p(out), _p(info), st), "mass_project")
    c = info.cpu().numpy()
    if not np.isfinite(c).all():
        raise ValueError("droplet mass out of reach of the prediction")
    return out.cpu().numpy().reshape(ny, nx)


def warm_start_fields(pred, phi0s: Sequence[np.ndarray], targets: Sequence[float]) -> List[Optional[np.ndarray]]:
    """warm_start_field for a batch of predictions already on the device
    ([N,256,256] FP32 tensor): resampling (skipped for 256 x 256 domains, where
    the corner-aligned map is the identity) and mass projection are queued for
    all N on the current stream and the fields come back in one transfer.
    None where the prediction is not finite or the mass is out of its reach."""
    import torch
    lib = nnlib()
    N = pred.shape[0]
    dev = pred.device
    st = V(torch.cuda.current_stream(dev).cuda_stream)
    flat = pred.reshape(N, RES * RES)
    finite = torch.isfinite(flat).all(dim=1).cpu().numpy()
    sizes = [f.shape for f in phi0s]
    offs = np.concatenate([[0], np.cumsum([h * w for h, w in sizes])])
    out = torch.zeros(int(offs[-1]), dtype=torch.float64, device=dev)
    info = torch.full((N, 2), float("nan"), dtype=torch.float64, device=dev)
    keep = []
    if all(sz == sizes[0] for sz in sizes):
        # equal sizes: one batched resampling (if needed) and one projection launch
        ny, nx = sizes[0]
        n = ny * nx
        if (ny, nx) != (RES, RES):
            p = torch.empty(N * n, dtype=torch.float32, device=dev)
            _ck(lib.tpfnn_resample(_p(flat), N, RES, RES, _p(p), ny, nx, st), "resample")
        else:
            p = flat
        t0 = torch.tensor(np.ascontiguousarray(np.stack(phi0s), np.float32), device=dev)
        tg = torch.tensor(np.where(finite, np.asarray(targets, np.float64), np.nan), device=dev)
        _ck(lib.tpfnn_mass_project_batch(_p(p), _p(t0), N, n, _p(tg), _p(out), _p(info), st), "mass_project_batch")
        keep.append((p, t0, tg))
    else:
        for d in range(N):
            if not finite[d]:
                continue
            ny, nx = sizes[d]
            n = ny * nx
            src = flat[d]
            if (ny, nx) != (RES, RES):
                p = torch.empty(n, dtype=torch.float32, device=dev)
                _ck(lib.tpfnn_resample(_p(src), 1, RES, RES, _p(p), ny, nx, st), "resample")
            else:
                p = src
            t0 = torch.tensor(np.ascontiguousarray(phi0s[d], np.float32).ravel(), device=dev)
            _ck(lib.tpfnn_mass_project(_p(p), _p(t0), n, float(targets[d]), _p(out[int(offs[d]):]), _p(info[d]),
                                       st), "mass_project")
            keep.append((p, t0))  # alive until the queued kernels ran
    fields = out.cpu().numpy()
    infos = info.cpu().numpy()
    del keep
    res: List[Optional[np.ndarray]] = []
    for d in range(N):
        ok = finite[d] and np.isfinite(infos[d]).all()
        res.append(fields[int(offs[d]):int(offs[d + 1])].reshape(sizes[d]).copy() if ok else None)
    return res


def time_layers(N: int, reps: int):
    """Forward 3x3 convolution of every layer of the network at batch N on
    random bf16 operands: microseconds per call (HIP events around reps
    back-to-back calls) and TFLOP/s (2 x 9 x Cin x Cout multiply-adds per
    output pixel); printed as one JSON line per layer."""
    import json
    import torch
    lib = nnlib()
    dev = torch.device("cuda")
    for name, cin, cout in layer_table():
        lev = int(name[1])
        r = RES >> lev
        x = torch.randn(N * r * r * cin, device=dev).to(torch.bfloat16)
        w = (torch.randn(cout * 9 * cin, device=dev) / math.sqrt(9 * cin)).to(torch.bfloat16)
        b = torch.zeros(cout, device=dev)
        y = torch.empty(N * r * r * cout, device=dev, dtype=torch.bfloat16)

        def call():
            _ck(lib.tpfnn_conv3x3_fwd(_p(x), N, r, r, cin, _p(w), _p(b), cout, 1, _p(y), None), "conv3x3_fwd")
        for _ in range(3):
            call()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            call()
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        fl = 2.0 * 9 * cin * cout * r * r * N
        print(json.dumps({"layer": name, "batch": N, "H": r, "W": r, "Cin": cin, "Cout": cout, "us": round(us, 2),
                          "tflops": round(fl / us / 1e6, 1), "frac_of_bf16_peak": round(fl / us / 1e6 / 2500.0, 4)}),
              flush=True)


def main(argv=None):
    """Times forward passes and training steps of the network on synthetic
    inputs (smooth random fields): ms per step and effective TFLOP/s, with
    3 x the forward multiply-adds counted per training sample."""
    import argparse
    import json
    import time
    import torch
    ap = argparse.ArgumentParser(description="surrogate throughput on synthetic inputs")
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--layers", action="store_true",
                    help="time the forward 3x3 convolution of every layer at this batch instead")
    args = ap.parse_args(argv)
    if args.layers:
        return time_layers(args.batch, max(args.steps, 5))
    rng = np.random.default_rng(0)
    N = args.batch
    yy, xx = np.mgrid[0:RES, 0:RES]
    phi0 = np.stack([0.5 - 0.5 * np.tanh((yy - 24 - 8 * np.sin(2 * np.pi * xx / RES + rng.uniform(0, 6))) / 2.0)
                     for _ in range(N)])
    phi1 = np.stack([(1 - phi0[i]) * (0.5 + 0.5 * np.tanh((50 - np.hypot(xx - 128, yy - 30)) / 2.0))
                     for i in range(N)])
    net = UNet(seed=0)
    net.pack(phi0, rng.uniform(30, 150, N), np.full(N, 0.6), phi1)
    tgt = torch.tensor(phi1.astype(np.float32).ravel(), device=net.dev)
    for _ in range(args.warmup):
        net.train_step(N, tgt, lr=1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        net.train_step(N, tgt, lr=1e-4)
    torch.cuda.synchronize()
    t_train = (time.perf_counter() - t0) / args.steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        net.forward(N)
    torch.cuda.synchronize()
    t_fwd = (time.perf_counter() - t0) / args.steps
    f = net.flops_per_sample()
    print(json.dumps({"batch": N, "train_ms": round(t_train * 1e3, 3), "forward_ms": round(t_fwd * 1e3, 3),
                      "train_tflops": round(3 * f * N / t_train / 1e12, 2),
                      "forward_tflops": round(f * N / t_fwd / 1e12, 2)}), flush=True)


if __name__ == "__main__":
    main()
