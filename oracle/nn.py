"""Plain FP64 numpy oracle of the learned warm start's building blocks.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Written from the
definitions, not for speed: NHWC tensors, 3x3 convolutions with zero
padding as a sum over the nine taps, their adjoints, 2x2 average pooling,
nearest upsampling, the sigmoid output head with the binary cross-entropy, Adam,
bilinear resampling, the mass projection of the warm start and the encoder-decoder assembled from them.  Shares no
code with the HIP kernels.
"""
from __future__ import annotations

import numpy as np


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round FP32 values to bfloat16 (nearest even) and return them as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def to_bf16_bits(a: np.ndarray) -> np.ndarray:
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def from_bf16_bits(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint32) << 16).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# convolution and its adjoints
# ---------------------------------------------------------------------------
def conv3x3(x, w, b=None):
    """y[n,h,w,co] = b[co] + sum_{ky,kx,ci} w[co,ky,kx,ci] x[n,h+ky-1,w+kx-1,ci]."""
    N, H, W, _ = x.shape
    Cout = w.shape[0]
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    y = np.zeros((N, H, W, Cout))
    for ky in range(3):
        for kx in range(3):
            y += xp[:, ky:ky + H, kx:kx + W, :] @ w[:, ky, kx, :].T
    if b is not None:
        y += b
    return y


def conv3x3_dx(dy, w):
    """Adjoint in x: dx[n,h,w,ci] = sum dy[n,h-ky+1,w-kx+1,co] w[co,ky,kx,ci]."""
    N, H, W, _ = dy.shape
    Cin = w.shape[3]
    dx = np.zeros((N, H + 2, W + 2, Cin))
    for ky in range(3):
        for kx in range(3):
            dx[:, ky:ky + H, kx:kx + W, :] += dy @ w[:, ky, kx, :]
    return dx[:, 1:H + 1, 1:W + 1, :]


def conv3x3_dw(x, dy):
    """Adjoint in w: dw[co,ky,kx,ci] = sum_{n,h,w} dy[n,h,w,co] x[n,h+ky-1,w+kx-1,ci]."""
    N, H, W, Cin = x.shape
    Cout = dy.shape[3]
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dw = np.zeros((Cout, 3, 3, Cin))
    d2 = dy.reshape(-1, Cout)
    for ky in range(3):
        for kx in range(3):
            dw[:, ky, kx, :] = d2.T @ xp[:, ky:ky + H, kx:kx + W, :].reshape(-1, Cin)
    return dw


def relu(x):
    return np.maximum(x, 0.0)


def avgpool2(x):
    N, H, W, C = x.shape
    return x.reshape(N, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def avgpool2_dx(dy):
    return 0.25 * np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2)


def upsample2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def upsample2_dx(dy):
    N, H, W, C = dy.shape
    return dy.reshape(N, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def head(x, w, b, target=None):
    """pred = sigmoid(z), z = b + x.w; with a target in [0, 1] also the mean
    binary cross-entropy loss = mean(softplus(z) - target z) and its gradients
    (dz = (pred - target)/npix)."""
    z = x @ w + b
    pred = 1.0 / (1.0 + np.exp(-z))
    if target is None:
        return pred
    npix = pred.size
    loss = float(np.mean(np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z))) - target * z))
    dz = (pred - target) / npix
    dx = dz[..., None] * w
    dw = (x * dz[..., None]).reshape(-1, x.shape[-1]).sum(0)
    db = float(dz.sum())
    return pred, loss, dx, dw, db


def adam(p, m, v, g, lr, b1, b2, eps, t):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    p = p - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
    return p, m, v


def resample(src, dh, dw):
    """Bilinear resampling [N,sh,sw] -> [N,dh,dw]; corner nodes map onto corner nodes."""
    N, sh, sw = src.shape
    fy = np.arange(dh) * ((sh - 1) / (dh - 1) if dh > 1 else 0.0)
    fx = np.arange(dw) * ((sw - 1) / (dw - 1) if dw > 1 else 0.0)
    y0 = np.clip(np.floor(fy).astype(int), 0, sh - 1)
    x0 = np.clip(np.floor(fx).astype(int), 0, sw - 1)
    y1 = np.minimum(y0 + 1, sh - 1)
    x1 = np.minimum(x0 + 1, sw - 1)
    ty = (fy - y0)[None, :, None]
    tx = (fx - x0)[None, None, :]
    a = src[:, y0][:, :, x0]
    b = src[:, y0][:, :, x1]
    c = src[:, y1][:, :, x0]
    d = src[:, y1][:, :, x1]
    return (1 - ty) * ((1 - tx) * a + tx * b) + ty * ((1 - tx) * c + tx * d)


def mass_project(pred, phi0, target, clip=1e-7):
    """Warm-start projection: phi1 = sigmoid(logit(p) + c) (1 - phi0), p = pred
    clipped to [clip, 1 - clip], with the scalar shift c chosen by bisection so
    that sum(phi1) = target (the sum increases monotonically with c).  Returns
    (phi1, c)."""
    p = np.clip(np.asarray(pred, np.float64), clip, 1.0 - clip)
    z = np.log(p) - np.log1p(-p)
    w = 1.0 - np.asarray(phi0, np.float64)

    def mass(c):
        return float(np.sum(w / (1.0 + np.exp(-(z + c)))))

    lo, hi = -40.0, 40.0
    if not (mass(lo) < target < mass(hi)):
        raise ValueError("target mass out of reach")
    for _ in range(200):
        c = 0.5 * (lo + hi)
        if c in (lo, hi):
            break
        if mass(c) < target:
            lo = c
        else:
            hi = c
    c = 0.5 * (lo + hi)
    return w / (1.0 + np.exp(-(z + c))), c


# ---------------------------------------------------------------------------
# encoder-decoder (same wiring as the GPU network)
# ---------------------------------------------------------------------------
def unet_forward(params, x, widths=(32, 64, 128, 256)):
    """Forward pass keeping every activation; params[name] = (w, b)."""
    acts = {"in": x}
    h = x
    skips = []
    L = len(widths)
    for l in range(L):
        if l > 0:
            h = avgpool2(h)
        h = relu(conv3x3(h, *params["e%da" % l]))
        acts["e%da" % l] = h
        h = relu(conv3x3(h, *params["e%db" % l]))
        acts["e%db" % l] = h
        skips.append(h)
    for l in range(L - 2, -1, -1):
        h = upsample2(h)
        h = relu(conv3x3(h, *params["d%du" % l]))
        acts["d%du" % l] = h
        h = np.concatenate([h, skips[l]], axis=-1)
        h = relu(conv3x3(h, *params["d%da" % l]))
        acts["d%da" % l] = h
        h = relu(conv3x3(h, *params["d%db" % l]))
        acts["d%db" % l] = h
    acts["last"] = h
    return acts


def unet_loss(params, x, target, widths=(32, 64, 128, 256)):
    acts = unet_forward(params, x, widths)
    wh, bh = params["head"]
    pred, loss, *_ = head(acts["last"], wh, bh, target)
    return loss
