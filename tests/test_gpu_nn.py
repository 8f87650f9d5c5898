"""Parity of the surrogate's HIP kernels (BF16 matrix cores, FP32 accumulation)
with the FP64 numpy oracle, run on an MI355X.

Inputs are rounded to bf16 before both sides see them, so the oracle computes
the exact result of the same operands; the remaining differences are FP32
accumulation order and the final bf16 rounding of activations (relative
2^-8), which set the tolerances."""
import sys

import numpy as np
import pytest

from oracle import nn as O

pytestmark = pytest.mark.gpu
rng = np.random.default_rng(11)


def _say(*a):
    print("[case]", *a, flush=True)


def _torch():
    import torch
    return torch


# device tensors handed to the kernels as raw pointers must outlive the call:
# every helper keeps a reference here (cleared per test)
_KEEP = []


@pytest.fixture(autouse=True)
def _keep_alive():
    yield
    _torch().cuda.synchronize()
    _KEEP.clear()


def _bf16_dev(a):
    torch = _torch()
    bits = O.to_bf16_bits(a).view(np.int16)
    t = torch.tensor(bits, device="cuda").view(torch.bfloat16)
    _KEEP.append(t)
    return t


def _from_dev_bf16(t, shape):
    torch = _torch()
    bits = t.view(torch.int16).cpu().numpy().view(np.uint16)
    return O.from_bf16_bits(bits).reshape(shape)


def _f32_dev(a):
    t = _torch().tensor(np.asarray(a, np.float32), device="cuda")
    _KEEP.append(t)
    return t


def _lib():
    from paper_2311_05091_amd.surrogate import nnlib
    return nnlib()


def _p(t):
    import ctypes
    return ctypes.c_void_p(t.data_ptr())


def test_mfma_operand_layout():
    """Small integers are exact in bf16 and FP32: the 16x32 by 32x16 product must be exact."""
    _say("mfma selftest")
    torch = _torch()
    A = rng.integers(-4, 5, size=(16, 32)).astype(np.float32)
    B = rng.integers(-4, 5, size=(32, 16)).astype(np.float32)
    D = torch.zeros(256, dtype=torch.float32, device="cuda")
    assert _lib().tpfnn_mfma_selftest(_p(_bf16_dev(A)), _p(_bf16_dev(B)), _p(D), None) == 0
    assert np.array_equal(D.cpu().numpy().reshape(16, 16), A @ B)


@pytest.mark.parametrize("N,H,W,Cin,Cout,relu", [(2, 16, 16, 32, 32, 1), (1, 8, 16, 64, 128, 0),
                                                 (3, 32, 8, 96, 64, 1), (1, 16, 8, 256, 256, 1),
                                                 (3, 8, 8, 128, 128, 0), (8, 64, 64, 128, 128, 1),
                                                 (8, 64, 64, 256, 128, 1), (8, 32, 32, 256, 256, 1),
                                                 (2, 32, 32, 32, 384, 0), (1, 4, 256, 64, 64, 1),
                                                 (2, 16, 128, 32, 64, 1), (8, 128, 128, 32, 64, 1),
                                                 (16, 32, 32, 64, 256, 0), (12, 32, 32, 64, 256, 1)])
def test_conv_forward(N, H, W, Cin, Cout, relu):
    """Output channels that are a multiple of 64 take the patch-staging
    kernel where the width allows (W a multiple of 128, or 16, 32, 64 with
    the rows to fill 128 pixels): widths 16, 32, 64, 128 and 256 here, with
    256-pixel blocks at batch 8 (W = 64, 128) and 16 (W = 32) and 128-pixel
    blocks elsewhere (12 x 32 x 32 among them); the others (W = 8) take the
    K-step kernels."""
    _say("conv fwd", N, H, W, Cin, Cout)
    torch = _torch()
    x = O.bf16_round(rng.normal(size=(N, H, W, Cin)))
    w = O.bf16_round(rng.normal(size=(Cout, 3, 3, Cin)) / np.sqrt(9 * Cin))
    b = rng.normal(size=Cout).astype(np.float32).astype(np.float64)
    y = torch.empty(N * H * W * Cout, dtype=torch.bfloat16, device="cuda")
    rc = _lib().tpfnn_conv3x3_fwd(_p(_bf16_dev(x)), N, H, W, Cin, _p(_bf16_dev(w)), _p(_f32_dev(b)), Cout,
                                  relu, _p(y), None)
    assert rc == 0
    ref = O.conv3x3(x, w, b)
    if relu:
        ref = O.relu(ref)
    got = _from_dev_bf16(y, ref.shape)
    err = np.abs(got - ref)
    assert np.all(err <= 2 ** -8 * np.abs(ref) + 1e-5 * np.abs(ref).max())


@pytest.mark.parametrize("N,H,W,Cin,Cout", [(2, 16, 8, 64, 32), (4, 32, 32, 256, 128)])
def test_conv_input_gradient_via_flipped_weights(N, H, W, Cin, Cout):
    _say("dgrad", N, H, W, Cin, Cout)
    torch = _torch()
    dy = O.bf16_round(rng.normal(size=(N, H, W, Cout)))
    w = O.bf16_round(rng.normal(size=(Cout, 3, 3, Cin)) / np.sqrt(9 * Cin))
    wt = torch.empty(w.size, dtype=torch.bfloat16, device="cuda")
    dx = torch.empty(N * H * W * Cin, dtype=torch.bfloat16, device="cuda")
    lib = _lib()
    assert lib.tpfnn_weight_flip(_p(_bf16_dev(w)), Cout, Cin, _p(wt), None) == 0
    assert lib.tpfnn_conv3x3_fwd(_p(_bf16_dev(dy)), N, H, W, Cout, _p(wt), None, Cin, 0, _p(dx), None) == 0
    ref = O.conv3x3_dx(dy, w)
    got = _from_dev_bf16(dx, ref.shape)
    assert np.all(np.abs(got - ref) <= 2 ** -8 * np.abs(ref) + 1e-5 * np.abs(ref).max())


@pytest.mark.parametrize("N,H,W,Cin,Cout", [(2, 16, 16, 32, 64), (1, 32, 32, 64, 32), (4, 8, 8, 128, 256),
                                             (2, 8, 64, 32, 64), (1, 4, 32, 256, 256), (3, 16, 32, 32, 32),
                                             (2, 256, 256, 32, 32), (2, 64, 64, 128, 128)])
def test_conv_weight_gradient(N, H, W, Cin, Cout):
    """Rows of width a multiple of 32 take the nine-tap kernel, the others the
    per-tap one; both against the FP64 oracle."""
    _say("wgrad", N, H, W, Cin, Cout)
    torch = _torch()
    lib = _lib()
    x = O.bf16_round(rng.normal(size=(N, H, W, Cin)))
    dy = O.bf16_round(rng.normal(size=(N, H, W, Cout)))
    ws = lib.tpfnn_wgrad_workspace(N, H, W, Cin, Cout)
    work = torch.empty(int(ws), dtype=torch.uint8, device="cuda")
    dw = torch.empty(Cout * 9 * Cin, dtype=torch.float32, device="cuda")
    db = torch.empty(Cout, dtype=torch.float32, device="cuda")
    rc = lib.tpfnn_conv3x3_wgrad(_p(_bf16_dev(x)), _p(_bf16_dev(dy)), N, H, W, Cin, Cout, _p(dw), _p(db), _p(work),
                                 work.numel(), None)
    assert rc == 0
    ref = O.conv3x3_dw(x, dy)
    got = dw.cpu().numpy().reshape(ref.shape)
    scale = np.sqrt(N * H * W)
    assert np.abs(got - ref).max() <= 1e-5 * scale
    assert np.allclose(db.cpu().numpy(), dy.reshape(-1, Cout).sum(0), atol=1e-4 * scale)


def test_pool_upsample_concat_split_exact():
    _say("elementwise")
    torch = _torch()
    lib = _lib()
    N, H, W, C = 2, 8, 16, 32
    x = O.bf16_round(rng.normal(size=(N, H, W, C)))
    y = torch.empty(N * H * W * C // 4, dtype=torch.bfloat16, device="cuda")
    assert lib.tpfnn_avgpool2_fwd(_p(_bf16_dev(x)), N, H, W, C, _p(y), None) == 0
    ref = O.bf16_round(O.avgpool2(x))
    assert np.array_equal(_from_dev_bf16(y, ref.shape), ref)
    u = torch.empty(N * H * W * C, dtype=torch.bfloat16, device="cuda")
    assert lib.tpfnn_upsample2_fwd(_p(y), N, H // 2, W // 2, C, _p(u), None) == 0
    assert np.array_equal(_from_dev_bf16(u, x.shape), O.upsample2(ref))
    a = O.bf16_round(rng.normal(size=(N * H * W, 32)))
    b = O.bf16_round(rng.normal(size=(N * H * W, 64)))
    cat = torch.empty(N * H * W * 96, dtype=torch.bfloat16, device="cuda")
    assert lib.tpfnn_concat(_p(_bf16_dev(a)), 32, _p(_bf16_dev(b)), 64, N * H * W, _p(cat), None) == 0
    assert np.array_equal(_from_dev_bf16(cat, (N * H * W, 96)), np.concatenate([a, b], 1))
    da = torch.empty(N * H * W * 32, dtype=torch.bfloat16, device="cuda")
    dbb = torch.empty(N * H * W * 64, dtype=torch.bfloat16, device="cuda")
    assert lib.tpfnn_split(_p(cat), 32, 64, N * H * W, _p(da), _p(dbb), None) == 0
    assert np.array_equal(_from_dev_bf16(da, a.shape), a) and np.array_equal(_from_dev_bf16(dbb, b.shape), b)


def test_relu_backward_and_upsample_at_network_size():
    """The 16-byte paths of the ReLU mask and the upsampling against their
    definitions on a level-0 sized tensor."""
    _say("relu upsample large")
    torch = _torch()
    lib = _lib()
    N, H, W, C = 2, 128, 128, 64
    y = O.bf16_round(rng.normal(size=(N, 2 * H, 2 * W, C // 2)))
    g = O.bf16_round(rng.normal(size=y.shape))
    gd = _bf16_dev(g)
    assert lib.tpfnn_relu_bwd(_p(_bf16_dev(y)), _p(gd), y.size, None) == 0
    assert np.array_equal(_from_dev_bf16(gd, g.shape), np.where(y > 0, g, 0.0))
    x = O.bf16_round(rng.normal(size=(N, H, W, C)))
    u = torch.empty(N * 4 * H * W * C, dtype=torch.bfloat16, device="cuda")
    assert lib.tpfnn_upsample2_fwd(_p(_bf16_dev(x)), N, H, W, C, _p(u), None) == 0
    assert np.array_equal(_from_dev_bf16(u, (N, 2 * H, 2 * W, C)), O.upsample2(x))


def test_head_loss_and_gradients():
    _say("head")
    torch = _torch()
    lib = _lib()
    rng = np.random.default_rng(29)   # inputs independent of the other tests' draws
    npix, C = 4096, 32
    x = O.bf16_round(rng.normal(size=(npix, C)) * 0.5)
    w = rng.normal(size=C).astype(np.float32).astype(np.float64) * 0.3
    b = np.array([0.1], np.float32).astype(np.float64)
    t = rng.uniform(size=npix).astype(np.float32).astype(np.float64)
    pred = torch.empty(npix, dtype=torch.float32, device="cuda")
    dx = torch.empty(npix * C, dtype=torch.bfloat16, device="cuda")
    dw = torch.empty(C, dtype=torch.float32, device="cuda")
    db = torch.empty(1, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    ws = lib.tpfnn_head_workspace(npix, C)
    work = torch.empty(int(ws), dtype=torch.uint8, device="cuda")
    rc = lib.tpfnn_head(_p(_bf16_dev(x)), npix, C, _p(_f32_dev(w)), _p(_f32_dev(b)), _p(pred), _p(_f32_dev(t)),
                        _p(dx), _p(dw), _p(db), _p(loss), _p(work), work.numel(), None)
    assert rc == 0
    rp, rl, rdx, rdw, rdb = O.head(x, w, b[0], t)
    assert np.abs(pred.cpu().numpy() - rp).max() < 1e-6
    assert abs(loss.item() - rl) < 1e-5 * rl
    assert np.abs(dw.cpu().numpy() - rdw).max() < 1e-6 * np.abs(rdw).max() + 1e-9
    assert abs(db.item() - rdb) < 1e-6 * abs(rdb) + 1e-9
    got_dx = _from_dev_bf16(dx, rdx.shape)
    # bf16 rounding (unit roundoff 2^-8) of a value evaluated in FP32 (a few
    # FP32 ulps, covered by 2^-18)
    assert np.all(np.abs(got_dx - rdx) <= (2 ** -8 + 2 ** -18) * np.abs(rdx) + 1e-12)


def test_pack_input_channels():
    """Channel layout of the network input: phi0, scaled angle, volume, plain
    phi1, zeros; with no phi1 given, channel 3 is zero."""
    _say("pack")
    torch = _torch()
    lib = _lib()
    N, H, W = 2, 4, 8
    phi0 = rng.uniform(size=(N, H, W))
    phi1 = rng.uniform(size=(N, H, W))
    th, vol = np.array([30.0, 150.0]), np.array([0.5, 1.5])
    x = torch.empty(N * H * W * 32, dtype=torch.bfloat16, device="cuda")
    for with_phi1 in (True, False):
        p1 = _p(_f32_dev(phi1)) if with_phi1 else None
        assert lib.tpfnn_pack_input(_p(_f32_dev(phi0)), p1, _p(_f32_dev(th)), _p(_f32_dev(vol)), N, H, W,
                                    _p(x), None) == 0
        got = _from_dev_bf16(x, (N, H, W, 32))
        assert np.array_equal(got[..., 0], O.bf16_round(phi0.astype(np.float32)))
        assert np.array_equal(got[..., 1], O.bf16_round(((th - 90) / 60)[:, None, None] + 0 * phi0))
        assert np.array_equal(got[..., 2], O.bf16_round(vol[:, None, None] + 0 * phi0))
        want3 = O.bf16_round(phi1.astype(np.float32)) if with_phi1 else 0 * phi1
        assert np.array_equal(got[..., 3], want3)
        assert not got[..., 4:].any()


def test_mass_project_matches_oracle():
    """Warm-start projection: the kernel's field follows the FP64 oracle (FP32
    sigmoid), its sum is the target, and an unreachable target is reported."""
    _say("mass project")
    torch = _torch()
    lib = _lib()
    ny, nx = 217, 300
    yy, xx = np.mgrid[0:ny, 0:nx]
    phi0 = 0.5 - 0.5 * np.tanh((yy - 20.0) / 2.0)
    pred = np.clip(0.5 + 0.5 * np.tanh((60.0 - np.hypot(xx - 150, yy - 20)) / 3.0)
                   + 0.05 * rng.normal(size=(ny, nx)), 0.0, 1.0).astype(np.float32)
    phi0 = phi0.astype(np.float32).astype(np.float64)
    out = torch.empty(ny * nx, dtype=torch.float64, device="cuda")
    info = torch.empty(2, dtype=torch.float64, device="cuda")
    for target in (3000.0, 6000.0, 9000.0):
        rc = lib.tpfnn_mass_project(_p(_f32_dev(pred.ravel())), _p(_f32_dev(phi0.ravel())), ny * nx, target,
                                    _p(out), _p(info), None)
        assert rc == 0
        ref, c = O.mass_project(pred.astype(np.float64), phi0, target)
        got = out.cpu().numpy().reshape(ny, nx)
        ci = info.cpu().numpy()
        assert abs(ci[0] - c) < 1e-4 * max(1.0, abs(c))
        assert abs(got.sum() - target) < 1e-10 * target
        assert np.abs(got - ref).max() < 2e-5
    rc = lib.tpfnn_mass_project(_p(_f32_dev(pred.ravel())), _p(_f32_dev(phi0.ravel())), ny * nx,
                                float(ny * nx), _p(out), _p(info), None)
    assert rc == 0 and np.isnan(info.cpu().numpy()).all()


def test_adam_and_resample():
    _say("adam resample")
    torch = _torch()
    lib = _lib()
    n = 1000
    p, g = rng.normal(size=n), rng.normal(size=n)
    m, v = rng.normal(size=n) * 0.1, rng.uniform(size=n) * 0.1
    P, M, Vv, Gt = (_f32_dev(a) for a in (p, m, v, g))
    assert lib.tpfnn_adam(_p(P), _p(M), _p(Vv), _p(Gt), None, n, 1e-3, 0.9, 0.999, 1e-8, 5, None) == 0
    rp, rm, rv = O.adam(p.astype(np.float32).astype(np.float64), m.astype(np.float32), v.astype(np.float32),
                        g.astype(np.float32), 1e-3, 0.9, 0.999, 1e-8, 5)
    assert np.abs(P.cpu().numpy() - rp).max() < 1e-6
    src = rng.uniform(size=(3, 37, 53))
    from paper_2311_05091_amd.surrogate import resample
    got = resample(src, 64, 29)
    ref = O.resample(src.astype(np.float32).astype(np.float64), 64, 29)
    assert np.abs(got - ref).max() < 1e-5


def test_unet_forward_matches_oracle_and_gradients_are_consistent():
    """Whole network at 256 x 256: the GPU prediction follows the FP64 oracle
    (bf16 activations, so within a few percent), and the GPU gradient agrees
    with a central finite difference of the FP64 oracle's loss along a random
    direction in the weights of every layer."""
    from paper_2311_05091_amd.surrogate import UNet, init_params, RES
    _say("unet")
    torch = _torch()
    params = init_params(seed=5)
    # bf16-representable weights so both sides start from the same model
    params = {k: (O.bf16_round(w), b) for k, (w, b) in params.items()}
    net = UNet(params=params)
    N = 1
    phi0 = np.zeros((N, RES, RES))
    yy, xx = np.mgrid[0:RES, 0:RES]
    phi0[0] = 0.5 - 0.5 * np.tanh((yy - 40) / 2.0)
    target = (1 - phi0) * (0.5 + 0.5 * np.tanh((60 - np.hypot(xx - 128, yy - 40)) / 2.0))
    th, vol = np.array([70.0]), np.array([0.9])
    net.pack(phi0, th, vol)
    pred = net.forward(N).reshape(RES, RES).cpu().numpy()
    x = np.zeros((N, RES, RES, 32))
    x[..., 0] = O.bf16_round(phi0)
    x[..., 1] = O.bf16_round(np.full_like(phi0, (70.0 - 90.0) / 60.0))
    x[..., 2] = O.bf16_round(np.full_like(phi0, 0.9))
    acts = O.unet_forward(params, x)
    ref = O.head(acts["last"], *params["head"])[0]
    assert np.abs(pred - ref).max() < 3e-2
    tgt = _f32_dev(target.ravel())
    net.forward(N)
    loss = net.loss_and_grads(N, tgt).item()
    ref_loss = O.unet_loss(params, x, target)
    assert abs(loss / ref_loss - 1) < 3e-2
    # directional derivative along the GPU gradient itself: sum g.g against a
    # central finite difference of the FP64 oracle's loss along g (a wrong
    # gradient, or one with a wrong sign in some layer, misses the slope; the
    # bf16 activations leave a few per cent)
    d = {k: net.gw[k].cpu().numpy().astype(np.float64).reshape(np.shape(w)) for k, (w, b) in params.items()}
    gd = float(sum(np.sum(v * v) for v in d.values()))
    eps = 1e-3 / np.sqrt(gd)
    pp = {k: (w + eps * d[k], b) for k, (w, b) in params.items()}
    pm = {k: (w - eps * d[k], b) for k, (w, b) in params.items()}
    fd = (O.unet_loss(pp, x, target) - O.unet_loss(pm, x, target)) / (2 * eps)
    print("slope along the gradient: gpu %.6e fd %.6e" % (gd, fd))
    assert abs(gd - fd) <= 0.05 * abs(fd)


def test_training_reduces_loss():
    from paper_2311_05091_amd.surrogate import UNet, RES
    _say("train")
    torch = _torch()
    net = UNet(seed=1)
    N = 2
    yy, xx = np.mgrid[0:RES, 0:RES]
    phi0 = np.stack([0.5 - 0.5 * np.tanh((yy - h) / 2.0) for h in (30, 50)])
    target = np.stack([(1 - phi0[i]) * (0.5 + 0.5 * np.tanh((r - np.hypot(xx - 128, yy - h)) / 2.0))
                       for i, (h, r) in enumerate(((30, 50), (50, 70)))])
    net.pack(phi0, np.array([60.0, 120.0]), np.array([0.8, 1.2]))
    tgt = _f32_dev(target.ravel())

    def mse():
        return float(np.mean((net.forward(N).cpu().numpy().reshape(target.shape) - target) ** 2))

    mse0 = mse()
    # learning rate ramped up over the first 10 updates (no normalisation layers)
    losses = [net.train_step(N, tgt, lr=5e-4 * min(1.0, (k + 1) / 10)).item() for k in range(60)]
    assert np.isfinite(losses).all()
    assert losses[-1] < losses[0]
    assert mse() < 0.5 * mse0
