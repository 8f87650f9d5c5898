"""Pins of the surrogate's FP64 oracle (oracle/nn.py) against mathematics:
adjoint identities, finite differences, exact bf16 rounding of known values,
and exactness of bilinear resampling on linear fields."""
import numpy as np
import pytest

from oracle import nn as O

rng = np.random.default_rng(7)


def test_bf16_rounding_known_values():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -2.5, 3.0e38, 1e-40], np.float32)
    r = O.bf16_round(x)
    # 1 + 2^-8 is a tie -> even (1.0); 1 + 3*2^-8 is a tie -> even (1 + 2^-6)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -7 and r[3] == 1.0 + 2 ** -6
    assert r[4] == -2.5
    assert np.array_equal(O.from_bf16_bits(O.to_bf16_bits(x)), r)


def test_conv_adjoints():
    """<conv(x, w), y> = <x, conv_dx(y, w)> = <w, conv_dw(x, y)> (no bias)."""
    x = rng.normal(size=(2, 8, 6, 5))
    w = rng.normal(size=(4, 3, 3, 5))
    y = rng.normal(size=(2, 8, 6, 4))
    a = np.sum(O.conv3x3(x, w) * y)
    assert abs(a - np.sum(x * O.conv3x3_dx(y, w))) < 1e-10 * abs(a)
    assert abs(a - np.sum(w * O.conv3x3_dw(x, y))) < 1e-10 * abs(a)


def test_conv_single_tap_is_shift():
    """A weight with only the centre tap is a 1x1 channel mix; a corner tap shifts."""
    x = rng.normal(size=(1, 5, 5, 2))
    w = np.zeros((1, 3, 3, 2))
    w[0, 0, 0, 1] = 1.0  # ky = kx = 0 reads x[h-1, w-1]
    y = O.conv3x3(x, w)
    assert np.allclose(y[0, 1:, 1:, 0], x[0, :-1, :-1, 1]) and np.all(y[0, 0, :, 0] == 0)


def test_pool_upsample_adjoints():
    x = rng.normal(size=(2, 8, 4, 3))
    y = rng.normal(size=(2, 4, 2, 3))
    assert abs(np.sum(O.avgpool2(x) * y) - np.sum(x * O.avgpool2_dx(y))) < 1e-12
    z = rng.normal(size=(2, 8, 4, 3))
    assert abs(np.sum(O.upsample2(y) * z) - np.sum(y * O.upsample2_dx(z))) < 1e-12


def test_head_gradients_finite_difference():
    x = rng.normal(size=(2, 4, 4, 3))
    w = rng.normal(size=3)
    b = 0.3
    t = rng.uniform(size=(2, 4, 4))
    pred, loss, dx, dw, db = O.head(x, w, b, t)
    eps = 1e-6
    for i in range(3):
        e = np.zeros(3)
        e[i] = eps
        num = (O.head(x, w + e, b, t)[1] - O.head(x, w - e, b, t)[1]) / (2 * eps)
        assert abs(num - dw[i]) < 1e-7
    num = (O.head(x, w, b + eps, t)[1] - O.head(x, w, b - eps, t)[1]) / (2 * eps)
    assert abs(num - db) < 1e-7
    e = np.zeros_like(x)
    e[1, 2, 3, 1] = eps
    num = (O.head(x + e, w, b, t)[1] - O.head(x - e, w, b, t)[1]) / (2 * eps)
    assert abs(num - dx[1, 2, 3, 1]) < 1e-7


def test_head_loss_is_cross_entropy():
    """With x = 0 the logit is the bias: the loss is -t log p - (1 - t) log(1 - p),
    p = 1/(1 + e^-b), written out in logarithms of probabilities; large logits
    of the right sign give a vanishing loss."""
    t = np.array([[[0.0, 0.25], [0.5, 1.0]]])
    x = np.zeros((1, 2, 2, 3))
    for b in (-3.0, 0.0, 0.7, 4.0):
        p = np.exp(b) / (np.exp(b) + 1.0)
        want = np.mean(-t * np.log(p) - (1 - t) * np.log(1 - p))
        assert abs(O.head(x, np.ones(3), b, t)[1] - want) < 1e-12
    tt = np.array([[[0.0, 1.0]]])
    xx = np.array([[[[-40.0], [40.0]]]])
    assert O.head(xx, np.ones(1), 0.0, tt)[1] < 1e-16


def test_adam_first_step_is_sign_step():
    """With bias correction the first Adam step is lr * g/(|g| + eps)."""
    p = rng.normal(size=10)
    g = rng.normal(size=10)
    p1, m, v = O.adam(p, 0 * p, 0 * p, g, 1e-3, 0.9, 0.999, 1e-8, 1)
    assert np.allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), atol=1e-12)


def test_resample_exact_on_linear_fields():
    sh, sw = 7, 9
    yy, xx = np.mgrid[0:sh, 0:sw].astype(float)
    f = (2.0 * yy / (sh - 1) - 0.5 * xx / (sw - 1) + 0.25)[None]
    g = O.resample(f, 13, 5)
    Y, X = np.mgrid[0:13, 0:5].astype(float)
    assert np.allclose(g[0], 2.0 * Y / 12 - 0.5 * X / 4 + 0.25, atol=1e-12)
    assert np.array_equal(O.resample(f, sh, sw), f)


def test_unet_forward_shapes_and_range():
    from paper_2311_05091_amd.surrogate import init_params
    widths = (4, 8)
    params = init_params(widths=widths, seed=3)
    x = rng.uniform(size=(1, 16, 16, 32)) * (np.arange(32) < 3)
    acts = O.unet_forward(params, x, widths)
    assert acts["e1b"].shape == (1, 8, 8, 8) and acts["last"].shape == (1, 16, 16, 4)
    pred = O.head(acts["last"], *params["head"])
    assert pred.shape == (1, 16, 16) and np.all((pred > 0) & (pred < 1))


def test_mass_project_recovers_a_known_shift():
    """A prediction sigmoid(z0) and the mass of sigmoid(z0 + c0)(1 - phi0) as the
    target: the projection returns c0 and that field; the field stays in
    [0, 1 - phi0]; a target equal to the unshifted mass gives c = 0."""
    z0 = rng.normal(size=(20, 30)) * 3.0
    phi0 = rng.uniform(size=(20, 30)) * (rng.uniform(size=(20, 30)) < 0.3)
    pred = 1.0 / (1.0 + np.exp(-z0))
    for c0 in (-2.5, 0.0, 0.7):
        want = (1.0 - phi0) / (1.0 + np.exp(-(z0 + c0)))
        f, c = O.mass_project(pred, phi0, want.sum())
        assert abs(c - c0) < 1e-9
        assert np.abs(f - want).max() < 1e-9
        assert abs(f.sum() - want.sum()) < 1e-9 * want.sum()
        assert np.all(f >= 0) and np.all(f <= 1.0 - phi0 + 1e-15)
    with pytest.raises(ValueError):
        O.mass_project(pred, phi0, 2.0 * np.sum(1.0 - phi0))


def test_avgpool_of_constant_and_ramp_fields():
    """2x2 average pooling keeps a constant field (a sum-pool would scale it
    by 4) and maps a ramp x to the mean of each pair, x + 1/2."""
    c = np.full((1, 6, 8, 3), 2.5)
    assert np.array_equal(O.avgpool2(c), np.full((1, 3, 4, 3), 2.5))
    ramp = np.tile(np.arange(8.0)[None, None, :, None], (2, 4, 1, 1))
    pooled = O.avgpool2(ramp)
    assert np.allclose(pooled[..., 0], np.arange(0, 8, 2)[None, None, :] + 0.5)


@pytest.mark.parametrize("t_end", [2, 5])
def test_adam_constant_gradient_closed_form(t_end):
    """Under a constant gradient g the bias-corrected moments are exactly g and
    g^2 at every step t, so each step moves by lr g/(|g| + eps): after t
    steps p = p0 - t lr g/(|g| + eps).  A bias correction with the wrong power
    of beta breaks this from t = 2 on."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p0 = np.array([1.0, -1.0, 0.5, 2.0])
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    p, m, v = p0.copy(), np.zeros(4), np.zeros(4)
    for t in range(1, t_end + 1):
        p, m, v = O.adam(p, m, v, g, lr, b1, b2, eps, t)
    expect = p0 - t_end * lr * g / (np.abs(g) + eps)
    assert np.allclose(p, expect, rtol=0, atol=1e-12)


def test_unet_wiring_with_hand_set_weights():
    """A two-level network of one channel per layer whose convolutions are the
    centre tap (identity) except the decoder's first convolution after the
    concatenation, which weighs the upsampled path by a and the skip by b:
    for a non-negative input x (ReLU passes) the last activation is
    a upsample(avgpool(x)) + b x, and the head with weight 1 and bias -0.3
    gives sigmoid of that minus 0.3.  Pins the order of pooling, upsampling,
    concatenation (upsampled path first) and which skip joins which level."""
    rng2 = np.random.default_rng(3)
    x = rng2.uniform(0.0, 1.0, size=(2, 8, 8, 1))

    def ident(cin=1):
        w = np.zeros((1, 3, 3, cin))
        w[0, 1, 1, 0] = 1.0
        return w, np.zeros(1)
    a, b = 0.7, 0.2
    wcat = np.zeros((1, 3, 3, 2))
    wcat[0, 1, 1, 0], wcat[0, 1, 1, 1] = a, b
    params = {"e0a": ident(), "e0b": ident(), "e1a": ident(), "e1b": ident(), "d0u": ident(),
              "d0a": (wcat, np.zeros(1)), "d0b": ident(), "head": (np.ones(1), -0.3)}
    acts = O.unet_forward(params, x, widths=(1, 1))
    expect = a * O.upsample2(O.avgpool2(x)) + b * x
    assert np.allclose(acts["last"], expect, atol=1e-14)
    pred = O.head(acts["last"], *params["head"])
    assert np.allclose(pred, 1.0 / (1.0 + np.exp(-(expect[..., 0] - 0.3))), atol=1e-14)
