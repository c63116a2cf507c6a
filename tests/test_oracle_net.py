"""Pins of the oracle learned force correction (net.c): special cases that
reduce to a library routine or a closed form, the plain PM force when the
output layers are zero, and central finite differences of every reverse-mode
function (conv, radial table, the full force-matching loss)."""
import numpy as np
import pytest

import oracle as O
from paper_2007_13394_amd import inputs as I


def _rel(a, b):
    return abs(a - b) / max(abs(a), abs(b), 1e-300)


def _random_params(seed, scale_mlp=0.3, scale_cnn=0.15):
    rng = np.random.default_rng(seed)
    th = np.zeros(O.NET_NPARAM)
    for k, (o, n) in O.NET_OFF.items():
        fan = {"W0": 2, "W1": O.NET_H, "W2": O.NET_H, "W3": O.NET_H, "C1W": 27, "C2W": 27 * O.NET_C,
               "C3W": 27 * O.NET_C}.get(k, 1)
        s = (scale_mlp if k.startswith(("W", "B")) else scale_cnn) / np.sqrt(fan)
        th[o:o + n] = rng.standard_normal(n) * s
    return th


def test_single_tap_conv_is_a_periodic_shift():
    rng = np.random.default_rng(1)
    n = 8
    x = rng.standard_normal((1, n, n, n))
    for t in (0, 4, 13, 22, 26):
        W = np.zeros(27)
        W[t] = 1.0
        out = O.conv3(x, W, np.zeros(1))
        o = (t // 9 - 1, (t // 3) % 3 - 1, t % 3 - 1)
        ref = np.roll(x[0], shift=(-o[0], -o[1], -o[2]), axis=(0, 1, 2))
        assert np.array_equal(out[0], ref)


def test_conv_channel_mixing_and_bias():
    """Centre-tap weights mix channels pointwise: out = W x + b per voxel."""
    rng = np.random.default_rng(2)
    n, ci, co = 6, 3, 4
    x = rng.standard_normal((ci, n, n, n))
    Wm = rng.standard_normal((co, ci))
    W = np.zeros((co, ci, 27))
    W[:, :, 13] = Wm
    b = rng.standard_normal(co)
    out = O.conv3(x, W, b)
    ref = np.einsum("oi,ixyz->oxyz", Wm, x) + b[:, None, None, None]
    assert np.allclose(out, ref, rtol=0, atol=1e-13)


def test_conv_vjp_finite_differences():
    rng = np.random.default_rng(3)
    n, ci, co = 6, 4, 5
    x = rng.standard_normal((ci, n, n, n))
    W = rng.standard_normal(co * ci * 27)
    b = rng.standard_normal(co)
    G = rng.standard_normal((co, n, n, n))
    dx, dW, db = O.conv3_vjp(x, W, co, G)
    h = 1e-6
    for _ in range(3):
        vx, vW, vb = rng.standard_normal(x.shape), rng.standard_normal(W.shape), rng.standard_normal(b.shape)
        f = lambda s: np.sum(G * O.conv3(x + s * vx, W + s * vW, b + s * vb))  # noqa: E731
        fd = (f(h) - f(-h)) / (2 * h)
        assert _rel(fd, np.sum(dx * vx) + np.sum(dW * vW) + np.sum(db * vb)) < 1e-8


def test_table_closed_form_and_identity():
    th = np.zeros(O.NET_NPARAM)
    assert np.array_equal(O.net_table(th, 0.5), np.ones(O.NET_NB))
    # only the last hidden bias and the output layer: h = W3 . silu(b2) + b3
    rng = np.random.default_rng(4)
    o, n = O.NET_OFF["B2"]
    th[o:o + n] = rng.standard_normal(n)
    o3, n3 = O.NET_OFF["W3"]
    th[o3:o3 + n3] = rng.standard_normal(n3)
    th[O.NET_OFF["B3"][0]] = 0.25
    b2 = th[o:o + n]
    expect = 1.0 + th[o3:o3 + n3] @ (b2 / (1 + np.exp(-b2))) + 0.25
    assert np.allclose(O.net_table(th, 0.3), expect, rtol=1e-14, atol=0)
    assert abs(O.net_kt(O.NET_NB - 1) - np.sqrt(3.0)) < 1e-15


def test_table_vjp_finite_differences():
    rng = np.random.default_rng(5)
    th = _random_params(6)
    tbar = rng.standard_normal(O.NET_NB)
    d = O.net_table_vjp(th, 0.4, tbar)
    h = 1e-6
    for _ in range(3):
        v = rng.standard_normal(th.shape)
        fd = (np.sum(tbar * O.net_table(th + h * v, 0.4)) - np.sum(tbar * O.net_table(th - h * v, 0.4))) / (2 * h)
        assert _rel(fd, np.sum(d * v)) < 1e-8


def test_zero_output_layers_give_the_plain_force():
    cfg = I.config("C5_fd16")
    sim = O.make_sim(cfg)
    x32, _ = I.synthetic_state(cfg, seed=7)
    x = x32.astype(np.float64)
    th = _random_params(8)
    for k in ("W3", "B3", "C3W", "C3B"):
        o, n = O.NET_OFF[k]
        th[o:o + n] = 0.0
    acc = O.learned_force(sim, th, 0.5, x)
    ref = O.force_cont(sim, x)
    assert np.linalg.norm(acc - ref) / np.linalg.norm(ref) < 1e-12


@pytest.mark.parametrize("name", ["C5_fd16"])
def test_learned_loss_gradient_finite_differences(name):
    cfg = I.config(name)
    sim = O.make_sim(cfg)
    x32, _ = I.synthetic_state(cfg, seed=9)
    x = x32.astype(np.float64)
    rng = np.random.default_rng(10)
    th = _random_params(11)
    target = O.force_cont(sim, x) * (1.0 + 0.2 * rng.standard_normal(x.shape))
    a = 0.6
    loss, d = O.learned_loss(sim, th, a, x, target)
    assert loss > 0
    # Richardson-extrapolated central differences: O(h^4) truncation, and a
    # step large enough that the loss's roundoff stays ~1e-9 relative
    h = 1e-5

    def cd(v, hh):
        lp, _ = O.learned_loss(sim, th + hh * v, a, x, target, grad=False)
        lm, _ = O.learned_loss(sim, th - hh * v, a, x, target, grad=False)
        return (lp - lm) / (2 * hh)

    for part in ("W1", "C2W", "B0", "C1W", "C3W", None):
        v = np.zeros_like(th)
        if part is None:
            v = rng.standard_normal(th.shape)
        else:
            o, n = O.NET_OFF[part]
            v[o:o + n] = rng.standard_normal(n)
        fd = (4.0 * cd(v, h / 2) - cd(v, h)) / 3.0
        assert _rel(fd, np.sum(d * v)) < 1e-7, part


def test_mlp_hidden_layers_closed_form_through_silu_pairs():
    """silu(z) - silu(-z) = z for every z, so two hidden units fed +z and -z,
    read with weights +1 and -1 by the next layer, pass z through exactly.
    Chaining such pairs through all three hidden layers at unrelated unit
    indices makes the MLP the affine map h = c0 + c1 kt + c2 a.  A transposed
    weight matrix, swapped inputs (kt, a), a misplaced bias or a dropped
    layer breaks the identity."""
    H = O.NET_H
    th = np.zeros(O.NET_NPARAM)
    W0, B0 = O.NET_OFF["W0"][0], O.NET_OFF["B0"][0]
    W1, B1 = O.NET_OFF["W1"][0], O.NET_OFF["B1"][0]
    W2, B2 = O.NET_OFF["W2"][0], O.NET_OFF["B2"][0]
    W3, B3 = O.NET_OFF["W3"][0], O.NET_OFF["B3"][0]
    c1, c2, c0 = 0.37, -1.9, 0.125
    u0, v0 = 3, 70        # layer-0 pair: z0 = c1 kt + c2 a + c0
    u1, v1 = 11, 40       # layer-1 pair: z1 = 2 z0 - 0.5
    u2, v2 = 90, 5        # layer-2 pair: z2 = -z1 + 0.25
    for j, sg in ((u0, 1.0), (v0, -1.0)):
        th[W0 + j * 2 + 0] = sg * c1
        th[W0 + j * 2 + 1] = sg * c2
        th[B0 + j] = sg * c0
    for j, sg in ((u1, 1.0), (v1, -1.0)):
        th[W1 + j * H + u0] = sg * 2.0
        th[W1 + j * H + v0] = -sg * 2.0
        th[B1 + j] = -sg * 0.5
    for j, sg in ((u2, 1.0), (v2, -1.0)):
        th[W2 + j * H + u1] = -sg
        th[W2 + j * H + v1] = sg
        th[B2 + j] = sg * 0.25
    th[W3 + u2], th[W3 + v2], th[B3] = 3.0, -3.0, -0.75
    for a in (0.05, 0.4, 1.0):
        kt = np.array([O.net_kt(b) for b in range(O.NET_NB)])
        z0 = c1 * kt + c2 * a + c0
        z2 = -(2 * z0 - 0.5) + 0.25
        expect = 1.0 + 3.0 * z2 - 0.75
        assert np.allclose(O.net_table(th, a), expect, rtol=0, atol=1e-13)
