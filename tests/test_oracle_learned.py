"""Pins of the learned-predictor oracle (``oracle.learned``) against facts that
do not come from the oracle itself: the plain 5/3 lifting (pinned to the
paper's matrix A and F(4,4) taps elsewhere), closed forms of special
networks written with numpy's own reflect padding, finite differences of
the loss, and the first Adam step's closed form."""
import math

import numpy as np
import pytest

from oracle import dwt53
from oracle import learned as L


def one_tap_net(j, w2=1, b2=-128, shift=0, b1=128):
    """Hidden unit 0 reads context j alone: h0 = c_j + b1 (>= 0 for b1 = 128)."""
    w1 = np.zeros((16, 8), np.int64)
    w1[0, j] = 1
    b1v = np.zeros(16, np.int64)
    b1v[0] = b1
    w2v = np.zeros(16, np.int64)
    w2v[0] = w2
    return L.Predictor(w1, b1v, w2v, b2, shift)


def reflect(x, pad):
    """numpy's whole-sample ('reflect') extension along the last axis."""
    return np.pad(x, [(0, 0)] * (x.ndim - 1) + [(pad, pad)], mode="reflect")


def rand_net(rng, scale=128, bias=4000, shift=None):
    return L.Predictor(rng.integers(-scale, scale, (16, 8)), rng.integers(-bias, bias, 16),
                       rng.integers(-scale, scale, 16), int(rng.integers(-bias, bias)),
                       int(rng.integers(4, 14)) if shift is None else shift)


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_zero_network_is_plain_53(levels):
    rng = np.random.default_rng(5)
    for h in (1, 2, 3, 7, 16, 33):
        for w in (1, 2, 5, 9, 32):
            a = rng.integers(0, 256, (h, w))
            ll0, det0 = L.fwd_multilevel(a, levels, L.Predictor.zero())
            ll1, det1 = dwt53.fwd_multilevel(a, levels)
            assert np.array_equal(ll0, ll1)
            for x, y in zip(det0, det1):
                for b0, b1 in zip(x, y):
                    assert np.array_equal(b0, b1)


@pytest.mark.parametrize("j", range(8))
def test_one_tap_network_is_a_difference_filter(j):
    """corr = x(i + o_j) - base, so d(i) = x(i) - x(m(i + o_j)) when every
    difference is inside the int8 context range."""
    rng = np.random.default_rng(10 + j)
    n = 40
    x = rng.integers(100, 160, (3, n))       # |x - base| < 64: no clamping
    y = L.fwd_1d(x, one_tap_net(j))
    ext = reflect(x, 8)
    odd = np.arange(1, n, 2)
    d = x[:, odd] - ext[:, odd + 8 + L.OFFSETS[j]]
    assert np.array_equal(y[:, (n + 1) // 2:], d)
    # update of eq. (5.2) on those highs, neighbours mirrored
    dfull = np.zeros_like(x)
    dfull[:, odd] = d
    de = reflect(dfull, 1)
    even = np.arange(0, n, 2)
    s = x[:, even] + ((de[:, even] + de[:, even + 2] + 2) // 4)
    assert np.array_equal(y[:, :(n + 1) // 2], s)


def test_context_clamp_relu_floor_and_saturation():
    rng = np.random.default_rng(3)
    x = rng.integers(0, 256, (4, 64))       # large jumps: contexts clamp
    ext = reflect(x, 8)
    odd = np.arange(1, 64, 2)
    base = (ext[:, odd + 7] + ext[:, odd + 9]) // 2
    raw = ext[:, odd + 8 + 3] - base           # offset +3 is context 5
    highs = lambda net: L.fwd_1d(x, net)[:, 32:]
    # clamp to the int8 range
    assert np.array_equal(highs(one_tap_net(5)), x[:, odd] - base - np.clip(raw, -128, 127))
    # ReLU: b1 = 0 keeps the positive part only
    assert np.array_equal(highs(one_tap_net(5, b1=0, b2=0)),
                          x[:, odd] - base - np.maximum(np.clip(raw, -128, 127), 0))
    # floor division by 2^shift (towards minus infinity, not zero)
    want = np.floor(3 * (np.clip(raw, -128, 127) + 128 - 128) / 4.0).astype(np.int64)
    assert np.array_equal(highs(one_tap_net(5, w2=3, b2=-384, shift=2)), x[:, odd] - base - want)
    # correction saturates at +-255
    big = np.clip(2 * np.clip(raw, -128, 127), -255, 255)
    assert np.array_equal(highs(one_tap_net(5, w2=2, b2=-256)), x[:, odd] - base - big)


def test_constant_correction_shifts_bands():
    """W1 = 0, b1 = 2c0 on one unit, W2 = 1, shift 1: corr = c0 everywhere;
    highs drop by c0 and, for even c0, lows by c0 / 2 (eq. (5.2) is affine
    in the highs)."""
    rng = np.random.default_rng(4)
    for c0 in (-20, 6, 100):
        net = L.Predictor(np.zeros((16, 8)), [max(2 * c0, 0)] + [0] * 15, [1] + [0] * 15,
                          min(2 * c0, 0), 1)
        x = rng.integers(0, 256, (5, 27))
        y, y0 = L.fwd_1d(x, net), dwt53.fwd_1d(x)
        assert np.array_equal(y[:, 14:], y0[:, 14:] - c0)
        assert np.array_equal(y[:, :14], y0[:, :14] - c0 // 2)


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_roundtrip_random_networks(levels):
    rng = np.random.default_rng(20 + levels)
    for shape in ((1, 1), (1, 9), (9, 1), (2, 2), (13, 17), (32, 24), (40, 65)):
        for _ in range(3):
            net = rand_net(rng)
            a = rng.integers(0, 256, shape)
            ll, det = L.fwd_multilevel(a, levels, net)
            assert np.array_equal(L.inv_multilevel(ll, det, net), a)


def test_inverse_of_arbitrary_coefficients():
    """Restore side: any integer bands invert back through the forward."""
    rng = np.random.default_rng(7)
    net = rand_net(rng)
    y = rng.integers(-30000, 30000, (6, 31))
    assert np.array_equal(L.fwd_1d(L.inv_1d(y, net), net), y)


def test_int16_bound_holds_and_fits():
    assert L.int16_bound(3) < 2 ** 15
    assert L.int16_bound(4) >= 2 ** 15          # why levels stop at 3
    rng = np.random.default_rng(8)
    worst = 0
    for _ in range(6):
        net = rand_net(rng, bias=2 ** 16, shift=0)      # corrections saturate
        a = np.where(rng.random((48, 48)) < 0.5, 0, 255)
        ll, det = L.fwd_multilevel(a, 3, net)
        worst = max(worst, np.abs(ll).max(), *(np.abs(b).max() for lv in det for b in lv))
    assert worst <= L.int16_bound(3)


def test_levels_limited():
    with pytest.raises(ValueError):
        L.fwd_multilevel(np.zeros((8, 8)), 4, L.Predictor.zero())


def test_blob_roundtrip_and_range_checks():
    rng = np.random.default_rng(9)
    net = rand_net(rng)
    blob = net.to_bytes()
    assert len(blob) == 216
    back = L.Predictor.from_bytes(blob)
    assert np.array_equal(back.w1, net.w1) and np.array_equal(back.w2, net.w2)
    assert np.array_equal(back.b1, net.b1) and (back.b2, back.shift) == (net.b2, net.shift)
    with pytest.raises(ValueError):
        L.Predictor(np.full((16, 8), 128), np.zeros(16), np.zeros(16), 0, 0)
    with pytest.raises(ValueError):
        L.Predictor(np.zeros((16, 8)), np.zeros(16), np.zeros(16), 0, 31)


def test_entropy_closed_forms():
    assert L.entropy_bits([]) == 0.0
    assert L.entropy_bits([5] * 10) == 0.0
    assert L.entropy_bits(np.arange(256)) == pytest.approx(8.0)
    assert L.entropy_bits([0, 0, 0, 1]) == pytest.approx(-(0.75 * math.log2(0.75) + 0.25 * math.log2(0.25)))


def test_training_pairs_targets_are_plain_highs():
    rng = np.random.default_rng(11)
    a = rng.integers(0, 256, (21, 30))
    ctx, t = L.training_pairs(a, 2)
    want, ll = [], a
    for _ in range(2):
        h, w = ll.shape
        rows = dwt53.fwd_1d(ll)
        want.append(rows[:, (w + 1) // 2:].reshape(-1))
        cols = dwt53.fwd_1d(rows.T)
        want.append(cols[:, (h + 1) // 2:].reshape(-1))
        ll = cols.T[:(h + 1) // 2, :(w + 1) // 2]
    assert np.array_equal(t, np.concatenate(want))
    assert ctx.shape == (t.size, 8) and ctx.min() >= -128 and ctx.max() <= 127


def test_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(12)
    ctx = rng.integers(-128, 128, (300, 8))
    t = rng.integers(-60, 60, 300)
    theta = rng.normal(0, 0.1, L.N_PARAMS)
    theta[128:144] += 0.3
    _, g = L.loss_grad(theta, ctx, t)
    eps = 1e-6
    for k in rng.choice(L.N_PARAMS, 40, replace=False):
        e = np.zeros(L.N_PARAMS)
        e[k] = eps
        fd = (L.loss_grad(theta + e, ctx, t)[0] - L.loss_grad(theta - e, ctx, t)[0]) / (2 * eps)
        assert fd == pytest.approx(g[k], rel=1e-4, abs=1e-7)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(13)
    theta, g = rng.normal(size=20), rng.normal(size=20)
    new, m, v = L.adam_step(theta, g, np.zeros(20), np.zeros(20), 1, 0.01, eps=0.0)
    assert np.allclose(new, theta - 0.01 * np.sign(g))
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_pow2_exponent_definition():
    for m in (1e-9, 0.0123, 0.5, 1.0, 0.99609375, 127.0, 127.5, 1000.0):
        k = L.pow2_exponent(m)
        assert m * 2.0 ** k < 127.5 and (k == 30 or m * 2.0 ** (k + 1) >= 127.5)
    assert L.pow2_exponent(0.0) == 30


def test_quantized_network_tracks_float_network():
    rng = np.random.default_rng(14)
    theta = rng.normal(0, 0.05, L.N_PARAMS).astype(np.float32)
    net = L.quantize(theta)
    ctx = rng.integers(-128, 128, (2000, 8))
    w1, b1, w2, b2 = L.unpack_params(theta.astype(np.float64))
    y = np.maximum(ctx @ w1.T + b1, 0) @ w2 + b2
    corr = net.correction(ctx)
    # rounding W1, b1, W2 to the power-of-two grid moves y by a bounded amount
    assert np.abs(corr - np.floor(y)).max() <= 3
    fq = L.fake_quant(theta)
    w1q, b1q, w2q, b2q = L.unpack_params(fq)
    yq = np.maximum(ctx @ w1q.T + b1q, 0) @ w2q + b2q
    assert np.array_equal(corr, np.clip(np.floor(yq), -255, 255).astype(np.int64))


def test_training_lowers_loss_and_entropy():
    import synth
    img = synth.smooth(96, 96, 31).astype(np.int64)
    ctx, t = L.training_pairs(img, 2)
    theta0 = synth.mlp_init(L.N_PARAMS, 32)
    loss0 = L.loss_grad(L.fake_quant(theta0), ctx, t)[0]
    theta = L.train(theta0, ctx, t, steps=150, lr=0.01, batch=4096)
    loss1 = L.loss_grad(L.fake_quant(theta), ctx, t)[0]
    assert loss1 < loss0 and loss1 < 0.95 * np.abs(t).mean()    # beats the plain predict
    net = L.quantize(theta)
    _, det = L.fwd_multilevel(img, 2, net)
    _, det0 = dwt53.fwd_multilevel(img, 2)
    assert L.detail_entropy(det) < L.detail_entropy(det0)


def test_fragments_zero_network_and_roundtrip():
    """Learned fragments with the zero network are the plain fragments; with
    any network restore inverts protect."""
    from oracle import fragment
    rng = np.random.default_rng(15)
    buf = rng.integers(0, 256, 5000).astype(np.uint8)
    key, nonce = rng.bytes(16), rng.bytes(16)
    assert L.protect(buf, 77, 3, key, nonce, L.Predictor.zero()) == \
        fragment.protect(buf, 77, 3, key, nonce)
    net = rand_net(rng)
    priv, pub = L.protect(buf, 77, 3, key, nonce, net)
    assert L.restore(priv, pub, 5000, 77, 3, key, nonce, net) == buf.tobytes()
