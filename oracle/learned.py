"""Learned-predictor variant of the 5/3 lifting: the oracle's definition.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Not a method of the paper: an extension that plugs into the predict slot of
its lifting scheme (Ch. 5 section 5.1.1, eqs. (5.1)-(5.2)) and is judged by
the entropy of eq. (5.6) (section 5.3).  The predict step keeps the paper's
two-tap prediction as a base and adds a correction computed by a small integer
network from the even neighbours; the update step is the paper's, unchanged.
Every quantity is an integer, so the map stays an exact integer-to-integer
bijection, which is what makes the fragments lossless (section 5.2.3).

One predict step at odd position i of a signal x of length N >= 2
(m = whole-sample mirror, as in ``dwt53.mirror``):

  base(i) = floor((x(m(i-1)) + x(m(i+1))) / 2)                   eq. (5.1)
  c_j     = clamp(x(m(i + o_j)) - base(i), -128, 127),  o = (-7,-5,-3,-1,1,3,5,7)
  h_k     = max(0, sum_j W1[k][j] c_j + b1[k])                   k = 0..15
  corr    = clamp(floor((sum_k W2[k] h_k + b2) / 2^shift), -255, 255)
  d(i)    = x(i) - (base(i) + corr)

and the update at even i is eq. (5.2) with the additive sign (the reading the
plain oracle uses): s(i) = x(i) + floor((d(m(i-1)) + d(m(i+1)) + 2) / 4).

W1 and W2 are int8, b1 and b2 int32 with |b1| <= 2^16 and |b2| <= 2^26, and
0 <= shift <= 30; the sums are exact in int32 (|c| <= 128, so |W1 c| <= 2^17,
0 <= h < 2^18 and |W2 . h + b2| < 2^30).  Every i + o_j is even, so the context
reads only even samples; the inverse reconstructs the evens first (undo the
update) and then recomputes the very same context to undo the predict.  With
every weight and bias zero the correction is zero and the transform is the
plain 5/3 lifting.  One network serves every predict step: rows and columns,
every level.  Levels are limited to 3, for which every coefficient of a byte
input fits int16 (``int16_bound``).

Training (section "training" below) fits the real-valued network
y = W2 relu(W1 c + b1) + b2 to the target t = x(i) - base(i) of the predict
steps of a plain decomposition, under the mean absolute error.
"""
from __future__ import annotations

import numpy as np

from .dwt53 import fwd_1d as plain_fwd_1d
from .dwt53 import mirror

OFFSETS = (-7, -5, -3, -1, 1, 3, 5, 7)
CTX = len(OFFSETS)
HIDDEN = 16
CORR_LIMIT = 255
MAX_LEVELS = 3
B1_LIMIT = 1 << 16
B2_LIMIT = 1 << 26
N_PARAMS = HIDDEN * CTX + HIDDEN + HIDDEN + 1      # w1, b1, w2, b2 = 161


class Predictor:
    """Integer network: int8 W1 (16x8) and W2 (16), int32 b1 (16), b2, shift."""

    def __init__(self, w1, b1, w2, b2, shift):
        self.w1 = np.asarray(w1, dtype=np.int64).reshape(HIDDEN, CTX)
        self.b1 = np.asarray(b1, dtype=np.int64).reshape(HIDDEN)
        self.w2 = np.asarray(w2, dtype=np.int64).reshape(HIDDEN)
        self.b2 = int(b2)
        self.shift = int(shift)
        if not (-128 <= self.w1.min() and self.w1.max() <= 127
                and -128 <= self.w2.min() and self.w2.max() <= 127
                and np.abs(self.b1).max() <= B1_LIMIT and abs(self.b2) <= B2_LIMIT
                and 0 <= self.shift <= 30):
            raise ValueError("predictor parameters out of range")

    @staticmethod
    def zero():
        return Predictor(np.zeros((HIDDEN, CTX)), np.zeros(HIDDEN), np.zeros(HIDDEN), 0, 0)

    def correction(self, ctx):
        """corr of a (..., 8) array of clamped contexts."""
        ctx = np.asarray(ctx, dtype=np.int64)
        h = np.maximum(0, ctx @ self.w1.T + self.b1)
        acc = h @ self.w2 + self.b2
        return np.clip(acc >> self.shift, -CORR_LIMIT, CORR_LIMIT)

    def to_bytes(self) -> bytes:
        """Blob: int8 W1 (16x8 row-major, 128 B), int8 W2 (16 B), int32 LE
        b1 (64 B), b2, shift: 216 bytes."""
        return (self.w1.astype(np.int8).tobytes() + self.w2.astype(np.int8).tobytes()
                + self.b1.astype("<i4").tobytes()
                + np.array([self.b2, self.shift], dtype="<i4").tobytes())

    @staticmethod
    def from_bytes(blob: bytes) -> "Predictor":
        if len(blob) != 216:
            raise ValueError("predictor blob must be 216 bytes")
        w1 = np.frombuffer(blob, np.int8, 128, 0)
        w2 = np.frombuffer(blob, np.int8, 16, 128)
        b1 = np.frombuffer(blob, "<i4", 16, 144)
        b2, shift = np.frombuffer(blob, "<i4", 2, 208)
        return Predictor(w1, b1, w2, int(b2), int(shift))


# ------------------------------------------------------------- lifting --

def contexts(x):
    """(ctx, base, odd): for every odd position of the last axis of x, the
    clamped context (..., n_odd, 8), the two-tap base (..., n_odd) and the
    positions themselves."""
    x = np.asarray(x, dtype=np.int64)
    n = x.shape[-1]
    odd = np.arange(1, n, 2)
    taps = np.array([[mirror(i + o, n) for o in OFFSETS] for i in odd], dtype=np.int64)
    taps = taps.reshape(len(odd), CTX)
    left = np.array([mirror(i - 1, n) for i in odd], dtype=np.int64)
    right = np.array([mirror(i + 1, n) for i in odd], dtype=np.int64)
    base = (x[..., left] + x[..., right]) >> 1
    ctx = np.clip(x[..., taps] - base[..., None], -128, 127)
    return ctx, base, odd


def _even_neighbours(n):
    even = np.arange(0, n, 2)
    left = np.array([mirror(i - 1, n) for i in even], dtype=np.int64)
    right = np.array([mirror(i + 1, n) for i in even], dtype=np.int64)
    return even, left, right


def fwd_1d(x, net: Predictor):
    """Learned predict, then the plain update, along the last axis; returns
    [lows | highs] like ``dwt53.fwd_1d``."""
    x = np.asarray(x, dtype=np.int64)
    n = x.shape[-1]
    if n == 1:
        return x.copy()
    ctx, base, odd = contexts(x)
    d = np.zeros_like(x)
    d[..., odd] = x[..., odd] - (base + net.correction(ctx))
    even, left, right = _even_neighbours(n)
    s = x[..., even] + ((d[..., left] + d[..., right] + 2) >> 2)
    return np.concatenate([s, d[..., odd]], axis=-1)


def inv_1d(y, net: Predictor):
    """Inverse of :func:`fwd_1d`: undo the update, then the predict."""
    y = np.asarray(y, dtype=np.int64)
    n = y.shape[-1]
    if n == 1:
        return y.copy()
    n_low = (n + 1) // 2
    even, left, right = _even_neighbours(n)
    odd = np.arange(1, n, 2)
    d = np.zeros_like(y)
    d[..., odd] = y[..., n_low:]
    x = np.zeros_like(y)
    x[..., even] = y[..., :n_low] - ((d[..., left] + d[..., right] + 2) >> 2)
    ctx, base, _ = contexts(x)            # reads the even samples only
    x[..., odd] = d[..., odd] + base + net.correction(ctx)
    return x


def fwd_2d_level(a, net: Predictor):
    """Rows, then columns (the paper's order); returns (LL, HL, LH, HH)."""
    a = np.asarray(a, dtype=np.int64)
    h, w = a.shape
    rows = fwd_1d(a, net)
    full = fwd_1d(rows.T, net).T
    hl_, wl_ = (h + 1) // 2, (w + 1) // 2
    return (full[:hl_, :wl_].copy(), full[:hl_, wl_:].copy(),
            full[hl_:, :wl_].copy(), full[hl_:, wl_:].copy())


def inv_2d_level(ll, hl, lh, hh, net: Predictor):
    full = np.block([[np.asarray(ll, np.int64), np.asarray(hl, np.int64)],
                     [np.asarray(lh, np.int64), np.asarray(hh, np.int64)]])
    rows = inv_1d(full.T, net).T
    return inv_1d(rows, net)


def fwd_multilevel(a, levels, net: Predictor):
    """L levels on LL; returns (LL_L, [(HL_l, LH_l, HH_l) for l = 1..L])."""
    if not 1 <= levels <= MAX_LEVELS:
        raise ValueError("learned lifting supports 1..3 levels")
    ll = np.asarray(a, dtype=np.int64)
    details = []
    for _ in range(levels):
        ll, hl, lh, hh = fwd_2d_level(ll, net)
        details.append((hl, lh, hh))
    return ll, details


def inv_multilevel(ll, details, net: Predictor):
    cur = np.asarray(ll, dtype=np.int64)
    for hl, lh, hh in reversed(details):
        cur = inv_2d_level(cur, hl, lh, hh, net)
    return cur


def int16_bound(levels, corr_limit=CORR_LIMIT):
    """Interval bound on |coefficient| of a byte input after ``levels``
    levels of the learned lifting with |corr| <= corr_limit: each pass maps
    an input interval [lo, hi] to highs in [lo-hi-C, hi-lo+C] and lows in
    [lo + floor((2 dmin + 2)/4), hi + floor((2 dmax + 2)/4)]; the column
    pass sees the row lows (towards LL and LH) and the row highs (towards HL
    and HH) separately."""
    def one_pass(lo, hi):
        dmin, dmax = lo - hi - corr_limit, hi - lo + corr_limit
        return (dmin, dmax), (lo + ((2 * dmin + 2) >> 2), hi + ((2 * dmax + 2) >> 2))

    lo, hi = 0, 255
    worst = 0
    for _ in range(levels):
        (dmin, dmax), (smin, smax) = one_pass(lo, hi)          # rows
        for a, b in ((smin, smax), (dmin, dmax)):              # columns
            (e, f), (g, k) = one_pass(a, b)
            worst = max(worst, abs(e), abs(f), abs(g), abs(k))
        worst = max(worst, abs(dmin), abs(dmax))
        (_, _), (lo, hi) = one_pass(smin, smax)
    return worst


# ------------------------------------------------------------- entropy --

def entropy_bits(values) -> float:
    """Zeroth-order entropy of eq. (5.6), read as H = -sum p log2 p (the
    printed form has a sign garble), in bits per symbol."""
    v = np.asarray(values).reshape(-1)
    if v.size == 0:
        return 0.0
    _, counts = np.unique(v, return_counts=True)
    p = counts / v.size
    return float(-(p * np.log2(p)).sum())


def detail_entropy(details) -> float:
    """Entropy of all detail coefficients of a decomposition, pooled."""
    return entropy_bits(np.concatenate([b.reshape(-1) for lv in details for b in lv]))


# ------------------------------------------------------------ training --

def training_pairs(a, levels):
    """(ctx (P, 8) int, target (P,) int) of every predict step of a PLAIN 5/3
    decomposition of the matrix a: row pass then column pass of each level,
    positions in row-major order of the pass's array (rows: row by row;
    columns: column by column)."""
    ctxs, targets = [], []
    ll = np.asarray(a, dtype=np.int64)
    for _ in range(levels):
        h, w = ll.shape
        rows = plain_fwd_1d(ll) if w > 1 else ll.copy()
        for arr in (ll, rows.T):
            if arr.shape[-1] < 2:
                continue
            ctx, base, odd = contexts(arr)
            ctxs.append(ctx.reshape(-1, CTX))
            targets.append((arr[..., odd] - base).reshape(-1))
        cols = plain_fwd_1d(rows.T).T if h > 1 else rows
        ll = cols[:(h + 1) // 2, :(w + 1) // 2]
    if not ctxs:
        return np.zeros((0, CTX), np.int64), np.zeros(0, np.int64)
    return np.concatenate(ctxs), np.concatenate(targets)


def unpack_params(theta):
    """Flat vector (161) -> (W1 (16x8), b1 (16), W2 (16), b2)."""
    t = np.asarray(theta, dtype=np.float64)
    return (t[:128].reshape(HIDDEN, CTX), t[128:144], t[144:160], t[160])


def loss_grad(theta, ctx, target):
    """Mean |y - t| of the real-valued network y = W2 relu(W1 c + b1) + b2
    and its gradient with respect to the flat parameter vector, in fp64.
    Conventions at the kinks: relu'(0) = 0 and sign(0) = 0."""
    w1, b1, w2, b2 = unpack_params(theta)
    c = np.asarray(ctx, dtype=np.float64)
    t = np.asarray(target, dtype=np.float64)
    n = max(c.shape[0], 1)
    pre = c @ w1.T + b1
    hid = np.maximum(pre, 0.0)
    r = hid @ w2 + b2 - t
    loss = np.abs(r).sum() / n
    gy = np.sign(r) / n
    g_w2 = hid.T @ gy
    g_b2 = gy.sum()
    g_pre = np.outer(gy, w2) * (pre > 0)
    g_w1 = g_pre.T @ c
    g_b1 = g_pre.sum(axis=0)
    return loss, np.concatenate([g_w1.reshape(-1), g_b1, g_w2, [g_b2]])


def adam_step(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015), ``step`` counted from 1:
    m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
    theta -= lr * (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps)."""
    g = np.asarray(grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return np.asarray(theta, np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v


def pow2_exponent(maxabs, limit=127.5, lo=-30, hi=30):
    """Largest k in [lo, hi] with maxabs * 2^k < limit (hi if maxabs == 0).
    Multiplication by a power of two is exact, so this is the same in any
    binary floating point format that holds maxabs."""
    maxabs = float(maxabs)
    if maxabs == 0.0:
        return hi
    k = hi
    while k > lo and maxabs * 2.0 ** k >= limit:
        k -= 1
    return k


def quantize(theta):
    """Integer network from float32 parameters, power-of-two scales:
    k1 = pow2_exponent(max|W1|), shift = clamp(k1 + pow2_exponent(max|W2|),
    0, 30), k2 = shift - k1;  W1q = clamp(rint(W1 2^k1)), b1q = clamp(rint(b1
    2^k1), +-2^16), W2q = clamp(rint(W2 2^k2)), b2q = clamp(rint(b2 2^shift),
    +-2^26), round half to even.  Then corr ~ floor(y).  Every product is by a
    power of two, so the float32 arithmetic here is exact and any faithful
    implementation reproduces it bit for bit."""
    t = np.asarray(theta, dtype=np.float32).astype(np.float64)   # float32 values, exact in fp64
    w1, b1, w2, b2 = unpack_params(t)
    k1 = pow2_exponent(np.abs(w1).max())
    shift = int(np.clip(k1 + pow2_exponent(np.abs(w2).max()), 0, 30))
    k2 = shift - k1
    q_w1 = np.clip(np.rint(w1 * 2.0 ** k1), -128, 127)
    q_b1 = np.clip(np.rint(b1 * 2.0 ** k1), -B1_LIMIT, B1_LIMIT)
    q_w2 = np.clip(np.rint(w2 * 2.0 ** k2), -128, 127)
    q_b2 = float(np.clip(np.rint(b2 * 2.0 ** shift), -B2_LIMIT, B2_LIMIT))
    return Predictor(q_w1, q_b1, q_w2, int(q_b2), shift)


def fake_quant(theta):
    """The float values the integer network of :func:`quantize` stands for:
    W1q 2^-k1, b1q 2^-k1, W2q 2^-k2, b2q 2^-shift (the fake-quantised
    parameters of quantisation-aware training, where the gradient taken at
    these values is applied to the float parameters unchanged: the
    straight-through estimator)."""
    t = np.asarray(theta, dtype=np.float32).astype(np.float64)
    w1, b1, w2, b2 = unpack_params(t)
    k1 = pow2_exponent(np.abs(w1).max())
    shift = int(np.clip(k1 + pow2_exponent(np.abs(w2).max()), 0, 30))
    k2 = shift - k1
    q = quantize(t)
    return np.concatenate([(q.w1 * 2.0 ** -k1).reshape(-1), q.b1 * 2.0 ** -k1,
                           q.w2 * 2.0 ** -k2, [q.b2 * 2.0 ** -shift]])


def train(theta0, ctx, target, steps, lr, batch):
    """Quantisation-aware training: ``steps`` Adam steps over nb = max(1,
    floor(P / batch)) interleaved batches, step s on the pairs i, i + nb,
    i + 2 nb, ... with i = (s-1) mod nb (every batch samples every region
    and pass of the pairs), each gradient taken at the fake-quantised
    parameters.  Returns the final float parameters."""
    theta = np.asarray(theta0, np.float64).copy()
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    nb = max(len(target) // batch, 1)
    for step in range(1, steps + 1):
        i = (step - 1) % nb
        _, g = loss_grad(fake_quant(theta), ctx[i::nb], target[i::nb])
        theta, m, v = adam_step(theta, g, m, v, step, lr)
    return theta


# ----------------------------------------------------------- fragments --

def protect(buf, width, levels, key, nonce, net: Predictor):
    """(priv, pub) fragments with the learned lifting: the plain fragment
    layout and AES-128-CTR of ``fragment.protect``, this module's transform."""
    from . import aes128, fragment
    mat = fragment.view(buf, width)
    ll, details = fwd_multilevel(mat, levels, net)
    priv_plain, pub = fragment.serialize(ll, details)
    return aes128.ctr_xor(key, nonce, priv_plain).tobytes(), pub


def restore(priv, pub, n, width, levels, key, nonce, net: Predictor):
    """The first n bytes (each sample modulo 256) from learned fragments."""
    from . import aes128, fragment
    geom = fragment.geometry(n, width, levels)
    if len(priv) != geom["priv_bytes"] or len(pub) != geom["pub_bytes"]:
        raise ValueError("fragment sizes do not match the geometry")
    ll, details = fragment.deserialize(aes128.ctr_xor(key, nonce, priv).tobytes(), pub, geom)
    mat = inv_multilevel(ll, details, net)
    return (mat.reshape(-1)[:n] & 0xFF).astype(np.uint8).tobytes()
