"""Integer LeGall 5/3 lifting DWT: the oracle's plain definition.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper passages followed
  * Ch. 5 section 5.1.1 ("DWT"), eqs. (5.1)-(5.2): predict on odd samples with
    floor((x(2n)+x(2n+2))/2), update on even samples with
    floor((y(2n-1)+y(2n+1)+2)/4); floor is "the largest integer not exceeding".
  * Ch. 5 section 5.1.1: the 2-D transform is two 1-D passes (horizontal, then
    vertical) giving LL, HL, LH, HH; further levels transform LL only (dyadic).
  * Ch. 5 section 5.2.2.1: the horizontal pass runs first, then the vertical
    one, and the 8x8 operator is matrix A.

Readings where the paper is ambiguous (each is pinned by a test):
  * update sign: the update ADDS the floored term.  Eq. (5.2) as printed
    subtracts it, but matrix A and the F(4,4) taps of section 5.2.2.2 are only
    reproduced with the additive update.
  * extension: whole-sample symmetric at every level: x(-i) = x(i) and
    x(N-1+i) = x(N-1-i) for the signal of length N at that level (matrix A's
    last column x7 - x6 and the F(4,4) taps fix this).
  * odd lengths: ceil(N/2) lows, floor(N/2) highs; N == 1 passes through.
  * no DC level shift: bytes enter as 0..255.
  * floor: arithmetic right shift on Python/NumPy signed integers.

Layout conventions
  * a 1-D pass returns [lows | highs]: lows are the even input positions,
    highs the odd ones, each in increasing order.
  * one 2-D level of an h x w array returns the four bands
    LL (ceil(h/2) x ceil(w/2)), HL (ceil(h/2) x floor(w/2)),
    LH (floor(h/2) x ceil(w/2)), HH (floor(h/2) x floor(w/2)),
    where the first letter is the horizontal (row) filter and the second the
    vertical (column) filter: HL is horizontal-high, vertical-low.
"""
from __future__ import annotations

import numpy as np


def mirror(i: int, n: int) -> int:
    """Whole-sample symmetric extension index for a signal of length ``n``.

    Reflection about 0 and about n-1 (period 2(n-1)).  For n == 1 every index
    maps to 0.
    """
    if n == 1:
        return 0
    period = 2 * (n - 1)
    i %= period
    return period - i if i >= n else i


def _as_i64(x) -> np.ndarray:
    return np.asarray(x, dtype=np.int64)


def _neighbours(positions, n):
    """Mirrored left and right neighbour indices of each position."""
    left = np.array([mirror(i - 1, n) for i in positions], dtype=np.int64)
    right = np.array([mirror(i + 1, n) for i in positions], dtype=np.int64)
    return left, right


def fwd_1d(x) -> np.ndarray:
    """One forward 5/3 lifting pass along the LAST axis.

    Eq. (5.1): every odd sample first becomes
        d(i) = x(i) - floor((x(i-1) + x(i+1)) / 2)
    Eq. (5.2), additive reading: then every even sample becomes
        s(i) = x(i) + floor((d(i-1) + d(i+1) + 2) / 4)
    with out-of-range indices mirrored.  Returns [s(0), s(2), ... | d(1), ...].
    """
    x = _as_i64(x)
    n = x.shape[-1]
    if n == 1:
        return x.copy()
    odd = np.arange(1, n, 2)
    even = np.arange(0, n, 2)
    # predict, eq. (5.1): neighbours of an odd index are even indices
    ol, orr = _neighbours(odd, n)
    d = np.zeros_like(x)  # d[..., i] meaningful for odd i only
    d[..., odd] = x[..., odd] - ((x[..., ol] + x[..., orr]) >> 1)
    # update, eq. (5.2): neighbours of an even index are odd indices
    el, er = _neighbours(even, n)
    s = x[..., even] + ((d[..., el] + d[..., er] + 2) >> 2)
    return np.concatenate([s, d[..., odd]], axis=-1)


def inv_1d(y) -> np.ndarray:
    """Inverse of :func:`fwd_1d` along the LAST axis.

    Undo the update on even samples, then undo the predict on odd samples:
        x(i even) = s(i) - floor((d(i-1) + d(i+1) + 2) / 4)
        x(i odd)  = d(i) + floor((x(i-1) + x(i+1)) / 2)
    """
    y = _as_i64(y)
    n = y.shape[-1]
    if n == 1:
        return y.copy()
    n_low = (n + 1) // 2
    odd = np.arange(1, n, 2)
    even = np.arange(0, n, 2)
    d = np.zeros_like(y)
    d[..., odd] = y[..., n_low:]
    x = np.zeros_like(y)
    el, er = _neighbours(even, n)
    x[..., even] = y[..., :n_low] - ((d[..., el] + d[..., er] + 2) >> 2)
    ol, orr = _neighbours(odd, n)
    x[..., odd] = d[..., odd] + ((x[..., ol] + x[..., orr]) >> 1)
    return x


def fwd_2d_level(a) -> tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
    """One 2-D level: horizontal pass on every row, then vertical on every column.

    Returns (LL, HL, LH, HH) as described in the module docstring.
    """
    a = _as_i64(a)
    h, w = a.shape
    rows = fwd_1d(a)                      # horizontal pass: [L | H] per row
    cols = fwd_1d(rows.T).T               # vertical pass on every column
    hl, wl = (h + 1) // 2, (w + 1) // 2
    ll = cols[:hl, :wl]
    hl_band = cols[:hl, wl:]
    lh_band = cols[hl:, :wl]
    hh = cols[hl:, wl:]
    return ll.copy(), hl_band.copy(), lh_band.copy(), hh.copy()


def inv_2d_level(ll, hl_band, lh_band, hh) -> np.ndarray:
    """Inverse of :func:`fwd_2d_level`: vertical inverse, then horizontal."""
    top = np.concatenate([_as_i64(ll), _as_i64(hl_band)], axis=1)
    bottom = np.concatenate([_as_i64(lh_band), _as_i64(hh)], axis=1)
    cols = np.concatenate([top, bottom], axis=0)
    rows = inv_1d(cols.T).T
    return inv_1d(rows)


def level_shapes(h: int, w: int, levels: int) -> list[tuple[int, int]]:
    """(h_l, w_l) for l = 0..levels: h_l = ceil(h_{l-1}/2), same for w."""
    shapes = [(h, w)]
    for _ in range(levels):
        ph, pw = shapes[-1]
        shapes.append(((ph + 1) // 2, (pw + 1) // 2))
    return shapes


def fwd_multilevel(a, levels: int):
    """Dyadic decomposition: level l+1 transforms LL_l only (section 5.1.1).

    Returns (LL_L, details) with details[l-1] = (HL_l, LH_l, HH_l), l = 1..L.
    """
    ll = _as_i64(a)
    details = []
    for _ in range(levels):
        ll, hl_band, lh_band, hh = fwd_2d_level(ll)
        details.append((hl_band, lh_band, hh))
    return ll, details


def inv_multilevel(ll, details) -> np.ndarray:
    """Inverse of :func:`fwd_multilevel`, levels L..1."""
    cur = _as_i64(ll)
    for hl_band, lh_band, hh in reversed(details):
        cur = inv_2d_level(cur, hl_band, lh_band, hh)
    return cur
