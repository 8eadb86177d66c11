"""The 16-bit inverse's range argument, checked on the CPU.

The GPU inverse lifts in packed int16 and trusts the result when every value
a level reads lies in [-4096, 4095] (else it redoes the wavefront in 32 bits).
These tests run one inverse level (vertical, then horizontal, as Ch. 5
section 5.2.3 inverts the forward order) with every operation in wrapping
int16 NumPy arithmetic and compare it with the exact integer inverse of the
oracle: equal for inputs inside the range, including the extreme patterns
that maximise every sum, and different for an input outside it (so the
check is needed).  They also pin the intermediate bounds the kernel's comment
states (|x| <= 10240 after the vertical step, sums <= 30720).
"""
import numpy as np
import pytest

from oracle import dwt53

LO, HI = -4096, 4095


def _mirror_idx(positions, n):
    """Whole-sample symmetric neighbour indices (left, right) of positions."""
    def m(i):
        if n == 1:
            return 0
        p = 2 * (n - 1)
        i %= p
        return p - i if i >= n else i
    left = np.array([m(i - 1) for i in positions], dtype=np.int64)
    right = np.array([m(i + 1) for i in positions], dtype=np.int64)
    return left, right


def _inv_1d(y, dtype, track=None):
    """Inverse 5/3 lifting along the last axis in the given integer dtype
    (int16 wraps).  track: optional list collecting |intermediate| maxima."""
    y = np.asarray(y, dtype=dtype)
    n = y.shape[-1]
    if n == 1:
        return y.copy()
    n_low = (n + 1) // 2
    odd, even = np.arange(1, n, 2), np.arange(0, n, 2)
    d = np.zeros_like(y)
    d[..., odd] = y[..., n_low:]
    x = np.zeros_like(y)
    el, er = _mirror_idx(even, n)
    s1 = d[..., el] + d[..., er] + dtype(2)
    x[..., even] = y[..., :n_low] - (s1 >> dtype(2))
    ol, orr = _mirror_idx(odd, n)
    s2 = x[..., ol] + x[..., orr]
    x[..., odd] = d[..., odd] + (s2 >> dtype(1))
    if track is not None:
        track.append(max(int(np.abs(s1.astype(np.int64)).max()), int(np.abs(s2.astype(np.int64)).max())))
        track.append(int(np.abs(x.astype(np.int64)).max()))
    return x


def _inv_level(ll, hl, lh, hh, dtype, track=None):
    top = np.concatenate([ll, hl], axis=1)
    bottom = np.concatenate([lh, hh], axis=1)
    cols = np.concatenate([top, bottom], axis=0).astype(dtype)
    vert = _inv_1d(cols.T, dtype, track).T
    return _inv_1d(vert, dtype, track)


def _bands(h, w, fill):
    hl_, wl_ = (h + 1) // 2, (w + 1) // 2
    return (fill(hl_, wl_), fill(hl_, w - wl_), fill(h - hl_, wl_), fill(h - hl_, w - wl_))


@pytest.mark.parametrize("h,w,seed", [(8, 8, 1), (9, 7, 2), (16, 33, 3), (2, 2, 4), (3, 5, 5), (31, 16, 6)])
def test_int16_inverse_is_exact_inside_the_range(h, w, seed):
    rng = np.random.default_rng(seed)
    bands = _bands(h, w, lambda a, b: rng.integers(LO, HI + 1, (a, b)))
    exact = dwt53.inv_2d_level(*bands)
    got = _inv_level(*bands, np.int16).astype(np.int64)
    assert np.array_equal(got, exact)


PATTERNS = {
    "all_max": lambda a, b: np.full((a, b), HI),
    "all_min": lambda a, b: np.full((a, b), LO),
    "checker": lambda a, b: np.where((np.add.outer(np.arange(a), np.arange(b)) & 1) == 0, HI, LO),
    "rows": lambda a, b: np.where((np.arange(a)[:, None] & 1) == 0, HI, LO) + 0 * np.arange(b)[None, :],
    "cols": lambda a, b: np.where((np.arange(b)[None, :] & 1) == 0, LO, HI) + 0 * np.arange(a)[:, None],
}


@pytest.mark.parametrize("ll_p,d_p", [(a, b) for a in PATTERNS for b in PATTERNS])
def test_int16_inverse_is_exact_at_the_extremes(ll_p, d_p):
    """LL and detail bands at the ends of the range in every combination of
    patterns (the sums the kernel forms are largest there)."""
    h, w = 12, 10
    ll, hl, lh, hh = _bands(h, w, PATTERNS[d_p])
    ll = PATTERNS[ll_p](*ll.shape)
    track = []
    exact = dwt53.inv_2d_level(ll, hl, lh, hh)
    _inv_level(ll, hl, lh, hh, np.int64, track)
    got = _inv_level(ll, hl, lh, hh, np.int16).astype(np.int64)
    assert np.array_equal(got, exact)
    # vertical step: sums and values; horizontal step: sums and values
    assert track[0] <= 12288 and track[1] <= 10240
    assert track[2] <= 30720 and track[3] <= 25600


def test_int16_inverse_fails_outside_the_range():
    """A patch of coefficients far outside: 16 bits wrap and the result differs, which
    is why the kernel checks its inputs and falls back to 32 bits."""
    rng = np.random.default_rng(9)
    ll, hl, lh, hh = (b.copy() for b in _bands(16, 16, lambda a, b: rng.integers(LO, HI + 1, (a, b))))
    for band in (hl, lh, hh):   # a patch of large details: their sums leave int16
        band[2:5, 2:5] = 20000
    exact = dwt53.inv_2d_level(ll, hl, lh, hh)
    got = _inv_level(ll, hl, lh, hh, np.int16).astype(np.int64)
    assert not np.array_equal(got, exact)
