"""Brute-force pointwise twin of the multi-level 5/3 transform.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  It exists to pin
``oracle.dwt53``: every output coefficient is evaluated on its own from the
input matrix through the nested-floor closed form of eqs. (5.1)-(5.2)
(Ch. 5 section 5.1.1, additive update), with explicit whole-sample mirror
indexing at every level and no arrays shared with ``dwt53``.

Coordinates are "in place": after level l the coefficient of band b at band
index (i, j) sits at position (2i + bv, 2j + bh) of the level-(l-1) LL grid,
where bh / bv are 0 for low and 1 for high in the horizontal / vertical pass.
Only tiny shapes are practical (the recursion re-derives every dependency).
"""
from __future__ import annotations

from functools import lru_cache


def _m(i: int, n: int) -> int:
    if n == 1:
        return 0
    p = 2 * (n - 1)
    i %= p
    return p - i if i >= n else i


def _floor_div(a: int, b: int) -> int:
    return a // b  # Python's // is floor division for ints


def make_twin(mat, levels: int):
    """Return a function coef(level, band, i, j) for the matrix ``mat``."""
    rows = [list(map(int, r)) for r in mat]
    h0, w0 = len(rows), len(rows[0])
    dims = [(h0, w0)]
    for _ in range(levels):
        h, w = dims[-1]
        dims.append(((h + 1) // 2, (w + 1) // 2))

    @lru_cache(maxsize=None)
    def ll(lv: int, r: int, c: int) -> int:
        """LL_lv(r, c); LL_0 is the input matrix."""
        if lv == 0:
            return rows[r][c]
        return col_out(lv, 2 * r, 2 * c)

    @lru_cache(maxsize=None)
    def row_out(lv: int, r: int, c: int) -> int:
        """Horizontal pass of level lv at (r, c) of the level-(lv-1) grid."""
        _, w = dims[lv - 1]
        x = lambda cc: ll(lv - 1, r, _m(cc, w))
        if w == 1:
            return x(c)
        if c % 2 == 1:  # eq. (5.1)
            return x(c) - _floor_div(x(c - 1) + x(c + 1), 2)
        # eq. (5.2), additive; neighbours c-1 and c+1 mirrored onto odd indices
        def d(cc):
            cc = _m(cc, w)
            return x(cc) - _floor_div(x(cc - 1) + x(cc + 1), 2)
        return x(c) + _floor_div(d(c - 1) + d(c + 1) + 2, 4)

    @lru_cache(maxsize=None)
    def col_out(lv: int, r: int, c: int) -> int:
        """Vertical pass of level lv at (r, c), applied to the horizontal output."""
        h, _ = dims[lv - 1]
        y = lambda rr: row_out(lv, _m(rr, h), c)
        if h == 1:
            return y(r)
        if r % 2 == 1:
            return y(r) - _floor_div(y(r - 1) + y(r + 1), 2)

        def d(rr):
            rr = _m(rr, h)
            return y(rr) - _floor_div(y(rr - 1) + y(rr + 1), 2)
        return y(r) + _floor_div(d(r - 1) + d(r + 1) + 2, 4)

    def coef(lv: int, band: str, i: int, j: int) -> int:
        bh = 1 if band in ("HL", "HH") else 0
        bv = 1 if band in ("LH", "HH") else 0
        return col_out(lv, 2 * i + bv, 2 * j + bh)

    return coef, dims


def decompose(mat, levels: int):
    """(LL_L, details) in the same shapes as ``dwt53.fwd_multilevel``, as
    nested Python lists, computed coefficient by coefficient."""
    coef, dims = make_twin(mat, levels)
    details = []
    for lv in range(1, levels + 1):
        h, w = dims[lv - 1]
        hl, wl = (h + 1) // 2, (w + 1) // 2
        bands = []
        for band, bh_, bw_ in (("HL", hl, w - wl), ("LH", h - hl, wl), ("HH", h - hl, w - wl)):
            bands.append([[coef(lv, band, i, j) for j in range(bw_)] for i in range(bh_)])
        details.append(tuple(bands))
    hL, wL = dims[levels]
    if levels == 0:
        ll = [list(r) for r in mat]
    else:
        ll = [[coef(levels, "LL", i, j) for j in range(wL)] for i in range(hL)]
    return ll, details
