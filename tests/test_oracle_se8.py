"""Pins of the per-8x8-block protection oracle (``oracle.se8``, ``oracle.sha2``)
against what the paper and the mathematics fix, without any implementation of
the GPU path.

  * SHA-256 / SHA-512: a library routine (hashlib) on messages of every
    padding case, one- and multi-block.
  * storage budget: 40 / 124 / 480 bits per 8x8 block and the 7.8 / 24.2 /
    93.8 % fragment fractions the paper prints (Ch. 5 sections 5.2.2.2 and
    5.5) are the fragment byte counts.
  * 10/11-bit packing is lossless: a sound bound (exact linear part plus an
    interval for every floor) puts every coefficient of every byte block
    inside its width.
  * record layout and hash messages: closed forms from hashlib and the pinned
    AES for zero and constant blocks, where the transform is known exactly.
  * bit packing by hand; the block transform is the pinned whole-matrix
    lifting on the tile; restore(protect(x)) == x; equal blocks differ
    (the counter in the hash input); one key bit changes about half of the
    public bits (the paper's key-sensitivity claim).
"""
import hashlib

import numpy as np
import pytest

from oracle import aes128, dwt53, se8, sha2


@pytest.mark.parametrize("length", [0, 1, 3, 45, 55, 56, 57, 63, 64, 65, 111, 112, 113,
                                    127, 128, 129, 255, 1000])
def test_sha2_against_hashlib(length):
    rng = np.random.default_rng(length)
    for _ in range(3):
        m = rng.bytes(length)
        assert sha2.sha256(m) == hashlib.sha256(m).digest()
        assert sha2.sha512(m) == hashlib.sha512(m).digest()


def test_sha2_constants_are_prime_roots():
    # FIPS 180-4: 64 / 80 round constants from cube roots, 8 initial values
    # from square roots; a wrong prime list or root breaks the digests above,
    # this checks the derivation's own arithmetic on its first entries.
    assert sha2.primes(10) == [2, 3, 5, 7, 11, 13, 17, 19, 23, 29]
    for x in (0, 1, 7, 8, 9, 2**96 - 1, 3 * 2**96, 10**40):
        for k in (2, 3):
            r = sha2.iroot(x, k)
            assert r ** k <= x < (r + 1) ** k
    assert len(sha2.K256) == 64 and len(sha2.K512) == 80
    # the SHA-512 constants extend the SHA-256 ones (same roots, more bits)
    assert all(k512 >> 32 == k256 for k512, k256 in zip(sha2.K512, sha2.K256))
    assert all(h512 >> 32 == h256 for h512, h256 in zip(sha2.H512, sha2.H256))


def test_storage_budget_and_fractions():
    # 40 + 124 + 480 bits per 64-byte block (Ch. 5 section 5.2.2.2), i.e.
    # 7.8 %, 24.2 % and 93.8 % of the input (section 5.5)
    for n, width in [(64, 8), (64 * 1000, 64), (4800 * 4800, 4800)]:
        g = se8.geometry(n, width)
        blocks = g["blocks"]
        assert blocks * 64 == n
        assert 8 * g["priv_bytes"] == 40 * blocks
        assert 8 * g["pub1_bytes"] == 124 * blocks + (4 if blocks % 2 else 0)
        assert 8 * g["pub2_bytes"] == 480 * blocks
        assert round(100 * 8 * g["priv_bytes"] / (8 * n), 1) == 7.8
        assert round(100 * 124 * blocks / (8 * n), 1) == 24.2
        assert round(100 * 8 * g["pub2_bytes"] / (8 * n), 1) == 93.8
    assert sum(w * 4 for _, w in se8.RECORDS["priv"]) == se8.PRIV_BITS == 40
    assert sum(w * 4 for _, w in se8.RECORDS["pub1"]) == se8.PUB1_BITS == 124
    assert sum(w * 16 for _, w in se8.RECORDS["pub2"]) == se8.PUB2_BITS == 480


def _lifted_bounds():
    """Per coefficient of the two-level 8x8 transform: [min, max] over every
    byte block.  Each sample is tracked as an exact linear form of the 64
    inputs plus an interval for the accumulated floor offsets (a predict
    floor((a + b) / 2) is (a + b) / 2 minus 0 or 1/2; an update
    floor((a + b + 2) / 4) is (a + b) / 4 plus an offset in [-1/4, 1/2])."""

    def fwd1(samples):
        n = len(samples)
        if n == 1:
            return samples
        m = dwt53.mirror
        d = {}
        for i in range(1, n, 2):
            (vi, li, hi), (vl, ll, hl), (vr, lr, hr) = samples[i], samples[m(i - 1, n)], samples[m(i + 1, n)]
            d[i] = (vi - (vl + vr) / 2, li - (hl + hr) / 2, hi - (ll + lr) / 2 + 0.5)
        s = {}
        for i in range(0, n, 2):
            ve, le, he = samples[i]
            (vl, ll, hl), (vr, lr, hr) = d[m(i - 1, n)], d[m(i + 1, n)]
            s[i] = (ve + (vl + vr) / 4, le + (ll + lr) / 4 - 0.25, he + (hl + hr) / 4 + 0.5)
        return [s[i] for i in range(0, n, 2)] + [d[i] for i in range(1, n, 2)]

    def level(grid):
        rows = [fwd1(r) for r in grid]
        h, w = len(rows), len(rows[0])
        cols = [fwd1([rows[r][c] for r in range(h)]) for c in range(w)]
        return [[cols[c][r] for c in range(w)] for r in range(h)]

    eye = np.eye(64)
    g1 = level([[(eye[8 * r + c], 0.0, 0.0) for c in range(8)] for r in range(8)])
    g2 = level([row[:4] for row in g1[:4]])
    lo, hi = np.zeros((8, 8)), np.zeros((8, 8))
    for r in range(8):
        for c in range(8):
            v, elo, ehi = g2[r][c] if (r < 4 and c < 4) else g1[r][c]
            hi[r, c] = 255 * v[v > 0].sum() + ehi
            lo[r, c] = 255 * v[v < 0].sum() + elo
    return lo, hi


def test_packing_widths_hold_for_every_byte_block():
    lo, hi = _lifted_bounds()
    width = np.full((8, 8), 10)
    width[2:4, 2:4] = 11          # HH2, the four 11-bit values
    assert np.all(lo >= -(2.0 ** (width - 1)))
    assert np.all(hi <= 2.0 ** (width - 1) - 1)
    # HH2 needs its eleventh bit: its bound passes 511
    assert hi[2:4, 2:4].max() > 511
    # each coefficient's extreme byte block (the sign pattern of its linear
    # form) comes within the floor offsets of the bound: it is not vacuous
    eye_bound = _extreme_values()
    assert np.all(eye_bound[0] >= lo - 1e-9) and np.all(eye_bound[1] <= hi + 1e-9)
    assert np.all(hi - eye_bound[1] <= 10) and np.all(eye_bound[0] - lo <= 10)


def _extreme_values():
    """Oracle values at each coefficient's extreme byte block (255 where the
    linear form is positive, else 0, and the reverse)."""
    lo, hi = np.zeros((8, 8)), np.zeros((8, 8))
    for r in range(8):
        for c in range(8):
            # linear form of coefficient (r, c) from 2^12-scaled unit blocks
            # (exact regime of the lifting: no rounding at 2^12 for 2 levels)
            form = np.zeros(64)
            for k in range(64):
                e = np.zeros(64, dtype=np.int64)
                e[k] = 1 << 12
                b = se8.block_bands(e.reshape(8, 8))
                full = _mallat(b)
                form[k] = full[r, c] / 4096.0
            xp = np.where(form > 0, 255, 0).reshape(8, 8)
            xn = np.where(form < 0, 255, 0).reshape(8, 8)
            hi[r, c] = _mallat(se8.block_bands(xp))[r, c]
            lo[r, c] = _mallat(se8.block_bands(xn))[r, c]
    return lo, hi


def _mallat(b):
    out = np.zeros((8, 8), dtype=np.int64)
    out[0:2, 0:2], out[0:2, 2:4], out[2:4, 0:2], out[2:4, 2:4] = b["LL2"], b["HL2"], b["LH2"], b["HH2"]
    out[0:4, 4:8], out[4:8, 0:4], out[4:8, 4:8] = b["HL1"], b["LH1"], b["HH1"]
    return out


def test_pack_by_hand():
    # 1, -1, -512, 511 in 10 bits, least significant first:
    # 0b0000000001 | 0b1111111111 << 10 | 0b1000000000 << 20 | 0b0111111111 << 30
    rec = se8.pack([(1, 10), (-1, 10), (-512, 10), (511, 10)])
    assert rec == 1 + (1023 << 10) + (512 << 20) + (511 << 30)
    assert rec.to_bytes(5, "little") == bytes([0x01, 0xFC, 0x0F, 0xE0, 0x7F])
    assert se8.unpack(rec, [10] * 4) == [1, -1, -512, 511]
    with pytest.raises(OverflowError):
        se8.pack([(512, 10)])
    with pytest.raises(OverflowError):
        se8.pack([(-1025, 11)])
    assert se8.unpack(se8.pack([(-1024, 11), (1023, 11)]), [11, 11]) == [-1024, 1023]


def test_block_transform_is_the_pinned_lifting_on_the_tile():
    rng = np.random.default_rng(7)
    x = rng.integers(0, 256, (16, 24)).astype(np.uint8)
    mat = se8.view(x.reshape(-1), 24)
    for by in range(2):
        for bx in range(3):
            tile = mat[8 * by:8 * by + 8, 8 * bx:8 * bx + 8]
            ll, det = dwt53.fwd_multilevel(tile, 2)
            b = se8.block_bands(tile)
            assert np.array_equal(b["LL2"], ll)
            assert np.array_equal(b["HH1"], det[0][2]) and np.array_equal(b["HL2"], det[1][0])


def test_zero_block_closed_form():
    """An all-zero block has all-zero coefficients, so its fragments are the
    key streams alone: AES-CTR of 5 zero bytes, the first 124 bits of
    SHA-256(m1) and the first 480 bits of SHA-512(m2) (hashlib)."""
    rng = np.random.default_rng(3)
    key, nonce = rng.bytes(16), rng.bytes(16)
    priv, pub1, pub2 = se8.protect(np.zeros(64, np.uint8), 8, key, nonce)
    assert priv == aes128.ctr_keystream(key, nonce, 5).tobytes()
    d1 = hashlib.sha256(bytes(5) + key + nonce + bytes(8)).digest()
    assert pub1 == d1[:15] + bytes([d1[15] & 0x0F])
    d2 = hashlib.sha512(pub1 + key + nonce + bytes(8)).digest()
    assert pub2 == d2[:60]


def test_constant_blocks_closed_form():
    """A constant block v has zero details and LL2 = v (the lifting of a
    constant: predict 0, update v + floor(2/4) = v); block b's hash
    messages carry b big-endian."""
    rng = np.random.default_rng(4)
    key, nonce = rng.bytes(16), rng.bytes(16)
    vals = [200, 17, 255]
    x = np.concatenate([np.full((8, 8), v, np.uint8) for v in vals], axis=1).reshape(-1)
    priv, pub1, pub2 = se8.protect(x, 24, key, nonce)
    plain = b"".join((v | v << 10 | v << 20 | v << 30).to_bytes(5, "little") for v in vals)
    assert aes128.ctr_xor(key, nonce, priv).tobytes() == plain
    acc1 = 0
    for b, v in enumerate(vals):
        d1 = hashlib.sha256((v | v << 10 | v << 20 | v << 30).to_bytes(5, "little") + key + nonce
                            + b.to_bytes(8, "big")).digest()
        rec1 = int.from_bytes(d1[:16], "little") & ((1 << 124) - 1)
        acc1 |= rec1 << (124 * b)
        d2 = hashlib.sha512(rec1.to_bytes(16, "little") + key + nonce + b.to_bytes(8, "big")).digest()
        assert pub2[60 * b:60 * b + 60] == d2[:60]
    assert pub1 == acc1.to_bytes(47, "little")


@pytest.mark.parametrize("n,width", [(1, 8), (64, 8), (65, 8), (1000, 16), (4096, 64),
                                     (12345, 40), (30001, 128)])
def test_roundtrip(n, width):
    rng = np.random.default_rng(n)
    x = rng.integers(0, 256, n, dtype=np.uint8)
    key, nonce = rng.bytes(16), rng.bytes(16)
    frags = se8.protect(x, width, key, nonce)
    g = se8.geometry(n, width)
    assert tuple(map(len, frags)) == (g["priv_bytes"], g["pub1_bytes"], g["pub2_bytes"])
    assert se8.restore(*frags, n, width, key, nonce) == x.tobytes()


def test_restore_of_tampered_fragments_returns_n_bytes():
    rng = np.random.default_rng(9)
    n, width = 5000, 64
    g = se8.geometry(n, width)
    key, nonce = rng.bytes(16), rng.bytes(16)
    out = se8.restore(rng.bytes(g["priv_bytes"]), rng.bytes(g["pub1_bytes"]),
                      rng.bytes(g["pub2_bytes"]), n, width, key, nonce)
    assert len(out) == n


def test_equal_blocks_give_different_public_fragments():
    key, nonce = bytes(range(16)), bytes(range(16, 32))
    x = np.tile(np.arange(64, dtype=np.uint8).reshape(8, 8), (1, 4)).reshape(-1)
    priv, pub1, pub2 = se8.protect(x, 32, key, nonce)
    recs = [pub2[60 * b:60 * b + 60] for b in range(4)]
    assert len(set(recs)) == 4


def test_one_key_bit_changes_about_half_the_public_bits():
    rng = np.random.default_rng(11)
    x = rng.integers(0, 256, 64 * 64, dtype=np.uint8)
    key, nonce = bytearray(rng.bytes(16)), rng.bytes(16)
    a = se8.protect(x, 64, bytes(key), nonce)
    key[5] ^= 0x10
    b = se8.protect(x, 64, bytes(key), nonce)
    for fa, fb in zip(a, b):
        diff = np.unpackbits(np.frombuffer(fa, np.uint8) ^ np.frombuffer(fb, np.uint8)).mean()
        assert 0.45 < diff < 0.55


def test_geometry_errors():
    for n, w in [(0, 8), (10, 0), (10, 12), (-1, 8)]:
        with pytest.raises(ValueError):
            se8.geometry(n, w)
