"""The oracle against brute force, invariants and an independent AES.

* dwt53 vs the pointwise nested-floor twin (direct53) on every shape
  1..12 x 1..12 and L = 1..3, plus exhaustive 1-D inputs over edge values.
* restore(protect(x)) == x (the 5/3 map is an invertible integer-to-integer
  map, Ch. 5 section 5.2.3) on random buffers, odd n, many widths, L = 1..6.
* fragment layout (private = LL_L, public = coarsest level first, HL|LH|HH).
* AES-128 / CTR against the ``openssl`` command-line tool (skipped when absent).
"""
import itertools
import shutil
import subprocess

import numpy as np
import pytest

from oracle import aes128, direct53, dwt53, fragment


def _same(twin, arr):
    return np.array_equal(np.array(twin, dtype=np.int64).reshape(arr.shape), arr)


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_twin_all_small_shapes(levels):
    rng = np.random.default_rng(100 + levels)
    for h in range(1, 13):
        for w in range(1, 13):
            X = rng.integers(0, 256, (h, w))
            ll, det = dwt53.fwd_multilevel(X, levels)
            tll, tdet = direct53.decompose(X, levels)
            assert _same(tll, ll), (h, w, levels)
            for lv in range(levels):
                for b in range(3):
                    assert _same(tdet[lv][b], det[lv][b]), (h, w, levels, lv, b)


def test_twin_signed_inputs():
    """Negative values exercise floor (not truncation) of negative sums."""
    rng = np.random.default_rng(5)
    for h, w in [(7, 9), (10, 5), (12, 12)]:
        X = rng.integers(-600, 600, (h, w))
        ll, det = dwt53.fwd_multilevel(X, 2)
        tll, tdet = direct53.decompose(X, 2)
        assert _same(tll, ll)
        for lv in range(2):
            for b in range(3):
                assert _same(tdet[lv][b], det[lv][b])


def _direct_1d(x):
    """Eqs. (5.1)-(5.2) for one short signal, written out per output."""
    n = len(x)
    if n == 1:
        return list(x)
    m = lambda i: dwt53.mirror(i, n)
    def d(j):
        j = m(j)
        return x[j] - (x[m(j - 1)] + x[m(j + 1)]) // 2
    lows = [x[i] + (d(i - 1) + d(i + 1) + 2) // 4 for i in range(0, n, 2)]
    highs = [d(i) for i in range(1, n, 2)]
    return lows + highs


def test_exhaustive_1d_edge_values():
    vals = [0, 1, 127, 128, 254, 255]
    for n in range(1, 6):
        combos = np.array(list(itertools.product(vals, repeat=n)), dtype=np.int64)
        got = dwt53.fwd_1d(combos)
        want = np.array([_direct_1d(list(map(int, c))) for c in combos])
        np.testing.assert_array_equal(got, want)
        np.testing.assert_array_equal(dwt53.inv_1d(got), combos)


@pytest.mark.parametrize("levels", [1, 2, 3, 4, 6])
def test_roundtrip_random_buffers(levels):
    rng = np.random.default_rng(200 + levels)
    key, nonce = rng.bytes(16), rng.bytes(16)
    for _ in range(25):
        n = int(rng.integers(1, 5000))
        width = int(rng.integers(1, 300))
        buf = rng.integers(0, 256, n, dtype=np.uint8).tobytes()
        priv, pub = fragment.protect(buf, width, levels, key, nonce)
        geom = fragment.geometry(n, width, levels)
        assert len(priv) == geom["priv_bytes"] and len(pub) == geom["pub_bytes"]
        assert len(priv) + len(pub) == 2 * geom["height"] * width
        assert fragment.restore(priv, pub, n, width, levels, key, nonce) == buf


def test_fragment_layout_matches_bands():
    rng = np.random.default_rng(11)
    key, nonce = rng.bytes(16), rng.bytes(16)
    n, width, levels = 11 * 13 - 5, 13, 2
    buf = rng.integers(0, 256, n, dtype=np.uint8)
    X = np.zeros(11 * 13, dtype=np.int64)
    X[:n] = buf
    X = X.reshape(11, 13)
    tll, tdet = direct53.decompose(X, levels)
    priv, pub = fragment.protect(buf.tobytes(), width, levels, key, nonce)
    plain = aes128.ctr_xor(key, nonce, priv)
    np.testing.assert_array_equal(np.frombuffer(plain.tobytes(), "<i2"),
                                  np.array(tll).reshape(-1))
    expect = []
    for lv in (2, 1):                       # coarsest level first
        for band in tdet[lv - 1]:           # HL, LH, HH
            expect.extend(np.array(band, dtype=np.int64).reshape(-1).tolist())
    np.testing.assert_array_equal(np.frombuffer(pub, "<i2"), np.array(expect))


def test_geometry_and_widths():
    g = fragment.geometry(1 << 28, 32768, 3)
    assert (g["height"], g["ll_h"], g["ll_w"]) == (8192, 1024, 4096)
    assert g["priv_bytes"] == 8388608 and g["pub_bytes"] == 528482304
    g = fragment.geometry(512 * 512, 512, 1)
    assert g["priv_bytes"] == 131072 and g["pub_bytes"] == 393216
    assert [fragment.default_width(n) for n in (1, 2, 4, 5, 4096, 4097, 1 << 26)] == \
        [1, 2, 2, 4, 64, 128, 4096]
    with pytest.raises(ValueError):
        fragment.geometry(0, 1, 1)


def test_restore_of_tampered_fragments_is_local():
    """A flipped public coefficient changes only samples inside its support
    (radius 2^(L+1) - 2), the analogue of Ch. 5 section 'Propagation of errors'."""
    rng = np.random.default_rng(12)
    key, nonce = rng.bytes(16), rng.bytes(16)
    H = W = 64
    buf = rng.integers(0, 256, H * W, dtype=np.uint8).tobytes()
    for levels in (1, 2, 3):
        priv, pub = fragment.protect(buf, W, levels, key, nonce)
        p = bytearray(pub)
        pos = len(p) - 2 * (3 * 32 * 32) + 2 * (16 * 32 + 16)  # HL_1 (16, 16)
        p[pos] ^= 0x04
        out = np.frombuffer(fragment.restore(priv, bytes(p), H * W, W, levels, key, nonce),
                            np.uint8).reshape(H, W)
        diff = np.argwhere(out != np.frombuffer(buf, np.uint8).reshape(H, W))
        assert diff.size
        # HL_1 (16,16) sits at level-0 position (32, 33)
        assert np.abs(diff - np.array([32, 33])).max() <= 2


# ------------------------------------------------------------------- AES --

_OPENSSL = shutil.which("openssl")
needs_openssl = pytest.mark.skipif(_OPENSSL is None, reason="openssl CLI not installed")


def _openssl(args, data):
    r = subprocess.run([_OPENSSL, "enc"] + args, input=data, capture_output=True, check=True)
    return r.stdout


def test_sbox_is_a_permutation_without_fixed_points():
    s = aes128.SBOX.astype(int)
    assert sorted(s) == list(range(256))
    assert all(s[a] != a and s[a] != (a ^ 0xFF) for a in range(256))


@needs_openssl
def test_aes128_fips197_example_inputs():
    """The inputs of the AES-128 example of FIPS-197 (Appendix C.1): key
    00 01 .. 0f, plaintext 00 11 22 .. ff.  The expected ciphertext is not
    typed here: it is what the openssl CLI returns for these inputs."""
    key = bytes(range(16))
    pt = bytes(((i << 4) | i) for i in range(16))   # 00 11 22 .. ff
    want = _openssl(["-aes-128-ecb", "-K", key.hex(), "-nopad"], pt)
    assert len(want) == 16
    assert aes128.encrypt_blocks(key, np.frombuffer(pt, np.uint8).reshape(1, 16)).tobytes() == want


@needs_openssl
def test_aes_ecb_against_openssl():
    rng = np.random.default_rng(21)
    for _ in range(8):
        key = rng.bytes(16)
        data = rng.bytes(16 * int(rng.integers(1, 9)))
        ours = aes128.encrypt_blocks(key, np.frombuffer(data, np.uint8).reshape(-1, 16)).tobytes()
        assert ours == _openssl(["-aes-128-ecb", "-K", key.hex(), "-nopad"], data)


@needs_openssl
@pytest.mark.parametrize("nonce_hex", [
    None,
    "00112233445566770000000000000000",
    "0011223344556677fffffffffffffffe",   # carry across the 64-bit halves
    "ffffffffffffffffffffffffffffffff",   # wrap modulo 2^128
])
def test_aes_ctr_against_openssl(nonce_hex):
    rng = np.random.default_rng(22)
    key = rng.bytes(16)
    nonce = rng.bytes(16) if nonce_hex is None else bytes.fromhex(nonce_hex)
    for length in (1, 15, 16, 17, 100, 1000):
        data = rng.bytes(length)
        ours = aes128.ctr_xor(key, nonce, data).tobytes()
        assert ours == _openssl(["-aes-128-ctr", "-K", key.hex(), "-iv", nonce.hex()], data)


def test_ctr_keystream_offset_consistency():
    rng = np.random.default_rng(23)
    key, nonce = rng.bytes(16), rng.bytes(16)
    full = aes128.ctr_keystream(key, nonce, 16 * 40)
    part = aes128.ctr_keystream(key, nonce, 16 * 10, offset_blocks=30)
    np.testing.assert_array_equal(full[16 * 30:], part)
