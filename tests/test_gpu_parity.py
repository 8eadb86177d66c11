"""GPU parity: the HIP path against the CPU oracle, byte for byte.

Every case draws seeded random (or synthetic) bytes, runs protect / restore
through the C ABI on cuda:0 and compares with ``oracle.fragment``.  The method
is exact integer arithmetic, so the tolerance is zero everywhere.
"""
import hashlib
import json
import os

import numpy as np
import pytest

from conftest import GOLDEN, gpu_available

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import torch  # noqa: E402

import paper_1803_04880_amd as dwtfrag  # noqa: E402
import synth  # noqa: E402
from oracle import aes128, fragment  # noqa: E402

DEV = "cuda:0"


def _say(msg):
    print(msg, flush=True)


def _gpu_protect(buf, width, levels, key, nonce, launch=None):
    x = torch.from_numpy(np.ascontiguousarray(buf)).to(DEV)
    priv, pub = dwtfrag.protect(x, width, levels, key, nonce, launch=launch)
    torch.cuda.synchronize()
    return priv.cpu().numpy().tobytes(), pub.cpu().numpy().tobytes()


def _gpu_restore(priv, pub, n, width, levels, key, nonce, launch=None):
    p = torch.from_numpy(np.frombuffer(priv, np.uint8).copy()).to(DEV)
    q = torch.from_numpy(np.frombuffer(pub, "<i2").copy()).to(DEV)
    out = dwtfrag.restore(p, q, n, width, levels, key, nonce, launch=launch)
    torch.cuda.synchronize()
    return out.cpu().numpy().tobytes()


# (n, width, levels): degenerate shapes, ragged tails, one and several
# windows / segments, every fused depth and multi-stage depths.
CASES = [
    (1, 1, 1), (2, 1, 1), (2, 2, 1), (3, 2, 2), (5, 2, 2), (7, 3, 2), (64, 8, 3),
    (100, 7, 1), (1000, 1000, 2), (1000, 1, 3), (4097, 64, 4), (12345, 97, 3),
    (100003, 317, 3), (513 * 37, 513, 1), (1500 * 40 - 3, 1500, 2),
    (2000 * 50, 2000, 3), (3000 * 33 + 5, 3000, 4), (70000, 4096, 4),
    (262144, 512, 1), (5000, 71, 5), (20000, 150, 6), (3, 2, 32), (300000, 1031, 8),
]


@pytest.mark.parametrize("n,width,levels", CASES)
def test_protect_matches_oracle_and_roundtrips(n, width, levels):
    rng = np.random.default_rng(n * 131 + width * 7 + levels)
    buf = rng.integers(0, 256, n, dtype=np.uint8)
    key, nonce = rng.bytes(16), rng.bytes(16)
    _say(f"case n={n} width={width} levels={levels}")
    priv, pub = _gpu_protect(buf, width, levels, key, nonce)
    opriv, opub = fragment.protect(buf, width, levels, key, nonce)
    assert len(priv) == len(opriv) and len(pub) == len(opub)
    assert priv == opriv, "private fragment differs"
    assert pub == opub, "public fragment differs"
    back = _gpu_restore(priv, pub, n, width, levels, key, nonce)
    assert back == buf.tobytes()


@pytest.mark.parametrize("nonce_hex", ["0011223344556677ffffffffffffff9c", "ffffffffffffffffffffffffffffff9c"])
def test_protect_counter_carries_match_oracle(nonce_hex):
    """Counters that carry from the nonce's low 64 bits into its high half
    (and wrap at 2^128) inside the LL band, which several forward wavefronts
    encrypt: the same fragments as the oracle, and an exact restore."""
    n, width, levels = 2000 * 50, 2000, 3   # LL 7 x 250: 219 keystream blocks
    rng = np.random.default_rng(91)
    buf = rng.integers(0, 256, n, dtype=np.uint8)
    key, nonce = rng.bytes(16), bytes.fromhex(nonce_hex)
    _say(f"case nonce={nonce_hex}")
    priv, pub = _gpu_protect(buf, width, levels, key, nonce)
    opriv, opub = fragment.protect(buf, width, levels, key, nonce)
    assert priv == bytes(opriv) and pub == bytes(opub)
    assert _gpu_restore(priv, pub, n, width, levels, key, nonce) == buf.tobytes()


@pytest.mark.parametrize("n,width,levels", [c for c in CASES if c[0] <= 300000])
def test_restore_of_arbitrary_fragments_matches_oracle(n, width, levels):
    """The inverse on its own: random (not protect-produced) fragments."""
    rng = np.random.default_rng(7 * n + width + levels)
    g = fragment.geometry(n, width, levels)
    priv = rng.integers(0, 256, g["priv_bytes"], dtype=np.uint8).tobytes()
    pub = rng.integers(-600, 600, g["pub_bytes"] // 2).astype("<i2").tobytes()
    key, nonce = rng.bytes(16), rng.bytes(16)
    _say(f"restore-only n={n} width={width} levels={levels}")
    got = _gpu_restore(priv, pub, n, width, levels, key, nonce)
    assert got == fragment.restore(priv, pub, n, width, levels, key, nonce)


def _fragments_from_values(ll, pub, key, nonce):
    """Fragments holding the given LL plaintext and public coefficients."""
    priv = aes128.ctr_xor(key, nonce, np.asarray(ll, "<i2").tobytes()).tobytes()
    return priv, np.asarray(pub, "<i2").tobytes()


@pytest.mark.parametrize("n,width", [(100003, 317), (262144, 512), (513 * 37, 513)])
def test_restore_at_the_packed_range_limits(n, width):
    """One level, every coefficient in [-4096, 4095] and half of them at the
    two ends: the 16-bit inverse runs at its largest sums and must still give
    the exact integer inverse."""
    rng = np.random.default_rng(n + 1)
    g = fragment.geometry(n, width, 1)
    key, nonce = rng.bytes(16), rng.bytes(16)

    def draw(count):
        v = rng.integers(-4096, 4096, count)
        ends = rng.random(count) < 0.5
        v[ends] = np.where(rng.random(int(ends.sum())) < 0.5, -4096, 4095)
        return v

    priv, pub = _fragments_from_values(draw(g["priv_bytes"] // 2), draw(g["pub_bytes"] // 2), key, nonce)
    _say(f"range limits n={n} width={width}")
    got = _gpu_restore(priv, pub, n, width, 1, key, nonce)
    assert got == fragment.restore(priv, pub, n, width, 1, key, nonce)


@pytest.mark.parametrize("levels,where,value", [
    (1, "pub", 4096), (1, "ll", -4097), (2, "pub", -4097), (2, "ll", 4096), (3, "pub", 30000),
    (3, "ll", -32768), (4, "pub", 4096),
])
def test_restore_with_one_value_outside_packed_range(levels, where, value):
    """Fragments of real data with one coefficient moved just outside the
    16-bit stream's range: the wavefronts that read it redo their rectangle
    in 32 bits, the others keep the packed result; all bytes must equal the
    exact inverse."""
    n, width = 300000, 1031
    rng = np.random.default_rng(levels * 10 + len(where))
    buf = rng.integers(0, 256, n, dtype=np.uint8)
    key, nonce = rng.bytes(16), rng.bytes(16)
    opriv, opub = fragment.protect(buf, width, levels, key, nonce)
    ll = np.frombuffer(aes128.ctr_xor(key, nonce, opriv).tobytes(), "<i2").copy()
    pub = np.frombuffer(opub, "<i2").copy()
    target = ll if where == "ll" else pub
    target[int(rng.integers(0, target.size))] = value
    priv, pubb = _fragments_from_values(ll, pub, key, nonce)
    _say(f"one value outside: levels={levels} {where}={value}")
    got = _gpu_restore(priv, pubb, n, width, levels, key, nonce)
    assert got == fragment.restore(priv, pubb, n, width, levels, key, nonce)


@pytest.mark.parametrize("levels", [1, 2, 3, 4])
def test_large_restore_with_values_outside_packed_range(levels):
    """A restore large enough for the two-launch form (packed streams, then
    the 32-bit redo of the rectangles they mark): fragments of real data with
    values moved outside the packed range in the private band, in the first
    and last columns of detail rows and at random places; every byte must
    equal the exact inverse."""
    n, width = (1 << 24) + 12345, 4096
    rng = np.random.default_rng(400 + levels)
    buf = rng.integers(0, 256, n, dtype=np.uint8)
    key, nonce = rng.bytes(16), rng.bytes(16)
    opriv, opub = fragment.protect(buf, width, levels, key, nonce)
    ll = np.frombuffer(aes128.ctr_xor(key, nonce, opriv).tobytes(), "<i2").copy()
    pub = np.frombuffer(opub, "<i2").copy()
    g = fragment.geometry(n, width, levels)
    wl = g["shapes"][1][1]          # level-1 LL width = HL row stride start
    ll[int(rng.integers(0, ll.size))] = -30000
    pub[-1] = 5000                   # last coefficient (bottom-right HH)
    pub[pub.size - wl] = -5000       # start of the last HH row
    for idx in rng.integers(0, pub.size, 5):
        pub[int(idx)] = int(rng.choice([-32768, 32767, 4096, -4097]))
    priv, pubb = _fragments_from_values(ll, pub, key, nonce)
    _say(f"large restore with values outside: levels={levels}")
    got = _gpu_restore(priv, pubb, n, width, levels, key, nonce)
    assert got == fragment.restore(priv, pubb, n, width, levels, key, nonce)


@pytest.mark.parametrize("levels", [2, 3])
def test_restore_of_small_arbitrary_fragments(levels):
    """Arbitrary coefficients in [-600, 600] (LL included): packed where the
    reconstructed rows stay in range, 32-bit where they do not."""
    n, width = 200003, 613
    rng = np.random.default_rng(70 + levels)
    g = fragment.geometry(n, width, levels)
    key, nonce = rng.bytes(16), rng.bytes(16)
    priv, pub = _fragments_from_values(rng.integers(-600, 601, g["priv_bytes"] // 2),
                                       rng.integers(-600, 601, g["pub_bytes"] // 2), key, nonce)
    _say(f"small arbitrary fragments levels={levels}")
    got = _gpu_restore(priv, pub, n, width, levels, key, nonce)
    assert got == fragment.restore(priv, pub, n, width, levels, key, nonce)


LAUNCHES = [None, (8, 8), (16, 8), (24, 16), (64, 16), (200, 8)]


@pytest.mark.parametrize("levels", [1, 2, 3, 4])
def test_launch_shape_invariance(levels):
    """Identical bytes for every segment height / lane width (a missing halo
    row or column would show up as a mismatch)."""
    rng = np.random.default_rng(40 + levels)
    width, rows = 1500, 301
    n = width * rows - 11
    buf = rng.integers(0, 256, n, dtype=np.uint8)
    key, nonce = rng.bytes(16), rng.bytes(16)
    opriv, opub = fragment.protect(buf, width, levels, key, nonce)
    for launch in LAUNCHES:
        if launch is not None and levels == 4 and launch[1] == 8:
            launch = (launch[0], 16)
        _say(f"launch {launch} levels={levels}")
        priv, pub = _gpu_protect(buf, width, levels, key, nonce, launch=launch)
        assert priv == opriv and pub == opub, launch
        assert _gpu_restore(priv, pub, n, width, levels, key, nonce, launch=launch) == buf.tobytes()


@pytest.mark.parametrize("nbytes,first_block,nonce_hex", [
    (1, 0, None), (15, 0, None), (16, 3, None), (17, 0, "00112233445566770000000000000000"),
    (1000, 5, "0011223344556677fffffffffffffffe"), ((1 << 20) + 3, 0, "ffffffffffffffffffffffffffffffff"),
])
def test_aes_ctr_kernel_matches_oracle(nbytes, first_block, nonce_hex):
    rng = np.random.default_rng(nbytes + first_block)
    key = rng.bytes(16)
    nonce = rng.bytes(16) if nonce_hex is None else bytes.fromhex(nonce_hex)
    data = rng.integers(0, 256, nbytes, dtype=np.uint8)
    _say(f"ctr nbytes={nbytes}")
    x = torch.from_numpy(data).to(DEV)
    y = dwtfrag.aes128_ctr(x, key, nonce, first_block)
    dwtfrag.aes128_ctr(x, key, nonce, first_block, out=x)  # in place
    torch.cuda.synchronize()
    ks = aes128.ctr_keystream(key, nonce, nbytes, offset_blocks=first_block)
    assert np.array_equal(y.cpu().numpy(), data ^ ks)
    assert np.array_equal(x.cpu().numpy(), data ^ ks)


def _digests():
    with open(os.path.join(GOLDEN, "oracle_digests.json")) as f:
        return json.load(f)


def test_small_workload_elementwise():
    """512 x 512 smooth field, one level: every byte against the oracle."""
    cfg = synth.config_small()
    gold = _digests()["small"]
    buf = cfg["buf"]
    assert hashlib.sha256(buf.tobytes()).hexdigest() == gold["input_sha256"]
    _say("small workload")
    priv, pub = _gpu_protect(buf, cfg["width"], cfg["levels"], cfg["key"], cfg["nonce"])
    opriv, opub = fragment.protect(buf, cfg["width"], cfg["levels"], cfg["key"], cfg["nonce"])
    a, b = np.frombuffer(pub, "<i2"), np.frombuffer(opub, "<i2")
    assert np.array_equal(a, b), f"{np.count_nonzero(a != b)} public coefficients differ"
    assert priv == opriv
    assert hashlib.sha256(priv).hexdigest() == gold["priv_sha256"]
    assert hashlib.sha256(pub).hexdigest() == gold["pub_sha256"]
    assert _gpu_restore(priv, pub, buf.size, cfg["width"], cfg["levels"], cfg["key"],
                        cfg["nonce"]) == buf.tobytes()


def test_large_workload_digest_and_roundtrip():
    """256 MiB, 8192 x 32768, three levels, in the benchmark's launch shape:
    SHA-256 of both fragments against the oracle's (written by
    tests/golden/make_digests.py), then restore on the GPU."""
    gold = _digests()["large"]
    _say("large workload: generating input")
    cfg = synth.config_large()
    buf = cfg["buf"]
    assert hashlib.sha256(buf.tobytes()).hexdigest() == gold["input_sha256"]
    x = torch.from_numpy(buf).to(DEV)
    del buf, cfg["buf"]
    _say("large workload: protect")
    priv, pub = dwtfrag.protect(x, cfg["width"], cfg["levels"], cfg["key"], cfg["nonce"])
    torch.cuda.synchronize()
    assert hashlib.sha256(priv.cpu().numpy().tobytes()).hexdigest() == gold["priv_sha256"]
    assert hashlib.sha256(pub.cpu().numpy().tobytes()).hexdigest() == gold["pub_sha256"]
    _say("large workload: restore")
    back = dwtfrag.restore(priv, pub, x.numel(), cfg["width"], cfg["levels"], cfg["key"],
                           cfg["nonce"])
    torch.cuda.synchronize()
    assert torch.equal(back, x)


@pytest.mark.parametrize("n,width,levels,launch", [
    (1000 * 37 + 5, 1000, 1, None), (268568, 1024, 1, None), (31683, 256, 2, (0, 16)),
    (4097, 64, 3, None), (100003, 317, 3, (16, 8)), (70000, 4096, 4, None), (5000, 71, 5, None),
])
def test_restore_writes_nothing_past_n(n, width, levels, launch):
    """The last row of the view is partial: restore writes exactly n bytes
    (a guard region right after the output keeps its pattern)."""
    rng = np.random.default_rng(n + levels)
    buf = rng.integers(0, 256, n, dtype=np.uint8)
    key, nonce = rng.bytes(16), rng.bytes(16)
    _say(f"guard n={n} width={width} levels={levels} launch={launch}")
    x = torch.from_numpy(buf).to(DEV)
    priv, pub = dwtfrag.protect(x, width, levels, key, nonce, launch=launch)
    guard = 16384
    big = torch.full((n + guard,), 0xA5, dtype=torch.uint8, device=DEV)
    dwtfrag.restore(priv, pub, n, width, levels, key, nonce, out=big[:n], launch=launch)
    torch.cuda.synchronize()
    assert torch.equal(big[:n], x)
    assert bool((big[n:] == 0xA5).all()), "restore wrote past n"
