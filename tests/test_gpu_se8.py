"""GPU parity of the per-8x8-block protection (``dwtfrag_se8_*``) against
``oracle.se8``, byte for byte (exact integer and bit arithmetic: tolerance 0).

Shapes cover one block, rows that are not a multiple of 8, ragged tails, one
and several 256-block workgroups with an odd block count (two first-public
records share a byte), counter carries in the private fragment's keystream,
restore of the oracle's fragments and of arbitrary (tampered) fragments,
and sampled blocks of a 256 MiB buffer in the launch shape the benchmark
times.
"""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import torch  # noqa: E402

import paper_1803_04880_amd as dwtfrag  # noqa: E402
from oracle import aes128, se8  # noqa: E402

DEV = "cuda:0"

CASES = [  # (n, width)
    (1, 8), (64, 8), (65, 8), (100, 16), (1000, 8), (64 * 7 + 5, 16),
    (256 * 64, 64), (255 * 64 + 1, 8), (257 * 64, 128), (12345, 96), (40000, 520),
    (513 * 64 * 3 - 11, 1024),
]


def _gpu(arr):
    return torch.from_numpy(np.ascontiguousarray(arr)).to(DEV)


def _frags(t):
    return tuple(x.cpu().numpy().tobytes() for x in t)


@pytest.mark.parametrize("n,width", CASES)
def test_protect_and_restore_match_oracle(n, width):
    print(f"se8 case n={n} width={width}", flush=True)
    rng = np.random.default_rng(n * 7 + width)
    buf = rng.integers(0, 256, n, dtype=np.uint8)
    key, nonce = rng.bytes(16), rng.bytes(16)
    g = dwtfrag.se8_geometry(n, width)
    og = se8.geometry(n, width)
    assert (g["priv_bytes"], g["pub1_bytes"], g["pub2_bytes"]) == \
        (og["priv_bytes"], og["pub1_bytes"], og["pub2_bytes"])
    frags = dwtfrag.se8_protect(_gpu(buf), width, key, nonce)
    torch.cuda.synchronize()
    want = se8.protect(buf, width, key, nonce)
    got = _frags(frags)
    for name, a, b in zip(("priv", "pub1", "pub2"), got, want):
        assert a == b, f"{name} differs from the oracle"
    back = dwtfrag.se8_restore(*frags, n, width, key, nonce)
    torch.cuda.synchronize()
    assert np.array_equal(back.cpu().numpy(), buf)


def test_counter_carries_in_private_keystream():
    n, width = 300 * 64 + 17, 80
    rng = np.random.default_rng(5)
    buf = rng.integers(0, 256, n, dtype=np.uint8)
    key = rng.bytes(16)
    for nonce in (bytes([0xFF] * 16), bytes(8) + bytes([0xFF] * 7) + bytes([0xF0])):
        got = _frags(dwtfrag.se8_protect(_gpu(buf), width, key, nonce))
        assert got == se8.protect(buf, width, key, nonce)


def test_restore_of_arbitrary_fragments_matches_oracle():
    # random bits in every record (values anywhere in their 10/11-bit range):
    # restore reconstructs with the same arithmetic and keeps bytes modulo 256
    n, width = 211 * 64 + 9, 104
    rng = np.random.default_rng(9)
    key, nonce = rng.bytes(16), rng.bytes(16)
    g = se8.geometry(n, width)
    priv = rng.bytes(g["priv_bytes"])
    pub1 = bytearray(rng.bytes(g["pub1_bytes"]))
    if g["blocks"] % 2:
        pub1[-1] &= 0x0F  # bits past the last record are zero in any fragment
    pub2 = rng.bytes(g["pub2_bytes"])
    want = se8.restore(priv, bytes(pub1), pub2, n, width, key, nonce)
    got = dwtfrag.se8_restore(_gpu(np.frombuffer(priv, np.uint8)),
                              _gpu(np.frombuffer(bytes(pub1), np.uint8)),
                              _gpu(np.frombuffer(pub2, np.uint8)), n, width, key, nonce)
    torch.cuda.synchronize()
    assert got.cpu().numpy().tobytes() == want


def test_restore_of_oracle_fragments():
    n, width = 100 * 64 + 3, 64
    rng = np.random.default_rng(11)
    buf = rng.integers(0, 256, n, dtype=np.uint8)
    key, nonce = rng.bytes(16), rng.bytes(16)
    priv, pub1, pub2 = se8.protect(buf, width, key, nonce)
    got = dwtfrag.se8_restore(*(_gpu(np.frombuffer(f, np.uint8)) for f in (priv, pub1, pub2)),
                              n, width, key, nonce)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), buf)


def _bits(data: bytes, start: int, count: int) -> int:
    lo, hi = start // 8, (start + count + 7) // 8
    return (int.from_bytes(data[lo:hi], "little") >> (start % 8)) & ((1 << count) - 1)


def test_sampled_blocks_of_256MiB_buffer():
    # 8192 x 32768 bytes: the records of sampled blocks (workgroup edges, the
    # first and last blocks, random ones) against the oracle's per-block
    # definition; the whole buffer round trips
    n, width = 1 << 28, 32768
    gen = torch.Generator(device=DEV)
    gen.manual_seed(28)
    x = torch.randint(0, 256, (n,), dtype=torch.uint8, device=DEV, generator=gen)
    key, nonce = bytes(range(16)), bytes([0xFF] * 12) + bytes([0, 0, 0xFF, 0xF0])
    g = dwtfrag.se8_geometry(n, width)
    priv, pub1, pub2 = dwtfrag.se8_protect(x, width, key, nonce)
    back = dwtfrag.se8_restore(priv, pub1, pub2, n, width, key, nonce)
    torch.cuda.synchronize()
    assert torch.equal(back, x)
    rng = np.random.default_rng(1)
    blocks = g["blocks"]
    sample = sorted({0, 1, 255, 256, 257, 511, 4095, 4096, blocks - 257, blocks - 256,
                     blocks - 1} | set(int(v) for v in rng.integers(0, blocks, 40)))
    wb = g["block_cols"]
    for b in sample:
        by, bx = divmod(b, wb)
        rows = torch.stack([x[(8 * by + r) * width + 8 * bx:(8 * by + r) * width + 8 * bx + 8]
                            for r in range(8)]).cpu().numpy()
        bands = se8.block_bands(rows)
        pr = se8.record(bands, "priv")
        p1 = se8.record(bands, "pub1") ^ se8.pub1_keystream(pr, key, nonce, b)
        p2 = se8.record(bands, "pub2") ^ se8.pub2_keystream(p1, key, nonce, b)
        # private record b: bytes 5b..5b+4 of the encrypted stream
        j0, j1 = (5 * b) // 16, (5 * b + 4) // 16
        ks = aes128.ctr_keystream(key, nonce, 16 * (j1 - j0 + 1), offset_blocks=j0).tobytes()
        off = 5 * b - 16 * j0
        enc = bytes(a ^ k for a, k in zip(pr.to_bytes(5, "little"), ks[off:off + 5]))
        assert priv[5 * b:5 * b + 5].cpu().numpy().tobytes() == enc, b
        lo = (124 * b) // 8
        seg = pub1[lo:lo + 17].cpu().numpy().tobytes()
        assert _bits(seg, 124 * b - 8 * lo, 124) == p1, b
        assert int.from_bytes(pub2[60 * b:60 * b + 60].cpu().numpy().tobytes(), "little") == p2, b
