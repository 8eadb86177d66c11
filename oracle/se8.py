"""The thesis's own per-8x8-block protection: block DWT, SHA keystreams over
the public fragments, packed 10/11-bit storage.  The oracle's plain definition.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper passages followed
  * Ch. 5 section 5.2.1 ("Designs"): the chunk is a matrix of bytes, cut into
    8x8 blocks; each block gets two levels of the 5/3 lifting.  Its level-2
    LL (4 of 64 coefficients) is the private fragment, encrypted with AES-128.
    SHA-256 of the private fragment and the key gives a bit sequence XORed
    over the remaining level-2 coefficients (the first public and protected
    fragment); SHA-512 of that first public and protected fragment and the
    key gives the bit sequence XORed over the level-1 detail coefficients
    (the second public and protected fragment).
  * Ch. 5 section 5.2.2.2 and "Storage space usage": every coefficient is
    stored in 10 bits except the four level-2 HH values (11 bits): 40 bits of
    private fragment, 40 + 40 + 44 = 124 bits of first public fragment and
    480 bits of second public fragment per 64-byte block.
  * Ch. 5 section 5.4 ("Sensitivity Test", "Key Sensitivity"): a counter
    (nonce) may be added to the hash input so that equal blocks give
    different fragments, and a per-chunk IV may vary the key stream.

Readings (the paper leaves these open; each is fixed here):
  * view: row width W a multiple of 8; H = ceil(n / W) rows, padded with zero
    rows up to a multiple of 8 (and the last row's tail with zeros); blocks
    are numbered row-major, b = (r / 8) * (W / 8) + c / 8.
  * block transform: the whole-matrix 5/3 lifting of ``dwt53`` applied to the
    8x8 block alone (mirrored at the block's own edges), rows first, 2 levels.
  * the "1st LL" that the thesis lists in the second public fragment is the
    level-1 LL the second level transforms; the second fragment is HL1, LH1,
    HH1 (3 x 16 coefficients, 480 bits).
  * records, coefficients in band row-major order:
      private  LL2                        4 x 10 bits =  40 bits
      public1  HL2, LH2 (10 bits), HH2 (11 bits)    = 124 bits
      public2  HL1, LH1, HH1              48 x 10 bits = 480 bits
    each value two's complement in its width; bit i of a record stream is bit
    i % 8 of byte i // 8 (least significant first), a value's bit j at
    position start + j.  Each fragment is the concatenation of the block
    records (public1 is a continuous 124-bit stream, so two blocks share a
    byte).
  * hash messages (one compression each):
      m1 = private record (5 bytes, before encryption) | key | nonce | b
      m2 = protected public1 record (124 bits + 4 zero bits, 16 bytes)
           | key | nonce | b
    with b as 8 bytes big-endian; the first 124 bits of SHA-256(m1) are XORed
    over the public1 record, the first 480 bits of SHA-512(m2) over the
    public2 record (bit i of a digest = bit i % 8 of its byte i // 8).
  * private fragment: AES-128-CTR (as the whole-matrix path) over the
    concatenated private records, keystream block j = AES_K(nonce + j).
  * restore writes every reconstructed sample modulo 256.
"""
from __future__ import annotations

import numpy as np

from . import aes128, dwt53, sha2

BLOCK = 8
LEVELS = 2
# (band, bits) of each record, bands in the 8x8 block's Mallat layout after
# two levels: rows / columns [0:2] LL2, HL2 = [0:2, 2:4], LH2 = [2:4, 0:2],
# HH2 = [2:4, 2:4], HL1 = [0:4, 4:8], LH1 = [4:8, 0:4], HH1 = [4:8, 4:8]
PRIV_BITS = 40
PUB1_BITS = 124
PUB2_BITS = 480


def geometry(n: int, width: int) -> dict:
    if n <= 0 or width <= 0 or width % BLOCK:
        raise ValueError("n > 0 and a width that is a positive multiple of 8 are required")
    height = -(-n // width)
    hb, wb = -(-height // BLOCK), width // BLOCK
    blocks = hb * wb
    return dict(n=n, width=width, height=height, block_rows=hb, block_cols=wb, blocks=blocks,
                priv_bytes=PRIV_BITS // 8 * blocks, pub1_bytes=-(-PUB1_BITS * blocks // 8),
                pub2_bytes=PUB2_BITS // 8 * blocks)


def view(buf, width: int) -> np.ndarray:
    """H8 x W byte matrix (H rounded up to whole blocks), zero padded."""
    data = np.asarray(np.frombuffer(bytes(buf), np.uint8) if isinstance(buf, (bytes, bytearray))
                      else buf, dtype=np.uint8).reshape(-1)
    g = geometry(data.size, width)
    mat = np.zeros(g["block_rows"] * BLOCK * width, dtype=np.uint8)
    mat[:data.size] = data
    return mat.reshape(-1, width)


def block_bands(block) -> dict:
    """Two-level lifting of one 8x8 block: the seven bands."""
    ll, details = dwt53.fwd_multilevel(block, LEVELS)
    (hl1, lh1, hh1), (hl2, lh2, hh2) = details
    return dict(LL2=ll, HL2=hl2, LH2=lh2, HH2=hh2, HL1=hl1, LH1=lh1, HH1=hh1)


def block_from_bands(b: dict) -> np.ndarray:
    return dwt53.inv_multilevel(b["LL2"], [(b["HL1"], b["LH1"], b["HH1"]),
                                           (b["HL2"], b["LH2"], b["HH2"])])


RECORDS = {
    "priv": [("LL2", 10)],
    "pub1": [("HL2", 10), ("LH2", 10), ("HH2", 11)],
    "pub2": [("HL1", 10), ("LH1", 10), ("HH1", 10)],
}


def pack(values_bits) -> int:
    """(value, width) pairs -> a record as a Python integer, first value in
    the lowest bits."""
    rec, pos = 0, 0
    for v, w in values_bits:
        v = int(v)
        if not -(1 << (w - 1)) <= v < (1 << (w - 1)):
            raise OverflowError(f"coefficient {v} does not fit {w} bits")
        rec |= (v & ((1 << w) - 1)) << pos
        pos += w
    return rec


def unpack(rec: int, widths) -> list[int]:
    out, pos = [], 0
    for w in widths:
        u = (rec >> pos) & ((1 << w) - 1)
        out.append(u - (1 << w) if u >> (w - 1) else u)
        pos += w
    return out


def record(bands: dict, kind: str) -> int:
    return pack((v, w) for name, w in RECORDS[kind] for v in np.asarray(bands[name]).reshape(-1))


def bands_from_records(priv: int, pub1: int, pub2: int) -> dict:
    out = {}
    for kind, rec in (("priv", priv), ("pub1", pub1), ("pub2", pub2)):
        widths = []
        names = []
        for name, w in RECORDS[kind]:
            side = 2 if name.endswith("2") else 4
            widths += [w] * (side * side)
            names.append((name, side))
        vals = unpack(rec, widths)
        pos = 0
        for name, side in names:
            out[name] = np.array(vals[pos:pos + side * side], dtype=np.int64).reshape(side, side)
            pos += side * side
    return out


def _digest_bits(d: bytes, bits: int) -> int:
    """First ``bits`` bits of a digest as an integer (bit i of the stream =
    bit i % 8 of byte i // 8)."""
    return int.from_bytes(d, "little") & ((1 << bits) - 1)


def pub1_keystream(priv_record: int, key: bytes, nonce: bytes, b: int) -> int:
    m1 = priv_record.to_bytes(5, "little") + key + nonce + b.to_bytes(8, "big")
    return _digest_bits(sha2.sha256(m1), PUB1_BITS)


def pub2_keystream(pub1_protected: int, key: bytes, nonce: bytes, b: int) -> int:
    m2 = pub1_protected.to_bytes(16, "little") + key + nonce + b.to_bytes(8, "big")
    return _digest_bits(sha2.sha512(m2), PUB2_BITS)


def _group(bits: int) -> int:
    """Records per whole number of bytes (2 for 124-bit records, else 1)."""
    g = 1
    while (g * bits) % 8:
        g += 1
    return g


def _concat(records, bits: int, nbytes: int) -> bytes:
    """Records laid end to end as one bit stream (record i at bit bits * i)."""
    g = _group(bits)
    out = []
    for i in range(0, len(records), g):
        acc = 0
        for k, r in enumerate(records[i:i + g]):
            acc |= r << (bits * k)
        out.append(acc.to_bytes(g * bits // 8, "little"))
    return b"".join(out)[:nbytes]


def _split(data: bytes, bits: int, count: int) -> list[int]:
    g = _group(bits)
    step = g * bits // 8
    mask = (1 << bits) - 1
    out = []
    for i in range(0, count, g):
        acc = int.from_bytes(data[(i // g) * step:(i // g + 1) * step], "little")
        out += [(acc >> (bits * k)) & mask for k in range(min(g, count - i))]
    return out


def protect(buf, width: int, key: bytes, nonce: bytes) -> tuple[bytes, bytes, bytes]:
    """(priv, pub1, pub2) fragments of a byte buffer."""
    key, nonce = bytes(key), bytes(nonce)
    n = len(buf) if isinstance(buf, (bytes, bytearray)) else np.asarray(buf).size
    mat = view(buf, width)
    g = geometry(n, width)
    privs, pub1s, pub2s = [], [], []
    for by in range(g["block_rows"]):
        for bx in range(g["block_cols"]):
            b = by * g["block_cols"] + bx
            bands = block_bands(mat[8 * by:8 * by + 8, 8 * bx:8 * bx + 8])
            pr = record(bands, "priv")
            p1 = record(bands, "pub1") ^ pub1_keystream(pr, key, nonce, b)
            p2 = record(bands, "pub2") ^ pub2_keystream(p1, key, nonce, b)
            privs.append(pr)
            pub1s.append(p1)
            pub2s.append(p2)
    priv_plain = _concat(privs, PRIV_BITS, g["priv_bytes"])
    priv = aes128.ctr_xor(key, nonce, priv_plain).tobytes()
    return (priv, _concat(pub1s, PUB1_BITS, g["pub1_bytes"]),
            _concat(pub2s, PUB2_BITS, g["pub2_bytes"]))


def restore(priv: bytes, pub1: bytes, pub2: bytes, n: int, width: int, key: bytes,
            nonce: bytes) -> bytes:
    """The original n bytes from the three fragments."""
    key, nonce = bytes(key), bytes(nonce)
    g = geometry(n, width)
    if (len(priv), len(pub1), len(pub2)) != (g["priv_bytes"], g["pub1_bytes"], g["pub2_bytes"]):
        raise ValueError("fragment sizes do not match the geometry")
    privs = _split(aes128.ctr_xor(key, nonce, priv).tobytes(), PRIV_BITS, g["blocks"])
    pub1s = _split(pub1, PUB1_BITS, g["blocks"])
    pub2s = _split(pub2, PUB2_BITS, g["blocks"])
    mat = np.zeros((g["block_rows"] * BLOCK, width), dtype=np.int64)
    for b in range(g["blocks"]):
        by, bx = divmod(b, g["block_cols"])
        p1 = pub1s[b] ^ pub1_keystream(privs[b], key, nonce, b)
        p2 = pub2s[b] ^ pub2_keystream(pub1s[b], key, nonce, b)
        mat[8 * by:8 * by + 8, 8 * bx:8 * bx + 8] = block_from_bands(
            bands_from_records(privs[b], p1, p2))
    return (mat.reshape(-1)[:n] & 0xFF).astype(np.uint8).tobytes()
