"""Byte buffer -> matrix view -> (private, public) fragments, and back.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper passages followed
  * Ch. 5 section 5.2.1 ("Designs"): any data is cut into fixed-size 2-D
    matrices of bytes, every byte treated as an 8-bit pixel.
  * Ch. 5 sections 5.1.1 and 5.2.1: the low-frequency band of the last DWT
    level is the private fragment, protected with AES-128; the remaining
    (detail) coefficients form the public fragment.
  * Ch. 5 section 5.2.3: the 5/3 DWT is an invertible integer-to-integer map,
    so restore is exact.

Readings (the paper is silent on these; each is fixed here):
  * view: H = ceil(n / W) rows of W bytes, row-major; the tail of the last row
    is zero padding, transformed like data; restore returns the first n bytes.
  * the whole matrix is transformed (not independent 8x8 blocks) for
    L = ``levels`` levels.
  * coefficients are stored as int16 little-endian.
  * private plaintext = LL_L row-major; public = for l = L down to 1,
    HL_l | LH_l | HH_l, each row-major (coarsest level first).
  * private fragment = AES-128-CTR(key, nonce) of the private plaintext.
  * restore of arbitrary (possibly tampered) fragments writes each
    reconstructed sample modulo 256.
"""
from __future__ import annotations

import numpy as np

from . import aes128, dwt53


def ceil_div(a: int, b: int) -> int:
    return -(-a // b)


def geometry(n: int, width: int, levels: int) -> dict:
    """Matrix view and fragment sizes for an n-byte buffer of row width W."""
    if n <= 0 or width <= 0 or levels <= 0:
        raise ValueError("n, width and levels must be positive")
    height = ceil_div(n, width)
    shapes = dwt53.level_shapes(height, width, levels)
    ll_h, ll_w = shapes[-1]
    priv_bytes = 2 * ll_h * ll_w
    pub_bytes = 2 * (height * width - ll_h * ll_w)
    return dict(n=n, width=width, height=height, levels=levels, shapes=shapes,
                ll_h=ll_h, ll_w=ll_w, priv_bytes=priv_bytes, pub_bytes=pub_bytes)


def default_width(n: int) -> int:
    """min(4096, next power of two >= ceil(sqrt(n))): the width rule used for
    batches of uneven buffers."""
    r = 1
    while r * r < n:
        r += 1
    p = 1
    while p < r:
        p *= 2
    return min(4096, p)


def view(buf, width: int) -> np.ndarray:
    """The H x W uint8 matrix of a byte buffer, zero-padded at the tail."""
    data = np.frombuffer(bytes(buf), dtype=np.uint8) if isinstance(buf, (bytes, bytearray)) \
        else np.asarray(buf, dtype=np.uint8).reshape(-1)
    n = data.size
    height = ceil_div(n, width)
    mat = np.zeros(height * width, dtype=np.uint8)
    mat[:n] = data
    return mat.reshape(height, width)


def _to_i16_bytes(a: np.ndarray) -> bytes:
    a = np.asarray(a, dtype=np.int64)
    if a.size and (a.min() < -32768 or a.max() > 32767):
        raise OverflowError("coefficient outside int16")
    return a.astype("<i2").tobytes()


def serialize(ll, details) -> tuple[bytes, bytes]:
    """(private plaintext, public) byte strings from the decomposition."""
    priv_plain = _to_i16_bytes(ll)
    pub = b"".join(_to_i16_bytes(band)
                   for level in reversed(details) for band in level)
    return priv_plain, pub


def deserialize(priv_plain: bytes, pub: bytes, geom: dict):
    """Inverse of :func:`serialize` for the given geometry."""
    shapes = geom["shapes"]
    ll_h, ll_w = shapes[-1]
    ll = np.frombuffer(priv_plain, dtype="<i2", count=ll_h * ll_w).astype(np.int64)
    ll = ll.reshape(ll_h, ll_w)
    coeffs = np.frombuffer(pub, dtype="<i2").astype(np.int64)
    details = [None] * geom["levels"]
    pos = 0
    for lvl in range(geom["levels"], 0, -1):
        h, w = shapes[lvl - 1]
        hl, wl = (h + 1) // 2, (w + 1) // 2
        dims = [(hl, w - wl), (h - hl, wl), (h - hl, w - wl)]
        bands = []
        for bh, bw in dims:
            cnt = bh * bw
            bands.append(coeffs[pos:pos + cnt].reshape(bh, bw))
            pos += cnt
        details[lvl - 1] = tuple(bands)
    assert pos == coeffs.size
    return ll, details


def protect(buf, width: int, levels: int, key: bytes, nonce: bytes) -> tuple[bytes, bytes]:
    """(priv, pub) fragments of a byte buffer."""
    mat = view(buf, width)
    ll, details = dwt53.fwd_multilevel(mat, levels)
    priv_plain, pub = serialize(ll, details)
    priv = aes128.ctr_xor(key, nonce, priv_plain).tobytes()
    return priv, pub


def restore(priv: bytes, pub: bytes, n: int, width: int, levels: int,
            key: bytes, nonce: bytes) -> bytes:
    """The original n bytes from the two fragments."""
    geom = geometry(n, width, levels)
    if len(priv) != geom["priv_bytes"] or len(pub) != geom["pub_bytes"]:
        raise ValueError("fragment sizes do not match the geometry")
    priv_plain = aes128.ctr_xor(key, nonce, priv).tobytes()
    ll, details = deserialize(priv_plain, pub, geom)
    mat = dwt53.inv_multilevel(ll, details)
    out = (mat.reshape(-1)[:n] & 0xFF).astype(np.uint8)
    return out.tobytes()
