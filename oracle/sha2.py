"""SHA-256 and SHA-512 (FIPS 180-4): the oracle's plain definition.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper passages followed
  * Ch. 5 section 5.2.1 ("Designs"): per 8x8 block, SHA-256 over the private
    fragment and the key gives the bit sequence XORed over the first public
    fragment; SHA-512 over the first public and protected fragment and the key
    gives the one XORed over the second.  The paper cites FIPS 180 for both
    and prints no part of them; this module is the standard's definition.

Every constant is derived here rather than typed (FIPS 180-4 section 4.2.2 /
4.2.3 and 5.3.3 / 5.3.5): round constants are the first 32 (SHA-256) or 64
(SHA-512) bits of the fractional parts of the cube roots of the first 64 / 80
primes, initial hash values those of the square roots of the first 8 primes,
computed with exact integer roots.  Plain Python integers, one block at a
time, no vectorisation.
"""
from __future__ import annotations


def primes(count: int) -> list[int]:
    """The first ``count`` primes (trial division)."""
    out: list[int] = []
    k = 2
    while len(out) < count:
        if all(k % p for p in out if p * p <= k):
            out.append(k)
        k += 1
    return out


def iroot(x: int, k: int) -> int:
    """floor(x ** (1/k)) for a non-negative integer x (exact, Newton)."""
    if x < 2:
        return x
    r = 1 << ((x.bit_length() + k - 1) // k)   # >= the root
    while True:
        s = ((k - 1) * r + x // r ** (k - 1)) // k
        if s >= r:
            break
        r = s
    while r ** k > x:
        r -= 1
    while (r + 1) ** k <= x:
        r += 1
    return r


def frac_bits(p: int, k: int, bits: int) -> int:
    """First ``bits`` bits of the fractional part of p ** (1/k)."""
    return iroot(p << (k * bits), k) & ((1 << bits) - 1)


K256 = [frac_bits(p, 3, 32) for p in primes(64)]
H256 = [frac_bits(p, 2, 32) for p in primes(8)]
K512 = [frac_bits(p, 3, 64) for p in primes(80)]
H512 = [frac_bits(p, 2, 64) for p in primes(8)]


def _rotr(x: int, n: int, w: int) -> int:
    return ((x >> n) | (x << (w - n))) & ((1 << w) - 1)


def _pad(msg: bytes, block: int, len_bytes: int) -> bytes:
    """FIPS 180-4 section 5.1: a 1 bit, zeros, the bit length big-endian."""
    ml = 8 * len(msg)
    m = msg + b"\x80"
    while (len(m) + len_bytes) % block:
        m += b"\x00"
    return m + ml.to_bytes(len_bytes, "big")


def _compress(state, chunk: bytes, w: int, rounds: int, K, sig):
    """One compression (section 6.2.2 / 6.4.2) of a block of 16 words."""
    mask = (1 << w) - 1
    nb = w // 8
    S0, S1, s0, s1 = sig
    W = [int.from_bytes(chunk[nb * t:nb * (t + 1)], "big") for t in range(16)]
    for t in range(16, rounds):
        x, y = W[t - 15], W[t - 2]
        lo = _rotr(x, s0[0], w) ^ _rotr(x, s0[1], w) ^ (x >> s0[2])
        hi = _rotr(y, s1[0], w) ^ _rotr(y, s1[1], w) ^ (y >> s1[2])
        W.append((hi + W[t - 7] + lo + W[t - 16]) & mask)
    a, b, c, d, e, f, g, h = state
    for t in range(rounds):
        big1 = _rotr(e, S1[0], w) ^ _rotr(e, S1[1], w) ^ _rotr(e, S1[2], w)
        ch = (e & f) ^ (~e & mask & g)
        t1 = (h + big1 + ch + K[t] + W[t]) & mask
        big0 = _rotr(a, S0[0], w) ^ _rotr(a, S0[1], w) ^ _rotr(a, S0[2], w)
        maj = (a & b) ^ (a & c) ^ (b & c)
        t2 = (big0 + maj) & mask
        h, g, f, e, d, c, b, a = g, f, e, (d + t1) & mask, c, b, a, (t1 + t2) & mask
    return [(x + y) & mask for x, y in zip(state, (a, b, c, d, e, f, g, h))]


# rotation / shift amounts, section 4.1.2 (SHA-256) and 4.1.3 (SHA-512):
# Sigma0, Sigma1 (three rotations), sigma0, sigma1 (two rotations, a shift)
_SIG256 = ((2, 13, 22), (6, 11, 25), (7, 18, 3), (17, 19, 10))
_SIG512 = ((28, 34, 39), (14, 18, 41), (1, 8, 7), (19, 61, 6))


def sha256(msg: bytes) -> bytes:
    m = _pad(bytes(msg), 64, 8)
    st = list(H256)
    for i in range(0, len(m), 64):
        st = _compress(st, m[i:i + 64], 32, 64, K256, _SIG256)
    return b"".join(x.to_bytes(4, "big") for x in st)


def sha512(msg: bytes) -> bytes:
    m = _pad(bytes(msg), 128, 16)
    st = list(H512)
    for i in range(0, len(m), 128):
        st = _compress(st, m[i:i + 128], 64, 80, K512, _SIG512)
    return b"".join(x.to_bytes(8, "big") for x in st)
