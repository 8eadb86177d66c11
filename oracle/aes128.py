"""AES-128 and counter mode for the private fragment: the oracle's definition.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper passages followed
  * Ch. 2 section "Our SE approach": AES-128 protects the most important
    fragment; the cipher is replaceable.
  * Ch. 2 section "Performance issue of SE": counter mode is the AES mode that
    can run in parallel.
  * Ch. 5 section "Cryptanalysis Discussion": an initialisation vector per
    chunk is suggested; here it is the 16-byte initial counter block (nonce).

The cipher itself is FIPS-197 (AES-128: 10 rounds, 4-word key).  Nothing is
typed from a table: the S-box is computed as the multiplicative inverse in
GF(2^8) modulo x^8 + x^4 + x^3 + x + 1 followed by the FIPS-197 affine map,
and the round constants are successive powers of x in the same field.

Counter mode: keystream block j = AES_K(T_j) with
T_j = (nonce as a 128-bit big-endian integer + j) mod 2^128; data is XORed
with the keystream and a final partial block uses the keystream's prefix.
"""
from __future__ import annotations

import numpy as np

_POLY = 0x11B  # x^8 + x^4 + x^3 + x + 1


def gf_mul(a: int, b: int) -> int:
    """Product in GF(2^8) (shift-and-add, reduce by the AES polynomial)."""
    r = 0
    while b:
        if b & 1:
            r ^= a
        a <<= 1
        if a & 0x100:
            a ^= _POLY
        b >>= 1
    return r


def gf_inv(a: int) -> int:
    """Multiplicative inverse in GF(2^8), with 0 mapped to 0 (a^254)."""
    if a == 0:
        return 0
    r, base, e = 1, a, 254
    while e:
        if e & 1:
            r = gf_mul(r, base)
        base = gf_mul(base, base)
        e >>= 1
    return r


def _affine(b: int) -> int:
    """FIPS-197 affine map: bit i of the result is
    b_i ^ b_{i+4} ^ b_{i+5} ^ b_{i+6} ^ b_{i+7} ^ c_i (indices mod 8), c = 0x63.
    """
    c = 0x63
    out = 0
    for i in range(8):
        bit = ((b >> i) ^ (b >> ((i + 4) % 8)) ^ (b >> ((i + 5) % 8))
               ^ (b >> ((i + 6) % 8)) ^ (b >> ((i + 7) % 8)) ^ (c >> i)) & 1
        out |= bit << i
    return out


SBOX = np.array([_affine(gf_inv(a)) for a in range(256)], dtype=np.uint8)
XTIME = np.array([gf_mul(a, 2) for a in range(256)], dtype=np.uint8)


def round_constants(count: int = 10) -> list[int]:
    """Rcon_i = x^(i-1) in GF(2^8), i = 1..count."""
    out, r = [], 1
    for _ in range(count):
        out.append(r)
        r = gf_mul(r, 2)
    return out


def expand_key(key: bytes) -> np.ndarray:
    """AES-128 key schedule: 44 words of 4 bytes -> (11, 16) round keys."""
    assert len(key) == 16
    rcon = round_constants(10)
    words = [list(key[4 * i:4 * i + 4]) for i in range(4)]
    for i in range(4, 44):
        temp = list(words[i - 1])
        if i % 4 == 0:
            temp = temp[1:] + temp[:1]                 # RotWord
            temp = [int(SBOX[b]) for b in temp]        # SubWord
            temp[0] ^= rcon[i // 4 - 1]
        words.append([words[i - 4][k] ^ temp[k] for k in range(4)])
    flat = np.array(words, dtype=np.uint8).reshape(11, 16)
    return flat


# State layout: a block's 16 bytes in input order; byte index r + 4c is row r,
# column c of the FIPS-197 state.


def _sub_bytes(s: np.ndarray) -> np.ndarray:
    return SBOX[s]


def _shift_rows(s: np.ndarray) -> np.ndarray:
    # destination index r + 4c takes state[r][(c + r) mod 4]
    dst = np.empty_like(s)
    for c in range(4):
        for r in range(4):
            dst[:, r + 4 * c] = s[:, r + 4 * ((c + r) % 4)]
    return dst


def _mix_columns(s: np.ndarray) -> np.ndarray:
    out = np.empty_like(s)
    for c in range(4):
        a0, a1, a2, a3 = (s[:, 4 * c + r] for r in range(4))
        t = a0 ^ a1 ^ a2 ^ a3
        out[:, 4 * c + 0] = a0 ^ t ^ XTIME[a0 ^ a1]
        out[:, 4 * c + 1] = a1 ^ t ^ XTIME[a1 ^ a2]
        out[:, 4 * c + 2] = a2 ^ t ^ XTIME[a2 ^ a3]
        out[:, 4 * c + 3] = a3 ^ t ^ XTIME[a3 ^ a0]
    return out


def encrypt_blocks(key: bytes, blocks: np.ndarray) -> np.ndarray:
    """AES-128 encryption of a (B, 16) uint8 array of blocks (FIPS-197 Cipher)."""
    rk = expand_key(key)
    s = np.asarray(blocks, dtype=np.uint8).reshape(-1, 16) ^ rk[0]
    for rnd in range(1, 10):
        s = _mix_columns(_shift_rows(_sub_bytes(s))) ^ rk[rnd]
    s = _shift_rows(_sub_bytes(s)) ^ rk[10]
    return s


def counter_blocks(nonce: bytes, count: int, first: int = 0) -> np.ndarray:
    """T_j = (int(nonce, big-endian) + j) mod 2^128 for j = first..first+count-1."""
    assert len(nonce) == 16
    base = int.from_bytes(nonce, "big")
    hi0, lo0 = base >> 64, base & ((1 << 64) - 1)
    j = np.arange(first, first + count, dtype=np.uint64)
    lo = np.uint64(lo0) + j                       # wraps mod 2^64
    carry = (lo < np.uint64(lo0)).astype(np.uint64)
    hi = np.uint64(hi0) + carry                   # wraps mod 2^64 (mod 2^128 overall)
    out = np.empty((count, 16), dtype=np.uint8)
    for k in range(8):
        out[:, k] = ((hi >> np.uint64(56 - 8 * k)) & np.uint64(0xFF)).astype(np.uint8)
        out[:, 8 + k] = ((lo >> np.uint64(56 - 8 * k)) & np.uint64(0xFF)).astype(np.uint8)
    return out


def ctr_keystream(key: bytes, nonce: bytes, nbytes: int, offset_blocks: int = 0) -> np.ndarray:
    """First ``nbytes`` of the CTR keystream starting at block ``offset_blocks``."""
    nblk = (nbytes + 15) // 16
    if nblk == 0:
        return np.zeros(0, dtype=np.uint8)
    ks = encrypt_blocks(key, counter_blocks(nonce, nblk, offset_blocks))
    return ks.reshape(-1)[:nbytes]


def ctr_xor(key: bytes, nonce: bytes, data) -> np.ndarray:
    """AES-128-CTR encryption (== decryption) of a byte array."""
    data = np.frombuffer(bytes(data), dtype=np.uint8) if isinstance(data, (bytes, bytearray)) \
        else np.asarray(data, dtype=np.uint8).reshape(-1)
    return data ^ ctr_keystream(key, nonce, data.size)
