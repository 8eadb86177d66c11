"""Seeded synthetic inputs with the shapes and content mix of the workloads.

This module holds no part of the protect/restore arithmetic; it only draws
bytes.  Tests, the benchmark and the oracle-digest script all take their inputs
from here, so the GPU path and the oracle see identical bytes.

The thesis measures on images (Lenna, barbara), English text and video files
(Ch. 5 section 5.3), none of which ship with it.  These generators stand in:
  smooth   image-like field: 8 random plane waves, min-max scaled, plus small
           integer noise (stands in for bitmaps);
  markov   order-1 chain over a skewed 16-symbol alphabet (stands in for text
           and other low-entropy formatted data);
  uniform  i.i.d. bytes (stands in for compressed/encrypted media).
"""
from __future__ import annotations

import math

import numpy as np

_BLOCK_ROWS = 256


def smooth(height: int, width: int, seed: int) -> np.ndarray:
    """height x width uint8 smooth field.

    Sum of 8 plane waves amp*sin(2*pi*(fx*c + fy*r) + phi) with amp ~ U(0.5, 1),
    phi ~ U(0, 2*pi), spatial frequency |f| ~ U(1/512, 12/512) cycles/pixel in
    a uniformly random direction; min-max scaled to 0..255 over the generated
    rows; then integer noise U{-8..8} is added, rounded and clipped.  Noise for
    row block k (256 rows) comes from ``default_rng([seed, 1, k])``.
    """
    rng = np.random.default_rng(seed)
    amp = rng.uniform(0.5, 1.0, 8)
    phi = rng.uniform(0.0, 2 * math.pi, 8)
    fmag = rng.uniform(1 / 512, 12 / 512, 8)
    theta = rng.uniform(0.0, 2 * math.pi, 8)
    fx, fy = fmag * np.cos(theta), fmag * np.sin(theta)
    cols = np.arange(width, dtype=np.float64)
    # sin(a_c + b_r) = sin(a_c) cos(b_r) + cos(a_c) sin(b_r): 1-D tables only
    sa = [np.sin(2 * math.pi * fx[k] * cols + phi[k]) for k in range(8)]
    ca = [np.cos(2 * math.pi * fx[k] * cols + phi[k]) for k in range(8)]

    def field(r0: int, r1: int) -> np.ndarray:
        rows = np.arange(r0, r1, dtype=np.float64)
        acc = np.zeros((r1 - r0, width), dtype=np.float64)
        for k in range(8):
            b = 2 * math.pi * fy[k] * rows
            acc += amp[k] * (np.outer(np.cos(b), sa[k]) + np.outer(np.sin(b), ca[k]))
        return acc

    lo, hi = np.inf, -np.inf
    for r0 in range(0, height, _BLOCK_ROWS):
        f = field(r0, min(height, r0 + _BLOCK_ROWS))
        lo, hi = min(lo, f.min()), max(hi, f.max())
    scale = 255.0 / (hi - lo) if hi > lo else 0.0
    out = np.empty((height, width), dtype=np.uint8)
    for k, r0 in enumerate(range(0, height, _BLOCK_ROWS)):
        r1 = min(height, r0 + _BLOCK_ROWS)
        f = (field(r0, r1) - lo) * scale
        noise = np.random.default_rng([seed, 1, k]).integers(-8, 9, (r1 - r0, width))
        out[r0:r1] = np.clip(np.rint(f + noise), 0, 255).astype(np.uint8)
    return out


def markov(length: int, seed: int, chain_len: int = 4096) -> np.ndarray:
    """Order-1 Markov byte stream over 16 distinct byte values.

    Row i of the transition matrix gives probability proportional to 2^-j to
    symbol perm_i[j] (perm_i a seeded permutation): about 2 bits per symbol.
    Built as ceil(length / chain_len) independent chains laid end to end, each
    starting from a draw of row 0.
    """
    rng = np.random.default_rng(seed)
    alphabet = rng.choice(256, 16, replace=False).astype(np.uint8)
    weights = 2.0 ** -np.arange(16)
    trans = np.zeros((16, 16))
    for i in range(16):
        trans[i, rng.permutation(16)] = weights
    trans /= trans.sum(axis=1, keepdims=True)
    cdf = np.cumsum(trans, axis=1)
    cdf[:, -1] = 1.0
    n_chains = max(1, -(-length // chain_len))
    u = rng.random((chain_len, n_chains))
    states = np.empty((chain_len, n_chains), dtype=np.int64)
    cur = np.zeros(n_chains, dtype=np.int64)
    for t in range(chain_len):
        cur = (u[t][:, None] >= cdf[cur]).sum(axis=1)
        states[t] = cur
    return alphabet[states.T.reshape(-1)[:length]]


def uniform(length: int, seed: int) -> np.ndarray:
    """i.i.d. uniform bytes."""
    return np.random.default_rng(seed).integers(0, 256, length, dtype=np.uint8)


def key_nonce(key_seed: int, nonce_seed: int) -> tuple[bytes, bytes]:
    return (np.random.default_rng(key_seed).bytes(16),
            np.random.default_rng(nonce_seed).bytes(16))


def mixed(length: int, width: int, seed: int) -> np.ndarray:
    """Three equal thirds: smooth field, Markov stream, uniform bytes."""
    a, b = length // 3, (2 * length) // 3
    rows = -(-a // width) if a else 0
    out = np.empty(length, dtype=np.uint8)
    if a:
        out[:a] = smooth(rows, width, seed).reshape(-1)[:a]
    out[a:b] = markov(b - a, seed)
    out[b:] = uniform(length - b, seed)
    return out


# ---------------------------------------------------------------- workloads --

def config_small():
    """512 x 512 smooth field, 1 level."""
    buf = smooth(512, 512, 1).reshape(-1)
    key, nonce = key_nonce(101, 201)
    return dict(name="512x512 smooth field, 1 level", buf=buf, width=512, levels=1,
                key=key, nonce=nonce)


def config_large():
    """256 MiB = 8192 rows x 32768 columns, thirds smooth/markov/uniform, 3 levels."""
    n, width = 1 << 28, 32768
    buf = mixed(n, width, 2)
    key, nonce = key_nonce(102, 202)
    return dict(name="256 MiB (8192x32768) mixed thirds, 3 levels", buf=buf, width=width,
                levels=3, key=key, nonce=nonce)


LEARNED_IMAGES = 64


def learned_image(i: int) -> np.ndarray:
    """Image i of the learned-predictor workload: a 4096 x 4096 smooth field
    (seed 4000 + i), as a flat byte buffer."""
    return smooth(4096, 4096, 4000 + i).reshape(-1)


def learned_key_nonce(i: int) -> tuple[bytes, bytes]:
    """Key (shared) and per-image nonce of the learned-predictor workload."""
    return np.random.default_rng(104).bytes(16), np.random.default_rng(5000 + i).bytes(16)


def default_width(n: int) -> int:
    """min(4096, next power of two >= ceil(sqrt(n)))."""
    r = math.isqrt(n)
    if r * r < n:
        r += 1
    return min(4096, 1 << max(0, (r - 1).bit_length()))


def batch_specs(count: int = 2048, seed_base: int = 3000, lo_log2: int = 12, hi_log2: int = 26):
    """Sizes, kinds, levels and seeds of the uneven batch (no bytes drawn)."""
    specs = []
    for i in range(count):
        rng = np.random.default_rng(seed_base + i)
        size = int(math.floor(math.exp(rng.uniform(lo_log2 * math.log(2), hi_log2 * math.log(2)))))
        kind = ("smooth", "markov", "uniform")[int(rng.integers(0, 3))]
        levels = int(rng.integers(1, 5))
        nonce = rng.bytes(16)
        specs.append(dict(seed=seed_base + i, n=size, kind=kind, levels=levels,
                          width=default_width(size), nonce=nonce))
    return specs


def batch_buffer(spec) -> np.ndarray:
    n, w, kind, seed = spec["n"], spec["width"], spec["kind"], spec["seed"]
    if kind == "smooth":
        return smooth(-(-n // w), w, seed).reshape(-1)[:n]
    if kind == "markov":
        return markov(n, seed)
    return uniform(n, seed)


def mlp_init(n_params: int, seed: int) -> np.ndarray:
    """Seeded float32 starting point of the 8-16-1 context network: the flat
    vector (W1 16x8, b1 16, W2 16, b2) with W1, W2 ~ N(0, 0.05^2), b1 = 1
    (hidden units start active) and b2 = 0."""
    rng = np.random.default_rng(seed)
    theta = rng.normal(0.0, 0.05, n_params)
    theta[128:144] = 1.0
    theta[160] = 0.0
    return theta.astype(np.float32)


def random_predictor(seed: int, weight: int = 128, bias: int = 4000, shift_range=(4, 14)):
    """Seeded raw integer parameters (w1 16x8, b1 16, w2 16, b2, shift) of the
    context network, for parity cases: int8 weights uniform in
    [-weight, weight), biases uniform in [-bias, bias), shift uniform in
    shift_range."""
    rng = np.random.default_rng(seed)
    w1 = rng.integers(-weight, weight, (16, 8)).astype(np.int8)
    b1 = rng.integers(-bias, bias, 16).astype(np.int32)
    w2 = rng.integers(-weight, weight, 16).astype(np.int8)
    b2 = int(rng.integers(-bias, bias))
    shift = int(rng.integers(shift_range[0], shift_range[1]))
    return w1, b1, w2, b2, shift
