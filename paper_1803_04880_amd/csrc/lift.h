// Per-row lifting primitives and per-wavefront helpers shared by the forward
// and inverse streaming kernels.
//
// Lane layout: at level l a lane holds C = C1 >> (l-1) consecutive samples of
// the level-(l-1) LL row, indices j0 .. j0+C-1 with j0 even.  Even positions
// become lows, odd positions highs (Ch. 5 eqs. (5.1)-(5.2)).  The neighbour
// beyond the lane's last sample comes from the next lane, the one before its
// first sample from the previous lane (one DPP move each).
#pragma once

#include "common.h"

namespace dwtfrag {

// Forward 1-D lifting of one row held across the wavefront.
// Predict, eq. (5.1): d(j) = x(j) - floor((x(j-1) + x(j+1)) / 2), j odd.
// Update, eq. (5.2) additive: s(j) = x(j) + floor((d(j-1) + d(j+1) + 2) / 4).
// EDGE: the wavefront covers index 0 or N-1, where whole-sample mirroring
// replaces the missing neighbour by the one on the other side.
template <int C, bool EDGE>
__device__ __forceinline__ void hfwd(int (&v)[C], int j0, int N) {
  const int right0 = from_next_lane(v[0]);
#pragma unroll
  for (int t = 1; t < C; t += 2) {
    int r = (t + 1 < C) ? v[t + 1] : right0;
    if (EDGE && j0 + t == N - 1) r = v[t - 1];
    v[t] -= (v[t - 1] + r) >> 1;
  }
  const int left_d = from_prev_lane(v[C - 1]);
#pragma unroll
  for (int t = 0; t < C; t += 2) {
    int l = (t > 0) ? v[t - 1] : left_d;
    int r = v[t + 1];
    if (EDGE) {
      if (j0 + t == 0) l = r;
      if (j0 + t == N - 1) r = l;
    }
    v[t] += (l + r + 2) >> 2;
  }
}

// Inverse of hfwd: undo the update on even positions, then the predict on odd.
template <int C, bool EDGE>
__device__ __forceinline__ void hinv(int (&v)[C], int j0, int N) {
  const int left_d = from_prev_lane(v[C - 1]);
#pragma unroll
  for (int t = 0; t < C; t += 2) {
    int l = (t > 0) ? v[t - 1] : left_d;
    int r = v[t + 1];
    if (EDGE) {
      if (j0 + t == 0) l = r;
      if (j0 + t == N - 1) r = l;
    }
    v[t] -= (l + r + 2) >> 2;
  }
  const int right0 = from_next_lane(v[0]);
#pragma unroll
  for (int t = 1; t < C; t += 2) {
    int r = (t + 1 < C) ? v[t + 1] : right0;
    if (EDGE && j0 + t == N - 1) r = v[t - 1];
    v[t] += (v[t - 1] + r) >> 1;
  }
}

template <int C>
__device__ __forceinline__ void hfwd_any(int (&v)[C], int j0, int N, bool edge) {
  if (N == 1) return;  // a length-1 signal passes through
  if (edge) hfwd<C, true>(v, j0, N);
  else hfwd<C, false>(v, j0, N);
}

template <int C>
__device__ __forceinline__ void hinv_any(int (&v)[C], int j0, int N, bool edge) {
  if (N == 1) return;
  if (edge) hinv<C, true>(v, j0, N);
  else hinv<C, false>(v, j0, N);
}

// ------------------------------------------------------- int16 row I/O --
// U consecutive int16 band values starting at element index idx.  The first
// `nvalid` of them exist (nvalid may exceed U); vector access when all U exist
// and idx is U-aligned.
template <int U>
__device__ __forceinline__ void store_i16(int16_t *base, int64_t idx, int nvalid, const int (&v)[U]) {
  if (nvalid <= 0) return;
  if (U >= 2 && nvalid >= U && (idx & (U - 1)) == 0) {
    uint32_t w[U / 2 > 0 ? U / 2 : 1];
#pragma unroll
    for (int i = 0; i < U / 2; ++i)
      w[i] = (uint32_t(v[2 * i]) & 0xFFFFu) | (uint32_t(v[2 * i + 1]) << 16);
    if constexpr (U == 2) {
      *(gptr<uint32_t>)(glob(base) + idx) = w[0];
    } else if constexpr (U == 4) {
      *(gptr<u32x2>)(glob(base) + idx) = u32x2{w[0], w[1]};
    } else if constexpr (U == 8) {
      *(gptr<u32x4>)(glob(base) + idx) = u32x4{w[0], w[1], w[2], w[3]};
    } else {
#pragma unroll
      for (int i = 0; i < U / 8; ++i)
        ((gptr<u32x4>)(glob(base) + idx))[i] =
            u32x4{w[4 * i], w[4 * i + 1], w[4 * i + 2], w[4 * i + 3]};
    }
    return;
  }
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (u < nvalid) glob(base)[idx + u] = int16_t(v[u]);
}

template <int U>
__device__ __forceinline__ void load_i16(const int16_t *base, int64_t idx, int nvalid, int (&v)[U]) {
  if (U >= 2 && nvalid >= U && (idx & (U - 1)) == 0) {
    uint32_t w[U / 2 > 0 ? U / 2 : 1];
    if constexpr (U == 2) {
      w[0] = *(gptr<const uint32_t>)(glob(base) + idx);
    } else if constexpr (U == 4) {
      u32x2 q = *(gptr<const u32x2>)(glob(base) + idx);
      w[0] = q.x; w[1] = q.y;
    } else if constexpr (U == 8) {
      u32x4 q = *(gptr<const u32x4>)(glob(base) + idx);
      w[0] = q.x; w[1] = q.y; w[2] = q.z; w[3] = q.w;
    } else {
#pragma unroll
      for (int i = 0; i < U / 8; ++i) {
        u32x4 q = ((gptr<const u32x4>)(glob(base) + idx))[i];
        w[4 * i] = q.x; w[4 * i + 1] = q.y; w[4 * i + 2] = q.z; w[4 * i + 3] = q.w;
      }
    }
#pragma unroll
    for (int i = 0; i < U / 2; ++i) {
      v[2 * i] = int(int16_t(w[i] & 0xFFFFu));
      v[2 * i + 1] = int(int32_t(w[i]) >> 16);
    }
    return;
  }
#pragma unroll
  for (int u = 0; u < U; ++u) v[u] = (u < nvalid) ? int(glob(base)[idx + u]) : 0;
}

// Raw form: U int16 values as W = max(1, U/2) packed words (value u in the
// low / high half of word u/2), for rows loaded ahead of their use.
template <int U> struct Raw { static constexpr int W = U >= 2 ? U / 2 : 1; };

template <int U>
__device__ __forceinline__ void load_raw(const int16_t *base, int64_t idx, int nvalid,
                                         uint32_t (&w)[Raw<U>::W]) {
  if (U >= 2 && nvalid >= U && (idx & (U - 1)) == 0) {
    if constexpr (U == 2) {
      w[0] = *(gptr<const uint32_t>)(glob(base) + idx);
    } else if constexpr (U == 4) {
      const u32x2 q = *(gptr<const u32x2>)(glob(base) + idx);
      w[0] = q.x; w[1] = q.y;
    } else {
#pragma unroll
      for (int i = 0; i < U / 8; ++i) {
        const u32x4 q = ((gptr<const u32x4>)(glob(base) + idx))[i];
        w[4 * i] = q.x; w[4 * i + 1] = q.y; w[4 * i + 2] = q.z; w[4 * i + 3] = q.w;
      }
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < Raw<U>::W; ++i) w[i] = 0;
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (u < nvalid) w[u >> 1] |= uint32_t(uint16_t(glob(base)[idx + u])) << (16 * (u & 1));
}

template <int U>
__device__ __forceinline__ void unpack_raw(const uint32_t (&w)[Raw<U>::W], int (&v)[U]) {
#pragma unroll
  for (int u = 0; u < U; ++u)
    v[u] = (u & 1) ? int(int32_t(w[u >> 1]) >> 16) : int(int16_t(uint16_t(w[u >> 1] & 0xFFFFu)));
}

// ------------------------------------------------------ keystream ring --
// AES-CTR keystream for the LL band, computed ks_rows LL rows at a time into a
// per-wavefront LDS ring so that all 64 lanes share the AES work.  For LL row
// k the wavefront needs the bytes of columns [col_lo, col_hi).
struct KsRing {
  uint32_t *ring;       // kRingBlocks * 4 words, this wavefront's
  const uint32_t *te;   // AES tables in LDS
  const uint32_t *kw;   // round keys + nonce in LDS
  int rows, blocks;     // rows per refill, blocks per row slot
  int col_lo, col_hi;   // LL columns needed (clipped to the band)
  int64_t wL;           // LL row length
  int base;             // first row held, or -1

  __device__ __forceinline__ int64_t first_block(int k) const { return (2 * (int64_t(k) * wL + col_lo)) >> 4; }

  // Make row k resident; called with the whole wavefront converged, rows in
  // increasing order.  row_end bounds the rows worth computing.
  __device__ __forceinline__ void ensure(int k, int row_end, int lane) {
    if (base >= 0 && k >= base && k < base + rows) return;
    base = k;
    if (col_hi > col_lo) {
      for (int idx = lane; idx < rows * blocks; idx += 64) {
        const int g = idx / blocks, b = idx - g * blocks;
        const int r = k + g;
        if (r >= row_end) break;
        const int64_t b0 = first_block(r);
        const int64_t blast = (2 * (int64_t(r) * wL + col_hi) - 1) >> 4;
        if (b0 + b <= blast) {
          uint32_t w[4];
          counter_block(kw, uint64_t(b0 + b), w);
          aes_encrypt(te, kw, w);
          uint32_t *dst = ring + idx * 4;
          dst[0] = w[0]; dst[1] = w[1]; dst[2] = w[2]; dst[3] = w[3];
        }
      }
    }
    wave_lds_sync();
  }

  // Keystream bytes for LL(k, col) as a little-endian 16-bit value.
  __device__ __forceinline__ uint32_t ks16(int k, int col) const {
    const int64_t off = 2 * (int64_t(k) * wL + col) - 16 * first_block(k);
    const uint16_t *r16 = reinterpret_cast<const uint16_t *>(ring);
    return r16[(k - base) * blocks * 8 + int(off >> 1)];
  }
};

}  // namespace dwtfrag
