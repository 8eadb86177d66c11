// Packed 16-bit lifting arithmetic.
//
// Forward coefficients of byte inputs stay far inside int16 (|c| < 1100 at any
// depth; sums of two stay below 2^12), so two samples share one 32-bit
// register and every lifting operation is one v_pk_* instruction on both.
// The inverse runs on the same layout when its inputs are bounded (see
// hinv_pk and the inverse kernel's range check).
//
// Register layout at a level where a lane holds M even and M odd samples
// (indices j0 .. j0+2M-1, j0 even) in P = max(1, M/2) registers per parity:
//   E[j] = (x[j0+4j],   x[j0+4j+2])   evens: lo half, hi half
//   O[j] = (x[j0+4j+1], x[j0+4j+3])   odds
// (for M == 1 only the lo halves are meaningful).  The neighbour pair of
// E[j] shifted by one even sample is one v_alignbit of two registers.  After
// the horizontal pass E holds lows and O highs in band order, which is the
// storage order of LL/LH and HL/HH, so no repacking is needed to store.
#pragma once

#include "common.h"

namespace dwtfrag {

typedef short v2s __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pk_u32(v2s v) { return __builtin_bit_cast(uint32_t, v); }
__device__ __forceinline__ v2s pk_v2(uint32_t u) { return __builtin_bit_cast(v2s, u); }
__device__ __forceinline__ uint32_t pk_add(uint32_t a, uint32_t b) { return pk_u32(pk_v2(a) + pk_v2(b)); }
__device__ __forceinline__ uint32_t pk_sub(uint32_t a, uint32_t b) { return pk_u32(pk_v2(a) - pk_v2(b)); }
__device__ __forceinline__ uint32_t pk_sra(uint32_t a, short s) { return pk_u32(pk_v2(a) >> s); }

// eq. (5.1): o - floor((a + b) / 2) on both halves
__device__ __forceinline__ uint32_t pk_predict(uint32_t o, uint32_t a, uint32_t b) {
  return pk_sub(o, pk_sra(pk_add(a, b), 1));
}
// eq. (5.2), additive: e + floor((a + b + 2) / 4) on both halves
__device__ __forceinline__ uint32_t pk_update(uint32_t e, uint32_t a, uint32_t b) {
  return pk_add(e, pk_sra(pk_add(pk_add(a, b), 0x00020002u), 2));
}

// (lo.hi, hi.lo): the pair one 16-bit slot further along
__device__ __forceinline__ uint32_t align16(uint32_t hi, uint32_t lo) {
  return __builtin_amdgcn_alignbit(hi, lo, 16);
}
// lo halves of two registers -> (lo(a), lo(b)); hi halves -> (hi(a), hi(b))
__device__ __forceinline__ uint32_t lo_halves(uint32_t a, uint32_t b) {
  return __builtin_amdgcn_perm(b, a, 0x05040100u);
}
__device__ __forceinline__ uint32_t hi_halves(uint32_t a, uint32_t b) {
  return __builtin_amdgcn_perm(b, a, 0x07060302u);
}
// bitwise select: bits of a where m is set, else b
__device__ __forceinline__ uint32_t bsel(uint32_t m, uint32_t a, uint32_t b) { return (a & m) | (b & ~m); }

// Mask of the half of register j that holds position `target` (relative to
// the lane's first sample), for positions base (lo) and base + 2 (hi).
__device__ __forceinline__ uint32_t half_at(int target, int base) {
  return target == base ? 0x0000FFFFu : (target == base + 2 ? 0xFFFF0000u : 0u);
}

template <int M> struct Pk { static constexpr int P = M >= 2 ? M / 2 : 1; };

// Forward 1-D lifting of one row across the wavefront, packed layout.
// EDGE: the lane group may hold index 0 or N-1 of the level's signal, where
// whole-sample mirroring replaces the missing neighbour.
template <int M, bool EDGE>
__device__ __forceinline__ void hfwd_pk(uint32_t (&E)[Pk<M>::P], uint32_t (&O)[Pk<M>::P], int j0, int N) {
  constexpr int P = Pk<M>::P;
  const uint32_t nxt = uint32_t(from_next_lane(int(E[0])));
  int tgt = N - 1 - j0;
  if (EDGE) {
    // recompute the edge masks at every use rather than keeping them live in
    // registers for the whole stream (only edge wavefronts run this)
    asm volatile("" : "+v"(tgt), "+v"(j0));
  }
  uint32_t D[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    uint32_t en = (j + 1 < P) ? align16(E[j + 1], E[j]) : (M >= 2 ? align16(nxt, E[j]) : nxt);
    if (EDGE) en = bsel(half_at(tgt, 4 * j + 1), E[j], en);   // x(N) = x(N-2)
    D[j] = pk_predict(O[j], E[j], en);
  }
  const uint32_t prv = uint32_t(from_prev_lane(int(D[P - 1])));
#pragma unroll
  for (int j = 0; j < P; ++j) {
    uint32_t dl = (j > 0) ? align16(D[j], D[j - 1]) : (M >= 2 ? align16(D[0], prv) : prv);
    uint32_t dr = D[j];
    if (EDGE) {
      if (j == 0) dl = bsel(j0 == 0 ? 0x0000FFFFu : 0u, D[0], dl);  // d(-1) = d(1)
      dr = bsel(half_at(tgt, 4 * j), dl, dr);                       // d(N) = d(N-2)
    }
    E[j] = pk_update(E[j], dl, dr);
  }
#pragma unroll
  for (int j = 0; j < P; ++j) O[j] = D[j];
}

template <int M>
__device__ __forceinline__ void hfwd_pk_any(uint32_t (&E)[Pk<M>::P], uint32_t (&O)[Pk<M>::P], int j0,
                                            int N, bool edge) {
  if (N == 1) return;
  if (edge) hfwd_pk<M, true>(E, O, j0, N);
  else hfwd_pk<M, false>(E, O, j0, N);
}

// Inverse of hfwd_pk: E holds lows, O highs; undo the update (5.2) on the
// evens, then the predict (5.1) on the odds.  The same neighbour pairs and
// mirror rules as the forward, taken in reverse order.
template <int M, bool EDGE>
__device__ __forceinline__ void hinv_pk(uint32_t (&E)[Pk<M>::P], uint32_t (&O)[Pk<M>::P], int j0, int N) {
  constexpr int P = Pk<M>::P;
  int tgt = N - 1 - j0;
  if (EDGE) asm volatile("" : "+v"(tgt), "+v"(j0));
  const uint32_t prv = uint32_t(from_prev_lane(int(O[P - 1])));
#pragma unroll
  for (int j = 0; j < P; ++j) {
    uint32_t dl = (j > 0) ? align16(O[j], O[j - 1]) : (M >= 2 ? align16(O[0], prv) : prv);
    uint32_t dr = O[j];
    if (EDGE) {
      if (j == 0) dl = bsel(j0 == 0 ? 0x0000FFFFu : 0u, O[0], dl);  // d(-1) = d(1)
      dr = bsel(half_at(tgt, 4 * j), dl, dr);                       // d(N) = d(N-2)
    }
    E[j] = pk_sub(E[j], pk_sra(pk_add(pk_add(dl, dr), 0x00020002u), 2));
  }
  const uint32_t nxt = uint32_t(from_next_lane(int(E[0])));
#pragma unroll
  for (int j = 0; j < P; ++j) {
    uint32_t en = (j + 1 < P) ? align16(E[j + 1], E[j]) : (M >= 2 ? align16(nxt, E[j]) : nxt);
    if (EDGE) en = bsel(half_at(tgt, 4 * j + 1), E[j], en);   // x(N) = x(N-2)
    O[j] = pk_add(O[j], pk_sra(pk_add(E[j], en), 1));
  }
}

template <int M>
__device__ __forceinline__ void hinv_pk_any(uint32_t (&E)[Pk<M>::P], uint32_t (&O)[Pk<M>::P], int j0,
                                            int N, bool edge) {
  if (N == 1) return;
  if (edge) hinv_pk<M, true>(E, O, j0, N);
  else hinv_pk<M, false>(E, O, j0, N);
}

}  // namespace dwtfrag
