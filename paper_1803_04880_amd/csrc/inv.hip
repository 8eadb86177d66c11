// Inverse path: AES-CTR decryption of the LL band fused with the multi-level
// inverse 5/3 lifting, as one streaming kernel (Ch. 5 section 5.2.3: the map
// is an invertible integer-to-integer map, so restore is exact).
//
// Within a level the vertical pass is undone first, then the horizontal one
// (the reverse of the forward order).  A wavefront streams the LL rows of the
// coarsest level; a step of level l consumes LL_l row k together with the
// detail rows k of HL_l / LH_l / HH_l and emits rows 2k-1 and 2k of the
// level-(l-1) grid, which are inverted horizontally and become LL_(l-1) rows
// for level l-1.  Level 1 emits output rows.
#include "batch.h"
#include "lift.h"
#include "pack.h"

namespace dwtfrag {

template <int L, int C1, bool U8OUT>
struct InvWave {
  template <int l> static constexpr int C = C1 >> (l - 1);

  const StageParams &P;
  const int16_t *llin;     // LL_L (priv bytes or int16 scratch)
  const int16_t *pub;
  uint8_t *out8;
  int16_t *out16;
  KsRing ks;
  int lane;
  int c0;
  int X0, Y0, X1, Y1;
  bool last_win, last_seg;

  // detail rows of the next step of each level, loaded one step ahead
  template <int l> static constexpr int U = (C<l> / 2) > 0 ? C<l> / 2 : 1;
  template <int l> static constexpr int RWd = Raw<U<l>>::W;
  uint32_t Fh1[RWd<1>], Fl1[RWd<1>], Fx1[RWd<1>];
  uint32_t Fh2[RWd<2>], Fl2[RWd<2>], Fx2[RWd<2>];
  uint32_t Fh3[RWd<3>], Fl3[RWd<3>], Fx3[RWd<3>];
  uint32_t Fh4[RWd<4>], Fl4[RWd<4>], Fx4[RWd<4>];

  int Dp1[C<1>], Xp1[C<1>];
  int Dp2[C1 >= 2 ? C<2> : 1], Xp2[C1 >= 2 ? C<2> : 1];
  int Dp3[C1 >= 4 ? C<3> : 1], Xp3[C1 >= 4 ? C<3> : 1];
  int Dp4[C1 >= 8 ? C<4> : 1], Xp4[C1 >= 8 ? C<4> : 1];
  int k0[kMaxFused + 1];   // first step index of each level's stream
  bool hedge[kMaxFused + 1];

  template <int l> __device__ auto &Dp() {
    if constexpr (l == 1) return Dp1; else if constexpr (l == 2) return Dp2;
    else if constexpr (l == 3) return Dp3; else return Dp4;
  }
  template <int l> __device__ auto &Xp() {
    if constexpr (l == 1) return Xp1; else if constexpr (l == 2) return Xp2;
    else if constexpr (l == 3) return Xp3; else return Xp4;
  }
  template <int l> __device__ auto &Fh() {
    if constexpr (l == 1) return Fh1; else if constexpr (l == 2) return Fh2;
    else if constexpr (l == 3) return Fh3; else return Fh4;
  }
  template <int l> __device__ auto &Fl() {
    if constexpr (l == 1) return Fl1; else if constexpr (l == 2) return Fl2;
    else if constexpr (l == 3) return Fl3; else return Fl4;
  }
  template <int l> __device__ auto &Fx() {
    if constexpr (l == 1) return Fx1; else if constexpr (l == 2) return Fx2;
    else if constexpr (l == 3) return Fx3; else return Fx4;
  }

  // Issue the loads of step k's detail rows of level l (HL_l row k; LH_l and
  // HH_l row k when they exist), to be consumed by that step.
  template <int l> __device__ __forceinline__ void prefetch(int k) {
    constexpr int UU = C<l> / 2;
    const int N = P.hdim[l - 1];
    const int Nw = P.wdim[l - 1];
    const int wl = P.wdim[l];
    const int bc = c0 >> l;
    if (k < P.hdim[l])
      load_raw<UU>(pub + P.off_hl[l], int64_t(k) * (Nw - wl) + bc, (Nw - wl) - bc, Fh<l>());
    if (2 * k + 1 < N) {
      load_raw<UU>(pub + P.off_lh[l], int64_t(k) * wl + bc, wl - bc, Fl<l>());
      load_raw<UU>(pub + P.off_hh[l], int64_t(k) * (Nw - wl) + bc, (Nw - wl) - bc, Fx<l>());
    }
  }

  // Row i of the level-(l-1) grid after the vertical inverse of level l:
  // undo the horizontal pass, then hand it down.
  template <int l> __device__ __forceinline__ void emit_row(int (&x)[C<l>], int i) {
    constexpr int CC = C<l>;
    hinv_any<CC>(x, c0 >> (l - 1), P.wdim[l - 1], hedge[l]);
    if constexpr (l > 1) {
      push_ll<l - 1>(x, i);
    } else {
      if (i < Y0 || (!last_seg && i >= Y1)) return;
      if (c0 < X0 || (!last_win && c0 >= X1)) return;
      const int64_t idx = int64_t(i) * P.W + c0;
      if constexpr (U8OUT) {
        // bytes of this lane's columns inside the view: the row's end, and n
        // (the last row may be partial)
        const int64_t lim = min(int64_t(P.W - c0), P.n_valid - idx);
        if (lim >= C1 && (idx & (C1 - 1)) == 0) {
          uint32_t w[C1 / 4];
#pragma unroll
          for (int q = 0; q < C1 / 4; ++q)
            w[q] = (uint32_t(x[4 * q]) & 0xFFu) | ((uint32_t(x[4 * q + 1]) & 0xFFu) << 8) |
                   ((uint32_t(x[4 * q + 2]) & 0xFFu) << 16) | (uint32_t(x[4 * q + 3]) << 24);
          if constexpr (C1 == 8) *(gptr<u32x2>)(glob(out8) + idx) = u32x2{w[0], w[1]};
          else *(gptr<u32x4>)(glob(out8) + idx) = u32x4{w[0], w[1], w[2], w[3]};
        } else {
#pragma unroll
          for (int t = 0; t < C1; ++t)
            if (t < lim) glob(out8)[idx + t] = uint8_t(x[t]);
        }
      } else {
        store_i16<C1>(out16, idx, P.W - c0, x);
      }
    }
  }

  // Step k of level l: LL_l row k arrives (values of this lane's LL columns).
  // The step yields up to three rows of the level-(l-1) grid (2k-1, 2k and,
  // at the end of an even-length signal, 2k+1), emitted from one call site.
  template <int l> __device__ __forceinline__ void push_ll(const int (&ll)[C<l> / 2], int k) {
    constexpr int CC = C<l>;
    constexpr int U = CC / 2;
    const int N = P.hdim[l - 1];
    int hl[U];
    unpack_raw<U>(Fh<l>(), hl);
    int S[CC];
#pragma unroll
    for (int u = 0; u < U; ++u) { S[2 * u] = ll[u]; S[2 * u + 1] = hl[u]; }
    auto &Dv = Dp<l>();
    auto &Xv = Xp<l>();
    int R0[CC], R1[CC], R2[CC];
    int e_begin = 1, e_end = 2;
    if (N == 1) {  // no vertical pass at this level: the row is row 0
#pragma unroll
      for (int t = 0; t < CC; ++t) R1[t] = S[t];
    } else {
      int Dn[CC];
      const bool has_d = (2 * k + 1 < N);
      if (has_d) {
        int lh[U], hh[U];
        unpack_raw<U>(Fl<l>(), lh);
        unpack_raw<U>(Fx<l>(), hh);
#pragma unroll
        for (int u = 0; u < U; ++u) { Dn[2 * u] = lh[u]; Dn[2 * u + 1] = hh[u]; }
      } else {  // odd length, last step: d(N) = d(N-2)
#pragma unroll
        for (int t = 0; t < CC; ++t) Dn[t] = Dv[t];
      }
      prefetch<l>(k + 1);
      const bool top = (k == 0);
#pragma unroll
      for (int t = 0; t < CC; ++t) {
        const int X = S[t] - (((top ? Dn[t] : Dv[t]) + Dn[t] + 2) >> 2);
        R0[t] = Dv[t] + ((Xv[t] + X) >> 1);  // x(2k-1)
        R1[t] = X;                             // x(2k)
        R2[t] = Dn[t] + X;                     // x(2k+1) when 2k+1 == N-1
        Dv[t] = Dn[t];
        Xv[t] = X;
      }
      if (k != k0[l]) e_begin = 0;
      if (2 * k + 1 == N - 1) e_end = 3;
    }
#pragma unroll 1
    for (int e = e_begin; e < e_end; ++e) {
      int row[CC];
#pragma unroll
      for (int t = 0; t < CC; ++t) row[t] = e == 0 ? R0[t] : (e == 1 ? R1[t] : R2[t]);
      emit_row<l>(row, 2 * k - 1 + e);
    }
  }

  __device__ __forceinline__ void load_ll(int k, int (&ll)[C<L> / 2]) {
    constexpr int U = C<L> / 2;
    const int wl = P.wdim[L];
    const int bc = c0 >> L;
    load_i16<U>(llin, int64_t(k) * wl + bc, wl - bc, ll);
  }

  __device__ __forceinline__ void run(int wave) {
    const int win = wave % P.n_win;
    const int seg = wave / P.n_win;
    X0 = win * P.own_w;
    last_win = (win == P.n_win - 1);
    last_seg = (seg == P.n_seg - 1);
    Y0 = seg_start(P, seg);
    X1 = last_win ? P.W : X0 + P.own_w;
    Y1 = last_seg ? P.H : seg_start(P, seg + 1);
    const int cbase = window_base(P, win);
    c0 = cbase + lane * C1;
    const int kbeg = (Y0 > P.halo_t ? Y0 - P.halo_t : 0) >> L;
    const int kend = min(P.hdim[L], (Y1 + P.halo_b) >> L);
#pragma unroll
    for (int l = 1; l <= L; ++l) {
      k0[l] = kbeg << (L - l);
      const int N = P.wdim[l - 1];
      const int j0 = cbase >> (l - 1);
      const int span = (64 * C1) >> (l - 1);
      hedge[l] = (j0 == 0) || (N - 1 >= j0 && N - 1 < j0 + span);
    }
    for (int t = 0; t < C<1>; ++t) { Dp1[t] = 0; Xp1[t] = 0; }
    for (int t = 0; t < (C1 >= 2 ? C<2> : 1); ++t) { Dp2[t] = 0; Xp2[t] = 0; }
    for (int t = 0; t < (C1 >= 4 ? C<3> : 1); ++t) { Dp3[t] = 0; Xp3[t] = 0; }
    for (int t = 0; t < (C1 >= 8 ? C<4> : 1); ++t) { Dp4[t] = 0; Xp4[t] = 0; }
    ks.col_lo = min(P.wdim[L], cbase >> L);
    ks.col_hi = min(P.wdim[L], (cbase + 64 * C1) >> L);
    ks.wL = P.wdim[L];
    ks.base = -1;

    if (kbeg >= kend) return;
    prefetch<1>(k0[1]);
    if constexpr (L >= 2) prefetch<2>(k0[2]);
    if constexpr (L >= 3) prefetch<3>(k0[3]);
    if constexpr (L >= 4) prefetch<4>(k0[4]);
    constexpr int U = C<L> / 2;
    int nxt[U];
    load_ll(kbeg, nxt);
    for (int k = kbeg; k < kend; ++k) {
      int cur[U];
#pragma unroll
      for (int u = 0; u < U; ++u) cur[u] = nxt[u];
      if (k + 1 < kend) load_ll(k + 1, nxt);
      if (P.use_aes) {
        ks.ensure(k, kend, lane);
        const int nv = P.wdim[L] - (c0 >> L);
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (u < nv) cur[u] = int(int16_t(uint16_t(cur[u]) ^ uint16_t(ks.ks16(k, (c0 >> L) + u))));
      }
      push_ll<L>(cur, k);
    }
  }
};

// Packed form of the same stream (two int16 samples per register, the
// forward's layout: E = lows, O = highs, see pack.h).  Exact when every value
// a level reads (LL row, HL, LH, HH) lies in [-4096, 4095]: then the vertical
// inverse gives |x| <= 10240, the horizontal one evens <= 15360 and odds
// <= 25600, and no sum exceeds 30720, so 16 bits never wrap.  Fragments made
// by protect stay far inside that range.  The stream checks every value it
// reads; run() returns false when one was outside, and the caller then redoes
// the wavefront's rectangle with the 32-bit stream above (same output bytes
// as the exact integer inverse for any fragments).
template <int L, int C1, bool U8OUT, bool FAST>
struct InvWavePk {
  template <int l> static constexpr int M = (C1 >> (l - 1)) / 2;  // evens per lane at level l
  template <int l> static constexpr int NP = Pk<M<l>>::P;         // words per parity
  template <int l> static constexpr int R = 2 * NP<l>;            // words per row: E then O
  static constexpr uint32_t kBias = 0x10001000u;   // [-4096, 4095] -> [0, 8191]
  static constexpr uint32_t kOutside = 0xE000E000u;

  const StageParams &P;
  const int16_t *llin;
  const int16_t *pub;
  uint8_t *out8;
  int16_t *out16;
  KsRing ks;
  int lane;
  int c0;
  int X0, Y0, X1, Y1;
  bool last_win, last_seg;
  uint32_t chk;            // OR of every biased value read

  // detail rows of the next step of each level, as loaded (band order is
  // the packed order: HL / HH words are O words, LH words E words)
  uint32_t Fh1[NP<1>], Fl1[NP<1>], Fx1[NP<1>];
  uint32_t Fh2[NP<2>], Fl2[NP<2>], Fx2[NP<2>];
  uint32_t Fh3[NP<3>], Fl3[NP<3>], Fx3[NP<3>];
  uint32_t Fh4[NP<4>], Fl4[NP<4>], Fx4[NP<4>];
  // vertical state: previous detail row and previous even row (E then O)
  uint32_t Dp1[R<1>], Xp1[R<1>];
  uint32_t Dp2[R<2>], Xp2[R<2>];
  uint32_t Dp3[R<3>], Xp3[R<3>];
  uint32_t Dp4[R<4>], Xp4[R<4>];
  int k0[kMaxFused + 1];
  bool hedge[kMaxFused + 1];
  // FAST (chosen per wavefront, see wave_is_fast): every lane's vector of
  // every band row lies inside its band, band rows are vector aligned and
  // every lane's output bytes lie inside a row.  Rows are then read at
  // (uniform row address + this lane's byte offset) with no per-lane bounds,
  // and output rows are written the same way under the column ownership.
  uint32_t voff[kMaxFused + 1];  // this lane's byte offset in a band row of level l
  bool own_col;                  // this lane's output columns belong to the wavefront

  template <int l> __device__ auto &Dp() {
    if constexpr (l == 1) return Dp1; else if constexpr (l == 2) return Dp2;
    else if constexpr (l == 3) return Dp3; else return Dp4;
  }
  template <int l> __device__ auto &Xp() {
    if constexpr (l == 1) return Xp1; else if constexpr (l == 2) return Xp2;
    else if constexpr (l == 3) return Xp3; else return Xp4;
  }
  template <int l> __device__ auto &Fh() {
    if constexpr (l == 1) return Fh1; else if constexpr (l == 2) return Fh2;
    else if constexpr (l == 3) return Fh3; else return Fh4;
  }
  template <int l> __device__ auto &Fl() {
    if constexpr (l == 1) return Fl1; else if constexpr (l == 2) return Fl2;
    else if constexpr (l == 3) return Fl3; else return Fl4;
  }
  template <int l> __device__ auto &Fx() {
    if constexpr (l == 1) return Fx1; else if constexpr (l == 2) return Fx2;
    else if constexpr (l == 3) return Fx3; else return Fx4;
  }

  template <int n> __device__ __forceinline__ void check(const uint32_t (&w)[n]) {
    if constexpr (n == 1) {
      chk |= pk_add(w[0], kBias);
    } else {
#pragma unroll
      for (int j = 0; j + 1 < n; j += 2) chk = chk | pk_add(w[j], kBias) | pk_add(w[j + 1], kBias);
    }
  }

  // UU int16 values at (row + off), UU-aligned: one vector load.
  template <int UU> __device__ __forceinline__ static void load_vec(const char *row, uint32_t off,
                                                                     uint32_t (&w)[Raw<UU>::W]) {
    const gptr<const char> p = glob(row) + off;
    if constexpr (UU == 1) {
      w[0] = *(gptr<const uint16_t>)p;
    } else if constexpr (UU == 2) {
      w[0] = *(gptr<const uint32_t>)p;
    } else if constexpr (UU == 4) {
      const u32x2 q = *(gptr<const u32x2>)p;
      w[0] = q.x; w[1] = q.y;
    } else {
      const u32x4 q = *(gptr<const u32x4>)p;
      w[0] = q.x; w[1] = q.y; w[2] = q.z; w[3] = q.w;
    }
  }

  template <int l> __device__ __forceinline__ void prefetch(int k) {
    constexpr int UU = M<l>;
    const int N = P.hdim[l - 1];
    const int Nw = P.wdim[l - 1];
    const int wl = P.wdim[l];
    const int bc = c0 >> l;
    if constexpr (FAST) {
      const char *base = reinterpret_cast<const char *>(pub);
      if (k < P.hdim[l])
        load_vec<UU>(base + 2 * (P.off_hl[l] + int64_t(k) * (Nw - wl)), voff[l], Fh<l>());
      if (2 * k + 1 < N) {
        load_vec<UU>(base + 2 * (P.off_lh[l] + int64_t(k) * wl), voff[l], Fl<l>());
        load_vec<UU>(base + 2 * (P.off_hh[l] + int64_t(k) * (Nw - wl)), voff[l], Fx<l>());
      }
    } else {
    if (k < P.hdim[l])
      load_raw<UU>(pub + P.off_hl[l], int64_t(k) * (Nw - wl) + bc, (Nw - wl) - bc, Fh<l>());
    if (2 * k + 1 < N) {
      load_raw<UU>(pub + P.off_lh[l], int64_t(k) * wl + bc, wl - bc, Fl<l>());
      load_raw<UU>(pub + P.off_hh[l], int64_t(k) * (Nw - wl) + bc, (Nw - wl) - bc, Fx<l>());
    }
    }
  }

  // Row i of the level-(l-1) grid after the vertical inverse of level l.
  template <int l> __device__ __forceinline__ void emit_row(const uint32_t (&x)[R<l>], int i) {
    constexpr int Np = NP<l>;
    uint32_t E[Np], O[Np];
#pragma unroll
    for (int j = 0; j < Np; ++j) { E[j] = x[j]; O[j] = x[Np + j]; }
    hinv_pk_any<M<l>>(E, O, c0 >> (l - 1), P.wdim[l - 1], hedge[l]);
    if constexpr (l > 1) {
      // the row in memory order is the LL row of level l-1
      uint32_t ll[NP<l - 1>];
#pragma unroll
      for (int j = 0; j < Np; ++j) {
        ll[2 * j] = lo_halves(E[j], O[j]);
        if constexpr (M<l> >= 2) ll[2 * j + 1] = hi_halves(E[j], O[j]);
      }
      push_ll<l - 1>(ll, i);
    } else {
      if (i < Y0 || (!last_seg && i >= Y1)) return;
      if constexpr (U8OUT) {
        if (FAST && int64_t(i + 1) * P.W <= P.n_valid) {
          uint32_t w[C1 / 4];
#pragma unroll
          for (int q = 0; q < C1 / 4; ++q) w[q] = __builtin_amdgcn_perm(O[q], E[q], 0x06020400u);
          const gptr<uint8_t> row = glob(out8) + int64_t(i) * P.W;
          if (own_col) {
            if constexpr (C1 == 8) *(gptr<u32x2>)(row + uint32_t(c0)) = u32x2{w[0], w[1]};
            else *(gptr<u32x4>)(row + uint32_t(c0)) = u32x4{w[0], w[1], w[2], w[3]};
          }
          return;
        }
      }
      if (c0 < X0 || (!last_win && c0 >= X1)) return;
      const int64_t idx = int64_t(i) * P.W + c0;
      if constexpr (U8OUT) {
        // bytes of this lane's columns inside the view: the row's end, and n
        const int64_t lim = min(int64_t(P.W - c0), P.n_valid - idx);
        uint32_t w[C1 / 4];
#pragma unroll
        for (int q = 0; q < C1 / 4; ++q) w[q] = __builtin_amdgcn_perm(O[q], E[q], 0x06020400u);
        if (lim >= C1 && (idx & (C1 - 1)) == 0) {
          if constexpr (C1 == 8) *(gptr<u32x2>)(glob(out8) + idx) = u32x2{w[0], w[1]};
          else *(gptr<u32x4>)(glob(out8) + idx) = u32x4{w[0], w[1], w[2], w[3]};
        } else {
#pragma unroll
          for (int t = 0; t < C1; ++t)
            if (t < lim) glob(out8)[idx + t] = uint8_t(w[t >> 2] >> (8 * (t & 3)));
        }
      } else {
        uint32_t w[C1 / 2];
#pragma unroll
        for (int q = 0; q < C1 / 4; ++q) {
          w[2 * q] = lo_halves(E[q], O[q]);
          w[2 * q + 1] = hi_halves(E[q], O[q]);
        }
        const int64_t lim = int64_t(P.W - c0);
        if (lim >= C1 && (idx & (C1 - 1)) == 0) {
#pragma unroll
          for (int q = 0; q < C1 / 8; ++q)
            ((gptr<u32x4>)(glob(out16) + idx))[q] =
                u32x4{w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]};
        } else {
#pragma unroll
          for (int t = 0; t < C1; ++t)
            if (t < lim) glob(out16)[idx + t] = int16_t(uint16_t(w[t >> 1] >> (16 * (t & 1))));
        }
      }
    }
  }

  // Step k of level l: LL_l row k arrives as E words (band order).
  template <int l> __device__ __forceinline__ void push_ll(const uint32_t (&ll)[NP<l>], int k) {
    constexpr int Np = NP<l>;
    constexpr int Rl = R<l>;
    const int N = P.hdim[l - 1];
    uint32_t S[Rl];
#pragma unroll
    for (int j = 0; j < Np; ++j) { S[j] = ll[j]; S[Np + j] = Fh<l>()[j]; }
    check(S);
    auto &Dv = Dp<l>();
    auto &Xv = Xp<l>();
    uint32_t Ra[Rl], Rb[Rl];   // rows 2k-1 and 2k
    bool last_pair = false;
    int e_begin = 1;
    if (N == 1) {  // no vertical pass at this level: the row is row 0
#pragma unroll
      for (int t = 0; t < Rl; ++t) Rb[t] = S[t];
    } else {
      uint32_t Dn[Rl];
      if (2 * k + 1 < N) {
#pragma unroll
        for (int j = 0; j < Np; ++j) { Dn[j] = Fl<l>()[j]; Dn[Np + j] = Fx<l>()[j]; }
        check(Dn);
      } else {  // odd length, last step: d(N) = d(N-2)
#pragma unroll
        for (int t = 0; t < Rl; ++t) Dn[t] = Dv[t];
      }
      prefetch<l>(k + 1);
      const bool top = (k == 0);
#pragma unroll
      for (int t = 0; t < Rl; ++t) {
        const uint32_t X = pk_sub(S[t], pk_sra(pk_add(pk_add(top ? Dn[t] : Dv[t], Dn[t]), 0x00020002u), 2));
        Ra[t] = pk_add(Dv[t], pk_sra(pk_add(Xv[t], X), 1));
        Rb[t] = X;
        Dv[t] = Dn[t];
        Xv[t] = X;
      }
      last_pair = (2 * k + 1 == N - 1);  // even length: row 2k+1 = d + x(2k)
      if (k != k0[l]) e_begin = 0;
    }
    if constexpr (l == 1) {
      // level-1 rows end in stores, not in further levels: a call site per
      // row costs little code and needs no row selects
      if (e_begin == 0) emit_row<1>(Ra, 2 * k - 1);
      emit_row<1>(Rb, 2 * k);
      if (last_pair) {
#pragma unroll
        for (int t = 0; t < Rl; ++t) Ra[t] = pk_add(Dv[t], Xv[t]);
        emit_row<1>(Ra, 2 * k + 1);
      }
    } else {
      const int e_end = last_pair ? 3 : 2;
      // one call site per level (each inlines the finer levels): the rows
      // go through a loop
#pragma unroll 1
      for (int e = e_begin; e < e_end; ++e) {
        uint32_t row[Rl];
#pragma unroll
        for (int t = 0; t < Rl; ++t) row[t] = (e & 1) ? Rb[t] : Ra[t];
        emit_row<l>(row, 2 * k - 1 + e);
        if (e == 1 && last_pair) {
#pragma unroll
          for (int t = 0; t < Rl; ++t) Ra[t] = pk_add(Dv[t], Xv[t]);
        }
      }
    }
  }

  __device__ __forceinline__ void load_ll(int k, uint32_t (&ll)[NP<L>]) {
    const int wl = P.wdim[L];
    const int bc = c0 >> L;
    load_raw<M<L>>(llin, int64_t(k) * wl + bc, wl - bc, ll);
  }

  // Returns false when a value outside [-4096, 4095] was read (the packed
  // results are then not trusted).
  __device__ __forceinline__ bool run(int wave) {
    const int win = wave % P.n_win;
    const int seg = wave / P.n_win;
    X0 = win * P.own_w;
    last_win = (win == P.n_win - 1);
    last_seg = (seg == P.n_seg - 1);
    Y0 = seg_start(P, seg);
    X1 = last_win ? P.W : X0 + P.own_w;
    Y1 = last_seg ? P.H : seg_start(P, seg + 1);
    const int cbase = window_base(P, win);
    c0 = cbase + lane * C1;
    const int kbeg = (Y0 > P.halo_t ? Y0 - P.halo_t : 0) >> L;
    const int kend = min(P.hdim[L], (Y1 + P.halo_b) >> L);
#pragma unroll
    for (int l = 1; l <= L; ++l) {
      k0[l] = kbeg << (L - l);
      const int N = P.wdim[l - 1];
      const int j0 = cbase >> (l - 1);
      const int span = (64 * C1) >> (l - 1);
      hedge[l] = (j0 == 0) || (N - 1 >= j0 && N - 1 < j0 + span);
    }
#pragma unroll
    for (int l = 1; l <= L; ++l) voff[l] = 2u * uint32_t(c0 >> l);
    own_col = c0 >= X0 && (last_win || c0 < X1);
    chk = 0;
#pragma unroll
    for (int t = 0; t < R<1>; ++t) { Dp1[t] = 0; Xp1[t] = 0; }
#pragma unroll
    for (int t = 0; t < R<2>; ++t) { Dp2[t] = 0; Xp2[t] = 0; }
#pragma unroll
    for (int t = 0; t < R<3>; ++t) { Dp3[t] = 0; Xp3[t] = 0; }
#pragma unroll
    for (int t = 0; t < R<4>; ++t) { Dp4[t] = 0; Xp4[t] = 0; }
    ks.col_lo = min(P.wdim[L], cbase >> L);
    ks.col_hi = min(P.wdim[L], (cbase + 64 * C1) >> L);
    ks.wL = P.wdim[L];
    ks.base = -1;

    if (kbeg >= kend) return true;
    prefetch<1>(k0[1]);
    if constexpr (L >= 2) prefetch<2>(k0[2]);
    if constexpr (L >= 3) prefetch<3>(k0[3]);
    if constexpr (L >= 4) prefetch<4>(k0[4]);
    constexpr int Np = NP<L>;
    uint32_t nxt[Np];
    load_ll(kbeg, nxt);
    for (int k = kbeg; k < kend; ++k) {
      uint32_t cur[Np];
#pragma unroll
      for (int j = 0; j < Np; ++j) cur[j] = nxt[j];
      if (k + 1 < kend) load_ll(k + 1, nxt);
      if (P.use_aes) {
        ks.ensure(k, kend, lane);
        const int bc = c0 >> L;
        const int nv = P.wdim[L] - bc;
#pragma unroll
        for (int u = 0; u < (M<L> >= 2 ? 2 * Np : 1); ++u)
          if (u < nv) cur[u >> 1] ^= ks.ks16(k, bc + u) << (16 * (u & 1));
      }
      push_ll<L>(cur, k);
    }
    return __builtin_amdgcn_ballot_w64((chk & kOutside) != 0) == 0;
  }
};

template <class Wv>
__device__ __forceinline__ void inv_setup(Wv &w, const int16_t *llin, const int16_t *pub, void *out,
                                          int lane, uint32_t *ring, const uint32_t *te,
                                          const uint32_t *kw) {
  w.llin = llin;
  w.pub = pub;
  w.out8 = static_cast<uint8_t *>(out);
  w.out16 = static_cast<int16_t *>(out);
  w.lane = lane;
  w.ks.ring = ring;
  w.ks.te = te;
  w.ks.kw = kw;
  w.ks.rows = w.P.ks_rows;
  w.ks.blocks = w.P.ks_blocks;
}

// Whether the wavefront's lanes all read whole, aligned vectors from every
// band row of every level and write whole output vectors (wave-uniform).
template <int L, int C1, bool U8OUT>
__device__ __forceinline__ bool wave_is_fast(const StageParams &P, int wave, int lane) {
  const int win = wave % P.n_win;
  const int cbase = window_base(P, win);
  const int c0 = cbase + lane * C1;
  bool bad = !U8OUT || P.W % C1 != 0 || c0 + C1 > P.W;
#pragma unroll
  for (int l = 1; l <= L; ++l) {
    const int uu = (C1 >> (l - 1)) / 2;
    const int wl = P.wdim[l];
    const int wh = P.wdim[l - 1] - wl;
    const int bc = c0 >> l;
    bad = bad || wl % uu != 0 || wh % uu != 0 || P.off_hl[l] % uu != 0 || P.off_lh[l] % uu != 0 ||
          P.off_hh[l] % uu != 0 || wl - bc < uu || wh - bc < uu;
  }
  return __builtin_amdgcn_ballot_w64(bad) == 0;
}

// One wavefront's rectangle: the packed stream, redone with the 32-bit
// stream when a value fell outside the packed range.
template <int L, int C1, bool U8OUT>
__device__ __forceinline__ void inv_wave(const StageParams &P, int wave, const int16_t *llin,
                                         const int16_t *pub, void *out, int lane, uint32_t *ring,
                                         const uint32_t *te, const uint32_t *kw) {
  if (wave_is_fast<L, C1, U8OUT>(P, wave, lane)) {
    InvWavePk<L, C1, U8OUT, true> w{P};
    inv_setup(w, llin, pub, out, lane, ring, te, kw);
    if (w.run(wave)) return;
  } else {
    InvWavePk<L, C1, U8OUT, false> w{P};
    inv_setup(w, llin, pub, out, lane, ring, te, kw);
    if (w.run(wave)) return;
  }
  wave_lds_sync();
  InvWave<L, C1, U8OUT> x{P};
  inv_setup(x, llin, pub, out, lane, ring, te, kw);
  x.run(wave);
}

template <int L, int C1, bool U8OUT>
__device__ __forceinline__ void inv_body(const int16_t *__restrict__ llin,
                                         const int16_t *__restrict__ pub, void *__restrict__ out,
                                         const StageParams &P) {
  __shared__ uint32_t s_te[1024];
  __shared__ uint32_t s_kw[kKeyWords];
  __shared__ uint32_t s_ring[kWavesPerBlock][kRingBlocks * 4];
  if (P.use_aes) load_aes_tables(s_te, s_kw, P.key);
  __syncthreads();
  // the wavefront index is uniform; readfirstlane lets the compiler see that,
  // so all row / level bookkeeping derived from it stays scalar
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wave = blockIdx.x * kWavesPerBlock + wib;
  if (wave >= P.n_waves) return;
  inv_wave<L, C1, U8OUT>(P, wave, llin, pub, out, int(threadIdx.x & 63), s_ring[wib], s_te, s_kw);
}

// Eight columns per lane: held to 128 VGPRs (four wavefronts per SIMD), the
// occupancy that hides the detail-row loads.
template <int L, bool U8OUT>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(4)))
void inv_kernel8(const int16_t *__restrict__ llin, const int16_t *__restrict__ pub,
                 void *__restrict__ out, const StageParams P) {
  inv_body<L, 8, U8OUT>(llin, pub, out, P);
}

// Sixteen columns per lane need more registers than that: two wavefronts
// per SIMD (256 VGPRs).
template <int L, bool U8OUT>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(2)))
void inv_kernel16(const int16_t *__restrict__ llin, const int16_t *__restrict__ pub,
                  void *__restrict__ out, const StageParams P) {
  inv_body<L, 16, U8OUT>(llin, pub, out, P);
}

// ---- split restore -----------------------------------------------------
// The 32-bit redo of a wavefront whose fragments hold values outside the
// packed range is rare, but its code in the same kernel as the packed streams
// costs those streams registers (spills).  For large byte outputs the restore
// therefore runs as two launches: the packed kernel (no redo code) writes
// kRedoMark into the first 16 bytes of a failed wavefront's output rectangle
// after all of its stores; the redo kernel then reads those 16 bytes of every
// rectangle and redoes, with the exact 32-bit stream, each one that holds the
// mark.  A rectangle whose correct output happens to equal the mark is redone
// too, which writes the same bytes: the mark decides only whether work is
// repeated, never the result.
__device__ __forceinline__ uint8_t redo_mark(int t) {
  constexpr uint32_t kRedoMark[4] = {0x3C8E15A7u, 0xD24B96F1u, 0x0B7F63E9u, 0x95A1C40Du};
  return uint8_t(kRedoMark[t >> 2] >> (8 * (t & 3)));
}

// Byte offset of a wavefront's output rectangle origin (its first owned row
// and column).
__device__ __forceinline__ int64_t rect_origin(const StageParams &P, int wave) {
  const int win = wave % P.n_win;
  const int seg = wave / P.n_win;
  return int64_t(seg_start(P, seg)) * P.W + int64_t(win) * P.own_w;
}

// ALL_FAST: the host found every wavefront FAST (see inv_all_fast), so only
// that stream is compiled in; a wavefront that is not (none, when the host is
// right) marks its rectangle for the redo without streaming.
template <int L, int C1, bool ALL_FAST>
__device__ __forceinline__ void inv_split_pk_body(const int16_t *__restrict__ llin,
                                                  const int16_t *__restrict__ pub,
                                                  uint8_t *__restrict__ out, const StageParams &P) {
  __shared__ uint32_t s_te[1024];
  __shared__ uint32_t s_kw[kKeyWords];
  __shared__ uint32_t s_ring[kWavesPerBlock][kRingBlocks * 4];
  if (P.use_aes) load_aes_tables(s_te, s_kw, P.key);
  __syncthreads();
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wave = blockIdx.x * kWavesPerBlock + wib;
  if (wave >= P.n_waves) return;
  const int lane = int(threadIdx.x & 63);
  bool ok = false;
  if (wave_is_fast<L, C1, true>(P, wave, lane)) {
    InvWavePk<L, C1, true, true> w{P};
    inv_setup(w, llin, pub, out, lane, s_ring[wib], s_te, s_kw);
    ok = w.run(wave);
  } else if constexpr (!ALL_FAST) {
    InvWavePk<L, C1, true, false> w{P};
    inv_setup(w, llin, pub, out, lane, s_ring[wib], s_te, s_kw);
    ok = w.run(wave);
  }
  if (!ok) {
    __threadfence();  // the wavefront's output stores land before the mark
    if (lane < 16) glob(out)[rect_origin(P, wave) + lane] = redo_mark(lane);
  }
}

template <int L, int C1>
__device__ __forceinline__ void inv_split_redo_body(const int16_t *__restrict__ llin,
                                                    const int16_t *__restrict__ pub,
                                                    uint8_t *__restrict__ out, const StageParams &P) {
  __shared__ uint32_t s_te[1024];
  __shared__ uint32_t s_kw[kKeyWords];
  __shared__ uint32_t s_ring[kWavesPerBlock][kRingBlocks * 4];
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wave = blockIdx.x * kWavesPerBlock + wib;
  const int lane = int(threadIdx.x & 63);
  bool marked = false;
  if (wave < P.n_waves) {
    const bool diff = lane < 16 && glob(out)[rect_origin(P, wave) + lane] != redo_mark(lane);
    marked = __builtin_amdgcn_ballot_w64(diff) == 0;
  }
  // tables only for workgroups with a marked rectangle
  const bool any = __syncthreads_or(marked) != 0;
  if (!any) return;
  if (P.use_aes) load_aes_tables(s_te, s_kw, P.key);
  __syncthreads();
  if (!marked) return;
  InvWave<L, C1, true> x{P};
  inv_setup(x, llin, pub, out, lane, s_ring[wib], s_te, s_kw);
  x.run(wave);
}

template <int L, bool ALL_FAST>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(4)))
void inv_split_pk8(const int16_t *__restrict__ llin, const int16_t *__restrict__ pub,
                   uint8_t *__restrict__ out, const StageParams P) {
  inv_split_pk_body<L, 8, ALL_FAST>(llin, pub, out, P);
}
template <int L, bool ALL_FAST>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(2)))
void inv_split_pk16(const int16_t *__restrict__ llin, const int16_t *__restrict__ pub,
                    uint8_t *__restrict__ out, const StageParams P) {
  inv_split_pk_body<L, 16, ALL_FAST>(llin, pub, out, P);
}
template <int L, int C1>
__global__ __launch_bounds__(kBlockThreads)
void inv_split_redo(const int16_t *__restrict__ llin, const int16_t *__restrict__ pub,
                    uint8_t *__restrict__ out, const StageParams P) {
  inv_split_redo_body<L, C1>(llin, pub, out, P);
}

// Whether a byte-output stage runs as the split pair: large enough that the
// second launch is negligible, and every rectangle's first row is complete
// and holds at least 16 owned columns (room for the mark).
static bool inv_split_ok(const StageParams &P) {
  if (P.n_valid < (int64_t(1) << 24)) return false;
  const int last_w = P.W - (P.n_win - 1) * P.own_w;
  if ((P.n_win > 1 && P.own_w < 16) || last_w < 16) return false;
  const int64_t last_y0 = int64_t(P.unit_rows) * ((int64_t(P.n_seg - 1) * P.units) / P.n_seg);
  return (last_y0 + 1) * P.W <= P.n_valid;
}

// Host mirror of wave_is_fast over every window (the lane with the largest
// column decides each window): whether all wavefronts of the stage are FAST.
static bool inv_all_fast(const StageParams &P, int L, int C1) {
  if (P.W % C1 != 0) return false;
  for (int win = 0; win < P.n_win; ++win) {
    const int cbase = win == 0 ? 0 : (win == P.n_win - 1 ? P.last_base : win * P.own_w - P.halo_l);
    const int64_t c0 = int64_t(cbase) + 63 * C1;
    if (c0 + C1 > P.W) return false;
    for (int l = 1; l <= L; ++l) {
      const int uu = (C1 >> (l - 1)) / 2;
      const int64_t wl = P.wdim[l], wh = P.wdim[l - 1] - P.wdim[l], bc = c0 >> l;
      if (wl % uu || wh % uu || P.off_hl[l] % uu || P.off_lh[l] % uu || P.off_hh[l] % uu ||
          wl - bc < uu || wh - bc < uu)
        return false;
    }
  }
  return true;
}

template <int L, int C1>
static hipError_t launch_inv_split(const int16_t *llin, const int16_t *pub, uint8_t *out,
                                   const StageParams &P, hipStream_t s) {
  const int blocks = (P.n_waves + kWavesPerBlock - 1) / kWavesPerBlock;
  const bool all_fast = inv_all_fast(P, L, C1);
  if constexpr (C1 == 8) {
    if (all_fast)
      hipLaunchKernelGGL((inv_split_pk8<L, true>), dim3(blocks), dim3(kBlockThreads), 0, s, llin, pub, out, P);
    else
      hipLaunchKernelGGL((inv_split_pk8<L, false>), dim3(blocks), dim3(kBlockThreads), 0, s, llin, pub, out, P);
  } else {
    if (all_fast)
      hipLaunchKernelGGL((inv_split_pk16<L, true>), dim3(blocks), dim3(kBlockThreads), 0, s, llin, pub, out, P);
    else
      hipLaunchKernelGGL((inv_split_pk16<L, false>), dim3(blocks), dim3(kBlockThreads), 0, s, llin, pub, out, P);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((inv_split_redo<L, C1>), dim3(blocks), dim3(kBlockThreads), 0, s, llin, pub, out, P);
  return hipGetLastError();
}

template <int L, int C1, bool U8OUT>
static const void *inv_fn() {
  if constexpr (C1 == 8) return reinterpret_cast<const void *>(&inv_kernel8<L, U8OUT>);
  else return reinterpret_cast<const void *>(&inv_kernel16<L, U8OUT>);
}

template <int L, int C1, bool U8OUT>
static hipError_t launch_inv_t(const int16_t *llin, const int16_t *pub, void *out,
                               const StageParams &P, hipStream_t s) {
  const int blocks = (P.n_waves + kWavesPerBlock - 1) / kWavesPerBlock;
  if constexpr (C1 == 8)
    hipLaunchKernelGGL((inv_kernel8<L, U8OUT>), dim3(blocks), dim3(kBlockThreads), 0, s, llin, pub,
                       out, P);
  else
    hipLaunchKernelGGL((inv_kernel16<L, U8OUT>), dim3(blocks), dim3(kBlockThreads), 0, s, llin,
                       pub, out, P);
  return hipGetLastError();
}

// Batch form: one persistent launch drains the batch's tile queue.  Items
// carry their own keys: each wavefront stages its tile's round keys and
// nonce in its own LDS slot; a tile runs the inverse of its item's depth.
// Sixteen columns per lane: two wavefronts per SIMD (256 VGPRs).
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(2)))
void inv_batch_kernel(const BatchItem *__restrict__ items, const int2 *__restrict__ tiles,
                      int64_t n_tiles, BatchCounters *__restrict__ ctr) {
  __shared__ uint32_t s_te[1024];
  __shared__ uint32_t s_kw[kWavesPerBlock][kKeyWords];
  __shared__ uint32_t s_ring[kWavesPerBlock][kRingBlocks * 4];
  load_aes_te(s_te);
  __syncthreads();
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  for (;;) {
    unsigned int t = 0;
    if (lane == 0) t = atomicAdd(&ctr->head, 1u);
    t = __builtin_amdgcn_readfirstlane(t);
    if (int64_t(t) >= n_tiles) break;
    const int2 e = tiles[t];
    const BatchItem &it = items[e.x];
    if (lane < kKeyWords) s_kw[wib][lane] = key_word(it.inv.key, lane);  // this item's keys
    wave_lds_sync();
    const int16_t *ll = reinterpret_cast<const int16_t *>(it.priv);
    switch (__builtin_amdgcn_readfirstlane(it.levels)) {
      case 1: inv_wave<1, kBatchCols, true>(it.inv, e.y, ll, it.pub, it.out, lane, s_ring[wib], s_te, s_kw[wib]); break;
      case 2: inv_wave<2, kBatchCols, true>(it.inv, e.y, ll, it.pub, it.out, lane, s_ring[wib], s_te, s_kw[wib]); break;
      case 3: inv_wave<3, kBatchCols, true>(it.inv, e.y, ll, it.pub, it.out, lane, s_ring[wib], s_te, s_kw[wib]); break;
      default: inv_wave<4, kBatchCols, true>(it.inv, e.y, ll, it.pub, it.out, lane, s_ring[wib], s_te, s_kw[wib]); break;
    }
    wave_lds_sync();
  }
  batch_finish(ctr);
}

hipError_t launch_inv_batch(const BatchItem *items, const int2 *tiles, int64_t n_tiles,
                            BatchCounters *ctr, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(inv_batch_kernel, dim3(blocks), dim3(kBlockThreads), 0, s, items, tiles,
                     n_tiles, ctr);
  return hipGetLastError();
}

// Resident workgroups per CU of the batch inverse kernel.
int inv_batch_blocks_per_cu() {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, reinterpret_cast<const void *>(&inv_batch_kernel),
                                                   kBlockThreads, 0) != hipSuccess)
    return 0;
  return blocks;
}

// Resident wavefronts per CU of the inverse kernel for (L, C1).
int inv_waves_per_cu(int L, int C1, bool u8out) {
  const void *fn = nullptr;
#define DWTFRAG_FN(LL, CC) \
  if (L == LL && C1 == CC) fn = u8out ? inv_fn<LL, CC, true>() : inv_fn<LL, CC, false>();
  DWTFRAG_FN(1, 8) DWTFRAG_FN(2, 8) DWTFRAG_FN(3, 8)
  DWTFRAG_FN(1, 16) DWTFRAG_FN(2, 16) DWTFRAG_FN(3, 16) DWTFRAG_FN(4, 16)
#undef DWTFRAG_FN
  int blocks = 0;
  if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, kBlockThreads, 0) != hipSuccess)
    return 0;
  return blocks * kWavesPerBlock;
}

// The split restore for the planner: whether a byte-output stage runs as
// the split pair, whether all its wavefronts are FAST (the packed kernel's
// variant), and that variant's resident wavefronts per compute unit.
bool inv_stage_split_ok(const StageParams &P) { return inv_split_ok(P); }
bool inv_stage_all_fast(const StageParams &P, int L, int C1) { return inv_all_fast(P, L, C1); }

template <int L, int C1, bool ALL_FAST>
static const void *inv_split_fn() {
  if constexpr (C1 == 8) return reinterpret_cast<const void *>(&inv_split_pk8<L, ALL_FAST>);
  else return reinterpret_cast<const void *>(&inv_split_pk16<L, ALL_FAST>);
}

int inv_split_waves_per_cu(int L, int C1, bool all_fast) {
  const void *fn = nullptr;
#define DWTFRAG_FN(LL, CC) \
  if (L == LL && C1 == CC) fn = all_fast ? inv_split_fn<LL, CC, true>() : inv_split_fn<LL, CC, false>();
  DWTFRAG_FN(1, 8) DWTFRAG_FN(2, 8) DWTFRAG_FN(3, 8)
  DWTFRAG_FN(1, 16) DWTFRAG_FN(2, 16) DWTFRAG_FN(3, 16) DWTFRAG_FN(4, 16)
#undef DWTFRAG_FN
  int blocks = 0;
  if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, kBlockThreads, 0) != hipSuccess)
    return 0;
  return blocks * kWavesPerBlock;
}

hipError_t launch_inv(int L, int C1, bool u8out, const int16_t *llin, const int16_t *pub,
                      void *out, const StageParams &P, hipStream_t s) {
  const bool split = u8out && inv_split_ok(P);
#define DWTFRAG_CASE(LL, CC)                                                   \
  if (L == LL && C1 == CC)                                                     \
    return split ? launch_inv_split<LL, CC>(llin, pub, static_cast<uint8_t *>(out), P, s) \
         : u8out ? launch_inv_t<LL, CC, true>(llin, pub, out, P, s)            \
                 : launch_inv_t<LL, CC, false>(llin, pub, out, P, s);
  DWTFRAG_CASE(1, 8) DWTFRAG_CASE(2, 8) DWTFRAG_CASE(3, 8)
  DWTFRAG_CASE(1, 16) DWTFRAG_CASE(2, 16) DWTFRAG_CASE(3, 16) DWTFRAG_CASE(4, 16)
#undef DWTFRAG_CASE
  return hipErrorInvalidValue;
}

}  // namespace dwtfrag
