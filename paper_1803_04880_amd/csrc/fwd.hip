// Forward path: fused multi-level 5/3 lifting with band scatter, as one
// streaming kernel.  The last LL band is written in clear to the private
// fragment's buffer and encrypted in place by the counter-mode kernel
// (ctr.hip) launched right after.
//
// Ch. 5 section 5.1.1: each level runs the horizontal pass (eqs. (5.1)-(5.2)
// along rows), then the vertical pass, and the next level transforms LL only.
//
// One wavefront owns a rectangle of the level-0 grid (a column window times a
// row segment).  It streams the rows of its window top to bottom, starting
// halo_t rows above its rectangle and stopping halo_b rows below.  Rows are
// fetched K at a time into an LDS staging buffer while the previous K rows
// are being transformed.  Each row is lifted horizontally across the 64 lanes
// (packed 16-bit arithmetic, see pack.h); the vertical lifting of level l is a
// per-column state machine in registers that consumes the level's rows as they
// are produced and emits one low row and one high row per row pair.  Low rows
// feed level l+1; everything inside the owned rectangle is stored.
#include "lift.h"
#include "pack.h"

namespace dwtfrag {

template <int L, int C1, bool U8IN>
struct FwdWave {
  template <int l> static constexpr int M = (C1 >> (l - 1)) / 2;  // evens per lane at level l
  template <int l> static constexpr int NP = Pk<M<l>>::P;         // packed regs per parity
  static constexpr int RB = U8IN ? C1 : 2 * C1;                   // input bytes per lane and row
  static constexpr int RW = RB / 4;                               // ... in dwords
  static constexpr int K = (4096 / (64 * RB)) >= 2 ? 4096 / (64 * RB) : 2;  // rows per batch

  const StageParams &G;
  const uint8_t *in8;
  const int16_t *in16;
  int16_t *pub;
  int16_t *llout;
  uint32_t *stage;        // this wavefront's LDS staging rows: K * 64 * RW dwords
  int lane;
  int c0;                 // level-0 column of this lane's first sample
  int X0, Y0, X1, Y1;     // owned rectangle (level 0), X1 / Y1 exclusive
  bool last_win, last_seg;

  uint32_t Ev1[2 * NP<1>], Ov1[2 * NP<1>], Dv1[2 * NP<1>];
  uint32_t Ev2[2 * NP<2>], Ov2[2 * NP<2>], Dv2[2 * NP<2>];
  uint32_t Ev3[L >= 3 ? 2 * NP<3> : 1], Ov3[L >= 3 ? 2 * NP<3> : 1], Dv3[L >= 3 ? 2 * NP<3> : 1];
  uint32_t Ev4[L >= 4 ? 2 * NP<4> : 1], Ov4[L >= 4 ? 2 * NP<4> : 1], Dv4[L >= 4 ? 2 * NP<4> : 1];
  int i0[kMaxFused + 1];  // first row of each level's stream
  bool hedge[kMaxFused + 1];
  bool lown[kMaxFused + 1];

  template <int l> __device__ __forceinline__ auto &E() {
    if constexpr (l == 1) return Ev1; else if constexpr (l == 2) return Ev2;
    else if constexpr (l == 3) return Ev3; else return Ev4;
  }
  template <int l> __device__ __forceinline__ auto &O() {
    if constexpr (l == 1) return Ov1; else if constexpr (l == 2) return Ov2;
    else if constexpr (l == 3) return Ov3; else return Ov4;
  }
  template <int l> __device__ __forceinline__ auto &D() {
    if constexpr (l == 1) return Dv1; else if constexpr (l == 2) return Dv2;
    else if constexpr (l == 3) return Dv3; else return Dv4;
  }

  template <int l> __device__ __forceinline__ bool row_owned(int k) const {
    return k >= (Y0 >> l) && (last_seg || k < (Y1 >> l));
  }

  // Store Mv int16 values (packed pairs) at band columns bc.. of a band row.
  template <int Mv>
  __device__ __forceinline__ void store_band(int16_t *row, int bc, int nvalid, const uint32_t *R) {
    if (nvalid <= 0) return;
    int16_t *dst = reinterpret_cast<int16_t *>(reinterpret_cast<char *>(row) + 2u * uint32_t(bc));
    const bool aligned = (reinterpret_cast<uintptr_t>(row) & (2 * Mv - 1)) == 0;
    if (nvalid >= Mv && aligned) {
      if constexpr (Mv == 1) *dst = int16_t(R[0]);
      else if constexpr (Mv == 2) *reinterpret_cast<uint32_t *>(dst) = R[0];
      else if constexpr (Mv == 4) *reinterpret_cast<uint2 *>(dst) = make_uint2(R[0], R[1]);
      else *reinterpret_cast<uint4 *>(dst) = make_uint4(R[0], R[1], R[2], R[3]);
      return;
    }
#pragma unroll
    for (int u = 0; u < Mv; ++u)
      if (u < nvalid) dst[u] = int16_t(Mv == 1 ? R[0] : (R[u >> 1] >> (16 * (u & 1))));
  }

  // Low row k of level l: lows -> LL_l (next level / private fragment), highs -> HL_l.
  template <int l> __device__ __forceinline__ void emit_low(const uint32_t (&s)[2 * NP<l>], int k) {
    constexpr int Np = NP<l>;
    const int N = G.wdim[l - 1];
    const int wl = G.wdim[l];
    const int bc = c0 >> l;
    const bool rown = row_owned<l>(k);
    if (rown && lown[l])
      store_band<M<l>>(pub + G.off_hl[l] + int64_t(k) * (N - wl), bc, (N - wl) - bc, s + Np);
    if constexpr (l < L) {
      constexpr int Mn = M<l + 1>;
      constexpr int Nn = NP<l + 1>;
      uint32_t E2[Nn], O2[Nn];
      if constexpr (Mn >= 2) {
#pragma unroll
        for (int j = 0; j < Nn; ++j) {
          E2[j] = lo_halves(s[2 * j], s[2 * j + 1]);
          O2[j] = hi_halves(s[2 * j], s[2 * j + 1]);
        }
      } else {
        E2[0] = s[0];
        O2[0] = s[0] >> 16;
      }
      push_row<l + 1>(E2, O2, k);
    } else {
      if (rown && lown[l]) store_band<M<l>>(llout + int64_t(k) * wl, bc, wl - bc, s);
    }
  }

  // High row k of level l: lows -> LH_l, highs -> HH_l.
  template <int l> __device__ __forceinline__ void emit_high(const uint32_t (&d)[2 * NP<l>], int k) {
    if (!(row_owned<l>(k) && lown[l])) return;
    constexpr int Np = NP<l>;
    const int N = G.wdim[l - 1];
    const int wl = G.wdim[l];
    const int bc = c0 >> l;
    store_band<M<l>>(pub + G.off_lh[l] + int64_t(k) * wl, bc, wl - bc, d);
    store_band<M<l>>(pub + G.off_hh[l] + int64_t(k) * (N - wl), bc, (N - wl) - bc, d + Np);
  }

  // Row i of the level-(l-1) LL arrives at level l in even/odd packed form.
  // While streaming, a row yields at most one low and one high row: the even
  // rows complete the pair (i-2, i-1), the last row of an even-length signal
  // completes the final pair.  The extra low row of an odd-length signal is
  // produced by flush_tail once the stream has ended.
  template <int l>
  __device__ __forceinline__ void push_row(uint32_t (&Ein)[NP<l>], uint32_t (&Oin)[NP<l>], int i) {
    constexpr int Np = NP<l>;
    constexpr int R = 2 * Np;
    hfwd_pk_any<M<l>>(Ein, Oin, c0 >> (l - 1), G.wdim[l - 1], hedge[l]);
    uint32_t x[R];
#pragma unroll
    for (int j = 0; j < Np; ++j) { x[j] = Ein[j]; x[Np + j] = Oin[j]; }
    const int N = G.hdim[l - 1];
    if (N == 1) {  // no vertical pass: the row is the low row
      emit_low<l>(x, 0);
      return;
    }
    auto &Ev = E<l>();
    auto &Ov = O<l>();
    auto &Dv = D<l>();
    const bool even = (i & 1) == 0;
    if (even && i == i0[l]) {
#pragma unroll
      for (int t = 0; t < R; ++t) Ev[t] = x[t];
      return;
    }
    if (!even && i != N - 1) {
#pragma unroll
      for (int t = 0; t < R; ++t) Ov[t] = x[t];
      return;
    }
    // even i: rows i-2 (Ev), i-1 (Ov), i (x) give d(i-1), s(i-2);
    // odd i = N-1: rows i-1 (Ev), i (x) with x(N) = x(N-2) give d(i), s(i-1)
    const int k = even ? (i - 2) >> 1 : (i - 1) >> 1;
    const bool top = (k == 0);
    uint32_t low[R], high[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const uint32_t dn = even ? pk_predict(Ov[t], Ev[t], x[t]) : pk_sub(x[t], Ev[t]);
      low[t] = pk_update(Ev[t], top ? dn : Dv[t], dn);
      high[t] = dn;
      Dv[t] = dn;
      if (even) Ev[t] = x[t];
    }
    emit_high<l>(high, k);
    emit_low<l>(low, k);
  }

  // End of the stream at the bottom edge: odd-length levels still owe their
  // last low row s(N-1) = x(N-1) + floor((d(N-2) + d(N) + 2) / 4), d(N) = d(N-2).
  // Levels are flushed in order, so a flushed row reaches the coarser levels
  // before they flush themselves.
  template <int l> __device__ __forceinline__ void flush_tail() {
    const int N = G.hdim[l - 1];
    if (N > 1 && (N & 1)) {
      constexpr int R = 2 * NP<l>;
      auto &Ev = E<l>();
      auto &Dv = D<l>();
      uint32_t low[R];
#pragma unroll
      for (int t = 0; t < R; ++t) low[t] = pk_update(Ev[t], Dv[t], Dv[t]);
      emit_low<l>(low, (N - 1) >> 1);
    }
    if constexpr (l < L) flush_tail<l + 1>();
  }

  // ---- input rows --------------------------------------------------------
  // Every lane's C1 columns of row r lie inside the input buffer and are
  // aligned for one vector load (lanes past the right edge read bytes of the
  // next row, which no valid sample uses).  Uniform across the wavefront.
  __device__ __forceinline__ bool row_fast(int r, int cbase) const {
    const int64_t end = int64_t(r) * G.W + cbase + 64 * C1;
    return (G.W % C1 == 0) && end <= G.n_valid;
  }

  // Vector load of row r (row_fast(r) holds).
  __device__ __forceinline__ void load_row_fast(int r, uint32_t (&w)[RW]) const {
    const uint32_t off = uint32_t(c0) * (U8IN ? 1u : 2u);
    const char *src = reinterpret_cast<const char *>(U8IN ? static_cast<const void *>(in8)
                                                          : static_cast<const void *>(in16)) +
                      int64_t(r) * G.W * (U8IN ? 1 : 2);
#pragma unroll
    for (int q = 0; q < RW; q += (RW >= 4 ? 4 : 2)) {
      if constexpr (RW >= 4) {
        const uint4 v = *reinterpret_cast<const uint4 *>(src + off + 4u * q);
        w[q] = v.x; w[q + 1] = v.y; w[q + 2] = v.z; w[q + 3] = v.w;
      } else {
        const uint2 v = *reinterpret_cast<const uint2 *>(src + off + 4u * q);
        w[q] = v.x; w[q + 1] = v.y;
      }
    }
  }

  // Element-wise load of row r with zeros outside the view.
  __device__ __forceinline__ void load_row_slow(int r, uint32_t (&w)[RW]) const {
    const int64_t rowbase = int64_t(r) * G.W;
#pragma unroll
    for (int q = 0; q < RW; ++q) w[q] = 0;
    for (int t = 0; t < C1; ++t) {
      const int c = c0 + t;
      if (c < G.W && rowbase + c < G.n_valid) {
        if constexpr (U8IN) w[t >> 2] |= uint32_t(in8[rowbase + c]) << (8 * (t & 3));
        else w[t >> 1] |= uint32_t(uint16_t(in16[rowbase + c])) << (16 * (t & 1));
      }
    }
  }

  // Staged row -> even / odd packed registers of level 1.
  __device__ __forceinline__ void unpack(const uint32_t (&w)[RW], uint32_t (&Ein)[NP<1>],
                                         uint32_t (&Oin)[NP<1>]) const {
    if constexpr (U8IN) {
#pragma unroll
      for (int j = 0; j < NP<1>; ++j) {
        Ein[j] = __builtin_amdgcn_perm(0u, w[j], 0x0C020C00u);  // (b0, b2)
        Oin[j] = __builtin_amdgcn_perm(0u, w[j], 0x0C030C01u);  // (b1, b3)
      }
    } else {
#pragma unroll
      for (int j = 0; j < NP<1>; ++j) {
        Ein[j] = lo_halves(w[2 * j], w[2 * j + 1]);
        Oin[j] = hi_halves(w[2 * j], w[2 * j + 1]);
      }
    }
  }

  __device__ __forceinline__ void stage_write(int k, const uint32_t (&w)[RW]) {
    uint32_t *dst = stage + (k * 64 + lane) * RW;
    if constexpr (RW == 2) {
      *reinterpret_cast<uint2 *>(dst) = make_uint2(w[0], w[1]);
    } else {
#pragma unroll
      for (int q = 0; q < RW / 4; ++q)
        reinterpret_cast<uint4 *>(dst)[q] = make_uint4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
    }
  }
  __device__ __forceinline__ void stage_read(int k, uint32_t (&w)[RW]) const {
    const uint32_t *src = stage + (k * 64 + lane) * RW;
    if constexpr (RW == 2) {
      const uint2 v = *reinterpret_cast<const uint2 *>(src);
      w[0] = v.x; w[1] = v.y;
    } else {
#pragma unroll
      for (int q = 0; q < RW / 4; ++q) {
        const uint4 v = reinterpret_cast<const uint4 *>(src)[q];
        w[4 * q] = v.x; w[4 * q + 1] = v.y; w[4 * q + 2] = v.z; w[4 * q + 3] = v.w;
      }
    }
  }

  __device__ __forceinline__ void run(int wave) {
    const int win = wave % G.n_win;
    const int seg = wave / G.n_win;
    X0 = win * G.own_w;
    Y0 = seg * G.own_h;
    last_win = (win == G.n_win - 1);
    last_seg = (seg == G.n_seg - 1);
    X1 = last_win ? G.W : X0 + G.own_w;
    Y1 = last_seg ? G.H : Y0 + G.own_h;
    const int cbase = (win == 0) ? 0 : X0 - G.halo_l;
    c0 = cbase + lane * C1;
    const int r0 = Y0 > G.halo_t ? Y0 - G.halo_t : 0;
    const int r1 = min(G.H, Y1 + G.halo_b);
#pragma unroll
    for (int l = 1; l <= L; ++l) {
      i0[l] = r0 >> (l - 1);
      const int N = G.wdim[l - 1];
      const int j0 = cbase >> (l - 1);
      const int span = (64 * C1) >> (l - 1);
      hedge[l] = (j0 == 0) || (N - 1 >= j0 && N - 1 < j0 + span);
      const int bc = c0 >> l;
      lown[l] = bc >= (X0 >> l) && (last_win || bc < (X1 >> l));
    }
#pragma unroll
    for (int t = 0; t < 2 * NP<1>; ++t) { Ev1[t] = 0; Ov1[t] = 0; Dv1[t] = 0; }
#pragma unroll
    for (int t = 0; t < 2 * NP<2>; ++t) { Ev2[t] = 0; Ov2[t] = 0; Dv2[t] = 0; }
#pragma unroll
    for (int t = 0; t < (L >= 3 ? 2 * NP<3> : 1); ++t) { Ev3[t] = 0; Ov3[t] = 0; Dv3[t] = 0; }
#pragma unroll
    for (int t = 0; t < (L >= 4 ? 2 * NP<4> : 1); ++t) { Ev4[t] = 0; Ov4[t] = 0; Dv4[t] = 0; }
    if (r0 >= r1) return;

    // Batches of K rows: while batch b is transformed from the LDS staging
    // buffer, the vector loads of batch b+1 are in flight in registers.  Rows
    // that cannot be loaded as one vector per lane are read element-wise
    // when they are transformed.
    uint32_t q[K][RW];
    const int cbase_ = cbase;
    bool fast_cur = row_fast(min(r1, r0 + K) - 1, cbase_);
    if (fast_cur) {
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (r0 + k < r1) load_row_fast(r0 + k, q[k]);
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (r0 + k < r1) stage_write(k, q[k]);
      wave_lds_sync();
    }
    for (int rb = r0; rb < r1; rb += K) {
      const int nb = min(K, r1 - rb);
      const int rn = rb + K;
      const bool fast_next = rn < r1 && row_fast(min(r1, rn + K) - 1, cbase_);
      if (fast_next) {
#pragma unroll
        for (int k = 0; k < K; ++k)
          if (rn + k < r1) load_row_fast(rn + k, q[k]);  // next batch in flight
      }
#pragma unroll 1
      for (int k = 0; k < nb; ++k) {
        uint32_t w[RW], Ein[NP<1>], Oin[NP<1>];
        if (fast_cur) stage_read(k, w);
        else load_row_slow(rb + k, w);
        unpack(w, Ein, Oin);
        push_row<1>(Ein, Oin, rb + k);
      }
      if (fast_next) {
        wave_lds_sync();
#pragma unroll
        for (int k = 0; k < K; ++k)
          if (rn + k < r1) stage_write(k, q[k]);
        wave_lds_sync();
      }
      fast_cur = fast_next;
    }
    if (r1 == G.H) flush_tail<1>();
  }
};

template <int L, int C1, bool U8IN>
__global__ __launch_bounds__(kBlockThreads) void fwd_kernel(const void *__restrict__ in,
                                                            int16_t *__restrict__ pub,
                                                            int16_t *__restrict__ llout,
                                                            const StageParams P) {
  using W = FwdWave<L, C1, U8IN>;
  __shared__ uint32_t s_stage[kWavesPerBlock][W::K * 64 * W::RW];
  const int wib = threadIdx.x >> 6;
  const int wave = blockIdx.x * kWavesPerBlock + wib;
  if (wave >= P.n_waves) return;
  W w{P};
  w.in8 = static_cast<const uint8_t *>(in);
  w.in16 = static_cast<const int16_t *>(in);
  w.pub = pub;
  w.llout = llout;
  w.stage = s_stage[wib];
  w.lane = threadIdx.x & 63;
  w.run(wave);
}

template <int L, int C1, bool U8IN>
static hipError_t launch_fwd_t(const void *in, int16_t *pub, int16_t *llout, const StageParams &P,
                               hipStream_t s) {
  const int blocks = (P.n_waves + kWavesPerBlock - 1) / kWavesPerBlock;
  hipLaunchKernelGGL((fwd_kernel<L, C1, U8IN>), dim3(blocks), dim3(kBlockThreads), 0, s, in, pub,
                     llout, P);
  return hipGetLastError();
}

hipError_t launch_fwd(int L, int C1, bool u8in, const void *in, int16_t *pub, int16_t *llout,
                      const StageParams &P, hipStream_t s) {
#define DWTFRAG_CASE(LL, CC)                                                           \
  if (L == LL && C1 == CC)                                                             \
    return u8in ? launch_fwd_t<LL, CC, true>(in, pub, llout, P, s)                     \
                : launch_fwd_t<LL, CC, false>(in, pub, llout, P, s);
  DWTFRAG_CASE(1, 8) DWTFRAG_CASE(2, 8) DWTFRAG_CASE(3, 8)
  DWTFRAG_CASE(1, 16) DWTFRAG_CASE(2, 16) DWTFRAG_CASE(3, 16) DWTFRAG_CASE(4, 16)
#undef DWTFRAG_CASE
  return hipErrorInvalidValue;
}

}  // namespace dwtfrag
