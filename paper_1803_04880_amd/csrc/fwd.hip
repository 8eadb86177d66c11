// Forward path: fused multi-level 5/3 lifting with band scatter and the
// AES-CTR encryption of the last LL band, as one streaming kernel.
//
// Ch. 5 section 5.1.1: each level runs the horizontal pass (eqs. (5.1)-(5.2)
// along rows), then the vertical pass, and the next level transforms LL only.
//
// One wavefront owns a rectangle of the level-0 grid (a column window times a
// row segment).  It streams the rows of its window top to bottom, starting
// halo_t rows above its rectangle and stopping halo_b rows below.  Each row is
// lifted horizontally across the 64 lanes; the vertical lifting of level l
// is a small state machine per lane column that consumes the level's rows as
// they are produced and emits one low row and one high row per row pair.
// Low rows feed level l+1; everything inside the owned rectangle is stored.
#include "lift.h"

namespace dwtfrag {

template <int L, int C1, bool U8IN>
struct FwdWave {
  template <int l> static constexpr int C = C1 >> (l - 1);

  const StageParams &P;
  const uint8_t *in8;
  const int16_t *in16;
  int16_t *pub;
  int16_t *llout;
  KsRing ks;
  int lane;
  int c0;                 // level-0 column of this lane's first sample
  int X0, Y0;             // owned rectangle origin (level 0)
  bool last_win, last_seg;
  int X1, Y1;             // owned rectangle end (exclusive, level 0)

  // per-level state (index by level 1..4; unused levels are size 1)
  int E1[C<1>], O1[C<1>], D1[C<1>];
  int E2[C1 >= 2 ? C<2> : 1], O2[C1 >= 2 ? C<2> : 1], D2[C1 >= 2 ? C<2> : 1];
  int E3[C1 >= 4 ? C<3> : 1], O3[C1 >= 4 ? C<3> : 1], D3[C1 >= 4 ? C<3> : 1];
  int E4[C1 >= 8 ? C<4> : 1], O4[C1 >= 8 ? C<4> : 1], D4[C1 >= 8 ? C<4> : 1];
  int i0[kMaxFused + 1];  // first row of each level's stream
  bool hedge[kMaxFused + 1];

  template <int l> __device__ auto &E() {
    if constexpr (l == 1) return E1; else if constexpr (l == 2) return E2;
    else if constexpr (l == 3) return E3; else return E4;
  }
  template <int l> __device__ auto &O() {
    if constexpr (l == 1) return O1; else if constexpr (l == 2) return O2;
    else if constexpr (l == 3) return O3; else return O4;
  }
  template <int l> __device__ auto &D() {
    if constexpr (l == 1) return D1; else if constexpr (l == 2) return D2;
    else if constexpr (l == 3) return D3; else return D4;
  }

  // ownership of band row k / this lane's band columns at level l
  template <int l> __device__ bool row_owned(int k) const {
    return k >= (Y0 >> l) && (last_seg || k < (Y1 >> l));
  }
  template <int l> __device__ bool lane_owned() const {
    const int bc = c0 >> l;
    return bc >= (X0 >> l) && (last_win || bc < (X1 >> l));
  }

  // Low row k of level l: even positions -> LL_l, odd positions -> HL_l.
  template <int l> __device__ __forceinline__ void emit_low(const int (&s)[C<l>], int k) {
    constexpr int U = C<l> / 2;
    const int N = P.wdim[l - 1];
    const int wl = P.wdim[l];
    const int bc = c0 >> l;  // first band column of this lane
    int hi[U], lo[U];
#pragma unroll
    for (int u = 0; u < U; ++u) { lo[u] = s[2 * u]; hi[u] = s[2 * u + 1]; }
    const bool rown = row_owned<l>(k);
    const bool lown = lane_owned<l>();
    if (rown && lown)
      store_i16<U>(pub + P.off_hl[l], int64_t(k) * (N - wl) + bc, (N - wl) - bc, hi);
    if constexpr (l < L) {
      push_row<l + 1>(lo, k);
    } else {
      if (rown) {
        if (P.use_aes) ks.ensure(k, last_seg ? P.hdim[l] : (Y1 >> l), P.key, lane);
        if (lown) {
          const int nv = wl - bc;
          if (P.use_aes) {
#pragma unroll
            for (int u = 0; u < U; ++u)
              if (u < nv) lo[u] ^= int(ks.ks16(k, bc + u));
          }
          store_i16<U>(llout, int64_t(k) * wl + bc, nv, lo);
        }
      }
    }
  }

  // High row k of level l: even positions -> LH_l, odd positions -> HH_l.
  template <int l> __device__ __forceinline__ void emit_high(const int (&d)[C<l>], int k) {
    constexpr int U = C<l> / 2;
    if (!(row_owned<l>(k) && lane_owned<l>())) return;
    const int N = P.wdim[l - 1];
    const int wl = P.wdim[l];
    const int bc = c0 >> l;
    int lo[U], hi[U];
#pragma unroll
    for (int u = 0; u < U; ++u) { lo[u] = d[2 * u]; hi[u] = d[2 * u + 1]; }
    store_i16<U>(pub + P.off_lh[l], int64_t(k) * wl + bc, wl - bc, lo);
    store_i16<U>(pub + P.off_hh[l], int64_t(k) * (N - wl) + bc, (N - wl) - bc, hi);
  }

  // Row i of the level-(l-1) LL arrives at level l (not yet lifted).  The
  // row yields at most one high row and two low rows; they are emitted from
  // one call site each so that the levels below are instantiated once.
  template <int l> __device__ __forceinline__ void push_row(int (&x)[C<l>], int i) {
    constexpr int CC = C<l>;
    hfwd_any<CC>(x, c0 >> (l - 1), P.wdim[l - 1], hedge[l]);
    const int N = P.hdim[l - 1];
    auto &Ev = E<l>();
    auto &Ov = O<l>();
    auto &Dv = D<l>();
    int lowA[CC], lowB[CC], high[CC];
    int nlow = 0, k_lowA = 0, k_lowB = 0, k_high = -1;
    if (N == 1) {  // no vertical pass: the row is the low row
#pragma unroll
      for (int t = 0; t < CC; ++t) lowA[t] = x[t];
      nlow = 1;
    } else if ((i & 1) == 0) {
      if (i != i0[l]) {
        // rows i-2 (even, Ev), i-1 (odd, Ov), i (even, x): d(i-1), s(i-2)
        const bool top = (i == 2);
#pragma unroll
        for (int t = 0; t < CC; ++t) {
          const int dn = Ov[t] - ((Ev[t] + x[t]) >> 1);
          const int dp = top ? dn : Dv[t];
          lowA[t] = Ev[t] + ((dp + dn + 2) >> 2);
          high[t] = dn;
          Dv[t] = dn;
        }
        nlow = 1;
        k_lowA = k_high = (i - 2) >> 1;
      }
#pragma unroll
      for (int t = 0; t < CC; ++t) Ev[t] = x[t];
      if (i == N - 1) {  // odd length, last (even) row: d(N) = d(N-2)
#pragma unroll
        for (int t = 0; t < CC; ++t) lowB[t] = Ev[t] + ((Dv[t] + Dv[t] + 2) >> 2);
        k_lowB = i >> 1;
        nlow += 1;
      }
    } else {
#pragma unroll
      for (int t = 0; t < CC; ++t) Ov[t] = x[t];
      if (i == N - 1) {  // even length, last (odd) row: x(N) = x(N-2)
        const bool top = (i == 1);
#pragma unroll
        for (int t = 0; t < CC; ++t) {
          const int dn = Ov[t] - Ev[t];
          const int dp = top ? dn : Dv[t];
          lowA[t] = Ev[t] + ((dp + dn + 2) >> 2);
          high[t] = dn;
        }
        nlow = 1;
        k_lowA = k_high = (i - 1) >> 1;
      }
    }
    if (k_high >= 0) emit_high<l>(high, k_high);
    // with a single low row from the flush alone it sits in lowB
    const int e0 = (nlow == 1 && k_lowB > 0 && k_high < 0 && N != 1) ? 1 : 0;
#pragma unroll 1
    for (int e = e0; e < e0 + nlow; ++e) {
      int row[CC];
#pragma unroll
      for (int t = 0; t < CC; ++t) row[t] = e ? lowB[t] : lowA[t];
      emit_low<l>(row, e ? k_lowB : k_lowA);
    }
  }

  // ---- input rows --------------------------------------------------------
  using Raw = typename std::conditional<U8IN, typename std::conditional<C1 == 16, uint4, uint2>::type,
                                        typename std::conditional<C1 == 16, uint4, uint4>::type>::type;
  struct RawRow { Raw a, b; };

  __device__ __forceinline__ RawRow load_row(int r) const {
    RawRow q{};
    const int64_t rowbase = int64_t(r) * P.W;
    if constexpr (U8IN) {
      const int64_t idx = rowbase + c0;
      if (c0 + C1 <= P.W && idx + C1 <= P.n_valid && (idx & (C1 - 1)) == 0) {
        q.a = *reinterpret_cast<const Raw *>(in8 + idx);
      } else {
        uint8_t tmp[16] = {0};
#pragma unroll
        for (int t = 0; t < C1; ++t) {
          const int c = c0 + t;
          if (c < P.W && rowbase + c < P.n_valid) tmp[t] = in8[rowbase + c];
        }
        uint32_t w[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
          w[i] = uint32_t(tmp[4 * i]) | (uint32_t(tmp[4 * i + 1]) << 8) |
                 (uint32_t(tmp[4 * i + 2]) << 16) | (uint32_t(tmp[4 * i + 3]) << 24);
        if constexpr (C1 == 16) q.a = make_uint4(w[0], w[1], w[2], w[3]);
        else q.a = make_uint2(w[0], w[1]);
      }
    } else {
      const int64_t idx = rowbase + c0;
      const int nv = P.W - c0;
      if (nv >= C1 && (idx & 7) == 0) {
        q.a = *reinterpret_cast<const uint4 *>(in16 + idx);
        if constexpr (C1 == 16) q.b = *reinterpret_cast<const uint4 *>(in16 + idx + 8);
      } else {
        uint32_t w[8] = {0};
#pragma unroll
        for (int t = 0; t < C1; ++t) {
          uint32_t v = (t < nv) ? uint32_t(uint16_t(in16[idx + t])) : 0u;
          w[t >> 1] |= v << (16 * (t & 1));
        }
        q.a = make_uint4(w[0], w[1], w[2], w[3]);
        if constexpr (C1 == 16) q.b = make_uint4(w[4], w[5], w[6], w[7]);
      }
    }
    return q;
  }

  __device__ __forceinline__ void unpack(const RawRow &q, int (&x)[C1]) const {
    if constexpr (U8IN) {
      uint32_t w[4] = {0, 0, 0, 0};
      if constexpr (C1 == 16) { w[0] = q.a.x; w[1] = q.a.y; w[2] = q.a.z; w[3] = q.a.w; }
      else { w[0] = q.a.x; w[1] = q.a.y; }
#pragma unroll
      for (int t = 0; t < C1; ++t) x[t] = int((w[t >> 2] >> (8 * (t & 3))) & 0xFFu);
    } else {
      uint32_t w[8] = {q.a.x, q.a.y, q.a.z, q.a.w, 0, 0, 0, 0};
      if constexpr (C1 == 16) { w[4] = q.b.x; w[5] = q.b.y; w[6] = q.b.z; w[7] = q.b.w; }
#pragma unroll
      for (int t = 0; t < C1; ++t) x[t] = int(int32_t(w[t >> 1] << (16 * (1 - (t & 1)))) >> 16);
    }
  }

  __device__ __forceinline__ void run(int wave) {
    const int win = wave % P.n_win;
    const int seg = wave / P.n_win;
    X0 = win * P.own_w;
    Y0 = seg * P.own_h;
    last_win = (win == P.n_win - 1);
    last_seg = (seg == P.n_seg - 1);
    X1 = last_win ? P.W : X0 + P.own_w;
    Y1 = last_seg ? P.H : Y0 + P.own_h;
    const int cbase = (win == 0) ? 0 : X0 - P.halo_l;
    c0 = cbase + lane * C1;
    const int r0 = Y0 > P.halo_t ? Y0 - P.halo_t : 0;
    const int r1 = min(P.H, Y1 + P.halo_b);
#pragma unroll
    for (int l = 1; l <= L; ++l) {
      i0[l] = r0 >> (l - 1);
      const int N = P.wdim[l - 1];
      const int j0 = cbase >> (l - 1);
      const int span = (64 * C1) >> (l - 1);
      hedge[l] = (j0 == 0) || (N - 1 >= j0 && N - 1 < j0 + span);
    }
#pragma unroll
    for (int t = 0; t < C<1>; ++t) { E1[t] = 0; O1[t] = 0; D1[t] = 0; }
    for (int t = 0; t < (C1 >= 2 ? C<2> : 1); ++t) { E2[t] = 0; O2[t] = 0; D2[t] = 0; }
    for (int t = 0; t < (C1 >= 4 ? C<3> : 1); ++t) { E3[t] = 0; O3[t] = 0; D3[t] = 0; }
    for (int t = 0; t < (C1 >= 8 ? C<4> : 1); ++t) { E4[t] = 0; O4[t] = 0; D4[t] = 0; }
    // keystream columns: the LL columns this wavefront stores
    ks.col_lo = X0 >> L;
    ks.col_hi = min(P.wdim[L], last_win ? P.wdim[L] : (X1 >> L));
    ks.wL = P.wdim[L];
    ks.base = -1;

    if (r0 >= r1) return;
    RawRow cur = load_row(r0);
    RawRow nxt = (r0 + 1 < r1) ? load_row(r0 + 1) : cur;
    for (int r = r0; r < r1; ++r) {
      RawRow q = cur;
      cur = nxt;
      if (r + 2 < r1) nxt = load_row(r + 2);
      int x[C1];
      unpack(q, x);
      push_row<1>(x, r);
    }
  }
};

template <int L, int C1, bool U8IN>
__global__ __launch_bounds__(kBlockThreads) void fwd_kernel(const void *__restrict__ in,
                                                            int16_t *__restrict__ pub,
                                                            int16_t *__restrict__ llout,
                                                            const StageParams P) {
  __shared__ uint32_t s_te[1024];
  __shared__ uint32_t s_ring[kWavesPerBlock][kRingBlocks * 4];
  if (P.use_aes) load_aes_tables(s_te);
  __syncthreads();
  const int wib = threadIdx.x >> 6;
  const int wave = blockIdx.x * kWavesPerBlock + wib;
  if (wave >= P.n_waves) return;
  FwdWave<L, C1, U8IN> w{P};
  w.in8 = static_cast<const uint8_t *>(in);
  w.in16 = static_cast<const int16_t *>(in);
  w.pub = pub;
  w.llout = llout;
  w.lane = threadIdx.x & 63;
  w.ks.ring = s_ring[wib];
  w.ks.te = s_te;
  w.ks.rows = P.ks_rows;
  w.ks.blocks = P.ks_blocks;
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
