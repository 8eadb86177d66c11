// Forward path: fused multi-level 5/3 lifting with band scatter and the
// counter-mode encryption of the last LL band, as one streaming kernel.  A
// wavefront writes its owned LL rectangle in clear while it streams, then
// encrypts it in place once its stream has ended (so the AES rounds do not
// share registers with the stream).
//
// Ch. 5 section 5.1.1: each level runs the horizontal pass (eqs. (5.1)-(5.2)
// along rows), then the vertical pass, and the next level transforms LL only.
//
// One wavefront owns a rectangle of the level-0 grid (a column window times a
// row segment) and streams the rows of its window top to bottom, starting
// halo_t rows above its rectangle and stopping halo_b rows below.  Work goes
// in batches of K level-0 rows: the batch sits in an LDS staging buffer (the
// next batch's vector loads are in flight meanwhile) and is pushed through the
// levels one after the other.  Level l takes its rows from an LDS queue,
// lifts each row horizontally across the 64 lanes (packed 16-bit arithmetic,
// see pack.h) and runs the vertical lifting as a per-column state machine in
// registers: an odd row waits, the following even row completes the pair
// (2k+1, 2k+2), which yields low row k and high row k.  Low rows go to level
// l+1's queue (or, at the last level, to the LL output), detail rows inside the
// owned rectangle are stored.  Rows a level cannot pair yet stay in registers
// until the next batch.
#include "batch.h"
#include "lift.h"
#include "pack.h"

namespace dwtfrag {

template <int L, int C1, bool U8IN>
struct FwdWave {
  template <int l> static constexpr int M = (C1 >> (l - 1)) / 2;  // evens per lane at level l
  template <int l> static constexpr int NP = Pk<M<l>>::P;         // packed regs per parity
  template <int l> static constexpr int R = 2 * NP<l>;            // packed regs per row
  static constexpr int RB = U8IN ? C1 : 2 * C1;                   // input bytes per lane and row
  static constexpr int RW = RB / 4;                               // ... in dwords
  static constexpr int K = 8;                                     // level-0 rows per batch
  // queue capacity (rows) of level l >= 2: rows level l-1 can emit in one batch
  template <int l> static constexpr int QC = (K >> (l - 1)) + 2;
  static constexpr int kStageWords = K * 64 * RW;
  static constexpr int kQueueWords = 64 * (QC<2> * R<2> + (L >= 3 ? QC<3> * R<3> : 0) +
                                           (L >= 4 ? QC<4> * R<4> : 0));
  static constexpr int kLdsWords = kStageWords + kQueueWords;

  const StageParams &G;
  const uint8_t *in8;
  const int16_t *in16;
  int16_t *pub;
  int16_t *llout;
  uint32_t *lds;          // this wavefront's staging rows, then the level queues
  const uint32_t *te;     // AES tables in LDS (use_aes)
  const uint32_t *kw;     // round keys + nonce in LDS
  int lane;
  int c0;                 // level-0 column of this lane's first sample
  int X0, Y0, X1, Y1;     // owned rectangle (level 0), X1 / Y1 exclusive
  bool last_win, last_seg;
  int r0;                 // first level-0 row streamed (level l starts at r0 >> (l-1))

  // per-level registers: previous even row, previous high row, waiting odd row
  uint32_t E1[R<1>], D1[R<1>], P1[R<1>];
  uint32_t E2[R<2>], D2[R<2>], P2[R<2>];
  uint32_t E3[L >= 3 ? R<3> : 1], D3[L >= 3 ? R<3> : 1], P3[L >= 3 ? R<3> : 1];
  uint32_t E4[L >= 4 ? R<4> : 1], D4[L >= 4 ? R<4> : 1], P4[L >= 4 ? R<4> : 1];
  int icnt[kMaxFused + 1];  // next row index of each level's stream
  int qn[kMaxFused + 1];    // rows waiting in each level's queue this batch
  bool hedge[kMaxFused + 1];
  bool lown[kMaxFused + 1];
  // Direct band stores (a wave-uniform choice per level): every lane keeps a
  // pointer to its columns of the next owned row of HL and LH (and of the LL
  // output) and advances it by the band's row length after each row; the HH
  // row sits at a fixed distance from the HL row.  Used when no lane of the
  // wavefront holds a partial vector and every row of the level's bands is
  // vector aligned; otherwise store_band.
  bool fast[kMaxFused + 1];
  char *pHL[kMaxFused + 1], *pLH[kMaxFused + 1], *pLL;
  int64_t dHH[kMaxFused + 1];                       // HH row - HL row (bytes)
  uint32_t sLo[kMaxFused + 1], sHi[kMaxFused + 1];  // bytes per row step
  bool flo[kMaxFused + 1], fhi[kMaxFused + 1];      // lane stores this class

  template <int l> __device__ __forceinline__ auto &E() {
    if constexpr (l == 1) return E1; else if constexpr (l == 2) return E2;
    else if constexpr (l == 3) return E3; else return E4;
  }
  template <int l> __device__ __forceinline__ auto &D() {
    if constexpr (l == 1) return D1; else if constexpr (l == 2) return D2;
    else if constexpr (l == 3) return D3; else return D4;
  }
  template <int l> __device__ __forceinline__ auto &Pw() {
    if constexpr (l == 1) return P1; else if constexpr (l == 2) return P2;
    else if constexpr (l == 3) return P3; else return P4;
  }

  // LDS queue of level l >= 2: QC<l> rows of R<l> words per lane, after the
  // staging rows and the queues of the finer levels.
  template <int l> __device__ __forceinline__ uint32_t *queue() const {
    int off = kStageWords;
    if constexpr (l >= 3) off += 64 * QC<2> * R<2>;
    if constexpr (l >= 4) off += 64 * QC<3> * R<3>;
    return lds + off;
  }

  template <int l> __device__ __forceinline__ bool row_owned(int k) const {
    return k >= (Y0 >> l) && (last_seg || k < (Y1 >> l));
  }

  // Store Mv int16 values (packed pairs) at band columns bc.. of a band row.
  template <int Mv>
  __device__ __forceinline__ void store_band(int16_t *row, int bc, int nvalid, const uint32_t *V) {
    if (nvalid <= 0) return;
    gptr<int16_t> dst = glob(row) + bc;
    const bool aligned = (reinterpret_cast<uintptr_t>(row) & (2 * Mv - 1)) == 0;
    if (nvalid >= Mv && aligned) {
      if constexpr (Mv == 1) *dst = int16_t(V[0]);
      else if constexpr (Mv == 2) *(gptr<uint32_t>)dst = V[0];
      else if constexpr (Mv == 4) *(gptr<u32x2>)dst = u32x2{V[0], V[1]};
      else *(gptr<u32x4>)dst = u32x4{V[0], V[1], V[2], V[3]};
      return;
    }
#pragma unroll
    for (int u = 0; u < Mv; ++u)
      if (u < nvalid) dst[u] = int16_t(Mv == 1 ? V[0] : (V[u >> 1] >> (16 * (u & 1))));
  }

  // Mv int16 values at an aligned address (Mv-element vector).
  template <int Mv> __device__ __forceinline__ static void store_vec(char *p, const uint32_t *V) {
    const gptr<char> g = glob(p);
    if constexpr (Mv == 1) *(gptr<int16_t>)g = int16_t(V[0]);
    else if constexpr (Mv == 2) *(gptr<uint32_t>)g = V[0];
    else if constexpr (Mv == 4) *(gptr<u32x2>)g = u32x2{V[0], V[1]};
    else *(gptr<u32x4>)g = u32x4{V[0], V[1], V[2], V[3]};
  }

  // Low row k of level l: lows -> LL_l (next level's queue / LL output),
  // highs -> HL_l.
  template <int l> __device__ __forceinline__ void emit_low(const uint32_t (&s)[R<l>], int k) {
    constexpr int Np = NP<l>;
    const int N = G.wdim[l - 1];
    const int wl = G.wdim[l];
    const int bc = c0 >> l;
    const bool rown = row_owned<l>(k);
    if (rown && fast[l]) {
      if (fhi[l]) store_vec<M<l>>(pHL[l], s + Np);
      pHL[l] += sHi[l];
    } else if (rown && lown[l]) {
      store_band<M<l>>(pub + G.off_hl[l] + int64_t(k) * (N - wl), bc, (N - wl) - bc, s + Np);
    }
    if constexpr (l < L) {
      constexpr int Mn = M<l + 1>;
      constexpr int Nn = NP<l + 1>;
      uint32_t *dst = queue<l + 1>() + (qn[l + 1] * 64 + lane) * R<l + 1>;
      uint32_t e[Nn], o[Nn];
      if constexpr (Mn >= 2) {
#pragma unroll
        for (int j = 0; j < Nn; ++j) {
          e[j] = lo_halves(s[2 * j], s[2 * j + 1]);
          o[j] = hi_halves(s[2 * j], s[2 * j + 1]);
        }
      } else {
        e[0] = s[0];
        o[0] = s[0] >> 16;
      }
#pragma unroll
      for (int j = 0; j < Nn; ++j) { dst[j] = e[j]; dst[Nn + j] = o[j]; }
      qn[l + 1] += 1;
    } else {
      if (rown && fast[l]) {
        if (flo[l]) store_vec<M<l>>(pLL, s);
        pLL += sLo[l];
      } else if (rown && lown[l]) {
        store_band<M<l>>(llout + int64_t(k) * wl, bc, wl - bc, s);
      }
    }
  }

  // High row k of level l: lows -> LH_l, highs -> HH_l.
  template <int l> __device__ __forceinline__ void emit_high(const uint32_t (&d)[R<l>], int k) {
    if (!row_owned<l>(k)) return;
    constexpr int Np = NP<l>;
    if (fast[l]) {
      if (flo[l]) store_vec<M<l>>(pLH[l], d);
      if (fhi[l]) store_vec<M<l>>(pHL[l] + dHH[l], d + Np);
      pLH[l] += sLo[l];
      return;
    }
    if (!lown[l]) return;
    const int N = G.wdim[l - 1];
    const int wl = G.wdim[l];
    const int bc = c0 >> l;
    store_band<M<l>>(pub + G.off_lh[l] + int64_t(k) * wl, bc, wl - bc, d);
    store_band<M<l>>(pub + G.off_hh[l] + int64_t(k) * (N - wl), bc, (N - wl) - bc, d + Np);
  }

  // Row i of level l, already lifted horizontally (x = lows | highs).
  template <int l> __device__ __forceinline__ void vertical(const uint32_t (&x)[R<l>], int i) {
    constexpr int Rl = R<l>;
    const int N = G.hdim[l - 1];
    auto &Ev = E<l>();
    auto &Dv = D<l>();
    auto &Pv = Pw<l>();
    if (N == 1) {  // no vertical pass: the row is the low row
      emit_low<l>(x, 0);
      return;
    }
    if (i == (r0 >> (l - 1))) {  // first row of this stream (even)
#pragma unroll
      for (int t = 0; t < Rl; ++t) Ev[t] = x[t];
      return;
    }
    const bool odd = (i & 1) != 0;
    if (odd && i != N - 1) {  // waits for its even partner
#pragma unroll
      for (int t = 0; t < Rl; ++t) Pv[t] = x[t];
      return;
    }
    // pair (2k+1, 2k+2): odd row o, even row e; at the end of an even-length
    // signal the odd row is x itself and x(N) = x(N-2), the previous even row
    const int k = odd ? (i - 1) >> 1 : (i - 2) >> 1;
    const bool top = (k == 0);
    uint32_t low[Rl], high[Rl];
#pragma unroll
    for (int t = 0; t < Rl; ++t) {
      const uint32_t o = odd ? x[t] : Pv[t];
      const uint32_t e = odd ? Ev[t] : x[t];
      const uint32_t dn = pk_predict(o, Ev[t], e);
      low[t] = pk_update(Ev[t], top ? dn : Dv[t], dn);
      high[t] = dn;
      Dv[t] = dn;
      Ev[t] = e;
    }
    emit_high<l>(high, k);
    emit_low<l>(low, k);
    if (!odd && i == N - 1) {  // odd length: s(N-1) with d(N) = d(N-2)
#pragma unroll
      for (int t = 0; t < Rl; ++t) low[t] = pk_update(Ev[t], Dv[t], Dv[t]);
      emit_low<l>(low, (N - 1) >> 1);
    }
  }

  // ---- steady-state batches ---------------------------------------------
  // Inside the image and away from the stream's first rows, a batch hands
  // level l a whole number of (odd, even) row pairs: level 1 gets K rows
  // starting with an even row (completing the pair whose odd row waits in
  // P), level l >= 2 gets K >> (l-1) rows starting with an odd row.  Such
  // batches run without the per-row parity / first / last tests, and with
  // the row's edge handling fixed for the whole batch.

  // Pair (2k+1, 2k+2) away from the top: odd row o, even row e.
  template <int l> __device__ __forceinline__ void pair_step(const uint32_t (&o)[R<l>],
                                                             const uint32_t (&e)[R<l>], int k) {
    constexpr int Rl = R<l>;
    auto &Ev = E<l>();
    auto &Dv = D<l>();
    uint32_t low[Rl], high[Rl];
#pragma unroll
    for (int t = 0; t < Rl; ++t) {
      const uint32_t dn = pk_predict(o[t], Ev[t], e[t]);
      low[t] = pk_update(Ev[t], Dv[t], dn);
      high[t] = dn;
      Dv[t] = dn;
      Ev[t] = e[t];
    }
    emit_high<l>(high, k);
    emit_low<l>(low, k);
  }

  // Level 1: K staged rows from even row rb; requires a batch after the
  // stream's first, rb >= 4 and rb + K < H (no first, top or last row).
  template <bool EDGE> __device__ __forceinline__ void phase1_steady(int rb) {
    constexpr int Np = NP<1>;
#pragma unroll 1
    for (int r = 0; r < K; r += 2) {
      uint32_t x[R<1>];
      {
        uint32_t w[RW], Ein[Np], Oin[Np];
        stage_read(r, w);
        unpack(w, Ein, Oin);
        hfwd_pk<M<1>, EDGE>(Ein, Oin, c0, G.wdim[0]);
#pragma unroll
        for (int j = 0; j < Np; ++j) { x[j] = Ein[j]; x[Np + j] = Oin[j]; }
      }
      pair_step<1>(P1, x, (rb + r - 2) >> 1);
      {
        uint32_t w[RW], Ein[Np], Oin[Np];
        stage_read(r + 1, w);
        unpack(w, Ein, Oin);
        hfwd_pk<M<1>, EDGE>(Ein, Oin, c0, G.wdim[0]);
#pragma unroll
        for (int j = 0; j < Np; ++j) { P1[j] = Ein[j]; P1[Np + j] = Oin[j]; }
      }
    }
    icnt[1] += K;
  }

  // Level l >= 2: n queued rows from odd row i0 = icnt[l]; requires i0 >= 3
  // and i0 + n < N.
  template <int l, bool EDGE> __device__ __forceinline__ void phase_steady() {
    constexpr int Np = NP<l>;
    const int n = qn[l];
    const int i0 = icnt[l];
    qn[l] = 0;
    const uint32_t *q = queue<l>();
    auto &Pv = Pw<l>();
#pragma unroll 1
    for (int r = 0; r < n; r += 2) {
      {
        const uint32_t *src = q + (r * 64 + lane) * R<l>;
        uint32_t Ein[Np], Oin[Np];
#pragma unroll
        for (int j = 0; j < Np; ++j) { Ein[j] = src[j]; Oin[j] = src[Np + j]; }
        hfwd_pk<M<l>, EDGE>(Ein, Oin, c0 >> (l - 1), G.wdim[l - 1]);
#pragma unroll
        for (int j = 0; j < Np; ++j) { Pv[j] = Ein[j]; Pv[Np + j] = Oin[j]; }
      }
      uint32_t x[R<l>];
      {
        const uint32_t *src = q + ((r + 1) * 64 + lane) * R<l>;
        uint32_t Ein[Np], Oin[Np];
#pragma unroll
        for (int j = 0; j < Np; ++j) { Ein[j] = src[j]; Oin[j] = src[Np + j]; }
        hfwd_pk<M<l>, EDGE>(Ein, Oin, c0 >> (l - 1), G.wdim[l - 1]);
#pragma unroll
        for (int j = 0; j < Np; ++j) { x[j] = Ein[j]; x[Np + j] = Oin[j]; }
      }
      pair_step<l>(Pv, x, (i0 + r - 1) >> 1);
    }
    icnt[l] += n;
  }

  // Level l's part of a batch: the steady form when it applies.
  template <int l> __device__ __forceinline__ void level_phase() {
    const int n = qn[l];
    const int i0 = icnt[l];
    const int N = G.hdim[l - 1];
    const bool steady = n == (K >> (l - 1)) && n >= 2 && (i0 & 1) && i0 >= 3 && i0 + n < N &&
                        G.wdim[l - 1] > 1;
    if (steady) {
      if (hedge[l]) phase_steady<l, true>();
      else phase_steady<l, false>();
    } else {
      phase<l>();
    }
  }

  // ---- level phases ------------------------------------------------------
  // Level 1 consumes nb staged rows starting at level-0 row rb.
  __device__ __forceinline__ void phase1(int rb, int nb, bool staged) {
#pragma unroll 1
    for (int r = 0; r < nb; ++r) {
      uint32_t w[RW], Ein[NP<1>], Oin[NP<1>];
      if (staged) stage_read(r, w);
      else load_row_slow(rb + r, w);
      unpack(w, Ein, Oin);
      hfwd_pk_any<M<1>>(Ein, Oin, c0, G.wdim[0], hedge[1]);
      uint32_t x[R<1>];
#pragma unroll
      for (int j = 0; j < NP<1>; ++j) { x[j] = Ein[j]; x[NP<1> + j] = Oin[j]; }
      vertical<1>(x, icnt[1]);
      icnt[1] += 1;
    }
  }

  // Level l >= 2 consumes the rows level l-1 queued in this batch.
  template <int l> __device__ __forceinline__ void phase() {
    constexpr int Np = NP<l>;
    const int n = qn[l];
    qn[l] = 0;
    const uint32_t *q = queue<l>();
#pragma unroll 1
    for (int r = 0; r < n; ++r) {
      const uint32_t *src = q + (r * 64 + lane) * R<l>;
      uint32_t Ein[Np], Oin[Np];
#pragma unroll
      for (int j = 0; j < Np; ++j) { Ein[j] = src[j]; Oin[j] = src[Np + j]; }
      hfwd_pk_any<M<l>>(Ein, Oin, c0 >> (l - 1), G.wdim[l - 1], hedge[l]);
      uint32_t x[R<l>];
#pragma unroll
      for (int j = 0; j < Np; ++j) { x[j] = Ein[j]; x[Np + j] = Oin[j]; }
      vertical<l>(x, icnt[l]);
      icnt[l] += 1;
    }
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
        const u32x4 v = *(gptr<const u32x4>)(glob(src) + off + 4u * q);
        w[q] = v.x; w[q + 1] = v.y; w[q + 2] = v.z; w[q + 3] = v.w;
      } else {
        const u32x2 v = *(gptr<const u32x2>)(glob(src) + off + 4u * q);
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
        if constexpr (U8IN) w[t >> 2] |= uint32_t(glob(in8)[rowbase + c]) << (8 * (t & 3));
        else w[t >> 1] |= uint32_t(uint16_t(glob(in16)[rowbase + c])) << (16 * (t & 1));
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
    uint32_t *dst = lds + (k * 64 + lane) * RW;
    if constexpr (RW == 2) {
      *reinterpret_cast<uint2 *>(dst) = make_uint2(w[0], w[1]);
    } else {
#pragma unroll
      for (int q = 0; q < RW / 4; ++q)
        reinterpret_cast<uint4 *>(dst)[q] = make_uint4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
    }
  }
  __device__ __forceinline__ void stage_read(int k, uint32_t (&w)[RW]) const {
    const uint32_t *src = lds + (k * 64 + lane) * RW;
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

  template <int l> __device__ __forceinline__ void setup_stores() {
    constexpr int Mv = M<l>;
    const int wl = G.wdim[l];
    const int wh = G.wdim[l - 1] - wl;
    const int bc = c0 >> l;
    const bool full_lo = lown[l] && wl - bc >= Mv;
    const bool full_hi = lown[l] && wh - bc >= Mv;
    const bool part = lown[l] && ((wl - bc > 0 && wl - bc < Mv) || (wh - bc > 0 && wh - bc < Mv));
    const bool aligned = wl % Mv == 0 && wh % Mv == 0 && G.off_hl[l] % Mv == 0 &&
                         G.off_lh[l] % Mv == 0 && G.off_hh[l] % Mv == 0;
    fast[l] = aligned && __builtin_amdgcn_ballot_w64(part) == 0;
    const int64_t k0 = Y0 >> l;  // first owned row of the level
    pHL[l] = reinterpret_cast<char *>(pub + G.off_hl[l] + k0 * wh + bc);
    dHH[l] = 2 * (G.off_hh[l] - G.off_hl[l]);
    pLH[l] = reinterpret_cast<char *>(pub + G.off_lh[l] + k0 * wl + bc);
    if constexpr (l == L) pLL = reinterpret_cast<char *>(llout + k0 * wl + bc);
    sHi[l] = 2u * uint32_t(wh);
    sLo[l] = 2u * uint32_t(wl);
    flo[l] = full_lo;
    fhi[l] = full_hi;
  }

  __device__ __forceinline__ void run(int wave) {
    const int win = wave % G.n_win;
    const int seg = wave / G.n_win;
    X0 = win * G.own_w;
    last_win = (win == G.n_win - 1);
    last_seg = (seg == G.n_seg - 1);
    Y0 = seg_start(G, seg);
    X1 = last_win ? G.W : X0 + G.own_w;
    Y1 = last_seg ? G.H : seg_start(G, seg + 1);
    const int cbase = (win == 0) ? 0 : X0 - G.halo_l;
    c0 = cbase + lane * C1;
    r0 = Y0 > G.halo_t ? Y0 - G.halo_t : 0;
    const int r1 = min(G.H, Y1 + G.halo_b);
#pragma unroll
    for (int l = 1; l <= L; ++l) {
      const int N = G.wdim[l - 1];
      const int j0 = cbase >> (l - 1);
      const int span = (64 * C1) >> (l - 1);
      hedge[l] = (j0 == 0) || (N - 1 >= j0 && N - 1 < j0 + span);
      const int bc = c0 >> l;
      lown[l] = bc >= (X0 >> l) && (last_win || bc < (X1 >> l));
      icnt[l] = r0 >> (l - 1);
      qn[l] = 0;
    }
    setup_stores<1>();
    if constexpr (L >= 2) setup_stores<2>();
    if constexpr (L >= 3) setup_stores<3>();
    if constexpr (L >= 4) setup_stores<4>();
#pragma unroll
    for (int t = 0; t < R<1>; ++t) { E1[t] = 0; D1[t] = 0; P1[t] = 0; }
#pragma unroll
    for (int t = 0; t < R<2>; ++t) { E2[t] = 0; D2[t] = 0; P2[t] = 0; }
#pragma unroll
    for (int t = 0; t < (L >= 3 ? R<3> : 1); ++t) { E3[t] = 0; D3[t] = 0; P3[t] = 0; }
#pragma unroll
    for (int t = 0; t < (L >= 4 ? R<4> : 1); ++t) { E4[t] = 0; D4[t] = 0; P4[t] = 0; }
    if (r0 >= r1) return;

    uint32_t q[K][RW];
    bool fast_cur = row_fast(min(r1, r0 + K) - 1, cbase);
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
      const bool fast_next = rn < r1 && row_fast(min(r1, rn + K) - 1, cbase);
      if (fast_next) {
#pragma unroll
        for (int k = 0; k < K; ++k)
          if (rn + k < r1) load_row_fast(rn + k, q[k]);  // next batch in flight
      }
      if (fast_cur && nb == K && rb != r0 && rb >= 4 && rb + K < G.H && G.W > 1) {
        if (hedge[1]) phase1_steady<true>(rb);
        else phase1_steady<false>(rb);
      } else {
        phase1(rb, nb, fast_cur);
      }
      wave_lds_sync();
      if constexpr (L >= 2) { level_phase<2>(); wave_lds_sync(); }
      if constexpr (L >= 3) { level_phase<3>(); wave_lds_sync(); }
      if constexpr (L >= 4) { level_phase<4>(); wave_lds_sync(); }
      if (fast_next) {
#pragma unroll
        for (int k = 0; k < K; ++k)
          if (rn + k < r1) stage_write(k, q[k]);
        wave_lds_sync();
      }
      fast_cur = fast_next;
    }
    if (G.use_aes) encrypt_owned();
  }

  // AES-128-CTR over this wavefront's owned LL_L rectangle, in place: the
  // keystream is indexed by the byte offset in the LL band, so each 16-byte
  // block is computed where needed and only the owned elements are XORed
  // (blocks shared with a neighbour's rectangle are computed by both; each
  // writes its own bytes).
  __device__ __forceinline__ void encrypt_owned() {
    const int kr0 = Y0 >> L;
    const int kr1 = last_seg ? G.hdim[L] : min(G.hdim[L], Y1 >> L);
    const int cc0 = min(G.wdim[L], X0 >> L);
    const int cc1 = last_win ? G.wdim[L] : min(G.wdim[L], X1 >> L);
    if (kr0 >= kr1 || cc0 >= cc1) return;
    // this wavefront's clear LL stores complete before it reads them back
    // (the same compute unit; no other wavefront touches these elements)
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    const int64_t wL = G.wdim[L];
    const int64_t band = int64_t(G.hdim[L]) * wL;      // elements in the LL band
    const int nb = ((2 * (cc1 - cc0) + 30) >> 4) + 1;  // blocks a row can touch
    const int total = (kr1 - kr0) * nb;
    const gptr<uint16_t> ll = glob(reinterpret_cast<uint16_t *>(llout));
    // lane work item i = (row kr0 + i / nb, block i % nb of that row); the
    // pair is stepped by 64 items per pass instead of divided each time
    const int step_r = 64 / nb, step_c = 64 % nb;
    int r = kr0 + lane / nb, c = lane % nb;
    for (int i = lane; i < total; i += 64) {
      const int64_t e0 = int64_t(r) * wL + cc0, e1 = int64_t(r) * wL + cc1;  // elements [e0, e1)
      const int64_t b = ((2 * e0) >> 4) + c;
      if (b <= ((2 * e1 - 1) >> 4)) {
        uint32_t w[4];
        counter_block(kw, uint64_t(b), w);
        aes_encrypt(te, kw, w);
        const gptr<u32x4> p = (gptr<u32x4>)(ll + 8 * b);
        if (8 * b + 8 <= band) {
          // the block lies in the band: one 16-byte read; written back whole
          // when all of it is owned, else only the owned elements (bytes of
          // a neighbour's rectangle read with them are discarded, never
          // written)
          u32x4 v = *p;
          v.x ^= w[0]; v.y ^= w[1]; v.z ^= w[2]; v.w ^= w[3];
          if (8 * b >= e0 && 8 * b + 8 <= e1) {
            *p = v;
          } else {
            const uint32_t vw[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int t = 0; t < 8; ++t) {
              const int64_t e = 8 * b + t;
              if (e >= e0 && e < e1) ll[e] = uint16_t(vw[t >> 1] >> (16 * (t & 1)));
            }
          }
        } else {
          // the band's last block runs past its end: element by element
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const int64_t e = 8 * b + t;
            if (e >= e0 && e < e1) ll[e] ^= uint16_t(w[t >> 1] >> (16 * (t & 1)));
          }
        }
      }
      c += step_c;
      r += step_r;
      if (c >= nb) { c -= nb; ++r; }
    }
  }
};

template <int L, int C1, bool U8IN>
__global__ __launch_bounds__(kBlockThreads) void fwd_kernel(const void *__restrict__ in,
                                                            int16_t *__restrict__ pub,
                                                            int16_t *__restrict__ llout,
                                                            const StageParams P) {
  using W = FwdWave<L, C1, U8IN>;
  __shared__ uint32_t s_lds[kWavesPerBlock][W::kLdsWords];
  __shared__ uint32_t s_te[1024];
  __shared__ uint32_t s_kw[kKeyWords];
  if (P.use_aes) load_aes_tables(s_te, s_kw, P.key);
  __syncthreads();
  // the wavefront index is uniform; readfirstlane lets the compiler see that,
  // so all row / level bookkeeping derived from it stays scalar
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wave = blockIdx.x * kWavesPerBlock + wib;
  if (wave >= P.n_waves) return;
  W w{P};
  w.te = s_te;
  w.kw = s_kw;
  w.in8 = static_cast<const uint8_t *>(in);
  w.in16 = static_cast<const int16_t *>(in);
  w.pub = pub;
  w.llout = llout;
  w.lds = s_lds[wib];
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

// Batch form: one persistent launch drains the batch's tile queue; each tile
// is one wavefront rectangle of one item (the item's own plan, buffers and
// keys), run by the streaming code of the item's depth.
template <int L> using FwdB = FwdWave<L, kBatchCols, true>;
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int kFwdBatchLds = cmax(cmax(FwdB<1>::kLdsWords, FwdB<2>::kLdsWords),
                                  cmax(FwdB<3>::kLdsWords, FwdB<4>::kLdsWords));

template <int L>
__device__ __forceinline__ void fwd_batch_tile(const BatchItem &it, int wave, uint32_t *lds,
                                               const uint32_t *te, const uint32_t *kw, int lane) {
  FwdB<L> w{it.fwd};
  w.te = te;
  w.kw = kw;
  w.in8 = it.in;
  w.in16 = nullptr;
  w.pub = it.pub;
  w.llout = reinterpret_cast<int16_t *>(it.priv);
  w.lds = lds;
  w.lane = lane;
  w.run(wave);
}

__global__ __launch_bounds__(kBlockThreads) void fwd_batch_kernel(const BatchItem *__restrict__ items,
                                                                  const int2 *__restrict__ tiles,
                                                                  int64_t n_tiles,
                                                                  BatchCounters *__restrict__ ctr) {
  __shared__ uint32_t s_lds[kWavesPerBlock][kFwdBatchLds];
  __shared__ uint32_t s_te[1024];
  __shared__ uint32_t s_kw[kWavesPerBlock][kKeyWords];
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
    if (lane < kKeyWords) s_kw[wib][lane] = key_word(it.fwd.key, lane);  // this item's keys
    wave_lds_sync();
    switch (__builtin_amdgcn_readfirstlane(it.levels)) {
      case 1: fwd_batch_tile<1>(it, e.y, s_lds[wib], s_te, s_kw[wib], lane); break;
      case 2: fwd_batch_tile<2>(it, e.y, s_lds[wib], s_te, s_kw[wib], lane); break;
      case 3: fwd_batch_tile<3>(it, e.y, s_lds[wib], s_te, s_kw[wib], lane); break;
      default: fwd_batch_tile<4>(it, e.y, s_lds[wib], s_te, s_kw[wib], lane); break;
    }
    wave_lds_sync();
  }
  batch_finish(ctr);
}

hipError_t launch_fwd_batch(const BatchItem *items, const int2 *tiles, int64_t n_tiles,
                            BatchCounters *ctr, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(fwd_batch_kernel, dim3(blocks), dim3(kBlockThreads), 0, s, items, tiles,
                     n_tiles, ctr);
  return hipGetLastError();
}

// Resident workgroups per CU of the batch forward kernel.
int fwd_batch_blocks_per_cu() {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, reinterpret_cast<const void *>(&fwd_batch_kernel),
                                                   kBlockThreads, 0) != hipSuccess)
    return 0;
  return blocks;
}

// Resident wavefronts per CU of the forward kernel for (L, C1).
int fwd_waves_per_cu(int L, int C1, bool u8in) {
  const void *fn = nullptr;
#define DWTFRAG_FN(LL, CC)                                                              \
  if (L == LL && C1 == CC)                                                              \
    fn = u8in ? reinterpret_cast<const void *>(&fwd_kernel<LL, CC, true>)               \
              : reinterpret_cast<const void *>(&fwd_kernel<LL, CC, false>);
  DWTFRAG_FN(1, 8) DWTFRAG_FN(2, 8) DWTFRAG_FN(3, 8)
  DWTFRAG_FN(1, 16) DWTFRAG_FN(2, 16) DWTFRAG_FN(3, 16) DWTFRAG_FN(4, 16)
#undef DWTFRAG_FN
  int blocks = 0;
  if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, kBlockThreads, 0) != hipSuccess)
    return 0;
  return blocks * kWavesPerBlock;
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
