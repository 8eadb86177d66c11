// Learned-predictor lifting and its trainer.
//
// The predict step of the 5/3 lifting (Ch. 5 section 5.1.1, eq. (5.1)) gains
// an integer correction from a small context network; the update step
// (eq. (5.2), additive reading) is unchanged, so the map stays an exact
// integer bijection and the fragments stay lossless (section 5.2.3).  At an
// odd position i of a signal x of length N >= 2 (m = whole-sample mirror):
//   base = floor((x(m(i-1)) + x(m(i+1))) / 2)
//   c_j  = clamp(x(m(i + 2j - 7)) - base, -128, 127)               j = 0..7
//   h_k  = max(0, sum_j W1[k][j] c_j + b1[k])                       k = 0..15
//   corr = clamp(floor((sum_k W2[k] h_k + b2) / 2^shift), -255, 255)
//   d(i) = x(i) - base - corr
// The context reads even samples only, which the inverse rebuilds first.
//
// Layout of the work: the network's hidden layer runs on the matrix cores
// (int8 MFMA, see correction_mfma), its output layer and the context on the
// VALU; that is still ~60 operations per predicted sample against ~2 for the
// plain predict, so this path is ALU-bound.  Protect and restore run one
// fused kernel per level and direction (both 1-D passes of a 32 x 128 tile
// in LDS, int16 samples, halos recomputed), so the only HBM traffic is each
// level's input and output.  The training-pair capture keeps one kernel per
// 1-D pass: a block takes SEG positions of LINES independent lines (rows: 1
// line of 2048 positions; columns: 64 lines of 64 positions), loads them with
// an 8-sample halo on each side, mirrored at the signal edges, into LDS as
// separate even and odd planes, then predicts the odd samples and updates
// the even ones.
//
// The trainer fits the network with quantisation-aware Adam.  Its gradient
// is taken at the fake-quantised parameters (integers over powers of two),
// where every quantity of the real-valued network is a dyadic rational: the
// kernels accumulate exact integer sums and scale them once at the end, so
// the gradient is the exact one rounded to float.
#include "dwtfrag.h"

#include "common.h"

namespace dwtfrag {

constexpr int kHidden = 16;
constexpr int kCtx = 8;
constexpr int kParams = kHidden * kCtx + kHidden + kHidden + 1;  // 161
constexpr int kSums = kParams + 1;                               // + loss
constexpr int kGradBlocks = 512;
constexpr int kHalo = 8;

// Network as kernel argument: W1 rows packed as two int8x4 words (c_0 in the
// low byte), W2 sign-extended.
struct Net {
  uint32_t w1[kHidden][2];
  int32_t b1[kHidden];
  int32_t w2[kHidden];
  int32_t b2, shift;
};

Net pack_net(const dwtfrag_predictor &p) {
  Net n{};
  for (int k = 0; k < kHidden; ++k) {
    for (int h = 0; h < 2; ++h) {
      uint32_t w = 0;
      for (int b = 0; b < 4; ++b) w |= uint32_t(uint8_t(p.w1[k][4 * h + b])) << (8 * b);
      n.w1[k][h] = w;
    }
    n.b1[k] = p.b1[k];
    n.w2[k] = p.w2[k];
  }
  n.b2 = p.b2;
  n.shift = p.shift;
  return n;
}

// ------------------------------------------------------------ network --

__device__ __forceinline__ int clamp_i(int v, int lo, int hi) { return min(max(v, lo), hi); }

// four int8 values (low bytes of a..d) -> one word, a in the low byte
__device__ __forceinline__ uint32_t pack4(int a, int b, int c, int d) {
  const uint32_t ab = __builtin_amdgcn_perm(uint32_t(b), uint32_t(a), 0x0c0c0400u);
  const uint32_t cd = __builtin_amdgcn_perm(uint32_t(d), uint32_t(c), 0x0c0c0400u);
  return __builtin_amdgcn_perm(cd, ab, 0x05040100u);
}

// Hidden pre-activations of a packed context.
__device__ __forceinline__ int hidden_pre(const uint32_t (&w1)[2], int b1, uint32_t lo, uint32_t hi) {
  const int p = __builtin_amdgcn_sdot4(int(lo), int(w1[0]), b1, false);
  return __builtin_amdgcn_sdot4(int(hi), int(w1[1]), p, false);
}

// corr of 64 contexts at once, one per lane of a wavefront (context of lane
// l = sample l), on the matrix cores.  The hidden layer is
// D = A_g x B + bias with v_mfma_i32_16x16x32_i8: B (32 x 16) holds, in
// k-group g = l / 16 and column l % 16, the eight context bytes of lane l;
// A_g (16 x 32) holds W1 in k-group g and zeros elsewhere, so D_g's column j
// is the 16 hidden pre-activations of sample 16 g + j.  Lane l receives rows
// 4 (l / 16) .. +3 of column l % 16; ReLU, the W2 products and a sum over
// the four 16-lane rows give the output of sample 16 g + l % 16, which lane
// 16 g + l % 16 keeps.  Every step is exact integer arithmetic; h < 2^18
// under the parameter limits the entry points check, so the clamp to
// 2^23 - 1 is a no-op that lets W2 h run as a 24-bit multiply.  All 64 lanes
// must call it together.
typedef int v4i __attribute__((ext_vector_type(4)));

struct MfmaNet {
  long a[4];   // A_g operand of this lane: W1 row (l % 16) in k-group l / 16 == g
  v4i bias;    // b1 of hidden rows 4 (l / 16) + r
  int w2[4];   // W2 of the same rows
  int b2, shift;
};

// Net staged in LDS as words: w1 (32), b1 (16), w2 (16).
__device__ __forceinline__ MfmaNet mfma_net(const uint32_t *s_net, int b2, int shift, int lane) {
  MfmaNet m;
  const int h = lane & 15, g0 = lane >> 4;
  const long w = long(s_net[2 * h]) | (long(s_net[2 * h + 1]) << 32);
#pragma unroll
  for (int g = 0; g < 4; ++g) m.a[g] = (g == g0) ? w : 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    m.bias[r] = int(s_net[32 + 4 * g0 + r]);
    m.w2[r] = (int(s_net[48 + 4 * g0 + r]) << 24) >> 24;
  }
  m.b2 = b2;
  m.shift = shift;
  return m;
}

// v_mad_i32_i24 as one instruction: the products of the output layer are
// chained through it (the compiler would otherwise regroup four products as
// three multiplies, a multiply-add and a three-input add).
__device__ __forceinline__ int mad24(int a, int b, int c) {
  int r;
  asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

// Eight int8 context bytes (c_0 in the low byte) of int32 samples.
__device__ __forceinline__ long pack_context(const int (&e)[kCtx], int base) {
  int c[kCtx];
#pragma unroll
  for (int j = 0; j < kCtx; ++j) c[j] = clamp_i(e[j] - base, -128, 127);
  return long(pack4(c[0], c[1], c[2], c[3])) | (long(pack4(c[4], c[5], c[6], c[7])) << 32);
}

__device__ __forceinline__ int correction_packed(const MfmaNet &m, long b) {
  // p[g]: this lane's quarter of the output sum of group g's sample l % 16
  // (its four hidden units 4q..4q+3, q = l / 16); the four products are
  // independent, so they are all issued before the first result is read
  v4i d[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) d[g] = __builtin_amdgcn_mfma_i32_16x16x32_i8(m.a[g], b, m.bias, 0, 0, 0);
  int p[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    int sum = __mul24(clamp_i(d[g][0], 0, 0x7fffff), m.w2[0]);
#pragma unroll
    for (int r = 1; r < 4; ++r) sum = mad24(clamp_i(d[g][r], 0, 0x7fffff), m.w2[r], sum);
    p[g] = sum;
  }
  // Lane l needs group q's total: the sum of p[q] over lanes s, s+16, s+32,
  // s+48 (s = l % 16, q = l / 16).  Swapping the upper 32 lanes of p[0]
  // (p[1]) with the lower 32 lanes of p[2] (p[3]) leaves each lane both
  // halves' terms of group 0 (1) in the lower half and of group 2 (3) in the
  // upper half: k0 (k1) sums quarters {q, q ^ 2}.  Swapping the odd 16-lane
  // rows of k0 with the even rows of k1 then gives every row r the two
  // partial sums of group r.
  const auto s02 = __builtin_amdgcn_permlane32_swap(unsigned(p[0]), unsigned(p[2]), false, false);
  const auto s13 = __builtin_amdgcn_permlane32_swap(unsigned(p[1]), unsigned(p[3]), false, false);
  const unsigned k0 = s02[0] + s02[1], k1 = s13[0] + s13[1];
  const auto s01 = __builtin_amdgcn_permlane16_swap(k0, k1, false, false);
  const int mine = int(s01[0] + s01[1]);
  return clamp_i((mine + m.b2) >> m.shift, -255, 255);
}

__device__ __forceinline__ int correction_mfma(const MfmaNet &m, const int (&e)[kCtx], int base) {
  return correction_packed(m, pack_context(e, base));
}

// The context of eight int16 samples at[0], at[2 s], .., at[14 s] in packed
// 16-bit arithmetic: base = floor((at[6 s] + at[8 s]) / 2) is returned
// through *base; the differences saturate at the int16 range, which leaves
// their clamp to [-128, 127] unchanged, and the bytes are gathered by two
// permutes.
typedef short s16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ long context16(const int16_t *at, int s, int *base) {
  const s16x2 e01 = {at[0], at[2 * s]}, e23 = {at[4 * s], at[6 * s]};
  const s16x2 e45 = {at[8 * s], at[10 * s]}, e67 = {at[12 * s], at[14 * s]};
  const int bs = (int(e23.y) + int(e45.x)) >> 1;
  *base = bs;
  const s16x2 b2 = {short(bs), short(bs)}, lo = {-128, -128}, hi = {127, 127};
  const auto cl = [&](s16x2 v) {
    return __builtin_bit_cast(
        uint32_t, __builtin_elementwise_min(__builtin_elementwise_max(__builtin_elementwise_sub_sat(v, b2), lo), hi));
  };
  const uint32_t a = __builtin_amdgcn_perm(cl(e23), cl(e01), 0x06040200u);
  const uint32_t b = __builtin_amdgcn_perm(cl(e67), cl(e45), 0x06040200u);
  return long(a) | (long(b) << 32);
}

// Stage the network in LDS (one copy per block) for mfma_net.
__device__ __forceinline__ void stage_net(uint32_t *s_net, const Net &net) {
  const int t = int(threadIdx.x);
  if (t < 32) s_net[t] = net.w1[t >> 1][t & 1];
  else if (t < 48) s_net[t] = uint32_t(net.b1[t - 32]);
  else if (t < 64) s_net[t] = uint32_t(net.w2[t - 48]);
}

// whole-sample symmetric index for a signal of length N
__device__ __forceinline__ int mirror_pos(int g, int N) {
  if (g >= 0 && g < N) return g;
  if (N == 1) return 0;
  const int P = 2 * (N - 1);
  int r = g % P;
  if (r < 0) r += P;
  return r >= N ? P - r : r;
}

// ------------------------------------------------ sources and sinks --
// A pass sees its array as LINES independent 1-D signals of length N:
// (line, pos) = (row, column) for row passes, (column, row) for columns.

struct SrcView {  // level-0 byte view, zero past n
  const uint8_t *p;
  int64_t n;
  int pitch;
  __device__ int operator()(int line, int pos) const {
    const int64_t o = int64_t(line) * pitch + pos;
    return o < n ? int(p[o]) : 0;
  }
};
struct SrcRows {
  const int32_t *p;
  int pitch;
  __device__ int operator()(int line, int pos) const { return p[int64_t(line) * pitch + pos]; }
};
struct SrcCols {
  const int32_t *p;
  int pitch;
  __device__ int operator()(int line, int pos) const { return p[int64_t(pos) * pitch + line]; }
};

// Row pass output: [lows | highs] per row.
struct SinkRows {
  int32_t *p;
  int pitch, nlow;
  __device__ void low(int line, int k, int v) const { p[int64_t(line) * pitch + k] = v; }
  __device__ void high(int line, int k, int v) const { p[int64_t(line) * pitch + nlow + k] = v; }
};
// Column pass output: the four bands of the level.  Column c < wl of the
// row-pass output holds row lows (LL above, LH below), the others row highs
// (HL, HH).  LL goes to int32 (next level) or int16 (last level); a null
// pointer discards the band.
struct Bands {
  int32_t *ll32;
  int16_t *ll16, *hl, *lh, *hh;
  int wl, wh;
  __device__ void low(int c, int r, int v) const {
    if (c < wl) {
      if (ll32) ll32[int64_t(r) * wl + c] = v;
      else if (ll16) ll16[int64_t(r) * wl + c] = int16_t(v);
    } else if (hl) {
      hl[int64_t(r) * wh + (c - wl)] = int16_t(v);
    }
  }
  __device__ void high(int c, int r, int v) const {
    if (c < wl) {
      if (lh) lh[int64_t(r) * wl + c] = int16_t(v);
    } else if (hh) {
      hh[int64_t(r) * wh + (c - wl)] = int16_t(v);
    }
  }
};

// (context, target) capture of every predict step, for training: pair index
// off + line * per_line + (i - 1) / 2.
struct Capture {
  uint2 *ctx;
  int32_t *target;
  int64_t off;
  int64_t per_line;
};

// ------------------------------------------------------------ kernels --

template <int LINES, int SEG>
struct Tile {
  static constexpr int NE = SEG / 2 + kHalo;  // even slots: positions s0-8 .. s0+SEG+6
  static constexpr int NO = SEG / 2 + 1;      // odd slots: positions s0-1 .. s0+SEG-1
  static constexpr int kThreads = 256;
  static_assert((LINES & (LINES - 1)) == 0 && kThreads % LINES == 0, "LINES: power of two");
};

__device__ __forceinline__ void tile_coords(int n_seg, int SEG, int LINES, int *s0, int *l0) {
  const int b = int(blockIdx.x);
  *s0 = (b % n_seg) * SEG;
  *l0 = (b / n_seg) * LINES;
}

template <int LINES, int SEG, class Src, class Sink, bool CAPTURE>
__global__ __launch_bounds__(256) void lfwd_kernel(Src src, Sink sink, const Net net, int N,
                                                   int n_lines, int n_seg, Capture cap) {
  using T = Tile<LINES, SEG>;
  __shared__ int32_t sE[T::NE * LINES];
  __shared__ int32_t sO[T::NO * LINES];
  __shared__ int32_t sD[T::NO * LINES];
  __shared__ uint32_t s_net[64];
  int s0, l0;
  tile_coords(n_seg, SEG, LINES, &s0, &l0);
  const int tid = int(threadIdx.x);
  stage_net(s_net, net);

  // positions s0-8 .. s0+SEG+7 (mirrored), split by parity
  for (int idx = tid; idx < (SEG + 2 * kHalo) * LINES; idx += T::kThreads) {
    const int li = idx % LINES, k = idx / LINES, line = l0 + li;
    if (!(k & 1)) {
      sE[(k >> 1) * LINES + li] = line < n_lines ? src(line, mirror_pos(s0 - kHalo + k, N)) : 0;
    } else {
      const int q = (k - 7) >> 1;
      if (k >= 7 && q < T::NO)
        sO[q * LINES + li] = line < n_lines ? src(line, mirror_pos(s0 - kHalo + k, N)) : 0;
    }
  }
  __syncthreads();

  // predict, eq. (5.1) plus the correction, at odd i = s0 - 1 + 2q; the
  // loop trip count is uniform per wavefront (the network runs on the matrix
  // cores with every lane active), lanes past the end only pad
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const MfmaNet mn = mfma_net(s_net, net.b2, net.shift, lane);
  for (int base0 = wave * 64; base0 < T::NO * LINES; base0 += T::kThreads) {
    const int idx = base0 + lane;
    const bool in = idx < T::NO * LINES;
    const int li = in ? idx % LINES : 0, q = in ? idx / LINES : 0, line = l0 + li;
    const int i = s0 - 1 + 2 * q;
    const bool valid = in && i > 0 && i < N && line < n_lines;
    int e[kCtx];
#pragma unroll
    for (int j = 0; j < kCtx; ++j) e[j] = sE[(q + j) * LINES + li];
    const int base = (e[3] + e[4]) >> 1;
    const int corr = correction_mfma(mn, e, base);
    if (!valid) continue;
    const int x = sO[q * LINES + li];
    sD[q * LINES + li] = x - base - corr;
    if (CAPTURE && q >= 1 && i < s0 + SEG) {
      int c[kCtx];
#pragma unroll
      for (int j = 0; j < kCtx; ++j) c[j] = clamp_i(e[j] - base, -128, 127);
      const int64_t at = cap.off + int64_t(line) * cap.per_line + ((i - 1) >> 1);
      cap.ctx[at] = make_uint2(pack4(c[0], c[1], c[2], c[3]), pack4(c[4], c[5], c[6], c[7]));
      cap.target[at] = x - base;
    }
  }
  __syncthreads();

  // update, eq. (5.2), at even i = s0 + 2 e2; store lows and highs
  for (int idx = tid; idx < (SEG / 2) * LINES; idx += T::kThreads) {
    const int li = idx % LINES, e2 = idx / LINES, line = l0 + li;
    const int i = s0 + 2 * e2;
    if (i >= N || line >= n_lines) continue;
    const int x = sE[(e2 + 4) * LINES + li];
    if (N == 1) {
      sink.low(line, 0, x);
      continue;
    }
    const int dl = sD[(i == 0 ? 1 : e2) * LINES + li];          // d(m(i-1))
    const int dr = sD[(i == N - 1 ? e2 : e2 + 1) * LINES + li];  // d(m(i+1))
    sink.low(line, i >> 1, x + ((dl + dr + 2) >> 2));
    if (i + 1 < N) sink.high(line, i >> 1, sD[(e2 + 1) * LINES + li]);
  }
}

// Launch shapes: rows take one line of 2048 positions per block, columns 64
// lines (adjacent columns: coalesced rows of 256 bytes) of 64 positions.
constexpr int kRowSeg = 2048;
constexpr int kColLines = 64;
constexpr int kColSeg = 64;

template <int LINES, int SEG>
bool grid_for(int N, int n_lines, int *n_seg, unsigned *grid) {
  *n_seg = (N + SEG - 1) / SEG;
  const int64_t blocks = int64_t(*n_seg) * ((n_lines + LINES - 1) / LINES);
  if (blocks <= 0 || blocks > 0x7fffffff) return false;
  *grid = unsigned(blocks);
  return true;
}

template <class Src, class Sink>
hipError_t row_fwd(Src src, Sink sink, const Net &net, int N, int lines, const Capture *cap,
                   hipStream_t s) {
  int n_seg;
  unsigned grid;
  if (!grid_for<1, kRowSeg>(N, lines, &n_seg, &grid)) return hipErrorInvalidValue;
  if (cap)
    hipLaunchKernelGGL((lfwd_kernel<1, kRowSeg, Src, Sink, true>), dim3(grid), dim3(256), 0, s, src,
                       sink, net, N, lines, n_seg, *cap);
  else
    hipLaunchKernelGGL((lfwd_kernel<1, kRowSeg, Src, Sink, false>), dim3(grid), dim3(256), 0, s,
                       src, sink, net, N, lines, n_seg, Capture{});
  return hipGetLastError();
}

template <class Src, class Sink>
hipError_t col_fwd(Src src, Sink sink, const Net &net, int N, int lines, const Capture *cap,
                   hipStream_t s) {
  int n_seg;
  unsigned grid;
  if (!grid_for<kColLines, kColSeg>(N, lines, &n_seg, &grid)) return hipErrorInvalidValue;
  if (cap)
    hipLaunchKernelGGL((lfwd_kernel<kColLines, kColSeg, Src, Sink, true>), dim3(grid), dim3(256), 0,
                       s, src, sink, net, N, lines, n_seg, *cap);
  else
    hipLaunchKernelGGL((lfwd_kernel<kColLines, kColSeg, Src, Sink, false>), dim3(grid), dim3(256),
                       0, s, src, sink, net, N, lines, n_seg, Capture{});
  return hipGetLastError();
}

// ------------------------------------------------ fused per-level kernels --
// Protect and restore run one launch per level and direction.  A block owns
// an Ht x kLvW rectangle of the level's sample grid (first row r0 and first
// column c0, both even) and runs both 1-D passes of the level over it in
// LDS, with the halos they need:
//   forward: the row pass over the rows the column pass reads (even rows
//     r0-8 .. r0+Ht+6, odd rows r0-1 .. r0+Ht-1), on columns
//     c0-8 .. c0+kLvW+6; then the column pass on the owned columns;
//   inverse: the column pass over columns c0-7 .. c0+kLvW+7 (rows
//     r0-7 .. r0+Ht+7 loaded), then the row pass on the owned rows.
// Rows and columns outside the level are loaded mirrored (whole-sample),
// the extension the definition uses: the update and its inverse are
// symmetric about each edge, the context reads mirrored samples by
// definition, and a predict at a mirrored position outside the signal is
// never used (the update of the first and last sample takes the mirrored
// real neighbour instead).  Samples are updated in place in LDS: int16 in
// the forward (every coefficient and intermediate of a byte input fits for
// up to three levels), int32 in the inverse, which must reproduce the
// definition for any fragment contents, also those no protect produces.
// Predicts go in batches of 64, one per lane, so that each wavefront calls
// the matrix-core network with every lane active.
// Ht is 32 in both directions: a taller forward tile recomputes fewer halo
// rows in its row pass, but its LDS holds fewer blocks per compute unit, and
// the wavefronts need the occupancy more (measured: 32 rows beat 48 and 64,
// and in the inverse 16 and 48).
constexpr int kFwdH = 32, kInvH = 32, kLvW = 128;
constexpr int kLvPitch = kLvW + 16;  // local column q <-> c0 - 8 + q; local row k <-> r0 - 8 + k
static_assert(kLvW == 128, "the row passes give each lane two columns of a 128-column tile");

// Tile loads: each thread keeps eight global loads in flight, then writes
// them to LDS (load(idx) reads element idx of the tile, store(idx, v)
// places it).
template <int TOTAL, class Load, class Store>
__device__ __forceinline__ void tile_load(const Load &load, const Store &store) {
  constexpr int kU = 8;
  for (int base = 0; base < TOTAL; base += 256 * kU) {
    int v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int idx = base + u * 256 + int(threadIdx.x);
      v[u] = idx < TOTAL ? load(idx) : 0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int idx = base + u * 256 + int(threadIdx.x);
      if (idx < TOTAL) store(idx, v[u]);
    }
  }
}

// Sources and sinks of the fused kernels.  quad(r, c, W, &ok) reads the
// four samples c .. c+3 of row r (c a multiple of 4) with one vector load,
// raw; ok says whether that form applies (every sample inside the row and
// the buffer).  Where it does not, the load reads the start of the row
// instead, so that the loads of a thread carry no branch and can all be in
// flight together; the caller then reads single samples.  Only called where
// the host set vec: the alignment holds, and every row start read this way
// is inside its band (with vec unset a band may be empty, its pointer null).
struct LvSrc8 {  // level-0 bytes, zero past n
  const uint8_t *p;
  int64_t n;
  int pitch;
  int vec;  // pitch and p 4-byte aligned, n >= 4
  __device__ int operator()(int r, int c) const {
    const int64_t o = int64_t(r) * pitch + c;
    return o < n ? int(p[o]) : 0;
  }
  __device__ uint32_t quad(int r, int c, int W, bool *ok) const {
    const int64_t o = int64_t(r) * pitch + c;
    *ok = vec && c >= 0 && c + 4 <= W && o + 4 <= n;
    return *reinterpret_cast<const uint32_t *>(p + (*ok ? o : 0));
  }
  // the raw quad as four int16 lanes
  static __device__ uint2 widen(uint32_t w) {
    return make_uint2(__builtin_amdgcn_perm(0u, w, 0x0c010c00u), __builtin_amdgcn_perm(0u, w, 0x0c030c02u));
  }
};
struct LvSrc16 {  // an LL band of the previous level
  const int16_t *p;
  int pitch;
  int vec;  // pitch a multiple of 4, p 8-byte aligned
  __device__ int operator()(int r, int c) const { return p[int64_t(r) * pitch + c]; }
  __device__ uint2 quad(int r, int c, int W, bool *ok) const {
    *ok = vec && c >= 0 && c + 4 <= W;
    return *reinterpret_cast<const uint2 *>(p + int64_t(r) * pitch + (*ok ? c : 0));
  }
  static __device__ uint2 widen(uint2 v) { return v; }
};
// The four bands of a level (LL: next level's input or the private
// fragment); wl / wh: columns of the row lows / highs.
struct LvBands {
  int16_t *ll, *hl, *lh, *hh;
  int wl, wh;
};
// Coefficient (r, c) of a level's interleaved grid: the band by the
// parities; LL from int16 (the private fragment) or int32 (a level below).
struct LvCoef {
  const int16_t *ll16;
  const int32_t *ll32;
  const int16_t *hl, *lh, *hh;
  int wl, wh;
  int vec;  // H >= 2; wl, wh even; the int16 bands 4-byte and ll32 8-byte aligned
  __device__ int operator()(int r, int c) const {
    const int64_t rr = r >> 1, cc = c >> 1;
    if (!(r & 1)) {
      if (c & 1) return hl[rr * wh + cc];
      return ll32 ? ll32[rr * wl + cc] : int(ll16[rr * wl + cc]);
    }
    return (c & 1) ? hh[rr * wh + cc] : lh[rr * wl + cc];
  }
  // Samples c .. c+3 of row r: two of the even-column band (a: int16 pair,
  // or a32: int32 pair where the row is even and LL is int32) and two of the
  // odd one (b).  The row's parity and LL's width are fixed per call site.
  template <bool ODD, bool LL32>
  __device__ void quad(int r, int c, int W, bool *ok, uint32_t *a, uint2 *a32, uint32_t *b) const {
    *ok = vec && c >= 0 && c + 4 <= W;
    const int64_t rr = r >> 1, cc = *ok ? (c >> 1) : 0;
    if (ODD) {
      *a = *reinterpret_cast<const uint32_t *>(lh + rr * wl + cc);
      *b = *reinterpret_cast<const uint32_t *>(hh + rr * wh + cc);
    } else {
      if (LL32) *a32 = *reinterpret_cast<const uint2 *>(ll32 + rr * wl + cc);
      else *a = *reinterpret_cast<const uint32_t *>(ll16 + rr * wl + cc);
      *b = *reinterpret_cast<const uint32_t *>(hl + rr * wh + cc);
    }
  }
};
struct LvDst8 {  // level-0 bytes, first n only, modulo 256
  uint8_t *p;
  int64_t n;
  int pitch;
  __device__ void operator()(int r, int c, int v) const {
    const int64_t o = int64_t(r) * pitch + c;
    if (o < n) p[o] = uint8_t(v);
  }
};
struct LvDst32 {
  int32_t *p;
  int pitch;
  __device__ void operator()(int r, int c, int v) const { p[int64_t(r) * pitch + c] = v; }
};

template <class T>
__device__ __forceinline__ void load_context(const T *at, int stride, int (&e)[kCtx]) {
#pragma unroll
  for (int j = 0; j < kCtx; ++j) e[j] = at[2 * j * stride];
}

template <class Src>
__global__ __launch_bounds__(256) void lfwd_level_kernel(Src src, LvBands out, const Net net, int H,
                                                         int W, int tiles_x) {
  __shared__ int16_t X[(kFwdH + 16) * kLvPitch];
  __shared__ uint32_t s_net[64];
  constexpr int P = kLvPitch;
  constexpr int kEvRows = kFwdH / 2 + 8;                // even local rows 0, 2, .., kFwdH+14
  constexpr int kRows = kEvRows + kFwdH / 2 + 1;        // + odd local rows 7, 9, .., kFwdH+7
  constexpr int kCols = kLvW + 15;                     // local columns 0 .. kLvW+14
  const int tid = int(threadIdx.x);
  const int r0 = int(blockIdx.x / unsigned(tiles_x)) * kFwdH;
  const int c0 = int(blockIdx.x % unsigned(tiles_x)) * kLvW;
  const auto local_row = [](int t) { return t < kEvRows ? 2 * t : 7 + 2 * (t - kEvRows); };
  stage_net(s_net, net);
  // tile loads: groups of 36 threads take a row, four samples each (local
  // columns 0 .. 143); where a quad cannot be read whole, the block reads
  // every sample of the tile singly instead
  bool miss = !src.vec;
  if (src.vec) {
    const int slot = tid % 36, grp = tid / 36;  // 7 groups; threads 252 .. 255 idle
    constexpr int kU = 4;
    for (int t0 = 0; t0 < kRows; t0 += 7 * kU) {
      decltype(src.quad(0, 0, 0, &miss)) v[kU];
      bool ok[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int t = min(t0 + grp + 7 * u, kRows - 1);
        v[u] = src.quad(mirror_pos(r0 - 8 + local_row(t), H), c0 - 8 + 4 * slot, W, &ok[u]);
        ok[u] = ok[u] && grp < 7 && t0 + grp + 7 * u < kRows;
        miss |= grp < 7 && t0 + grp + 7 * u < kRows && !ok[u];
      }
#pragma unroll
      for (int u = 0; u < kU; ++u)
        if (ok[u])
          *reinterpret_cast<uint2 *>(X + local_row(t0 + grp + 7 * u) * P + 4 * slot) = Src::widen(v[u]);
    }
  }
  if (__syncthreads_or(miss)) {
    tile_load<kRows * kCols>(
        [&](int idx) {
          const int t = idx / kCols, q = idx - t * kCols;
          return src(mirror_pos(r0 - 8 + local_row(t), H), mirror_pos(c0 - 8 + q, W));
        },
        [&](int idx, int v) {
          const int t = idx / kCols, q = idx - t * kCols;
          X[local_row(t) * P + q] = int16_t(v);
        });
  }
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const MfmaNet mn = mfma_net(s_net, net.b2, net.shift, lane);

  // row pass, predict: a batch per row at the owned odd columns (q = 9 +
  // 2 lane), then batches of 64 rows at the odd column q = 7 (c0 - 1), on
  // the waves the row batches leave least loaded
  {
    const int q = 9 + 2 * lane;
    const bool col_ok = c0 + 1 + 2 * lane < W;
    for (int t = wave; t < kRows; t += 4) {
      int16_t *row = X + local_row(t) * P;
      int base;
      const int corr = correction_packed(mn, context16(row + q - 7, 1, &base));
      if (col_ok) row[q] = int16_t(row[q] - base - corr);
    }
    for (int b = (wave + 4 - kRows % 4) % 4; b < (kRows + 63) / 64; b += 4) {
      const int t = b * 64 + lane;
      const bool in = t < kRows;
      int16_t *at = X + local_row(in ? t : 0) * P + 7;
      int base;
      const int corr = correction_packed(mn, context16(at - 7, 1, &base));
      if (in && c0 > 0) *at = int16_t(*at - base - corr);
    }
  }
  __syncthreads();
  // row pass, update at the owned even columns (q = 8 + 2 lane)
  if (W > 1) {
    for (int t = wave; t < kRows; t += 4) {
      const int k = local_row(t), q = 8 + 2 * lane, c = c0 + 2 * lane;
      if (c < W) {
        int16_t *row = X + k * P;
        const int dl = row[c == 0 ? q + 1 : q - 1];
        const int dr = row[c == W - 1 ? q - 1 : q + 1];
        row[q] = int16_t(row[q] + ((dl + dr + 2) >> 2));
      }
    }
  }
  __syncthreads();
  // column pass, predict at the odd rows k = 7 (r0 - 1), 9, .., kFwdH+7 of
  // the owned columns, 64 columns per batch
  for (int b = wave; b < (kFwdH / 2 + 1) * 2; b += 4) {
    const int k = 7 + 2 * (b >> 1), q = 8 + 64 * (b & 1) + lane;
    int base;
    const int corr = correction_packed(mn, context16(X + (k - 7) * P + q, P, &base));
    const int i = r0 - 8 + k;
    if (i > 0 && i < H && c0 - 8 + q < W) X[k * P + q] = int16_t(X[k * P + q] - base - corr);
  }
  __syncthreads();
  // column pass, update at the owned even rows; each lane stores the band
  // samples of the column pair c0 + 2 lane, +1 (band column c0/2 + lane)
  const int64_t cc = c0 / 2 + lane;
  for (int m = wave; m < kFwdH / 2; m += 4) {
    const int k = 8 + 2 * m, r = r0 + 2 * m;
    if (r >= H) break;
    const int64_t rr = r >> 1;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int q = 8 + 2 * lane + h, c = c0 + 2 * lane + h;
      if (c >= W) continue;
      int v = X[k * P + q];
      if (H > 1) {
        const int dl = X[(r == 0 ? k + 1 : k - 1) * P + q];
        const int dr = X[(r == H - 1 ? k - 1 : k + 1) * P + q];
        v += (dl + dr + 2) >> 2;
      }
      if (h == 0) {
        if (out.ll) out.ll[rr * out.wl + cc] = int16_t(v);
      } else {
        out.hl[rr * out.wh + cc] = int16_t(v);
      }
      if (r + 1 < H) {
        const int16_t d = X[(k + 1) * P + q];
        if (h == 0) out.lh[rr * out.wl + cc] = d;
        else out.hh[rr * out.wh + cc] = d;
      }
    }
  }
}

// Inverse tile loads in quads: local rows 1 .. kInvH+15 (global rows
// r0-7 ..), local columns 0 .. 143.  Local row 1 + t holds an even global
// row when t is odd (mirroring keeps parity), so the two parities run as
// separate passes, each with fixed bands.  Returns whether a quad was
// missed (the caller then reads the tile singly).
template <bool ODD, bool LL32>
__device__ __forceinline__ bool inv_quads_parity(const LvCoef &src, int32_t *Z, int r0, int c0, int H,
                                                 int W) {
  constexpr int P = kLvPitch, kR = kInvH + 15;
  const int tid = int(threadIdx.x), slot = tid % 36, grp = tid / 36;
  bool miss = false;
  // rows of this parity: t = t_first + 2 i
  constexpr int t_first = ODD ? 0 : 1;
  constexpr int n_rows = (kR - t_first + 1) / 2;
  constexpr int kU = 4;
  for (int i0 = 0; i0 < n_rows; i0 += 7 * kU) {
    uint32_t a[kU], b[kU];
    uint2 a32[kU];
    bool ok[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int i = min(i0 + grp + 7 * u, n_rows - 1);
      src.quad<ODD, LL32>(mirror_pos(r0 - 7 + t_first + 2 * i, H), c0 - 8 + 4 * slot, W, &ok[u], &a[u],
                          &a32[u], &b[u]);
      const bool mine = grp < 7 && i0 + grp + 7 * u < n_rows;
      miss |= mine && !ok[u];
      ok[u] = ok[u] && mine;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (!ok[u]) continue;
      const int t = t_first + 2 * (i0 + grp + 7 * u);
      const int b0 = int(b[u] << 16) >> 16, b1 = int(b[u]) >> 16;
      int a0, a1;
      if (!ODD && LL32) {
        a0 = int(a32[u].x);
        a1 = int(a32[u].y);
      } else {
        a0 = int(a[u] << 16) >> 16;
        a1 = int(a[u]) >> 16;
      }
      *reinterpret_cast<int4 *>(Z + (1 + t) * P + 4 * slot) = make_int4(a0, b0, a1, b1);
    }
  }
  return miss;
}

template <bool LL32>
__device__ __forceinline__ bool inv_tile_quads(const LvCoef &src, int32_t *Z, int r0, int c0, int H,
                                               int W) {
  const bool m0 = inv_quads_parity<false, LL32>(src, Z, r0, c0, H, W);
  const bool m1 = inv_quads_parity<true, LL32>(src, Z, r0, c0, H, W);
  return m0 || m1;
}

template <class Dst>
__global__ __launch_bounds__(256) void linv_level_kernel(LvCoef src, Dst dst, const Net net, int H,
                                                         int W, int tiles_x) {
  __shared__ int32_t Z[(kInvH + 16) * kLvPitch];
  __shared__ uint32_t s_net[64];
  constexpr int P = kLvPitch;
  constexpr int kR = kInvH + 15, kC = kLvW + 15;  // local rows / columns 1 .. 15 + tile
  const int tid = int(threadIdx.x);
  const int r0 = int(blockIdx.x / unsigned(tiles_x)) * kInvH;
  const int c0 = int(blockIdx.x % unsigned(tiles_x)) * kLvW;
  stage_net(s_net, net);
  // tile loads as in the forward: local rows 1 .. kInvH+15, local columns
  // 0 .. 143 in quads, or every sample singly where a quad is missing
  bool miss = !src.vec;
  if (src.vec) miss = src.ll32 ? inv_tile_quads<true>(src, Z, r0, c0, H, W)
                               : inv_tile_quads<false>(src, Z, r0, c0, H, W);
  if (__syncthreads_or(miss)) {
    tile_load<kR * kC>(
        [&](int idx) {
          const int t = idx / kC, q = 1 + idx - t * kC;
          return src(mirror_pos(r0 - 7 + t, H), mirror_pos(c0 - 8 + q, W));
        },
        [&](int idx, int v) {
          const int t = idx / kC, q = 1 + idx - t * kC;
          Z[(1 + t) * P + q] = v;
        });
  }
  __syncthreads();
  // column pass, undo the update at the even rows k = 2 .. kInvH+14
  if (H > 1) {
    constexpr int kEv = kInvH / 2 + 7;
    for (int idx = tid; idx < kEv * kC; idx += 256) {
      const int t = idx / kC, k = 2 + 2 * t, q = 1 + idx - t * kC;
      Z[k * P + q] -= (Z[(k - 1) * P + q] + Z[(k + 1) * P + q] + 2) >> 2;
    }
  }
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const MfmaNet mn = mfma_net(s_net, net.b2, net.shift, lane);
  // column pass, undo the predict at the owned odd rows k = 9 .. kInvH+7,
  // every loaded column (1 .. 143): per group of four rows, two batches of 64
  // columns per row, then one batch of the last 15 columns of the four rows
  static_assert(kC == 143 && (kInvH / 2) % 4 == 0, "column batches of the inverse tile");
  constexpr int kGroups = kInvH / 2 / 4, kPerGroup = 9;
  for (int b = wave; b < kGroups * kPerGroup; b += 4) {
    const int g = b / kPerGroup, j = b - g * kPerGroup;  // wave-uniform
    int k, q;
    bool in = true;
    if (j < 8) {
      k = 9 + 2 * (4 * g + (j >> 1));
      q = 1 + 64 * (j & 1) + lane;
    } else {
      const int rsub = lane >> 4, csub = lane & 15;
      in = rsub < 4 && csub < 15;
      k = 9 + 2 * (4 * g + (in ? rsub : 0));
      q = 129 + (in ? csub : 0);
    }
    int32_t *at = Z + k * P + q;
    int e[kCtx];
    load_context(at - 7 * P, P, e);
    const int base = (e[3] + e[4]) >> 1;
    const int corr = correction_mfma(mn, e, base);
    if (in && r0 - 8 + k < H) *at += base + corr;
  }
  __syncthreads();
  // row pass, undo the update at the even columns q = 2 .. kLvW+14 of the
  // owned rows
  if (W > 1) {
    constexpr int kEv = kLvW / 2 + 7;
    for (int idx = tid; idx < kInvH * kEv; idx += 256) {
      const int t = idx / kEv, k = 8 + t, q = 2 + 2 * (idx - t * kEv);
      int32_t *row = Z + k * P;
      row[q] -= (row[q - 1] + row[q + 1] + 2) >> 2;
    }
  }
  __syncthreads();
  // row pass, undo the predict at the owned odd columns (q = 9 + 2 lane) and
  // store the column pair c0 + 2 lane, +1 of each owned row
  for (int t = wave; t < kInvH; t += 4) {
    const int k = 8 + t, r = r0 + t;
    if (r >= H) break;
    const int q = 9 + 2 * lane, c = c0 + 2 * lane;
    int e[kCtx];
    load_context(Z + k * P + q - 7, 1, e);
    const int base = (e[3] + e[4]) >> 1;
    const int corr = correction_mfma(mn, e, base);
    if (c < W) dst(r, c, Z[k * P + q - 1]);
    if (c + 1 < W) dst(r, c + 1, Z[k * P + q] + base + corr);
  }
}

template <class Src>
hipError_t fwd_level(Src src, const LvBands &out, const Net &net, int h, int w, hipStream_t s) {
  const int tx = (w + kLvW - 1) / kLvW, ty = (h + kFwdH - 1) / kFwdH;
  const int64_t grid = int64_t(tx) * ty;
  if (grid <= 0 || grid > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((lfwd_level_kernel<Src>), dim3(unsigned(grid)), dim3(256), 0, s, src, out, net,
                     h, w, tx);
  return hipGetLastError();
}

template <class Dst>
hipError_t inv_level(const LvCoef &src, Dst dst, const Net &net, int h, int w, hipStream_t s) {
  const int tx = (w + kLvW - 1) / kLvW, ty = (h + kInvH - 1) / kInvH;
  const int64_t grid = int64_t(tx) * ty;
  if (grid <= 0 || grid > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((linv_level_kernel<Dst>), dim3(unsigned(grid)), dim3(256), 0, s, src, dst, net,
                     h, w, tx);
  return hipGetLastError();
}

// Per-level description the host hands to the passes.
struct LearnedLevel {
  int h, w;                 // LL_{l-1} dims (the level's input)
  int16_t *hl, *lh, *hh;    // bands of the level in pub (null: discard)
  const int16_t *chl, *clh, *chh;
};

// Forward over all levels as separate 1-D passes, for the training-pair
// capture (the pairs are taken in each pass's own order).  T: int32 H x W
// scratch; B: int32 h1 x w1 scratch for LL_1 .. LL_{L-1}; ll_out: int16 LL_L
// (null: discard).
hipError_t learned_forward(const uint8_t *in, int64_t n, int W, int L, const LearnedLevel *lv,
                           int32_t *T, int32_t *B, int16_t *ll_out, const Net &net,
                           const int64_t *cap_off, uint2 *cap_ctx, int32_t *cap_tgt,
                           hipStream_t s) {
  for (int l = 1; l <= L; ++l) {
    const LearnedLevel &v = lv[l - 1];
    const int h = v.h, w = v.w, wl = (w + 1) / 2;
    SinkRows rows{T, w, wl};
    Capture crow{cap_ctx, cap_tgt, cap_off ? cap_off[2 * (l - 1)] : 0, w / 2};
    const Capture *pr = (cap_off && w > 1) ? &crow : nullptr;
    hipError_t e = (l == 1) ? row_fwd(SrcView{in, n, W}, rows, net, w, h, pr, s)
                            : row_fwd(SrcRows{B, w}, rows, net, w, h, pr, s);
    if (e != hipSuccess) return e;
    Bands bands{l < L ? B : nullptr, l == L ? ll_out : nullptr, v.hl, v.lh, v.hh, wl, w - wl};
    Capture ccol{cap_ctx, cap_tgt, cap_off ? cap_off[2 * (l - 1) + 1] : 0, h / 2};
    const Capture *pc = (cap_off && h > 1) ? &ccol : nullptr;
    e = col_fwd(SrcCols{T, w}, bands, net, h, w, pc, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

inline bool aligned(const void *p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// Protect over all levels with the fused kernels.  LL_1 goes to T16, LL_2
// to B16 (int16, each level's own width), LL_L to ll_out.
hipError_t learned_protect_levels(const uint8_t *in, int64_t n, int W, int L, const LearnedLevel *lv,
                                  int16_t *T16, int16_t *B16, int16_t *ll_out, const Net &net,
                                  hipStream_t s) {
  for (int l = 1; l <= L; ++l) {
    const LearnedLevel &v = lv[l - 1];
    const int wl = (v.w + 1) / 2;
    const LvBands bands{l == L ? ll_out : (l == 1 ? T16 : B16), v.hl, v.lh, v.hh, wl, v.w - wl};
    const int16_t *ll_in = l == 2 ? T16 : B16;
    const hipError_t e =
        l == 1 ? fwd_level(LvSrc8{in, n, W, W % 4 == 0 && n >= 4 && aligned(in, 4)}, bands, net, v.h,
                           v.w, s)
               : fwd_level(LvSrc16{ll_in, v.w, v.w % 4 == 0 && aligned(ll_in, 8)}, bands, net, v.h,
                           v.w, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Restore over all levels, from int16 LL_L (already decrypted) and the bands;
// LL_1 in T32, LL_2 in B32 (int32: fragments no protect produced may leave
// int16).
hipError_t learned_restore_levels(const int16_t *ll_in, const LearnedLevel *lv, int L, int32_t *T32,
                                  int32_t *B32, uint8_t *out, int64_t n, int W, const Net &net,
                                  hipStream_t s) {
  for (int l = L; l >= 1; --l) {
    const LearnedLevel &v = lv[l - 1];
    const int wl = (v.w + 1) / 2;
    LvCoef coef{l == L ? ll_in : nullptr, l == L ? nullptr : (l == 1 ? T32 : B32),
                v.chl, v.clh, v.chh, wl, v.w - wl, 0};
    // (two rows at least: the quads take each row's parity from its
    // unmirrored index, which mirroring keeps only then)
    coef.vec = v.h >= 2 && wl % 2 == 0 && (v.w - wl) % 2 == 0 && aligned(coef.ll16, 4) &&
               aligned(coef.ll32, 8) && aligned(coef.hl, 4) && aligned(coef.lh, 4) &&
               aligned(coef.hh, 4);
    const hipError_t e =
        l == 1 ? inv_level(coef, LvDst8{out, n, W}, net, v.h, v.w, s)
               : inv_level(coef, LvDst32{l == 2 ? T32 : B32, v.w}, net, v.h, v.w, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ------------------------------------------------------------ trainer --

// Exponent k in [-30, 30]: the largest with maxabs * 2^k < 127.5 (30 for 0).
// Products with powers of two are exact, so this matches any exact reference.
__device__ int pow2_exponent(float maxabs) {
  int k = 30;
  while (k > -30 && maxabs * ldexpf(1.0f, k) >= 127.5f) --k;
  return k;
}

__device__ float block_max_abs(float v, float *red) {
  v = fabsf(v);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  const int wave = int(threadIdx.x) >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[wave] = v;
  __syncthreads();
  float m = red[0];
  for (int w = 1; w < int(blockDim.x) / 64; ++w) m = fmaxf(m, red[w]);
  return m;
}

// Integer network from the float parameters: power-of-two scales, round half
// to even, clamps to the parameter ranges.  Run by one 256-thread block.
__device__ void quantize_block(dwtfrag_trainer *st) {
  __shared__ float red[8];
  const int t = int(threadIdx.x);
  const float th = t < kParams ? st->theta[t] : 0.0f;
  const float m1 = block_max_abs(t < 128 ? th : 0.0f, red);
  const float m2 = block_max_abs((t >= 144 && t < 160) ? th : 0.0f, red);
  const int k1 = pow2_exponent(m1);
  const int shift = min(max(k1 + pow2_exponent(m2), 0), 30);
  const int k2 = shift - k1;
  if (t < 128) {
    st->net.w1[t >> 3][t & 7] = int8_t(fminf(fmaxf(rintf(th * ldexpf(1.0f, k1)), -128.f), 127.f));
  } else if (t < 144) {
    st->net.b1[t - 128] = int32_t(fminf(fmaxf(rintf(th * ldexpf(1.0f, k1)), -65536.f), 65536.f));
  } else if (t < 160) {
    st->net.w2[t - 144] = int8_t(fminf(fmaxf(rintf(th * ldexpf(1.0f, k2)), -128.f), 127.f));
  } else if (t == 160) {
    st->net.b2 = int32_t(fminf(fmaxf(rintf(th * ldexpf(1.0f, shift)), -67108864.f), 67108864.f));
    st->net.shift = shift;
    st->k1 = k1;
    st->k2 = k2;
  }
}

struct Theta {
  float v[kParams];
};

__global__ __launch_bounds__(256) void trainer_init_kernel(dwtfrag_trainer *st, const Theta theta0) {
  const int t = int(threadIdx.x);
  if (t < kParams) {
    st->theta[t] = theta0.v[t];
    st->m[t] = 0.0f;
    st->v[t] = 0.0f;
    st->grad[t] = 0.0f;
  }
  if (t == 0) {
    st->loss = 0.0f;
    st->step = 0;
  }
  __syncthreads();
  quantize_block(st);
}

__device__ __forceinline__ int64_t wave_sum(int64_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Stage 1: per-block integer sums over the pairs, for the current network:
//   S_w1[k][j] = sum sg [pre_k > 0] c_j,   S_b1[k] = sum sg [pre_k > 0],
//   S_w2[k] = sum sg h_k,   S_b2 = sum sg,   S_loss = sum |acc - t 2^shift|,
// with acc = W2 . h + b2 (the network output times 2^shift) and
// sg = sign(acc - t 2^shift).
__global__ __launch_bounds__(256) void grad_partial_kernel(const uint2 *__restrict__ ctx,
                                                           const int32_t *__restrict__ tgt,
                                                           int64_t count, int64_t stride,
                                                           const dwtfrag_trainer *__restrict__ st,
                                                           int64_t *__restrict__ partial) {
  __shared__ int64_t red[4][kSums];
  Net net;
  {
    const dwtfrag_predictor &q = st->net;
    net = Net{};
    for (int k = 0; k < kHidden; ++k) {
      net.w1[k][0] = uint32_t(uint8_t(q.w1[k][0])) | (uint32_t(uint8_t(q.w1[k][1])) << 8) |
                     (uint32_t(uint8_t(q.w1[k][2])) << 16) | (uint32_t(uint8_t(q.w1[k][3])) << 24);
      net.w1[k][1] = uint32_t(uint8_t(q.w1[k][4])) | (uint32_t(uint8_t(q.w1[k][5])) << 8) |
                     (uint32_t(uint8_t(q.w1[k][6])) << 16) | (uint32_t(uint8_t(q.w1[k][7])) << 24);
      net.b1[k] = q.b1[k];
      net.w2[k] = q.w2[k];
    }
    net.b2 = q.b2;
    net.shift = q.shift;
  }
  int32_t s_w1[kHidden][kCtx], s_b1[kHidden];
  int64_t s_w2[kHidden];
  int64_t s_b2 = 0, s_loss = 0;
#pragma unroll
  for (int k = 0; k < kHidden; ++k) {
    s_b1[k] = 0;
    s_w2[k] = 0;
#pragma unroll
    for (int j = 0; j < kCtx; ++j) s_w1[k][j] = 0;
  }
  const int64_t grid_threads = int64_t(gridDim.x) * blockDim.x;
  for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < count; p += grid_threads) {
    const uint2 cw = ctx[p * stride];
    const int64_t t = tgt[p * stride];
    int c[kCtx];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      c[j] = int(int8_t(uint8_t(cw.x >> (8 * j))));
      c[4 + j] = int(int8_t(uint8_t(cw.y >> (8 * j))));
    }
    int h[kHidden];
    int acc = net.b2;
#pragma unroll
    for (int k = 0; k < kHidden; ++k) {
      h[k] = hidden_pre(net.w1[k], net.b1[k], cw.x, cw.y);
      acc += clamp_i(h[k], 0, 0x7fffff) * ((net.w2[k] << 24) >> 24);
    }
    const int64_t r = int64_t(acc) - (t << net.shift);
    const int sg = (r > 0) - (r < 0);
    s_loss += r < 0 ? -r : r;
    s_b2 += sg;
#pragma unroll
    for (int k = 0; k < kHidden; ++k) {
      const int hk = max(h[k], 0);
      s_w2[k] += sg * hk;
      const int mk = h[k] > 0 ? sg : 0;
      s_b1[k] += mk;
#pragma unroll
      for (int j = 0; j < kCtx; ++j) s_w1[k][j] += mk * c[j];
    }
  }
  const int wave = int(threadIdx.x) >> 6, lane = int(threadIdx.x) & 63;
#pragma unroll
  for (int k = 0; k < kHidden; ++k) {
#pragma unroll
    for (int j = 0; j < kCtx; ++j) {
      const int64_t v = wave_sum(int64_t(s_w1[k][j]));
      if (lane == 0) red[wave][k * kCtx + j] = v;
    }
    const int64_t vb = wave_sum(int64_t(s_b1[k]));
    const int64_t vw = wave_sum(s_w2[k]);
    if (lane == 0) {
      red[wave][128 + k] = vb;
      red[wave][144 + k] = vw;
    }
  }
  {
    const int64_t vb = wave_sum(s_b2), vl = wave_sum(s_loss);
    if (lane == 0) {
      red[wave][160] = vb;
      red[wave][161] = vl;
    }
  }
  __syncthreads();
  for (int i = int(threadIdx.x); i < kSums; i += blockDim.x)
    partial[int64_t(blockIdx.x) * kSums + i] = red[0][i] + red[1][i] + red[2][i] + red[3][i];
}

// Stage 2 (one block): total sums -> loss and gradient at the fake-quantised
// point, Adam step on the float parameters, re-quantisation.
__global__ __launch_bounds__(256) void adam_kernel(dwtfrag_trainer *st, const int64_t *partial,
                                                   int nblocks, int64_t count, float lr) {
  __shared__ int64_t S[kSums];
  const int t = int(threadIdx.x);
  if (t < kSums) {
    int64_t v = 0;
    for (int b = 0; b < nblocks; ++b) v += partial[int64_t(b) * kSums + t];
    S[t] = v;
  }
  __syncthreads();
  const double inv_n = 1.0 / double(count > 0 ? count : 1);
  const int k1 = st->k1, k2 = st->k2, shift = st->net.shift;
  double g = 0.0;
  if (t < 128) {
    g = double(st->net.w2[t >> 3]) * double(S[t]) * ldexp(1.0, -k2) * inv_n;
  } else if (t < 144) {
    g = double(st->net.w2[t - 128]) * double(S[t]) * ldexp(1.0, -k2) * inv_n;
  } else if (t < 160) {
    g = double(S[t]) * ldexp(1.0, -k1) * inv_n;
  } else if (t == 160) {
    g = double(S[t]) * inv_n;
  }
  __syncthreads();  // every thread has read the old network
  const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
  const int step = st->step + 1;
  if (t < kParams) {
    const float gf = float(g);
    st->grad[t] = gf;
    const float m = beta1 * st->m[t] + (1.0f - beta1) * gf;
    const float v = beta2 * st->v[t] + (1.0f - beta2) * gf * gf;
    st->m[t] = m;
    st->v[t] = v;
    const float mh = m / (1.0f - powf(beta1, float(step)));
    const float vh = v / (1.0f - powf(beta2, float(step)));
    st->theta[t] -= lr * mh / (sqrtf(vh) + eps);
  }
  if (t == 0) {
    st->loss = float(double(S[161]) * ldexp(1.0, -shift) * inv_n);
    st->step = step;
  }
  __syncthreads();
  quantize_block(st);
}

}  // namespace dwtfrag

// ---------------------------------------------------------- C ABI --

using namespace dwtfrag;

namespace {

// Same row and column limit as the plain path (int32 indexing with margins).
constexpr uint64_t kMaxDim = 0x7FFF0000ull;

uint64_t a256(uint64_t v) { return (v + 255) & ~uint64_t(255); }

struct LGeom {
  uint64_t n;
  int W, H, L;
  int h[4], w[4];
  uint64_t priv_bytes, pub_bytes;
  uint64_t off_T, off_B, off_LL, ws_bytes;
  uint64_t pairs;
  int64_t pair_off[6];
  int64_t band_off[4][3];  // element offsets in pub of HL, LH, HH of level l
};

int lgeom(uint64_t n, uint32_t width, uint32_t levels, LGeom *g) {
  if (n == 0 || width == 0 || levels == 0 || levels > 3) return DWTFRAG_EINVAL;
  if (width > kMaxDim) return DWTFRAG_ERANGE;
  const uint64_t H = (n + width - 1) / width;
  if (H > kMaxDim || H * uint64_t(width) > (uint64_t(1) << 40)) return DWTFRAG_ERANGE;
  g->n = n;
  g->W = int(width);
  g->H = int(H);
  g->L = int(levels);
  g->h[0] = g->H;
  g->w[0] = g->W;
  for (int l = 1; l <= g->L; ++l) {
    g->h[l] = (g->h[l - 1] + 1) / 2;
    g->w[l] = (g->w[l - 1] + 1) / 2;
  }
  const uint64_t ll = uint64_t(g->h[g->L]) * g->w[g->L];
  g->priv_bytes = 2 * ll;
  g->pub_bytes = 2 * (H * width - ll);
  g->off_T = 0;
  g->off_B = a256(4 * H * width);
  g->off_LL = g->off_B + a256(4 * uint64_t(g->h[1]) * g->w[1]);
  g->ws_bytes = g->off_LL + a256(2 * ll);
  uint64_t pairs = 0;
  for (int l = 1; l <= g->L; ++l) {
    const uint64_t h = g->h[l - 1], w = g->w[l - 1];
    g->pair_off[2 * (l - 1)] = int64_t(pairs);
    if (w > 1) pairs += h * (w / 2);
    g->pair_off[2 * (l - 1) + 1] = int64_t(pairs);
    if (h > 1) pairs += w * (h / 2);
  }
  g->pairs = pairs;
  uint64_t off = 0;
  for (int l = g->L; l >= 1; --l) {
    const uint64_t h = g->h[l - 1], w = g->w[l - 1], hl = g->h[l], wl = g->w[l];
    g->band_off[l][0] = int64_t(off);
    g->band_off[l][1] = int64_t(off + hl * (w - wl));
    g->band_off[l][2] = int64_t(off + hl * (w - wl) + (h - hl) * wl);
    off += h * w - hl * wl;
  }
  return DWTFRAG_OK;
}

bool net_ok(const dwtfrag_predictor *p) {
  if (!p || p->shift < 0 || p->shift > 30) return false;
  if (p->b2 < -(1 << 26) || p->b2 > (1 << 26)) return false;
  for (int k = 0; k < kHidden; ++k)
    if (p->b1[k] < -(1 << 16) || p->b1[k] > (1 << 16)) return false;
  return true;
}

bool al16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

void fill_levels(const LGeom &g, int16_t *pub, const int16_t *cpub, LearnedLevel *lv) {
  for (int l = 1; l <= g.L; ++l) {
    LearnedLevel &v = lv[l - 1];
    v.h = g.h[l - 1];
    v.w = g.w[l - 1];
    v.hl = pub ? pub + g.band_off[l][0] : nullptr;
    v.lh = pub ? pub + g.band_off[l][1] : nullptr;
    v.hh = pub ? pub + g.band_off[l][2] : nullptr;
    v.chl = cpub ? cpub + g.band_off[l][0] : nullptr;
    v.clh = cpub ? cpub + g.band_off[l][1] : nullptr;
    v.chh = cpub ? cpub + g.band_off[l][2] : nullptr;
  }
}

}  // namespace

namespace dwtfrag {
hipError_t launch_ctr(const uint8_t *in, uint8_t *out, uint64_t nbytes, const AesKey &key,
                      uint64_t first_block, hipStream_t s);
}

extern "C" {

int dwtfrag_learned_geometry(uint64_t n, uint32_t width, uint32_t levels,
                             uint64_t *workspace_bytes, uint64_t *pairs) {
  LGeom g;
  const int rc = lgeom(n, width, levels, &g);
  if (rc != DWTFRAG_OK) return rc;
  if (workspace_bytes) *workspace_bytes = g.ws_bytes;
  if (pairs) *pairs = g.pairs;
  return DWTFRAG_OK;
}

int dwtfrag_protect_learned(const uint8_t *in, uint64_t n, uint32_t width, uint32_t levels,
                            const uint8_t key[16], const uint8_t nonce[16],
                            const dwtfrag_predictor *predictor, uint8_t *priv, int16_t *pub,
                            void *workspace, uint64_t workspace_bytes, void *stream) {
  if (!in || !key || !nonce || !priv || !workspace || !net_ok(predictor)) return DWTFRAG_EINVAL;
  LGeom g;
  const int rc = lgeom(n, width, levels, &g);
  if (rc != DWTFRAG_OK) return rc;
  if (!pub && g.pub_bytes) return DWTFRAG_EINVAL;
  if (workspace_bytes < g.ws_bytes) return DWTFRAG_EWORKSPACE;
  if (!al16(in) || !al16(priv) || !al16(pub) || !al16(workspace)) return DWTFRAG_EINVAL;
  AesKey k;
  expand_key(key, nonce, &k);
  const Net net = pack_net(*predictor);
  LearnedLevel lv[3];
  fill_levels(g, pub, nullptr, lv);
  char *ws = static_cast<char *>(workspace);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (learned_protect_levels(in, int64_t(n), g.W, g.L, lv, reinterpret_cast<int16_t *>(ws + g.off_T),
                             reinterpret_cast<int16_t *>(ws + g.off_B),
                             reinterpret_cast<int16_t *>(priv), net, st) != hipSuccess)
    return DWTFRAG_EDEVICE;
  if (launch_ctr(priv, priv, g.priv_bytes, k, 0, st) != hipSuccess) return DWTFRAG_EDEVICE;
  return DWTFRAG_OK;
}

int dwtfrag_restore_learned(const uint8_t *priv, const int16_t *pub, uint64_t n, uint32_t width,
                            uint32_t levels, const uint8_t key[16], const uint8_t nonce[16],
                            const dwtfrag_predictor *predictor, uint8_t *out, void *workspace,
                            uint64_t workspace_bytes, void *stream) {
  if (!priv || !key || !nonce || !out || !workspace || !net_ok(predictor)) return DWTFRAG_EINVAL;
  LGeom g;
  const int rc = lgeom(n, width, levels, &g);
  if (rc != DWTFRAG_OK) return rc;
  if (!pub && g.pub_bytes) return DWTFRAG_EINVAL;
  if (workspace_bytes < g.ws_bytes) return DWTFRAG_EWORKSPACE;
  if (!al16(out) || !al16(priv) || !al16(pub) || !al16(workspace)) return DWTFRAG_EINVAL;
  AesKey k;
  expand_key(key, nonce, &k);
  const Net net = pack_net(*predictor);
  LearnedLevel lv[3];
  fill_levels(g, nullptr, pub, lv);
  char *ws = static_cast<char *>(workspace);
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint8_t *ll = reinterpret_cast<uint8_t *>(ws + g.off_LL);
  if (launch_ctr(priv, ll, g.priv_bytes, k, 0, st) != hipSuccess) return DWTFRAG_EDEVICE;
  if (learned_restore_levels(reinterpret_cast<const int16_t *>(ll), lv, g.L,
                             reinterpret_cast<int32_t *>(ws + g.off_T),
                             reinterpret_cast<int32_t *>(ws + g.off_B), out, int64_t(n), g.W, net,
                             st) != hipSuccess)
    return DWTFRAG_EDEVICE;
  return DWTFRAG_OK;
}

int dwtfrag_learned_pairs(const uint8_t *in, uint64_t n, uint32_t width, uint32_t levels,
                          int8_t *ctx, int32_t *target, void *workspace, uint64_t workspace_bytes,
                          void *stream) {
  if (!in || !workspace) return DWTFRAG_EINVAL;
  LGeom g;
  const int rc = lgeom(n, width, levels, &g);
  if (rc != DWTFRAG_OK) return rc;
  if (g.pairs && (!ctx || !target)) return DWTFRAG_EINVAL;
  if (workspace_bytes < g.ws_bytes) return DWTFRAG_EWORKSPACE;
  if ((reinterpret_cast<uintptr_t>(ctx) & 7) || (reinterpret_cast<uintptr_t>(target) & 3) ||
      !al16(in) || !al16(workspace))
    return DWTFRAG_EINVAL;
  const Net zero{};
  LearnedLevel lv[3];
  fill_levels(g, nullptr, nullptr, lv);
  char *ws = static_cast<char *>(workspace);
  if (learned_forward(in, int64_t(n), g.W, g.L, lv, reinterpret_cast<int32_t *>(ws + g.off_T),
                      reinterpret_cast<int32_t *>(ws + g.off_B), nullptr, zero, g.pair_off,
                      reinterpret_cast<uint2 *>(ctx), target,
                      static_cast<hipStream_t>(stream)) != hipSuccess)
    return DWTFRAG_EDEVICE;
  return DWTFRAG_OK;
}

uint64_t dwtfrag_trainer_workspace_bytes(void) { return uint64_t(kGradBlocks) * kSums * 8; }

int dwtfrag_trainer_init(dwtfrag_trainer *state, const float theta0[161], void *stream) {
  if (!state || !theta0 || (reinterpret_cast<uintptr_t>(state) & 7)) return DWTFRAG_EINVAL;
  Theta th;
  for (int i = 0; i < kParams; ++i) th.v[i] = theta0[i];
  hipLaunchKernelGGL(trainer_init_kernel, dim3(1), dim3(256), 0, static_cast<hipStream_t>(stream),
                     state, th);
  return hipGetLastError() == hipSuccess ? DWTFRAG_OK : DWTFRAG_EDEVICE;
}

int dwtfrag_trainer_step(dwtfrag_trainer *state, const int8_t *ctx, const int32_t *target,
                         uint64_t count, uint64_t stride, float lr, void *workspace,
                         uint64_t workspace_bytes, void *stream) {
  if (!state || !ctx || !target || count == 0 || stride == 0 || !workspace) return DWTFRAG_EINVAL;
  if ((reinterpret_cast<uintptr_t>(state) & 7) || (reinterpret_cast<uintptr_t>(ctx) & 7) ||
      (reinterpret_cast<uintptr_t>(target) & 3) || (reinterpret_cast<uintptr_t>(workspace) & 7))
    return DWTFRAG_EINVAL;
  if (workspace_bytes < dwtfrag_trainer_workspace_bytes()) return DWTFRAG_EWORKSPACE;
  if (count > (uint64_t(1) << 40) || stride > (uint64_t(1) << 40) ||
      (count - 1) > ((uint64_t(1) << 62) / stride))
    return DWTFRAG_ERANGE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const uint64_t want = (count + 255) / 256;
  const int blocks = int(want < uint64_t(kGradBlocks) ? want : uint64_t(kGradBlocks));
  int64_t *partial = static_cast<int64_t *>(workspace);
  hipLaunchKernelGGL(grad_partial_kernel, dim3(blocks), dim3(256), 0, st,
                     reinterpret_cast<const uint2 *>(ctx), target, int64_t(count), int64_t(stride),
                     state, partial);
  if (hipGetLastError() != hipSuccess) return DWTFRAG_EDEVICE;
  hipLaunchKernelGGL(adam_kernel, dim3(1), dim3(256), 0, st, state, partial, blocks,
                     int64_t(count), lr);
  return hipGetLastError() == hipSuccess ? DWTFRAG_OK : DWTFRAG_EDEVICE;
}

}  // extern "C"
