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
// plain predict, so this path is ALU-bound and each 1-D pass runs as its own
// kernel over int32 intermediates in HBM.  A block
// takes SEG positions of LINES independent lines (rows: 1 line of 2048
// positions; columns: 64 lines of 64 positions), loads them with an 8-sample
// halo on each side, mirrored at the signal edges, into LDS as separate even
// and odd planes (line index fastest, so lanes hit consecutive banks), then
// predicts the odd samples and updates the even ones.
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

__device__ __forceinline__ int correction_mfma(const MfmaNet &m, const int (&e)[kCtx], int base,
                                               int lane) {
  int c[kCtx];
#pragma unroll
  for (int j = 0; j < kCtx; ++j) c[j] = clamp_i(e[j] - base, -128, 127);
  const long b = long(pack4(c[0], c[1], c[2], c[3])) | (long(pack4(c[4], c[5], c[6], c[7])) << 32);
  // p[g]: this lane's quarter of the output sum of group g's sample l % 16
  // (its four hidden units 4q..4q+3, q = l / 16)
  int p[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const v4i d = __builtin_amdgcn_mfma_i32_16x16x32_i8(m.a[g], b, m.bias, 0, 0, 0);
    int sum = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) sum += clamp_i(d[r], 0, 0x7fffff) * m.w2[r];
    p[g] = sum;
  }
  // Lane l needs group q's total: the sum of p[q] over lanes s, s+16, s+32,
  // s+48 (s = l % 16).  Two exchange rounds: across lane halves (q ^ 2) each
  // lane keeps the pair of groups {2(q/2), 2(q/2)+1} and sends the other
  // pair; then across q ^ 1 it keeps group q and sends the other.
  const int q = lane >> 4;
  const bool hi = (q & 2) != 0;
  const int k0 = (hi ? p[2] : p[0]) + __shfl_xor(hi ? p[0] : p[2], 32);
  const int k1 = (hi ? p[3] : p[1]) + __shfl_xor(hi ? p[1] : p[3], 32);
  const bool odd = (q & 1) != 0;
  const int mine = (odd ? k1 : k0) + __shfl_xor(odd ? k0 : k1, 16);
  return clamp_i((mine + m.b2) >> m.shift, -255, 255);
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

// Inverse sources: lows and highs of a line.
struct InvRows {
  const int32_t *p;
  int pitch, nlow;
  __device__ int low(int line, int k) const { return p[int64_t(line) * pitch + k]; }
  __device__ int high(int line, int k) const { return p[int64_t(line) * pitch + nlow + k]; }
};
struct InvBands {
  const int32_t *ll32;
  const int16_t *ll16, *hl, *lh, *hh;
  int wl, wh;
  __device__ int low(int c, int r) const {
    if (c < wl) return ll32 ? ll32[int64_t(r) * wl + c] : int(ll16[int64_t(r) * wl + c]);
    return hl[int64_t(r) * wh + (c - wl)];
  }
  __device__ int high(int c, int r) const {
    if (c < wl) return lh[int64_t(r) * wl + c];
    return hh[int64_t(r) * wh + (c - wl)];
  }
};
// Inverse sinks: reconstructed samples.
struct OutCols {
  int32_t *p;
  int pitch;
  __device__ void operator()(int line, int pos, int v) const { p[int64_t(pos) * pitch + line] = v; }
};
struct OutRows {
  int32_t *p;
  int pitch;
  __device__ void operator()(int line, int pos, int v) const { p[int64_t(line) * pitch + pos] = v; }
};
struct OutView {  // level-0 bytes, first n only, modulo 256
  uint8_t *p;
  int64_t n;
  int pitch;
  __device__ void operator()(int line, int pos, int v) const {
    const int64_t o = int64_t(line) * pitch + pos;
    if (o < n) p[o] = uint8_t(v);
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
    const int corr = correction_mfma(mn, e, base, lane);
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

template <int LINES, int SEG, class Src, class Out>
__global__ __launch_bounds__(256) void linv_kernel(Src src, Out out, const Net net, int N,
                                                   int n_lines, int n_seg) {
  using T = Tile<LINES, SEG>;
  __shared__ int32_t sE[T::NE * LINES];
  __shared__ uint32_t s_net[64];
  int s0, l0;
  tile_coords(n_seg, SEG, LINES, &s0, &l0);
  const int tid = int(threadIdx.x);
  stage_net(s_net, net);

  // undo the update at the (mirrored) even positions s0-8 .. s0+SEG+6
  for (int idx = tid; idx < T::NE * LINES; idx += T::kThreads) {
    const int li = idx % LINES, e = idx / LINES, line = l0 + li;
    int v = 0;
    if (line < n_lines) {
      const int p = mirror_pos(s0 - kHalo + 2 * e, N);
      v = src.low(line, p >> 1);
      if (N > 1) {
        const int pl = p == 0 ? 1 : p - 1;
        const int pr = p == N - 1 ? N - 2 : p + 1;
        v -= (src.high(line, pl >> 1) + src.high(line, pr >> 1) + 2) >> 2;
      }
    }
    sE[e * LINES + li] = v;
  }
  __syncthreads();

  // owned positions: evens as rebuilt, odds by undoing the predict (the
  // network on the matrix cores: uniform trip count per wavefront)
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const MfmaNet mn = mfma_net(s_net, net.b2, net.shift, lane);
  for (int base0 = wave * 64; base0 < (SEG / 2) * LINES; base0 += T::kThreads) {
    const int idx = base0 + lane;
    const bool in = idx < (SEG / 2) * LINES;
    const int li = in ? idx % LINES : 0, e2 = in ? idx / LINES : 0, line = l0 + li;
    const int i = s0 + 2 * e2;
    const bool valid = in && i < N && line < n_lines;
    if (valid) out(line, i, sE[(e2 + 4) * LINES + li]);
    const int q = e2 + 1;
    int e[kCtx];
#pragma unroll
    for (int j = 0; j < kCtx; ++j) e[j] = sE[(q + j) * LINES + li];
    const int base = (e[3] + e[4]) >> 1;
    const int corr = correction_mfma(mn, e, base, lane);
    if (valid && i + 1 < N) out(line, i + 1, src.high(line, i >> 1) + base + corr);
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

template <int LINES, int SEG, class Src, class Out>
hipError_t inv_pass(Src src, Out out, const Net &net, int N, int lines, hipStream_t s) {
  int n_seg;
  unsigned grid;
  if (!grid_for<LINES, SEG>(N, lines, &n_seg, &grid)) return hipErrorInvalidValue;
  hipLaunchKernelGGL((linv_kernel<LINES, SEG, Src, Out>), dim3(grid), dim3(256), 0, s, src, out,
                     net, N, lines, n_seg);
  return hipGetLastError();
}

// Per-level description the host hands to the passes.
struct LearnedLevel {
  int h, w;                 // LL_{l-1} dims (the level's input)
  int16_t *hl, *lh, *hh;    // bands of the level in pub (null: discard)
  const int16_t *chl, *clh, *chh;
};

// Forward over all levels.  T: int32 H x W scratch; B: int32 h1 x w1
// scratch for LL_1 .. LL_{L-1}; ll_out: int16 LL_L (null: discard).
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

// Inverse over all levels, from int16 LL_L (already decrypted) and the bands.
hipError_t learned_inverse(const int16_t *ll_in, const LearnedLevel *lv, int L, int32_t *T,
                           int32_t *B, uint8_t *out, int64_t n, int W, const Net &net,
                           hipStream_t s) {
  for (int l = L; l >= 1; --l) {
    const LearnedLevel &v = lv[l - 1];
    const int h = v.h, w = v.w, wl = (w + 1) / 2;
    InvBands bands{l < L ? B : nullptr, l == L ? ll_in : nullptr, v.chl, v.clh, v.chh, wl, w - wl};
    hipError_t e = inv_pass<kColLines, kColSeg>(bands, OutCols{T, w}, net, h, w, s);
    if (e != hipSuccess) return e;
    InvRows rows{T, w, wl};
    e = (l == 1) ? inv_pass<1, kRowSeg>(rows, OutView{out, n, W}, net, w, h, s)
                 : inv_pass<1, kRowSeg>(rows, OutRows{B, w}, net, w, h, s);
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
  if (learned_forward(in, int64_t(n), g.W, g.L, lv, reinterpret_cast<int32_t *>(ws + g.off_T),
                      reinterpret_cast<int32_t *>(ws + g.off_B), reinterpret_cast<int16_t *>(priv),
                      net, nullptr, nullptr, nullptr, st) != hipSuccess)
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
  if (learned_inverse(reinterpret_cast<const int16_t *>(ll), lv, g.L,
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
