// The thesis's per-8x8-block protection (Ch. 5 section 5.2.1 "Designs"):
// every 8x8 block of the byte matrix gets two levels of the 5/3 lifting; its
// level-2 LL (4 coefficients) is the private fragment, encrypted with
// AES-128; a SHA-256 digest of the private part and the key is XORed over
// the rest of level 2 (first public fragment), and a SHA-512 digest of that
// protected first public fragment and the key over the level-1 details
// (second public fragment).  Coefficients are stored in 10 bits, the four
// level-2 HH values in 11 (section 5.2.2.2: 40 / 124 / 480 bits per block).
//
// One thread per block, 256 blocks per workgroup.  A thread lifts its block
// in registers, packs the three records, runs one SHA-256 and one SHA-512
// compression and writes the records into the workgroup's LDS copy of its
// three fragment ranges; the ranges are then written with 16-byte stores and
// the private range is encrypted in LDS on the way (its keystream blocks
// never straddle two workgroups: 256 records are 80 AES blocks).  Restore
// runs the same steps backwards.  Hash messages (one compression each; the
// paper leaves their exact content open):
//   m1 = private record (5 bytes, clear) | key | nonce | block index (8 bytes,
//        big-endian)
//   m2 = protected first public record (16 bytes, 4 zero bits at the top) |
//        key | nonce | block index
// The first 124 / 480 digest bits (bit i = bit i % 8 of digest byte i / 8)
// are XORed over the records, which are bit streams in the same order.
#include "dwtfrag.h"
#include "se8.h"

namespace dwtfrag {

namespace {

constexpr int kSeThreads = 256;                 // blocks per workgroup
constexpr int kPrivRange = kSeThreads * 5;      // 1280 bytes = 80 AES blocks
constexpr int kPub1Range = kSeThreads * 31 / 2; // 3968 bytes
constexpr int kPub2Range = kSeThreads * 60;     // 15360 bytes

// ------------------------------------------------------------- lifting ----
// One forward 5/3 lifting pass over N (even) samples v[0], v[S], ...:
// predict the odd samples, update the even ones, whole-sample mirror, then
// reorder to [evens | odds].
template <int N, int S>
__device__ __forceinline__ void lift_fwd(int *v) {
  int t[N];
#pragma unroll
  for (int i = 0; i < N; ++i) t[i] = v[i * S];
#pragma unroll
  for (int i = 1; i < N; i += 2) {
    const int right = (i + 1 < N) ? t[i + 1] : t[N - 2];
    t[i] -= (t[i - 1] + right) >> 1;
  }
#pragma unroll
  for (int i = 0; i < N; i += 2) {
    const int left = (i == 0) ? t[1] : t[i - 1];
    t[i] += (left + t[i + 1] + 2) >> 2;
  }
#pragma unroll
  for (int i = 0; i < N / 2; ++i) {
    v[i * S] = t[2 * i];
    v[(N / 2 + i) * S] = t[2 * i + 1];
  }
}

// Inverse of lift_fwd: undo the update on the evens, then the predict on the
// odds.
template <int N, int S>
__device__ __forceinline__ void lift_inv(int *v) {
  int t[N];
#pragma unroll
  for (int i = 0; i < N / 2; ++i) {
    t[2 * i] = v[i * S];
    t[2 * i + 1] = v[(N / 2 + i) * S];
  }
#pragma unroll
  for (int i = 0; i < N; i += 2) {
    const int left = (i == 0) ? t[1] : t[i - 1];
    t[i] -= (left + t[i + 1] + 2) >> 2;
  }
#pragma unroll
  for (int i = 1; i < N; i += 2) {
    const int right = (i + 1 < N) ? t[i + 1] : t[N - 2];
    t[i] += (t[i - 1] + right) >> 1;
  }
#pragma unroll
  for (int i = 0; i < N; ++i) v[i * S] = t[i];
}

// Two levels on an 8x8 block (m[8 r + c]): rows then columns, then the same
// on the 4x4 LL.
__device__ __forceinline__ void block_fwd(int *m) {
#pragma unroll
  for (int r = 0; r < 8; ++r) lift_fwd<8, 1>(m + 8 * r);
#pragma unroll
  for (int c = 0; c < 8; ++c) lift_fwd<8, 8>(m + c);
#pragma unroll
  for (int r = 0; r < 4; ++r) lift_fwd<4, 1>(m + 8 * r);
#pragma unroll
  for (int c = 0; c < 4; ++c) lift_fwd<4, 8>(m + c);
}

__device__ __forceinline__ void block_inv(int *m) {
#pragma unroll
  for (int c = 0; c < 4; ++c) lift_inv<4, 8>(m + c);
#pragma unroll
  for (int r = 0; r < 4; ++r) lift_inv<4, 1>(m + 8 * r);
#pragma unroll
  for (int c = 0; c < 8; ++c) lift_inv<8, 8>(m + c);
#pragma unroll
  for (int r = 0; r < 8; ++r) lift_inv<8, 1>(m + 8 * r);
}

// ------------------------------------------------------------- records ----
// Band cells of the records, in band row-major order: (row, col) in the
// block's two-level layout.  LL2 [0:2,0:2]; HL2 [0:2,2:4]; LH2 [2:4,0:2];
// HH2 [2:4,2:4]; HL1 [0:4,4:8]; LH1 [4:8,0:4]; HH1 [4:8,4:8].
__device__ constexpr int cell_priv(int k) { return 8 * (k >> 1) + (k & 1); }
__device__ constexpr int cell_pub1(int k) {
  return k < 4 ? 8 * (k >> 1) + 2 + (k & 1)
       : k < 8 ? 8 * (2 + ((k - 4) >> 1)) + ((k - 4) & 1)
               : 8 * (2 + ((k - 8) >> 1)) + 2 + ((k - 8) & 1);
}
__device__ constexpr int pub1_pos(int k) { return k < 8 ? 10 * k : 80 + 11 * (k - 8); }
__device__ constexpr int pub1_bits(int k) { return k < 8 ? 10 : 11; }
__device__ constexpr int cell_pub2(int k) {
  return k < 16 ? 8 * (k >> 2) + 4 + (k & 3)
       : k < 32 ? 8 * (4 + ((k - 16) >> 2)) + ((k - 16) & 3)
                : 8 * (4 + ((k - 32) >> 2)) + 4 + ((k - 32) & 3);
}

// value's low `bits` bits at bit `pos` of a little-endian word stream
template <int kWords>
__device__ __forceinline__ void put_bits(uint32_t (&w)[kWords], int pos, int bits, int value) {
  const uint32_t v = uint32_t(value) & ((1u << bits) - 1u);
  const int q = pos >> 5, s = pos & 31;
  w[q] |= v << s;
  if (s + bits > 32) w[q + 1] |= v >> (32 - s);
}

// sign-extended `bits`-bit field at bit `pos`
template <int kWords>
__device__ __forceinline__ int get_bits(const uint32_t (&w)[kWords], int pos, int bits) {
  const int q = pos >> 5, s = pos & 31;
  uint32_t v = w[q] >> s;
  if (s + bits > 32) v |= w[q + 1] << (32 - s);
  return int(v << (32 - bits)) >> (32 - bits);
}

// ---------------------------------------------------------------- SHA-2 ----
// FIPS 180-4 compressions of one padded message block.  Every logical
// function maps onto single gfx950 instructions: a 32-bit rotate is one
// funnel shift (v_alignbit), a 64-bit rotate or shift two (one per half), a
// three-way XOR, choose or majority one three-input bit operation per 32
// bits (v_bitop3 truth tables 0x96, 0xCA, 0xE8), and 64-bit additions stay
// 64-bit operations.
__device__ __forceinline__ uint32_t rotr32(uint32_t x, int n) {
  return __builtin_amdgcn_alignbit(x, x, n);
}
__device__ __forceinline__ uint32_t ch32(uint32_t e, uint32_t f, uint32_t g) {
  return __builtin_amdgcn_bitop3_b32(e, f, g, 0xCA);  // e ? f : g
}
__device__ __forceinline__ uint32_t maj32(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8);  // majority
}

__device__ __forceinline__ uint32_t lo32(uint64_t x) { return uint32_t(x); }
__device__ __forceinline__ uint32_t hi32(uint64_t x) { return uint32_t(x >> 32); }
__device__ __forceinline__ uint64_t join(uint32_t hi, uint32_t lo) { return (uint64_t(hi) << 32) | lo; }

// rotate right by a constant 0 < N < 64: bits of the two halves funnel
// through each other
template <int N> __device__ __forceinline__ uint64_t rotr64(uint64_t x) {
  const uint32_t lo = N >= 32 ? hi32(x) : lo32(x), hi = N >= 32 ? lo32(x) : hi32(x);
  constexpr int n = N % 32;
  if constexpr (n == 0) return join(hi, lo);
  else return join(__builtin_amdgcn_alignbit(lo, hi, n), __builtin_amdgcn_alignbit(hi, lo, n));
}
// logical shift right by a constant 0 < N < 32
template <int N> __device__ __forceinline__ uint64_t shr64(uint64_t x) {
  return join(hi32(x) >> N, __builtin_amdgcn_alignbit(hi32(x), lo32(x), N));
}
__device__ __forceinline__ uint64_t xor3_64(uint64_t a, uint64_t b, uint64_t c) {
  return join(xor3(hi32(a), hi32(b), hi32(c)), xor3(lo32(a), lo32(b), lo32(c)));
}
__device__ __forceinline__ uint64_t ch64(uint64_t e, uint64_t f, uint64_t g) {
  return join(ch32(hi32(e), hi32(f), hi32(g)), ch32(lo32(e), lo32(f), lo32(g)));
}
__device__ __forceinline__ uint64_t maj64(uint64_t a, uint64_t b, uint64_t c) {
  return join(maj32(hi32(a), hi32(b), hi32(c)), maj32(lo32(a), lo32(b), lo32(c)));
}

__device__ __forceinline__ void sha256_block(const Sha2Tables &T, uint32_t (&W)[16], uint32_t (&H)[8]) {
  uint32_t a = T.h256[0], b = T.h256[1], c = T.h256[2], d = T.h256[3];
  uint32_t e = T.h256[4], f = T.h256[5], g = T.h256[6], h = T.h256[7];
#pragma unroll
  for (int t = 0; t < 64; ++t) {
    uint32_t wt;
    if (t < 16) {
      wt = W[t];
    } else {
      const uint32_t w15 = W[(t - 15) & 15], w2 = W[(t - 2) & 15];
      const uint32_t s0 = xor3(rotr32(w15, 7), rotr32(w15, 18), w15 >> 3);
      const uint32_t s1 = xor3(rotr32(w2, 17), rotr32(w2, 19), w2 >> 10);
      wt = W[t & 15] = W[t & 15] + s0 + W[(t - 7) & 15] + s1;
    }
    const uint32_t S1 = xor3(rotr32(e, 6), rotr32(e, 11), rotr32(e, 25));
    const uint32_t t1 = h + S1 + ch32(e, f, g) + T.k256[t] + wt;
    const uint32_t S0 = xor3(rotr32(a, 2), rotr32(a, 13), rotr32(a, 22));
    const uint32_t mj = maj32(a, b, c);
    h = g; g = f; f = e; e = d + t1;
    d = c; c = b; b = a; a = t1 + S0 + mj;
  }
  H[0] = T.h256[0] + a; H[1] = T.h256[1] + b; H[2] = T.h256[2] + c; H[3] = T.h256[3] + d;
  H[4] = T.h256[4] + e; H[5] = T.h256[5] + f; H[6] = T.h256[6] + g; H[7] = T.h256[7] + h;
}

__device__ __forceinline__ void sha512_block(const Sha2Tables &T, uint64_t (&W)[16], uint64_t (&H)[8]) {
  uint64_t a = T.h512[0], b = T.h512[1], c = T.h512[2], d = T.h512[3];
  uint64_t e = T.h512[4], f = T.h512[5], g = T.h512[6], h = T.h512[7];
#pragma unroll
  for (int t = 0; t < 80; ++t) {
    uint64_t wt;
    if (t < 16) {
      wt = W[t];
    } else {
      const uint64_t w15 = W[(t - 15) & 15], w2 = W[(t - 2) & 15];
      const uint64_t s0 = xor3_64(rotr64<1>(w15), rotr64<8>(w15), shr64<7>(w15));
      const uint64_t s1 = xor3_64(rotr64<19>(w2), rotr64<61>(w2), shr64<6>(w2));
      wt = W[t & 15] = W[t & 15] + s0 + W[(t - 7) & 15] + s1;
    }
    const uint64_t S1 = xor3_64(rotr64<14>(e), rotr64<18>(e), rotr64<41>(e));
    const uint64_t t1 = h + S1 + ch64(e, f, g) + T.k512[t] + wt;
    const uint64_t S0 = xor3_64(rotr64<28>(a), rotr64<34>(a), rotr64<39>(a));
    const uint64_t mj = maj64(a, b, c);
    h = g; g = f; f = e; e = d + t1;
    d = c; c = b; b = a; a = t1 + S0 + mj;
  }
  H[0] = T.h512[0] + a; H[1] = T.h512[1] + b; H[2] = T.h512[2] + c; H[3] = T.h512[3] + d;
  H[4] = T.h512[4] + e; H[5] = T.h512[5] + f; H[6] = T.h512[6] + g; H[7] = T.h512[7] + h;
}

// Keystream of the first public record: SHA-256 of m1, XORed in place.
__device__ __forceinline__ void pub1_xor(const Se8Params &P, uint32_t priv_lo, uint32_t priv_hi,
                                         uint64_t b, uint32_t (&pub1)[4]) {
  uint32_t W[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) W[t] = P.m1[t];
  // bytes 0..4: the private record (little-endian bit stream), big-endian words
  W[0] = __builtin_bswap32(priv_lo);
  W[1] |= (priv_hi & 0xFFu) << 24;
  // bytes 37..44: the block index, big-endian
  W[9] |= uint32_t(b >> 40) & 0xFFFFFFu;
  W[10] = uint32_t(b >> 8);
  W[11] |= uint32_t(b & 0xFF) << 24;
  uint32_t H[8];
  sha256_block(P.tab, W, H);
#pragma unroll
  for (int k = 0; k < 4; ++k) pub1[k] ^= __builtin_bswap32(H[k]);
  pub1[3] &= 0x0FFFFFFFu;  // 124 bits
}

// Keystream of the second public record: SHA-512 of m2, XORed in place.
__device__ __forceinline__ void pub2_xor(const Se8Params &P, const uint32_t (&pub1)[4], uint64_t b,
                                         uint32_t (&pub2)[15]) {
  uint64_t W[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) W[t] = 0;
  W[0] = __builtin_bswap64(uint64_t(pub1[0]) | (uint64_t(pub1[1]) << 32));
  W[1] = __builtin_bswap64(uint64_t(pub1[2]) | (uint64_t(pub1[3]) << 32));
  W[2] = P.m2_key[0];
  W[3] = P.m2_key[1];
  W[4] = P.m2_nonce[0];
  W[5] = P.m2_nonce[1];
  W[6] = b;
  W[7] = uint64_t(0x80) << 56;  // padding after 56 message bytes
  W[15] = 56 * 8;               // message length in bits
  uint64_t H[8];
  sha512_block(P.tab, W, H);
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    pub2[2 * j] ^= __builtin_bswap32(uint32_t(H[j] >> 32));
    if (2 * j + 1 < 15) pub2[2 * j + 1] ^= __builtin_bswap32(uint32_t(H[j]));
  }
}

// ------------------------------------------------------------- LDS ranges --
struct SeLds {
  uint32_t priv[kPrivRange / 4];
  uint32_t pub1[kPub1Range / 4];
  uint32_t pub2[kPub2Range / 4];
  uint32_t te[1024];
  uint32_t kw[kKeyWords];
};

// Byte counts of this workgroup's three ranges (the last workgroup may hold
// fewer than 256 blocks).
__device__ __forceinline__ void range_bytes(uint32_t nb, uint32_t &pr, uint32_t &p1, uint32_t &p2) {
  pr = 5 * nb;
  p1 = (124 * nb + 7) / 8;
  p2 = 60 * nb;
}

// LDS range <-> global range (16-byte vectors, bytes for the tail); the
// global range starts 16-byte aligned.
__device__ __forceinline__ void range_store(uint8_t *dst, const uint32_t *lds, uint32_t bytes) {
  const uint32_t vecs = bytes / 16;
  for (uint32_t i = threadIdx.x; i < vecs; i += kSeThreads) {
    const uint32_t *s = lds + 4 * i;
    *(gptr<u32x4>)(glob(dst) + 16 * i) = u32x4{s[0], s[1], s[2], s[3]};
  }
  const uint32_t tail = bytes - 16 * vecs;
  if (threadIdx.x < tail) {
    const uint32_t o = 16 * vecs + threadIdx.x;
    glob(dst)[o] = uint8_t(lds[o >> 2] >> (8 * (o & 3)));
  }
}

__device__ __forceinline__ void range_load(uint32_t *lds, const uint8_t *src, uint32_t bytes,
                                           uint32_t words_total) {
  const uint32_t vecs = bytes / 16;
  for (uint32_t i = threadIdx.x; i < vecs; i += kSeThreads) {
    const u32x4 v = *(gptr<const u32x4>)(glob(src) + 16 * i);
    lds[4 * i] = v.x; lds[4 * i + 1] = v.y; lds[4 * i + 2] = v.z; lds[4 * i + 3] = v.w;
  }
  // the tail words (zero past `bytes`), one thread per word
  for (uint32_t wi = 4 * vecs + threadIdx.x; wi < words_total; wi += kSeThreads) {
    uint32_t w = 0;
    for (int k = 0; k < 4; ++k) {
      const uint32_t o = 4 * wi + k;
      if (o < bytes) w |= uint32_t(glob(src)[o]) << (8 * k);
    }
    lds[wi] = w;
  }
}

// AES-128-CTR over the private range in LDS: global keystream block
// 80 * group + j, one thread per 16-byte block.
__device__ __forceinline__ void ctr_range(SeLds &S, uint64_t group, uint32_t bytes) {
  const uint32_t nblk = (bytes + 15) / 16;
  if (threadIdx.x < nblk) {
    uint32_t w[4];
    counter_block(S.kw, group * (kPrivRange / 16) + threadIdx.x, w);
    aes_encrypt(S.te, S.kw, w);
#pragma unroll
    for (int k = 0; k < 4; ++k) S.priv[4 * threadIdx.x + k] ^= w[k];
  }
}

__device__ __forceinline__ void load_block(const Se8Params &P, uint64_t b, int (&m)[64]) {
  const uint32_t by = uint32_t(b / P.wb), bx = uint32_t(b % P.wb);
  const uint64_t base = uint64_t(8 * by) * P.W + 8 * bx;
  if (base + 7 * uint64_t(P.W) + 8 <= P.n) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const u32x2 v = *(gptr<const u32x2>)(glob(P.in) + base + uint64_t(r) * P.W);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        m[8 * r + c] = int((v.x >> (8 * c)) & 0xFF);
        m[8 * r + 4 + c] = int((v.y >> (8 * c)) & 0xFF);
      }
    }
  } else {
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const uint64_t o = base + uint64_t(r) * P.W + c;
        m[8 * r + c] = o < P.n ? int(glob(P.in)[o]) : 0;
      }
  }
}

__device__ __forceinline__ void store_block(const Se8Params &P, uint64_t b, const int (&m)[64]) {
  const uint32_t by = uint32_t(b / P.wb), bx = uint32_t(b % P.wb);
  const uint64_t base = uint64_t(8 * by) * P.W + 8 * bx;
  if (base + 7 * uint64_t(P.W) + 8 <= P.n) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      uint32_t lo = 0, hi = 0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        lo |= (uint32_t(m[8 * r + c]) & 0xFF) << (8 * c);
        hi |= (uint32_t(m[8 * r + 4 + c]) & 0xFF) << (8 * c);
      }
      *(gptr<u32x2>)(glob(P.out) + base + uint64_t(r) * P.W) = u32x2{lo, hi};
    }
  } else {
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const uint64_t o = base + uint64_t(r) * P.W + c;
        if (o < P.n) glob(P.out)[o] = uint8_t(m[8 * r + c]);
      }
  }
}

}  // namespace

__global__ __launch_bounds__(kSeThreads) void se8_protect_kernel(const Se8Params P) {
  __shared__ SeLds S;
  const uint64_t group = blockIdx.x;
  const uint64_t b0 = group * kSeThreads;
  const uint32_t nb = uint32_t(min<uint64_t>(kSeThreads, P.blocks - b0));
  load_aes_tables(S.te, S.kw, P.key);
  for (int i = threadIdx.x; i < kPrivRange / 4; i += kSeThreads) S.priv[i] = 0;
  for (int i = threadIdx.x; i < kPub1Range / 4; i += kSeThreads) S.pub1[i] = 0;
  __syncthreads();
  const uint32_t t = threadIdx.x;
  if (t < nb) {
    const uint64_t b = b0 + t;
    uint32_t pr[2] = {0, 0}, p1[4] = {0, 0, 0, 0}, p2[15];
    {
      int m[64];
      load_block(P, b, m);
      block_fwd(m);
#pragma unroll
      for (int k = 0; k < 4; ++k) put_bits(pr, 10 * k, 10, m[cell_priv(k)]);
#pragma unroll
      for (int k = 0; k < 12; ++k) put_bits(p1, pub1_pos(k), pub1_bits(k), m[cell_pub1(k)]);
#pragma unroll
      for (int k = 0; k < 15; ++k) p2[k] = 0;
#pragma unroll
      for (int k = 0; k < 48; ++k) put_bits(p2, 10 * k, 10, m[cell_pub2(k)]);
    }
    pub1_xor(P, pr[0], pr[1], b, p1);
    pub2_xor(P, p1, b, p2);
    // records into the LDS ranges: private at byte 5t, first public at bit
    // 124t (two records share a byte), second public at byte 60t
    {
      const uint32_t bit = 40 * t, q = bit >> 5, s = bit & 31;
      atomicOr(&S.priv[q], pr[0] << s);
      atomicOr(&S.priv[q + 1], (s ? pr[0] >> (32 - s) : 0u) | (pr[1] << s));
      if (s + 8 > 32) atomicOr(&S.priv[q + 2], pr[1] >> (32 - s));
    }
    {
      const uint32_t bit = 124 * t, q = bit >> 5, s = bit & 31;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        atomicOr(&S.pub1[q + k], (p1[k] << s) | (s && k ? p1[k - 1] >> (32 - s) : 0u));
      }
      if (s && q + 4 < kPub1Range / 4) atomicOr(&S.pub1[q + 4], p1[3] >> (32 - s));
    }
#pragma unroll
    for (int k = 0; k < 15; ++k) S.pub2[15 * t + k] = p2[k];
  }
  __syncthreads();
  uint32_t bpr, bp1, bp2;
  range_bytes(nb, bpr, bp1, bp2);
  ctr_range(S, group, bpr);
  __syncthreads();
  range_store(P.priv + group * kPrivRange, S.priv, bpr);
  range_store(P.pub1 + group * kPub1Range, S.pub1, bp1);
  range_store(P.pub2 + group * kPub2Range, S.pub2, bp2);
}

// Restore hashes in sequence (SHA-256 unmasks the level-2 details that
// SHA-512 then hashes), so a wavefront has less independent work to issue
// than in the protect, where the two hashes interleave: three wavefronts per
// SIMD (168 VGPRs, a few spilled) hide that chain better than two
// (measured 758-768 against 785-800 us on the 256 MiB workload).
__global__ __launch_bounds__(kSeThreads) __attribute__((amdgpu_waves_per_eu(3)))
void se8_restore_kernel(const Se8Params P) {
  __shared__ SeLds S;
  const uint64_t group = blockIdx.x;
  const uint64_t b0 = group * kSeThreads;
  const uint32_t nb = uint32_t(min<uint64_t>(kSeThreads, P.blocks - b0));
  uint32_t bpr, bp1, bp2;
  range_bytes(nb, bpr, bp1, bp2);
  load_aes_tables(S.te, S.kw, P.key);
  range_load(S.priv, P.priv_in + group * kPrivRange, bpr, kPrivRange / 4);
  range_load(S.pub1, P.pub1_in + group * kPub1Range, bp1, kPub1Range / 4);
  range_load(S.pub2, P.pub2_in + group * kPub2Range, bp2, kPub2Range / 4);
  __syncthreads();
  ctr_range(S, group, bpr);
  __syncthreads();
  const uint32_t t = threadIdx.x;
  if (t >= nb) return;
  const uint64_t b = b0 + t;
  uint32_t pr[2], p1[4], p1s[4], p2[15];
  {
    const uint32_t bit = 40 * t, q = bit >> 5, s = bit & 31;
    const uint32_t w0 = S.priv[q], w1 = S.priv[q + 1], w2 = (q + 2 < kPrivRange / 4) ? S.priv[q + 2] : 0u;
    pr[0] = s ? (w0 >> s) | (w1 << (32 - s)) : w0;
    pr[1] = (s ? (w1 >> s) | (w2 << (32 - s)) : w1) & 0xFFu;
  }
  {
    const uint32_t bit = 124 * t, q = bit >> 5, s = bit & 31;
    uint32_t w[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) w[k] = (q + k < kPub1Range / 4) ? S.pub1[q + k] : 0u;
#pragma unroll
    for (int k = 0; k < 4; ++k) p1s[k] = s ? (w[k] >> s) | (w[k + 1] << (32 - s)) : w[k];
    p1s[3] &= 0x0FFFFFFFu;
  }
#pragma unroll
  for (int k = 0; k < 15; ++k) p2[k] = S.pub2[15 * t + k];
#pragma unroll
  for (int k = 0; k < 4; ++k) p1[k] = p1s[k];
  pub1_xor(P, pr[0], pr[1], b, p1);  // clear first public record
  pub2_xor(P, p1s, b, p2);           // keyed on the stored (protected) record
  int m[64];
#pragma unroll
  for (int k = 0; k < 4; ++k) m[cell_priv(k)] = get_bits(pr, 10 * k, 10);
#pragma unroll
  for (int k = 0; k < 12; ++k) m[cell_pub1(k)] = get_bits(p1, pub1_pos(k), pub1_bits(k));
#pragma unroll
  for (int k = 0; k < 48; ++k) m[cell_pub2(k)] = get_bits(p2, 10 * k, 10);
  block_inv(m);
  store_block(P, b, m);
}

// ------------------------------------------------------------ host side ----
namespace {

// Integer k-th root of a 256-bit value (limbs little-endian), bit by bit.
struct U256 {
  uint64_t w[4];
};

U256 mul(const U256 &a, const U256 &b) {
  U256 r{{0, 0, 0, 0}};
  for (int i = 0; i < 4; ++i) {
    unsigned __int128 carry = 0;
    for (int j = 0; i + j < 4; ++j) {
      const unsigned __int128 cur = (unsigned __int128)a.w[i] * b.w[j] + r.w[i + j] + carry;
      r.w[i + j] = uint64_t(cur);
      carry = cur >> 64;
    }
  }
  return r;
}

bool le(const U256 &a, const U256 &b) {
  for (int i = 3; i >= 0; --i)
    if (a.w[i] != b.w[i]) return a.w[i] < b.w[i];
  return true;
}

// floor(p^(1/k) * 2^frac_bits) mod 2^64 (the first frac_bits bits of the
// fractional part of the root, below its integer part)
uint64_t root_bits(uint64_t p, int k, int frac_bits) {
  U256 N{{0, 0, 0, 0}};
  const int sh = k * frac_bits;  // N = p * 2^(k * frac_bits)
  N.w[sh / 64] = p << (sh % 64);
  if (sh % 64) N.w[sh / 64 + 1] = p >> (64 - sh % 64);
  U256 x{{0, 0, 0, 0}};
  for (int bit = frac_bits + 3; bit >= 0; --bit) {  // roots of primes < 512 are < 8
    U256 y = x;
    y.w[bit / 64] |= uint64_t(1) << (bit % 64);
    U256 pw = y;
    for (int e = 1; e < k; ++e) pw = mul(pw, y);
    if (le(pw, N)) x = y;
  }
  return frac_bits == 64 ? x.w[0] : (x.w[0] & ((uint64_t(1) << frac_bits) - 1));
}

Sha2Tables make_tables() {
  Sha2Tables T{};
  uint64_t primes[80];
  int np = 0;
  for (uint64_t c = 2; np < 80; ++c) {
    bool prime = true;
    for (uint64_t d = 2; d * d <= c; ++d)
      if (c % d == 0) { prime = false; break; }
    if (prime) primes[np++] = c;
  }
  for (int i = 0; i < 80; ++i) T.k512[i] = root_bits(primes[i], 3, 64);
  for (int i = 0; i < 64; ++i) T.k256[i] = uint32_t(root_bits(primes[i], 3, 32));
  for (int i = 0; i < 8; ++i) {
    T.h512[i] = root_bits(primes[i], 2, 64);
    T.h256[i] = uint32_t(root_bits(primes[i], 2, 32));
  }
  return T;
}

const Sha2Tables &tables() {
  static const Sha2Tables T = make_tables();
  return T;
}

uint64_t load_be64(const uint8_t *p) {
  uint64_t v = 0;
  for (int i = 0; i < 8; ++i) v = (v << 8) | p[i];
  return v;
}

}  // namespace

int se8_make_geometry(uint64_t n, uint32_t width, Se8Geometry *g) {
  if (n == 0 || width == 0 || width % 8) return -1;
  const uint64_t H = (n + width - 1) / width;
  const uint64_t hb = (H + 7) / 8, wb = width / 8;
  const uint64_t blocks = hb * wb;
  // one workgroup per 256 blocks; the grid holds at most 2^31 - 1 of them
  if (blocks > (uint64_t(0x7FFFFFFF) << 8) || H > 0x7FFF0000ull) return -2;
  g->H = H;
  g->hb = hb;
  g->wb = wb;
  g->blocks = blocks;
  g->priv_bytes = 5 * blocks;
  g->pub1_bytes = (124 * blocks + 7) / 8;
  g->pub2_bytes = 60 * blocks;
  return 0;
}

void se8_fill_params(const Se8Geometry &g, uint64_t n, uint32_t width, const uint8_t key[16],
                     const uint8_t nonce[16], Se8Params *P) {
  std::memset(P, 0, sizeof(*P));
  P->n = n;
  P->W = width;
  P->wb = uint32_t(g.wb);
  P->blocks = g.blocks;
  expand_key(key, nonce, &P->key);
  P->tab = tables();
  // m1 template (SHA-256 big-endian words): bytes 5..20 key, 21..36 nonce,
  // 0x80 at 45, message length 45 * 8 bits in the last word
  uint8_t m1[64] = {0};
  for (int i = 0; i < 16; ++i) {
    m1[5 + i] = key[i];
    m1[21 + i] = nonce[i];
  }
  m1[45] = 0x80;
  m1[62] = uint8_t((45 * 8) >> 8);
  m1[63] = uint8_t(45 * 8);
  for (int t = 0; t < 16; ++t)
    P->m1[t] = (uint32_t(m1[4 * t]) << 24) | (uint32_t(m1[4 * t + 1]) << 16) |
               (uint32_t(m1[4 * t + 2]) << 8) | uint32_t(m1[4 * t + 3]);
  P->m2_key[0] = load_be64(key);
  P->m2_key[1] = load_be64(key + 8);
  P->m2_nonce[0] = load_be64(nonce);
  P->m2_nonce[1] = load_be64(nonce + 8);
}

hipError_t launch_se8(bool forward, const Se8Params &P, hipStream_t s) {
  const uint64_t groups = (P.blocks + kSeThreads - 1) / kSeThreads;
  if (forward)
    hipLaunchKernelGGL(se8_protect_kernel, dim3(unsigned(groups)), dim3(kSeThreads), 0, s, P);
  else
    hipLaunchKernelGGL(se8_restore_kernel, dim3(unsigned(groups)), dim3(kSeThreads), 0, s, P);
  return hipGetLastError();
}

}  // namespace dwtfrag

using namespace dwtfrag;

extern "C" {

int dwtfrag_se8_geometry(uint64_t n, uint32_t width, dwtfrag_se8_geom *out) {
  if (!out) return DWTFRAG_EINVAL;
  Se8Geometry g;
  const int rc = se8_make_geometry(n, width, &g);
  if (rc) return rc == -1 ? DWTFRAG_EINVAL : DWTFRAG_ERANGE;
  out->n = n;
  out->width = width;
  out->height = g.H;
  out->block_rows = g.hb;
  out->block_cols = g.wb;
  out->blocks = g.blocks;
  out->priv_bytes = g.priv_bytes;
  out->pub1_bytes = g.pub1_bytes;
  out->pub2_bytes = g.pub2_bytes;
  return DWTFRAG_OK;
}

int dwtfrag_se8_protect(const uint8_t *in, uint64_t n, uint32_t width, const uint8_t key[16],
                        const uint8_t nonce[16], uint8_t *priv, uint8_t *pub1, uint8_t *pub2,
                        void *stream) {
  if (!in || !key || !nonce || !priv || !pub1 || !pub2) return DWTFRAG_EINVAL;
  Se8Geometry g;
  const int rc = se8_make_geometry(n, width, &g);
  if (rc) return rc == -1 ? DWTFRAG_EINVAL : DWTFRAG_ERANGE;
  if (((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(priv) |
        reinterpret_cast<uintptr_t>(pub1) | reinterpret_cast<uintptr_t>(pub2)) & 15))
    return DWTFRAG_EINVAL;
  Se8Params P;
  se8_fill_params(g, n, width, key, nonce, &P);
  P.in = in;
  P.priv = priv;
  P.pub1 = pub1;
  P.pub2 = pub2;
  return launch_se8(true, P, static_cast<hipStream_t>(stream)) == hipSuccess ? DWTFRAG_OK
                                                                             : DWTFRAG_EDEVICE;
}

int dwtfrag_se8_restore(const uint8_t *priv, const uint8_t *pub1, const uint8_t *pub2, uint64_t n,
                        uint32_t width, const uint8_t key[16], const uint8_t nonce[16],
                        uint8_t *out, void *stream) {
  if (!priv || !pub1 || !pub2 || !key || !nonce || !out) return DWTFRAG_EINVAL;
  Se8Geometry g;
  const int rc = se8_make_geometry(n, width, &g);
  if (rc) return rc == -1 ? DWTFRAG_EINVAL : DWTFRAG_ERANGE;
  if (((reinterpret_cast<uintptr_t>(out) | reinterpret_cast<uintptr_t>(priv) |
        reinterpret_cast<uintptr_t>(pub1) | reinterpret_cast<uintptr_t>(pub2)) & 15))
    return DWTFRAG_EINVAL;
  Se8Params P;
  se8_fill_params(g, n, width, key, nonce, &P);
  P.priv_in = priv;
  P.pub1_in = pub1;
  P.pub2_in = pub2;
  P.out = out;
  return launch_se8(false, P, static_cast<hipStream_t>(stream)) == hipSuccess ? DWTFRAG_OK
                                                                              : DWTFRAG_EDEVICE;
}

}  // extern "C"
