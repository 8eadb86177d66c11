// Shared definitions of the HIP path: launch parameters, wavefront neighbour
// taps, and AES-128 (tables derived at compile time from GF(2^8) arithmetic).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dwtfrag {

// Levels fused into one streaming kernel; deeper transforms run as further
// stages over the LL band of the previous stage.
constexpr int kMaxFused = 4;
constexpr int kWavesPerBlock = 4;
constexpr int kBlockThreads = 64 * kWavesPerBlock;
// Keystream ring per wavefront: up to 96 AES blocks of 16 bytes.
constexpr int kRingBlocks = 96;

// ----------------------------------------------------------------- AES-128 --
// FIPS-197 S-box: multiplicative inverse in GF(2^8) mod x^8+x^4+x^3+x+1, then
// the affine map b_i ^ b_{i+4} ^ b_{i+5} ^ b_{i+6} ^ b_{i+7} ^ 0x63_i.
constexpr uint8_t gf_mul(uint8_t a, uint8_t b) {
  uint8_t r = 0;
  for (int i = 0; i < 8; ++i) {
    if (b & 1) r ^= a;
    bool hi = a & 0x80;
    a = uint8_t(a << 1);
    if (hi) a ^= 0x1B;
    b >>= 1;
  }
  return r;
}

constexpr uint8_t gf_inv(uint8_t a) {
  if (a == 0) return 0;
  uint8_t r = 1, base = a;
  int e = 254;
  while (e) {
    if (e & 1) r = gf_mul(r, base);
    base = gf_mul(base, base);
    e >>= 1;
  }
  return r;
}

constexpr uint8_t rotl8(uint8_t v, int s) { return uint8_t((v << s) | (v >> (8 - s))); }

constexpr uint8_t sbox_entry(uint8_t a) {
  uint8_t b = gf_inv(a);
  return uint8_t(b ^ rotl8(b, 1) ^ rotl8(b, 2) ^ rotl8(b, 3) ^ rotl8(b, 4) ^ 0x63);
}

struct AesTables {
  uint8_t sbox[256];
  // te0[x]: MixColumns column of a substituted byte in row 0, as a
  // little-endian word (bytes 2S, S, S, 3S); rows 1..3 are byte rotations.
  uint32_t te0[256];
};

constexpr AesTables make_aes_tables() {
  AesTables t{};
  for (int x = 0; x < 256; ++x) {
    uint8_t s = sbox_entry(uint8_t(x));
    uint8_t s2 = gf_mul(s, 2), s3 = uint8_t(s2 ^ s);
    t.sbox[x] = s;
    t.te0[x] = uint32_t(s2) | (uint32_t(s) << 8) | (uint32_t(s) << 16) | (uint32_t(s3) << 24);
  }
  return t;
}

// Round keys as little-endian column words (44 words); nonce as two 64-bit
// big-endian halves.
struct AesKey {
  uint32_t rk[44];
  uint64_t nonce_hi, nonce_lo;
};

void expand_key(const uint8_t key[16], const uint8_t nonce[16], AesKey *out);

__device__ __forceinline__ uint32_t bswap32(uint32_t v) { return __builtin_bswap32(v); }

// Key material as staged in LDS: 44 round-key words, then the nonce as
// (hi low word, hi high word, lo low word, lo high word).
constexpr int kKeyWords = 48;

// Block j of the counter sequence as 4 little-endian state words.
__device__ __forceinline__ void counter_block(const uint32_t *kw, uint64_t j, uint32_t w[4]) {
  const uint64_t nhi = uint64_t(kw[44]) | (uint64_t(kw[45]) << 32);
  const uint64_t nlo = uint64_t(kw[46]) | (uint64_t(kw[47]) << 32);
  uint64_t lo = nlo + j;
  uint64_t hi = nhi + (lo < nlo ? 1ull : 0ull);
  w[0] = bswap32(uint32_t(hi >> 32));
  w[1] = bswap32(uint32_t(hi));
  w[2] = bswap32(uint32_t(lo >> 32));
  w[3] = bswap32(uint32_t(lo));
}

// One AES-128 encryption; `te` points at four 256-word tables in LDS
// (te[256 r + x] = rotl(te0[x], 8 r)), `rk` at the 44 round-key words.
// Each column of a middle round is four table words and a round-key word
// XORed together: two 3-input bit operations (truth table 0x96 = a ^ b ^ c).
// The last round takes the S-box byte (byte 1 of te0[x]) of four lookups
// with two byte permutes and joins them with the round key in one 3-input
// operation (truth table 0x56 = (a | b) ^ c).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ void aes_encrypt(const uint32_t *te, const uint32_t *rk, uint32_t w[4]) {
  uint32_t s0 = w[0] ^ rk[0], s1 = w[1] ^ rk[1], s2 = w[2] ^ rk[2], s3 = w[3] ^ rk[3];
#define DWTFRAG_TE(r, v) te[256 * (r) + (((v) >> (8 * (r))) & 0xFF)]
#pragma unroll
  for (int rnd = 1; rnd < 10; ++rnd) {
    const uint32_t t0 = xor3(xor3(DWTFRAG_TE(0, s0), DWTFRAG_TE(1, s1), DWTFRAG_TE(2, s2)), DWTFRAG_TE(3, s3), rk[4 * rnd + 0]);
    const uint32_t t1 = xor3(xor3(DWTFRAG_TE(0, s1), DWTFRAG_TE(1, s2), DWTFRAG_TE(2, s3)), DWTFRAG_TE(3, s0), rk[4 * rnd + 1]);
    const uint32_t t2 = xor3(xor3(DWTFRAG_TE(0, s2), DWTFRAG_TE(1, s3), DWTFRAG_TE(2, s0)), DWTFRAG_TE(3, s1), rk[4 * rnd + 2]);
    const uint32_t t3 = xor3(xor3(DWTFRAG_TE(0, s3), DWTFRAG_TE(1, s0), DWTFRAG_TE(2, s1)), DWTFRAG_TE(3, s2), rk[4 * rnd + 3]);
    s0 = t0; s1 = t1; s2 = t2; s3 = t3;
  }
#undef DWTFRAG_TE
  // last round: SubBytes + ShiftRows + the last round key
#define DWTFRAG_L(v, r) te[((v) >> (8 * (r))) & 0xFF]
#define DWTFRAG_LAST(a, b, c, d, k)                                                             \
  __builtin_amdgcn_bitop3_b32(__builtin_amdgcn_perm(DWTFRAG_L(b, 1), DWTFRAG_L(a, 0), 0x0c0c0501u), \
                              __builtin_amdgcn_perm(DWTFRAG_L(d, 3), DWTFRAG_L(c, 2), 0x05010c0cu), \
                              (k), 0x56)
  w[0] = DWTFRAG_LAST(s0, s1, s2, s3, rk[40]);
  w[1] = DWTFRAG_LAST(s1, s2, s3, s0, rk[41]);
  w[2] = DWTFRAG_LAST(s2, s3, s0, s1, rk[42]);
  w[3] = DWTFRAG_LAST(s3, s0, s1, s2, rk[43]);
#undef DWTFRAG_LAST
#undef DWTFRAG_L
}

static __constant__ AesTables c_aes = make_aes_tables();

// The four byte-rotated T-tables (1024 words) into LDS, loaded by the whole
// block; the caller synchronises the block afterwards.
__device__ __forceinline__ void load_aes_te(uint32_t *te) {
  for (int i = threadIdx.x; i < 1024; i += blockDim.x) {
    const uint32_t v = c_aes.te0[i & 255];
    const int r = 8 * (i >> 8);
    te[i] = r ? ((v << r) | (v >> (32 - r))) : v;
  }
}

// Word i (< kKeyWords) of the LDS key block: 44 round-key words, then the
// nonce's two 64-bit halves as low / high words.
__device__ __forceinline__ uint32_t key_word(const AesKey &key, int i) {
  if (i < 44) return key.rk[i];
  if (i == 44) return uint32_t(key.nonce_hi);
  if (i == 45) return uint32_t(key.nonce_hi >> 32);
  if (i == 46) return uint32_t(key.nonce_lo);
  return uint32_t(key.nonce_lo >> 32);
}

// Tables and key words together, for a block that uses one key.
__device__ __forceinline__ void load_aes_tables(uint32_t *te, uint32_t *kw, const AesKey &key) {
  load_aes_te(te);
  for (int i = threadIdx.x; i < kKeyWords; i += blockDim.x) kw[i] = key_word(key, i);
}

// --------------------------------------------------------- launch geometry --
// One stage = up to kMaxFused levels over an H x W input.  Wavefronts own
// rectangles of the level-0 grid: window k owns columns [k*own_w, ...);
// the rows are cut into `units` units of unit_rows = 2^L rows, and segment s
// owns units [floor(s*units/n_seg), floor((s+1)*units/n_seg)), so segment
// lengths differ by at most one unit.
struct StageParams {
  int64_t n_valid;            // valid input elements (byte view: n; else H*W)
  int32_t H, W;               // stage input dims
  int32_t hdim[kMaxFused + 1], wdim[kMaxFused + 1];  // level dims, [0] = input
  int64_t off_hl[kMaxFused + 1], off_lh[kMaxFused + 1], off_hh[kMaxFused + 1];
  int32_t own_w, n_win;       // owned columns per window, number of windows
  int32_t unit_rows, units;   // 2^L, ceil(H / 2^L)
  int32_t n_seg;              // number of row segments
  int32_t halo_l;             // columns before the owned range (multiple of lane_cols)
  int32_t last_base;          // first column of the last window's lanes (n_win > 1)
  int32_t halo_t, halo_b;     // rows streamed before / after the owned range
  int32_t n_waves;
  int32_t use_aes;            // LL output / input goes through AES-CTR
  int32_t ks_rows, ks_blocks; // keystream ring: rows per refill, blocks per row
  AesKey key;
};

// First level-0 column of window win's lanes: the owned range minus the left
// halo, from column 0 for the first window; the last window's lanes may start
// further left (last_base) so that they end inside the row.
__device__ __forceinline__ int window_base(const StageParams &P, int win) {
  if (win == 0) return 0;
  return win == P.n_win - 1 ? P.last_base : win * P.own_w - P.halo_l;
}

// First level-0 row of segment s (s == n_seg gives units * unit_rows).
__device__ __forceinline__ int seg_start(const StageParams &P, int s) {
  return P.unit_rows * int((int64_t(s) * P.units) / P.n_seg);
}

// ------------------------------------------------------ global pointers --
// Buffer accesses go through these: a pointer into device global memory, so
// that loads and stores compile to global (not flat) instructions also where
// the address was read from memory (batch items), which the compiler cannot
// place in an address space by itself.  Cast with glob() first, then change
// the pointee type.
template <class T> using gptr = __attribute__((address_space(1))) T *;
template <class T> __device__ __forceinline__ gptr<T> glob(T *p) { return (gptr<T>)p; }
// 8- and 16-byte vectors for those accesses (plain vector types, which can be
// read from any address space).
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------- wavefront taps --
// wave_shl:1 -> lane i receives lane i+1; wave_shr:1 -> lane i receives
// lane i-1 (the lane with no source receives 0).
__device__ __forceinline__ int from_next_lane(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xF, 0xF, false);
}
__device__ __forceinline__ int from_prev_lane(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xF, 0xF, false);
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace dwtfrag
