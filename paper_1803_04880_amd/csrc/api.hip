// C ABI of the library: validation, geometry, AES key schedule, stage and
// launch planning.  Declarations and contracts are in include/dwtfrag.h.
#include "dwtfrag.h"

#include <algorithm>
#include <atomic>
#include <cstring>
#include <mutex>

#include "common.h"

namespace dwtfrag {

hipError_t launch_fwd(int L, int C1, bool u8in, const void *in, int16_t *pub, int16_t *llout,
                      const StageParams &P, hipStream_t s);
hipError_t launch_inv(int L, int C1, bool u8out, const int16_t *llin, const int16_t *pub,
                      void *out, const StageParams &P, hipStream_t s);
hipError_t launch_ctr(const uint8_t *in, uint8_t *out, uint64_t nbytes, const AesKey &key,
                      uint64_t first_block, hipStream_t s);
int fwd_waves_per_cu(int L, int C1, bool u8in);
int inv_waves_per_cu(int L, int C1, bool u8out);
int inv_split_waves_per_cu(int L, int C1, bool all_fast);
bool inv_stage_split_ok(const StageParams &P);
bool inv_stage_all_fast(const StageParams &P, int L, int C1);

static constexpr AesTables kHostTables = make_aes_tables();

void expand_key(const uint8_t key[16], const uint8_t nonce[16], AesKey *out) {
  // FIPS-197 key expansion, Nk = 4, Nr = 10.  Words are kept little-endian
  // (byte 0 of a word in bits 0..7), matching the device state layout.
  uint32_t *w = out->rk;
  for (int i = 0; i < 4; ++i)
    w[i] = uint32_t(key[4 * i]) | (uint32_t(key[4 * i + 1]) << 8) |
           (uint32_t(key[4 * i + 2]) << 16) | (uint32_t(key[4 * i + 3]) << 24);
  uint8_t rcon = 1;
  for (int i = 4; i < 44; ++i) {
    uint32_t t = w[i - 1];
    if (i % 4 == 0) {
      t = (t >> 8) | (t << 24);  // RotWord on bytes (a0 a1 a2 a3) -> (a1 a2 a3 a0)
      t = uint32_t(kHostTables.sbox[t & 0xFF]) | (uint32_t(kHostTables.sbox[(t >> 8) & 0xFF]) << 8) |
          (uint32_t(kHostTables.sbox[(t >> 16) & 0xFF]) << 16) |
          (uint32_t(kHostTables.sbox[t >> 24]) << 24);
      t ^= rcon;
      rcon = gf_mul(rcon, 2);
    }
    w[i] = w[i - 4] ^ t;
  }
  uint64_t hi = 0, lo = 0;
  for (int i = 0; i < 8; ++i) {
    hi = (hi << 8) | nonce[i];
    lo = (lo << 8) | nonce[8 + i];
  }
  out->nonce_hi = hi;
  out->nonce_lo = lo;
}

namespace {

// Rows and columns of a view.  The launch planning and the kernels index rows
// and columns in int32 with margins of up to a window (1024 columns) and a
// unit plus halos (under 64 rows) past the end, so the limit keeps 2^16 below
// 2^31.
constexpr uint64_t kMaxDim = 0x7FFF0000ull;

// Bytes of the static workspace behind dwtfrag_protect_noalloc (16 MiB).
constexpr uint64_t kScratchBytes = uint64_t(16) << 20;

// Deepest decomposition accepted, and the fused stages it takes.  Geometry and
// launch plans live in fixed arrays of these sizes, so planning a call
// allocates nothing, on the host or the device.
constexpr uint32_t kMaxLevels = 32;
constexpr int kMaxStages = int((kMaxLevels + kMaxFused - 1) / kMaxFused);

struct Geometry {
  uint64_t n;
  uint32_t W, H, levels;
  uint64_t h[kMaxLevels + 1], w[kMaxLevels + 1];  // level dims 0..levels
  uint64_t priv_bytes, pub_bytes, ws_bytes;
  uint64_t ws_off[kMaxStages];  // workspace byte offset of LL_{4(s+1)}, s = 0..stages-2
  int stages;
};

uint64_t align256(uint64_t v) { return (v + 255) & ~uint64_t(255); }

int make_geometry(uint64_t n, uint32_t width, uint32_t levels, Geometry *g) {
  if (n == 0 || width == 0 || levels == 0 || levels > kMaxLevels) return DWTFRAG_EINVAL;
  if (width > kMaxDim) return DWTFRAG_ERANGE;
  const uint64_t H = (n + width - 1) / width;
  if (H > kMaxDim) return DWTFRAG_ERANGE;
  if (H * uint64_t(width) > (uint64_t(1) << 62)) return DWTFRAG_ERANGE;
  g->n = n;
  g->W = width;
  g->H = uint32_t(H);
  g->levels = levels;
  std::memset(g->h, 0, sizeof(g->h));
  std::memset(g->w, 0, sizeof(g->w));
  std::memset(g->ws_off, 0, sizeof(g->ws_off));
  g->h[0] = H;
  g->w[0] = width;
  for (uint32_t l = 1; l <= levels; ++l) {
    g->h[l] = (g->h[l - 1] + 1) / 2;
    g->w[l] = (g->w[l - 1] + 1) / 2;
  }
  const uint64_t ll = g->h[levels] * g->w[levels];
  g->priv_bytes = 2 * ll;
  g->pub_bytes = 2 * (H * width - ll);
  g->stages = int((levels + kMaxFused - 1) / kMaxFused);
  uint64_t ws = 0;
  for (int s = 0; s + 1 < g->stages; ++s) {
    g->ws_off[s] = ws;
    const int lv = kMaxFused * (s + 1);
    ws += align256(2 * g->h[lv] * g->w[lv]);
  }
  g->ws_bytes = ws;
  return DWTFRAG_OK;
}

// Element offset in pub of level l's three bands (levels stored coarsest
// first: L, L-1, ..., 1).
void level_offsets(const Geometry &g, uint32_t l, int64_t *hl, int64_t *lh, int64_t *hh) {
  uint64_t off = 0;
  for (uint32_t m = g.levels; m > l; --m) off += g.h[m - 1] * g.w[m - 1] - g.h[m] * g.w[m];
  *hl = int64_t(off);
  *lh = int64_t(off + g.h[l] * (g.w[l - 1] - g.w[l]));
  *hh = int64_t(off + g.h[l] * (g.w[l - 1] - g.w[l]) + (g.h[l - 1] - g.h[l]) * g.w[l]);
}

int round_up(int v, int m) { return (v + m - 1) / m * m; }

// Wavefronts the current device keeps resident at once for the kernel of a
// stage: compute units x resident wavefronts per CU (queried once per device
// and kernel variant; falls back to 256 x 16 if the queries fail).  split:
// 0 for the one-launch kernels, 1 / 2 for the split restore's packed kernel
// with every wavefront FAST / not.
int64_t device_slots(bool forward, int L, int C1, bool bytes, int split = 0) {
  constexpr int kDev = 16, kVar = 2 * 5 * 3 * 2 * 2;
  static std::atomic<int> cache[kDev][kVar];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kDev) dev = -1;
  const int var = (((forward ? 1 : 0) * 5 + L) * 3 + split) * 4 + (C1 == 16 ? 2 : 0) + (bytes ? 1 : 0);
  if (dev >= 0) {
    const int v = cache[dev][var].load(std::memory_order_relaxed);
    if (v > 0) return v;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev < 0 ? 0 : dev) != hipSuccess)
    cus = 0;
  const int per_cu = forward ? fwd_waves_per_cu(L, C1, bytes)
                     : split ? inv_split_waves_per_cu(L, C1, split == 1)
                             : inv_waves_per_cu(L, C1, bytes);
  const int slots = (cus > 0 && per_cu > 0) ? cus * per_cu : 256 * 16;
  if (dev >= 0) cache[dev][var].store(slots, std::memory_order_relaxed);
  return slots;
}

// SIMDs of the current device (4 per compute unit), cached per device.
int64_t device_simds() {
  constexpr int kDev = 16;
  static std::atomic<int> cache[kDev];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kDev) dev = -1;
  if (dev >= 0) {
    const int v = cache[dev].load(std::memory_order_relaxed);
    if (v > 0) return v;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev < 0 ? 0 : dev) != hipSuccess)
    cus = 0;
  const int simds = cus > 0 ? 4 * cus : 1024;
  if (dev >= 0) cache[dev].store(simds, std::memory_order_relaxed);
  return simds;
}

// Fill stage s's parameters.  forward selects the halo shape of the direction;
// alone: the stage runs as its own launch (not as one item of a batch that
// shares the device).
int plan_stage(const Geometry &g, int s, bool forward, const dwtfrag_launch *launch,
               const AesKey &key, StageParams *P, int *L_out, int *C1_out, bool alone) {
  std::memset(P, 0, sizeof(*P));
  const int lv0 = kMaxFused * s;  // global level of the stage input
  const int L = int(std::min<uint32_t>(kMaxFused, g.levels - lv0));
  // Default columns per lane: 16 for a stage of at least 64 Mi elements (the
  // per-row work is spread over twice the columns and the device stays full
  // at two wavefronts per SIMD; 256 MiB at three levels: forward 237 -> 224
  // us, inverse 248 -> 227 us in its two-launch form), else 8 (more, shorter
  // streams for smaller stages).
  const bool wide = uint64_t(g.h[lv0]) * g.w[lv0] >= (uint64_t(1) << 26);
  int C1 = (launch && launch->lane_cols) ? int(launch->lane_cols) : (wide ? 16 : 8);
  if (C1 != 8 && C1 != 16) return DWTFRAG_EINVAL;
  if (L == 4) C1 = 16;
  P->H = int32_t(g.h[lv0]);
  P->W = int32_t(g.w[lv0]);
  P->n_valid = (s == 0) ? int64_t(g.n) : int64_t(g.h[lv0] * g.w[lv0]);
  for (int l = 0; l <= L; ++l) {
    P->hdim[l] = int32_t(g.h[lv0 + l]);
    P->wdim[l] = int32_t(g.w[lv0 + l]);
  }
  for (int l = 1; l <= L; ++l)
    level_offsets(g, uint32_t(lv0 + l), &P->off_hl[l], &P->off_lh[l], &P->off_hh[l]);
  // halos (level-0 samples of this stage): forward needs 2^(L+1)-2 before and
  // 2^L-1 after an owned range, inverse the reverse; rows are streamed with
  // 2^(L+1) / 2^L (forward) and 2^L / 2^L (inverse) extra rows.
  const int big = (1 << (L + 1)) - 2, small = (1 << L) - 1;
  const int hl = round_up(forward ? big : small, C1);
  const int hr = round_up(forward ? small : big, C1);
  const int span = 64 * C1;
  if (P->W <= span) {
    P->own_w = P->W;
    P->n_win = 1;
  } else {
    P->own_w = span - hl - hr;
    P->n_win = (P->W + P->own_w - 1) / P->own_w;
  }
  P->halo_l = hl;
  // The inverse's last window: when the row is a whole number of lane
  // vectors, its lanes are placed to end at the row's end (a larger left
  // halo), so every lane reads whole vectors inside every band row.  The
  // forward keeps the plain placement.
  P->last_base = P->n_win > 1 ? (P->n_win - 1) * P->own_w - hl : 0;
  if (!forward && P->n_win > 1 && P->W % C1 == 0 && P->W >= span)
    P->last_base = std::min(P->last_base, P->W - span);
  P->halo_t = forward ? (1 << (L + 1)) : (1 << L);
  P->halo_b = 1 << L;
  const int unit = 1 << L;
  P->unit_rows = unit;
  P->units = (P->H + unit - 1) / unit;
  int64_t n_seg;
  if (launch && launch->seg_rows) {
    const int own_h = std::max(unit, round_up(int(std::min<uint32_t>(launch->seg_rows, uint32_t(P->H))), unit));
    n_seg = (int64_t(P->H) + own_h - 1) / own_h;
  } else {
    // one round of resident wavefronts: as many segments as fill the device
    // once, each at least two units long (halo work stays below the owned).
    // A launch of its own whose grid stays within one wavefront per SIMD
    // even at one unit per segment takes one unit per segment: the extra
    // halo rows run on otherwise idle SIMDs and each stream is shorter.
    // A restore's byte stage that runs as the split pair is filled to the
    // packed kernel's own residency (three wavefronts per SIMD at 16
    // columns, where the one-launch kernel holds two: 256 MiB at three
    // levels, restore 210 -> 195 us), and planned again with the one-launch
    // kernel's when the finished plan turns out not to run split.
    const int min_units = (alone && int64_t(P->units) * P->n_win <= device_simds()) ? 1 : 2;
    const auto segments = [&](int split) {
      const int64_t slots = device_slots(forward, L, C1, s == 0, split);
      const int64_t k = std::max<int64_t>(1, slots / P->n_win);
      return std::min<int64_t>(k, std::max(1, P->units / min_units));
    };
    const int split = (alone && !forward && s == 0 && P->n_valid >= (int64_t(1) << 24))
                          ? (inv_stage_all_fast(*P, L, C1) ? 1 : 2) : 0;
    n_seg = segments(split);
    if (split) {
      P->n_seg = int32_t(std::min<int64_t>(n_seg, P->units));
      if (!inv_stage_split_ok(*P)) n_seg = segments(0);
    }
  }
  P->n_seg = int32_t(std::min<int64_t>(std::max<int64_t>(n_seg, 1), P->units));
  const int64_t waves = int64_t(P->n_win) * P->n_seg;
  if (waves > (int64_t(1) << 30)) return DWTFRAG_ERANGE;
  P->n_waves = int32_t(waves);
  const bool last = (s == g.stages - 1);
  P->use_aes = last ? 1 : 0;
  // keystream ring: LL columns per wavefront (forward: owned, inverse: lanes)
  const int ll_cols = forward ? std::min<int>(P->wdim[L], (P->own_w >> L) + 1)
                              : std::min<int>(P->wdim[L], span >> L);
  P->ks_blocks = (2 * ll_cols + 30) / 16;
  P->ks_rows = std::max(1, 64 / P->ks_blocks);
  if (P->ks_rows * P->ks_blocks > kRingBlocks) P->ks_rows = kRingBlocks / P->ks_blocks;
  if (P->ks_rows < 1) return DWTFRAG_ERANGE;
  P->key = key;
  *L_out = L;
  *C1_out = C1;
  return DWTFRAG_OK;
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

}  // namespace

// Plan of a buffer whose levels fit one fused stage (levels <= kMaxFused).
int plan_single_stage(uint64_t n, uint32_t width, uint32_t levels, bool forward,
                      const dwtfrag_launch *launch, const AesKey &key, StageParams *P, int *L,
                      int *C1, uint64_t *priv_bytes) {
  if (levels > uint32_t(kMaxFused)) return DWTFRAG_EINVAL;
  Geometry g;
  const int rc = make_geometry(n, width, levels, &g);
  if (rc != DWTFRAG_OK) return rc;
  *priv_bytes = g.priv_bytes;
  return plan_stage(g, 0, forward, launch, key, P, L, C1, false);
}
// Forward stages of a planned geometry: validation of the buffers, key
// expansion, launch planning and the launches (workspace: g.ws_bytes bytes, or
// null when that is 0).
int protect_planned(const Geometry &g, const uint8_t *in, const uint8_t key[16],
                    const uint8_t nonce[16], uint8_t *priv, int16_t *pub, void *workspace,
                    const dwtfrag_launch *launch, void *stream) {
  if (!pub && g.pub_bytes) return DWTFRAG_EINVAL;  // pub may be NULL only when empty
  if (!aligned16(in) || !aligned16(priv) || !aligned16(pub) || (workspace && !aligned16(workspace)))
    return DWTFRAG_EINVAL;
  AesKey k;
  expand_key(key, nonce, &k);
  StageParams plans[kMaxStages];
  int Ls[kMaxStages], C1s[kMaxStages];
  for (int s = 0; s < g.stages; ++s) {
    const int rc = plan_stage(g, s, true, launch, k, &plans[s], &Ls[s], &C1s[s], true);
    if (rc != DWTFRAG_OK) return rc;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  for (int s = 0; s < g.stages; ++s) {
    const bool last = (s == g.stages - 1);
    const void *src = (s == 0) ? static_cast<const void *>(in)
                               : static_cast<const char *>(workspace) + g.ws_off[s - 1];
    int16_t *dst = last ? reinterpret_cast<int16_t *>(priv)
                        : reinterpret_cast<int16_t *>(static_cast<char *>(workspace) + g.ws_off[s]);
    if (launch_fwd(Ls[s], C1s[s], s == 0, src, pub, dst, plans[s], st) != hipSuccess)
      return DWTFRAG_EDEVICE;
  }
  return DWTFRAG_OK;
}

// Static workspace of dwtfrag_protect_noalloc: one array per device, kept
// until the process ends.  Its host-side name is not a device address; the
// device address is looked up once per device (with that device current) and
// only that address is handed to kernels.  Every call on a device shares the
// array: each stage writes every element of its LL output before the next
// stage reads it, so nothing needs clearing, and calls that overlap on one
// device race on it.
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

int device_scratch(void **out) {
  constexpr int kDev = 64;
  static std::mutex mu;
  static void *ptr[kDev] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kDev) return DWTFRAG_EDEVICE;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return DWTFRAG_EDEVICE;
    ptr[dev] = p;
  }
  *out = ptr[dev];
  return DWTFRAG_OK;
}

}  // namespace dwtfrag

using namespace dwtfrag;

extern "C" {

int dwtfrag_geometry(uint64_t n, uint32_t width, uint32_t levels, dwtfrag_geom *out) {
  if (!out) return DWTFRAG_EINVAL;
  Geometry g;
  const int rc = make_geometry(n, width, levels, &g);
  if (rc != DWTFRAG_OK) return rc;
  out->n = n;
  out->width = width;
  out->height = g.H;
  out->levels = levels;
  out->ll_h = uint32_t(g.h[levels]);
  out->ll_w = uint32_t(g.w[levels]);
  out->priv_bytes = g.priv_bytes;
  out->pub_bytes = g.pub_bytes;
  out->workspace_bytes = g.ws_bytes;
  return DWTFRAG_OK;
}

uint32_t dwtfrag_default_width(uint64_t n) {
  if (n == 0) return 0;
  uint64_t r = 1;
  while (r * r < n) r <<= 1;  // smallest power of two whose square reaches n
  // r is now the smallest power of two >= sqrt(n); that equals the smallest
  // power of two >= ceil(sqrt(n)).
  return uint32_t(std::min<uint64_t>(4096, r));
}

int dwtfrag_protect(const uint8_t *in, uint64_t n, uint32_t width, uint32_t levels,
                    const uint8_t key[16], const uint8_t nonce[16], uint8_t *priv, int16_t *pub,
                    void *workspace, uint64_t workspace_bytes, const dwtfrag_launch *launch,
                    void *stream) {
  if (!in || !key || !nonce || !priv) return DWTFRAG_EINVAL;
  Geometry g;
  int rc = make_geometry(n, width, levels, &g);
  if (rc != DWTFRAG_OK) return rc;
  if (!pub && g.pub_bytes) return DWTFRAG_EINVAL;  // pub may be NULL only when empty
  if (g.ws_bytes && (!workspace || workspace_bytes < g.ws_bytes)) return DWTFRAG_EWORKSPACE;
  return protect_planned(g, in, key, nonce, priv, pub, workspace, launch, stream);
}

int dwtfrag_protect_noalloc(const uint8_t *in, uint64_t n, uint32_t width, uint32_t levels,
                            const uint8_t key[16], const uint8_t nonce[16], uint8_t *priv,
                            int16_t *pub, const dwtfrag_launch *launch, void *stream) {
  if (!in || !key || !nonce || !priv) return DWTFRAG_EINVAL;
  Geometry g;
  int rc = make_geometry(n, width, levels, &g);
  if (rc != DWTFRAG_OK) return rc;
  if (g.ws_bytes > kScratchBytes) return DWTFRAG_ESCRATCH;
  void *ws = nullptr;
  if (g.ws_bytes) {
    rc = device_scratch(&ws);
    if (rc != DWTFRAG_OK) return rc;
  }
  return protect_planned(g, in, key, nonce, priv, pub, ws, launch, stream);
}

int dwtfrag_restore(const uint8_t *priv, const int16_t *pub, uint64_t n, uint32_t width,
                    uint32_t levels, const uint8_t key[16], const uint8_t nonce[16], uint8_t *out,
                    void *workspace, uint64_t workspace_bytes, const dwtfrag_launch *launch,
                    void *stream) {
  if (!priv || !key || !nonce || !out) return DWTFRAG_EINVAL;
  Geometry g;
  int rc = make_geometry(n, width, levels, &g);
  if (rc != DWTFRAG_OK) return rc;
  if (!pub && g.pub_bytes) return DWTFRAG_EINVAL;  // pub may be NULL only when empty
  if (g.ws_bytes && (!workspace || workspace_bytes < g.ws_bytes)) return DWTFRAG_EWORKSPACE;
  if (!aligned16(out) || !aligned16(priv) || !aligned16(pub) || (workspace && !aligned16(workspace)))
    return DWTFRAG_EINVAL;
  AesKey k;
  expand_key(key, nonce, &k);
  StageParams plans[kMaxStages];
  int Ls[kMaxStages], C1s[kMaxStages];
  for (int s = 0; s < g.stages; ++s) {
    rc = plan_stage(g, s, false, launch, k, &plans[s], &Ls[s], &C1s[s], true);
    if (rc != DWTFRAG_OK) return rc;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  for (int s = g.stages - 1; s >= 0; --s) {
    const bool last = (s == g.stages - 1);
    const int16_t *src = last ? reinterpret_cast<const int16_t *>(priv)
                              : reinterpret_cast<const int16_t *>(
                                    static_cast<const char *>(workspace) + g.ws_off[s]);
    void *dst = (s == 0) ? static_cast<void *>(out)
                         : static_cast<void *>(static_cast<char *>(workspace) + g.ws_off[s - 1]);
    if (launch_inv(Ls[s], C1s[s], s == 0, src, pub, dst, plans[s], st) != hipSuccess)
      return DWTFRAG_EDEVICE;
  }
  return DWTFRAG_OK;
}

int dwtfrag_aes128_ctr(const uint8_t *in, uint8_t *out, uint64_t nbytes, const uint8_t key[16],
                       const uint8_t nonce[16], uint64_t first_block, void *stream) {
  if (!in || !out || !key || !nonce || nbytes == 0) return DWTFRAG_EINVAL;
  AesKey k;
  expand_key(key, nonce, &k);
  if (launch_ctr(in, out, nbytes, k, first_block, static_cast<hipStream_t>(stream)) != hipSuccess)
    return DWTFRAG_EDEVICE;
  return DWTFRAG_OK;
}

int dwtfrag_autotune(const uint8_t *in, uint64_t n, uint32_t width, uint32_t levels,
                     void *scratch, uint64_t scratch_bytes, uint32_t trials,
                     dwtfrag_launch *best, float *best_us, void *stream) {
  if (!in || !scratch || !best || trials == 0) return DWTFRAG_EINVAL;
  Geometry g;
  int rc = make_geometry(n, width, levels, &g);
  if (rc != DWTFRAG_OK) return rc;
  const uint64_t o_pub = align256(g.priv_bytes);
  const uint64_t o_out = o_pub + align256(g.pub_bytes);
  const uint64_t o_ws = o_out + align256(n);
  if (scratch_bytes < o_ws + g.ws_bytes || (reinterpret_cast<uintptr_t>(scratch) & 255))
    return DWTFRAG_EWORKSPACE;
  char *base = static_cast<char *>(scratch);
  uint8_t *priv = reinterpret_cast<uint8_t *>(base);
  int16_t *pub = g.pub_bytes ? reinterpret_cast<int16_t *>(base + o_pub) : nullptr;
  uint8_t *out = reinterpret_cast<uint8_t *>(base + o_out);
  void *ws = g.ws_bytes ? base + o_ws : nullptr;
  const uint8_t key[16] = {0}, nonce[16] = {0};
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return DWTFRAG_EDEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return DWTFRAG_EDEVICE;
  }
  float best_t = -1.0f;
  dwtfrag_launch best_l{0, 0};
  const uint32_t rows[] = {0, 64, 128, 256};
  const uint32_t cols[] = {8, 16};
  rc = DWTFRAG_OK;
  for (uint32_t c : cols) {
    if (levels % kMaxFused == 0 && c == 8) continue;  // a four-level stage needs 16 columns
    for (uint32_t r : rows) {
      const dwtfrag_launch ln{r, c};
      // one untimed pair, then `trials` timed pairs; the first failing call's
      // code is returned
      auto pair = [&]() {
        const int r = dwtfrag_protect(in, n, width, levels, key, nonce, priv, pub, ws, g.ws_bytes, &ln, st);
        return r != DWTFRAG_OK ? r
                               : dwtfrag_restore(priv, pub, n, width, levels, key, nonce, out, ws,
                                                 g.ws_bytes, &ln, st);
      };
      rc = pair();
      if (rc != DWTFRAG_OK) break;
      if (hipEventRecord(e0, st) != hipSuccess) {
        rc = DWTFRAG_EDEVICE;
        break;
      }
      for (uint32_t t = 0; t < trials && rc == DWTFRAG_OK; ++t) rc = pair();
      if (rc != DWTFRAG_OK) break;
      float ms = 0.0f;
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        rc = DWTFRAG_EDEVICE;
        break;
      }
      const float us = 1000.0f * ms / float(trials);
      if (best_t < 0.0f || us < best_t) {
        best_t = us;
        best_l = ln;
      }
    }
    if (rc != DWTFRAG_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != DWTFRAG_OK) return rc;
  *best = best_l;
  if (best_us) *best_us = best_t;
  return DWTFRAG_OK;
}

const char *dwtfrag_strerror(int code) {
  switch (code) {
    case DWTFRAG_OK: return "ok";
    case DWTFRAG_EINVAL: return "invalid argument (null or misaligned pointer, zero size, bad levels or launch shape)";
    case DWTFRAG_ERANGE: return "geometry out of range";
    case DWTFRAG_EDEVICE: return "HIP runtime or launch error";
    case DWTFRAG_EWORKSPACE: return "workspace missing or too small";
    case DWTFRAG_ESCRATCH: return "the transform needs more workspace than the library's 16 MiB static buffer holds";
    default: return "unknown status";
  }
}

}  // extern "C"
