// Batches of independent buffers: host planning and the C ABI.
//
// The thesis cuts data into many fixed-size chunks (Ch. 5 section 5.2.1) and
// its GPU runs take many chunks per call.  Here a batch is planned once on the
// host (every item's geometry and launch plan with 16 columns per lane, and
// one tile list per direction, longest tiles first), copied into a
// caller-owned device buffer, and then run by one persistent launch per
// direction that drains the direction's queue: protect = the forward drain
// (encryption fused), restore = the inverse drain (decryption fused).  The
// kernels reset their own queue counters when they finish, so a direction is
// one kernel launch and can be captured in a HIP graph.
#include "dwtfrag.h"

#include <algorithm>
#include <atomic>
#include <cstring>
#include <new>
#include <vector>

#include "batch.h"

namespace dwtfrag {

hipError_t launch_fwd_batch(const BatchItem *items, const int2 *tiles, int64_t n_tiles,
                            BatchCounters *ctr, int blocks, hipStream_t s);
hipError_t launch_inv_batch(const BatchItem *items, const int2 *tiles, int64_t n_tiles,
                            BatchCounters *ctr, int blocks, hipStream_t s);
int fwd_batch_blocks_per_cu();
int inv_batch_blocks_per_cu();
int plan_single_stage(uint64_t n, uint32_t width, uint32_t levels, bool forward,
                      const dwtfrag_launch *launch, const AesKey &key, StageParams *P, int *L,
                      int *C1, uint64_t *priv_bytes);

}  // namespace dwtfrag

using namespace dwtfrag;

struct dwtfrag_batch {
  uint32_t count = 0;
  std::vector<BatchItem> items;
  std::vector<int2> tiles;                 // forward queue, then inverse queue
  int64_t n_fwd = 0, n_inv = 0;            // tiles per direction
  int fwd_blocks = 0, inv_blocks = 0;      // persistent grid per direction
  uint64_t off_ctr = 0, off_items = 0, off_tiles = 0, bytes = 0;
  char *dev = nullptr;                     // caller's device copy, set by upload
  hipEvent_t uploaded = nullptr;           // the last upload's copies are done
};

namespace {

uint64_t a256(uint64_t v) { return (v + 255) & ~uint64_t(255); }

const dwtfrag_launch *tuned_launch(const dwtfrag_tune_entry *tune, uint32_t n_tune, uint32_t width,
                                   uint32_t levels) {
  for (uint32_t i = 0; i < n_tune; ++i)
    if (tune[i].width == width && tune[i].levels == levels) return &tune[i].launch;
  return nullptr;
}

// Persistent grid of a batch kernel: resident workgroups per CU x CUs.
int persistent_blocks(int per_cu) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    cus = 256;
  return cus * std::max(1, per_cu);
}

}  // namespace

extern "C" {

int dwtfrag_batch_create(const dwtfrag_item *items, uint32_t count, const dwtfrag_tune_entry *tune,
                         uint32_t n_tune, dwtfrag_batch **out) {
  if (!out) return DWTFRAG_EINVAL;
  *out = nullptr;
  if (!items || count == 0 || count > (1u << 30) || (n_tune && !tune)) return DWTFRAG_EINVAL;
  dwtfrag_batch *b = new (std::nothrow) dwtfrag_batch();
  if (!b) return DWTFRAG_ERANGE;
  b->count = count;
  b->items.resize(count);
  // tiles (item, wavefront) of every item, one list per direction
  std::vector<int2> ft, it;
  for (uint32_t i = 0; i < count; ++i) {
    const dwtfrag_item &src = items[i];
    if (!src.in || !src.priv || src.levels == 0 || src.levels > uint32_t(kMaxFused)) {
      delete b;
      return DWTFRAG_EINVAL;
    }
    const auto al16 = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
    if (!al16(src.in) || !al16(src.priv) || !al16(src.pub) || !al16(src.out)) {
      delete b;
      return DWTFRAG_EINVAL;
    }
    // batches fill the device with many items: 128-row tiles unless tuned;
    // every tile has kBatchCols columns per lane (one kernel serves all depths)
    const dwtfrag_launch *tl = tuned_launch(tune, n_tune, src.width, src.levels);
    if (tl && tl->lane_cols != 0 && tl->lane_cols != 8 && tl->lane_cols != 16) {
      delete b;
      return DWTFRAG_EINVAL;
    }
    const dwtfrag_launch ln{tl && tl->seg_rows ? tl->seg_rows : 128u, uint32_t(kBatchCols)};
    AesKey key;
    expand_key(src.key, src.nonce, &key);
    BatchItem &bi = b->items[i];
    std::memset(&bi, 0, sizeof(bi));
    int Lf = 0, Cf = 0, Li = 0, Ci = 0;
    uint64_t priv_bytes = 0;
    int rc = plan_single_stage(src.n, src.width, src.levels, true, &ln, key, &bi.fwd, &Lf, &Cf, &priv_bytes);
    if (rc == DWTFRAG_OK)
      rc = plan_single_stage(src.n, src.width, src.levels, false, &ln, key, &bi.inv, &Li, &Ci, &priv_bytes);
    if (rc != DWTFRAG_OK) {
      delete b;
      return rc;
    }
    const uint64_t pub_bytes = 2 * (uint64_t(bi.fwd.H) * bi.fwd.W) - priv_bytes;
    if (pub_bytes && !src.pub) {
      delete b;
      return DWTFRAG_EINVAL;
    }
    bi.in = src.in;
    bi.priv = src.priv;
    bi.pub = src.pub;
    bi.out = src.out;
    bi.priv_bytes = priv_bytes;
    bi.levels = int32_t(src.levels);
    for (int w = 0; w < bi.fwd.n_waves; ++w) ft.push_back(make_int2(int(i), w));
    for (int w = 0; w < bi.inv.n_waves; ++w) it.push_back(make_int2(int(i), w));
  }
  // Longest tiles first, so the short tiles of small items fill the end of a
  // drain instead of extending it.  A tile's cost is the rows it streams
  // (segment plus halos) times the columns of its window.
  const auto tile_cost = [](const StageParams &P) {
    const int64_t seg = int64_t(P.unit_rows) * ((P.units + P.n_seg - 1) / P.n_seg);
    return std::min<int64_t>(P.H, seg + P.halo_t + P.halo_b) * std::min(P.W, P.own_w);
  };
  std::vector<int64_t> fcost(count), icost(count);
  for (uint32_t i = 0; i < count; ++i) {
    fcost[i] = tile_cost(b->items[i].fwd);
    icost[i] = tile_cost(b->items[i].inv);
  }
  std::stable_sort(ft.begin(), ft.end(), [&](const int2 &x, const int2 &y) { return fcost[x.x] > fcost[y.x]; });
  std::stable_sort(it.begin(), it.end(), [&](const int2 &x, const int2 &y) { return icost[x.x] > icost[y.x]; });
  if (ft.size() + it.size() > 0x7fffffffull) {
    delete b;
    return DWTFRAG_ERANGE;
  }
  b->n_fwd = int64_t(ft.size());
  b->n_inv = int64_t(it.size());
  b->tiles = std::move(ft);
  b->tiles.insert(b->tiles.end(), it.begin(), it.end());
  b->fwd_blocks = persistent_blocks(fwd_batch_blocks_per_cu());
  b->inv_blocks = persistent_blocks(inv_batch_blocks_per_cu());
  b->off_ctr = 0;
  b->off_items = a256(2 * sizeof(BatchCounters));
  b->off_tiles = a256(b->off_items + count * sizeof(BatchItem));
  b->bytes = a256(b->off_tiles + b->tiles.size() * sizeof(int2));
  *out = b;
  return DWTFRAG_OK;
}

uint64_t dwtfrag_batch_device_bytes(const dwtfrag_batch *b) { return b ? b->bytes : 0; }

int dwtfrag_batch_upload(dwtfrag_batch *b, void *device_plan, uint64_t device_bytes, void *stream) {
  if (!b || !device_plan || (reinterpret_cast<uintptr_t>(device_plan) & 255)) return DWTFRAG_EINVAL;
  if (device_bytes < b->bytes) return DWTFRAG_EWORKSPACE;
  char *dev = static_cast<char *>(device_plan);
  hipStream_t st = static_cast<hipStream_t>(stream);
  // The copies run asynchronously on the stream: their sources (the zero
  // counters below, the plan's own tables) stay in place until
  // dwtfrag_batch_destroy, which waits for the event recorded behind them.
  // The queue counters start at zero (the kernels leave them at zero).
  static const BatchCounters zero[2] = {};
  if (hipMemcpyAsync(dev + b->off_ctr, zero, sizeof(zero), hipMemcpyHostToDevice, st) != hipSuccess)
    return DWTFRAG_EDEVICE;
  if (hipMemcpyAsync(dev + b->off_items, b->items.data(), b->items.size() * sizeof(BatchItem),
                     hipMemcpyHostToDevice, st) != hipSuccess)
    return DWTFRAG_EDEVICE;
  if (!b->tiles.empty() &&
      hipMemcpyAsync(dev + b->off_tiles, b->tiles.data(), b->tiles.size() * sizeof(int2),
                     hipMemcpyHostToDevice, st) != hipSuccess)
    return DWTFRAG_EDEVICE;
  if (!b->uploaded && hipEventCreateWithFlags(&b->uploaded, hipEventDisableTiming) != hipSuccess) {
    b->uploaded = nullptr;
    return DWTFRAG_EDEVICE;
  }
  if (hipEventRecord(b->uploaded, st) != hipSuccess) return DWTFRAG_EDEVICE;
  b->dev = dev;
  return DWTFRAG_OK;
}

int dwtfrag_batch_protect(const dwtfrag_batch *b, void *stream) {
  if (!b || !b->dev) return DWTFRAG_EINVAL;
  if (b->n_fwd == 0) return DWTFRAG_OK;
  BatchCounters *ctr = reinterpret_cast<BatchCounters *>(b->dev + b->off_ctr);
  const BatchItem *items = reinterpret_cast<const BatchItem *>(b->dev + b->off_items);
  const int2 *tiles = reinterpret_cast<const int2 *>(b->dev + b->off_tiles);
  const int blocks = int(std::min<int64_t>(b->fwd_blocks, (b->n_fwd + kWavesPerBlock - 1) / kWavesPerBlock));
  if (launch_fwd_batch(items, tiles, b->n_fwd, ctr, blocks, static_cast<hipStream_t>(stream)) != hipSuccess)
    return DWTFRAG_EDEVICE;
  return DWTFRAG_OK;
}

int dwtfrag_batch_restore(const dwtfrag_batch *b, void *stream) {
  if (!b || !b->dev) return DWTFRAG_EINVAL;
  for (const BatchItem &i : b->items)
    if (!i.out) return DWTFRAG_EINVAL;
  if (b->n_inv == 0) return DWTFRAG_OK;
  BatchCounters *ctr = reinterpret_cast<BatchCounters *>(b->dev + b->off_ctr) + 1;
  const BatchItem *items = reinterpret_cast<const BatchItem *>(b->dev + b->off_items);
  const int2 *tiles = reinterpret_cast<const int2 *>(b->dev + b->off_tiles) + b->n_fwd;
  const int blocks = int(std::min<int64_t>(b->inv_blocks, (b->n_inv + kWavesPerBlock - 1) / kWavesPerBlock));
  if (launch_inv_batch(items, tiles, b->n_inv, ctr, blocks, static_cast<hipStream_t>(stream)) != hipSuccess)
    return DWTFRAG_EDEVICE;
  return DWTFRAG_OK;
}

void dwtfrag_batch_destroy(dwtfrag_batch *b) {
  if (!b) return;
  if (b->uploaded) {  // the copies read the plan's tables until then
    hipEventSynchronize(b->uploaded);
    hipEventDestroy(b->uploaded);
  }
  delete b;
}

}  // extern "C"
