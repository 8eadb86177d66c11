// Batches of independent buffers: host planning and the C ABI.
//
// The thesis cuts data into many fixed-size chunks (Ch. 5 section 5.2.1) and
// its GPU runs take many chunks per call.  Here a batch is planned once on the
// host (every item's geometry and launch plan, grouped into classes of equal
// kernel shape, with one tile list per class), copied into a caller-owned
// device buffer, and then run by persistent launches that drain each class's
// tile queue: protect = forward drains (encryption fused), restore = inverse
// drains (decryption fused).  The run calls launch kernels only, so they can
// be captured in a HIP graph.
#include "dwtfrag.h"

#include <algorithm>
#include <atomic>
#include <cstring>
#include <new>
#include <vector>

#include "batch.h"

namespace dwtfrag {

hipError_t launch_fwd_batch(int L, int C1, const BatchItem *items, const int2 *tiles, int64_t n_tiles,
                            unsigned int *head, int blocks, hipStream_t s);
hipError_t launch_inv_batch(int L, int C1, const BatchItem *items, const int2 *tiles, int64_t n_tiles,
                            unsigned int *head, int blocks, hipStream_t s);
int fwd_waves_per_cu(int L, int C1, bool u8in);
int inv_waves_per_cu(int L, int C1, bool u8out);
int plan_single_stage(uint64_t n, uint32_t width, uint32_t levels, bool forward,
                      const dwtfrag_launch *launch, const AesKey &key, StageParams *P, int *L,
                      int *C1, uint64_t *priv_bytes);

__global__ void reset_heads_kernel(unsigned int *heads, int n) {
  const int i = int(threadIdx.x);
  if (i < n) heads[i] = 0u;
}

}  // namespace dwtfrag

using namespace dwtfrag;

struct dwtfrag_batch {
  uint32_t count = 0;
  std::vector<BatchItem> items;
  std::vector<int2> tiles;                 // forward classes, then inverse classes
  std::vector<BatchClass> fwd_cls, inv_cls;
  std::vector<int> fwd_blocks, inv_blocks; // persistent grid per class
  uint64_t off_items = 0, off_tiles = 0, off_heads = 0, bytes = 0;
  char *dev = nullptr;                     // caller's device copy, set by upload
};

namespace {

uint64_t a256(uint64_t v) { return (v + 255) & ~uint64_t(255); }

const dwtfrag_launch *tuned_launch(const dwtfrag_tune_entry *tune, uint32_t n_tune, uint32_t width,
                                   uint32_t levels) {
  for (uint32_t i = 0; i < n_tune; ++i)
    if (tune[i].width == width && tune[i].levels == levels) return &tune[i].launch;
  return nullptr;
}

int class_index(std::vector<BatchClass> &cls, int L, int C1) {
  for (size_t i = 0; i < cls.size(); ++i)
    if (cls[i].L == L && cls[i].C1 == C1) return int(i);
  cls.push_back(BatchClass{L, C1, 0, 0});
  return int(cls.size()) - 1;
}

int persistent_blocks(bool forward, int L, int C1) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    cus = 256;
  const int per_cu = forward ? fwd_waves_per_cu(L, C1, true) : inv_waves_per_cu(L, C1, true);
  return cus * std::max(1, per_cu / kWavesPerBlock);
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
  // per class: tiles (item, wavefront) of every member item, in item order
  std::vector<std::vector<int2>> ft, it;
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
    dwtfrag_launch def{128, 0};  // batches fill the device with many items: 128-row tiles
    const dwtfrag_launch *ln = tuned_launch(tune, n_tune, src.width, src.levels);
    if (!ln) ln = &def;
    AesKey key;
    expand_key(src.key, src.nonce, &key);
    BatchItem &bi = b->items[i];
    std::memset(&bi, 0, sizeof(bi));
    int Lf = 0, Cf = 0, Li = 0, Ci = 0;
    uint64_t priv_bytes = 0;
    int rc = plan_single_stage(src.n, src.width, src.levels, true, ln, key, &bi.fwd, &Lf, &Cf, &priv_bytes);
    if (rc == DWTFRAG_OK)
      rc = plan_single_stage(src.n, src.width, src.levels, false, ln, key, &bi.inv, &Li, &Ci, &priv_bytes);
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
    const int cf = class_index(b->fwd_cls, Lf, Cf);
    const int ci = class_index(b->inv_cls, Li, Ci);
    if (int(b->fwd_cls.size()) > kBatchClasses || int(b->inv_cls.size()) > kBatchClasses) {
      delete b;
      return DWTFRAG_ERANGE;
    }
    ft.resize(b->fwd_cls.size());
    it.resize(b->inv_cls.size());
    for (int w = 0; w < bi.fwd.n_waves; ++w) ft[cf].push_back(make_int2(int(i), w));
    for (int w = 0; w < bi.inv.n_waves; ++w) it[ci].push_back(make_int2(int(i), w));
  }
  // Longest tiles first within a queue, so the short tiles of small items
  // fill the end of a drain instead of extending it.  A tile's cost is the
  // rows it streams (segment plus halos) times the columns of its window.
  const auto tile_cost = [](const StageParams &P) {
    const int64_t seg = int64_t(P.unit_rows) * ((P.units + P.n_seg - 1) / P.n_seg);
    return std::min<int64_t>(P.H, seg + P.halo_t + P.halo_b) * std::min(P.W, P.own_w);
  };
  std::vector<int64_t> fcost(count), icost(count);
  for (uint32_t i = 0; i < count; ++i) {
    fcost[i] = tile_cost(b->items[i].fwd);
    icost[i] = tile_cost(b->items[i].inv);
  }
  for (auto &v : ft)
    std::stable_sort(v.begin(), v.end(), [&](const int2 &x, const int2 &y) { return fcost[x.x] > fcost[y.x]; });
  for (auto &v : it)
    std::stable_sort(v.begin(), v.end(), [&](const int2 &x, const int2 &y) { return icost[x.x] > icost[y.x]; });
  for (size_t c = 0; c < b->fwd_cls.size(); ++c) {
    b->fwd_cls[c].tile_off = int64_t(b->tiles.size());
    b->fwd_cls[c].n_tiles = int64_t(ft[c].size());
    b->tiles.insert(b->tiles.end(), ft[c].begin(), ft[c].end());
    b->fwd_blocks.push_back(persistent_blocks(true, b->fwd_cls[c].L, b->fwd_cls[c].C1));
  }
  for (size_t c = 0; c < b->inv_cls.size(); ++c) {
    b->inv_cls[c].tile_off = int64_t(b->tiles.size());
    b->inv_cls[c].n_tiles = int64_t(it[c].size());
    b->tiles.insert(b->tiles.end(), it[c].begin(), it[c].end());
    b->inv_blocks.push_back(persistent_blocks(false, b->inv_cls[c].L, b->inv_cls[c].C1));
  }
  if (b->tiles.size() > 0x7fffffffull) {
    delete b;
    return DWTFRAG_ERANGE;
  }
  b->off_heads = 0;
  b->off_items = a256(2 * kBatchClasses * sizeof(unsigned int));
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
  // pageable sources: the copies are staged before the calls return
  if (hipMemcpyAsync(dev + b->off_items, b->items.data(), b->items.size() * sizeof(BatchItem),
                     hipMemcpyHostToDevice, st) != hipSuccess)
    return DWTFRAG_EDEVICE;
  if (!b->tiles.empty() &&
      hipMemcpyAsync(dev + b->off_tiles, b->tiles.data(), b->tiles.size() * sizeof(int2),
                     hipMemcpyHostToDevice, st) != hipSuccess)
    return DWTFRAG_EDEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return DWTFRAG_EDEVICE;
  b->dev = dev;
  return DWTFRAG_OK;
}

int dwtfrag_batch_protect(const dwtfrag_batch *b, void *stream) {
  if (!b || !b->dev) return DWTFRAG_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  unsigned int *heads = reinterpret_cast<unsigned int *>(b->dev + b->off_heads);
  const BatchItem *items = reinterpret_cast<const BatchItem *>(b->dev + b->off_items);
  const int2 *tiles = reinterpret_cast<const int2 *>(b->dev + b->off_tiles);
  hipLaunchKernelGGL(reset_heads_kernel, dim3(1), dim3(64), 0, st, heads, 2 * kBatchClasses);
  if (hipGetLastError() != hipSuccess) return DWTFRAG_EDEVICE;
  for (size_t c = 0; c < b->fwd_cls.size(); ++c) {
    const BatchClass &k = b->fwd_cls[c];
    if (k.n_tiles == 0) continue;
    const int blocks = int(std::min<int64_t>(b->fwd_blocks[c], (k.n_tiles + kWavesPerBlock - 1) / kWavesPerBlock));
    if (launch_fwd_batch(k.L, k.C1, items, tiles + k.tile_off, k.n_tiles, heads + c, blocks, st) != hipSuccess)
      return DWTFRAG_EDEVICE;
  }
  return DWTFRAG_OK;
}

int dwtfrag_batch_restore(const dwtfrag_batch *b, void *stream) {
  if (!b || !b->dev) return DWTFRAG_EINVAL;
  for (const BatchItem &i : b->items)
    if (!i.out) return DWTFRAG_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  unsigned int *heads = reinterpret_cast<unsigned int *>(b->dev + b->off_heads);
  const BatchItem *items = reinterpret_cast<const BatchItem *>(b->dev + b->off_items);
  const int2 *tiles = reinterpret_cast<const int2 *>(b->dev + b->off_tiles);
  hipLaunchKernelGGL(reset_heads_kernel, dim3(1), dim3(64), 0, st, heads, 2 * kBatchClasses);
  if (hipGetLastError() != hipSuccess) return DWTFRAG_EDEVICE;
  for (size_t c = 0; c < b->inv_cls.size(); ++c) {
    const BatchClass &k = b->inv_cls[c];
    if (k.n_tiles == 0) continue;
    const int blocks = int(std::min<int64_t>(b->inv_blocks[c], (k.n_tiles + kWavesPerBlock - 1) / kWavesPerBlock));
    if (launch_inv_batch(k.L, k.C1, items, tiles + k.tile_off, k.n_tiles, heads + kBatchClasses + c,
                         blocks, st) != hipSuccess)
      return DWTFRAG_EDEVICE;
  }
  return DWTFRAG_OK;
}

void dwtfrag_batch_destroy(dwtfrag_batch *b) { delete b; }

}  // extern "C"
