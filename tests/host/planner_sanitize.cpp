// Host-only check of the library's planning code under AddressSanitizer and
// UndefinedBehaviorSanitizer: geometry, stage and launch planning, batch
// planning, and the argument checks of every entry point, over extreme
// sizes, widths and depths.  Built from api.hip, batch.hip and se8.hip for
// the host only (no device code); the kernel launchers of the other sources
// are replaced below by stubs that report a failed launch, so every call
// runs its planning and returns before touching memory.  No GPU is needed.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "dwtfrag.h"
#include "batch.h"

namespace dwtfrag {
hipError_t launch_fwd(int, int, bool, const void *, int16_t *, int16_t *, const StageParams &,
                      hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_inv(int, int, bool, const int16_t *, const int16_t *, void *,
                      const StageParams &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_ctr(const uint8_t *, uint8_t *, uint64_t, const AesKey &, uint64_t,
                      hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_fwd_batch(const BatchItem *, const int2 *, int64_t, BatchCounters *, int,
                            hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_inv_batch(const BatchItem *, const int2 *, int64_t, BatchCounters *, int,
                            hipStream_t) { return hipErrorInvalidValue; }
int fwd_waves_per_cu(int L, int C1, bool) { return C1 == 16 ? 8 : 12 + L % 2; }
int inv_waves_per_cu(int L, int C1, bool) { return C1 == 16 ? 8 : 16 - L % 2; }
int inv_split_waves_per_cu(int L, int C1, bool all_fast) { return C1 == 16 ? 12 - !all_fast : 16 - L % 2; }
bool inv_stage_split_ok(const StageParams &P) { return P.n_valid >= (int64_t(1) << 24) && P.n_seg > 1; }
bool inv_stage_all_fast(const StageParams &P, int, int C1) { return P.W % C1 == 0; }
int fwd_batch_blocks_per_cu() { return 2; }
int inv_batch_blocks_per_cu() { return 2; }
}  // namespace dwtfrag

static int failures = 0;
#define EXPECT(cond)                                                     \
  do {                                                                   \
    if (!(cond)) {                                                       \
      std::fprintf(stderr, "%s:%d: expected %s\n", __FILE__, __LINE__, #cond); \
      ++failures;                                                        \
    }                                                                    \
  } while (0)

int main() {
  const uint8_t key[16] = {1}, nonce[16] = {2};
  // fake, 256-byte aligned device pointers: every call below returns before
  // any access (planning ends in a stubbed launch, or the arguments fail)
  uint8_t *fp = reinterpret_cast<uint8_t *>(uintptr_t(1) << 20);
  int16_t *fq = reinterpret_cast<int16_t *>(uintptr_t(1) << 21);
  const uint64_t lim = 0x7FFF0000ull;
  const uint64_t ns[] = {1, 2, 3, 7, 64, 4097, 100003, uint64_t(1) << 28, (uint64_t(1) << 31) + 5,
                         uint64_t(1) << 36, lim * 3, lim * lim, uint64_t(1) << 62};
  const uint32_t widths[] = {1, 2, 3, 8, 317, 512, 4096, 32768, 1u << 20, uint32_t(lim),
                             uint32_t(lim) + 1, 0xFFFFFFFFu};
  const uint32_t levels[] = {1, 2, 3, 4, 5, 8, 9, 16, 31, 32};
  const dwtfrag_launch shapes[] = {{0, 0}, {0, 16}, {1, 8}, {64, 8}, {1000000, 16}, {0xFFFFFFFFu, 0}};
  long planned = 0, reached_launch = 0;
  for (uint64_t n : ns)
    for (uint32_t w : widths)
      for (uint32_t L : levels) {
        dwtfrag_geom g;
        const int rc = dwtfrag_geometry(n, w, L, &g);
        if (rc != DWTFRAG_OK) {
          EXPECT(rc == DWTFRAG_ERANGE || rc == DWTFRAG_EINVAL);
          continue;
        }
        EXPECT(g.height == (n + w - 1) / w);
        EXPECT(g.priv_bytes + g.pub_bytes == 2 * uint64_t(g.height) * w);
        for (const dwtfrag_launch &ln : shapes) {
          const int p = dwtfrag_protect(fp, n, w, L, key, nonce, fp, fq, fp, g.workspace_bytes, &ln,
                                        nullptr);
          EXPECT(p == DWTFRAG_EDEVICE || p == DWTFRAG_ERANGE || p == DWTFRAG_EINVAL);
          reached_launch += (p == DWTFRAG_EDEVICE);
          const int r = dwtfrag_restore(fp, fq, n, w, L, key, nonce, fp, fp, g.workspace_bytes,
                                        &ln, nullptr);
          EXPECT(r == DWTFRAG_EDEVICE || r == DWTFRAG_ERANGE || r == DWTFRAG_EINVAL);
          const int a = dwtfrag_protect_noalloc(fp, n, w, L, key, nonce, fp, fq, &ln, nullptr);
          EXPECT(a == DWTFRAG_EDEVICE || a == DWTFRAG_ERANGE || a == DWTFRAG_EINVAL ||
                 a == DWTFRAG_ESCRATCH);
          ++planned;
        }
        dwtfrag_se8_geom s;
        (void)dwtfrag_se8_geometry(n, w, &s);
      }
  // batches: many items of extreme shapes, tuned and default tiles
  std::vector<dwtfrag_item> items;
  for (uint64_t n : {uint64_t(1), uint64_t(4096), uint64_t(100003), uint64_t(1) << 26,
                     uint64_t(3) << 30})
    for (uint32_t L = 1; L <= 4; ++L) {
      dwtfrag_item it{};
      it.in = fp;
      it.out = fp;
      it.priv = fp;
      it.pub = fq;
      it.n = n;
      it.width = dwtfrag_default_width(n);
      it.levels = L;
      items.push_back(it);
    }
  const dwtfrag_tune_entry tune[] = {{4096, 3, {256, 16}}, {1, 1, {1, 8}}, {64, 4, {64, 16}}};
  dwtfrag_batch *b = nullptr;
  EXPECT(dwtfrag_batch_create(items.data(), uint32_t(items.size()), tune, 3, &b) == DWTFRAG_OK);
  EXPECT(b && dwtfrag_batch_device_bytes(b) > 0);
  EXPECT(dwtfrag_batch_protect(b, nullptr) == DWTFRAG_EINVAL);  // not uploaded
  EXPECT(dwtfrag_batch_restore(b, nullptr) == DWTFRAG_EINVAL);
  dwtfrag_batch_destroy(b);
  items[3].levels = 5;
  EXPECT(dwtfrag_batch_create(items.data(), uint32_t(items.size()), nullptr, 0, &b) == DWTFRAG_EINVAL);
  EXPECT(b == nullptr);
  // most geometries are in range: their planning ran to the (stubbed) launch
  EXPECT(reached_launch > planned / 4);
  std::printf("planned %ld calls, %ld reached the launch, %d failures\n", planned, reached_launch,
              failures);
  return failures ? 1 : 0;
}
