// Device-side tables of a batch of independent buffers (protect / restore of
// many chunks in one go: the thesis cuts data into many equal chunks, Ch. 5
// section 5.2.1, and its GPU runs take many chunks as input).
//
// Each buffer ("item") is one fused stage (levels <= 4) planned with 16
// columns per lane, the layout every depth up to four levels can use, so one
// kernel per direction serves all items: its tiles (item, wavefront index
// within the item) form a single queue, longest first, that one persistent
// launch drains with an atomic head counter, dispatching each tile on its
// item's depth.  The last workgroup to finish resets the counters, so a
// batch direction is exactly one kernel launch.
#pragma once

#include "common.h"

namespace dwtfrag {

// Columns per lane of every batch tile.
constexpr int kBatchCols = 16;

struct BatchItem {
  StageParams fwd;     // forward plan (halo shape of the forward kernel)
  StageParams inv;     // inverse plan
  const uint8_t *in;   // protect input (device)
  uint8_t *priv;       // private fragment (device)
  int16_t *pub;        // public fragment (device)
  uint8_t *out;        // restore output (device)
  uint64_t priv_bytes; // 2 * h_L * w_L
  int32_t levels;      // 1..4
  int32_t pad;
};

// Queue counters of one direction: [0] next tile, [1] finished workgroups.
struct BatchCounters {
  unsigned int head, done;
};

// Called by every workgroup once its wavefronts have left the tile loop: the
// last one resets both counters for the next launch (no other workgroup pops
// a tile any more at that point).
__device__ __forceinline__ void batch_finish(BatchCounters *c) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned int d = atomicAdd(&c->done, 1u);
    if (d == gridDim.x - 1) {
      atomicExch(&c->head, 0u);
      atomicExch(&c->done, 0u);
    }
  }
}

}  // namespace dwtfrag
