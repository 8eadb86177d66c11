// Device-side tables of a batch of independent buffers (protect / restore of
// many chunks in one go: the thesis cuts data into many equal chunks, Ch. 5
// section 5.2.1, and its GPU runs take many chunks as input).
//
// Each buffer ("item") is one fused stage (levels <= 4).  Items are grouped
// into classes of equal kernel shape (levels, columns per lane); a class's
// tiles (item, wavefront index within the item) form one queue that a
// persistent launch drains with an atomic head counter, so uneven buffers
// share the device without a tail per buffer.
#pragma once

#include "common.h"

namespace dwtfrag {

struct BatchItem {
  StageParams fwd;     // forward plan (halo shape of the forward kernel)
  StageParams inv;     // inverse plan
  const uint8_t *in;   // protect input (device)
  uint8_t *priv;       // private fragment (device)
  int16_t *pub;        // public fragment (device)
  uint8_t *out;        // restore output (device)
  uint64_t priv_bytes; // 2 * h_L * w_L
};

// Tile queue head counters, reset by a kernel before every drain: one per
// class and direction.
constexpr int kBatchClasses = 8;

struct BatchClass {
  int L, C1;
  int64_t n_tiles;
  int64_t tile_off;    // first tile of the class in the tile array
};

}  // namespace dwtfrag
