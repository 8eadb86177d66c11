/*
 * dwtfrag: DWT fragmentation protect / restore on one MI355X (gfx950).
 *
 * Method (Qiu Han, "An Efficient Data Protection Architecture Based on
 * Fragmentation and Encryption", arXiv 1803.04880):
 *   - Ch. 5 section 5.2.1: any byte buffer is viewed as a 2-D matrix of bytes.
 *   - Ch. 5 section 5.1.1, eqs. (5.1)-(5.2): integer LeGall 5/3 lifting,
 *     horizontal pass then vertical pass, dyadic levels on LL.  The update
 *     step adds its floored term and the signal is extended whole-sample
 *     symmetrically at every level (both fixed by matrix A and F(4,4) of
 *     section 5.2.2.2).
 *   - Ch. 5 sections 5.1.1 / 5.2.1 and Ch. 2 "Our SE approach": the last LL
 *     band is the private fragment, encrypted with AES-128; the detail bands
 *     are the public fragment.  Ch. 2 "Performance issue of SE" names counter
 *     mode as the parallel AES mode; Ch. 5 "Cryptanalysis Discussion" suggests
 *     a per-chunk IV, which is the nonce here.
 *   - Ch. 5 section 5.2.3: the map is integer-to-integer and invertible, so
 *     restore is exact.
 *
 * Data layout (all multi-byte values little-endian):
 *   view      H = ceil(n / width) rows of `width` bytes, row-major; the tail of
 *             the last row is zero padding, transformed like data.
 *   levels    (h_0, w_0) = (H, width); (h_l, w_l) = (ceil(h_{l-1}/2),
 *             ceil(w_{l-1}/2)).  Level l splits the h_{l-1} x w_{l-1} LL into
 *             LL_l (h_l x w_l), HL_l (h_l x (w_{l-1}-w_l)), LH_l ((h_{l-1}-h_l)
 *             x w_l), HH_l ((h_{l-1}-h_l) x (w_{l-1}-w_l)); HL is the
 *             horizontal-high / vertical-low band.
 *   priv      AES-128-CTR(key, nonce) of LL_L as int16, row-major:
 *             priv_bytes = 2 * h_L * w_L.  Keystream block j encrypts the
 *             counter (nonce + j) mod 2^128, nonce read as a big-endian
 *             128-bit integer; the last block is truncated.
 *   pub       int16 bands, for l = L down to 1: HL_l | LH_l | HH_l, each
 *             row-major: pub_bytes = 2 * (H * width - h_L * w_L).
 *
 * Conventions for every entry point below:
 *   - data pointers are DEVICE pointers (HBM of the current HIP device);
 *     key / nonce are HOST pointers, read before the call returns.
 *   - work is enqueued on `stream` (a hipStream_t; NULL = the null stream)
 *     and the call returns without waiting; results are valid once the
 *     stream has reached that point.
 *   - the caller owns every buffer.  The library allocates no device memory.
 *   - arguments are validated before anything is launched; on an error
 *     return nothing has been written.
 *   - input and output buffers must not overlap.
 *   - device buffers of dwtfrag_protect / dwtfrag_restore (in, out, priv, pub,
 *     workspace) and of batch items must start at 16-byte aligned addresses:
 *     rows are read and written with 16-byte vector accesses from the buffer
 *     base.  A misaligned pointer returns DWTFRAG_EINVAL before any launch
 *     (copy a buffer that starts at an odd offset into an aligned one first;
 *     hipMalloc and torch allocations are 256-byte aligned).  n itself may be
 *     any length.
 *   - calls may come from several host threads; there is no mutable global
 *     state besides per-device constant tables set up on first use.
 */
#ifndef DWTFRAG_H
#define DWTFRAG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DWTFRAG_OK = 0,
  DWTFRAG_EINVAL = -1,     /* null pointer, n == 0, width == 0, levels == 0 or > 32 */
  DWTFRAG_ERANGE = -2,     /* rows or width above 2^31-2^16, or a byte count overflows */
  DWTFRAG_EDEVICE = -3,    /* a HIP call or kernel launch failed */
  DWTFRAG_EWORKSPACE = -4, /* workspace missing or smaller than workspace_bytes */
  DWTFRAG_ESCRATCH = -5    /* dwtfrag_protect_noalloc: workspace_bytes above its 16 MiB */
} dwtfrag_status;

/* Geometry of one buffer; filled by dwtfrag_geometry. */
typedef struct {
  uint64_t n;               /* buffer length in bytes */
  uint32_t width;           /* row width W */
  uint32_t height;          /* H = ceil(n / W) */
  uint32_t levels;          /* L */
  uint32_t ll_h, ll_w;      /* h_L, w_L */
  uint64_t priv_bytes;      /* 2 * h_L * w_L */
  uint64_t pub_bytes;       /* 2 * (H * W - h_L * w_L) */
  uint64_t workspace_bytes; /* device scratch needed by protect / restore (0 if L <= 4) */
} dwtfrag_geom;

/* Optional launch shape (0 in a field = library default).  Results do not
 * depend on it; it only trades parallelism against halo recomputation.  The
 * default cuts the rows into as many segments as the device keeps wavefronts
 * resident for that kernel (one round), at least two 2^levels-row units each. */
typedef struct {
  uint32_t seg_rows;        /* rows per segment (rounded up to 2^levels; segments are
                               balanced to within 2^levels rows) */
  uint32_t lane_cols;       /* columns per lane at level 1: 8 or 16 (16 needed for 4 levels) */
} dwtfrag_launch;

/* Host-only, pure: geometry of an n-byte buffer viewed with row width `width`
 * and transformed over `levels` levels (Ch. 5 section 5.2.1 view, section
 * 5.1.1 dyadic levels).  Returns DWTFRAG_OK, DWTFRAG_EINVAL or DWTFRAG_ERANGE. */
int dwtfrag_geometry(uint64_t n, uint32_t width, uint32_t levels, dwtfrag_geom *out);

/* Host-only, pure: min(4096, smallest power of two >= ceil(sqrt(n))), the row
 * width used for batches of uneven buffers; 0 for n == 0. */
uint32_t dwtfrag_default_width(uint64_t n);

/* Forward path: view -> L-level 5/3 lifting -> priv = AES-128-CTR(LL_L),
 * pub = detail bands (layout above).  Every device pointer 16-byte aligned.
 *   in        device, n bytes
 *   priv      device, geom.priv_bytes bytes (written)
 *   pub       device, geom.pub_bytes / 2 int16 values (written); may be NULL
 *             when pub_bytes is 0 (a 1 x 1 view)
 *   workspace device scratch of at least geom.workspace_bytes bytes when
 *             that is non-zero (levels > 4), else may be NULL
 *   launch    NULL for the default launch shape */
int dwtfrag_protect(const uint8_t *in, uint64_t n, uint32_t width, uint32_t levels,
                    const uint8_t key[16], const uint8_t nonce[16],
                    uint8_t *priv, int16_t *pub,
                    void *workspace, uint64_t workspace_bytes,
                    const dwtfrag_launch *launch, void *stream);

/* dwtfrag_protect for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same fragments, with the workspace of levels > 4 taken from a static
 * 16 MiB device array inside the library instead of a caller buffer.  The
 * call allocates nothing.  Each GPU the library runs on holds its own copy
 * of the array until the process ends; its device address is looked up on
 * the first call on that device.  Every call on one device shares the array,
 * so calls that may overlap on one device (several streams, several host
 * threads) race and must be ordered by the caller; calls with levels <= 4 do
 * not touch it.  Arguments as dwtfrag_protect; DWTFRAG_ESCRATCH (before any
 * launch) when geom.workspace_bytes exceeds 16 MiB (about n > 2 GiB at
 * levels > 4); DWTFRAG_EDEVICE if the array's address cannot be found. */
int dwtfrag_protect_noalloc(const uint8_t *in, uint64_t n, uint32_t width, uint32_t levels,
                            const uint8_t key[16], const uint8_t nonce[16],
                            uint8_t *priv, int16_t *pub,
                            const dwtfrag_launch *launch, void *stream);

/* Inverse path (Ch. 5 section 5.2.3, exact inverse): decrypt priv with the
 * same keystream, inverse lifting levels L..1 (vertical then horizontal
 * within a level), write the first n bytes; every reconstructed sample is
 * stored modulo 256, so tampered fragments still produce n bytes.
 *   priv, pub fragments as produced by dwtfrag_protect (device, read only)
 *   out       device, n bytes (written)
 * Every device pointer 16-byte aligned; EINVAL otherwise. */
int dwtfrag_restore(const uint8_t *priv, const int16_t *pub, uint64_t n, uint32_t width,
                    uint32_t levels, const uint8_t key[16], const uint8_t nonce[16],
                    uint8_t *out, void *workspace, uint64_t workspace_bytes,
                    const dwtfrag_launch *launch, void *stream);

/* AES-128-CTR on its own (Ch. 2 "Performance issue of SE": counter mode):
 * out[i] = in[i] ^ keystream[16 * first_block + i] for i < nbytes, keystream
 * block j = AES_K((nonce + j) mod 2^128).  in and out (device) may be equal. */
int dwtfrag_aes128_ctr(const uint8_t *in, uint8_t *out, uint64_t nbytes,
                       const uint8_t key[16], const uint8_t nonce[16],
                       uint64_t first_block, void *stream);

/* ------------------------------------------------------------------------
 * Batches of independent buffers (the thesis cuts data into many fixed-size
 * chunks, Ch. 5 section 5.2.1, and feeds many chunks per GPU call).  A batch
 * is planned once on the host, copied into a caller-owned device buffer, and
 * run by one persistent launch per direction that drains a single tile queue
 * (every item's tiles, longest first, 16 columns per lane), so buffers of
 * uneven sizes and depths share the device in one kernel.  Each item's
 * fragments are exactly those of dwtfrag_protect on that item alone.  The
 * run calls launch one kernel each (no allocation, copy or memset; the
 * kernels leave their queue counters reset): they can be captured in a HIP
 * graph and replayed.  Calls on one plan must be ordered on one stream.
 * ------------------------------------------------------------------------ */

typedef struct {
  const uint8_t *in;       /* device, n bytes (protect input), 16-byte aligned */
  uint8_t *out;            /* device, n bytes (restore output) or NULL */
  uint8_t *priv;           /* device, geometry priv_bytes, 16-byte aligned */
  int16_t *pub;            /* device, geometry pub_bytes / 2 values (NULL if 0) */
  uint64_t n;
  uint32_t width;
  uint32_t levels;         /* 1..4 */
  uint8_t key[16];
  uint8_t nonce[16];
} dwtfrag_item;

/* A launch shape for the buffers of one (width, levels) class, as chosen by
 * dwtfrag_autotune. */
typedef struct {
  uint32_t width, levels;
  dwtfrag_launch launch;
} dwtfrag_tune_entry;

typedef struct dwtfrag_batch dwtfrag_batch;  /* opaque host-side plan */

/* Host only: plan `count` items (host array, read before return).  Items of a
 * (width, levels) class listed in `tune` use that entry's rows per tile,
 * others 128-row tiles; batch tiles always have 16 columns per lane (the
 * entry's lane_cols must be 0, 8 or 16 and is not otherwise used).  *out
 * receives a plan owned by the caller (free it with dwtfrag_batch_destroy).
 * EINVAL for a null or misaligned pointer, levels outside 1..4 or a bad
 * lane_cols; ERANGE for geometry out of range. */
int dwtfrag_batch_create(const dwtfrag_item *items, uint32_t count,
                         const dwtfrag_tune_entry *tune, uint32_t n_tune,
                         dwtfrag_batch **out);

/* Device bytes the plan needs (256-byte aligned buffer). */
uint64_t dwtfrag_batch_device_bytes(const dwtfrag_batch *plan);

/* Copy the plan's tables into `device_plan` (device, 256-byte aligned, at
 * least dwtfrag_batch_device_bytes), asynchronously on `stream`: launches
 * that use the plan must be ordered after it (the same stream, or a stream
 * made to wait for this one).  The host tables the copies read stay with the
 * plan; dwtfrag_batch_destroy waits for the last upload's copies before it
 * frees them.  The buffer must stay allocated and untouched while the plan
 * is used. */
int dwtfrag_batch_upload(dwtfrag_batch *plan, void *device_plan, uint64_t device_bytes,
                         void *stream);

/* Protect every item (fragments as dwtfrag_protect), or restore every item
 * (outputs as dwtfrag_restore; every item needs `out`). */
int dwtfrag_batch_protect(const dwtfrag_batch *plan, void *stream);
int dwtfrag_batch_restore(const dwtfrag_batch *plan, void *stream);

/* Free a plan (NULL is a no-op); waits for its last upload's copies. */
void dwtfrag_batch_destroy(dwtfrag_batch *plan);

/* Autotuner: time protect + restore of one buffer (device `in`, n bytes)
 * under each candidate launch shape (rows per tile 0 = the single-buffer
 * default, 64, 128, 256; 8 and 16 columns per lane where the levels allow),
 * `trials` times each, with HIP events on `stream`, and return the fastest in
 * *best (and its time in microseconds in *best_us).  `scratch` (device) holds
 * the fragments, the output and the workspace: at least
 * geom.priv_bytes + geom.pub_bytes + n + geom.workspace_bytes + 768 bytes,
 * 256-byte aligned.  Synchronises `stream`.  Errors: EINVAL for a null
 * pointer or trials == 0, EWORKSPACE for a short or misaligned scratch,
 * the geometry's own errors, else the first failing protect / restore
 * call's code, or EDEVICE for a failing event call. */
int dwtfrag_autotune(const uint8_t *in, uint64_t n, uint32_t width, uint32_t levels,
                     void *scratch, uint64_t scratch_bytes, uint32_t trials,
                     dwtfrag_launch *best, float *best_us, void *stream);

/* ------------------------------------------------------------------------
 * Learned predictor (an extension of the predict slot of the Ch. 5 section
 * 5.1.1 lifting, eq. (5.1); judged by the entropy of eq. (5.6)).  At an odd
 * position i of a signal x of length N >= 2, m the whole-sample mirror:
 *   base = floor((x(m(i-1)) + x(m(i+1))) / 2)
 *   c_j  = clamp(x(m(i + 2j - 7)) - base, -128, 127)                 j = 0..7
 *   h_k  = max(0, sum_j w1[k][j] c_j + b1[k])                         k = 0..15
 *   corr = clamp(floor((sum_k w2[k] h_k + b2) / 2^shift), -255, 255)
 *   d(i) = x(i) - base - corr
 * and the update is eq. (5.2) unchanged; every predict step (rows and
 * columns, every level) uses the same network.  All zero = the plain 5/3
 * lifting.  Levels are limited to 1..3, for which every coefficient of a
 * byte input fits int16.  Fragment layout, AES-CTR and the modulo-256 restore
 * are those of dwtfrag_protect / dwtfrag_restore.
 * ------------------------------------------------------------------------ */

/* Integer network, 216 bytes, no padding (also the serialised blob). */
typedef struct {
  int8_t w1[16][8];   /* hidden weights */
  int8_t w2[16];      /* output weights */
  int32_t b1[16];     /* hidden biases, |b1| <= 2^16 */
  int32_t b2;         /* output bias, |b2| <= 2^26 */
  int32_t shift;      /* 0..30 */
} dwtfrag_predictor;

/* Host-only, pure: device workspace bytes of the learned entry points and
 * the number of (context, target) training pairs of a buffer:
 * sum over levels of h*floor(w/2) (rows, if w > 1) + w*floor(h/2) (columns,
 * if h > 1), (h, w) the level's input dims.  DWTFRAG_EINVAL for levels > 3. */
int dwtfrag_learned_geometry(uint64_t n, uint32_t width, uint32_t levels,
                             uint64_t *workspace_bytes, uint64_t *pairs);

/* dwtfrag_protect with the learned predict step.
 *   predictor  HOST pointer, read before return; limits above (else EINVAL)
 *   workspace  device, >= workspace_bytes of dwtfrag_learned_geometry; holds
 *              the intermediate LL bands until the call's work on `stream` has
 *              completed, so calls that can overlap (other streams) need
 *              workspaces of their own; the same holds for the restore */
int dwtfrag_protect_learned(const uint8_t *in, uint64_t n, uint32_t width, uint32_t levels,
                            const uint8_t key[16], const uint8_t nonce[16],
                            const dwtfrag_predictor *predictor,
                            uint8_t *priv, int16_t *pub,
                            void *workspace, uint64_t workspace_bytes, void *stream);

/* Exact inverse of dwtfrag_protect_learned for the same predictor. */
int dwtfrag_restore_learned(const uint8_t *priv, const int16_t *pub, uint64_t n, uint32_t width,
                            uint32_t levels, const uint8_t key[16], const uint8_t nonce[16],
                            const dwtfrag_predictor *predictor,
                            uint8_t *out, void *workspace, uint64_t workspace_bytes,
                            void *stream);

/* Training pairs of a buffer: for every predict step of its PLAIN 5/3
 * decomposition (level by level; the row pass, row by row, then the column
 * pass, column by column; odd positions in increasing order) the clamped
 * context c_0..c_7 (8 int8, device, 8-byte aligned) and the target
 * x(i) - base (int32, device).  Writes exactly `pairs` entries. */
int dwtfrag_learned_pairs(const uint8_t *in, uint64_t n, uint32_t width, uint32_t levels,
                          int8_t *ctx, int32_t *target,
                          void *workspace, uint64_t workspace_bytes, void *stream);

/* Trainer state (device memory, caller-owned, 8-byte aligned).  theta is the
 * float network y = w2 . relu(W1 c + b1) + b2 flattened as W1 (16x8 row-
 * major), b1 (16), w2 (16), b2.  net is its quantisation: power-of-two
 * scales k1 = largest k <= 30 with max|W1| 2^k < 127.5, shift =
 * clamp(k1 + k(max|w2|), 0, 30), k2 = shift - k1, values rounded half to
 * even and clamped to the limits above. */
typedef struct {
  float theta[161];
  float m[161];         /* Adam first moment */
  float v[161];         /* Adam second moment */
  float grad[161];      /* gradient of the last step */
  float loss;           /* mean |y - t| of the last step, before its update */
  int32_t step;         /* Adam steps taken */
  int32_t k1, k2;       /* scales of net */
  dwtfrag_predictor net;
} dwtfrag_trainer;

/* Device workspace bytes of dwtfrag_trainer_step (a constant). */
uint64_t dwtfrag_trainer_workspace_bytes(void);

/* theta = theta0 (HOST, 161 floats), zero moments and step, net = its
 * quantisation. */
int dwtfrag_trainer_init(dwtfrag_trainer *state, const float theta0[161], void *stream);

/* One step of quantisation-aware Adam (beta1 0.9, beta2 0.999, eps 1e-8) on
 * the `count` pairs at indices 0, stride, 2 stride, ... of ctx / target
 * (stride >= 1; offset the pointers to pick another interleaved batch):
 * the mean absolute error of y against the target and its
 * gradient are taken at the fake-quantised parameters (net's integers over
 * their powers of two), the gradient is applied to theta, and net is
 * re-quantised.  ctx / target as written by dwtfrag_learned_pairs. */
int dwtfrag_trainer_step(dwtfrag_trainer *state, const int8_t *ctx, const int32_t *target,
                         uint64_t count, uint64_t stride, float lr,
                         void *workspace, uint64_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------
 * The thesis's own per-8x8-block protection (Ch. 5 section 5.2.1 "Designs";
 * bit budget of section 5.2.2.2).  The byte matrix (row width a multiple of
 * 8, rows padded with zeros to a multiple of 8) is cut into 8x8 blocks,
 * numbered row-major; each gets two levels of the 5/3 lifting (whole-sample
 * mirror at the block's own edges, rows first).  Per block:
 *   private record   LL2 (4 x 10 bits)                         40 bits
 *   first public     HL2, LH2 (10 bits each), HH2 (11 bits)     124 bits
 *   second public    HL1, LH1, HH1 (48 x 10 bits)               480 bits
 * values two's complement in their width, bands row-major, records as bit
 * streams (bit i = bit i % 8 of byte i / 8) laid end to end in block order.
 * The first public record is XORed with the first 124 bits of
 *   SHA-256(private record (5 bytes) | key | nonce | block index (8 bytes BE)),
 * the second with the first 480 bits of
 *   SHA-512(protected first record (16 bytes, 4 zero bits on top) | key | nonce
 *           | block index),
 * and the private fragment is AES-128-CTR(key, nonce) of the concatenated
 * private records, as dwtfrag_protect's.  Restore writes every sample modulo
 * 256.  Every device pointer 16-byte aligned (EINVAL otherwise); EINVAL also
 * for n == 0 or a width that is not a positive multiple of 8.
 * ------------------------------------------------------------------------ */

typedef struct {
  uint64_t n;
  uint32_t width;
  uint64_t height;          /* ceil(n / width) */
  uint64_t block_rows;      /* ceil(height / 8) */
  uint64_t block_cols;      /* width / 8 */
  uint64_t blocks;          /* block_rows * block_cols */
  uint64_t priv_bytes;      /* 5 * blocks */
  uint64_t pub1_bytes;      /* ceil(124 * blocks / 8) */
  uint64_t pub2_bytes;      /* 60 * blocks */
} dwtfrag_se8_geom;

/* Host-only, pure: geometry of the blocked form. */
int dwtfrag_se8_geometry(uint64_t n, uint32_t width, dwtfrag_se8_geom *out);

/* Forward: in (device, n bytes) -> priv, pub1, pub2 (device, sizes above). */
int dwtfrag_se8_protect(const uint8_t *in, uint64_t n, uint32_t width,
                        const uint8_t key[16], const uint8_t nonce[16],
                        uint8_t *priv, uint8_t *pub1, uint8_t *pub2, void *stream);

/* Inverse: the three fragments -> out (device, n bytes). */
int dwtfrag_se8_restore(const uint8_t *priv, const uint8_t *pub1, const uint8_t *pub2,
                        uint64_t n, uint32_t width, const uint8_t key[16],
                        const uint8_t nonce[16], uint8_t *out, void *stream);

/* ------------------------------------------------------------------------
 * Reference streams, for measurement context only (not part of the method;
 * for callers that compare the lifting kernels with the plainest kernel of
 * the same traffic): one-shot launches that move the same bytes as the
 * forward and the inverse of a whole buffer.
 *   widen:  out[i] = in[i] zero-extended to int16   (reads n, writes 2n bytes)
 *   narrow: out[i] = low byte of in[i]              (reads 2n, writes n bytes)
 * in, out: device, not overlapping, 16-byte aligned; n a positive multiple of
 * 16 below 2^43.  DWTFRAG_EINVAL otherwise; DWTFRAG_EDEVICE if the launch
 * fails.  Asynchronous on stream.
 * ------------------------------------------------------------------------ */
int dwtfrag_ref_widen(const uint8_t *in, int16_t *out, uint64_t n, void *stream);
int dwtfrag_ref_narrow(const int16_t *in, uint8_t *out, uint64_t n, void *stream);

/* Static text for a status code. */
const char *dwtfrag_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* DWTFRAG_H */
