// AES-128-CTR over a byte range on its own (Ch. 2 "Performance issue of SE":
// counter mode is the parallel AES mode).  One thread per 16-byte block; the
// four T-tables sit in LDS.
#include "batch.h"
#include "common.h"

namespace dwtfrag {

__global__ __launch_bounds__(256) void ctr_kernel(const uint8_t *__restrict__ in,
                                                  uint8_t *__restrict__ out, uint64_t nbytes,
                                                  const AesKey key, uint64_t first_block) {
  __shared__ uint32_t s_te[1024];
  __shared__ uint32_t s_kw[kKeyWords];
  load_aes_tables(s_te, s_kw, key);
  __syncthreads();
  const uint64_t nblk = (nbytes + 15) / 16;
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t b = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; b < nblk; b += stride) {
    uint32_t w[4];
    counter_block(s_kw, first_block + b, w);
    aes_encrypt(s_te, s_kw, w);
    const uint64_t off = b * 16;
    const bool vec = off + 16 <= nbytes &&
                     ((reinterpret_cast<uintptr_t>(in + off) | reinterpret_cast<uintptr_t>(out + off)) & 15) == 0;
    if (vec) {
      uint4 v = *reinterpret_cast<const uint4 *>(in + off);
      v.x ^= w[0]; v.y ^= w[1]; v.z ^= w[2]; v.w ^= w[3];
      *reinterpret_cast<uint4 *>(out + off) = v;
    } else {
      for (int i = 0; i < 16 && off + i < nbytes; ++i)
        out[off + i] = uint8_t(in[off + i] ^ uint8_t(w[i >> 2] >> (8 * (i & 3))));
    }
  }
}

hipError_t launch_ctr(const uint8_t *in, uint8_t *out, uint64_t nbytes, const AesKey &key,
                      uint64_t first_block, hipStream_t s) {
  const uint64_t nblk = (nbytes + 15) / 16;
  const uint64_t grid = std::min<uint64_t>((nblk + 255) / 256, 4096);
  hipLaunchKernelGGL(ctr_kernel, dim3(unsigned(grid)), dim3(256), 0, s, in, out, nbytes, key,
                     first_block);
  return hipGetLastError();
}

// Batch form: the private fragments of all items in place, each with its own
// key and nonce.  Global block b belongs to the item whose prefix range
// [aes_first, aes_first + aes_blocks) holds it (binary search).
__global__ __launch_bounds__(256) void ctr_batch_kernel(const BatchItem *__restrict__ items, int count,
                                                        uint64_t total_blocks) {
  __shared__ uint32_t s_te[1024];
  for (int i = threadIdx.x; i < 1024; i += blockDim.x) {
    const uint32_t v = c_aes.te0[i & 255];
    const int r = 8 * (i >> 8);
    s_te[i] = r ? ((v << r) | (v >> (32 - r))) : v;
  }
  __syncthreads();
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t b = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; b < total_blocks; b += stride) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (items[mid].aes_first <= b) lo = mid;
      else hi = mid - 1;
    }
    const BatchItem &it = items[lo];
    const AesKey &key = it.fwd.key;
    const uint64_t j = b - it.aes_first;
    uint32_t kw[kKeyWords];
#pragma unroll
    for (int i = 0; i < 44; ++i) kw[i] = key.rk[i];
    kw[44] = uint32_t(key.nonce_hi);
    kw[45] = uint32_t(key.nonce_hi >> 32);
    kw[46] = uint32_t(key.nonce_lo);
    kw[47] = uint32_t(key.nonce_lo >> 32);
    uint32_t w[4];
    counter_block(kw, j, w);
    aes_encrypt(s_te, kw, w);
    uint8_t *p = it.priv + 16 * j;
    if (16 * (j + 1) <= it.priv_bytes) {  // priv is 16-byte aligned (checked by the planner)
      uint4 v = *reinterpret_cast<const uint4 *>(p);
      v.x ^= w[0]; v.y ^= w[1]; v.z ^= w[2]; v.w ^= w[3];
      *reinterpret_cast<uint4 *>(p) = v;
    } else {
      const int len = int(it.priv_bytes - 16 * j);
      for (int i = 0; i < len; ++i) p[i] ^= uint8_t(w[i >> 2] >> (8 * (i & 3)));
    }
  }
}

hipError_t launch_ctr_batch(const BatchItem *items, int count, uint64_t total_blocks, hipStream_t s) {
  const uint64_t grid = std::min<uint64_t>((total_blocks + 255) / 256, 4096);
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL(ctr_batch_kernel, dim3(unsigned(grid)), dim3(256), 0, s, items, count,
                     total_blocks);
  return hipGetLastError();
}

}  // namespace dwtfrag
