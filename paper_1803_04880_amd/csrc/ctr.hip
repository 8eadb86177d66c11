// AES-128-CTR over a byte range on its own (Ch. 2 "Performance issue of SE":
// counter mode is the parallel AES mode).  One thread per 16-byte block; the
// four T-tables sit in LDS.
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

}  // namespace dwtfrag
