// Reference streams for measurement context, not part of the method: a
// plain conversion that moves the same bytes as the streaming lifting
// kernels, in the same directions.  widen reads n bytes and writes n int16
// (zero-extended), as the forward reads the bytes and writes the int16
// fragments; narrow reads n int16 and writes their low bytes, as the inverse
// does.  Both are one-shot launches: a thread converts one 16-byte vector of
// bytes and exits, so no thread ever waits on a load behind its own stores.
#include "dwtfrag.h"

#include "common.h"

namespace dwtfrag {

__global__ __launch_bounds__(256) void ref_widen_kernel(const uint8_t *__restrict__ in,
                                                        int16_t *__restrict__ out, uint64_t nvec) {
  const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nvec) return;
  const u32x4 v = *(glob(reinterpret_cast<const u32x4 *>(in)) + i);
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
  uint32_t o[8];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    o[2 * k] = __builtin_amdgcn_perm(0u, w[k], 0x0C010C00u);      // bytes 0, 1
    o[2 * k + 1] = __builtin_amdgcn_perm(0u, w[k], 0x0C030C02u);  // bytes 2, 3
  }
  const gptr<u32x4> dst = glob(reinterpret_cast<u32x4 *>(out)) + 2 * i;
  dst[0] = u32x4{o[0], o[1], o[2], o[3]};
  dst[1] = u32x4{o[4], o[5], o[6], o[7]};
}

__global__ __launch_bounds__(256) void ref_narrow_kernel(const int16_t *__restrict__ in,
                                                         uint8_t *__restrict__ out, uint64_t nvec) {
  const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nvec) return;
  const gptr<const u32x4> src = glob(reinterpret_cast<const u32x4 *>(in)) + 2 * i;
  const u32x4 a = src[0], b = src[1];
  const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
  uint32_t o[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) o[k] = __builtin_amdgcn_perm(w[2 * k + 1], w[2 * k], 0x06040200u);
  *(glob(reinterpret_cast<u32x4 *>(out)) + i) = u32x4{o[0], o[1], o[2], o[3]};
}

namespace {

bool ref_args_ok(const void *a, const void *b, uint64_t n) {
  return a && b && n && n % 16 == 0 && (n / 16 + 255) / 256 < (1ull << 31) &&
         ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b)) & 15) == 0;
}

}  // namespace

}  // namespace dwtfrag

using namespace dwtfrag;

extern "C" {

int dwtfrag_ref_widen(const uint8_t *in, int16_t *out, uint64_t n, void *stream) {
  if (!ref_args_ok(in, out, n)) return DWTFRAG_EINVAL;
  const uint64_t nvec = n / 16;
  hipLaunchKernelGGL(ref_widen_kernel, dim3(unsigned((nvec + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), in, out, nvec);
  return hipGetLastError() == hipSuccess ? DWTFRAG_OK : DWTFRAG_EDEVICE;
}

int dwtfrag_ref_narrow(const int16_t *in, uint8_t *out, uint64_t n, void *stream) {
  if (!ref_args_ok(in, out, n)) return DWTFRAG_EINVAL;
  const uint64_t nvec = n / 16;
  hipLaunchKernelGGL(ref_narrow_kernel, dim3(unsigned((nvec + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), in, out, nvec);
  return hipGetLastError() == hipSuccess ? DWTFRAG_OK : DWTFRAG_EDEVICE;
}

}  // extern "C"
