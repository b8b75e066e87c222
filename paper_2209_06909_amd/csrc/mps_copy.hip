// mps_copy.hip -- a streaming device-to-device copy: the reference point for
// the HBM bandwidth a one-pass kernel reaches on this device (every byte read
// once and written once), against which the merge levels are measured.
#include "mps_internal.h"
#include "mps.h"

namespace mps {
namespace {

constexpr int kCopyThreads = 256;
constexpr unsigned kCopyGrid = 1024;   // 4 workgroups per CU

__global__ __launch_bounds__(kCopyThreads) void k_stream_copy(const uint4 *__restrict__ src,
                                                              uint4 *__restrict__ dst, uint64_t n16,
                                                              const uint8_t *__restrict__ tail_src,
                                                              uint8_t *__restrict__ tail_dst,
                                                              uint32_t tail) {
  const uint64_t stride = (uint64_t)gridDim.x * kCopyThreads;
  for (uint64_t i = (uint64_t)blockIdx.x * kCopyThreads + threadIdx.x; i < n16; i += stride)
    dst[i] = src[i];
  if (blockIdx.x == 0 && threadIdx.x < tail) tail_dst[threadIdx.x] = tail_src[threadIdx.x];
}

}  // namespace
}  // namespace mps

extern "C" int mps_stream_copy(const void *src, void *dst, uint64_t bytes, void *stream) {
  using namespace mps;
  if (bytes == 0) return MPS_OK;
  if (!src || !dst) return fail_msg(MPS_E_INVALID, "NULL pointer");
  if (((uintptr_t)src | (uintptr_t)dst) & 15)
    return fail_msg(MPS_E_INVALID, "src and dst must be 16-byte aligned");
  const uint64_t n16 = bytes / 16;
  const uint32_t tail = (uint32_t)(bytes % 16);
  const uint64_t want = (n16 + kCopyThreads - 1) / kCopyThreads;
  const unsigned grid = want == 0 ? 1u : (want < kCopyGrid ? (unsigned)want : kCopyGrid);
  hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(kCopyThreads), 0, (hipStream_t)stream,
                     (const uint4 *)src, (uint4 *)dst, n16,
                     (const uint8_t *)src + n16 * 16, (uint8_t *)dst + n16 * 16, tail);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail_msg(MPS_E_HIP, hipGetErrorString(e));
  return MPS_OK;
}
