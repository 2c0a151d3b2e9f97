// Reference kernels for hardware traffic counters (measurement only).
//
// A counter such as FETCH_SIZE reports bytes per kernel in units that
// depend on how the kernel's requests reach memory; these kernels move a
// known number of bytes in the two ways the library's kernels read:
//   k_copy_vector : a plain copy, 16 bytes per lane per load and store
//                   (the expansion's operand and output traffic);
//   k_read_scalar : wave-uniform 64-byte reads through the scalar cache
//                   (the ascent kernel's class weights), summed into one
//                   value per workgroup so that the reads are not removed.
#include "bh_internal.h"

namespace bh {
namespace {

__global__ __launch_bounds__(256) void k_copy_vector(const float4* __restrict__ src,
                                                     float4* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// One wave per workgroup; workgroup g reads the 64-byte blocks
// [g * per, min((g + 1) * per, n_blocks)).
__global__ __launch_bounds__(64) void k_read_scalar(const double* __restrict__ src,
                                                    int64_t n_blocks, int64_t per,
                                                    double* __restrict__ out) {
  const int64_t b0 = (int64_t)blockIdx.x * per;
  const int64_t b1 = b0 + per < n_blocks ? b0 + per : n_blocks;
  double acc = 0.0;
  for (int64_t b = b0; b < b1; ++b) {
    const double* p = src + b * 8;
    acc += ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]));
  }
  if (threadIdx.x == 0) out[blockIdx.x] = acc;
}

}  // namespace
}  // namespace bh

using namespace bh;

extern "C" int bh_calib_copy(void* dst, const void* src, int64_t bytes, int mode, void* stream) {
  if (!dst || !src) return set_error(BH_EINVAL, "NULL buffer");
  const hipStream_t s = (hipStream_t)stream;
  if (mode == BH_CALIB_COPY_VECTOR) {
    if (bytes <= 0 || bytes % 16) return set_error(BH_EINVAL, "bytes must be a positive multiple of 16");
    hipLaunchKernelGGL(k_copy_vector, dim3(4096), dim3(256), 0, s,
                       reinterpret_cast<const float4*>(src), reinterpret_cast<float4*>(dst),
                       bytes / 16);
  } else if (mode == BH_CALIB_READ_SCALAR) {
    if (bytes <= 0 || bytes % 64) return set_error(BH_EINVAL, "bytes must be a positive multiple of 64");
    const int64_t n_blocks = bytes / 64;
    const int64_t per = (n_blocks + BH_CALIB_READ_GROUPS - 1) / BH_CALIB_READ_GROUPS;
    hipLaunchKernelGGL(k_read_scalar, dim3(BH_CALIB_READ_GROUPS), dim3(64), 0, s,
                       reinterpret_cast<const double*>(src), n_blocks, per,
                       reinterpret_cast<double*>(dst));
  } else {
    return set_error(BH_EINVAL, "unknown calibration mode");
  }
  BH_HIP(hipGetLastError());
  return BH_OK;
}
