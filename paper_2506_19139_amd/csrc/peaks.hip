// Instrumentation, not part of the method: two kernels that measure the machine peaks the
// benchmark reports beside the vendor figures.  A streaming copy (16-byte loads and stores,
// grid-stride) gives the reachable HBM bandwidth; a chain of independent fused multiply-adds
// per lane gives the reachable float32 vector rate of this build (packed float32 is disabled
// for all device code, so one lane issues one FMA per instruction).
#include "launch.h"

namespace sof {

__global__ __launch_bounds__(256) void k_peak_copy(const float4* __restrict__ src, float4* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// 16 independent accumulators per lane, `iters` rounds of 16 FMAs each; the result is stored
// so that nothing can be folded away.  Flops = 2 x 16 x iters x lanes.
__global__ __launch_bounds__(256) void k_peak_fma(float* out, int iters, float a, float b) {
  float acc[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) acc[k] = (float)(threadIdx.x + k) * 1e-3f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = fmaf(acc[k], a, b);
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 16; ++k) s += acc[k];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace sof

using namespace sof;

extern "C" int sof_bench_copy(const void* src, void* dst, int64_t n_vec4, hipStream_t stream) {
  if (n_vec4 < 0 || (n_vec4 > 0 && (!src || !dst))) return SOF_E_ARG;
  if (n_vec4 == 0) return SOF_OK;
  const int64_t blocks = div_up(n_vec4, 256) < 256 * 64 ? div_up(n_vec4, 256) : 256 * 64;
  hipLaunchKernelGGL(k_peak_copy, dim3((unsigned)blocks), dim3(256), 0, stream, (const float4*)src, (float4*)dst, n_vec4);
  return hipGetLastError() == hipSuccess ? SOF_OK : SOF_E_HIP;
}

extern "C" int sof_bench_fma(float* out, int64_t n_blocks, int32_t iters, hipStream_t stream) {
  if (n_blocks < 0 || iters < 0 || (n_blocks > 0 && !out)) return SOF_E_ARG;
  if (n_blocks == 0) return SOF_OK;
  hipLaunchKernelGGL(k_peak_fma, dim3((unsigned)n_blocks), dim3(256), 0, stream, out, iters, 0.999f, 1e-4f);
  return hipGetLastError() == hipSuccess ? SOF_OK : SOF_E_HIP;
}
