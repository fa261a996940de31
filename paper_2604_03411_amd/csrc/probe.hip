// Calibration probe for the matrix-core counters: a kernel that issues only
// FP64 16x16x4 matrix products (4 independent accumulation chains per wave,
// 4 waves per block), so that the MFMA-busy counter of a profiled run can be
// related to a known number of products, as a device copy of known size
// relates the byte counters to bytes.  Launched as many short blocks, so that
// the dispatcher's uneven placement of blocks on compute units averages out.
#include "gedmg_internal.h"

namespace gedmg {

typedef double d4_t __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void mfma_probe_kernel(double* sink, int iters) {
  d4_t c0 = {0.0, 0.0, 0.0, 0.0}, c1 = c0, c2 = c0, c3 = c0;
  const double a = 1.0 + 1e-3 * (threadIdx.x & 63);
  const double b = 1.0 - 1e-3 * (threadIdx.x & 63);
  for (int i = 0; i < iters; ++i) {
    c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(b, a, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, a, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f64_16x16x4f64(b, b, c3, 0, 0, 0);
  }
  const d4_t s = c0 + c1 + c2 + c3;
  sink[(long)blockIdx.x * blockDim.x + threadIdx.x] = s[0] + s[1] + s[2] + s[3];
}

}  // namespace gedmg

extern "C" int gedmg_probe_mfma(double* sink, int32_t blocks, int32_t iters, void* hip_stream) {
  if (!sink || blocks <= 0 || iters <= 0) return GEDMG_E_ARG;
  hipLaunchKernelGGL(gedmg::mfma_probe_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)hip_stream, sink, iters);
  return hipGetLastError() == hipSuccess ? GEDMG_OK : GEDMG_E_HIP;
}
