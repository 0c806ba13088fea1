// FP64 throughput probes, the measured denominators beside the published
// peak: back-to-back v_mfma_f64_16x16x4 instructions in four independent
// accumulator chains per wave, and FP64 VALU fused multiply-adds in eight
// independent chains per lane.  Each block writes one value per wave so that
// no chain is optimised away.
#include <hip/hip_runtime.h>

namespace mpe {

typedef double v4dp __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_peak_mfma(int iters, double seed, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const double a = seed + 1e-3 * lane, b = 1.0 - seed;
  v4dp c0 = v4dp{0.0, 0.0, 0.0, 0.0}, c1 = c0, c2 = c0, c3 = c0;
  for (int i = 0; i < iters; i++) {
    c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(b, a, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, a, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f64_16x16x4f64(b, b, c3, 0, 0, 0);
  }
  const double s = (c0[0] + c1[1]) + (c2[2] + c3[3]);
  if (lane == 0) out[blockIdx.x * 4 + (threadIdx.x >> 6)] = s;
}

__global__ __launch_bounds__(256) void k_peak_valu(int iters, double seed, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const double a = 1.0 - 1e-9, b = seed * 1e-9;
  double x[8];
#pragma unroll
  for (int u = 0; u < 8; u++) x[u] = seed + 1e-3 * u + 1e-6 * threadIdx.x;
  for (int i = 0; i < iters; i++) {
#pragma unroll
    for (int u = 0; u < 8; u++) x[u] = fma(x[u], a, b);
  }
  const double s = ((x[0] + x[1]) + (x[2] + x[3])) + ((x[4] + x[5]) + (x[6] + x[7]));
  if (lane == 0) out[blockIdx.x * 4 + (threadIdx.x >> 6)] = s;
}

// flops of one launch: kind 0: blocks * 4 waves * 4 chains * 2048 per
// iteration; kind 1: blocks * 256 lanes * 8 chains * 2 per iteration
hipError_t launch_peak_probe(int kind, int blocks, int iters, double* out, hipStream_t s, double* flops) {
  if (kind == 0) {
    hipLaunchKernelGGL(k_peak_mfma, dim3(blocks), dim3(256), 0, s, iters, 0.25, out);
    *flops = (double)blocks * 4.0 * 4.0 * 2048.0 * iters;
  } else {
    hipLaunchKernelGGL(k_peak_valu, dim3(blocks), dim3(256), 0, s, iters, 0.25, out);
    *flops = (double)blocks * 256.0 * 8.0 * 2.0 * iters;
  }
  return hipGetLastError();
}

}  // namespace mpe
