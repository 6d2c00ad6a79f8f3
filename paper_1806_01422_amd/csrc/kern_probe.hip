// Diagnostic kernels: FP64 issue rate of the matrix cores (v_mfma_f64_16x16x4f64) and of the
// vector units (v_fma_f64), each alone and both interleaved in one instruction stream.  They
// measure the choice made for the line contractions of the operators (Sec. 3.3 sum
// factorisation): whether moving contractions onto the matrix cores could run beside the vector
// work that stays on the vector units.
#include "sem_internal.h"

namespace sem {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// MODE 0: matrix cores only (four independent accumulators), 1: vector FMAs only (eight
// independent chains, 64 FMAs per lane per iteration), 2: both in each iteration.
template <int MODE>
__global__ __launch_bounds__(256) void fp64_rate_kernel(double* __restrict__ out, int iters) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const double a = 1.0 + 1e-12 * threadIdx.x, b = 1.0 - 1e-12 * threadIdx.x;
  d4 m0 = {0, 0, 0, 0}, m1 = m0, m2 = m0, m3 = m0;
  double v[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) v[r] = 1e-3 * (r + 1);
  for (int k = 0; k < iters; ++k) {
    if constexpr (MODE != 1) {
      m0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, m0, 0, 0, 0);
      m1 = __builtin_amdgcn_mfma_f64_16x16x4f64(b, a, m1, 0, 0, 0);
      m2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, a, m2, 0, 0, 0);
      m3 = __builtin_amdgcn_mfma_f64_16x16x4f64(b, b, m3, 0, 0, 0);
    }
    if constexpr (MODE != 0) {
#pragma unroll
      for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int r = 0; r < 8; ++r) v[r] = __builtin_fma(v[r], a, b);
    }
  }
  double acc = m0.x + m1.y + m2.z + m3.w;
#pragma unroll
  for (int r = 0; r < 8; ++r) acc += v[r];
  out[t] = acc;  // keeps every chain live
}

}  // namespace

constexpr int PROBE_BLOCKS = 4096, PROBE_THREADS = 256;

int64_t fp64_probe_values() { return (int64_t)PROBE_BLOCKS * PROBE_THREADS; }

hipError_t launch_fp64_probe(int mode, double* out, int iters, hipStream_t s) {
  const dim3 grid(PROBE_BLOCKS), block(PROBE_THREADS);
  if (mode == 0)
    hipLaunchKernelGGL((fp64_rate_kernel<0>), grid, block, 0, s, out, iters);
  else if (mode == 1)
    hipLaunchKernelGGL((fp64_rate_kernel<1>), grid, block, 0, s, out, iters);
  else
    hipLaunchKernelGGL((fp64_rate_kernel<2>), grid, block, 0, s, out, iters);
  return hipGetLastError();
}

// Flops one wavefront issues per iteration: a 16x16x4 FP64 MFMA is 16*16*4 multiply-adds; the
// vector part is 64 FMAs per lane.
double fp64_probe_mfma_flops_per_wave_iter() { return 4 * 16.0 * 16 * 4 * 2; }
double fp64_probe_valu_flops_per_wave_iter() { return 64 * 64.0 * 2; }

}  // namespace sem
