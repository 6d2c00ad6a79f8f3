// Vector kernels for the Newton-Krylov solvers: dot products of one vector with several others
// (deterministic two-stage reduction in FP64: fixed-order partial sums per block, then a fixed
// tree per vector) and combinations y = a y + sum_j c_j x_j with the
// coefficients read from device memory, so a Gram-Schmidt step needs no host round trip between
// its projection and its update.
#include "sem_internal.h"

namespace sem {
namespace {

constexpr int BT = 256;          // threads per block
constexpr int MAXV = 40;         // most vectors in one multi-dot or combination
constexpr int CH = 8;            // vectors per multi-dot chunk (blockIdx.y)
constexpr int DOT_BLOCKS = 2048; // partial sums per vector

// partial[b][j] = sum over block b's strided range of x_j[i] * w[i], for the chunk of vectors
// j0 = CH * blockIdx.y .. j0 + CH - 1 (fixed order within the block: per thread, then per wavefront
// by shuffles, then over the wavefronts)
template <typename T>
__global__ __launch_bounds__(BT) void multidot_partial(const T* __restrict__ X, int64_t ldx, int nv,
                                                       const T* __restrict__ w, int64_t n,
                                                       double* __restrict__ partial) {
  __shared__ double red[BT / 64][CH];
  const int j0 = CH * blockIdx.y;
  const int nc = nv - j0 < CH ? nv - j0 : CH;
  double acc[CH];
#pragma unroll
  for (int j = 0; j < CH; ++j) acc[j] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x; i < n; i += (int64_t)gridDim.x * BT) {
    const double wi = (double)w[i];
#pragma unroll
    for (int j = 0; j < CH; ++j)
      if (j < nc) acc[j] += (double)X[(j0 + j) * ldx + i] * wi;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < CH; ++j) {
    double v = acc[j];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[wave][j] = v;
  }
  __syncthreads();
  if (threadIdx.x < nc) {
    double s = 0.0;
    for (int k = 0; k < BT / 64; ++k) s += red[k][threadIdx.x];
    partial[(int64_t)blockIdx.x * MAXV + j0 + threadIdx.x] = s;
  }
}

// out[j] = sum over blocks of partial[b][j]: block j, each thread a strided subset in order, then a
// tree over the threads (the same order on every call)
__global__ __launch_bounds__(BT) void multidot_final(const double* __restrict__ partial, int nblocks,
                                                     double* __restrict__ out) {
  __shared__ double red[BT];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += BT) s += partial[(int64_t)b * MAXV + j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = BT / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = red[0];
}

// Gram-Schmidt update fused with the next reduction: y <- y + sign sum_j coef[j] x_j, then
// partial sums of <x_j, y_new> (j < nv) or, with SELF, of <y_new, y_new> (one value); the partial
// layout and the final reduction are those of multidot.  NV bounds nv (registers per thread).
template <typename T, int NV, bool SELF>
__global__ __launch_bounds__(BT) void combine_dot_partial(T* __restrict__ y, const T* __restrict__ X, int64_t ldx,
                                                          int nv, const double* __restrict__ coef, double sign,
                                                          int64_t n, double* __restrict__ partial) {
  constexpr int NA = SELF ? 1 : NV;
  __shared__ double c[MAXV];
  __shared__ double red[BT / 64][NA];
  if (threadIdx.x < nv) c[threadIdx.x] = sign * coef[threadIdx.x];
  __syncthreads();
  double acc[NA];
#pragma unroll
  for (int j = 0; j < NA; ++j) acc[j] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x; i < n; i += (int64_t)gridDim.x * BT) {
    double xv[NV];
    double sum = (double)y[i];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      xv[j] = j < nv ? (double)X[j * ldx + i] : 0.0;
      if (j < nv) sum += c[j] * xv[j];
    }
    const T yn = (T)sum;
    y[i] = yn;
    if constexpr (SELF) {
      acc[0] += (double)yn * (double)yn;
    } else {
#pragma unroll
      for (int j = 0; j < NV; ++j)
        if (j < nv) acc[j] += xv[j] * (double)yn;
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < NA; ++j) {
    double v = acc[j];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[wave][j] = v;
  }
  __syncthreads();
  const int na = SELF ? 1 : nv;
  if ((int)threadIdx.x < na) {
    double s = 0.0;
    for (int k = 0; k < BT / 64; ++k) s += red[k][threadIdx.x];
    partial[(int64_t)blockIdx.x * MAXV + threadIdx.x] = s;
  }
}

// y = alpha * y + sum_j sign * coef[j] * x_j   (coef in device memory)
template <typename T>
__global__ __launch_bounds__(BT) void combine(T* __restrict__ y, double alpha, const T* __restrict__ X, int64_t ldx,
                                              int nv, const double* __restrict__ coef, double sign, int64_t n) {
  __shared__ double c[MAXV];
  if (threadIdx.x < nv) c[threadIdx.x] = sign * coef[threadIdx.x];
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x; i < n; i += (int64_t)gridDim.x * BT) {
    double s = alpha == 0.0 ? 0.0 : alpha * (double)y[i];
    for (int j = 0; j < nv; ++j) s += c[j] * (double)X[j * ldx + i];
    y[i] = (T)s;
  }
}

// z = a x + b y
template <typename T>
__global__ __launch_bounds__(BT) void axpby_kernel(T* __restrict__ z, double a, const T* __restrict__ x, double b,
                                                   const T* __restrict__ y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x; i < n; i += (int64_t)gridDim.x * BT)
    z[i] = (T)(a * (double)x[i] + (y ? b * (double)y[i] : 0.0));
}

unsigned grid_for(int64_t n) {
  const int64_t b = (n + BT - 1) / BT;
  return (unsigned)(b < 2048 ? (b < 1 ? 1 : b) : 2048);
}

}  // namespace

int blas_max_vectors() { return MAXV; }
size_t blas_partial_bytes() { return sizeof(double) * DOT_BLOCKS * MAXV; }

hipError_t blas_multidot(int dtype, const void* X, int64_t ldx, int nv, const void* w, int64_t n, double* partial,
                         double* out, hipStream_t s) {
  if (nv < 1 || nv > MAXV) return hipErrorInvalidValue;
  const int64_t need = (n + BT - 1) / BT;
  const int nb = (int)(need < DOT_BLOCKS ? (need < 1 ? 1 : need) : DOT_BLOCKS);
  const dim3 grid(nb, (nv + CH - 1) / CH);
  if (dtype == SEM_F64)
    hipLaunchKernelGGL(multidot_partial<double>, grid, dim3(BT), 0, s, static_cast<const double*>(X), ldx, nv,
                       static_cast<const double*>(w), n, partial);
  else
    hipLaunchKernelGGL(multidot_partial<float>, grid, dim3(BT), 0, s, static_cast<const float*>(X), ldx, nv,
                       static_cast<const float*>(w), n, partial);
  hipLaunchKernelGGL(multidot_final, dim3(nv), dim3(BT), 0, s, partial, nb, out);
  return hipGetLastError();
}

template <typename T, bool SELF>
static hipError_t run_combine_dot(T* y, const T* X, int64_t ldx, int nv, const double* coef, double sign, int64_t n,
                                  double* partial, double* out, hipStream_t s) {
  const int64_t need = (n + BT - 1) / BT;
  const int nb = (int)(need < DOT_BLOCKS ? (need < 1 ? 1 : need) : DOT_BLOCKS);
  if (nv <= 8)
    hipLaunchKernelGGL((combine_dot_partial<T, 8, SELF>), dim3(nb), dim3(BT), 0, s, y, X, ldx, nv, coef, sign, n,
                       partial);
  else if (nv <= 16)
    hipLaunchKernelGGL((combine_dot_partial<T, 16, SELF>), dim3(nb), dim3(BT), 0, s, y, X, ldx, nv, coef, sign, n,
                       partial);
  else if (nv <= 32)
    hipLaunchKernelGGL((combine_dot_partial<T, 32, SELF>), dim3(nb), dim3(BT), 0, s, y, X, ldx, nv, coef, sign, n,
                       partial);
  else
    hipLaunchKernelGGL((combine_dot_partial<T, MAXV, SELF>), dim3(nb), dim3(BT), 0, s, y, X, ldx, nv, coef, sign, n,
                       partial);
  hipLaunchKernelGGL(multidot_final, dim3(SELF ? 1 : nv), dim3(BT), 0, s, partial, nb, out);
  return hipGetLastError();
}

hipError_t blas_combine_dot(int dtype, void* y, const void* X, int64_t ldx, int nv, const double* coef, double sign,
                            int64_t n, bool self, double* partial, double* out, hipStream_t s) {
  if (nv < 1 || nv > MAXV) return hipErrorInvalidValue;
  if (dtype == SEM_F64) {
    auto* yy = static_cast<double*>(y);
    const auto* xx = static_cast<const double*>(X);
    return self ? run_combine_dot<double, true>(yy, xx, ldx, nv, coef, sign, n, partial, out, s)
                : run_combine_dot<double, false>(yy, xx, ldx, nv, coef, sign, n, partial, out, s);
  }
  auto* yy = static_cast<float*>(y);
  const auto* xx = static_cast<const float*>(X);
  return self ? run_combine_dot<float, true>(yy, xx, ldx, nv, coef, sign, n, partial, out, s)
              : run_combine_dot<float, false>(yy, xx, ldx, nv, coef, sign, n, partial, out, s);
}

hipError_t blas_combine(int dtype, void* y, double alpha, const void* X, int64_t ldx, int nv, const double* coef,
                        double sign, int64_t n, hipStream_t s) {
  if (dtype == SEM_F64)
    hipLaunchKernelGGL(combine<double>, dim3(grid_for(n)), dim3(BT), 0, s, static_cast<double*>(y), alpha,
                       static_cast<const double*>(X), ldx, nv, coef, sign, n);
  else
    hipLaunchKernelGGL(combine<float>, dim3(grid_for(n)), dim3(BT), 0, s, static_cast<float*>(y), alpha,
                       static_cast<const float*>(X), ldx, nv, coef, sign, n);
  return hipGetLastError();
}

hipError_t blas_axpby(int dtype, void* z, double a, const void* x, double b, const void* y, int64_t n,
                      hipStream_t s) {
  if (dtype == SEM_F64)
    hipLaunchKernelGGL(axpby_kernel<double>, dim3(grid_for(n)), dim3(BT), 0, s, static_cast<double*>(z), a,
                       static_cast<const double*>(x), b, static_cast<const double*>(y), n);
  else
    hipLaunchKernelGGL(axpby_kernel<float>, dim3(grid_for(n)), dim3(BT), 0, s, static_cast<float*>(z), a,
                       static_cast<const float*>(x), b, static_cast<const float*>(y), n);
  return hipGetLastError();
}

}  // namespace sem
