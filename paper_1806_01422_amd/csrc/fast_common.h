// Building blocks shared by the tuned order-7 kernels (kern_fast2d.hip, kern_fast3d.hip): the
// even/odd split GLL derivative table, raw buffer accesses, the 8-point line contractions and
// the per-direction element residual contribution of the Burgers operators (Sec. 3.3).
#pragma once
#include "sem_internal.h"

namespace sem {
namespace fast {

constexpr int NQ = 7;  // order

// The even/odd blocks of D are A[i][m] = (D_im - D_i,7-m)/2 and B[i][m] = (D_im + D_i,7-m)/2
// (i, m < 4).  Centro-antisymmetry makes the blocks of D^T their transposes (A' = B^T, B' = A^T),
// so one 32-entry table serves both contractions.
template <typename T>
struct FastTab {
  T A[16], B[16];
  T w[8];            // GLL weights
  T imq[8];          // 1 / (assembled 1-D reference mass at local index q): 1/(2 w_0) at q = 0, 7
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Raw buffer accesses: a lane whose byte offset is out of range (OOB) stores nothing and loads 0,
// so lane predicates become offsets and the store sequence stays free of branches (which keeps
// the compiler's wait counts exact: loads and stores share one counter on this architecture).
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
constexpr uint32_t OOB = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t brsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, (int)off, 0, 0);
}
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, (int)off, 0, 0);
}
// with a wave-uniform part soff of the offset in a scalar register
template <typename T>
__device__ __forceinline__ T bload_s(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, (int)soff, 0));
  else
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, (int)soff, 0));
}
__device__ __forceinline__ void bstore_s(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, (int)off, (int)soff, 0);
}
__device__ __forceinline__ void bstore_s(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, (int)off, (int)soff, 0);
}
template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
  else
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}

// y = D x (TR = false) or y = D^T x (TR = true) on one 8-point line, even/odd split:
//   e_m = x_m + x_{7-m}, o_m = x_m - x_{7-m};  y_i = s_i + d_i, y_{7-i} = s_i - d_i  (i < 4)
//   D:   s_i = sum_m A[i][m] o_m,  d_i = sum_m B[i][m] e_m
//   D^T: s_i = sum_m B[m][i] o_m,  d_i = sum_m A[m][i] e_m
template <bool TR, typename T>
__device__ __forceinline__ void contract(const T (&x)[8], T (&y)[8], const FastTab<T>* __restrict__ tb) {
  const T e0 = x[0] + x[7], e1 = x[1] + x[6], e2 = x[2] + x[5], e3 = x[3] + x[4];
  const T o0 = x[0] - x[7], o1 = x[1] - x[6], o2 = x[2] - x[5], o3 = x[3] - x[4];
  const T* __restrict__ A = tb->A;
  const T* __restrict__ B = tb->B;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    T s, d;
    if constexpr (!TR) {
      s = A[4 * i] * o0 + A[4 * i + 1] * o1 + A[4 * i + 2] * o2 + A[4 * i + 3] * o3;
      d = B[4 * i] * e0 + B[4 * i + 1] * e1 + B[4 * i + 2] * e2 + B[4 * i + 3] * e3;
    } else {
      s = B[i] * o0 + B[4 + i] * o1 + B[8 + i] * o2 + B[12 + i] * o3;
      d = A[i] * e0 + A[4 + i] * e1 + A[8 + i] * e2 + A[12 + i] * e3;
    }
    y[i] = s + d;
    y[7 - i] = s - d;
  }
}

// Contribution of direction j (the lane's register direction) to the element residual of each of
// the NC components.  ldU(i, U) / ldV(i, V) fill the 8 register values of component i of the state and of
// the direction (J v) or scaled adjoint input Z = M^{-1} w (J^T) in the current map; emit(i, P)
// receives the contribution to component i.  om[s] is the quadrature weight at register s (an array
// or an indexable object),
// K1 = nu sc_j^2, K2 = sc_j (the 2/h_j of D on the physical element folded in).
template <typename T, int OP, int NC, typename LU, typename LV, typename OM, typename EM>
__device__ __forceinline__ void map_contrib(int j, LU ldU, LV ldV, const OM& om, T K1, T K2,
                                            const FastTab<T>* __restrict__ tb, EM emit) {
  T c1[8], cu[8];
  {
    T Uj[8];
    ldU(j, Uj);
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      c1[s] = K1 * om[s];
      cu[s] = K2 * om[s] * Uj[s];
    }
  }
  if constexpr (OP == OP_RHS) {
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      T Ui[8], G[8], f[8], t[8];
      ldU(i, Ui);
      contract<false>(Ui, G, tb);
#pragma unroll
      for (int s = 0; s < 8; ++s) f[s] = c1[s] * G[s];
      contract<true>(f, t, tb);
#pragma unroll
      for (int s = 0; s < 8; ++s) t[s] = -(t[s] + cu[s] * G[s]);
      emit(i, t);
    }
  } else if constexpr (OP == OP_JAC) {
    T cv[8];
    {
      T Vj[8];
      ldV(j, Vj);
#pragma unroll
      for (int s = 0; s < 8; ++s) cv[s] = K2 * om[s] * Vj[s];
    }
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      T X[8], G[8], H[8], t[8];
      ldU(i, X);
      contract<false>(X, G, tb);
      ldV(i, X);
      contract<false>(X, H, tb);
#pragma unroll
      for (int s = 0; s < 8; ++s) X[s] = c1[s] * H[s];
      contract<true>(X, t, tb);
#pragma unroll
      for (int s = 0; s < 8; ++s) t[s] = -(t[s] + cv[s] * G[s] + cu[s] * H[s]);
      emit(i, t);
    }
  } else {  // OP_JACT: V holds Z = M^{-1} w
    T acc[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) acc[s] = 0;
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      T X[8], G[8];
      ldU(i, X);
      contract<false>(X, G, tb);
      ldV(i, X);
#pragma unroll
      for (int s = 0; s < 8; ++s) acc[s] += X[s] * G[s];
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) acc[s] *= K2 * om[s];
#pragma unroll
    for (int l = 0; l < NC; ++l) {
      T Zl[8], H[8], t[8];
      ldV(l, Zl);
      contract<false>(Zl, H, tb);
#pragma unroll
      for (int s = 0; s < 8; ++s) H[s] = c1[s] * H[s] + cu[s] * Zl[s];
      contract<true>(H, t, tb);
#pragma unroll
      for (int s = 0; s < 8; ++s) t[s] = (l == j) ? -(t[s] + acc[s]) : -t[s];
      emit(l, t);
    }
  }
}

template <typename T>
__device__ __forceinline__ T coef(const Coef& c, double dt) {
  return (T)(c.c0 + c.cdt * dt);
}

// Workgroup (X, ey) of block `bid`.  Blocks are dealt round-robin to the 8 XCDs; when the count
// allows, consecutive logical workgroups are given to the same XCD so that it sweeps a contiguous
// band of element rows and its L2 serves the rows shared by neighbouring workgroups.
__device__ __forceinline__ int logical_wg(int bid, int nwg) {
  return (nwg % 8 == 0) ? (bid % 8) * (nwg / 8) + bid / 8 : bid;
}

template <typename T>
void fill_tab(int N, FastTab<T>* t) {
  double xi[MAXP], w[MAXP], D[MAXP * MAXP];
  gll_tables(N, xi, w, D);
  for (int i = 0; i < 4; ++i)
    for (int m = 0; m < 4; ++m) {
      const double dim = D[i * 8 + m], dimr = D[i * 8 + 7 - m];
      t->A[4 * i + m] = (T)(0.5 * (dim - dimr));
      t->B[4 * i + m] = (T)(0.5 * (dim + dimr));
    }
  for (int q = 0; q < 8; ++q) {
    t->w[q] = (T)w[q];
    t->imq[q] = (T)(1.0 / ((q == 0 || q == 7) ? 2.0 * w[0] : w[q]));
  }
}

}  // namespace fast
}  // namespace sem
