// Building blocks shared by the tuned kernels (kern_fast2d.hip: orders 3, 5, 7; kern_fast3d.hip:
// order 7): the even/odd split GLL derivative table, raw buffer accesses, the line contractions
// and the per-direction element residual contribution of the Burgers operators (Sec. 3.3).  P is
// the number of GLL points per line (N + 1, even).
#pragma once
#include "sem_internal.h"

namespace sem {
namespace fast {

constexpr int NQ = 7;  // order

// The even/odd blocks of D are A[i][m] = (D_im - D_i,P-1-m)/2 and B[i][m] = (D_im + D_i,P-1-m)/2
// (i, m < P/2).  Centro-antisymmetry makes the blocks of D^T their transposes (A' = B^T,
// B' = A^T), so one table of P^2/2 entries serves both contractions.
template <typename T, int P = 8>
struct FastTab {
  static constexpr int H = P / 2;
  T A[H * H], B[H * H];
  T w[P];    // GLL weights
  T imq[P];  // 1 / (assembled 1-D reference mass at local index q): 1/(2 w_0) at q = 0, P - 1
  // A line's last point (used where a tile completes a face from a neighbour's line):
  //   D7[n] = D_{P-1,n}  (the derivative there),
  //   Kw[n] = K_{P-1,n} / w_{P-1} with K = D^T W D the 1-D stiffness (the weak second derivative
  //           of D^T (w D x) evaluated there, divided by the point's weight),
  //   Dw[m] = D_{m,P-1} w_m / w_{P-1}  (D^T (w y) evaluated there, divided by the point's weight).
  T D7[P], Kw[P], Dw[P];
};

// The same (uniform) table pointer, opaque to the compiler and in the constant address space:
// loads through it are scalar loads that cannot be hoisted across the point where it is taken.
// A kernel that sweeps a loop takes one per phase of the loop body, so the table's coefficients
// are re-read from the scalar cache where a phase needs them instead of being held in scalar
// registers for the whole loop (which overflows them: the compiler then parks the values in
// vector-register lanes and restores each with two lane reads before every use).
template <typename P>
using const_ptr = const __attribute__((address_space(4))) P*;
template <typename P>
__device__ __forceinline__ const_ptr<P> phase_ptr(const P* p) {
  uint64_t v = reinterpret_cast<uint64_t>(p);
  asm volatile("" : "+s"(v));
  return reinterpret_cast<const_ptr<P>>(v);
}

// omega at register s: a lane factor times a GLL weight (uniform, read through WP), formed where
// it is used
template <typename T, typename WP>
struct OmLane {
  T f;
  WP w;
  __device__ __forceinline__ T operator[](int s) const { return f * w[s]; }
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

// y = D x (TR = false) or y = D^T x (TR = true) on one P-point line, even/odd split (H = P/2):
//   e_m = x_m + x_{P-1-m}, o_m = x_m - x_{P-1-m};  y_i = s_i + d_i, y_{P-1-i} = s_i - d_i  (i < H)
//   D:   s_i = sum_m A[i][m] o_m,  d_i = sum_m B[i][m] e_m
//   D^T: s_i = sum_m B[m][i] o_m,  d_i = sum_m A[m][i] e_m
template <bool TR, typename T, int P, typename TB>
__device__ __forceinline__ void contract(const T (&x)[P], T (&y)[P], TB tb) {
  constexpr int H = P / 2;
  T e[H], o[H];
#pragma unroll
  for (int m = 0; m < H; ++m) {
    e[m] = x[m] + x[P - 1 - m];
    o[m] = x[m] - x[P - 1 - m];
  }
  const auto A = tb->A;
  const auto B = tb->B;
#pragma unroll
  for (int i = 0; i < H; ++i) {
    T s, d;
    if constexpr (!TR) {
      s = A[H * i] * o[0];
      d = B[H * i] * e[0];
#pragma unroll
      for (int m = 1; m < H; ++m) {
        s += A[H * i + m] * o[m];
        d += B[H * i + m] * e[m];
      }
    } else {
      s = B[i] * o[0];
      d = A[i] * e[0];
#pragma unroll
      for (int m = 1; m < H; ++m) {
        s += B[H * m + i] * o[m];
        d += A[H * m + i] * e[m];
      }
    }
    y[i] = s + d;
    y[P - 1 - i] = s - d;
  }
}

// Contribution of direction j (the lane's register direction) to the element residual of each of
// the NC components.  ldU(i, U) / ldV(i, V) fill the P register values of component i of the state and of
// the direction (J v) or scaled adjoint input Z = M^{-1} w (J^T) in the current map; emit(i, P)
// receives the contribution to component i.  om[s] is the quadrature weight at register s (an array
// or an indexable object),
// K1 = nu sc_j^2, K2 = sc_j (the 2/h_j of D on the physical element folded in).
template <typename T, int OP, int NC, int P = 8, typename LU, typename LV, typename OM, typename TB, typename EM>
__device__ __forceinline__ void map_contrib(int j, LU ldU, LV ldV, const OM& om, T K1, T K2, TB tb, EM emit) {
  T c1[P], cu[P];
  {
    T Uj[P];
    ldU(j, Uj);
#pragma unroll
    for (int s = 0; s < P; ++s) {
      c1[s] = K1 * om[s];
      cu[s] = K2 * om[s] * Uj[s];
    }
  }
  if constexpr (OP == OP_RHS) {
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      T Ui[P], G[P], f[P], t[P];
      ldU(i, Ui);
      contract<false>(Ui, G, tb);
#pragma unroll
      for (int s = 0; s < P; ++s) f[s] = c1[s] * G[s];
      contract<true>(f, t, tb);
#pragma unroll
      for (int s = 0; s < P; ++s) t[s] = -(t[s] + cu[s] * G[s]);
      emit(i, t);
    }
  } else if constexpr (OP == OP_JAC) {
    T cv[P];
    {
      T Vj[P];
      ldV(j, Vj);
#pragma unroll
      for (int s = 0; s < P; ++s) cv[s] = K2 * om[s] * Vj[s];
    }
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      T X[P], G[P], H[P], t[P];
      ldU(i, X);
      contract<false>(X, G, tb);
      ldV(i, X);
      contract<false>(X, H, tb);
#pragma unroll
      for (int s = 0; s < P; ++s) X[s] = c1[s] * H[s];
      contract<true>(X, t, tb);
#pragma unroll
      for (int s = 0; s < P; ++s) t[s] = -(t[s] + cv[s] * G[s] + cu[s] * H[s]);
      emit(i, t);
    }
  } else {  // OP_JACT: V holds Z = M^{-1} w
    T acc[P];
#pragma unroll
    for (int s = 0; s < P; ++s) acc[s] = 0;
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      T X[P], G[P];
      ldU(i, X);
      contract<false>(X, G, tb);
      ldV(i, X);
#pragma unroll
      for (int s = 0; s < P; ++s) acc[s] += X[s] * G[s];
    }
#pragma unroll
    for (int s = 0; s < P; ++s) acc[s] *= K2 * om[s];
#pragma unroll
    for (int l = 0; l < NC; ++l) {
      T Zl[P], H[P], t[P];
      ldV(l, Zl);
      contract<false>(Zl, H, tb);
#pragma unroll
      for (int s = 0; s < P; ++s) H[s] = c1[s] * H[s] + cu[s] * Zl[s];
      contract<true>(H, t, tb);
#pragma unroll
      for (int s = 0; s < P; ++s) t[s] = (l == j) ? -(t[s] + acc[s]) : -t[s];
      emit(l, t);
    }
  }
}

// Direction-j terms of an element's residual (the map_contrib terms) at the last point of its
// lines, from whole lines: UL[i] / VL[i] hold component i of the state and of the second input
// (J v: v; J^T: Z = M^{-1} w) at the P points of the lane's line, om7 the quadrature weight at the
// last point, K1 = nu sc_j^2 and K2 = sc_j as for map_contrib.  With the stiffness row
// K_{P-1,.} = sum_m D_{m,P-1} w_m D_{m,.} the two contractions collapse to dot products:
//   F:   out_i = -om7 (K1 Kw.U_i + K2 U_j(P-1) D7.U_i)
//   J v: out_i = -om7 (K1 Kw.V_i + K2 (V_j(P-1) D7.U_i + U_j(P-1) D7.V_i))
//   J^T: out_l = -om7 (K1 Kw.Z_l + K2 Dw.(U_j Z_l)) - [l = j] om7 K2 sum_i Z_i(P-1) D7.U_i
template <typename T, int OP, int NC, int P = 8, typename TB>
__device__ __forceinline__ void line_end_terms(int j, const T (&UL)[NC][P], const T (&VL)[NC][P], T om7, T K1, T K2,
                                               TB tb, T (&out)[NC]) {
  constexpr int L = P - 1;
  const auto D7 = tb->D7;
  const auto Kw = tb->Kw;
  if constexpr (OP == OP_RHS) {
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      T k = Kw[0] * UL[i][0], d = D7[0] * UL[i][0];
#pragma unroll
      for (int n = 1; n < P; ++n) {
        k += Kw[n] * UL[i][n];
        d += D7[n] * UL[i][n];
      }
      out[i] = -om7 * (K1 * k + K2 * UL[j][L] * d);
    }
  } else if constexpr (OP == OP_JAC) {
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      T k = Kw[0] * VL[i][0], du = D7[0] * UL[i][0], dv = D7[0] * VL[i][0];
#pragma unroll
      for (int n = 1; n < P; ++n) {
        k += Kw[n] * VL[i][n];
        du += D7[n] * UL[i][n];
        dv += D7[n] * VL[i][n];
      }
      out[i] = -om7 * (K1 * k + K2 * (VL[j][L] * du + UL[j][L] * dv));
    }
  } else {
    const auto Dw = tb->Dw;
    T acc = 0;
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      T du = D7[0] * UL[i][0];
#pragma unroll
      for (int n = 1; n < P; ++n) du += D7[n] * UL[i][n];
      acc += VL[i][L] * du;
    }
#pragma unroll
    for (int l = 0; l < NC; ++l) {
      T k = Kw[0] * VL[l][0], a = Dw[0] * (UL[j][0] * VL[l][0]);
#pragma unroll
      for (int n = 1; n < P; ++n) {
        k += Kw[n] * VL[l][n];
        a += Dw[n] * (UL[j][n] * VL[l][n]);
      }
      out[l] = -om7 * (K1 * k + K2 * a + (l == j ? K2 * acc : (T)0));
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

template <typename T, int P>
void fill_tab(FastTab<T, P>* t) {
  constexpr int H = P / 2;
  double xi[MAXP], w[MAXP], D[MAXP * MAXP];
  gll_tables(P - 1, xi, w, D);
  for (int i = 0; i < H; ++i)
    for (int m = 0; m < H; ++m) {
      const double dim = D[i * P + m], dimr = D[i * P + P - 1 - m];
      t->A[H * i + m] = (T)(0.5 * (dim - dimr));
      t->B[H * i + m] = (T)(0.5 * (dim + dimr));
    }
  for (int q = 0; q < P; ++q) {
    t->w[q] = (T)w[q];
    t->imq[q] = (T)(1.0 / ((q == 0 || q == P - 1) ? 2.0 * w[0] : w[q]));
  }
  const int L = P - 1;
  for (int n = 0; n < P; ++n) {
    long double k = 0;
    for (int m = 0; m < P; ++m) k += (long double)D[m * P + L] * w[m] * D[m * P + n];
    t->D7[n] = (T)D[L * P + n];
    t->Kw[n] = (T)(k / w[L]);
    t->Dw[n] = (T)((long double)D[n * P + L] * w[n] / w[L]);
  }
}

}  // namespace fast
}  // namespace sem
