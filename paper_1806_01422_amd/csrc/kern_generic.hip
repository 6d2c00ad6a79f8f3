// Generic SEM Burgers kernels for any dimension (1-3) and order: one workgroup covers EPB
// elements with one thread per element-local GLL point.
//
//  elem_kernel : gather Q (periodic), sum-factorised contractions with D along each direction
//                (Sec. 3.3: each Kronecker factor acts on one direction), the pointwise flux, the
//                transposed contractions, and a store of the element-local residual R(e, q).
//  dss_kernel  : direct-stiffness summation Q^T at every unique node (1, 2, 4 or 8 element
//                contributions, fixed order), the inverse assembled mass for F and J v, and a fused
//                epilogue (plain store, or the RK4 stage / adjoint-stage updates).
//
//  persist2d_kernel : elem_kernel's work for a batched 2-D set of mixed orders as one persistent
//                launch over a cost-sorted work list.
//
// The element-local residual goes through a scratch array between the element and summation
// kernels; the tuned paths sum inside the workgroup instead (kern_fast2d.hip completely,
// kern_fast3d.hip with a small face fixup).
#include "sem_internal.h"

namespace sem {

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

// Element-launch default: elements per workgroup giving ~256 threads.
constexpr int default_epb(int dim, int P) {
  int nl = ipow(P, dim);
  int e = 256 / nl;
  if (e < 1) e = 1;
  if (e > 32) e = 32;
  // round down to a power of two
  int p = 1;
  while (p * 2 <= e) p *= 2;
  return p;
}

__device__ inline int find_item(const ProbDev* __restrict__ p, int n, int64_t item) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (p[mid].item0 <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ inline int find_node(const ProbDev* __restrict__ p, int n, int64_t item) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (p[mid].node0 <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// loc = b * per + r with per < 2^31 (checked at setup): 32-bit division unless loc itself needs 64
// bits (batches beyond 2^31 values), which keeps the common path free of 64-bit division sequences
__device__ __forceinline__ void split_item(int64_t loc, int64_t per, int& b, int& r) {
  if (loc <= 0x7fffffff) {
    const unsigned l = (unsigned)loc, p = (unsigned)per;
    const unsigned q = l / p;
    b = (int)q;
    r = (int)(l - q * p);
  } else {
    const int64_t q = loc / per;
    b = (int)q;
    r = (int)(loc - q * per);
  }
}

// (D_j S)(q) = sum_m D[q_j][m] S(q; q_j <- m)   (unscaled; caller multiplies by 2/h_j)
template <typename T, int P>
__device__ inline T contract(const T* __restrict__ s, const T* __restrict__ D, int row, int base, int st) {
  T acc = 0;
#pragma unroll
  for (int m = 0; m < P; ++m) acc += D[row * P + m] * s[base + m * st];
  return acc;
}
// (D_j^T S)(q) = sum_m D[m][q_j] S(q; q_j <- m)
template <typename T, int P>
__device__ inline T contract_t(const T* __restrict__ s, const T* __restrict__ D, int col, int base, int st) {
  T acc = 0;
#pragma unroll
  for (int m = 0; m < P; ++m) acc += D[m * P + col] * s[base + m * st];
  return acc;
}

// Element residual of OP for the EPB elements of one workgroup.  Thread tid covers local point
// q of element le = tid / P^DIM; `pr` / `loc` give that element's problem and its index among the
// problem's batch-flattened elements (loc < 0: no element).  sD (P*P), sIn (EPB*NIN*C*NL) and
// sT (EPB*C*DIM*NL) are LDS buffers.  Every thread of the workgroup must call this.
template <typename T, int DIM, int P, int OP, int EPB>
__device__ __forceinline__ void elem_body(int tid, const ProbDev* __restrict__ pr, int64_t loc,
                                          const T* __restrict__ Dg, T* __restrict__ sD, T* __restrict__ sInb,
                                          T* __restrict__ sTb, const T* __restrict__ u, const T* __restrict__ v,
                                          T* __restrict__ L, Coef in_scale) {
  constexpr int NL = ipow(P, DIM);
  constexpr int C = DIM;
  constexpr int NIN = (OP == OP_RHS) ? 1 : 2;
  const int le = tid / NL;
  const int q = tid - le * NL;
  for (int i = tid; i < P * P; i += EPB * NL) sD[i] = Dg[i];
  const bool valid = loc >= 0;
  T* __restrict__ sIn = sInb + le * NIN * C * NL;  // [NIN][C][NL] of this element
  T* __restrict__ sT = sTb + le * C * DIM * NL;    // [C][DIM][NL]
  int qd[3] = {0, 0, 0};
  {
    int t = q;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      qd[k] = t % P;
      t /= P;
    }
  }

  T U[C], V[C];
  T om = 0, nu = 0, sc[3] = {0, 0, 0};
  int64_t lbase = 0;
  if (valid) {
    const int N = pr->N;
    int b, e;
    split_item(loc, pr->nelem, b, e);
    int ed[3];
    {
      const unsigned E0 = (unsigned)pr->E[0], E1 = (unsigned)pr->E[1];
      const unsigned e1 = (unsigned)e / E0;
      ed[0] = (int)((unsigned)e - e1 * E0);
      ed[1] = (int)(e1 % E1);
      ed[2] = (int)(e1 / E1);
    }
    int g = 0, stride = 1;
    double omd = 1.0, mass = 1.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      const int gk = (ed[k] * N + qd[k]) % pr->n[k];
      g += gk * stride;
      stride *= pr->n[k];
      omd *= pr->hh[k] * pr->w[qd[k]];
      mass *= pr->hh[k] * ((qd[k] == 0 || qd[k] == N) ? 2.0 * pr->w[0] : pr->w[qd[k]]);
      sc[k] = (T)pr->sc[k];
    }
    om = (T)omd;
    nu = (T)pr->nu;
    const int64_t base = pr->off + (int64_t)b * C * pr->nodes + g;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      U[c] = u[base + c * pr->nodes];
      sIn[c * NL + q] = U[c];
    }
    if (OP != OP_RHS) {
      T s = 1;
      if (OP == OP_JACT) s = (T)((in_scale.c0 + in_scale.cdt * pr->dt) / mass);  // Z = scale * M^{-1} w
#pragma unroll
      for (int c = 0; c < C; ++c) {
        V[c] = v[base + c * pr->nodes] * s;
        sIn[((NIN - 1) * C + c) * NL + q] = V[c];
      }
    }
    lbase = pr->loff + loc * C * NL + q;
  }
  __syncthreads();

  T adv[C];
  if (valid) {
    T G[C][DIM];
#pragma unroll
    for (int i = 0; i < C; ++i)
#pragma unroll
      for (int j = 0; j < DIM; ++j) {
        const int st = ipow(P, j);
        G[i][j] = sc[j] * contract<T, P>(sIn + i * NL, sD, qd[j], q - qd[j] * st, st);
      }
    if (OP == OP_RHS) {
#pragma unroll
      for (int i = 0; i < C; ++i) {
        T a = 0;
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
          sT[(i * DIM + j) * NL + q] = nu * om * G[i][j];
          a += U[j] * G[i][j];
        }
        adv[i] = om * a;
      }
    } else {
      T H[C][DIM];  // H[i][j] = D_j V_i
#pragma unroll
      for (int i = 0; i < C; ++i)
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
          const int st = ipow(P, j);
          H[i][j] = sc[j] * contract<T, P>(sIn + (C + i) * NL, sD, qd[j], q - qd[j] * st, st);
        }
      if (OP == OP_JAC) {
#pragma unroll
        for (int i = 0; i < C; ++i) {
          T a = 0;
#pragma unroll
          for (int j = 0; j < DIM; ++j) {
            sT[(i * DIM + j) * NL + q] = nu * om * H[i][j];
            a += V[j] * G[i][j] + U[j] * H[i][j];
          }
          adv[i] = om * a;
        }
      } else {  // OP_JACT: V holds Z = M^{-1} w
#pragma unroll
        for (int l = 0; l < C; ++l) {
          T a = 0;
#pragma unroll
          for (int j = 0; j < DIM; ++j) sT[(l * DIM + j) * NL + q] = om * (nu * H[l][j] + U[j] * V[l]);
#pragma unroll
          for (int i = 0; i < C; ++i) a += V[i] * G[i][l];
          adv[l] = om * a;
        }
      }
    }
  }
  __syncthreads();
  if (valid) {
#pragma unroll
    for (int i = 0; i < C; ++i) {
      T r = 0;
#pragma unroll
      for (int j = 0; j < DIM; ++j) {
        const int st = ipow(P, j);
        r += sc[j] * contract_t<T, P>(sT + (i * DIM + j) * NL, sD, qd[j], q - qd[j] * st, st);
      }
      L[lbase + i * NL] = -r - adv[i];
    }
  }
}

template <typename T, int DIM, int P, int OP, int EPB>
__global__ __launch_bounds__(EPB* ipow(P, DIM)) void elem_kernel(const ProbDev* __restrict__ probs, int nprobs,
                                                                  int64_t nitems, const Tables<T>* __restrict__ tab,
                                                                  const T* __restrict__ u, const T* __restrict__ v,
                                                                  T* __restrict__ L, Coef in_scale) {
  constexpr int NL = ipow(P, DIM);
  constexpr int NIN = (OP == OP_RHS) ? 1 : 2;
  __shared__ T sD[P * P];
  __shared__ T sIn[EPB * NIN * DIM * NL];
  __shared__ T sT[EPB * DIM * DIM * NL];
  const int tid = threadIdx.x;
  const int64_t item = (int64_t)blockIdx.x * EPB + tid / NL;
  const bool valid = item < nitems;
  // a workgroup inside one problem (the common case) reads that problem's entry through
  // workgroup-uniform (scalar) loads
  const int64_t first = (int64_t)blockIdx.x * EPB;
  const int64_t last = first + EPB <= nitems ? first + EPB - 1 : nitems - 1;
  const int pf = find_item(probs, nprobs, first);
  if (pf == find_item(probs, nprobs, last)) {
    const ProbDev* pr = probs + pf;
    elem_body<T, DIM, P, OP, EPB>(tid, pr, valid ? item - pr->item0 : -1, tab->D, sD, sIn, sT, u, v, L, in_scale);
  } else {
    const ProbDev* pr = probs + (valid ? find_item(probs, nprobs, item) : 0);
    elem_body<T, DIM, P, OP, EPB>(tid, pr, valid ? item - pr->item0 : -1, tab->D, sD, sIn, sT, u, v, L, in_scale);
  }
}

// Persistent element kernel over a 2-D problem set of mixed orders: workgroup b processes work
// items b, b + G, b + 2G, ... of a list sorted by decreasing cost; each item is up to NT / P^2
// elements of one problem, dispatched on its order.  LDS is sized per thread, so one buffer fits
// every order.
template <typename T, int OP, int NT>
__global__ __launch_bounds__(NT) void persist2d_kernel(const ProbDev* __restrict__ probs,
                                                       const WorkItem* __restrict__ items, int nitems,
                                                       const Tables<T>* __restrict__ tabs,
                                                       const T* __restrict__ u, const T* __restrict__ v,
                                                       T* __restrict__ L, Coef in_scale) {
  constexpr int NIN = (OP == OP_RHS) ? 1 : 2;
  __shared__ T sD[MAXP * MAXP];
  __shared__ T sIn[NT * NIN * 2];
  __shared__ T sT[NT * 4];
  const int tid = threadIdx.x;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const WorkItem w = items[it];
    const ProbDev* pr = probs + w.prob;
    const int NL = w.P * w.P;
    const int le = tid / NL;
    const int64_t loc = (le < w.ne) ? w.e0 + le : -1;
    const T* Dg = tabs[w.P].D;
    switch (w.P) {
#define SEM_PCASE(PV)                                                                                  \
  case PV: {                                                                                           \
    /* one uniform call: threads past the last whole element pass no element */                       \
    constexpr int EPBV = NT / (PV * PV);                                                               \
    const bool act = tid < EPBV * PV * PV;                                                             \
    elem_body<T, 2, PV, OP, EPBV>(act ? tid : EPBV * PV * PV, pr, act ? loc : -1, Dg, sD, sIn, sT, u, v, \
                                  L, in_scale);                                                        \
    break;                                                                                             \
  }
      SEM_PCASE(2) SEM_PCASE(3) SEM_PCASE(4) SEM_PCASE(5) SEM_PCASE(6) SEM_PCASE(7) SEM_PCASE(8)
      SEM_PCASE(9) SEM_PCASE(10) SEM_PCASE(11) SEM_PCASE(12) SEM_PCASE(13)
#undef SEM_PCASE
      default: break;
    }
    __syncthreads();  // the next item overwrites the LDS buffers
  }
}

template <typename T, int DIM, bool DIV>
__device__ __forceinline__ void dss_node(const ProbDev* __restrict__ pr, int64_t item, const T* __restrict__ L,
                                         const Epi& epi) {
  const int N = pr->N, P = pr->P;
  int b, g;
  split_item(item - pr->node0, pr->nodes, b, g);
  int gd[3] = {0, 0, 0};
  {
    unsigned t = (unsigned)g;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      const unsigned nk = (unsigned)pr->n[k], q = t / nk;
      gd[k] = (int)(t - q * nk);
      t = q;
    }
  }
  // contributing (element, local index) pairs per direction: (g/N, g%N) and, on an element
  // face (g%N == 0), also the previous element's last point (periodic wrap)
  int ne[3] = {1, 1, 1}, ee[3][2] = {{0, 0}, {0, 0}, {0, 0}}, qq[3][2] = {{0, 0}, {0, 0}, {0, 0}};
  double mass = 1.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    ee[k][0] = gd[k] / N;
    qq[k][0] = gd[k] - ee[k][0] * N;
    if (qq[k][0] == 0) {
      ne[k] = 2;
      ee[k][1] = (ee[k][0] - 1 + pr->E[k]) % pr->E[k];
      qq[k][1] = N;
      mass *= pr->hh[k] * 2.0 * pr->w[0];
    } else {
      mass *= pr->hh[k] * pr->w[qq[k][0]];
    }
  }
  const int NL = (DIM == 1) ? P : (DIM == 2) ? P * P : P * P * P;
  const int64_t lb = pr->loff + (int64_t)b * pr->nelem * DIM * (int64_t)NL;
  const double dt = pr->dt;
  const T b1 = (T)(epi.b1.c0 + epi.b1.cdt * dt), a1 = (T)(epi.a1.c0 + epi.a1.cdt * dt);
  const T b2 = (T)(epi.b2.c0 + epi.b2.cdt * dt), a2 = (T)(epi.a2.c0 + epi.a2.cdt * dt);
  const T c1 = (T)(epi.c1.c0 + epi.c1.cdt * dt), c2 = (T)(epi.c2.c0 + epi.c2.cdt * dt);
  const int64_t ob = pr->off + (int64_t)b * DIM * pr->nodes + g;
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    T s = 0;
    for (int x = 0; x < ne[0]; ++x)
      for (int y = 0; y < ne[1]; ++y)
        for (int z = 0; z < ne[2]; ++z) {
          const int e = ee[0][x] + pr->E[0] * (ee[1][y] + pr->E[1] * ee[2][z]);  // < nelem < 2^31
          const int q = qq[0][x] + P * (qq[1][y] + P * qq[2][z]);
          s += L[lb + ((int64_t)e * DIM + c) * NL + q];
        }
    if (DIV) s = s / (T)mass;
    const int64_t o = ob + c * pr->nodes;
    // o2 may alias x2: both operands are read before either output is written
    const T v1 = epi.x1 ? static_cast<const T*>(epi.x1)[o] : (T)0;
    const T v2 = epi.x2 ? static_cast<const T*>(epi.x2)[o] : (T)0;
    if (epi.o2) static_cast<T*>(epi.o2)[o] = b2 * s + a2 * v2 + c2 * v1;
    static_cast<T*>(epi.o1)[o] = b1 * s + a1 * v1 + c1 * v2;
  }
}

template <typename T, int DIM, bool DIV>
__global__ __launch_bounds__(256) void dss_kernel(const ProbDev* __restrict__ probs, int nprobs, int64_t nitems,
                                                  const T* __restrict__ L, Epi epi) {
  const int64_t first = (int64_t)blockIdx.x * 256;
  const int64_t item = first + threadIdx.x;
  const int64_t last = first + 256 <= nitems ? first + 255 : nitems - 1;
  // a workgroup inside one problem (the common case) reads its entry through uniform loads
  const int pf = find_node(probs, nprobs, first);
  const bool uniform = pf == find_node(probs, nprobs, last);
  if (item >= nitems) return;
  if (uniform)
    dss_node<T, DIM, DIV>(probs + pf, item, L, epi);
  else
    dss_node<T, DIM, DIV>(probs + find_node(probs, nprobs, item), item, L, epi);
}

// ------------------------------------------------------------------------------------------------
// Dispatch
// ------------------------------------------------------------------------------------------------
template <typename T, int DIM, int P, int OP, int EPB>
static hipError_t run_elem(const ElemLaunch& el, const void* u, const void* v, void* L, Coef sc, const void* tab,
                           hipStream_t s) {
  constexpr int NT = EPB * ipow(P, DIM);
  static_assert(NT <= 1024, "workgroup too large");
  const int64_t blocks = (el.nitems + EPB - 1) / EPB;
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL((elem_kernel<T, DIM, P, OP, EPB>), dim3((unsigned)blocks), dim3(NT), 0, s, el.probs,
                     el.nprobs, el.nitems, static_cast<const Tables<T>*>(tab), static_cast<const T*>(u),
                     static_cast<const T*>(v), static_cast<T*>(L), sc);
  return hipGetLastError();
}

template <typename T, int DIM, int P, int OP>
static hipError_t run_elem_epb(const ElemLaunch& el, const void* u, const void* v, void* L, Coef sc, const void* tab,
                               hipStream_t s) {
  constexpr int DEF = default_epb(DIM, P);
  const int epb = el.epb ? el.epb : DEF;
  // tunable workgroup sizes only for the 2-D batched orders; everything else uses the default
  if constexpr (DIM == 2 && (P == 6 || P == 8 || P == 10)) {
    switch (epb) {
      case 1: return run_elem<T, DIM, P, OP, 1>(el, u, v, L, sc, tab, s);
      case 2: return run_elem<T, DIM, P, OP, 2>(el, u, v, L, sc, tab, s);
      case 4: return run_elem<T, DIM, P, OP, 4>(el, u, v, L, sc, tab, s);
      case 8:
        if constexpr (8 * P * P <= 1024) return run_elem<T, DIM, P, OP, 8>(el, u, v, L, sc, tab, s);
        break;
      case 16:
        if constexpr (16 * P * P <= 1024) return run_elem<T, DIM, P, OP, 16>(el, u, v, L, sc, tab, s);
        break;
      default: break;
    }
    return hipErrorInvalidValue;
  } else {
    if (epb != DEF) return hipErrorInvalidValue;
    return run_elem<T, DIM, P, OP, DEF>(el, u, v, L, sc, tab, s);
  }
}

hipError_t launch_persist2d(const ProbDev* probs, const WorkItem* items, int nitems, int grid, int op, int dtype,
                            const void* tabs, const void* u, const void* v, void* lvec, Coef in_scale, hipStream_t s) {
  constexpr int NT = 256;
  if (nitems <= 0) return hipSuccess;
  if (dtype == SEM_F64) {
    const auto* tb = static_cast<const Tables<double>*>(tabs);
    const auto* uu = static_cast<const double*>(u);
    const auto* vv = static_cast<const double*>(v);
    auto* L = static_cast<double*>(lvec);
    if (op == OP_RHS)
      hipLaunchKernelGGL((persist2d_kernel<double, OP_RHS, NT>), dim3(grid), dim3(NT), 0, s, probs, items, nitems, tb, uu,
                         vv, L, in_scale);
    else if (op == OP_JAC)
      hipLaunchKernelGGL((persist2d_kernel<double, OP_JAC, NT>), dim3(grid), dim3(NT), 0, s, probs, items, nitems, tb, uu,
                         vv, L, in_scale);
    else
      hipLaunchKernelGGL((persist2d_kernel<double, OP_JACT, NT>), dim3(grid), dim3(NT), 0, s, probs, items, nitems, tb,
                         uu, vv, L, in_scale);
  } else {
    const auto* tb = static_cast<const Tables<float>*>(tabs);
    const auto* uu = static_cast<const float*>(u);
    const auto* vv = static_cast<const float*>(v);
    auto* L = static_cast<float*>(lvec);
    if (op == OP_RHS)
      hipLaunchKernelGGL((persist2d_kernel<float, OP_RHS, NT>), dim3(grid), dim3(NT), 0, s, probs, items, nitems, tb, uu,
                         vv, L, in_scale);
    else if (op == OP_JAC)
      hipLaunchKernelGGL((persist2d_kernel<float, OP_JAC, NT>), dim3(grid), dim3(NT), 0, s, probs, items, nitems, tb, uu,
                         vv, L, in_scale);
    else
      hipLaunchKernelGGL((persist2d_kernel<float, OP_JACT, NT>), dim3(grid), dim3(NT), 0, s, probs, items, nitems, tb,
                         uu, vv, L, in_scale);
  }
  return hipGetLastError();
}

int persist2d_elems_per_item(int P) { return 256 / (P * P); }

int elem_epb_choices(int dim, int P, int* out, int max_out) {
  int n = 0;
  if (dim == 2 && (P == 6 || P == 8 || P == 10)) {
    for (int e : {1, 2, 4, 8, 16})
      if (e * P * P <= 1024 && n < max_out) out[n++] = e;
  } else if (n < max_out) {
    out[n++] = default_epb(dim, P);
  }
  return n;
}

template <typename T, int DIM, int P>
static hipError_t run_elem_op(const ElemLaunch& el, int op, const void* u, const void* v, void* L, Coef sc,
                              const void* tab, hipStream_t s) {
  switch (op) {
    case OP_RHS: return run_elem_epb<T, DIM, P, OP_RHS>(el, u, v, L, sc, tab, s);
    case OP_JAC: return run_elem_epb<T, DIM, P, OP_JAC>(el, u, v, L, sc, tab, s);
    case OP_JACT: return run_elem_epb<T, DIM, P, OP_JACT>(el, u, v, L, sc, tab, s);
  }
  return hipErrorInvalidValue;
}

#define SEM_P_CASE(DIMV, PV) \
  case PV: return run_elem_op<T, DIMV, PV>(el, op, u, v, L, sc, tab, s);

template <typename T>
static hipError_t run_elem_dim(const ElemLaunch& el, int op, const void* u, const void* v, void* L, Coef sc,
                               const void* tab, hipStream_t s) {
  if (el.dim == 1) {
    switch (el.P) {
      SEM_P_CASE(1, 2) SEM_P_CASE(1, 3) SEM_P_CASE(1, 4) SEM_P_CASE(1, 5) SEM_P_CASE(1, 6) SEM_P_CASE(1, 7)
      SEM_P_CASE(1, 8) SEM_P_CASE(1, 9) SEM_P_CASE(1, 10) SEM_P_CASE(1, 11) SEM_P_CASE(1, 12) SEM_P_CASE(1, 13)
    }
  } else if (el.dim == 2) {
    switch (el.P) {
      SEM_P_CASE(2, 2) SEM_P_CASE(2, 3) SEM_P_CASE(2, 4) SEM_P_CASE(2, 5) SEM_P_CASE(2, 6) SEM_P_CASE(2, 7)
      SEM_P_CASE(2, 8) SEM_P_CASE(2, 9) SEM_P_CASE(2, 10) SEM_P_CASE(2, 11) SEM_P_CASE(2, 12) SEM_P_CASE(2, 13)
    }
  } else if (el.dim == 3) {
    switch (el.P) {
      SEM_P_CASE(3, 2) SEM_P_CASE(3, 3) SEM_P_CASE(3, 4) SEM_P_CASE(3, 5) SEM_P_CASE(3, 6) SEM_P_CASE(3, 7)
      SEM_P_CASE(3, 8) SEM_P_CASE(3, 9) SEM_P_CASE(3, 10)
    }
  }
  return hipErrorInvalidValue;
}
#undef SEM_P_CASE

hipError_t launch_elem(const ElemLaunch& el, int op, const void* u, const void* v, void* lvec, Coef in_scale,
                       const void* tables, hipStream_t s) {
  if (el.dtype == SEM_F64) return run_elem_dim<double>(el, op, u, v, lvec, in_scale, tables, s);
  return run_elem_dim<float>(el, op, u, v, lvec, in_scale, tables, s);
}

template <typename T, int DIM>
static hipError_t run_dss(const ProbDev* probs, int32_t nprobs, int64_t nitems, int div, const void* L,
                          const Epi& epi, hipStream_t s) {
  const int64_t blocks = (nitems + 255) / 256;
  if (blocks <= 0) return hipSuccess;
  if (div)
    hipLaunchKernelGGL((dss_kernel<T, DIM, true>), dim3((unsigned)blocks), dim3(256), 0, s, probs, nprobs, nitems,
                       static_cast<const T*>(L), epi);
  else
    hipLaunchKernelGGL((dss_kernel<T, DIM, false>), dim3((unsigned)blocks), dim3(256), 0, s, probs, nprobs, nitems,
                       static_cast<const T*>(L), epi);
  return hipGetLastError();
}

hipError_t launch_dss(const ProbDev* probs, int32_t nprobs, int64_t nitems, int dim, int dtype, int div,
                      const void* lvec, const Epi& epi, hipStream_t s) {
  if (dtype == SEM_F64) {
    if (dim == 1) return run_dss<double, 1>(probs, nprobs, nitems, div, lvec, epi, s);
    if (dim == 2) return run_dss<double, 2>(probs, nprobs, nitems, div, lvec, epi, s);
    return run_dss<double, 3>(probs, nprobs, nitems, div, lvec, epi, s);
  }
  if (dim == 1) return run_dss<float, 1>(probs, nprobs, nitems, div, lvec, epi, s);
  if (dim == 2) return run_dss<float, 2>(probs, nprobs, nitems, div, lvec, epi, s);
  return run_dss<float, 3>(probs, nprobs, nitems, div, lvec, epi, s);
}

// Assembled diagonal GLL mass (Sec. 3.2: the lumped mass of the collocation quadrature) of every
// node of one problem-table entry, written to every component of its fields:
//   M[g] = prod_k (h_k / 2) (2 w_0 if g_k mod N = 0, else w_{g_k mod N}).
template <typename T>
__global__ __launch_bounds__(256) void mass_kernel(ProbDev p, T* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)p.batch * p.nodes) return;
  const int64_t b = t / p.nodes, g = t - b * p.nodes;
  int64_t r = g;
  double m = 1.0;
  for (int k = 0; k < p.dim; ++k) {
    const int64_t gk = r % p.n[k];
    r /= p.n[k];
    const int q = (int)(gk % p.N);
    m *= p.hh[k] * (q == 0 ? 2.0 * p.w[0] : p.w[q]);
  }
  T* __restrict__ o = out + p.off + b * p.dim * p.nodes + g;
  for (int c = 0; c < p.dim; ++c) o[c * p.nodes] = (T)m;
}

hipError_t launch_mass(const ProbDev& hp, void* out, int dtype, hipStream_t s) {
  const int64_t blocks = ((int64_t)hp.batch * hp.nodes + 255) / 256;
  if (blocks <= 0) return hipSuccess;
  if (dtype == SEM_F64)
    hipLaunchKernelGGL(mass_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s, hp, static_cast<double*>(out));
  else
    hipLaunchKernelGGL(mass_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s, hp, static_cast<float*>(out));
  return hipGetLastError();
}

}  // namespace sem
