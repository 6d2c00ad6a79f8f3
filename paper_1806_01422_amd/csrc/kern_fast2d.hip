// Tuned 2-D kernel for the odd orders N = 3, 5, 7 (P = N + 1 = 4, 6, 8 GLL points per direction) on
// gfx950: element contractions, direct-stiffness summation Q^T, inverse mass and the stage
// epilogue in one launch, with no element-local scratch array.
//
// Work decomposition.  A workgroup owns one whole element row along x (Ex = 8 * nw elements,
// wavefront w takes elements 8w .. 8w + 7) and sweeps a segment of S element rows along y, one
// row per step.  The wavefronts of a workgroup therefore read and write whole grid rows.
//
// Every lane holds element lines of P points in one of two maps:
//     y-map  lane = a + 8e, register b      (global loads and stores: 8N + 1 / 8N contiguous values)
//     x-map  lane = b + 8e, register a
// Each element has 8 lanes; for P < 8 the lanes with a (or b) >= P only pad: their values are
// never read by a point of the element, and they store nothing.
// with e the element slot of the wavefront and (a, b) the element-local (x, y) GLL indices.  The
// y-direction part of the residual is formed in the y-map from registers, the x-direction part
// in the x-map from an XOR-swizzled LDS tile, and the x part returns to the y-map through the
// same tile (Sec. 3.3: sum factorisation, one direction at a time, with the even/odd split of D).
//
// Direct-stiffness summation.
//   x: point a = N of slot e is point a = 0 of slot e + 1; the partial sums are added through
//      LDS, across wavefronts (and periodically from the last wavefront to the first) after one
//      workgroup barrier per step.  Lanes with a >= N store nothing.
//   y: point b = N of row ey is point b = 0 of row ey + 1: its partial sum is carried in
//      registers along the sweep, as is the input line b = N (N new grid rows per step).  The
//      first step of a segment recomputes the row before it (periodically) without storing, so
//      the carry into the segment's first grid row is complete and every node is written once,
//      by one lane, as part of whole row segments of 8N nodes.
#include "fast_common.h"

namespace sem {
namespace {

using namespace fast;
constexpr int EW = 8;    // elements per wavefront along x
constexpr int MAXW = 8;  // wavefronts per workgroup

// omega at register s: a lane factor times a GLL weight (uniform), formed where it is used
template <typename T>
struct OmLane {
  T f;
  const T* __restrict__ w;
  __device__ __forceinline__ T operator[](int s) const { return f * w[s]; }
};

struct Fast2Args {
  int Ex, Ey, nx, ny;
  int nw;    // wavefronts per workgroup (Ex / 8)
  int S;     // element rows per segment
  int nseg;  // segments per batch member
  int nwg;   // workgroups (batch * nseg)
  double hh[2], sc[2], nu;
  int64_t nodes;  // per component
  const ProbDev* prob;
};

// Padded LDS index of point (a, b) of element slot e: 72e + 9b + a (rows of 9, elements of 72).
// Modulo 32 (the 8-byte bank pairs of 64 banks) this is 8e + a + 9b: with b fixed (y-map) the
// 32 lanes e in 0..3 (or 4..7), a in 0..7 hit 32 distinct pairs, and with a fixed (x-map)
// 8 ((e + b) mod 4) + b is distinct over b in 0..7, e in 0..3.  Either map addresses its 8
// registers as one lane base plus immediate offsets.
constexpr int TE = 72, TB = 9, TC = EW * TE;  // element, row and component strides
__device__ __forceinline__ int tix2(int e, int a, int b) { return TE * e + TB * b + a; }

// LDS per workgroup: per wavefront a tile of NIN * 2 components x TC points, then the x-face
// exchange between wavefronts [step parity][wavefront][component][b].
template <typename T>
constexpr size_t lds_bytes(int nin, int nw) {
  return sizeof(T) * ((size_t)nw * nin * 2 * TC + (size_t)2 * nw * 2 * 8);
}

// The work of one workgroup: a row segment of one field (all values wavefront-uniform).
struct Fast2Job {
  int Ey, nx, ny, nw, y0, nrows;
  int64_t nodes;  // per component
  int64_t bo;     // values before the field (batch member or packed problem)
  double hh[2], sc[2], nu, dt;
};

// EP: epilogue variant known at compile time: 0 = o1 = b1 s; 1 = o1 = a1 x1 + b1 s;
// 2 = o1 = a1 x1 + c1 x2 + b1 s and (when o2 is given) o2 = a2 x2 + c2 x1 + b2 s.
template <typename T, int OP, int EP, int P>
__device__ __forceinline__ void fast2d_body(const Fast2Job& g, const FastTab<T, P>* __restrict__ tb,
                                            const T* __restrict__ u, const T* __restrict__ v, const Epi& epi,
                                            Coef in_scale, T* __restrict__ lds) {
  constexpr bool HASV = OP != OP_RHS;
  constexpr int NIN = HASV ? 2 : 1;
  constexpr int N = P - 1;

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nw = g.nw;
  const int y0 = g.y0, nrows = g.nrows;
  const int64_t bo = g.bo;
  const uint32_t fbytes = (uint32_t)(2 * g.nodes * sizeof(T));
  const __amdgpu_buffer_rsrc_t r_u = brsrc(u + bo, fbytes);
  const __amdgpu_buffer_rsrc_t r_v = brsrc(HASV ? v + bo : u, HASV ? fbytes : 0);
  const __amdgpu_buffer_rsrc_t r_o1 = brsrc(static_cast<T*>(epi.o1) + bo, fbytes);
  // a missing operand gets an empty range: its loads return 0 and its stores are dropped
  const bool hx1 = EP >= 1 && epi.x1, ho2 = EP >= 2 && epi.o2, hx2 = EP >= 2 && epi.x2;
  const __amdgpu_buffer_rsrc_t r_x1 = brsrc(hx1 ? static_cast<const T*>(epi.x1) + bo : u, hx1 ? fbytes : 0);
  const __amdgpu_buffer_rsrc_t r_o2 = brsrc(ho2 ? static_cast<T*>(epi.o2) + bo : u, ho2 ? fbytes : 0);
  const __amdgpu_buffer_rsrc_t r_x2 = brsrc(hx2 ? static_cast<const T*>(epi.x2) + bo : u, hx2 ? fbytes : 0);
  const double dt = g.dt;
  const T a1 = coef<T>(epi.a1, dt), b1 = coef<T>(epi.b1, dt), a2 = coef<T>(epi.a2, dt), b2 = coef<T>(epi.b2, dt);
  const T c1 = coef<T>(epi.c1, dt), c2 = coef<T>(epi.c2, dt);

  const int l0 = lane & 7, e = lane >> 3;  // y-map: a = l0; x-map: b = l0
  const int a = l0;
  const int lp = l0 < P ? l0 : N;  // table index of the lane's point (padding lanes: any valid one)
  // quadrature weight omega = (h_x h_y / 4) w_a w_b; with the lane holding one index and the
  // register the other, the same lane factor serves both maps
  const OmLane<T> om{(T)(g.hh[0] * g.hh[1]) * tb->w[lp], tb->w};
  const T K1x = (T)(g.nu * g.sc[0] * g.sc[0]), K1y = (T)(g.nu * g.sc[1] * g.sc[1]);
  const T K2x = (T)g.sc[0], K2y = (T)g.sc[1];
  // inverse assembled mass, lane factor of the y-map
  const T mlane = tb->imq[lp] * (T)(1.0 / (g.hh[0] * g.hh[1]));
  const T zin = (T)(in_scale.c0 + in_scale.cdt * dt) * mlane;  // J^T input: scale * M^{-1} w

  T* __restrict__ tU = lds + (size_t)wave * NIN * 2 * TC;
  T* __restrict__ tV = tU + 2 * TC;
  T* __restrict__ sEx = lds + (size_t)nw * NIN * 2 * TC;  // [2][nw][2][8]

  // y-map global addressing: column of the lane's line, periodic in x and y
  int col = N * (EW * wave + e) + (a <= N ? a : N);
  if (col >= g.nx) col -= g.nx;

  // the lane's byte offset in a grid row; the row and component part is uniform (scalar offset)
  const uint32_t lcol = (uint32_t)(col * sizeof(T));
  auto rowoff = [&](int i, int y) { return (uint32_t)((i * g.nodes + (int64_t)y * g.nx) * sizeof(T)); };
  // lines b0..7 of element row ey of the state (WU) and of the second input (WV)
  auto load_rows = [&](int ey, int b0, bool WU, bool WV, T (&UU)[2][P], T (&VV)[2][P]) {
#pragma unroll
    for (int b = 0; b < P; ++b) {
      if (b < b0) continue;
      int yb = N * ey + b;
      if (yb >= g.ny) yb -= g.ny;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        if (WU) UU[i][b] = bload_s<T>(r_u, lcol, rowoff(i, yb));
        if (HASV && WV) VV[i][b] = bload_s<T>(r_v, lcol, rowoff(i, yb));
      }
    }
  };

  T cu[2][P], cv[2][P];
  const int ey_first = y0 == 0 ? g.Ey - 1 : y0 - 1;
  load_rows(ey_first, 0, true, true, cu, cv);
  T carry[2] = {0, 0};

  // step 0 recomputes the row before the segment (carry only); steps 1..nrows own rows y0 + k - 1
  for (int k = 0; k <= nrows; ++k) {
    const int ey = k == 0 ? ey_first : y0 + k - 1;
    const bool st = k > 0;
    // ---- y-map: stage the element tile, y-direction part in registers
    T vlast[2];  // unscaled input line b = N, the next row's line b = 0
#pragma unroll
    for (int i = 0; i < 2; ++i) vlast[i] = cv[i][N];
    if constexpr (OP == OP_JACT) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int b = 0; b < P; ++b) cv[i][b] *= zin * tb->imq[b];
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int b = 0; b < P; ++b) {
        tU[i * TC + tix2(e, a, b)] = cu[i][b];
        if constexpr (HASV) tV[i * TC + tix2(e, a, b)] = cv[i][b];
      }
    T r[2][P];
    map_contrib<T, OP, 2, P>(
        1,
        [&](int i, T (&X)[P]) {
#pragma unroll
          for (int b = 0; b < P; ++b) X[b] = cu[i][b];
        },
        [&](int i, T (&X)[P]) {
#pragma unroll
          for (int b = 0; b < P; ++b) X[b] = cv[i][b];
        },
        om, K1y, K2y, tb,
        [&](int i, const T (&Pv)[P]) {
#pragma unroll
          for (int b = 0; b < P; ++b) r[i][b] = Pv[b];
        });
    // the y-map lines are no longer needed: move line 7 to line 0 and prefetch the next row's
    // lines 1..7 (unconditionally: the last step loads the row after the segment).  With a second
    // input (J v, J^T) both prefetches wait until after the x part: in flight during it, they
    // would push the kernel past its 256 registers.
    const int ey_next = ey + 1 < g.Ey ? ey + 1 : 0;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      cu[i][0] = cu[i][N];
      if constexpr (HASV) cv[i][0] = vlast[i];
    }
    if constexpr (!HASV) load_rows(ey_next, 1, true, false, cu, cv);
    wave_sync();
    // ---- x-map (lane (b = l0, e), register a): x-direction part, written over component i of
    // the state tile once that component has been read
    map_contrib<T, OP, 2, P>(
        0,
        [&](int i, T (&X)[P]) {
#pragma unroll
          for (int q = 0; q < P; ++q) X[q] = tU[i * TC + tix2(e, q, l0)];
        },
        [&](int i, T (&X)[P]) {
#pragma unroll
          for (int q = 0; q < P; ++q) X[q] = tV[i * TC + tix2(e, q, l0)];
        },
        om, K1x, K2x, tb,
        [&](int i, const T (&Pv)[P]) {
#pragma unroll
          for (int q = 0; q < P; ++q) tU[i * TC + tix2(e, q, l0)] = Pv[q];
        });
    if constexpr (HASV) load_rows(ey_next, 1, true, true, cu, cv);
    wave_sync();
    // ---- back to the y-map: element residual r = y part + x part
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int b = 0; b < P; ++b) r[i][b] += tU[i * TC + tix2(e, a, b)];
    // ---- x-direction summation: the a = N line of slot e goes to the a = 0 line of slot e + 1
    // (inside the wavefront through the tile, across wavefronts through sEx, double-buffered by
    // step parity: one barrier per step)
    const int par = k & 1;
    wave_sync();
    if (a == N) {
      T* __restrict__ dst = (e < EW - 1) ? tU + 8 * e : sEx + ((par * nw + wave) * 2) * 8;
      const int ist = (e < EW - 1) ? 64 : 8;
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int b = 0; b < P; ++b) dst[i * ist + b] = r[i][b];
    }
    __syncthreads();
    if (a == 0) {
      const int wl = wave == 0 ? nw - 1 : wave - 1;
      const T* __restrict__ src = (e > 0) ? tU + 8 * (e - 1) : sEx + ((par * nw + wl) * 2) * 8;
      const int ist = (e > 0) ? 64 : 8;
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int b = 0; b < P; ++b) r[i][b] += src[i * ist + b];
    }
    // ---- y-direction summation: carry the shared line
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      r[i][0] += carry[i];
      carry[i] = r[i][N];
    }
    // ---- outputs: grid rows N ey .. N ey + N - 1, lanes a < N (inverse mass for F and J v); all
    // epilogue operands are read first (o2 may alias x2)
    const uint32_t vo = (st && a < N) ? lcol : OOB;
    T E1[2][N], E2[2][N];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int b = 0; b < N; ++b) {
        E1[i][b] = (EP >= 1) ? bload_s<T>(r_x1, vo, rowoff(i, N * ey + b)) : (T)0;
        E2[i][b] = (EP >= 2) ? bload_s<T>(r_x2, vo, rowoff(i, N * ey + b)) : (T)0;
      }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int b = 0; b < N; ++b) {
        const T sm = (OP != OP_JACT) ? r[i][b] * (mlane * tb->imq[b]) : r[i][b];
        T r1 = b1 * sm;
        if (EP >= 1) r1 += a1 * E1[i][b];
        if (EP >= 2) r1 += c1 * E2[i][b];
        bstore_s(r_o1, vo, rowoff(i, N * ey + b), r1);
        if (EP >= 2) bstore_s(r_o2, vo, rowoff(i, N * ey + b), a2 * E2[i][b] + c2 * E1[i][b] + b2 * sm);
      }
  }
}

// One field or a same-shape batch: workgroup L takes segment L % nseg of batch member L / nseg.
template <typename T, int OP, int EP, int P>
__global__ __launch_bounds__(64 * MAXW) void fast2d_kernel(Fast2Args a, const FastTab<T, P>* __restrict__ tb,
                                                           const T* __restrict__ u, const T* __restrict__ v,
                                                           Epi epi, Coef in_scale) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int L = logical_wg(blockIdx.x, a.nwg);
  const int bm = L / a.nseg, seg = L - bm * a.nseg;
  Fast2Job g;
  g.Ey = a.Ey, g.nx = a.nx, g.ny = a.ny, g.nw = a.nw;
  g.y0 = seg * a.S;
  g.nrows = min(a.S, a.Ey - g.y0);
  g.nodes = a.nodes;
  g.bo = (int64_t)bm * 2 * a.nodes;
  g.hh[0] = a.hh[0], g.hh[1] = a.hh[1], g.sc[0] = a.sc[0], g.sc[1] = a.sc[1], g.nu = a.nu;
  g.dt = a.prob->dt;
  fast2d_body<T, OP, EP, P>(g, tb, u, v, epi, in_scale, reinterpret_cast<T*>(lds_raw));
}

// Problems of a batched set with the same x element count: workgroup b takes work item b, a row
// segment of one packed problem (its constants read from the problem table).
template <typename T, int OP, int EP, int P>
__global__ __launch_bounds__(64 * MAXW) void fast2d_batch_kernel(const ProbDev* __restrict__ probs,
                                                                 const Fast2Item* __restrict__ items,
                                                                 const FastTab<T, P>* __restrict__ tb,
                                                                 const T* __restrict__ u, const T* __restrict__ v,
                                                                 Epi epi, Coef in_scale) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const Fast2Item it = items[blockIdx.x];
  const ProbDev* __restrict__ pr = probs + it.prob;
  Fast2Job g;
  g.Ey = pr->E[1], g.nx = pr->n[0], g.ny = pr->n[1], g.nw = pr->E[0] / EW;
  g.y0 = it.y0;
  g.nrows = it.nrows;
  g.nodes = pr->nodes;
  g.bo = pr->off;
  g.hh[0] = pr->hh[0], g.hh[1] = pr->hh[1], g.sc[0] = pr->sc[0], g.sc[1] = pr->sc[1], g.nu = pr->nu;
  g.dt = pr->dt;
  fast2d_body<T, OP, EP, P>(g, tb, u, v, epi, in_scale, reinterpret_cast<T*>(lds_raw));
}

// Segment length: about one workgroup per CU (256), so every workgroup starts in the first wave
// of dispatch and the recomputed rows stay few (measured on 64 fields of 64 x 64 elements: 128,
// 512, 1024 or 4096 workgroups are 5-50% slower for F, J v and J^T alike).  Small launches go down
// to one row per segment: recomputing every row is cheaper there than running half as many
// workgroups (one 64 x 64 field: 10.7 instead of 14.3 us for F).
#ifndef SEM_FAST2D_TARGET_F
#define SEM_FAST2D_TARGET_F 256
#endif
#ifndef SEM_FAST2D_TARGET_J
#define SEM_FAST2D_TARGET_J 256
#endif

Fast2Args make_args(const ProbDev& hp, const ProbDev* dprob, int op) {
  Fast2Args g;
  g.Ex = hp.E[0];
  g.Ey = hp.E[1];
  g.nx = hp.n[0];
  g.ny = hp.n[1];
  g.nw = hp.E[0] / EW;
  const int64_t target = op == OP_RHS ? SEM_FAST2D_TARGET_F : SEM_FAST2D_TARGET_J;
  int64_t s = ((int64_t)hp.E[1] * hp.batch + target - 1) / target;
  if (s < 1) s = 1;
  if (s > hp.E[1]) s = hp.E[1];
  g.S = (int)s;
  g.nseg = (hp.E[1] + g.S - 1) / g.S;
  g.nwg = g.nseg * hp.batch;
  for (int k = 0; k < 2; ++k) {
    g.hh[k] = hp.hh[k];
    g.sc[k] = hp.sc[k];
  }
  g.nu = hp.nu;
  g.nodes = hp.nodes;
  g.prob = dprob;
  return g;
}

template <typename T, int OP, int EP, int P>
hipError_t launch_one(const Fast2Args& g, const FastTab<T, P>* tb, const T* u, const T* v, const Epi& epi,
                      Coef in_scale, hipStream_t s) {
  constexpr int NIN = OP == OP_RHS ? 1 : 2;
  hipLaunchKernelGGL((fast2d_kernel<T, OP, EP, P>), dim3(g.nwg), dim3(64 * g.nw), lds_bytes<T>(NIN, g.nw), s, g, tb,
                     u, v, epi, in_scale);
  return hipGetLastError();
}

template <typename T, int OP, int P>
hipError_t launch_ep(const Fast2Args& g, const FastTab<T, P>* tb, const T* u, const T* v, const Epi& epi,
                     Coef in_scale, hipStream_t s) {
  const int ep = (epi.o2 || epi.x2) ? 2 : (epi.x1 ? 1 : 0);
  if (ep == 0) return launch_one<T, OP, 0, P>(g, tb, u, v, epi, in_scale, s);
  if (ep == 1) return launch_one<T, OP, 1, P>(g, tb, u, v, epi, in_scale, s);
  return launch_one<T, OP, 2, P>(g, tb, u, v, epi, in_scale, s);
}

template <typename T, int P>
hipError_t run_fast2(const ProbDev& hp, const ProbDev* dprob, int op, const void* u, const void* v, const Epi& epi,
                     Coef in_scale, const void* dtab, hipStream_t s) {
  const Fast2Args g = make_args(hp, dprob, op);
  const auto* tb = static_cast<const FastTab<T, P>*>(dtab);
  const T* uu = static_cast<const T*>(u);
  const T* vv = static_cast<const T*>(v);
  if (op == OP_RHS) return launch_ep<T, OP_RHS, P>(g, tb, uu, vv, epi, in_scale, s);
  if (op == OP_JAC) return launch_ep<T, OP_JAC, P>(g, tb, uu, vv, epi, in_scale, s);
  return launch_ep<T, OP_JACT, P>(g, tb, uu, vv, epi, in_scale, s);
}

template <typename T, int OP, int P>
hipError_t allow_lds_op() {
  constexpr int NIN = OP == OP_RHS ? 1 : 2;
  const int bytes = (int)lds_bytes<T>(NIN, MAXW);
  const void* fns[6] = {reinterpret_cast<const void*>(&fast2d_kernel<T, OP, 0, P>),
                        reinterpret_cast<const void*>(&fast2d_kernel<T, OP, 1, P>),
                        reinterpret_cast<const void*>(&fast2d_kernel<T, OP, 2, P>),
                        reinterpret_cast<const void*>(&fast2d_batch_kernel<T, OP, 0, P>),
                        reinterpret_cast<const void*>(&fast2d_batch_kernel<T, OP, 1, P>),
                        reinterpret_cast<const void*>(&fast2d_batch_kernel<T, OP, 2, P>)};
  for (const void* f : fns) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T, int OP, int P>
hipError_t run_batch_op(const ProbDev* probs, const Fast2Item* items, int nitems, int nw, const T* u, const T* v,
                        const Epi& epi, Coef in_scale, const FastTab<T, P>* tb, hipStream_t s) {
  constexpr int NIN = OP == OP_RHS ? 1 : 2;
  const int ep = (epi.o2 || epi.x2) ? 2 : (epi.x1 ? 1 : 0);
  const dim3 grid(nitems), block(64 * nw);
  const size_t lds = lds_bytes<T>(NIN, nw);
  if (ep == 0)
    hipLaunchKernelGGL((fast2d_batch_kernel<T, OP, 0, P>), grid, block, lds, s, probs, items, tb, u, v, epi, in_scale);
  else if (ep == 1)
    hipLaunchKernelGGL((fast2d_batch_kernel<T, OP, 1, P>), grid, block, lds, s, probs, items, tb, u, v, epi, in_scale);
  else
    hipLaunchKernelGGL((fast2d_batch_kernel<T, OP, 2, P>), grid, block, lds, s, probs, items, tb, u, v, epi, in_scale);
  return hipGetLastError();
}

template <typename T, int P>
hipError_t run_batch(const ProbDev* probs, const Fast2Item* items, int nitems, int nw, int op, const void* u,
                     const void* v, const Epi& epi, Coef in_scale, const void* dtab, hipStream_t s) {
  const auto* tb = static_cast<const FastTab<T, P>*>(dtab);
  const T* uu = static_cast<const T*>(u);
  const T* vv = static_cast<const T*>(v);
  if (op == OP_RHS) return run_batch_op<T, OP_RHS, P>(probs, items, nitems, nw, uu, vv, epi, in_scale, tb, s);
  if (op == OP_JAC) return run_batch_op<T, OP_JAC, P>(probs, items, nitems, nw, uu, vv, epi, in_scale, tb, s);
  return run_batch_op<T, OP_JACT, P>(probs, items, nitems, nw, uu, vv, epi, in_scale, tb, s);
}

template <typename T, int P>
hipError_t allow_lds() {
  hipError_t e;
  if ((e = allow_lds_op<T, OP_RHS, P>()) != hipSuccess) return e;
  if ((e = allow_lds_op<T, OP_JAC, P>()) != hipSuccess) return e;
  return allow_lds_op<T, OP_JACT, P>();
}

// device tables of order N: FastTab<double, N + 1> followed by FastTab<float, N + 1>
template <int P>
size_t table_bytes() {
  return sizeof(FastTab<double, P>) + sizeof(FastTab<float, P>);
}
template <int P>
void fill_tables(void* host) {
  fill_tab<double, P>(static_cast<FastTab<double, P>*>(host));
  fill_tab<float, P>(reinterpret_cast<FastTab<float, P>*>(static_cast<char*>(host) + sizeof(FastTab<double, P>)));
}

}  // namespace

bool fast2d_supported(const ProbDev& hp) {
  // odd orders up to 7 (P = N + 1 even, at most the 8 lanes of an element); one workgroup spans a
  // whole element row (8 elements per wavefront, at most 8 wavefronts); buffer offsets are 32-bit:
  // one batch member (both components, FP64) must stay below 2 GiB
  return hp.dim == 2 && (hp.N == 3 || hp.N == 5 || hp.N == 7) && hp.E[0] % EW == 0 && hp.E[0] >= EW &&
         hp.E[0] <= EW * MAXW && hp.E[1] >= 1 && (int64_t)2 * hp.nodes * 8 < ((int64_t)1 << 31);
}

// the tuned orders N = 3, 5, 7 have P = N + 1 = 4, 6, 8 points per line
#define SEM_FAST2D_ORDERS(X) \
  case 3: X(4);              \
  case 5: X(6);              \
  default: X(8);

size_t fast_table_bytes(int N) {
#define SEM_X(PV) return table_bytes<PV>()
  switch (N) { SEM_FAST2D_ORDERS(SEM_X) }
#undef SEM_X
}

void fast_fill_tables(int N, void* host) {
#define SEM_X(PV) return fill_tables<PV>(host)
  switch (N) { SEM_FAST2D_ORDERS(SEM_X) }
#undef SEM_X
}

hipError_t fast2d_prepare(int N, int dtype) {
#define SEM_X(PV) return dtype == SEM_F64 ? allow_lds<double, PV>() : allow_lds<float, PV>()
  switch (N) { SEM_FAST2D_ORDERS(SEM_X) }
#undef SEM_X
}

int fast2d_waves(const ProbDev& hp) { return hp.E[0] / EW; }

hipError_t launch_fast2d_batch(const ProbDev* dprobs, const Fast2Item* items, int nitems, int nw, int N, int op,
                               const void* u, const void* v, const Epi& epi, Coef in_scale, const void* dtables,
                               int dtype, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  if (nw < 1 || nw > MAXW) return hipErrorInvalidValue;
#define SEM_X(PV)                                                                                                   \
  return dtype == SEM_F64                                                                                           \
             ? run_batch<double, PV>(dprobs, items, nitems, nw, op, u, v, epi, in_scale, dtables, s)               \
             : run_batch<float, PV>(dprobs, items, nitems, nw, op, u, v, epi, in_scale,                            \
                                    static_cast<const char*>(dtables) + sizeof(FastTab<double, PV>), s)
  switch (N) { SEM_FAST2D_ORDERS(SEM_X) }
#undef SEM_X
}

hipError_t launch_fast2d(const ProbDev& hp, const ProbDev* dprob, int op, const void* u, const void* v, const Epi& epi,
                         Coef in_scale, const void* dtables, int dtype, hipStream_t s) {
#define SEM_X(PV)                                                                                    \
  return dtype == SEM_F64 ? run_fast2<double, PV>(hp, dprob, op, u, v, epi, in_scale, dtables, s)  \
                          : run_fast2<float, PV>(hp, dprob, op, u, v, epi, in_scale,               \
                                                 static_cast<const char*>(dtables) + sizeof(FastTab<double, PV>), s)
  switch (hp.N) { SEM_FAST2D_ORDERS(SEM_X) }
#undef SEM_X
}
#undef SEM_FAST2D_ORDERS

}  // namespace sem
