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
#include "fast_consts.h"  // written by the build (gen/fast_consts_gen.hip)

namespace sem {
namespace {

using namespace fast;
// Lane layout per order.  Up to 8 points per line (orders 3, 5, 7) an element has 8 lanes and a
// wavefront 8 elements; with 10 points (order 9) an element has 16 lanes (6 of them padding) and a
// wavefront 4 elements.  A workgroup holds at most MAXW wavefronts: a whole element row for
// P <= 8 (up to 64 elements); for P = 10 at most 16 elements, so longer rows are split into
// x-segments of one workgroup each (see "x-segments" above).
template <int P>
struct Lay {
  static constexpr int LPE = P <= 8 ? 8 : 16;  // lanes per element
  static constexpr int EW = 64 / LPE;          // elements per wavefront along x
  static constexpr int MAXW = P <= 8 ? 8 : 4;  // wavefronts per workgroup
  // Padded LDS index of point (a, b) of element slot e: TE e + TB b + a.  Modulo 32 (the 8-byte
  // bank pairs of 64 banks), with LPE = 8: 8e + a + 9b, so with b fixed (y-map) the 32 lanes
  // e in 0..3 (or 4..7), a in 0..7 hit 32 distinct pairs, and with a fixed (x-map)
  // 8 ((e + b) mod 4) + b is distinct over b in 0..7, e in 0..3.  With LPE = 16: 16e + 17b + a,
  // so with b fixed a + 16e (a in 0..15, e in 0..1) is distinct, and with a fixed 17b + 16e is:
  // 17b mod 32 runs through the even residues 0..14 and the odd ones 17..31 for b in 0..15.
  // Either map addresses its registers as one lane base plus immediate offsets.
  static constexpr int TB = LPE + 1;
  static constexpr int TE = LPE == 8 ? 72 : 176;  // >= P TB, and 8 (or 16) modulo 32
  static constexpr int TC = EW * TE;              // component stride
};


struct Fast2Args {
  int Ex, Ey, nx, ny;
  int nw;    // wavefronts per workgroup
  int nxs;   // x-segments per element row (Ex / (nw EW))
  int S;     // element rows per segment
  int nseg;  // row segments per batch member
  int nwg;   // workgroups (batch * nseg * nxs)
  double hh[2], sc[2], nu;
  int64_t nodes;  // per component
  const ProbDev* prob;
};

template <int P>
__device__ __forceinline__ int tix2(int e, int a, int b) {
  return Lay<P>::TE * e + Lay<P>::TB * b + a;
}

// LDS per workgroup: per wavefront a tile of NIN * 2 components x TC points, then the x-face
// exchange between wavefronts [step parity][wavefront][component][b].
// Order 9 adds a copy of the coefficient table (read from LDS by J^T; see fast2d_body).
template <typename T, int P>
constexpr size_t lds_bytes(int nin, int nw) {
  return sizeof(T) * ((size_t)nw * nin * 2 * Lay<P>::TC + (size_t)2 * nw * 2 * Lay<P>::LPE) +
         (P > 8 ? sizeof(FastTab<T, P>) : 0);
}

// The work of one workgroup: a row segment of one field, or of one x-segment of it (all values
// wavefront-uniform).
struct Fast2Job {
  int Ey, nx, ny, nw, y0, nrows;
  int x0;      // first element column of the workgroup
  bool xsplit; // the row is split into x-segments: the left face is completed here
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
  constexpr int LPE = Lay<P>::LPE, EW = Lay<P>::EW, TC = Lay<P>::TC;
  // The coefficient table of a phase.  Orders up to 7: a fresh pointer per phase (phase_ptr),
  // except for J^T, which measured 4-5% faster reading the table through the kernel argument.
  // Order 9: the two 5 x 5 blocks alone (100 scalar registers) overflow the scalar file, and the
  // compiler then parks the coefficients of a run-time table in vector-register lanes and
  // restores each with two lane reads before every use (over half of the loop's VALU
  // instructions).
  //   F and J v (FP64) take the coefficients as compile-time constants (FastConst, written by the
  //     build from the same table routine): each is formed with two scalar moves next to its use,
  //     and the kernel keeps two wavefronts per SIMD (order-9 F 112 -> 82 us).
  //   J^T copies the table into LDS once and reads each coefficient with a broadcast LDS read
  //     into a vector register: no lane moves, at one wavefront per SIMD instead of two, 10%
  //     faster; with the constants it needs one register more than two wavefronts allow and is
  //     slower than from LDS.
  //   FP32 keeps the run-time table (its scalar file holds the single-precision blocks).
  constexpr bool CTAB = P == 10 && sizeof(T) == 8 && OP != OP_JACT;
  constexpr bool LTAB = P > 8 && OP == OP_JACT;
  FastTab<T, P>* ltab = nullptr;
  if constexpr (LTAB) {
    ltab = reinterpret_cast<FastTab<T, P>*>(lds + (size_t)g.nw * NIN * 2 * TC + (size_t)2 * g.nw * 2 * LPE);
    const T* __restrict__ src = reinterpret_cast<const T*>(tb);
    T* __restrict__ dst = reinterpret_cast<T*>(ltab);
    for (int k = threadIdx.x; k < (int)(sizeof(FastTab<T, P>) / sizeof(T)); k += blockDim.x) dst[k] = src[k];
    __syncthreads();
  }
  static constexpr FastConst<10> ctab{};
  auto tph = [&]() {
    if constexpr (CTAB) return &ctab;
    else if constexpr (LTAB) return static_cast<const FastTab<T, P>*>(ltab);
    else if constexpr (OP == OP_JACT) return tb;
    else return phase_ptr(tb);
  };

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

  const int e = lane / LPE;  // element slot of the wavefront
  const int a = lane % LPE;  // y-map: column a of the lane's line (>= P: padding)
  // x-map: row b = l0.  Padding rows of the 8-lane layout stay inside the 72-value element block;
  // with 16 lanes they would not, so those padding lanes take row N (and write the same values
  // as its own lane).
  const int l0 = P > 8 ? min(a, N) : a;
  const int lp = min(a, N);  // table index of the lane's point (padding lanes: point N)
  // quadrature weight omega = (h_x h_y / 4) w_a w_b; with the lane holding one index and the
  // register the other, the same lane factor serves both maps
  const T omf = (T)(g.hh[0] * g.hh[1]) * tb->w[lp];
  // x-segmented rows: the workgroup's left face (column N x0, point a = 0 of wavefront 0's slot
  // 0) is completed here.  The missing left element shares the own element's y-lines there, so
  // its y-terms equal the own ones and are doubled; its x-terms come from its x-lines
  // (line_end_terms).  The right face is left to the next x-segment.
  constexpr bool SPLITS = P > 8;  // only order 9 splits rows into x-segments
  const bool lface = SPLITS && g.xsplit && wave == 0 && e == 0;
  const T omyf = (lface && a == 0) ? (T)2 * omf : omf;
  const T K1x = (T)(g.nu * g.sc[0] * g.sc[0]), K1y = (T)(g.nu * g.sc[1] * g.sc[1]);
  const T K2x = (T)g.sc[0], K2y = (T)g.sc[1];
  // inverse assembled mass, lane factor of the y-map
  const T mlane = tb->imq[lp] * (T)(1.0 / (g.hh[0] * g.hh[1]));
  const T zin = (T)(in_scale.c0 + in_scale.cdt * dt) * mlane;  // J^T input: scale * M^{-1} w

  T* __restrict__ tU = lds + (size_t)wave * NIN * 2 * TC;
  T* __restrict__ tV = tU + 2 * TC;
  T* __restrict__ sEx = lds + (size_t)nw * NIN * 2 * TC;  // [2][nw][2][LPE]

  // y-map global addressing: column of the lane's line, periodic in x and y
  int col = N * (g.x0 + EW * wave + e) + (a <= N ? a : N);
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
      const auto ts = tph();
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int b = 0; b < P; ++b) cv[i][b] *= zin * ts->imq[b];
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int b = 0; b < P; ++b) {
        tU[i * TC + tix2<P>(e, a, b)] = cu[i][b];
        if constexpr (HASV) tV[i * TC + tix2<P>(e, a, b)] = cv[i][b];
      }
    T r[2][P];
    const auto ty = tph();
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
        OmLane<T, decltype(ty->w + 0)>{omyf, ty->w}, K1y, K2y, ty,
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
    // the state tile once that component has been read.  On a left face, the left element's
    // x-terms at its last point are added at a = 0 (its lines' last point is the own node).
    T lowX[2] = {0, 0};
    if (SPLITS && lface) {
      const auto tl = tph();
      T XU[2][P], XV[2][P];
      const uint32_t rb = (uint32_t)((int64_t)((N * ey + l0) % g.ny) * g.nx * sizeof(T));
      const int xl0 = (g.x0 == 0 ? g.nx : N * g.x0) - N;  // first column of the left element
#pragma unroll
      for (int p = 0; p < N; ++p)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const uint32_t uni = (uint32_t)((i * g.nodes + xl0 + p) * sizeof(T));
          XU[i][p] = bload_s<T>(r_u, rb, uni);
          if constexpr (HASV) XV[i][p] = bload_s<T>(r_v, rb, uni);
        }
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        XU[i][N] = tU[i * TC + tix2<P>(e, 0, l0)];
        if constexpr (HASV) {
          XV[i][N] = tV[i * TC + tix2<P>(e, 0, l0)];
          if constexpr (OP == OP_JACT) {
#pragma unroll
            for (int p = 0; p < N; ++p) XV[i][p] *= zin * tl->imq[p];
          }
        }
      }
      line_end_terms<T, OP, 2, P>(0, XU, XV, omf * tl->w[N], K1x, K2x, tl, lowX);
    }
    const auto tx = tph();
    map_contrib<T, OP, 2, P>(
        0,
        [&](int i, T (&X)[P]) {
#pragma unroll
          for (int q = 0; q < P; ++q) X[q] = tU[i * TC + tix2<P>(e, q, l0)];
        },
        [&](int i, T (&X)[P]) {
#pragma unroll
          for (int q = 0; q < P; ++q) X[q] = tV[i * TC + tix2<P>(e, q, l0)];
        },
        OmLane<T, decltype(tx->w + 0)>{omf, tx->w}, K1x, K2x, tx,
        [&](int i, const T (&Pv)[P]) {
          tU[i * TC + tix2<P>(e, 0, l0)] = SPLITS ? Pv[0] + lowX[i] : Pv[0];
#pragma unroll
          for (int q = 1; q < P; ++q) tU[i * TC + tix2<P>(e, q, l0)] = Pv[q];
        });
    if constexpr (HASV) load_rows(ey_next, 1, true, true, cu, cv);
    wave_sync();
    // ---- back to the y-map: element residual r = y part + x part
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int b = 0; b < P; ++b) r[i][b] += tU[i * TC + tix2<P>(e, a, b)];
    // ---- x-direction summation: the a = N line of slot e goes to the a = 0 line of slot e + 1
    // (inside the wavefront through the tile, across wavefronts through sEx, double-buffered by
    // step parity: one barrier per step)
    const int par = k & 1;
    wave_sync();
    if (a == N) {
      T* __restrict__ dst = (e < EW - 1) ? tU + LPE * e : sEx + ((par * nw + wave) * 2) * LPE;
      const int ist = (e < EW - 1) ? 64 : LPE;
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int b = 0; b < P; ++b) dst[i * ist + b] = r[i][b];
    }
    __syncthreads();
    if (a == 0 && !lface) {  // a left face has its left element's terms already
      const int wl = wave == 0 ? nw - 1 : wave - 1;
      const T* __restrict__ src = (e > 0) ? tU + LPE * (e - 1) : sEx + ((par * nw + wl) * 2) * LPE;
      const int ist = (e > 0) ? 64 : LPE;
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
    const auto te = tph();
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
        const T sm = (OP != OP_JACT) ? r[i][b] * (mlane * te->imq[b]) : r[i][b];
        T r1 = b1 * sm;
        if (EP >= 1) r1 += a1 * E1[i][b];
        if (EP >= 2) r1 += c1 * E2[i][b];
        bstore_s(r_o1, vo, rowoff(i, N * ey + b), r1);
        if (EP >= 2) bstore_s(r_o2, vo, rowoff(i, N * ey + b), a2 * E2[i][b] + c2 * E1[i][b] + b2 * sm);
      }
  }
}

// One field or a same-shape batch: workgroup L takes x-segment L % nxs of row segment
// (L / nxs) % nseg of batch member L / (nxs nseg).
template <typename T, int OP, int EP, int P>
__global__ __launch_bounds__(64 * Lay<P>::MAXW) void fast2d_kernel(Fast2Args a, const FastTab<T, P>* __restrict__ tb,
                                                                   const T* __restrict__ u, const T* __restrict__ v,
                                                                   Epi epi, Coef in_scale) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int L = logical_wg(blockIdx.x, a.nwg);
  const int per = a.nseg * a.nxs;
  const int bm = L / per, rem = L - bm * per, seg = rem / a.nxs, xs = rem - seg * a.nxs;
  Fast2Job g;
  g.Ey = a.Ey, g.nx = a.nx, g.ny = a.ny, g.nw = a.nw;
  g.x0 = xs * a.nw * Lay<P>::EW;
  g.xsplit = a.nxs > 1;
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
__global__ __launch_bounds__(64 * Lay<P>::MAXW) void fast2d_batch_kernel(const ProbDev* __restrict__ probs,
                                                                 const Fast2Item* __restrict__ items,
                                                                 const FastTab<T, P>* __restrict__ tb,
                                                                 const T* __restrict__ u, const T* __restrict__ v,
                                                                 Epi epi, Coef in_scale) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const Fast2Item it = items[blockIdx.x];
  const ProbDev* __restrict__ pr = probs + it.prob;
  Fast2Job g;
  g.Ey = pr->E[1], g.nx = pr->n[0], g.ny = pr->n[1], g.nw = blockDim.x >> 6;
  g.x0 = it.x0;
  g.xsplit = pr->E[0] > g.nw * Lay<P>::EW;
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

// Wavefronts per workgroup for a row of ex elements: the whole row up to MAXW wavefronts, else
// the largest divisor of the row's wavefront count that fits (x-segments of equal length).
template <int P>
int waves_of(int ex) {
  int nw = ex / Lay<P>::EW;
  if (nw <= Lay<P>::MAXW) return nw;
  for (int d = Lay<P>::MAXW; d >= 1; --d)
    if (nw % d == 0) return d;
  return 1;
}

template <int P>
Fast2Args make_args(const ProbDev& hp, const ProbDev* dprob, int op) {
  Fast2Args g;
  g.Ex = hp.E[0];
  g.Ey = hp.E[1];
  g.nx = hp.n[0];
  g.ny = hp.n[1];
  g.nw = waves_of<P>(hp.E[0]);
  g.nxs = hp.E[0] / (g.nw * Lay<P>::EW);
  const int64_t target = op == OP_RHS ? SEM_FAST2D_TARGET_F : SEM_FAST2D_TARGET_J;
  int64_t s = ((int64_t)hp.E[1] * hp.batch * g.nxs + target - 1) / target;
  if (s < 1) s = 1;
  if (s > hp.E[1]) s = hp.E[1];
  g.S = (int)s;
  g.nseg = (hp.E[1] + g.S - 1) / g.S;
  g.nwg = g.nseg * g.nxs * hp.batch;
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
  const size_t lds = lds_bytes<T, P>(NIN, g.nw);
  hipLaunchKernelGGL((fast2d_kernel<T, OP, EP, P>), dim3(g.nwg), dim3(64 * g.nw), lds, s, g, tb,
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
  const Fast2Args g = make_args<P>(hp, dprob, op);
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
  const int bytes = (int)lds_bytes<T, P>(NIN, Lay<P>::MAXW);
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
  const size_t lds = lds_bytes<T, P>(NIN, nw);
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
  // odd orders 3, 5, 7 (P = N + 1 even, at most the 8 lanes of an element): one workgroup spans a
  // whole element row (8 elements per wavefront, at most 8 wavefronts).  Order 9: 16 lanes and
  // 4 elements per wavefront, rows of any multiple of 4 elements in x-segments of at most 16.
  // Buffer offsets are 32-bit: one batch member (both components, FP64) must stay below 2 GiB.
  const bool rows = (hp.N == 3 || hp.N == 5 || hp.N == 7) ? (hp.E[0] % 8 == 0 && hp.E[0] <= 64)
                    : hp.N == 9                             ? hp.E[0] % 4 == 0
                                                            : false;
  return hp.dim == 2 && rows && hp.E[0] >= 1 && hp.E[1] >= 1 && (int64_t)2 * hp.nodes * 8 < ((int64_t)1 << 31);
}

// the tuned orders N = 3, 5, 7, 9 have P = N + 1 = 4, 6, 8, 10 points per line
#define SEM_FAST2D_ORDERS(X) \
  case 3: X(4);              \
  case 5: X(6);              \
  case 9: X(10);             \
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

int fast2d_waves(const ProbDev& hp) { return hp.N == 9 ? waves_of<10>(hp.E[0]) : waves_of<8>(hp.E[0]); }

int fast2d_xsegments(const ProbDev& hp) { return hp.E[0] / (fast2d_waves(hp) * (hp.N == 9 ? 4 : 8)); }

hipError_t launch_fast2d_batch(const ProbDev* dprobs, const Fast2Item* items, int nitems, int nw, int N, int op,
                               const void* u, const void* v, const Epi& epi, Coef in_scale, const void* dtables,
                               int dtype, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  if (nw < 1 || nw > (N == 9 ? Lay<10>::MAXW : Lay<8>::MAXW)) return hipErrorInvalidValue;
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
