// Tuned 3-D kernels for order N = 7 (8 GLL points per direction) on gfx950.
//
// Work decomposition.  A workgroup of 4 wavefronts owns 4 consecutive elements along x of one
// element row in y (wavefront w takes element 4X + w) and sweeps that block along z, one element
// layer per step.  Concurrently running wavefronts therefore touch contiguous x-ranges: the 4
// wavefronts of a workgroup read and write 224 contiguous bytes of every grid row they cover, and
// the workgroups of one XCD (block ids are remapped so that each XCD holds a contiguous band of
// element rows) cover whole rows.  Lines shared by neighbouring elements are then fetched once and
// written whole, instead of once per element step as in a sweep along x.
//
// Every lane keeps whole element lines in registers in one of three maps:
//     z-map  lane = a + 8b, register c      (global loads and stores: 8 lanes, 64 contiguous bytes)
//     y-map  lane = a + 8c, register b
//     x-map  lane = b + 8c, register a      (x-direction summation)
// with (a, b, c) the element-local (x, y, z) GLL indices.  The element tile moves between maps
// through an XOR-swizzled LDS tile.  The contraction with D along the register direction uses
// the centro-antisymmetry of the GLL differentiation matrix (D_{N-i,N-j} = -D_ij): even/odd
// halves of the line need 32 multiply-adds instead of 64 (Sec. 3.3 sum factorisation, one
// direction at a time).
//
// Direct-stiffness summation (Q^T).
//   z: the last plane (c = 7) of an element is the first plane (c = 0) of the next one in the
//      sweep; its partial sum is carried in registers, and the periodic wrap is closed after the
//      sweep.  The input plane is carried too, so each step loads 7 new planes.  A sweep split
//      into z-segments instead starts each segment by recomputing the layer before it.
//   x: inside a workgroup the shared face of wavefronts w and w + 1 is added through LDS.
//   workgroup faces: a workgroup owns the nodes x in [28X, 28X + 28), y in [7ey, 7ey + 7) and
//      completes them itself, so every output node is written once, by one lane, and no other
//      launch follows.  The element residual is a sum of per-direction terms, each a function of
//      the element's line through the node along that direction only (Sec. 3.3: the operators
//      are sums over directions j of D_j^T(.) and pointwise D_j terms; for J v and J^T the same
//      holds with the second input's line beside the state's).  At a node of the lower face
//      (y = 7ey) the missing element row below shares the own element's x- and z-lines (GLL
//      weights w_0 = w_7, equal element sizes), so its x- and z-terms equal the own ones: they
//      are doubled, and only its y-term is formed, from its y-lines (line_end_terms).  The left
//      face (x = 28X, wavefront 0) is completed the same way with the left element's x-lines; at
//      the corner line both rules apply (the diagonal element's terms are the doubled y-term of
//      the lower and x-term of the left element).  The upper and right faces are left to the
//      workgroups that own them.
//   workgroup faces of the segmented FP32 J^T (face_buffer_variant):
//      the workgroup writes its finished nodes to the output and, to a face buffer, its partial sums of the lower y-row (y = 7ey), its contributions to the upper
//      y-row and upper x-column (owned by the neighbours), and the first 32-byte sector of each
//      interior row (x in [28X, 28X + 4): the x = 28X node still lacks the left neighbour's
//      part).  fast3d_fixup adds the parts and applies M^{-1} (J v) and the epilogue, and writes
//      those nodes as whole row segments and whole sectors, so no 32-byte sector of the output is
//      written twice.
#include "fast_common.h"

namespace sem {
namespace {

using namespace fast;
constexpr int WX = 4;  // elements per workgroup along x, one per wavefront
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
// Face buffer of one batch member: four regions, each [workgroup][component][grid plane z][width]
// so that every region is read by one neighbour's fixup as a run contiguous in z.
//   LY  own lower y-row y = 7ey, x-local 0..27 (partial sums)             width 28
//   UY  upper y-row y = 7ey + 7, x-local 0..28 (contribution to neighbours) width 29
//   UX  upper x-column x = 28X + 28, y-local 0..6                          width 7
//   LX  first sector x-local 0..3 of the rows y-local 1..6                 width 24
// Region g starts at NWG * 3 * nz * (sum of the widths before it).
constexpr int W_LY = 28, W_UY = 29, W_UX = 7, W_LX = 24;
constexpr int O_LY = 0, O_UY = 28, O_UX = 57, O_LX = 64;
constexpr int FROWS = 88;  // total width
constexpr int FSEC = 13;   // 32-byte sectors the fixup completes per (workgroup, component, z): 7 + 6

struct FastArgs {
  int Ex, Ey, Ez, nx, ny, nz;
  int NX, NWG;  // workgroups along x (Ex / 4) and per field and z-segment (NX * Ey)
  int nseg, S;  // z-segments per column and element layers per segment
  double hh[3], sc[3], nu;
  double ihhh;    // 1 / (h_x h_y h_z)
  int64_t nodes;  // per component
  const ProbDev* prob;
};

// Swizzled LDS tile index of element-local point (a, b, c): (c, b ^ c, a ^ b).  In each of the
// three maps (lanes over (a, b), (a, c) or (b, c)) every group of 32 consecutive lanes hits 32
// distinct 8-byte bank pairs, so 64-bit accesses are free of bank conflicts with 64 banks (and
// 32-bit accesses with all 64 lanes at once).
__device__ __forceinline__ int tix(int a, int b, int c) { return (c << 6) + ((b ^ c) << 3) + (a ^ b); }

// The variant that leaves its workgroup faces to the face buffer and fast3d_fixup: the segmented
// J^T (FP32), whose register budget (two wavefronts per SIMD) leaves no room for the neighbours'
// lines.  Every other variant completes its faces in the kernel.  With a stage epilogue the fixup
// would read the epilogue operands of its nodes as scattered sectors; the plain J v and J^T
// complete theirs too since their lower state lines are loaded a step ahead (J^T 402 -> 393 us,
// J v 407 -> 379 us per apply on the 32^3 field, against main kernel + fixup).
constexpr bool face_buffer_variant(int op, int ep, bool seg) {
  (void)ep;
  return seg && op == OP_JACT;
}

// EP: epilogue variant known at compile time: 0 = o1 = b1 s; 1 = o1 = a1 x1 + b1 s;
// 2 = o1 = a1 x1 + c1 x2 + b1 s and (when o2 is given) o2 = a2 x2 + c2 x1 + b2 s.
// SEG: the z-sweep split into g.nseg segments (else one sweep closed by the periodic wrap), for
// two workgroups per CU: the register budget is then that of two wavefronts per SIMD.
template <typename T, int OP, int EP, bool SEG>
__global__ __launch_bounds__(256, SEG ? 2 : 1) void fast3d_kernel(FastArgs g, const FastTab<T>* __restrict__ tb,
                                                     const T* __restrict__ u, const T* __restrict__ v,
                                                     T* __restrict__ face, Epi epi, Coef in_scale) {
  // The workgroup faces are completed in the kernel, except by the variants of face_buffer_variant
  constexpr bool CMPL = !face_buffer_variant(OP, EP, SEG);
  constexpr bool HASV = OP != OP_RHS;
  __shared__ T sU[4][3][512];
  __shared__ T sV[4][HASV ? 3 : 1][HASV ? 512 : 1];
  __shared__ T sQ[4][3][512];
  __shared__ T sEx[2][3][3][64];  // [step parity][sending wavefront][component][x-map lane]
  // F: the left element's block at the workgroup's left face, staged by wavefront 0 (see XT;
  // FP64 F 263 -> 258 us on the 32^3 field)
  constexpr bool LTILE = OP == OP_RHS;
  __shared__ T sXL[LTILE ? 3 : 1][LTILE ? 512 : 1];

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int LS = logical_wg(blockIdx.x, g.NWG * (SEG ? g.nseg : 1));
  const int seg = SEG ? LS / g.NWG : 0, L = LS - seg * g.NWG;
  const int X = L % g.NX, ey = L / g.NX;
  const int ex = WX * X + wave;
  const int64_t bo = (int64_t)blockIdx.y * 3 * g.nodes;  // batch member offset
  const T* __restrict__ ub = u + bo;
  const T* __restrict__ vb = HASV ? v + bo : nullptr;
  const uint32_t fbytes = (uint32_t)(3 * g.nodes * sizeof(T));  // one batch member, all components
  const __amdgpu_buffer_rsrc_t r_o1 = brsrc(static_cast<T*>(epi.o1) + bo, fbytes);
  // a missing operand gets an empty range: its loads return 0 and its stores are dropped
  const bool hx1 = EP >= 1 && epi.x1, ho2 = EP >= 2 && epi.o2, hx2 = EP >= 2 && epi.x2;
  const __amdgpu_buffer_rsrc_t r_x1 = brsrc(hx1 ? static_cast<const T*>(epi.x1) + bo : u, hx1 ? fbytes : 0);
  const __amdgpu_buffer_rsrc_t r_o2 = brsrc(ho2 ? static_cast<T*>(epi.o2) + bo : u, ho2 ? fbytes : 0);
  const __amdgpu_buffer_rsrc_t r_x2 = brsrc(hx2 ? static_cast<const T*>(epi.x2) + bo : u, hx2 ? fbytes : 0);
  const __amdgpu_buffer_rsrc_t r_fb =
      CMPL ? brsrc(u, 0)
           : brsrc(face + (int64_t)blockIdx.y * g.NWG * 3 * g.nz * FROWS,
                   (uint32_t)((int64_t)g.NWG * 3 * g.nz * FROWS * sizeof(T)));
  const __amdgpu_buffer_rsrc_t r_u = brsrc(ub, fbytes);
  const __amdgpu_buffer_rsrc_t r_v = brsrc(HASV ? vb : ub, HASV ? fbytes : 0);
  const double dt = g.prob->dt;
  const T a1 = coef<T>(epi.a1, dt), b1 = coef<T>(epi.b1, dt), a2 = coef<T>(epi.a2, dt), b2 = coef<T>(epi.b2, dt);
  const T c1 = coef<T>(epi.c1, dt), c2 = coef<T>(epi.c2, dt);

  const int l0 = lane & 7, l1 = lane >> 3;
  const T ihhh = (T)(1.0 / (g.hh[0] * g.hh[1] * g.hh[2]));
  // quadrature weight omega = (h_x h_y h_z / 8) w_a w_b w_c (hh = h / 2); with the lane holding
  // the two fixed indices (l0, l1) and the register the third, the same 8 values serve all maps
  T om[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) om[s] = (T)(g.hh[0] * g.hh[1] * g.hh[2]) * tb->w[l0] * tb->w[l1] * tb->w[s];
  const T K1x = (T)(g.nu * g.sc[0] * g.sc[0]), K1y = (T)(g.nu * g.sc[1] * g.sc[1]), K1z = (T)(g.nu * g.sc[2] * g.sc[2]);
  const T K2x = (T)g.sc[0], K2y = (T)g.sc[1], K2z = (T)g.sc[2];
  // inverse assembled mass, lane factor of the z-map (a = l0, b = l1)
  const T mlane = tb->imq[l0] * tb->imq[l1] * ihhh;
  const T zin = (T)(in_scale.c0 + in_scale.cdt * dt) * mlane;  // J^T input: scale * M^{-1} w

  // z-map global addressing: lane (a = l0, b = l1), register c
  const int64_t plane = (int64_t)g.ny * g.nx;
  const int64_t lrow = (int64_t)((7 * ey + l1) % g.ny) * g.nx + (7 * ex + l0) % g.nx;
  // Output roles of the lane's node (7ex + a, 7ey + b, z).  F: owned (stored here) for a < 7 and
  // b < 7; the upper x- and y-faces belong to the neighbouring workgroups (a = 7 of wavefronts
  // 0..2 is added into the next wavefront's a = 0).  J v, J^T:
  //   own   finished here: a < 7, 1 <= b < 7, outside the first sector of the row
  //   face  face-buffer slot (lower and upper y-rows, upper x-column, first sectors), if any
  //         (a = 7 of wavefronts 0..2 has none: it is added into the next wavefront's a = 0)
  const int a = l0, b = l1;
  const bool lsec = !CMPL && wave == 0 && a < 4 && b >= 1 && b < 7;
  const bool own = a < 7 && b < 7 && (CMPL || (b >= 1 && !lsec));
  int fo = -1, fw = 0, fk = 0;  // region offset (widths before it), width, index; fo < 0: none
  if (!CMPL) {
    if (b == 7) {
      if (a < 7 || wave == WX - 1) fo = O_UY, fw = W_UY, fk = 7 * wave + a;
    } else if (a == 7) {
      if (wave == WX - 1) fo = O_UX, fw = W_UX, fk = b;
    } else if (b == 0) {
      fo = O_LY, fw = W_LY, fk = 7 * wave + a;
    } else if (lsec) {
      fo = O_LX, fw = W_LX, fk = 4 * (b - 1) + a;
    }
  }
  const int64_t fslab = (int64_t)g.NWG * 3 * g.nz;  // values per unit of region width
  const int64_t flane = fo * fslab + ((int64_t)L * 3 * g.nz) * fw + fk;
  const int64_t orow = (int64_t)(7 * ey + b) * g.nx + 7 * ex + a;  // valid when own
  // Doubling factors of the per-direction terms on the workgroup's lower face (b = 0, every
  // wavefront) and left face (a = 0 of wavefront 0): there the missing neighbour's terms along the
  // other directions equal the own element's.  z-map lanes (a = l0, b = l1), y-map (a = l0,
  // c = l1), x-map (b = l0, c = l1).
  const T fleft = (CMPL && wave == 0 && l0 == 0) ? (T)2 : (T)1;
  const T fz = fleft * ((CMPL && l1 == 0) ? (T)2 : (T)1), fy = fleft, fx = (CMPL && l0 == 0) ? (T)2 : (T)1;
  // y-map lanes (a, c): the lower element row's y-lines (rows 7 eym .. 7 eym + 6; row 7 is the own
  // row 7 ey); x-map lanes (b, c) of wavefront 0: the left element's x-lines (columns
  // 28X - 7 .. 28X - 1).  Byte offsets: a lane part and a uniform part per line point.
  const int eym = ey == 0 ? g.Ey - 1 : ey - 1;
  const int xl0 = (WX * 7 * X == 0 ? g.nx : WX * 7 * X) - 7;  // first column of the left element
  const int yrow_b = (7 * ey + l0) % g.ny;                    // x-map lane row (b = l0)
  const int xcol_a = (7 * ex + l0) % g.nx;                    // y-map lane column (a = l0)
  // Load planes c in [c0, 8) of element layer ez (plane 7ez + c, periodic in z).
  auto load_z = [&](int ez, int c0, T (&UU)[3][8], T (&VV)[3][8]) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      if (c < c0) continue;
      int zc = 7 * ez + c;
      if (zc >= g.nz) zc -= g.nz;
      const int64_t off = zc * plane + lrow;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        UU[i][c] = ub[i * g.nodes + off];
        if constexpr (HASV) VV[i][c] = vb[i * g.nodes + off];
      }
    }
  };

  // Write planes c in [c_lo, c_hi) of element layer ez from the summed z-map values Zv: inverse
  // mass and epilogue for the owned nodes, raw sums to the face-buffer slots (J v, J^T).  Every
  // lane issues the same stores; inactive ones drop theirs, each at its own offset beyond the
  // range (with bit 31 set; a batch member and its face buffer stay below 2 GiB), so that the
  // compiler keeps every dropped store as a distinct access.
  auto emit = [&](int ez, const T (&Zv)[3][8], int c_lo, int c_hi, const T (&E1)[3][7], const T (&E2)[3][7]) {
    const auto te = phase_ptr(tb);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int c = 0; c < 7; ++c) {
        const bool inc = c >= c_lo && c < c_hi;
        const int z = 7 * ez + c;  // < nz: c < 7
        const T r = Zv[i][c];
        const uint32_t no = (uint32_t)((i * g.nodes + z * plane + orow) * sizeof(T));
        const T sm = (OP != OP_JACT) ? r * (mlane * te->imq[c]) : r;
        T r1 = b1 * sm;
        if (EP >= 1) r1 += a1 * E1[i][c];
        if (EP >= 2) r1 += c1 * E2[i][c];
        bstore(r_o1, (own && inc) ? no : (OOB | no), r1);
        if (EP >= 2) bstore(r_o2, (own && inc) ? no : (OOB | no), a2 * E2[i][c] + c2 * E1[i][c] + b2 * sm);
        if constexpr (!CMPL) {
          const uint32_t fb = (uint32_t)((flane + ((int64_t)i * g.nz + z) * fw) * sizeof(T));
          bstore(r_fb, (fo >= 0 && inc) ? fb : (OOB | fb), r);
        }
      }
  };

  auto load_epi = [&](int ez, T (&E1)[3][7], T (&E2)[3][7], int c_lo, int c_hi) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int c = 0; c < 7; ++c) {
        const bool inc = c >= c_lo && c < c_hi;
        const uint32_t no = (own && inc)
                                ? (uint32_t)((i * g.nodes + (7 * ez + c) * plane + orow) * sizeof(T))
                                : OOB;
        E1[i][c] = (EP >= 1) ? bload<T>(r_x1, no) : (T)0;
        E2[i][c] = (EP >= 2) ? bload<T>(r_x2, no) : (T)0;
      }
  };

  T* __restrict__ tU = sU[wave][0];
  T* __restrict__ tQ = sQ[wave][0];
  T* __restrict__ tV = HASV ? sV[wave][0] : sU[wave][0];
  // Lines of a neighbouring element through the lane's face node, points 0..6 (point 7 is the
  // own node and comes from the tile): the lower element's y-lines in the y-map (ylow) or the
  // left element's x-lines in the x-map (xleft), for layer ez, of one input field (r_u or r_v).
  // lines_node fills point 7 from the tile; J^T scales its second input to Z = M^{-1} w like
  // the tile's.
  // An x-line's points 0..6 lie in one grid row, one row per lane.  FP64 reads them with three
  // 16-byte loads and one 8-byte load per lane instead of seven 8-byte ones: a load touches a cache
  // line per lane, so fewer, wider loads cost the cache less (F 271 -> 263 us on the 32^3 field).
  // FP32 keeps one load per point: a 16- plus 12-byte version gave wrong results (cause not
  // traced; F's FP32 lines now go through the LDS tile below).
  auto load_lines = [&](bool ylow, int ez, __amdgpu_buffer_rsrc_t r, T (&L)[3][8]) {
    int zc = 7 * ez + l1;
    if (zc >= g.nz) zc -= g.nz;
    const uint32_t lane_off = (uint32_t)(((int64_t)zc * plane + (ylow ? xcol_a : (int64_t)yrow_b * g.nx)) * sizeof(T));
    if constexpr (sizeof(T) == 8) {
      if (!ylow) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const uint32_t uni = (uint32_t)(((int64_t)i * g.nodes + xl0) * sizeof(T));
#pragma unroll
          for (int n = 0; n < 6; n += 2) {
            const u32x4_t q = __builtin_amdgcn_raw_buffer_load_b128(r, (int)lane_off, (int)(uni + 8 * n), 0);
            L[i][n] = __builtin_bit_cast(double, u32x2_t{q.x, q.y});
            L[i][n + 1] = __builtin_bit_cast(double, u32x2_t{q.z, q.w});
          }
          L[i][6] = bload_s<T>(r, lane_off, uni + 48);
        }
        return;
      }
    }
#pragma unroll
    for (int n = 0; n < 7; ++n) {
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const int64_t uni = (int64_t)i * g.nodes + (ylow ? (int64_t)(7 * eym + n) * g.nx : (int64_t)(xl0 + n));
        L[i][n] = bload_s<T>(r, lane_off, (uint32_t)(uni * sizeof(T)));
      }
    }
  };
  auto lines_node = [&](bool ylow, const T* __restrict__ tile, bool scale, T (&L)[3][8]) {
    const int t = ylow ? tix(l0, 0, l1) : tix(0, l0, l1);
    const auto tl = phase_ptr(tb);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      L[i][7] = tile[i * 512 + t];
      if (scale) {
#pragma unroll
        for (int n = 0; n < 7; ++n) L[i][n] *= zin * tl->imq[n];
      }
    }
  };

  // The sweep.  One segment (wrap): layers 0 .. Ez - 1, plane c = 0 of layer 0 completed by the
  // periodic wrap after the sweep.  Several: layers z0 .. z0 + nl - 1 after a first step that
  // recomputes layer z0 - 1 (periodically) without storing, so that the carry into plane 0 of
  // layer z0 is complete and every plane is stored by the segment that owns it.
  constexpr bool wrap = !SEG;
  const int z0 = seg * g.S, nl = min(g.S, g.Ez - z0);
  const int nstep = wrap ? g.Ez : nl + 1;
  const int zfirst = wrap ? 0 : (z0 == 0 ? g.Ez - 1 : z0 - 1);
  T cu[3][8], cv[3][8];
  load_z(zfirst, 0, cu, cv);
  // the neighbouring elements' lines through the layer's face nodes (the left ones: wavefront
  // 0), used right after the tile is staged; load_neighbours issues those loaded a step ahead
  T YU[3][8], YV[3][8], XU[3][8], XV[3][8];
  // F (wavefront 0): the left element's columns x = xl0 + a (a < 7; lanes a = 7 repeat a = 6) of
  // the workgroup's rows, in the z-map (lane (a, b), register c).  Loaded like the own layer (8
  // lanes read a contiguous row piece), they reach the x-map through LDS: read directly in the
  // x-map, each load would touch a cache line per lane.
  T XT[3][8];
  const uint32_t xt_lane = (uint32_t)(((int64_t)((7 * ey + l1) % g.ny) * g.nx + xl0 + min(l0, 6)) * sizeof(T));
  auto load_left_block = [&](int ez) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      int zc = 7 * ez + c;
      if (zc >= g.nz) zc -= g.nz;
#pragma unroll
      for (int i = 0; i < 3; ++i) XT[i][c] = bload_s<T>(r_u, xt_lane, (uint32_t)((i * g.nodes + zc * plane) * sizeof(T)));
    }
  };
  // F prefetches them a step ahead.  J v and J^T hold twice the lines (both inputs): they
  // prefetch the lower element's state lines (RK4 adjoint with stored stages 2.03 -> 1.98 ms per
  // step) and load the second input's lines and wavefront 0's left lines where they are used
  // (prefetched too, they spilled 17-139 registers and ran slower)
  auto load_neighbours = [&](int ez) {
    if constexpr (!CMPL) return;
    load_lines(true, ez, r_u, YU);
    if constexpr (LTILE) {
      if (wave == 0) load_left_block(ez);
    }
  };
  load_neighbours(zfirst);
  T carry[3] = {0, 0, 0}, first0[3] = {0, 0, 0};
  {
    // The store sequence of a step, with every store dropped.  Loads and stores share one
    // completion counter that drains in issue order, and the compiler's wait for a load in the
    // loop allows only the memory operations issued after it on every path into the loop.  On
    // the back edge the previous step's stores follow the layer and neighbour loads; issuing the
    // same sequence before the loop lets those waits leave the stores in flight (else every step
    // would first wait for the previous step's stores to complete).
    T Z0[3][8] = {}, E0[3][7] = {};
    // after the loads above (the asm may read the inputs, so their loads cannot move below it)
    asm volatile("" ::"s"(ub), "s"(HASV ? vb : ub) : "memory");
    __builtin_amdgcn_sched_barrier(0);
    emit(zfirst, Z0, 0, 0, E0, E0);
  }

  for (int k = 0; k < nstep; ++k) {
    const int ez = wrap ? k : (k == 0 ? zfirst : z0 + k - 1);
    const int c_lo = (wrap && k == 0) ? 1 : 0, c_hi = (wrap || k > 0) ? 7 : 0;  // planes stored
    // ---- z-map (lane (a=l0, b=l1), register c): stage the element tile, z-direction part
    T wlast[3];  // unscaled input plane c = 7, the next layer's plane c = 0
#pragma unroll
    for (int i = 0; i < 3; ++i) wlast[i] = cv[i][7];
    if constexpr (OP == OP_JACT) {
      const auto ts = phase_ptr(tb);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int c = 0; c < 8; ++c) cv[i][c] *= zin * ts->imq[c];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        tU[i * 512 + tix(l0, l1, c)] = cu[i][c];
        if constexpr (HASV) tV[i * 512 + tix(l0, l1, c)] = cv[i][c];
      }
    map_contrib<T, OP, 3>(
        2,
        [&](int i, T (&Xr)[8]) {
#pragma unroll
          for (int c = 0; c < 8; ++c) Xr[c] = cu[i][c];
        },
        [&](int i, T (&Xr)[8]) {
#pragma unroll
          for (int c = 0; c < 8; ++c) Xr[c] = cv[i][c];
        },
        om, K1z * fz, K2z * fz, phase_ptr(tb),
        [&](int i, const T (&P)[8]) {
#pragma unroll
          for (int c = 0; c < 8; ++c) tQ[i * 512 + tix(l0, l1, c)] = P[c];
        });
    // the lower element's y-terms at its b = 7 (y-map lanes (a, c)), added at b = 0, and, in
    // wavefront 0, the left element's x-terms at its a = 7 (x-map lanes (b, c)), added at a = 0:
    // their lines' last point is the own node, read from the tile
    if constexpr (CMPL) {
    wave_sync();
    {
      T low[3];
      if constexpr (HASV) load_lines(true, ez, r_v, YV);
      lines_node(true, tU, false, YU);
      if constexpr (HASV) lines_node(true, tV, OP == OP_JACT, YV);
      line_end_terms<T, OP, 3>(1, YU, YV, om[7], K1y * fy, K2y * fy, phase_ptr(tb), low);
#pragma unroll
      for (int i = 0; i < 3; ++i) tQ[i * 512 + tix(l0, 0, l1)] += low[i];
    }
    if (wave == 0) {
      T low[3];
      if constexpr (HASV) {
        load_lines(false, ez, r_u, XU);
        load_lines(false, ez, r_v, XV);
      }
      if constexpr (LTILE) {
        T* __restrict__ tL = sXL[0];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int c = 0; c < 8; ++c) tL[i * 512 + tix(l0, l1, c)] = XT[i][c];
        wave_sync();
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int n = 0; n < 7; ++n) XU[i][n] = tL[i * 512 + tix(n, l0, l1)];
      }
      lines_node(false, tU, false, XU);
      if constexpr (HASV) lines_node(false, tV, OP == OP_JACT, XV);
      line_end_terms<T, OP, 3>(0, XU, XV, om[7], K1x * fx, K2x * fx, phase_ptr(tb), low);
      wave_sync();
#pragma unroll
      for (int i = 0; i < 3; ++i) tQ[i * 512 + tix(0, l0, l1)] += low[i];
    }
    }
    // the z-map lines are no longer needed: move plane 7 to plane 0 and prefetch the next layer's
    // planes 1..7 into the same registers (unconditionally: the last step reloads layer 0, so the
    // memory-op sequence is fixed)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      cu[i][0] = cu[i][7];
      if constexpr (HASV) cv[i][0] = wlast[i];
    }
    load_z(ez + 1 < g.Ez ? ez + 1 : 0, 1, cu, cv);  // the last step loads one layer more
    wave_sync();
    // ---- y-map (lane (a=l0, c=l1), register b)
    map_contrib<T, OP, 3>(
        1,
        [&](int i, T (&Xr)[8]) {
#pragma unroll
          for (int q = 0; q < 8; ++q) Xr[q] = tU[i * 512 + tix(l0, q, l1)];
        },
        [&](int i, T (&Xr)[8]) {
#pragma unroll
          for (int q = 0; q < 8; ++q) Xr[q] = tV[i * 512 + tix(l0, q, l1)];
        },
        om, K1y * fy, K2y * fy, phase_ptr(tb),
        [&](int i, const T (&P)[8]) {
          // read the 8 values first, then write: one LDS round trip per component instead of
          // one per value (the compiler cannot prove the swizzled addresses distinct)
          T qv[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) qv[q] = tQ[i * 512 + tix(l0, q, l1)];
#pragma unroll
          for (int q = 0; q < 8; ++q) tQ[i * 512 + tix(l0, q, l1)] = qv[q] + P[q];
        });
    wave_sync();
    // ---- x-map (lane (b=l0, c=l1), register a): accumulate into the tile, keep face a = 7;
    // wavefront 0 adds the left element's x-terms at its a = 7 to a = 0
    T R7[3];
    map_contrib<T, OP, 3>(
        0,
        [&](int i, T (&Xr)[8]) {
#pragma unroll
          for (int q = 0; q < 8; ++q) Xr[q] = tU[i * 512 + tix(q, l0, l1)];
        },
        [&](int i, T (&Xr)[8]) {
#pragma unroll
          for (int q = 0; q < 8; ++q) Xr[q] = tV[i * 512 + tix(q, l0, l1)];
        },
        om, K1x * fx, K2x * fx, phase_ptr(tb),
        [&](int i, const T (&P)[8]) {
          T qv[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) qv[q] = tQ[i * 512 + tix(q, l0, l1)];
#pragma unroll
          for (int q = 0; q < 8; ++q) tQ[i * 512 + tix(q, l0, l1)] = qv[q] + P[q];
          R7[i] = qv[7] + P[7];
        });
    // epilogue operands of this layer: issued before the barrier so that their latency overlaps it
    T E1[3][7], E2[3][7];
    load_epi(ez, E1, E2, c_lo, c_hi);
    // The next layer's neighbour lines (F; the last step loads one layer more).  Loads and stores
    // share one completion counter that drains in issue order, so lines loaded after this step's
    // stores would wait for them too: the plain apply issues them here, before its stores (F
    // 278 -> 268 us on the 32^3 field).  The stage variants issue them after their stores: here,
    // behind the epilogue operands, they made an RK4 step 4% slower.
    const int ezn = ez + 1 < g.Ez ? ez + 1 : 0;
    if constexpr (EP == 0) load_neighbours(ezn);
    // ---- x-direction summation inside the workgroup: wavefront w's face a = 7 is wavefront
    // w + 1's face a = 0 (double-buffered by step parity: one barrier per step)
    const int par = k & 1;
    if (wave < WX - 1) {
#pragma unroll
      for (int i = 0; i < 3; ++i) sEx[par][wave][i][lane] = R7[i];
    }
    __syncthreads();
    if (wave > 0) {
#pragma unroll
      for (int i = 0; i < 3; ++i) tQ[i * 512 + tix(0, l0, l1)] += sEx[par][wave - 1][i][lane];
    }
    // ---- read the summed tile in the z-map; z-direction summation: carry the shared plane
    wave_sync();
    T Zv[3][8];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int c = 0; c < 8; ++c) Zv[i][c] = tQ[i * 512 + tix(l0, l1, c)];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Zv[i][0] += carry[i];
      carry[i] = Zv[i][7];
    }
    if (wrap && k == 0) {
#pragma unroll
      for (int i = 0; i < 3; ++i) first0[i] = Zv[i][0];
    }
    // ---- outputs (with one segment, plane c = 0 of layer 0 waits for the periodic wrap)
    emit(ez, Zv, c_lo, c_hi, E1, E2);
    if constexpr (EP != 0) load_neighbours(ezn);
  }
  // periodic wrap along z: the carried plane of the last layer is plane c = 0 of layer 0
  if (wrap) {
    T Zv[3][8], E1[3][7], E2[3][7];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int c = 0; c < 8; ++c) Zv[i][c] = (c == 0) ? first0[i] + carry[i] : (T)0;
    load_epi(0, E1, E2, 0, 1);
    emit(0, Zv, 0, 1, E1, E2);
  }
}

// Completes, for every workgroup (X, ey), component and grid plane z, the nodes of its lower
// y-row (own partial plus the lower neighbour's upper-y contribution) and of the first sectors of
// its interior rows (own value plus, at x = 28X, the left neighbour's upper-x contribution); the
// node (28X, 7ey) also receives the diagonal neighbour's corner.  Then the inverse mass (J v) and
// the epilogue.  One thread per 32-byte output sector (4 nodes along x); blockIdx.x is
// (workgroup, component), blockIdx.y a range of (z, sector) pairs, blockIdx.z the batch member.
template <typename T, bool DIV>
__global__ __launch_bounds__(256) void fast3d_fixup(FastArgs g, const FastTab<T>* __restrict__ tb,
                                                    const T* __restrict__ face, Epi epi) {
  const int t = blockIdx.y * 256 + threadIdx.x;
  if (t >= g.nz * FSEC) return;
  const int sct = t % FSEC, z = t / FSEC;
  const int L = blockIdx.x / 3, i = blockIdx.x % 3;
  const int X = L % g.NX, ey = L / g.NX;
  const int Xm = X == 0 ? g.NX - 1 : X - 1, eym = ey == 0 ? g.Ey - 1 : ey - 1;
  const int xl0 = sct < 7 ? 4 * sct : 0;
  const int yl = sct < 7 ? 0 : sct - 6;
  const int64_t fslab = (int64_t)g.NWG * 3 * g.nz;
  const T* __restrict__ fm = face + (int64_t)blockIdx.z * fslab * FROWS;
  // start of (workgroup W, this component, this z) in region (offset o, width w)
  auto rec = [&](int W, int o, int w) { return fm + o * fslab + (((int64_t)W * 3 + i) * g.nz + z) * w; };
  T s[4];
  if (yl == 0) {
    const T* __restrict__ own = rec(L, O_LY, W_LY) + xl0;
    const T* __restrict__ up = rec(X + g.NX * eym, O_UY, W_UY) + xl0;
#pragma unroll
    for (int q = 0; q < 4; ++q) s[q] = own[q] + up[q];
    if (xl0 == 0) s[0] += rec(Xm + g.NX * ey, O_UX, W_UX)[0] + rec(Xm + g.NX * eym, O_UY, W_UY)[28];
  } else {
    const T* __restrict__ own = rec(L, O_LX, W_LX) + 4 * (yl - 1);
#pragma unroll
    for (int q = 0; q < 4; ++q) s[q] = own[q];
    s[0] += rec(Xm + g.NX * ey, O_UX, W_UX)[yl];
  }
  const double dt = g.prob->dt;
  if (DIV) {
    const T m = tb->imq[yl] * tb->imq[z % NQ] * (T)g.ihhh;
#pragma unroll
    for (int q = 0; q < 4; ++q) s[q] *= m * tb->imq[(xl0 + q) % NQ];
  }
  const int64_t o = (int64_t)blockIdx.z * 3 * g.nodes + i * g.nodes +
                    ((int64_t)z * g.ny + 7 * ey + yl) * g.nx + 7 * WX * X + xl0;
  const T a1 = coef<T>(epi.a1, dt), b1 = coef<T>(epi.b1, dt), a2 = coef<T>(epi.a2, dt), b2 = coef<T>(epi.b2, dt);
  const T c1 = coef<T>(epi.c1, dt), c2 = coef<T>(epi.c2, dt);
  // o2 may alias x2 (in-place accumulation): each element is read before it is written
  T* o1 = static_cast<T*>(epi.o1) + o;
  const T* x1 = epi.x1 ? static_cast<const T*>(epi.x1) + o : nullptr;
  T* o2 = epi.o2 ? static_cast<T*>(epi.o2) + o : nullptr;
  const T* x2 = epi.x2 ? static_cast<const T*>(epi.x2) + o : nullptr;
  // all operands first: a store may alias a later operand, so the loads must not wait behind it.
  // A sector is 4 contiguous nodes, so each operand moves as one vector (16-byte accesses)
  // instead of four scalar ones.  The vector type assumes only the element's alignment; within
  // a field the sectors are 32-byte aligned (28X and x-local 4k nodes, rows of 7 E_x nodes).
  typedef T T4 __attribute__((ext_vector_type(4), aligned(sizeof(T))));
  const T4 zero = {0, 0, 0, 0};
  const T4 v1 = x1 ? *reinterpret_cast<const T4*>(x1) : zero;
  const T4 v2 = x2 ? *reinterpret_cast<const T4*>(x2) : zero;
  T4 r1, r2;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    r1[q] = b1 * s[q] + a1 * v1[q] + c1 * v2[q];
    r2[q] = b2 * s[q] + a2 * v2[q] + c2 * v1[q];
  }
  if (o2) *reinterpret_cast<T4*>(o2) = r2;
  *reinterpret_cast<T4*>(o1) = r1;
}

// z-segments per column: the FP32 F and J^T kernels (54 and 78 KB of LDS, at most 256 registers)
// fit two workgroups per CU, which needs twice as many workgroups as CUs; every other variant
// holds one workgroup per CU, where a segment would only add its recomputed layer.
int z_segments(const ProbDev& hp, int op, bool f32) {
  return (f32 && (op == OP_RHS || op == OP_JACT) && hp.E[2] >= 4) ? 2 : 1;
}

// whether a launch goes through the face buffer and fast3d_fixup
bool fast3d_face_buffer(const ProbDev& hp, int op, int ep, bool f32) {
  return face_buffer_variant(op, ep, z_segments(hp, op, f32) > 1);
}

FastArgs make_args(const ProbDev& hp, const ProbDev* dprob, int nseg) {
  FastArgs g;
  g.Ex = hp.E[0];
  g.Ey = hp.E[1];
  g.Ez = hp.E[2];
  g.nx = hp.n[0];
  g.ny = hp.n[1];
  g.nz = hp.n[2];
  g.NX = hp.E[0] / WX;
  g.NWG = g.NX * hp.E[1];
  g.nseg = nseg;
  g.S = (hp.E[2] + nseg - 1) / nseg;
  for (int k = 0; k < 3; ++k) {
    g.hh[k] = hp.hh[k];
    g.sc[k] = hp.sc[k];
  }
  g.nu = hp.nu;
  g.ihhh = 1.0 / (hp.hh[0] * hp.hh[1] * hp.hh[2]);
  g.nodes = hp.nodes;
  g.prob = dprob;
  return g;
}

template <typename T>
hipError_t run_fast(const ProbDev& hp, const ProbDev* dprob, int op, const void* u, const void* v, void* face,
                    const Epi& epi, Coef in_scale, const void* dtab, hipStream_t s) {
  const FastArgs g = make_args(hp, dprob, z_segments(hp, op, sizeof(T) == 4));
  const auto* tb = static_cast<const FastTab<T>*>(dtab);
  const dim3 grid(g.NWG * g.nseg, hp.batch);
  const T* uu = static_cast<const T*>(u);
  const T* vv = static_cast<const T*>(v);
  T* fc = static_cast<T*>(face);
  const int ep = (epi.o2 || epi.x2) ? 2 : (epi.x1 ? 1 : 0);
#define SEM_FAST_LAUNCH(OPV, EPV)                                                                           \
  hipLaunchKernelGGL((fast3d_kernel<T, OPV, EPV, false>), grid, dim3(256), 0, s, g, tb, uu, vv, fc, epi, in_scale)
#define SEM_FAST_EP(OPV)          \
  if (ep == 0) SEM_FAST_LAUNCH(OPV, 0); \
  else if (ep == 1) SEM_FAST_LAUNCH(OPV, 1); \
  else SEM_FAST_LAUNCH(OPV, 2);
#define SEM_FAST_LAUNCH_SEG(OPV, EPV)                                                                       \
  hipLaunchKernelGGL((fast3d_kernel<T, OPV, EPV, true>), grid, dim3(256), 0, s, g, tb, uu, vv, fc, epi, in_scale)
#define SEM_FAST_EP_SEG(OPV)                \
  if (ep == 0) SEM_FAST_LAUNCH_SEG(OPV, 0); \
  else if (ep == 1) SEM_FAST_LAUNCH_SEG(OPV, 1); \
  else SEM_FAST_LAUNCH_SEG(OPV, 2);
  if (g.nseg > 1) {
    if constexpr (sizeof(T) == 4) {  // the segmented variants (z_segments): FP32 F and J^T
      if (op == OP_RHS) {
        SEM_FAST_EP_SEG(OP_RHS)
      } else {
        SEM_FAST_EP_SEG(OP_JACT)
      }
    }
  } else if (op == OP_RHS) {
    SEM_FAST_EP(OP_RHS)
  } else if (op == OP_JAC) {
    SEM_FAST_EP(OP_JAC)
  } else {
    SEM_FAST_EP(OP_JACT)
  }
#undef SEM_FAST_EP_SEG
#undef SEM_FAST_LAUNCH_SEG
#undef SEM_FAST_EP
#undef SEM_FAST_LAUNCH
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !fast3d_face_buffer(hp, op, ep, sizeof(T) == 4)) return e;  // faces completed in the kernel
  const dim3 fgrid((unsigned)(g.NWG * 3), (unsigned)((g.nz * FSEC + 255) / 256), hp.batch);
  if (op == OP_JACT)
    hipLaunchKernelGGL((fast3d_fixup<T, false>), fgrid, dim3(256), 0, s, g, tb, fc, epi);
  else
    hipLaunchKernelGGL((fast3d_fixup<T, true>), fgrid, dim3(256), 0, s, g, tb, fc, epi);
  return hipGetLastError();
}

}  // namespace

bool fast3d_supported(const ProbDev& hp) {
  // buffer offsets are 32-bit: one batch member (all components, FP64) must stay below 2 GiB
  return hp.dim == 3 && hp.N == NQ && hp.E[0] % WX == 0 && hp.E[1] >= 1 && hp.E[2] >= 1 &&
         (int64_t)3 * hp.nodes * 8 < ((int64_t)1 << 31);
}


bool fast3d_needs_face(const ProbDev& hp, bool f32) {
  return fast3d_face_buffer(hp, OP_JACT, 0, f32) || fast3d_face_buffer(hp, OP_JAC, 0, f32) ||
         fast3d_face_buffer(hp, OP_RHS, 0, f32);
}

int64_t fast3d_face_values(const ProbDev& hp) {
  return (int64_t)hp.batch * (hp.E[0] / WX) * hp.E[1] * 3 * hp.n[2] * FROWS;
}

hipError_t launch_fast3d(const ProbDev& hp, const ProbDev* dprob, int op, const void* u, const void* v, void* face,
                         const Epi& epi, Coef in_scale, const void* dtables, int dtype, hipStream_t s) {
  if (dtype == SEM_F64) return run_fast<double>(hp, dprob, op, u, v, face, epi, in_scale, dtables, s);
  return run_fast<float>(hp, dprob, op, u, v, face, epi, in_scale,
                         static_cast<const char*>(dtables) + sizeof(FastTab<double>), s);
}

}  // namespace sem
