// Private declarations shared by libsem's translation units (host launchers + HIP kernels).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>
#include <string>

#include "sem.h"

namespace sem {

// Largest supported number of GLL points per direction (order N = MAXP - 1 in 1-D and 2-D).
constexpr int MAXP = 13;
constexpr int MAXP3 = 10;  // 3-D: (N+1)^3 threads per element must fit one workgroup

// GLL differentiation matrix and weights for one order (device-resident; kernels get a pointer).
template <typename T>
struct Tables {
  T D[MAXP * MAXP];  // D[i*P + j] = l_j'(xi_i)
  T w[MAXP];
};

// One problem of a launch (device-resident array, read-only in kernels).  A context with a
// same-shape batch is one entry with batch > 1; a batched uneven set has one entry per problem.
struct ProbDev {
  int32_t E[3], n[3];
  int32_t N, P, dim, batch;
  double sc[3];  // 2 / h_k: scale of D on the physical element
  double hh[3];  // h_k / 2
  double nu, dt;
  double w[MAXP];  // GLL weights of this order
  int64_t off;     // offset (values) of this problem's batch member 0 in the packed field arrays
  int64_t loff;    // offset (values) of its element-local scratch
  int64_t nelem;   // elements per batch member
  int64_t nodes;   // unique nodes per component per batch member
  int64_t item0;   // first element work item of this problem in its element launch
  int64_t node0;   // first node work item of this problem in the summation launch
};

// Coefficient evaluated per problem: c0 + cdt * dt_p.
struct Coef {
  double c0, cdt;
};

// Epilogue of the summation (DSS) kernels: s is the assembled operator value at a node;
//   o1 = a1 * x1 + c1 * x2 + b1 * s   (a NULL x contributes 0)
//   o2 = a2 * x2 + c2 * x1 + b2 * s   (optional; o2 may equal x2; o1 never aliases x1 or x2)
struct Epi {
  void* o1;
  const void* x1;
  Coef a1, b1;
  void* o2;
  const void* x2;
  Coef a2, b2;
  Coef c1, c2;  // cross terms: o1 += c1 x2, o2 += c2 x1 (RK-3 stage combinations)
};

enum Op { OP_RHS = 0, OP_JAC = 1, OP_JACT = 2 };

// A set of problems of one order and dimension that an element launch covers.
struct ElemLaunch {
  const ProbDev* probs;  // device array
  int32_t nprobs;
  int64_t nitems;  // total element items
  int32_t dim, P, dtype;
  int32_t epb;  // elements per workgroup (tunable); 0 = default
};

// Launchers (kern_generic.hip).  Return hipSuccess or the launch error.  `tables` is a device
// pointer to Tables<T> of the launch's order.
hipError_t launch_elem(const ElemLaunch& el, int op, const void* u, const void* v, void* lvec, Coef in_scale,
                       const void* tables, hipStream_t s);
hipError_t launch_dss(const ProbDev* probs, int32_t nprobs, int64_t nitems, int dim, int dtype, int divide_by_mass,
                      const void* lvec, const Epi& epi, hipStream_t s);
// assembled diagonal mass of every node of one problem-table entry, into every component of the
// field layout at the entry's offset
hipError_t launch_mass(const ProbDev& hp, void* out, int dtype, hipStream_t s);
// elements-per-workgroup choices accepted by launch_elem for (dim, P); returns count, fills out[]
int elem_epb_choices(int dim, int P, int* out, int max_out);

// Work item of the persistent 2-D element kernel: elements [e0, e0 + ne) (batch-flattened) of
// problem `prob` (index into the problem table), whose order has P points per direction.
struct WorkItem {
  int32_t prob;
  int32_t P;
  int64_t e0;
  int32_t ne;
  int32_t pad;
};
// One launch over all items of a mixed-order 2-D set; tabs: device array of Tables<T> indexed by
// P (entries 0..MAXP).  Each workgroup of 256 threads walks items blockIdx.x + k * grid.
hipError_t launch_persist2d(const ProbDev* probs, const WorkItem* items, int nitems, int grid, int op, int dtype,
                            const void* tabs, const void* u, const void* v, void* lvec, Coef in_scale, hipStream_t s);
int persist2d_elems_per_item(int P);  // elements per work item for order P

// Host GLL tables in long double (gll.cpp)
void gll_tables(int N, double* xi, double* w, double* D);

// Tuned paths (kern_fast3d.hip: 3-D order 7; kern_fast2d.hip: 2-D orders 3, 5, 7, 9) for one
// problem (any batch).  The epilogue output o1 must alias neither operator input: other
// workgroups still read the input nodes that a workgroup has finished.  Both take the device
// table of their order (fast_fill_tables).
bool fast3d_supported(const ProbDev& hp);
int64_t fast3d_face_values(const ProbDev& hp);
bool fast3d_needs_face(const ProbDev& hp, bool f32);  // whether any 3-D launch uses the face buffer

// FP64 rate diagnostic (kern_probe.hip): mode 0 matrix cores, 1 vector FMAs, 2 both interleaved;
// `out` holds fp64_probe_values() doubles.
int64_t fp64_probe_values();
hipError_t launch_fp64_probe(int mode, double* out, int iters, hipStream_t s);
double fp64_probe_mfma_flops_per_wave_iter();
double fp64_probe_valu_flops_per_wave_iter();  // face-buffer values per launch (plain J v, J^T)
bool fast2d_supported(const ProbDev& hp);
// lets the 2-D kernels of order N and dtype use their workgroup LDS (more than the default limit)
hipError_t fast2d_prepare(int N, int dtype);
size_t fast_table_bytes(int N);            // N = 3, 5 or 7
void fast_fill_tables(int N, void* host);  // fills fast_table_bytes(N) bytes

// Vector kernels (kern_blas.hip): out[j] = <X_j, w> for nv <= blas_max_vectors() vectors X_j at
// stride ldx (FP64 accumulation, fixed order; partial holds blas_partial_bytes()), and
// y = alpha y + sign * sum_j coef[j] X_j with coef in device memory, and z = a x + b y (y may be NULL).
int blas_max_vectors();
size_t blas_partial_bytes();
hipError_t blas_multidot(int dtype, const void* X, int64_t ldx, int nv, const void* w, int64_t n, double* partial,
                         double* out, hipStream_t s);
hipError_t blas_combine(int dtype, void* y, double alpha, const void* X, int64_t ldx, int nv, const double* coef,
                        double sign, int64_t n, hipStream_t s);
hipError_t blas_axpby(int dtype, void* z, double a, const void* x, double b, const void* y, int64_t n, hipStream_t s);
// y <- y + sign sum_j coef[j] X_j (coef in device memory), then out[j] = <X_j, y> for j < nv, or
// with self out[0] = <y, y>: one pass over the vectors (partial as for blas_multidot)
hipError_t blas_combine_dot(int dtype, void* y, const void* X, int64_t ldx, int nv, const double* coef, double sign,
                            int64_t n, bool self, double* partial, double* out, hipStream_t s);

// Binomial checkpointing schedule (revolve.cpp).  Actions, in order: RESTORE slot (current state
// <- snapshot slot), ADVANCE k (k forward steps), STORE slot (snapshot slot <- current state),
// ADJOINT i (adjoint of step i on the current state, which is u_i).  Slot 0 holds u_0.
enum { REV_RESTORE = 0, REV_ADVANCE = 1, REV_STORE = 2, REV_ADJOINT = 3 };
struct RevolveAct {
  int kind;
  int64_t arg;
};
// Fills acts for nsteps steps and snaps snapshot slots; returns the number of forward steps the
// schedule advances (-1 for invalid sizes).
int64_t revolve_plan(int64_t nsteps, int64_t snaps, std::vector<RevolveAct>& acts);
hipError_t launch_fast3d(const ProbDev& hp, const ProbDev* dprob, int op, const void* u, const void* v, void* face,
                         const Epi& epi, Coef in_scale, const void* dtables, int dtype, hipStream_t s);
hipError_t launch_fast2d(const ProbDev& hp, const ProbDev* dprob, int op, const void* u, const void* v, const Epi& epi,
                         Coef in_scale, const void* dtables, int dtype, hipStream_t s);
// Batched sets: problems that fast2d_supported accepts run the tuned 2-D kernel, one launch per
// (order, x element count) (fast2d_waves wavefronts per workgroup) over work items = row segments.
struct Fast2Item {
  int32_t prob;   // index into the problem table
  int32_t y0;     // first element row of the segment
  int32_t nrows;  // element rows of the segment
  int32_t x0;     // first element column of the segment (rows split into x-segments: order 9)
};
int fast2d_waves(const ProbDev& hp);      // wavefronts per workgroup
int fast2d_xsegments(const ProbDev& hp);  // workgroups per element row
hipError_t launch_fast2d_batch(const ProbDev* dprobs, const Fast2Item* items, int nitems, int nw, int N, int op,
                               const void* u, const void* v, const Epi& epi, Coef in_scale, const void* dtables,
                               int dtype, hipStream_t s);

}  // namespace sem
