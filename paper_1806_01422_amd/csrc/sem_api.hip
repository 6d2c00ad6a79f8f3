// libsem C ABI: contexts, operator entry points, RK4 forward/adjoint with uniform checkpoints, and
// the batched uneven problem set.  Host code only; kernels live in kern_*.hip.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "sem_internal.h"

using namespace sem;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(x)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) return fail(SEM_ERR_HIP, "%s: %s", #x, hipGetErrorString(e_));  \
  } while (0)

// A device allocation released with the owner.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) {
    o.p = nullptr;
    o.bytes = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      o.p = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  int alloc(size_t n) {
    release();
    if (n == 0) n = 256;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      return fail(SEM_ERR_NOMEM, "hipMalloc(%zu bytes) failed: %s", n, hipGetErrorString(e));
    }
    bytes = n;
    return SEM_OK;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  ~DevBuf() { release(); }
};

// Sets dt of every problem entry of a device table (stream-ordered, capturable).
__global__ void set_dt_kernel(ProbDev* probs, int n, const double* dts, double dt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) probs[i].dt = dts ? dts[i] : dt;
}

template <typename T>
__global__ void finite_kernel(const T* __restrict__ x, int64_t n, int* __restrict__ flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int bad = 0;
  for (; i < n; i += stride) bad |= !isfinite((double)x[i]);
  if (bad) atomicOr(flag, 1);
}

int validate_desc(const sem_desc* d) {
  if (!d) return fail(SEM_ERR_ARG, "null descriptor");
  if (d->dim < 1 || d->dim > 3) return fail(SEM_ERR_UNSUPPORTED, "dim %d outside 1..3", d->dim);
  const int maxN = (d->dim == 3) ? MAXP3 - 1 : MAXP - 1;
  if (d->order < 1 || d->order > maxN)
    return fail(SEM_ERR_UNSUPPORTED, "order %d outside 1..%d for dim %d", d->order, maxN, d->dim);
  if (d->dtype != SEM_F64 && d->dtype != SEM_F32) return fail(SEM_ERR_ARG, "dtype %d", d->dtype);
  if (d->batch < 1) return fail(SEM_ERR_ARG, "batch %d < 1", d->batch);
  if (!(d->nu >= 0.0) || !std::isfinite(d->nu)) return fail(SEM_ERR_ARG, "nu must be finite and >= 0");
  int64_t nodes = 1;
  for (int k = 0; k < d->dim; ++k) {
    if (d->elems[k] < 1) return fail(SEM_ERR_ARG, "elems[%d] = %d < 1", k, d->elems[k]);
    if (!(d->length[k] > 0.0) || !std::isfinite(d->length[k])) return fail(SEM_ERR_ARG, "length[%d] must be > 0", k);
    if ((int64_t)d->elems[k] * d->order > (int64_t)1 << 30) return fail(SEM_ERR_ARG, "mesh too large");
    nodes *= (int64_t)d->elems[k] * d->order;
  }
  // kernel index arithmetic is 32-bit within one batch member
  if (nodes >= ((int64_t)1 << 31)) return fail(SEM_ERR_ARG, "mesh too large: %lld nodes per component", (long long)nodes);
  if (nodes * d->dim * (int64_t)d->batch > ((int64_t)1 << 40)) return fail(SEM_ERR_ARG, "field too large");
  return SEM_OK;
}

// Fill a problem entry (offsets left to the caller).
void fill_prob(const sem_desc* d, ProbDev* p) {
  std::memset(p, 0, sizeof(*p));
  double xi[MAXP], w[MAXP], D[MAXP * MAXP];
  gll_tables(d->order, xi, w, D);
  p->N = d->order;
  p->P = d->order + 1;
  p->dim = d->dim;
  p->batch = d->batch;
  p->nelem = 1;
  p->nodes = 1;
  for (int k = 0; k < 3; ++k) {
    if (k < d->dim) {
      p->E[k] = d->elems[k];
      p->n[k] = d->elems[k] * d->order;
      const double h = d->length[k] / d->elems[k];
      p->sc[k] = 2.0 / h;
      p->hh[k] = 0.5 * h;
    } else {
      p->E[k] = 1;
      p->n[k] = 1;
      p->sc[k] = 0.0;
      p->hh[k] = 1.0;
    }
    p->nelem *= p->E[k];
    p->nodes *= p->n[k];
  }
  p->nu = d->nu;
  p->dt = 0.0;
  for (int i = 0; i < p->P; ++i) p->w[i] = w[i];
}

// Device tables (D, w) of one order, both precisions.
struct DevTables {
  DevBuf t64, t32;
  int make(int N) {
    double xi[MAXP], w[MAXP], D[MAXP * MAXP];
    gll_tables(N, xi, w, D);
    const int P = N + 1;
    Tables<double> a{};
    Tables<float> b{};
    for (int i = 0; i < P * P; ++i) {
      a.D[i] = D[i];
      b.D[i] = (float)D[i];
    }
    for (int i = 0; i < P; ++i) {
      a.w[i] = w[i];
      b.w[i] = (float)w[i];
    }
    int rc;
    if ((rc = t64.alloc(sizeof(a)))) return rc;
    if ((rc = t32.alloc(sizeof(b)))) return rc;
    HIPCHK(hipMemcpy(t64.p, &a, sizeof(a), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(t32.p, &b, sizeof(b), hipMemcpyHostToDevice));
    return SEM_OK;
  }
  const void* get(int dtype) const { return dtype == SEM_F64 ? t64.p : t32.p; }
};

// Operator application over a set of problems: element launches (one per order class, or the
// tuned 3-D kernel) followed by one summation launch.
struct OpSet {
  int dim = 0, dtype = 0;
  size_t ts = 8;
  std::vector<ProbDev> hp;  // host copy of the table (offsets, items)
  DevBuf dprob;             // device table
  struct Class {
    int P;
    int64_t nitems;
    int first, count;  // problems [first, first+count) of dprob, sorted by order
    DevTables tab;
    int epb = 0;
  };
  std::vector<Class> classes;
  int64_t total_vals = 0, total_nodes = 0, lvals = 0;
  DevBuf lvec;
  DevBuf face;  // face buffer of the tuned 3-D J v and J^T
  int fast = 0;  // one problem handled by a tuned kernel: 3 (kern_fast3d) or 2 (kern_fast2d)
  DevBuf fast_tab;
  // persistent mixed-order launch (2-D sets): cost-sorted work list and per-order tables
  int persistent = 0;  // 0: one launch per order class, 1: one persistent launch
  int pgrid = 1024;    // persistent grid size (workgroups)
  DevBuf items, ptabs64, ptabs32;
  int nitems = 0;
  // Batched 2-D sets: the table entries [0, ngeneric) run the element + summation kernels; the
  // rest (orders 3, 5, 7 with 8 | E_x <= 64) run the tuned 2-D kernel, one launch per (order,
  // x element count).
  int ngeneric = 0;
  struct TunedGroup {
    int N;   // order
    int nw;  // wavefronts per workgroup (E_x / 8)
    int nitems;
    DevBuf items;  // Fast2Item[nitems]
    DevBuf tab;    // device tables of order N
  };
  std::vector<TunedGroup> tuned;

  int finalize() {
    int rc;
    if ((rc = dprob.alloc(sizeof(ProbDev) * hp.size()))) return rc;
    HIPCHK(hipMemcpy(dprob.p, hp.data(), sizeof(ProbDev) * hp.size(), hipMemcpyHostToDevice));
    if (!fast && lvals > 0 && (rc = lvec.alloc(lvals * ts))) return rc;
    return SEM_OK;
  }

  hipError_t apply(int op, const void* u, const void* v, Coef in_scale, const Epi& epi, hipStream_t s) {
    if (fast == 3)
      return launch_fast3d(hp[0], static_cast<const ProbDev*>(dprob.p), op, u, v, face.p, epi, in_scale, fast_tab.p,
                           dtype, s);
    if (fast == 2)
      return launch_fast2d(hp[0], static_cast<const ProbDev*>(dprob.p), op, u, v, epi, in_scale, fast_tab.p, dtype, s);
    const ProbDev* dp = static_cast<const ProbDev*>(dprob.p);
    hipError_t e;
    if (ngeneric > 0) {
      if (persistent && nitems > 0) {
        e = launch_persist2d(dp, static_cast<const WorkItem*>(items.p), nitems, pgrid, op, dtype,
                             dtype == SEM_F64 ? ptabs64.p : ptabs32.p, u, v, lvec.p, in_scale, s);
        if (e != hipSuccess) return e;
      } else {
        for (auto& c : classes) {
          ElemLaunch el{dp + c.first, c.count, c.nitems, dim, c.P, dtype, c.epb};
          if ((e = launch_elem(el, op, u, v, lvec.p, in_scale, c.tab.get(dtype), s)) != hipSuccess) return e;
        }
      }
      if ((e = launch_dss(dp, ngeneric, total_nodes, dim, dtype, op != OP_JACT, lvec.p, epi, s)) != hipSuccess)
        return e;
    }
    for (auto& g : tuned)
      if ((e = launch_fast2d_batch(dp, static_cast<const Fast2Item*>(g.items.p), g.nitems, g.nw, g.N, op, u, v, epi,
                                   in_scale, g.tab.p, dtype, s)) != hipSuccess)
        return e;
    return hipSuccess;
  }
};

// Builds an OpSet for problems given by descriptors (packed back to back, sorted internally by
// order so that each order class is a contiguous table range; packed offsets keep input order).
int build_opset(OpSet& os, const sem_desc* descs, int count, bool allow_fast) {
  os.dim = descs[0].dim;
  os.dtype = descs[0].dtype;
  os.ts = os.dtype == SEM_F64 ? 8 : 4;
  std::vector<int64_t> off(count + 1, 0);
  std::vector<ProbDev> tmp(count);
  for (int i = 0; i < count; ++i) {
    fill_prob(&descs[i], &tmp[i]);
    off[i + 1] = off[i] + tmp[i].nodes * tmp[i].dim * tmp[i].batch;
    tmp[i].off = off[i];
  }
  os.total_vals = off[count];
  // the tuned 3-D kernel addresses a batch member and its face buffer with 32-bit byte offsets
  // and drops accesses by setting bit 31, so both must stay below 2 GiB
  const bool fast3 = count == 1 && fast3d_supported(tmp[0]) &&
                     fast3d_face_values(tmp[0]) / tmp[0].batch * 8 < ((int64_t)1 << 31);
  os.fast = !allow_fast || count != 1 ? 0 : fast3 ? 3 : fast2d_supported(tmp[0]) ? 2 : 0;
  // a batched 2-D set runs its problems of order 3, 5 or 7 with 8 | E_x <= 64 on the tuned kernel:
  // they go after every order class, so the generic launches cover a prefix of the table
  std::vector<char> is_tuned(count, 0);
  if (count > 1 && os.dim == 2)
    for (int i = 0; i < count; ++i) is_tuned[i] = fast2d_supported(tmp[i]) ? 1 : 0;
  // order classes of the generic problems
  std::vector<int> idx;
  for (int i = 0; i < count; ++i)
    if (!is_tuned[i]) idx.push_back(i);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return tmp[a].P < tmp[b].P; });
  const int ngen = (int)idx.size();
  os.hp.clear();
  os.classes.clear();
  int64_t lv = 0, nodes0 = 0;
  for (int k = 0; k < ngen;) {
    int P = tmp[idx[k]].P;
    OpSet::Class c;
    c.P = P;
    c.first = (int)os.hp.size();
    c.count = 0;
    int64_t items = 0;
    while (k < ngen && tmp[idx[k]].P == P) {
      ProbDev p = tmp[idx[k]];
      p.item0 = items;
      p.loff = lv;
      p.node0 = nodes0;
      items += p.nelem * p.batch;
      lv += p.nelem * p.batch * p.dim * (int64_t)std::pow(P, p.dim);
      nodes0 += p.nodes * p.batch;
      os.hp.push_back(p);
      ++c.count;
      ++k;
    }
    c.nitems = items;
    int rc = c.tab.make(P - 1);
    if (rc) return rc;
    os.classes.push_back(std::move(c));
  }
  // item0 must be class-relative for element launches but node0 global: already so.
  os.lvals = lv;
  os.ngeneric = ngen;
  // tuned problems: table entries after the generic ones, grouped by (order, x element count).  Each
  // group's launch splits its problems into row segments of S rows, S = rows / 256 clamped to
  // 1..4: a group's launch gets about one workgroup per CU or more, because these launches are
  // short and latency-bound (a segment costs S + 1 row steps: the row before it is recomputed).
  os.tuned.clear();
  {
    std::vector<int> tid;
    for (int i = 0; i < count; ++i)
      if (is_tuned[i]) tid.push_back(i);
    std::stable_sort(tid.begin(), tid.end(), [&](int a, int b) {
      return tmp[a].N != tmp[b].N ? tmp[a].N < tmp[b].N : tmp[a].E[0] < tmp[b].E[0];
    });
    for (size_t k = 0; k < tid.size();) {
      const int nw = fast2d_waves(tmp[tid[k]]), N = tmp[tid[k]].N;
      size_t k1 = k;
      int64_t rows = 0;
      for (; k1 < tid.size() && fast2d_waves(tmp[tid[k1]]) == nw && tmp[tid[k1]].N == N; ++k1)
        rows += (int64_t)tmp[tid[k1]].E[1] * fast2d_xsegments(tmp[tid[k1]]);
      const int SEG = (int)std::max<int64_t>(1, std::min<int64_t>(4, rows / 256));
      std::vector<Fast2Item> its;
      for (; k < k1; ++k) {
        ProbDev p = tmp[tid[k]];
        p.item0 = p.loff = p.node0 = 0;  // unused: no element items, scratch or summation items
        const int t = (int)os.hp.size();
        os.hp.push_back(p);
        const int nxs = fast2d_xsegments(p), xw = p.E[0] / nxs;
        for (int y0 = 0; y0 < p.E[1]; y0 += SEG)
          for (int xs = 0; xs < nxs; ++xs) its.push_back({t, y0, std::min(SEG, p.E[1] - y0), xs * xw});
      }
      OpSet::TunedGroup g;
      g.N = N;
      g.nw = nw;
      g.nitems = (int)its.size();
      int rc;
      if ((rc = g.items.alloc(sizeof(Fast2Item) * its.size()))) return rc;
      HIPCHK(hipMemcpy(g.items.p, its.data(), sizeof(Fast2Item) * its.size(), hipMemcpyHostToDevice));
      std::vector<char> host(fast_table_bytes(N));
      fast_fill_tables(N, host.data());
      if ((rc = g.tab.alloc(host.size()))) return rc;
      HIPCHK(hipMemcpy(g.tab.p, host.data(), host.size(), hipMemcpyHostToDevice));
      HIPCHK(fast2d_prepare(N, os.dtype));
      os.tuned.push_back(std::move(g));
    }
  }
  if (os.dim == 2 && count > 1 && ngen > 0) {
    // persistent work list: chunks of whole elements per 256-thread workgroup, largest cost first
    struct It {
      WorkItem w;
      double cost;
    };
    std::vector<It> its;
    for (size_t t = 0; t < (size_t)ngen; ++t) {
      const ProbDev& p = os.hp[t];
      const int per = persist2d_elems_per_item(p.P);
      const int64_t tot = p.nelem * p.batch;
      for (int64_t e0 = 0; e0 < tot; e0 += per) {
        WorkItem w{(int32_t)t, p.P, e0, (int32_t)std::min<int64_t>(per, tot - e0), 0};
        its.push_back({w, (double)w.ne * p.P * p.P * p.P});
      }
    }
    std::stable_sort(its.begin(), its.end(), [](const It& a, const It& b) { return a.cost > b.cost; });
    std::vector<WorkItem> wl(its.size());
    for (size_t i = 0; i < its.size(); ++i) wl[i] = its[i].w;
    os.nitems = (int)wl.size();
    int rc;
    if ((rc = os.items.alloc(sizeof(WorkItem) * wl.size()))) return rc;
    HIPCHK(hipMemcpy(os.items.p, wl.data(), sizeof(WorkItem) * wl.size(), hipMemcpyHostToDevice));
    std::vector<Tables<double>> t64(MAXP + 1);
    std::vector<Tables<float>> t32(MAXP + 1);
    for (int P = 2; P <= MAXP; ++P) {
      double xi[MAXP], w[MAXP], D[MAXP * MAXP];
      gll_tables(P - 1, xi, w, D);
      for (int i = 0; i < P * P; ++i) {
        t64[P].D[i] = D[i];
        t32[P].D[i] = (float)D[i];
      }
      for (int i = 0; i < P; ++i) {
        t64[P].w[i] = w[i];
        t32[P].w[i] = (float)w[i];
      }
    }
    if ((rc = os.ptabs64.alloc(sizeof(Tables<double>) * t64.size()))) return rc;
    if ((rc = os.ptabs32.alloc(sizeof(Tables<float>) * t32.size()))) return rc;
    HIPCHK(hipMemcpy(os.ptabs64.p, t64.data(), sizeof(Tables<double>) * t64.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(os.ptabs32.p, t32.data(), sizeof(Tables<float>) * t32.size(), hipMemcpyHostToDevice));
    os.persistent = 1;
  }
  os.total_nodes = nodes0;
  if (os.fast) {
    int rc;
    std::vector<char> host(fast_table_bytes(descs[0].order));
    fast_fill_tables(descs[0].order, host.data());
    if ((rc = os.fast_tab.alloc(host.size()))) return rc;
    HIPCHK(hipMemcpy(os.fast_tab.p, host.data(), host.size(), hipMemcpyHostToDevice));
    if (os.fast == 3 && fast3d_needs_face(os.hp[0], os.dtype == SEM_F32) &&
        (rc = os.face.alloc(fast3d_face_values(os.hp[0]) * os.ts)))
      return rc;
    if (os.fast == 2) HIPCHK(fast2d_prepare(descs[0].order, os.dtype));
  }
  return os.finalize();
}

// RK4 forward/adjoint machinery shared by contexts and batches.
struct Integrator {
  OpSet* os = nullptr;
  int64_t n = 0;  // values per state (all problems / batch members)
  size_t ts = 8;
  enum { STATE, S1, S2, ACC, USTATE, A2, A3, A4, T1, T2, LACC, LAMB, NBUF };
  DevBuf buf[NBUF];
  static constexpr int NSCHEME = 2;  // SEM_RK4, SEM_RK3
  bool ready[NSCHEME] = {};
  hipStream_t cap = nullptr;
  hipGraphExec_t gstep[NSCHEME] = {}, gadj[NSCHEME] = {};
  DevBuf dts;  // per-problem dt table for the batch
  // Adjoint with uniform checkpoints: the segment recompute writes every step's stage states to
  // the work buffer and the adjoint steps read them (as an adjoint with stored stages does, Sec.
  // 4.1), instead of recomputing them in each adjoint step.  Those launches address a different
  // work slot every step, so they run uncaptured; for small states, where launch overhead would
  // dominate, the captured recompute-in-step graphs run instead.  Both give the same values.
  int adj_mode = SEM_ADJ_AUTO;
  static constexpr int64_t STORE_MIN_VALUES = (int64_t)1 << 22;  // auto: stored stages from 4M values
  static constexpr int MAX_STAGE_STATES = 4;                       // u, U2, U3, U4 (RK4)
  static int stage_states(int scheme) { return scheme == SEM_RK3 ? 3 : 4; }
  bool stores_stages() const {
    return adj_mode == SEM_ADJ_STORE || (adj_mode == SEM_ADJ_AUTO && n >= STORE_MIN_VALUES);
  }
  // states the caller's adjoint work buffer holds for ckpt_every K
  int64_t work_states(int32_t K) const { return (int64_t)K * (stores_stages() ? MAX_STAGE_STATES : 1); }

  ~Integrator() {
    reset_graphs(nullptr);
    if (cap) (void)hipStreamDestroy(cap);
  }
  void* b(int i) { return buf[i].p; }

  // Drop the captured graphs (after the operator's launch configuration changed).  Graph launches
  // may still be in flight on the handle's stream s (every earlier stream of the handle is
  // chained into it), so s is synchronised before any executable graph is destroyed; null s: the
  // caller has already waited (the handle's destroy).
  void reset_graphs(hipStream_t s, bool wait = false) {
    bool any = false;
    for (int k = 0; k < NSCHEME; ++k) any = any || gstep[k] || gadj[k];
    if (any && wait) (void)hipStreamSynchronize(s);
    for (int k = 0; k < NSCHEME; ++k) {
      if (gstep[k]) (void)hipGraphExecDestroy(gstep[k]);
      if (gadj[k]) (void)hipGraphExecDestroy(gadj[k]);
      gstep[k] = gadj[k] = nullptr;
      ready[k] = false;
    }
  }

  hipError_t enqueue_step(hipStream_t s, int scheme) {
    return scheme == SEM_RK3 ? enqueue_step_rk3(s) : enqueue_step_rk4(s);
  }
  hipError_t enqueue_adjoint_step(hipStream_t s, int scheme) {
    return scheme == SEM_RK3 ? enqueue_adjoint_step_rk3(s) : enqueue_adjoint_step_rk4(s);
  }

  // one step of Kutta's third-order method on STATE, stage updates fused into the epilogues:
  //   U2 = u + dt/2 k1,  U3 = u - dt k1 + 2 dt k2 = 3u - 2 U2 + 2 dt k2,
  //   u+ = u + dt/6 k1 + 2dt/3 k2 + dt/6 k3 = [(2/3) u + (1/3) U2 + (2dt/3) k2] + dt/6 k3
  hipError_t enqueue_step_rk3(hipStream_t s) {
    hipError_t e;
    const Coef one{1, 0}, zero{0, 0};
    Epi ep{b(S1), b(STATE), one, {0, 0.5}, nullptr, nullptr, zero, zero};
    if ((e = os->apply(OP_RHS, b(STATE), nullptr, one, ep, s))) return e;
    ep = Epi{b(S2), b(STATE), {3, 0}, {0, 2.0}, b(ACC), b(S1), {1.0 / 3, 0}, {0, 2.0 / 3}, {-2, 0}, {2.0 / 3, 0}};
    if ((e = os->apply(OP_RHS, b(S1), nullptr, one, ep, s))) return e;
    ep = Epi{b(STATE), b(ACC), one, {0, 1.0 / 6}, nullptr, nullptr, zero, zero};
    return os->apply(OP_RHS, b(S2), nullptr, one, ep, s);
  }

  // reverse sweep through one step of Kutta's method taken from USTATE (tableau A21 = 1/2,
  // A31 = -1, A32 = 2, b = 1/6, 2/3, 1/6), updating LAMB in place:
  //   a3 = J(U3)^T (dt/6 lam);  a2 = J(U2)^T (2dt/3 lam + 2 dt a3);
  //   a1 = J(u)^T (dt/6 lam + dt/2 a2 - dt a3);  lam <- lam + a1 + a2 + a3.
  // With S = lam + a3 kept in LACC, the input of a1 is (7dt/6) lam - dt S + dt/2 a2.
  hipError_t enqueue_adjoint_step_rk3(hipStream_t s) {
    hipError_t e;
    const Coef one{1, 0}, zero{0, 0};
    Epi ep{b(A2), b(USTATE), one, {0, 0.5}, nullptr, nullptr, zero, zero};
    if ((e = os->apply(OP_RHS, b(USTATE), nullptr, one, ep, s))) return e;
    ep = Epi{b(A3), b(USTATE), {3, 0}, {0, 2.0}, nullptr, b(A2), zero, zero, {-2, 0}, zero};
    if ((e = os->apply(OP_RHS, b(A2), nullptr, one, ep, s))) return e;
    const void* st[2] = {b(A2), b(A3)};
    return enqueue_adjoint_jt_rk3(s, b(USTATE), st);
  }
  // the J^T part of the RK-3 adjoint step from u and its stage states st = {U2, U3}, updating
  // the adjoint state lam in place (LAMB unless a caller buffer is given)
  hipError_t enqueue_adjoint_jt_rk3(hipStream_t s, const void* u, const void* const* st, void* lam = nullptr) {
    hipError_t e;
    const Coef one{1, 0}, zero{0, 0};
    void* L = lam ? lam : b(LAMB);
    Epi ep{b(T1), L, {0, 2.0 / 3}, {0, 2.0}, b(LACC), L, one, one};
    if ((e = os->apply(OP_JACT, st[1], L, {0, 1.0 / 6}, ep, s))) return e;
    ep = Epi{b(T2), L, {0, 7.0 / 6}, {0, 0.5}, b(LACC), b(LACC), one, one, {0, -1.0}, zero};
    if ((e = os->apply(OP_JACT, st[0], b(T1), one, ep, s))) return e;
    ep = Epi{L, b(LACC), one, one, nullptr, nullptr, zero, zero};
    return os->apply(OP_JACT, u, b(T2), one, ep, s);
  }

  // one RK4 step on STATE (stage updates fused into the summation epilogues)
  hipError_t enqueue_step_rk4(hipStream_t s) {
    hipError_t e;
    Epi ep{};
    // k1 = F(u):  S1 = u + dt/2 k1;  ACC = u + dt/6 k1
    ep = Epi{b(S1), b(STATE), {1, 0}, {0, 0.5}, b(ACC), b(STATE), {1, 0}, {0, 1.0 / 6}};
    if ((e = os->apply(OP_RHS, b(STATE), nullptr, {1, 0}, ep, s))) return e;
    // k2 = F(S1): S2 = u + dt/2 k2;  ACC += dt/3 k2
    ep = Epi{b(S2), b(STATE), {1, 0}, {0, 0.5}, b(ACC), b(ACC), {1, 0}, {0, 1.0 / 3}};
    if ((e = os->apply(OP_RHS, b(S1), nullptr, {1, 0}, ep, s))) return e;
    // k3 = F(S2): S1 = u + dt k3;  ACC += dt/3 k3
    ep = Epi{b(S1), b(STATE), {1, 0}, {0, 1.0}, b(ACC), b(ACC), {1, 0}, {0, 1.0 / 3}};
    if ((e = os->apply(OP_RHS, b(S2), nullptr, {1, 0}, ep, s))) return e;
    // k4 = F(S1): u = ACC + dt/6 k4
    ep = Epi{b(STATE), b(ACC), {1, 0}, {0, 1.0 / 6}, nullptr, nullptr, {0, 0}, {0, 0}};
    return os->apply(OP_RHS, b(S1), nullptr, {1, 0}, ep, s);
  }

  // reverse sweep through one RK4 step taken from USTATE, updating LAMB in place:
  //   U2 = u + dt/2 F(u), U3 = u + dt/2 F(U2), U4 = u + dt F(U3)   (recomputed)
  //   a4 = J(U4)^T (dt/6 lam); a3 = J(U3)^T (dt/3 lam + dt a4); a2 = J(U2)^T (dt/3 lam + dt/2 a3);
  //   a1 = J(u)^T (dt/6 lam + dt/2 a2); lam <- lam + a1 + a2 + a3 + a4
  hipError_t enqueue_adjoint_step_rk4(hipStream_t s) {
    hipError_t e;
    const Coef one{1, 0}, zero{0, 0};
    Epi ep{b(A2), b(USTATE), one, {0, 0.5}, nullptr, nullptr, zero, zero};
    if ((e = os->apply(OP_RHS, b(USTATE), nullptr, one, ep, s))) return e;
    ep = Epi{b(A3), b(USTATE), one, {0, 0.5}, nullptr, nullptr, zero, zero};
    if ((e = os->apply(OP_RHS, b(A2), nullptr, one, ep, s))) return e;
    ep = Epi{b(A4), b(USTATE), one, {0, 1.0}, nullptr, nullptr, zero, zero};
    if ((e = os->apply(OP_RHS, b(A3), nullptr, one, ep, s))) return e;
    const void* st[3] = {b(A2), b(A3), b(A4)};
    return enqueue_adjoint_jt_rk4(s, b(USTATE), st);
  }
  // the J^T part of the RK4 adjoint step from u and its stage states st = {U2, U3, U4}, updating
  // the adjoint state lam in place (LAMB unless a caller buffer is given)
  hipError_t enqueue_adjoint_jt_rk4(hipStream_t s, const void* u, const void* const* st, void* lam = nullptr) {
    hipError_t e;
    const Coef one{1, 0}, zero{0, 0};
    void* L = lam ? lam : b(LAMB);
    Epi ep{b(T1), L, {0, 1.0 / 3}, {0, 1.0}, b(LACC), L, one, one};
    if ((e = os->apply(OP_JACT, st[2], L, {0, 1.0 / 6}, ep, s))) return e;
    ep = Epi{b(T2), L, {0, 1.0 / 3}, {0, 0.5}, b(LACC), b(LACC), one, one};
    if ((e = os->apply(OP_JACT, st[1], b(T1), one, ep, s))) return e;
    ep = Epi{b(T1), L, {0, 1.0 / 6}, {0, 0.5}, b(LACC), b(LACC), one, one};
    if ((e = os->apply(OP_JACT, st[0], b(T2), one, ep, s))) return e;
    ep = Epi{L, b(LACC), one, one, nullptr, nullptr, zero, zero};
    return os->apply(OP_JACT, u, b(T1), one, ep, s);
  }

  // One step from u with its stage states written to st (RK4: U2, U3, U4; RK-3: U2, U3) and the
  // new state to unext: the same launches and coefficients as the captured step, so the states
  // are the same values.  With unext null (the last step of a segment) only the stage states are
  // formed, without the accumulator, as in the adjoint step's own recompute.
  hipError_t enqueue_step_stages(hipStream_t s, int scheme, const void* u, void* const* st, void* unext,
                                 void* accbuf = nullptr) {
    hipError_t e;
    const Coef one{1, 0}, zero{0, 0};
    void* acc = unext ? (accbuf ? accbuf : b(ACC)) : nullptr;
    Epi ep{};
    if (scheme == SEM_RK3) {
      ep = Epi{st[0], u, one, {0, 0.5}, nullptr, nullptr, zero, zero};
      if ((e = os->apply(OP_RHS, u, nullptr, one, ep, s))) return e;
      ep = unext ? Epi{st[1], u, {3, 0}, {0, 2.0}, acc, st[0], {1.0 / 3, 0}, {0, 2.0 / 3}, {-2, 0}, {2.0 / 3, 0}}
                 : Epi{st[1], u, {3, 0}, {0, 2.0}, nullptr, st[0], zero, zero, {-2, 0}, zero};
      if ((e = os->apply(OP_RHS, st[0], nullptr, one, ep, s))) return e;
      if (!unext) return hipSuccess;
      ep = Epi{unext, acc, one, {0, 1.0 / 6}, nullptr, nullptr, zero, zero};
      return os->apply(OP_RHS, st[1], nullptr, one, ep, s);
    }
    ep = Epi{st[0], u, one, {0, 0.5}, acc, unext ? u : nullptr, one, {0, 1.0 / 6}};
    if ((e = os->apply(OP_RHS, u, nullptr, one, ep, s))) return e;
    ep = Epi{st[1], u, one, {0, 0.5}, acc, acc, one, {0, 1.0 / 3}};
    if ((e = os->apply(OP_RHS, st[0], nullptr, one, ep, s))) return e;
    ep = Epi{st[2], u, one, {0, 1.0}, acc, acc, one, {0, 1.0 / 3}};
    if ((e = os->apply(OP_RHS, st[1], nullptr, one, ep, s))) return e;
    if (!unext) return hipSuccess;
    ep = Epi{unext, acc, one, {0, 1.0 / 6}, nullptr, nullptr, zero, zero};
    return os->apply(OP_RHS, st[2], nullptr, one, ep, s);
  }

  int alloc_buffers() {
    for (int i = 0; i < NBUF; ++i) {
      if (buf[i].p) continue;
      int rc = buf[i].alloc(n * ts);
      if (rc) return rc;
    }
    return SEM_OK;
  }

  int prepare(int scheme) {
    if (ready[scheme]) return SEM_OK;
    if (int rc = alloc_buffers()) return rc;
    if (!cap) HIPCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue_step(cap, scheme);
    hipError_t e2 = hipStreamEndCapture(cap, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(SEM_ERR_HIP, "capturing the time step: %s", hipGetErrorString(e ? e : e2));
    }
    e = hipGraphInstantiate(&gstep[scheme], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHK(e);
    g = nullptr;
    HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    e = enqueue_adjoint_step(cap, scheme);
    e2 = hipStreamEndCapture(cap, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(SEM_ERR_HIP, "capturing the adjoint step: %s", hipGetErrorString(e ? e : e2));
    }
    e = hipGraphInstantiate(&gadj[scheme], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHK(e);
    ready[scheme] = true;
    return SEM_OK;
  }

  // dt: a single value for every table entry, or per-entry values in dts (device) when per_problem
  int set_dt(double dt, bool per_problem, hipStream_t s) {
    const int np = (int)os->hp.size();
    hipLaunchKernelGGL(set_dt_kernel, dim3((np + 63) / 64), dim3(64), 0, s, static_cast<ProbDev*>(os->dprob.p), np,
                       per_problem ? static_cast<const double*>(dts.p) : nullptr, dt);
    HIPCHK(hipGetLastError());
    return SEM_OK;
  }

  int forward(int scheme, void* u, int32_t nsteps, int32_t K, void* ckpt, hipStream_t s) {
    const size_t bytes = n * ts;
    HIPCHK(hipMemcpyAsync(b(STATE), u, bytes, hipMemcpyDeviceToDevice, s));
    for (int k = 0; k < nsteps; ++k) {
      if (ckpt && k % K == 0)
        HIPCHK(hipMemcpyAsync(static_cast<char*>(ckpt) + (size_t)(k / K) * bytes, b(STATE), bytes,
                              hipMemcpyDeviceToDevice, s));
      HIPCHK(hipGraphLaunch(gstep[scheme], s));
    }
    HIPCHK(hipMemcpyAsync(u, b(STATE), bytes, hipMemcpyDeviceToDevice, s));
    return SEM_OK;
  }

  int adjoint(int scheme, const void* ckpt, int32_t nsteps, int32_t K, void* lam, void* work, hipStream_t s) {
    const size_t bytes = n * ts;
    char* wk = static_cast<char*>(work);
    if (stores_stages()) {
      // work: [K][stage_states][n]; slot (k, 0) holds u_k (k >= 1; u_0 is read from its
      // checkpoint), slots (k, 1..) its stage states.  These launches are not captured, so the
      // adjoint state is updated in the caller's buffer (no copy in or out); it must not overlap
      // the checkpoints or the work slots, which are read until the last step.
      const int ns = stage_states(scheme);
      {
        const char* l0 = static_cast<const char*>(lam);
        const char* c0 = static_cast<const char*>(ckpt);
        const size_t cb = (size_t)(nsteps / K) * bytes, wb = (size_t)K * ns * bytes;
        if ((nsteps > 0 && l0 < c0 + cb && c0 < l0 + bytes) || (l0 < wk + wb && wk < l0 + bytes))
          return fail(SEM_ERR_ARG, "lam overlaps the checkpoints or the work buffer");
      }
      auto slot = [&](int k, int j) -> void* { return wk + ((size_t)k * ns + j) * bytes; };
      for (int sg = nsteps / K - 1; sg >= 0; --sg) {
        const void* u0 = static_cast<const char*>(ckpt) + (size_t)sg * bytes;
        auto state = [&](int k) -> const void* { return k == 0 ? u0 : slot(k, 0); };
        for (int k = 0; k < K; ++k) {
          void* st[3] = {slot(k, 1), slot(k, 2), ns > 3 ? slot(k, 3) : nullptr};
          HIPCHK(enqueue_step_stages(s, scheme, state(k), st, k + 1 < K ? slot(k + 1, 0) : nullptr));
        }
        for (int k = K - 1; k >= 0; --k) {
          const void* st[3] = {slot(k, 1), slot(k, 2), ns > 3 ? slot(k, 3) : nullptr};
          HIPCHK(scheme == SEM_RK3 ? enqueue_adjoint_jt_rk3(s, state(k), st, lam)
                                   : enqueue_adjoint_jt_rk4(s, state(k), st, lam));
        }
      }
      return SEM_OK;
    }
    HIPCHK(hipMemcpyAsync(b(LAMB), lam, bytes, hipMemcpyDeviceToDevice, s));
    for (int sg = nsteps / K - 1; sg >= 0; --sg) {
      HIPCHK(hipMemcpyAsync(b(STATE), static_cast<const char*>(ckpt) + (size_t)sg * bytes, bytes,
                            hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpyAsync(wk, b(STATE), bytes, hipMemcpyDeviceToDevice, s));
      for (int k = 1; k < K; ++k) {
        HIPCHK(hipGraphLaunch(gstep[scheme], s));
        HIPCHK(hipMemcpyAsync(wk + (size_t)k * bytes, b(STATE), bytes, hipMemcpyDeviceToDevice, s));
      }
      for (int k = K - 1; k >= 0; --k) {
        HIPCHK(hipMemcpyAsync(b(USTATE), wk + (size_t)k * bytes, bytes, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipGraphLaunch(gadj[scheme], s));
      }
    }
    HIPCHK(hipMemcpyAsync(lam, b(LAMB), bytes, hipMemcpyDeviceToDevice, s));
    return SEM_OK;
  }

  // Every stage stored by the forward sweep: stages[k][S][n] holds u_k and its stage states, formed
  // by the same launches as the stage-storing segment recompute (so the same values as the
  // captured step), and the adjoint applies only the J^T part of each step.
  void* stage_slot(void* stages, int scheme, int k, int j) const {
    return static_cast<char*>(stages) + ((size_t)k * stage_states(scheme) + j) * (size_t)n * ts;
  }
  int forward_stored(int scheme, void* u, int32_t nsteps, void* stages, hipStream_t s) {
    if (nsteps == 0) return SEM_OK;
    const int ns = stage_states(scheme);
    HIPCHK(hipMemcpyAsync(stage_slot(stages, scheme, 0, 0), u, (size_t)n * ts, hipMemcpyDeviceToDevice, s));
    for (int k = 0; k < nsteps; ++k) {
      void* st[3] = {stage_slot(stages, scheme, k, 1), stage_slot(stages, scheme, k, 2),
                     ns > 3 ? stage_slot(stages, scheme, k, 3) : nullptr};
      void* unext = k + 1 < nsteps ? stage_slot(stages, scheme, k + 1, 0) : u;
      HIPCHK(enqueue_step_stages(s, scheme, stage_slot(stages, scheme, k, 0), st, unext));
    }
    return SEM_OK;
  }
  // The adjoint state is updated in the caller's buffer (in: lam_T, out: lam_0), so no copy in
  // or out: these launches are not captured, so they may take any buffer.  lam must therefore not
  // overlap the stage states, which are read until the last step.
  int adjoint_stored(int scheme, const void* stages, int32_t nsteps, void* lam, hipStream_t s) {
    if (nsteps == 0) return SEM_OK;
    const int ns = stage_states(scheme);
    {
      const char* s0 = static_cast<const char*>(stages);
      const char* s1 = s0 + (size_t)nsteps * ns * n * ts;
      const char* l0 = static_cast<const char*>(lam);
      if (l0 < s1 && s0 < l0 + (size_t)n * ts) return fail(SEM_ERR_ARG, "lam overlaps the stage states");
    }
    void* sb = const_cast<void*>(stages);  // read only
    for (int k = nsteps - 1; k >= 0; --k) {
      const void* st[3] = {stage_slot(sb, scheme, k, 1), stage_slot(sb, scheme, k, 2),
                           ns > 3 ? stage_slot(sb, scheme, k, 3) : nullptr};
      const void* uk = stage_slot(sb, scheme, k, 0);
      HIPCHK(scheme == SEM_RK3 ? enqueue_adjoint_jt_rk3(s, uk, st, lam) : enqueue_adjoint_jt_rk4(s, uk, st, lam));
    }
    return SEM_OK;
  }

  // Binomial checkpointing.  The forward sweep stores the schedule's first snapshots (the states
  // its actions store before the first adjoint step) into ckpt slots; the adjoint sweep copies
  // them to work and runs the rest of the schedule there.
  static size_t first_adjoint(const std::vector<RevolveAct>& acts) {
    size_t k = 0;
    while (k < acts.size() && acts[k].kind != REV_ADJOINT) ++k;
    while (k > 0 && acts[k].kind != REV_RESTORE) --k;  // its restore starts the adjoint sweep
    return k;
  }

  int forward_revolve(int scheme, void* u, int32_t nsteps, const std::vector<RevolveAct>& acts, void* ckpt,
                      hipStream_t s) {
    const size_t bytes = n * ts;
    std::vector<int64_t> slot_at(nsteps, -1);  // snapshot slot taking the state before step k
    int64_t p = 0;
    std::vector<int64_t> slot_pos(1, 0);  // step index held by each slot
    for (size_t k = 0; k < first_adjoint(acts); ++k) {
      const RevolveAct& a = acts[k];
      if (a.kind == REV_RESTORE) {
        if (a.arg >= (int64_t)slot_pos.size()) return fail(SEM_ERR_ARG, "schedule restores an empty slot");
        p = slot_pos[a.arg];
      }
      if (a.kind == REV_ADVANCE) p += a.arg;
      if (a.kind == REV_STORE) {
        if ((int64_t)slot_pos.size() <= a.arg) slot_pos.resize(a.arg + 1, 0);
        slot_pos[a.arg] = p;
        slot_at[p] = a.arg;
      }
    }
    slot_at[0] = 0;
    HIPCHK(hipMemcpyAsync(b(STATE), u, bytes, hipMemcpyDeviceToDevice, s));
    for (int32_t k = 0; k < nsteps; ++k) {
      if (slot_at[k] >= 0)
        HIPCHK(hipMemcpyAsync(static_cast<char*>(ckpt) + (size_t)slot_at[k] * bytes, b(STATE), bytes,
                              hipMemcpyDeviceToDevice, s));
      HIPCHK(hipGraphLaunch(gstep[scheme], s));
    }
    HIPCHK(hipMemcpyAsync(u, b(STATE), bytes, hipMemcpyDeviceToDevice, s));
    return SEM_OK;
  }

  int adjoint_revolve(int scheme, const void* ckpt, int32_t snaps, const std::vector<RevolveAct>& acts, void* lam,
                      void* work, hipStream_t s) {
    const size_t bytes = n * ts;
    char* wk = static_cast<char*>(work);
    HIPCHK(hipMemcpyAsync(wk, ckpt, (size_t)snaps * bytes, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(b(LAMB), lam, bytes, hipMemcpyDeviceToDevice, s));
    for (size_t k = first_adjoint(acts); k < acts.size(); ++k) {
      const RevolveAct& a = acts[k];
      switch (a.kind) {
        case REV_RESTORE: {
          // a restore followed directly by an adjoint step goes straight to the step's input
          const bool direct = k + 1 < acts.size() && acts[k + 1].kind == REV_ADJOINT;
          HIPCHK(hipMemcpyAsync(b(direct ? USTATE : STATE), wk + (size_t)a.arg * bytes, bytes,
                                hipMemcpyDeviceToDevice, s));
          if (direct) {
            HIPCHK(hipGraphLaunch(gadj[scheme], s));
            ++k;
          }
          break;
        }
        case REV_ADVANCE:
          for (int64_t i = 0; i < a.arg; ++i) HIPCHK(hipGraphLaunch(gstep[scheme], s));
          break;
        case REV_STORE:
          HIPCHK(hipMemcpyAsync(wk + (size_t)a.arg * bytes, b(STATE), bytes, hipMemcpyDeviceToDevice, s));
          break;
        default:  // REV_ADJOINT after an advance
          HIPCHK(hipMemcpyAsync(b(USTATE), b(STATE), bytes, hipMemcpyDeviceToDevice, s));
          HIPCHK(hipGraphLaunch(gadj[scheme], s));
      }
    }
    HIPCHK(hipMemcpyAsync(lam, b(LAMB), bytes, hipMemcpyDeviceToDevice, s));
    return SEM_OK;
  }
};

// Crank-Nicolson with Newton-Krylov solves on the integrator's state buffers plus a caller work
// buffer (GMRES basis, and the recomputed states of an adjoint segment).
struct Implicit {
  Integrator* in = nullptr;
  double* partial = nullptr;  // blas_partial_bytes()
  double* dvec = nullptr;     // 3 * blas_max_vectors() doubles: dot results and combination weights
  hipStream_t s = nullptr;
  double newton_rtol = 0, gmres_rtol = 0;
  int newton_maxit = 0, restart = 0, gmres_maxit = 0;
  sem_nk_stats st{};

  int dtype() const { return in->os->dtype; }
  int64_t n() const { return in->n; }
  size_t bytes() const { return (size_t)in->n * in->ts; }

  int configure(const sem_nk_opts* o) {
    const bool f64 = dtype() == SEM_F64;
    newton_rtol = (o && o->newton_rtol > 0) ? o->newton_rtol : (f64 ? 1e-13 : 1e-6);
    gmres_rtol = (o && o->gmres_rtol > 0) ? o->gmres_rtol : (f64 ? 1e-11 : 1e-5);
    newton_maxit = (o && o->newton_maxit > 0) ? o->newton_maxit : 25;
    restart = (o && o->gmres_restart > 0) ? o->gmres_restart : 30;
    gmres_maxit = (o && o->gmres_maxit > 0) ? o->gmres_maxit : 300;
    if (restart > blas_max_vectors() - 1)
      return fail(SEM_ERR_ARG, "gmres_restart %d exceeds %d", restart, blas_max_vectors() - 1);
    st = sem_nk_stats{};
    return SEM_OK;
  }

  // host copies of <X_j, w>, j < nv (the device copy stays in dvec for a following combination)
  int dots(const void* X, int nv, const void* w, double* h) {
    HIPCHK(blas_multidot(dtype(), X, in->n, nv, w, in->n, partial, dvec, s));
    HIPCHK(hipMemcpyAsync(h, dvec, sizeof(double) * nv, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return SEM_OK;
  }
  int norm(const void* w, double* r) {
    double h = 0;
    if (int rc = dots(w, 1, w, &h)) return rc;
    *r = std::sqrt(h > 0 ? h : 0.0);
    return SEM_OK;
  }

  // out = p + cdt * dt * op(at) p  (op: J or J^T at the state `at`)
  hipError_t matvec(int op, const void* at, double cdt, const void* p, void* out) {
    const Coef one{1, 0}, zero{0, 0};
    Epi ep{out, p, one, {0, cdt}, nullptr, nullptr, zero, zero};
    return in->os->apply(op, at, p, one, ep, s);
  }

  // Restarted GMRES for (I + cdt dt op(at)) x = b from x = 0; basis: restart + 1 vectors, then one
  // more vector of scratch.  Classical Gram-Schmidt, applied twice.
  int gmres(int op, const void* at, double cdt, const void* b, void* x, char* basis) {
    const size_t B = bytes();
    const int m = restart;
    auto V = [&](int j) { return basis + (size_t)j * B; };
    char* tmp = V(m + 1);
    double bnorm = 0;
    if (int rc = norm(b, &bnorm)) return rc;
    HIPCHK(blas_axpby(dtype(), x, 0.0, b, 0.0, nullptr, in->n, s));  // x = 0
    ++st.linear_solves;
    if (!(bnorm > 0)) return std::isfinite(bnorm) ? SEM_OK : fail(SEM_ERR_NONFINITE, "non-finite Krylov right-hand side");
    std::vector<double> H((m + 1) * m), cs(m), sn(m), g(m + 1), y(m), h(m + 1), h2(m + 1);
    int total = 0;
    double res = bnorm;
    bool first = true;
    while (true) {
      // r = b - A x  (x = 0 on the first cycle)
      if (first) {
        HIPCHK(blas_axpby(dtype(), V(0), 1.0 / bnorm, b, 0.0, nullptr, in->n, s));
        res = bnorm;
      } else {
        HIPCHK(matvec(op, at, cdt, x, tmp));
        HIPCHK(blas_axpby(dtype(), tmp, 1.0, b, -1.0, tmp, in->n, s));
        if (int rc = norm(tmp, &res)) return rc;
        if (!(res > 0)) break;
        HIPCHK(blas_axpby(dtype(), V(0), 1.0 / res, tmp, 0.0, nullptr, in->n, s));
      }
      first = false;
      std::fill(g.begin(), g.end(), 0.0);
      g[0] = res;
      int k = 0;
      for (; k < m && total < gmres_maxit; ++k, ++total) {
        HIPCHK(matvec(op, at, cdt, V(k), V(k + 1)));
        // w = V(k+1): h = V^T w; w -= V h fused with h2 = V^T w; w -= V h2 fused with |w|^2.
        // Three passes over the basis, coefficients kept on the device, one host sync.
        const int MV = blas_max_vectors();
        HIPCHK(blas_multidot(dtype(), V(0), in->n, k + 1, V(k + 1), in->n, partial, dvec, s));
        HIPCHK(blas_combine_dot(dtype(), V(k + 1), V(0), in->n, k + 1, dvec, -1.0, in->n, false, partial, dvec + MV,
                                s));
        HIPCHK(blas_combine_dot(dtype(), V(k + 1), V(0), in->n, k + 1, dvec + MV, -1.0, in->n, true, partial,
                                dvec + 2 * MV, s));
        double hn2 = 0;
        HIPCHK(hipMemcpyAsync(h.data(), dvec, sizeof(double) * (k + 1), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(h2.data(), dvec + MV, sizeof(double) * (k + 1), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&hn2, dvec + 2 * MV, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const double hn = std::sqrt(hn2 > 0 ? hn2 : 0.0);
        for (int i = 0; i <= k; ++i) H[i * m + k] = h[i] + h2[i];
        H[(k + 1) * m + k] = hn;
        if (hn > 0) HIPCHK(blas_axpby(dtype(), V(k + 1), 1.0 / hn, V(k + 1), 0.0, nullptr, in->n, s));
        for (int i = 0; i < k; ++i) {  // earlier rotations
          const double a = H[i * m + k], c = H[(i + 1) * m + k];
          H[i * m + k] = cs[i] * a + sn[i] * c;
          H[(i + 1) * m + k] = -sn[i] * a + cs[i] * c;
        }
        const double a = H[k * m + k], c = H[(k + 1) * m + k], r = std::hypot(a, c);
        cs[k] = r > 0 ? a / r : 1.0;
        sn[k] = r > 0 ? c / r : 0.0;
        H[k * m + k] = r;
        H[(k + 1) * m + k] = 0.0;
        g[k + 1] = -sn[k] * g[k];
        g[k] = cs[k] * g[k];
        if (!std::isfinite(g[k + 1])) return fail(SEM_ERR_NONFINITE, "non-finite GMRES residual");
        if (std::fabs(g[k + 1]) <= gmres_rtol * bnorm || hn == 0.0) {
          ++k, ++total;
          break;
        }
      }
      // x += V y with H y = g (upper triangular k x k)
      for (int i = k - 1; i >= 0; --i) {
        double t = g[i];
        for (int j = i + 1; j < k; ++j) t -= H[i * m + j] * y[j];
        y[i] = t / H[i * m + i];
      }
      HIPCHK(hipMemcpyAsync(dvec, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
      HIPCHK(blas_combine(dtype(), x, 1.0, V(0), in->n, k, dvec, 1.0, in->n, s));
      res = std::fabs(g[k]);
      if (res <= gmres_rtol * bnorm) break;
      if (total >= gmres_maxit)
        return fail(SEM_ERR_NOCONV, "GMRES stopped at relative residual %.3g after %d iterations", res / bnorm, total);
    }
    st.gmres_iters += total;
    st.max_rel_residual = std::max(st.max_rel_residual, res / bnorm);
    return SEM_OK;
  }

  // one Crank-Nicolson step on u (device state, overwritten), Newton from the predictor u + dt F(u)
  int cn_step(void* u, char* basis) {
    using I = Integrator;
    const Coef one{1, 0}, zero{0, 0};
    void* Bv = in->b(I::S1);  // u + dt/2 F(u)
    void* v = in->b(I::S2);   // Newton iterate
    void* R = in->b(I::ACC);  // residual
    void* d = in->b(I::T1);   // correction
    Epi ep{Bv, u, one, {0, 0.5}, v, u, one, {0, 1.0}};
    HIPCHK(in->os->apply(OP_RHS, u, nullptr, one, ep, s));
    double bn = 0;
    if (int rc = norm(Bv, &bn)) return rc;
    const double scale = bn > 0 ? bn : 1.0;
    double rn = 0;
    for (int it = 0;; ++it) {
      ep = Epi{R, v, one, {0, -0.5}, nullptr, Bv, zero, zero, {-1, 0}, zero};  // R = v - B - dt/2 F(v)
      HIPCHK(in->os->apply(OP_RHS, v, nullptr, one, ep, s));
      if (int rc = norm(R, &rn)) return rc;
      if (!std::isfinite(rn)) return fail(SEM_ERR_NONFINITE, "non-finite Newton residual (dt too large?)");
      if (rn <= newton_rtol * scale) break;
      if (it >= newton_maxit)
        return fail(SEM_ERR_NOCONV, "Newton stopped at relative residual %.3g after %d iterations", rn / scale, it);
      ++st.newton_iters;
      if (int rc = gmres(OP_JAC, v, -0.5, R, d, basis)) return rc;
      HIPCHK(blas_axpby(dtype(), v, 1.0, v, -1.0, d, in->n, s));
    }
    st.max_rel_residual = std::max(st.max_rel_residual, rn / scale);
    HIPCHK(hipMemcpyAsync(u, v, bytes(), hipMemcpyDeviceToDevice, s));
    return SEM_OK;
  }

  int forward(void* u, int32_t nsteps, int32_t K, void* ckpt, char* work) {
    using I = Integrator;
    void* x = in->b(I::STATE);
    HIPCHK(hipMemcpyAsync(x, u, bytes(), hipMemcpyDeviceToDevice, s));
    for (int32_t k = 0; k < nsteps; ++k) {
      if (ckpt && k % K == 0)
        HIPCHK(hipMemcpyAsync(static_cast<char*>(ckpt) + (size_t)(k / K) * bytes(), x, bytes(),
                              hipMemcpyDeviceToDevice, s));
      if (int rc = cn_step(x, work)) return rc;
    }
    HIPCHK(hipMemcpyAsync(u, x, bytes(), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return SEM_OK;
  }

  // work: K + 1 states of the segment, then the GMRES basis
  int adjoint(const void* ckpt, int32_t nsteps, int32_t K, void* lam, char* work) {
    using I = Integrator;
    const Coef one{1, 0}, zero{0, 0};
    const size_t B = bytes();
    char* basis = work + (size_t)(K + 1) * B;
    void* L = in->b(I::LAMB);
    void* mu = in->b(I::T2);
    HIPCHK(hipMemcpyAsync(L, lam, B, hipMemcpyDeviceToDevice, s));
    for (int sg = nsteps / K - 1; sg >= 0; --sg) {
      HIPCHK(hipMemcpyAsync(work, static_cast<const char*>(ckpt) + (size_t)sg * B, B, hipMemcpyDeviceToDevice, s));
      for (int k = 1; k <= K; ++k) {
        HIPCHK(hipMemcpyAsync(work + (size_t)k * B, work + (size_t)(k - 1) * B, B, hipMemcpyDeviceToDevice, s));
        if (int rc = cn_step(work + (size_t)k * B, basis)) return rc;
      }
      for (int k = K - 1; k >= 0; --k) {
        // (I - dt/2 J(u_{k+1}))^T mu = lam;  lam = mu + dt/2 J(u_k)^T mu
        if (int rc = gmres(OP_JACT, work + (size_t)(k + 1) * B, -0.5, L, mu, basis)) return rc;
        Epi ep{L, mu, one, {0, 0.5}, nullptr, nullptr, zero, zero};
        HIPCHK(in->os->apply(OP_JACT, work + (size_t)k * B, mu, one, ep, s));
      }
    }
    HIPCHK(hipMemcpyAsync(lam, L, B, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return SEM_OK;
  }
};

// LMVM for the optimal initial condition: device vectors in one work buffer, host scalars.
struct Lmvm {
  Integrator* in = nullptr;
  Implicit* im = nullptr;  // set for SEM_CN
  int scheme = SEM_RK4;
  hipStream_t s = nullptr;
  double* partial = nullptr;
  double* dvec = nullptr;
  int32_t nsteps = 0, K = 1;
  const void* target = nullptr;
  char* ckpt = nullptr;   // nsteps / K states
  char* adjw = nullptr;   // adjoint work
  char* resid = nullptr;  // u(T) - u*
  int evals = 0;

  int dtype() const { return in->os->dtype; }
  size_t bytes() const { return (size_t)in->n * in->ts; }

  int dot(const void* a, const void* b, double* r) {
    HIPCHK(blas_multidot(dtype(), a, in->n, 1, b, in->n, partial, dvec, s));
    HIPCHK(hipMemcpyAsync(r, dvec, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return SEM_OK;
  }
  hipError_t axpby(void* z, double a, const void* x, double b, const void* y) {
    return blas_axpby(dtype(), z, a, x, b, y, in->n, s);
  }

  // Phi(x) and its gradient g (discrete adjoint of the scheme)
  int evaluate(const void* x, void* g, double* f) {
    ++evals;
    HIPCHK(hipMemcpyAsync(resid, x, bytes(), hipMemcpyDeviceToDevice, s));
    int rc = im ? im->forward(resid, nsteps, K, ckpt, adjw) : in->forward(scheme, resid, nsteps, K, ckpt, s);
    if (rc) return rc;
    HIPCHK(axpby(resid, 1.0, resid, -1.0, target));
    double rr = 0;
    if ((rc = dot(resid, resid, &rr))) return rc;
    *f = 0.5 * rr;
    if (!std::isfinite(*f)) return fail(SEM_ERR_NONFINITE, "non-finite objective (dt too large?)");
    HIPCHK(hipMemcpyAsync(g, resid, bytes(), hipMemcpyDeviceToDevice, s));
    rc = im ? im->adjoint(ckpt, nsteps, K, g, adjw) : in->adjoint(scheme, ckpt, nsteps, K, g, adjw, s);
    return rc;
  }

  int run(void* u0, char* vecs, int memory, const sem_lmvm_opts& o, double* history, sem_lmvm_stats& st) {
    const size_t B = bytes();
    char* x = vecs;
    char* g = vecs + B;
    char* d = vecs + 2 * B;
    char* xt = vecs + 3 * B;
    char* gt = vecs + 4 * B;
    char* tmp = vecs + 5 * B;
    char* S = vecs + 6 * B;                        // memory pairs: S_i, then Y_i
    char* Y = S + (size_t)memory * B;
    std::vector<double> rho(memory), alpha(memory);
    int npairs = 0, newest = -1;
    HIPCHK(hipMemcpyAsync(x, u0, B, hipMemcpyDeviceToDevice, s));
    double f = 0, gn = 0;
    int rc = evaluate(x, g, &f);
    if (rc) return rc;
    st.f0 = f;
    if (history) history[0] = f;
    st.reason = 0;
    int k = 0;
    for (;; ++k) {
      double gg = 0;
      if ((rc = dot(g, g, &gg))) return rc;
      gn = std::sqrt(gg);
      if (gn <= o.gatol) { st.reason = 1; break; }
      if (gn <= o.grtol * std::fabs(f)) { st.reason = 2; break; }
      if (k >= o.max_iters) { st.reason = 3; break; }
      // direction: two-loop recursion (or steepest descent when no pair is stored)
      double stp0 = 1.0;
      HIPCHK(hipMemcpyAsync(d, g, B, hipMemcpyDeviceToDevice, s));
      if (npairs > 0) {
        for (int c = 0, i = newest; c < npairs; ++c, i = (i - 1 + memory) % memory) {
          double sq = 0;
          if ((rc = dot(S + (size_t)i * B, d, &sq))) return rc;
          alpha[i] = rho[i] * sq;
          HIPCHK(axpby(d, 1.0, d, -alpha[i], Y + (size_t)i * B));
        }
        double sy = 0, yy = 0;
        if ((rc = dot(S + (size_t)newest * B, Y + (size_t)newest * B, &sy)) ||
            (rc = dot(Y + (size_t)newest * B, Y + (size_t)newest * B, &yy)))
          return rc;
        HIPCHK(axpby(d, sy / yy, d, 0.0, nullptr));
        const int oldest = (newest - npairs + 1 + memory) % memory;
        for (int c = 0, i = oldest; c < npairs; ++c, i = (i + 1) % memory) {
          double yr = 0;
          if ((rc = dot(Y + (size_t)i * B, d, &yr))) return rc;
          HIPCHK(axpby(d, 1.0, d, alpha[i] - rho[i] * yr, S + (size_t)i * B));
        }
      }
      HIPCHK(axpby(d, -1.0, d, 0.0, nullptr));
      double gd = 0;
      if ((rc = dot(g, d, &gd))) return rc;
      if (npairs == 0 || !(gd < 0)) {  // steepest descent, first step of unit length
        if (npairs > 0) HIPCHK(axpby(d, -1.0, g, 0.0, nullptr));
        npairs = 0, newest = -1;
        gd = -gg;
        stp0 = 1.0 / gn;
      }
      // More-Thuente line search on phi(t) = Phi(x + t d)
      sem_line_search ls{};
      ls.ftol = o.ftol, ls.gtol = o.gtol, ls.xtol = o.xtol, ls.stpmin = 0.0, ls.stpmax = 1e10;
      int32_t task = SEM_LS_START;
      double stp = stp0, last = -1.0, ft = f;
      sem_line_search_step(&ls, &task, &stp, f, gd);
      int n_eval = 0;
      while (task == SEM_LS_FG && n_eval < o.max_evals) {
        HIPCHK(axpby(xt, 1.0, x, stp, d));
        if ((rc = evaluate(xt, gt, &ft))) return rc;
        double gtd = 0;
        if ((rc = dot(gt, d, &gtd))) return rc;
        last = stp;
        ++n_eval;
        sem_line_search_step(&ls, &task, &stp, ft, gtd);
      }
      if (task != SEM_LS_CONVERGED && task != SEM_LS_WARNING) { st.reason = -1; break; }
      if (stp != last) {  // the line search settled on its best earlier step
        HIPCHK(axpby(xt, 1.0, x, stp, d));
        if ((rc = evaluate(xt, gt, &ft))) return rc;
      }
      if (!(ft < f)) { st.reason = -1; break; }
      // new pair s = xt - x, y = gt - g (into scratch: the direction is spent), kept if s.y > 0
      HIPCHK(axpby(d, 1.0, xt, -1.0, x));
      HIPCHK(axpby(tmp, 1.0, gt, -1.0, g));
      double sy = 0;
      if ((rc = dot(d, tmp, &sy))) return rc;
      if (sy > 0) {
        const int slot = (newest + 1) % memory;
        HIPCHK(hipMemcpyAsync(S + (size_t)slot * B, d, B, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(Y + (size_t)slot * B, tmp, B, hipMemcpyDeviceToDevice, s));
        rho[slot] = 1.0 / sy;
        newest = slot;
        npairs = std::min(npairs + 1, memory);
      }
      std::swap(x, xt);
      std::swap(g, gt);
      f = ft;
      if (history) history[k + 1] = f;
    }
    st.iters = k;
    st.evals = evals;
    st.f = f;
    st.gnorm = gn;
    HIPCHK(hipMemcpyAsync(u0, x, B, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return SEM_OK;
  }
};

}  // namespace

// Scratch of the allocation-free RK4 forward (sem_rk4_forward_noalloc): its three stage states and
// the stage accumulator.  Each device holds its own copy of the array for the life of the process;
// host code reaches it only through the address that hipGetSymbolAddress returns for the current
// device (the array's name is a host-side stand-in, not a device address).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// This device's scratch address, resolved once per device with that device current.
int scratch_address(void** out) {
  *out = nullptr;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES)
    return fail(SEM_ERR_UNSUPPORTED, "device %d beyond the %d devices the scratch table covers", dev,
                SCRATCH_MAX_DEVICES);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(SEM_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SEM_OK;
}
}  // namespace

struct sem_ctx_s {
  sem_desc d{};
  hipStream_t stream = nullptr;
  void* scratch = nullptr;     // this device's allocation-free scratch (scratch_address)
  hipEvent_t chain = nullptr;  // orders work across a change of stream (chain_streams)
  OpSet os;
  Integrator integ;
  int64_t ndof = 0, nodes = 0;
  bool check_finite = false;
  DevBuf flag;
  DevBuf nk;  // Newton-Krylov reductions: partial sums, then dot results / combination weights
};

struct sem_batch_s {
  std::vector<sem_desc> descs;
  std::vector<double> dts;
  std::vector<int64_t> offsets;
  hipStream_t stream = nullptr;
  hipEvent_t chain = nullptr;
  OpSet os;
  Integrator integ;
};

namespace {
// A handle's internal buffers and graphs are shared by all of its calls, so its work must form
// one ordered chain even when the caller moves it to another stream: the new stream first waits
// for everything already enqueued on the old one.  Synchronising the current stream then also
// waits for the work of every stream the handle used before.
int chain_streams(hipStream_t from, hipStream_t to, hipEvent_t& ev) {
  if (from == to) return SEM_OK;
  if (!ev) HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  HIPCHK(hipEventRecord(ev, from));
  HIPCHK(hipStreamWaitEvent(to, ev, 0));
  return SEM_OK;
}
}  // namespace

extern "C" {

const char* sem_last_error(void) { return g_err.c_str(); }

int sem_setup(const sem_desc* desc, void* stream, sem_ctx* out) {
  if (!out) return fail(SEM_ERR_ARG, "null output pointer");
  *out = nullptr;
  int rc = validate_desc(desc);
  if (rc) return rc;
  sem_ctx c = new (std::nothrow) sem_ctx_s();
  if (!c) return fail(SEM_ERR_NOMEM, "host allocation failed");
  c->d = *desc;
  c->stream = static_cast<hipStream_t>(stream);
  if ((rc = build_opset(c->os, desc, 1, true))) {
    delete c;
    return rc;
  }
  if ((rc = scratch_address(&c->scratch))) {
    delete c;
    return rc;
  }
  c->nodes = c->os.hp[0].nodes;
  c->ndof = c->nodes * desc->dim;
  c->integ.os = &c->os;
  c->integ.n = c->ndof * desc->batch;
  c->integ.ts = c->os.ts;
  if ((rc = c->flag.alloc(sizeof(int))) || (rc = c->nk.alloc(blas_partial_bytes() + 3 * sizeof(double) * blas_max_vectors()))) {
    delete c;
    return rc;
  }
  g_err.clear();
  *out = c;
  return SEM_OK;
}

int sem_destroy(sem_ctx c) {
  if (!c) return fail(SEM_ERR_ARG, "null context");
  // the current stream carries the handle's whole chain of work (chain_streams)
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  if (c->chain) (void)hipEventDestroy(c->chain);
  delete c;
  return SEM_OK;
}

int sem_set_stream(sem_ctx c, void* stream) {
  if (!c) return fail(SEM_ERR_ARG, "null context");
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if (int rc = chain_streams(c->stream, s, c->chain)) return rc;
  c->stream = s;
  return SEM_OK;
}

int sem_query(sem_ctx c, int64_t* ndof, int64_t* nodes) {
  if (!c) return fail(SEM_ERR_ARG, "null context");
  if (ndof) *ndof = c->ndof;
  if (nodes) *nodes = c->nodes;
  return SEM_OK;
}

int sem_query_path(sem_ctx c, int32_t* path) {
  if (!c || !path) return fail(SEM_ERR_ARG, "null argument");
  *path = c->os.fast;
  return SEM_OK;
}

int sem_node_coords(sem_ctx c, int32_t dir, double* x) {
  if (!c || !x) return fail(SEM_ERR_ARG, "null argument");
  if (dir < 0 || dir >= c->d.dim) return fail(SEM_ERR_ARG, "dir %d outside 0..%d", dir, c->d.dim - 1);
  double xi[MAXP], w[MAXP], D[MAXP * MAXP];
  const int N = c->d.order;
  gll_tables(N, xi, w, D);
  const double h = c->d.length[dir] / c->d.elems[dir];
  const int64_t n = (int64_t)c->d.elems[dir] * N;
  for (int64_t g = 0; g < n; ++g) x[g] = (double)(g / N) * h + 0.5 * (xi[g % N] + 1.0) * h;
  return SEM_OK;
}

static int apply_entry(sem_ctx c, int op, const void* u, const void* v, void* out) {
  if (!c) return fail(SEM_ERR_ARG, "null context");
  if (!u || !out || (op != OP_RHS && !v)) return fail(SEM_ERR_ARG, "null field pointer");
  if (out == u || (v && out == v)) return fail(SEM_ERR_ARG, "output aliases an input");
  Epi ep{out, nullptr, {0, 0}, {1, 0}, nullptr, nullptr, {0, 0}, {0, 0}};
  HIPCHK(c->os.apply(op, u, v, {1, 0}, ep, c->stream));
  return SEM_OK;
}

int sem_mass(sem_ctx c, void* m) {
  if (!c || !m) return fail(SEM_ERR_ARG, "null argument");
  for (const auto& hp : c->os.hp) HIPCHK(launch_mass(hp, m, c->d.dtype, c->stream));
  return SEM_OK;
}

int sem_rhs(sem_ctx c, const void* u, void* f) { return apply_entry(c, OP_RHS, u, nullptr, f); }
int sem_jac_vec(sem_ctx c, const void* u, const void* v, void* jv) { return apply_entry(c, OP_JAC, u, v, jv); }
int sem_jact_vec(sem_ctx c, const void* u, const void* w, void* jtw) { return apply_entry(c, OP_JACT, u, w, jtw); }

static int check_scheme(int32_t scheme) {
  if (scheme != SEM_RK4 && scheme != SEM_RK3) return fail(SEM_ERR_ARG, "unknown time-integration scheme %d", scheme);
  return SEM_OK;
}

static int check_steps(double dt, int32_t nsteps, int32_t K, bool need_k) {
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(SEM_ERR_ARG, "dt must be finite and > 0");
  if (nsteps < 0) return fail(SEM_ERR_ARG, "nsteps %d < 0", nsteps);
  if (need_k && (K < 1 || (nsteps % K) != 0))
    return fail(SEM_ERR_ARG, "ckpt_every %d must be >= 1 and divide nsteps %d", K, nsteps);
  return SEM_OK;
}

int sem_probe_fp64_rates(void* stream, int32_t iters, double* tflops) {
  if (!tflops || iters < 1) return fail(SEM_ERR_ARG, "sem_probe_fp64_rates: null result or iters < 1");
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevBuf out;
  if (int rc = out.alloc(fp64_probe_values() * sizeof(double))) return rc;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const double waves = (double)fp64_probe_values() / 64;
  const double fm = waves * iters * fp64_probe_mfma_flops_per_wave_iter();
  const double fv = waves * iters * fp64_probe_valu_flops_per_wave_iter();
  int rc = SEM_OK;
  float ms[3] = {0, 0, 0};
  for (int mode = 0; mode < 3 && rc == SEM_OK; ++mode) {
    hipError_t he = launch_fp64_probe(mode, static_cast<double*>(out.p), iters, s);  // warm-up
    if (he == hipSuccess) he = hipEventRecord(e0, s);
    if (he == hipSuccess) he = launch_fp64_probe(mode, static_cast<double*>(out.p), iters, s);
    if (he == hipSuccess) he = hipEventRecord(e1, s);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    if (he == hipSuccess) he = hipEventElapsedTime(&ms[mode], e0, e1);
    if (he != hipSuccess) rc = fail(SEM_ERR_HIP, "sem_probe_fp64_rates: %s", hipGetErrorString(he));
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  tflops[0] = fm / (ms[0] * 1e-3) / 1e12;
  tflops[1] = fv / (ms[1] * 1e-3) / 1e12;
  tflops[2] = fm / (ms[2] * 1e-3) / 1e12;
  tflops[3] = fv / (ms[2] * 1e-3) / 1e12;
  return SEM_OK;
}

int sem_set_check_finite(sem_ctx c, int32_t on) {
  if (!c) return fail(SEM_ERR_ARG, "null context");
  c->check_finite = on != 0;
  return SEM_OK;
}

// With sem_set_check_finite on: SEM_ERR_NONFINITE if the final state holds a non-finite value.
static int check_final_state(sem_ctx c, const void* u, double dt) {
  if (!c->check_finite) return SEM_OK;
  HIPCHK(hipMemsetAsync(c->flag.p, 0, sizeof(int), c->stream));
  const int64_t n = c->integ.n;
  if (c->d.dtype == SEM_F64)
    hipLaunchKernelGGL(finite_kernel<double>, dim3(1024), dim3(256), 0, c->stream, static_cast<const double*>(u), n,
                       static_cast<int*>(c->flag.p));
  else
    hipLaunchKernelGGL(finite_kernel<float>, dim3(1024), dim3(256), 0, c->stream, static_cast<const float*>(u), n,
                       static_cast<int*>(c->flag.p));
  HIPCHK(hipGetLastError());
  int h = 0;
  HIPCHK(hipMemcpyAsync(&h, c->flag.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (h) return fail(SEM_ERR_NONFINITE, "trajectory produced a non-finite value (dt = %g too large?)", dt);
  return SEM_OK;
}

int sem_rk_forward(sem_ctx c, int32_t scheme, void* u, double dt, int32_t nsteps, int32_t K, void* ckpt) {
  if (!c) return fail(SEM_ERR_ARG, "null context");
  if (!u) return fail(SEM_ERR_ARG, "null u");
  int rc = check_scheme(scheme);
  if (rc) return rc;
  if ((rc = check_steps(dt, nsteps, K, ckpt != nullptr))) return rc;
  if (ckpt && ckpt == u) return fail(SEM_ERR_ARG, "ckpt aliases u");
  if ((rc = c->integ.prepare(scheme))) return rc;
  if ((rc = c->integ.set_dt(dt, false, c->stream))) return rc;
  if ((rc = c->integ.forward(scheme, u, nsteps, K, ckpt, c->stream))) return rc;
  return check_final_state(c, u, dt);
}

int sem_rk_stages_bytes(sem_ctx c, int32_t scheme, int32_t nsteps, int64_t* bytes) {
  if (!c || !bytes) return fail(SEM_ERR_ARG, "null argument");
  int rc = check_scheme(scheme);
  if (rc) return rc;
  if (nsteps < 0) return fail(SEM_ERR_ARG, "nsteps %d < 0", nsteps);
  *bytes = (int64_t)nsteps * Integrator::stage_states(scheme) * c->integ.n * (int64_t)c->os.ts;
  return SEM_OK;
}

int sem_rk_forward_stored(sem_ctx c, int32_t scheme, void* u, double dt, int32_t nsteps, void* stages) {
  if (!c) return fail(SEM_ERR_ARG, "null context");
  if (!u || (!stages && nsteps > 0)) return fail(SEM_ERR_ARG, "null pointer");
  if (stages == u) return fail(SEM_ERR_ARG, "stages alias u");
  int rc = check_scheme(scheme);
  if (rc) return rc;
  if ((rc = check_steps(dt, nsteps, 1, false))) return rc;
  if ((rc = c->integ.alloc_buffers())) return rc;
  if ((rc = c->integ.set_dt(dt, false, c->stream))) return rc;
  if ((rc = c->integ.forward_stored(scheme, u, nsteps, stages, c->stream))) return rc;
  return check_final_state(c, u, dt);
}

int sem_rk_adjoint_stored(sem_ctx c, int32_t scheme, const void* stages, double dt, int32_t nsteps, void* lam) {
  if (!c) return fail(SEM_ERR_ARG, "null context");
  if (!lam || (!stages && nsteps > 0)) return fail(SEM_ERR_ARG, "null pointer");
  if (stages == lam) return fail(SEM_ERR_ARG, "stages alias lam");
  int rc = check_scheme(scheme);
  if (rc) return rc;
  if ((rc = check_steps(dt, nsteps, 1, false))) return rc;
  if ((rc = c->integ.alloc_buffers())) return rc;
  if ((rc = c->integ.set_dt(dt, false, c->stream))) return rc;
  return c->integ.adjoint_stored(scheme, stages, nsteps, lam, c->stream);
}

int sem_workspace_bytes(sem_ctx c, int32_t K, int64_t* bytes) {
  if (!c || !bytes) return fail(SEM_ERR_ARG, "null argument");
  if (K < 1) return fail(SEM_ERR_ARG, "ckpt_every %d < 1", K);
  *bytes = c->integ.work_states(K) * c->integ.n * (int64_t)c->os.ts;
  return SEM_OK;
}

int sem_set_adjoint_stages(sem_ctx c, int32_t mode) {
  if (!c) return fail(SEM_ERR_ARG, "null context");
  if (mode != SEM_ADJ_AUTO && mode != SEM_ADJ_STORE && mode != SEM_ADJ_RECOMPUTE)
    return fail(SEM_ERR_ARG, "adjoint stage mode %d", mode);
  c->integ.adj_mode = mode;
  return SEM_OK;
}

int sem_rk4_forward(sem_ctx c, void* u, double dt, int32_t nsteps, int32_t K, void* ckpt) {
  return sem_rk_forward(c, SEM_RK4, u, dt, nsteps, K, ckpt);
}

int sem_rk4_forward_noalloc(sem_ctx c, void* u, double dt, int32_t nsteps, int32_t K, void* ckpt) {
  if (!c) return fail(SEM_ERR_ARG, "null context");
  if (!u) return fail(SEM_ERR_ARG, "null u");
  int rc = check_steps(dt, nsteps, K, ckpt != nullptr);
  if (rc) return rc;
  if (ckpt && ckpt == u) return fail(SEM_ERR_ARG, "ckpt aliases u");
  // three stage states and the accumulator, each rounded up to the array's 256-byte alignment
  const int64_t bytes = c->integ.n * (int64_t)c->os.ts;
  const int64_t slot = (bytes + 255) / 256 * 256;
  if (4 * slot > (int64_t)NOALLOC_SCRATCH_BYTES)
    return fail(SEM_ERR_ARG,
                "state of %lld bytes: the allocation-free RK4 forward keeps 4 states (%lld bytes) in a scratch of "
                "%zu bytes; use sem_rk4_forward",
                (long long)bytes, (long long)(4 * slot), NOALLOC_SCRATCH_BYTES);
  if (!c->scratch) return fail(SEM_ERR_HIP, "scratch address not resolved");
  char* sp = static_cast<char*>(c->scratch);
  void* const st[3] = {sp, sp + slot, sp + 2 * slot};
  void* const acc = sp + 3 * slot;
  if ((rc = c->integ.set_dt(dt, false, c->stream))) return rc;
  for (int32_t k = 0; k < nsteps; ++k) {
    if (ckpt && k % K == 0)
      HIPCHK(hipMemcpyAsync(static_cast<char*>(ckpt) + (size_t)(k / K) * bytes, u, bytes, hipMemcpyDeviceToDevice,
                            c->stream));
    // the captured step's launches and coefficients, the new state written over u
    HIPCHK(c->integ.enqueue_step_stages(c->stream, SEM_RK4, u, st, u, acc));
  }
  return SEM_OK;
}

int sem_rk_adjoint(sem_ctx c, int32_t scheme, const void* ckpt, double dt, int32_t nsteps, int32_t K, void* lam,
                   void* work) {
  if (!c) return fail(SEM_ERR_ARG, "null context");
  // with no steps there are no checkpoints to read (an empty array may come as NULL)
  if ((!ckpt && nsteps > 0) || !lam || !work) return fail(SEM_ERR_ARG, "null pointer");
  int rc = check_scheme(scheme);
  if (rc) return rc;
  if ((rc = check_steps(dt, nsteps, K, true))) return rc;
  if (lam == ckpt || lam == work || work == ckpt) return fail(SEM_ERR_ARG, "aliased buffers");
  if ((rc = c->integ.prepare(scheme))) return rc;
  if ((rc = c->integ.set_dt(dt, false, c->stream))) return rc;
  return c->integ.adjoint(scheme, ckpt, nsteps, K, lam, work, c->stream);
}

int sem_rk4_adjoint(sem_ctx c, const void* ckpt, double dt, int32_t nsteps, int32_t K, void* lam, void* work) {
  return sem_rk_adjoint(c, SEM_RK4, ckpt, dt, nsteps, K, lam, work);
}

static int cn_setup(sem_ctx c, const sem_nk_opts* opts, Implicit& im) {
  im.in = &c->integ;
  im.partial = static_cast<double*>(c->nk.p);
  im.dvec = reinterpret_cast<double*>(static_cast<char*>(c->nk.p) + blas_partial_bytes());
  im.s = c->stream;
  if (int rc = im.configure(opts)) return rc;
  return c->integ.alloc_buffers();
}

int sem_cn_workspace_bytes(sem_ctx c, int32_t K, const sem_nk_opts* opts, int64_t* bytes) {
  if (!c || !bytes) return fail(SEM_ERR_ARG, "null argument");
  if (K < 1) return fail(SEM_ERR_ARG, "ckpt_every %d < 1", K);
  const int restart = (opts && opts->gmres_restart > 0) ? opts->gmres_restart : 30;
  *bytes = (int64_t)(K + 1 + restart + 2) * c->integ.n * (int64_t)c->os.ts;
  return SEM_OK;
}

int sem_cn_forward(sem_ctx c, void* u, double dt, int32_t nsteps, int32_t K, void* ckpt, const sem_nk_opts* opts,
                   void* work, sem_nk_stats* stats) {
  if (!c) return fail(SEM_ERR_ARG, "null context");
  if (!u || !work) return fail(SEM_ERR_ARG, "null pointer");
  if ((ckpt && (ckpt == u || ckpt == work)) || work == u) return fail(SEM_ERR_ARG, "aliased buffers");
  int rc = check_steps(dt, nsteps, K, ckpt != nullptr);
  if (rc) return rc;
  Implicit im;
  if ((rc = cn_setup(c, opts, im))) return rc;
  if ((rc = c->integ.set_dt(dt, false, c->stream))) return rc;
  rc = im.forward(u, nsteps, K, ckpt, static_cast<char*>(work));
  if (stats) *stats = im.st;
  return rc;
}

int sem_cn_adjoint(sem_ctx c, const void* ckpt, double dt, int32_t nsteps, int32_t K, void* lam,
                   const sem_nk_opts* opts, void* work, sem_nk_stats* stats) {
  if (!c) return fail(SEM_ERR_ARG, "null context");
  if ((!ckpt && nsteps > 0) || !lam || !work) return fail(SEM_ERR_ARG, "null pointer");
  if (lam == ckpt || lam == work || work == ckpt) return fail(SEM_ERR_ARG, "aliased buffers");
  int rc = check_steps(dt, nsteps, K, true);
  if (rc) return rc;
  Implicit im;
  if ((rc = cn_setup(c, opts, im))) return rc;
  if ((rc = c->integ.set_dt(dt, false, c->stream))) return rc;
  rc = im.adjoint(ckpt, nsteps, K, lam, static_cast<char*>(work));
  if (stats) *stats = im.st;
  return rc;
}

static sem_lmvm_opts lmvm_defaults(const sem_lmvm_opts* o) {
  sem_lmvm_opts r{};
  r.max_iters = (o && o->max_iters > 0) ? o->max_iters : 50;
  r.memory = (o && o->memory > 0) ? o->memory : 5;
  r.gatol = (o && o->gatol > 0) ? o->gatol : 1e-10;
  r.grtol = (o && o->grtol > 0) ? o->grtol : 1e-10;
  r.ftol = (o && o->ftol > 0) ? o->ftol : 1e-4;
  r.gtol = (o && o->gtol > 0) ? o->gtol : 0.9;
  r.xtol = (o && o->xtol > 0) ? o->xtol : 1e-10;
  r.max_evals = (o && o->max_evals > 0) ? o->max_evals : 30;
  return r;
}

// states of the LMVM work buffer: 6 iterate/scratch vectors, 2 m pairs, the residual, the checkpoints and
// the adjoint work of the scheme
static int64_t lmvm_states(const Integrator& in, int32_t scheme, int32_t nsteps, int32_t K, const sem_lmvm_opts& o) {
  const int64_t adj = scheme == SEM_CN ? (int64_t)K + 1 + 30 + 2 : in.work_states(K);
  return 6 + 2 * (int64_t)o.memory + 1 + nsteps / K + adj;
}

int sem_lmvm_workspace_bytes(sem_ctx c, int32_t scheme, int32_t nsteps, int32_t K, const sem_lmvm_opts* opts,
                             int64_t* bytes) {
  if (!c || !bytes) return fail(SEM_ERR_ARG, "null argument");
  if (scheme != SEM_RK4 && scheme != SEM_RK3 && scheme != SEM_CN) return fail(SEM_ERR_ARG, "unknown scheme %d", scheme);
  if (int rc = check_steps(1.0, nsteps, K, true)) return rc;
  const sem_lmvm_opts o = lmvm_defaults(opts);
  *bytes = lmvm_states(c->integ, scheme, nsteps, K, o) * c->integ.n * (int64_t)c->os.ts;
  return SEM_OK;
}

int sem_lmvm_initial_condition(sem_ctx c, int32_t scheme, void* u0, const void* target, double dt, int32_t nsteps,
                               int32_t K, const sem_lmvm_opts* opts, void* work, double* history,
                               sem_lmvm_stats* stats) {
  if (!c) return fail(SEM_ERR_ARG, "null context");
  if (!u0 || !target || !work) return fail(SEM_ERR_ARG, "null pointer");
  if (u0 == target || work == u0 || work == target) return fail(SEM_ERR_ARG, "aliased buffers");
  if (scheme != SEM_RK4 && scheme != SEM_RK3 && scheme != SEM_CN) return fail(SEM_ERR_ARG, "unknown scheme %d", scheme);
  int rc = check_steps(dt, nsteps, K, true);
  if (rc) return rc;
  if (nsteps < 1) return fail(SEM_ERR_ARG, "nsteps must be >= 1");
  const sem_lmvm_opts o = lmvm_defaults(opts);
  if (o.memory > 20) return fail(SEM_ERR_ARG, "memory %d > 20", o.memory);
  Implicit im;
  Lmvm L;
  L.in = &c->integ;
  L.scheme = scheme;
  L.s = c->stream;
  L.partial = static_cast<double*>(c->nk.p);
  L.dvec = reinterpret_cast<double*>(static_cast<char*>(c->nk.p) + blas_partial_bytes());
  if (scheme == SEM_CN) {
    if ((rc = cn_setup(c, nullptr, im))) return rc;
    L.im = &im;
  } else if ((rc = c->integ.prepare(scheme))) {
    return rc;
  }
  if ((rc = c->integ.set_dt(dt, false, c->stream))) return rc;
  L.nsteps = nsteps, L.K = K, L.target = target;
  const size_t B = (size_t)c->integ.n * c->os.ts;
  char* w = static_cast<char*>(work);
  char* vecs = w;
  L.resid = w + (size_t)(6 + 2 * o.memory) * B;
  L.ckpt = L.resid + B;
  L.adjw = L.ckpt + (size_t)(nsteps / K) * B;
  sem_lmvm_stats st{};
  rc = L.run(u0, vecs, o.memory, o, history, st);
  if (stats) *stats = st;
  return rc;
}

int sem_revolve_plan(int32_t nsteps, int32_t snaps, int64_t* nactions, int64_t* actions, int64_t capacity,
                     int64_t* advances) {
  if (!nactions) return fail(SEM_ERR_ARG, "null nactions");
  if (nsteps < 1 || snaps < 1) return fail(SEM_ERR_ARG, "need nsteps >= 1 and snaps >= 1 (got %d, %d)", nsteps, snaps);
  std::vector<RevolveAct> acts;
  const int64_t adv = revolve_plan(nsteps, snaps, acts);
  *nactions = (int64_t)acts.size();
  if (advances) *advances = adv;
  if (!actions) return SEM_OK;
  if (capacity < (int64_t)acts.size())
    return fail(SEM_ERR_ARG, "action buffer holds %lld actions, the schedule has %lld", (long long)capacity,
                (long long)acts.size());
  for (size_t k = 0; k < acts.size(); ++k) {
    actions[2 * k] = acts[k].kind;
    actions[2 * k + 1] = acts[k].arg;
  }
  return SEM_OK;
}

int sem_revolve_workspace_bytes(sem_ctx c, int32_t snaps, int64_t* bytes) {
  if (!c || !bytes) return fail(SEM_ERR_ARG, "null argument");
  if (snaps < 1) return fail(SEM_ERR_ARG, "snaps %d < 1", snaps);
  *bytes = (int64_t)snaps * c->integ.n * (int64_t)c->os.ts;
  return SEM_OK;
}

int sem_rk_forward_revolve(sem_ctx c, int32_t scheme, void* u, double dt, int32_t nsteps, int32_t snaps, void* ckpt) {
  if (!c) return fail(SEM_ERR_ARG, "null context");
  if (!u || !ckpt) return fail(SEM_ERR_ARG, "null pointer");
  if (ckpt == u) return fail(SEM_ERR_ARG, "ckpt aliases u");
  int rc = check_scheme(scheme);
  if (rc) return rc;
  if ((rc = check_steps(dt, nsteps, 1, false))) return rc;
  if (nsteps < 1 || snaps < 1) return fail(SEM_ERR_ARG, "need nsteps >= 1 and snaps >= 1 (got %d, %d)", nsteps, snaps);
  std::vector<RevolveAct> acts;
  revolve_plan(nsteps, snaps, acts);
  if ((rc = c->integ.prepare(scheme))) return rc;
  if ((rc = c->integ.set_dt(dt, false, c->stream))) return rc;
  return c->integ.forward_revolve(scheme, u, nsteps, acts, ckpt, c->stream);
}

int sem_rk_adjoint_revolve(sem_ctx c, int32_t scheme, const void* ckpt, double dt, int32_t nsteps, int32_t snaps,
                           void* lam, void* work) {
  if (!c) return fail(SEM_ERR_ARG, "null context");
  if (!ckpt || !lam || !work) return fail(SEM_ERR_ARG, "null pointer");
  if (lam == ckpt || lam == work || work == ckpt) return fail(SEM_ERR_ARG, "aliased buffers");
  int rc = check_scheme(scheme);
  if (rc) return rc;
  if ((rc = check_steps(dt, nsteps, 1, false))) return rc;
  if (nsteps < 1 || snaps < 1) return fail(SEM_ERR_ARG, "need nsteps >= 1 and snaps >= 1 (got %d, %d)", nsteps, snaps);
  std::vector<RevolveAct> acts;
  revolve_plan(nsteps, snaps, acts);
  if ((rc = c->integ.prepare(scheme))) return rc;
  if ((rc = c->integ.set_dt(dt, false, c->stream))) return rc;
  return c->integ.adjoint_revolve(scheme, ckpt, snaps, acts, lam, work, c->stream);
}

// ------------------------------------------------------------------------------------------------
// Batched uneven problems
// ------------------------------------------------------------------------------------------------
int sem_batch_setup(const sem_desc* descs, const double* dts, int32_t count, void* stream, sem_batch* out) {
  if (!out) return fail(SEM_ERR_ARG, "null output pointer");
  *out = nullptr;
  if (!descs || !dts || count < 1) return fail(SEM_ERR_ARG, "need count >= 1 descriptors and step sizes");
  for (int i = 0; i < count; ++i) {
    int rc = validate_desc(&descs[i]);
    if (rc) return rc;
    if (descs[i].batch != 1) return fail(SEM_ERR_ARG, "batched problem %d has batch %d != 1", i, descs[i].batch);
    if (descs[i].dim != descs[0].dim || descs[i].dtype != descs[0].dtype)
      return fail(SEM_ERR_ARG, "problem %d differs in dim or dtype", i);
    if (!(dts[i] > 0.0) || !std::isfinite(dts[i])) return fail(SEM_ERR_ARG, "dt of problem %d must be > 0", i);
  }
  sem_batch b = new (std::nothrow) sem_batch_s();
  if (!b) return fail(SEM_ERR_NOMEM, "host allocation failed");
  b->descs.assign(descs, descs + count);
  b->dts.assign(dts, dts + count);
  b->stream = static_cast<hipStream_t>(stream);
  int rc = build_opset(b->os, descs, count, false);
  if (rc) {
    delete b;
    return rc;
  }
  b->offsets.assign(count + 1, 0);
  for (int i = 0; i < count; ++i) {
    int64_t v = 1;
    for (int k = 0; k < descs[i].dim; ++k) v *= (int64_t)descs[i].elems[k] * descs[i].order;
    b->offsets[i + 1] = b->offsets[i] + v * descs[i].dim;
  }
  // per-table-entry dt (table entries are sorted by order; match by packed offset)
  std::vector<double> tdt(b->os.hp.size());
  for (size_t t = 0; t < b->os.hp.size(); ++t) {
    int64_t off = b->os.hp[t].off;
    int i = (int)(std::lower_bound(b->offsets.begin(), b->offsets.end(), off) - b->offsets.begin());
    tdt[t] = dts[i];
  }
  b->integ.os = &b->os;
  b->integ.n = b->os.total_vals;
  b->integ.ts = b->os.ts;
  if ((rc = b->integ.dts.alloc(sizeof(double) * tdt.size()))) {
    delete b;
    return rc;
  }
  if (hipMemcpy(b->integ.dts.p, tdt.data(), sizeof(double) * tdt.size(), hipMemcpyHostToDevice) != hipSuccess) {
    delete b;
    return fail(SEM_ERR_HIP, "copying step sizes");
  }
  if ((rc = b->integ.set_dt(0.0, true, nullptr))) {
    delete b;
    return rc;
  }
  if (hipDeviceSynchronize() != hipSuccess) {
    delete b;
    return fail(SEM_ERR_HIP, "batch setup synchronisation");
  }
  g_err.clear();
  *out = b;
  return SEM_OK;
}

int sem_batch_destroy(sem_batch b) {
  if (!b) return fail(SEM_ERR_ARG, "null batch");
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  else (void)hipDeviceSynchronize();
  if (b->chain) (void)hipEventDestroy(b->chain);
  delete b;
  return SEM_OK;
}

int sem_batch_set_stream(sem_batch b, void* stream) {
  if (!b) return fail(SEM_ERR_ARG, "null batch");
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if (int rc = chain_streams(b->stream, s, b->chain)) return rc;
  b->stream = s;
  return SEM_OK;
}

int sem_batch_query(sem_batch b, int64_t* offsets) {
  if (!b || !offsets) return fail(SEM_ERR_ARG, "null argument");
  std::copy(b->offsets.begin(), b->offsets.end(), offsets);
  return SEM_OK;
}

static int batch_apply(sem_batch b, int op, const void* u, const void* v, void* out) {
  if (!b) return fail(SEM_ERR_ARG, "null batch");
  if (!u || !out || (op != OP_RHS && !v)) return fail(SEM_ERR_ARG, "null field pointer");
  if (out == u || (v && out == v)) return fail(SEM_ERR_ARG, "output aliases an input");
  Epi ep{out, nullptr, {0, 0}, {1, 0}, nullptr, nullptr, {0, 0}, {0, 0}};
  HIPCHK(b->os.apply(op, u, v, {1, 0}, ep, b->stream));
  return SEM_OK;
}

int sem_batch_mass(sem_batch b, void* m) {
  if (!b || !m) return fail(SEM_ERR_ARG, "null argument");
  for (const auto& hp : b->os.hp) HIPCHK(launch_mass(hp, m, b->descs[0].dtype, b->stream));
  return SEM_OK;
}

int sem_batch_rhs(sem_batch b, const void* u, void* f) { return batch_apply(b, OP_RHS, u, nullptr, f); }
int sem_batch_jact_vec(sem_batch b, const void* u, const void* w, void* jtw) {
  return batch_apply(b, OP_JACT, u, w, jtw);
}

int sem_batch_workspace_bytes(sem_batch b, int32_t K, int64_t* bytes) {
  if (!b || !bytes) return fail(SEM_ERR_ARG, "null argument");
  if (K < 1) return fail(SEM_ERR_ARG, "ckpt_every %d < 1", K);
  *bytes = b->integ.work_states(K) * b->integ.n * (int64_t)b->os.ts;
  return SEM_OK;
}

int sem_batch_set_adjoint_stages(sem_batch b, int32_t mode) {
  if (!b) return fail(SEM_ERR_ARG, "null batch");
  if (mode != SEM_ADJ_AUTO && mode != SEM_ADJ_STORE && mode != SEM_ADJ_RECOMPUTE)
    return fail(SEM_ERR_ARG, "adjoint stage mode %d", mode);
  b->integ.adj_mode = mode;
  return SEM_OK;
}

int sem_batch_rk_forward(sem_batch b, int32_t scheme, void* u, int32_t nsteps, int32_t K, void* ckpt) {
  if (!b) return fail(SEM_ERR_ARG, "null batch");
  if (!u) return fail(SEM_ERR_ARG, "null u");
  int rc = check_scheme(scheme);
  if (rc) return rc;
  if ((rc = check_steps(1.0, nsteps, K, ckpt != nullptr))) return rc;
  if (ckpt && ckpt == u) return fail(SEM_ERR_ARG, "ckpt aliases u");
  if ((rc = b->integ.prepare(scheme))) return rc;
  return b->integ.forward(scheme, u, nsteps, K, ckpt, b->stream);
}

int sem_batch_rk4_forward(sem_batch b, void* u, int32_t nsteps, int32_t K, void* ckpt) {
  return sem_batch_rk_forward(b, SEM_RK4, u, nsteps, K, ckpt);
}

int sem_batch_rk_adjoint(sem_batch b, int32_t scheme, const void* ckpt, int32_t nsteps, int32_t K, void* lam,
                         void* work) {
  if (!b) return fail(SEM_ERR_ARG, "null batch");
  if ((!ckpt && nsteps > 0) || !lam || !work) return fail(SEM_ERR_ARG, "null pointer");
  int rc = check_scheme(scheme);
  if (rc) return rc;
  if ((rc = check_steps(1.0, nsteps, K, true))) return rc;
  if (lam == ckpt || lam == work || work == ckpt) return fail(SEM_ERR_ARG, "aliased buffers");
  if ((rc = b->integ.prepare(scheme))) return rc;
  return b->integ.adjoint(scheme, ckpt, nsteps, K, lam, work, b->stream);
}

int sem_batch_rk4_adjoint(sem_batch b, const void* ckpt, int32_t nsteps, int32_t K, void* lam, void* work) {
  return sem_batch_rk_adjoint(b, SEM_RK4, ckpt, nsteps, K, lam, work);
}

int sem_batch_rk_stages_bytes(sem_batch b, int32_t scheme, int32_t nsteps, int64_t* bytes) {
  if (!b || !bytes) return fail(SEM_ERR_ARG, "null argument");
  int rc = check_scheme(scheme);
  if (rc) return rc;
  if (nsteps < 0) return fail(SEM_ERR_ARG, "nsteps %d < 0", nsteps);
  *bytes = (int64_t)nsteps * Integrator::stage_states(scheme) * b->integ.n * (int64_t)b->os.ts;
  return SEM_OK;
}

int sem_batch_rk_forward_stored(sem_batch b, int32_t scheme, void* u, int32_t nsteps, void* stages) {
  if (!b) return fail(SEM_ERR_ARG, "null batch");
  if (!u || (!stages && nsteps > 0)) return fail(SEM_ERR_ARG, "null pointer");
  if (stages == u) return fail(SEM_ERR_ARG, "stages alias u");
  int rc = check_scheme(scheme);
  if (rc) return rc;
  if ((rc = check_steps(1.0, nsteps, 1, false))) return rc;
  if ((rc = b->integ.alloc_buffers())) return rc;
  return b->integ.forward_stored(scheme, u, nsteps, stages, b->stream);
}

int sem_batch_rk_adjoint_stored(sem_batch b, int32_t scheme, const void* stages, int32_t nsteps, void* lam) {
  if (!b) return fail(SEM_ERR_ARG, "null batch");
  if (!lam || (!stages && nsteps > 0)) return fail(SEM_ERR_ARG, "null pointer");
  if (stages == lam) return fail(SEM_ERR_ARG, "stages alias lam");
  int rc = check_scheme(scheme);
  if (rc) return rc;
  if ((rc = check_steps(1.0, nsteps, 1, false))) return rc;
  if ((rc = b->integ.alloc_buffers())) return rc;
  return b->integ.adjoint_stored(scheme, stages, nsteps, lam, b->stream);
}

int sem_batch_configure(sem_batch b, int32_t persistent, int32_t param) {
  if (!b) return fail(SEM_ERR_ARG, "null batch");
  OpSet& os = b->os;
  if (persistent) {
    if (os.nitems == 0) return fail(SEM_ERR_UNSUPPORTED, "persistent launch needs a 2-D set of more than one problem");
    if (param < 1 || param > 65535) return fail(SEM_ERR_ARG, "persistent grid %d outside 1..65535", param);
    os.persistent = 1;
    os.pgrid = param;
  } else {
    int choices[8];
    for (auto& c : os.classes) {
      const int n = elem_epb_choices(os.dim, c.P, choices, 8);
      bool ok = param == 0;
      for (int i = 0; i < n && !ok; ++i) ok = choices[i] == param;
      c.epb = ok ? param : 0;  // orders without that choice keep their default
    }
    os.persistent = 0;
  }
  b->integ.reset_graphs(b->stream, true);
  return SEM_OK;
}

namespace {
struct TuneResult {
  int persistent, param;
  double ms;
};
std::mutex g_tune_mu;
std::map<std::string, TuneResult> g_tune_cache;

std::string batch_signature(const sem_batch_s* b) {
  std::string k = std::to_string(b->descs[0].dim) + ":" + std::to_string(b->descs[0].dtype);
  for (const auto& d : b->descs)
    k += "|" + std::to_string(d.order) + "," + std::to_string(d.elems[0]) + "," + std::to_string(d.elems[1]) + "," +
         std::to_string(d.elems[2]);
  return k;
}
}  // namespace

int sem_batch_autotune(sem_batch b, double* best_ms) {
  if (!b) return fail(SEM_ERR_ARG, "null batch");
  const std::string key = batch_signature(b);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      int rc = sem_batch_configure(b, it->second.persistent, it->second.param);
      if (best_ms) *best_ms = it->second.ms;
      return rc;
    }
  }
  std::vector<std::pair<int, int>> cand = {{0, 0}, {0, 1}, {0, 2}, {0, 4}, {0, 8}, {0, 16}};
  if (b->os.nitems > 0)
    for (int g : {256, 512, 1024, 2048, 4096}) cand.push_back({1, g});
  hipStream_t s = b->stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  TuneResult best{0, 0, 1e30};
  int rc = SEM_OK;
  for (auto [pm, prm] : cand) {
    if ((rc = sem_batch_configure(b, pm, prm))) break;
    if ((rc = b->integ.prepare(SEM_RK4))) break;
    // time the captured RK4 step on a zero state (values do not change the work)
    hipError_t he = hipMemsetAsync(b->integ.b(Integrator::STATE), 0, b->integ.n * b->integ.ts, s);
    for (int w = 0; w < 2 && he == hipSuccess; ++w) he = hipGraphLaunch(b->integ.gstep[SEM_RK4], s);
    if (he == hipSuccess) he = hipEventRecord(e0, s);
    const int R = 5;
    for (int r = 0; r < R && he == hipSuccess; ++r) he = hipGraphLaunch(b->integ.gstep[SEM_RK4], s);
    if (he == hipSuccess) he = hipEventRecord(e1, s);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    float ms = 0;
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    if (he != hipSuccess) {
      rc = fail(SEM_ERR_HIP, "autotune timing: %s", hipGetErrorString(he));
      break;
    }
    if (ms / R < best.ms) best = {pm, prm, ms / R};
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  if ((rc = sem_batch_configure(b, best.persistent, best.param))) return rc;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = best;
  }
  if (best_ms) *best_ms = best.ms;
  return SEM_OK;
}

}  // extern "C"
