/*
 * sem.h -- C ABI of libsem: matrix-free spectral-element viscous-Burgers operators, their
 * Jacobian products, and RK4 forward/adjoint integration on one AMD Instinct MI355X (gfx950).
 *
 * Method: Marin, Constantinescu & Smith, "A scalable matrix-free spectral element approach for
 * unsteady PDE constrained optimization using PETSc/TAO", arXiv 1806.01422.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Mesh.   A periodic box [0,L_1]x..x[0,L_d] (d = 1, 2, 3) split into E_1 x .. x E_d equal
 *         elements, each carrying (N+1)^d Gauss-Lobatto-Legendre (GLL) points (order N).
 *         Along direction k there are n_k = E_k * N unique nodes; node g_k lies at
 *         x = (g_k div N) h_k + (xi_{g_k mod N} + 1) h_k / 2, h_k = L_k / E_k.
 * Fields. A field is a velocity with C = d components stored as a contiguous device array
 *         [batch][C][n_3][n_2][n_1] (x fastest) of the context's dtype (double or float).
 *         ndof = C * n_1 * n_2 * n_3 values per batch member.
 * Memory. Every pointer argument named u, v, w, f, jv, jtw, lam, ckpt, work is a DEVICE pointer
 *         owned by the caller, who keeps it alive until the stream work completes.  libsem
 *         never frees caller memory.  The context owns its tables and scratch, released in
 *         sem_destroy: the operators' tables and face buffer are allocated in sem_setup, the
 *         time integrators' state buffers (twelve states) and captured step graphs at the first
 *         call of an integrator entry point (so a context used for operator products only never
 *         holds them).
 * Streams. All work is enqueued on the context stream (a hipStream_t passed as void*, NULL for
 *         the null stream) and returns without synchronising, except where documented.
 * Errors. Every function returns SEM_OK (0) or a negative sem_status and sets a thread-local
 *         message readable with sem_last_error().  Inputs are validated before anything is
 *         enqueued; on error nothing has been enqueued.  Outputs must not alias inputs
 *         (checked by pointer equality, SEM_ERR_ARG).  A context is not thread-safe.
 */
#ifndef SEM_H
#define SEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SEM_OK = 0,
  SEM_ERR_ARG = -1,         /* invalid argument: sizes, null/aliased pointers, dt, nsteps */
  SEM_ERR_UNSUPPORTED = -2, /* order N or dimension outside the compiled range */
  SEM_ERR_HIP = -3,         /* a HIP runtime call failed (message carries the HIP error) */
  SEM_ERR_NOMEM = -4,       /* device allocation failed */
  SEM_ERR_NONFINITE = -5,   /* a trajectory produced a non-finite value (when checking is on) */
  SEM_ERR_NOCONV = -6       /* a Newton or Krylov iteration did not reach its tolerance */
} sem_status;

typedef enum { SEM_F64 = 0, SEM_F32 = 1 } sem_dtype;

/* Explicit time integrators.  SEM_RK4: the classical four-stage method.  SEM_RK3: the three-stage
   explicit RK-3 of the paper's scalability runs (Sec. 6.3), which prints no tableau; libsem takes
   Kutta's third-order method (c = 0, 1/2, 1; a21 = 1/2, a31 = -1, a32 = 2; b = 1/6, 2/3, 1/6). */
typedef enum { SEM_RK4 = 0, SEM_RK3 = 1, SEM_CN = 2 } sem_scheme;  /* SEM_CN: Crank-Nicolson (sem_cn_*) */

/* Problem descriptor.  Supported: dim 1..3; order 1..12 for dim 1 and 2, 1..9 for dim 3;
   elems[k] >= 1; length[k] > 0; nu >= 0; batch >= 1.  Entries past dim are ignored. */
typedef struct {
  int32_t dim;
  int32_t elems[3];
  int32_t order;
  double length[3];
  double nu;
  int32_t dtype; /* sem_dtype */
  int32_t batch; /* number of same-shape fields stacked on the leading axis */
} sem_desc;

typedef struct sem_ctx_s* sem_ctx;

/* Create a context: computes the GLL tables (Sec. 3.2: Legendre polynomials on GLL points,
   nodes, weights and the differentiation matrix D), the 1-D assembled lumped masses, and
   allocates the scratch the operators need (the integrators allocate theirs on first use).
   stream: hipStream_t or NULL. */
int sem_setup(const sem_desc* desc, void* stream, sem_ctx* out);
/* Waits for the context's work (on its current stream, which carries the work of every stream
   it used before: see sem_set_stream), then frees its tables, scratch and graphs. */
int sem_destroy(sem_ctx ctx);
/* Rebind the stream used by later calls.  The new stream first waits (a device-side event wait,
   no host synchronisation) for everything already enqueued on the old one: the context's scratch
   and graphs are shared by all its calls, so its work stays one ordered chain. */
int sem_set_stream(sem_ctx ctx, void* stream);
/* ndof per batch member (C * nodes) and unique nodes per component. Either pointer may be NULL. */
int sem_query(sem_ctx ctx, int64_t* ndof, int64_t* nodes);
/* Operator implementation the context runs (host only, no GPU work): 0 the element kernel plus
   node summation kernel (any dimension and order), 2 the tuned 2-D kernel for orders 3, 5, 7 (x element
   count a multiple of 8, at most 64), 3 the tuned 3-D order-7 kernel (x element count a multiple
   of 4).  All three compute the same operators (Sec. 3.3); they differ in summation order only. */
int sem_query_path(sem_ctx ctx, int32_t* path);
/* Host copy of the 1-D node coordinates of direction dir (n_dir doubles into x_host). */
int sem_node_coords(sem_ctx ctx, int32_t dir, double* x_host);

/* m = the assembled diagonal GLL mass M (Sec. 3.2: the lumped mass of the collocation quadrature,
   M[g] = prod_k (h_k / 2) (2 w_0 if g_k mod N = 0, else w_{g_k mod N})), written to every component
   of every batch member: m is a device array shaped like a field. */
int sem_mass(sem_ctx ctx, void* m);

/* f = F(u) = M^{-1} Q^T a(Q u): the semi-discrete right-hand side of u_t = nu Lap u - (u.grad)u
   in the explicit form u' = M^{-1} P(u) (Sec. 3.4), where a(.) is the per-element weak form
   -sum_j D_j^T(nu W D_j U_i) - W sum_j U_j D_j U_i (Sec. 3.3, eq. rhsvec; signs of eq. burgers23d),
   Q the periodic gather to elements, Q^T the direct-stiffness summation and M the assembled
   diagonal GLL mass.  u, f: [batch][C][...] device arrays; f must not alias u. */
int sem_rhs(sem_ctx ctx, const void* u, void* f);

/* jv = J(u) v, the Jacobian of F at u applied to v (Sec. 3.3, eq. jacvec, with the M^{-1} of the
   explicit form).  jv must alias neither u nor v. */
int sem_jac_vec(sem_ctx ctx, const void* u, const void* v, void* jv);

/* jtw = J(u)^T w, the Euclidean transpose of J(u) on the unique nodes (Sec. 3.3, eq. jactransvec):
   J^T w = Q^T a'(Qu)^T Q M^{-1} w, i.e. the inverse mass scales the input before the gather and
   the summed result is not divided.  jtw must alias neither u nor w. */
int sem_jact_vec(sem_ctx ctx, const void* u, const void* w, void* jtw);

/* Classical RK4 with fixed step dt, nsteps steps, applied in place to u (u0 in, u(T) out) for
   every batch member.  If ckpt is non-NULL, u_{sK} (K = ckpt_every) is copied to
   ckpt[s][batch][ndof] for s = 0 .. nsteps/K - 1 before step sK (nsteps % K must be 0).
   The four stage updates are fused into the summation kernels; one step is a captured graph. */
int sem_rk4_forward(sem_ctx ctx, void* u, double dt, int32_t nsteps, int32_t ckpt_every, void* ckpt);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
   loops, harnesses that forbid hipMalloc): sem_rk4_forward with the same arguments, results and
   checkpoints, that allocates nothing.  Its three stage states and its stage accumulator live in a
   64 MiB file-scope device array that each GPU holds for the life of the process (its address is
   resolved in sem_setup); a state may therefore hold at most (64 MiB / 4) rounded down to 256 bytes,
   i.e. about 2.1 M FP64 values (batch * ndof), else SEM_ERR_ARG with a message naming the limit.
   The steps are launched one by one (no graph is captured or instantiated) and no non-finite check
   runs.  Every call on one GPU shares that GPU's array and leaves its contents behind: calls that
   overlap in time on one GPU (other streams, other contexts, other threads) race on it and must be
   ordered by the caller.  The context itself comes from sem_setup, which does allocate. */
int sem_rk4_forward_noalloc(sem_ctx ctx, void* u, double dt, int32_t nsteps, int32_t ckpt_every, void* ckpt);

/* Discrete adjoint of sem_rk4_forward (Sec. 4.1, eqs. adjointloop, initadj, gradient, adjtime,
   for the classical RK4 tableau): on entry lam holds lambda_N = dPhi/du(T); on exit lambda_0 =
   dPhi/du_0.  Uses the checkpoints written by sem_rk4_forward with the same dt, nsteps and
   ckpt_every, and recomputes each segment of K states into work (Sec. 5.3).  work: device buffer
   of at least sem_workspace_bytes(ctx, ckpt_every) bytes.  Stage states: by default, states of
   4M values or more have the segment recompute store every step's stage states in work (4 F per
   step, as an adjoint with stored stages), and each adjoint step then only applies the four J^T
   products; smaller states keep one state per step and recompute the stage states in each
   adjoint step (3 F more per step, but every step is one captured graph).  Both give the same
   values; sem_set_adjoint_stages overrides the choice.  With stored stages lam is updated in place
   through the sweep, so lam overlapping ckpt or work is SEM_ERR_ARG.  With nsteps = 0, lam is
   left unchanged and ckpt may be NULL (as for every adjoint entry point below). */
int sem_rk4_adjoint(sem_ctx ctx, const void* ckpt, double dt, int32_t nsteps, int32_t ckpt_every,
                    void* lam, void* work);
/* The same two calls for any sem_scheme: the stage updates of every scheme are fused into the
   summation kernels and one step is a captured graph.  RK-3: a step applies F three times; its
   discrete adjoint (Sec. 4.1 for a general tableau: a_i = J(U_i)^T dt (b_i lam + sum_{j>i} A_ji a_j),
   lam <- lam + sum_i a_i) recomputes two stage states (2 F) and applies three J^T.  ckpt, work and
   errors as for RK4; an unknown scheme is SEM_ERR_ARG. */
int sem_rk_forward(sem_ctx ctx, int32_t scheme, void* u, double dt, int32_t nsteps, int32_t ckpt_every, void* ckpt);
int sem_rk_adjoint(sem_ctx ctx, int32_t scheme, const void* ckpt, double dt, int32_t nsteps, int32_t ckpt_every,
                   void* lam, void* work);
/* Every stage stored (the adjoint of Sec. 4.1 fed with the forward sweep's own stage states, as
   an adjoint with stored stages and no checkpoint recompute does):
   - sem_rk_stages_bytes (host only): bytes of the stage buffer for nsteps steps of the scheme:
     nsteps * S states, S = 4 for RK4 (u_k, U2, U3, U4) and 3 for RK-3 (u_k, U2, U3).
   - sem_rk_forward_stored: u in: u_0, out: u(T), bitwise equal to sem_rk_forward.  Writes state
     u_k and its stage states to stages[k][s][batch][ndof] (s < S) as the stage launches form them.
   - sem_rk_adjoint_stored: lam in: lambda_N, out: lambda_0 from those stages (read only), with the
     same scheme, dt and nsteps: only the J^T products of each step (RK4: 4, RK-3: 3) and their
     fused updates.  Bitwise equal to sem_rk_adjoint with the stage states stored
     (SEM_ADJ_STORE).
   With nsteps = 0 the stage buffer may be NULL; lam (and u) pass through unchanged.  An unknown
   scheme, a non-positive dt or aliased buffers are SEM_ERR_ARG; sem_rk_adjoint_stored updates lam
   in place, so lam overlapping the stage states is SEM_ERR_ARG too. */
int sem_rk_stages_bytes(sem_ctx ctx, int32_t scheme, int32_t nsteps, int64_t* bytes);
int sem_rk_forward_stored(sem_ctx ctx, int32_t scheme, void* u, double dt, int32_t nsteps, void* stages);
int sem_rk_adjoint_stored(sem_ctx ctx, int32_t scheme, const void* stages, double dt, int32_t nsteps, void* lam);
/* Binomial (revolve) checkpointing (Sec. 5.3: recompute the forward trajectory from a few stored
   states; the paper's runs use PETSc's revolve).  With `snaps` state slots the adjoint advances
   the least number of forward steps any schedule with that many slots needs.
   - sem_revolve_plan (host only): the schedule as `nactions` (kind, arg) pairs in `actions`
     (host int64 array of 2 * capacity entries; NULL to query nactions).  Kinds: 0 RESTORE slot
     (current state <- slot), 1 ADVANCE k steps, 2 STORE slot (slot <- current state), 3 ADJOINT i
     (adjoint of step i from the current state u_i).  Slot 0 holds u_0.  advances (may be NULL)
     receives the number of forward steps in the schedule.  SEM_ERR_ARG if capacity is too small.
   - sem_rk_forward_revolve: like sem_rk_forward (u in: u_0, out: u(T)) and stores the
     schedule's first snapshots into ckpt[snaps][batch][ndof].
   - sem_rk_adjoint_revolve: lam in: lambda_N, out: lambda_0 from that ckpt (read only); work
     holds sem_revolve_workspace_bytes(ctx, snaps) bytes.  Bitwise equal to sem_rk_adjoint with the
     same scheme, dt and nsteps. */
int sem_revolve_plan(int32_t nsteps, int32_t snaps, int64_t* nactions, int64_t* actions, int64_t capacity,
                     int64_t* advances);
int sem_rk_forward_revolve(sem_ctx ctx, int32_t scheme, void* u, double dt, int32_t nsteps, int32_t snaps, void* ckpt);
int sem_rk_adjoint_revolve(sem_ctx ctx, int32_t scheme, const void* ckpt, double dt, int32_t nsteps, int32_t snaps,
                           void* lam, void* work);
int sem_revolve_workspace_bytes(sem_ctx ctx, int32_t snaps, int64_t* bytes);
/* Crank-Nicolson, the paper's implicit scheme (Sec. 6.3), with a Newton-Krylov solve per step
   (Sec. 2: Newton-type nonlinear solves with Krylov linear solves and matrix-free Jacobians).
   Each step solves R(v) = v - u - dt/2 (F(u) + F(v)) = 0 by Newton's method from the predictor
   u + dt F(u); the corrections solve (I - dt/2 J(v)) d = R(v) by restarted GMRES with matrix-free
   J v products.  The discrete adjoint of the exact step map (Sec. 4.1, eq. adjtime) needs linear
   solves only: (I - dt/2 J(u_{n+1}))^T mu = lambda_{n+1} by GMRES with J^T products, then
   lambda_n = mu + dt/2 J(u_n)^T mu.  Each adjoint segment recomputes its K + 1 states from the
   checkpoint.  Both calls synchronise the stream (the iterations read norms on the host) and are
   not capturable.  A batch (desc.batch > 1) is solved as one block-diagonal system.
   opts may be NULL (defaults); stats (may be NULL) receives the iteration counts. */
typedef struct {
  double newton_rtol;    /* stop when ||R||_2 <= newton_rtol ||u + dt/2 F(u)||_2; 0: 1e-13 (FP64), 1e-6 (FP32) */
  int32_t newton_maxit;  /* Newton iterations per step; 0: 25 */
  double gmres_rtol;     /* relative residual of each linear solve; 0: 1e-11 (FP64), 1e-5 (FP32) */
  int32_t gmres_restart; /* Krylov basis size between restarts, 1..39; 0: 30 */
  int32_t gmres_maxit;   /* GMRES iterations per linear solve; 0: 300 */
} sem_nk_opts;
typedef struct {
  int64_t newton_iters;    /* Newton iterations, all steps */
  int64_t linear_solves;   /* GMRES solves */
  int64_t gmres_iters;     /* GMRES iterations (J v or J^T w products), all solves */
  double max_rel_residual; /* largest final relative residual of any Newton or GMRES solve */
} sem_nk_stats;
/* Bytes of the caller work buffer of sem_cn_forward and sem_cn_adjoint (the adjoint's is larger:
   (K + 1) + (restart + 2) states; the forward needs restart + 2). */
int sem_cn_workspace_bytes(sem_ctx ctx, int32_t ckpt_every, const sem_nk_opts* opts, int64_t* bytes);
/* u in: u_0, out: u(T); checkpoints as in sem_rk4_forward (ckpt may be NULL).  SEM_ERR_NOCONV when
   Newton or GMRES does not converge within its iteration limit. */
int sem_cn_forward(sem_ctx ctx, void* u, double dt, int32_t nsteps, int32_t ckpt_every, void* ckpt,
                   const sem_nk_opts* opts, void* work, sem_nk_stats* stats);
/* lam in: lambda_N, out: lambda_0, from sem_cn_forward's checkpoints. */
int sem_cn_adjoint(sem_ctx ctx, const void* ckpt, double dt, int32_t nsteps, int32_t ckpt_every, void* lam,
                   const sem_nk_opts* opts, void* work, sem_nk_stats* stats);
/* Line search with guaranteed sufficient decrease (More and Thuente, the step-length rule of the
   paper's LMVM optimiser, Sec. 5), host only, by reverse communication.  It seeks stp with
   phi(stp) <= phi(0) + ftol stp phi'(0) and |phi'(stp)| <= gtol |phi'(0)|, stpmin <= stp <= stpmax.
   Call first with *task = SEM_LS_START, f = phi(0), g = phi'(0) < 0 and *stp the initial step;
   while it returns *task = SEM_LS_FG, evaluate f = phi(*stp), g = phi'(*stp) and call again.
   It ends with SEM_LS_CONVERGED, SEM_LS_WARNING (no further progress: the interval reached xtol
   relative width, rounding, or stp hit stpmin / stpmax; *stp is the best step) or SEM_LS_ERROR
   (invalid start).  work/iwork carry the state between calls. */
enum { SEM_LS_START = 0, SEM_LS_FG = 1, SEM_LS_CONVERGED = 2, SEM_LS_WARNING = 3, SEM_LS_ERROR = 4 };
typedef struct {
  double ftol, gtol, xtol, stpmin, stpmax; /* inputs */
  double work[14];                         /* state, owned by the line search */
  int32_t iwork[4];
} sem_line_search;
int sem_line_search_step(sem_line_search* ls, int32_t* task, double* stp, double f, double g);
/* Optimal initial condition by LMVM (Sec. 5: limited-memory variable-metric directions with
   More-Thuente step lengths; Sec. 6.1: recover u_0 from the state at time T).  Minimises
   Phi(u_0) = 1/2 sum (u(T) - u*)^2 over all nodes, components and batch members, with u(T) from
   `scheme` (SEM_RK4, SEM_RK3 or SEM_CN, nsteps of dt, checkpoints every ckpt_every) and the
   gradient from its discrete adjoint.  Directions: -g first (tried with a step of length 1 in
   the 2-norm), then the two-loop recursion over the last `memory` pairs (s, y) with s.y > 0 and
   initial inverse Hessian (s.y / y.y) I, tried with step 1; a direction that does not descend
   restarts from -g.  u0: in the initial guess, out the final iterate.  work: device buffer of
   sem_lmvm_workspace_bytes bytes.  history (host, may be NULL) receives Phi at iterates 0..iters.
   Synchronises the stream. */
typedef struct {
  int32_t max_iters;       /* 0: 50 */
  int32_t memory;          /* stored pairs, 1..20; 0: 5 */
  double gatol, grtol;     /* stop when ||g||_2 <= gatol or <= grtol |Phi|; 0: 1e-10 each */
  double ftol, gtol, xtol; /* line search (sem_line_search); 0: 1e-4, 0.9, 1e-10 */
  int32_t max_evals;       /* evaluations per line search; 0: 30 */
} sem_lmvm_opts;
typedef struct {
  int32_t iters, evals;  /* iterations, objective-and-gradient evaluations */
  int32_t reason;        /* 1 gatol, 2 grtol, 3 max_iters; -1 line search failed or exhausted */
  double f0, f, gnorm;   /* first and last Phi, last ||g||_2 */
} sem_lmvm_stats;
int sem_lmvm_workspace_bytes(sem_ctx ctx, int32_t scheme, int32_t nsteps, int32_t ckpt_every,
                             const sem_lmvm_opts* opts, int64_t* bytes);
int sem_lmvm_initial_condition(sem_ctx ctx, int32_t scheme, void* u0, const void* target, double dt, int32_t nsteps,
                               int32_t ckpt_every, const sem_lmvm_opts* opts, void* work, double* history,
                               sem_lmvm_stats* stats);
/* Bytes of caller work buffer needed by sem_rk4_adjoint / sem_rk_adjoint for a given ckpt_every:
   ckpt_every states, or 4 ckpt_every states when stage states are stored (query again after
   sem_set_adjoint_stages). */
int sem_workspace_bytes(sem_ctx ctx, int32_t ckpt_every, int64_t* bytes);
/* How the RK adjoints obtain the stage states of a step (host only): SEM_ADJ_AUTO (default:
   stored for states of 4M values or more), SEM_ADJ_STORE (always stored: the segment recompute
   writes them to work), SEM_ADJ_RECOMPUTE (never: each adjoint step recomputes them, 2 F for
   RK-3 and 3 F for RK4).  Other values are SEM_ERR_ARG. */
typedef enum { SEM_ADJ_AUTO = 0, SEM_ADJ_STORE = 1, SEM_ADJ_RECOMPUTE = 2 } sem_adj_stages;
int sem_set_adjoint_stages(sem_ctx ctx, int32_t mode);
/* Enable (1) or disable (0, default) the non-finite check at the end of sem_rk4_forward (one
   host synchronisation per call). */
int sem_set_check_finite(sem_ctx ctx, int32_t on);

/* Message of the last failure on the calling thread ("" if none).  Valid until the next call. */
const char* sem_last_error(void);

/* Diagnostic, outside the operator path: the FP64 rates of this GPU's matrix cores
 * (v_mfma_f64_16x16x4f64) and vector units (v_fma_f64), each alone and both interleaved in one
 * instruction stream of 4096 x 256 threads, `iters` loop iterations each.  This is the measurement
 * behind contracting the element lines (Sec. 3.3, sum factorisation) with vector FMAs.  Writes
 * tflops[0] = matrix cores alone, [1] = vector units alone, [2] and [3] = the matrix and vector
 * parts of the interleaved run (host array of 4, TFLOP/s).  Allocates and frees an 8 MiB device
 * buffer; `stream` may be NULL (the default stream); synchronises it.  SEM_ERR_ARG for a NULL
 * result or iters < 1. */
int sem_probe_fp64_rates(void* stream, int32_t iters, double* tflops);

/* ---------------------------------------------------------------------------------------------
 * Batched uneven problems: `count` independent problems of possibly different dim-2 shapes,
 * orders, viscosities and step sizes, packed back to back in one device array (problem p
 * occupies [offset_p, offset_p + ndof_p) values; offsets from sem_batch_query).  Each RK4 stage
 * runs as one persistent launch over all problems (work items sorted by cost) and one
 * summation launch; a full RK4 step is captured in a HIP graph and replayed.  Descriptors must
 * share dim and dtype and have batch == 1.
 * ------------------------------------------------------------------------------------------- */
typedef struct sem_batch_s* sem_batch;
/* dts: host array of count step sizes.  stream: hipStream_t or NULL. */
int sem_batch_setup(const sem_desc* descs, const double* dts, int32_t count, void* stream, sem_batch* out);
/* Waits for the set's work (as sem_destroy), then frees it. */
int sem_batch_destroy(sem_batch b);
/* Rebind the stream used by later calls on the set (as sem_set_stream: the new stream waits for
   the old one's work). */
int sem_batch_set_stream(sem_batch b, void* stream);
/* offsets: host array of count+1 entries (in values, not bytes); offsets[count] = total. */
int sem_batch_query(sem_batch b, int64_t* offsets);
/* The assembled diagonal mass of every problem (as sem_mass) on a packed array. */
int sem_batch_mass(sem_batch b, void* m);
/* F of every problem: f = F(u) on packed arrays. */
int sem_batch_rhs(sem_batch b, const void* u, void* f);
/* J_p(u_p)^T w_p for every problem p on packed arrays. */
int sem_batch_jact_vec(sem_batch b, const void* u, const void* w, void* jtw);
/* RK4 forward for every problem with its own dt (nsteps shared); ckpt as in sem_rk4_forward with
   the packed layout: ckpt[s][total]. */
int sem_batch_rk4_forward(sem_batch b, void* u, int32_t nsteps, int32_t ckpt_every, void* ckpt);
/* Discrete adjoint for every problem; work must hold sem_batch_workspace_bytes bytes. */
int sem_batch_rk4_adjoint(sem_batch b, const void* ckpt, int32_t nsteps, int32_t ckpt_every, void* lam,
                          void* work);
/* The same for any sem_scheme. */
int sem_batch_rk_forward(sem_batch b, int32_t scheme, void* u, int32_t nsteps, int32_t ckpt_every, void* ckpt);
int sem_batch_rk_adjoint(sem_batch b, int32_t scheme, const void* ckpt, int32_t nsteps, int32_t ckpt_every,
                         void* lam, void* work);
/* The stored-stage pair for a batch (each problem with its own dt): stages[k][s][total]. */
int sem_batch_rk_stages_bytes(sem_batch b, int32_t scheme, int32_t nsteps, int64_t* bytes);
int sem_batch_rk_forward_stored(sem_batch b, int32_t scheme, void* u, int32_t nsteps, void* stages);
int sem_batch_rk_adjoint_stored(sem_batch b, int32_t scheme, const void* stages, int32_t nsteps, void* lam);
int sem_batch_workspace_bytes(sem_batch b, int32_t ckpt_every, int64_t* bytes);
/* sem_set_adjoint_stages for a batch (the state is the whole packed set). */
int sem_batch_set_adjoint_stages(sem_batch b, int32_t mode);
/* Launch shape of the element stage.  persistent = 1: one persistent launch over all problems
   (2-D sets of more than one problem) with `param` workgroups walking a cost-sorted work list;
   persistent = 0: one launch per order class with `param` elements per workgroup (0 = default;
   orders without that choice keep their default).  Drops the captured RK4 graphs (recaptured on
   the next integration); when graphs exist it first synchronises the set's stream, so that no
   graph launch is still in flight when its executable is destroyed. */
int sem_batch_configure(sem_batch b, int32_t persistent, int32_t param);
/* Time the candidate launch shapes on the captured RK4 step of this problem set and keep the
   fastest (synchronises the stream; overwrites the integrator's internal state buffers, not
   caller data; results are cached per problem set for the process).  best_ms (host, may be NULL)
   receives the fastest step time in milliseconds. */
int sem_batch_autotune(sem_batch b, double* best_ms);

#ifdef __cplusplus
}
#endif
#endif /* SEM_H */
