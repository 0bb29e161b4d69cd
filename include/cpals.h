/*
 * cpals.h -- C ABI of the MI355X (gfx950) implicit CP-ALS library (libcpals.so).
 *
 * The library implements the hot path of the canonical-tensor (CP) time stepper of
 * Boelens, Venturi & Tartakovsky, "Parallel numerical tensor methods for
 * high-dimensional PDEs":
 *   - a CP tensor f = sum_l prod_k U_k[:, l]                  (Section 2.1, eq. functional-SSE)
 *   - separable operators A = sum_e eta_e kron_k E_k^e        (Section 3, eqs. Lz and BLs)
 *   - the implicit step A f_{n+1} = B f_n solved by alternating least squares over the
 *     dimensions, one convex problem per dimension               (Section 3.1, eqs. ALS2, ML, MR)
 *   - rank reduction by the same ALS with A = B = I           (Section 2.1, Section 3.2)
 *   - scalar products and operator application on CP tensors  (Sections 2.2 and 3.2)
 *
 * Memory and ownership
 *   - Every factor panel (cp_tensor.U[k]) is DEVICE memory owned by the caller; the
 *     library never frees or keeps it past the call.  Panels are column-major n_k x r with
 *     leading dimension ld[k] >= n[k] (element (i, l) at U[k][i + l * ld[k]]).
 *   - Operator descriptions (cp_operator, cp_op1d and everything they point to) are HOST
 *     memory; the library copies them to the device during the call.
 *   - Scalar outputs named *_dev are DEVICE pointers; report structs are HOST memory.
 *   - Device workspace: by default the library owns one per handle (grown on demand, freed
 *     by cp_destroy).  After cp_set_workspace the caller's buffer is used instead and no
 *     call on the handle allocates device memory; a call that needs more than the buffer
 *     holds returns CP_ERR_WORKSPACE before launching anything.  The cp_workspace_size_*
 *     queries give the bytes a call needs.
 *
 * Execution: calls are enqueued on the handle's HIP stream.  Calls that return a report
 * synchronise that stream once before returning.  One handle per host thread.
 *
 * Errors never cross the ABI as exceptions: every call returns a cp_status, and
 * cp_last_error() gives a message for the last failing call on the handle.  Shape and
 * argument checks happen before anything is launched.
 */
#ifndef CPALS_H
#define CPALS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CP_MAX_DIMS 8
#define CP_MAX_OPS 4
#define CP_MAX_TERMS 64
#define CP_MAX_RANK 64
#define CP_MAX_N 4096

typedef enum {
    CP_OK = 0,
    CP_ERR_INVALID_ARG = 1,  /* null pointer, bad enum, bad option value          */
    CP_ERR_SHAPE = 2,        /* dimensions, ranks or sizes inconsistent / too big */
    CP_ERR_UNSUPPORTED = 3,  /* valid request that the library does not implement */
    CP_ERR_HIP = 4,          /* HIP runtime error (allocation, launch, copy)      */
    CP_ERR_NOT_CONVERGED = 5, /* soft: results written, report.flags says why     */
    CP_ERR_WORKSPACE = 6     /* the caller's workspace (cp_set_workspace) is too small */
} cp_status;

/* report.flags bits */
#define CP_FLAG_NOT_CONVERGED 1u  /* max_sweeps reached with eps_conv > tol            */
#define CP_FLAG_PCG_MAXITER 2u    /* a per-dimension solve hit pcg_max_iter            */
#define CP_FLAG_REGULARIZED 4u    /* a Gauss-Jordan pivot of H_q + lambda_q I fell     */
                                  /* below 1e-12 of its largest diagonal entry         */
#define CP_FLAG_NONFINITE 8u      /* a NaN/Inf was produced                            */
#define CP_FLAG_SYNC_TIMEOUT 16u  /* a workgroup of a cluster waited too long for the    */
                                  /* others at a barrier; the result is not valid       */

typedef struct cp_handle_s* cp_handle;

/* Create a handle bound to the current HIP device and to `hip_stream` (a hipStream_t;
 * NULL = the null stream). */
cp_status cp_create(cp_handle* handle, void* hip_stream);
cp_status cp_destroy(cp_handle handle);
/* Caller-owned device workspace: `dev_ptr` (256-byte aligned, `bytes` long) is used by
 * every later call on the handle in place of library-allocated memory, until the next
 * cp_set_workspace; (NULL, 0) returns to the library's own workspace.  The buffer must stay
 * allocated while calls on the handle may run; calls that overlap on one buffer race.
 * INVALID_ARG for a misaligned pointer or a null pointer with nonzero bytes. */
cp_status cp_set_workspace(cp_handle handle, void* dev_ptr, size_t bytes);
cp_status cp_set_stream(cp_handle handle, void* hip_stream);
const char* cp_last_error(cp_handle handle);
/* Largest number of workgroups that may advance one problem together (default 16; 1 keeps
 * every problem on one workgroup).  A call that advances a single problem (cp_als_step,
 * cp_als_run, cp_truncate) splits its grid rows over a cluster of W workgroups, W the largest
 * power of two <= max_workgroups with every n_k divisible by 16 W, when no operator of A or B
 * is rank-1; batched calls always use one workgroup per problem.  The clusters meet at
 * device-wide barriers, and partial sums are added in a fixed order, so results are
 * deterministic for a given W (and agree across W to rounding).  INVALID_ARG outside 1..256. */
cp_status cp_set_cluster(cp_handle handle, int32_t max_workgroups);
/* Library version string (static storage). */
const char* cp_version(void);

/* A CP tensor of dimension d and separation rank r (Section 2.1).  U[k] are device
 * pointers to column-major n[k] x r panels with leading dimension ld[k]. */
typedef struct {
    int32_t d;
    int32_t r;
    int32_t n[CP_MAX_DIMS];
    int32_t ld[CP_MAX_DIMS];
    double* U[CP_MAX_DIMS];
} cp_tensor;

/* A one-dimensional linear operator on a periodic grid of n points (HOST data):
 *   CP_OP_IDENTITY : data unused
 *   CP_OP_DIAG     : data[n], O = diag(data)
 *   CP_OP_BAND     : data[(2*half_bw+1) * n], O[i, (i + j - half_bw) mod n] += data[j*n + i]
 *                    (periodic band, e.g. the central difference with half_bw = 1)
 *   CP_OP_RANK1    : data[2*n] = [m ; w], O = m w^T (e.g. a velocity-moment projector) */
typedef enum { CP_OP_IDENTITY = 0, CP_OP_DIAG = 1, CP_OP_BAND = 2, CP_OP_RANK1 = 3 } cp_op_kind;

typedef struct {
    int32_t kind;
    int32_t n;
    int32_t half_bw;
    const double* data;
} cp_op1d;

/* A separable operator sum_{e < n_terms} coef[e] * kron_k ops[k][op_index[e*d + k]]
 * (eq. Lz / eq. BLs).  ops[k] lists the DISTINCT 1-D operators of dimension k
 * (n_ops[k] <= CP_MAX_OPS), which is the paper's map of unique one-dimensional integrals
 * (Section 3.1, "Summary of the Algorithm").  All HOST memory. */
typedef struct {
    int32_t d;
    int32_t n_terms;
    const double* coef;
    const int32_t* op_index;
    int32_t n_ops[CP_MAX_DIMS];
    const cp_op1d* ops[CP_MAX_DIMS];
} cp_operator;

typedef enum { CP_PREC_FP64 = 0, CP_PREC_MIXED = 1 } cp_precision;
typedef enum { CP_RANK_FIXED = 0, CP_RANK_ADAPTIVE = 1 } cp_rank_mode;
typedef enum { CP_SWEEP_GAUSS_SEIDEL = 0, CP_SWEEP_JACOBI = 1 } cp_sweep_mode;

/* ALS options.
 *  tol          : stop when eps_conv = max_q ||Delta f_q|| / ||f|| <= tol after a sweep
 *                 (increment test of Section 3.1 / Appendix B, on the represented tensor)
 *  max_sweeps   : cap on Gauss-Seidel sweeps per solve (>= 1)
 *  precision    : CP_PREC_FP64, or CP_PREC_MIXED: sweeps with the Gram, right-hand-side and
 *                 matvec contractions in FP32 on the matrix cores (solves, scalars and checks
 *                 in FP64) until the increment stalls at the FP32 floor, then the Grams in
 *                 FP64 and FP64 sweeps until eps_conv <= tol
 *  eps_reg      : every per-dimension system is shifted by
 *                 lambda_q = eps_reg * trace(M_q) / (n_q r)  (regularisation, Section 2.1)
 *  pcg_tol      : relative residual target of the per-dimension PCG solve
 *  pcg_max_iter : PCG iteration cap per dimension update
 *  rank_mode    : CP_RANK_FIXED: the rank of the guess is kept.  CP_RANK_ADAPTIVE: the
 *                 separation rank is chosen per step (Section 4.1: adaptive rank up to a
 *                 maximum): after a converged solve at rank r the step residual
 *                 rho = ||A f - g|| / ||g|| (g = B f_n) is formed in double-double; while
 *                 rho > tau_rank (or, when replay_rank >= 0, while r < replay_rank) and
 *                 r < rank_cap, one term is appended -- three sweeps of rank-1 ALS fitting
 *                 the residual tensor g - A f from a seeded start (SplitMix64 of `seed`,
 *                 counter ((step*64 + r)*8 + k)*2^32 + i, 2u - 1 in every dimension k > 0)
 *                 -- and the step is solved again at rank r + 1.  Terms of weight
 *                 prod_k ||U_k[:, l]|| below 1e-14 of the largest are then dropped (the
 *                 kept columns move to the front, in order).  Later steps start from f_n
 *                 at its own rank.  Problems in adaptive mode run on one workgroup.
 *  tau_rank, rank_cap, replay_rank, seed : see rank_mode (rank_cap <= CP_MAX_RANK; the
 *                 output panels must hold rank_cap columns)
 *  report_residual : 1: every step's rho (double-double) into report.rel_residual (the
 *                 problem then runs on one workgroup); adaptive mode always reports it
 *  sweep_mode   : CP_SWEEP_GAUSS_SEIDEL (Section 3.1: q = 1..d in turn, each update from the
 *                 factors already updated) or CP_SWEEP_JACOBI (Appendix B, Algorithm 1: every
 *                 dimension solved from the factors at the start of the sweep, then every
 *                 factor moved by `damping` of its change, U_q <- U_q + damping (U_q' - U_q);
 *                 the paper divides the change by 4).  eps_conv uses the undamped changes.
 *  damping      : the Jacobi step fraction, 0 < damping <= 1 (default 0.25) */
typedef struct {
    double tol;
    int32_t max_sweeps;
    int32_t precision;
    double eps_reg;
    double pcg_tol;
    int32_t pcg_max_iter;
    int32_t rank_mode;
    double tau_rank;
    int32_t rank_cap;
    int32_t replay_rank;
    uint64_t seed;
    int32_t report_residual;
    int32_t sweep_mode;
    double damping;
} cp_als_opts;

/* Per-step report (HOST memory, filled after the call's single stream synchronisation). */
typedef struct {
    int32_t sweeps;        /* sweeps performed (summed over the solves of the step)     */
    int32_t pcg_iters;     /* PCG iterations summed over all updates                    */
    double eps_conv;       /* eps_conv after the last sweep                             */
    double fnorm;          /* ||f_{n+1}||                                               */
    double rel_residual;   /* rho = ||A f_{n+1} - g|| / ||g|| in double-double, or -1   */
                           /* when not formed (fixed rank without report_residual)      */
    uint32_t flags;        /* CP_FLAG_* bits of the last solve                          */
    int32_t final_rank;    /* rank of f_{n+1}                                           */
    int32_t grown_rank;    /* rank before small terms were dropped (replay_rank value   */
                           /* that reproduces this step's growth decisions)             */
    int32_t low_sweeps;    /* sweeps with FP32 contractions (CP_PREC_MIXED), of sweeps  */
} cp_als_report;

/* Fill `opts` with the defaults (tol 1e-8, max_sweeps 200, FP64, eps_reg 1e-10, pcg_tol
 * 1e-14, pcg_max_iter 100, fixed rank, tau_rank 1e-6, rank_cap CP_MAX_RANK, replay_rank -1,
 * seed 0, report_residual 0, Gauss-Seidel sweeps, damping 0.25). */
cp_status cp_als_default_opts(cp_als_opts* opts);

/* <x, y> = sum_{l,l'} prod_k <X_k[:,l], Y_k[:,l']>  (scalar product of CP tensors,
 * Section 2.2).  out_dev: one double in device memory.  Requires x.d == y.d, equal n. */
cp_status cp_inner(cp_handle h, const cp_tensor* x, const cp_tensor* y, double* out_dev);
/* ||x|| = sqrt(max(<x,x>, 0)).  out_dev: one double in device memory. */
cp_status cp_norm(cp_handle h, const cp_tensor* x, double* out_dev);

/* cp_inner for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same scalar product and kernels,
 * with the chunk partials in a file-scope device array of the library (4 MiB per GPU, held
 * until the process ends) instead of the handle's workspace.  The call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine); the array's device address is taken
 * once per device by cp_create.  The row chunks are capped so that the partials and the d
 * Grams fit in the array (fewer, longer chunks for large ranks), so the result may differ
 * from cp_inner's by reduction order (rounding).  Every call on a GPU shares that GPU's array
 * and every entry it reads is written first by the same call; calls that overlap on one GPU
 * (other streams, other threads) race.  CP_ERR_SHAPE when the partials of one chunk per
 * dimension and the Grams, (2 d rank(x) rank(y)) doubles, do not fit -- never for
 * d <= CP_MAX_DIMS and ranks <= CP_MAX_RANK (at most 1 MiB). */
cp_status cp_inner_noalloc(cp_handle h, const cp_tensor* x, const cp_tensor* y, double* out_dev);

/* y = L x as a CP tensor of rank n_terms * x.r (operator application, Section 3.2):
 * column e*x.r + l of y.U[k] is E_k^e X_k[:, l], with coef[e] multiplied into dimension 0.
 * y must have y.r == L.n_terms * x.r and the same n; y's panels are overwritten and must not
 * overlap x's panels (not checked; overlapping panels give undefined results). */
cp_status cp_apply_operator(cp_handle h, const cp_operator* L, const cp_tensor* x, cp_tensor* y);

/* One implicit time step: minimise ||A f_{n+1} - B f_n|| over rank-r CP tensors
 * (eqs. rRr1, resnorm) by Gauss-Seidel ALS over q = 1..d (eqs. sequential_min, ALS2).
 * f_next is in/out: on entry the initial guess (rank r = f_next.r), on exit f_{n+1}.
 * The columns of the result are balanced (equal factor norms per column).
 * With opts.rank_mode = CP_RANK_ADAPTIVE the panels of f_next hold opts.rank_cap columns;
 * on return f_next->r is the final rank (report.final_rank).
 * Returns CP_ERR_NOT_CONVERGED (results still written) if max_sweeps was reached. */
cp_status cp_als_step(cp_handle h, const cp_operator* A, const cp_operator* B, const cp_tensor* f_n,
                      cp_tensor* f_next, const cp_als_opts* opts, cp_als_report* report);

/* The implicit step with a source term, A f_{n+1} = B f_n + c (the time step of Section 3.1
 * with the source of the paper's forced equations, already scaled, e.g. c = dt C).  c is a
 * CP tensor (device panels owned by the caller, same d and n_k as f_n; null: cp_als_step).
 * The right-hand side g = B f_n + c is formed in the workspace as one CP tensor (the
 * applied terms of B f_n, as cp_apply_operator, followed by c's columns) and the step
 * A f_{n+1} = g is solved as cp_als_step does (same options, report and errors).  Requires
 * n_terms(B) * f_n.r + c.r <= CP_MAX_RANK. */
cp_status cp_als_step_source(cp_handle h, const cp_operator* A, const cp_operator* B, const cp_tensor* f_n,
                             const cp_tensor* source, cp_tensor* f_next, const cp_als_opts* opts,
                             cp_als_report* report);

/* Relative residual of the implicit step, rho = ||A f - B f_n|| / ||B f_n|| (the residual
 * of eqs. rRr1 / resnorm that drives rank control, Section 3.2).  Formed on the device in
 * double-double: the Grams of the stacked applied panels [O_A^a U_k | O_B^b V_k] by
 * compensated dot products (Dot2), their Hadamard products over the dimensions and the sum
 * over all term pairs in double-double, so rho is resolved down to ~1e-15 (a plain FP64
 * expansion <Af,Af> - 2<Af,Bf_n> + <Bf_n,Bf_n> cancels below ~1e-8).  One workgroup.
 * Written to *rel_residual (host) after one stream synchronisation. */
cp_status cp_residual(cp_handle h, const cp_operator* A, const cp_operator* B, const cp_tensor* f,
                      const cp_tensor* f_n, double* rel_residual);

/* cp_als_step with opts.rank_mode = CP_RANK_ADAPTIVE, opts.tau_rank = tau and
 * opts.rank_cap = f_next->r: the panels of f_next hold f_next->r columns, the first r_start
 * of them are the initial guess.  Output: the factors in the first *final_rank columns,
 * *rel_residual the last rho (double-double).  Errors as cp_als_step; CP_ERR_INVALID_ARG
 * unless 1 <= r_start <= f_next->r and tau >= 0. */
cp_status cp_als_step_adaptive(cp_handle h, const cp_operator* A, const cp_operator* B, const cp_tensor* f_n,
                               cp_tensor* f_next, int32_t r_start, double tau, const cp_als_opts* opts,
                               cp_als_report* report, int32_t* final_rank, double* rel_residual);

/* n_steps implicit steps in one device-resident launch: f_0 = f_init, guess for step s is
 * f_{s-1} (the first step uses f_io as guess), result f_{n_steps} written to f_io.
 * reports: host array of n_steps.  traj (nullable): device buffer of
 * n_steps * sum_k n_k * rc doubles (rc = f_io.r, or opts.rank_cap in adaptive mode)
 * receiving every step's factors, packed dimension after dimension, column-major n_k x rc
 * (in adaptive mode the first final_rank columns of each step are valid).  Adaptive mode:
 * f_io's panels hold opts.rank_cap columns; on return f_io->r is the last step's rank. */
cp_status cp_als_run(cp_handle h, const cp_operator* A, const cp_operator* B, const cp_tensor* f_init,
                     cp_tensor* f_io, int32_t n_steps, const cp_als_opts* opts, cp_als_report* reports,
                     double* traj);

/* Rank reduction: minimise ||f - g|| over rank-f.r CP tensors by ALS (Section 2.1).
 * f is in/out (initial guess in, result out). */
cp_status cp_truncate(cp_handle h, const cp_tensor* g, cp_tensor* f, const cp_als_opts* opts,
                      cp_als_report* report);

/* One explicit second-order Adams-Bashforth step f_{n+2} = f_{n+1} + (dt/2) L (3 f_{n+1} - f_n)
 * (Section 3.2, eq. AB2_), split as the paper splits it into additions, one operator
 * application and rank reductions to at most cap = f_next->r columns:
 *   i)   w = 3 f_{n+1} - f_n (f_cur's columns scaled by 3, then f_prev's by -1, the scalars in
 *        dimension 0), reduced by ALS (cp_truncate) from its leading cap columns when its
 *        rank rank(f_prev) + rank(f_cur) exceeds cap;
 *   ii)  y = L w, reduced when L.n_terms * rank(w) > cap: the ALS fit of L w at rank cap
 *        (cp_als_step with A = I, B = L, f_n = w, so L w is never formed) from the leading cap
 *        columns of L w (the first terms of L applied to w);
 *   iii) f_{n+2} = f_{n+1} + (dt/2) y (f_cur's columns, then y's), reduced from its leading
 *        cap columns when rank(f_cur) + rank(y) > cap.
 * Reductions use opts (fixed rank).  reports: 3 entries (sweeps 0 for a reduction that was
 * not needed).  f_next (capacity cap columns, not overlapping the inputs) receives the result
 * and f_next->r its rank.  Requires rank(f_prev) + rank(f_cur) <= CP_MAX_RANK and
 * rank(f_cur) + rank(y) <= CP_MAX_RANK.  Temporaries live in the workspace
 * (cp_workspace_size_ab2). */
cp_status cp_ab2_step(cp_handle h, const cp_operator* L, double dt, const cp_tensor* f_prev, const cp_tensor* f_cur,
                      cp_tensor* f_next, const cp_als_opts* opts, cp_als_report* reports);

/* Many independent problems advanced in one persistent launch (one workgroup per problem, or
 * the tuned cluster sizes: see cp_tune_cluster).
 * Arrays of length count: A[i], B[i] (host descriptions), f_init[i], f_io[i] and opts[i]
 * (each problem has its own options: tolerance, rank mode and cap) as in cp_als_run;
 * reports: count * n_steps entries, problem-major; traj (nullable, host array of count device
 * pointers, entries nullable): problem i's trajectory buffer as cp_als_run's.  In adaptive
 * mode f_io[i].r is updated to problem i's final rank. */
cp_status cp_als_run_batched(cp_handle h, int32_t count, const cp_operator* A, const cp_operator* B,
                             const cp_tensor* f_init, cp_tensor* f_io, int32_t n_steps,
                             const cp_als_opts* opts, cp_als_report* reports, double* const* traj);

/* The batched run captured once and replayed (the many-instance form of Section 3.1's time
 * stepping, launched as a HIP graph).
 *
 * cp_batch_plan_create validates and packs the count problems exactly as cp_als_run_batched
 * (same arguments, opts[count]), uploads their operator data once into device memory owned by the plan,
 * and captures one run into a graph on a stream of the plan's own: copies of the f_init[i]
 * and f_io[i] panels into the plan, the persistent kernel, the results back into f_io[i],
 * the reports into pinned host memory of the plan.  The graph keeps the device pointers of
 * f_init[i] and f_io[i]: those buffers must stay allocated, with the same shapes, until the
 * plan is destroyed; their contents may change between runs.
 *
 * cp_batch_plan_run replays the graph after the work already queued on the handle's stream
 * and waits for it; reports: count * n_steps entries, problem-major, as cp_als_run_batched
 * (and the same CP_ERR_NOT_CONVERGED rule; in adaptive mode the final ranks are in the
 * reports, the f_io descriptors given at creation are not updated).  A plan is used by one thread at a time.
 * cp_batch_plan_destroy waits for the plan's stream and frees everything the plan owns.
 * Errors: those of cp_als_run_batched; CP_ERR_HIP when the capture or instantiation fails. */
typedef struct cp_batch_plan_s* cp_batch_plan;
cp_status cp_batch_plan_create(cp_handle h, int32_t count, const cp_operator* A, const cp_operator* B,
                               const cp_tensor* f_init, cp_tensor* f_io, int32_t n_steps,
                               const cp_als_opts* opts, cp_batch_plan* plan);
cp_status cp_batch_plan_run(cp_handle h, cp_batch_plan plan, cp_als_report* reports);
cp_status cp_batch_plan_destroy(cp_batch_plan plan);

/* Cluster-size tuning.  A problem can be advanced by a cluster of W workgroups that split its
 * grid rows (W a power of two <= the cp_set_cluster limit, every n_k a multiple of 16 W, no
 * rank-1 operator); the handle keeps a table of tuned W per problem shape (d, n_k, r, the
 * rank of f_n, the operator counts per dimension, the precision).
 *
 * cp_tune_cluster times `sweeps` sweeps (tol 0) of the implicit step of Section 3.1 for f_n
 * from guess with every admissible W (each once to warm up, then timed with HIP events on the
 * handle's stream), records the fastest in the table and returns it in *best_w and its time
 * in *best_ms (nullable).  guess is left untouched (trials run on a copy of it in the
 * workspace).
 * Use of the table: a single problem (cp_als_step, cp_als_run, a plan of one problem) runs
 * with its tuned W when one is recorded, else with the largest admissible W.  A batch
 * (cp_als_run_batched, cp_batch_plan_create) gives every problem its tuned W (1 where none
 * is recorded) when all workgroups of the launch fit on the device at once (at most one
 * workgroup per compute unit), else one workgroup to each problem.
 * cp_tune_save writes the table as JSON, {"cluster": {"<shape>": W, ...}}; cp_tune_load
 * merges such a file into the table (CP_ERR_INVALID_ARG for a file that cannot be read or
 * parsed, or a W that is not a power of two in 1..256); cp_tune_clear empties it. */
cp_status cp_tune_cluster(cp_handle h, const cp_operator* A, const cp_operator* B, const cp_tensor* f_n,
                          const cp_tensor* guess, const cp_als_opts* opts, int32_t sweeps, int32_t* best_w,
                          float* best_ms);
cp_status cp_tune_save(cp_handle h, const char* path);
cp_status cp_tune_load(cp_handle h, const char* path);
cp_status cp_tune_clear(cp_handle h);

/* Workspace sizes (bytes) for a caller-owned workspace (cp_set_workspace).  Arguments as in
 * the calls they size; nothing is launched.
 *  cp_workspace_size_step  : cp_als_run / cp_als_step (n_steps = 1) with these shapes and
 *                            options, and with source non-null cp_als_step_source; also
 *                            enough for cp_residual(A, B, f_io, f_init), cp_tune_cluster and
 *                            cp_als_step_adaptive on f_io
 *  cp_workspace_size_batched : cp_als_run_batched with these arguments
 *  cp_workspace_size_inner : cp_inner(x, y) and cp_norm(x) (pass y = x)
 *  cp_workspace_size_apply : cp_apply_operator(L, x, .)
 *  cp_workspace_size_ab2   : cp_ab2_step(L, ., f_prev, f_cur, f_next, opts, .) */
cp_status cp_workspace_size_step(cp_handle h, const cp_operator* A, const cp_operator* B, const cp_tensor* f_init,
                                 const cp_tensor* source, const cp_tensor* f_io, int32_t n_steps,
                                 const cp_als_opts* opts, size_t* bytes);
cp_status cp_workspace_size_batched(cp_handle h, int32_t count, const cp_operator* A, const cp_operator* B,
                                    const cp_tensor* f_init, const cp_tensor* f_io, int32_t n_steps,
                                    const cp_als_opts* opts, size_t* bytes);
cp_status cp_workspace_size_inner(cp_handle h, const cp_tensor* x, const cp_tensor* y, size_t* bytes);
cp_status cp_workspace_size_apply(cp_handle h, const cp_operator* L, const cp_tensor* x, size_t* bytes);
cp_status cp_workspace_size_ab2(cp_handle h, const cp_operator* L, const cp_tensor* f_prev, const cp_tensor* f_cur,
                                const cp_tensor* f_next, const cp_als_opts* opts, size_t* bytes);

#ifdef __cplusplus
}
#endif

#endif /* CPALS_H */
