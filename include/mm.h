/*
 * mm.h -- C ABI of the MI355X map-making library (block-Jacobi PCG for the maximum-likelihood
 * map-making system of arXiv:2112.03370).
 *
 * The library solves, on one GPU,
 *
 *     (P^T N^-1 P) m = P^T N^-1 d                      (Eq. genMapEstimator with F_T = N^-1)
 *
 * where P is the pointing matrix with three non-zeros per row, (1, cos 2psi, sin 2psi), in the
 * columns of the pixel observed by the sample (Eq. dataModelSingleSlot, Eq. dataModelHwp), and
 * N^-1 is block-diagonal with one symmetric banded Toeplitz block per stationary interval
 * (Eq. MADCAP; the stbmm product of the Toeplitz algebra package: samples outside every block
 * are passed through unchanged).  The solver is PCG (Alg. 1) with the block-Jacobi
 * preconditioner M_BD = (P^T diag(N^-1) P)^-1 (BJ paragraph of the preconditioner section).
 *
 * Conventions
 *   - Every function returns an mm_status; none aborts, throws or exits.  On error the
 *     thread-local detail string is available from mm_last_error().
 *   - "DEVICE" pointers are HIP device (HBM) addresses owned by the caller; "HOST" pointers are
 *     ordinary host memory owned by the caller.  The library never frees caller memory.
 *   - Pixel-domain vectors are FP64, pixel-major: [k][n_kept][3] (I, Q, U), where n_kept is
 *     the number of kept pixels of the plan, ordered by ascending global pixel id.
 *   - Time-domain vectors are FP32 with n_samples entries per right-hand side, detector-major.
 *   - stream is a hipStream_t passed as void* (NULL = the default stream).  Asynchronous calls
 *     are ordered on that stream; calls on one plan must not overlap (they share its workspace;
 *     mm_pcg_solve serializes itself, the asynchronous calls are ordered by the caller).  The
 *     serving calls below run solves on one plan concurrently, each with its own workspace.
 */
#ifndef MM_H
#define MM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mm_status;

enum {
  MM_OK = 0,
  MM_PENDING = 1,            /* mm_poll: request not finished yet */
  MM_ERR_INVALID = -1,       /* bad argument, index out of range, overlapping blocks, ... */
  MM_ERR_NOT_SPD = -2,       /* band symbol <= 0, or p^T A p <= 0 / r^T z <= 0 in PCG */
  MM_ERR_NO_CONV = -3,       /* max_iter reached; the last iterate is returned */
  MM_ERR_OOM = -4,           /* device allocation failed */
  MM_ERR_HIP = -5,           /* a HIP runtime call failed */
  MM_ERR_BUDGET = -6,        /* serving: request can never fit the memory budget */
  MM_ERR_UNSUPPORTED = -7,   /* valid input outside what the library implements */
  MM_ERR_NOT_FOUND = -8      /* serving: unknown ticket */
};

enum { MM_TOEPLITZ_AUTO = 0, MM_TOEPLITZ_DIRECT = 1, MM_TOEPLITZ_FFT = 2 };

/* mm_geometry.precision: arithmetic of the time-domain products inside the PCG loop.
 *   MM_PRECISION_MIXED  FP32 time-domain vectors and FP32 Toeplitz arithmetic; FP64 pointing
 *                       sums, P^T accumulation, pixel domain and CG recurrences (default).
 *   MM_PRECISION_FP64   every product (b and A x) in FP64 throughout (slower; the reference
 *                       precision, and the product used by the FP64 exit check). */
enum { MM_PRECISION_MIXED = 0, MM_PRECISION_FP64 = 1 };

typedef struct mm_plan mm_plan_t;
typedef struct mm_server mm_server_t;

/*
 * Problem geometry (pointing + block-Toeplitz inverse noise).
 *   pix[s]      DEVICE int32 [n_samples]  global pixel id in [0, n_pix_global), -1 = flagged.
 *   w_q, w_u    DEVICE float [n_samples]  cos 2psi_s, sin 2psi_s (the I weight is 1).
 *   blk_*       HOST [n_blocks]            stationary intervals: first sample, length >= 1,
 *                                          band index.  Blocks must not overlap and, when
 *                                          det_offset is given, must not cross detectors.
 *   band_*      HOST [n_bands]             band b holds band_ncoef[b] = lambda_b + 1 FP32
 *                                          coefficients c_0..c_lambda at band_coef +
 *                                          band_offset[b] (first row of the Toeplitz block).
 *   det_offset  HOST [n_dets + 1] or NULL  first sample of each detector (validation only).
 *   cond_max    excision threshold on the 2-norm condition number of each pixel's 3x3 BJ
 *               block; <= 0 selects 1e3.  Pixels with fewer than 3 hits are excised too.
 *   toeplitz_algo  MM_TOEPLITZ_*; fft_size  real FFT length for the overlap-save product
 *               (power of two in [2^11, 2^17], > 2 lambda_max), 0 = automatic (the smallest
 *               power of two >= 4 lambda_max, with the exceptions of the kernels' limits),
 *               -1 = tuned: the plan is built at that length N0 and at 2 N0 and 4 N0 (up to
 *               2^17), one system product is timed on each and the fastest is kept; the choice
 *               is remembered for plans of the same shape (samples, blocks, lambda_max, flags,
 *               precision, device) for the life of the process.  Lengths up
 *               to 2^15 run in one CU's LDS (fused with the pointing products); 2^16 and 2^17
 *               (lambda up to 2^15 and beyond) use a four-step transform through one device
 *               tile per CU, fused with the pointing products as well.
 *   flags       MM_FLAG_* bits.
 *   precision   MM_PRECISION_*.
 *   n_poly, n_baselines, base_start, base_len
 *               template map-making (Eq. defFT with the Legendre baselines of Appendix A,
 *               Eq. polytemplate): n_poly > 0 deprojects, on every baseline interval
 *               [base_start[i], base_start[i] + base_len[i]) (HOST int64 arrays), the Legendre
 *               polynomials of degrees 0 .. n_poly - 1, each scaled to unit norm on the
 *               interval's sample grid.  The weights W^-1 are then diagonal: every band must
 *               have band_ncoef = 1 (its c_0 is the weight of the block's samples; 1 outside
 *               blocks), otherwise MM_ERR_UNSUPPORTED.  Baselines must not overlap and, when
 *               det_offset is given, must not cross detectors.  n_poly = 0 (the default): no
 *               templates, F_T = N^-1 (the maximum-likelihood system).
 * All pointers are read only during mm_plan and may be released afterwards.
 */
typedef struct {
  int64_t n_samples;
  const int32_t* pix;
  const float* w_q;
  const float* w_u;
  int64_t n_pix_global;
  int32_t n_blocks;
  const int64_t* blk_start;
  const int64_t* blk_len;
  const int32_t* blk_band;
  int32_t n_bands;
  const int32_t* band_ncoef;
  const int64_t* band_offset;
  const float* band_coef;
  int32_t n_dets;
  const int64_t* det_offset;
  double cond_max;
  int32_t toeplitz_algo;
  int32_t fft_size;
  int32_t flags;            /* MM_FLAG_* bits, 0 = defaults */
  int32_t precision;        /* MM_PRECISION_*, 0 = MM_PRECISION_MIXED */
  int32_t n_poly;           /* Legendre templates per baseline, 0 = none */
  int32_t pad0;
  int64_t n_baselines;
  const int64_t* base_start;
  const int64_t* base_len;
} mm_geometry;

/* mm_geometry.flags: MM_FLAG_UNFUSED keeps the FFT path's gather, Toeplitz product and scatter
 * as three kernels with FP32 time-domain vectors in HBM (the fused kernel is the default).
 * MM_FLAG_LDS_FFT keeps fused 2^15-sample segments in the LDS-resident kernel (one workgroup
 * per CU); by default segments of that length with at most 2^14 outputs (lambda >= 2^13) use
 * the register-resident kernel, which runs two workgroups per CU. */
enum { MM_FLAG_UNFUSED = 1, MM_FLAG_LDS_FFT = 2 };

typedef struct {
  int64_t n_samples;
  int64_t n_pix_global;
  int64_t n_obs;          /* pixels with at least one unflagged sample */
  int64_t n_kept;         /* pixels solved for */
  int64_t n_excised;      /* n_obs - n_kept */
  int64_t n_gap_samples;  /* flagged or excised samples (zero rows of P) */
  int64_t device_bytes;   /* device memory owned by the plan */
  int32_t lambda_max;
  int32_t toeplitz_algo;  /* algorithm actually used */
  int32_t fft_size;       /* 0 when not using the FFT product */
  int32_t n_blocks;
  int32_t n_chunks;       /* overlap-save segments (FFT) or tiles (direct) per product */
  int32_t fused;          /* 1: gather, Toeplitz and scatter run as one kernel per segment
                             (LDS-resident FFT), 2: the same with the register-resident FFT,
                             3: the same with the four-step FFT of long segments */
  int32_t precision;      /* MM_PRECISION_* of the plan */
  int32_t n_poly;         /* template orders per baseline (0: maximum-likelihood system) */
  int64_t n_baselines;
} mm_plan_info_t;

typedef struct {
  double tol;             /* stop when ||r_k||_2 < tol ||b||_2 (Alg. 1); <= 0 selects 1e-8 */
  int32_t max_iter;       /* <= 0 selects 10000 */
  int32_t use_x0;         /* nonzero: start from the x passed in (restart); else x0 = 0 */
  int32_t check_every;    /* iterations between host convergence checks; <= 0 automatic */
  int32_t use_graph;      /* nonzero: replay iterations from a captured HIP graph */
  int32_t block;          /* right-hand sides solved together (Alg. 2 on stacked columns):
                             0 or 1 each column alone (Alg. 1); 2..32 that many at a time;
                             < 0 tune among 1 (each alone), 8, 16, 32 on the first column
                             groups; the choice is kept (per plan, and per problem shape for
                             the life of the process) and later tuned solves start with it */
  int32_t precond;        /* 0 block-Jacobi M_BD; 1 two-level M_2lvl (Eq. 2lvlDef), which needs
                             mm_deflation_build on the plan and block 0/1 */
  int32_t refine;         /* MM_PRECISION_MIXED plans, block 0/1: up to `refine` steps of
                             iterative refinement after the solve: r = b - A x with b and A in
                             FP64, an inner PCG on A d = r with the plan's products to the
                             relative tolerance that brings ||r|| under tol ||b||, x += d; stops
                             once the FP64 true residual (Eq. CGresidual) is below tol.  0: none */
  int32_t check_fp64;     /* nonzero: report the FP64 true residual ||b - A x|| / ||b|| with
                             b and A in FP64 (two FP64 products; implied by refine > 0) */
} mm_solve_opts;

typedef struct {
  int32_t iterations;     /* PCG iterations (A products inside the loop) */
  int32_t converged;      /* 1 when the stopping test passed */
  double relres;          /* recursive ||r_k|| / ||b|| */
  double true_relres;     /* ||b - A x_k|| / ||b|| of the PCG iterate x_k with one more product,
                             FP64 reductions: the plan's product, or the FP64 one when an FP64
                             residual is taken anyway (refine > 0 or check_fp64 on a Toeplitz
                             FFT plan, whose FP64 product forms b - A x in one pass) */
  double bnorm;           /* ||b||_2 */
  double ms;              /* wall time of the solve (of the column's group when block >= 2) */
  int32_t block;          /* columns solved together with this one (1: alone) */
  int32_t refine_steps;   /* refinement updates applied */
  double true_relres64;   /* ||b - A x|| / ||b|| with b and A in FP64 (Eq. CGresidual), when
                             refine > 0, check_fp64, or an MM_PRECISION_FP64 plan; else -1 */
  int32_t inner_iterations;  /* PCG iterations of the refinement solves */
  int32_t pad0;
} mm_solve_info;

/* mm_plan -- build the device plan: copy the pointing to the device plan, count hits, build
 * the 3x3 BJ blocks sum_s diag(N^-1)_s w_s w_s^T (diag(N^-1) = c_0 of the sample's band, 1
 * outside blocks), excise pixels with < 3 hits or condition number > cond_max together with
 * their samples (Degeneracy section), compact global -> local pixels (MAPMAT local indexing),
 * invert the kept blocks, and check that every band's symbol c_0 + 2 sum_k c_k cos(k w) is
 * positive (so every Toeplitz block and A are SPD).  Synchronous on `stream`.  The plan owns
 * all its device memory and is immutable.
 * Errors: MM_ERR_INVALID (bad sizes, pixel id out of range, overlapping blocks), MM_ERR_NOT_SPD
 * (non-positive symbol), MM_ERR_UNSUPPORTED (lambda beyond the implemented products),
 * MM_ERR_OOM, MM_ERR_HIP.  *out is NULL on error. */
mm_status mm_plan(const mm_geometry* g, void* stream, mm_plan_t** out);

/* Release a plan (NULL allowed).  The caller must have synchronised its streams. */
mm_status mm_plan_destroy(mm_plan_t* plan);

/* Plan statistics (host struct). */
mm_status mm_plan_info(const mm_plan_t* plan, mm_plan_info_t* out);

/* Kept pixels: HOST outputs with n_kept entries each (either may be NULL): ascending global
 * ids and their hit counts (unflagged samples).  Bit-exact integers.  Synchronous. */
mm_status mm_plan_pixels(const mm_plan_t* plan, int64_t* global_ids, int32_t* hits);

/* t = P x: the un-pointing step of the system product (the pointing matrix of
 * Eq. dataModelSingleSlot / Eq. dataModelHwp applied to a map; first of the three operations of
 * the right-to-left product in the solvers section).  x DEVICE double [n_kept][3]; t DEVICE
 * float [n_samples]; gap samples get 0.  Sums in FP64, stored FP32.  Asynchronous.  Errors:
 * MM_ERR_INVALID (NULL plan or vector, wrong device), MM_ERR_HIP. */
mm_status mm_unpoint(const mm_plan_t* plan, const double* x, float* t, void* stream);

/* u = N^-1 t: the block-diagonal banded Toeplitz product of the inverse noise weights
 * (Eq. MADCAP; the stbmm product of the Toeplitz algebra package: identity outside blocks,
 * truncated at block edges, shift-and-overlap segments of the plan's FFT length).  Template
 * plans apply F_T of Eq. defFT on the same call path only inside mm_apply_A / mm_rhs; here they
 * apply the diagonal weights.  t, u DEVICE float [n_samples], must not alias.  FP32.
 * Asynchronous.  Errors: MM_ERR_INVALID (NULL, aliasing, wrong device), MM_ERR_HIP. */
mm_status mm_noise_weight(const mm_plan_t* plan, const float* t, float* u, void* stream);

/* y = P^T u: the pointing (binning) step, last of the three operations of the system product:
 * y[p] = sum over samples of p of (1, cos 2psi, sin 2psi) u_s, FP64 accumulation.  u DEVICE
 * float [n_samples]; y DEVICE double [n_kept][3] is overwritten.  Asynchronous.  Errors:
 * MM_ERR_INVALID, MM_ERR_HIP. */
mm_status mm_point(const mm_plan_t* plan, const float* u, double* y, void* stream);

/* b = P^T F_T d, the right-hand side of Eq. genMapEstimator (F_T = N^-1 for the
 * maximum-likelihood system, Eq. defFT for template plans), for k right-hand sides; d DEVICE
 * float, column j at d + j*ld_d (ld_d >= n_samples); gap samples of d are ignored.  b DEVICE
 * double [k][n_kept][3].  FP64 products on MM_PRECISION_FP64 and template plans (synchronous
 * there), else FP32 time domain.  Asynchronous otherwise.  Errors: MM_ERR_INVALID, MM_ERR_OOM,
 * MM_ERR_HIP. */
mm_status mm_rhs(const mm_plan_t* plan, const float* d, int32_t k, int64_t ld_d, double* b,
                 void* stream);

/* y = P^T F_T P x, the system matrix of Eq. genMapEstimator applied right to left as the
 * solvers section describes (un-pointing, noise weighting / template filter, pointing), k
 * columns.  x, y DEVICE double [k][n_kept][3], must not alias.  Precision as mm_rhs.
 * Asynchronous (synchronous for FP64 products).  Errors: MM_ERR_INVALID, MM_ERR_OOM,
 * MM_ERR_HIP. */
mm_status mm_apply_A(const mm_plan_t* plan, const double* x, double* y, int32_t k,
                     void* stream);

/* z = M_BD r, the block-Jacobi preconditioner (P^T diag(N^-1) P)^-1 of the preconditioner
 * section: one symmetric 3x3 FP64 block per kept pixel, inverted at plan time.  r, z DEVICE
 * double [k][n_kept][3] (may alias).  Asynchronous.  Errors: MM_ERR_INVALID, MM_ERR_HIP. */
mm_status mm_precond_bj(const mm_plan_t* plan, const double* r, double* z, int32_t k,
                        void* stream);

/* Solve A x = P^T N^-1 d for k right-hand sides.  opts->block 0/1: PCG (Alg. 1) on each
 * column alone.  opts->block >= 2 (or < 0, tuned): columns are taken in groups of t and each
 * group is solved by the enlarged-CG recurrences (Alg. 2, Orthomin form, search block
 * Z = M_BD R with one column per right-hand side, t x t systems by an FP64 eigen
 * pseudo-inverse, a column leaves the block once ||r_j|| < tol ||b_j||); one multi-column
 * product per iteration serves the whole group; use_x0, use_graph and check_every do not
 * apply (x starts at 0).  d as in mm_rhs; x DEVICE double [k][n_kept][3] (read when
 * opts->use_x0); info HOST array of k entries (may be NULL).  opts may be NULL (defaults).
 * Synchronous: returns when x holds the maps.  Errors: MM_ERR_NO_CONV (x = last iterate),
 * MM_ERR_NOT_SPD, MM_ERR_OOM (block workspace: 4 t n_kept 3 doubles), MM_ERR_HIP. */
mm_status mm_pcg_solve(const mm_plan_t* plan, const float* d, int32_t k, int64_t ld_d,
                       double* x, const mm_solve_opts* opts, mm_solve_info* info,
                       void* stream);

/* mm_pcg_solve_noalloc -- mm_pcg_solve for callers that cannot allocate device memory
 * (serving loops with a fixed footprint, code run where hipMalloc is forbidden).  It allocates
 * nothing: the solve's pixel-domain vectors, reduction partials and device scalars live in a
 * static device array of the library (64 MiB per GPU, held until the process ends), so
 * 40 * n_kept bytes (five FP64 vectors of 3 n_kept) plus a few KB must fit: MM_ERR_INVALID
 * beyond that.  Same arguments and results as mm_pcg_solve, restricted to PCG per column
 * with block-Jacobi (opts->block 0/1, precond 0, refine 0, check_fp64 0; use_graph is
 * ignored: launches are eager) on plans whose product keeps the time domain on chip (fused
 * FFT product or diagonal weights, MM_PRECISION_MIXED, no templates); otherwise
 * MM_ERR_UNSUPPORTED.  Per-kernel timing must be off.  All calls on one GPU share its array:
 * calls are serialised per device inside the process; concurrent calls are therefore safe
 * but never overlap.  Synchronous. */
mm_status mm_pcg_solve_noalloc(const mm_plan_t* plan, const float* d, int32_t k, int64_t ld_d,
                               double* x, const mm_solve_opts* opts, mm_solve_info* info,
                               void* stream);

/* ---- Two-level a posteriori preconditioner (Eq. 2lvlDef, A-DEF1; Alg. 3) ------------------
 * mm_deflation_build runs m steps of Lanczos (Alg. 3) on A = P^T N^-1 P from r0 = b =
 * P^T N^-1 d (d: one right-hand side, DEVICE float [n_samples]), keeps the Lanczos vectors
 * V_m and the products A V_m on the device (the plan owns them: 2 m + 1 pixel-domain FP64
 * vectors), forms the coarse matrix E = V_m^T A V_m and its FP64 pseudo-inverse
 * (eigen-directions below 1e-12 of the largest dropped; the paper's Ritz rotation of V_m is
 * not needed since M_2lvl depends on span(V_m) only).  Later solves with opts.precond = 1
 * apply M_2lvl = M_BD (I - A Q) + Q, Q = Z E^+ Z^T, as in Eq. 2lvlDef0.  Synchronous; m in
 * [1, 128]; the process stops early when beta_(k+1) falls below machine precision.  Errors:
 * MM_ERR_INVALID (m out of range, b = 0), MM_ERR_OOM, MM_ERR_HIP.  A new build replaces the
 * previous one; mm_deflation_clear releases it. */
typedef struct {
  int32_t m;              /* Lanczos steps taken = columns of the deflation space */
  int32_t rank;           /* directions kept by the pseudo-inverse of E */
  double e_min;           /* smallest kept eigenvalue of E */
  double e_max;           /* largest eigenvalue of E */
  double build_ms;
  int64_t device_bytes;
} mm_deflation_info_t;

mm_status mm_deflation_build(mm_plan_t* plan, const float* d, int32_t m, void* stream);
mm_status mm_deflation_info(const mm_plan_t* plan, mm_deflation_info_t* out);
mm_status mm_deflation_clear(mm_plan_t* plan);
/* Copies the deflation vectors V_m to z (DEVICE double [m][n_kept][3], m from the info). */
mm_status mm_deflation_vectors(const mm_plan_t* plan, double* z, void* stream);
/* z = M_2lvl r (Eq. 2lvlDef0), r and z DEVICE double [k][n_kept][3], must not alias.  Needs a
 * built deflation space (MM_ERR_INVALID otherwise).  Asynchronous. */
mm_status mm_precond_2lvl(const mm_plan_t* plan, const double* r, double* z, int32_t k,
                          void* stream);

/* Per-kernel timing (HIP events recorded on the launch stream around every launch of the
 * plan's kernels while enabled; graphs are not used then).  kind: 0 un-pointing, 1 Toeplitz
 * product, 2 pointing (P^T), 3 CG vector kernels.  Outputs total milliseconds and launch count
 * since the last reset.  Synchronous. */
mm_status mm_set_timing(mm_plan_t* plan, int32_t enable);
mm_status mm_kernel_time(mm_plan_t* plan, int32_t kind, double* total_ms, int64_t* launches);

/* ---- Serving: many solves of uneven size, continuously batched on one GPU ------------------
 *
 * A server keeps plans on the device (a cache keyed by a caller-chosen 64-bit geometry key) and
 * runs submitted solves on n_slots host threads, each with its own HIP stream and per-request
 * workspace, so the solves of different requests overlap on the device.  A request is admitted
 * when a slot is free and its workspace fits the device-memory budget next to the cached plans
 * and the running requests; a request that does not fit lets later ones start (up to
 * max_bypass times, then it waits at the head of the queue).  Idle workspaces are kept per plan
 * for reuse and released, then unpinned plans evicted least recently used first, when memory is
 * needed.  Each request runs exactly the computation of mm_pcg_solve on its own (its columns
 * never share a block with another request's), so its result does not depend on the mix apart
 * from the order of FP64 atomic additions.  With size classes (large_work > 0), requests whose
 * work n_samples x k reaches large_work run at most large_slots at a time: on a saturated
 * device concurrency only divides a large solve's share, so large requests keep close to their
 * run-alone time while small ones flow past them on the other slots. */
typedef struct {
  int64_t hbm_budget;    /* device bytes for cached plans + request workspaces; <= 0: 80% of
                            the free device memory at creation */
  int32_t n_slots;       /* solves running at once; <= 0: 4 */
  int32_t max_bypass;    /* later requests that may start before a waiting one; < 0: 16 */
  int64_t large_work;    /* size classes: a request of n_samples x k >= large_work is large;
                            <= 0: one class (no size rule) */
  int32_t large_slots;   /* large requests running at once (<= 0: 1); small requests take the
                            other slots, and a large request held by this rule lets later
                            requests pass without counting as bypassed */
  int32_t pad0;
} mm_server_opts;

typedef struct {
  double queued_ms;      /* submit -> start on a slot */
  double run_ms;         /* start -> result ready */
  double total_ms;       /* submit -> result ready */
  int32_t slot;          /* slot that ran the request */
  int32_t pad;
} mm_request_times;

typedef struct {
  int64_t hbm_budget;
  int64_t bytes_in_use;  /* cached plans + workspaces (idle and running) */
  int64_t peak_bytes;
  int64_t submitted;
  int64_t completed;
  int64_t plan_hits;
  int64_t plan_misses;
  int64_t evictions;
  int32_t queued;
  int32_t running;
  int32_t peak_running;  /* most requests that ran at once */
  int32_t n_plans;
  int32_t peak_large;    /* most large requests that ran at once */
  int32_t pad0;
} mm_server_stats_t;

/* Create a server on the current device.  opts may be NULL (defaults).  Errors: MM_ERR_INVALID,
 * MM_ERR_HIP. */
mm_status mm_server_create(const mm_server_opts* opts, mm_server_t** out);

/* Stop the server: queued requests are dropped (never run), running solves finish, then every
 * cached plan and workspace is released.  Tickets are invalid afterwards.  NULL is accepted. */
mm_status mm_server_destroy(mm_server_t* server);

/* Make the plan of geometry g available under `key` (mm_plan semantics; the geometry's device
 * arrays must stay valid until this call returns).  A cached key is a hit and g is not read (it
 * may be NULL then).  info (HOST, may be NULL) receives the plan's mm_plan_info.  Blocks while
 * another thread builds the same key.  Errors: those of mm_plan; MM_ERR_INVALID (g NULL on a
 * miss); MM_ERR_BUDGET (the plan alone exceeds the budget). */
mm_status mm_server_plan(mm_server_t* server, const mm_geometry* g, uint64_t key,
                         mm_plan_info_t* info);

/* Queue a solve of k right-hand sides on the cached plan `key`; arguments as mm_pcg_solve
 * (d, x DEVICE, caller-owned; they must stay valid, and x untouched, until mm_poll reports the
 * result).  Non-blocking; *ticket identifies the request.  The plan stays cached while the
 * request is queued or running.  Errors: MM_ERR_NOT_FOUND (key not cached), MM_ERR_INVALID,
 * MM_ERR_BUDGET (plan + workspace can never fit the budget). */
mm_status mm_submit(mm_server_t* server, uint64_t key, const float* d, int32_t k, int64_t ld_d,
                    double* x, const mm_solve_opts* opts, uint64_t* ticket);

/* MM_PENDING while the request is queued or running.  Otherwise the solve's status (as
 * mm_pcg_solve), with info (HOST, k entries, may be NULL) and times (may be NULL) filled; the
 * ticket is released by that call.  MM_ERR_NOT_FOUND for an unknown or released ticket. */
mm_status mm_poll(mm_server_t* server, uint64_t ticket, mm_solve_info* info,
                  mm_request_times* times);

/* Like mm_poll but blocks until the request has finished. */
mm_status mm_wait(mm_server_t* server, uint64_t ticket, mm_solve_info* info,
                  mm_request_times* times);

mm_status mm_server_stats(mm_server_t* server, mm_server_stats_t* out);

const char* mm_status_string(mm_status s);
const char* mm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MM_H */
