// Internal declarations shared by the library's HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <mutex>
#include <shared_mutex>
#include <string>
#include <vector>

#include "../../include/mm.h"

namespace mm {

// ---------------------------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------------------------

void set_error(const std::string& msg);
const char* last_error_cstr();
mm_status fail(mm_status s, const std::string& msg);

#define MM_HIP_TRY(expr)                                                                 \
  do {                                                                                   \
    hipError_t e__ = (expr);                                                             \
    if (e__ != hipSuccess)                                                               \
      return ::mm::fail(MM_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e__)); \
  } while (0)

#define MM_TRY(expr)                 \
  do {                               \
    mm_status s__ = (expr);          \
    if (s__ != MM_OK) return s__;    \
  } while (0)

// ---------------------------------------------------------------------------------------------
// Plan
// ---------------------------------------------------------------------------------------------

// One overlap-save segment of the FFT Toeplitz product: outputs [out0, out0 + out_len) of the
// block [blk_start, blk_start + blk_len) with band `band`.
struct Chunk {
  int64_t out0;
  int64_t blk_start;
  int32_t blk_len;
  int32_t out_len;
  int32_t band;
  int32_t pad;
};

// Samples [start, start + len) with one diagonal weight c0 (plan-time tiles).
struct Tile {
  int64_t start;
  int32_t len;
  float c0;
};

// A template baseline (template map-making): samples [start, start + len) with the diagonal
// weight w of the stationary interval that holds them.
constexpr int kMaxTemplates = 8;
struct TBase {
  int64_t start;
  int32_t len;
  float w;
};

// Device-resident PCG scalars.
struct CgState {
  double rz;        // <r, z> of the current iterate
  double alpha;
  double beta;
  double bb;        // ||b||^2
  double rr;        // ||r||^2 of the latest iterate
  double tol2bb;    // tol^2 ||b||^2
  double pq;
  double spare;
  int32_t iter;
  int32_t done;     // 0 running, 1 converged, 2 breakdown, 3 iteration limit
  int32_t max_iter;
  int32_t iter_next;  // number of the iteration being completed (set with alpha)
  double rz_prev;     // <r, z> before the update (set with alpha), beta's denominator
};

enum KernelKind { K_UNPOINT = 0, K_TOEPLITZ = 1, K_POINT = 2, K_CG = 3, K_NKINDS = 4 };

struct TimedPair {
  hipEvent_t e0, e1;
  int32_t tag;  // PCG iteration the launch belongs to (0 = outside the loop)
};

struct Timing {
  bool enabled = false;
  int32_t tag = 0;
  int32_t next_tag = 1;  // tags of successive PCG runs do not overlap (refinement solves)
  std::vector<TimedPair> pending[K_NKINDS];
  double total_ms[K_NKINDS] = {0, 0, 0, 0};
  int64_t count[K_NKINDS] = {0, 0, 0, 0};
};


// Per-solve device workspace: time-domain buffers (unfused and direct products), long-segment
// tiles, the PCG vectors and scalars.  A plan holds one for the plain calls; a server gives every
// running request its own, so that solves on one plan can overlap.
// An instantiated graph of `chunk` PCG iterations, as captured for one solution vector and
// deflation space (the plan and workspace buffers are fixed for the workspace's life).  A key
// seen once holds no graph yet: its first chunk runs eagerly, the next use captures it.
struct GraphSlot {
  bool used = false;
  hipGraphExec_t exec = nullptr;
  const double* x = nullptr;
  int32_t chunk = 0;
  bool two_level = false;
  uint64_t defl_gen = 0;
  uint64_t last_use = 0;
};
constexpr int kGraphSlots = 8;

struct Work {
  float* t = nullptr;           // [n_samples] (only when the product is not fused)
  float* u = nullptr;
  float2* scratch = nullptr;    // long segments: one NC-point complex tile per workgroup
  double* r = nullptr;          // [3 n_kept] each
  double* z = nullptr;
  double* p = nullptr;
  double* q = nullptr;
  double* b = nullptr;
  double* partial = nullptr;    // reduction partials, 4 slots of nrb
  int32_t nrb = 0;
  CgState* state = nullptr;
  CgState* h_state = nullptr;   // pinned host mirror
  int64_t bytes = 0;
  // Iteration graphs kept across solves (workspaces from work_alloc; they are destroyed with
  // the workspace).  A workspace runs one solve at a time, always with the same plan.
  bool cache_graphs = false;
  GraphSlot graphs[kGraphSlots];
  uint64_t graph_clock = 0;
};

// Two-level preconditioner state (deflation.hip): Lanczos basis V_m (Z), the stored products
// A V_m (Zp), the pseudo-inverse of E = Z^T Zp, and scratch for its application.
constexpr int32_t kMaxDeflation = 128;

struct Deflation {
  int32_t m = 0;               // columns of Z (Lanczos steps taken)
  int32_t rank = 0;            // rank kept by the pseudo-inverse of E
  double e_min = 0.0;          // smallest kept eigenvalue of E
  double e_max = 0.0;          // largest eigenvalue of E
  double build_ms = 0.0;
  int64_t bytes = 0;
  double* Z = nullptr;         // [m + 1][3 n_kept]
  double* Zp = nullptr;        // [m][3 n_kept]
  double* einv = nullptr;      // [m][m]
  double* partial = nullptr;   // dot partials
  double* c = nullptr;         // [kMaxDeflation] coefficients + scalars
  uint64_t gen = 0;            // unique per build (0: none); keys the cached iteration graphs
};

struct Plan;
// Time-domain work vectors are needed by unfused and direct products (plan.hip).
bool needs_time_buffers(const Plan* P);
// Workgroups of the pixel-domain reductions for n_kept pixels (the partials hold 4 x that).
int32_t reduction_blocks(int64_t n_kept);
int64_t work_bytes(const Plan* P);
mm_status work_alloc(const Plan* P, Work* W);
void work_free(Work* W);

// Device allocation and release.  Allocation calls and graph captures exclude each other
// (gate_capture / gate_alloc), so that solves capturing graphs on one thread never see a
// concurrent hipMalloc / hipFree of another thread (a server runs both at once).
std::shared_mutex& alloc_gate();
hipError_t dev_malloc(void** p, size_t bytes);
void dev_free(void* p);

struct Plan {
  int device = 0;
  int64_t n_samples = 0;
  int64_t n_pix_global = 0;
  int64_t n_obs = 0;
  int64_t n_kept = 0;
  int64_t n_gap = 0;
  int32_t lambda_max = 0;
  int32_t algo = MM_TOEPLITZ_FFT;
  int32_t fft_n = 0;       // real FFT length
  int32_t n_blocks = 0;
  int32_t n_bands = 0;
  int64_t device_bytes = 0;
  int32_t precision = MM_PRECISION_MIXED;
  int32_t n_poly = 0;           // template map-making: Legendre orders per baseline
  int64_t n_baselines = 0;

  // pointing (device)
  int32_t* lpix = nullptr;  // local pixel or -1
  float* wq = nullptr;
  float* wu = nullptr;

  // pixel domain (device)
  double* minv = nullptr;   // [n_kept][6]: 00 01 02 11 12 22 of B^-1
  int32_t* hits = nullptr;  // [n_kept]
  int64_t* kept_ids = nullptr;

  // Toeplitz (device)
  float* band_coef = nullptr;   // concatenated c_0..c_lambda
  int64_t* band_off = nullptr;
  int32_t* band_ncoef = nullptr;
  float* spec = nullptr;        // [n_bands][fft_n/2 + 1], scaled for the in-kernel transform
  float2* spec_reg = nullptr;   // symbol pairs in the register FFT kernel's read order
  float4* long_pq = nullptr;    // spectrum-step coefficient pairs in the long kernel's read order
  float2* tw0 = nullptr;        // fine twiddles exp(-2 pi i m / fft_n), m < 128
  float2* tw1 = nullptr;        // coarse twiddles exp(-2 pi i 128 m / fft_n)
  Chunk* chunks = nullptr;      // FFT segments or direct tiles
  Tile* tiles = nullptr;        // <= 4096-sample tiles with their diagonal weight c_0
  int32_t n_tiles = 0;
  Tile* id_tiles = nullptr;     // the tiles of samples outside every block (weight 1)
  int32_t n_id_tiles = 0;
  bool fused = true;            // FFT path: gather + Toeplitz + scatter in one kernel
  bool reg_fft = false;         // fused 2^15 segments in the register-resident kernel
  int32_t n_cu = 0;             // compute units of the plan's device
  std::atomic<int32_t> tuned_block{0};  // block size chosen by a tuned stacked solve (0: none)
  int32_t n_chunks = 0;
  int64_t* id_seg = nullptr;    // identity segments: pairs (start, len)
  int32_t n_id_seg = 0;
  std::vector<int64_t> h_id_seg;

  // template map-making (templates.hip): baselines, pseudo-inverted kernel blocks
  // [n_baselines][n_poly][n_poly], and the tiles of samples outside every baseline
  TBase* tbases = nullptr;
  double* tkinv = nullptr;
  Tile* free_tiles = nullptr;
  int32_t n_free_tiles = 0;

  // FP64 product (exact.hip): symbol of every band at fft_n in FP64 and exp(-2 pi i k/fft_n)
  // for k < fft_n / 2, built on first use under x_mu
  double* x_spec = nullptr;
  double2* x_tw = nullptr;
  bool x_ready = false;
  std::mutex x_mu;

  Work work;                    // workspace of the plain calls (serialized by mu)
  Deflation defl;               // two-level preconditioner (built on request, under mu)
  hipStream_t aux = nullptr;    // plan-owned stream for graph replay when the caller's is null

  Timing timing;
  std::mutex mu;
};

// Drop timed launches tagged first..last (PCG iterations queued after convergence: they exit at
// once and are not kernel work).
void timing_drop_range(Plan* P, int32_t first, int32_t last);

// Allocation helper tracking plan bytes.
template <class T>
mm_status dalloc(Plan* P, T** ptr, size_t count) {
  *ptr = nullptr;
  if (count == 0) return MM_OK;
  hipError_t e = dev_malloc(reinterpret_cast<void**>(ptr), count * sizeof(T));
  if (e != hipSuccess) {
    *ptr = nullptr;
    return fail(MM_ERR_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  }
  P->device_bytes += static_cast<int64_t>(count * sizeof(T));
  return MM_OK;
}

// Timing scope: records events around launches of one kernel kind when enabled.
struct TimedLaunch {
  Plan* P;
  int kind;
  hipStream_t s;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  TimedLaunch(Plan* plan, int k, hipStream_t st);
  ~TimedLaunch();
};

// ---------------------------------------------------------------------------------------------
// Kernel launchers (all asynchronous on `s`; `done` may be null, else kernels exit when *done)
// ---------------------------------------------------------------------------------------------

mm_status launch_unpoint(Plan* P, const double* x, float* t, const int32_t* done, hipStream_t s);
mm_status launch_mask_data(Plan* P, const float* d, float* t, hipStream_t s);
mm_status launch_noise_weight(Plan* P, const float* t, float* u, float2* scratch,
                              const int32_t* done, hipStream_t s);
mm_status launch_point(Plan* P, const float* u, double* y, bool zero_first, const int32_t* done,
                       hipStream_t s);
mm_status launch_precond(Plan* P, const double* r, double* z, hipStream_t s);
mm_status launch_precond_multi(Plan* P, const double* r, double* z, int32_t ncol,
                               hipStream_t s);
// Diagonal weights (lambda_max = 0): y += P^T diag(c_0) (P x or masked d), all in FP64.
mm_status launch_diag_apply(Plan* P, const double* x, const float* d, double* y,
                            const int32_t* done, hipStream_t s);
// Same over an explicit tile list.
mm_status launch_diag_tiles(Plan* P, const Tile* tiles, int32_t n_tiles, const double* x,
                            const float* d, double* y, const int32_t* done, hipStream_t s);
// FFT path, fused: y += P^T N^-1 (P x) (d == nullptr) or y += P^T N^-1 d (x == nullptr), for
// ncol columns (x or d column j at + j ldx, y column j at + j ldy; 0 = packed defaults).
// Long segments (2^16, 2^17) need the solve's tiles.
mm_status launch_apply_fused(Plan* P, const double* x, const float* d, double* y,
                             const int32_t* done, hipStream_t s, float2* tiles,
                             int32_t ncol = 1, int64_t ldx = 0, int64_t ldy = 0);
// Register-resident variant for 2^15-sample segments with at most 2^14 outputs (apply_reg.hip).
bool apply_reg_supported(const Plan* P);
mm_status build_reg_table(Plan* P, hipStream_t s);  // after the band spectra
mm_status launch_apply_reg(Plan* P, const double* x, const float* d, int64_t ldx, double* y,
                           int64_t ldy, int32_t ncol, const int32_t* done, hipStream_t s);
mm_status launch_zero(double* y, int64_t n, hipStream_t s);

// b = P^T N^-1 d (b overwritten).
mm_status compute_rhs(Plan* P, Work& W, const float* d, double* b, hipStream_t s);

// A x -> y (y overwritten), done-gated.
mm_status apply_A(Plan* P, Work& W, const double* x, double* y, const int32_t* done,
                  hipStream_t s);
// A X -> Y for ncol columns with leading dimensions ldx, ldy (Y overwritten).
mm_status apply_A_multi(Plan* P, Work& W, const double* x, int64_t ldx, double* y, int64_t ldy,
                        int32_t ncol, hipStream_t s);
// Stacked right-hand sides by the enlarged-CG recurrences (block.hip).
mm_status block_solve(Plan* P, Work& W, const float* d, int32_t k, int64_t ld_d, double* x,
                      const mm_solve_opts* o, mm_solve_info* info, hipStream_t s);

// Pseudo-inverse of a symmetric positive semi-definite n x n matrix (row-major, host FP64) by
// cyclic Jacobi; eigenvalues <= rtol * largest are dropped (block.hip).
struct SymPinvInfo {
  int rank;
  double wmin;   // smallest kept eigenvalue
  double wmax;   // largest eigenvalue
};
void sym_pinv(const std::vector<double>& G, int n, double rtol, std::vector<double>& out,
              SymPinvInfo* info = nullptr);

// Two-level preconditioner (deflation.hip): build from d (Lanczos on A from b = P^T N^-1 d),
// release, and apply z = M_2lvl r (p = z too when p != null) writing the <r, z> partials to
// partial[nrb + block] as the CG scalar kernels expect (launch grid nrb).
mm_status deflation_build(Plan* P, const float* d, int32_t m, hipStream_t s);
void deflation_free(Deflation* D);
mm_status deflation_apply(Plan* P, const double* r, double* z, double* p, double* partial, int nrb,
                          const int32_t* done, hipStream_t s);

// FP64 band symbols at the plan's FFT length (plan.hip).
mm_status launch_band_symbol64(Plan* P, double* spec64, hipStream_t s);
// FP64 product (exact.hip): y = P^T N^-1 P x (d == nullptr), y = P^T N^-1 d (x == nullptr) or,
// with both, y = P^T N^-1 (d - P x) = b - A x (plans with exact_residual_supported only), every
// step in FP64, y overwritten.  Synchronous (staging tiles are allocated per call).
mm_status exact_product(Plan* P, const double* x, const float* d, double* y, hipStream_t s);
bool exact_residual_supported(const Plan* P);

// Template map-making (templates.hip): tables and kernel blocks at plan time (tiles: the
// plan's weight tiles, sorted, covering every sample), and y += P^T F_T P x (d == nullptr) or
// y += P^T F_T d (x == nullptr), FP64, done-gated.
mm_status build_templates(Plan* P, const mm_geometry* g, const std::vector<Tile>& tiles,
                          hipStream_t s);
mm_status launch_template_apply(Plan* P, const double* x, const float* d, double* y,
                                const int32_t* done, hipStream_t s);

// Plan construction (plan.hip).
mm_status build_plan(const mm_geometry* g, hipStream_t s, Plan** out);
void destroy_plan(Plan* P);  // releases the device memory and deletes P

// PCG (cg.hip).  alloc_free: no device or host allocation inside the call (no graphs, no
// events, no plan-owned stream); W then holds caller-provided buffers.
mm_status pcg_solve(Plan* P, Work& W, const float* d, double* x, const mm_solve_opts* o,
                    mm_solve_info* info, hipStream_t s, bool alloc_free = false);
struct PcgParams {
  double tol = 1e-8;
  int32_t max_iter = 10000;
  bool use_x0 = false;
  int32_t check_every = 0;
  bool use_graph = true;
  bool two_level = false;
};
// Alg. 1 on the right-hand side already in W.b (x in/out); the final device state is copied
// to *out.  Synchronous.
mm_status pcg_iterate(Plan* P, Work& W, double* x, const PcgParams& prm, hipStream_t s,
                      CgState* out);
// FP64 true residual and iterative refinement after a solve (cg.hip); bb_solve = ||b||^2 of
// the solve's right-hand side; *rel_first = the FP64 relative residual of the incoming x.
mm_status refine_fp64(Plan* P, Work& W, const float* d, double* x, const PcgParams& outer,
                      int32_t max_steps, double bb_solve, hipStream_t s, double* rel64,
                      int32_t* steps, int32_t* inner_its, double* rel_first);
// ||W.b - A x||^2 with the plan's product (uses W.q and the partials).  Synchronous.
mm_status residual_norm2(Plan* P, Work& W, const double* x, double* rr, hipStream_t s);

// FFT sizing helpers (toeplitz.hip).
int32_t choose_fft_size(int32_t lambda_max);
bool fft_size_supported(int32_t n);
int32_t max_direct_lambda();
// Long segments (toeplitz_long.hip): N = 2^16, 2^17 through a global tile per segment.
bool long_fft_size(int32_t n);
int32_t long_fine_size();
mm_status launch_toeplitz_long(Plan* P, const float* t, float* u, float2* scratch,
                               const int32_t* done, hipStream_t s);
mm_status build_long_table(Plan* P, hipStream_t s);  // after the band spectra
// Workgroups (and tiles) of the persistent long-segment kernels.
int32_t long_slots(const Plan* P);
// Fused long-segment product: y += P^T N^-1 (P x) or P^T N^-1 d for ncol columns (layout as
// launch_apply_fused), through `tiles` (long_slots(P) tiles of fft_n / 2 points).
mm_status launch_apply_long(Plan* P, const double* x, const float* d, int64_t ldx, double* y,
                            int64_t ldy, int32_t ncol, float2* tiles, const int32_t* done,
                            hipStream_t s);

}  // namespace mm
