// Preconditioned conjugate gradient (Alg. 1) on the device.
//
// Per iteration: q = A p (un-pointing, Toeplitz product, pointing), then three pixel-domain
// kernels and two one-workgroup scalar kernels:
//   k_dot_pq     partial sums of <p, q>
//   k_alpha      alpha = <r, z> / <p, q> (breakdown flag when <p, q> <= 0)
//   k_update     x += alpha p, r -= alpha q, z = M_BD r, q = 0; partials of ||r||^2, <r, z>
//   k_beta       stop test ||r|| < eps ||b||, beta = <r', z'> / <r, z>, iteration count
//   k_direction  p = z + beta p
// All scalars live in a device CgState and all reductions are FP64 with a fixed summation
// order (deterministic).  Every kernel returns at once when the state's `done` flag is set,
// so iterations can be queued (or replayed from a captured graph) in chunks and the host only
// reads the state between chunks.  Zeroing is done by kernels (no memset nodes in graphs).
#include <chrono>
#include <cmath>

#include "mm_internal.h"

namespace mm {

namespace {

constexpr int kThreads = 256;
constexpr int kPerBlock = 1024;  // elements per workgroup per grid-stride step

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kThreads / 64; ++i) s += sh[i];
  __syncthreads();
  return s;  // valid in thread 0
}

// Sum of partials[0..n) by one workgroup in a fixed order.
__device__ __forceinline__ double reduce_partials(const double* p, int n, double* sh) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) v += p[i];
  return block_sum(v, sh);
}

// z = M_BD r for pixel i of a [*, n_kept, 3] layout (minv shared across columns).
__device__ __forceinline__ void bj_apply(const double* __restrict__ m6, const double* r,
                                         double* z) {
  const double r0 = r[0], r1 = r[1], r2 = r[2];
  z[0] = m6[0] * r0 + m6[1] * r1 + m6[2] * r2;
  z[1] = m6[1] * r0 + m6[3] * r1 + m6[4] * r2;
  z[2] = m6[2] * r0 + m6[4] * r1 + m6[5] * r2;
}

__global__ __launch_bounds__(kThreads) void k_precond(const double* __restrict__ minv,
                                                      const double* r, double* z, int64_t n_kept,
                                                      int64_t n_pix_total) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n_pix_total;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    const double* m6 = minv + 6 * (i % n_kept);
    double zz[3];
    bj_apply(m6, r + 3 * i, zz);
    z[3 * i] = zz[0];
    z[3 * i + 1] = zz[1];
    z[3 * i + 2] = zz[2];
  }
}

// r = b - Ax (use_x0) or r = b; z = M r; p = z; q = 0; partials: [0] b.b, [1] r.z, [2] r.r
__global__ __launch_bounds__(kThreads) void k_init(const double* __restrict__ minv,
                                                   const double* __restrict__ b,
                                                   const double* __restrict__ ax, double* r,
                                                   double* z, double* p, double* q,
                                                   double* x, int use_x0, int64_t n_kept,
                                                   double* partial, int nrb) {
  __shared__ double sh[kThreads / 64];
  double bb = 0.0, rz = 0.0, rr = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n_kept;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    double rv[3], zv[3];
    for (int c = 0; c < 3; ++c) {
      const double bv = b[3 * i + c];
      bb += bv * bv;
      rv[c] = use_x0 ? bv - ax[3 * i + c] : bv;
      rr += rv[c] * rv[c];
    }
    bj_apply(minv + 6 * i, rv, zv);
    for (int c = 0; c < 3; ++c) {
      r[3 * i + c] = rv[c];
      z[3 * i + c] = zv[c];
      p[3 * i + c] = zv[c];
      q[3 * i + c] = 0.0;
      if (!use_x0) x[3 * i + c] = 0.0;
      rz += rv[c] * zv[c];
    }
  }
  const double s0 = block_sum(bb, sh);
  const double s1 = block_sum(rz, sh);
  const double s2 = block_sum(rr, sh);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = s0;
    partial[nrb + blockIdx.x] = s1;
    partial[2 * nrb + blockIdx.x] = s2;
  }
}

__global__ __launch_bounds__(kThreads) void k_init_state(CgState* st, const double* partial,
                                                         int nrb, double tol, int max_iter) {
  __shared__ double sh[kThreads / 64];
  const double bb = reduce_partials(partial, nrb, sh);
  const double rz = reduce_partials(partial + nrb, nrb, sh);
  const double rr = reduce_partials(partial + 2 * nrb, nrb, sh);
  if (threadIdx.x == 0) {
    st->bb = bb;
    st->rz = rz;
    st->rr = rr;
    st->tol2bb = tol * tol * bb;
    st->alpha = 0.0;
    st->beta = 0.0;
    st->pq = 0.0;
    st->iter = 0;
    st->max_iter = max_iter;
    if (bb == 0.0 || rr < st->tol2bb) {
      st->done = 1;
    } else if (!(rz > 0.0)) {
      st->done = 2;
    } else {
      st->done = 0;
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_dot_pq(const double* __restrict__ p,
                                                     const double* __restrict__ q, int64_t n,
                                                     double* partial, const CgState* st) {
  __shared__ double sh[kThreads / 64];
  if (st->done) return;
  double v = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads)
    v += p[i] * q[i];
  const double s = block_sum(v, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_alpha(CgState* st, const double* partial, int nrb) {
  __shared__ double sh[kThreads / 64];
  if (st->done) return;
  const double pq = reduce_partials(partial, nrb, sh);
  if (threadIdx.x == 0) {
    st->pq = pq;
    if (!(pq > 0.0)) {
      st->done = 2;
    } else {
      st->alpha = st->rz / pq;
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_update(const double* __restrict__ minv, double* x,
                                                     double* r, double* z,
                                                     const double* __restrict__ p, double* q,
                                                     int64_t n_kept, double* partial, int nrb,
                                                     const CgState* st) {
  __shared__ double sh[kThreads / 64];
  if (st->done) return;
  const double alpha = st->alpha;
  double rr = 0.0, rz = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n_kept;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    double rv[3], zv[3];
    for (int c = 0; c < 3; ++c) {
      const int64_t j = 3 * i + c;
      x[j] += alpha * p[j];
      rv[c] = r[j] - alpha * q[j];
      q[j] = 0.0;
      r[j] = rv[c];
      rr += rv[c] * rv[c];
    }
    bj_apply(minv + 6 * i, rv, zv);
    for (int c = 0; c < 3; ++c) {
      z[3 * i + c] = zv[c];
      rz += rv[c] * zv[c];
    }
  }
  const double s0 = block_sum(rr, sh);
  const double s1 = block_sum(rz, sh);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = s0;
    partial[nrb + blockIdx.x] = s1;
  }
}

__global__ __launch_bounds__(kThreads) void k_beta(CgState* st, const double* partial, int nrb) {
  __shared__ double sh[kThreads / 64];
  if (st->done) return;
  const double rr = reduce_partials(partial, nrb, sh);
  const double rz = reduce_partials(partial + nrb, nrb, sh);
  if (threadIdx.x == 0) {
    st->iter += 1;
    st->rr = rr;
    if (rr < st->tol2bb) {
      st->done = 1;
    } else if (st->iter >= st->max_iter) {
      st->done = 3;
    } else if (!(rz > 0.0)) {
      st->done = 2;
    } else {
      st->beta = rz / st->rz;
      st->rz = rz;
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_direction(const double* __restrict__ z, double* p,
                                                        int64_t n, const CgState* st) {
  if (st->done) return;
  const double beta = st->beta;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads)
    p[i] = z[i] + beta * p[i];
}

// partial = ||b - y||^2 per block
__global__ __launch_bounds__(kThreads) void k_resid(const double* __restrict__ b,
                                                    const double* __restrict__ y, int64_t n,
                                                    double* partial) {
  __shared__ double sh[kThreads / 64];
  double v = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    const double d = b[i] - y[i];
    v += d * d;
  }
  const double s = block_sum(v, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_reduce_to(double* out, const double* partial,
                                                        int nrb) {
  __shared__ double sh[kThreads / 64];
  const double s = reduce_partials(partial, nrb, sh);
  if (threadIdx.x == 0) *out = s;
}

// One PCG iteration (all launches gated by state->done).  With the two-level preconditioner,
// z = M_2lvl r replaces the block-Jacobi z of k_update (and its <r, z> partials) before beta.
mm_status iteration(Plan* P, Work& W, double* x, bool two_level, hipStream_t s) {
  const int32_t* done = &W.state->done;
  const int nrb = W.nrb;
  const int64_t nk = P->n_kept;
  if (P->lambda_max == 0) {
    MM_TRY(launch_diag_apply(P, W.p, nullptr, W.q, done, s));  // q was zeroed by k_update
  } else if (P->algo == MM_TOEPLITZ_FFT && P->fused) {
    MM_TRY(launch_apply_fused(P, W.p, nullptr, W.q, done, s));
  } else {
    MM_TRY(launch_unpoint(P, W.p, W.t, done, s));
    MM_TRY(launch_noise_weight(P, W.t, W.u, W.scratch, done, s));
    MM_TRY(launch_point(P, W.u, W.q, false, done, s));
  }
  TimedLaunch tl(P, K_CG, s);
  hipLaunchKernelGGL(k_dot_pq, dim3(nrb), dim3(kThreads), 0, s, W.p, W.q, 3 * nk, W.partial,
                     W.state);
  hipLaunchKernelGGL(k_alpha, dim3(1), dim3(kThreads), 0, s, W.state, W.partial, nrb);
  hipLaunchKernelGGL(k_update, dim3(nrb), dim3(kThreads), 0, s, P->minv, x, W.r, W.z, W.p,
                     W.q, nk, W.partial, nrb, W.state);
  if (two_level) MM_TRY(deflation_apply(P, W.r, W.z, nullptr, W.partial, nrb, done, s));
  hipLaunchKernelGGL(k_beta, dim3(1), dim3(kThreads), 0, s, W.state, W.partial, nrb);
  hipLaunchKernelGGL(k_direction, dim3(nrb), dim3(kThreads), 0, s, W.z, W.p, 3 * nk, W.state);
  MM_HIP_TRY(hipGetLastError());
  return MM_OK;
}

}  // namespace

mm_status launch_precond(Plan* P, const double* r, double* z, hipStream_t s) {
  // r and z may alias: each element is read (all three components) before written.
  const int64_t n = P->n_kept;
  if (n == 0) return MM_OK;
  int64_t g = (n + kThreads - 1) / kThreads;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_precond, dim3(static_cast<unsigned>(g)), dim3(kThreads), 0, s, P->minv, r,
                     z, n, n);
  MM_HIP_TRY(hipGetLastError());
  return MM_OK;
}

mm_status launch_precond_multi(Plan* P, const double* r, double* z, int32_t ncol,
                               hipStream_t s) {
  // ncol contiguous columns of 3 n_kept values each (column j at offset 3 j n_kept).
  const int64_t n = P->n_kept;
  if (n == 0 || ncol <= 0) return MM_OK;
  int64_t g = (n * ncol + kThreads - 1) / kThreads;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_precond, dim3(static_cast<unsigned>(g)), dim3(kThreads), 0, s, P->minv, r,
                     z, n, n * ncol);
  MM_HIP_TRY(hipGetLastError());
  return MM_OK;
}

mm_status compute_rhs(Plan* P, Work& W, const float* d, double* b, hipStream_t s) {
  if (P->lambda_max == 0) {
    MM_TRY(launch_zero(b, 3 * P->n_kept, s));
    return launch_diag_apply(P, nullptr, d, b, nullptr, s);
  }
  if (P->algo == MM_TOEPLITZ_FFT && P->fused) {
    MM_TRY(launch_zero(b, 3 * P->n_kept, s));
    return launch_apply_fused(P, nullptr, d, b, nullptr, s);
  }
  MM_TRY(launch_mask_data(P, d, W.t, s));
  MM_TRY(launch_noise_weight(P, W.t, W.u, W.scratch, nullptr, s));
  return launch_point(P, W.u, b, true, nullptr, s);
}

mm_status apply_A(Plan* P, Work& W, const double* x, double* y, const int32_t* done,
                  hipStream_t s) {
  if (P->lambda_max == 0) {
    MM_TRY(launch_zero(y, 3 * P->n_kept, s));
    return launch_diag_apply(P, x, nullptr, y, done, s);
  }
  if (P->algo == MM_TOEPLITZ_FFT && P->fused) {
    MM_TRY(launch_zero(y, 3 * P->n_kept, s));
    return launch_apply_fused(P, x, nullptr, y, done, s);
  }
  MM_TRY(launch_unpoint(P, x, W.t, done, s));
  MM_TRY(launch_noise_weight(P, W.t, W.u, W.scratch, done, s));
  MM_TRY(launch_point(P, W.u, y, true, done, s));
  return MM_OK;
}

mm_status apply_A_multi(Plan* P, Work& W, const double* x, int64_t ldx, double* y, int64_t ldy,
                        int32_t ncol, hipStream_t s) {
  if (ncol <= 0 || P->n_kept == 0) return MM_OK;
  if (P->lambda_max != 0 && P->algo == MM_TOEPLITZ_FFT && P->fused) {
    for (int32_t j = 0; j < ncol; ++j) MM_TRY(launch_zero(y + j * ldy, 3 * P->n_kept, s));
    return launch_apply_fused(P, x, nullptr, y, nullptr, s, ncol, ldx, ldy);
  }
  for (int32_t j = 0; j < ncol; ++j) MM_TRY(apply_A(P, W, x + j * ldx, y + j * ldy, nullptr, s));
  return MM_OK;
}

namespace {

// Host-side clock or HIP events for the solve's wall time (no events in allocation-free mode).
struct SolveClock {
  bool events = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  std::chrono::steady_clock::time_point t0;
  ~SolveClock() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
  mm_status start(bool use_events, hipStream_t s) {
    events = use_events;
    if (!events) {
      t0 = std::chrono::steady_clock::now();
      return MM_OK;
    }
    MM_HIP_TRY(hipEventCreate(&e0));
    MM_HIP_TRY(hipEventCreate(&e1));
    MM_HIP_TRY(hipEventRecord(e0, s));
    return MM_OK;
  }
  mm_status stop(hipStream_t s) {
    if (events) MM_HIP_TRY(hipEventRecord(e1, s));
    return MM_OK;
  }
  mm_status elapsed_ms(double* ms) {  // after the stream has been synchronised
    if (!events) {
      *ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      return MM_OK;
    }
    float f = 0.0f;
    MM_HIP_TRY(hipEventElapsedTime(&f, e0, e1));
    *ms = f;
    return MM_OK;
  }
};

}  // namespace

mm_status pcg_iterate(Plan* P, Work& W, double* x, const PcgParams& prm, hipStream_t s,
                      CgState* out) {
  const int nrb = W.nrb;
  const int64_t nk = P->n_kept;
  if (prm.use_x0) MM_TRY(apply_A(P, W, x, W.q, nullptr, s));
  hipLaunchKernelGGL(k_init, dim3(nrb), dim3(kThreads), 0, s, P->minv, W.b, W.q, W.r, W.z,
                     W.p, W.q, x, prm.use_x0 ? 1 : 0, nk, W.partial, nrb);
  if (prm.two_level) {
    if (P->defl.m == 0) return fail(MM_ERR_INVALID, "precond = 1 needs a deflation space");
    MM_TRY(deflation_apply(P, W.r, W.z, W.p, W.partial, nrb, nullptr, s));  // z0 = p0 = M r0
  }
  hipLaunchKernelGGL(k_init_state, dim3(1), dim3(kThreads), 0, s, W.state, W.partial, nrb,
                     prm.tol, prm.max_iter);
  MM_HIP_TRY(hipGetLastError());

  // Iterate in chunks; the host reads the state between chunks.  Launches queued past
  // convergence exit at once; with per-kernel timing on they carry their iteration number and
  // are dropped from the timings afterwards, and the launches are eager (events per launch)
  // instead of graph replays.
  int chunk = prm.check_every > 0 ? prm.check_every : 4;
  const bool use_graph = prm.use_graph && !P->timing.enabled;
  hipGraphExec_t gexec = nullptr;
  int graph_chunk = 0;
  struct GraphGuard {
    hipGraphExec_t* e;
    ~GraphGuard() {
      if (*e) {
        std::unique_lock<std::shared_mutex> lock(alloc_gate());
        (void)hipGraphExecDestroy(*e);
      }
    }
  } gg{&gexec};
  int queued = 0;
  while (true) {
    MM_HIP_TRY(hipMemcpyAsync(W.h_state, W.state, sizeof(CgState), hipMemcpyDeviceToHost, s));
    MM_HIP_TRY(hipStreamSynchronize(s));
    if (W.h_state->done) break;
    if (queued >= prm.max_iter + 1) break;  // safety: the device stops at max_iter
    if (use_graph) {
      if (gexec == nullptr || graph_chunk != chunk) {
        if (gexec) {
          std::unique_lock<std::shared_mutex> lock(alloc_gate());
          const hipError_t de = hipGraphExecDestroy(gexec);
          gexec = nullptr;
          if (de != hipSuccess) return fail(MM_ERR_HIP, std::string("graph destroy: ") + hipGetErrorString(de));
        }
        hipGraph_t graph = nullptr;
        std::shared_lock<std::shared_mutex> gate(alloc_gate());
        MM_HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        mm_status st = MM_OK;
        for (int i = 0; i < chunk && st == MM_OK; ++i) st = iteration(P, W, x, prm.two_level, s);
        hipError_t ce = hipStreamEndCapture(s, &graph);
        gate.unlock();
        if (st != MM_OK) {
          if (graph) (void)hipGraphDestroy(graph);
          return st;
        }
        if (ce != hipSuccess) return fail(MM_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(ce));
        hipError_t ie;
        {
          // instantiation may allocate device memory: keep it apart from other captures
          std::unique_lock<std::shared_mutex> lock(alloc_gate());
          ie = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
          (void)hipGraphDestroy(graph);
        }
        if (ie != hipSuccess) return fail(MM_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(ie));
        graph_chunk = chunk;
      }
      MM_HIP_TRY(hipGraphLaunch(gexec, s));
    } else {
      for (int i = 0; i < chunk; ++i) {
        if (P->timing.enabled) P->timing.tag = queued + i + 1;
        MM_TRY(iteration(P, W, x, prm.two_level, s));
      }
      if (P->timing.enabled) P->timing.tag = 0;
    }
    queued += chunk;
    if (prm.check_every <= 0 && chunk < 16) chunk *= 2;
  }
  *out = *W.h_state;
  if (P->timing.enabled) timing_drop_after(P, out->iter);
  return MM_OK;
}

mm_status residual_norm2(Plan* P, Work& W, const double* x, double* rr, hipStream_t s) {
  const int nrb = W.nrb;
  const int64_t nk = P->n_kept;
  *rr = 0.0;
  if (nk == 0) return MM_OK;
  MM_TRY(apply_A(P, W, x, W.q, nullptr, s));
  hipLaunchKernelGGL(k_resid, dim3(nrb), dim3(kThreads), 0, s, W.b, W.q, 3 * nk, W.partial);
  hipLaunchKernelGGL(k_reduce_to, dim3(1), dim3(kThreads), 0, s, &W.state->spare, W.partial,
                     nrb);
  MM_HIP_TRY(hipGetLastError());
  MM_HIP_TRY(hipMemcpyAsync(&W.h_state->spare, &W.state->spare, sizeof(double),
                            hipMemcpyDeviceToHost, s));
  MM_HIP_TRY(hipStreamSynchronize(s));
  *rr = W.h_state->spare;
  return MM_OK;
}

mm_status pcg_solve(Plan* P, Work& W, const float* d, double* x, const mm_solve_opts* o,
                    mm_solve_info* info, hipStream_t caller, bool alloc_free) {
  mm_solve_opts opts{};
  if (o) opts = *o;
  if (alloc_free) opts.use_graph = 0;  // instantiating a graph allocates
  // The legacy null stream cannot be captured: replay graphs on a plan-owned stream that
  // waits for the caller's prior work (the solve is synchronous, so no join is needed after).
  hipStream_t s = caller;
  if (caller == nullptr && opts.use_graph && !P->timing.enabled) {
    if (P->aux == nullptr) MM_HIP_TRY(hipStreamCreateWithFlags(&P->aux, hipStreamNonBlocking));
    MM_HIP_TRY(hipStreamSynchronize(caller));
    s = P->aux;
  }
  PcgParams prm;
  prm.tol = opts.tol > 0 ? opts.tol : 1e-8;
  prm.max_iter = opts.max_iter > 0 ? opts.max_iter : 10000;
  prm.use_x0 = opts.use_x0 != 0;
  prm.check_every = opts.check_every;
  prm.use_graph = opts.use_graph != 0;
  prm.two_level = opts.precond == 1;
  SolveClock clock;
  MM_TRY(clock.start(!alloc_free, s));

  // b = P^T N^-1 d
  if (P->timing.enabled) P->timing.tag = 0;
  MM_TRY(compute_rhs(P, W, d, W.b, s));
  CgState st{};
  MM_TRY(pcg_iterate(P, W, x, prm, s, &st));

  // True residual with one more product.
  double true_rr = 0.0;
  if (st.bb > 0.0) MM_TRY(residual_norm2(P, W, x, &true_rr, s));
  MM_TRY(clock.stop(s));
  MM_HIP_TRY(hipStreamSynchronize(s));
  double ms = 0.0;
  MM_TRY(clock.elapsed_ms(&ms));
  if (info) {
    info->iterations = st.iter;
    info->converged = st.done == 1 ? 1 : 0;
    info->bnorm = std::sqrt(st.bb);
    info->relres = st.bb > 0 ? std::sqrt(st.rr / st.bb) : 0.0;
    info->true_relres = st.bb > 0 ? std::sqrt(true_rr / st.bb) : 0.0;
    info->ms = ms;
    info->block = 1;
    info->refine_steps = 0;
    info->true_relres64 = -1.0;
    info->inner_iterations = 0;
    info->pad0 = 0;
  }
  if (st.done == 2) return fail(MM_ERR_NOT_SPD, "PCG breakdown: p^T A p <= 0 or r^T z <= 0");
  if (st.done != 1) return fail(MM_ERR_NO_CONV, "PCG reached max_iter without converging");
  return MM_OK;
}

}  // namespace mm
