// Preconditioned conjugate gradient (Alg. 1) on the device.
//
// Per iteration: q = A p (un-pointing, Toeplitz product, pointing), then three pixel-domain
// kernels:
//   k_dot_pq     partial sums of <p, q>
//   k_update     alpha = <r, z> / <p, q> from those partials (breakdown flag when <p, q> <= 0),
//                x += alpha p, r -= alpha q, z = M_BD r, q = 0; partials of ||r||^2, <r, z>
//                (the two-level preconditioner then replaces z and its <r, z> partials)
//   k_direction  the stop test ||r|| < eps ||b||, the iteration count and beta = <r', z'> /
//                <r, z> from those partials, then p = z + beta p
// All scalars live in a device CgState and all reductions are FP64 with a fixed summation
// order (deterministic): each workgroup that needs a scalar sums all partials of the previous
// kernel in index order, so every workgroup holds the same value.  Every kernel returns at once
// when the state's `done` flag is set, so iterations can be queued (or replayed from a captured
// graph) in chunks and the host only reads the state between chunks.  Zeroing is done by
// kernels (no memset nodes in graphs).
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

// Scalars of the recurrence: every workgroup of the kernel that needs alpha or beta sums the
// previous kernel's per-workgroup partials itself, in the same fixed order, so all of them hold
// the same value (the kernel boundary makes the partials visible; no fence or counter).
// Workgroup 0 alone records the scalars in the state; the state fields that the other
// workgroups read in that kernel were written one kernel earlier.

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
    st->iter_next = 0;
    st->rz_prev = 0.0;
    if (bb == 0.0 || rr < st->tol2bb) {
      st->done = 1;
    } else if (!(rz > 0.0)) {
      st->done = 2;
    } else {
      st->done = 0;
    }
  }
}

// Partial slots: ||r||^2 at [0, nrb), <r, z> at [nrb, 2 nrb), <p, q> at [2 nrb, 3 nrb).
// <p, q> partials.
__global__ __launch_bounds__(kThreads) void k_dot_pq(const double* __restrict__ p,
                                                     const double* __restrict__ q, int64_t n,
                                                     double* partial, const CgState* st,
                                                     int nrb) {
  __shared__ double sh[kThreads / 64];
  if (st->done) return;
  double v = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads)
    v += p[i] * q[i];
  const double s = block_sum(v, sh);
  if (threadIdx.x == 0) partial[2 * nrb + blockIdx.x] = s;
}

// alpha = <r, z> / <p, q> from the <p, q> partials, then x += alpha p, r -= alpha q,
// z = M_BD r, q = 0, with the partials of ||r||^2 and <r, z>.
__global__ __launch_bounds__(kThreads) void k_update(const double* __restrict__ minv, double* x,
                                                     double* r, double* z,
                                                     const double* __restrict__ p, double* q,
                                                     int64_t n_kept, double* partial, int nrb,
                                                     CgState* st) {
  __shared__ double sh[kThreads / 64];
  __shared__ double s_pq;
  if (st->done) return;
  const double pq0 = reduce_partials(partial + 2 * nrb, nrb, sh);
  if (threadIdx.x == 0) s_pq = pq0;
  __syncthreads();
  const double pq = s_pq;
  if (!(pq > 0.0)) {  // the same test in every workgroup
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->pq = pq;
      st->done = 2;
    }
    return;
  }
  const double alpha = st->rz / pq;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->pq = pq;
    st->alpha = alpha;
    st->rz_prev = st->rz;
    st->iter_next = st->iter + 1;
  }
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

// The stop test and beta = <r', z'> / <r, z> from the ||r||^2 and <r, z> partials, then
// p = z + beta p.  Workgroup 0 writes the iteration's outcome; a workgroup that starts after it
// has set `done` skips, as it would have after the same test.
__global__ __launch_bounds__(kThreads) void k_direction(const double* __restrict__ z, double* p,
                                                        int64_t n, const double* partial,
                                                        int nrb, CgState* st) {
  __shared__ double sh[kThreads / 64];
  __shared__ double s_rr, s_rz;
  if (st->done) return;
  const double rr0 = reduce_partials(partial, nrb, sh);
  const double rz0 = reduce_partials(partial + nrb, nrb, sh);
  if (threadIdx.x == 0) {
    s_rr = rr0;
    s_rz = rz0;
  }
  __syncthreads();
  const double rr = s_rr, rz = s_rz;
  const int iter = st->iter_next;
  int done = 0;
  if (rr < st->tol2bb) {
    done = 1;
  } else if (iter >= st->max_iter) {
    done = 3;
  } else if (!(rz > 0.0)) {
    done = 2;
  }
  const double beta = done ? 0.0 : rz / st->rz_prev;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->iter = iter;
    st->rr = rr;
    if (done) {
      st->done = done;
    } else {
      st->beta = beta;
      st->rz = rz;
    }
  }
  if (done) return;
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

// out = a - q (q may be null: out = a), partials of ||out||^2 per workgroup.
__global__ __launch_bounds__(kThreads) void k_sub_norm(const double* __restrict__ a,
                                                       const double* __restrict__ q,
                                                       double* __restrict__ out, int64_t n,
                                                       double* partial) {
  __shared__ double sh[kThreads / 64];
  double v = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    const double r = q != nullptr ? a[i] - q[i] : a[i];
    if (out != nullptr) out[i] = r;
    v += r * r;
  }
  const double s = block_sum(v, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_add(double* __restrict__ x,
                                                  const double* __restrict__ dx, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads)
    x[i] += dx[i];
}

// One PCG iteration (all launches gated by state->done).  With the two-level preconditioner,
// z = M_2lvl r replaces the block-Jacobi z of k_update (and its <r, z> partials) before beta.
mm_status iteration(Plan* P, Work& W, double* x, bool two_level, hipStream_t s) {
  const int32_t* done = &W.state->done;
  const int nrb = W.nrb;
  const int64_t nk = P->n_kept;
  if (P->n_poly > 0) {
    MM_TRY(launch_template_apply(P, W.p, nullptr, W.q, done, s));  // q was zeroed by k_update
  } else if (P->lambda_max == 0) {
    MM_TRY(launch_diag_apply(P, W.p, nullptr, W.q, done, s));  // q was zeroed by k_update
  } else if (P->precision == MM_PRECISION_FP64) {
    // synchronous and not gated by `done`: such plans run one iteration per host check
    MM_TRY(exact_product(P, W.p, nullptr, W.q, s));
  } else if (P->algo == MM_TOEPLITZ_FFT && P->fused) {
    MM_TRY(launch_apply_fused(P, W.p, nullptr, W.q, done, s, W.scratch));
  } else {
    MM_TRY(launch_unpoint(P, W.p, W.t, done, s));
    MM_TRY(launch_noise_weight(P, W.t, W.u, W.scratch, done, s));
    MM_TRY(launch_point(P, W.u, W.q, false, done, s));
  }
  TimedLaunch tl(P, K_CG, s);
  hipLaunchKernelGGL(k_dot_pq, dim3(nrb), dim3(kThreads), 0, s, W.p, W.q, 3 * nk, W.partial,
                     W.state, nrb);
  hipLaunchKernelGGL(k_update, dim3(nrb), dim3(kThreads), 0, s, P->minv, x, W.r, W.z, W.p, W.q,
                     nk, W.partial, nrb, W.state);
  // z = M_2lvl r and its <r, z> partials replace those of the block-Jacobi z
  if (two_level) MM_TRY(deflation_apply(P, W.r, W.z, nullptr, W.partial, nrb, done, s));
  hipLaunchKernelGGL(k_direction, dim3(nrb), dim3(kThreads), 0, s, W.z, W.p, 3 * nk, W.partial,
                     nrb, W.state);
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
  if (P->n_poly > 0) {
    MM_TRY(launch_zero(b, 3 * P->n_kept, s));
    return launch_template_apply(P, nullptr, d, b, nullptr, s);
  }
  if (P->lambda_max == 0) {
    MM_TRY(launch_zero(b, 3 * P->n_kept, s));
    return launch_diag_apply(P, nullptr, d, b, nullptr, s);
  }
  if (P->precision == MM_PRECISION_FP64) return exact_product(P, nullptr, d, b, s);
  if (P->algo == MM_TOEPLITZ_FFT && P->fused) {
    MM_TRY(launch_zero(b, 3 * P->n_kept, s));
    return launch_apply_fused(P, nullptr, d, b, nullptr, s, W.scratch);
  }
  MM_TRY(launch_mask_data(P, d, W.t, s));
  MM_TRY(launch_noise_weight(P, W.t, W.u, W.scratch, nullptr, s));
  return launch_point(P, W.u, b, true, nullptr, s);
}

mm_status apply_A(Plan* P, Work& W, const double* x, double* y, const int32_t* done,
                  hipStream_t s) {
  if (P->n_poly > 0) {
    MM_TRY(launch_zero(y, 3 * P->n_kept, s));
    return launch_template_apply(P, x, nullptr, y, done, s);
  }
  if (P->lambda_max == 0) {
    MM_TRY(launch_zero(y, 3 * P->n_kept, s));
    return launch_diag_apply(P, x, nullptr, y, done, s);
  }
  if (P->precision == MM_PRECISION_FP64) return exact_product(P, x, nullptr, y, s);
  if (P->algo == MM_TOEPLITZ_FFT && P->fused) {
    MM_TRY(launch_zero(y, 3 * P->n_kept, s));
    return launch_apply_fused(P, x, nullptr, y, done, s, W.scratch);
  }
  MM_TRY(launch_unpoint(P, x, W.t, done, s));
  MM_TRY(launch_noise_weight(P, W.t, W.u, W.scratch, done, s));
  MM_TRY(launch_point(P, W.u, y, true, done, s));
  return MM_OK;
}

mm_status apply_A_multi(Plan* P, Work& W, const double* x, int64_t ldx, double* y, int64_t ldy,
                        int32_t ncol, hipStream_t s) {
  if (ncol <= 0 || P->n_kept == 0) return MM_OK;
  if (P->lambda_max != 0 && P->algo == MM_TOEPLITZ_FFT && P->fused &&
      P->precision == MM_PRECISION_MIXED) {
    if (ldy == 3 * P->n_kept) {
      MM_TRY(launch_zero(y, ncol * ldy, s));  // the columns are contiguous: one launch
    } else {
      for (int32_t j = 0; j < ncol; ++j) MM_TRY(launch_zero(y + j * ldy, 3 * P->n_kept, s));
    }
    return launch_apply_fused(P, x, nullptr, y, nullptr, s, W.scratch, ncol, ldx, ldy);
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
  // FP64 plans: their product is synchronous and not gated by the stop flag, so the host checks
  // after every iteration and nothing is captured
  const bool one_by_one = P->precision == MM_PRECISION_FP64 && P->lambda_max > 0;
  int chunk = one_by_one ? 1 : (prm.check_every > 0 ? prm.check_every : 4);
  // Graphs of `chunk` iterations are kept in the workspace and replayed by later solves with the
  // same solution vector: capturing and instantiating one costs more than a tiny solve's eager
  // launches, so a key's first chunk runs eagerly and its second use captures the graph.
  // A workspace without a cache captures every time and destroys its graphs on return.
  const bool use_graph = prm.use_graph && !P->timing.enabled && !one_by_one;
  const uint64_t defl_gen = prm.two_level ? P->defl.gen : 0;
  hipGraphExec_t gexec = nullptr;  // the graph being replayed (null: eager launches)
  hipGraphExec_t owned = nullptr;  // instantiated here and not cached
  int graph_chunk = 0;
  struct GraphGuard {
    hipGraphExec_t* e;
    ~GraphGuard() {
      if (*e) {
        std::unique_lock<std::shared_mutex> lock(alloc_gate());
        (void)hipGraphExecDestroy(*e);
      }
    }
  } gg{&owned};
  auto capture = [&](hipGraphExec_t* out) -> mm_status {
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
      ie = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
    }
    if (ie != hipSuccess) {
      *out = nullptr;
      return fail(MM_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(ie));
    }
    return MM_OK;
  };
  int queued = 0;
  const int32_t tag_base = P->timing.next_tag;
  while (true) {
    MM_HIP_TRY(hipMemcpyAsync(W.h_state, W.state, sizeof(CgState), hipMemcpyDeviceToHost, s));
    MM_HIP_TRY(hipStreamSynchronize(s));
    if (W.h_state->done) break;
    if (queued >= prm.max_iter + 1) break;  // safety: the device stops at max_iter
    // the stream is idle from here to the launches below: a graph destroyed or evicted here
    // is not in flight
    if (use_graph && graph_chunk != chunk) {
      gexec = nullptr;
      graph_chunk = chunk;
      if (W.cache_graphs) {
        GraphSlot* hit = nullptr;
        for (GraphSlot& g : W.graphs)
          if (g.used && g.x == x && g.chunk == chunk && g.two_level == prm.two_level &&
              g.defl_gen == defl_gen)
            hit = &g;
        if (hit == nullptr) {
          // first use of this key: remember it (an unused slot, else the least recently used
          // one) and run the chunk eagerly
          hit = &W.graphs[0];
          for (GraphSlot& g : W.graphs) {
            if (!g.used) {
              hit = &g;
              break;
            }
            if (g.last_use < hit->last_use) hit = &g;
          }
          if (hit->exec) {
            std::unique_lock<std::shared_mutex> lock(alloc_gate());
            (void)hipGraphExecDestroy(hit->exec);
          }
          *hit = GraphSlot{true, nullptr, x, chunk, prm.two_level, defl_gen, ++W.graph_clock};
        } else {
          if (hit->exec == nullptr) MM_TRY(capture(&hit->exec));
          hit->last_use = ++W.graph_clock;
          gexec = hit->exec;
        }
      } else {
        if (owned) {
          std::unique_lock<std::shared_mutex> lock(alloc_gate());
          const hipError_t de = hipGraphExecDestroy(owned);
          owned = nullptr;
          if (de != hipSuccess) return fail(MM_ERR_HIP, std::string("graph destroy: ") + hipGetErrorString(de));
        }
        MM_TRY(capture(&owned));
        gexec = owned;
      }
    }
    if (gexec != nullptr) {
      MM_HIP_TRY(hipGraphLaunch(gexec, s));
    } else {
      for (int i = 0; i < chunk; ++i) {
        if (P->timing.enabled) P->timing.tag = tag_base + queued + i + 1;
        MM_TRY(iteration(P, W, x, prm.two_level, s));
      }
      if (P->timing.enabled) P->timing.tag = 0;
    }
    queued += chunk;
    if (prm.check_every <= 0 && chunk < 16 && !one_by_one) chunk *= 2;
  }
  *out = *W.h_state;
  if (P->timing.enabled) {
    timing_drop_range(P, tag_base + out->iter + 1, tag_base + queued);
    P->timing.next_tag = tag_base + queued + 1;
  }
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

namespace {

// ||a - q||^2 (q may be null) into *out, with out_vec = a - q when given.  Synchronous.
mm_status sub_norm2(Work& W, const double* a, const double* q, double* out_vec, int64_t n,
                    double* out, hipStream_t s) {
  const int nrb = W.nrb;
  hipLaunchKernelGGL(k_sub_norm, dim3(nrb), dim3(kThreads), 0, s, a, q, out_vec, n, W.partial);
  hipLaunchKernelGGL(k_reduce_to, dim3(1), dim3(kThreads), 0, s, &W.state->spare, W.partial, nrb);
  MM_HIP_TRY(hipGetLastError());
  MM_HIP_TRY(hipMemcpyAsync(&W.h_state->spare, &W.state->spare, sizeof(double),
                            hipMemcpyDeviceToHost, s));
  MM_HIP_TRY(hipStreamSynchronize(s));
  *out = W.h_state->spare;
  return MM_OK;
}

template <class T>
struct DevVec {
  T* p = nullptr;
  ~DevVec() { dev_free(p); }
  mm_status alloc(size_t n) {
    const hipError_t e = dev_malloc(reinterpret_cast<void**>(&p), n * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      return fail(MM_ERR_OOM, std::string("hipMalloc (refinement): ") + hipGetErrorString(e));
    }
    return MM_OK;
  }
};

}  // namespace

// FP64 true residual of x, and up to max_steps refinement updates: r = b - A x with b and A in
// FP64; inner PCG with the plan's own product on A dx = r to the relative tolerance that
// brings ||r|| under tol ||b|| with a factor 2 to spare; x += dx.  Stops when the FP64
// residual is below tol.  *rel64 is the FP64 relative residual of the returned x.
// r = b - A x in FP64 (Eq. CGresidual), and refinement steps on it.  Where the FP64 product
// takes the time-domain residual, r = P^T N^-1 (d - P x) is one product (no cancellation
// between two large vectors) and ||b|| is that of the solve's right-hand side (its FP32
// time-domain rounding moves the ratio by ~1e-7 of itself); otherwise r is the FP64
// right-hand side minus the FP64 product, relative to the FP64 right-hand side.
mm_status refine_fp64(Plan* P, Work& W, const float* d, double* x, const PcgParams& outer,
                      int32_t max_steps, double bb_solve, hipStream_t s, double* rel64,
                      int32_t* steps, int32_t* inner_its, double* rel_first) {
  const int64_t nu = 3 * P->n_kept;
  const bool one_product = exact_residual_supported(P);
  DevVec<double> b64, dx;
  double bb = bb_solve;
  if (!one_product) {
    MM_TRY(b64.alloc(static_cast<size_t>(nu)));
    MM_TRY(exact_product(P, nullptr, d, b64.p, s));
    MM_TRY(sub_norm2(W, b64.p, nullptr, nullptr, nu, &bb, s));
  }
  *steps = 0;
  *inner_its = 0;
  *rel_first = 0.0;
  if (!(bb > 0.0)) {
    *rel64 = 0.0;
    return MM_OK;
  }
  if (max_steps > 0) MM_TRY(dx.alloc(static_cast<size_t>(nu)));
  while (true) {
    double rr = 0.0;
    if (one_product) {
      MM_TRY(exact_product(P, x, d, W.b, s));  // W.b = r = P^T N^-1 (d - P x)
      MM_TRY(sub_norm2(W, W.b, nullptr, nullptr, nu, &rr, s));
    } else {
      MM_TRY(exact_product(P, x, nullptr, W.q, s));
      MM_TRY(sub_norm2(W, b64.p, W.q, W.b, nu, &rr, s));  // W.b = r = b - A x
    }
    *rel64 = std::sqrt(rr / bb);
    if (*steps == 0) *rel_first = *rel64;
    if (*rel64 < outer.tol || *steps >= max_steps) break;
    PcgParams inner = outer;
    inner.use_x0 = false;
    inner.two_level = outer.two_level;
    inner.tol = std::min(0.5, std::max(1e-6, 0.5 * outer.tol / *rel64));
    CgState st{};
    MM_TRY(pcg_iterate(P, W, dx.p, inner, s, &st));
    *inner_its += st.iter;
    if (st.done == 2) return fail(MM_ERR_NOT_SPD, "refinement PCG breakdown");
    int64_t g = (nu + kThreads - 1) / kThreads;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_add, dim3(static_cast<unsigned>(g)), dim3(kThreads), 0, s, x, dx.p, nu);
    MM_HIP_TRY(hipGetLastError());
    *steps += 1;
  }
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

  // FP64 true residual (Eq. CGresidual) and iterative refinement for mixed-precision plans.
  const bool fp64_products = P->precision == MM_PRECISION_FP64 || P->lambda_max == 0;
  const bool run_refine = st.bb > 0.0 && (opts.refine > 0 || (opts.check_fp64 && !fp64_products));
  if (run_refine && alloc_free) return fail(MM_ERR_UNSUPPORTED, "FP64 check or refinement allocates");
  // True residual of the PCG iterate with one more product: the FP64 residual that the check
  // or refinement forms first when its FP64 product takes the time-domain residual, else the
  // plan's own product.
  const bool true_from_fp64 = run_refine && exact_residual_supported(P);
  double true_rr = 0.0;
  if (st.bb > 0.0 && !true_from_fp64) MM_TRY(residual_norm2(P, W, x, &true_rr, s));
  double rel64 = -1.0, rel_first = 0.0;
  int32_t steps = 0, inner_its = 0;
  if (run_refine) {
    MM_TRY(refine_fp64(P, W, d, x, prm, opts.refine > 0 ? opts.refine : 0, st.bb, s, &rel64,
                       &steps, &inner_its, &rel_first));
    if (true_from_fp64) true_rr = rel_first * rel_first * st.bb;
  } else if (opts.check_fp64 && st.bb > 0.0) {
    rel64 = std::sqrt(true_rr / st.bb);  // the products are FP64 already
  } else if (opts.refine > 0 || opts.check_fp64) {
    rel64 = 0.0;  // b = 0
  }
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
    info->refine_steps = steps;
    info->true_relres64 = rel64;
    info->inner_iterations = inner_its;
    info->pad0 = 0;
    if (opts.refine > 0 && rel64 >= 0.0) info->converged = rel64 < prm.tol ? 1 : 0;
  }
  if (st.done == 2) return fail(MM_ERR_NOT_SPD, "PCG breakdown: p^T A p <= 0 or r^T z <= 0");
  if (opts.refine > 0 && rel64 >= prm.tol)
    return fail(MM_ERR_NO_CONV, "refinement did not bring the FP64 true residual under tol");
  if (st.done != 1) return fail(MM_ERR_NO_CONV, "PCG reached max_iter without converging");
  return MM_OK;
}

}  // namespace mm
