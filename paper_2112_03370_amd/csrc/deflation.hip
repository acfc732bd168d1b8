// Two-level a posteriori preconditioner (Eq. 2lvlDef, A-DEF1 variant; Alg. 3).
//
// Build: m steps of Lanczos on A itself from r0 = b (x0 = 0): w = A v_k - beta_k v_(k-1) with
// A v_k stored, alpha_k = <w, v_k>, w -= alpha_k v_k, beta_(k+1) = ||w||, v_(k+1) = w / beta.
// The deflation space is spanned by V_m = [v_1 .. v_m] with Z' = A V_m the stored products,
// and the coarse matrix E = V_m^T (A V_m) is formed explicitly and pseudo-inverted in FP64 on
// the host (eigen-directions below 1e-12 of the largest eigenvalue dropped).  The paper rotates
// V_m to the Ritz vectors Z = V_m X of T_m first; Q = Z E^-1 Z^T depends only on span(Z), and
// an orthogonal rotation leaves the eigen-truncation of E unchanged, so the operator below is
// the same without the rotation.
//
// Apply (once per PCG iteration, graph-capturable, done-gated), Eq. 2lvlDef0:
//   s = Z^T r (k_defl_dots: per-workgroup partials for 8 columns at a time),
//   c = E^+ s (k_defl_coef: one workgroup),
//   z = M_BD (r - Z' c) + Z c  and the partial sums of <r, z> (k_defl_apply).
#include <atomic>
#include <chrono>
#include <cmath>

#include "mm_internal.h"

namespace mm {

namespace {

constexpr int kThreads = 256;
constexpr int kDotCols = 8;      // deflation columns per workgroup in k_defl_dots
constexpr int kDotChunks = 256;  // row chunks of k_defl_dots

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  return v;
}

// Sum over the workgroup into thread 0 (fixed order).
__device__ __forceinline__ double group_sum(double v, double* sh) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kThreads / 64; ++i) s += sh[i];
  __syncthreads();
  return s;
}

// ---- Lanczos steps ----------------------------------------------------------------------------

// w = av - beta v_prev (v_prev may be null), partial <w, v>
__global__ __launch_bounds__(kThreads) void k_lz_prep(double* __restrict__ w,
                                                      const double* __restrict__ av,
                                                      const double* __restrict__ v,
                                                      const double* __restrict__ v_prev,
                                                      double beta, int64_t n,
                                                      double* __restrict__ partial) {
  __shared__ double sh[kThreads / 64];
  double acc = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    const double wi = av[i] - (v_prev ? beta * v_prev[i] : 0.0);
    w[i] = wi;
    acc += wi * v[i];
  }
  const double s = group_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// w -= alpha v, partial ||w||^2
__global__ __launch_bounds__(kThreads) void k_lz_update(double* __restrict__ w,
                                                        const double* __restrict__ v,
                                                        double alpha, int64_t n,
                                                        double* __restrict__ partial) {
  __shared__ double sh[kThreads / 64];
  double acc = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    const double wi = w[i] - alpha * v[i];
    w[i] = wi;
    acc += wi * wi;
  }
  const double s = group_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_sumsq(const double* __restrict__ v, int64_t n,
                                                    double* __restrict__ partial) {
  __shared__ double sh[kThreads / 64];
  double acc = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads)
    acc += v[i] * v[i];
  const double s = group_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_lz_scale(double* __restrict__ v, double scale,
                                                       int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads)
    v[i] *= scale;
}

__global__ __launch_bounds__(kThreads) void k_sum_to(const double* __restrict__ partial, int n,
                                                     double* __restrict__ out) {
  __shared__ double sh[kThreads / 64];
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) v += partial[i];
  const double s = group_sum(v, sh);
  if (threadIdx.x == 0) *out = s;
}

// ---- deflation apply ---------------------------------------------------------------------------

// partial[chunk][i] = sum over the chunk's rows of Z_i[row] r[row], for columns
// i in [blockIdx.y * kDotCols, +kDotCols)
__global__ __launch_bounds__(kThreads) void k_defl_dots(const double* __restrict__ Z, int m,
                                                        int64_t nu, const double* __restrict__ r,
                                                        double* __restrict__ partial,
                                                        const int32_t* __restrict__ done) {
  __shared__ double sh[kThreads / 64];
  if (done != nullptr && *done) return;
  const int i0 = blockIdx.y * kDotCols;
  double acc[kDotCols];
#pragma unroll
  for (int q = 0; q < kDotCols; ++q) acc[q] = 0.0;
  for (int64_t row = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; row < nu;
       row += static_cast<int64_t>(gridDim.x) * kThreads) {
    const double rv = r[row];
#pragma unroll
    for (int q = 0; q < kDotCols; ++q)
      if (i0 + q < m) acc[q] += Z[static_cast<int64_t>(i0 + q) * nu + row] * rv;
  }
#pragma unroll
  for (int q = 0; q < kDotCols; ++q) {
    const double s = group_sum(acc[q], sh);
    if (threadIdx.x == 0 && i0 + q < m) partial[static_cast<int64_t>(blockIdx.x) * m + i0 + q] = s;
  }
}

// s_i = sum_chunks partial[chunk][i] (fixed order); c = E^+ s
__global__ __launch_bounds__(kThreads) void k_defl_coef(const double* __restrict__ partial,
                                                        int n_chunks, int m,
                                                        const double* __restrict__ einv,
                                                        double* __restrict__ c,
                                                        const int32_t* __restrict__ done) {
  __shared__ double s[kMaxDeflation];
  __shared__ double red[kThreads];
  if (done != nullptr && *done) return;
  // s_i = sum of the chunk partials: tpe threads per entry, each summing every tpe-th chunk,
  // then a fixed tree (m <= 128, so tpe >= 2)
  int tpe = 1;
  while (tpe < 16 && 2 * tpe * m <= kThreads) tpe *= 2;
  const int e = threadIdx.x / tpe, sub = threadIdx.x % tpe;
  double v = 0.0;
  if (e < m)
    for (int k = sub; k < n_chunks; k += tpe) v += partial[static_cast<int64_t>(k) * m + e];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = tpe / 2; h > 0; h >>= 1) {
    if (sub < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (sub == 0 && e < m) s[e] = red[threadIdx.x];
  __syncthreads();
  for (int j = threadIdx.x; j < m; j += kThreads) {
    double v = 0.0;
    for (int i = 0; i < m; ++i) v += einv[j * m + i] * s[i];
    c[j] = v;
  }
}

// z = M_BD (r - Z' c) + Z c per pixel; p = z when p != null; partial[nrb + block] = <r, z>
// (the slot that the CG scalar kernels read).  Launch with exactly nrb workgroups.
__global__ __launch_bounds__(kThreads) void k_defl_apply(
    const double* __restrict__ Z, const double* __restrict__ Zp, int m, int64_t n_kept,
    const double* __restrict__ c_g, const double* __restrict__ minv, const double* __restrict__ r,
    double* __restrict__ z, double* __restrict__ p, double* __restrict__ partial, int nrb,
    const int32_t* __restrict__ done) {
  __shared__ double c[kMaxDeflation];
  __shared__ double sh[kThreads / 64];
  if (done != nullptr && *done) return;
  for (int i = threadIdx.x; i < m; i += kThreads) c[i] = c_g[i];
  __syncthreads();
  const int64_t nu = 3 * n_kept;
  double rz = 0.0;
  for (int64_t px = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; px < n_kept;
       px += static_cast<int64_t>(gridDim.x) * kThreads) {
    double t[3], add[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      t[a] = r[3 * px + a];
      add[a] = 0.0;
    }
    for (int i = 0; i < m; ++i) {
      const double ci = c[i];
      const int64_t o = static_cast<int64_t>(i) * nu + 3 * px;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        t[a] -= Zp[o + a] * ci;
        add[a] += Z[o + a] * ci;
      }
    }
    const double* m6 = minv + 6 * px;
    const double zz[3] = {m6[0] * t[0] + m6[1] * t[1] + m6[2] * t[2] + add[0],
                          m6[1] * t[0] + m6[3] * t[1] + m6[4] * t[2] + add[1],
                          m6[2] * t[0] + m6[4] * t[1] + m6[5] * t[2] + add[2]};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      z[3 * px + a] = zz[a];
      if (p != nullptr) p[3 * px + a] = zz[a];
      rz += r[3 * px + a] * zz[a];
    }
  }
  const double s = group_sum(rz, sh);
  if (threadIdx.x == 0) partial[nrb + blockIdx.x] = s;
}

int grid_rows(int64_t n) {
  int64_t g = (n + kThreads - 1) / kThreads;
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(g, 1024)));
}

// Device sum of partial[0..g) to the host.
mm_status sum_to_host(const double* partial, int g, double* dev_out, double* host_out,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_sum_to, dim3(1), dim3(kThreads), 0, s, partial, g, dev_out);
  MM_HIP_TRY(hipGetLastError());
  MM_HIP_TRY(hipMemcpyAsync(host_out, dev_out, sizeof(double), hipMemcpyDeviceToHost, s));
  MM_HIP_TRY(hipStreamSynchronize(s));
  return MM_OK;
}

}  // namespace

void deflation_free(Deflation* D) {
  for (void* p : {static_cast<void*>(D->Z), static_cast<void*>(D->Zp),
                  static_cast<void*>(D->einv), static_cast<void*>(D->partial),
                  static_cast<void*>(D->c)})
    dev_free(p);
  *D = Deflation{};
}

mm_status deflation_build(Plan* P, const float* d, int32_t m, hipStream_t s) {
  if (m < 1 || m > kMaxDeflation)
    return fail(MM_ERR_INVALID, "deflation size must be in [1, " + std::to_string(kMaxDeflation) + "]");
  const auto t_start = std::chrono::steady_clock::now();
  deflation_free(&P->defl);
  Deflation D;
  struct Guard {
    Deflation* d;
    bool keep = false;
    ~Guard() {
      if (!keep) deflation_free(d);
    }
  } guard{&D};
  const int64_t nu = 3 * P->n_kept;
  auto get = [&](double** p, size_t count) -> mm_status {
    if (dev_malloc(reinterpret_cast<void**>(p), std::max<size_t>(count, 1) * sizeof(double)) !=
        hipSuccess) {
      *p = nullptr;
      return fail(MM_ERR_OOM, "hipMalloc (deflation) failed");
    }
    D.bytes += static_cast<int64_t>(std::max<size_t>(count, 1) * sizeof(double));
    return MM_OK;
  };
  MM_TRY(get(&D.Z, static_cast<size_t>(m + 1) * nu));  // v_1 .. v_(m+1)
  MM_TRY(get(&D.Zp, static_cast<size_t>(m) * nu));
  MM_TRY(get(&D.partial, static_cast<size_t>(std::max(kDotChunks * m, 1024))));
  MM_TRY(get(&D.c, static_cast<size_t>(kMaxDeflation) + 2));
  double* scal = D.c + kMaxDeflation;  // device scalar for Lanczos reductions

  // r0 = b = P^T N^-1 d into v_1's slot, then normalize
  Work& W = P->work;
  MM_TRY(compute_rhs(P, W, d, D.Z, s));
  const int g = grid_rows(nu);
  double bb = 0.0;
  hipLaunchKernelGGL(k_sumsq, dim3(g), dim3(kThreads), 0, s, D.Z, nu, D.partial);
  MM_TRY(sum_to_host(D.partial, g, scal, &bb, s));
  const double beta1 = std::sqrt(bb);
  if (!(beta1 > 0.0)) return fail(MM_ERR_INVALID, "deflation start vector b is zero");
  hipLaunchKernelGGL(k_lz_scale, dim3(g), dim3(kThreads), 0, s, D.Z, 1.0 / beta1, nu);
  const double eps = 2.220446049250313e-16 * std::max(beta1, 1.0);
  double beta = 0.0;
  int done_steps = m;
  for (int k = 0; k < m; ++k) {
    double* v = D.Z + static_cast<int64_t>(k) * nu;
    double* av = D.Zp + static_cast<int64_t>(k) * nu;
    double* w = D.Z + static_cast<int64_t>(k + 1) * nu;
    MM_TRY(apply_A(P, W, v, av, nullptr, s));
    double alpha = 0.0, ww = 0.0;
    hipLaunchKernelGGL(k_lz_prep, dim3(g), dim3(kThreads), 0, s, w, av, v,
                       k > 0 ? v - nu : nullptr, beta, nu, D.partial);
    MM_TRY(sum_to_host(D.partial, g, scal, &alpha, s));
    hipLaunchKernelGGL(k_lz_update, dim3(g), dim3(kThreads), 0, s, w, v, alpha, nu, D.partial);
    MM_TRY(sum_to_host(D.partial, g, scal, &ww, s));
    beta = std::sqrt(std::max(ww, 0.0));
    if (beta < eps) {
      done_steps = k + 1;
      break;
    }
    if (k + 1 < m) hipLaunchKernelGGL(k_lz_scale, dim3(g), dim3(kThreads), 0, s, w, 1.0 / beta, nu);
  }
  D.m = done_steps;

  // E = V^T (A V), column by column: E[:, j] = V^T (A v_j)
  const int mm = D.m;
  std::vector<double> E(static_cast<size_t>(mm) * mm);
  std::vector<double> col(static_cast<size_t>(mm));
  const int groups = (mm + kDotCols - 1) / kDotCols;
  for (int j = 0; j < mm; ++j) {
    hipLaunchKernelGGL(k_defl_dots, dim3(kDotChunks, groups), dim3(kThreads), 0, s, D.Z, mm, nu,
                       D.Zp + static_cast<int64_t>(j) * nu, D.partial, nullptr);
    MM_HIP_TRY(hipGetLastError());
    std::vector<double> part(static_cast<size_t>(kDotChunks) * mm);
    MM_HIP_TRY(hipMemcpyAsync(part.data(), D.partial, part.size() * sizeof(double),
                              hipMemcpyDeviceToHost, s));
    MM_HIP_TRY(hipStreamSynchronize(s));
    for (int i = 0; i < mm; ++i) {
      double v = 0.0;
      for (int c = 0; c < kDotChunks; ++c) v += part[static_cast<size_t>(c) * mm + i];
      E[static_cast<size_t>(i) * mm + j] = v;
    }
  }
  for (int i = 0; i < mm; ++i)
    for (int j = 0; j < i; ++j) {
      const double a = 0.5 * (E[i * mm + j] + E[j * mm + i]);
      E[i * mm + j] = E[j * mm + i] = a;
    }
  std::vector<double> Einv;
  SymPinvInfo pi{};
  sym_pinv(E, mm, 1e-12, Einv, &pi);
  D.rank = pi.rank;
  D.e_min = pi.wmin;
  D.e_max = pi.wmax;
  MM_TRY(get(&D.einv, Einv.size()));
  MM_HIP_TRY(hipMemcpyAsync(D.einv, Einv.data(), Einv.size() * sizeof(double),
                            hipMemcpyHostToDevice, s));
  MM_HIP_TRY(hipStreamSynchronize(s));
  D.build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  static std::atomic<uint64_t> builds{0};
  D.gen = ++builds;
  guard.keep = true;
  P->defl = D;
  return MM_OK;
}

mm_status deflation_apply(Plan* P, const double* r, double* z, double* p, double* partial, int nrb,
                          const int32_t* done, hipStream_t s) {
  const Deflation& D = P->defl;
  const int64_t nu = 3 * P->n_kept;
  const int groups = (D.m + kDotCols - 1) / kDotCols;
  hipLaunchKernelGGL(k_defl_dots, dim3(kDotChunks, groups), dim3(kThreads), 0, s, D.Z, D.m, nu, r,
                     D.partial, done);
  hipLaunchKernelGGL(k_defl_coef, dim3(1), dim3(kThreads), 0, s, D.partial, kDotChunks, D.m,
                     D.einv, D.c, done);
  hipLaunchKernelGGL(k_defl_apply, dim3(nrb), dim3(kThreads), 0, s, D.Z, D.Zp, D.m, P->n_kept,
                     D.c, P->minv, r, z, p, partial, nrb, done);
  MM_HIP_TRY(hipGetLastError());
  return MM_OK;
}

}  // namespace mm
