// Stacked right-hand sides solved together by the enlarged-CG recurrences (Alg. 2, Orthomin
// variant) applied to t right-hand sides that share P and N^-1:
//
//   R = B, Z = M R;  repeat:  W = A Z (one multi-column product), G = Z^T W, H1 = Z^T R,
//   X += Z G^+ H1,  R -= W G^+ H1,  stop columns with ||R_j|| < eps ||B_j||,
//   Z <- M R - Z G^+ (W^T M R)
//
// (P_k = Z G^-1/2 folds into G^+ = G^-1/2 G^-1/2).  G^+ is an FP64 eigen pseudo-inverse that
// drops directions below 1e-12 of the largest eigenvalue, a safeguard against the rank loss of
// the search block (the paper's Cholesky square root has none).  Converged columns leave the
// block (their X is final).  The t x t algebra runs on the host in FP64; the tall-skinny Gram
// products, updates and the block-Jacobi apply run in the kernels below, in FP64.
//
// Block size: opts->block >= 2 fixes t; opts->block < 0 tunes it: the first column groups are
// solved with t = 1 (8 columns, each alone by Alg. 1), 8, 16, 32 in turn (real work, not a
// rehearsal); the candidate with the lowest time per right-hand side then solves the remaining
// columns and is kept in the plan and, for the life of the process, for plans of the same
// shape, so later tuned solves start with it.  When
// the stacked recurrences do not shorten the iteration enough to pay for their extra
// tall-skinny work, t = 1 wins.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <mutex>
#include <numeric>
#include <tuple>

#include "mm_internal.h"

namespace mm {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxT = 32;

// Gram partials partial[x][i * tv + j] = sum over workgroup x's rows of U_i[r] V_j[r], streamed:
// workgroup (x, y) takes the 8 x 8 block y of column pairs and
// a grid-stride share of the rows; each thread keeps its 64 pair sums in registers over all its
// rows (8 + 8 coalesced loads and 64 FMAs per row, no barrier in the loop), then the workgroup
// reduces them once (wavefront shuffles, then LDS across the 4 wavefronts) in a fixed order.
// (A tiled form that staged 64-row tiles of U and V in LDS waited on memory at every tile and
// took ~160 us per call for t = 8.)
constexpr int kGB = 8;

// Two products against the same U in one launch: pair blocks y < nb1 belong to U^T V1, the
// rest to U^T V2 (tv2 = 0: one product); partial[x] holds the tu x tv1 entries, then the
// tu x tv2 entries.
__global__ __launch_bounds__(kThreads) void k_gram_rb(const double* __restrict__ U, int tu,
                                                      int64_t ldu, const double* __restrict__ V1,
                                                      int tv1, const double* __restrict__ V2,
                                                      int tv2, int64_t ldv, int64_t n,
                                                      double* __restrict__ partial) {
  __shared__ double red[kThreads / 64][kGB * kGB];
  const int nbu = (tu + kGB - 1) / kGB;
  const int nb1 = nbu * ((tv1 + kGB - 1) / kGB);
  const bool second = static_cast<int>(blockIdx.y) >= nb1;
  const double* __restrict__ V = second ? V2 : V1;
  const int tv = second ? tv2 : tv1;
  const int yb = second ? static_cast<int>(blockIdx.y) - nb1 : static_cast<int>(blockIdx.y);
  const int64_t off = second ? static_cast<int64_t>(tu) * tv1 : 0;
  const int nbv = (tv + kGB - 1) / kGB;
  const int i0 = (yb / nbv) * kGB, j0 = (yb % nbv) * kGB;
  const int nu = min(kGB, tu - i0), nv = min(kGB, tv - j0);
  double acc[kGB][kGB];
#pragma unroll
  for (int a = 0; a < kGB; ++a)
#pragma unroll
    for (int b = 0; b < kGB; ++b) acc[a][b] = 0.0;
  for (int64_t r = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; r < n;
       r += static_cast<int64_t>(gridDim.x) * kThreads) {
    double u[kGB], v[kGB];
#pragma unroll
    for (int a = 0; a < kGB; ++a) u[a] = a < nu ? U[(i0 + a) * ldu + r] : 0.0;
#pragma unroll
    for (int b = 0; b < kGB; ++b) v[b] = b < nv ? V[(j0 + b) * ldv + r] : 0.0;
#pragma unroll
    for (int a = 0; a < kGB; ++a)
#pragma unroll
      for (int b = 0; b < kGB; ++b) acc[a][b] = fma(u[a], v[b], acc[a][b]);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int a = 0; a < kGB; ++a)
#pragma unroll
    for (int b = 0; b < kGB; ++b) {
      double x = acc[a][b];
      for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o);
      if (lane == 0) red[wv][a * kGB + b] = x;
    }
  __syncthreads();
  if (threadIdx.x < kGB * kGB) {
    const int a = threadIdx.x / kGB, b = threadIdx.x % kGB;
    if (a < nu && b < nv) {
      double x = 0.0;
#pragma unroll
      for (int w = 0; w < kThreads / 64; ++w) x += red[w][threadIdx.x];
      partial[static_cast<int64_t>(blockIdx.x) * tu * (tv1 + tv2) + off + (i0 + a) * tv +
              (j0 + b)] = x;
    }
  }
}

// out[e] = sum_w partial[w][e] in a fixed order: kRedEntries entries per workgroup, 16 threads
// per entry each summing every 16th partial, then a fixed tree over the 16 sums (one thread per
// entry walking all partials serially took ~150 us for 512 partials)
constexpr int kRedEntries = kThreads / 16;

__global__ __launch_bounds__(kThreads) void k_gram_reduce(const double* __restrict__ partial,
                                                          int nwg, int count,
                                                          double* __restrict__ out) {
  __shared__ double red[kThreads];
  const int le = threadIdx.x >> 4, lw = threadIdx.x & 15;
  const int e = blockIdx.x * kRedEntries + le;
  double s = 0.0;
  if (e < count)
    for (int w = lw; w < nwg; w += 16) s += partial[static_cast<int64_t>(w) * count + e];
  red[threadIdx.x] = s;
  __syncthreads();
#pragma unroll
  for (int h = 8; h > 0; h >>= 1) {
    if (lw < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (lw == 0 && e < count) out[e] = red[threadIdx.x];
}

inline unsigned reduce_grid(int count) {
  return static_cast<unsigned>((count + kRedEntries - 1) / kRedEntries);
}

// The coefficient table's address, opaque to the optimiser: read inside the row loop (broadcast
// LDS reads) instead of hoisting up to t x t coefficients into registers across all rows.
__device__ __forceinline__ const double* row_coefs(const double* p) {
  asm volatile("" : "+v"(p));
  return p;
}

// X_cols[j] += sum_i Z_i a1[i][j];  R_j -= sum_i W_i a1[i][j];  rr partial of ||R_j||^2
template <int TM>
__global__ __launch_bounds__(kThreads) void k_block_update(
    const double* __restrict__ Z, const double* __restrict__ W, int tz, double* __restrict__ R,
    int ta, int64_t nu, double* __restrict__ x, const int32_t* __restrict__ cols,
    const double* __restrict__ a1, double* __restrict__ rr_partial) {
  __shared__ double sa[kMaxT * kMaxT];
  __shared__ double red[kThreads / 64][TM];
  for (int e = threadIdx.x; e < tz * ta; e += kThreads) sa[e] = a1[e];
  __syncthreads();
  double rr[TM];
#pragma unroll
  for (int j = 0; j < TM; ++j) rr[j] = 0.0;
  for (int64_t r = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; r < nu;
       r += static_cast<int64_t>(gridDim.x) * kThreads) {
    {  // X += Z a1 (one row of Z live at a time)
      double z[TM];
#pragma unroll
      for (int i = 0; i < TM; ++i) z[i] = i < tz ? Z[i * nu + r] : 0.0;
      const double* c = row_coefs(sa);
#pragma unroll
      for (int j = 0; j < TM; ++j) {
        if (j < ta) {
          double dx = 0.0;
#pragma unroll
          for (int i = 0; i < TM; ++i)
            if (i < tz) dx += z[i] * c[i * ta + j];
          x[static_cast<int64_t>(cols[j]) * nu + r] += dx;
        }
      }
    }
    {  // R -= W a1, with the norms
      double w[TM];
#pragma unroll
      for (int i = 0; i < TM; ++i) w[i] = i < tz ? W[i * nu + r] : 0.0;
      const double* c = row_coefs(sa);
#pragma unroll
      for (int j = 0; j < TM; ++j) {
        if (j < ta) {
          double dr = 0.0;
#pragma unroll
          for (int i = 0; i < TM; ++i)
            if (i < tz) dr += w[i] * c[i * ta + j];
          const double rn = R[j * nu + r] - dr;
          R[j * nu + r] = rn;
          rr[j] += rn * rn;
        }
      }
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < TM; ++j) {
    double v = rr[j];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    if (lane == 0) red[wv][j] = v;
  }
  __syncthreads();
  if (threadIdx.x < ta) {
    double s = 0.0;
    for (int q = 0; q < kThreads / 64; ++q) s += red[q][threadIdx.x];
    rr_partial[static_cast<int64_t>(blockIdx.x) * ta + threadIdx.x] = s;
  }
}

// Z_j <- MR_j - sum_i Z_i a2[i][j]  for j < tn (in place: each row reads all old Z first)
template <int TM>
__global__ __launch_bounds__(kThreads) void k_block_direction(double* __restrict__ Z, int tz,
                                                              const double* __restrict__ MR,
                                                              int tn, int64_t nu,
                                                              const double* __restrict__ a2) {
  __shared__ double sa[kMaxT * kMaxT];
  for (int e = threadIdx.x; e < tz * tn; e += kThreads) sa[e] = a2[e];
  __syncthreads();
  for (int64_t r = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; r < nu;
       r += static_cast<int64_t>(gridDim.x) * kThreads) {
    double z[TM];
#pragma unroll
    for (int i = 0; i < TM; ++i) z[i] = i < tz ? Z[i * nu + r] : 0.0;
    const double* c = row_coefs(sa);
#pragma unroll
    for (int j = 0; j < TM; ++j) {
      if (j < tn) {
        double s = MR[j * nu + r];
#pragma unroll
        for (int i = 0; i < TM; ++i)
          if (i < tz) s -= z[i] * c[i * tn + j];
        Z[j * nu + r] = s;
      }
    }
  }
}

// rr_partial[wg][j] = partial sum of (B_j - Y_j)^2 (or B_j^2 when Y is null)
template <int TM>
__global__ __launch_bounds__(kThreads) void k_col_norms(const double* __restrict__ B, int t,
                                                        const double* __restrict__ Y, int64_t nu,
                                                        double* __restrict__ partial) {
  __shared__ double red[kThreads / 64][TM];
  double acc[TM];
#pragma unroll
  for (int j = 0; j < TM; ++j) acc[j] = 0.0;
  for (int64_t r = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; r < nu;
       r += static_cast<int64_t>(gridDim.x) * kThreads) {
#pragma unroll
    for (int j = 0; j < TM; ++j) {
      if (j < t) {
        const double v = B[j * nu + r] - (Y ? Y[j * nu + r] : 0.0);
        acc[j] += v * v;
      }
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < TM; ++j) {
    double v = acc[j];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    if (lane == 0) red[wv][j] = v;
  }
  __syncthreads();
  if (threadIdx.x < t) {
    double s = 0.0;
    for (int q = 0; q < kThreads / 64; ++q) s += red[q][threadIdx.x];
    partial[static_cast<int64_t>(blockIdx.x) * t + threadIdx.x] = s;
  }
}

__global__ void k_zero_cols(double* __restrict__ x, const int32_t* __restrict__ cols, int t,
                            int64_t nu) {
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < t * nu;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int j = static_cast<int>(e / nu);
    x[static_cast<int64_t>(cols[j]) * nu + (e % nu)] = 0.0;
  }
}

#define MM_TM_DISPATCH(KERNEL, t, grid, s, ...)                                             \
  do {                                                                                      \
    if ((t) <= 8)                                                                           \
      hipLaunchKernelGGL(KERNEL<8>, dim3(grid), dim3(kThreads), 0, s, __VA_ARGS__);         \
    else if ((t) <= 16)                                                                     \
      hipLaunchKernelGGL(KERNEL<16>, dim3(grid), dim3(kThreads), 0, s, __VA_ARGS__);        \
    else                                                                                    \
      hipLaunchKernelGGL(KERNEL<32>, dim3(grid), dim3(kThreads), 0, s, __VA_ARGS__);        \
  } while (0)

// ---- host-side t x t algebra (FP64) ---------------------------------------------------------

// C (n x m) = A (n x n) B (n x m), row-major
void matmul(const std::vector<double>& A, const std::vector<double>& B, int n, int m,
            std::vector<double>& C) {
  C.assign(static_cast<size_t>(n) * m, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      const double aik = A[i * n + k];
      for (int j = 0; j < m; ++j) C[i * m + j] += aik * B[k * m + j];
    }
}

struct BlockWs {
  double* R = nullptr;
  double* Z = nullptr;
  double* W = nullptr;
  double* MR = nullptr;
  double* small = nullptr;    // t x t matrices
  double* partial = nullptr;  // Gram / norm partials
  int32_t* cols = nullptr;
  int cap = 0;
  int nwg = 0;
};

// Rows per workgroup of the streamed Gram kernel: enough rows per thread that the final
// reduction is a small share of the work.
int gram_rb_grid(int64_t nu) {
  int64_t g = (nu + 16 * kThreads - 1) / (16 * kThreads);
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(g, 256)));
}

int rows_grid(int64_t nu) {
  int64_t g = (nu + kThreads - 1) / kThreads;
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(g, 1024)));
}

mm_status ensure_ws(Plan* P, BlockWs& ws, int t) {
  if (ws.cap >= t) return MM_OK;
  const int64_t nu = 3 * P->n_kept;
  for (void* p : {static_cast<void*>(ws.R), static_cast<void*>(ws.Z), static_cast<void*>(ws.W),
                  static_cast<void*>(ws.MR), static_cast<void*>(ws.small),
                  static_cast<void*>(ws.partial), static_cast<void*>(ws.cols)})
    dev_free(p);
  ws = BlockWs{};
  auto alloc = [&](void** p, size_t bytes) -> mm_status {
    if (dev_malloc(p, std::max<size_t>(bytes, 8)) != hipSuccess) {
      *p = nullptr;
      return fail(MM_ERR_OOM, "hipMalloc (block workspace) failed");
    }
    return MM_OK;
  };
  const size_t vec = sizeof(double) * static_cast<size_t>(t) * nu;
  MM_TRY(alloc(reinterpret_cast<void**>(&ws.R), vec));
  MM_TRY(alloc(reinterpret_cast<void**>(&ws.Z), vec));
  MM_TRY(alloc(reinterpret_cast<void**>(&ws.W), vec));
  MM_TRY(alloc(reinterpret_cast<void**>(&ws.MR), vec));
  MM_TRY(alloc(reinterpret_cast<void**>(&ws.small), sizeof(double) * 4 * kMaxT * kMaxT));
  ws.nwg = std::max(gram_rb_grid(nu), rows_grid(nu));
  MM_TRY(alloc(reinterpret_cast<void**>(&ws.partial),
               sizeof(double) * static_cast<size_t>(ws.nwg) * kMaxT * kMaxT));
  MM_TRY(alloc(reinterpret_cast<void**>(&ws.cols), sizeof(int32_t) * kMaxT));
  ws.cap = t;
  return MM_OK;
}

void free_ws(BlockWs& ws) {
  for (void* p : {static_cast<void*>(ws.R), static_cast<void*>(ws.Z), static_cast<void*>(ws.W),
                  static_cast<void*>(ws.MR), static_cast<void*>(ws.small),
                  static_cast<void*>(ws.partial), static_cast<void*>(ws.cols)})
    dev_free(p);
  ws = BlockWs{};
}

// Gram U^T V (tu x tv, row-major) to the host.
void launch_gram(const double* U, int tu, const double* V1, int tv1, const double* V2, int tv2,
                 int64_t nu, double* partial, int g, hipStream_t s) {
  const int nbu = (tu + kGB - 1) / kGB;
  const int nb = nbu * ((tv1 + kGB - 1) / kGB) + nbu * ((tv2 + kGB - 1) / kGB);
  hipLaunchKernelGGL(k_gram_rb, dim3(static_cast<unsigned>(g), static_cast<unsigned>(nb)),
                     dim3(kThreads), 0, s, U, tu, nu, V1, tv1, V2, tv2, nu, nu, partial);
}

mm_status gram(const double* U, int tu, const double* V, int tv, int64_t nu, BlockWs& ws,
               std::vector<double>& out, hipStream_t s) {
  const int g = gram_rb_grid(nu);
  launch_gram(U, tu, V, tv, nullptr, 0, nu, ws.partial, g, s);
  const int count = tu * tv;
  hipLaunchKernelGGL(k_gram_reduce, dim3(reduce_grid(count)), dim3(kThreads), 0, s, ws.partial, g,
                     count, ws.small);
  MM_HIP_TRY(hipGetLastError());
  out.resize(count);
  MM_HIP_TRY(hipMemcpyAsync(out.data(), ws.small, sizeof(double) * count, hipMemcpyDeviceToHost, s));
  MM_HIP_TRY(hipStreamSynchronize(s));
  return MM_OK;
}

// U^T V1 and U^T V2 to the host, one launch, one reduction and one synchronization.
mm_status gram_pair(const double* U, int tu, const double* V1, int tv1, const double* V2, int tv2,
                    int64_t nu, BlockWs& ws, std::vector<double>& out1, std::vector<double>& out2,
                    hipStream_t s) {
  const int g = gram_rb_grid(nu);
  const int c1 = tu * tv1, c2 = tu * tv2;
  launch_gram(U, tu, V1, tv1, V2, tv2, nu, ws.partial, g, s);
  hipLaunchKernelGGL(k_gram_reduce, dim3(reduce_grid(c1 + c2)), dim3(kThreads), 0, s, ws.partial,
                     g, c1 + c2, ws.small);
  MM_HIP_TRY(hipGetLastError());
  std::vector<double> both(c1 + c2);
  MM_HIP_TRY(hipMemcpyAsync(both.data(), ws.small, sizeof(double) * (c1 + c2),
                            hipMemcpyDeviceToHost, s));
  MM_HIP_TRY(hipStreamSynchronize(s));
  out1.assign(both.begin(), both.begin() + c1);
  out2.assign(both.begin() + c1, both.end());
  return MM_OK;
}

// Per-column ||B_j - Y_j||^2 (Y may be null) to the host.
mm_status col_norms(const double* B, const double* Y, int t, int64_t nu, BlockWs& ws,
                    std::vector<double>& out, hipStream_t s) {
  const int g = rows_grid(nu);
  MM_TM_DISPATCH(k_col_norms, t, g, s, B, t, Y, nu, ws.partial);
  hipLaunchKernelGGL(k_gram_reduce, dim3(reduce_grid(t)), dim3(kThreads), 0, s, ws.partial, g, t,
                     ws.small);
  MM_HIP_TRY(hipGetLastError());
  out.resize(t);
  MM_HIP_TRY(hipMemcpyAsync(out.data(), ws.small, sizeof(double) * t, hipMemcpyDeviceToHost, s));
  MM_HIP_TRY(hipStreamSynchronize(s));
  return MM_OK;
}

// Solve the columns `cols` (at most kMaxT) together.
mm_status solve_group(Plan* P, Work& Wk, const float* d, int64_t ld_d, double* x,
                      const std::vector<int32_t>& cols, double tol, int max_iter,
                      mm_solve_info* info, int block_used, BlockWs& ws, hipStream_t s) {
  const int t = static_cast<int>(cols.size());
  const int64_t nu = 3 * P->n_kept;
  MM_TRY(ensure_ws(P, ws, t));
  auto ev = std::chrono::steady_clock::now();

  // R_j = b_j = P^T N^-1 d_j, X_j = 0
  MM_HIP_TRY(hipMemcpyAsync(ws.cols, cols.data(), sizeof(int32_t) * t, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_zero_cols, dim3(rows_grid(t * nu)), dim3(kThreads), 0, s, x, ws.cols, t, nu);
  for (int j = 0; j < t; ++j) MM_TRY(compute_rhs(P, Wk, d + cols[j] * ld_d, ws.R + j * nu, s));
  std::vector<double> bb;
  MM_TRY(col_norms(ws.R, nullptr, t, nu, ws, bb, s));
  std::vector<double> bnorm(t);
  for (int j = 0; j < t; ++j) bnorm[j] = std::sqrt(bb[j]);

  // active slots: columns with b != 0 (others are solved by x = 0)
  std::vector<int32_t> act;           // user column of each active slot
  std::vector<int> slot_of;           // original position of each active slot
  std::vector<int> iters(t, 0), conv(t, 0);
  std::vector<double> relres(t, 0.0);
  for (int j = 0; j < t; ++j) {
    if (bnorm[j] > 0.0) {
      if (static_cast<int>(act.size()) != j)
        MM_HIP_TRY(hipMemcpyAsync(ws.R + act.size() * nu, ws.R + j * nu, sizeof(double) * nu,
                                  hipMemcpyDeviceToDevice, s));
      act.push_back(cols[j]);
      slot_of.push_back(j);
    } else {
      conv[j] = 1;
    }
  }
  int ta = static_cast<int>(act.size());
  int tz = ta;
  std::vector<double> G, H, Gi, A;
  if (ta > 0) {
    MM_TRY(launch_precond_multi(P, ws.R, ws.Z, ta, s));  // Z = M R
  }
  int k = 0;
  while (ta > 0 && k < max_iter) {
    MM_TRY(apply_A_multi(P, Wk, ws.Z, nu, ws.W, nu, tz, s));  // W = A Z
    MM_TRY(gram_pair(ws.Z, tz, ws.W, tz, ws.R, ta, nu, ws, G, H, s));  // G = Z^T W, H1 = Z^T R
    sym_pinv(G, tz, 1e-12, Gi);
    matmul(Gi, H, tz, ta, A);                              // a1 = G^+ H1  (tz x ta)
    MM_HIP_TRY(hipMemcpyAsync(ws.cols, act.data(), sizeof(int32_t) * ta, hipMemcpyHostToDevice, s));
    MM_HIP_TRY(hipMemcpyAsync(ws.small + kMaxT * kMaxT, A.data(), sizeof(double) * A.size(),
                              hipMemcpyHostToDevice, s));
    const int g = rows_grid(nu);
    MM_TM_DISPATCH(k_block_update, tz, g, s, ws.Z, ws.W, tz, ws.R, ta, nu, x, ws.cols,
                   ws.small + kMaxT * kMaxT, ws.partial);
    // ||R_j||^2, then MR = M R and H2 = W^T MR for every column still in the block, read back
    // together behind one synchronization
    constexpr int kRrOff = 2 * kMaxT * kMaxT, kH2Off = kRrOff + kMaxT;
    hipLaunchKernelGGL(k_gram_reduce, dim3(reduce_grid(ta)), dim3(kThreads), 0, s, ws.partial, g,
                       ta, ws.small + kRrOff);
    MM_TRY(launch_precond_multi(P, ws.R, ws.MR, ta, s));
    const int gg = gram_rb_grid(nu);
    launch_gram(ws.W, tz, ws.MR, ta, nullptr, 0, nu, ws.partial, gg, s);
    hipLaunchKernelGGL(k_gram_reduce, dim3(reduce_grid(tz * ta)), dim3(kThreads), 0, s,
                       ws.partial, gg, tz * ta, ws.small + kH2Off);
    MM_HIP_TRY(hipGetLastError());
    std::vector<double> back(kMaxT + static_cast<size_t>(tz) * ta);
    MM_HIP_TRY(hipMemcpyAsync(back.data(), ws.small + kRrOff, sizeof(double) * back.size(),
                              hipMemcpyDeviceToHost, s));
    MM_HIP_TRY(hipStreamSynchronize(s));
    ++k;
    // stop test per column; compact R and MR to the remaining columns
    std::vector<int32_t> nact;
    std::vector<int> nslot, keep_idx;
    for (int i = 0; i < ta; ++i) {
      const int j = slot_of[i];
      const double rel = std::sqrt(std::max(back[i], 0.0)) / bnorm[j];
      relres[j] = rel;
      iters[j] = k;
      if (rel < tol) {
        conv[j] = 1;
      } else {
        if (static_cast<int>(nact.size()) != i) {
          MM_HIP_TRY(hipMemcpyAsync(ws.R + nact.size() * nu, ws.R + i * nu, sizeof(double) * nu,
                                    hipMemcpyDeviceToDevice, s));
          MM_HIP_TRY(hipMemcpyAsync(ws.MR + nact.size() * nu, ws.MR + i * nu,
                                    sizeof(double) * nu, hipMemcpyDeviceToDevice, s));
        }
        nact.push_back(act[i]);
        nslot.push_back(j);
        keep_idx.push_back(i);
      }
    }
    const int tn = static_cast<int>(nact.size());
    if (tn == 0) {
      ta = 0;
      break;
    }
    H.assign(static_cast<size_t>(tz) * tn, 0.0);  // H2 = W^T MR on the remaining columns
    for (int i = 0; i < tz; ++i)
      for (int jj = 0; jj < tn; ++jj) H[i * tn + jj] = back[kMaxT + i * ta + keep_idx[jj]];
    matmul(Gi, H, tz, tn, A);                              // a2 = G^+ H2  (tz x tn)
    MM_HIP_TRY(hipMemcpyAsync(ws.small + kMaxT * kMaxT, A.data(), sizeof(double) * A.size(),
                              hipMemcpyHostToDevice, s));
    MM_TM_DISPATCH(k_block_direction, tz, g, s, ws.Z, tz, ws.MR, tn, nu,
                   ws.small + kMaxT * kMaxT);
    MM_HIP_TRY(hipGetLastError());
    act.swap(nact);
    slot_of.swap(nslot);
    ta = tz = tn;
  }

  // true residuals ||b - A x|| (W = A X, R = b)
  std::vector<double> tr(t, 0.0);
  MM_HIP_TRY(hipMemcpyAsync(ws.cols, cols.data(), sizeof(int32_t) * t, hipMemcpyHostToDevice, s));
  for (int j = 0; j < t; ++j) {
    MM_TRY(compute_rhs(P, Wk, d + cols[j] * ld_d, ws.R + j * nu, s));
    MM_TRY(apply_A(P, Wk, x + static_cast<int64_t>(cols[j]) * nu, ws.W + j * nu, nullptr, s));
  }
  MM_TRY(col_norms(ws.R, ws.W, t, nu, ws, tr, s));
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - ev).count();
  for (int j = 0; j < t; ++j) {
    mm_solve_info& in = info[cols[j]];
    in.iterations = iters[j];
    in.converged = conv[j];
    in.relres = relres[j];
    in.bnorm = bnorm[j];
    in.true_relres = bnorm[j] > 0 ? std::sqrt(tr[j]) / bnorm[j] : 0.0;
    in.ms = ms;
    in.block = block_used;
    in.refine_steps = 0;
    in.true_relres64 = -1.0;
    in.inner_iterations = 0;
    in.pad0 = 0;
  }
  return MM_OK;
}

}  // namespace

// Pseudo-inverse of a symmetric positive semi-definite n x n matrix (row-major) by cyclic
// Jacobi eigen-decomposition; eigenvalues below rtol * largest are dropped.
void sym_pinv(const std::vector<double>& G, int n, double rtol, std::vector<double>& out,
              SymPinvInfo* info) {
  std::vector<double> a(G), v(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) v[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += a[i * n + j] * a[i * n + j];
        if (i != j) off += a[i * n + j] * a[i * n + j];
      }
    if (off <= 1e-30 * tot || tot == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[p * n + q];
        if (apq == 0.0) continue;
        const double theta = (a[q * n + q] - a[p * n + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = a[k * n + p], akq = a[k * n + q];
          a[k * n + p] = c * akp - s * akq;
          a[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = a[p * n + k], aqk = a[q * n + k];
          a[p * n + k] = c * apk - s * aqk;
          a[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {  // eigenvectors
          const double vkp = v[k * n + p], vkq = v[k * n + q];
          v[k * n + p] = c * vkp - s * vkq;
          v[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  double wmax = 0.0;
  for (int i = 0; i < n; ++i) wmax = std::max(wmax, a[i * n + i]);
  out.assign(static_cast<size_t>(n) * n, 0.0);
  if (info) *info = SymPinvInfo{0, INFINITY, wmax};
  for (int e = 0; e < n; ++e) {
    const double w = a[e * n + e];
    if (!(w > rtol * wmax) || w <= 0.0) continue;
    if (info) {
      info->rank += 1;
      info->wmin = std::min(info->wmin, w);
    }
    const double inv = 1.0 / w;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) out[i * n + j] += v[i * n + e] * inv * v[j * n + e];
  }
}


// Tuned block sizes by problem shape, kept for the life of the process: a plan rebuilt for the
// same geometry starts with the size an earlier plan found.
namespace {
struct ShapeKey {
  int64_t n_samples, n_kept;
  int32_t lambda_max, fft_n, algo, fused;
  bool operator<(const ShapeKey& o) const {
    return std::tie(n_samples, n_kept, lambda_max, fft_n, algo, fused) <
           std::tie(o.n_samples, o.n_kept, o.lambda_max, o.fft_n, o.algo, o.fused);
  }
};
std::mutex g_tuned_mu;
std::map<ShapeKey, int32_t> g_tuned;

ShapeKey shape_of(const Plan* P) {
  return ShapeKey{P->n_samples, P->n_kept, P->lambda_max, P->fft_n, P->algo, P->fused ? 1 : 0};
}
}  // namespace

mm_status block_solve(Plan* P, Work& Wk, const float* d, int32_t k, int64_t ld_d, double* x,
                      const mm_solve_opts* o, mm_solve_info* info, hipStream_t s) {
  if (o->block < 0 && P->tuned_block.load() == 0) {
    std::lock_guard<std::mutex> lock(g_tuned_mu);
    auto it = g_tuned.find(shape_of(P));
    if (it != g_tuned.end()) P->tuned_block = it->second;
  }
  const double tol = o->tol > 0 ? o->tol : 1e-8;
  const int max_iter = o->max_iter > 0 ? o->max_iter : 10000;
  std::vector<mm_solve_info> local(static_cast<size_t>(k));
  mm_solve_info* inf = info ? info : local.data();
  BlockWs ws;
  struct Guard {
    BlockWs& w;
    ~Guard() { free_ws(w); }
  } guard{ws};
  std::vector<int> candidates;
  int best = 0;
  if (o->block < 0 && P->tuned_block.load() > 0) {
    best = P->tuned_block.load();  // chosen by an earlier tuned solve on this plan
  } else if (o->block < 0) {
    candidates = {1, 8, 16, 32};  // 1: each column alone by Alg. 1
    best = candidates[0];
  } else {
    best = std::min(std::max(2, static_cast<int>(o->block)), kMaxT);
  }
  int32_t next = 0;
  size_t ci = 0;
  double best_cost = INFINITY;
  mm_solve_opts alone = *o;  // the t = 1 candidate: Alg. 1 per column
  alone.block = 0;
  alone.use_x0 = 0;
  alone.precond = 0;
  while (next < k) {
    const bool tuning = ci < candidates.size();
    const int t = tuning ? candidates[ci] : best;
    const int group = t == 1 ? kMaxT / 4 : t;  // columns per group (8 for the t = 1 candidate)
    const int n = std::min<int32_t>(group, k - next);
    std::vector<int32_t> cols(n);
    std::iota(cols.begin(), cols.end(), next);
    const auto t0 = std::chrono::steady_clock::now();
    if (t == 1) {
      for (int32_t j : cols) {
        const mm_status st = pcg_solve(P, Wk, d + j * ld_d, x + static_cast<int64_t>(j) * 3 * P->n_kept,
                                       &alone, &inf[j], s);
        if (st != MM_OK && st != MM_ERR_NO_CONV && st != MM_ERR_NOT_SPD) return st;
      }
    } else {
      MM_TRY(solve_group(P, Wk, d, ld_d, x, cols, tol, max_iter, inf, t, ws, s));
    }
    const double cost = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() / n;
    if (tuning) {
      if (n == group && cost < best_cost) {
        best_cost = cost;
        best = t;
      }
      ++ci;
      if (ci == candidates.size() && best_cost < INFINITY) {
        P->tuned_block = best;
        std::lock_guard<std::mutex> lock(g_tuned_mu);
        g_tuned[shape_of(P)] = best;
      }
    }
    next += n;
  }
  for (int j = 0; j < k; ++j) {
    if (inf[j].converged != 1) return fail(MM_ERR_NO_CONV, "block solve reached max_iter");
  }
  return MM_OK;
}

}  // namespace mm
