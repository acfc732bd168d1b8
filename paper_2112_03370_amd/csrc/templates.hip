// Template map-making: the system product P^T F_T P with
//
//     F_T = W^-1 (I - T (T^T W^-1 T)^+ T^T W^-1)                                (Eq. defFT)
//
// for diagonal weights W^-1 and Legendre baselines (Appendix A, Eq. polytemplate): on every
// baseline interval of L samples the templates are sqrt((2k+1)/L) P_k(x_j), k < n_poly, at the
// midpoints x_j = (2j+1)/L - 1.  The orthogonalisation kernel T^T W^-1 T is block-diagonal, one
// n_poly x n_poly block per baseline, built on the device in FP64 at plan time and
// pseudo-inverted on the host (eigen-directions below 1e-12 of the largest dropped, the paper's
// SVD threshold).  A baseline lies inside one stationary interval (or outside all of them), so
// its weight w is the c_0 of that interval's band; gap samples (flagged or excised) weigh 0.
//
// The product runs as one kernel, one workgroup per baseline, every step in FP64:
//   1. t_s = (P x)_s (or the data sample), weighted v_s = w t_s; projections a_k = sum_s T_sk v_s
//      reduced over the workgroup (the time-domain projection of the templates algebra)
//   2. c = K_b^+ a
//   3. u_s = w (t_s - sum_k T_sk c_k)  (template projection subtracted); y += P^T u through the
//      wavefront run merge
// Samples of the first kCached steps of a baseline stay in registers between 1 and 3, so
// baselines of up to kCached x 2048 samples read their pointing once; longer ones re-gather the
// rest.  Samples outside every baseline get u = w t through the diagonal product.
#include <algorithm>
#include <cmath>

#include "mm_internal.h"
#include "wave_runs.h"

namespace mm {

namespace {

constexpr int kTT = 512;          // threads per workgroup
constexpr int kStep = 4 * kTT;    // samples per step (4 consecutive per lane)
constexpr int kCached = 4;        // steps kept in registers

struct TFlush {
  double* y;
  __device__ void operator()(int key, const double (&v)[3]) const {
    double* dst = y + 3 * static_cast<int64_t>(key);
    unsafeAtomicAdd(dst + 0, v[0]);
    unsafeAtomicAdd(dst + 1, v[1]);
    unsafeAtomicAdd(dst + 2, v[2]);
  }
};

// Scaled Legendre values T_k = scale_k P_k(x), k < NP, by the three-term recurrence
// k P_k = (2k - 1) x P_(k-1) - (k - 1) P_(k-2), with 1/k as a constant.
template <int NP>
__device__ __forceinline__ void legendre(double x, const double* scale, double (&T)[NP]) {
  double p0 = 1.0, p1 = x;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    double pk;
    if (k == 0) {
      pk = p0;
    } else if (k == 1) {
      pk = p1;
    } else {
      constexpr double kInv[kMaxTemplates] = {0.0, 1.0, 1.0 / 2, 1.0 / 3, 1.0 / 4, 1.0 / 5,
                                               1.0 / 6, 1.0 / 7};
      pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) * kInv[k];
      p0 = p1;
      p1 = pk;
    }
    T[k] = scale[k] * pk;
  }
}

// Samples j0 .. j0 + 3 of a baseline: pixel, weights and t = (P x)_s (or the data sample) in
// FP64; key -1 for gap samples and samples past the end.  A lane whose 4 samples lie inside the
// baseline at a 16-byte boundary loads its pointing with 16-byte loads, and since scan runs keep
// a pixel for several samples, it loads the pixel values of its first and last samples once
// each and a third pixel only when one occurs.  The sums are those of the one-sample form.
template <bool kData>
__device__ __forceinline__ void load4(const int32_t* __restrict__ lpix,
                                      const float* __restrict__ wq,
                                      const float* __restrict__ wu,
                                      const double* __restrict__ x,
                                      const float* __restrict__ d, int64_t start, int len,
                                      int j0, int (&key)[4], double (&t)[4], float (&q)[4],
                                      float (&u)[4]) {
  const int64_t g0 = start + j0;
  const bool vec = j0 + 4 <= len && (g0 & 3) == 0 &&
                   (!kData || (reinterpret_cast<uintptr_t>(d + g0) & 15u) == 0);
  if (vec) {
    const int4 k4 = *reinterpret_cast<const int4*>(lpix + g0);
    const float4 q4 = *reinterpret_cast<const float4*>(wq + g0);
    const float4 u4 = *reinterpret_cast<const float4*>(wu + g0);
    key[0] = k4.x;
    key[1] = k4.y;
    key[2] = k4.z;
    key[3] = k4.w;
    q[0] = q4.x;
    q[1] = q4.y;
    q[2] = q4.z;
    q[3] = q4.w;
    u[0] = u4.x;
    u[1] = u4.y;
    u[2] = u4.z;
    u[3] = u4.w;
    if constexpr (kData) {
      const float4 d4 = *reinterpret_cast<const float4*>(d + g0);
      t[0] = key[0] < 0 ? 0.0 : static_cast<double>(d4.x);
      t[1] = key[1] < 0 ? 0.0 : static_cast<double>(d4.y);
      t[2] = key[2] < 0 ? 0.0 : static_cast<double>(d4.z);
      t[3] = key[3] < 0 ? 0.0 : static_cast<double>(d4.w);
    } else {
      const int ka = key[0], kb = key[3];
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, b0 = 0.0, b1 = 0.0, b2 = 0.0;
      if (ka >= 0) {
        const double* m = x + 3 * static_cast<int64_t>(ka);
        a0 = m[0];
        a1 = m[1];
        a2 = m[2];
      }
      if (kb >= 0 && kb != ka) {
        const double* m = x + 3 * static_cast<int64_t>(kb);
        b0 = m[0];
        b1 = m[1];
        b2 = m[2];
      }
      bool other = false;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = key[i];
        other |= k >= 0 && k != ka && k != kb;
        const double qd = static_cast<double>(q[i]), ud = static_cast<double>(u[i]);
        const double ta = a0 + qd * a1 + ud * a2;
        const double tb = b0 + qd * b1 + ud * b2;
        t[i] = k < 0 ? 0.0 : (k == ka ? ta : tb);
      }
      if (other) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int k = key[i];
          if (k >= 0 && k != ka && k != kb) {
            const double* m = x + 3 * static_cast<int64_t>(k);
            t[i] = m[0] + static_cast<double>(q[i]) * m[1] + static_cast<double>(u[i]) * m[2];
          }
        }
      }
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int j = j0 + i;
    key[i] = -1;
    t[i] = 0.0;
    q[i] = u[i] = 0.0f;
    if (j < len) {
      const int64_t g = start + j;
      const int p = lpix[g];
      if (p >= 0) {
        key[i] = p;
        q[i] = wq[g];
        u[i] = wu[g];
        if (kData) {
          t[i] = static_cast<double>(d[g]);
        } else {
          const double* m = x + 3 * static_cast<int64_t>(p);
          t[i] = m[0] + static_cast<double>(q[i]) * m[1] + static_cast<double>(u[i]) * m[2];
        }
      }
    }
  }
}

// Projections of 4 samples onto the templates: a_k += T_k(x_j) w t_j.
template <int NP>
__device__ __forceinline__ void project4(const int (&key)[4], const double (&t)[4], int j0,
                                         double invL, double w, const double* scale,
                                         double (&a)[NP]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (key[i] < 0) continue;
    double T[NP];
    legendre<NP>(fma(2.0, static_cast<double>(j0 + i), 1.0) * invL - 1.0, scale, T);
    const double v = w * t[i];
#pragma unroll
    for (int k = 0; k < NP; ++k) a[k] = fma(T[k], v, a[k]);
  }
}

// u_j = w (t_j - sum_k T_k c_k) for 4 samples, then the pointing sums.
template <int NP>
__device__ __forceinline__ void subtract_point4(const int (&key)[4], const double (&t)[4],
                                                const float (&q)[4], const float (&u)[4],
                                                int j0, double invL, double w,
                                                const double* scale, const double (&c)[NP],
                                                double* y) {
  double v[4][3];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double r = 0.0;
    if (key[i] >= 0) {
      double T[NP];
      legendre<NP>(fma(2.0, static_cast<double>(j0 + i), 1.0) * invL - 1.0, scale, T);
      double fit = 0.0;
#pragma unroll
      for (int k = 0; k < NP; ++k) fit = fma(T[k], c[k], fit);
      r = w * (t[i] - fit);
    }
    v[i][0] = r;
    v[i][1] = static_cast<double>(q[i]) * r;
    v[i][2] = static_cast<double>(u[i]) * r;
  }
  wave_merge_runs<3>(key, v, TFlush{y});
}

template <bool kData, int NP>
__global__ __launch_bounds__(kTT) void k_template_apply(
    const int32_t* __restrict__ lpix, const float* __restrict__ wq, const float* __restrict__ wu,
    const double* __restrict__ x, const float* __restrict__ d, const TBase* __restrict__ bases,
    const double* __restrict__ kinv, double* __restrict__ y, const int32_t* __restrict__ done) {
  constexpr int n_poly = NP;
  if (done != nullptr && *done) return;
  __shared__ double red[kMaxTemplates][kTT / 64];
  __shared__ double scale[kMaxTemplates];
  __shared__ double coef[kMaxTemplates];
  const TBase B = bases[blockIdx.x];
  const int tid = threadIdx.x;
  const double invL = 1.0 / static_cast<double>(B.len);
  const double w = static_cast<double>(B.w);
  if (tid < kMaxTemplates) scale[tid] = sqrt((2.0 * tid + 1.0) * invL);
  __syncthreads();
  const int nsteps = (B.len + kStep - 1) / kStep;

  // ---- 1. gather and project ------------------------------------------------------------------
  double a[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) a[k] = 0.0;
  int ck[kCached][4];
  double ct[kCached][4];
  float cq[kCached][4], cu[kCached][4];
#pragma unroll
  for (int sidx = 0; sidx < kCached; ++sidx) {
    if (sidx < nsteps) {
      const int j0 = sidx * kStep + 4 * tid;
      load4<kData>(lpix, wq, wu, x, d, B.start, B.len, j0, ck[sidx], ct[sidx], cq[sidx], cu[sidx]);
      project4<NP>(ck[sidx], ct[sidx], j0, invL, w, scale, a);
    }
  }
  for (int sidx = kCached; sidx < nsteps; ++sidx) {
    const int j0 = sidx * kStep + 4 * tid;
    int k4[4];
    double t4[4];
    float q4[4], u4[4];
    load4<kData>(lpix, wq, wu, x, d, B.start, B.len, j0, k4, t4, q4, u4);
    project4<NP>(k4, t4, j0, invL, w, scale, a);
  }
  // workgroup sums in a fixed order
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    double v = a[k];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    if ((tid & 63) == 0) red[k][tid >> 6] = v;
  }
  __syncthreads();

  // ---- 2. c = K^+ a ---------------------------------------------------------------------------
  if (tid < kMaxTemplates) {
    double acc = 0.0;
    if (tid < n_poly) {
      const double* K = kinv + static_cast<int64_t>(blockIdx.x) * n_poly * n_poly + tid * n_poly;
      for (int k = 0; k < n_poly; ++k) {
        double ak = 0.0;
        for (int wv = 0; wv < kTT / 64; ++wv) ak += red[k][wv];
        acc = fma(K[k], ak, acc);
      }
    }
    coef[tid] = acc;
  }
  __syncthreads();
  double c[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) c[k] = coef[k];

  // ---- 3. subtract the fit, weight, point -----------------------------------------------------
#pragma unroll
  for (int sidx = 0; sidx < kCached; ++sidx) {
    if (sidx < nsteps)
      subtract_point4<NP>(ck[sidx], ct[sidx], cq[sidx], cu[sidx], sidx * kStep + 4 * tid, invL,
                          w, scale, c, y);
  }
  for (int sidx = kCached; sidx < nsteps; ++sidx) {
    const int j0 = sidx * kStep + 4 * tid;
    int k4[4];
    double t4[4];
    float q4[4], u4[4];
    load4<kData>(lpix, wq, wu, x, d, B.start, B.len, j0, k4, t4, q4, u4);
    subtract_point4<NP>(k4, t4, q4, u4, j0, invL, w, scale, c, y);
  }
}

// Pseudo-inverse of a symmetric positive semi-definite NP x NP block by cyclic Jacobi rotations
// (eigenvalues below rtol times the largest dropped), in registers: the same algorithm as the
// host routine used for the block recurrences.
template <int NP>
__device__ __forceinline__ void small_sym_pinv(double (&a)[NP][NP], double (&v)[NP][NP],
                                               double rtol, double (&out)[NP][NP]) {
#pragma unroll
  for (int i = 0; i < NP; ++i)
#pragma unroll
    for (int j = 0; j < NP; ++j) v[i][j] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i)
#pragma unroll
      for (int j = 0; j < NP; ++j) {
        tot += a[i][j] * a[i][j];
        if (i != j) off += a[i][j] * a[i][j];
      }
    if (off <= 1e-30 * tot || tot == 0.0) break;
#pragma unroll
    for (int p = 0; p < NP - 1; ++p)
#pragma unroll
      for (int q = p + 1; q < NP; ++q) {
        const double apq = a[p][q];
        if (apq == 0.0) continue;
        const double theta = (a[q][q] - a[p][p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
#pragma unroll
        for (int k = 0; k < NP; ++k) {  // columns p, q
          const double akp = a[k][p], akq = a[k][q];
          a[k][p] = c * akp - sn * akq;
          a[k][q] = sn * akp + c * akq;
        }
#pragma unroll
        for (int k = 0; k < NP; ++k) {  // rows p, q
          const double apk = a[p][k], aqk = a[q][k];
          a[p][k] = c * apk - sn * aqk;
          a[q][k] = sn * apk + c * aqk;
        }
#pragma unroll
        for (int k = 0; k < NP; ++k) {  // eigenvectors
          const double vkp = v[k][p], vkq = v[k][q];
          v[k][p] = c * vkp - sn * vkq;
          v[k][q] = sn * vkp + c * vkq;
        }
      }
  }
  double wmax = 0.0;
#pragma unroll
  for (int i = 0; i < NP; ++i) wmax = fmax(wmax, a[i][i]);
#pragma unroll
  for (int i = 0; i < NP; ++i)
#pragma unroll
    for (int j = 0; j < NP; ++j) out[i][j] = 0.0;
#pragma unroll
  for (int e = 0; e < NP; ++e) {
    const double w = a[e][e];
    if (!(w > rtol * wmax) || w <= 0.0) continue;
    const double inv = 1.0 / w;
#pragma unroll
    for (int i = 0; i < NP; ++i)
#pragma unroll
      for (int j = 0; j < NP; ++j) out[i][j] += v[i][e] * inv * v[j][e];
  }
}

// Kernel block of one baseline, K = sum_j w T(j) T(j)^T over its unflagged samples (Legendre
// templates T), and its pseudo-inverse (zero for a block of zeros), one workgroup per baseline:
// every pair (i <= k) is accumulated in the same pass over the samples, reduced across the
// workgroup, and the first thread inverts the block.
template <int NP>
__global__ __launch_bounds__(kTT) void k_template_kernel(const int32_t* __restrict__ lpix,
                                                         const TBase* __restrict__ bases,
                                                         double* __restrict__ Kinv) {
  constexpr int NPAIR = NP * (NP + 1) / 2;
  __shared__ double red[NPAIR][kTT / 64];
  __shared__ double scale[kMaxTemplates];
  const TBase B = bases[blockIdx.x];
  const int tid = threadIdx.x;
  const double invL = 1.0 / static_cast<double>(B.len);
  if (tid < kMaxTemplates) scale[tid] = sqrt((2.0 * tid + 1.0) * invL);
  __syncthreads();
  const double w = static_cast<double>(B.w);
  double acc[NPAIR];
#pragma unroll
  for (int q = 0; q < NPAIR; ++q) acc[q] = 0.0;
  for (int j = tid; j < B.len; j += kTT) {
    if (lpix[B.start + j] < 0) continue;
    double T[NP];
    legendre<NP>(fma(2.0, static_cast<double>(j), 1.0) * invL - 1.0, scale, T);
    int q = 0;
#pragma unroll
    for (int i = 0; i < NP; ++i)
#pragma unroll
      for (int k = i; k < NP; ++k, ++q) acc[q] = fma(w * T[i], T[k], acc[q]);
  }
#pragma unroll
  for (int q = 0; q < NPAIR; ++q) {
    double v = acc[q];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    if ((tid & 63) == 0) red[q][tid >> 6] = v;
  }
  __syncthreads();
  if (tid != 0) return;
  // the rotations work in registers for up to five templates, in LDS beyond (register room)
  constexpr bool kRegs = NP <= 5;
  __shared__ double lds_g[kRegs ? 1 : NP][NP], lds_v[kRegs ? 1 : NP][NP],
      lds_o[kRegs ? 1 : NP][NP];
  double reg_g[kRegs ? NP : 1][NP], reg_v[kRegs ? NP : 1][NP], reg_o[kRegs ? NP : 1][NP];
  auto& G = *reinterpret_cast<double(*)[NP][NP]>(kRegs ? &reg_g[0][0] : &lds_g[0][0]);
  auto& V = *reinterpret_cast<double(*)[NP][NP]>(kRegs ? &reg_v[0][0] : &lds_v[0][0]);
  auto& Gi = *reinterpret_cast<double(*)[NP][NP]>(kRegs ? &reg_o[0][0] : &lds_o[0][0]);
  bool zero = true;
  int q = 0;
#pragma unroll
  for (int i = 0; i < NP; ++i)
#pragma unroll
    for (int k = i; k < NP; ++k, ++q) {
      double sum = 0.0;
#pragma unroll
      for (int wv = 0; wv < kTT / 64; ++wv) sum += red[q][wv];
      G[i][k] = G[k][i] = sum;
      zero = zero && sum == 0.0;
    }
  double* out = Kinv + static_cast<int64_t>(blockIdx.x) * NP * NP;
  if (zero) {
#pragma unroll
    for (int i = 0; i < NP * NP; ++i) out[i] = 0.0;
    return;
  }
  small_sym_pinv<NP>(G, V, 1e-12, Gi);
#pragma unroll
  for (int i = 0; i < NP; ++i)
#pragma unroll
    for (int k = 0; k < NP; ++k) out[i * NP + k] = Gi[i][k];
}

}  // namespace

mm_status build_templates(Plan* P, const mm_geometry* g, const std::vector<Tile>& tiles,
                          hipStream_t s) {
  const int n_poly = g->n_poly;
  if (n_poly <= 0) return MM_OK;
  if (n_poly > kMaxTemplates)
    return fail(MM_ERR_UNSUPPORTED, "n_poly > " + std::to_string(kMaxTemplates));
  if (P->lambda_max != 0)
    return fail(MM_ERR_UNSUPPORTED, "template map-making takes diagonal weights (band_ncoef = 1)");
  if (g->n_baselines < 0) return fail(MM_ERR_INVALID, "n_baselines < 0");
  if (g->n_baselines > 0 && (!g->base_start || !g->base_len))
    return fail(MM_ERR_INVALID, "baseline table pointers are NULL");
  if (g->n_baselines > INT32_MAX) return fail(MM_ERR_INVALID, "too many baselines");
  const int64_t nb = g->n_baselines;
  std::vector<int64_t> order(static_cast<size_t>(nb));
  for (int64_t i = 0; i < nb; ++i) order[static_cast<size_t>(i)] = i;
  std::sort(order.begin(), order.end(),
            [&](int64_t a, int64_t b) { return g->base_start[a] < g->base_start[b]; });
  // weights: the c_0 of the tile holding the baseline; the baseline must stay inside one block
  // (or outside all blocks) and, with detector offsets, inside one detector
  std::vector<int64_t> bstart, bend;  // blocks, sorted by start
  {
    std::vector<int> bo(static_cast<size_t>(g->n_blocks));
    for (int i = 0; i < g->n_blocks; ++i) bo[static_cast<size_t>(i)] = i;
    std::sort(bo.begin(), bo.end(), [&](int a, int b) { return g->blk_start[a] < g->blk_start[b]; });
    for (int i : bo) {
      bstart.push_back(g->blk_start[i]);
      bend.push_back(g->blk_start[i] + g->blk_len[i]);
    }
  }
  std::vector<TBase> bases;
  bases.reserve(static_cast<size_t>(nb));
  int64_t prev_end = 0;
  for (int64_t i : order) {
    const int64_t s0 = g->base_start[i], L = g->base_len[i];
    if (s0 < 0 || L < 1 || s0 + L > g->n_samples)
      return fail(MM_ERR_INVALID, "baseline " + std::to_string(i) + " outside [0, n_samples)");
    if (L > INT32_MAX) return fail(MM_ERR_INVALID, "baseline longer than 2^31 samples");
    if (s0 < prev_end) return fail(MM_ERR_INVALID, "baselines overlap");
    prev_end = s0 + L;
    // block containing s0 (last block starting at or before s0)
    const auto it = std::upper_bound(bstart.begin(), bstart.end(), s0);
    const int64_t bi = (it - bstart.begin()) - 1;
    const bool inside = bi >= 0 && s0 < bend[static_cast<size_t>(bi)];
    if (inside && s0 + L > bend[static_cast<size_t>(bi)])
      return fail(MM_ERR_INVALID, "baseline " + std::to_string(i) + " crosses a stationary interval");
    if (!inside) {
      const int64_t next = bi + 1;
      if (next < static_cast<int64_t>(bstart.size()) && bstart[static_cast<size_t>(next)] < s0 + L)
        return fail(MM_ERR_INVALID, "baseline " + std::to_string(i) + " crosses a stationary interval");
    }
    if (g->det_offset != nullptr && g->n_dets > 0) {
      const int64_t* de = g->det_offset;
      const auto dt = std::upper_bound(de, de + g->n_dets + 1, s0);
      if (dt == de + g->n_dets + 1 || s0 + L > *dt)
        return fail(MM_ERR_INVALID, "baseline " + std::to_string(i) + " crosses a detector");
    }
    // weight of the covering tile (tiles are sorted and cover [0, n_samples))
    const auto ti = std::upper_bound(tiles.begin(), tiles.end(), s0,
                                     [](int64_t v, const Tile& t) { return v < t.start; });
    const float w = (ti == tiles.begin()) ? 1.0f : (ti - 1)->c0;
    bases.push_back(TBase{s0, static_cast<int32_t>(L), w});
  }
  // samples outside every baseline: the tiles with the baselines cut out
  std::vector<Tile> free_tiles;
  {
    size_t bix = 0;
    for (const Tile& t : tiles) {
      int64_t a = t.start;
      const int64_t e = t.start + t.len;
      while (a < e) {
        while (bix < bases.size() && bases[bix].start + bases[bix].len <= a) ++bix;
        int64_t stop = e;
        if (bix < bases.size() && bases[bix].start <= a) {
          a = std::min<int64_t>(e, bases[bix].start + bases[bix].len);  // skip the covered part
          continue;
        }
        if (bix < bases.size()) stop = std::min<int64_t>(e, bases[bix].start);
        free_tiles.push_back(Tile{a, static_cast<int32_t>(stop - a), t.c0});
        a = stop;
      }
    }
  }
  P->n_poly = n_poly;
  P->n_baselines = nb;
  MM_TRY(dalloc(P, &P->tbases, bases.size()));
  MM_TRY(dalloc(P, &P->tkinv, bases.size() * static_cast<size_t>(n_poly * n_poly)));
  MM_TRY(dalloc(P, &P->free_tiles, free_tiles.size()));
  P->n_free_tiles = static_cast<int32_t>(free_tiles.size());
  if (!bases.empty())
    MM_HIP_TRY(hipMemcpyAsync(P->tbases, bases.data(), bases.size() * sizeof(TBase), hipMemcpyHostToDevice, s));
  if (!free_tiles.empty())
    MM_HIP_TRY(hipMemcpyAsync(P->free_tiles, free_tiles.data(), free_tiles.size() * sizeof(Tile),
                              hipMemcpyHostToDevice, s));
  if (bases.empty()) {
    MM_HIP_TRY(hipStreamSynchronize(s));
    return MM_OK;
  }
  // kernel blocks and their pseudo-inverses on the device, one workgroup per baseline
  const dim3 grid(static_cast<unsigned>(bases.size()));
  switch (n_poly) {
    case 1: hipLaunchKernelGGL(k_template_kernel<1>, grid, dim3(kTT), 0, s, P->lpix, P->tbases, P->tkinv); break;
    case 2: hipLaunchKernelGGL(k_template_kernel<2>, grid, dim3(kTT), 0, s, P->lpix, P->tbases, P->tkinv); break;
    case 3: hipLaunchKernelGGL(k_template_kernel<3>, grid, dim3(kTT), 0, s, P->lpix, P->tbases, P->tkinv); break;
    case 4: hipLaunchKernelGGL(k_template_kernel<4>, grid, dim3(kTT), 0, s, P->lpix, P->tbases, P->tkinv); break;
    case 5: hipLaunchKernelGGL(k_template_kernel<5>, grid, dim3(kTT), 0, s, P->lpix, P->tbases, P->tkinv); break;
    case 6: hipLaunchKernelGGL(k_template_kernel<6>, grid, dim3(kTT), 0, s, P->lpix, P->tbases, P->tkinv); break;
    case 7: hipLaunchKernelGGL(k_template_kernel<7>, grid, dim3(kTT), 0, s, P->lpix, P->tbases, P->tkinv); break;
    default: hipLaunchKernelGGL(k_template_kernel<8>, grid, dim3(kTT), 0, s, P->lpix, P->tbases, P->tkinv); break;
  }
  MM_HIP_TRY(hipGetLastError());
  MM_HIP_TRY(hipStreamSynchronize(s));  // the host tables above are released on return
  return MM_OK;
}

namespace {

template <int NP>
mm_status launch_np(Plan* P, const double* x, const float* d, double* y, const int32_t* done,
                    hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(P->n_baselines));
  if (x != nullptr)
    hipLaunchKernelGGL((k_template_apply<false, NP>), grid, dim3(kTT), 0, s, P->lpix, P->wq,
                       P->wu, x, d, P->tbases, P->tkinv, y, done);
  else
    hipLaunchKernelGGL((k_template_apply<true, NP>), grid, dim3(kTT), 0, s, P->lpix, P->wq,
                       P->wu, x, d, P->tbases, P->tkinv, y, done);
  MM_HIP_TRY(hipGetLastError());
  return MM_OK;
}

}  // namespace

mm_status launch_template_apply(Plan* P, const double* x, const float* d, double* y,
                                const int32_t* done, hipStream_t s) {
  TimedLaunch tl(P, K_TOEPLITZ, s);
  if (P->n_baselines > 0) {
    switch (P->n_poly) {
      case 1: MM_TRY(launch_np<1>(P, x, d, y, done, s)); break;
      case 2: MM_TRY(launch_np<2>(P, x, d, y, done, s)); break;
      case 3: MM_TRY(launch_np<3>(P, x, d, y, done, s)); break;
      case 4: MM_TRY(launch_np<4>(P, x, d, y, done, s)); break;
      case 5: MM_TRY(launch_np<5>(P, x, d, y, done, s)); break;
      case 6: MM_TRY(launch_np<6>(P, x, d, y, done, s)); break;
      case 7: MM_TRY(launch_np<7>(P, x, d, y, done, s)); break;
      default: MM_TRY(launch_np<8>(P, x, d, y, done, s)); break;
    }
  }
  if (P->n_free_tiles > 0)
    MM_TRY(launch_diag_tiles(P, P->free_tiles, P->n_free_tiles, x, d, y, done, s));
  return MM_OK;
}

}  // namespace mm
