// Plan construction: hits, block-Jacobi blocks, excision, compaction, band symbols.
//
// Follows the block-Jacobi preconditioner construction (accumulate P^T diag(N^-1) P per pixel,
// then invert each 3x3 block and evaluate its condition number, excising ill-conditioned
// pixels and their samples, Degeneracy section) and MAPMAT's global/local pixel indexing (the
// local index of a kept pixel is the rank of its global id).  All per-sample and per-pixel work
// runs in the kernels below; the host only validates the small block/band tables, lays out
// the segment tables and sizes the allocations.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <numeric>
#include <tuple>
#include <type_traits>
#include <unordered_map>

#include "mm_internal.h"
#include "wave_runs.h"

namespace mm {

namespace {

constexpr int kThreads = 256;
constexpr int kTile = 4096;        // samples per plan tile (never crossing a block edge)
constexpr int kScanChunk = 4096;   // pixels per compaction workgroup
constexpr int kAccLane = 8;        // consecutive samples per lane in the BJ accumulation
constexpr int kAccListed = 64;     // listed runs per wavefront there

// ---- hits + BJ blocks over global pixels ---------------------------------------------------

struct BjFlush {
  double* B;        // [n_pix_global][6]
  int32_t* hits;    // [n_pix_global]
  __device__ void operator()(int key, const double (&v)[7]) const {
    double* dst = B + 6 * static_cast<int64_t>(key);
#pragma unroll
    for (int c = 0; c < 6; ++c) unsafeAtomicAdd(dst + c, v[c]);
    atomicAdd(hits + key, static_cast<int32_t>(v[6] + 0.5));
  }
  __device__ void one(int key, int c, double v) const {
    if (c < 6) {
      unsafeAtomicAdd(B + 6 * static_cast<int64_t>(key) + c, v);
    } else {
      atomicAdd(hits + key, static_cast<int32_t>(v + 0.5));
    }
  }
};

__global__ __launch_bounds__(kThreads) void k_plan_accumulate(
    const int32_t* __restrict__ pix, const float* __restrict__ wq, const float* __restrict__ wu,
    const Tile* __restrict__ tiles, int64_t n_pix_global, double* __restrict__ B,
    int32_t* __restrict__ hits, int32_t* __restrict__ err) {
  const Tile tl = tiles[blockIdx.x];
  const BjFlush flush{B, hits};
  // per wavefront: the runs it completes, listed before the atomics
  __shared__ int skey[kThreads / 64][kAccListed];
  __shared__ double sval[kThreads / 64][7 * kAccListed];
  const int wave = static_cast<int>(threadIdx.x >> 6);
  const double c0 = tl.c0;
  for (int off = 0; off < tl.len; off += kThreads * kAccLane) {  // same trip count for all lanes
    const int o0 = off + threadIdx.x * kAccLane;
    const int64_t i0 = tl.start + o0;
    int gg[kAccLane];
    float qq[kAccLane], uu[kAccLane];
    bool in[kAccLane];
    if (o0 + kAccLane <= tl.len && (i0 & 3) == 0) {  // 16-byte loads per stream
#pragma unroll
      for (int h = 0; h < kAccLane / 4; ++h) {
        const int4 g4 = *reinterpret_cast<const int4*>(pix + i0 + 4 * h);
        const float4 q4 = *reinterpret_cast<const float4*>(wq + i0 + 4 * h);
        const float4 u4 = *reinterpret_cast<const float4*>(wu + i0 + 4 * h);
        gg[4 * h] = g4.x; gg[4 * h + 1] = g4.y; gg[4 * h + 2] = g4.z; gg[4 * h + 3] = g4.w;
        qq[4 * h] = q4.x; qq[4 * h + 1] = q4.y; qq[4 * h + 2] = q4.z; qq[4 * h + 3] = q4.w;
        uu[4 * h] = u4.x; uu[4 * h + 1] = u4.y; uu[4 * h + 2] = u4.z; uu[4 * h + 3] = u4.w;
      }
#pragma unroll
      for (int j = 0; j < kAccLane; ++j) in[j] = true;
    } else {
#pragma unroll
      for (int j = 0; j < kAccLane; ++j) {
        in[j] = o0 + j < tl.len;
        gg[j] = in[j] ? pix[i0 + j] : -1;
        qq[j] = in[j] ? wq[i0 + j] : 0.0f;
        uu[j] = in[j] ? wu[i0 + j] : 0.0f;
      }
    }
    int key[kAccLane];
    double v[kAccLane][7];
#pragma unroll
    for (int j = 0; j < kAccLane; ++j) {
      key[j] = -1;
#pragma unroll
      for (int c = 0; c < 7; ++c) v[j][c] = 0.0;
      if (in[j]) {
        int g = gg[j];
        if (g < -1 || g >= n_pix_global) {
          atomicOr(err, 1);
          g = -1;
        }
        key[j] = g;
        const double q = qq[j], u = uu[j];
        v[j][0] = c0;
        v[j][1] = c0 * q;
        v[j][2] = c0 * u;
        v[j][3] = c0 * q * q;
        v[j][4] = c0 * q * u;
        v[j][5] = c0 * u * u;
        v[j][6] = 1.0;
      }
    }
    wave_merge_runs_listed<kAccLane, 7, kAccListed, BjFlush, true>(key, v, flush, skey[wave],
                                                                  sval[wave]);
  }
}

// ---- per-pixel classification: keep when hits >= 3 and cond(B) <= cond_max ----------------

// Eigenvalues of a symmetric 3x3 matrix by cyclic Jacobi rotations (FP64).
__device__ void sym3_eigs(const double* b6, double& lo, double& hi) {
  double a[3][3] = {{b6[0], b6[1], b6[2]}, {b6[1], b6[3], b6[4]}, {b6[2], b6[4], b6[5]}};
  for (int sweep = 0; sweep < 12; ++sweep) {
    const double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    const double diag = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
    if (off <= 1e-34 * diag) break;
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0;
      const int q = pq == 0 ? 1 : 2;
      const double apq = a[p][q];
      if (apq == 0.0) continue;
      const double theta = (a[q][q] - a[p][p]) / (2.0 * apq);
      const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
      const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
      for (int k = 0; k < 3; ++k) {  // A <- A J  (columns p, q)
        const double akp = a[k][p], akq = a[k][q];
        a[k][p] = c * akp - s * akq;
        a[k][q] = s * akp + c * akq;
      }
      for (int k = 0; k < 3; ++k) {  // A <- J^T A  (rows p, q)
        const double apk = a[p][k], aqk = a[q][k];
        a[p][k] = c * apk - s * aqk;
        a[q][k] = s * apk + c * aqk;
      }
    }
  }
  lo = fmin(a[0][0], fmin(a[1][1], a[2][2]));
  hi = fmax(a[0][0], fmax(a[1][1], a[2][2]));
}

__global__ __launch_bounds__(kThreads) void k_plan_classify(const double* __restrict__ B,
                                                            const int32_t* __restrict__ hits,
                                                            int64_t n, double cond_max,
                                                            uint8_t* __restrict__ keep,
                                                            unsigned long long* __restrict__ n_obs) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  int observed = 0;
  if (g < n) {
    const int h = hits[g];
    uint8_t k = 0;
    if (h > 0) {
      observed = 1;
      if (h >= 3) {
        double lo, hi;
        sym3_eigs(B + 6 * g, lo, hi);
        if (lo > 0.0 && hi <= cond_max * lo) k = 1;
      }
    }
    keep[g] = k;
  }
  const unsigned long long cnt = __ballot(observed);
  if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(n_obs, static_cast<unsigned long long>(__popcll(cnt)));
}

// ---- compaction: prefix sum of keep flags --------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_scan_count(const uint8_t* __restrict__ keep,
                                                         int64_t n, int32_t* __restrict__ counts) {
  __shared__ int red[kThreads / 64];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanChunk;
  int c = 0;
  for (int i = threadIdx.x; i < kScanChunk; i += kThreads) {
    const int64_t g = base + i;
    if (g < n) c += keep[g];
  }
  for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int w = 0; w < kThreads / 64; ++w) s += red[w];
    counts[blockIdx.x] = s;
  }
}

// Exclusive scan of the per-chunk counts by one workgroup; the total goes to *total.
__global__ __launch_bounds__(1024) void k_scan_offsets(int32_t* __restrict__ counts, int n,
                                                       int64_t* __restrict__ total) {
  __shared__ int64_t part[1024];
  const int per = (n + 1023) / 1024;
  const int lo = threadIdx.x * per, hi = min(n, lo + per);
  int64_t s = 0;
  for (int i = lo; i < hi; ++i) s += counts[i];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int i = 0; i < 1024; ++i) {
      const int64_t v = part[i];
      part[i] = run;
      run += v;
    }
    *total = run;
  }
  __syncthreads();
  int64_t run = part[threadIdx.x];
  for (int i = lo; i < hi; ++i) {
    const int32_t v = counts[i];
    counts[i] = static_cast<int32_t>(run);
    run += v;
  }
}

// Local ids for kept pixels; kept ids, hits and inverted BJ blocks in local order.
__global__ __launch_bounds__(kThreads) void k_scan_write(
    const uint8_t* __restrict__ keep, int64_t n, const int32_t* __restrict__ offsets,
    const double* __restrict__ B, const int32_t* __restrict__ hits_g, int32_t* __restrict__ local,
    int64_t* __restrict__ kept_ids, int32_t* __restrict__ hits, double* __restrict__ minv) {
  __shared__ int wsum[kThreads / 64];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanChunk;
  int run = offsets[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i0 = 0; i0 < kScanChunk; i0 += kThreads) {
    const int64_t g = base + i0 + threadIdx.x;
    const int k = (g < n) ? keep[g] : 0;
    const unsigned long long m = __ballot(k);
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wave] = __popcll(m);
    __syncthreads();
    int woff = 0;
    for (int w = 0; w < wave; ++w) woff += wsum[w];
    int tot = 0;
    for (int w = 0; w < kThreads / 64; ++w) tot += wsum[w];
    if (g < n) {
      if (k) {
        const int l = run + woff + before;
        local[g] = l;
        kept_ids[l] = g;
        hits[l] = hits_g[g];
        const double* b = B + 6 * g;
        const double a = b[0], bb = b[1], c = b[2], d = b[3], e = b[4], f = b[5];
        const double A00 = d * f - e * e, A01 = c * e - bb * f, A02 = bb * e - c * d;
        const double A11 = a * f - c * c, A12 = bb * c - a * e, A22 = a * d - bb * bb;
        const double inv = 1.0 / (a * A00 + bb * A01 + c * A02);
        double* mo = minv + 6 * static_cast<int64_t>(l);
        mo[0] = A00 * inv;
        mo[1] = A01 * inv;
        mo[2] = A02 * inv;
        mo[3] = A11 * inv;
        mo[4] = A12 * inv;
        mo[5] = A22 * inv;
      } else {
        local[g] = -1;
      }
    }
    run += tot;
    __syncthreads();
  }
}

// lpix[s] = local id of pix[s] (or -1); counts gap samples.
__global__ __launch_bounds__(kThreads) void k_plan_remap(const int32_t* __restrict__ pix,
                                                         const int32_t* __restrict__ local,
                                                         int32_t* __restrict__ lpix, int64_t n,
                                                         unsigned long long* __restrict__ n_gap) {
  int gaps = 0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    const int g = pix[i];
    const int l = g >= 0 ? local[g] : -1;
    lpix[i] = l;
    gaps += (l < 0);
  }
  for (int o = 32; o > 0; o >>= 1) gaps += __shfl_down(gaps, o);
  if ((threadIdx.x & 63) == 0 && gaps) atomicAdd(n_gap, static_cast<unsigned long long>(gaps));
}

// ---- band symbols f(w) = c_0 + 2 sum_k c_k cos(k w) on an M-point grid (Clenshaw, FP64) -----
// Each thread runs kSymPts independent recurrences (grid points k, k + S, k + 2S, ... with S the
// number of threads of the band) that share every coefficient load: one chain alone would wait
// on its own FMA latency at every step.  A step is b_j = 2x b_{j+1} + (2c_j - b_{j+2}): the
// bracket is known a step early, so each chain's critical path is one FMA per coefficient.
constexpr int kSymPts = 8;

__global__ __launch_bounds__(kThreads) void k_band_symbol(
    const float* __restrict__ coef, const int64_t* __restrict__ off,
    const int32_t* __restrict__ ncoef, int M, int fft_n, float* __restrict__ spec,
    double* __restrict__ spec64, double* __restrict__ block_min) {
  __shared__ double red[kThreads / 64];
  const int band = blockIdx.y;
  const int nc = ncoef[band];
  const float* cs = coef + off[band];  // every lane reads the same coefficient: broadcast loads
  const int stride = gridDim.x * kThreads;
  int k[kSymPts];
  double x[kSymPts], x2[kSymPts], b1[kSymPts], b2[kSymPts];
#pragma unroll
  for (int p = 0; p < kSymPts; ++p) {
    k[p] = blockIdx.x * kThreads + threadIdx.x + p * stride;
    x[p] = cospi(2.0 * static_cast<double>(k[p]) / static_cast<double>(M));
    x2[p] = 2.0 * x[p];
    b1[p] = 0.0;
    b2[p] = 0.0;
  }
  // eight steps per round with their eight coefficients loaded first: one wait per round
  // instead of one per step
  int j = nc - 1;
  for (; j >= 8; j -= 8) {
    double c2[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) c2[q] = 2.0 * static_cast<double>(cs[j - q]);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
#pragma unroll
      for (int p = 0; p < kSymPts; ++p) {
        const double b0 = fma(x2[p], b1[p], c2[q] - b2[p]);  // b2 is known a step early
        b2[p] = b1[p];
        b1[p] = b0;
      }
    }
  }
  for (; j >= 1; --j) {
    const double c2 = 2.0 * static_cast<double>(cs[j]);
#pragma unroll
    for (int p = 0; p < kSymPts; ++p) {
      const double b0 = fma(x2[p], b1[p], c2 - b2[p]);
      b2[p] = b1[p];
      b1[p] = b0;
    }
  }
  double m = INFINITY;
  const double c0 = static_cast<double>(cs[0]);
#pragma unroll
  for (int p = 0; p < kSymPts; ++p) {
    if (k[p] > M / 2) continue;
    const double f = c0 + x[p] * b1[p] - b2[p];
    m = fmin(m, f);
    if (spec != nullptr || spec64 != nullptr) {
      const int step = M / fft_n;
      if (k[p] % step == 0) {
        const int kk = k[p] / step;  // 0 .. fft_n / 2
        const int64_t at = static_cast<int64_t>(band) * (fft_n / 2 + 1) + kk;
        if (spec != nullptr) spec[at] = static_cast<float>(f / (2.0 * static_cast<double>(fft_n)));
        if (spec64 != nullptr) spec64[at] = f;
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) m = fmin(m, __shfl_down(m, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int w = 1; w < kThreads / 64; ++w) r = fmin(r, red[w]);
    block_min[static_cast<int64_t>(band) * gridDim.x + blockIdx.x] = r;
  }
}

// The same symbol on large grids (M >= 4096) in two levels, with j = p + 64 q and the grid
// point k = r + (M/64) s:
//   f(2 pi k / M) = Re sum_p e^{2 pi i p k / M} G_p(r),   G_p(r) = sum_q w_{p+64q} e^{2 pi i q r / (M/64)}
// (w_0 = c_0, w_j = 2 c_j): the inner sums depend on k only through r, so each is formed once for
// the 64 values of s that share it, about a tenth of the Clenshaw work at lambda = M/8.  A
// workgroup takes 16 consecutive r for one band: phase 1 builds its 64 x 16 inner sums in LDS
// (powers of e^{2 pi i r/(M/64)} by multiplication, re-anchored every 32 steps), phase 2 the grid
// points k <= M/2 with those r.  All FP64.
constexpr int kSymP = 64;   // inner stride
constexpr int kSymR = 16;   // r values per workgroup

__global__ __launch_bounds__(kThreads) void k_band_symbol2(
    const float* __restrict__ coef, const int64_t* __restrict__ off,
    const int32_t* __restrict__ ncoef, int M, int fft_n, float* __restrict__ spec,
    double* __restrict__ spec64, double* __restrict__ block_min) {
  static_assert(kThreads == 256 && kSymP * kSymR == 4 * kThreads, "thread mapping");
  __shared__ double gr[kSymP * kSymR], gi[kSymP * kSymR];
  __shared__ double red[kThreads / 64];
  const int band = blockIdx.y;
  const int nc = ncoef[band];
  const float* cs = coef + off[band];
  const int MP = M / kSymP;
  const int r0 = blockIdx.x * kSymR;
  const int tid = threadIdx.x;
  // ---- phase 1: inner sums G_p(r) for p = 4 g .. 4 g + 3 and r = r0 + rr ---------------------
  {
    const int rr = tid & (kSymR - 1), g = tid >> 4;
    const int r = r0 + rr;
    double zs, zc;
    sincospi(2.0 * static_cast<double>(r) / static_cast<double>(MP), &zs, &zc);
    double ar[4] = {0.0, 0.0, 0.0, 0.0}, ai[4] = {0.0, 0.0, 0.0, 0.0};
    double qr = 1.0, qi = 0.0;
    const int Q = (nc + kSymP - 1) / kSymP;
    for (int q = 0; q < Q; ++q) {
      if ((q & 31) == 0 && q > 0) {  // re-anchor z^q
        const int64_t e = (static_cast<int64_t>(q) * r) % MP;
        sincospi(2.0 * static_cast<double>(e) / static_cast<double>(MP), &qi, &qr);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int j = 4 * g + i + kSymP * q;
        const double w = j >= nc ? 0.0 : (j == 0 ? 1.0 : 2.0) * static_cast<double>(cs[j]);
        ar[i] = fma(w, qr, ar[i]);
        ai[i] = fma(w, qi, ai[i]);
      }
      const double nr = qr * zc - qi * zs, ni = qr * zs + qi * zc;
      qr = nr;
      qi = ni;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      gr[(4 * g + i) * kSymR + rr] = ar[i];
      gi[(4 * g + i) * kSymR + rr] = ai[i];
    }
  }
  __syncthreads();
  // ---- phase 2: grid points k = r0 + rr + MP s <= M/2 ----------------------------------------
  double m = INFINITY;
  for (int pt = tid; pt < kSymR * (kSymP / 2 + 1); pt += kThreads) {
    const int rr = pt & (kSymR - 1), sidx = pt >> 4;
    const int k = r0 + rr + MP * sidx;
    if (k > M / 2) continue;
    double us, uc;
    sincospi(2.0 * static_cast<double>(k) / static_cast<double>(M), &us, &uc);
    double vr = 1.0, vi = 0.0, f = 0.0;
    for (int p = 0; p < kSymP; ++p) {
      if ((p & 15) == 0 && p > 0) {  // re-anchor u^p
        const int64_t e = (static_cast<int64_t>(p) * k) % M;
        sincospi(2.0 * static_cast<double>(e) / static_cast<double>(M), &vi, &vr);
      }
      f = fma(vr, gr[p * kSymR + rr], f);
      f = fma(-vi, gi[p * kSymR + rr], f);
      const double nr = vr * uc - vi * us, ni = vr * us + vi * uc;
      vr = nr;
      vi = ni;
    }
    m = fmin(m, f);
    if (spec != nullptr || spec64 != nullptr) {
      const int step = M / fft_n;
      if (k % step == 0) {
        const int64_t at = static_cast<int64_t>(band) * (fft_n / 2 + 1) + k / step;
        if (spec != nullptr) spec[at] = static_cast<float>(f / (2.0 * static_cast<double>(fft_n)));
        if (spec64 != nullptr) spec64[at] = f;
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) m = fmin(m, __shfl_down(m, o));
  if ((tid & 63) == 0) red[tid >> 6] = m;
  __syncthreads();
  if (tid == 0) {
    double rm = red[0];
    for (int w = 1; w < kThreads / 64; ++w) rm = fmin(rm, red[w]);
    block_min[static_cast<int64_t>(band) * gridDim.x + blockIdx.x] = rm;
  }
}

}  // namespace

// FP64 symbol S[k] = c_0 + 2 sum_j c_j cos(2 pi j k / N), k = 0 .. N/2, of every band at the
// plan's FFT length N (unscaled), for the FP64 product.  Synchronous.
mm_status launch_band_symbol64(Plan* P, double* spec64, hipStream_t s) {
  const int M = P->fft_n;
  if (P->n_bands == 0 || M <= 0) return MM_OK;
  const bool two_level = M >= 4096;
  const int gx = two_level ? M / (kSymP * kSymR)
                           : (M / 2 + 1 + kThreads * kSymPts - 1) / (kThreads * kSymPts);
  double* mins = nullptr;
  const hipError_t e = dev_malloc(reinterpret_cast<void**>(&mins),
                                  sizeof(double) * static_cast<size_t>(gx) * P->n_bands);
  if (e != hipSuccess) return fail(MM_ERR_OOM, std::string("hipMalloc (symbol): ") + hipGetErrorString(e));
  if (two_level)
    hipLaunchKernelGGL(k_band_symbol2, dim3(gx, P->n_bands), dim3(kThreads), 0, s, P->band_coef,
                       P->band_off, P->band_ncoef, M, M, static_cast<float*>(nullptr), spec64, mins);
  else
    hipLaunchKernelGGL(k_band_symbol, dim3(gx, P->n_bands), dim3(kThreads), 0, s, P->band_coef,
                       P->band_off, P->band_ncoef, M, M, static_cast<float*>(nullptr), spec64, mins);
  const hipError_t le = hipGetLastError();
  const hipError_t se = hipStreamSynchronize(s);
  dev_free(mins);
  if (le != hipSuccess) return fail(MM_ERR_HIP, std::string("symbol launch: ") + hipGetErrorString(le));
  if (se != hipSuccess) return fail(MM_ERR_HIP, std::string("symbol: ") + hipGetErrorString(se));
  return MM_OK;
}

namespace {

// Stream-ordered upload (no legacy-stream operation: other threads may be capturing graphs on
// their own streams meanwhile); synchronous, since h is released by the caller afterwards.
template <class T>
mm_status upload(Plan* P, T** dst, const T* h, size_t n, hipStream_t s) {
  MM_TRY(dalloc(P, dst, n));
  if (n > 0) {
    MM_HIP_TRY(hipMemcpyAsync(*dst, h, n * sizeof(T), hipMemcpyHostToDevice, s));
    MM_HIP_TRY(hipStreamSynchronize(s));
  }
  return MM_OK;
}

template <class T>
mm_status upload(Plan* P, T** dst, const std::vector<T>& h, hipStream_t s) {
  return upload(P, dst, h.data(), h.size(), s);
}

// Temporary device buffer freed at scope exit.
template <class T>
struct Scratch {
  T* p = nullptr;
  ~Scratch() {
    if (p) dev_free(p);
  }
  mm_status alloc(size_t n) {
    if (n == 0) n = 1;
    hipError_t e = dev_malloc(reinterpret_cast<void**>(&p), n * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      return fail(MM_ERR_OOM, std::string("hipMalloc (plan scratch): ") + hipGetErrorString(e));
    }
    return MM_OK;
  }
};

mm_status validate(const mm_geometry* g, std::vector<int>& order, int32_t& lambda_max) {
  if (g->n_samples < 0) return fail(MM_ERR_INVALID, "n_samples < 0");
  if (g->n_samples > (int64_t(1) << 40)) return fail(MM_ERR_INVALID, "n_samples too large");
  if (g->n_pix_global < 0 || g->n_pix_global > INT32_MAX)
    return fail(MM_ERR_INVALID, "n_pix_global out of [0, 2^31)");
  if (g->n_samples > 0 && (!g->pix || !g->w_q || !g->w_u))
    return fail(MM_ERR_INVALID, "pix / w_q / w_u must be device pointers");
  if (g->n_blocks < 0 || g->n_bands < 0) return fail(MM_ERR_INVALID, "negative table size");
  if (g->n_blocks > 0 && (!g->blk_start || !g->blk_len || !g->blk_band))
    return fail(MM_ERR_INVALID, "block table pointers are NULL");
  if (g->n_bands > 0 && (!g->band_ncoef || !g->band_offset || !g->band_coef))
    return fail(MM_ERR_INVALID, "band table pointers are NULL");
  if (g->n_blocks > 0 && g->n_bands == 0) return fail(MM_ERR_INVALID, "blocks without bands");
  lambda_max = 0;
  for (int b = 0; b < g->n_bands; ++b) {
    if (g->band_ncoef[b] < 1) return fail(MM_ERR_INVALID, "band_ncoef < 1");
    if (g->band_offset[b] < 0) return fail(MM_ERR_INVALID, "band_offset < 0");
  }
  std::vector<char> used(static_cast<size_t>(g->n_bands), 0);
  for (int i = 0; i < g->n_blocks; ++i) {
    const int64_t s = g->blk_start[i], L = g->blk_len[i];
    const int b = g->blk_band[i];
    if (s < 0 || L < 1 || s + L > g->n_samples)
      return fail(MM_ERR_INVALID, "block " + std::to_string(i) + " outside [0, n_samples)");
    if (L > INT32_MAX) return fail(MM_ERR_INVALID, "block longer than 2^31 samples");
    if (b < 0 || b >= g->n_bands) return fail(MM_ERR_INVALID, "block band index out of range");
    used[b] = 1;
  }
  for (int b = 0; b < g->n_bands; ++b)
    if (used[b]) lambda_max = std::max(lambda_max, g->band_ncoef[b] - 1);
  order.resize(g->n_blocks);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(),
            [&](int a, int b) { return g->blk_start[a] < g->blk_start[b]; });
  for (size_t i = 1; i < order.size(); ++i) {
    const int a = order[i - 1], b = order[i];
    if (g->blk_start[a] + g->blk_len[a] > g->blk_start[b])
      return fail(MM_ERR_INVALID, "blocks overlap");
  }
  if (g->det_offset != nullptr && g->n_dets > 0) {
    if (g->det_offset[0] != 0 || g->det_offset[g->n_dets] != g->n_samples)
      return fail(MM_ERR_INVALID, "det_offset must span [0, n_samples]");
    for (int d = 0; d < g->n_dets; ++d)
      if (g->det_offset[d + 1] < g->det_offset[d])
        return fail(MM_ERR_INVALID, "det_offset not ascending");
    for (int i = 0; i < g->n_blocks; ++i) {
      const int64_t s = g->blk_start[i], e = s + g->blk_len[i];
      const int64_t* it = std::upper_bound(g->det_offset, g->det_offset + g->n_dets + 1, s);
      const int64_t det_end = *it;
      if (e > det_end) return fail(MM_ERR_INVALID, "block crosses a detector boundary");
    }
  }
  return MM_OK;
}

}  // namespace

std::shared_mutex& alloc_gate() {
  static std::shared_mutex m;
  return m;
}

// Device memory of plans, workspaces and temporaries goes through a caching allocator.  A freed
// block is kept (per device, keyed by its size) and handed to a later allocation that it fits
// within an eighth, so that the repeated plan builds and solves of a serving loop do not map and
// unmap gigabytes each time.  A free first synchronises the block's device, as hipFree does, so a
// block is never handed out while earlier work may still touch it (the allocation gate keeps
// that synchronisation away from graph captures).  Each device's cache holds at most a quarter
// of its memory, the largest blocks released first beyond that, and is emptied when hipMalloc
// fails.
namespace {

struct DevCache {
  std::multimap<size_t, void*> blocks;  // cached blocks by size
  size_t bytes = 0;
  size_t cap = 0;
};

struct Allocation {
  int device;
  size_t bytes;
};

std::unordered_map<void*, Allocation>& allocations() {
  static std::unordered_map<void*, Allocation> m;
  return m;
}

std::map<int, DevCache>& dev_caches() {
  static std::map<int, DevCache> m;
  return m;
}

size_t rounded(size_t b) {
  const size_t g = b <= (size_t{1} << 20) ? 256 : (size_t{1} << 16);
  return (b + g - 1) / g * g;
}

// Release cached blocks of `c` (current device) until at most `keep` bytes stay cached.
void release_cached(DevCache& c, size_t keep) {
  while (c.bytes > keep && !c.blocks.empty()) {
    auto it = std::prev(c.blocks.end());
    c.bytes -= it->first;
    allocations().erase(it->second);
    (void)hipFree(it->second);
    c.blocks.erase(it);
  }
}

}  // namespace

hipError_t dev_malloc(void** p, size_t bytes) {
  std::unique_lock<std::shared_mutex> lock(alloc_gate());
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  DevCache& c = dev_caches()[dev];
  if (c.cap == 0) {
    size_t free_b = 0, total_b = 0;
    c.cap = hipMemGetInfo(&free_b, &total_b) == hipSuccess ? total_b / 4 : (size_t{1} << 30);
  }
  const size_t want = rounded(bytes == 0 ? 1 : bytes);
  auto it = c.blocks.lower_bound(want);
  if (it != c.blocks.end() && it->first <= want + want / 8) {
    *p = it->second;
    c.bytes -= it->first;
    c.blocks.erase(it);
    return hipSuccess;
  }
  e = hipMalloc(p, want);
  if (e != hipSuccess && !c.blocks.empty()) {
    (void)hipGetLastError();  // the failure is recovered from: do not leave it for later checks
    release_cached(c, 0);
    e = hipMalloc(p, want);
  }
  if (e != hipSuccess) {
    *p = nullptr;
    return e;
  }
  allocations()[*p] = Allocation{dev, want};
  return hipSuccess;
}

void dev_free(void* p) {
  if (p == nullptr) return;
  std::unique_lock<std::shared_mutex> lock(alloc_gate());
  auto it = allocations().find(p);
  if (it == allocations().end()) {
    (void)hipFree(p);
    return;
  }
  const Allocation a = it->second;
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) cur = a.device;
  if (cur != a.device) (void)hipSetDevice(a.device);
  (void)hipDeviceSynchronize();
  DevCache& c = dev_caches()[a.device];
  if (a.bytes > c.cap) {
    allocations().erase(it);
    (void)hipFree(p);
  } else {
    c.blocks.emplace(a.bytes, p);
    c.bytes += a.bytes;
    release_cached(c, c.cap);
  }
  if (cur != a.device) (void)hipSetDevice(cur);
}

bool needs_time_buffers(const Plan* P) {
  return P->lambda_max > 0 && !(P->algo == MM_TOEPLITZ_FFT && P->fused);
}

int32_t reduction_blocks(int64_t n_kept) {
  int64_t nrb = (n_kept + 1023) / 1024;
  return static_cast<int32_t>(std::min<int64_t>(std::max<int64_t>(nrb, 1), 1024));
}

int64_t work_bytes(const Plan* P) {
  int64_t b = 0;
  if (needs_time_buffers(P)) b += 2 * P->n_samples * static_cast<int64_t>(sizeof(float));
  if (P->algo == MM_TOEPLITZ_FFT && long_fft_size(P->fft_n) && P->n_chunks > 0)
    b += static_cast<int64_t>(long_slots(P)) * (P->fft_n / 2) * static_cast<int64_t>(sizeof(float2));
  b += 5 * 3 * P->n_kept * static_cast<int64_t>(sizeof(double));
  b += 4 * static_cast<int64_t>(reduction_blocks(P->n_kept)) * sizeof(double);
  b += sizeof(CgState);
  return b;
}

mm_status work_alloc(const Plan* P, Work* W) {
  *W = Work{};
  struct Guard {
    Work* w;
    bool keep = false;
    ~Guard() {
      if (!keep) work_free(w);
    }
  } guard{W};
  auto get = [&](auto** ptr, size_t count) -> mm_status {
    using T = std::remove_pointer_t<std::remove_reference_t<decltype(*ptr)>>;
    *ptr = nullptr;
    if (count == 0) return MM_OK;
    hipError_t e = dev_malloc(reinterpret_cast<void**>(ptr), count * sizeof(T));
    if (e != hipSuccess) {
      *ptr = nullptr;
      return fail(MM_ERR_OOM, std::string("hipMalloc (solve workspace): ") + hipGetErrorString(e));
    }
    W->bytes += static_cast<int64_t>(count * sizeof(T));
    return MM_OK;
  };
  if (needs_time_buffers(P)) {
    MM_TRY(get(&W->t, static_cast<size_t>(P->n_samples)));
    MM_TRY(get(&W->u, static_cast<size_t>(P->n_samples)));
  }
  if (P->algo == MM_TOEPLITZ_FFT && long_fft_size(P->fft_n) && P->n_chunks > 0)
    MM_TRY(get(&W->scratch, static_cast<size_t>(long_slots(P)) * (P->fft_n / 2)));
  const size_t nu = static_cast<size_t>(3 * P->n_kept);
  MM_TRY(get(&W->r, nu));
  MM_TRY(get(&W->z, nu));
  MM_TRY(get(&W->p, nu));
  MM_TRY(get(&W->q, nu));
  MM_TRY(get(&W->b, nu));
  W->nrb = reduction_blocks(P->n_kept);
  MM_TRY(get(&W->partial, static_cast<size_t>(4 * W->nrb)));
  MM_TRY(get(&W->state, 1));
  {
    std::unique_lock<std::shared_mutex> lock(alloc_gate());
    MM_HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&W->h_state), sizeof(CgState),
                             hipHostMallocDefault));
  }
  W->cache_graphs = true;
  guard.keep = true;
  return MM_OK;
}

void work_free(Work* W) {
  {
    std::unique_lock<std::shared_mutex> lock(alloc_gate());
    for (GraphSlot& g : W->graphs)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
  }
  void* ptrs[] = {W->t, W->u, W->scratch, W->r, W->z, W->p, W->q, W->b, W->partial, W->state};
  for (void* p : ptrs) dev_free(p);
  if (W->h_state) {
    std::unique_lock<std::shared_mutex> lock(alloc_gate());
    (void)hipHostFree(W->h_state);
  }
  *W = Work{};
}

void destroy_plan(Plan* P) {
  if (!P) return;
  void* ptrs[] = {P->lpix,       P->wq,       P->wu,      P->minv,     P->hits,
                  P->kept_ids,   P->band_coef, P->band_off, P->band_ncoef, P->spec,
                  P->spec_reg,   P->long_pq,  P->tw0,     P->tw1,      P->chunks,
                  P->tiles,      P->id_tiles, P->id_seg};
  for (void* p : ptrs) dev_free(p);
  dev_free(P->x_spec);
  dev_free(P->x_tw);
  dev_free(P->tbases);
  dev_free(P->tkinv);
  dev_free(P->free_tiles);
  work_free(&P->work);
  deflation_free(&P->defl);
  if (P->aux) (void)hipStreamDestroy(P->aux);
  for (int k = 0; k < K_NKINDS; ++k)
    for (const TimedPair& t : P->timing.pending[k]) {
      (void)hipEventDestroy(t.e0);
      (void)hipEventDestroy(t.e1);
    }
  delete P;
}

namespace {

// FFT-length tuning (fft_size = -1): the shapes already tuned in this process, keyed by what
// decides the segment table and its kernels.
struct FftTuneKey {
  int64_t n_samples;
  int32_t n_blocks, lambda_max, flags, precision, device;
  bool operator<(const FftTuneKey& o) const {
    return std::tie(n_samples, n_blocks, lambda_max, flags, precision, device) <
           std::tie(o.n_samples, o.n_blocks, o.lambda_max, o.flags, o.precision, o.device);
  }
};

std::mutex& fft_tune_mutex() {
  static std::mutex m;
  return m;
}

std::map<FftTuneKey, int32_t>& fft_tuned() {
  static std::map<FftTuneKey, int32_t> m;
  return m;
}

// Milliseconds of one system product of a built plan (mean of three after one warm-up).
mm_status time_product(Plan* P, hipStream_t s, double* ms) {
  const int64_t nu = 3 * P->n_kept;
  double* x = nullptr;
  double* y = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  struct Cleanup {
    double*& x;
    double*& y;
    hipEvent_t& e0;
    hipEvent_t& e1;
    ~Cleanup() {
      dev_free(x);
      dev_free(y);
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    }
  } cleanup{x, y, e0, e1};
  if (dev_malloc(reinterpret_cast<void**>(&x), sizeof(double) * std::max<int64_t>(nu, 1)) !=
          hipSuccess ||
      dev_malloc(reinterpret_cast<void**>(&y), sizeof(double) * std::max<int64_t>(nu, 1)) !=
          hipSuccess)
    return fail(MM_ERR_OOM, "hipMalloc (FFT-length tuning)");
  MM_TRY(launch_zero(x, nu, s));  // the product's work does not depend on the values
  MM_HIP_TRY(hipEventCreate(&e0));
  MM_HIP_TRY(hipEventCreate(&e1));
  MM_TRY(apply_A(P, P->work, x, y, nullptr, s));
  MM_HIP_TRY(hipEventRecord(e0, s));
  for (int i = 0; i < 3; ++i) MM_TRY(apply_A(P, P->work, x, y, nullptr, s));
  MM_HIP_TRY(hipEventRecord(e1, s));
  MM_HIP_TRY(hipEventSynchronize(e1));
  float t = 0.0f;
  MM_HIP_TRY(hipEventElapsedTime(&t, e0, e1));
  *ms = t / 3.0;
  return MM_OK;
}

}  // namespace

mm_status build_plan_fixed(const mm_geometry* g, hipStream_t s, Plan** out);

// fft_size = -1: the plan is built at the rule's length N0 and at 2 N0 and 4 N0 (up to 2^17),
// one system product is timed on each, and the fastest is kept.  The choice is remembered for
// the shape, so later plans of the same shape are built once.
mm_status build_plan(const mm_geometry* g, hipStream_t s, Plan** out) {
  *out = nullptr;
  if (g->fft_size < -1) return fail(MM_ERR_INVALID, "fft_size must be -1 (tuned), 0 or a length");
  if (g->fft_size != -1) return build_plan_fixed(g, s, out);
  int32_t lambda_max = 0;
  for (int32_t b = 0; b < g->n_bands; ++b)
    if (g->band_ncoef) lambda_max = std::max(lambda_max, g->band_ncoef[b] - 1);
  mm_geometry h = *g;
  h.fft_size = 0;
  const bool fft = g->toeplitz_algo == MM_TOEPLITZ_FFT ||
                   (g->toeplitz_algo == MM_TOEPLITZ_AUTO && lambda_max > 32);
  if (!fft || lambda_max <= 0 || g->n_poly > 0) return build_plan_fixed(&h, s, out);
  int dev = 0;
  MM_HIP_TRY(hipGetDevice(&dev));
  const FftTuneKey key{g->n_samples, g->n_blocks, lambda_max, g->flags, g->precision, dev};
  {
    std::lock_guard<std::mutex> lk(fft_tune_mutex());
    auto it = fft_tuned().find(key);
    if (it != fft_tuned().end()) {
      h.fft_size = it->second;
      return build_plan_fixed(&h, s, out);
    }
  }
  const int32_t n0 = choose_fft_size(lambda_max);
  if (n0 == 0) return build_plan_fixed(&h, s, out);  // reports the unsupported length
  Plan* best = nullptr;
  double best_ms = 0.0;
  for (int32_t n = n0; n <= (1 << 17); n *= 2) {
    if (!fft_size_supported(n)) continue;
    h.fft_size = n;
    Plan* cand = nullptr;
    const mm_status st = build_plan_fixed(&h, s, &cand);
    if (st != MM_OK) {
      if (best == nullptr && n == n0) return st;  // the rule's own length must build
      continue;
    }
    double ms = 0.0;
    const mm_status tt = time_product(cand, s, &ms);
    if (tt != MM_OK) {
      destroy_plan(cand);
      if (best) destroy_plan(best);
      return tt;
    }
    if (best == nullptr || ms < best_ms) {
      if (best) destroy_plan(best);
      best = cand;
      best_ms = ms;
    } else {
      destroy_plan(cand);
    }
  }
  {
    std::lock_guard<std::mutex> lk(fft_tune_mutex());
    fft_tuned()[key] = best->fft_n;
  }
  *out = best;
  return MM_OK;
}

mm_status build_plan_fixed(const mm_geometry* g, hipStream_t s, Plan** out) {
  *out = nullptr;
  std::vector<int> order;
  int32_t lambda_max = 0;
  MM_TRY(validate(g, order, lambda_max));

  if (g->precision != MM_PRECISION_MIXED && g->precision != MM_PRECISION_FP64)
    return fail(MM_ERR_INVALID, "unknown precision");
  if (g->n_poly < 0) return fail(MM_ERR_INVALID, "n_poly < 0");

  // Algorithm selection.
  int32_t algo = g->toeplitz_algo;
  int32_t fft_n = 0;
  if (algo != MM_TOEPLITZ_AUTO && algo != MM_TOEPLITZ_DIRECT && algo != MM_TOEPLITZ_FFT)
    return fail(MM_ERR_INVALID, "unknown toeplitz_algo");
  if (algo == MM_TOEPLITZ_AUTO) algo = (lambda_max <= 32) ? MM_TOEPLITZ_DIRECT : MM_TOEPLITZ_FFT;
  if (algo == MM_TOEPLITZ_FFT) {
    fft_n = g->fft_size > 0 ? g->fft_size : choose_fft_size(lambda_max);
    if (fft_n == 0 || !fft_size_supported(fft_n))
      return fail(MM_ERR_UNSUPPORTED, "no supported FFT size for lambda = " + std::to_string(lambda_max));
    if (fft_n <= 2 * lambda_max) return fail(MM_ERR_INVALID, "fft_size must exceed 2 lambda");
  } else if (lambda_max > max_direct_lambda()) {
    return fail(MM_ERR_UNSUPPORTED, "direct product limited to lambda <= " +
                                        std::to_string(max_direct_lambda()));
  }

  Plan* P = new Plan();
  struct Guard {
    Plan*& p;
    bool keep = false;
    ~Guard() {
      if (!keep) destroy_plan(p);
    }
  } guard{P};
  MM_HIP_TRY(hipGetDevice(&P->device));
  MM_HIP_TRY(hipDeviceGetAttribute(&P->n_cu, hipDeviceAttributeMultiprocessorCount, P->device));
  P->n_samples = g->n_samples;
  P->n_pix_global = g->n_pix_global;
  P->lambda_max = lambda_max;
  P->algo = algo;
  P->fft_n = fft_n;
  P->n_blocks = g->n_blocks;
  P->n_bands = g->n_bands;
  P->precision = g->precision;
  const int64_t n = g->n_samples;
  const int64_t ng = g->n_pix_global;

  // ---- segment tables: blocks and identity gaps ------------------------------------------
  std::vector<Tile> tiles, id_tiles;
  std::vector<int64_t> idseg;
  auto add_tiles = [&](int64_t s0, int64_t len, float c0) {
    for (int64_t o = 0; o < len; o += kTile)
      tiles.push_back(Tile{s0 + o, static_cast<int32_t>(std::min<int64_t>(kTile, len - o)), c0});
  };
  auto add_identity = [&](int64_t s0, int64_t len) {
    add_tiles(s0, len, 1.0f);
    for (int64_t o = 0; o < len; o += kTile)
      id_tiles.push_back(Tile{s0 + o, static_cast<int32_t>(std::min<int64_t>(kTile, len - o)), 1.0f});
    for (int64_t o = 0; o < len; o += 65536) {
      idseg.push_back(s0 + o);
      idseg.push_back(std::min<int64_t>(65536, len - o));
    }
  };
  int64_t cursor = 0;
  for (int i : order) {
    const int64_t s0 = g->blk_start[i], len = g->blk_len[i];
    if (s0 > cursor) add_identity(cursor, s0 - cursor);
    const int b = g->blk_band[i];
    add_tiles(s0, len, g->band_coef[g->band_offset[b]]);
    cursor = s0 + len;
  }
  if (cursor < n) add_identity(cursor, n - cursor);

  // Segment order: with detector offsets, blocks run by time within their detector first and
  // detector second, so that the segments resident together come from many detectors observing
  // at the same moment (the same patch of sky) and share pixels in L2; the segments of one block
  // stay consecutive (their windows overlap).
  std::vector<int> seg_order(order);
  if (g->det_offset != nullptr && g->n_dets > 0) {
    auto key = [g](int b) {
      const int64_t s0 = g->blk_start[b];
      const int64_t* it = std::upper_bound(g->det_offset, g->det_offset + g->n_dets + 1, s0);
      const int64_t d = (it - g->det_offset) - 1;
      return std::make_pair(s0 - g->det_offset[d], d);
    };
    std::stable_sort(seg_order.begin(), seg_order.end(),
                     [&](int a, int b) { return key(a) < key(b); });
  }
  std::vector<Chunk> chunks;
  if (algo == MM_TOEPLITZ_FFT) {
    const int64_t L = fft_n - 2 * lambda_max;
    for (int i : seg_order) {
      const int64_t s0 = g->blk_start[i], len = g->blk_len[i];
      for (int64_t o = 0; o < len; o += L)
        chunks.push_back(Chunk{s0 + o, s0, static_cast<int32_t>(len),
                               static_cast<int32_t>(std::min<int64_t>(L, len - o)),
                               g->blk_band[i], 0});
    }
  } else {
    for (int i : seg_order) {
      const int64_t s0 = g->blk_start[i], len = g->blk_len[i];
      for (int64_t o = 0; o < len; o += 1024)
        chunks.push_back(Chunk{s0 + o, s0, static_cast<int32_t>(len),
                               static_cast<int32_t>(std::min<int64_t>(1024, len - o)),
                               g->blk_band[i], 0});
    }
  }
  if (chunks.size() > static_cast<size_t>(INT32_MAX) || idseg.size() / 2 > static_cast<size_t>(INT32_MAX))
    return fail(MM_ERR_UNSUPPORTED, "too many segments");
  P->n_chunks = static_cast<int32_t>(chunks.size());
  P->n_id_seg = static_cast<int32_t>(idseg.size() / 2);
  P->h_id_seg = idseg;
  MM_TRY(upload(P, &P->chunks, chunks, s));
  MM_TRY(upload(P, &P->id_tiles, id_tiles, s));
  P->n_id_tiles = static_cast<int32_t>(id_tiles.size());
  P->fused = (g->flags & MM_FLAG_UNFUSED) == 0;
  MM_TRY(upload(P, &P->id_seg, idseg, s));

  // ---- bands -------------------------------------------------------------------------------
  int64_t n_coef_total = 0;
  for (int b = 0; b < g->n_bands; ++b)
    n_coef_total = std::max<int64_t>(n_coef_total, g->band_offset[b] + g->band_ncoef[b]);
  // straight from the caller's tables (validated above)
  MM_TRY(upload(P, &P->band_coef, g->band_coef, static_cast<size_t>(n_coef_total), s));
  MM_TRY(upload(P, &P->band_off, g->band_offset, static_cast<size_t>(g->n_bands), s));
  MM_TRY(upload(P, &P->band_ncoef, g->band_ncoef, static_cast<size_t>(g->n_bands), s));

  // ---- pointing copies + global accumulation -------------------------------------------------
  MM_TRY(dalloc(P, &P->lpix, n));
  MM_TRY(dalloc(P, &P->wq, n));
  MM_TRY(dalloc(P, &P->wu, n));
  if (n > 0) {
    MM_HIP_TRY(hipMemcpyAsync(P->wq, g->w_q, n * sizeof(float), hipMemcpyDeviceToDevice, s));
    MM_HIP_TRY(hipMemcpyAsync(P->wu, g->w_u, n * sizeof(float), hipMemcpyDeviceToDevice, s));
  }
  Scratch<double> Bg;
  Scratch<int32_t> hits_g, local, counts, err;
  Scratch<uint8_t> keep;
  Scratch<unsigned long long> ctr;  // [0] observed, [1] gap samples
  Scratch<int64_t> total;
  MM_TRY(Bg.alloc(6 * std::max<int64_t>(ng, 1)));
  MM_TRY(hits_g.alloc(std::max<int64_t>(ng, 1)));
  MM_TRY(local.alloc(ng));
  MM_TRY(keep.alloc(ng));
  MM_TRY(err.alloc(1));
  MM_TRY(ctr.alloc(2));
  MM_TRY(total.alloc(1));
  MM_TRY(dalloc(P, &P->tiles, tiles.size()));
  P->n_tiles = static_cast<int32_t>(tiles.size());
  const int n_scan = static_cast<int>((ng + kScanChunk - 1) / kScanChunk);
  MM_TRY(counts.alloc(n_scan + 1));
  MM_HIP_TRY(hipMemsetAsync(Bg.p, 0, sizeof(double) * 6 * std::max<int64_t>(ng, 1), s));
  MM_HIP_TRY(hipMemsetAsync(hits_g.p, 0, sizeof(int32_t) * std::max<int64_t>(ng, 1), s));
  MM_HIP_TRY(hipMemsetAsync(err.p, 0, sizeof(int32_t), s));
  MM_HIP_TRY(hipMemsetAsync(ctr.p, 0, 2 * sizeof(unsigned long long), s));
  MM_HIP_TRY(hipMemsetAsync(total.p, 0, sizeof(int64_t), s));
  if (!tiles.empty()) {
    MM_HIP_TRY(hipMemcpyAsync(P->tiles, tiles.data(), tiles.size() * sizeof(Tile),
                              hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_plan_accumulate, dim3(static_cast<unsigned>(tiles.size())), dim3(kThreads),
                       0, s, g->pix, g->w_q, g->w_u, P->tiles, ng, Bg.p, hits_g.p, err.p);
    MM_HIP_TRY(hipGetLastError());
  }
  int32_t h_err = 0;
  MM_HIP_TRY(hipMemcpyAsync(&h_err, err.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MM_HIP_TRY(hipStreamSynchronize(s));
  if (h_err) return fail(MM_ERR_INVALID, "pixel index out of [-1, n_pix_global)");

  // ---- classify + compact --------------------------------------------------------------------
  const double cond_max = g->cond_max > 0 ? g->cond_max : 1.0e3;
  if (ng > 0) {
    hipLaunchKernelGGL(k_plan_classify, dim3(static_cast<unsigned>((ng + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, s, Bg.p, hits_g.p, ng, cond_max, keep.p, ctr.p);
    MM_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_scan_count, dim3(n_scan), dim3(kThreads), 0, s, keep.p, ng, counts.p);
    MM_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_scan_offsets, dim3(1), dim3(1024), 0, s, counts.p, n_scan, total.p);
    MM_HIP_TRY(hipGetLastError());
  }
  int64_t n_kept = 0;
  unsigned long long h_ctr[2] = {0, 0};
  MM_HIP_TRY(hipMemcpyAsync(&n_kept, total.p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MM_HIP_TRY(hipMemcpyAsync(h_ctr, ctr.p, sizeof(h_ctr), hipMemcpyDeviceToHost, s));
  MM_HIP_TRY(hipStreamSynchronize(s));
  P->n_kept = n_kept;
  P->n_obs = static_cast<int64_t>(h_ctr[0]);
  MM_TRY(dalloc(P, &P->kept_ids, n_kept));
  MM_TRY(dalloc(P, &P->hits, n_kept));
  MM_TRY(dalloc(P, &P->minv, 6 * n_kept));
  if (ng > 0) {
    hipLaunchKernelGGL(k_scan_write, dim3(n_scan), dim3(kThreads), 0, s, keep.p, ng, counts.p,
                       Bg.p, hits_g.p, local.p, P->kept_ids, P->hits, P->minv);
    MM_HIP_TRY(hipGetLastError());
  }
  if (n > 0) {
    int64_t gr = (n + kThreads - 1) / kThreads;
    if (gr > 65536) gr = 65536;
    hipLaunchKernelGGL(k_plan_remap, dim3(static_cast<unsigned>(gr)), dim3(kThreads), 0, s, g->pix,
                       local.p, P->lpix, n, ctr.p + 1);
    MM_HIP_TRY(hipGetLastError());
  }

  // ---- band symbols: positivity on a grid of >= 8 lambda points; FFT spectra ----------------
  if (g->n_bands > 0) {
    int M = 16;
    while (M < 8 * lambda_max) M *= 2;
    if (fft_n > M) M = fft_n;
    if (algo == MM_TOEPLITZ_FFT) MM_TRY(dalloc(P, &P->spec, static_cast<size_t>(g->n_bands) * (fft_n / 2 + 1)));
    const bool two_level = M >= 4096;  // Clenshaw below: small grids are cheap either way
    const int gx = two_level ? M / (kSymP * kSymR)
                             : (M / 2 + 1 + kThreads * kSymPts - 1) / (kThreads * kSymPts);
    Scratch<double> mins;
    MM_TRY(mins.alloc(static_cast<size_t>(gx) * g->n_bands));
    if (two_level)
      hipLaunchKernelGGL(k_band_symbol2, dim3(gx, g->n_bands), dim3(kThreads), 0, s, P->band_coef,
                         P->band_off, P->band_ncoef, M, fft_n > 0 ? fft_n : M, P->spec,
                         static_cast<double*>(nullptr), mins.p);
    else
      hipLaunchKernelGGL(k_band_symbol, dim3(gx, g->n_bands), dim3(kThreads), 0, s, P->band_coef,
                         P->band_off, P->band_ncoef, M, fft_n > 0 ? fft_n : M, P->spec,
                         static_cast<double*>(nullptr), mins.p);
    MM_HIP_TRY(hipGetLastError());
    std::vector<double> h_mins(static_cast<size_t>(gx) * g->n_bands);
    MM_HIP_TRY(hipMemcpyAsync(h_mins.data(), mins.p, h_mins.size() * sizeof(double),
                              hipMemcpyDeviceToHost, s));
    MM_HIP_TRY(hipStreamSynchronize(s));
    for (int b = 0; b < g->n_bands; ++b) {
      double m = INFINITY;
      for (int x = 0; x < gx; ++x) m = std::min(m, h_mins[static_cast<size_t>(b) * gx + x]);
      if (!(m > 0.0))
        return fail(MM_ERR_NOT_SPD, "band " + std::to_string(b) + " has a non-positive symbol (" +
                                        std::to_string(m) + ")");
    }
  }
  if (algo == MM_TOEPLITZ_FFT) {
    // exp(-2 pi i m / fft_n) = coarse[m / F] * fine[m % F]; F = 128 (LDS kernels) or 512
    // (four-step kernel)
    const int F = long_fft_size(fft_n) ? long_fine_size() : 128;
    std::vector<float2> t0(F), t1(fft_n / F);
    const double two_pi = 6.283185307179586476925286766559;
    for (int m = 0; m < F; ++m) {
      const double a = -two_pi * m / fft_n;
      t0[m] = make_float2(static_cast<float>(std::cos(a)), static_cast<float>(std::sin(a)));
    }
    for (int m = 0; m < fft_n / F; ++m) {
      const double a = -two_pi * (static_cast<double>(F) * m) / fft_n;
      t1[m] = make_float2(static_cast<float>(std::cos(a)), static_cast<float>(std::sin(a)));
    }
    MM_TRY(upload(P, &P->tw0, t0, s));
    MM_TRY(upload(P, &P->tw1, t1, s));
  }

  // ---- workspace -----------------------------------------------------------------------------
  P->reg_fft = algo == MM_TOEPLITZ_FFT && P->fused && (g->flags & MM_FLAG_LDS_FFT) == 0 &&
               apply_reg_supported(P);
  if (P->reg_fft) MM_TRY(build_reg_table(P, s));
  if (algo == MM_TOEPLITZ_FFT) MM_TRY(build_long_table(P, s));
  MM_TRY(work_alloc(P, &P->work));
  P->device_bytes += P->work.bytes;

  unsigned long long h_gap = 0;
  MM_HIP_TRY(hipMemcpyAsync(&h_gap, ctr.p + 1, sizeof(h_gap), hipMemcpyDeviceToHost, s));
  MM_HIP_TRY(hipStreamSynchronize(s));
  P->n_gap = static_cast<int64_t>(h_gap);
  MM_TRY(build_templates(P, g, tiles, s));
  guard.keep = true;
  *out = P;
  return MM_OK;
}

}  // namespace mm
