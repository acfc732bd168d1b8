// Pointing products on the GPU: un-pointing t = P x and pointing y = P^T u (MAPMAT core
// operations), plus the data mask used for the right-hand side.
//
// Layout: per-sample arrays are separate coalesced streams (local pixel int32, cos/sin FP32);
// each thread owns 8 consecutive samples, read with two 16-byte loads per stream.  Pixel-domain
// vectors are FP64 [n_kept][3] and stay cache-resident while the time streams go by; the
// un-pointing loads the pixels of a thread's first and last samples together and a third pixel
// only when one occurs (scan runs make that rare), since these kernels are bound by the count
// and the latency of vector memory instructions rather than by bytes.  P^T accumulates in FP64: samples of one
// pixel arrive in runs (the scan dwells on a pixel for several samples), so each thread first
// sums its own run pieces, then a wavefront segmented scan merges runs that continue across
// lanes, and only the lane that closes a run issues the three FP64 atomic adds.
#include "mm_internal.h"
#include "wave_runs.h"

namespace mm {

namespace {

constexpr int kThreads = 256;
constexpr int kPerThread = 4;              // diagonal kernel
constexpr int kPerBlock = kThreads * kPerThread;
constexpr int kLane = 8;                   // un-pointing and pointing
constexpr int kLaneBlock = kThreads * kLane;
constexpr int kListed = 128;                // listed runs per wavefront in the scatter

inline int grid_for(int64_t n, int per_block = kPerBlock) {
  int64_t g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return static_cast<int>(g);
}

__global__ __launch_bounds__(kThreads) void k_unpoint(const int32_t* __restrict__ lpix,
                                                      const float* __restrict__ wq,
                                                      const float* __restrict__ wu,
                                                      const double* __restrict__ x,
                                                      float* __restrict__ t, int64_t n,
                                                      const int32_t* __restrict__ done) {
  if (done != nullptr && *done) return;
  for (int64_t i0 = (static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x) * kLane;
       i0 < n; i0 += static_cast<int64_t>(gridDim.x) * kLaneBlock) {
    if (i0 + kLane <= n) {
      int key[kLane];
      float qq[kLane], uu[kLane], out[kLane];
#pragma unroll
      for (int c = 0; c < kLane / 4; ++c) {
        const int4 k4 = *reinterpret_cast<const int4*>(lpix + i0 + 4 * c);
        const float4 q4 = *reinterpret_cast<const float4*>(wq + i0 + 4 * c);
        const float4 u4 = *reinterpret_cast<const float4*>(wu + i0 + 4 * c);
        key[4 * c] = k4.x; key[4 * c + 1] = k4.y; key[4 * c + 2] = k4.z; key[4 * c + 3] = k4.w;
        qq[4 * c] = q4.x; qq[4 * c + 1] = q4.y; qq[4 * c + 2] = q4.z; qq[4 * c + 3] = q4.w;
        uu[4 * c] = u4.x; uu[4 * c + 1] = u4.y; uu[4 * c + 2] = u4.z; uu[4 * c + 3] = u4.w;
      }
      // the pixels of the first and last samples are loaded together behind one wait; a third
      // pixel inside the lane (rare along scan runs) is loaded afterwards
      const int ka = key[0], kb = key[kLane - 1];
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
      for (int j = 0; j < kLane; ++j) {
        other |= key[j] >= 0 && key[j] != ka && key[j] != kb;
        // both candidate pixels' sums, then one select
        const double q = static_cast<double>(qq[j]), u = static_cast<double>(uu[j]);
        const double ta = a0 + q * a1 + u * a2;
        const double tb = b0 + q * b1 + u * b2;
        out[j] = key[j] < 0 ? 0.0f : static_cast<float>(key[j] == ka ? ta : tb);
      }
      if (other) {
#pragma unroll
        for (int j = 0; j < kLane; ++j) {
          if (key[j] >= 0 && key[j] != ka && key[j] != kb) {
            const double* m = x + 3 * static_cast<int64_t>(key[j]);
            out[j] = static_cast<float>(m[0] + static_cast<double>(qq[j]) * m[1] +
                                        static_cast<double>(uu[j]) * m[2]);
          }
        }
      }
#pragma unroll
      for (int c = 0; c < kLane / 4; ++c)
        *reinterpret_cast<float4*>(t + i0 + 4 * c) =
            make_float4(out[4 * c], out[4 * c + 1], out[4 * c + 2], out[4 * c + 3]);
    } else {
      for (int64_t i = i0; i < n; ++i) {
        const int k = lpix[i];
        double v = 0.0;
        if (k >= 0) {
          const double* m = x + 3 * static_cast<int64_t>(k);
          v = m[0] + static_cast<double>(wq[i]) * m[1] + static_cast<double>(wu[i]) * m[2];
        }
        t[i] = static_cast<float>(v);
      }
    }
  }
}

// Scalar variant for unaligned caller buffers.
__global__ __launch_bounds__(kThreads) void k_unpoint_scalar(const int32_t* __restrict__ lpix,
                                                             const float* __restrict__ wq,
                                                             const float* __restrict__ wu,
                                                             const double* __restrict__ x,
                                                             float* __restrict__ t, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    const int k = lpix[i];
    double v = 0.0;
    if (k >= 0) {
      const double* m = x + 3 * static_cast<int64_t>(k);
      v = m[0] + static_cast<double>(wq[i]) * m[1] + static_cast<double>(wu[i]) * m[2];
    }
    t[i] = static_cast<float>(v);
  }
}

// t = d at kept samples, 0 at gap samples (flagged or excised: zero rows of P).
__global__ __launch_bounds__(kThreads) void k_mask_data(const int32_t* __restrict__ lpix,
                                                        const float* __restrict__ d,
                                                        float* __restrict__ t, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    t[i] = lpix[i] >= 0 ? d[i] : 0.0f;
  }
}

struct PointFlush {
  double* y;
  __device__ void operator()(int key, const double (&v)[3]) const {
    double* dst = y + 3 * static_cast<int64_t>(key);
    unsafeAtomicAdd(dst + 0, v[0]);
    unsafeAtomicAdd(dst + 1, v[1]);
    unsafeAtomicAdd(dst + 2, v[2]);
  }
  __device__ void one(int key, int c, double v) const {
    unsafeAtomicAdd(y + 3 * static_cast<int64_t>(key) + c, v);
  }
};

template <bool kVec>
__global__ __launch_bounds__(kThreads) void k_point(const int32_t* __restrict__ lpix,
                                                    const float* __restrict__ wq,
                                                    const float* __restrict__ wu,
                                                    const float* __restrict__ u,
                                                    double* __restrict__ y, int64_t n,
                                                    const int32_t* __restrict__ done) {
  if (done != nullptr && *done) return;
  const PointFlush flush{y};
  // per wavefront: the runs it completes, listed before the atomics
  __shared__ int skey[kThreads / 64][kListed];
  __shared__ double sval[kThreads / 64][3 * kListed];
  const int wave = static_cast<int>(threadIdx.x >> 6);
  // Every lane of the block runs the same number of iterations (wavefront-collective scan).
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * kLaneBlock; base < n;
       base += static_cast<int64_t>(gridDim.x) * kLaneBlock) {
    const int64_t i0 = base + static_cast<int64_t>(threadIdx.x) * kLane;
    int key[kLane];
    double v[kLane][3];
    if (kVec && i0 + kLane <= n) {
#pragma unroll
      for (int c = 0; c < kLane / 4; ++c) {
        const int4 k4 = *reinterpret_cast<const int4*>(lpix + i0 + 4 * c);
        const float4 q4 = *reinterpret_cast<const float4*>(wq + i0 + 4 * c);
        const float4 w4 = *reinterpret_cast<const float4*>(wu + i0 + 4 * c);
        const float4 t4 = *reinterpret_cast<const float4*>(u + i0 + 4 * c);
        const int kq[4] = {k4.x, k4.y, k4.z, k4.w};
        const float qq[4] = {q4.x, q4.y, q4.z, q4.w};
        const float ww[4] = {w4.x, w4.y, w4.z, w4.w};
        const float tt[4] = {t4.x, t4.y, t4.z, t4.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const double tv = tt[j];
          key[4 * c + j] = kq[j];
          v[4 * c + j][0] = tv;
          v[4 * c + j][1] = static_cast<double>(qq[j]) * tv;
          v[4 * c + j][2] = static_cast<double>(ww[j]) * tv;
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < kLane; ++j) {
        const int64_t i = i0 + j;
        key[j] = -1;
        v[j][0] = v[j][1] = v[j][2] = 0.0;
        if (i < n) {
          key[j] = lpix[i];
          const double tv = u[i];
          v[j][0] = tv;
          v[j][1] = static_cast<double>(wq[i]) * tv;
          v[j][2] = static_cast<double>(wu[i]) * tv;
        }
      }
    }
    wave_merge_runs_listed<kLane, 3, kListed, PointFlush, true>(key, v, flush, skey[wave],
                                                               sval[wave]);
  }
}

// Diagonal weights: per tile of samples with one weight c_0, y += P^T (c_0 (P x)) or
// y += P^T (c_0 d) with every product in FP64 (no FP32 time-domain intermediate).
__global__ __launch_bounds__(kThreads) void k_diag_apply(const int32_t* __restrict__ lpix,
                                                         const float* __restrict__ wq,
                                                         const float* __restrict__ wu,
                                                         const Tile* __restrict__ tiles,
                                                         const double* __restrict__ x,
                                                         const float* __restrict__ d,
                                                         double* __restrict__ y,
                                                         const int32_t* __restrict__ done) {
  if (done != nullptr && *done) return;
  const Tile tl = tiles[blockIdx.x];
  const PointFlush flush{y};
  const double c0 = tl.c0;
  for (int off = 0; off < tl.len; off += kPerBlock) {
    int key[4];
    double v[4][3];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int o = off + threadIdx.x * kPerThread + j;
      key[j] = -1;
      v[j][0] = v[j][1] = v[j][2] = 0.0;
      if (o < tl.len) {
        const int64_t i = tl.start + o;
        const int k = lpix[i];
        if (k >= 0) {
          const double q = wq[i], w = wu[i];
          double tv;
          if (x != nullptr) {
            const double* m = x + 3 * static_cast<int64_t>(k);
            tv = m[0] + q * m[1] + w * m[2];
          } else {
            tv = d[i];
          }
          tv *= c0;
          key[j] = k;
          v[j][0] = tv;
          v[j][1] = q * tv;
          v[j][2] = w * tv;
        }
      }
    }
    wave_merge_runs<3>(key, v, flush);
  }
}

__global__ void k_zero(double* __restrict__ y, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    y[i] = 0.0;
}

inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

mm_status launch_diag_tiles(Plan* P, const Tile* tiles, int32_t n_tiles, const double* x,
                            const float* d, double* y, const int32_t* done, hipStream_t s) {
  if (n_tiles == 0 || P->n_kept == 0) return MM_OK;
  TimedLaunch tl(P, K_POINT, s);
  hipLaunchKernelGGL(k_diag_apply, dim3(n_tiles), dim3(kThreads), 0, s, P->lpix, P->wq, P->wu,
                     tiles, x, d, y, done);
  MM_HIP_TRY(hipGetLastError());
  return MM_OK;
}

mm_status launch_diag_apply(Plan* P, const double* x, const float* d, double* y,
                            const int32_t* done, hipStream_t s) {
  return launch_diag_tiles(P, P->tiles, P->n_tiles, x, d, y, done, s);
}

mm_status launch_zero(double* y, int64_t n, hipStream_t s) {
  if (n <= 0) return MM_OK;
  int64_t g = (n + 255) / 256;
  if (g > 16384) g = 16384;
  hipLaunchKernelGGL(k_zero, dim3(static_cast<unsigned>(g)), dim3(256), 0, s, y, n);
  MM_HIP_TRY(hipGetLastError());
  return MM_OK;
}

mm_status launch_unpoint(Plan* P, const double* x, float* t, const int32_t* done,
                         hipStream_t s) {
  const int64_t n = P->n_samples;
  if (n == 0) return MM_OK;
  TimedLaunch tl(P, K_UNPOINT, s);
  if (aligned16(t)) {
    hipLaunchKernelGGL(k_unpoint, dim3(grid_for(n, kLaneBlock)), dim3(kThreads), 0, s, P->lpix, P->wq, P->wu,
                       x, t, n, done);
  } else {
    int64_t g = (n + kThreads - 1) / kThreads;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_unpoint_scalar, dim3(static_cast<unsigned>(g)), dim3(kThreads), 0, s,
                       P->lpix, P->wq, P->wu, x, t, n);
  }
  MM_HIP_TRY(hipGetLastError());
  return MM_OK;
}

mm_status launch_mask_data(Plan* P, const float* d, float* t, hipStream_t s) {
  const int64_t n = P->n_samples;
  if (n == 0) return MM_OK;
  int64_t g = (n + kThreads - 1) / kThreads;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_mask_data, dim3(static_cast<unsigned>(g)), dim3(kThreads), 0, s, P->lpix,
                     d, t, n);
  MM_HIP_TRY(hipGetLastError());
  return MM_OK;
}

mm_status launch_point(Plan* P, const float* u, double* y, bool zero_first, const int32_t* done,
                       hipStream_t s) {
  if (zero_first) MM_TRY(launch_zero(y, 3 * P->n_kept, s));
  const int64_t n = P->n_samples;
  if (n == 0 || P->n_kept == 0) return MM_OK;
  TimedLaunch tl(P, K_POINT, s);
  if (aligned16(u)) {
    hipLaunchKernelGGL(k_point<true>, dim3(grid_for(n, kLaneBlock)), dim3(kThreads), 0, s, P->lpix, P->wq,
                       P->wu, u, y, n, done);
  } else {
    hipLaunchKernelGGL(k_point<false>, dim3(grid_for(n, kLaneBlock)), dim3(kThreads), 0, s, P->lpix, P->wq,
                       P->wu, u, y, n, done);
  }
  MM_HIP_TRY(hipGetLastError());
  return MM_OK;
}

}  // namespace mm
