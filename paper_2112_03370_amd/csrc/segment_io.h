// Per-segment time-domain I/O shared by the fused system-product kernels: the gather of
// t = P x (or of the data d) for a lane of consecutive samples, and the FP64 atomic flush of
// merged scatter runs into y = P^T u.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mm {

struct AtomicFlush {
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

template <bool kFromData>
__device__ __forceinline__ float gather_one(int key, float q, float w, const double* __restrict__ x,
                                            float dv) {
  if (key < 0) return 0.0f;
  if constexpr (kFromData) {
    return dv;
  } else {
    const double* m = x + 3 * static_cast<int64_t>(key);
    return static_cast<float>(m[0] + static_cast<double>(q) * m[1] + static_cast<double>(w) * m[2]);
  }
}

// Pointing of one lane: window samples [g, g + S), inside the block and 16-byte aligned (the
// data instead of the weights when gathering d).
template <int S, bool kFromData>
struct LanePointing {
  int kk[S];
  float qq[S], uu[S];

  __device__ __forceinline__ void load(const int32_t* __restrict__ lpix,
                                       const float* __restrict__ wq, const float* __restrict__ wu,
                                       const float* __restrict__ d, int64_t g) {
#pragma unroll
    for (int c = 0; c < S / 4; ++c) {
      const int4 k4 = *reinterpret_cast<const int4*>(lpix + g + 4 * c);
      kk[4 * c] = k4.x;
      kk[4 * c + 1] = k4.y;
      kk[4 * c + 2] = k4.z;
      kk[4 * c + 3] = k4.w;
      const float4 q4 = *reinterpret_cast<const float4*>((kFromData ? d : wq) + g + 4 * c);
      qq[4 * c] = q4.x;
      qq[4 * c + 1] = q4.y;
      qq[4 * c + 2] = q4.z;
      qq[4 * c + 3] = q4.w;
      if constexpr (!kFromData) {
        const float4 u4 = *reinterpret_cast<const float4*>(wu + g + 4 * c);
        uu[4 * c] = u4.x;
        uu[4 * c + 1] = u4.y;
        uu[4 * c + 2] = u4.z;
        uu[4 * c + 3] = u4.w;
      }
    }
  }

  // Scan runs keep a pixel for several consecutive samples, so a lane usually sees one or two
  // pixels: it loads the pixels of its first and last samples together, behind a single wait,
  // and goes back for a third pixel only when one occurs.
  __device__ __forceinline__ void resolve(const double* __restrict__ x, float (&v)[S]) const {
    if constexpr (kFromData) {
#pragma unroll
      for (int j = 0; j < S; ++j) v[j] = kk[j] < 0 ? 0.0f : qq[j];
    } else {
      const int ka = kk[0], kb = kk[S - 1];
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
      for (int j = 0; j < S; ++j) {
        const int key = kk[j];
        other |= key >= 0 && key != ka && key != kb;
        // both candidate pixels' sums, then one select (cheaper than selecting three FP64
        // pixel values)
        const double q = static_cast<double>(qq[j]), u = static_cast<double>(uu[j]);
        const double ta = a0 + q * a1 + u * a2;
        const double tb = b0 + q * b1 + u * b2;
        v[j] = key < 0 ? 0.0f : static_cast<float>(key == ka ? ta : tb);
      }
      if (other) {  // a third pixel inside the lane
#pragma unroll
        for (int j = 0; j < S; ++j) {
          const int key = kk[j];
          if (key >= 0 && key != ka && key != kb) {
            const double* m = x + 3 * static_cast<int64_t>(key);
            v[j] = static_cast<float>(m[0] + static_cast<double>(qq[j]) * m[1] +
                                      static_cast<double>(uu[j]) * m[2]);
          }
        }
      }
    }
  }
};

}  // namespace mm
