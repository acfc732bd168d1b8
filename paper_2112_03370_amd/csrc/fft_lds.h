// LDS-resident FP32 FFT building blocks for the overlap-save Toeplitz product.
//
// NC = 2^LOG complex points live in LDS (one pad slot per 16 values); T = NC/16 threads each
// move 16 values per Stockham pass (radix 16, then one radix-8/4/2 pass).  Twiddles
// exp(-2 pi i m / N), N = 2 NC, come from a two-level table (coarse[m >> 7] * fine[m & 127]).
#pragma once

#include <hip/hip_runtime.h>

namespace mm {
namespace fft {


__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }  // -i a

// Forward radix-4 butterfly in place (X_k = sum_n x_n exp(-2 pi i nk/4)).
__device__ __forceinline__ void dft4(float2& x0, float2& x1, float2& x2, float2& x3) {
  const float2 t0 = cadd(x0, x2), t1 = csub(x0, x2), t2 = cadd(x1, x3), t3 = mul_mi(csub(x1, x3));
  x0 = cadd(t0, t2);
  x2 = csub(t0, t2);
  x1 = cadd(t1, t3);
  x3 = csub(t1, t3);
}

constexpr float kC1 = 0.92387953251128674f;  // cos(pi/8)
constexpr float kS1 = 0.38268343236508978f;  // sin(pi/8)
constexpr float kR2 = 0.70710678118654752f;  // sqrt(2)/2

// Radix-R forward DFT on v[0..R); result X_m is left at v[perm(m)], see out_slot().
template <int R>
__device__ __forceinline__ void dft(float2* v);

template <>
__device__ __forceinline__ void dft<2>(float2* v) {
  const float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <>
__device__ __forceinline__ void dft<4>(float2* v) {
  dft4(v[0], v[1], v[2], v[3]);
}

// 8 = 4 x 2: n = 2 n1 + n2, k = k1 + 4 k2; X[k1 + 4 k2] ends at v[2 k1 + k2].
template <>
__device__ __forceinline__ void dft<8>(float2* v) {
  dft4(v[0], v[2], v[4], v[6]);
  dft4(v[1], v[3], v[5], v[7]);
  v[3] = cmul(v[3], make_float2(kR2, -kR2));
  v[5] = mul_mi(v[5]);
  v[7] = cmul(v[7], make_float2(-kR2, -kR2));
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    const float2 a = v[2 * k1], b = v[2 * k1 + 1];
    v[2 * k1] = cadd(a, b);
    v[2 * k1 + 1] = csub(a, b);
  }
}

// 16 = 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2; X[k1 + 4 k2] ends at v[4 k1 + k2].
template <>
__device__ __forceinline__ void dft<16>(float2* v) {
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
  // twiddles W16^(n2 k1) on v[4 k1 + n2]
  const float2 w1 = make_float2(kC1, -kS1), w2 = make_float2(kR2, -kR2), w3 = make_float2(kS1, -kC1);
  const float2 w6 = make_float2(-kR2, -kR2), w9 = make_float2(-kC1, kS1);
  v[5] = cmul(v[5], w1);
  v[6] = cmul(v[6], w2);
  v[7] = cmul(v[7], w3);
  v[9] = cmul(v[9], w2);
  v[10] = mul_mi(v[10]);
  v[11] = cmul(v[11], w6);
  v[13] = cmul(v[13], w3);
  v[14] = cmul(v[14], w6);
  v[15] = cmul(v[15], w9);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) dft4(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
}

template <int R>
__device__ __forceinline__ int out_slot(int m) {
  if constexpr (R == 16) return 4 * (m & 3) + (m >> 2);
  if constexpr (R == 8) return 2 * (m & 3) + (m >> 2);
  return m;
}

// LDS index with one pad slot per 16 complex values (spreads power-of-two strides over banks).
__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }

// exp(-2 pi i m / N) from the two-level table (m in [0, N)).
__device__ __forceinline__ float2 twiddle(const float2* tw0, const float2* tw1, int m) {
  return cmul(tw1[m >> 7], tw0[m & 127]);
}

// One Stockham pass of radix R over NC complex points held in LDS (T threads; every thread
// handles 16 / R butterflies so that each pass moves 16 values per thread).
template <int NC, int T, int R>
__device__ __forceinline__ void fft_pass(float2* buf, int p, const float2* tw0, const float2* tw1) {
  constexpr int B = NC / R;       // butterflies in the pass
  constexpr int PER = B / T;      // butterflies per thread
  static_assert(PER * R == 16, "16 values per thread per pass");
  const int tid = threadIdx.x;
  const int stride_n = (2 * NC) / (p * R);  // twiddle index step on the 2*NC grid
  float2 v[16];
#pragma unroll
  for (int bi = 0; bi < PER; ++bi) {
    const int b = tid + bi * T;
    const int k = b & (p - 1);
    float2* u = v + bi * R;
#pragma unroll
    for (int j = 0; j < R; ++j) u[j] = buf[pad(b + j * B)];
    if (p > 1) {
      const int base = k * stride_n;  // angle index of j = 1, < 2*NC
      float2 w[16];
      w[1] = twiddle(tw0, tw1, base);
      if constexpr (R >= 4) w[2] = twiddle(tw0, tw1, (2 * base) & (2 * NC - 1));
      if constexpr (R >= 8) w[4] = twiddle(tw0, tw1, (4 * base) & (2 * NC - 1));
      if constexpr (R >= 16) w[8] = twiddle(tw0, tw1, (8 * base) & (2 * NC - 1));
      if constexpr (R >= 4) w[3] = cmul(w[1], w[2]);
      if constexpr (R >= 8) {
        w[5] = cmul(w[1], w[4]);
        w[6] = cmul(w[2], w[4]);
        w[7] = cmul(w[3], w[4]);
      }
      if constexpr (R >= 16) {
#pragma unroll
        for (int j = 9; j < 16; ++j) w[j] = cmul(w[j - 8], w[8]);
      }
#pragma unroll
      for (int j = 1; j < R; ++j) u[j] = cmul(u[j], w[j]);
    }
    dft<R>(u);
  }
  __syncthreads();
#pragma unroll
  for (int bi = 0; bi < PER; ++bi) {
    const int b = tid + bi * T;
    const int k = b & (p - 1);
    const int base = (b - k) * R + k;
    const float2* u = v + bi * R;
#pragma unroll
    for (int m = 0; m < R; ++m) buf[pad(base + m * p)] = u[out_slot<R>(m)];
  }
  __syncthreads();
}

// Forward complex FFT of NC = 2^LOG points in LDS: radix-16 passes, then one smaller pass.
template <int LOG, int T>
__device__ __forceinline__ void fft_forward(float2* buf, const float2* tw0, const float2* tw1) {
  constexpr int NC = 1 << LOG;
  constexpr int N16 = LOG / 4;
  constexpr int REM = LOG % 4;
  int p = 1;
#pragma unroll
  for (int i = 0; i < N16; ++i) {
    fft_pass<NC, T, 16>(buf, p, tw0, tw1);
    p *= 16;
  }
  if constexpr (REM == 3) fft_pass<NC, T, 8>(buf, p, tw0, tw1);
  if constexpr (REM == 2) fft_pass<NC, T, 4>(buf, p, tw0, tw1);
  if constexpr (REM == 1) fft_pass<NC, T, 2>(buf, p, tw0, tw1);
}

// Workgroups are dispatched to the 8 XCDs in turn: give each XCD a contiguous run of segments
// so neighbouring segments of a block (which share their lambda halos) meet in the same L2.
__device__ __forceinline__ int xcd_ordered(int bid, int nblocks) {
  const int x = bid & 7, r = bid >> 3;
  const int per = nblocks >> 3, extra = nblocks & 7;
  return x * per + (x < extra ? x : extra) + r;
}

template <int LOG>
struct FftCfg {
  static constexpr int NC = 1 << LOG;   // complex points
  static constexpr int N = 2 * NC;      // real samples per segment
  static constexpr int T = NC / 16;     // threads
  static constexpr int LDS = NC + NC / 16;
};


// Real spectrum step between the two transforms.  The N real samples are packed as NC complex
// values z[m] = t[2m] + i t[2m+1] with transform Z; the step unpacks the real spectrum X at k
// and NC - k, multiplies by the band symbol S (already scaled by 1/(2N)), repacks for the
// inverse transform and stores the conjugate (the inverse transform is the conjugate of the
// forward transform of the conjugate).  Written out, that chain of linear maps collapses to two
// real coefficients per output: with W = exp(-2 pi i k / N) = c - i s, sigma = S[k] + S[NC-k]
// and delta = S[k] - S[NC-k],
//   Z'[k]    = 2 (sigma - delta s) conj(Z[k])    - 2 i delta c Z[NC-k]
//   Z'[NC-k] = 2 (sigma + delta s) conj(Z[NC-k]) - 2 i delta c Z[k]
// Each thread owns R = NC / (2T) pairs (k, NC - k), k = tid + r T, and thread 0 also the middle
// bin k = NC/2.  The pairs are disjoint, so the loads of a batch of pairs (the symbol from
// global memory, the spectrum from LDS) are all issued before its stores: one memory latency
// per batch instead of one per pair.
template <int LOG, int T>
__device__ __forceinline__ void symbol_multiply(float2* buf, const float* __restrict__ S,
                                                const float2* tw0, const float2* tw1) {
  constexpr int NC = 1 << LOG;
  constexpr int R = NC / (2 * T);
  constexpr int B = 4;  // pairs per batch
  static_assert(R * 2 * T == NC && R % B == 0, "pairs per thread");
  const int tid = threadIdx.x;
  const float s_mid = tid == 0 ? S[NC / 2] : 0.0f;
#pragma unroll
  for (int r0 = 0; r0 < R; r0 += B) {
    float sa[B], sb[B];
    float2 Z[B], Z2[B], W[B];
#pragma unroll
    for (int r = 0; r < B; ++r) {
      const int k = tid + (r0 + r) * T;
      sa[r] = S[k];
      sb[r] = S[NC - k];
    }
#pragma unroll
    for (int r = 0; r < B; ++r) {
      const int k = tid + (r0 + r) * T;
      Z[r] = buf[pad(k)];
      Z2[r] = buf[pad((NC - k) & (NC - 1))];
      W[r] = twiddle(tw0, tw1, k);
    }
#pragma unroll
    for (int r = 0; r < B; ++r) {
      const int k = tid + (r0 + r) * T;
      const int k2 = (NC - k) & (NC - 1);
      const float a = 2.0f * sa[r], b = 2.0f * sb[r];
      const float sig = a + b, del = a - b;
      const float ds = del * W[r].y;  // -2 delta s
      const float p = sig + ds, p2 = sig - ds, q = del * W[r].x;
      buf[pad(k)] = make_float2(p * Z[r].x + q * Z2[r].y, -(p * Z[r].y + q * Z2[r].x));
      if (k2 != k)  // k = 0 pairs with itself
        buf[pad(k2)] = make_float2(p2 * Z2[r].x + q * Z[r].y, -(p2 * Z2[r].y + q * Z[r].x));
    }
  }
  if (tid == 0) {  // k = NC/2: s = 1, c = 0, delta = 0
    const float2 Z = buf[pad(NC / 2)];
    const float p = 4.0f * s_mid;
    buf[pad(NC / 2)] = make_float2(p * Z.x, -(p * Z.y));
  }
  __syncthreads();
}

// Real sample n of the inverse transform held in buf (y[2m] = Re, y[2m+1] = -Im).
__device__ __forceinline__ float real_out(const float2* buf, int n) {
  const float2 v = buf[pad(n >> 1)];
  return (n & 1) ? -v.y : v.x;
}

}  // namespace fft
}  // namespace mm
