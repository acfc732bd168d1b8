// FP64 system product: y = P^T N^-1 P x and b = P^T N^-1 d with every step in FP64.
//
// The mixed-precision products keep the time domain in FP32 and run the Toeplitz transform in
// FP32, which leaves an operator error of a few 1e-8 relative: enough to keep the true residual
// ||b - A x|| / ||b|| (Eq. CGresidual) of a converged solve above 1e-8 when b and A are taken
// in FP64.  This module computes the FP64 operator itself, for the exit check of that residual,
// for iterative refinement, and for plans built with MM_PRECISION_FP64.  Accuracy, not speed,
// sets its design; it runs on the plan's own segment table:
//
//   FFT plans      the overlap-save segments of the plan (N real samples each, N - 2 lambda
//                  outputs).  A batch of segments is staged in two device tiles of N/2 complex
//                  FP64 points per segment and transformed by radix-16 Stockham passes (a last
//                  pass of radix 2, 4 or 8), one kernel launch per pass for the whole batch:
//                    load      window samples t_s = x[p,0] + c_s x[p,1] + s_s x[p,2] (or the
//                              data sample), zero outside the block, packed as complex points
//                              z[n] = t[2n] + i t[2n+1]
//                    forward   Z = DFT_{N/2}(z)
//                    spectrum  real spectrum X[k] = E[k] + W_N^k O[k] from the pair Z[k],
//                              Z[N/2 - k], times the band symbol S[k] = c_0 + 2 sum c_j
//                              cos(2 pi j k / N) (FP64, unscaled), repacked for the half-length
//                              inverse and conjugated, so that a forward transform inverts it
//                    forward   G = DFT_{N/2}(conj Q); y[2n] = Re G[n] / N, y[2n+1] = -Im G[n] / N
//                    scatter   outputs lambda .. lambda + out_len of each segment, P^T in FP64
//                              through the wavefront run merge
//   direct plans   each tile of <= 1024 outputs stages its window of FP64 samples in LDS and
//                  sums c_|j| t_(i+j) over |j| <= lambda in FP64
//   lambda = 0     the diagonal product, which is FP64 already
// Samples outside every block (identity rows) use the FP64 diagonal product with weight 1.
#include <cmath>

#include "mm_internal.h"
#include "wave_runs.h"

namespace mm {

namespace {

constexpr int kXThreads = 256;
constexpr size_t kTileBudget = size_t{256} << 20;  // bytes per staging tile

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 mul_minus_i(double2 a) { return make_double2(a.y, -a.x); }

// exp(-2 pi i m / 16), m in [0, 16): exact constants cos(pi/8), sin(pi/8), sqrt(1/2).
__device__ __forceinline__ double2 w16(int m) {
  constexpr double c = 0.92387953251128675613, s = 0.38268343236508977173,
                   r = 0.70710678118654752440;
  constexpr double re[16] = {1, c, r, s, 0, -s, -r, -c, -1, -c, -r, -s, 0, s, r, c};
  constexpr double im[16] = {0, -s, -r, -c, -1, -c, -r, -s, 0, s, r, c, 1, c, r, s};
  return make_double2(re[m & 15], im[m & 15]);
}

__device__ __forceinline__ void dft2(double2& a, double2& b) {
  const double2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

// In-place 4-point forward DFT of (a0, a1, a2, a3), natural order out.
__device__ __forceinline__ void dft4(double2& a0, double2& a1, double2& a2, double2& a3) {
  const double2 s02 = cadd(a0, a2), d02 = csub(a0, a2);
  const double2 s13 = cadd(a1, a3), d13 = mul_minus_i(csub(a1, a3));
  a0 = cadd(s02, s13);
  a2 = csub(s02, s13);
  a1 = cadd(d02, d13);
  a3 = csub(d02, d13);
}

// Forward DFT of R points in registers, natural order in and out.  R = 8 and 16 split as
// (R/4 or 4) x 4: X[k1 + 4 k2] = sum_j1 W_R^(j1 k1) W_(R/4)^(j1 k2) sum_j2 v[j1 + A j2] W_4^(j2 k1)
// with A = R / 4 inner sequences.
template <int R>
__device__ __forceinline__ void dft(double2 (&v)[R]) {
  if constexpr (R == 2) {
    dft2(v[0], v[1]);
  } else if constexpr (R == 4) {
    dft4(v[0], v[1], v[2], v[3]);
  } else {
    constexpr int A = R / 4;  // 2 or 4
    double2 a[A][4];
#pragma unroll
    for (int j1 = 0; j1 < A; ++j1) {
      a[j1][0] = v[j1];
      a[j1][1] = v[j1 + A];
      a[j1][2] = v[j1 + 2 * A];
      a[j1][3] = v[j1 + 3 * A];
      dft4(a[j1][0], a[j1][1], a[j1][2], a[j1][3]);
#pragma unroll
      for (int k1 = 1; k1 < 4; ++k1)
        if (j1 > 0) a[j1][k1] = cmul(a[j1][k1], w16((16 / R) * j1 * k1));
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      if constexpr (A == 4) {
        double2 b0 = a[0][k1], b1 = a[1][k1], b2 = a[2][k1], b3 = a[3][k1];
        dft4(b0, b1, b2, b3);
        v[k1] = b0;
        v[k1 + 4] = b1;
        v[k1 + 8] = b2;
        v[k1 + 12] = b3;
      } else {
        double2 b0 = a[0][k1], b1 = a[1][k1];
        dft2(b0, b1);
        v[k1] = b0;
        v[k1 + 4] = b1;
      }
    }
  }
}

// exp(-2 pi i k / N) for k in [0, N) from the table of its first N/2 values.
__device__ __forceinline__ double2 tw_n(const double2* __restrict__ tw, int k, int NC) {
  if (k < NC) return tw[k];
  const double2 t = tw[k - NC];
  return make_double2(-t.x, -t.y);
}

// What the FP64 product gathers as its time stream: P x (kInMap), the data d (kInData), or the
// time-domain residual d - P x (kInResid; zero at flagged samples as d is), so that one product
// gives P^T N^-1 (d - P x) = b - A x without the cancellation of two large products.
enum : int { kInMap = 0, kInData = 1, kInResid = 2 };

// ---- load: window samples of each segment, packed as complex points -----------------------
template <int kIn>
__global__ __launch_bounds__(kXThreads) void k_x_load(
    const int32_t* __restrict__ lpix, const float* __restrict__ wq, const float* __restrict__ wu,
    const double* __restrict__ x, const float* __restrict__ d, const Chunk* __restrict__ chunks,
    int seg0, int lam, int NC, double2* __restrict__ tile) {
  const int n = blockIdx.x * kXThreads + threadIdx.x;
  if (n >= NC) return;
  const Chunk c = chunks[seg0 + blockIdx.y];
  const int64_t b0 = c.blk_start, b1 = c.blk_start + c.blk_len;
  double v[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int64_t g = c.out0 - lam + 2 * static_cast<int64_t>(n) + h;
    double t = 0.0;
    if (g >= b0 && g < b1) {
      const int p = lpix[g];
      if (p >= 0) {
        if constexpr (kIn == kInData) {
          t = static_cast<double>(d[g]);
        } else {
          const double* m = x + 3 * static_cast<int64_t>(p);
          t = m[0] + static_cast<double>(wq[g]) * m[1] + static_cast<double>(wu[g]) * m[2];
          if constexpr (kIn == kInResid) t = static_cast<double>(d[g]) - t;
        }
      }
    }
    v[h] = t;
  }
  tile[static_cast<int64_t>(blockIdx.y) * NC + n] = make_double2(v[0], v[1]);
}

// ---- one radix-R Stockham pass over every segment of the batch ---------------------------
// Butterfly b < NC / R with k = b mod p (p = product of the radices before): inputs at
// b + j NC/R, twiddles W_(pR)^(j k), outputs at (b - k) R + k + m p.
template <int R>
__global__ __launch_bounds__(kXThreads) void k_x_pass(const double2* __restrict__ in,
                                                      double2* __restrict__ out,
                                                      const double2* __restrict__ tw, int NC,
                                                      int p) {
  const int L = NC / R;
  const int b = blockIdx.x * kXThreads + threadIdx.x;
  if (b >= L) return;
  const int64_t base = static_cast<int64_t>(blockIdx.y) * NC;
  const int k = b & (p - 1);
  double2 v[R];
#pragma unroll
  for (int j = 0; j < R; ++j) v[j] = in[base + b + j * L];
  if (p > 1) {
    // W_(pR)^(j k) = W_N^(2 j k NC / (p R)) with N = 2 NC
    const int step = 2 * k * (NC / (p * R));
#pragma unroll
    for (int j = 1; j < R; ++j) v[j] = cmul(v[j], tw_n(tw, j * step, NC));
  }
  dft<R>(v);
  const int64_t o = base + static_cast<int64_t>(b - k) * R + k;
#pragma unroll
  for (int m = 0; m < R; ++m) out[o + m * p] = v[m];
}

// Radix-256 Stockham pass: the two radix-16 levels of a 256-point DFT in one read and one write
// of the batch.  With j = 16 j1 + j2 and m = m1 + 16 m2,
//   X[m1 + 16 m2] = sum_j2 W_16^(j2 m2) W_256^(j2 m1) sum_j1 W_16^(j1 m1) v[16 j1 + j2];
// a workgroup takes 16 consecutive butterflies b (g = b mod 16 fastest, so each load and store
// touches 16 consecutive points); thread (g, h) first runs the inner DFT over j1 for j2 = h, then,
// after the exchange in LDS, the outer DFT over j2 for m1 = h.
__global__ __launch_bounds__(kXThreads) void k_x_pass256(const double2* __restrict__ in,
                                                         double2* __restrict__ out,
                                                         const double2* __restrict__ tw, int NC,
                                                         int p) {
  static_assert(kXThreads == 256, "16 butterflies x 16 threads");
  constexpr int R = 256;
  __shared__ double2 sh[16 * 16 * 17];  // [m1][j2][g], rows of 16 padded to 17
  const int L = NC / R;
  const int g = static_cast<int>(threadIdx.x & 15u), h = static_cast<int>(threadIdx.x >> 4);
  const int b = blockIdx.x * 16 + g;
  const bool live = b < L;
  const int64_t base = static_cast<int64_t>(blockIdx.y) * NC;
  const int k = b & (p - 1);
  double2 v[16];
  if (live) {
#pragma unroll
    for (int j1 = 0; j1 < 16; ++j1) v[j1] = in[base + b + static_cast<int64_t>(16 * j1 + h) * L];
    if (p > 1) {
      // W_(pR)^(j k) = W_N^(2 j k NC / (p R)) with N = 2 NC, j = 16 j1 + h
      const int step = 2 * k * (NC / (p * R));
#pragma unroll
      for (int j1 = 0; j1 < 16; ++j1)
        if (16 * j1 + h > 0) v[j1] = cmul(v[j1], tw_n(tw, (16 * j1 + h) * step, NC));
    }
    dft<16>(v);
    // W_256^(h m1) = W_N^(h m1 2 NC / 256)
    const int s256 = 2 * NC / R;
#pragma unroll
    for (int m1 = 1; m1 < 16; ++m1) v[m1] = cmul(v[m1], tw_n(tw, h * m1 * s256, NC));
#pragma unroll
    for (int m1 = 0; m1 < 16; ++m1) sh[(m1 * 16 + h) * 17 + g] = v[m1];
  }
  __syncthreads();
  if (live) {
#pragma unroll
    for (int j2 = 0; j2 < 16; ++j2) v[j2] = sh[(h * 16 + j2) * 17 + g];
    dft<16>(v);
    const int64_t o = base + static_cast<int64_t>(b - k) * R + k;
#pragma unroll
    for (int m2 = 0; m2 < 16; ++m2) out[o + static_cast<int64_t>(h + 16 * m2) * p] = v[m2];
  }
}

// ---- real spectrum times the band symbol, repacked and conjugated -----------------------
// From Z[k] and Z[NC - k] of the packed forward transform: even / odd half spectra
// E = (Z[k] + conj Z[-k]) / 2, O = (Z[k] - conj Z[-k]) / (2i), X[k] = E + W_N^k O and
// X[NC - k] = conj(E - W_N^k O); Y = S X; the half-length inverse takes
// Q[k] = (Y[k] + Y[k + NC]) + i (Y[k] - Y[k + NC]) conj(W_N^k) with Y[k + NC] = conj Y[NC - k];
// returned conjugated, so that a forward transform inverts it.
__device__ __forceinline__ double2 spectrum_q(double2 zk, double2 zm, double2 w, double sk,
                                              double sm) {
  const double2 e = make_double2(0.5 * (zk.x + zm.x), 0.5 * (zk.y - zm.y));
  const double2 od = make_double2(0.5 * (zk.y + zm.y), -0.5 * (zk.x - zm.x));
  const double2 wo = cmul(w, od);
  const double2 xk = cadd(e, wo);           // X[k]
  const double2 xm = cconj(csub(e, wo));    // X[NC - k] (X[NC] for k = 0)
  const double2 yk = make_double2(sk * xk.x, sk * xk.y);
  const double2 ymc = make_double2(sm * xm.x, -sm * xm.y);  // conj Y[NC - k]
  const double2 fe = cadd(yk, ymc);
  const double2 fo = cmul(csub(yk, ymc), cconj(w));
  return make_double2(fe.x - fo.y, -(fe.y + fo.x));
}

__global__ __launch_bounds__(kXThreads) void k_x_spectrum(
    const double2* __restrict__ Z, double2* __restrict__ out, const double2* __restrict__ tw,
    const double* __restrict__ spec, const Chunk* __restrict__ chunks, int seg0, int NC) {
  const int k = blockIdx.x * kXThreads + threadIdx.x;
  if (k >= NC) return;
  const int64_t base = static_cast<int64_t>(blockIdx.y) * NC;
  const double* S = spec + static_cast<int64_t>(chunks[seg0 + blockIdx.y].band) * (NC + 1);
  out[base + k] = spectrum_q(Z[base + k], Z[base + ((NC - k) & (NC - 1))], tw[k], S[k], S[NC - k]);
}

struct XFlush {
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

// ---- outputs of each segment, pointed back into the pixel domain -------------------------
__global__ __launch_bounds__(kXThreads) void k_x_scatter(
    const double2* __restrict__ G, const int32_t* __restrict__ lpix,
    const float* __restrict__ wq, const float* __restrict__ wu, const Chunk* __restrict__ chunks,
    int seg0, int lam, int NC, double inv_n, double* __restrict__ y) {
  // per wavefront: the runs it completes, listed before the atomics (one value per lane)
  constexpr int kScatterListed = 64;
  __shared__ int skey[kXThreads / 64][kScatterListed];
  __shared__ double sval[kXThreads / 64][3 * kScatterListed];
  const int wave = static_cast<int>(threadIdx.x >> 6);
  const Chunk c = chunks[seg0 + blockIdx.y];
  const int64_t base = static_cast<int64_t>(blockIdx.y) * NC;
  const int j0 = 4 * (blockIdx.x * kXThreads + threadIdx.x);
  int key[4];
  double v[4][3];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int j = j0 + q;
    key[q] = -1;
    v[q][0] = v[q][1] = v[q][2] = 0.0;
    if (j < c.out_len) {
      const int64_t g = c.out0 + j;
      const int p = lpix[g];
      if (p >= 0) {
        const int n = lam + j;
        const double2 gv = G[base + (n >> 1)];
        const double u = ((n & 1) ? -gv.y : gv.x) * inv_n;
        key[q] = p;
        v[q][0] = u;
        v[q][1] = static_cast<double>(wq[g]) * u;
        v[q][2] = static_cast<double>(wu[g]) * u;
      }
    }
  }
  wave_merge_runs_listed<4, 3, kScatterListed, XFlush, true>(key, v, XFlush{y}, skey[wave],
                                                             sval[wave]);
}

// ---- direct product for short bands (direct plans) ---------------------------------------
template <bool kData>
__global__ __launch_bounds__(kXThreads) void k_x_direct(
    const int32_t* __restrict__ lpix, const float* __restrict__ wq, const float* __restrict__ wu,
    const double* __restrict__ x, const float* __restrict__ d, const Chunk* __restrict__ tiles,
    const float* __restrict__ band_coef, const int64_t* __restrict__ band_off,
    const int32_t* __restrict__ band_ncoef, double* __restrict__ y) {
  extern __shared__ double xs[];  // window: out_len + 2 lambda samples, then lambda + 1 coefs
  const Chunk c = tiles[blockIdx.x];
  const int lam = band_ncoef[c.band] - 1;
  const float* coef = band_coef + band_off[c.band];
  const int nin = c.out_len + 2 * lam;
  double* cs = xs + nin;
  const int64_t b0 = c.blk_start, b1 = c.blk_start + c.blk_len;
  for (int i = threadIdx.x; i < nin; i += kXThreads) {
    const int64_t g = c.out0 - lam + i;
    double t = 0.0;
    if (g >= b0 && g < b1) {
      const int p = lpix[g];
      if (p >= 0) {
        if (kData) {
          t = static_cast<double>(d[g]);
        } else {
          const double* m = x + 3 * static_cast<int64_t>(p);
          t = m[0] + static_cast<double>(wq[g]) * m[1] + static_cast<double>(wu[g]) * m[2];
        }
      }
    }
    xs[i] = t;
  }
  for (int i = threadIdx.x; i <= lam; i += kXThreads) cs[i] = static_cast<double>(coef[i]);
  __syncthreads();
  for (int o0 = 0; o0 < c.out_len; o0 += 4 * kXThreads) {
    int key[4];
    double v[4][3];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int o = o0 + 4 * threadIdx.x + q;
      key[q] = -1;
      v[q][0] = v[q][1] = v[q][2] = 0.0;
      if (o < c.out_len) {
        const int64_t g = c.out0 + o;
        const int p = lpix[g];
        if (p >= 0) {
          const double* xc = xs + o + lam;
          double acc = cs[0] * xc[0];
          for (int j = 1; j <= lam; ++j) acc += cs[j] * (xc[-j] + xc[j]);
          key[q] = p;
          v[q][0] = acc;
          v[q][1] = static_cast<double>(wq[g]) * acc;
          v[q][2] = static_cast<double>(wu[g]) * acc;
        }
      }
    }
    wave_merge_runs<3>(key, v, XFlush{y});
  }
}

// ---- one segment per workgroup: FP64 transform with the data in registers ----------------
// NC = 2^M complex points (M = 11..14), T = NC / 16 threads of 16 points each.  Stockham passes
// of radix 16, then (8 or) 4, then a last radix-4 pass; between passes the points move through
// LDS one component at a time (NC doubles, padded one per 16 against bank conflicts).  Pass
// butterflies b = t + i T (i < 16 / R); the last pass of the forward transform instead gives
// thread t the butterflies {t, 4T - t, t + T, 3T - t} (thread 0: {0, 2T, T, 3T}), so that every
// output k = b + m NC / 4 finds its mirror NC - k in the same thread and the real-spectrum step
// runs in registers.
template <int M>
struct XFused {
  static constexpr int NC = 1 << M;
  static constexpr int T = NC / 16;
  static constexpr int R2 = M == 11 ? 8 : 16;            // second pass
  static constexpr int R3 = M == 11 ? 4 : (M == 12 ? 4 : (M == 13 ? 8 : 16));
  static constexpr int LDS = NC + NC / 16;  // exchange area (32 more doubles: thread 0's slot)
};

__device__ __forceinline__ int xpad(int i) { return i + (i >> 4); }

// Butterfly i of thread t in a radix-R pass (16 / R per thread).
template <int R, int T>
__device__ __forceinline__ int xbutterfly(int t, int i, bool paired) {
  if (paired) {  // R == 4: {t, 4T - t, t + T, 3T - t}, thread 0 {0, 2T, T, 3T}
    if (i == 0) return t;
    if (i == 1) return t == 0 ? 2 * T : 4 * T - t;
    if (i == 2) return t + T;
    return 3 * T - t;
  }
  return t + i * T;
}

// Input slot s = i R + j of a radix-R pass: point b_i + j NC / R.
template <int R, int T>
__device__ __forceinline__ int xin_pos(int t, int s, bool paired) {
  constexpr int NB = 16 * T / R;
  return xbutterfly<R, T>(t, s / R, paired) + (s % R) * NB;
}

// Output slot s = i R + m of a radix-R pass after p points were transformed: (b - k) R + k + m p.
template <int R, int T>
__device__ __forceinline__ int xout_pos(int t, int s, int p, bool paired) {
  const int b = xbutterfly<R, T>(t, s / R, paired);
  const int k = b & (p - 1);
  return (b - k) * R + k + (s % R) * p;
}

// An opaque copy of a value: the compiler cannot prove it equal to the original, so addresses
// and table loads of the two transforms are not merged and kept live across both (the second
// transform recomputes them instead of holding the first one's in registers).
template <class V>
__device__ __forceinline__ V xopaque(V v) {
  asm volatile("" : "+v"(v));
  return v;
}

// One radix-R pass on the registers (inputs already in place).
template <int R, int T>
__device__ __forceinline__ void xpass(double2 (&v)[16], int t, int p, bool paired,
                                      const double2* __restrict__ tw) {
  constexpr int NC = 16 * T;
#pragma unroll
  for (int i = 0; i < 16 / R; ++i) {
    const int b = xbutterfly<R, T>(t, i, paired);
    const int k = b & (p - 1);
    double2(&u)[R] = *reinterpret_cast<double2(*)[R]>(v + i * R);
    if (p > 1) {
      // W_(pR)^(j k) from the table for j = 1, 2, 4, 8 and by products for the others
      const int step = 2 * k * (NC / (p * R));
      const double2 w1 = tw_n(tw, step, NC);
      double2 w2 = make_double2(1.0, 0.0), w4 = w2, w8 = w2;
      if (R > 2) w2 = tw_n(tw, 2 * step, NC);
      if (R > 4) w4 = tw_n(tw, 4 * step, NC);
      if (R > 8) w8 = tw_n(tw, 8 * step, NC);
#pragma unroll
      for (int j = 1; j < R; ++j) {
        double2 w = (j & 1) ? w1 : make_double2(1.0, 0.0);
        if (j & 2) w = (j & 1) ? cmul(w, w2) : w2;
        if (j & 4) w = (j & 3) ? cmul(w, w4) : w4;
        if (j & 8) w = (j & 7) ? cmul(w, w8) : w8;
        u[j] = cmul(u[j], w);
      }
    }
    dft<R>(u);
    __builtin_amdgcn_sched_barrier(0);  // one butterfly's twiddles in flight at a time
  }
}

// Move the points from the output slots of pass A to the input slots of pass B through LDS.
template <int RA, int RB, int T>
__device__ __forceinline__ void xexchange(double2 (&v)[16], double* sh, int t, int pa,
                                          bool paired_a, bool paired_b) {
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int tw_ = xopaque(t);  // addresses recomputed per component, not held across
#pragma unroll
    for (int s = 0; s < 16; ++s) sh[xpad(xout_pos<RA, T>(tw_, s, pa, paired_a))] = c ? v[s].y : v[s].x;
    __syncthreads();
    const int tr_ = xopaque(t);
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const double val = sh[xpad(xin_pos<RB, T>(tr_, s, paired_b))];
      if (c) v[s].y = val; else v[s].x = val;
    }
    __syncthreads();
  }
}

// Forward transform: inputs at the first pass's slots, outputs at the last pass's slots.
template <int M>
__device__ __forceinline__ void xfft(double2 (&v)[16], double* sh, int t, bool paired_last,
                                     const double2* __restrict__ tw) {
  using C = XFused<M>;
  constexpr int T = C::T, R2 = C::R2, R3 = C::R3;
  xpass<16, T>(v, t, 1, false, tw);
  xexchange<16, R2, T>(v, sh, t, 1, false, false);
  xpass<R2, T>(v, t, 16, false, tw);
  xexchange<R2, R3, T>(v, sh, t, 16, false, false);
  xpass<R3, T>(v, t, 16 * R2, false, tw);
  xexchange<R3, 4, T>(v, sh, t, 16 * R2, false, paired_last);
  xpass<4, T>(v, t, 16 * R2 * R3, paired_last, tw);
}

// FP64 samples of one lane of 8 consecutive window samples [g, g + 8), all inside the block and
// g a multiple of 4: the pointing comes in 16-byte loads, and scan runs keep a pixel for several
// samples, so the pixel values of the lane's first and last samples are loaded together and a
// third pixel only when one occurs.  The sums are those of the one-sample form.
template <int kIn>
__device__ __forceinline__ void xgather8(const int32_t* __restrict__ lpix,
                                         const float* __restrict__ wq,
                                         const float* __restrict__ wu,
                                         const double* __restrict__ x,
                                         const float* __restrict__ d, int64_t g,
                                         double (&o)[8]) {
  constexpr bool kData = kIn == kInData;
  int kk[8];
  float qq[8], uu[8], dd[8];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int4 k4 = *reinterpret_cast<const int4*>(lpix + g + 4 * c);
    kk[4 * c] = k4.x;
    kk[4 * c + 1] = k4.y;
    kk[4 * c + 2] = k4.z;
    kk[4 * c + 3] = k4.w;
    const float4 q4 = *reinterpret_cast<const float4*>((kData ? d : wq) + g + 4 * c);
    qq[4 * c] = q4.x;
    qq[4 * c + 1] = q4.y;
    qq[4 * c + 2] = q4.z;
    qq[4 * c + 3] = q4.w;
    if constexpr (!kData) {
      const float4 u4 = *reinterpret_cast<const float4*>(wu + g + 4 * c);
      uu[4 * c] = u4.x;
      uu[4 * c + 1] = u4.y;
      uu[4 * c + 2] = u4.z;
      uu[4 * c + 3] = u4.w;
    }
    if constexpr (kIn == kInResid) {
      const float4 d4 = *reinterpret_cast<const float4*>(d + g + 4 * c);
      dd[4 * c] = d4.x;
      dd[4 * c + 1] = d4.y;
      dd[4 * c + 2] = d4.z;
      dd[4 * c + 3] = d4.w;
    }
  }
  if constexpr (kData) {
#pragma unroll
    for (int j = 0; j < 8; ++j) o[j] = kk[j] < 0 ? 0.0 : static_cast<double>(qq[j]);
  } else {
    const int ka = kk[0], kb = kk[7];
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
    for (int j = 0; j < 8; ++j) {
      const int key = kk[j];
      other |= key >= 0 && key != ka && key != kb;
      const double q = static_cast<double>(qq[j]), u = static_cast<double>(uu[j]);
      const double ta = a0 + q * a1 + u * a2;
      const double tb = b0 + q * b1 + u * b2;
      o[j] = key < 0 ? 0.0 : (key == ka ? ta : tb);
    }
    if (other) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int key = kk[j];
        if (key >= 0 && key != ka && key != kb) {
          const double* m = x + 3 * static_cast<int64_t>(key);
          o[j] = m[0] + static_cast<double>(qq[j]) * m[1] + static_cast<double>(uu[j]) * m[2];
        }
      }
    }
    if constexpr (kIn == kInResid) {
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (kk[j] >= 0) o[j] = static_cast<double>(dd[j]) - o[j];
    }
  }
}

template <int M, int kIn>
__global__ __launch_bounds__(XFused<M>::T) void k_x_fused(
    const int32_t* __restrict__ lpix, const float* __restrict__ wq, const float* __restrict__ wu,
    const double* __restrict__ x, const float* __restrict__ d, int dvec,
    const Chunk* __restrict__ chunks, int lam, const double* __restrict__ spec,
    const double2* __restrict__ tw0, double inv_n, double* __restrict__ y) {
  using C = XFused<M>;
  constexpr int NC = C::NC, T = C::T, PL = NC / 4;
  static_assert(C::R2 * C::R3 * 16 * 4 == NC, "pass radices");
  __shared__ __align__(16) double sh[C::LDS + 32];
  const Chunk c = chunks[blockIdx.x];
  const int t = threadIdx.x;
  const int64_t b0 = c.blk_start, b1 = c.blk_start + c.blk_len;

  // ---- window samples, packed as complex points at the first pass's slots ------------------
  // Two halves of NC samples (NC / 2 points) staged through LDS, where sample n of a half sits
  // at n (point p at 2p and 2p + 1); lanes take 8 consecutive samples (two rounds per half)
  double2 v[16];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll 1
    for (int r = 0; r < 2; ++r) {
      const int n = 8 * (t + r * T);  // sample of the half
      const int64_t g = c.out0 - lam + static_cast<int64_t>(h) * NC + n;
      double o[8];
      if (g >= b0 && g + 8 <= b1 && (g & 3) == 0 && (kIn == kInMap || dvec)) {
        xgather8<kIn>(lpix, wq, wu, x, d, g, o);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int64_t gj = g + j;
          double val = 0.0;
          if (gj >= b0 && gj < b1) {
            const int p = lpix[gj];
            if (p >= 0) {
              if constexpr (kIn == kInData) {
                val = static_cast<double>(d[gj]);
              } else {
                const double* m = x + 3 * static_cast<int64_t>(p);
                val = m[0] + static_cast<double>(wq[gj]) * m[1] + static_cast<double>(wu[gj]) * m[2];
                if constexpr (kIn == kInResid) val = static_cast<double>(d[gj]) - val;
              }
            }
          }
          o[j] = val;
        }
      }
      double2* dst = reinterpret_cast<double2*>(sh + n);
#pragma unroll
      for (int j = 0; j < 4; ++j) dst[j] = make_double2(o[2 * j], o[2 * j + 1]);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 8; ++j) v[8 * h + j] = reinterpret_cast<const double2*>(sh)[t + j * T];
    __syncthreads();
  }

  // ---- forward transform; real spectrum x symbol with mirrors in the same thread -----------
  xfft<M>(v, sh, t, true, tw0);
  {
    const int t = xopaque(threadIdx.x);
    const double2* __restrict__ tw = reinterpret_cast<const double2*>(
        xopaque(reinterpret_cast<uintptr_t>(tw0)));
    // slot s = 4 i + m holds point k = b_i + m PL; its mirror NC - k is in the same thread:
    // slots (8 + m, 15 - m) always, (m, 7 - m) for t > 0; thread 0 holds k = 0 and NC/2 alone
    // (slots 0 and 2) and pairs (1, 3), (4, 7), (5, 6)
    const double* S = spec + static_cast<int64_t>(c.band) * (NC + 1);
    auto kpos = [&](int s) {
      return xbutterfly<4, T>(xopaque(t), s >> 2, true) + (s & 3) * PL;
    };
    auto pair = [&](int a, int b) {
      const int ka = kpos(a), kb = NC - ka;
      const double2 za = v[a], zb = v[b];
      const double sa = S[ka], sb = S[kb];
      v[a] = spectrum_q(za, zb, tw_n(tw, ka, NC), sa, sb);
      v[b] = spectrum_q(zb, za, tw_n(tw, kb, NC), sb, sa);
      __builtin_amdgcn_sched_barrier(0);  // bound the loads in flight (register pressure)
    };
    // Thread 0's first two butterflies (0 and 2T) pair within themselves: it parks their
    // points in a private LDS slot, runs the common pairing with everyone (its slots 0..7 come
    // out wrong there), lanes 0..7 of its wavefront redo one of those slots each from the
    // parked points, and thread 0 reloads them.
    double2* own = reinterpret_cast<double2*>(sh + C::LDS);  // [0, 8) parked, [8, 16) redone
    if (t == 0) {
#pragma unroll
      for (int s2 = 0; s2 < 8; ++s2) own[s2] = v[s2];
    }
    wave_lds_sync();
    // one half of the points at a time in registers, the other parked in the (idle) exchange
    // area at lane-consecutive addresses
    auto park = [&](int base) {
#pragma unroll
      for (int s2 = 0; s2 < 8; ++s2) {
        sh[(2 * s2) * T + t] = v[base + s2].x;
        sh[(2 * s2 + 1) * T + t] = v[base + s2].y;
      }
    };
    auto unpark = [&](int base) {
#pragma unroll
      for (int s2 = 0; s2 < 8; ++s2)
        v[base + s2] = make_double2(sh[(2 * s2) * T + t], sh[(2 * s2 + 1) * T + t]);
    };
    park(0);
#pragma unroll
    for (int m = 0; m < 4; ++m) pair(8 + m, 15 - m);
    __builtin_amdgcn_sched_barrier(0);
    unpark(0);
    park(8);
#pragma unroll
    for (int m = 0; m < 4; ++m) pair(m, 7 - m);
    __builtin_amdgcn_sched_barrier(0);
    unpark(8);
    if (t < 8) {
      // slot t of thread 0: butterfly 0 holds k = t PL (mirror slot (4 - t) mod 4), butterfly
      // 2T holds k = 2T + (t - 4) PL (mirror slot 11 - t)
      const int mir = t < 4 ? ((4 - t) & 3) : 11 - t;
      const int k = t < 4 ? t * PL : 2 * T + (t - 4) * PL;
      own[8 + t] = spectrum_q(own[t], own[mir], tw_n(tw, k, NC), S[k], S[NC - k]);
    }
    wave_lds_sync();
    if (t == 0) {
#pragma unroll
      for (int s2 = 0; s2 < 8; ++s2) v[s2] = own[8 + s2];
    }
  }
  // back to the first pass's slots, then the forward transform of conj Q
  __syncthreads();  // every thread has reloaded its parked points
  {
    const int t2 = xopaque(threadIdx.x);
    const double2* __restrict__ tw2 = reinterpret_cast<const double2*>(
        xopaque(reinterpret_cast<uintptr_t>(tw0)));
    xexchange<4, 16, T>(v, sh, t2, PL, true, false);
    xfft<M>(v, sh, t2, false, tw2);
  }

  // ---- outputs y[n] = Re G[n/2] / N (n even), -Im G[n/2] / N (n odd), staged in LDS -------
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const int k = xbutterfly<4, T>(t, s >> 2, false) + (s & 3) * PL;
    const int o0 = 2 * k - lam;
    if (o0 >= 0 && o0 < c.out_len) sh[xpad(o0)] = v[s].x * inv_n;
    if (o0 + 1 >= 0 && o0 + 1 < c.out_len) sh[xpad(o0 + 1)] = -v[s].y * inv_n;
  }
  __syncthreads();
  // Each wavefront reads its own 512 staged outputs per round (out_len <= NC, so every round's
  // slices lie inside sh); once read, that slice holds the wavefront's list of completed runs,
  // flushed one FP64 value per lane.
  constexpr int kXListed = 64;
  static_assert(3 * kXListed + kXListed / 2 <= 512, "run list must fit a wavefront's slice");
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  for (int base = 0; base < c.out_len; base += 8 * T) {  // same trip count for every lane
    const int i0 = base + 8 * t;
    const int64_t o = c.out0 + i0;
    int key[8];
    double vv[8][3];
    if (i0 + 8 <= c.out_len && (o & 3) == 0) {
      int kk[8];
      float qq[8], uu[8];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int4 k4 = *reinterpret_cast<const int4*>(lpix + o + 4 * q);
        const float4 q4 = *reinterpret_cast<const float4*>(wq + o + 4 * q);
        const float4 u4 = *reinterpret_cast<const float4*>(wu + o + 4 * q);
        kk[4 * q] = k4.x;
        kk[4 * q + 1] = k4.y;
        kk[4 * q + 2] = k4.z;
        kk[4 * q + 3] = k4.w;
        qq[4 * q] = q4.x;
        qq[4 * q + 1] = q4.y;
        qq[4 * q + 2] = q4.z;
        qq[4 * q + 3] = q4.w;
        uu[4 * q] = u4.x;
        uu[4 * q + 1] = u4.y;
        uu[4 * q + 2] = u4.z;
        uu[4 * q + 3] = u4.w;
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const double u = sh[xpad(i0 + i)];
        key[i] = kk[i];
        vv[i][0] = u;
        vv[i][1] = static_cast<double>(qq[i]) * u;
        vv[i][2] = static_cast<double>(uu[i]) * u;
      }
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int oi = i0 + i;
        key[i] = -1;
        vv[i][0] = vv[i][1] = vv[i][2] = 0.0;
        if (oi < c.out_len) {
          const int64_t g = c.out0 + oi;
          const int p = lpix[g];
          if (p >= 0) {
            const double u = sh[xpad(oi)];
            key[i] = p;
            vv[i][0] = u;
            vv[i][1] = static_cast<double>(wq[g]) * u;
            vv[i][2] = static_cast<double>(wu[g]) * u;
          }
        }
      }
    }
    double* sval = sh + xpad(base + 512 * wave);
    int* skey = reinterpret_cast<int*>(sval + 3 * kXListed);
    wave_merge_runs_listed<8, 3, kXListed, XFlush, true>(key, vv, XFlush{y}, skey, sval);
  }
}

template <int M>
mm_status launch_fused_m(Plan* P, const double* x, const float* d, double* y, hipStream_t s) {
  const double inv_n = 1.0 / static_cast<double>(P->fft_n);
  const int dvec = (reinterpret_cast<uintptr_t>(d) & 15u) == 0 ? 1 : 0;
  if (x == nullptr)
    hipLaunchKernelGGL((k_x_fused<M, kInData>), dim3(P->n_chunks), dim3(XFused<M>::T), 0, s,
                       P->lpix, P->wq, P->wu, x, d, dvec, P->chunks, P->lambda_max, P->x_spec,
                       P->x_tw, inv_n, y);
  else if (d == nullptr)
    hipLaunchKernelGGL((k_x_fused<M, kInMap>), dim3(P->n_chunks), dim3(XFused<M>::T), 0, s,
                       P->lpix, P->wq, P->wu, x, d, dvec, P->chunks, P->lambda_max, P->x_spec,
                       P->x_tw, inv_n, y);
  else
    hipLaunchKernelGGL((k_x_fused<M, kInResid>), dim3(P->n_chunks), dim3(XFused<M>::T), 0, s,
                       P->lpix, P->wq, P->wu, x, d, dvec, P->chunks, P->lambda_max, P->x_spec,
                       P->x_tw, inv_n, y);
  MM_HIP_TRY(hipGetLastError());
  return MM_OK;
}

// Device buffer released at scope exit (after the caller's stream has been synchronised).
template <class T>
struct XBuf {
  T* p = nullptr;
  ~XBuf() { dev_free(p); }
  mm_status alloc(size_t n) {
    const hipError_t e = dev_malloc(reinterpret_cast<void**>(&p), n * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      return fail(MM_ERR_OOM, std::string("hipMalloc (FP64 product): ") + hipGetErrorString(e));
    }
    return MM_OK;
  }
};

template <int R>
mm_status run_pass(const double2* in, double2* out, const double2* tw, int NC, int p, int nseg,
                   hipStream_t s) {
  const int L = NC / R;
  hipLaunchKernelGGL(k_x_pass<R>, dim3((L + kXThreads - 1) / kXThreads, nseg), dim3(kXThreads), 0,
                     s, in, out, tw, NC, p);
  MM_HIP_TRY(hipGetLastError());
  return MM_OK;
}

// Forward DFT of every segment of the batch: radix-256 passes (two radix-16 levels each
// through LDS), then radix-16 passes, then the remaining factor.
// Returns the tile holding the result (a or b).
mm_status batch_fft(double2* a, double2* b, const double2* tw, int NC, int nseg, hipStream_t s,
                    double2** result) {
  double2* in = a;
  double2* out = b;
  int p = 1;
  while (NC / p >= 256) {
    hipLaunchKernelGGL(k_x_pass256, dim3((NC / 256 + 15) / 16, nseg), dim3(kXThreads), 0, s, in,
                       out, tw, NC, p);
    MM_HIP_TRY(hipGetLastError());
    p *= 256;
    std::swap(in, out);
  }
  while (NC / p >= 16) {
    MM_TRY(run_pass<16>(in, out, tw, NC, p, nseg, s));
    p *= 16;
    std::swap(in, out);
  }
  const int rest = NC / p;
  if (rest > 1) {
    if (rest == 2) MM_TRY(run_pass<2>(in, out, tw, NC, p, nseg, s));
    if (rest == 4) MM_TRY(run_pass<4>(in, out, tw, NC, p, nseg, s));
    if (rest == 8) MM_TRY(run_pass<8>(in, out, tw, NC, p, nseg, s));
    std::swap(in, out);
  }
  *result = in;
  return MM_OK;
}

// FP64 symbol and twiddles of the plan's FFT length, built once.
mm_status prepare(Plan* P, hipStream_t s) {
  std::lock_guard<std::mutex> lk(P->x_mu);
  if (P->x_ready) return MM_OK;
  const int N = P->fft_n, NC = N / 2;
  MM_TRY(dalloc(P, &P->x_spec, static_cast<size_t>(P->n_bands) * (NC + 1)));
  MM_TRY(launch_band_symbol64(P, P->x_spec, s));
  std::vector<double2> tw(static_cast<size_t>(NC));
  for (int k = 0; k < NC; ++k) {
    double sn, cs;
    // exp(-2 pi i k / N) with the angle reduced exactly: k / N in [0, 1/2)
    const double a = 2.0 * 3.14159265358979323846264338327950288 * (static_cast<double>(k) / N);
    sn = std::sin(a);
    cs = std::cos(a);
    tw[static_cast<size_t>(k)] = make_double2(cs, -sn);
  }
  MM_TRY(dalloc(P, &P->x_tw, tw.size()));
  MM_HIP_TRY(hipMemcpyAsync(P->x_tw, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice, s));
  MM_HIP_TRY(hipStreamSynchronize(s));
  P->x_ready = true;
  return MM_OK;
}

}  // namespace

bool exact_residual_supported(const Plan* P) {
  return P->n_poly == 0 && P->lambda_max > 0 && P->algo == MM_TOEPLITZ_FFT &&
         P->n_id_tiles == 0;
}

mm_status exact_product(Plan* P, const double* x, const float* d, double* y, hipStream_t s) {
  if (x != nullptr && d != nullptr && !exact_residual_supported(P))
    return fail(MM_ERR_UNSUPPORTED, "FP64 residual product: Toeplitz FFT plans only");
  MM_TRY(launch_zero(y, 3 * P->n_kept, s));
  if (P->n_kept == 0) return MM_OK;
  const bool data = x == nullptr;
  if (P->n_poly > 0) return launch_template_apply(P, x, d, y, nullptr, s);  // FP64 already
  if (P->lambda_max == 0) return launch_diag_apply(P, x, d, y, nullptr, s);
  if (P->algo == MM_TOEPLITZ_FFT && P->n_chunks > 0 && P->fft_n >= (1 << 12) &&
      P->fft_n <= (1 << 15) && P->fft_n - 2 * P->lambda_max <= P->fft_n / 2) {
    // one workgroup per segment with the transform in registers and LDS
    MM_TRY(prepare(P, s));
    switch (P->fft_n) {
      case 1 << 12: MM_TRY(launch_fused_m<11>(P, x, d, y, s)); break;
      case 1 << 13: MM_TRY(launch_fused_m<12>(P, x, d, y, s)); break;
      case 1 << 14: MM_TRY(launch_fused_m<13>(P, x, d, y, s)); break;
      default: MM_TRY(launch_fused_m<14>(P, x, d, y, s)); break;
    }
    if (P->n_id_tiles > 0) MM_TRY(launch_diag_tiles(P, P->id_tiles, P->n_id_tiles, x, d, y, nullptr, s));
    return MM_OK;
  }
  if (P->algo == MM_TOEPLITZ_FFT) {
    MM_TRY(prepare(P, s));
    const int N = P->fft_n, NC = N / 2;
    const int per = static_cast<int>(std::max<size_t>(1, kTileBudget / (sizeof(double2) * NC)));
    const int batch = std::min(per, std::max(1, P->n_chunks));
    XBuf<double2> ta, tb;
    MM_TRY(ta.alloc(static_cast<size_t>(batch) * NC));
    MM_TRY(tb.alloc(static_cast<size_t>(batch) * NC));
    const int lam = P->lambda_max;
    const int out_max = N - 2 * lam;
    for (int seg0 = 0; seg0 < P->n_chunks; seg0 += batch) {
      const int nseg = std::min(batch, P->n_chunks - seg0);
      const dim3 gpts((NC + kXThreads - 1) / kXThreads, nseg);
      if (data)
        hipLaunchKernelGGL(k_x_load<kInData>, gpts, dim3(kXThreads), 0, s, P->lpix, P->wq,
                           P->wu, x, d, P->chunks, seg0, lam, NC, ta.p);
      else if (d == nullptr)
        hipLaunchKernelGGL(k_x_load<kInMap>, gpts, dim3(kXThreads), 0, s, P->lpix, P->wq,
                           P->wu, x, d, P->chunks, seg0, lam, NC, ta.p);
      else
        hipLaunchKernelGGL(k_x_load<kInResid>, gpts, dim3(kXThreads), 0, s, P->lpix, P->wq,
                           P->wu, x, d, P->chunks, seg0, lam, NC, ta.p);
      MM_HIP_TRY(hipGetLastError());
      double2* spec_in = nullptr;
      MM_TRY(batch_fft(ta.p, tb.p, P->x_tw, NC, nseg, s, &spec_in));
      double2* spec_out = spec_in == ta.p ? tb.p : ta.p;
      hipLaunchKernelGGL(k_x_spectrum, gpts, dim3(kXThreads), 0, s, spec_in, spec_out, P->x_tw,
                         P->x_spec, P->chunks, seg0, NC);
      MM_HIP_TRY(hipGetLastError());
      double2* other = spec_out == ta.p ? tb.p : ta.p;
      double2* res = nullptr;
      MM_TRY(batch_fft(spec_out, other, P->x_tw, NC, nseg, s, &res));
      const dim3 gout((out_max + 4 * kXThreads - 1) / (4 * kXThreads), nseg);
      hipLaunchKernelGGL(k_x_scatter, gout, dim3(kXThreads), 0, s, res, P->lpix, P->wq, P->wu,
                         P->chunks, seg0, lam, NC, 1.0 / static_cast<double>(N), y);
      MM_HIP_TRY(hipGetLastError());
    }
    if (P->n_id_tiles > 0) MM_TRY(launch_diag_tiles(P, P->id_tiles, P->n_id_tiles, x, d, y, nullptr, s));
    MM_HIP_TRY(hipStreamSynchronize(s));  // the tiles are released on return
    return MM_OK;
  }
  // direct plans: tiles of <= 1024 outputs with their lambda halo in LDS
  if (P->n_chunks > 0) {
    const size_t lds = sizeof(double) * (1024 + 2 * static_cast<size_t>(P->lambda_max) +
                                         static_cast<size_t>(P->lambda_max) + 1);
    if (lds > 160 * 1024) return fail(MM_ERR_UNSUPPORTED, "FP64 direct product: band too long");
    if (lds > 64 * 1024) {
      MM_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(k_x_direct<true>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
      MM_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(k_x_direct<false>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
    }
    if (data)
      hipLaunchKernelGGL(k_x_direct<true>, dim3(P->n_chunks), dim3(kXThreads), lds, s, P->lpix,
                         P->wq, P->wu, x, d, P->chunks, P->band_coef, P->band_off,
                         P->band_ncoef, y);
    else
      hipLaunchKernelGGL(k_x_direct<false>, dim3(P->n_chunks), dim3(kXThreads), lds, s, P->lpix,
                         P->wq, P->wu, x, d, P->chunks, P->band_coef, P->band_off,
                         P->band_ncoef, y);
    MM_HIP_TRY(hipGetLastError());
  }
  if (P->n_id_tiles > 0) MM_TRY(launch_diag_tiles(P, P->id_tiles, P->n_id_tiles, x, d, y, nullptr, s));
  return MM_OK;
}

}  // namespace mm
