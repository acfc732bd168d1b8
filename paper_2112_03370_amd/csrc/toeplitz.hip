// Block-diagonal banded Toeplitz product u = N^-1 t (Toeplitz algebra package: stbmm).
//
// FFT path (shift-and-overlap, Toeplitz product paragraph): each workgroup owns one segment of
// one stationary interval: N real inputs [out0 - lambda, out0 - lambda + N), zero outside the
// interval (truncation at block edges), producing N - 2 lambda outputs.  The N real samples
// are packed as N/2 complex points (even samples real, odd imaginary) and transformed in LDS
// by a radix-16/8/4/2 Stockham FFT; the half-length spectrum is unpacked into the real
// spectrum, multiplied by the band's symbol (real because the band is symmetric), repacked,
// and transformed back (inverse = conjugate of the forward transform of the conjugate).  All
// arithmetic is FP32; twiddles come from a two-level table (exp(-2 pi i m / N) =
// coarse[m >> 7] * fine[m & 127]) computed in FP64 on the host.  The symbol is precomputed per
// band at plan time with the 1/(2N) normalisation folded in.
//
// Direct path (short bands and tests): each workgroup owns 1024 outputs, stages the inputs
// with a lambda halo and the band in LDS, and evaluates y_i = c_0 x_i + sum_k c_k (x_{i-k} +
// x_{i+k}) in FP32.
#include "mm_internal.h"

namespace mm {

namespace {

// ---------------------------------------------------------------------------------------------
// Small complex helpers
// ---------------------------------------------------------------------------------------------

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

template <int LOG>
struct FftCfg {
  static constexpr int NC = 1 << LOG;   // complex points
  static constexpr int N = 2 * NC;      // real samples per segment
  static constexpr int T = NC / 16;     // threads
  static constexpr int LDS = NC + NC / 16;
};

template <int LOG>
__global__ __launch_bounds__(FftCfg<LOG>::T) void k_toeplitz_fft(
    const float* __restrict__ t, float* __restrict__ u, const Chunk* __restrict__ chunks,
    const float* __restrict__ spec, const float2* __restrict__ tw0g,
    const float2* __restrict__ tw1g, int lam, const int32_t* __restrict__ done) {
  using C = FftCfg<LOG>;
  constexpr int NC = C::NC, N = C::N, T = C::T;
  __shared__ float2 buf[C::LDS];
  __shared__ float2 tw0[128];
  __shared__ float2 tw1[N / 128];
  if (done != nullptr && *done) return;
  const int tid = threadIdx.x;
  for (int i = tid; i < 128; i += T) tw0[i] = tw0g[i];
  for (int i = tid; i < N / 128; i += T) tw1[i] = tw1g[i];

  const Chunk c = chunks[blockIdx.x];
  const int64_t in0 = c.out0 - lam;
  const int64_t b0 = c.blk_start, b1 = c.blk_start + c.blk_len;
  float* fbuf = reinterpret_cast<float*>(buf);
  for (int n = tid; n < N; n += T) {
    const int64_t g = in0 + n;
    const float val = (g >= b0 && g < b1) ? t[g] : 0.0f;
    fbuf[2 * pad(n >> 1) + (n & 1)] = val;
  }
  __syncthreads();
  fft_forward<LOG, T>(buf, tw0, tw1);

  // Unpack the real spectrum, multiply by the symbol, repack (conjugated for the inverse).
  const float* S = spec + static_cast<int64_t>(c.band) * (NC + 1);
  for (int k = tid; k <= NC / 2; k += T) {
    const int k2 = (NC - k) & (NC - 1);
    const float2 Z = buf[pad(k)], Z2 = buf[pad(k2)];
    const float2 E = make_float2(Z.x + Z2.x, Z.y - Z2.y);
    const float2 O = make_float2(Z.y + Z2.y, Z2.x - Z.x);  // -i (Z - conj(Z2))
    const float2 W = twiddle(tw0, tw1, k);
    const float2 WO = cmul(W, O);
    const float sa = S[k], sb = S[NC - k];
    const float2 Ya = make_float2(sa * (E.x + WO.x), sa * (E.y + WO.y));
    const float2 Yb = make_float2(sb * (E.x - WO.x), sb * (E.y - WO.y));
    const float2 Ye = cadd(Ya, Yb);
    const float2 Yo = cmulc(csub(Ya, Yb), W);
    // Z'[k] = Ye + i Yo ; Z'[NC-k] = conj(Ye) + i conj(Yo); store conjugates.
    buf[pad(k)] = make_float2(Ye.x - Yo.y, -(Ye.y + Yo.x));
    if (k2 != k) buf[pad(k2)] = make_float2(Ye.x + Yo.y, Ye.y - Yo.x);
  }
  __syncthreads();
  fft_forward<LOG, T>(buf, tw0, tw1);

  // y[2m] = Re R[m], y[2m+1] = -Im R[m]; outputs are y[lam .. lam + out_len).
  for (int n = lam + tid; n < lam + c.out_len; n += T) {
    const float2 v = buf[pad(n >> 1)];
    u[c.out0 + (n - lam)] = (n & 1) ? -v.y : v.x;
  }
}

// ---------------------------------------------------------------------------------------------
// Direct product
// ---------------------------------------------------------------------------------------------

constexpr int kDirectTile = 1024;
constexpr int kDirectThreads = 256;
constexpr int kDirectMaxLambda = 4096;

__global__ __launch_bounds__(kDirectThreads) void k_toeplitz_direct(
    const float* __restrict__ t, float* __restrict__ u, const Chunk* __restrict__ tiles,
    const float* __restrict__ band_coef, const int64_t* __restrict__ band_off,
    const int32_t* __restrict__ band_ncoef, const int32_t* __restrict__ done) {
  extern __shared__ float sh[];
  if (done != nullptr && *done) return;
  const Chunk c = tiles[blockIdx.x];
  const int lam = band_ncoef[c.band] - 1;
  const float* coef = band_coef + band_off[c.band];
  float* x = sh;                                  // kDirectTile + 2 lam
  float* cc = sh + kDirectTile + 2 * kDirectMaxLambda;  // lam + 1
  const int64_t b0 = c.blk_start, b1 = c.blk_start + c.blk_len;
  const int64_t in0 = c.out0 - lam;
  const int nin = c.out_len + 2 * lam;
  for (int i = threadIdx.x; i < nin; i += kDirectThreads) {
    const int64_t g = in0 + i;
    x[i] = (g >= b0 && g < b1) ? t[g] : 0.0f;
  }
  for (int i = threadIdx.x; i <= lam; i += kDirectThreads) cc[i] = coef[i];
  __syncthreads();
  for (int o = threadIdx.x; o < c.out_len; o += kDirectThreads) {
    const float* xc = x + o + lam;
    float acc = cc[0] * xc[0];
    for (int k = 1; k <= lam; ++k) acc = fmaf(cc[k], xc[-k] + xc[k], acc);
    u[c.out0 + o] = acc;
  }
}

// Identity rows (samples outside every block): u = t.
__global__ __launch_bounds__(256) void k_copy_segments(const float* __restrict__ t,
                                                       float* __restrict__ u,
                                                       const int64_t* __restrict__ seg,
                                                       const int32_t* __restrict__ done) {
  if (done != nullptr && *done) return;
  const int64_t s0 = seg[2 * blockIdx.x], len = seg[2 * blockIdx.x + 1];
  for (int64_t i = threadIdx.x; i < len; i += 256) u[s0 + i] = t[s0 + i];
}

template <int LOG>
mm_status launch_fft(Plan* P, const float* t, float* u, const int32_t* done, hipStream_t s) {
  using C = FftCfg<LOG>;
  hipLaunchKernelGGL(k_toeplitz_fft<LOG>, dim3(P->n_chunks), dim3(C::T), 0, s, t, u, P->chunks,
                     P->spec, P->tw0, P->tw1, P->lambda_max, done);
  MM_HIP_TRY(hipGetLastError());
  return MM_OK;
}

}  // namespace

int32_t max_direct_lambda() { return kDirectMaxLambda; }

bool fft_size_supported(int32_t n) {
  return n == (1 << 11) || n == (1 << 12) || n == (1 << 13) || n == (1 << 14) || n == (1 << 15);
}

int32_t choose_fft_size(int32_t lambda_max) {
  // Smallest supported power of two with at least half of every segment being output.
  int32_t n = 1 << 11;
  while (n < 4 * lambda_max && n < (1 << 15)) n *= 2;
  if (n <= 2 * lambda_max) return 0;
  return n;
}

mm_status launch_noise_weight(Plan* P, const float* t, float* u, const int32_t* done,
                              hipStream_t s) {
  if (P->n_samples == 0) return MM_OK;
  TimedLaunch tl(P, K_TOEPLITZ, s);
  if (P->n_chunks > 0) {
    if (P->algo == MM_TOEPLITZ_FFT) {
      switch (P->fft_n) {
        case 1 << 11: MM_TRY(launch_fft<10>(P, t, u, done, s)); break;
        case 1 << 12: MM_TRY(launch_fft<11>(P, t, u, done, s)); break;
        case 1 << 13: MM_TRY(launch_fft<12>(P, t, u, done, s)); break;
        case 1 << 14: MM_TRY(launch_fft<13>(P, t, u, done, s)); break;
        case 1 << 15: MM_TRY(launch_fft<14>(P, t, u, done, s)); break;
        default: return fail(MM_ERR_UNSUPPORTED, "FFT size not supported");
      }
    } else {
      const size_t lds = sizeof(float) * (kDirectTile + 2 * kDirectMaxLambda + kDirectMaxLambda + 1);
      hipLaunchKernelGGL(k_toeplitz_direct, dim3(P->n_chunks), dim3(kDirectThreads), lds, s, t, u,
                         P->chunks, P->band_coef, P->band_off, P->band_ncoef, done);
      MM_HIP_TRY(hipGetLastError());
    }
  }
  if (P->n_id_seg > 0) {
    hipLaunchKernelGGL(k_copy_segments, dim3(P->n_id_seg), dim3(256), 0, s, t, u, P->id_seg, done);
    MM_HIP_TRY(hipGetLastError());
  }
  return MM_OK;
}

}  // namespace mm
