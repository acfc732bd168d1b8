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
#include "fft_lds.h"
#include "mm_internal.h"

namespace mm {

namespace {

using namespace fft;

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

  const Chunk c = chunks[xcd_ordered(blockIdx.x, gridDim.x)];
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
  symbol_multiply<LOG, T>(buf, spec + static_cast<int64_t>(c.band) * (NC + 1), tw0, tw1);
  fft_forward<LOG, T>(buf, tw0, tw1);
  // outputs are y[lam .. lam + out_len)
  for (int n = lam + tid; n < lam + c.out_len; n += T) u[c.out0 + (n - lam)] = real_out(buf, n);
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
  return n == (1 << 11) || n == (1 << 12) || n == (1 << 13) || n == (1 << 14) ||
         n == (1 << 15) || long_fft_size(n);
}

int32_t choose_fft_size(int32_t lambda_max) {
  // Smallest power of two >= 4 lambda (at least half of every segment is output).  Up to 2^15
  // the segment fits one CU's LDS; bands a little longer still use 2^15 while at least 8,192
  // outputs per segment remain; longer bands go to the four-step kernel (up to 2^17).
  int64_t n = 1 << 11;
  while (n < 4 * static_cast<int64_t>(lambda_max)) n *= 2;
  if (n <= (1 << 15)) return static_cast<int32_t>(n);
  if ((1 << 15) - 2 * static_cast<int64_t>(lambda_max) >= 8192) return 1 << 15;
  if (n <= (1 << 17)) return static_cast<int32_t>(n);
  if ((1 << 17) - 2 * static_cast<int64_t>(lambda_max) >= 16384) return 1 << 17;
  return 0;
}

mm_status launch_noise_weight(Plan* P, const float* t, float* u, float2* scratch,
                              const int32_t* done, hipStream_t s) {
  if (P->n_samples == 0) return MM_OK;
  TimedLaunch tl(P, K_TOEPLITZ, s);
  if (P->n_chunks > 0) {
    if (P->algo == MM_TOEPLITZ_FFT && long_fft_size(P->fft_n)) {
      MM_TRY(launch_toeplitz_long(P, t, u, scratch, done, s));
    } else if (P->algo == MM_TOEPLITZ_FFT) {
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
