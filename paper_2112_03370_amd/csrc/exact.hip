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

// ---- load: window samples of each segment, packed as complex points -----------------------
template <bool kData>
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
        if (kData) {
          t = static_cast<double>(d[g]);
        } else {
          const double* m = x + 3 * static_cast<int64_t>(p);
          t = m[0] + static_cast<double>(wq[g]) * m[1] + static_cast<double>(wu[g]) * m[2];
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

// ---- real spectrum times the band symbol, repacked and conjugated -----------------------
__global__ __launch_bounds__(kXThreads) void k_x_spectrum(
    const double2* __restrict__ Z, double2* __restrict__ out, const double2* __restrict__ tw,
    const double* __restrict__ spec, const Chunk* __restrict__ chunks, int seg0, int NC) {
  const int k = blockIdx.x * kXThreads + threadIdx.x;
  if (k >= NC) return;
  const int64_t base = static_cast<int64_t>(blockIdx.y) * NC;
  const double* S = spec + static_cast<int64_t>(chunks[seg0 + blockIdx.y].band) * (NC + 1);
  const double2 zk = Z[base + k];
  const double2 zm = Z[base + ((NC - k) & (NC - 1))];
  // even / odd half spectra: E = (Z[k] + conj Z[-k]) / 2, O = (Z[k] - conj Z[-k]) / (2i)
  const double2 e = make_double2(0.5 * (zk.x + zm.x), 0.5 * (zk.y - zm.y));
  const double2 od = make_double2(0.5 * (zk.y + zm.y), -0.5 * (zk.x - zm.x));
  const double2 w = tw[k];  // W_N^k
  const double2 wo = cmul(w, od);
  const double2 xk = cadd(e, wo);           // X[k]
  const double2 xm = cconj(csub(e, wo));    // X[NC - k] (X[NC] for k = 0)
  const double2 yk = make_double2(S[k] * xk.x, S[k] * xk.y);
  const double2 ym = make_double2(S[NC - k] * xm.x, S[NC - k] * xm.y);
  // Q = (Y[k] + Y[k + NC]) + i (Y[k] - Y[k + NC]) conj(W_N^k), Y[k + NC] = conj Y[NC - k]
  const double2 ymc = cconj(ym);
  const double2 fe = cadd(yk, ymc);
  const double2 fo = cmul(csub(yk, ymc), cconj(w));
  const double2 q = make_double2(fe.x - fo.y, fe.y + fo.x);
  out[base + k] = cconj(q);
}

struct XFlush {
  double* y;
  __device__ void operator()(int key, const double (&v)[3]) const {
    double* dst = y + 3 * static_cast<int64_t>(key);
    unsafeAtomicAdd(dst + 0, v[0]);
    unsafeAtomicAdd(dst + 1, v[1]);
    unsafeAtomicAdd(dst + 2, v[2]);
  }
};

// ---- outputs of each segment, pointed back into the pixel domain -------------------------
__global__ __launch_bounds__(kXThreads) void k_x_scatter(
    const double2* __restrict__ G, const int32_t* __restrict__ lpix,
    const float* __restrict__ wq, const float* __restrict__ wu, const Chunk* __restrict__ chunks,
    int seg0, int lam, int NC, double inv_n, double* __restrict__ y) {
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
  wave_merge_runs<3>(key, v, XFlush{y});
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

// Forward DFT of every segment of the batch: radix-16 passes, then the remaining factor.
// Returns the tile holding the result (a or b).
mm_status batch_fft(double2* a, double2* b, const double2* tw, int NC, int nseg, hipStream_t s,
                    double2** result) {
  double2* in = a;
  double2* out = b;
  int p = 1;
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

mm_status exact_product(Plan* P, const double* x, const float* d, double* y, hipStream_t s) {
  MM_TRY(launch_zero(y, 3 * P->n_kept, s));
  if (P->n_kept == 0) return MM_OK;
  const bool data = x == nullptr;
  if (P->n_poly > 0) return launch_template_apply(P, x, d, y, nullptr, s);  // FP64 already
  if (P->lambda_max == 0) return launch_diag_apply(P, x, d, y, nullptr, s);
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
        hipLaunchKernelGGL(k_x_load<true>, gpts, dim3(kXThreads), 0, s, P->lpix, P->wq, P->wu,
                           x, d, P->chunks, seg0, lam, NC, ta.p);
      else
        hipLaunchKernelGGL(k_x_load<false>, gpts, dim3(kXThreads), 0, s, P->lpix, P->wq, P->wu,
                           x, d, P->chunks, seg0, lam, NC, ta.p);
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
