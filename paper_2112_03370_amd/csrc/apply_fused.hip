// Fused system product for the FFT path: one workgroup per overlap-save segment does
//
//   gather   t = P x (FP64 sums rounded to FP32) or t = d at kept samples, straight into LDS
//   Toeplitz u = N^-1 t by the LDS real FFT (shift-and-overlap segment, Toeplitz package)
//   scatter  y += P^T u for the segment's outputs, FP64, run-merged atomics
//
// so the time-domain vectors never go to HBM: per output sample the kernel reads the pointing
// of its input window (12 B per window sample, the lambda halo included) and again for its
// outputs, and issues the run-merged atomics.  Samples outside every block (identity rows of
// stbmm) are handled by the diagonal kernel over identity tiles.
//
// The gather is bound by the number of vector memory instructions, not by bytes: a lane takes
// 8 consecutive samples (two 16-byte loads per pointing array) and loads a pixel's three values
// only when the pixel changes, which scan runs make rare.
#include "fft_lds.h"
#include "mm_internal.h"
#include "segment_io.h"
#include "wave_runs.h"



namespace mm {

namespace {

using namespace fft;

// Consecutive samples per lane in the gather and in the scatter.  Wider lanes issue fewer,
// wider memory instructions and load a pixel's values once per run; 8 is the widest that
// 1,024-thread workgroups (128 registers per lane) hold without spilling.
constexpr int kGatherLane = 8;
constexpr int kScatterLane = 8;

template <int LOG, bool kFromData>
__global__ __launch_bounds__(FftCfg<LOG>::T) void k_apply_fused(
    const int32_t* __restrict__ lpix, const float* __restrict__ wq, const float* __restrict__ wu,
    const double* __restrict__ x0, const float* __restrict__ d0, int d_vec, double* __restrict__ y0,
    int ncol, int64_t ldx, int64_t ldy, const Chunk* __restrict__ chunks,
    const float* __restrict__ spec,
    const float2* __restrict__ tw0g, const float2* __restrict__ tw1g, int lam,
    const int32_t* __restrict__ done) {
  using C = FftCfg<LOG>;
  constexpr int NC = C::NC, N = C::N, T = C::T;
  __shared__ float2 buf[C::LDS];
  __shared__ float2 tw0[128];
  __shared__ float2 tw1[N / 128];
  if (done != nullptr && *done) return;
  const int tid = threadIdx.x;
  for (int i = tid; i < 128; i += T) tw0[i] = tw0g[i];
  for (int i = tid; i < N / 128; i += T) tw1[i] = tw1g[i];

  // workgroup -> (segment, column), columns fastest: an XCD runs all columns of a segment
  // back to back, so the pointing re-reads of the later columns hit its L2
  const int wg = xcd_ordered(blockIdx.x, gridDim.x);
  const int col = wg % ncol;
  const Chunk c = chunks[wg / ncol];
  const double* __restrict__ x = kFromData ? x0 : x0 + col * ldx;
  const float* __restrict__ d = kFromData ? d0 + col * ldx : d0;
  double* __restrict__ y = y0 + col * ldy;
  const int64_t in0 = c.out0 - lam;
  const int64_t b0 = c.blk_start, b1 = c.blk_start + c.blk_len;

  // ---- gather the N-sample window (zero outside the block) ---------------------------------
  // Four rounds of T SG samples, one window quarter each.  With N = 4 lambda the right half of
  // the window is the left half of the next segment's, and neighbouring segments run at the
  // same time on one XCD: even segments gather their right half first, odd ones their left
  // half first, so both readers of a shared half fetch it together and the second finds it in
  // L2.
  constexpr int SG = kGatherLane;
  static_assert(N == 4 * T * SG, "four gather rounds");
  const int rot = ((wg / ncol) & 1) == 0 ? 2 : 0;
  for (int rr = 0; rr < 4; ++rr) {
    const int n = ((rr + rot) & 3) * (T * SG) + tid * SG;
    const int64_t g = in0 + n;
    float v[SG];
    if (g >= b0 && g + SG <= b1 && (g & 3) == 0 && (!kFromData || d_vec)) {
      LanePointing<SG, kFromData> lane;
      lane.load(lpix, wq, wu, d, g);
      lane.resolve(x, v);
    } else {
#pragma unroll
      for (int j = 0; j < SG; ++j) {
        const int64_t gj = g + j;
        v[j] = 0.0f;
        if (gj >= b0 && gj < b1)
          v[j] = gather_one<kFromData>(lpix[gj], wq[gj], wu[gj], x, kFromData ? d[gj] : 0.0f);
      }
    }
    // samples n..n+SG-1 are complex points n/2.. (n/2 even: contiguous pairs after padding)
    float2* dst = buf + pad(n >> 1);
#pragma unroll
    for (int j = 0; j < SG / 2; ++j) dst[j] = make_float2(v[2 * j], v[2 * j + 1]);
  }
  __syncthreads();

  // ---- Toeplitz product in LDS ----------------------------------------------------------------
  fft_forward<LOG, T>(buf, tw0, tw1);
  symbol_multiply<LOG, T>(buf, spec + static_cast<int64_t>(c.band) * (NC + 1), tw0, tw1);
  fft_forward<LOG, T>(buf, tw0, tw1);

  // ---- scatter the segment's outputs ----------------------------------------------------------
  constexpr int SS = kScatterLane;
  const AtomicFlush flush{y};
  for (int base = 0; base < c.out_len; base += T * SS) {  // same trip count for every lane
    const int i0 = base + tid * SS;
    const int64_t o = c.out0 + i0;
    int key[SS];
    double v[SS][3];
    if (i0 + SS <= c.out_len && (o & 3) == 0) {
      LanePointing<SS, false> lane;
      lane.load(lpix, wq, wu, nullptr, o);
#pragma unroll
      for (int j = 0; j < SS; ++j) {
        const double tv = real_out(buf, lam + i0 + j);
        key[j] = lane.kk[j];
        v[j][0] = tv;
        v[j][1] = static_cast<double>(lane.qq[j]) * tv;
        v[j][2] = static_cast<double>(lane.uu[j]) * tv;
      }
    } else {
#pragma unroll
      for (int j = 0; j < SS; ++j) {
        key[j] = -1;
        v[j][0] = v[j][1] = v[j][2] = 0.0;
        if (i0 + j < c.out_len) {
          const int64_t oj = o + j;
          key[j] = lpix[oj];
          const double tv = real_out(buf, lam + i0 + j);
          v[j][0] = tv;
          v[j][1] = static_cast<double>(wq[oj]) * tv;
          v[j][2] = static_cast<double>(wu[oj]) * tv;
        }
      }
    }
    wave_merge_runs_n<SS, 3>(key, v, flush);
  }
}

template <int LOG>
mm_status launch(Plan* P, const double* x, const float* d, int64_t ldx, double* y, int64_t ldy,
                 int ncol, const int32_t* done, hipStream_t s) {
  using C = FftCfg<LOG>;
  const bool vec = (reinterpret_cast<uintptr_t>(d) & 15u) == 0 && (ldx & 3) == 0;
  const int d_vec = vec ? 1 : 0;
  const int64_t grid = static_cast<int64_t>(P->n_chunks) * ncol;
  if (grid > INT32_MAX) return fail(MM_ERR_UNSUPPORTED, "too many segment x column workgroups");
  if (d != nullptr) {
    hipLaunchKernelGGL((k_apply_fused<LOG, true>), dim3(static_cast<unsigned>(grid)), dim3(C::T), 0,
                       s, P->lpix, P->wq, P->wu, x, d, d_vec, y, ncol, ldx, ldy, P->chunks,
                       P->spec, P->tw0, P->tw1, P->lambda_max, done);
  } else {
    hipLaunchKernelGGL((k_apply_fused<LOG, false>), dim3(static_cast<unsigned>(grid)), dim3(C::T), 0,
                       s, P->lpix, P->wq, P->wu, x, d, d_vec, y, ncol, ldx, ldy, P->chunks,
                       P->spec, P->tw0, P->tw1, P->lambda_max, done);
  }
  MM_HIP_TRY(hipGetLastError());
  return MM_OK;
}

}  // namespace

mm_status launch_apply_fused(Plan* P, const double* x, const float* d, double* y,
                             const int32_t* done, hipStream_t s, float2* tiles, int32_t ncol,
                             int64_t ldx, int64_t ldy) {
  if (P->n_kept == 0 || ncol <= 0) return MM_OK;
  if (ldx == 0) ldx = d != nullptr ? P->n_samples : 3 * P->n_kept;
  if (ldy == 0) ldy = 3 * P->n_kept;
  if (P->n_chunks > 0 && long_fft_size(P->fft_n)) {
    TimedLaunch tl(P, K_TOEPLITZ, s);
    MM_TRY(launch_apply_long(P, x, d, ldx, y, ldy, ncol, tiles, done, s));
  } else if (P->n_chunks > 0 && P->reg_fft) {
    TimedLaunch tl(P, K_TOEPLITZ, s);
    MM_TRY(launch_apply_reg(P, x, d, ldx, y, ldy, ncol, done, s));
  } else if (P->n_chunks > 0) {
    TimedLaunch tl(P, K_TOEPLITZ, s);
    switch (P->fft_n) {
      case 1 << 11: MM_TRY(launch<10>(P, x, d, ldx, y, ldy, ncol, done, s)); break;
      case 1 << 12: MM_TRY(launch<11>(P, x, d, ldx, y, ldy, ncol, done, s)); break;
      case 1 << 13: MM_TRY(launch<12>(P, x, d, ldx, y, ldy, ncol, done, s)); break;
      case 1 << 14: MM_TRY(launch<13>(P, x, d, ldx, y, ldy, ncol, done, s)); break;
      case 1 << 15: MM_TRY(launch<14>(P, x, d, ldx, y, ldy, ncol, done, s)); break;
      default: return fail(MM_ERR_UNSUPPORTED, "FFT size not supported");
    }
  }
  if (P->n_id_tiles > 0) {
    for (int32_t j = 0; j < ncol; ++j)
      MM_TRY(launch_diag_tiles(P, P->id_tiles, P->n_id_tiles, d ? nullptr : x + j * ldx,
                               d ? d + j * ldx : nullptr, y + j * ldy, done, s));
  }
  return MM_OK;
}

}  // namespace mm
