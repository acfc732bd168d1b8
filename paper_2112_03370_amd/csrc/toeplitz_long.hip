// Toeplitz product for long bands (segment lengths N = 2^16, 2^17 real samples, i.e. lambda up
// to 2^15): the same shift-and-overlap segments as the LDS kernel, but a segment's NC = N/2
// complex points (256 KB or 512 KB) exceed one CU's LDS, so each workgroup runs a four-step
// transform through a per-segment tile in global memory (NC = N1 x 256, N1 = NC / 256):
//
//   F1  16 columns at a time: load the window's samples (complex point N2 n1 + n2), DFT over n1
//       in LDS, multiply by exp(-2 pi i n2 k1 / NC), store to tile row k1
//   F2  16 rows at a time, grouped as (k1, N1 - k1) pairs: DFT over n2 gives X[k1 + N1 k2];
//       with both rows of every pair in LDS, unpack the real spectrum, multiply by the band
//       symbol and repack (conjugated) in place; the inverse's first DFT (over k2) and its
//       twiddle exp(-2 pi i k1 m2 / NC) follow in LDS; store back to the same rows.  The
//       spectrum step is Z'[k] = p_k conj(Z[k]) - i q_k Z[NC - k] with two real coefficients
//       per bin (derivation with symbol_multiply); the plan stores (p_k, q_k) in exactly the
//       order F2 visits the bins, so that each lane reads them with one coalesced load.
//   F3  16 columns at a time: DFT over k1 yields the inverse in natural order; write the
//       segment's outputs (real parts at even samples, minus imaginary parts at odd ones)
//
// 256 threads and 35 KB of LDS per workgroup leave room for several workgroups per CU.
#include "fft_lds.h"
#include "mm_internal.h"

namespace mm {

namespace {

using namespace fft;

constexpr int kLongThreads = 256;
constexpr int kN2 = 256;        // row length of the tile
constexpr int kGroup = 16;      // rows or columns per LDS group
constexpr int kFine = 512;      // fine twiddle table size (exp(-2 pi i m / N), m < 512)

template <int NN>
struct LongTw {
  const float2* fine;
  const float2* coarse;
  __device__ __forceinline__ float2 operator()(int m) const {  // exp(-2 pi i m / NN), m < NN
    return cmul(coarse[m >> 9], fine[m & (kFine - 1)]);
  }
};

// One batched radix-R Stockham pass over NB contiguous transforms of length L held in LDS
// (transform b occupies [b L, (b + 1) L)); twiddles exp(-2 pi i j k / (p R)) from the table of
// the NN-point grid.
template <int L, int NB, int R, int NN>
__device__ __forceinline__ void batched_pass(float2* buf, int p, const LongTw<NN>& tw) {
  constexpr int BPT = L / R;
  constexpr int NBF = NB * BPT;
  constexpr int PER = (NBF + kLongThreads - 1) / kLongThreads;
  float2 v[PER][R];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int b = threadIdx.x + i * kLongThreads;
    if (b < NBF) {
      const int bt = b / BPT, bl = b % BPT, k = bl & (p - 1);
#pragma unroll
      for (int j = 0; j < R; ++j) v[i][j] = buf[pad(bt * L + bl + j * BPT)];
      if (p > 1) {
        const int step = k * (NN / (p * R));
#pragma unroll
        for (int j = 1; j < R; ++j) v[i][j] = cmul(v[i][j], tw((j * step) & (NN - 1)));
      }
      dft<R>(v[i]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int b = threadIdx.x + i * kLongThreads;
    if (b < NBF) {
      const int bt = b / BPT, bl = b % BPT, k = bl & (p - 1);
      const int base = bt * L + (bl - k) * R + k;
#pragma unroll
      for (int m = 0; m < R; ++m) buf[pad(base + m * p)] = v[i][out_slot<R>(m)];
    }
  }
  __syncthreads();
}

// NB forward DFTs of length L (256 = 16 x 16, 128 = 16 x 8) in LDS.
template <int L, int NB, int NN>
__device__ __forceinline__ void batched_fft(float2* buf, const LongTw<NN>& tw) {
  static_assert(L == 256 || L == 128, "transform length");
  batched_pass<L, NB, 16, NN>(buf, 1, tw);
  batched_pass<L, NB, L / 16, NN>(buf, 16, tw);
}

// Row k1 held in slot r of F2 group g: group 0 = {0, N1/2, 1, N1-1, ..., 7, N1-7}, group g > 0
// = {8g, N1-8g, ..., 8g+7, N1-8g-7}; the partner row N1 - k1 sits in slot r ^ 1 (itself for
// rows 0 and N1/2).
template <int N1>
__device__ __forceinline__ int row_of(int g, int r) {
  if (g == 0) {
    if (r == 0) return 0;
    if (r == 1) return N1 / 2;
    const int k = 1 + (r - 2) / 2;
    return (r & 1) ? N1 - k : k;
  }
  const int k = 8 * g + r / 2;
  return (r & 1) ? N1 - k : k;
}

// (p_k, q_k) for the bins of F2 in visiting order: entry (g 16 + r) 256 + k2 is bin
// k = row_of(g, r) + N1 k2, with p_k = 2 (sigma - delta sin(2 pi k / N)),
// q_k = 2 delta cos(2 pi k / N), sigma and delta the sum and difference of the symbol at k and
// NC - k.  FP64, rounded once.
template <int LOGNC>
__global__ __launch_bounds__(kLongThreads) void k_long_table(const float* __restrict__ spec,
                                                             float2* __restrict__ tab) {
  constexpr int NC = 1 << LOGNC, N1 = NC / kN2;
  const int e = blockIdx.x * kLongThreads + threadIdx.x;  // < NC
  const int band = blockIdx.y;
  const int g = e / (kGroup * kN2), r = (e / kN2) % kGroup, k2 = e % kN2;
  const int k = row_of<N1>(g, r) + N1 * k2;
  const float* S = spec + static_cast<int64_t>(band) * (NC + 1);
  const double sa = S[k], sb = S[NC - k];
  const double sig = 2.0 * (sa + sb), del = 2.0 * (sa - sb);
  double sn, cs;
  sincospi(static_cast<double>(k) / static_cast<double>(NC), &sn, &cs);  // angle 2 pi k / N
  tab[static_cast<int64_t>(band) * NC + e] =
      make_float2(static_cast<float>(sig - del * sn), static_cast<float>(del * cs));
}

// Four waves per SIMD (four workgroups per CU, 128 registers) for N = 2^17, where that costs a
// handful of spilled registers and hides more of each group's memory wait; N = 2^16 spills too
// much at that limit and keeps the compiler's choice.
template <int LOGNC>
__global__ __launch_bounds__(kLongThreads)
__attribute__((amdgpu_waves_per_eu(LOGNC == 16 ? 4 : 1))) void k_toeplitz_long(
    const float* __restrict__ t, float* __restrict__ u, const Chunk* __restrict__ chunks,
    const float2* __restrict__ pqtab, const float2* __restrict__ tw0g,
    const float2* __restrict__ tw1g, float2* __restrict__ scratch, int lam, int vec8,
    const int32_t* __restrict__ done) {
  // vec8: t and u are 8-byte aligned, so even sample indices allow 8-byte accesses
  constexpr int NC = 1 << LOGNC, NN = 2 * NC, N1 = NC / kN2;
  constexpr int GL = kGroup * kN2;
  static_assert(N1 == 128 || N1 == 256, "tile shape");
  __shared__ float2 buf[GL + GL / 16];
  __shared__ float2 fine[kFine];
  __shared__ float2 coarse[NN / kFine];
  if (done != nullptr && *done) return;
  const int tid = threadIdx.x;
  for (int i = tid; i < kFine; i += kLongThreads) fine[i] = tw0g[i];
  for (int i = tid; i < NN / kFine; i += kLongThreads) coarse[i] = tw1g[i];
  const LongTw<NN> tw{fine, coarse};

  const int seg = xcd_ordered(blockIdx.x, gridDim.x);
  const Chunk c = chunks[seg];
  float2* Z = scratch + static_cast<int64_t>(seg) * NC;
  const int64_t in0 = c.out0 - lam;
  const int64_t b0 = c.blk_start, b1 = c.blk_start + c.blk_len;
  __syncthreads();

  // ---- F1: column DFTs over n1 --------------------------------------------------------------
  for (int g = 0; g < kN2 / kGroup; ++g) {
    for (int idx = tid; idx < kGroup * N1; idx += kLongThreads) {
      const int n1 = idx >> 4, cc = idx & 15;
      const int64_t gs = in0 + 2 * (static_cast<int64_t>(n1) * kN2 + kGroup * g + cc);
      float2 ab;
      if (vec8 && gs >= b0 && gs + 1 < b1 && (gs & 1) == 0) {  // one 8-byte load
        ab = *reinterpret_cast<const float2*>(t + gs);
      } else {
        ab.x = (gs >= b0 && gs < b1) ? t[gs] : 0.0f;
        ab.y = (gs + 1 >= b0 && gs + 1 < b1) ? t[gs + 1] : 0.0f;
      }
      buf[pad(cc * N1 + n1)] = ab;
    }
    __syncthreads();
    batched_fft<N1, kGroup, NN>(buf, tw);
    for (int idx = tid; idx < kGroup * N1; idx += kLongThreads) {
      const int k1 = idx >> 4, cc = idx & 15, n2 = kGroup * g + cc;
      Z[k1 * kN2 + n2] = cmul(buf[pad(cc * N1 + k1)], tw((2 * ((n2 * k1) & (NC - 1))) & (NN - 1)));
    }
    __syncthreads();
  }

  // ---- F2: row DFTs, symbol, inverse row DFTs ----------------------------------------------
  const float2* __restrict__ PQ = pqtab + static_cast<int64_t>(c.band) * NC;
  for (int g = 0; g < N1 / kGroup; ++g) {
    for (int idx = tid; idx < GL; idx += kLongThreads) {
      const int r = idx >> 8, n2 = idx & 255;
      buf[pad(idx)] = Z[row_of<N1>(g, r) * kN2 + n2];
    }
    __syncthreads();
    batched_fft<kN2, kGroup, NN>(buf, tw);  // slot r, position k2: X[k1 + N1 k2]
    float2 w[GL / kLongThreads];
#pragma unroll
    for (int i = 0; i < GL / kLongThreads; ++i) {
      const int idx = tid + i * kLongThreads;
      const int r = idx >> 8, k2 = idx & 255;
      const int k1 = row_of<N1>(g, r);
      const int k = k1 + N1 * k2;
      const int kk = (NC - k) & (NC - 1);
      const int rp = (k1 == 0 || k1 == N1 / 2) ? r : (r ^ 1);
      const float2 Zk = buf[pad(idx)];
      const float2 Z2 = buf[pad(rp * kN2 + kk / N1)];
      const float2 pq = PQ[g * GL + idx];
      w[i] = make_float2(pq.x * Zk.x + pq.y * Z2.y, -(pq.x * Zk.y + pq.y * Z2.x));
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < GL / kLongThreads; ++i) buf[pad(tid + i * kLongThreads)] = w[i];
    __syncthreads();
    batched_fft<kN2, kGroup, NN>(buf, tw);  // slot r, position m2
    for (int idx = tid; idx < GL; idx += kLongThreads) {
      const int r = idx >> 8, m2 = idx & 255;
      const int k1 = row_of<N1>(g, r);
      Z[k1 * kN2 + m2] = cmul(buf[pad(idx)], tw((2 * ((k1 * m2) & (NC - 1))) & (NN - 1)));
    }
    __syncthreads();
  }

  // ---- F3: column DFTs over k1, outputs in natural order -----------------------------------
  for (int g = 0; g < kN2 / kGroup; ++g) {
    for (int idx = tid; idx < kGroup * N1; idx += kLongThreads) {
      const int k1 = idx >> 4, cc = idx & 15;
      buf[pad(cc * N1 + k1)] = Z[k1 * kN2 + kGroup * g + cc];
    }
    __syncthreads();
    batched_fft<N1, kGroup, NN>(buf, tw);
    for (int idx = tid; idx < kGroup * N1; idx += kLongThreads) {
      const int m1 = idx >> 4, cc = idx & 15;
      const int m = m1 * kN2 + kGroup * g + cc;
      const float2 F = buf[pad(cc * N1 + m1)];
      const int o = 2 * m - lam;  // segment output offset of the real sample 2m
      if (vec8 && o >= 0 && o + 1 < c.out_len && ((c.out0 + o) & 1) == 0) {  // one 8-byte store
        *reinterpret_cast<float2*>(u + c.out0 + o) = make_float2(F.x, -F.y);
      } else {
        if (o >= 0 && o < c.out_len) u[c.out0 + o] = F.x;
        if (o + 1 >= 0 && o + 1 < c.out_len) u[c.out0 + o + 1] = -F.y;
      }
    }
    __syncthreads();
  }
}

}  // namespace

bool long_fft_size(int32_t n) { return n == (1 << 16) || n == (1 << 17); }

mm_status build_long_table(Plan* P, hipStream_t s) {
  if (P->n_bands == 0 || !long_fft_size(P->fft_n)) return MM_OK;
  const int NC = P->fft_n / 2;
  MM_TRY(dalloc(P, &P->long_pq, static_cast<size_t>(P->n_bands) * NC));
  const dim3 grid(static_cast<unsigned>(NC / kLongThreads), static_cast<unsigned>(P->n_bands));
  if (P->fft_n == (1 << 16))
    hipLaunchKernelGGL(k_long_table<15>, grid, dim3(kLongThreads), 0, s, P->spec, P->long_pq);
  else
    hipLaunchKernelGGL(k_long_table<16>, grid, dim3(kLongThreads), 0, s, P->spec, P->long_pq);
  MM_HIP_TRY(hipGetLastError());
  return MM_OK;
}

int32_t long_fine_size() { return kFine; }

mm_status launch_toeplitz_long(Plan* P, const float* t, float* u, float2* scratch,
                               const int32_t* done, hipStream_t s) {
  if (P->n_chunks == 0) return MM_OK;
  if (scratch == nullptr) return fail(MM_ERR_INVALID, "long-segment product without its tiles");
  if (P->long_pq == nullptr) return fail(MM_ERR_INVALID, "long-segment product without its table");
  const int vec8 = ((reinterpret_cast<uintptr_t>(t) | reinterpret_cast<uintptr_t>(u)) & 7u) == 0;
  if (P->fft_n == (1 << 16)) {
    hipLaunchKernelGGL(k_toeplitz_long<15>, dim3(P->n_chunks), dim3(kLongThreads), 0, s, t, u,
                       P->chunks, P->long_pq, P->tw0, P->tw1, scratch, P->lambda_max, vec8, done);
  } else if (P->fft_n == (1 << 17)) {
    hipLaunchKernelGGL(k_toeplitz_long<16>, dim3(P->n_chunks), dim3(kLongThreads), 0, s, t, u,
                       P->chunks, P->long_pq, P->tw0, P->tw1, scratch, P->lambda_max, vec8, done);
  } else {
    return fail(MM_ERR_UNSUPPORTED, "long FFT size not supported");
  }
  MM_HIP_TRY(hipGetLastError());
  return MM_OK;
}

}  // namespace mm
