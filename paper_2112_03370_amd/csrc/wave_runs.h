// Wavefront merge of equal-key runs for scatter-adds (P^T and the block-Jacobi build).
//
// Each lane holds SPL consecutive samples (lane l + 1 continues lane l) with their keys (pixel
// ids, -1 = skip) and NV FP64 values.  Time-ordered data visit a pixel for several consecutive
// samples, so keys come in runs.  The lane first sums the pieces of its own runs; runs strictly inside the lane are
// flushed at once.  The run that ends the lane (its tail) may continue in the next lanes: an
// inclusive segmented scan over the lane tails (a new segment starts where the key changes or
// where a lane holds more than one run) gives every lane the sum of its chain so far.  The lane
// that closes a chain flushes it, unless the next lane's first run has the same key, in which
// case that lane adds the chain to its first run and flushes both together.  The result: one
// flush per run and wavefront instead of one atomic per sample.
#pragma once

#include <hip/hip_runtime.h>

namespace mm {

template <int SPL, int NV, class Flush>
__device__ __forceinline__ void wave_merge_runs_n(const int (&key)[SPL], const double (&v)[SPL][NV],
                                                  const Flush& flush) {
  const int lane = static_cast<int>(threadIdx.x & 63u);

  // ---- runs inside the lane --------------------------------------------------------------
  double acc[NV];
  double head[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    acc[c] = v[0][c];
    head[c] = 0.0;
  }
  int cur = key[0];
  int hk = -1;
  bool single = true;
#pragma unroll
  for (int j = 1; j < SPL; ++j) {
    if (key[j] != cur) {
      if (single) {
        hk = cur;
#pragma unroll
        for (int c = 0; c < NV; ++c) head[c] = acc[c];
        single = false;
      } else if (cur >= 0) {
        flush(cur, acc);
      }
      cur = key[j];
#pragma unroll
      for (int c = 0; c < NV; ++c) acc[c] = v[j][c];
    } else {
#pragma unroll
      for (int c = 0; c < NV; ++c) acc[c] += v[j][c];
    }
  }
  const int tk = cur;

  // ---- segmented inclusive scan of the lane tails ----------------------------------------
  const int prev_tk = __shfl_up(tk, 1);
  const bool start = (lane == 0) || !single || (prev_tk != tk);
  double S[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) S[c] = acc[c];
  int f = start ? 1 : 0;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    if (__ballot((!f) && lane >= d) == 0) break;  // wavefront-uniform exit
    double up[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) up[c] = __shfl_up(S[c], d);
    const int fup = __shfl_up(f, d);
    if (lane >= d && !f) {
#pragma unroll
      for (int c = 0; c < NV; ++c) S[c] += up[c];
      f = fup;
    }
  }

  // ---- flushes -----------------------------------------------------------------------------
  double prevS[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) prevS[c] = __shfl_up(S[c], 1);
  const int next_start = __shfl_down(start ? 1 : 0, 1);
  const int next_single = __shfl_down(single ? 1 : 0, 1);
  const int next_hk = __shfl_down(hk, 1);

  if (!single && hk >= 0) {
    if (lane > 0 && prev_tk == hk) {
#pragma unroll
      for (int c = 0; c < NV; ++c) head[c] += prevS[c];
    }
    flush(hk, head);
  }
  const bool ends = (lane == 63) || next_start;
  if (ends && tk >= 0) {
    const bool consumed = (lane < 63) && !next_single && next_hk == tk;
    if (!consumed) flush(tk, S);
  }
}

template <int NV, class Flush>
__device__ __forceinline__ void wave_merge_runs(const int (&key)[4], const double (&v)[4][NV],
                                                const Flush& flush) {
  wave_merge_runs_n<4, NV>(key, v, flush);
}

}  // namespace mm
