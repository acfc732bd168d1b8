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

// Orders LDS accesses of one wavefront across its lanes: what lanes wrote before the call is
// visible to reads by other lanes of the same wavefront after it, and reads before it complete
// before later writes to the same slots.  A wavefront-scope release/acquire fence pair around a
// wave barrier; it must be reached by the whole wavefront (uniform control flow).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

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

// Exclusive prefix sum over the wavefront of a small per-lane count c < 2^BITS.
template <int BITS>
__device__ __forceinline__ int wave_exclusive_count(int c, int lane, int& total) {
  const unsigned long long below = (1ull << lane) - 1ull;
  int before = 0;
  total = 0;
#pragma unroll
  for (int b = 0; b < BITS; ++b) {
    const unsigned long long m = __ballot((c >> b) & 1);
    before += __popcll(m & below) << b;
    total += __popcll(m) << b;
  }
  return before;
}

// The same merge, but the runs that the wavefront completes are first listed in LDS (CAP slots
// of one key and NV values per wavefront, `skey` and `sval`) and then flushed one run per lane:
// ceil(R / 64) rounds of NV atomics for R runs.  The direct form above issues one round at every
// lane position where some lane closes a run inside it, which on scans with short runs (a
// circle clipping pixel corners) means several rounds of nearly idle atomic instructions per
// wavefront.  Runs beyond CAP are flushed directly.
//
// kByComponent flushes the list one value per lane instead (lanes NV r .. NV r + NV - 1 take the
// NV values of run r, through flush.one(key, component, value)): ceil(NV R / 64) instructions,
// and the values of one run go out in one instruction.  Where the runs of a wavefront fall on
// different cache lines (pixel ids far apart along the scan), a run then costs one memory-side
// atomic request instead of NV.
template <int SPL, int NV, int CAP, class Flush, bool kByComponent = false>
__device__ __forceinline__ void wave_merge_runs_listed(const int (&key)[SPL],
                                                       const double (&v)[SPL][NV],
                                                       const Flush& flush, int* skey,
                                                       double* sval) {
  static_assert(SPL >= 2 && SPL <= 9, "inner-run counts must fit the 3-bit wavefront prefix");
  const int lane = static_cast<int>(threadIdx.x & 63u);

  // ---- runs inside the lane: count, then list ---------------------------------------------
  // A run starting at a key change j > 0 lies inside the lane when another change follows.
  int n_in = 0, last_keyed = 0;
#pragma unroll
  for (int j = 1; j < SPL; ++j) {
    if (key[j] != key[j - 1]) {
      n_in += last_keyed;
      last_keyed = key[j] >= 0 ? 1 : 0;
    }
  }
  int r_in = 0;
  const int in_base = wave_exclusive_count<3>(n_in, lane, r_in);
  wave_lds_sync();  // the previous call's listed runs have been read before slots are reused

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
  int slot = in_base;
#pragma unroll
  for (int j = 1; j < SPL; ++j) {
    if (key[j] != cur) {
      if (single) {
        hk = cur;
#pragma unroll
        for (int c = 0; c < NV; ++c) head[c] = acc[c];
        single = false;
      } else if (cur >= 0) {
        if (slot < CAP) {
          skey[slot] = cur;
#pragma unroll
          for (int c = 0; c < NV; ++c) sval[slot * NV + c] = acc[c];
        } else {
          flush(cur, acc);
        }
        ++slot;
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

  // ---- segmented inclusive scan of the lane tails (as in the direct form) -----------------
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

  // ---- the lane's head and closing tail ------------------------------------------------------
  double prevS[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) prevS[c] = __shfl_up(S[c], 1);
  const int next_start = __shfl_down(start ? 1 : 0, 1);
  const int next_single = __shfl_down(single ? 1 : 0, 1);
  const int next_hk = __shfl_down(hk, 1);

  const bool has_head = !single && hk >= 0;
  if (has_head && lane > 0 && prev_tk == hk) {
#pragma unroll
    for (int c = 0; c < NV; ++c) head[c] += prevS[c];
  }
  const bool ends = (lane == 63) || next_start;
  const bool has_tail =
      ends && tk >= 0 && !((lane < 63) && !next_single && next_hk == tk);
  const int n_ht = (has_head ? 1 : 0) + (has_tail ? 1 : 0);
  int r_ht = 0;
  int s2 = r_in + wave_exclusive_count<2>(n_ht, lane, r_ht);
  if (has_head) {
    if (s2 < CAP) {
      skey[s2] = hk;
#pragma unroll
      for (int c = 0; c < NV; ++c) sval[s2 * NV + c] = head[c];
    } else {
      flush(hk, head);
    }
    ++s2;
  }
  if (has_tail) {
    if (s2 < CAP) {
      skey[s2] = tk;
#pragma unroll
      for (int c = 0; c < NV; ++c) sval[s2 * NV + c] = S[c];
    } else {
      flush(tk, S);
    }
  }

  // ---- one listed run (or one value of one) per lane ---------------------------------------
  wave_lds_sync();  // runs listed by other lanes of the wavefront are visible
  const int listed = r_in + r_ht < CAP ? r_in + r_ht : CAP;
  if constexpr (kByComponent) {
    const int n = listed * NV;
    for (int e = lane; e - lane < n; e += 64) {
      if (e < n) {
        const int r = e / NV;
        flush.one(skey[r], e - r * NV, sval[e]);
      }
    }
  } else {
    for (int r = lane; r - lane < listed; r += 64) {
      if (r < listed) {
        double w[NV];
#pragma unroll
        for (int c = 0; c < NV; ++c) w[c] = sval[r * NV + c];
        flush(skey[r], w);
      }
    }
  }
}

template <int NV, class Flush>
__device__ __forceinline__ void wave_merge_runs(const int (&key)[4], const double (&v)[4][NV],
                                                const Flush& flush) {
  wave_merge_runs_n<4, NV>(key, v, flush);
}

}  // namespace mm
