// Toeplitz products for long bands: shift-and-overlap segments of N = 2^16 or 2^17 real samples
// (lambda up to 2^15 and beyond), in two forms that share one four-step transform:
//
//   plain  u = N^-1 t for FP32 time-domain vectors in HBM (the stand-alone N^-1 t product)
//   fused  y += P^T N^-1 (P x) or y += P^T N^-1 d: the gather fills the transform's input and
//          the run-merged FP64 scatter drains its output, so t and u never leave the CU
//
// A segment's NC = N / 2 complex points (256 KB or 512 KB) exceed one CU's LDS, so the transform
// runs in four steps through a tile in global memory (NC = N1 x 256, N1 = NC / 256):
//
//   F1  64 columns at a time: fill the window's complex points z[256 n1 + n2] (samples 2p and
//       2p + 1 of point p), DFT over n1 in LDS, multiply by exp(-2 pi i n2 k1 / NC), store to
//       tile row k1
//   F2  64 rows at a time, grouped as (k1, N1 - k1) pairs: DFT over n2 gives X[k1 + N1 k2];
//       with both rows of every pair in LDS, unpack the real spectrum, multiply by the band
//       symbol and repack (conjugated) in place; the inverse's first DFT (over k2) and its
//       twiddle exp(-2 pi i k1 m2 / NC) follow in LDS; store back to the same rows.  The
//       spectrum step is Z'[k] = p_k conj(Z[k]) - i q_k Z[NC - k] with two real coefficients
//       per bin (derivation with symbol_multiply); the plan stores (p_k, q_k) in exactly the
//       order F2 visits the bins, so that each wavefront reads them with one coalesced load.
//   F3  64 columns at a time: DFT over k1 yields the inverse in natural order; drain the
//       segment's outputs (real parts at even samples, minus imaginary parts at odd ones)
//
// Layout for the CDNA memory system:
//   * 512 threads and about 72 KB of LDS per workgroup: two workgroups per CU, so that one
//     workgroup's transform runs while the other waits on its fill, tile pass or drain.  A
//     group's 32 transforms are interleaved in LDS (element e of transform c at e * 33 + c) and
//     thread (c, b) runs butterfly b of transform c: a wavefront's butterfly accesses are runs of
//     32 consecutive slots, and row loads and stores (64 consecutive elements of one row,
//     stride 33) touch each bank the minimum number of times.
//   * Persistent workgroups: the grid is two workgroups per CU (at most), each takes segments
//     in turn and keeps ONE tile for all of them (256 MB in all for N = 2^17 on 256 CUs),
//     instead of a tile per segment (2 GB for the satellite-sized workload).
//   * The workgroups of one XCD take consecutive segments at the same time, so the shared
//     lambda halos of neighbouring windows are fetched together.
//   * Global accesses are wavefront-contiguous: 256 bytes per tile row piece, 8 samples per
//     lane in the fills and drains (64-sample row pieces).
// Measured on the satellite-sized workload (2^28 samples, N = 2^17): one fused product takes
// 5.4 ms, against 7.1 ms for the three kernels (gather, four-step product, scatter) with FP32
// time-domain vectors in HBM; of it about 1.9 ms is the FP64 atomic scatter, 1.1 ms the
// gather and 0.9 ms the tile passes.
#include "fft_lds.h"
#include "mm_internal.h"
#include "segment_io.h"
#include "wave_runs.h"

namespace mm {

namespace {

using namespace fft;

constexpr int kG = 32;        // columns (F1, F3) or rows (F2) per LDS group
constexpr int kLT = 16 * kG;  // threads per workgroup: 16 butterflies of each of kG transforms
constexpr int kN2 = 256;      // tile row length
constexpr int kS = kG + 1;    // LDS stride between consecutive elements of a group's transforms
constexpr int kRowLanes = 2 * kG / 8;        // lanes per row piece in the fills and drains
constexpr int kWaveRows = 64 / kRowLanes;    // row pieces per wavefront
constexpr int kFillRows = kLT / kRowLanes;   // row pieces per fill or drain round
constexpr int kFine = 512;  // fine twiddle table size (exp(-2 pi i m / N), m < 512)
constexpr int kLane = 8;    // consecutive samples per lane in the fills and drains

enum LongIo { kIoPlain = 0, kIoApply = 1, kIoRhs = 2 };

template <int NN>
struct LongTw {
  const float2* fine;
  const float2* coarse;
  __device__ __forceinline__ float2 operator()(int m) const {  // exp(-2 pi i m / NN), m < NN
    return cmul(coarse[m >> 9], fine[m & (kFine - 1)]);
  }
};

struct LongArgs {
  const float* t;  // plain: input and output vectors
  float* u;
  const int32_t* lpix;  // fused: pointing, map(s) or data, accumulated output map(s)
  const float* wq;
  const float* wu;
  const double* x0;
  const float* d0;
  double* y0;
  int64_t ldx, ldy;
  int ncol;
  int vec;  // plain: t and u 16-byte aligned; fused rhs: every data column 16-byte aligned
  const Chunk* chunks;
  int n_work;  // segments x columns
  const float4* pq;
  const float2* tw0;
  const float2* tw1;
  float2* tiles;  // one NC-point tile per workgroup
  int lam;
  const int32_t* done;
};

// One radix-R Stockham pass over the kG interleaved transforms of length L in LDS (element e of
// transform c at buf[e * kS + c]); thread (c, b) runs butterfly b of transform c, so a
// wavefront's accesses are runs of kG consecutive slots.
template <int L, int R, int NN>
__device__ __forceinline__ void ipass(float2* buf, int p, const LongTw<NN>& tw, int c, int b) {
  constexpr int BPT = L / R;  // butterflies per transform
  static_assert(BPT <= kLT / kG, "one butterfly per thread");
  const bool act = b < BPT;
  const int k = b & (p - 1);
  float2 v[R];
  if (act) {
#pragma unroll
    for (int j = 0; j < R; ++j) v[j] = buf[(b + j * BPT) * kS + c];
    if (p > 1) {
      const int step = k * (NN / (p * R));
#pragma unroll
      for (int j = 1; j < R; ++j) v[j] = cmul(v[j], tw((j * step) & (NN - 1)));
    }
    dft<R>(v);
  }
  __syncthreads();
  if (act) {
    const int base = (b - k) * R + k;
#pragma unroll
    for (int m = 0; m < R; ++m) buf[(base + m * p) * kS + c] = v[out_slot<R>(m)];
  }
  __syncthreads();
}

// kG interleaved forward DFTs of length L (256 = 16 x 16, 128 = 16 x 8), natural order out.
template <int L, int NN>
__device__ __forceinline__ void ifft(float2* buf, const LongTw<NN>& tw, int c, int b) {
  static_assert(L == 256 || L == 128, "transform length");
  ipass<L, 16, NN>(buf, 1, tw, c, b);
  ipass<L, L / 16, NN>(buf, 16, tw, c, b);
}

// Row k1 held in slot r of F2 group g: group 0 = {0, N1/2, 1, N1-1, ..., 31, N1-31}, group
// g > 0 = {32g, N1-32g, ..., 32g+31, N1-32g-31}; the partner row N1 - k1 sits in slot r ^ 1
// (itself for rows 0 and N1/2).
template <int N1>
__device__ __forceinline__ int row_of(int g, int r) {
  constexpr int H = kG / 2;
  if (g == 0) {
    if (r == 0) return 0;
    if (r == 1) return N1 / 2;
    const int k = 1 + (r - 2) / 2;
    return (r & 1) ? N1 - k : k;
  }
  const int k = H * g + r / 2;
  return (r & 1) ? N1 - k : k;
}

// Spectrum-step coefficients in F2's visiting order.  Every bin k of a row group is paired
// with its partner NC - k, and one thread handles both bins of a pair in place: in group g,
// thread (lane c, wavefront w) at step i < 8 takes position kl = w + 16 i and
//   lanes c = 2m, 2m + 1 (slots 2m, 2m + 1 hold rows k1 and N1 - k1): bin A = (slot 2m,
//     position kl + 128 (c & 1)), bin B = (slot 2m + 1, position 255 - position of A);
//   group 0, lane 0 (row 0, bins N1 k2): A = (0, kl), B = (0, (256 - kl) mod 256), and the
//     thread with kl = 0 also takes the single bin (0, 128);
//   group 0, lane 1 (row N1/2): A = (1, kl), B = (1, 255 - kl).
// Entry ((g 8 + i) 16 + w) 64 + c holds (p, q) of A and of B; entry NC / 2 holds (p, q) of the
// single bin.  p_k = 2 (sigma - delta sin(2 pi k / N)), q_k = 2 delta cos(2 pi k / N), sigma and
// delta the sum and difference of the symbol at k and NC - k; FP64, rounded once.
struct PairBins {
  int ra, ka, rb, kb;  // slots and positions of bins A and B
};

__device__ __forceinline__ PairBins pair_bins(int g, int c, int w, int i) {
  const int kl = w + 16 * i;
  PairBins p;
  if (g == 0 && c < 2) {
    p.ra = p.rb = c;
    p.ka = kl;
    p.kb = c == 0 ? ((kN2 - kl) & (kN2 - 1)) : kN2 - 1 - kl;
  } else {
    p.ra = c & ~1;
    p.rb = c | 1;
    p.ka = kl + (kN2 / 2) * (c & 1);
    p.kb = kN2 - 1 - p.ka;
  }
  return p;
}

__device__ __forceinline__ float2 spectrum_coef(const float* S, int NC, int k) {
  const double sa = S[k], sb = S[NC - k];
  const double sig = 2.0 * (sa + sb), del = 2.0 * (sa - sb);
  double sn, cs;
  sincospi(static_cast<double>(k) / static_cast<double>(NC), &sn, &cs);  // angle 2 pi k / N
  return make_float2(static_cast<float>(sig - del * sn), static_cast<float>(del * cs));
}

template <int LOGNC>
__global__ __launch_bounds__(256) void k_long_table(const float* __restrict__ spec,
                                                    float4* __restrict__ tab) {
  constexpr int NC = 1 << LOGNC, N1 = NC / kN2;
  const int e = blockIdx.x * 256 + threadIdx.x;  // <= NC / 2
  const int band = blockIdx.y;
  const float* S = spec + static_cast<int64_t>(band) * (NC + 1);
  float4* T = tab + static_cast<int64_t>(band) * (NC / 2 + 1);
  if (e == NC / 2) {
    const float2 a = spectrum_coef(S, NC, NC / 2);  // row 0, position 128
    T[e] = make_float4(a.x, a.y, a.x, a.y);
    return;
  }
  if (e > NC / 2) return;
  const int c = e % kG, w = (e / kG) % 16, i = (e / (kG * 16)) % 8, g = e / (kG * 16 * 8);
  const PairBins p = pair_bins(g, c, w, i);
  const float2 a = spectrum_coef(S, NC, row_of<N1>(g, p.ra) + N1 * p.ka);
  const float2 b = spectrum_coef(S, NC, row_of<N1>(g, p.rb) + N1 * p.kb);
  T[e] = make_float4(a.x, a.y, b.x, b.y);
}

// Window samples [g, g + kLane) of one segment (zero outside its block [b0, b1)).
template <int IO>
__device__ __forceinline__ void fill_lane(const LongArgs& a, const double* __restrict__ x,
                                          const float* __restrict__ d, int64_t g, int64_t b0,
                                          int64_t b1, float (&v)[kLane]) {
  if (g + kLane <= b0 || g >= b1) {
#pragma unroll
    for (int j = 0; j < kLane; ++j) v[j] = 0.0f;
    return;
  }
  const bool inside = g >= b0 && g + kLane <= b1 && (g & 3) == 0;
  if constexpr (IO == kIoPlain) {
    if (inside && a.vec) {
      const float4 lo = *reinterpret_cast<const float4*>(a.t + g);
      const float4 hi = *reinterpret_cast<const float4*>(a.t + g + 4);
      v[0] = lo.x; v[1] = lo.y; v[2] = lo.z; v[3] = lo.w;
      v[4] = hi.x; v[5] = hi.y; v[6] = hi.z; v[7] = hi.w;
    } else {
#pragma unroll
      for (int j = 0; j < kLane; ++j)
        v[j] = (g + j >= b0 && g + j < b1) ? a.t[g + j] : 0.0f;
    }
  } else {
    constexpr bool kD = IO == kIoRhs;
    if (inside && (!kD || a.vec)) {
      LanePointing<kLane, kD> lane;
      lane.load(a.lpix, a.wq, a.wu, d, g);
      lane.resolve(x, v);
    } else {
#pragma unroll
      for (int j = 0; j < kLane; ++j) {
        const int64_t gj = g + j;
        v[j] = 0.0f;
        if (gj >= b0 && gj < b1)
          v[j] = gather_one<kD>(a.lpix[gj], a.wq[gj], a.wu[gj], x, kD ? d[gj] : 0.0f);
      }
    }
  }
}

// Runs listed per wavefront and drain round before their atomics; the list lives in the
// wavefront's own row pieces of the group buffer, which it has read by then.
constexpr int kListed = 64;
static_assert(kListed * (3 * sizeof(double) + sizeof(int)) <= kWaveRows * kS * sizeof(float2),
              "run list must fit the wavefront's row pieces");

// Output samples [o, o + kLane) of a segment (only those in [0, out_len) exist).  The fused
// form must be reached by whole wavefronts (the run merge exchanges lanes); `list` is the
// wavefront's LDS for its run list (no other wavefront touches it during the call).
template <int IO>
__device__ __forceinline__ void drain_lane(const LongArgs& a, double* __restrict__ y,
                                           const Chunk& c, int o, const float (&v)[kLane],
                                           float2* list) {
  const int64_t go = c.out0 + o;
  const bool inside = o >= 0 && o + kLane <= c.out_len && (go & 3) == 0;
  if constexpr (IO == kIoPlain) {
    if (inside && a.vec) {
      *reinterpret_cast<float4*>(a.u + go) = make_float4(v[0], v[1], v[2], v[3]);
      *reinterpret_cast<float4*>(a.u + go + 4) = make_float4(v[4], v[5], v[6], v[7]);
    } else {
#pragma unroll
      for (int j = 0; j < kLane; ++j)
        if (o + j >= 0 && o + j < c.out_len) a.u[go + j] = v[j];
    }
  } else {
    int key[kLane];
    double val[kLane][3];
    if (inside) {
      LanePointing<kLane, false> lane;
      lane.load(a.lpix, a.wq, a.wu, nullptr, go);
#pragma unroll
      for (int j = 0; j < kLane; ++j) {
        const double tv = v[j];
        key[j] = lane.kk[j];
        val[j][0] = tv;
        val[j][1] = static_cast<double>(lane.qq[j]) * tv;
        val[j][2] = static_cast<double>(lane.uu[j]) * tv;
      }
    } else {
#pragma unroll
      for (int j = 0; j < kLane; ++j) {
        key[j] = -1;
        val[j][0] = val[j][1] = val[j][2] = 0.0;
        if (o + j >= 0 && o + j < c.out_len) {
          const int64_t oj = go + j;
          const double tv = v[j];
          key[j] = a.lpix[oj];
          val[j][0] = tv;
          val[j][1] = static_cast<double>(a.wq[oj]) * tv;
          val[j][2] = static_cast<double>(a.wu[oj]) * tv;
        }
      }
    }
    double* sval = reinterpret_cast<double*>(list);
    int* skey = reinterpret_cast<int*>(sval + 3 * kListed);
    wave_merge_runs_listed<kLane, 3, kListed, AtomicFlush, true>(key, val, AtomicFlush{y}, skey,
                                                                 sval);
  }
}

// The value itself, opaque to the optimiser: per-thread index arithmetic derived from it is
// redone in every round of the persistent loop instead of being hoisted out of it (64 twiddle
// and row indices held across the whole loop do not fit the 128 registers of a thread).
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Work item of workgroup b in round `round`: the 8 XCDs take workgroups in turn, so when the
// grid is a multiple of 8 the workgroups of one XCD get consecutive items in every round.
__device__ __forceinline__ int work_item(int b, int nb, int round) {
  if ((nb & 7) != 0) return round * nb + b;
  return round * nb + (b & 7) * (nb >> 3) + (b >> 3);
}

// Four waves per SIMD: two workgroups per CU (128 registers per lane).
template <int LOGNC, int IO>
__global__ __launch_bounds__(kLT) __attribute__((amdgpu_waves_per_eu(4))) void k_long(
    const LongArgs a) {
  constexpr int NC = 1 << LOGNC, NN = 2 * NC, N1 = NC / kN2;
  static_assert(N1 == 128 || N1 == 256, "tile shape");
  __shared__ float2 buf[kN2 * kS];
  __shared__ float2 fine[kFine];
  __shared__ float2 coarse[NN / kFine];
  if (a.done != nullptr && *a.done) return;
  const int tid = threadIdx.x;
  for (int i = tid; i < kFine; i += kLT) fine[i] = a.tw0[i];
  for (int i = tid; i < NN / kFine; i += kLT) coarse[i] = a.tw1[i];
  const LongTw<NN> tw{fine, coarse};
  float2* __restrict__ Z = a.tiles + static_cast<int64_t>(blockIdx.x) * NC;
  __syncthreads();

  for (int round = 0;; ++round) {
    const int item = work_item(blockIdx.x, gridDim.x, round);
    if (item >= a.n_work) break;
    // lane roles: transform slot (lane) and butterfly / row (wavefront); kRowLanes lanes of
    // 8 samples per 2 kG-sample row piece in the fills and drains
    const int lt = opaque(tid);
    const int tc = lt % kG, tw_ = lt / kG;                        // transform, butterfly
    const int fr = lt / kRowLanes, fq = lt % kRowLanes;           // row piece, lane in it
    const int wave = __builtin_amdgcn_readfirstlane(lt >> 6);     // wavefront (uniform)
    const int col = item % a.ncol;
    const Chunk c = a.chunks[item / a.ncol];
    const double* __restrict__ x = IO == kIoApply ? a.x0 + col * a.ldx : nullptr;
    const float* __restrict__ d = IO == kIoRhs ? a.d0 + col * a.ldx : nullptr;
    double* __restrict__ y = IO == kIoPlain ? nullptr : a.y0 + col * a.ldy;
    const int64_t in0 = c.out0 - a.lam;
    const int64_t b0 = c.blk_start, b1 = c.blk_start + c.blk_len;

    // ---- F1: fill 64 columns, DFT over n1, twiddle, store tile rows ----------------------
#pragma unroll 1
    for (int g = 0; g < kN2 / kG; ++g) {
#pragma unroll 1
      for (int rr = 0; rr < N1 / kFillRows; ++rr) {
        const int n1 = rr * kFillRows + fr;
        const int w = 2 * (n1 * kN2 + kG * g) + kLane * fq;  // window sample of the lane
        float v[kLane];
        fill_lane<IO>(a, x, d, in0 + w, b0, b1, v);
        float2* dst = buf + n1 * kS + 4 * fq;
#pragma unroll
        for (int j = 0; j < kLane / 2; ++j) dst[j] = make_float2(v[2 * j], v[2 * j + 1]);
      }
      __syncthreads();
      ifft<N1, NN>(buf, tw, tc, tw_);
#pragma unroll
      for (int i = 0; i < N1 / 16; ++i) {
        const int k1 = tw_ + 16 * i, n2 = kG * g + tc;
        Z[k1 * kN2 + n2] = cmul(buf[k1 * kS + tc], tw((2 * ((n2 * k1) & (NC - 1))) & (NN - 1)));
      }
      __syncthreads();
    }

    // ---- F2: row DFTs, symbol, inverse row DFTs ------------------------------------------
    const float4* __restrict__ PQ = a.pq + static_cast<int64_t>(c.band) * (NC / 2 + 1);
#pragma unroll 1
    for (int g = 0; g < N1 / kG; ++g) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int r = (kLT / kN2) * i + (wave >> 2), e = (lt & 255);
        buf[e * kS + r] = Z[row_of<N1>(g, r) * kN2 + e];
      }
      __syncthreads();
      ifft<kN2, NN>(buf, tw, tc, tw_);  // slot r, position k2: X[k1 + N1 k2]
      // spectrum step, one bin pair per thread and step, in place
#pragma unroll 4
      for (int i = 0; i < 8; ++i) {
        const PairBins p = pair_bins(g, tc, tw_, i);
        const float4 pq = PQ[((g * 8 + i) * 16 + tw_) * kG + tc];
        const float2 A = buf[p.ka * kS + p.ra], B = buf[p.kb * kS + p.rb];
        buf[p.ka * kS + p.ra] =
            make_float2(pq.x * A.x + pq.y * B.y, -(pq.x * A.y + pq.y * B.x));
        if (p.kb != p.ka || p.rb != p.ra)
          buf[p.kb * kS + p.rb] =
              make_float2(pq.z * B.x + pq.w * A.y, -(pq.z * B.y + pq.w * A.x));
      }
      if (g == 0 && tid == 0) {  // the single bin of row 0 at position 128
        const float4 pq = PQ[NC / 2];
        const float2 A = buf[(kN2 / 2) * kS];
        buf[(kN2 / 2) * kS] = make_float2(pq.x * A.x + pq.y * A.y, -(pq.x * A.y + pq.y * A.x));
      }
      __syncthreads();
      ifft<kN2, NN>(buf, tw, tc, tw_);  // slot r, position m2
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int r = (kLT / kN2) * i + (wave >> 2), m2 = (lt & 255);
        const int k1 = row_of<N1>(g, r);
        Z[k1 * kN2 + m2] = cmul(buf[m2 * kS + r], tw((2 * ((k1 * m2) & (NC - 1))) & (NN - 1)));
      }
      __syncthreads();
    }

    // ---- F3: column DFTs over k1, outputs in natural order --------------------------------
#pragma unroll 1
    for (int g = 0; g < kN2 / kG; ++g) {
#pragma unroll
      for (int i = 0; i < N1 / 16; ++i) {
        const int k1 = tw_ + 16 * i;
        buf[k1 * kS + tc] = Z[k1 * kN2 + kG * g + tc];
      }
      __syncthreads();
      ifft<N1, NN>(buf, tw, tc, tw_);
#pragma unroll 1
      for (int rr = 0; rr < N1 / kFillRows; ++rr) {
        // the wavefront's kWaveRows row pieces cover window samples [lo, hi); skip them
        // together when none of those samples is an output
        const int m1w = rr * kFillRows + kWaveRows * wave;
        const int lo = 2 * (m1w * kN2 + kG * g);
        const int hi = lo + (kWaveRows - 1) * 2 * kN2 + 2 * kG;
        if (hi <= a.lam || lo >= a.lam + c.out_len) continue;  // wavefront-uniform
        const int m1 = rr * kFillRows + fr;
        const float2* src = buf + m1 * kS + 4 * fq;
        float v[kLane];
#pragma unroll
        for (int j = 0; j < kLane / 2; ++j) {
          const float2 F = src[j];
          v[2 * j] = F.x;
          v[2 * j + 1] = -F.y;
        }
        const int o = 2 * (m1 * kN2 + kG * g) + kLane * fq - a.lam;
        drain_lane<IO>(a, y, c, o, v, buf + m1w * kS);
      }
      __syncthreads();
    }
  }
}

}  // namespace

bool long_fft_size(int32_t n) { return n == (1 << 16) || n == (1 << 17); }

int32_t long_fine_size() { return kFine; }

int32_t long_slots(const Plan* P) {
  // two workgroups (and tiles) per CU, fewer when a plan has few segments
  const int64_t want = static_cast<int64_t>(P->n_chunks) * 16;
  return static_cast<int32_t>(std::max<int64_t>(1, std::min<int64_t>(2 * P->n_cu, want)));
}

mm_status build_long_table(Plan* P, hipStream_t s) {
  if (P->n_bands == 0 || !long_fft_size(P->fft_n)) return MM_OK;
  const int NC = P->fft_n / 2;
  MM_TRY(dalloc(P, &P->long_pq, static_cast<size_t>(P->n_bands) * (NC / 2 + 1)));
  const dim3 grid(static_cast<unsigned>(NC / 512 + 1), static_cast<unsigned>(P->n_bands));
  if (P->fft_n == (1 << 16))
    hipLaunchKernelGGL(k_long_table<15>, grid, dim3(256), 0, s, P->spec, P->long_pq);
  else
    hipLaunchKernelGGL(k_long_table<16>, grid, dim3(256), 0, s, P->spec, P->long_pq);
  MM_HIP_TRY(hipGetLastError());
  return MM_OK;
}

namespace {

template <int IO>
mm_status launch_long(Plan* P, const LongArgs& a, hipStream_t s) {
  const int grid = std::min(a.n_work, long_slots(P));
  if (P->fft_n == (1 << 16))
    hipLaunchKernelGGL((k_long<15, IO>), dim3(grid), dim3(kLT), 0, s, a);
  else if (P->fft_n == (1 << 17))
    hipLaunchKernelGGL((k_long<16, IO>), dim3(grid), dim3(kLT), 0, s, a);
  else
    return fail(MM_ERR_UNSUPPORTED, "long FFT size not supported");
  MM_HIP_TRY(hipGetLastError());
  return MM_OK;
}

LongArgs base_args(Plan* P, float2* tiles, const int32_t* done) {
  LongArgs a{};
  a.chunks = P->chunks;
  a.pq = P->long_pq;
  a.tw0 = P->tw0;
  a.tw1 = P->tw1;
  a.tiles = tiles;
  a.lam = P->lambda_max;
  a.done = done;
  a.ncol = 1;
  return a;
}

}  // namespace

mm_status launch_toeplitz_long(Plan* P, const float* t, float* u, float2* tiles,
                               const int32_t* done, hipStream_t s) {
  if (P->n_chunks == 0) return MM_OK;
  if (tiles == nullptr) return fail(MM_ERR_INVALID, "long-segment product without its tiles");
  if (P->long_pq == nullptr) return fail(MM_ERR_INVALID, "long-segment product without its table");
  LongArgs a = base_args(P, tiles, done);
  a.t = t;
  a.u = u;
  a.vec = ((reinterpret_cast<uintptr_t>(t) | reinterpret_cast<uintptr_t>(u)) & 15u) == 0;
  a.n_work = P->n_chunks;
  return launch_long<kIoPlain>(P, a, s);
}

mm_status launch_apply_long(Plan* P, const double* x, const float* d, int64_t ldx, double* y,
                            int64_t ldy, int32_t ncol, float2* tiles, const int32_t* done,
                            hipStream_t s) {
  if (P->n_chunks == 0 || ncol <= 0) return MM_OK;
  if (tiles == nullptr) return fail(MM_ERR_INVALID, "long-segment product without its tiles");
  if (P->long_pq == nullptr) return fail(MM_ERR_INVALID, "long-segment product without its table");
  const int64_t n_work = static_cast<int64_t>(P->n_chunks) * ncol;
  if (n_work > INT32_MAX) return fail(MM_ERR_UNSUPPORTED, "too many segment x column items");
  LongArgs a = base_args(P, tiles, done);
  a.lpix = P->lpix;
  a.wq = P->wq;
  a.wu = P->wu;
  a.x0 = x;
  a.d0 = d;
  a.y0 = y;
  a.ldx = ldx;
  a.ldy = ldy;
  a.ncol = ncol;
  a.n_work = static_cast<int>(n_work);
  if (d != nullptr) {
    a.vec = (reinterpret_cast<uintptr_t>(d) & 15u) == 0 && (ldx & 3) == 0;
    return launch_long<kIoRhs>(P, a, s);
  }
  return launch_long<kIoApply>(P, a, s);
}

}  // namespace mm
