// Fused system product for 2^15-sample overlap-save segments with a register-resident FFT.
//
// Same operation as the LDS-resident fused kernel (gather t = P x, Toeplitz u = N^-1 t by the
// real FFT of the segment, scatter y += P^T u over the segment's outputs), laid out so that
// two workgroups share a CU: 512 threads each hold 32 of the 16,384 complex points in
// registers, and LDS (about 77 KB per workgroup) only stages the gather, the transposes between
// the three radix steps and the outputs.  While one workgroup waits on its gather or scatter
// the other keeps the vector ALUs busy with its transforms, which a single 142 KB workgroup
// per CU cannot do.
//
// Transform (NC = 16384 points z[n] = t[2n] + i t[2n+1], n = n1 + 16 n2 + 512 j,
// k = k3 + 32 k2 + 1024 k1):
//   A  thread t = n1 + 16 n2 holds z[t + 512 j], j < 32: radix-32 over j, twiddle W_NC^(t k3)
//   B  thread (k3, n1) holds slot n2:                  radix-32 over n2, twiddle W_512^(n1 k2)
//   C  thread holds two tasks (k3, k2), slot n1:       radix-16 over n1 -> Z[k], k1 < 16
// The two tasks of a thread are chosen so that the partner bin NC - k of each of its bins is
// also in the thread, so the real-spectrum step (unpack, band symbol, repack) stays in
// registers.  The inverse runs the same steps transposed (C, B, A with the same twiddles):
// the transposed factorisation of the symmetric DFT matrix is the DFT again, so it maps the
// repacked spectrum back to the natural order that the first step read.
#include "fft_lds.h"
#include "mm_internal.h"
#include "segment_io.h"
#include "wave_runs.h"

namespace mm {

namespace {

using namespace fft;

constexpr int kT = 512;            // threads per workgroup
constexpr int kNC = 16384;         // complex points per segment
constexpr int kN = 2 * kNC;        // real samples per segment
constexpr int kHalf = kNC;         // window samples staged per gather half; outputs at most
constexpr int kRowA = 528;         // LDS stride of a k3 row in the A <-> B transposes
constexpr int kRowB = 560;         // LDS stride of a k3 plane in the B <-> C transposes (measured:
                                   // 39 % fewer bank conflicts than 544)
constexpr int kLdsF = 32 * kRowB;  // floats of staging LDS
constexpr int kLane = 8;           // consecutive samples per lane in the gather and scatter
constexpr int kListed = 64;        // runs listed per wavefront and scatter round
constexpr int kTab = 16 * kT + 8;  // symbol pairs per band in the kernel's read order
constexpr int kW2 = 33;            // row stride of the W_512 table

typedef __attribute__((address_space(1))) const void* global_ptr;
typedef __attribute__((address_space(3))) void* lds_ptr;

// Direct load of 16 B per lane from global memory into LDS at (wave-uniform) wave_base +
// 16 B x lane, without passing through registers.
__device__ __forceinline__ void load_to_lds16(const void* src, void* wave_base) {
  __builtin_amdgcn_global_load_lds((global_ptr)src, (lds_ptr)wave_base, 16, 0, 0);
}

// Tasks of a thread in the C layout: (a3, a2) and its mirror (b3, b2).
__device__ __forceinline__ void reg_tasks(int tid, int& a3, int& a2, int& b3, int& b2) {
  if (tid >= 32) {
    a3 = tid >> 5;
    a2 = tid & 31;
    b3 = 32 - a3;
    b2 = 31 - a2;
  } else if (tid >= 16) {
    a3 = 16;
    a2 = tid - 16;
    b3 = 16;
    b2 = 47 - tid;
  } else {
    a3 = 0;
    a2 = tid;
    b3 = 0;
    b2 = tid == 0 ? 16 : 32 - tid;
  }
}

// cos and sin of 2 pi k / 32, k < 16
__device__ constexpr float kCos32[16] = {
    1.0f, 0.98078528040323043f, 0.92387953251128674f, 0.83146961230254524f,
    0.70710678118654752f, 0.55557023301960218f, 0.38268343236508978f, 0.19509032201612827f,
    0.0f, -0.19509032201612827f, -0.38268343236508978f, -0.55557023301960218f,
    -0.70710678118654752f, -0.83146961230254524f, -0.92387953251128674f, -0.98078528040323043f};
__device__ constexpr float kSin32[16] = {
    0.0f, 0.19509032201612827f, 0.38268343236508978f, 0.55557023301960218f,
    0.70710678118654752f, 0.83146961230254524f, 0.92387953251128674f, 0.98078528040323043f,
    1.0f, 0.98078528040323043f, 0.92387953251128674f, 0.83146961230254524f,
    0.70710678118654752f, 0.55557023301960218f, 0.38268343236508978f, 0.19509032201612827f};

// Radix-32 DFT on v[0..32) in natural order: two radix-16 DFTs (even and odd points) and a
// radix-2 step with W_32^k.
__device__ __forceinline__ void dft32(float2 (&v)[32]) {
  float2 e[16], o[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    e[i] = v[2 * i];
    o[i] = v[2 * i + 1];
  }
  dft<16>(e);
  dft<16>(o);
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const float2 E = e[out_slot<16>(k)];
    float2 O = o[out_slot<16>(k)];
    if (k == 8)
      O = mul_mi(O);
    else if (k != 0)
      O = cmul(O, make_float2(kCos32[k], -kSin32[k]));
    v[k] = cadd(E, O);
    v[k + 16] = csub(E, O);
  }
}

// Radix-16 DFT on v[off..off+16) in natural order.
template <int OFF>
__device__ __forceinline__ void dft16_at(float2 (&v)[32]) {
  float2 u[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) u[i] = v[OFF + i];
  dft<16>(u);
#pragma unroll
  for (int k = 0; k < 16; ++k) v[OFF + k] = u[out_slot<16>(k)];
}

// v[k] *= W_NC^(t k) = W_N^(2 t k), k < 32, from five table twiddles and their products
// (2 t k < 2^15 for t < 512: no reduction of the angle index).
__device__ __forceinline__ void twiddle_a(float2 (&v)[32], int t, const float2* tw0,
                                          const float2* tw1) {
  const float2 w1 = twiddle(tw0, tw1, 2 * t), w2 = twiddle(tw0, tw1, 4 * t);
  const float2 w4 = twiddle(tw0, tw1, 8 * t), w8 = twiddle(tw0, tw1, 16 * t);
  const float2 w16 = twiddle(tw0, tw1, 32 * t);
  float2 lo[8];
  lo[0] = make_float2(1.0f, 0.0f);
  lo[1] = w1;
  lo[2] = w2;
  lo[3] = cmul(w1, w2);
  lo[4] = w4;
  lo[5] = cmul(w1, w4);
  lo[6] = cmul(w2, w4);
  lo[7] = cmul(lo[3], w4);
  const float2 hi[4] = {make_float2(1.0f, 0.0f), w8, w16, cmul(w8, w16)};
#pragma unroll
  for (int h = 0; h < 4; ++h) {
#pragma unroll
    for (int l = 0; l < 8; ++l) {
      const int k = 8 * h + l;
      if (k == 0) continue;
      const float2 w = h == 0 ? lo[l] : (l == 0 ? hi[h] : cmul(hi[h], lo[l]));
      v[k] = cmul(v[k], w);
    }
  }
}

template <int C>
__device__ __forceinline__ float& part(float2& z) {
  if constexpr (C == 0) return z.x;
  else return z.y;
}

// A layout (thread t, slot k3) -> B layout (thread (k3, n1), slot n2), one component.
template <int C>
__device__ __forceinline__ void transpose_ab(float2 (&v)[32], float* lds, int tid, int k3b,
                                            int n1b) {
#pragma unroll
  for (int k = 0; k < 32; ++k) lds[k * kRowA + tid] = part<C>(v[k]);
  __syncthreads();
#pragma unroll
  for (int n2 = 0; n2 < 32; ++n2) part<C>(v[n2]) = lds[k3b * kRowA + n1b + 16 * n2];
  __syncthreads();
}

// B layout -> A layout.
template <int C>
__device__ __forceinline__ void transpose_ba(float2 (&v)[32], float* lds, int tid, int k3b,
                                            int n1b) {
#pragma unroll
  for (int n2 = 0; n2 < 32; ++n2) lds[k3b * kRowA + n1b + 16 * n2] = part<C>(v[n2]);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 32; ++k) part<C>(v[k]) = lds[k * kRowA + tid];
  __syncthreads();
}

// Task slots of the B <-> C transposes: plane k3, row k2 of 17 floats, column n1.
struct Tasks {
  int a, b;  // k3 * kRowB + 17 * k2 of the two tasks
};

// B layout (thread (k3, n1), slot k2) -> C layout (tasks a, b; slots n1 and 16 + n1).
template <int C>
__device__ __forceinline__ void transpose_bc(float2 (&v)[32], float* lds, Tasks tk, int k3b,
                                            int n1b) {
#pragma unroll
  for (int k2 = 0; k2 < 32; ++k2) lds[k3b * kRowB + 17 * k2 + n1b] = part<C>(v[k2]);
  __syncthreads();
#pragma unroll
  for (int n1 = 0; n1 < 16; ++n1) {
    part<C>(v[n1]) = lds[tk.a + n1];
    part<C>(v[16 + n1]) = lds[tk.b + n1];
  }
  __syncthreads();
}

// C layout -> B layout.
template <int C>
__device__ __forceinline__ void transpose_cb(float2 (&v)[32], float* lds, Tasks tk, int k3b,
                                            int n1b) {
#pragma unroll
  for (int n1 = 0; n1 < 16; ++n1) {
    lds[tk.a + n1] = part<C>(v[n1]);
    lds[tk.b + n1] = part<C>(v[16 + n1]);
  }
  __syncthreads();
#pragma unroll
  for (int k2 = 0; k2 < 32; ++k2) part<C>(v[k2]) = lds[k3b * kRowB + 17 * k2 + n1b];
  __syncthreads();
}

// Real-spectrum step for one bin pair: X1 = Z[k], X2 = Z[NC - k] (indices mod NC), sa = S[k],
// sb = S[NC - k], W = W_N^k; the repacked, conjugated inverse input replaces both (see
// symbol_multiply in the LDS kernels for the derivation).
__device__ __forceinline__ void spectrum_pair(float2& X1, float2& X2, float sa, float sb,
                                              float2 W) {
  const float a = 2.0f * sa, b = 2.0f * sb;
  const float sig = a + b, del = a - b;
  const float ds = del * W.y;
  const float p = sig + ds, p2 = sig - ds, q = del * W.x;
  const float2 y1 = make_float2(p * X1.x + q * X2.y, -(p * X1.y + q * X2.x));
  const float2 y2 = make_float2(p2 * X2.x + q * X1.y, -(p2 * X2.y + q * X1.x));
  X1 = y1;
  X2 = y2;
}

// A bin that is its own partner (k = 0 or NC/2).
__device__ __forceinline__ void spectrum_self(float2& X, float sa, float sb, float2 W) {
  const float a = 2.0f * sa, b = 2.0f * sb;
  const float sig = a + b, del = a - b;
  const float p = sig + del * W.y, q = del * W.x;
  X = make_float2(p * X.x + q * X.y, -(p * X.y + q * X.x));
}

// Window samples [H kHalf, (H + 1) kHalf) (zero outside the block [b0, b1)) through LDS into
// the A layout: z[t + 512 j] = (t[2m], t[2m+1]), m = t + 512 j, j in [16 H, 16 H + 16).
template <int H, bool kFromData>
__device__ __forceinline__ void gather_half(float2 (&v)[32], float* lds, int tid,
                                            const int32_t* __restrict__ lpix,
                                            const float* __restrict__ wq,
                                            const float* __restrict__ wu,
                                            const double* __restrict__ x,
                                            const float* __restrict__ d, int d_vec, int64_t in0,
                                            int64_t b0, int64_t b1) {
  for (int n = tid * kLane; n < kHalf; n += kT * kLane) {
    const int64_t g = in0 + H * kHalf + n;
    float s[kLane];
    if (g >= b0 && g + kLane <= b1 && (g & 3) == 0 && (!kFromData || d_vec)) {
      LanePointing<kLane, kFromData> lane;
      lane.load(lpix, wq, wu, d, g);
      lane.resolve(x, s);
    } else {
#pragma unroll
      for (int j = 0; j < kLane; ++j) {
        const int64_t gj = g + j;
        s[j] = 0.0f;
        if (gj >= b0 && gj < b1)
          s[j] = gather_one<kFromData>(lpix[gj], wq[gj], wu[gj], x, kFromData ? d[gj] : 0.0f);
      }
    }
    *reinterpret_cast<float4*>(lds + n) = make_float4(s[0], s[1], s[2], s[3]);
    *reinterpret_cast<float4*>(lds + n + 4) = make_float4(s[4], s[5], s[6], s[7]);
  }
  __syncthreads();
#pragma unroll
  for (int jj = 0; jj < 16; ++jj)
    v[16 * H + jj] = *reinterpret_cast<const float2*>(lds + 2 * (tid + kT * jj));
  __syncthreads();
}

template <bool kFromData>
__global__ __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(4))) void k_apply_reg(
    const int32_t* __restrict__ lpix, const float* __restrict__ wq, const float* __restrict__ wu,
    const double* __restrict__ x0, const float* __restrict__ d0, int d_vec, double* __restrict__ y0,
    int ncol, int64_t ldx, int64_t ldy, const Chunk* __restrict__ chunks,
    const float2* __restrict__ tab, const float2* __restrict__ tw0g,
    const float2* __restrict__ tw1g, int lam, const int32_t* __restrict__ done) {
  __shared__ __align__(16) float lds[kLdsF + 64];
  __shared__ float2 tw0[128];
  __shared__ float2 tw1[kN / 128];
  // W_512^(n1 k2) = W_N^(64 n1 k2) at [n1 * kW2 + k2], n1 < 16, k2 < 32: rows of 33 so that
  // both the step-B reads (lanes across n1, slot k2 fixed) and the inverse reads (lanes across
  // k2, n1 fixed) hit distinct banks
  __shared__ float2 w512[16 * kW2];
  if (done != nullptr && *done) return;
  const int tid = threadIdx.x;
  if (tid < 128) tw0[tid] = tw0g[tid];
  if (tid < kN / 128) tw1[tid] = tw1g[tid];
  {
    const int e = (tid >> 5) * (tid & 31);  // < 512
    w512[(tid >> 5) * kW2 + (tid & 31)] = cmul(tw1g[e >> 1], tw0g[(e & 1) * 64]);
  }

  const int wg = xcd_ordered(blockIdx.x, gridDim.x);
  const int col = wg % ncol;
  const Chunk c = chunks[wg / ncol];
  const double* __restrict__ x = kFromData ? x0 : x0 + col * ldx;
  const float* __restrict__ d = kFromData ? d0 + col * ldx : d0;
  double* __restrict__ y = y0 + col * ldy;
  const int64_t in0 = c.out0 - lam;
  const int64_t b0 = c.blk_start, b1 = c.blk_start + c.blk_len;

  // thread roles: A layout t = tid; B layout (k3, n1); C layout two mirror tasks
  const int k3b = tid >> 4, n1b = tid & 15;
  int a3, a2, b3, b2;
  reg_tasks(tid, a3, a2, b3, b2);
  const Tasks tk{a3 * kRowB + 17 * a2, b3 * kRowB + 17 * b2};

  float2 v[32];

  // ---- gather the window in two halves of 16,384 samples through LDS ----------------------
  // The gather runs at raised wave priority: its waves issue their loads and finish their FP64
  // sums ahead of the other workgroup's transform, which has VALU work to fill the wait
  // (measured: -4 % per solve on the ground workload; the same for the scatter gave nothing).
  __builtin_amdgcn_s_setprio(3);
  // The right half of a segment's window is the left half of the next segment's (lambda = 2^13;
  // nearly so otherwise), and neighbouring segments run at the same time on one XCD: even
  // segments gather their right half first and odd ones their left half first, so that both
  // readers of a shared half fetch it together and the second finds it in L2.
  if (((wg / ncol) & 1) == 0) {
    gather_half<1, kFromData>(v, lds, tid, lpix, wq, wu, x, d, d_vec, in0, b0, b1);
    gather_half<0, kFromData>(v, lds, tid, lpix, wq, wu, x, d, d_vec, in0, b0, b1);
  } else {
    gather_half<0, kFromData>(v, lds, tid, lpix, wq, wu, x, d, d_vec, in0, b0, b1);
    gather_half<1, kFromData>(v, lds, tid, lpix, wq, wu, x, d, d_vec, in0, b0, b1);
  }

  // ---- forward transform --------------------------------------------------------------------
  __builtin_amdgcn_s_setprio(0);
  dft32(v);
  twiddle_a(v, tid, tw0, tw1);
  transpose_ab<0>(v, lds, tid, k3b, n1b);
  transpose_ab<1>(v, lds, tid, k3b, n1b);
  dft32(v);
#pragma unroll
  for (int k2 = 1; k2 < 32; ++k2) v[k2] = cmul(v[k2], w512[n1b * kW2 + k2]);
  transpose_bc<0>(v, lds, tk, k3b, n1b);
  transpose_bc<1>(v, lds, tk, k3b, n1b);
  // The band's symbol pairs (kTab float2, in this kernel's read order) go straight from global
  // memory into the idle staging LDS while the radix-16 steps run: each wave's direct load of
  // 16 B per lane lands at its wave base + 16 B x lane.
  {
    const float4* __restrict__ tg = reinterpret_cast<const float4*>(tab + c.band * kTab);
    const int wbase = tid & ~63;
#pragma unroll
    for (int r = 0; r < 8; ++r)
      load_to_lds16(tg + r * kT + tid, lds + 4 * (r * kT + wbase));
    if (tid < (2 * kTab) / 4 - 8 * kT)
      load_to_lds16(tg + 8 * kT + tid, lds + 4 * 8 * kT);
  }
  dft16_at<0>(v);
  dft16_at<16>(v);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  // ---- real spectrum x band symbol, in registers --------------------------------------------
  // Slot k1 of task a is bin k = a3 + 32 a2 + 1024 k1 and its partner NC - k is slot 15 - k1 of
  // task b, for every thread but the first, whose tasks (0, 0) and (0, 16) are their own
  // partners.  All threads run the common pairing; thread 0 keeps its spectrum in a private LDS
  // slot, where lanes 0..16 of its wave redo its 17 bin pairs (two of them single bins) side by
  // side, and reloads it after the common pairing.  That keeps the common path free of a second
  // register pairing.  The slot is written and read by one wave only; wavefront-scope fences
  // order the hand-offs between its lanes.  (The side work comes before the common pairing: placed after it, the
  // compiler's schedule no longer fits the 128 registers of two workgroups per CU.)
  {
    const float2* stab = reinterpret_cast<const float2*>(lds);  // [k1][thread], then 8 extra
    float2* own = reinterpret_cast<float2*>(lds + kLdsF);  // thread 0 only; the transposes never
                                                            // reach past kLdsF
    if (tid == 0) {
#pragma unroll
      for (int i = 0; i < 32; ++i) own[i] = v[i];
    }
    wave_lds_sync();  // thread 0's slot is visible to lanes 0..16
    if (tid < 17) {
      // task (0, 0): bins 1024 k1, partners k1 <-> 16 - k1, bins 0 and NC/2 alone (lanes 0..8);
      // task (0, 16): bins 512 + 1024 k1, partners k1 <-> 15 - k1 (lanes 9..16)
      int i1, i2, k, e;
      if (tid == 0) {
        i1 = i2 = 0;
        k = 0;
        e = 0;
      } else if (tid == 1) {
        i1 = i2 = 8;
        k = kNC / 2;
        e = 8 * kT;
      } else if (tid <= 8) {
        i1 = tid - 1;
        i2 = 17 - tid;
        k = 1024 * i1;
        e = i1 * kT;
      } else {
        i1 = tid + 7;
        i2 = 40 - tid;
        k = 512 + 1024 * (tid - 9);
        e = 16 * kT + tid - 9;
      }
      float2 X1 = own[i1], X2 = own[i2];
      const float2 ss = stab[e];
      spectrum_pair(X1, X2, ss.x, ss.y, twiddle(tw0, tw1, k));
      own[i1] = X1;
      if (i2 != i1) own[i2] = X2;
    }
    const int ka = a3 + 32 * a2;
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) {
      const float2 ss = stab[k1 * kT + tid];
      spectrum_pair(v[k1], v[31 - k1], ss.x, ss.y, twiddle(tw0, tw1, ka + 1024 * k1));
    }
    wave_lds_sync();  // lanes 0..16 have written the slot back before thread 0 reloads it
    if (tid == 0) {
#pragma unroll
      for (int i = 0; i < 32; ++i) v[i] = own[i];
    }
  }
  __syncthreads();  // the staged symbol is read: the transposes may reuse the buffer

  // ---- inverse: the transposed steps --------------------------------------------------------
  dft16_at<0>(v);
  dft16_at<16>(v);
#pragma unroll
  for (int n1 = 1; n1 < 16; ++n1) {
    v[n1] = cmul(v[n1], w512[n1 * kW2 + a2]);
    v[16 + n1] = cmul(v[16 + n1], w512[n1 * kW2 + b2]);
  }
  transpose_cb<0>(v, lds, tk, k3b, n1b);
  transpose_cb<1>(v, lds, tk, k3b, n1b);
  dft32(v);
  transpose_ba<0>(v, lds, tid, k3b, n1b);
  transpose_ba<1>(v, lds, tid, k3b, n1b);
  twiddle_a(v, tid, tw0, tw1);
  dft32(v);

  // ---- outputs to LDS: sample 2m is Re, 2m+1 is -Im of point m = t + 512 j ------------------
  const int out_len = c.out_len;
  if ((lam & 1) == 0) {
#pragma unroll
    for (int j = 0; j < 32; ++j) {
      const int i = 2 * (tid + kT * j) - lam;  // even
      if (i >= 0 && i + 1 < out_len) {
        *reinterpret_cast<float2*>(lds + i) = make_float2(v[j].x, -v[j].y);
      } else if (i >= 0 && i < out_len) {
        lds[i] = v[j].x;
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < 32; ++j) {
      const int i = 2 * (tid + kT * j) - lam;
      if (i >= 0 && i < out_len) lds[i] = v[j].x;
      if (i + 1 >= 0 && i + 1 < out_len) lds[i + 1] = -v[j].y;
    }
  }
  __syncthreads();

  // ---- scatter the segment's outputs ----------------------------------------------------------
  // Each wavefront reads its own 512 staged outputs per round; once read, that slice holds the
  // wavefront's list of completed runs, flushed one FP64 value per lane.
  const AtomicFlush flush{y};
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  static_assert(kListed * (3 * sizeof(double) + sizeof(int)) <= 64 * kLane * sizeof(float),
                "run list must fit the wavefront's slice of the staged outputs");
  static_assert((kHalf + kT * kLane - 1) / (kT * kLane) * (kT * kLane) <= kLdsF,
                "every round's slices lie inside the staging buffer");
  for (int base = 0; base < out_len; base += kT * kLane) {  // same trip count for every lane
    const int i0 = base + tid * kLane;
    const int64_t o = c.out0 + i0;
    int key[kLane];
    double val[kLane][3];
    if (i0 + kLane <= out_len && (o & 3) == 0) {
      LanePointing<kLane, false> lane;
      lane.load(lpix, wq, wu, nullptr, o);
#pragma unroll
      for (int j = 0; j < kLane; ++j) {
        const double tv = lds[i0 + j];
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
        if (i0 + j < out_len) {
          const int64_t oj = o + j;
          key[j] = lpix[oj];
          const double tv = lds[i0 + j];
          val[j][0] = tv;
          val[j][1] = static_cast<double>(wq[oj]) * tv;
          val[j][2] = static_cast<double>(wu[oj]) * tv;
        }
      }
    }
    double* sval = reinterpret_cast<double*>(lds + base + 64 * kLane * wave);
    int* skey = reinterpret_cast<int*>(sval + 3 * kListed);
    wave_merge_runs_listed<kLane, 3, kListed, AtomicFlush, true>(key, val, flush, skey, sval);
  }
}

// Symbol pairs of every band in the register kernel's read order: entry [k1][thread] is
// (S[k], S[NC - k]) for bin k = a3 + 32 a2 + 1024 k1 of the thread's first task; then the 8
// bins 512 + 1024 j of the first thread's second task.
__global__ __launch_bounds__(kT) void k_reg_table(const float* __restrict__ spec,
                                                  float2* __restrict__ tab) {
  const int tid = threadIdx.x;
  const float* __restrict__ S = spec + static_cast<int64_t>(blockIdx.x) * (kNC + 1);
  float2* __restrict__ T = tab + static_cast<int64_t>(blockIdx.x) * kTab;
  int a3, a2, b3, b2;
  reg_tasks(tid, a3, a2, b3, b2);
  const int ka = a3 + 32 * a2;
  for (int k1 = 0; k1 < 16; ++k1) {
    const int k = ka + 1024 * k1;
    T[k1 * kT + tid] = make_float2(S[k], S[kNC - k]);
  }
  if (tid < 8) {
    const int k = 512 + 1024 * tid;
    T[16 * kT + tid] = make_float2(S[k], S[kNC - k]);
  }
}

}  // namespace

mm_status build_reg_table(Plan* P, hipStream_t s) {
  if (P->n_bands == 0) return MM_OK;
  MM_TRY(dalloc(P, &P->spec_reg, static_cast<size_t>(P->n_bands) * kTab));
  hipLaunchKernelGGL(k_reg_table, dim3(static_cast<unsigned>(P->n_bands)), dim3(kT), 0, s,
                     P->spec, P->spec_reg);
  MM_HIP_TRY(hipGetLastError());
  return MM_OK;
}

bool apply_reg_supported(const Plan* P) {
  return P->fft_n == kN && P->fft_n - 2 * static_cast<int64_t>(P->lambda_max) <= kHalf;
}

mm_status launch_apply_reg(Plan* P, const double* x, const float* d, int64_t ldx, double* y,
                           int64_t ldy, int32_t ncol, const int32_t* done, hipStream_t s) {
  if (!apply_reg_supported(P) || P->spec_reg == nullptr)
    return fail(MM_ERR_UNSUPPORTED, "register FFT kernel: segment shape");
  const bool vec = (reinterpret_cast<uintptr_t>(d) & 15u) == 0 && (ldx & 3) == 0;
  const int d_vec = vec ? 1 : 0;
  const int64_t grid = static_cast<int64_t>(P->n_chunks) * ncol;
  if (grid > INT32_MAX) return fail(MM_ERR_UNSUPPORTED, "too many segment x column workgroups");
  if (d != nullptr) {
    hipLaunchKernelGGL((k_apply_reg<true>), dim3(static_cast<unsigned>(grid)), dim3(kT), 0, s,
                       P->lpix, P->wq, P->wu, x, d, d_vec, y, ncol, ldx, ldy, P->chunks, P->spec_reg,
                       P->tw0, P->tw1, P->lambda_max, done);
  } else {
    hipLaunchKernelGGL((k_apply_reg<false>), dim3(static_cast<unsigned>(grid)), dim3(kT), 0, s,
                       P->lpix, P->wq, P->wu, x, d, d_vec, y, ncol, ldx, ldy, P->chunks, P->spec_reg,
                       P->tw0, P->tw1, P->lambda_max, done);
  }
  MM_HIP_TRY(hipGetLastError());
  return MM_OK;
}

}  // namespace mm
