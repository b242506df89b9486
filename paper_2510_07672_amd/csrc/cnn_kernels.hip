// HIP kernels of the convolutional coarse propagator G (Section 3.2):
// 3x3 convolutions with circular padding, an activation after every
// convolution except the last, a global residual u + net(u), an optional
// uniform mass fix and an optional bound limiter.
//
// Layers 1 -> C -> ... -> C -> 1.  Activations are stored channels-last,
// act[field][y][x][c], so the C channels of a pixel are contiguous.
//   k_cnn_first   1 -> C on the vector ALU (K = 9), reading the FP64 state
//                 unrounded, FP32 arithmetic.
//   k_cnn_hidden  C -> C as an implicit GEMM on the matrix cores: M = output
//                 channels (16 per block of a 16x16x32 bf16 MFMA), N = output
//                 pixels (16 per block), K = 9 C ordered (tap, channel)
//                 and padded to a multiple of 32; FP32 accumulation.  A
//                 work-group stages a (TH+2) x (TW+2) input tile in LDS
//                 (8 x 32 or, at 32 and 48 channels, 16 x 16 outputs);
//                 the weights stay in registers.  With SPLIT the activation
//                 is carried as hi + lo bfloat16 and every product is done
//                 twice (hi W + lo W), which keeps ~16 mantissa bits.
//   k_cnn_first_ref, k_cnn_hidden_ref, k_cnn_last_ref  the layers on the
//                 vector ALU in FP32 or FP64 (the reference precisions).
//   k_cnn_last_mma  C -> 1 on the matrix cores with the nine taps as the N
//                 dimension, then a 3x3 gather of the per-tap products;
//                 plus the residual, written in FP64, with per-tile FP64
//                 sums of (G(u) - u).
//   Folded inference plan: k_cnn_hidden computes the first layer on its own
//                 input tile (FIRST) and, at C = 32 or 48, the last layer's
//                 per-tap products in its epilogue (TAIL);
//                 k_cnn_last_gather / k_cnn_last_gather_lin then sum the
//                 products over the taps (k_cnn_gather_correct also applies
//                 the Parareal correction).
//   k_cnn_fused   all layers of a call in one launch (16 x 16 output tiles,
//                 halos recomputed, activations in LDS).
//   k_cnn_fix     the uniform mass fix and the limiter.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <type_traits>
#include <utility>

#include "internal.h"
#include "gelu_coef.h"

namespace pr {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) __bf16 bf16x4;
typedef __attribute__((ext_vector_type(4))) float f32x4;

// GELU(x) = x/2 (1 + erf(x / sqrt 2)) in FP32 without branches.  With
// z = |x| / sqrt 2, erfc(z) takes the form t exp(-z^2 + Q(t)),
// t = 1 / (1 + 0.3 z); with h = x erfc(z) / 2 the result is x - h for x >= 0
// and h for x < 0, and h has the sign of x, so both cases are
// max(x, 0) - |x t| 2^(P(t) - z^2 log2(e)), one FMA, where P = log2(e) Q - 1
// is a degree-7 polynomial fitted to that exponent on z in [0, 6.5]
// (gelu_coef.h, written by gelu_fit.py; its error there is below 2.5e-7,
// a relative error of erfc below 1.7e-7).
// One reciprocal, one exp2 and 13 other instructions, where the library's
// erff evaluates two branches across a wave.  Relative error of the result
// in FP32 with a correctly rounded reciprocal and exp2: below 8e-7 for
// |x| < 2 (5.9e-7 on a dense grid), 1.5e-6 down to x = -5 and a few 1e-6 of
// a value that is already below 1e-5 of x beyond.
__device__ __forceinline__ float gelu_f32(float x) {
  constexpr double L = 1.44269504088896340736;  // log2(e)
  const float t = __builtin_amdgcn_rcpf(fmaf(fabsf(x), kGeluT, 1.0f));
  float p = kGeluP[0];
#pragma unroll
  for (int i = 1; i <= kGeluDeg; ++i) p = fmaf(p, t, kGeluP[i]);
  const float e = __builtin_amdgcn_exp2f(fmaf(x * (float)(-0.5 * L), x, p));
  // max(x, 0) as a signed-integer max of the bit pattern (one instruction:
  // negative values, -0 included, have the sign bit set)
  const float relu = __int_as_float(max(__float_as_int(x), 0));
  return fmaf(-fabsf(x * t), e, relu);
}

__device__ __forceinline__ float act_fn(float x, int act) {
  if (act == kActTanh) return tanhf(x);
  return gelu_f32(x);
}

// The activation chosen at compile time (TANH: tanh, else GELU), for loops
// that branch once on the activation instead of once per value.
template <bool TANH> __device__ __forceinline__ float act_sel(float x) {
  if constexpr (TANH) return tanhf(x);
  else return gelu_f32(x);
}

template <typename T> __device__ __forceinline__ float to_f(T v) { return (float)v; }

// activation in the reference precisions (float or double)
template <typename T>
__device__ __forceinline__ T act_ref(T x, int act) {
  if (act == kActTanh) return tanh(x);
  return (T)0.5 * x * ((T)1 + erf(x * (T)0.70710678118654752440));
}

// derivative of the activation at the pre-activation z
template <typename T>
__device__ __forceinline__ T act_grad(T z, int act) {
  if (act == kActTanh) {
    const T t = tanh(z);
    return (T)1 - t * t;
  }
  // d/dz z Phi(z) = Phi(z) + z phi(z)
  const T phi = exp((T)-0.5 * z * z) * (T)0.39894228040143267794;
  return (T)0.5 * ((T)1 + erf(z * (T)0.70710678118654752440)) + z * phi;
}

// store a value as hi (and, with lo != nullptr, the bfloat16 remainder)
template <typename T>
__device__ __forceinline__ void store_act(T* hi, T* lo, int64_t i, float v) {
  const T h = (T)v;
  hi[i] = h;
  if (lo) lo[i] = (T)(v - (float)h);
}

// ------------------------------------------------------------- weights

// torch Conv2d weights [Cout][Cin][3][3] -> bfloat16 [Cout][KP], k = tap Cin + ci,
// tap = 3 ky + kx, zero for k >= 9 Cin.
__global__ void k_cnn_pack(const float* __restrict__ W, int cin, int cout, int kp,
                           __bf16* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)cout * kp) return;
  const int co = (int)(i / kp), k = (int)(i % kp);
  float v = 0.f;
  if (k < 9 * cin) {
    const int tap = k / cin, ci = k % cin;
    v = W[((co * cin + ci) * 3 + tap / 3) * 3 + tap % 3];
  }
  out[i] = (__bf16)v;
}

// ------------------------------------------------------------ first layer

constexpr int kTile = 16;  // output tile side of the first and last layers

// Each thread produces 8 consecutive channels of one pixel (one 16-byte
// store in bfloat16), so consecutive threads write consecutive memory.
template <int C, typename TO>
__global__ __launch_bounds__(256) void k_cnn_first(const double* __restrict__ u_base,
                                                   const int64_t* __restrict__ u_offs, int n,
                                                   const float* __restrict__ W,
                                                   const float* __restrict__ b, int act,
                                                   TO* __restrict__ out, TO* __restrict__ out_lo,
                                                   float* __restrict__ zout) {
  static_assert(C % 8 == 0, "width must be a multiple of 8");
  __shared__ float sw[C * 9], sb[C];
  __shared__ float tile[(kTile + 2) * (kTile + 2)];
  const int tid = threadIdx.x;
  const int tpr = n / kTile, m = n - 1;
  const int64_t f = blockIdx.x / (tpr * tpr);
  const int t = (int)(blockIdx.x % (tpr * tpr));
  const int y0 = (t / tpr) * kTile, x0 = (t % tpr) * kTile;
  const double* u = u_base + (u_offs ? u_offs[f] : f * (int64_t)n * n);
  for (int i = tid; i < C * 9; i += 256) sw[i] = W[i];
  for (int i = tid; i < C; i += 256) sb[i] = b[i];
  for (int i = tid; i < (kTile + 2) * (kTile + 2); i += 256) {
    const int ty = i / (kTile + 2), tx = i % (kTile + 2);
    tile[i] = (float)u[(int64_t)((y0 + ty - 1) & m) * n + ((x0 + tx - 1) & m)];
  }
  __syncthreads();
  constexpr int C8 = C / 8;
  for (int item = tid; item < kTile * kTile * C8; item += 256) {
    const int c8 = item % C8, px = item / C8;
    const int py = px / kTile, pxx = px % kTile;
    float v[9];
#pragma unroll
    for (int tp = 0; tp < 9; ++tp) v[tp] = tile[(py + tp / 3) * (kTile + 2) + pxx + tp % 3];
    float r8[8], z8[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int co = c8 * 8 + j;
      float s = sb[co];
#pragma unroll
      for (int tp = 0; tp < 9; ++tp) s += sw[co * 9 + tp] * v[tp];
      z8[j] = s;
      r8[j] = act_fn(s, act);
    }
    const int64_t o = ((f * n + y0 + py) * (int64_t)n + x0 + pxx) * C + c8 * 8;
    if (zout) {
#pragma unroll
      for (int j = 0; j < 8; ++j) zout[o + j] = z8[j];
    }
    if constexpr (sizeof(TO) == 2) {
      bf16x8 h, l;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        h[j] = (__bf16)r8[j];
        l[j] = (__bf16)(r8[j] - (float)h[j]);
      }
      *(bf16x8*)&out[o] = h;
      if (out_lo) *(bf16x8*)&out_lo[o] = l;
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) out[o + j] = r8[j];
    }
  }
}

// ----------------------------------------------------------- hidden layers

// x / D for 0 <= x < LIMIT as (x M) >> S with one 24-bit multiply (full
// rate on the vector ALU, where a 32-bit division by a constant takes
// quarter-rate high-half multiplies).  M and S are fixed at compile time and
// the quotient is checked against x / D for every x below LIMIT.
constexpr bool div24_exact(int d, int limit, unsigned m, int s) {
  for (int x = 0; x < limit; ++x)
    if ((unsigned long long)x * m >= (1ull << 32) || (int)(((unsigned long long)x * m) >> s) != x / d)
      return false;
  return true;
}
template <int D, int LIMIT> struct Div24 {
  static constexpr int S = 20;
  static constexpr unsigned M = ((1u << S) + D - 1) / D;
  static_assert(LIMIT < (1 << 24) && M < (1u << 24) && div24_exact(D, LIMIT, M, S),
                "24-bit reciprocal division is not exact on this range");
  __device__ static int div(int x) { return (int)(__umul24((unsigned)x, M) >> S); }
};

template <int C, int NWAVES = 4, int TH_ = 8, int TW_ = 32> struct HidCfg {
  static constexpr int TH = TH_, TW = TW_;           // output tile (rows, columns)
  static constexpr int NW = NWAVES, NT = 64 * NW;    // waves, threads
  static constexpr int CS = C + 8;                   // LDS pixel stride (elements), one plane
  static constexpr int KP = (9 * C + 31) / 32 * 32;  // K padded to the MFMA depth
  static constexpr int MB = TH * TW / 16;            // 16-pixel blocks per tile
  static constexpr int MBW = MB / NW;                // per wave
  static constexpr int NB = C / 16;                  // 16-channel blocks
  static constexpr int KB = KP / 32;                 // K steps
  static constexpr int TPIX = (TH + 2) * (TW + 2);
  static constexpr int TCH = TPIX * (C / 8);         // 16-byte chunks of an input tile
};

// LDS layout of the hidden layer's input tile: pixel p at p * PS; with
// SPLIT a pixel holds its C hi values then its C lo values, with one
// 8-element pad after both.  The 16 lanes of a fragment read then stride
// an odd number of 16-byte bank quads, as one plane of stride C + 8 would,
// while the pair costs 8 pad elements per pixel instead of 16 (at C = 32
// that lets 3 work-groups share a CU instead of 2).
template <int C, bool SPLIT, int TH_ = 8, int TW_ = 32> struct HidTile {
  using HC = HidCfg<C, 4, TH_, TW_>;
  static constexpr int PS = SPLIT ? 2 * C + 8 : C + 8;
  static constexpr int LO = SPLIT ? C : 0;   // offset of the lo values
  static constexpr size_t BYTES = (size_t)HC::TPIX * PS * 2;
  // With the first layer computed in the same launch: after the tile, the
  // (TH+4) x (TW+4) patch of the state that the tile's first-layer outputs
  // read, then the first layer's C x 9 weights and C biases (FP32).
  static constexpr int UH = HC::TH + 4, UW = HC::TW + 4;
  static constexpr size_t FIRST_BYTES = BYTES + (size_t)(UH * UW + 10 * C) * 4;
  // At C = 48 the layer's biases (FP32) and, with TAIL, the last layer's
  // packed weight fragments (2 LKB bf16x8 per lane) follow, staged once
  // per work-group and read from LDS per 16-pixel block.
  static constexpr int LKB = (C + 31) / 32;
  static constexpr size_t STAGE_BYTES = C == 48 ? (size_t)C * 4 + (size_t)2 * LKB * 64 * 16 : 0;
  static_assert(BYTES % 16 == 0 && FIRST_BYTES % 16 == 0, "staged block alignment");
};

// Tuning knobs (compile time): whether the last layer folds into the last
// hidden layer at 48 channels, the waves per SIMD the 48-channel hidden
// layer's registers are bounded to, and whether the 48-channel layers other
// than the folded last one split their output channels over waves.
#ifndef PR_TAIL48
#define PR_TAIL48 1
#endif
#ifndef PR_HID48_NBW
#define PR_HID48_NBW 0
#endif
#ifndef PR_HID48_WAVES
#define PR_HID48_WAVES 2
#endif

template <int C> struct LastCfg {
  static constexpr int T = 16, WI = T + 2, PX = WI * WI;
  static constexpr int KB = (C + 31) / 32;   // 32-channel steps
};

// The last layer's K order.  In each 32-deep step kb of the C -> 1
// product, lane group g (lanes 16 g .. 16 g + 15) supplies K slots
// 8 g .. 8 g + 7; last_chan gives the channel in slot j of that group, or
// -1 for a zero slot.  At C = 48 group g holds channels 12 g .. 12 g + 11,
// the first eight in step 0 and the last four in step 1 (its slots 4..7
// zero): exactly the channels a TAIL hidden layer leaves in the lanes of
// group g.  Other widths take channels 32 kb + 8 g + j in order.
template <int C>
__device__ __forceinline__ int last_chan(int kb, int g, int j) {
  if constexpr (C == 48) return kb == 0 ? 12 * g + j : (j < 4 ? 12 * g + 8 + j : -1);
  const int c = kb * 32 + 8 * g + j;
  return c < C ? c : -1;
}

// The A fragment of step kb for lane group g: the channels last_chan
// names, of the pixel whose channels start at a (8-byte aligned).
template <int C>
__device__ __forceinline__ bf16x8 last_frag(const __bf16* a, int kb, int g) {
  if constexpr (C == 48) {
    const bf16x4 x0 = *(const bf16x4*)&a[kb == 0 ? 12 * g : 12 * g + 8];
    const bf16x4 x1 = kb == 0 ? *(const bf16x4*)&a[12 * g + 4] : bf16x4{};
    return __builtin_shufflevector(x0, x1, 0, 1, 2, 3, 4, 5, 6, 7);
  } else {
    const int c0 = kb * 32 + 8 * g;
    return c0 < C ? *(const bf16x8*)&a[c0] : bf16x8{};
  }
}

// Lane (g, r) holds W[c = last_chan(kb, g, j)][tap r], j < 8, as hi and lo
// (zero in zero slots or beyond nine taps).
template <int C>
__device__ __forceinline__ void last_weights(const float* __restrict__ W, int lane,
                                             bf16x8* hi, bf16x8* lo) {
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int kb = 0; kb < LastCfg<C>::KB; ++kb) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int c = last_chan<C>(kb, g, j);
      const float v = (c >= 0 && r < 9) ? W[c * 9 + r] : 0.f;
      const __bf16 h = (__bf16)v;
      hi[kb][j] = h;
      lo[kb][j] = (__bf16)(v - (float)h);
    }
  }
}

// The last layer's weights as the per-lane B fragments last_weights forms:
// out[(2 kb + h) 64 + lane] = (h ? lo : hi)[kb] of that lane.
template <int C>
__global__ void k_cnn_pack_last(const float* __restrict__ W, bf16x8* __restrict__ out) {
  const int lane = threadIdx.x;
  if (lane >= 64) return;
  bf16x8 hi[LastCfg<C>::KB], lo[LastCfg<C>::KB];
  last_weights<C>(W, lane, hi, lo);
#pragma unroll
  for (int kb = 0; kb < LastCfg<C>::KB; ++kb) {
    out[(2 * kb) * 64 + lane] = hi[kb];
    out[(2 * kb + 1) * 64 + lane] = lo[kb];
  }
}

// The first layer's inputs, for a hidden-layer launch that also computes it.
struct FirstIn {
  const double* u_base;   // field f at u_base + (u_offs ? u_offs[f] : f N^2)
  const int64_t* u_offs;
  const float* W;         // [C][9] FP32, torch order
  const float* b;         // [C]
};

// A hidden layer C -> C, persistent over (TH x TW) output tiles.
//
// With FIRST the layer's input tile is not read from HBM: the work-group
// computes it, the first layer 1 -> C on the (TH+2) x (TW+2) tile pixels
// from the FP64 state, with the arithmetic of k_cnn_first (the same FP32
// multiply-add chain, activation and hi / lo rounding), so the result is
// bitwise that of the two launches.  Inference only: the first layer's
// activations and pre-activations are not kept.
//
// With TAIL (C = 32 or 48) the layer's activations are not stored: the epilogue
// multiplies them at once by the last layer's weights, as k_cnn_last_mma
// does after reloading them, and stores the nine per-tap products
// Y[t][pixel] (tap planes of nfields N^2 floats) for k_cnn_last_gather.
// For that the weight rows are permuted so that lane group g receives
// output channels 8 g .. 8 g + 7 of its pixel: those registers are then
// the 16x16x32 A fragment that k_cnn_last_mma loads for the pixel, and the
// same three products in the same order give Y bit for bit.
// Output tile shapes of the hidden layers: 0 is 8 x 32 pixels, 1 is 16 x 16
// (fewer halo pixels per tile, 324 instead of 340 for 256 outputs; rows of
// one 16-pixel block).  The per-pixel arithmetic does not depend on the
// shape, so both give the same bits; pr_autotune_coarse times them at 32
// and 48 channels, the only widths built with both.
template <int SHAPE> constexpr int tile_h() { return SHAPE ? 16 : 8; }
template <int SHAPE> constexpr int tile_w() { return SHAPE ? 16 : 32; }
template <int C> constexpr bool both_tile_shapes() { return C == 32 || C == 48; }

// Whether a hidden layer splits its output channels over waves: wave w then
// computes output-channel block w % NB (16 channels) of pixel group w / NB
// and holds only that block's weight fragments (KB x 4 registers instead of
// KB x NB x 4), so more waves share a SIMD, while each input fragment is
// read from LDS by NB waves instead of one.  Six waves per work-group at
// 48 channels (2 pixel groups of 8 blocks), 3 waves per SIMD.  Not with
// TAIL, whose folded last layer needs all of a pixel's channels in one wave.
// Off: measured slower (6 x 48 split network on 16 fields of 512^2: 2.37 ->
// 2.95 ms per call), the tripled LDS reads of the input fragments costing
// more than the third wave per SIMD gains.
template <int C, bool TAIL> constexpr bool hidden_nbw() { return PR_HID48_NBW && C == 48 && !TAIL; }
template <int C, bool TAIL> constexpr int hidden_waves() { return hidden_nbw<C, TAIL>() ? 6 : 4; }

// Waves per SIMD the register allocator must leave room for: at 48
// channels 2 (3 with the channel blocks split over waves); at 32 channels 3,
// which the compiler would otherwise give up for a few registers in some
// variants, except the bf16 kernel with both the first and the last layer
// folded in, which would then spill.
template <int C, bool SPLIT, bool FIRST, bool TAIL> constexpr int hidden_min_waves() {
  if constexpr (C == 48) return hidden_nbw<C, TAIL>() ? 3 : PR_HID48_WAVES;
  if constexpr (C == 32) return (FIRST && TAIL && !SPLIT) ? 1 : 3;
  return 1;
}

template <int C, bool SPLIT, bool FIRST = false, bool TAIL = false, int SHAPE = 0>
__global__ __launch_bounds__((HidCfg<C, hidden_waves<C, TAIL>()>::NT)) __attribute__((amdgpu_waves_per_eu(hidden_min_waves<C, SPLIT, FIRST, TAIL>()))) void k_cnn_hidden(
    const __bf16* __restrict__ in, const __bf16* __restrict__ in_lo, int n, int64_t nfields,
    const __bf16* __restrict__ Wp, const float* __restrict__ b, int act,
    __bf16* __restrict__ out, __bf16* __restrict__ out_lo, float* __restrict__ zout,
    FirstIn fi, const float* __restrict__ WL, const bf16x8* __restrict__ WLp,
    float* __restrict__ Yp) {
  using H = HidCfg<C, hidden_waves<C, TAIL>(), tile_h<SHAPE>(), tile_w<SHAPE>()>;
  static_assert(C % 16 == 0, "hidden width must be a multiple of 16");
  constexpr bool kNBW = hidden_nbw<C, TAIL>();
  constexpr int NBL = kNBW ? 1 : H::NB;              // channel blocks per wave
  constexpr int PG = kNBW ? H::NW / H::NB : H::NW;   // pixel groups
  static_assert(!kNBW || PG * H::NB == H::NW, "waves must cover the channel blocks");
  constexpr int MBW = H::MB / PG;                    // 16-pixel blocks per wave and tile
  // blocks whose products one pass over K computes together: 4 with one
  // channel block per wave, so consecutive MFMAs do not depend on each other
  constexpr int NBLK = kNBW ? 4 : 1;
  static_assert(MBW % NBLK == 0, "blocks per wave");
  static_assert(!TAIL || C == 32 || C == 48,
                "the last layer folds into a hidden layer of 32 or 48 channels");
  extern __shared__ __align__(16) unsigned char smem[];
  using HT = HidTile<C, SPLIT, tile_h<SHAPE>(), tile_w<SHAPE>()>;
  __bf16* tile = (__bf16*)smem;                               // [TPIX][PS]
  __bf16* tile_lo = tile + HT::LO;                            // SPLIT only
  float* su = (float*)(smem + HT::BYTES);                     // FIRST: [UH][UW]
  float* sw0 = su + HT::UH * HT::UW;                          // FIRST: [C][9]
  float* sb0 = sw0 + 9 * C;                                   // FIRST: [C]
  // C = 48: biases [C], then (TAIL) the last layer's fragments [2 LKB][64]
  float* sbias = (float*)(smem + (FIRST ? HT::FIRST_BYTES : HT::BYTES));
  bf16x8* swl = (bf16x8*)(sbias + C);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int tpy = n / H::TH, tpx = n / H::TW;
  const int64_t tiles = nfields * tpy * tpx;
  const int wpg = kNBW ? wave / H::NB : wave;         // the wave's pixel group
  // channel block of the wave's j-th set of fragments
  auto nbof = [&](int j) { return kNBW ? wave % H::NB : j; };

  // this lane's weight fragments and biases, for the whole kernel; och is
  // the output channel of row m of channel block nb
  auto och = [](int nb, int m) { return TAIL ? (C / 4) * (m / 4) + 4 * nb + m % 4 : nb * 16 + m; };
  bf16x8 bfr[H::KB][NBL];
  // biases of channels och(nb, 4 g + i), consecutive in i: in registers for
  // the whole kernel, or at C = 48 read per 16-pixel block (16-byte loads),
  // which leaves the registers the folded last layer needs at 2 waves per SIMD
  constexpr bool kBiasRegs = C != 48;
  if constexpr (!kBiasRegs) {
    // read after the tile loop's first barrier
    for (int i = tid; i < C; i += H::NT) sbias[i] = b[i];
    if constexpr (TAIL)
      for (int i = tid; i < 2 * HT::LKB * 64; i += H::NT) swl[i] = WLp[i];
  }
  float bias[NBL][4];
#pragma unroll
  for (int j = 0; j < NBL; ++j) {
    const int nb = nbof(j);
    if constexpr (kBiasRegs) {
#pragma unroll
      for (int i = 0; i < 4; ++i) bias[j][i] = b[och(nb, 4 * g + i)];
    }
#pragma unroll
    for (int kb = 0; kb < H::KB; ++kb)
      bfr[kb][j] = *(const bf16x8*)&Wp[(int64_t)och(nb, r) * H::KP + kb * 32 + 8 * g];
  }
  constexpr int LKB = LastCfg<C>::KB;
  // TAIL: the last layer's weights, as in k_cnn_last_mma; held in registers
  // at C = 32, loaded per 16-pixel block (packed by k_cnn_pack_last) at
  // C = 48, where the registers would cost a wave per SIMD
  constexpr bool kTailRegs = C == 32;
  bf16x8 lwhi[LKB], lwlo[LKB];
  if constexpr (TAIL && kTailRegs) last_weights<C>(WL, lane, lwhi, lwlo);
  const int64_t yplane = nfields * (int64_t)n * n;

  if constexpr (FIRST) {
    for (int i = tid; i < 9 * C; i += H::NT) sw0[i] = fi.W[i];
    for (int i = tid; i < C; i += H::NT) sb0[i] = fi.b[i];
  }
  // tile tt's decomposition: field, top row, left column
  auto tile_at = [&](int64_t tt, int64_t& f_, int& y0_, int& x0_) {
    f_ = tt / (tpy * tpx);
    const int r_ = (int)(tt % (tpy * tpx));
    y0_ = (r_ / tpx) * H::TH;
    x0_ = (r_ % tpx) * H::TW;
  };
  // the input tile of tile tt straight from HBM into LDS at dst (16 bytes
  // per lane, no registers), every load of the tile in flight at once:
  // lane l of a wave's load at slot base s0 fills slot s0 + l, slot s being
  // the 16-byte chunk s % SP of tile pixel s / SP (SP = PS / 8 chunks per
  // pixel: C / 8 hi chunks, with SPLIT C / 8 lo chunks, then the pad, which
  // no lane loads).
  // Each step covers DP whole pixels (STEP = DP SP slots, at most NT): a
  // lane keeps its chunk j, so its plane (hi or lo) and source base, and
  // its pixel advances by DP, i.e. DP / RW rows and DP % RW columns with at
  // most one more wrap.  The lane's first pixel and chunk come from 24-bit
  // reciprocal multiplies once per tile, the byte offset within the field is
  // 32-bit (n a power of two up to 4096), and the slot base is scalar (it
  // sets the LDS address of the wave's load).  Lanes past STEP and pad
  // chunks load nothing.
  auto load_tile = [&](int64_t tt, __bf16* dst) {
    int64_t f_;
    int y0_, x0_;
    tile_at(tt, f_, y0_, x0_);
    constexpr int SP = HT::PS / 8, NSLOT = H::TPIX * SP, DATA = (SPLIT ? 2 : 1) * (C / 8);
    constexpr int RW = H::TW + 2, DP = H::NT / SP, STEP = DP * SP;
    using DivS = Div24<SP, H::NT>;
    using DivR = Div24<RW, H::NT / SP + 1>;
    const int w0 = __builtin_amdgcn_readfirstlane(wave) * 64;
    const int q = w0 + lane;  // the lane's slot within a step
    const int pp = DivS::div(q), j = q - __mul24(pp, SP);
    int ty = DivR::div(pp), tx = pp - __mul24(ty, RW);
    const bool lo = SPLIT && j >= C / 8;
    const unsigned c16 = (unsigned)((lo ? j - C / 8 : j) * 16);
    const char* base = (const char*)((lo ? in_lo : in) + f_ * (int64_t)n * n * C);
    const bool live = q < STEP && j < DATA;
    const int ym = y0_ - 1, xm = x0_ - 1, msk = n - 1, ln = __builtin_ctz(n);
    for (int s0 = 0; s0 < NSLOT; s0 += STEP) {
      if (live && q < NSLOT - s0) {
        const int gy = (ym + ty) & msk, gx = (xm + tx) & msk;
        // byte offset of the chunk within its field's plane (< 2^31)
        const unsigned off = __umul24((unsigned)((gy << ln) | gx), (unsigned)(2 * C)) + c16;
        __builtin_amdgcn_global_load_lds((const void*)(base + off),
                                         (__attribute__((address_space(3))) void*)(dst + (s0 + w0) * 8),
                                         16, 0, 0);
      }
      tx += DP % RW;
      ty += DP / RW;
      if (tx >= RW) {
        tx -= RW;
        ++ty;
      }
    }
  };
  // the products, activation and stores of tile t from the input tile tl
  auto compute_tile = [&](int64_t t, const __bf16* tl) {
    int64_t f;
    int y0, x0;
    tile_at(t, f, y0, x0);
    const __bf16* tin = tl;              // the input tile
    const __bf16* tin_lo = tl + HT::LO;  // its lo values (SPLIT)
    // the products of blocks m0 .. m0 + NBLK - 1; every accumulator takes
    // its hi then its lo product at each K step, in K order
    auto mma_blocks = [&](int m0, f32x4 (*acc)[NBL]) {
      int aoff[NBLK];
#pragma unroll
      for (int q = 0; q < NBLK; ++q) {
        const int mb = wpg * MBW + m0 + q;
        aoff[q] = ((mb / (H::TW / 16)) * (H::TW + 2) + (mb % (H::TW / 16)) * 16 + r) * HT::PS;
#pragma unroll
        for (int j = 0; j < NBL; ++j) acc[q][j] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
      for (int kb = 0; kb < H::KB; ++kb) {
        const int k0 = kb * 32 + 8 * g;
        const bool live = k0 < 9 * C;
        const int tap = live ? k0 / C : 0, ci0 = live ? k0 % C : 0;
        const int kofs = ((tap / 3) * (H::TW + 2) + tap % 3) * HT::PS + ci0;
        bf16x8 afr[NBLK], alo[NBLK];
#pragma unroll
        for (int q = 0; q < NBLK; ++q) {
          afr[q] = *(const bf16x8*)&tin[aoff[q] + kofs];
          if (!live) afr[q] = bf16x8{};
          if constexpr (SPLIT) {
            alo[q] = *(const bf16x8*)&tin_lo[aoff[q] + kofs];
            if (!live) alo[q] = bf16x8{};
          }
        }
#pragma unroll
        for (int q = 0; q < NBLK; ++q)
#pragma unroll
          for (int j = 0; j < NBL; ++j)
            acc[q][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[kb][j], afr[q], acc[q][j], 0, 0, 0);
        if constexpr (SPLIT) {
#pragma unroll
          for (int q = 0; q < NBLK; ++q)
#pragma unroll
            for (int j = 0; j < NBL; ++j)
              acc[q][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[kb][j], alo[q], acc[q][j], 0, 0, 0);
        }
      }
    };
    // lane (r, g) holds channels nb 16 + 4 g + i of pixel ox0 + r: bias,
    // activation and hi / lo rounding in registers, 8-byte stores (4
    // consecutive channels) straight to the channels-last output
    auto epilogue_act = [&](int m, const f32x4* acc, auto tanh_tag) {
      constexpr bool kTanh = decltype(tanh_tag)::value;
      const int mb = wpg * MBW + m;
      const int oy = mb / (H::TW / 16), ox0 = (mb % (H::TW / 16)) * 16;
      const int64_t pb = ((f * n + y0 + oy) * (int64_t)n + x0 + ox0 + r) * C + 4 * g;
      // TAIL: the lane's channels (C/4) g + q of pixel ox0 + r, q = 4 nb + i,
      // as the last layer's A fragments: slot j of step kb holds q = 8 kb + j.
      // Step kb's products are issued as soon as its fragment is complete,
      // so one fragment pair is live at a time; lane (g, r) receives
      // Y[pixel ox0 + 4 g + e][tap r]
      bf16x8 xh = bf16x8{}, xl = bf16x8{};
      f32x4 y = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int j = 0; j < NBL; ++j) {
        const int nb = nbof(j);
        float z[4];
        if constexpr (kBiasRegs) {
#pragma unroll
          for (int i = 0; i < 4; ++i) z[i] = acc[j][i] + bias[j][i];
        } else {
          const float4 bv = *(const float4*)&sbias[och(nb, 4 * g)];
          z[0] = acc[j][0] + bv.x;
          z[1] = acc[j][1] + bv.y;
          z[2] = acc[j][2] + bv.z;
          z[3] = acc[j][3] + bv.w;
        }
        if (zout) *(float4*)&zout[pb + nb * 16] = float4{z[0], z[1], z[2], z[3]};
        bf16x4 h, l;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float v = act_sel<kTanh>(z[i]);
          h[i] = (__bf16)v;
          l[i] = (__bf16)(v - (float)h[i]);
        }
        if constexpr (TAIL) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            xh[(4 * nb + i) % 8] = h[i];
            xl[(4 * nb + i) % 8] = l[i];
          }
          if ((4 * nb + 4) % 8 == 0 || nb == H::NB - 1) {
            const int kb = (4 * nb) / 8;
            bf16x8 wh, wl;
            if constexpr (kTailRegs) {
              wh = lwhi[kb];
              wl = lwlo[kb];
            } else {
              wh = swl[(2 * kb) * 64 + lane];
              wl = swl[(2 * kb + 1) * 64 + lane];
            }
            y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, wh, y, 0, 0, 0);
            y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, wl, y, 0, 0, 0);
            if constexpr (SPLIT) y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, wh, y, 0, 0, 0);
            xh = bf16x8{};
            xl = bf16x8{};
          }
        } else {
          *(bf16x4*)&out[pb + nb * 16] = h;
          if constexpr (SPLIT) *(bf16x4*)&out_lo[pb + nb * 16] = l;
        }
      }
      if constexpr (TAIL) {
        if (r < 9)
          *(f32x4*)&Yp[r * yplane + (f * n + y0 + oy) * (int64_t)n + x0 + ox0 + 4 * g] = y;
      }
    };
    auto epilogue = [&](int m, const f32x4* acc) {
      if (act == kActTanh) epilogue_act(m, acc, std::true_type{});
      else epilogue_act(m, acc, std::false_type{});
    };
    for (int m = 0; m < MBW; m += NBLK) {
      f32x4 acc[NBLK][NBL];
      mma_blocks(m, acc);
#pragma unroll
      for (int q = 0; q < NBLK; ++q) epilogue(m + q, acc[q]);
    }
  };
  // FIRST: the state patch su[sy][sx] = u[y0 + sy - 2][x0 + sx - 2]
  // (periodic) of tile tt, this thread's entries tid, tid + NT, .. into
  // registers; the next tile's patch is fetched before the current tile's
  // products, so that its loads are in flight during them (not where the
  // registers would cost a wave per SIMD: 32 channels with TAIL)
  constexpr bool kPrefetch = FIRST && !(C == 32 && TAIL);
  constexpr int kUp = FIRST ? (HT::UH * HT::UW + H::NT - 1) / H::NT : 1;
  double upatch[kUp];
  auto fetch_patch = [&](int64_t tt) {
    int64_t f_;
    int y0_, x0_;
    tile_at(tt, f_, y0_, x0_);
    const double* u = fi.u_base + (fi.u_offs ? fi.u_offs[f_] : f_ * (int64_t)n * n);
#pragma unroll
    for (int k = 0; k < kUp; ++k) {
      const int i = tid + k * H::NT;
      if (i < HT::UH * HT::UW) {
        const int sy = i / HT::UW, sx = i % HT::UW;
        upatch[k] = u[(int64_t)((y0_ + sy - 2) & (n - 1)) * n + ((x0_ + sx - 2) & (n - 1))];
      }
    }
  };
  if constexpr (kPrefetch) {
    if (blockIdx.x < tiles) fetch_patch(blockIdx.x);
  }
  for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    int64_t f;
    int y0, x0;
    tile_at(t, f, y0, x0);
    __syncthreads();  // the previous tile is no longer read
    if constexpr (FIRST) {
      if constexpr (kPrefetch) {
#pragma unroll
        for (int k = 0; k < kUp; ++k) {
          const int i = tid + k * H::NT;
          if (i < HT::UH * HT::UW) su[i] = (float)upatch[k];
        }
      } else {
        const double* u = fi.u_base + (fi.u_offs ? fi.u_offs[f] : f * (int64_t)n * n);
        for (int i = tid; i < HT::UH * HT::UW; i += H::NT) {
          const int sy = i / HT::UW, sx = i % HT::UW;
          su[i] = (float)u[(int64_t)((y0 + sy - 2) & (n - 1)) * n + ((x0 + sx - 2) & (n - 1))];
        }
      }
      __syncthreads();
      // tile pixel (ty, tx) is state point (y0 + ty - 1, x0 + tx - 1); its
      // tap tp reads su[ty + tp / 3][tx + tp % 3].  Item = 8 channels of
      // one pixel, as in k_cnn_first.
      auto first_tile = [&](auto tanh_tag) {
        constexpr bool kTanh = decltype(tanh_tag)::value;
        // item -> (pixel, channel group) and pixel -> (row, column) by
        // 24-bit reciprocal multiplies, as in load_tile
        using DivG = Div24<C / 8, H::TCH>;
        using DivR = Div24<H::TW + 2, H::TPIX>;
        for (int item = tid; item < H::TCH; item += H::NT) {
          const int px = DivG::div(item), c8 = item - __mul24(px, C / 8);
          const int ty = DivR::div(px), tx = px - __mul24(ty, H::TW + 2);
          const int ub = __mul24(ty, HT::UW) + tx;
          float v[9];
#pragma unroll
          for (int tp = 0; tp < 9; ++tp) v[tp] = su[ub + (tp / 3) * HT::UW + tp % 3];
          bf16x8 h, l;
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int co = c8 * 8 + j;
            float s = sb0[co];
#pragma unroll
            for (int tp = 0; tp < 9; ++tp) s += sw0[co * 9 + tp] * v[tp];
            const float r = act_sel<kTanh>(s);
            h[j] = (__bf16)r;
            l[j] = (__bf16)(r - (float)h[j]);
          }
          // LDS element of the item's 16-byte chunk: pixel px, channels 8 c8 ..
          const int li = __mul24(px, HT::PS) + c8 * 8;
          *(bf16x8*)&tile[li] = h;
          if constexpr (SPLIT) *(bf16x8*)&tile_lo[li] = l;
        }
      };
      if (act == kActTanh) first_tile(std::true_type{});
      else first_tile(std::false_type{});
    } else {
      load_tile(t, tile);
      __builtin_amdgcn_s_waitcnt(0);   // this wave's loads have landed in LDS
    }
    __syncthreads();
    if constexpr (kPrefetch) {
      if (t + gridDim.x < tiles) fetch_patch(t + gridDim.x);
    }
    compute_tile(t, tile);
  }
}

// ------------------------------------------------------ last layer on MFMA
//
// C -> 1 as a GEMM whose N dimension is the nine taps:
//   Y[q][t] = sum_c a[q][c] W[c][t]   on the (16 + 2)^2 input pixels q,
//   out[p] = b + sum_t Y[p + (t / 3, t % 3)][t],
// on the 16x16x32 bf16 MFMA (A = activations, B = weights in columns 0..8).
// The FP32 weights enter as bfloat16 hi + lo (16 significant bits); split
// activations add their lo part, so a term costs 2 or 3 products instead
// of 9 C vector FMAs per pixel.

// Y for the input region in LDS (pixel stride CS; lo plane at a + plane
// with SPLIT), then the sum over taps for output pixel tid (< 256),
// without the bias.  Four waves of 64 lanes.  Y is LDS scratch of PX * 9
// floats and may alias the region: the products stay in registers until
// every wave has read its operands.  The region must be complete on
// entry; the function synchronises between its phases.
template <int C, bool SPLIT, int CS>
__device__ __forceinline__ float last_layer_mfma(const __bf16* a, int plane, float* Y,
                                                 const bf16x8* whi, const bf16x8* wlo, int tid) {
  using L = LastCfg<C>;
  constexpr int NBLK = (L::PX + 15) / 16, NW = 4, PER = (NBLK + NW - 1) / NW;
  const int lane = tid & 63, wave = tid >> 6, r = lane & 15, g = lane >> 4;
  f32x4 acc[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int mb = wave + NW * i;
    if (mb < NBLK) {
      const int p = mb * 16 + r, pc = p < L::PX ? p : L::PX - 1;
#pragma unroll
      for (int kb = 0; kb < L::KB; ++kb) {
        const bf16x8 x = last_frag<C>(a + pc * CS, kb, g);
        acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, whi[kb], acc[i], 0, 0, 0);
        acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, wlo[kb], acc[i], 0, 0, 0);
        if constexpr (SPLIT) {
          const bf16x8 xl = last_frag<C>(a + plane + pc * CS, kb, g);
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, whi[kb], acc[i], 0, 0, 0);
        }
      }
    }
  }
  __syncthreads();
  // lane (g, r) holds Y for pixels 16 mb + 4 g + i, tap r
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int mb = wave + NW * i;
    if (mb < NBLK && r < 9) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int q = mb * 16 + 4 * g + e;
        if (q < L::PX) Y[q * 9 + r] = acc[i][e];
      }
    }
  }
  __syncthreads();
  const int py = tid / L::T, px = tid % L::T;
  float s = 0.f;
#pragma unroll
  for (int t = 0; t < 9; ++t) s += Y[((py + t / 3) * L::WI + px + t % 3) * 9 + t];
  return s;
}

template <int C, bool SPLIT>
__global__ __launch_bounds__(256) void k_cnn_last_mma(
    const __bf16* __restrict__ in, const __bf16* __restrict__ in_lo, int n,
    const float* __restrict__ W, const float* __restrict__ b, const double* __restrict__ u_base,
    const int64_t* __restrict__ u_offs, double* __restrict__ g_base,
    const int64_t* __restrict__ g_offs, int residual, double* __restrict__ partials) {
  using L = LastCfg<C>;
  constexpr int CS = C + 8, C8 = C / 8;
  constexpr size_t TB = (size_t)(SPLIT ? 2 : 1) * L::PX * CS * 2, YB = (size_t)L::PX * 9 * 4;
  __shared__ __align__(16) unsigned char lds[TB > YB ? TB : YB];   // tile, then Y
  __shared__ double red[4];
  __bf16* tile = (__bf16*)lds;
  const int tid = threadIdx.x;
  const int tpr = n / L::T, m = n - 1;
  const int64_t f = blockIdx.x / (tpr * tpr);
  const int t = (int)(blockIdx.x % (tpr * tpr));
  const int y0 = (t / tpr) * L::T, x0 = (t % tpr) * L::T;
  bf16x8 whi[L::KB], wlo[L::KB];
  last_weights<C>(W, tid & 63, whi, wlo);
  for (int i = tid; i < L::PX * C8; i += 256) {
    const int p = i / C8, c8 = i % C8;
    const int ty = p / L::WI, tx = p % L::WI;
    const int64_t gi = ((f * n + ((y0 + ty - 1) & m)) * (int64_t)n + ((x0 + tx - 1) & m)) * C + c8 * 8;
    *(bf16x8*)&tile[p * CS + c8 * 8] = *(const bf16x8*)&in[gi];
    if constexpr (SPLIT) *(bf16x8*)&tile[L::PX * CS + p * CS + c8 * 8] = *(const bf16x8*)&in_lo[gi];
  }
  __syncthreads();
  const float s = b[0] + last_layer_mfma<C, SPLIT, CS>(tile, L::PX * CS, (float*)lds, whi, wlo, tid);
  const int py = tid / L::T, px = tid % L::T;
  const int64_t gi = (int64_t)(y0 + py) * n + x0 + px;
  const double u = u_base[(u_offs ? u_offs[f] : f * (int64_t)n * n) + gi];
  const double out = residual ? u + (double)s : (double)s;
  g_base[(g_offs ? g_offs[f] : f * (int64_t)n * n) + gi] = out;
  if (partials) {
    double d = out - u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
    if ((tid & 63) == 0) red[tid >> 6] = d;
    __syncthreads();
    if (tid == 0) partials[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
  }
}

// The last layer from per-tap products that a TAIL hidden layer stored:
// out[p] = b + sum_t Y[t][p + (t / 3 - 1, t % 3 - 1)], then the residual
// and the per-tile mass partials, each as k_cnn_last_mma forms them (same
// 16 x 16 tiles, same order of sums), so the output is bitwise the same.
// With g2_base the output also goes to a second destination.
__global__ __launch_bounds__(256) void k_cnn_last_gather(
    const float* __restrict__ Yp, int n, int64_t nfields, const float* __restrict__ b,
    const double* __restrict__ u_base, const int64_t* __restrict__ u_offs,
    double* __restrict__ g_base, const int64_t* __restrict__ g_offs, int residual,
    double* __restrict__ partials, double* __restrict__ g2_base,
    const int64_t* __restrict__ g2_offs) {
  constexpr int T = 16;
  __shared__ double red[4];
  const int tid = threadIdx.x;
  const int tpr = n / T, m = n - 1;
  const int64_t f = blockIdx.x / (tpr * tpr);
  const int t = (int)(blockIdx.x % (tpr * tpr));
  const int y0 = (t / tpr) * T, x0 = (t % tpr) * T;
  const int py = tid / T, px = tid % T;
  const int64_t plane = nfields * (int64_t)n * n;
  const float* Yf = Yp + f * (int64_t)n * n;
  float sum = 0.f;
#pragma unroll
  for (int tp = 0; tp < 9; ++tp)
    sum += Yf[tp * plane + (int64_t)((y0 + py + tp / 3 - 1) & m) * n + ((x0 + px + tp % 3 - 1) & m)];
  const float s = b[0] + sum;
  const int64_t gi = (int64_t)(y0 + py) * n + x0 + px;
  const double u = u_base[(u_offs ? u_offs[f] : f * (int64_t)n * n) + gi];
  const double out = residual ? u + (double)s : (double)s;
  g_base[(g_offs ? g_offs[f] : f * (int64_t)n * n) + gi] = out;
  if (g2_base) g2_base[(g2_offs ? g2_offs[f] : f * (int64_t)n * n) + gi] = out;
  if (partials) {
    double d = out - u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
    if ((tid & 63) == 0) red[tid >> 6] = d;
    __syncthreads();
    if (tid == 0) partials[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
  }
}

// k_cnn_last_gather without the tile sums (no mass fix): points in the
// linear order of k_cnn_gather_correct, two per thread, so more blocks and
// fewer dependent loads per block; each point's sum is formed as there.
__global__ __launch_bounds__(256) void k_cnn_last_gather_lin(
    const float* __restrict__ Yp, int n, int64_t nfields, const float* __restrict__ b,
    const double* __restrict__ u_base, const int64_t* __restrict__ u_offs,
    double* __restrict__ g_base, const int64_t* __restrict__ g_offs, int residual,
    double* __restrict__ g2_base, const int64_t* __restrict__ g2_offs, int blocks_per_field) {
  constexpr int PPT = 2;
  const int64_t n2 = (int64_t)n * n;
  const int64_t fld = blockIdx.x / blocks_per_field;
  const int64_t part = blockIdx.x % blocks_per_field;
  const int m = n - 1;
  const int64_t plane = nfields * n2;
  const float* Yf = Yp + fld * n2;
  const double* u = u_base + (u_offs ? u_offs[fld] : fld * n2);
  double* g = g_base + (g_offs ? g_offs[fld] : fld * n2);
  double* g2 = g2_base ? g2_base + (g2_offs ? g2_offs[fld] : fld * n2) : nullptr;
  const int64_t i0 = part * (256 * PPT) + threadIdx.x;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int64_t i = i0 + k * 256;
    if (i < n2) {
      const int y = (int)(i / n), x = (int)(i % n);
      float sum = 0.f;
#pragma unroll
      for (int tp = 0; tp < 9; ++tp)
        sum += Yf[tp * plane + (int64_t)((y + tp / 3 - 1) & m) * n + ((x + tp % 3 - 1) & m)];
      const float s = b[0] + sum;
      const double v = u[i];
      const double out = residual ? v + (double)s : (double)s;
      g[i] = out;
      if (g2) g2[i] = out;
    }
  }
}

// The same sum over the taps with the Parareal correction of the sweep
// applied at once (no mass fix or limiter): g1 = G(u) as k_cnn_last_gather
// forms it, then u <- f + (g1 - g_old), g_old <- g1 and the running sup
// norm of the update, each as k_correct does them, so G(u) itself is not
// stored.  Two points per thread (points part 512 + k 256 + thread) and at
// most one atomic per block, skipped when the block's maximum is not above
// the value already stored: the norm only grows, so a skipped update could
// not have changed it (measured: 2 points per thread with the skip 6.76 ms
// per 64-slice sweep, 4 points 6.85, 4 points always updating 7.0).
template <typename TF>
__global__ __launch_bounds__(256) void k_cnn_gather_correct(
    const float* __restrict__ Yp, int n, int64_t nfields, const float* __restrict__ b,
    const double* __restrict__ in_base, const int64_t* __restrict__ in_offs, int residual,
    const TF* __restrict__ fb, const int64_t* __restrict__ f_offs,
    double* __restrict__ gob, const int64_t* __restrict__ go_offs,
    double* __restrict__ ub, const int64_t* __restrict__ u_offs,
    unsigned long long* __restrict__ upd, const int32_t* __restrict__ upd_idx, int update_cache,
    int blocks_per_field) {
  constexpr int PPT = 2;
  __shared__ unsigned long long red[4];
  const int64_t n2 = (int64_t)n * n;
  const int64_t fld = blockIdx.x / blocks_per_field;
  const int64_t part = blockIdx.x % blocks_per_field;
  const int m = n - 1;
  const int64_t plane = nfields * n2;
  const float* Yf = Yp + fld * n2;
  const double* uin = in_base + (in_offs ? in_offs[fld] : fld * n2);
  const TF* fp = fb + (f_offs ? f_offs[fld] : fld * n2);
  double* go = gob + (go_offs ? go_offs[fld] : fld * n2);
  double* u = ub + (u_offs ? u_offs[fld] : fld * n2);
  const int64_t i0 = part * (256 * PPT) + threadIdx.x;
  double g1[PPT], f[PPT], g0[PPT], u0[PPT];
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int64_t i = i0 + k * 256;
    if (i < n2) {
      const int y = (int)(i / n), x = (int)(i % n);
      float sum = 0.f;
#pragma unroll
      for (int tp = 0; tp < 9; ++tp)
        sum += Yf[tp * plane + (int64_t)((y + tp / 3 - 1) & m) * n + ((x + tp % 3 - 1) & m)];
      const float s = b[0] + sum;
      const double v = uin[i];
      g1[k] = residual ? v + (double)s : (double)s;
      f[k] = (double)fp[i];
      g0[k] = go[i];
      u0[k] = u[i];
    }
  }
  unsigned long long mx = 0;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int64_t i = i0 + k * 256;
    if (i < n2) {
      const double un = f[k] + (g1[k] - g0[k]);
      const double d = fabs(un - u0[k]);
      u[i] = un;
      if (update_cache) go[i] = g1[k];
      const unsigned long long bits = (unsigned long long)__double_as_longlong(d);
      mx = bits > mx ? bits : mx;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long t = __shfl_xor(mx, o, 64);
    mx = t > mx ? t : mx;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long r = red[0];
#pragma unroll
    for (int w = 1; w < 4; ++w) r = red[w] > r ? red[w] : r;
    unsigned long long* dst = &upd[upd_idx ? upd_idx[fld] : fld];
    if (r > __atomic_load_n(dst, __ATOMIC_RELAXED)) atomicMax(dst, r);
  }
}

// ---------------------------------------------------------- fused network
//
// Inference with every layer of a network with NH hidden layers in one
// persistent kernel.  A work-group takes a 16 x 16 output tile, loads the
// (16 + 2L)^2 region of u around it, and computes each layer on the region
// the layers after it need (the halo shrinks by one pixel per layer), with
// the activations in LDS as bfloat16 (hi and lo planes with SPLIT),
// channels last.  Hidden layers run on the 16x16x32 bf16 MFMA with the
// weights as the A operand, held in registers for the whole kernel, and
// the activations as the B operand: lane l then receives output channels
// 4 (l / 16) .. +3 of pixel l % 16, one 8-byte LDS store per 16 channels.
// HBM traffic is u in and G(u) out; the layer-by-layer path instead moves
// 2 C (L - 1) activation words per pixel.

template <int C, int NH, bool SPLIT> struct FusedCfg {
  static constexpr int T = 16, NW = 4, NT = 256;
  static constexpr int CS = C + 8;                   // LDS pixel stride (elements)
  static constexpr int KP = (9 * C + 31) / 32 * 32, KB = KP / 32, NB = C / 16;
  static constexpr int W0 = T + 2 * (NH + 1);       // first layer's output region side
  static constexpr int WU = W0 + 2;                 // region of u
  static constexpr int PLANE_A = W0 * W0 * CS;      // one plane of buffer A (layer 0, 2, ...)
  static constexpr int PLANE_B = (W0 - 2) * (W0 - 2) * CS;   // buffer B (layer 1, 3, ...)
  static constexpr int P = SPLIT ? 2 : 1;
  static constexpr size_t LDS = (size_t)P * (PLANE_A + PLANE_B) * 2 + (size_t)WU * WU * 4 +
                                (size_t)C * 10 * 4 + 4 * 8;
  // the last layer's scratch aliases its input region
  static_assert((size_t)(T + 2) * (T + 2) * 9 * 4 <= (size_t)(T + 2) * (T + 2) * CS * 2,
                "last-layer scratch exceeds its input region");
  static constexpr bool kFits = LDS <= 160 * 1024;
};

template <int C, int NH, bool SPLIT>
__global__ __launch_bounds__(256) void k_cnn_fused(
    const double* __restrict__ u_base, const int64_t* __restrict__ u_offs, int n, int64_t nfields,
    const float* __restrict__ W0g, const float* __restrict__ b0g, const __bf16* __restrict__ Wp,
    const float* __restrict__ bh, const float* __restrict__ WL, const float* __restrict__ bL,
    int act, int residual, double* __restrict__ g_base, const int64_t* __restrict__ g_offs,
    double* __restrict__ partials) {
  using F = FusedCfg<C, NH, SPLIT>;
  static_assert(C % 16 == 0, "hidden width must be a multiple of 16");
  extern __shared__ __align__(16) unsigned char smem[];
  __bf16* bufA = (__bf16*)smem;                          // [P][W0^2][CS]
  __bf16* bufB = bufA + F::P * F::PLANE_A;               // [P][(W0-2)^2][CS]
  double* red = (double*)(bufB + F::P * F::PLANE_B);     // [4]
  float* ut = (float*)(red + 4);                         // [WU][WU]
  float* sw0 = ut + F::WU * F::WU;                       // [C][9]
  float* sb0 = sw0 + C * 9;                              // [C]

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int tpr = n / F::T, m = n - 1;
  const int64_t tiles = nfields * tpr * tpr;

  bf16x8 wfr[NH][F::KB][F::NB];
  float bias[NH][F::NB][4];
#pragma unroll
  for (int h = 0; h < NH; ++h)
#pragma unroll
    for (int nb = 0; nb < F::NB; ++nb) {
#pragma unroll
      for (int i = 0; i < 4; ++i) bias[h][nb][i] = bh[h * C + nb * 16 + 4 * g + i];
#pragma unroll
      for (int kb = 0; kb < F::KB; ++kb)
        wfr[h][kb][nb] = *(const bf16x8*)&Wp[((int64_t)h * C + nb * 16 + r) * F::KP + kb * 32 + 8 * g];
    }
  for (int i = tid; i < C * 9; i += F::NT) sw0[i] = W0g[i];
  for (int i = tid; i < C; i += F::NT) sb0[i] = b0g[i];
  bf16x8 wlh[LastCfg<C>::KB], wll[LastCfg<C>::KB];
  last_weights<C>(WL, lane, wlh, wll);

  for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    const int64_t f = t / (tpr * tpr);
    const int tt = (int)(t % (tpr * tpr));
    const int y0 = (tt / tpr) * F::T, x0 = (tt % tpr) * F::T;
    const double* u = u_base + (u_offs ? u_offs[f] : f * (int64_t)n * n);
    __syncthreads();  // the previous tile is no longer read
    constexpr int HU = NH + 2;
    for (int i = tid; i < F::WU * F::WU; i += F::NT) {
      const int ty = i / F::WU, tx = i % F::WU;
      ut[i] = (float)u[(int64_t)((y0 + ty - HU) & m) * n + ((x0 + tx - HU) & m)];
    }
    __syncthreads();
    // layer 0: 1 -> C on the W0 x W0 region, 8 channels per item
    {
      constexpr int C8 = C / 8, ITEMS = F::W0 * F::W0 * C8;
      for (int item = tid; item < ITEMS; item += F::NT) {
        const int c8 = item % C8, p = item / C8;
        const int py = p / F::W0, px = p % F::W0;
        float v[9];
#pragma unroll
        for (int tp = 0; tp < 9; ++tp) v[tp] = ut[(py + tp / 3) * F::WU + px + tp % 3];
        bf16x8 hv, lv;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int co = c8 * 8 + j;
          float s = sb0[co];
#pragma unroll
          for (int tp = 0; tp < 9; ++tp) s += sw0[co * 9 + tp] * v[tp];
          const float a = act_fn(s, act);
          hv[j] = (__bf16)a;
          lv[j] = (__bf16)(a - (float)hv[j]);
        }
        *(bf16x8*)&bufA[p * F::CS + c8 * 8] = hv;
        if constexpr (SPLIT) *(bf16x8*)&bufA[F::PLANE_A + p * F::CS + c8 * 8] = lv;
      }
    }
    __syncthreads();
    // hidden layers: layer h reads A (h even) or B and writes the other
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const __bf16* in = (h & 1) ? bufB : bufA;
      __bf16* out = (h & 1) ? bufA : bufB;
      const int in_plane = (h & 1) ? F::PLANE_B : F::PLANE_A;
      const int out_plane = (h & 1) ? F::PLANE_A : F::PLANE_B;
      const int Wi = F::W0 - 2 * h, Wo = Wi - 2, npx = Wo * Wo, nblk = (npx + 15) / 16;
      for (int mb = wave; mb < nblk; mb += F::NW) {
        const int p = mb * 16 + r, pc = p < npx ? p : npx - 1;
        const int py = pc / Wo, px = pc % Wo;
        f32x4 acc[F::NB];
#pragma unroll
        for (int nb = 0; nb < F::NB; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < F::KB; ++kb) {
          const int k0 = kb * 32 + 8 * g;
          const bool live = k0 < 9 * C;
          const int tap = live ? k0 / C : 0, ci0 = live ? k0 % C : 0;
          const int a = ((py + tap / 3) * Wi + px + tap % 3) * F::CS + ci0;
          bf16x8 b = *(const bf16x8*)&in[a];
          if (!live) b = bf16x8{};
#pragma unroll
          for (int nb = 0; nb < F::NB; ++nb)
            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wfr[h][kb][nb], b, acc[nb], 0, 0, 0);
          if constexpr (SPLIT) {
            bf16x8 bl = *(const bf16x8*)&in[in_plane + a];
            if (!live) bl = bf16x8{};
#pragma unroll
            for (int nb = 0; nb < F::NB; ++nb)
              acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wfr[h][kb][nb], bl, acc[nb], 0, 0, 0);
          }
        }
        if (p < npx) {
#pragma unroll
          for (int nb = 0; nb < F::NB; ++nb) {
            typedef __attribute__((ext_vector_type(4))) __bf16 bf16x4;
            bf16x4 hv, lv;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const float v = act_fn(acc[nb][i] + bias[h][nb][i], act);
              hv[i] = (__bf16)v;
              lv[i] = (__bf16)(v - (float)hv[i]);
            }
            const int o = p * F::CS + nb * 16 + 4 * g;
            *(bf16x4*)&out[o] = hv;
            if constexpr (SPLIT) *(bf16x4*)&out[out_plane + o] = lv;
          }
        }
      }
      __syncthreads();
    }
    // last layer: C -> 1 on the tile (MFMA over the taps), residual and
    // mass partials in FP64
    {
      __bf16* in = (NH & 1) ? bufB : bufA;
      const int plane = (NH & 1) ? F::PLANE_B : F::PLANE_A;
      const int py = tid / F::T, px = tid % F::T;
      const float s = bL[0] + last_layer_mfma<C, SPLIT, F::CS>(in, plane, (float*)in, wlh, wll, tid);
      const int64_t gi = (int64_t)(y0 + py) * n + x0 + px;
      const double uc = u[gi];
      const double o = residual ? uc + (double)s : (double)s;
      g_base[(g_offs ? g_offs[f] : f * (int64_t)n * n) + gi] = o;
      if (partials) {
        double d = o - uc;
#pragma unroll
        for (int sh = 32; sh > 0; sh >>= 1) d += __shfl_xor(d, sh, 64);
        if (lane == 0) red[wave] = d;
        __syncthreads();
        if (tid == 0) partials[t] = ((red[0] + red[1]) + red[2]) + red[3];
      }
    }
  }
}

// ------------------------------------------- reference-precision layers
//
// FP32 or FP64 throughout, on the vector ALU, with weights in the same
// precision; optionally storing the pre-activations z for a backward pass.

template <int C, typename T>
__global__ __launch_bounds__(256) void k_cnn_first_ref(const double* __restrict__ u_base,
                                                       const int64_t* __restrict__ u_offs, int n,
                                                       const T* __restrict__ W,
                                                       const T* __restrict__ b, int act,
                                                       T* __restrict__ out, T* __restrict__ zout) {
  __shared__ T tile[(kTile + 2) * (kTile + 2)];
  const int tid = threadIdx.x;
  const int tpr = n / kTile, m = n - 1;
  const int64_t f = blockIdx.x / (tpr * tpr);
  const int t = (int)(blockIdx.x % (tpr * tpr));
  const int y0 = (t / tpr) * kTile, x0 = (t % tpr) * kTile;
  const double* u = u_base + (u_offs ? u_offs[f] : f * (int64_t)n * n);
  for (int i = tid; i < (kTile + 2) * (kTile + 2); i += 256) {
    const int ty = i / (kTile + 2), tx = i % (kTile + 2);
    tile[i] = (T)u[(int64_t)((y0 + ty - 1) & m) * n + ((x0 + tx - 1) & m)];
  }
  __syncthreads();
  const int py = tid / kTile, px = tid % kTile;
  T v[9];
#pragma unroll
  for (int tp = 0; tp < 9; ++tp) v[tp] = tile[(py + tp / 3) * (kTile + 2) + px + tp % 3];
  const int64_t o = ((f * n + y0 + py) * (int64_t)n + x0 + px) * C;
  for (int co = 0; co < C; ++co) {
    T s = b[co];
#pragma unroll
    for (int tp = 0; tp < 9; ++tp) s += W[co * 9 + tp] * v[tp];
    if (zout) zout[o + co] = s;
    out[o + co] = act_ref<T>(s, act);
  }
}

template <int C, typename T>
__global__ __launch_bounds__(256) void k_cnn_hidden_ref(const T* __restrict__ in, int n,
                                                        const T* __restrict__ W,
                                                        const T* __restrict__ b, int act,
                                                        T* __restrict__ out, T* __restrict__ zout) {
  __shared__ T tile[(kTile + 2) * (kTile + 2) * (C + 1)];
  const int tid = threadIdx.x;
  const int tpr = n / kTile, m = n - 1;
  const int64_t f = blockIdx.x / (tpr * tpr);
  const int t = (int)(blockIdx.x % (tpr * tpr));
  const int y0 = (t / tpr) * kTile, x0 = (t % tpr) * kTile;
  for (int i = tid; i < (kTile + 2) * (kTile + 2) * C; i += 256) {
    const int p = i / C, c = i % C;
    const int ty = p / (kTile + 2), tx = p % (kTile + 2);
    tile[p * (C + 1) + c] =
        in[((f * n + ((y0 + ty - 1) & m)) * (int64_t)n + ((x0 + tx - 1) & m)) * C + c];
  }
  __syncthreads();
  const int py = tid / kTile, px = tid % kTile;
  T acc[C];
#pragma unroll
  for (int co = 0; co < C; ++co) acc[co] = b[co];
  for (int tp = 0; tp < 9; ++tp) {
    const int p = (py + tp / 3) * (kTile + 2) + px + tp % 3;
    for (int ci = 0; ci < C; ++ci) {
      const T x = tile[p * (C + 1) + ci];
#pragma unroll
      for (int co = 0; co < C; ++co) acc[co] += W[(co * C + ci) * 9 + tp] * x;
    }
  }
  const int64_t o = ((f * n + y0 + py) * (int64_t)n + x0 + px) * C;
#pragma unroll
  for (int co = 0; co < C; ++co) {
    if (zout) zout[o + co] = acc[co];
    out[o + co] = act_ref<T>(acc[co], act);
  }
}

template <int C, typename T>
__global__ __launch_bounds__(256) void k_cnn_last_ref(
    const T* __restrict__ in, int n, const T* __restrict__ W, const T* __restrict__ b,
    const double* __restrict__ u_base, const int64_t* __restrict__ u_offs,
    double* __restrict__ g_base, const int64_t* __restrict__ g_offs, int residual,
    double* __restrict__ partials) {
  __shared__ T tile[(kTile + 2) * (kTile + 2) * (C + 1)];
  __shared__ double red[4];
  const int tid = threadIdx.x;
  const int tpr = n / kTile, m = n - 1;
  const int64_t f = blockIdx.x / (tpr * tpr);
  const int t = (int)(blockIdx.x % (tpr * tpr));
  const int y0 = (t / tpr) * kTile, x0 = (t % tpr) * kTile;
  for (int i = tid; i < (kTile + 2) * (kTile + 2) * C; i += 256) {
    const int p = i / C, c = i % C;
    const int ty = p / (kTile + 2), tx = p % (kTile + 2);
    tile[p * (C + 1) + c] =
        in[((f * n + ((y0 + ty - 1) & m)) * (int64_t)n + ((x0 + tx - 1) & m)) * C + c];
  }
  __syncthreads();
  const int py = tid / kTile, px = tid % kTile;
  T s = b[0];
  for (int tp = 0; tp < 9; ++tp) {
    const int p = (py + tp / 3) * (kTile + 2) + px + tp % 3;
#pragma unroll 8
    for (int ci = 0; ci < C; ++ci) s += W[ci * 9 + tp] * tile[p * (C + 1) + ci];
  }
  const int64_t gi = (int64_t)(y0 + py) * n + x0 + px;
  const double u = u_base[(u_offs ? u_offs[f] : f * (int64_t)n * n) + gi];
  const double out = residual ? u + (double)s : (double)s;
  g_base[(g_offs ? g_offs[f] : f * (int64_t)n * n) + gi] = out;
  if (partials) {
    double d = out - u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
    if ((tid & 63) == 0) red[tid >> 6] = d;
    __syncthreads();
    if (tid == 0) partials[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
  }
}

// uniform mass fix (G(u) - mean(G(u) - u)) and bound limiter
__global__ __launch_bounds__(256) void k_cnn_fix(double* __restrict__ g_base,
                                                 const int64_t* __restrict__ g_offs, int n,
                                                 const double* __restrict__ partials, int tiles,
                                                 int mass_fix, int limiter, double lo, double hi,
                                                 int blocks_per_field) {
  __shared__ double corr_sh;
  const int64_t f = blockIdx.x / blocks_per_field;
  const int part = blockIdx.x % blocks_per_field;
  if (threadIdx.x == 0) {
    double s = 0.0;
    if (mass_fix)
      for (int i = 0; i < tiles; ++i) s += partials[f * tiles + i];
    corr_sh = s / ((double)n * (double)n);
  }
  __syncthreads();
  const double corr = corr_sh;
  double* g = g_base + (g_offs ? g_offs[f] : f * (int64_t)n * n);
  const int64_t n2 = (int64_t)n * n;
  for (int64_t i = (int64_t)part * blockDim.x + threadIdx.x; i < n2;
       i += (int64_t)blocks_per_field * blockDim.x) {
    double v = g[i] - corr;
    if (limiter) v = v < lo ? lo : (v > hi ? hi : v);
    g[i] = v;
  }
}

// --------------------------------------------------------------- backward
//
// For a convolution layer Y = conv(X, W) + b (3x3, circular, cross-
// correlation), given dY:
//   dX[q][ci] = sum_{co, ky, kx} W[co][ci][ky][kx] dY[q - (ky - 1, kx - 1)][co]
//   dW[co][ci][ky][kx] = sum_p dY[p][co] X[p + (ky - 1, kx - 1)][ci]
//   db[co] = sum_p dY[p][co]
// Weight and bias gradients are summed per 16 x 16 tile into FP64 partials
// and then over tiles in a fixed order, so results are deterministic.

// Wt[tap][co][ci] = W[co][ci][tap]: the data gradient's weights, laid out so
// that one (tap, co) step reads CI consecutive values.
template <int CI, int CO, typename TW>
__global__ void k_w_transpose(const TW* __restrict__ W, TW* __restrict__ Wt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= CO * CI * 9) return;
  const int tp = i % 9, ci = (i / 9) % CI, co = i / (9 * CI);
  Wt[(tp * CO + co) * CI + ci] = W[i];
}

template <int CI, int CO, typename T, typename TW>
__global__ __launch_bounds__(256) void k_conv_bwd_data(const T* __restrict__ dY, int n,
                                                       const TW* __restrict__ Wt,
                                                       T* __restrict__ dX) {
  __shared__ T tile[(kTile + 2) * (kTile + 2) * (CO + 1)];
  const int tid = threadIdx.x;
  const int tpr = n / kTile, m = n - 1;
  const int64_t f = blockIdx.x / (tpr * tpr);
  const int t = (int)(blockIdx.x % (tpr * tpr));
  const int y0 = (t / tpr) * kTile, x0 = (t % tpr) * kTile;
  for (int i = tid; i < (kTile + 2) * (kTile + 2) * CO; i += 256) {
    const int p = i / CO, c = i % CO;
    const int ty = p / (kTile + 2), tx = p % (kTile + 2);
    tile[p * (CO + 1) + c] =
        dY[((f * n + ((y0 + ty - 1) & m)) * (int64_t)n + ((x0 + tx - 1) & m)) * CO + c];
  }
  __syncthreads();
  const int py = tid / kTile, px = tid % kTile;
  T acc[CI];
#pragma unroll
  for (int ci = 0; ci < CI; ++ci) acc[ci] = (T)0;
  for (int tp = 0; tp < 9; ++tp) {
    const int ky = tp / 3, kx = tp % 3;
    // dY at q - (ky - 1, kx - 1): tile coordinates (py + 2 - ky, px + 2 - kx)
    const int p = (py + 2 - ky) * (kTile + 2) + px + 2 - kx;
    // unrolled by 4 so that the next channels' LDS value and scalar weight
    // loads are in flight during the current channel's products (each
    // accumulator still sums in (tp, co) order: the same bits; 32 -> 32 at
    // 32 fields of 256^2 with the weight pass below: pr_cnn_backward 7.5 ->
    // 6.2 ms)
#pragma unroll 4
    for (int co = 0; co < CO; ++co) {
      const T d = tile[p * (CO + 1) + co];
      const TW* w = Wt + (tp * CO + co) * CI;  // contiguous in ci: wide scalar loads
#pragma unroll
      for (int ci = 0; ci < CI; ++ci) acc[ci] += (T)w[ci] * d;
    }
  }
  const int64_t o = ((f * n + y0 + py) * (int64_t)n + x0 + px) * CI;
#pragma unroll
  for (int ci = 0; ci < CI; ++ci) dX[o + ci] = acc[ci];
}

// partial[block][q]: q < CO CI 9 weight entries ([co][ci][ky][kx]), then CO biases
template <int CI, int CO, typename T, typename TX>
__global__ __launch_bounds__(256) void k_conv_bwd_weight(const T* __restrict__ dY,
                                                         const TX* __restrict__ X,
                                                         const TX* __restrict__ X_lo, int n,
                                                         double* __restrict__ partial) {
  constexpr int NP = CO * CI * 9 + CO;
  __shared__ T xt[(kTile + 2) * (kTile + 2) * (CI + 1)];
  __shared__ T yt[kTile * kTile * (CO + 1)];
  const int tid = threadIdx.x;
  const int tpr = n / kTile, m = n - 1;
  const int64_t f = blockIdx.x / (tpr * tpr);
  const int t = (int)(blockIdx.x % (tpr * tpr));
  const int y0 = (t / tpr) * kTile, x0 = (t % tpr) * kTile;
  for (int i = tid; i < (kTile + 2) * (kTile + 2) * CI; i += 256) {
    const int p = i / CI, c = i % CI;
    const int ty = p / (kTile + 2), tx = p % (kTile + 2);
    const int64_t gi = ((f * n + ((y0 + ty - 1) & m)) * (int64_t)n + ((x0 + tx - 1) & m)) * CI + c;
    T v = (T)(float)0;
    v = (T)X[gi];
    if (X_lo) v += (T)X_lo[gi];
    xt[p * (CI + 1) + c] = v;
  }
  for (int i = tid; i < kTile * kTile * CO; i += 256) {
    const int p = i / CO, c = i % CO;
    yt[p * (CO + 1) + c] = dY[((f * n + y0 + p / kTile) * (int64_t)n + x0 + p % kTile) * CO + c];
  }
  __syncthreads();
  for (int q = tid; q < NP; q += 256) {
    double s = 0.0;
    if (q < CO * CI * 9) {
      const int co = q / (CI * 9), ci = (q / 9) % CI, tp = q % 9;
      const int ky = tp / 3, kx = tp % 3;
      // 8 pixels in flight; the sum still runs in pixel order (the same
      // bits; pr_cnn_backward at 32 fields of 256^2: 6.5 -> 6.2 ms)
#pragma unroll 8
      for (int p = 0; p < kTile * kTile; ++p) {
        const int py = p / kTile, px = p % kTile;
        s += (double)(yt[p * (CO + 1) + co] * xt[((py + ky) * (kTile + 2) + px + kx) * (CI + 1) + ci]);
      }
    } else {
      const int co = q - CO * CI * 9;
      for (int p = 0; p < kTile * kTile; ++p) s += (double)yt[p * (CO + 1) + co];
    }
    partial[(int64_t)blockIdx.x * NP + q] = s;
  }
}

// Byte offset of the bias sums in k_conv_bwd_weight_rb's partials, after
// the weight sums of all blocks (256-byte aligned).
__host__ __device__ constexpr size_t rb_bias_offset(int64_t blocks, int nw, size_t elem) {
  return ((size_t)blocks * nw * elem + 255) / 256 * 256;
}

// The same partial sums for wide layers (CI, CO >= 32), register-blocked:
// a task is 4 output channels x 9 taps of one input channel, so that per
// pixel a thread reads 4 values of dY and 9 of X for 36 products (instead
// of 2 reads per product).  Each task accumulates its tile's 256 pixels in
// T, in pixel order, and stores the sums as doubles; biases as above.
template <int CI, int CO, typename T, typename TX>
__global__ __launch_bounds__(256) void k_conv_bwd_weight_rb(const T* __restrict__ dY,
                                                            const TX* __restrict__ X,
                                                            const TX* __restrict__ X_lo, int n,
                                                            void* __restrict__ partial) {
  static_assert(CO % 4 == 0, "output channels in blocks of 4");
  constexpr int NW = CO * CI * 9, TASKS = (CO / 4) * CI;
  // Unpadded tiles: in the product loop every lane of a wave reads the same
  // pixel (its lanes differ in channels only), so there are no bank
  // conflicts to avoid, and dY's 4 channels come in one 16-byte read
  // (pr_cnn_backward at 32 fields of 256^2: 6.21 -> 6.10 ms, same bits).
  constexpr int XS = CI, YS = CO;
  typedef T T4 __attribute__((ext_vector_type(4)));
  __shared__ __align__(32) T xt[(kTile + 2) * (kTile + 2) * XS];
  __shared__ __align__(32) T yt[kTile * kTile * YS];
  const int tid = threadIdx.x;
  const int tpr = n / kTile, m = n - 1;
  const int64_t f = blockIdx.x / (tpr * tpr);
  const int t = (int)(blockIdx.x % (tpr * tpr));
  const int y0 = (t / tpr) * kTile, x0 = (t % tpr) * kTile;
  for (int i = tid; i < (kTile + 2) * (kTile + 2) * CI; i += 256) {
    const int p = i / CI, c = i % CI;
    const int ty = p / (kTile + 2), tx = p % (kTile + 2);
    const int64_t gi = ((f * n + ((y0 + ty - 1) & m)) * (int64_t)n + ((x0 + tx - 1) & m)) * CI + c;
    T v = (T)X[gi];
    if (X_lo) v += (T)X_lo[gi];
    xt[p * XS + c] = v;
  }
  for (int i = tid; i < kTile * kTile * CO; i += 256) {
    const int p = i / CO, c = i % CO;
    yt[p * YS + c] = dY[((f * n + y0 + p / kTile) * (int64_t)n + x0 + p % kTile) * CO + c];
  }
  __syncthreads();
  // the weight sums in T (the accumulators' own type, widened only when
  // reduced), the bias sums in FP64 after them
  T* out = (T*)partial + (int64_t)blockIdx.x * NW;
  double* outb = (double*)((char*)partial + rb_bias_offset(gridDim.x, NW, sizeof(T))) +
                 (int64_t)blockIdx.x * CO;
  for (int task = tid; task < TASKS; task += 256) {
    const int co0 = (task % (CO / 4)) * 4, ci = task / (CO / 4);
    T acc[4][9];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int tp = 0; tp < 9; ++tp) acc[k][tp] = (T)0;
    // 8 pixels in flight per thread (each accumulator still sums its 256
    // pixels in order: the same bits as unroll 2, 3% faster)
#pragma unroll 8
    for (int p = 0; p < kTile * kTile; ++p) {
      const int py = p / kTile, px = p % kTile;
      T y[4];
      const T4 yv = *(const T4*)&yt[p * YS + co0];
#pragma unroll
      for (int k = 0; k < 4; ++k) y[k] = yv[k];
#pragma unroll
      for (int tp = 0; tp < 9; ++tp) {
        const T x = xt[((py + tp / 3) * (kTile + 2) + px + tp % 3) * XS + ci];
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k][tp] += y[k] * x;
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int tp = 0; tp < 9; ++tp) out[((co0 + k) * CI + ci) * 9 + tp] = acc[k][tp];
  }
  for (int co = tid; co < CO; co += 256) {
    double s = 0.0;
    for (int p = 0; p < kTile * kTile; ++p) s += (double)yt[p * YS + co];
    outb[co] = s;
  }
}

// First stage of the deterministic weight-gradient reduction: group g
// (blockIdx.y) sums rows [g per, (g + 1) per) of partial, in row order, into
// part2[g][q].  Many groups keep the whole GPU reading the partial sums.
// Entries q < nw of block b at wp[b nw + q] (PW, widened exactly to
// double), the others at bp[b (np - nw) + q - nw]; nw = np for one array.
template <typename PW>
__global__ void k_reduce_groups(const PW* __restrict__ wp, const double* __restrict__ bp,
                                int64_t blocks, int nw, int np, int64_t per,
                                double* __restrict__ part2) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= np) return;
  const int64_t b0 = (int64_t)blockIdx.y * per;
  const int64_t b1 = b0 + per < blocks ? b0 + per : blocks;
  // unrolled so that several blocks' loads are in flight; the sum still
  // runs in block order
  double s = 0.0;
  if (q < nw) {
#pragma unroll 8
    for (int64_t b = b0; b < b1; ++b) s += (double)wp[b * nw + q];
  } else {
#pragma unroll 8
    for (int64_t b = b0; b < b1; ++b) s += bp[b * (np - nw) + q - nw];
  }
  part2[(int64_t)blockIdx.y * np + q] = s;
}

// out[q] = sum over blocks of partial[block][q], in block order
template <typename T>
__global__ void k_reduce_partials(const double* __restrict__ partial, int64_t blocks, int np,
                                  T* __restrict__ out_w, int nw, T* __restrict__ out_b) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= np) return;
  double s = 0.0;
#pragma unroll 8
  for (int64_t b = 0; b < blocks; ++b) s += partial[b * np + q];
  if (q < nw) out_w[q] = (T)s;
  else out_b[q - nw] = (T)s;
}

// dZ = dA * act'(z), in place on dA; four consecutive elements per thread
// (count is a multiple of 4: channels come in multiples of 8), so each
// lane moves 16-byte or wider words
template <typename T, typename TZ>
__global__ __launch_bounds__(256) void k_act_bwd(T* __restrict__ dA, const TZ* __restrict__ z,
                                                 int64_t count, int act) {
  typedef T T4 __attribute__((ext_vector_type(4)));
  typedef TZ Z4 __attribute__((ext_vector_type(4)));
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (i >= count) return;
  T4 d = *(const T4*)&dA[i];
  const Z4 zz = *(const Z4*)&z[i];
#pragma unroll
  for (int k = 0; k < 4; ++k) d[k] = d[k] * (T)act_grad<T>((T)zz[k], act);
  *(T4*)&dA[i] = d;
}

// Backward of the output stage.  Forward: o0 = [residual] u + net; o1 = o0 -
// mean(o0 - u) (mass fix); o2 = clamp(o1) (limiter).  Given dG = dL/do2 and
// o1, writes dnet = dL/dnet and du = the direct part of dL/du.
__global__ __launch_bounds__(256) void k_out_bwd_sum(const double* __restrict__ dG,
                                                     const double* __restrict__ o1, int n,
                                                     int limiter, double lo, double hi,
                                                     double* __restrict__ partials, int bpf) {
  __shared__ double red[4];
  const int64_t f = blockIdx.x / bpf;
  const int part = blockIdx.x % bpf;
  const int64_t n2 = (int64_t)n * n;
  double s = 0.0;
  for (int64_t i = (int64_t)part * 256 + threadIdx.x; i < n2; i += (int64_t)bpf * 256) {
    const double v = o1[f * n2 + i];
    const bool pass = !limiter || (v > lo && v < hi);
    s += pass ? dG[f * n2 + i] : 0.0;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

template <typename T>
__global__ __launch_bounds__(256) void k_out_bwd(const double* __restrict__ dG,
                                                 const double* __restrict__ o1, int n,
                                                 int residual, int mass_fix, int limiter,
                                                 double lo, double hi,
                                                 const double* __restrict__ partials, int bpf,
                                                 T* __restrict__ dnet, double* __restrict__ du) {
  __shared__ double mean_sh;
  const int64_t f = blockIdx.x / bpf;
  const int part = blockIdx.x % bpf;
  const int64_t n2 = (int64_t)n * n;
  if (threadIdx.x == 0) {
    double s = 0.0;
    if (mass_fix)
      for (int i = 0; i < bpf; ++i) s += partials[f * bpf + i];
    mean_sh = s / (double)n2;
  }
  __syncthreads();
  const double mean = mean_sh;
  for (int64_t i = (int64_t)part * 256 + threadIdx.x; i < n2; i += (int64_t)bpf * 256) {
    const double v = o1[f * n2 + i];
    const bool pass = !limiter || (v > lo && v < hi);
    const double d1 = pass ? dG[f * n2 + i] : 0.0;   // dL/do1
    const double d0 = d1 - mean;                       // dL/do0 (mean = 0 without mass fix)
    dnet[f * n2 + i] = (T)d0;
    du[f * n2 + i] = (residual ? d0 : 0.0) + mean;
  }
}

// du += dX of the first layer (one channel)
template <typename T>
__global__ void k_add_into(double* __restrict__ du, const T* __restrict__ d, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) du[i] += (double)d[i];
}

// --------------------------------------------------------------- launch

size_t cnn_lds_bytes(int C, bool split, bool first, int shape);

// Blocks of the persistent hidden-layer kernel that fill the GPU once.
template <int C, bool SPLIT, bool FIRST = false, bool TAIL = false, int SHAPE = 0>
static int hidden_cap() {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 512;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_cnn_hidden<C, SPLIT, FIRST, TAIL, SHAPE>,
                                                   HidCfg<C, hidden_waves<C, TAIL>()>::NT,
                                                   cnn_lds_bytes(C, SPLIT, FIRST, SHAPE)) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return cus * per_cu;
}

// offsets of layer l's weights / biases in the concatenated arrays
static int64_t cnn_woff(int l, int L, int C) {
  int64_t o = 0;
  for (int i = 0; i < l; ++i) o += (int64_t)(i == 0 ? 1 : C) * (i == L - 1 ? 1 : C) * 9;
  return o;
}
static int64_t cnn_boff(int l, int C) { return (int64_t)l * C; }

int cnn_act_bytes(int prec) { return prec == kCnnF64 ? 8 : prec == kCnnF32 ? 4 : prec == kCnnBf16x2 ? 4 : 2; }
int cnn_grad_bytes(int prec) { return prec == kCnnF64 ? 8 : 4; }

// per-tile sums of G(u) - u for the mass fix, or nullptr (the last layer
// then skips the reduction)
static double* mass_partials(const CnnJob& j) { return j.mass_fix ? j.ws.partials : nullptr; }

// activation (and pre-activation) buffer of layer l's output
static void* act_buf(const CnnJob& j, int l, bool train) {
  const size_t bytes = (size_t)j.nfields * j.n * j.n * j.channels * cnn_act_bytes(j.prec);
  return train ? (char*)j.ws.acts + (size_t)l * bytes : j.ws.act[l & 1];
}
static void* z_buf(const CnnJob& j, int l, bool train) {
  const size_t zb = (size_t)j.nfields * j.n * j.n * j.channels * cnn_grad_bytes(j.prec);
  return train ? (char*)j.ws.zs + (size_t)l * zb : nullptr;
}

template <int C, typename T>
static void cnn_fwd_ref(const CnnJob& j, bool train, double* g_out, hipStream_t st) {
  const int n = j.n, L = j.n_layers;
  const int64_t tiles16 = (int64_t)(n / kTile) * (n / kTile);
  const dim3 g16((unsigned)(j.nfields * tiles16)), b256(256);
  const T* W = (const T*)j.W;
  const T* B = (const T*)j.B;
  k_cnn_first_ref<C, T><<<g16, b256, 0, st>>>(j.in_base, j.in_offs, n, W, B, j.act,
                                              (T*)act_buf(j, 0, train), (T*)z_buf(j, 0, train));
  for (int l = 1; l < L - 1; ++l)
    k_cnn_hidden_ref<C, T><<<g16, b256, 0, st>>>(
        (const T*)act_buf(j, l - 1, train), n, W + cnn_woff(l, L, C), B + cnn_boff(l, C), j.act,
        (T*)act_buf(j, l, train), (T*)z_buf(j, l, train));
  k_cnn_last_ref<C, T><<<g16, b256, 0, st>>>((const T*)act_buf(j, L - 2, train), n,
                                             W + cnn_woff(L - 1, L, C), B + cnn_boff(L - 1, C),
                                             j.in_base, j.in_offs, g_out, train ? nullptr : j.out_offs,
                                             j.residual, mass_partials(j));
}

std::atomic<int> g_cnn_plan{0};          // pr_cnn_plan, process-wide setting
std::atomic<int> g_cnn_tile{0};          // pr_cnn_tile, process-wide setting
std::atomic<int> g_cnn_tile_tuned[2][2][7];  // [C 32 / 48][split][log2 N - 4]: measured tile + 1 (0 = none)
std::atomic<int> g_cnn_tuned[5][8][2];     // [C index][L - 3][split]: measured choice (0 = none)

static int c_index(int C) { return C == 8 ? 0 : C == 16 ? 1 : C == 32 ? 2 : C == 48 ? 3 : 4; }

template <int C, int NH, bool SPLIT>
static int fused_cap() {
  using F = FusedCfg<C, NH, SPLIT>;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_cnn_fused<C, NH, SPLIT>, F::NT, F::LDS) !=
          hipSuccess || per_cu < 1)
    per_cu = 1;
  return cus * per_cu;
}

// The fused kernel for (C, NH, SPLIT), if one is built and fits in LDS.
template <int C, int NH, bool SPLIT>
static bool launch_fused_nh(const CnnJob& j, double* g_out, hipStream_t st) {
  using F = FusedCfg<C, NH, SPLIT>;
  if constexpr (!F::kFits || C % 16 != 0) {
    return false;
  } else {
    if (j.n % F::T != 0) return false;
    const int L = j.n_layers;
    const float* W = (const float*)j.W;
    const float* B = (const float*)j.B;
    const int64_t tiles = j.nfields * (int64_t)(j.n / F::T) * (j.n / F::T);
    static const int cap = fused_cap<C, NH, SPLIT>();
    const dim3 grid((unsigned)std::min<int64_t>(tiles, cap)), block(F::NT);
    k_cnn_fused<C, NH, SPLIT><<<grid, block, F::LDS, st>>>(
        j.in_base, j.in_offs, j.n, j.nfields, W, B, (const __bf16*)j.ws.wpack, B + C,
        W + cnn_woff(L - 1, L, C), B + cnn_boff(L - 1, C), j.act, j.residual, g_out, j.out_offs,
        mass_partials(j));
    return true;
  }
}

template <int C, bool SPLIT>
static bool launch_fused_c(const CnnJob& j, double* g_out, hipStream_t st) {
  if constexpr (C == 16) {
    switch (j.n_layers - 2) {
      case 1: return launch_fused_nh<16, 1, SPLIT>(j, g_out, st);
      case 2: return launch_fused_nh<16, 2, SPLIT>(j, g_out, st);
      case 3: return launch_fused_nh<16, 3, SPLIT>(j, g_out, st);
      case 4: return launch_fused_nh<16, 4, SPLIT>(j, g_out, st);
      default: return false;
    }
  } else if constexpr (C == 32) {
    switch (j.n_layers - 2) {
      case 1: return launch_fused_nh<32, 1, SPLIT>(j, g_out, st);
      case 2: return launch_fused_nh<32, 2, SPLIT>(j, g_out, st);
      default: return false;
    }
  } else if constexpr (C == 48 && !SPLIT) {
    return j.n_layers == 3 && launch_fused_nh<48, 1, false>(j, g_out, st);
  } else {
    return false;
  }
}

// Whether a fused kernel exists for this network (inference, bf16 kinds).
template <int C, bool SPLIT>
static constexpr bool fused_exists(int nh) {
  if (C % 16 != 0 || C > 48) return false;
  switch (nh) {
    case 1: return (C <= 32 || !SPLIT) && FusedCfg<C, 1, SPLIT>::kFits;
    case 2: return C <= 32 && FusedCfg<C, 2, SPLIT>::kFits;
    case 3: return C <= 16 && FusedCfg<C, 3, SPLIT>::kFits;
    case 4: return C <= 16 && FusedCfg<C, 4, SPLIT>::kFits;
    default: return false;
  }
}

bool cnn_fused_available(int C, int L, int prec) {
  if (prec != kCnnBf16 && prec != kCnnBf16x2) return false;
  const bool sp = prec == kCnnBf16x2;
  switch (C) {
    case 16: return sp ? fused_exists<16, true>(L - 2) : fused_exists<16, false>(L - 2);
    case 32: return sp ? fused_exists<32, true>(L - 2) : fused_exists<32, false>(L - 2);
    case 48: return sp ? fused_exists<48, true>(L - 2) : fused_exists<48, false>(L - 2);
    default: return false;
  }
}

bool cnn_folded_available(int C, int L, int prec) {
  return (prec == kCnnBf16 || prec == kCnnBf16x2) && C % 16 == 0 && C <= 64 && L >= 3;
}

int cnn_effective_plan(int C, int L, int prec) {
  const bool fused = cnn_fused_available(C, L, prec) && L >= 3 && L <= 10;
  const bool folded = cnn_folded_available(C, L, prec);
  int pl = g_cnn_plan.load();
  if (pl == CNN_PLAN_AUTO && L >= 3 && L <= 10)
    pl = g_cnn_tuned[c_index(C)][L - 3][prec == kCnnBf16x2 ? 1 : 0].load();
  // untuned default: FOLDED for split networks and at 32 channels, where
  // it measured faster than LAYERED; other unsplit widths fold only the
  // first layer, whose hidden-layer variant needs more registers than 4
  // waves per SIMD allow, and LAYERED wins.  (The whole-network fused
  // kernel measured slower for the 4 x 32 network at 256^2, where the halo
  // recomputation adds more activation work than the saved HBM traffic is
  // worth.)
  if (pl == CNN_PLAN_AUTO)
    pl = folded && (prec == kCnnBf16x2 || C == 32) ? CNN_PLAN_FOLDED : CNN_PLAN_LAYERED;
  if ((pl == CNN_PLAN_FUSED && !fused) || (pl == CNN_PLAN_FOLDED && !folded)) pl = CNN_PLAN_LAYERED;
  return pl;
}

// Hidden-layer output tile shape (0 = 8 x 32, 1 = 16 x 16) for a bf16
// network of C channels on N x N fields: the pr_cnn_tile setting, else the
// autotuner's measured choice for (C, prec, N), else 16 x 16 at 48 channels
// (faster on every batch measured, 1-5%) and 8 x 32 at 32 (either way by
// batch and N, within 2%).
static int tile_slot(int n) {
  int lg = 0;
  while ((1 << lg) < n) ++lg;
  return lg - 4;
}
int cnn_effective_tile(int C, int prec, int n) {
  if (C != 32 && C != 48) return 0;
  const int t = g_cnn_tile.load();
  if (t == CNN_TILE_8X32) return 0;
  if (t == CNN_TILE_16X16) return 1;
  const int k = tile_slot(n);
  if (k < 0 || k > 6) return C == 48 ? 1 : 0;
  const int tuned = g_cnn_tile_tuned[C == 48][prec == kCnnBf16x2][k].load();
  return tuned > 0 ? tuned - 1 : (C == 48 ? 1 : 0);
}
void cnn_set_tile(int tile) { g_cnn_tile.store(tile); }
int cnn_get_tile() { return g_cnn_tile.load(); }
void cnn_record_tile(int C, int prec, int n, int shape) {
  const int k = tile_slot(n);
  if ((C == 32 || C == 48) && k >= 0 && k <= 6)
    g_cnn_tile_tuned[C == 48][prec == kCnnBf16x2][k].store(shape + 1);
}

void cnn_set_plan(int plan) { g_cnn_plan.store(plan); }
int cnn_get_plan() { return g_cnn_plan.load(); }
void cnn_record_tuned(int C, int L, int prec, int plan) {
  if (L >= 3 && L <= 10) g_cnn_tuned[c_index(C)][L - 3][prec == kCnnBf16x2 ? 1 : 0].store(plan);
}

// What the last kernel of a forward pass took over from the caller.
enum { kDidCorr = 1, kDidOut2 = 2 };

// Returns the kDid* flags of what the last kernel did.
template <int C>
static int cnn_fwd_bf16(const CnnJob& j, bool train, double* g_out, hipStream_t st) {
  const int n = j.n, L = j.n_layers;
  if (!train && cnn_effective_plan(C, L, j.prec) == CNN_PLAN_FUSED) {
    const bool done = j.prec == kCnnBf16x2 ? launch_fused_c<C, true>(j, g_out, st)
                                           : launch_fused_c<C, false>(j, g_out, st);
    if (done) return 0;
  }
  const int64_t tiles16 = (int64_t)(n / kTile) * (n / kTile);
  const dim3 g16((unsigned)(j.nfields * tiles16)), b256(256);
  const bool split = j.prec == kCnnBf16x2;
  const int64_t act_elems = j.nfields * (int64_t)n * n * C;
  const float* W = (const float*)j.W;
  const float* B = (const float*)j.B;
  auto hi = [&](int l) { return (__bf16*)act_buf(j, l, train); };
  auto lo = [&](int l) { return split ? hi(l) + act_elems : (__bf16*)nullptr; };
  // PR_CNN_PLAN_FOLDED (inference only; training keeps every layer's
  // activations): the first layer runs inside the first hidden layer's
  // launch, and at C = 32 or 48 the last layer's per-tap products inside the
  // last hidden layer's, summed over the taps by k_cnn_last_gather
  const bool folded = !train && cnn_effective_plan(C, L, j.prec) == CNN_PLAN_FOLDED;
  const bool tail = folded && (C == 32 || (C == 48 && PR_TAIL48));
  float* Yp = nullptr;
  if (!folded)
    k_cnn_first<C, __bf16><<<g16, b256, 0, st>>>(j.in_base, j.in_offs, n, W, B, j.act, hi(0), lo(0),
                                                 (float*)z_buf(j, 0, train));
  for (int l = 1; l < L - 1; ++l) {
    if constexpr (C % 16 == 0) {
      using H = HidCfg<C>;
      const __bf16* wp = (const __bf16*)j.ws.wpack + (int64_t)(l - 1) * C * H::KP;
      const bool first = folded && l == 1, last = tail && l == L - 2;
      const int shape = both_tile_shapes<C>() ? cnn_effective_tile(C, j.prec, n) : 0;
      const size_t lds = cnn_lds_bytes(C, split, first, shape);
      const int64_t tiles = j.nfields * (n / H::TH) * (n / H::TW);  // the same for both shapes
      const FirstIn fi{j.in_base, j.in_offs, W, B};
      const float* WL = W + cnn_woff(L - 1, L, C);
      const bf16x8* WLp = (const bf16x8*)((const __bf16*)j.ws.wpack + (int64_t)(L - 2) * C * H::KP);
      // the tap planes (9 floats per pixel) take the place of the layer's
      // output activations (2 C or 4 C bytes per pixel)
      if (last) Yp = (float*)hi(l);
      float* zo = (float*)z_buf(j, l, train);
      const __bf16* ih = first ? nullptr : hi(l - 1);
      const __bf16* il = first ? nullptr : lo(l - 1);
      __bf16* oh = last ? nullptr : hi(l);
      __bf16* ol = last ? nullptr : lo(l);
#define PR_HID_S(SP, FI, TA, SH)                                                                 \
  {                                                                                              \
    static const int cap = hidden_cap<C, SP, FI, TA, SH>();                                      \
    const dim3 gh((unsigned)std::min<int64_t>(tiles, cap));                                      \
    const dim3 bh(HidCfg<C, hidden_waves<C, TA>()>::NT);                                       \
    k_cnn_hidden<C, SP, FI, TA, SH><<<gh, bh, lds, st>>>(ih, il, n, j.nfields, wp,               \
                                                         B + cnn_boff(l, C), j.act, oh, ol, zo,  \
                                                         fi, WL, WLp, Yp);                       \
  }
#define PR_HID(SP, FI, TA)                                                                       \
  {                                                                                              \
    if constexpr (both_tile_shapes<C>()) {                                                       \
      if (shape) PR_HID_S(SP, FI, TA, 1)                                                         \
      else PR_HID_S(SP, FI, TA, 0)                                                               \
    } else PR_HID_S(SP, FI, TA, 0)                                                               \
  }
      if constexpr (C == 32 || C == 48) {
        if (split) {
          if (first && last) PR_HID(true, true, true)
          else if (first) PR_HID(true, true, false)
          else if (last) PR_HID(true, false, true)
          else PR_HID(true, false, false)
        } else {
          if (first && last) PR_HID(false, true, true)
          else if (first) PR_HID(false, true, false)
          else if (last) PR_HID(false, false, true)
          else PR_HID(false, false, false)
        }
      } else {
        if (split) {
          if (first) PR_HID(true, true, false)
          else PR_HID(true, false, false)
        } else {
          if (first) PR_HID(false, true, false)
          else PR_HID(false, false, false)
        }
      }
#undef PR_HID
#undef PR_HID_S
    }
  }
  const bool fold_corr = Yp && j.corr && !j.mass_fix && !j.limiter;
  if (fold_corr) {
    const CorrectJob& c = *j.corr;
    const int bpf = (int)((int64_t)n * n / 512);  // 256 threads x 2 points; N >= 32
    const dim3 gc((unsigned)(j.nfields * bpf));
    if (c.f_f32)
      k_cnn_gather_correct<float><<<gc, b256, 0, st>>>(
          Yp, n, j.nfields, B + cnn_boff(L - 1, C), j.in_base, j.in_offs, j.residual,
          (const float*)c.f, c.f_offs, c.g_old, c.go_offs, c.u, c.u_offs, c.upd, c.upd_idx,
          c.update_cache, bpf);
    else
      k_cnn_gather_correct<double><<<gc, b256, 0, st>>>(
          Yp, n, j.nfields, B + cnn_boff(L - 1, C), j.in_base, j.in_offs, j.residual,
          (const double*)c.f, c.f_offs, c.g_old, c.go_offs, c.u, c.u_offs, c.upd, c.upd_idx,
          c.update_cache, bpf);
  } else if (Yp) {
    // the second destination only where nothing changes the output later
    double* o2 = j.mass_fix || j.limiter ? nullptr : j.out2_base;
    if (j.mass_fix)
      k_cnn_last_gather<<<g16, b256, 0, st>>>(Yp, n, j.nfields, B + cnn_boff(L - 1, C), j.in_base,
                                              j.in_offs, g_out, train ? nullptr : j.out_offs,
                                              j.residual, mass_partials(j), o2, j.out2_offs);
    else
      k_cnn_last_gather_lin<<<dim3((unsigned)(j.nfields * (n * n / 512))), b256, 0, st>>>(
          Yp, n, j.nfields, B + cnn_boff(L - 1, C), j.in_base, j.in_offs, g_out,
          train ? nullptr : j.out_offs, j.residual, o2, j.out2_offs, n * n / 512);
    return o2 ? kDidOut2 : 0;
  }
  else if (split)
    k_cnn_last_mma<C, true><<<g16, b256, 0, st>>>(hi(L - 2), lo(L - 2), n, W + cnn_woff(L - 1, L, C),
                                                  B + cnn_boff(L - 1, C), j.in_base, j.in_offs,
                                                  g_out, train ? nullptr : j.out_offs, j.residual,
                                                  mass_partials(j));
  else
    k_cnn_last_mma<C, false><<<g16, b256, 0, st>>>(hi(L - 2), nullptr, n, W + cnn_woff(L - 1, L, C),
                                                   B + cnn_boff(L - 1, C), j.in_base, j.in_offs,
                                                   g_out, train ? nullptr : j.out_offs, j.residual,
                                                   mass_partials(j));
  return fold_corr ? kDidCorr : 0;
}

// Forward of G; in training mode every layer's activation and pre-activation
// is kept and the output (before the limiter) goes to ws.o1.
template <int C>
static hipError_t launch_cnn_fwd_c(const CnnJob& j, bool train, hipStream_t st) {
  const int n = j.n;
  double* g_out = train ? j.ws.o1 : j.out_base;
  if (train && (j.corr || j.out2_base)) return hipErrorInvalidValue;
  int did = 0;
  if (j.prec == kCnnF64) {
    if constexpr (C <= kCnnF64MaxC) cnn_fwd_ref<C, double>(j, train, g_out, st);
    else return hipErrorInvalidValue;
  } else if (j.prec == kCnnF32) {
    cnn_fwd_ref<C, float>(j, train, g_out, st);
  } else {
    if (j.n_layers > 2 && C % 16 != 0) return hipErrorInvalidValue;
    did = cnn_fwd_bf16<C>(j, train, g_out, st);
  }
  const int limiter = train ? 0 : j.limiter;
  if (!(did & kDidCorr) && (j.mass_fix || limiter)) {
    const int bpf = (int)std::max<int64_t>(1, (int64_t)n * n / 2048);
    const int64_t tiles16 = (int64_t)(n / kTile) * (n / kTile);
    k_cnn_fix<<<dim3((unsigned)(j.nfields * bpf)), dim3(256), 0, st>>>(
        g_out, train ? nullptr : j.out_offs, n, j.ws.partials, (int)tiles16, j.mass_fix, limiter,
        j.lim_lo, j.lim_hi, bpf);
  }
  // a correction the network's last kernel did not apply: on the stored
  // output (its g_new must address g_out as written above)
  if (j.corr && !(did & kDidCorr)) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_correct(*j.corr, st);
  }
  if (j.out2_base && !(did & kDidOut2)) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_copy(j.nfields, n, g_out, j.out_offs, j.out2_base, j.out2_offs, st);
  }
  return hipGetLastError();
}

template <int CI, int CO, typename TG, typename TX, typename TW>
static void conv_bwd(const CnnJob& j, const TG* dY, const TX* X, const TX* X_lo, const TW* W,
                     TW* dW, TW* db, TG* dX, hipStream_t st) {
  const int n = j.n;
  const int64_t tiles16 = j.nfields * (int64_t)(n / kTile) * (n / kTile);
  const dim3 g16((unsigned)tiles16), b256(256);
  constexpr int NP = CO * CI * 9 + CO;
  // tiles -> kWGradGroups group sums -> dW, each stage in a fixed order
  const int64_t per = (tiles16 + kWGradGroups - 1) / kWGradGroups;
  const dim3 gr((NP + 255) / 256, kWGradGroups);
  if constexpr (CI >= 32 && CO >= 32) {
    // weight sums stored in TG (half the bytes in FP32), biases in FP64
    constexpr int NW = CO * CI * 9;
    k_conv_bwd_weight_rb<CI, CO, TG, TX><<<g16, b256, 0, st>>>(dY, X, X_lo, n, j.ws.wpart);
    const double* bp = (const double*)((const char*)j.ws.wpart +
                                       rb_bias_offset(tiles16, NW, sizeof(TG)));
    k_reduce_groups<TG><<<gr, b256, 0, st>>>((const TG*)j.ws.wpart, bp, tiles16, NW, NP, per,
                                             j.ws.wpart2);
  } else {
    k_conv_bwd_weight<CI, CO, TG, TX><<<g16, b256, 0, st>>>(dY, X, X_lo, n, j.ws.wpart);
    k_reduce_groups<double><<<gr, b256, 0, st>>>(j.ws.wpart, nullptr, tiles16, NP, NP, per,
                                                 j.ws.wpart2);
  }
  k_reduce_partials<TW><<<dim3((NP + 255) / 256), b256, 0, st>>>(j.ws.wpart2, kWGradGroups, NP, dW,
                                                                 CO * CI * 9, db);
  if (dX) {
    // the weight partials are reduced by now: their buffer holds the
    // transposed weights
    TW* Wt = (TW*)j.ws.wpart;
    k_w_transpose<CI, CO, TW><<<dim3((CO * CI * 9 + 255) / 256), b256, 0, st>>>(W, Wt);
    k_conv_bwd_data<CI, CO, TG, TW><<<g16, b256, 0, st>>>(dY, n, Wt, dX);
  }
}

template <int C, typename TG, typename TA, typename TZ, typename TW>
static hipError_t cnn_bwd_layers(const CnnJob& j, const double* dG, double* du, TW* gW, TW* gB,
                                 hipStream_t st) {
  const int n = j.n, L = j.n_layers;
  const int64_t n2 = (int64_t)n * n, pix = j.nfields * n2;
  const bool split = j.prec == kCnnBf16x2;
  const int64_t act_elems = pix * C;
  const TW* W = (const TW*)j.W;
  auto A = [&](int l) { return (const TA*)act_buf(j, l, true); };
  auto Alo = [&](int l) { return split ? A(l) + act_elems : (const TA*)nullptr; };
  auto Z = [&](int l) { return (const TZ*)z_buf(j, l, true); };
  TG* d0 = (TG*)j.ws.d[0];
  TG* d1 = (TG*)j.ws.d[1];
  // output stage
  const int bpf = (int)std::max<int64_t>(1, n2 / 2048);
  k_out_bwd_sum<<<dim3((unsigned)(j.nfields * bpf)), dim3(256), 0, st>>>(
      dG, j.ws.o1, n, j.limiter, j.lim_lo, j.lim_hi, j.ws.fpart, bpf);
  k_out_bwd<TG><<<dim3((unsigned)(j.nfields * bpf)), dim3(256), 0, st>>>(
      dG, j.ws.o1, n, j.residual, j.mass_fix, j.limiter, j.lim_lo, j.lim_hi, j.ws.fpart, bpf, d0,
      du);
  // last layer: C -> 1
  conv_bwd<C, 1, TG, TA, TW>(j, d0, A(L - 2), Alo(L - 2), W + cnn_woff(L - 1, L, C),
                             gW + cnn_woff(L - 1, L, C), gB + cnn_boff(L - 1, C), d1, st);
  const dim3 ge((unsigned)((act_elems / 4 + 255) / 256)), b256(256);  // act_elems % 8 == 0
  k_act_bwd<TG, TZ><<<ge, b256, 0, st>>>(d1, Z(L - 2), act_elems, j.act);
  std::swap(d0, d1);  // d0 = dZ of layer L-2
  for (int l = L - 2; l >= 1; --l) {
    conv_bwd<C, C, TG, TA, TW>(j, d0, A(l - 1), Alo(l - 1), W + cnn_woff(l, L, C),
                               gW + cnn_woff(l, L, C), gB + cnn_boff(l, C), d1, st);
    k_act_bwd<TG, TZ><<<ge, b256, 0, st>>>(d1, Z(l - 1), act_elems, j.act);
    std::swap(d0, d1);
  }
  // first layer: 1 -> C, its input is the state itself
  conv_bwd<1, C, TG, double, TW>(j, d0, j.in_base, nullptr, W, gW, gB, d1, st);
  k_add_into<TG><<<dim3((unsigned)((pix + 255) / 256)), b256, 0, st>>>(du, d1, pix);
  return hipGetLastError();
}

template <int C>
static hipError_t launch_cnn_bwd_c(const CnnJob& j, const double* dG, double* du, void* gW,
                                   void* gB, hipStream_t st) {
  hipError_t e = launch_cnn_fwd_c<C>(j, true, st);
  if (e != hipSuccess) return e;
  if (j.prec == kCnnF64) {
    if constexpr (C <= kCnnF64MaxC)
      return cnn_bwd_layers<C, double, double, double, double>(j, dG, du, (double*)gW, (double*)gB, st);
    else
      return hipErrorInvalidValue;
  }
  if (j.prec == kCnnF32)
    return cnn_bwd_layers<C, float, float, float, float>(j, dG, du, (float*)gW, (float*)gB, st);
  return cnn_bwd_layers<C, float, __bf16, float, float>(j, dG, du, (float*)gW, (float*)gB, st);
}

hipError_t launch_cnn_pack(const CnnJob& j, hipStream_t st) {
  if (j.prec == kCnnF32 || j.prec == kCnnF64 || j.n_layers < 3) return hipSuccess;
  const int C = j.channels, L = j.n_layers;
  const int kp = (9 * C + 31) / 32 * 32;
  int64_t wo = (int64_t)C * 9;  // layer 0 is 1 -> C
  for (int l = 1; l < L - 1; ++l) {
    const int64_t cnt = (int64_t)C * kp;
    k_cnn_pack<<<dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st>>>(
        (const float*)j.W + wo, C, C, kp, (__bf16*)j.ws.wpack + (int64_t)(l - 1) * C * kp);
    wo += (int64_t)C * C * 9;
  }
  bf16x8* last = (bf16x8*)((__bf16*)j.ws.wpack + (int64_t)(L - 2) * C * kp);
  switch (C) {
    case 8: k_cnn_pack_last<8><<<1, 64, 0, st>>>((const float*)j.W + wo, last); break;
    case 16: k_cnn_pack_last<16><<<1, 64, 0, st>>>((const float*)j.W + wo, last); break;
    case 32: k_cnn_pack_last<32><<<1, 64, 0, st>>>((const float*)j.W + wo, last); break;
    case 48: k_cnn_pack_last<48><<<1, 64, 0, st>>>((const float*)j.W + wo, last); break;
    case 64: k_cnn_pack_last<64><<<1, 64, 0, st>>>((const float*)j.W + wo, last); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_cnn(const CnnJob& j, hipStream_t st) {
  if (j.nfields <= 0) return hipSuccess;
  switch (j.channels) {
    case 8: return launch_cnn_fwd_c<8>(j, false, st);
    case 16: return launch_cnn_fwd_c<16>(j, false, st);
    case 32: return launch_cnn_fwd_c<32>(j, false, st);
    case 48: return launch_cnn_fwd_c<48>(j, false, st);
    case 64: return launch_cnn_fwd_c<64>(j, false, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_cnn_backward(const CnnJob& j, const double* dG, double* du, void* gW, void* gB,
                               hipStream_t st) {
  if (j.nfields <= 0) return hipSuccess;
  switch (j.channels) {
    case 8: return launch_cnn_bwd_c<8>(j, dG, du, gW, gB, st);
    case 16: return launch_cnn_bwd_c<16>(j, dG, du, gW, gB, st);
    case 32: return launch_cnn_bwd_c<32>(j, dG, du, gW, gB, st);
    case 48: return launch_cnn_bwd_c<48>(j, dG, du, gW, gB, st);
    case 64: return launch_cnn_bwd_c<64>(j, dG, du, gW, gB, st);
    default: return hipErrorInvalidValue;
  }
}

template <int C, int SHAPE>
static size_t hid_lds(bool split, bool first) {
  using S = HidTile<C, true, tile_h<SHAPE>(), tile_w<SHAPE>()>;
  using U = HidTile<C, false, tile_h<SHAPE>(), tile_w<SHAPE>()>;
  return split ? (first ? S::FIRST_BYTES : S::BYTES) + S::STAGE_BYTES
               : (first ? U::FIRST_BYTES : U::BYTES) + U::STAGE_BYTES;
}

size_t cnn_lds_bytes(int C, bool split, bool first, int shape) {
  switch (C) {
    case 16: return hid_lds<16, 0>(split, first);
    case 32: return shape ? hid_lds<32, 1>(split, first) : hid_lds<32, 0>(split, first);
    case 48: return shape ? hid_lds<48, 1>(split, first) : hid_lds<48, 0>(split, first);
    case 64: return hid_lds<64, 0>(split, first);
    default: return 0;
  }
}

template <int C, int NH, bool SPLIT>
static hipError_t fused_lds_limit() {
  using F = FusedCfg<C, NH, SPLIT>;
  if constexpr (!F::kFits) {
    return hipSuccess;
  } else {
    return hipFuncSetAttribute((const void*)k_cnn_fused<C, NH, SPLIT>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)F::LDS);
  }
}

hipError_t cnn_set_lds_limits() {
  // raise the dynamic-LDS limit of each hidden-layer kernel to what it
  // uses; configurations beyond the 160 KB of a CU are rejected earlier
  constexpr size_t kMaxLds = 160 * 1024;
  hipError_t e = hipSuccess;
#define PR_F(CC, NH)                                                        \
  if (e == hipSuccess) e = fused_lds_limit<CC, NH, false>();                \
  if (e == hipSuccess) e = fused_lds_limit<CC, NH, true>();
  PR_F(16, 1) PR_F(16, 2) PR_F(16, 3) PR_F(16, 4) PR_F(32, 1) PR_F(32, 2)
#undef PR_F
  if (e == hipSuccess) e = fused_lds_limit<48, 1, false>();
#define PR_A(CC, SP, FI, TA, SH)                                                             \
  if (e == hipSuccess && cnn_lds_bytes(CC, SP, FI, SH) <= kMaxLds)                           \
    e = hipFuncSetAttribute((const void*)k_cnn_hidden<CC, SP, FI, TA, SH>,                   \
                            hipFuncAttributeMaxDynamicSharedMemorySize,                      \
                            (int)cnn_lds_bytes(CC, SP, FI, SH));
#define PR_B(CC, TA, SH) \
  PR_A(CC, false, false, TA, SH) PR_A(CC, true, false, TA, SH) PR_A(CC, false, true, TA, SH) PR_A(CC, true, true, TA, SH)
  PR_B(16, false, 0) PR_B(32, false, 0) PR_B(48, false, 0) PR_B(64, false, 0)
  PR_B(32, true, 0) PR_B(48, true, 0)
  PR_B(32, false, 1) PR_B(48, false, 1) PR_B(32, true, 1) PR_B(48, true, 1)
#undef PR_B
#undef PR_A
  return e;
}

}  // namespace pr
