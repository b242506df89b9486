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
//                 pixels (16 per block of a 16x16x32 bf16 MFMA), N = output
//                 channels (16 per block), K = 9 C ordered (tap, channel)
//                 and padded to a multiple of 32; FP32 accumulation.  A
//                 work-group stages a (TH+2) x (TW+2) input tile and the
//                 layer's packed weights in LDS.  With SPLIT the activation
//                 is carried as hi + lo bfloat16 and every product is done
//                 twice (hi W + lo W), which keeps ~16 mantissa bits.
//   k_cnn_hidden_f32  the same layer on the vector ALU in FP32 (reference
//                 precision).
//   k_cnn_last    C -> 1 on the vector ALU, plus the residual, written in
//                 FP64, with per-tile FP64 sums of (G(u) - u).
//   k_cnn_fix     the uniform mass fix and the limiter.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>

#include "internal.h"

namespace pr {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

__device__ __forceinline__ float act_fn(float x, int act) {
  if (act == kActTanh) return tanhf(x);
  return 0.5f * x * (1.0f + erff(x * 0.70710678118654752440f));  // exact GELU
}

template <typename T> __device__ __forceinline__ float to_f(T v) { return (float)v; }

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
                                                   TO* __restrict__ out, TO* __restrict__ out_lo) {
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
    float r8[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int co = c8 * 8 + j;
      float s = sb[co];
#pragma unroll
      for (int tp = 0; tp < 9; ++tp) s += sw[co * 9 + tp] * v[tp];
      r8[j] = act_fn(s, act);
    }
    const int64_t o = ((f * n + y0 + py) * (int64_t)n + x0 + pxx) * C + c8 * 8;
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

template <int C> struct HidCfg {
  static constexpr int TH = 8, TW = 32;              // output tile (rows, columns)
  static constexpr int NW = 4, NT = 64 * NW;         // waves, threads
  static constexpr int CS = C + 8;                   // LDS pixel stride (elements)
  static constexpr int KP = (9 * C + 31) / 32 * 32;  // K padded to the MFMA depth
  static constexpr int MB = TH * TW / 16;            // 16-pixel blocks per tile
  static constexpr int MBW = MB / NW;                // per wave
  static constexpr int NB = C / 16;                  // 16-channel blocks
  static constexpr int KB = KP / 32;                 // K steps
  static constexpr int TPIX = (TH + 2) * (TW + 2);
  static constexpr int OS = C + 8;                   // LDS stride of the output staging rows
};

// Persistent over tiles: each wave keeps the whole layer's weight fragments
// (KB x NB bfloat16x8 B operands) in registers, the block stages one input
// tile at a time in LDS, and each 16-pixel output block is staged in LDS
// (per wave) so that it leaves as 16-byte coalesced stores.
template <int C, bool SPLIT>
__global__ __launch_bounds__(HidCfg<C>::NT) void k_cnn_hidden(
    const __bf16* __restrict__ in, const __bf16* __restrict__ in_lo, int n, int64_t nfields,
    const __bf16* __restrict__ Wp, const float* __restrict__ b, int act,
    __bf16* __restrict__ out, __bf16* __restrict__ out_lo) {
  using H = HidCfg<C>;
  static_assert(C % 16 == 0, "hidden width must be a multiple of 16");
  extern __shared__ __align__(16) unsigned char smem[];
  __bf16* tile = (__bf16*)smem;                               // [TPIX][CS]
  __bf16* tile_lo = tile + H::TPIX * H::CS;                   // SPLIT only
  __bf16* stage = tile + (SPLIT ? 2 : 1) * H::TPIX * H::CS;   // [NW][(SPLIT?2:1)*16][OS]

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int tpy = n / H::TH, tpx = n / H::TW;
  const int64_t tiles = nfields * tpy * tpx;

  // this lane's weight fragments and biases, for the whole kernel
  bf16x8 bfr[H::KB][H::NB];
  float bias[H::NB];
#pragma unroll
  for (int nb = 0; nb < H::NB; ++nb) {
    bias[nb] = b[nb * 16 + r];
#pragma unroll
    for (int kb = 0; kb < H::KB; ++kb)
      bfr[kb][nb] = *(const bf16x8*)&Wp[(int64_t)(nb * 16 + r) * H::KP + kb * 32 + 8 * g];
  }
  __bf16* st = stage + wave * (SPLIT ? 2 : 1) * 16 * H::OS;

  for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    const int64_t f = t / (tpy * tpx);
    const int tt = (int)(t % (tpy * tpx));
    const int y0 = (tt / tpx) * H::TH, x0 = (tt % tpx) * H::TW;
    __syncthreads();  // the previous tile is no longer read
    constexpr int TCH = H::TPIX * (C / 8);
    for (int i = tid; i < TCH; i += H::NT) {
      const int p = i / (C / 8), c8 = i % (C / 8);
      const int ty = p / (H::TW + 2), tx = p % (H::TW + 2);
      const int gy = (y0 + ty - 1) & (n - 1), gx = (x0 + tx - 1) & (n - 1);
      const int64_t gi = ((f * n + gy) * (int64_t)n + gx) * C + c8 * 8;
      *(bf16x8*)&tile[p * H::CS + c8 * 8] = *(const bf16x8*)&in[gi];
      if constexpr (SPLIT) *(bf16x8*)&tile_lo[p * H::CS + c8 * 8] = *(const bf16x8*)&in_lo[gi];
    }
    __syncthreads();

    for (int m = 0; m < H::MBW; ++m) {
      const int mb = wave * H::MBW + m;
      const int oy = mb / (H::TW / 16), ox0 = (mb % (H::TW / 16)) * 16;
      f32x4 acc[H::NB];
#pragma unroll
      for (int nb = 0; nb < H::NB; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < H::KB; ++kb) {
        const int k0 = kb * 32 + 8 * g;
        const bool live = k0 < 9 * C;
        const int tap = live ? k0 / C : 0, ci0 = live ? k0 % C : 0;
        const int a_off = ((oy + tap / 3) * (H::TW + 2) + ox0 + r + tap % 3) * H::CS + ci0;
        bf16x8 afr = *(const bf16x8*)&tile[a_off];
        if (!live) afr = bf16x8{};
#pragma unroll
        for (int nb = 0; nb < H::NB; ++nb)
          acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr, bfr[kb][nb], acc[nb], 0, 0, 0);
        if constexpr (SPLIT) {
          bf16x8 alo = *(const bf16x8*)&tile_lo[a_off];
          if (!live) alo = bf16x8{};
#pragma unroll
          for (int nb = 0; nb < H::NB; ++nb)
            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bfr[kb][nb], acc[nb], 0, 0, 0);
        }
      }
      // bias + activation into the wave's staging rows: pixel 4 g + i, channel nb 16 + r
#pragma unroll
      for (int nb = 0; nb < H::NB; ++nb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float v = act_fn(acc[nb][i] + bias[nb], act);
          const __bf16 h = (__bf16)v;
          st[(4 * g + i) * H::OS + nb * 16 + r] = h;
          if constexpr (SPLIT) st[(16 + 4 * g + i) * H::OS + nb * 16 + r] = (__bf16)(v - (float)h);
        }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): staged values visible to the wave
      __builtin_amdgcn_wave_barrier();
      // 16 pixels x C channels are contiguous in the output: 16-byte stores
      const int64_t ob = ((f * n + y0 + oy) * (int64_t)n + x0 + ox0) * C;
      constexpr int CH = 16 * C / 8;
      for (int i = lane; i < CH; i += 64) {
        const int px = i / (C / 8), c8 = i % (C / 8);
        *(bf16x8*)&out[ob + px * C + c8 * 8] = *(const bf16x8*)&st[px * H::OS + c8 * 8];
        if constexpr (SPLIT)
          *(bf16x8*)&out_lo[ob + px * C + c8 * 8] = *(const bf16x8*)&st[(16 + px) * H::OS + c8 * 8];
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
}

// FP32 reference-precision hidden layer on the vector ALU: one pixel per
// thread, weights read uniformly across the wave (scalar loads).
template <int C>
__global__ __launch_bounds__(256) void k_cnn_hidden_f32(const float* __restrict__ in, int n,
                                                        const float* __restrict__ W,
                                                        const float* __restrict__ b, int act,
                                                        float* __restrict__ out) {
  __shared__ float tile[(kTile + 2) * (kTile + 2) * (C + 1)];
  const int tid = threadIdx.x;
  const int tpr = n / kTile;
  const int64_t f = blockIdx.x / (tpr * tpr);
  const int t = (int)(blockIdx.x % (tpr * tpr));
  const int y0 = (t / tpr) * kTile, x0 = (t % tpr) * kTile;
  for (int i = tid; i < (kTile + 2) * (kTile + 2) * C; i += 256) {
    const int p = i / C, c = i % C;
    const int ty = p / (kTile + 2), tx = p % (kTile + 2);
    const int gy = (y0 + ty - 1) & (n - 1), gx = (x0 + tx - 1) & (n - 1);
    tile[p * (C + 1) + c] = in[((f * n + gy) * (int64_t)n + gx) * C + c];
  }
  __syncthreads();
  const int py = tid / kTile, px = tid % kTile;
  float acc[C];
#pragma unroll
  for (int co = 0; co < C; ++co) acc[co] = b[co];
  for (int tp = 0; tp < 9; ++tp) {
    const int p = (py + tp / 3) * (kTile + 2) + px + tp % 3;
    for (int ci = 0; ci < C; ++ci) {
      const float x = tile[p * (C + 1) + ci];
#pragma unroll
      for (int co = 0; co < C; ++co) acc[co] += W[(co * C + ci) * 9 + tp] * x;
    }
  }
  const int64_t o = ((f * n + y0 + py) * (int64_t)n + x0 + px) * C;
#pragma unroll
  for (int co = 0; co < C; ++co) out[o + co] = act_fn(acc[co], act);
}

// ------------------------------------------------------------- last layer

// One pixel per thread.  The input tile is loaded with 16-byte vectors
// (8 channels) and kept in the input precision; the weights are read with
// wave-uniform addresses (scalar loads).
template <int C, typename TI>
__global__ __launch_bounds__(256) void k_cnn_last(
    const TI* __restrict__ in, const TI* __restrict__ in_lo, int n, const float* __restrict__ W,
    const float* __restrict__ b, const double* __restrict__ u_base,
    const int64_t* __restrict__ u_offs, double* __restrict__ g_base,
    const int64_t* __restrict__ g_offs, int residual, double* __restrict__ partials) {
  constexpr int C8 = C / 8;
  constexpr int PS = C + (sizeof(TI) == 2 ? 8 : 4);  // LDS pixel stride (elements)
  constexpr int TP = (kTile + 2) * (kTile + 2);
  __shared__ __align__(16) TI tile[TP * PS];
  __shared__ __align__(16) TI tile_lo[(sizeof(TI) == 2 ? TP * PS : 1)];
  __shared__ double red[4];
  const int tid = threadIdx.x;
  const int tpr = n / kTile, m = n - 1;
  const int64_t f = blockIdx.x / (tpr * tpr);
  const int t = (int)(blockIdx.x % (tpr * tpr));
  const int y0 = (t / tpr) * kTile, x0 = (t % tpr) * kTile;
  const bool split = sizeof(TI) == 2 && in_lo != nullptr;
  for (int i = tid; i < TP * C8; i += 256) {
    const int p = i / C8, c8 = i % C8;
    const int ty = p / (kTile + 2), tx = p % (kTile + 2);
    const int64_t gi = ((f * n + ((y0 + ty - 1) & m)) * (int64_t)n + ((x0 + tx - 1) & m)) * C + c8 * 8;
    if constexpr (sizeof(TI) == 2) {
      *(bf16x8*)&tile[p * PS + c8 * 8] = *(const bf16x8*)&in[gi];
      if (split) *(bf16x8*)&tile_lo[p * PS + c8 * 8] = *(const bf16x8*)&in_lo[gi];
    } else {
      *(float4*)&tile[p * PS + c8 * 8] = *(const float4*)&in[gi];
      *(float4*)&tile[p * PS + c8 * 8 + 4] = *(const float4*)&in[gi + 4];
    }
  }
  __syncthreads();
  const int py = tid / kTile, px = tid % kTile;
  float s = b[0];
  for (int tp = 0; tp < 9; ++tp) {
    const int p = (py + tp / 3) * (kTile + 2) + px + tp % 3;
#pragma unroll
    for (int c8 = 0; c8 < C8; ++c8) {
      float x[8];
      if constexpr (sizeof(TI) == 2) {
        const bf16x8 h = *(const bf16x8*)&tile[p * PS + c8 * 8];
#pragma unroll
        for (int j = 0; j < 8; ++j) x[j] = (float)h[j];
        if (split) {
          const bf16x8 l = *(const bf16x8*)&tile_lo[p * PS + c8 * 8];
#pragma unroll
          for (int j = 0; j < 8; ++j) x[j] += (float)l[j];
        }
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) x[j] = tile[p * PS + c8 * 8 + j];
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) s += W[(c8 * 8 + j) * 9 + tp] * x[j];
    }
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

// --------------------------------------------------------------- launch

size_t cnn_lds_bytes(int C, bool split);

// Blocks of the persistent hidden-layer kernel that fill the GPU once.
template <int C, bool SPLIT>
static int hidden_cap() {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 512;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_cnn_hidden<C, SPLIT>,
                                                   HidCfg<C>::NT, cnn_lds_bytes(C, SPLIT)) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return cus * per_cu;
}

template <int C>
static hipError_t launch_cnn_c(const CnnJob& j, hipStream_t st) {
  const int n = j.n;
  const int64_t tiles16 = (int64_t)(n / kTile) * (n / kTile);
  const int L = j.n_layers;
  const int64_t act_elems = j.nfields * (int64_t)n * n * C;
  const bool f32 = j.prec == kCnnF32;
  const bool split = j.prec == kCnnBf16x2;
  // weight / bias offsets of layer l in the concatenated arrays
  auto woff = [&](int l) {
    int64_t o = 0;
    for (int i = 0; i < l; ++i) o += (int64_t)(i == 0 ? 1 : C) * (i == L - 1 ? 1 : C) * 9;
    return o;
  };
  auto boff = [&](int l) { return (int64_t)l * C; };
  const dim3 g16((unsigned)(j.nfields * tiles16)), b256(256);

  if (f32) {
    float* a0 = (float*)j.ws.act[0];
    float* a1 = (float*)j.ws.act[1];
    k_cnn_first<C, float><<<g16, b256, 0, st>>>(j.in_base, j.in_offs, n, j.W, j.B, j.act, a0,
                                                nullptr);
    for (int l = 1; l < L - 1; ++l) {
      if constexpr (C >= 16) {
        k_cnn_hidden_f32<C><<<g16, b256, 0, st>>>(a0, n, j.W + woff(l), j.B + boff(l), j.act, a1);
      } else {
        return hipErrorInvalidValue;
      }
      std::swap(a0, a1);
    }
    k_cnn_last<C, float><<<g16, b256, 0, st>>>(a0, nullptr, n, j.W + woff(L - 1),
                                               j.B + boff(L - 1), j.in_base, j.in_offs,
                                               j.out_base, j.out_offs, j.residual,
                                               j.ws.partials);
  } else {
    __bf16* a0 = (__bf16*)j.ws.act[0];
    __bf16* a1 = (__bf16*)j.ws.act[1];
    __bf16* l0 = split ? a0 + act_elems : nullptr;
    __bf16* l1 = split ? a1 + act_elems : nullptr;
    k_cnn_first<C, __bf16><<<g16, b256, 0, st>>>(j.in_base, j.in_offs, n, j.W, j.B, j.act, a0, l0);
    for (int l = 1; l < L - 1; ++l) {
      if constexpr (C % 16 == 0) {
        using H = HidCfg<C>;
        const __bf16* wp = (const __bf16*)j.ws.wpack + (int64_t)(l - 1) * C * H::KP;
        const size_t lds = cnn_lds_bytes(C, split);
        const int64_t tiles = j.nfields * (n / H::TH) * (n / H::TW);
        static const int cap0 = hidden_cap<C, false>(), cap1 = hidden_cap<C, true>();
        const dim3 gh((unsigned)std::min<int64_t>(tiles, split ? cap1 : cap0)), bh(H::NT);
        if (split)
          k_cnn_hidden<C, true><<<gh, bh, lds, st>>>(a0, l0, n, j.nfields, wp, j.B + boff(l), j.act,
                                                     a1, l1);
        else
          k_cnn_hidden<C, false><<<gh, bh, lds, st>>>(a0, nullptr, n, j.nfields, wp, j.B + boff(l),
                                                      j.act, a1, nullptr);
      } else {
        return hipErrorInvalidValue;
      }
      std::swap(a0, a1);
      std::swap(l0, l1);
    }
    k_cnn_last<C, __bf16><<<g16, b256, 0, st>>>(a0, l0, n, j.W + woff(L - 1), j.B + boff(L - 1),
                                                j.in_base, j.in_offs, j.out_base, j.out_offs,
                                                j.residual, j.ws.partials);
  }
  if (j.mass_fix || j.limiter) {
    const int bpf = (int)std::max<int64_t>(1, (int64_t)n * n / 2048);
    k_cnn_fix<<<dim3((unsigned)(j.nfields * bpf)), b256, 0, st>>>(
        j.out_base, j.out_offs, n, j.ws.partials, (int)tiles16, j.mass_fix, j.limiter, j.lim_lo,
        j.lim_hi, bpf);
  }
  return hipGetLastError();
}

hipError_t launch_cnn_pack(const CnnJob& j, hipStream_t st) {
  if (j.prec == kCnnF32 || j.n_layers < 3) return hipSuccess;
  const int C = j.channels, L = j.n_layers;
  const int kp = (9 * C + 31) / 32 * 32;
  int64_t wo = (int64_t)C * 9;  // layer 0 is 1 -> C
  for (int l = 1; l < L - 1; ++l) {
    const int64_t cnt = (int64_t)C * kp;
    k_cnn_pack<<<dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st>>>(
        j.W + wo, C, C, kp, (__bf16*)j.ws.wpack + (int64_t)(l - 1) * C * kp);
    wo += (int64_t)C * C * 9;
  }
  return hipGetLastError();
}

hipError_t launch_cnn(const CnnJob& j, hipStream_t st) {
  if (j.nfields <= 0) return hipSuccess;
  switch (j.channels) {
    case 8: return launch_cnn_c<8>(j, st);
    case 16: return launch_cnn_c<16>(j, st);
    case 32: return launch_cnn_c<32>(j, st);
    case 48: return launch_cnn_c<48>(j, st);
    case 64: return launch_cnn_c<64>(j, st);
    default: return hipErrorInvalidValue;
  }
}

size_t cnn_lds_bytes(int C, bool split) {
  switch (C) {
#define PR_L(CC)                                                                               \
  case CC:                                                                                     \
    return ((split ? 2 : 1) * (HidCfg<CC>::TPIX * HidCfg<CC>::CS +                             \
                               HidCfg<CC>::NW * 16 * HidCfg<CC>::OS)) * 2;
    PR_L(16) PR_L(32) PR_L(48) PR_L(64)
#undef PR_L
    default: return 0;
  }
}

hipError_t cnn_set_lds_limits() {
  // raise the dynamic-LDS limit of each hidden-layer kernel to what it
  // uses; configurations beyond the 160 KB of a CU are rejected earlier
  constexpr size_t kMaxLds = 160 * 1024;
  hipError_t e = hipSuccess;
#define PR_A(CC, SP)                                                                         \
  if (e == hipSuccess && cnn_lds_bytes(CC, SP) <= kMaxLds)                                   \
    e = hipFuncSetAttribute((const void*)k_cnn_hidden<CC, SP>,                               \
                            hipFuncAttributeMaxDynamicSharedMemorySize,                      \
                            (int)cnn_lds_bytes(CC, SP));
  PR_A(16, false) PR_A(16, true) PR_A(32, false) PR_A(32, true)
  PR_A(48, false) PR_A(48, true) PR_A(64, false) PR_A(64, true)
#undef PR_A
  return e;
}

}  // namespace pr
