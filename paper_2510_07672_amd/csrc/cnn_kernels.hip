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

template <int C, typename TO>
__global__ __launch_bounds__(256) void k_cnn_first(const double* __restrict__ u_base,
                                                   const int64_t* __restrict__ u_offs, int n,
                                                   const float* __restrict__ W,
                                                   const float* __restrict__ b, int act,
                                                   TO* __restrict__ out, TO* __restrict__ out_lo) {
  __shared__ float sw[C * 9], sb[C];
  __shared__ float tile[(kTile + 2) * (kTile + 2)];
  const int tid = threadIdx.x;
  const int tpr = n / kTile;
  const int64_t f = blockIdx.x / (tpr * tpr);
  const int t = (int)(blockIdx.x % (tpr * tpr));
  const int y0 = (t / tpr) * kTile, x0 = (t % tpr) * kTile;
  const double* u = u_base + (u_offs ? u_offs[f] : f * (int64_t)n * n);
  for (int i = tid; i < C * 9; i += 256) sw[i] = W[i];
  for (int i = tid; i < C; i += 256) sb[i] = b[i];
  for (int i = tid; i < (kTile + 2) * (kTile + 2); i += 256) {
    const int ty = i / (kTile + 2), tx = i % (kTile + 2);
    const int gy = (y0 + ty - 1 + n) % n, gx = (x0 + tx - 1 + n) % n;
    tile[i] = (float)u[(int64_t)gy * n + gx];
  }
  __syncthreads();
  const int py = tid / kTile, px = tid % kTile;
  float v[9];
#pragma unroll
  for (int tp = 0; tp < 9; ++tp) v[tp] = tile[(py + tp / 3) * (kTile + 2) + px + tp % 3];
  const int64_t o = ((f * n + y0 + py) * (int64_t)n + x0 + px) * C;
#pragma unroll 4
  for (int co = 0; co < C; ++co) {
    float s = sb[co];
#pragma unroll
    for (int tp = 0; tp < 9; ++tp) s += sw[co * 9 + tp] * v[tp];
    store_act(out, out_lo, o + co, act_fn(s, act));
  }
}

// ----------------------------------------------------------- hidden layers

template <int C> struct HidCfg {
  static constexpr int TH = 8, TW = 32;              // output tile (rows, columns)
  static constexpr int NW = 4, NT = 64 * NW;         // waves, threads
  static constexpr int CS = C + 8;                   // LDS pixel stride (elements)
  static constexpr int KP = (9 * C + 31) / 32 * 32;  // K padded to the MFMA depth
  static constexpr int KS = KP + 8;                  // LDS weight-row stride
  static constexpr int MB = TH * TW / 16;            // 16-pixel blocks per tile
  static constexpr int MBW = MB / NW;                // per wave
  static constexpr int NB = C / 16;                  // 16-channel blocks
  static constexpr int KB = KP / 32;                 // K steps
  static constexpr int TPIX = (TH + 2) * (TW + 2);
};

template <int C, bool SPLIT>
__global__ __launch_bounds__(HidCfg<C>::NT) void k_cnn_hidden(
    const __bf16* __restrict__ in, const __bf16* __restrict__ in_lo, int n,
    const __bf16* __restrict__ Wp, const float* __restrict__ b, int act,
    __bf16* __restrict__ out, __bf16* __restrict__ out_lo) {
  using H = HidCfg<C>;
  static_assert(C % 16 == 0, "hidden width must be a multiple of 16");
  extern __shared__ __align__(16) unsigned char smem[];
  __bf16* tile = (__bf16*)smem;                                 // [TPIX][CS]
  __bf16* tile_lo = tile + H::TPIX * H::CS;                     // SPLIT only
  __bf16* wl = tile + (SPLIT ? 2 : 1) * H::TPIX * H::CS;        // [C][KS]
  __shared__ float sb[C];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tpy = n / H::TH, tpx = n / H::TW;
  const int64_t f = blockIdx.x / (tpy * tpx);
  const int t = (int)(blockIdx.x % (tpy * tpx));
  const int y0 = (t / tpx) * H::TH, x0 = (t % tpx) * H::TW;

  // weights and bias
  constexpr int WCH = C * H::KP / 8;
  for (int i = tid; i < WCH; i += H::NT) {
    const int co = i / (H::KP / 8), k8 = i % (H::KP / 8);
    *(bf16x8*)&wl[co * H::KS + k8 * 8] = *(const bf16x8*)&Wp[(int64_t)co * H::KP + k8 * 8];
  }
  for (int i = tid; i < C; i += H::NT) sb[i] = b[i];
  // input tile with a one-pixel periodic halo
  constexpr int TCH = H::TPIX * (C / 8);
  for (int i = tid; i < TCH; i += H::NT) {
    const int p = i / (C / 8), c8 = i % (C / 8);
    const int ty = p / (H::TW + 2), tx = p % (H::TW + 2);
    const int gy = (y0 + ty - 1 + n) % n, gx = (x0 + tx - 1 + n) % n;
    const int64_t g = ((f * n + gy) * (int64_t)n + gx) * C + c8 * 8;
    *(bf16x8*)&tile[p * H::CS + c8 * 8] = *(const bf16x8*)&in[g];
    if constexpr (SPLIT) *(bf16x8*)&tile_lo[p * H::CS + c8 * 8] = *(const bf16x8*)&in_lo[g];
  }
  __syncthreads();

  f32x4 acc[H::MBW][H::NB];
#pragma unroll
  for (int m = 0; m < H::MBW; ++m)
#pragma unroll
    for (int nb = 0; nb < H::NB; ++nb) acc[m][nb] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int r = lane & 15, g = lane >> 4;
  for (int kb = 0; kb < H::KB; ++kb) {
    const int k0 = kb * 32 + 8 * g;
    bf16x8 bfr[H::NB];
#pragma unroll
    for (int nb = 0; nb < H::NB; ++nb) bfr[nb] = *(const bf16x8*)&wl[(nb * 16 + r) * H::KS + k0];
    const bool live = k0 < 9 * C;
    const int tap = live ? k0 / C : 0, ci0 = live ? k0 % C : 0;
    const int ky = tap / 3, kx = tap % 3;
#pragma unroll
    for (int m = 0; m < H::MBW; ++m) {
      const int mb = wave * H::MBW + m;
      const int oy = mb / (H::TW / 16), ox0 = (mb % (H::TW / 16)) * 16;
      const int a_off = ((oy + ky) * (H::TW + 2) + ox0 + r + kx) * H::CS + ci0;
      bf16x8 afr = *(const bf16x8*)&tile[a_off];
      if (!live) afr = bf16x8{};
#pragma unroll
      for (int nb = 0; nb < H::NB; ++nb)
        acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr, bfr[nb], acc[m][nb], 0, 0, 0);
      if constexpr (SPLIT) {
        bf16x8 alo = *(const bf16x8*)&tile_lo[a_off];
        if (!live) alo = bf16x8{};
#pragma unroll
        for (int nb = 0; nb < H::NB; ++nb)
          acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bfr[nb], acc[m][nb], 0, 0, 0);
      }
    }
  }

  // bias, activation, store: lane holds pixels 4 g + i of the block, channel r
#pragma unroll
  for (int m = 0; m < H::MBW; ++m) {
    const int mb = wave * H::MBW + m;
    const int oy = mb / (H::TW / 16), ox0 = (mb % (H::TW / 16)) * 16;
#pragma unroll
    for (int nb = 0; nb < H::NB; ++nb) {
      const int co = nb * 16 + r;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int x = x0 + ox0 + 4 * g + i;
        const int64_t o = ((f * n + y0 + oy) * (int64_t)n + x) * C + co;
        store_act<__bf16>(out, SPLIT ? out_lo : nullptr, o, act_fn(acc[m][nb][i] + sb[co], act));
      }
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
    const int gy = (y0 + ty - 1 + n) % n, gx = (x0 + tx - 1 + n) % n;
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

template <int C, typename TI>
__global__ __launch_bounds__(256) void k_cnn_last(
    const TI* __restrict__ in, const TI* __restrict__ in_lo, int n, const float* __restrict__ W,
    const float* __restrict__ b, const double* __restrict__ u_base,
    const int64_t* __restrict__ u_offs, double* __restrict__ g_base,
    const int64_t* __restrict__ g_offs, int residual, double* __restrict__ partials) {
  __shared__ float tile[(kTile + 2) * (kTile + 2) * (C + 1)];
  __shared__ float sw[C * 9];
  __shared__ double red[4];
  const int tid = threadIdx.x;
  const int tpr = n / kTile;
  const int64_t f = blockIdx.x / (tpr * tpr);
  const int t = (int)(blockIdx.x % (tpr * tpr));
  const int y0 = (t / tpr) * kTile, x0 = (t % tpr) * kTile;
  for (int i = tid; i < C * 9; i += 256) sw[i] = W[i];
  for (int i = tid; i < (kTile + 2) * (kTile + 2) * C; i += 256) {
    const int p = i / C, c = i % C;
    const int ty = p / (kTile + 2), tx = p % (kTile + 2);
    const int gy = (y0 + ty - 1 + n) % n, gx = (x0 + tx - 1 + n) % n;
    const int64_t g = ((f * n + gy) * (int64_t)n + gx) * C + c;
    float v = to_f(in[g]);
    if (in_lo) v += to_f(in_lo[g]);
    tile[p * (C + 1) + c] = v;
  }
  __syncthreads();
  const int py = tid / kTile, px = tid % kTile;
  float s = b[0];
  for (int tp = 0; tp < 9; ++tp) {
    const int p = (py + tp / 3) * (kTile + 2) + px + tp % 3;
#pragma unroll 8
    for (int ci = 0; ci < C; ++ci) s += sw[ci * 9 + tp] * tile[p * (C + 1) + ci];
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
        const size_t lds = ((split ? 2 : 1) * H::TPIX * H::CS + C * H::KS) * sizeof(__bf16);
        const dim3 gh((unsigned)(j.nfields * (n / H::TH) * (n / H::TW))), bh(H::NT);
        if (split)
          k_cnn_hidden<C, true><<<gh, bh, lds, st>>>(a0, l0, n, wp, j.B + boff(l), j.act, a1, l1);
        else
          k_cnn_hidden<C, false><<<gh, bh, lds, st>>>(a0, nullptr, n, wp, j.B + boff(l), j.act, a1,
                                                      nullptr);
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
    return ((split ? 2 : 1) * HidCfg<CC>::TPIX * HidCfg<CC>::CS + CC * HidCfg<CC>::KS) * 2;
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
