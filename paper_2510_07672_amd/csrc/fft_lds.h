// Device building blocks: complex arithmetic, radix-2/4/8 butterflies, a
// batched Stockham FFT over lines held in LDS, and block reductions.
//
// The 2-D solve of the semi-implicit step (a real 2-D DFT, a division by
// the symbol of ((1 + S dt) I - dt eps^2 Lap_h), and the inverse DFT) is
// built from these length-N complex transforms.
//
// FFT scheme.  N = 8^a * {1, 2, 4}; stages run radix 8 first and the
// leftover 2 or 4 last.  Each stage is the self-sorting Stockham step: for
// butterfly j of a line (j < N/R) the R inputs sit at j + r N/R, are
// multiplied by w^(r k), k = j mod Ns (Ns = product of earlier radices,
// w = exp(sign 2 pi i / (Ns R))), transformed by a radix-R DFT, and land at
// (j / Ns) Ns R + k + r Ns.  Output is in natural order after the last
// stage.  The transform is in place in LDS: every thread reads its eight
// elements into registers, the block synchronises, then every thread
// writes.  So a block of NT threads handles NT * 8 complex elements at a
// time, and the panel it works on must hold exactly that many.
//
// The first stage may take its inputs from a prologue functor instead of
// LDS (e.g. straight from global memory, whose addresses j + r N/R are
// consecutive across threads), and the last stage may hand its outputs to
// an epilogue functor that either modifies them before the LDS write or
// stores them to global memory itself (addresses j + r N/R again).
//
// LDS layout.  Element e of line l sits at l * LS + e + e / 8: one pad slot
// after every eight elements, so the stride-8 writes of the first stage
// and the stride-LS accesses across lines (LS odd) spread over the banks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace pr {

template <typename T> struct cpx_sel;
template <> struct cpx_sel<float> { using type = float2; };
template <> struct cpx_sel<double> { using type = double2; };
template <typename T> using cpx = typename cpx_sel<T>::type;

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// multiply by sign * i
template <int SIGN, typename C> __device__ __forceinline__ C cmul_i(C a) {
  if constexpr (SIGN > 0) return C{-a.y, a.x};
  else return C{a.y, -a.x};
}

template <int SIGN, typename C>
__device__ __forceinline__ void dft2(C& a, C& b) {
  C t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <int SIGN, typename C>
__device__ __forceinline__ void dft4(C& v0, C& v1, C& v2, C& v3) {
  C t0 = cadd(v0, v2), t1 = csub(v0, v2), t2 = cadd(v1, v3);
  C t3 = cmul_i<SIGN>(csub(v1, v3));
  v0 = cadd(t0, t2);
  v2 = csub(t0, t2);
  v1 = cadd(t1, t3);
  v3 = csub(t1, t3);
}

template <int SIGN, typename C>
__device__ __forceinline__ void dft8(C* v) {
  using T = decltype(v[0].x);
  C e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  C o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<SIGN>(e0, e1, e2, e3);
  dft4<SIGN>(o0, o1, o2, o3);
  const T c = (T)0.70710678118654752440;
  const T s = (T)SIGN;
  // o_k *= exp(sign 2 pi i k / 8)
  o1 = C{c * (o1.x - s * o1.y), c * (o1.y + s * o1.x)};
  o2 = cmul_i<SIGN>(o2);
  o3 = C{-c * (o3.x + s * o3.y), c * (s * o3.x - o3.y)};
  v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
}

template <int R, int SIGN, typename C>
__device__ __forceinline__ void dft_r(C* v) {
  if constexpr (R == 8) dft8<SIGN>(v);
  else if constexpr (R == 4) dft4<SIGN>(v[0], v[1], v[2], v[3]);
  else if constexpr (R == 2) dft2<SIGN>(v[0], v[1]);
}

// One pad slot after every 2^PR_PAD_SHIFT elements of a line.
#ifndef PR_PAD_SHIFT
#define PR_PAD_SHIFT 3
#endif

// Padded line stride for lines of N elements: N + N/2^SH pad slots, made
// odd.
template <int N, int SH = PR_PAD_SHIFT> struct PadLS {
  static constexpr int value = N + (N >> SH) + 1;
};

// Panel layout: element e of line l at l * LS + e + (e >> SH).
template <int LS, int SH = PR_PAD_SHIFT> struct LinePanel {
  __device__ __forceinline__ int operator()(int line, int e) const {
    return line * LS + e + (e >> SH);
  }
};

// Twiddles.  Stage (Ns, R) needs w^(r k) = exp(-2 pi i r k / (Ns R)) for
// r = 1..R-1, k = 0..Ns-1.  They are kept per stage as [r-1][k], so the
// lanes of a wave (consecutive k) read consecutive entries.
// Radix split: the radix of the stage that follows Ns.
//   RS = 0: 8 while it fits, the leftover 2 or 4 last (N = 8^a * {1, 2, 4}).
//   RS = 1: the same, except that a trailing 8 x 2 becomes 4 x 4, so that
//           N = 8^a * 2 (16, 128, 1024) has no radix-2 stage; the other N
//           have no such split and take RS = 0's stages.
// Both take the fewest stages (LDS round trips) a thread's 8 elements
// allow; which is faster is measured (pr_autotune_fine).  (The leftover
// first measured 1.2-1.6x slower per step: a radix-2 or -4 first stage
// gives each thread two or four butterflies of strided global loads.)
template <int N, int RS = 0> constexpr int stage_radix(int ns) {
  return (RS == 1 && N / ns == 16) ? 4 : (N / ns) >= 8 ? 8 : N / ns;
}
// Whether RS = 1 differs from RS = 0 for length N.
template <int N> constexpr bool radix_split_differs() {
  int l = 0;
  while ((1 << l) < N) ++l;
  return N >= 16 && l % 3 == 1;   // N = 8^a * 2, a >= 1
}
static_assert(radix_split_differs<16>() && radix_split_differs<128>() &&
                  radix_split_differs<1024>() && !radix_split_differs<256>() &&
                  !radix_split_differs<512>() && !radix_split_differs<64>() &&
                  !radix_split_differs<32>(),
              "radix splits");

template <int N, int RS = 0> constexpr int tw_offset(int ns_target) {
  int off = 0;
  for (int ns = 1; ns < ns_target; ns *= stage_radix<N, RS>(ns))
    if (ns > 1) off += (stage_radix<N, RS>(ns) - 1) * ns;
  return off;
}

template <int N, int RS = 0> struct TwSize {
  static constexpr int value = tw_offset<N, RS>(N) > 0 ? tw_offset<N, RS>(N) : 1;
};

// Compact table: per stage only the r = 1 row, w^k for k < Ns; the other
// powers are formed by repeated multiplication in the butterfly (R - 2
// complex products, a few ulps of extra rounding).  Stages with Ns > 64
// store that row factored, w^k = w^(8 (k / 8)) w^(k % 8): Ns / 8 + 8
// entries and one more product.  Passed to the transforms wrapped in
// TwPow, so that the stage code selects the form.
constexpr int tw_pow_rows(int ns) { return ns > 64 ? ns / 8 + 8 : ns; }
template <int N, int RS = 0> constexpr int tw_offset_pow(int ns_target) {
  int off = 0;
  for (int ns = 1; ns < ns_target; ns *= stage_radix<N, RS>(ns))
    if (ns > 1) off += tw_pow_rows(ns);
  return off;
}
template <int N, int RS = 0> struct TwSizePow {
  static constexpr int value = tw_offset_pow<N, RS>(N) > 0 ? tw_offset_pow<N, RS>(N) : 1;
};
template <typename C> struct TwPow {
  const C* p;
};

// Fill the per-stage table from g[t] = exp(-2 pi i t / N).  The caller
// synchronises the block before the first transform.
template <int N, int NT, int RS = 0, typename C>
__device__ __forceinline__ void load_stage_twiddles(C* tw, const C* g, int tid) {
  for (int ns = 1; ns < N; ns *= stage_radix<N, RS>(ns)) {
    const int R = stage_radix<N, RS>(ns);
    if (ns == 1) continue;
    const int off = tw_offset<N, RS>(ns), cnt = (R - 1) * ns;
    for (int i = tid; i < cnt; i += NT) {
      const int r = i / ns + 1, k = i % ns;
      tw[off + i] = g[r * k * (N / (ns * R))];
    }
  }
}

// Pad shift of a transform block's panel of LINES lines of N elements of
// ESIZE bytes (line stride N + N/2^sh + PLUS), next to OTHER further bytes
// of LDS, for THREADS threads: one pad slot per 8 elements, or one per 16
// where that lets more blocks share a CU (160 KB of LDS, 2048 threads).
// Only for 16-byte elements: a wave's 16-byte accesses are served 8 lanes
// at a time from 16 bank quads, and the first stage's stride-8 writes,
// whose lane-to-lane slot distances then alternate 8 and 9, still hit
// distinct quads.
template <int N, int LINES, int ESIZE, int OTHER, int PLUS, int THREADS> struct LdsPlan {
  static constexpr int fit(int sh) {
    const int b = LINES * (N + (N >> sh) + PLUS) * ESIZE + OTHER;
    const int by_lds = 160 * 1024 / b, by_threads = 2048 / THREADS;
    return by_lds < by_threads ? by_lds : by_threads;
  }
  static constexpr bool k16 = ESIZE == 16 && PR_PAD_SHIFT == 3;
  static constexpr int SH = k16 && fit(4) > fit(PR_PAD_SHIFT) ? 4 : PR_PAD_SHIFT;
  static constexpr int FIT = fit(SH);  // blocks per CU
};

// Fill the compact table: stage (Ns, R) gets w^k = g[k N / (Ns R)], k < Ns
// (factored into w^(8a), a < Ns / 8, and w^b, b < 8, when Ns > 64).
template <int N, int NT, int RS = 0, typename C>
__device__ __forceinline__ void load_stage_twiddles_pow(C* tw, const C* g, int tid) {
  for (int ns = 1; ns < N; ns *= stage_radix<N, RS>(ns)) {
    const int R = stage_radix<N, RS>(ns);
    if (ns == 1) continue;
    const int off = tw_offset_pow<N, RS>(ns), stride = N / (ns * R);
    if (ns > 64) {
      for (int a = tid; a < ns / 8; a += NT) tw[off + a] = g[8 * a * stride];
      for (int b = tid; b < 8; b += NT) tw[off + ns / 8 + b] = g[b * stride];
    } else {
      for (int k = tid; k < ns; k += NT) tw[off + k] = g[k * stride];
    }
  }
}

// The twiddle source of a block: the full per-stage table, or the compact
// one wrapped in TwPow.
template <bool POW, typename C>
__device__ __forceinline__ auto twiddle_source(const C* tw) {
  if constexpr (POW) return TwPow<C>{tw};
  else return tw;
}

// Hooks.  A prologue provides `C load(int i, int line, int e)` for the
// first stage's i-th input of this thread (line `line`, element `e`) and
// `void after_reads()`, called once all of them have been taken; an
// epilogue provides `void apply(int line, int e, C& v)` and a constexpr
// kWritesLds telling whether the (possibly modified) value is still
// written to LDS afterwards.
struct NoPro {};
struct NoEpi {
  static constexpr bool kWritesLds = true;
};

// One Stockham stage over the panel.  tw gives the forward twiddles (the
// per-stage table of load_stage_twiddles, or TwPow over the compact one);
// SIGN = -1 forward,
// +1 inverse.  Each of the NT threads owns
// G groups of eight elements.
template <int N, int R, int NS, int SIGN, int NT, int G, bool LF, typename T, int RS, class TW,
          class Lay, class Pro, class Epi>
__device__ __forceinline__ void fft_stage(cpx<T>* buf, TW tw, Lay lay, int tid, Pro& pro,
                                          Epi& epi) {
  constexpr int NB = N / R;        // butterflies per line
  constexpr int BPT = G * 8 / R;   // butterflies per thread
  constexpr int LINES = NT * G * 8 / N;
  constexpr bool kFirst = NS == 1;
  constexpr bool kLast = NS * R == N;
  constexpr bool kFromPro = kFirst && !std::is_same<Pro, NoPro>::value;
  constexpr bool kToLds = !kLast || Epi::kWritesLds;
  cpx<T> v[8 * G];
  int line[BPT], jj[BPT];
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int b = tid + q * NT;
    line[q] = LF ? b % LINES : b / NB;
    jj[q] = LF ? b / LINES : b % NB;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if constexpr (kFromPro) v[q * R + r] = pro.load(q * R + r, line[q], jj[q] + r * NB);
      else v[q * R + r] = buf[lay(line[q], jj[q] + r * NB)];
    }
  }
  if constexpr (kFromPro) pro.after_reads();
  if constexpr (kToLds) __syncthreads();
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int k = jj[q] % NS;
    if constexpr (NS > 1) {
      if constexpr (std::is_same<TW, TwPow<cpx<T>>>::value) {
        constexpr int off = tw_offset_pow<N, RS>(NS);
        cpx<T> w1;
        if constexpr (NS > 64) w1 = cmul(tw.p[off + k / 8], tw.p[off + NS / 8 + k % 8]);
        else w1 = tw.p[off + k];
        if constexpr (SIGN > 0) w1.y = -w1.y;
        cpx<T> w = w1;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          v[q * R + r] = cmul(v[q * R + r], w);
          if (r + 1 < R) w = cmul(w, w1);
        }
      } else {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cpx<T> w = tw[tw_offset<N, RS>(NS) + (r - 1) * NS + k];
          if constexpr (SIGN > 0) w.y = -w.y;
          v[q * R + r] = cmul(v[q * R + r], w);
        }
      }
    }
    dft_r<R, SIGN>(&v[q * R]);
    const int base = (jj[q] / NS) * NS * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if constexpr (kLast && !std::is_same<Epi, NoEpi>::value) epi.apply(line[q], base + r * NS, v[q * R + r]);
      if constexpr (kToLds) buf[lay(line[q], base + r * NS)] = v[q * R + r];
    }
  }
  if constexpr (kToLds) __syncthreads();
}

template <int N, int NS, int SIGN, int NT, int G, bool LF, typename T, int RS, class TW, class Lay,
          class Pro, class Epi>
__device__ __forceinline__ void fft_from(cpx<T>* buf, TW tw, Lay lay, int tid, Pro& pro, Epi& epi) {
  if constexpr (NS < N) {
    constexpr int R = stage_radix<N, RS>(NS);
    fft_stage<N, R, NS, SIGN, NT, G, LF, T, RS>(buf, tw, lay, tid, pro, epi);
    fft_from<N, NS * R, SIGN, NT, G, LF, T, RS>(buf, tw, lay, tid, pro, epi);
  }
}

// Unnormalised length-N DFT of every line in the panel, in place.
// Requires NT * 8 * G == (number of lines) * N.  Unless a prologue
// supplies the inputs, `buf` must be complete (synchronised) on entry.  On
// exit the block is synchronised if the last stage wrote LDS.  Butterfly b
// of a stage belongs to line b / (N/R), position b % (N/R) (a line's
// elements in consecutive lanes) or, with LF, to line b % lines, position
// b / lines (the lines in consecutive lanes).
template <int N, int SIGN, int NT, typename T, int G = 1, bool LF = false, int RS = 0, class TW,
          class Lay, class Pro = NoPro, class Epi = NoEpi>
__device__ __forceinline__ void fft_lines(cpx<T>* buf, TW tw, Lay lay, int tid, Pro pro = Pro{},
                                          Epi epi = Epi{}) {
  fft_from<N, 1, SIGN, NT, G, LF, T, RS>(buf, tw, lay, tid, pro, epi);
}

// Deterministic block sum of one double per thread (fixed tree order).
// `red` is LDS scratch of at least NT/64 + 1 doubles.  Result valid in
// thread 0.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red, int tid) {
  constexpr int W = NT < 64 ? NT : 64;
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
  if constexpr (NT <= 64) {
    return v;
  } else {
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (tid == 0) {
#pragma unroll
      for (int w = 0; w < NT / 64; ++w) s += red[w];
    }
    __syncthreads();
    return s;
  }
}

}  // namespace pr
