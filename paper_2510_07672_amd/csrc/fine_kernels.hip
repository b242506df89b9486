// HIP kernels of the fine propagator (the stabilised semi-implicit step,
// Section 3.1 / eq. fine_operator), the Parareal correction and its norm
// (Section 3.3, Algorithm 2).
//
// One step maps u to u+ with
//     ((1 + S dt) I - dt eps^2 Lap_h) u+ = (1 + S dt) u + dt (f(u) - m),
// f(u) = u - u^3, m = 0 (classic) or the grid mean of f(u) (conservative).
// In Fourier space the operator is the scalar (1 + S dt) + dt eps^2 mu_k,
// mu_k = (4/h^2)(sin^2(pi kx/N) + sin^2(pi ky/N)) (5-point stencil).
//
// Spectral layout of a field between passes ("row spectra, column-major"):
// R_r[kx] is the length-N DFT of real row r.  Only kx = 0..N/2 is kept;
// columns kx = 1..N/2-1 are stored as complex column c = kx, and the two
// real columns kx = 0 and kx = N/2 share column c = 0 as R_r[0] + i R_r[N/2].
// So a field is N/2 columns of N complex values, spec[c][r], contiguous per
// column: exactly N*N real numbers.
//
// Row pass   (one block per tile of TR rows of one field): rows 2j and 2j+1
//   are carried as one complex row z = row_2j + i row_2j+1.  Rebuild Z from
//   the stored half spectra, inverse FFT, apply the pointwise right-hand
//   side r = (1 + S dt) v + dt f(v) (and sum f(v) in FP64 for the mass
//   multiplier), forward FFT, split Z back into R_2j and R_2j+1, store.
// Column pass (one block per CT columns of one field): forward column FFT,
//   multiply by 1 / (N^2 ((1 + S dt) + dt eps^2 mu_k)) (the 1/N^2 undoes
//   both unnormalised inverse transforms), subtract dt * sum f from the DC
//   bin in the conservative model (dt * N^2 * m), inverse column FFT.
// The first row pass reads the real state instead of spectra; the last
// writes the real state and does no forward transform.  Each step is one
// column pass plus one row pass: two read+write sweeps of the field.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <vector>

#include "fft_lds.h"
#include "internal.h"

// Whether the column passes stage the symbol table in LDS (1) or read it
// from global memory through the cache (0).
#ifndef PR_S2_LDS
#define PR_S2_LDS 0
#endif

namespace pr {

// ------------------------------------------------------------------ tables

// Twiddles exp(-2 pi i t / N) and the per-axis symbol table s2: the
// symbol of the discrete Laplacian is -(4/h^2)(s2[kx] + s2[ky]) with
// s2[t] = sin^2(pi t / N) for the 5-point stencil and (pi t~ / N)^2,
// t~ = min(t, N - t), for Fourier collocation ((4/h^2)(pi t~/N)^2 =
// (2 pi t~ / L)^2).
__global__ void k_tables(int n, int laplacian, double2* tw64, float2* tw32, double* s2) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) {
    double s, c;
    sincospi(2.0 * (double)t / (double)n, &s, &c);
    tw64[t] = double2{c, -s};
    tw32[t] = float2{(float)c, (float)-s};
    if (laplacian == LAP_SPECTRAL) {
      const double k = 3.141592653589793 * (double)(t <= n - t ? t : n - t) / (double)n;
      s2[t] = k * k;
    } else {
      const double sn = sinpi((double)t / (double)n);
      s2[t] = sn * sn;
    }
  }
}

// The thread index, made opaque to the optimiser.  Used at the top of a
// loop over steps or tiles so that the address arithmetic of the unrolled
// FFT stages is recomputed per iteration instead of being hoisted out of
// the loop and held in registers for its whole length.
__device__ __forceinline__ int opaque_tid(int tid) {
  asm volatile("" : "+v"(tid));
  return tid;
}

// ------------------------------------------------------- spectral layout
//
// A field's half spectrum (N/2 columns kx of N rows ky, complex) is stored
// in blocks of W columns, row-major inside a block: (c, r) at
// (c / W) N W + r W + c % W.  W = 1 is plain column-major.  At N >= 1024,
// W = ColCfg<N>::CT: a column tile is then one contiguous block and a row
// tile reads TR W consecutive values per block instead of TR (measured
// faster there; at N <= 512 the column pass lost more than the row pass
// gained).  The column transforms then put a tile's lines in consecutive
// lanes (fft_lines' LF), so that their global loads and stores run along
// the block.
template <int N> struct SpecLayout {
  static constexpr int W = N >= 1024 ? ColCfg<N>::CT : 1;
  static constexpr bool LF = W > 1;
};
template <int N> __device__ __forceinline__ int64_t spec_at(int c, int r) {
  constexpr int W = SpecLayout<N>::W;
  return (int64_t)(c / W) * N * W + (int64_t)r * W + (c % W);
}
// Offset of (line, e) from the start of a column tile (W divides CT).
template <int N> __device__ __forceinline__ int64_t col_at(int line, int e) {
  constexpr int W = SpecLayout<N>::W;
  return (int64_t)(line / W) * N * W + (int64_t)e * W + (line % W);
}
// Entry e of a row tile's (pair, column) loops: W consecutive columns in
// consecutive lanes, then the pairs, then the column blocks.
template <int N, int PAIRS> __device__ __forceinline__ void row_entry(int e, int& p, int& c) {
  constexpr int W = SpecLayout<N>::W;
  p = (e / W) % PAIRS;
  c = (e / (W * PAIRS)) * W + e % W;
}

// --------------------------------------------------------------- row pass

// What the row pass transforms, on the two rows carried by one complex
// value: the semi-implicit right-hand side r = (1 + S dt) v + dt f(v) (f
// also summed in FP64 for the mass multiplier), f(v), or v.
template <int RHS, typename T>
__device__ __forceinline__ cpx<T> rhs_pair(cpx<T> z, T a, T dt, double& fsum) {
  if constexpr (RHS == RHS_U) {
    return z;
  } else {
    const T f0 = z.x - z.x * z.x * z.x, f1 = z.y - z.y * z.y * z.y;
    if constexpr (RHS == RHS_F) {
      return cpx<T>{f0, f1};
    } else {
      fsum += (double)f0 + (double)f1;
      return cpx<T>{a * z.x + dt * f0, a * z.y + dt * f1};
    }
  }
}

// First forward stage reads rows r0+2p and r0+2p+1 of the real FP64 state,
// rounds them to T and forms the right-hand side.
template <int N, typename T, int RHS = RHS_SSI> struct RealRowsPro {
  const double* u;
  int r0;
  T a, dt;
  double* fsum;
  __device__ __forceinline__ cpx<T> load(int, int p, int x) const {
    const cpx<T> z{(T)u[(int64_t)(r0 + 2 * p) * N + x], (T)u[(int64_t)(r0 + 2 * p + 1) * N + x]};
    return rhs_pair<RHS, T>(z, a, dt, *fsum);
  }
  __device__ __forceinline__ void after_reads() const {}
};

// Last inverse stage: right-hand side of the next step, kept in LDS.
template <typename T, int RHS = RHS_SSI> struct RhsEpi {
  static constexpr bool kWritesLds = true;
  T a, dt;
  double* fsum;
  __device__ __forceinline__ void apply(int, int, cpx<T>& v) const {
    v = rhs_pair<RHS, T>(v, a, dt, *fsum);
  }
};

// Last inverse stage: the two real rows go straight to the output state.
template <int N, typename T> struct RealRowsStore {
  static constexpr bool kWritesLds = false;
  void* out;
  int64_t ob;
  int r0;
  int f32;
  __device__ __forceinline__ void apply(int p, int x, cpx<T>& v) const {
    const int64_t i0 = ob + (int64_t)(r0 + 2 * p) * N + x;
    if (f32) {
      float* o = (float*)out;
      o[i0] = (float)v.x;
      o[i0 + N] = (float)v.y;
    } else {
      double* o = (double*)out;
      o[i0] = (double)v.x;
      o[i0 + N] = (double)v.y;
    }
  }
};

// Split the pair-packed spectra Z of every row pair of the tile back into
// the two rows' half spectra and store them column-major.
template <int N, typename T, int PAIRS, int NT, class Lay>
__device__ __forceinline__ void row_split_store(const cpx<T>* panel, cpx<T>* S, int r0, int tid,
                                                Lay lay) {
  using C = cpx<T>;
  for (int e = tid; e < PAIRS * (N / 2); e += NT) {
    int p, c;
    row_entry<N, PAIRS>(e, p, c);
    C A, B;
    if (c == 0) {
      const C z0 = panel[lay(p, 0)], zn = panel[lay(p, N / 2)];
      A = C{z0.x, zn.x};
      B = C{z0.y, zn.y};
    } else {
      const C z = panel[lay(p, c)], w = panel[lay(p, N - c)];
      const T h = (T)0.5;
      A = C{h * (z.x + w.x), h * (z.y - w.y)};
      B = C{h * (z.y + w.y), h * (w.x - z.x)};
    }
    S[spec_at<N>(c, r0 + 2 * p)] = A;
    S[spec_at<N>(c, r0 + 2 * p + 1)] = B;
  }
}

// Line stride of the row-pass panel.  The rebuild and split loops put the
// row pairs of one column in consecutive lanes; with four pairs per tile
// a stride = 4 (mod 16) makes the 8 lanes served together (4 pairs x 2
// columns, direct or mirrored) fall in distinct 16-byte bank quads.
// The plan also picks the twiddle table: the full per-stage one, or (for
// 16-byte elements, where it lets one more work-group share a CU) the
// compact one of r = 1 rows, whose other powers the butterflies multiply
// out.  TWN is the table's length in elements.
template <int N, typename T, int RS = 0> struct RowLS {
  static constexpr bool kQuad = sizeof(T) == 8 && RowCfg<N, T>::PAIRS == 4 && N >= 128;
  static constexpr int E = (int)sizeof(cpx<T>), kOther = (RowCfg<N, T>::NT / 64 + 1) * 8 + 64;
  using PF = LdsPlan<N, RowCfg<N, T>::PAIRS, E, TwSize<N, RS>::value * E + kOther, kQuad ? 4 : 1,
                     RowCfg<N, T>::NT>;
  using PP = LdsPlan<N, RowCfg<N, T>::PAIRS, E, TwSizePow<N, RS>::value * E + kOther,
                     kQuad ? 4 : 1, RowCfg<N, T>::NT>;
  static constexpr bool TWP = E == 16 && PP::FIT > PF::FIT;
  static constexpr int TWN = TWP ? TwSizePow<N, RS>::value : TwSize<N, RS>::value;
  static constexpr int SH = TWP ? PP::SH : PF::SH;
  static constexpr int value = N + (N >> SH) + (kQuad ? 4 : 1);
};

// Column-pass panel: CT whole columns next to the twiddles (and, for the
// Picard pass, the symbol table).
template <int N, typename T, int EXTRA = 0, int RS = 0> struct ColLS {
  static constexpr int E = (int)sizeof(cpx<T>);
  using PF = LdsPlan<N, ColCfg<N>::CT, E, TwSize<N, RS>::value * E + EXTRA + 64, 1, ColCfg<N>::NT>;
  using PP =
      LdsPlan<N, ColCfg<N>::CT, E, TwSizePow<N, RS>::value * E + EXTRA + 64, 1, ColCfg<N>::NT>;
  static constexpr bool TWP = E == 16 && PP::FIT > PF::FIT;
  static constexpr int TWN = TWP ? TwSizePow<N, RS>::value : TwSize<N, RS>::value;
  static constexpr int SH = TWP ? PP::SH : PF::SH;
  static constexpr int value = N + (N >> SH) + 1;
};

// Stage the block's twiddle table in LDS in the plan's form, for radix
// split RS.
template <int N, int NT, bool TWP, int RS = 0, typename C>
__device__ __forceinline__ void load_twiddles(C* tw, const C* g, int tid) {
  if constexpr (TWP) load_stage_twiddles_pow<N, NT, RS>(tw, g, tid);
  else load_stage_twiddles<N, NT, RS>(tw, g, tid);
}

// The step parameters of field f: the launch argument, or the field's entry
// of the descriptor's parameter table.
__device__ __forceinline__ StepParams field_params(const CallDesc* desc, int64_t f,
                                                   const StepParams& arg) {
  if (!desc->params) return arg;
  return desc->params[desc->pidx ? desc->pidx[f] : 0];
}

// Rebuild of pair p's spectrum Z_p[kx] = R_2p[kx] + i R_2p+1[kx] at kx = c
// and N - c from the two rows' half-spectrum values A and B of column c
// (c = 0 carries kx = 0 and kx = N/2 as its real and imaginary parts).
template <int N, typename T, class Lay>
__device__ __forceinline__ void row_rebuild_entry(cpx<T>* panel, Lay lay, int p, int c, cpx<T> A,
                                                  cpx<T> B) {
  using C = cpx<T>;
  if (c == 0) {
    panel[lay(p, 0)] = C{A.x, B.x};
    panel[lay(p, N / 2)] = C{A.y, B.y};
  } else {
    panel[lay(p, c)] = C{A.x - B.y, A.y + B.x};
    panel[lay(p, N - c)] = C{A.x + B.y, B.x - A.y};
  }
}

// Middle row pass of one tile whose pair spectra are in the panel: inverse
// transforms, the right-hand side (with the tile's FP64 sum of f for the
// mass multiplier), forward transforms, split and store to S.
template <int N, typename T, int RHS, int RS = 0, class TW>
__device__ __forceinline__ void row_mid_tile(cpx<T>* panel, TW tw, double* red,
                                             double* __restrict__ partials, cpx<T>* S, int64_t f,
                                             int tile, T a, T dt, int conservative, int tid) {
  using Cfg = RowCfg<N, T>;
  constexpr int PAIRS = Cfg::PAIRS, NT = Cfg::NT, TILES = Cfg::TILES;
  using Lay = LinePanel<RowLS<N, T, RS>::value, RowLS<N, T, RS>::SH>;
  const Lay lay{};
  double fsum = 0.0;
  fft_lines<N, +1, NT, T, 1, false, RS>(panel, tw, lay, tid, NoPro{}, RhsEpi<T, RHS>{a, dt, &fsum});
  fft_lines<N, -1, NT, T, 1, false, RS>(panel, tw, lay, tid);
  if (RHS == RHS_SSI && conservative) {
    const double s = block_sum<NT>(fsum, red, tid);
    if (tid == 0) partials[f * TILES + tile] = s;
  }
  row_split_store<N, T, PAIRS, NT>(panel, S, tile * Cfg::TR, tid, lay);
}

// First row pass of a call: the real FP64 state in, half spectra out.
// Tile `tile` of field f; panel, tw_s and red are the block's LDS.
template <int N, typename T, int RHS = RHS_SSI, int RS = 0>
__device__ __forceinline__ void row_first_body(cpx<T>* panel, cpx<T>* tw_s, double* red,
                                               const CallDesc* __restrict__ desc,
                                               cpx<T>* __restrict__ spec,
                                               double* __restrict__ partials,
                                               const cpx<T>* __restrict__ tw_g,
                                               const StepParams& sp_arg, int64_t f, int tile,
                                               int tid) {
  using C = cpx<T>;
  using Cfg = RowCfg<N, T>;
  constexpr int TR = Cfg::TR, PAIRS = Cfg::PAIRS, NT = Cfg::NT, TILES = Cfg::TILES;
  using RL = RowLS<N, T, RS>;
  using Lay = LinePanel<RL::value, RL::SH>;
  const auto tw = twiddle_source<RL::TWP>((const C*)tw_s);
  const StepParams sp = field_params(desc, f, sp_arg);
  const int r0 = tile * TR;
  const Lay lay{};
  load_twiddles<N, NT, RL::TWP, RS>(tw_s, tw_g, tid);
  const T a = (T)sp.a, dt = (T)sp.dt;
  double fsum = 0.0;
  const double* u = desc->in_base + (desc->in_offs ? desc->in_offs[f] : f * (int64_t)N * N);
  __syncthreads();
  fft_lines<N, -1, NT, T, 1, false, RS>(panel, tw, lay, tid,
                                        RealRowsPro<N, T, RHS>{u, r0, a, dt, &fsum});
  if (RHS == RHS_SSI && sp.conservative) {
    const double s = block_sum<NT>(fsum, red, tid);
    if (tid == 0) partials[f * TILES + tile] = s;
  }
  row_split_store<N, T, PAIRS, NT>(panel, spec + f * (int64_t)(N / 2) * N, r0, tid, lay);
}

template <int N, typename T, int RHS = RHS_SSI, int RS = 0>
__global__ __attribute__((amdgpu_flat_work_group_size(1, RowCfg<N, T>::NT))) void k_row_first(
    const CallDesc* __restrict__ desc, cpx<T>* __restrict__ spec, double* __restrict__ partials,
    const cpx<T>* __restrict__ tw_g, StepParams sp_arg) {
  using C = cpx<T>;
  using Cfg = RowCfg<N, T>;
  __shared__ C panel[Cfg::PAIRS * RowLS<N, T, RS>::value];
  __shared__ C tw_s[RowLS<N, T, RS>::TWN];
  __shared__ double red[Cfg::NT / 64 + 1];
  const int64_t f = blockIdx.x / Cfg::TILES;
  if (f >= desc->nfields) return;
  row_first_body<N, T, RHS, RS>(panel, tw_s, red, desc, spec, partials, tw_g, sp_arg, f,
                                (int)(blockIdx.x % Cfg::TILES), threadIdx.x);
}

// Middle and last row passes: tile `tile` (TR rows) of field f.
template <int N, typename T, int MODE, int RHS = RHS_SSI, int RS = 0>
__device__ __forceinline__ void row_body(cpx<T>* panel, cpx<T>* tw_s, double* red,
                                         const CallDesc* __restrict__ desc,
                                         cpx<T>* __restrict__ spec, double* __restrict__ partials,
                                         const cpx<T>* __restrict__ tw_g, const StepParams& sp_arg,
                                         int64_t f, int tile, int tid) {
  using C = cpx<T>;
  using Cfg = RowCfg<N, T>;
  constexpr int TR = Cfg::TR, PAIRS = Cfg::PAIRS, NT = Cfg::NT;
  using RL = RowLS<N, T, RS>;
  using Lay = LinePanel<RL::value, RL::SH>;
  const auto tw = twiddle_source<RL::TWP>((const C*)tw_s);
  const StepParams sp = field_params(desc, f, sp_arg);
  const int r0 = tile * TR;
  const Lay lay{};
  load_twiddles<N, NT, RL::TWP, RS>(tw_s, tw_g, tid);
  C* S = spec + f * (int64_t)(N / 2) * N;
  const T a = (T)sp.a, dt = (T)sp.dt;
  // rebuild Z_j[kx] = R_2j[kx] + i R_2j+1[kx] for kx = 0..N-1
  for (int e = tid; e < PAIRS * (N / 2); e += NT) {
    int p, c;
    row_entry<N, PAIRS>(e, p, c);
    row_rebuild_entry<N, T>(panel, lay, p, c, S[spec_at<N>(c, r0 + 2 * p)],
                            S[spec_at<N>(c, r0 + 2 * p + 1)]);
  }
  __syncthreads();
  if constexpr (MODE == ROW_LAST) {
    const int64_t ob = desc->out_offs ? desc->out_offs[f] : f * (int64_t)N * N;
    fft_lines<N, +1, NT, T, 1, false, RS>(panel, tw, lay, tid, NoPro{},
                                          RealRowsStore<N, T>{desc->out_base, ob, r0, desc->out_f32});
  } else {
    row_mid_tile<N, T, RHS, RS>(panel, tw, red, partials, S, f, tile, a, dt, sp.conservative, tid);
  }
}

// One block per tile of TR rows of one field.
template <int N, typename T, int MODE, int RHS = RHS_SSI, int RS = 0>
__global__ __attribute__((amdgpu_flat_work_group_size(1, RowCfg<N, T>::NT))) void k_row(
    const CallDesc* __restrict__ desc, cpx<T>* __restrict__ spec, double* __restrict__ partials,
    const cpx<T>* __restrict__ tw_g, StepParams sp_arg) {
  using C = cpx<T>;
  using Cfg = RowCfg<N, T>;
  __shared__ C panel[Cfg::PAIRS * RowLS<N, T, RS>::value];
  __shared__ C tw_s[RowLS<N, T, RS>::TWN];
  __shared__ double red[Cfg::NT / 64 + 1];
  const int64_t f = blockIdx.x / Cfg::TILES;
  if (f >= desc->nfields) return;
  row_body<N, T, MODE, RHS, RS>(panel, tw_s, red, desc, spec, partials, tw_g, sp_arg, f,
                                (int)(blockIdx.x % Cfg::TILES), threadIdx.x);
}

// ------------------------------------------------------------ column pass

// Element e of line (column) `line` of the column tile starting at P.
template <int N, typename T> struct ColLoad {
  const cpx<T>* P;
  __device__ __forceinline__ cpx<T> load(int, int line, int e) const { return P[col_at<N>(line, e)]; }
  __device__ __forceinline__ void after_reads() const {}
};

template <int N, typename T> struct ColStore {
  static constexpr bool kWritesLds = false;
  cpx<T>* P;
  __device__ __forceinline__ void apply(int line, int e, cpx<T>& v) const { P[col_at<N>(line, e)] = v; }
};

// 1 / (N^2 ((1 + S dt) + dt eps^2 mu_k)) for bin (ky, kx)
__device__ __forceinline__ double inv_symbol(const StepParams& sp, const double* s2, int ky, int kx) {
  return sp.inv_n2 / (sp.a + sp.lam * (s2[kx] + s2[ky]));
}

// Last forward stage: divide every column except the packed one (c = 0).
template <typename T> struct DivideEpi {
  static constexpr bool kWritesLds = true;
  const double* s2;
  StepParams sp;
  int c0;
  __device__ __forceinline__ void apply(int line, int ky, cpx<T>& v) const {
    const int col = c0 + line;
    if (col != 0) {
      const T d = (T)inv_symbol(sp, s2, ky, col);
      v = cpx<T>{v.x * d, v.y * d};
    }
  }
};

// Column panel of CT columns next to the twiddles (and the symbol table
// when it is kept in LDS).
template <int N, typename T, int RS = 0> using ColPanel = ColLS<N, T, PR_S2_LDS ? N * 8 : 0, RS>;

// One column tile: CT columns of field f from c0, at P.  Forward transform
// (inputs from `pro`), division by the symbol (the packed column c = 0 with
// the mass correction), inverse transform straight to P.  corr_sh must not
// be read by any thread of the block from a previous tile any more.
template <int N, typename T, int RS = 0, class TW, class Pro>
__device__ __forceinline__ void col_tile(cpx<T>* panel, TW tw, double* corr_sh,
                                         const double* s2, const double* __restrict__ partials,
                                         cpx<T>* P, int64_t f, int c0, const StepParams& sp,
                                         int tid, Pro pro) {
  using C = cpx<T>;
  constexpr int NT = ColCfg<N>::NT;
  constexpr int TILES = RowCfg<N, T>::TILES;
  constexpr int E0 = (N + NT - 1) / NT;  // packed-column elements per thread
  using Lay = LinePanel<ColPanel<N, T, RS>::value, ColPanel<N, T, RS>::SH>;
  const Lay lay{};
  if (tid == 0) {
    double corr = 0.0;
    if (c0 == 0 && sp.conservative) {
      double sum = 0.0;
      for (int i = 0; i < TILES; ++i) sum += partials[f * TILES + i];
      corr = sp.dt * sum;  // dt * N^2 * mean f
    }
    *corr_sh = corr;
  }
  // the forward transform's last stage ends with a block barrier, which
  // also publishes corr_sh
  fft_lines<N, -1, NT, T, 1, SpecLayout<N>::LF, RS>(panel, tw, lay, tid, pro,
                                                     DivideEpi<T>{s2, sp, c0});
  if (c0 == 0) {
    // packed column: z = A + iB with A the kx = 0 and B the kx = N/2
    // column spectra (both Hermitian in ky); scale A and B separately
    const double corr = *corr_sh;
    C vals[E0];
#pragma unroll
    for (int q = 0; q < E0; ++q) {
      const int ky = tid + q * NT;
      if (ky < N) {
        const int kr = (N - ky) % N;
        C z = panel[lay(0, ky)], w = panel[lay(0, kr)];
        if (ky == 0) z.x = (T)((double)z.x - corr);
        if (kr == 0) w.x = (T)((double)w.x - corr);
        const double d0 = inv_symbol(sp, s2, ky, 0), dn = inv_symbol(sp, s2, ky, N / 2);
        const T pp = (T)(0.5 * (d0 + dn)), mm = (T)(0.5 * (d0 - dn));
        vals[q] = C{z.x * pp + w.x * mm, z.y * pp - w.y * mm};
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < E0; ++q) {
      const int ky = tid + q * NT;
      if (ky < N) panel[lay(0, ky)] = vals[q];
    }
    __syncthreads();
  }
  fft_lines<N, +1, NT, T, 1, SpecLayout<N>::LF, RS>(panel, tw, lay, tid, NoPro{},
                                                     ColStore<N, T>{P});
}

// Column tile `blk` (CT columns) of field f; panel, tw_s, s2_s (PR_S2_LDS
// only) and corr_sh are the block's LDS.
template <int N, typename T, int RS = 0>
__device__ __forceinline__ void col_body(cpx<T>* panel, cpx<T>* tw_s, double* s2_s,
                                         double* corr_sh, const CallDesc* __restrict__ desc,
                                         cpx<T>* __restrict__ spec,
                                         const double* __restrict__ partials,
                                         const cpx<T>* __restrict__ tw_g,
                                         const double* __restrict__ s2_g, const StepParams& sp_arg,
                                         int64_t f, int blk, int tid) {
  using C = cpx<T>;
  constexpr int CT = ColCfg<N>::CT, NT = ColCfg<N>::NT;
  const auto tw = twiddle_source<ColPanel<N, T, RS>::TWP>((const C*)tw_s);
#if PR_S2_LDS
  const double* s2 = s2_s;
#else
  const double* s2 = s2_g;
  (void)s2_s;
#endif
  const StepParams sp = field_params(desc, f, sp_arg);
  const int c0 = blk * CT;
  C* P = spec + f * (int64_t)(N / 2) * N + (int64_t)c0 * N;
  load_twiddles<N, NT, ColPanel<N, T, RS>::TWP, RS>(tw_s, tw_g, tid);
#if PR_S2_LDS
  for (int i = tid; i < N; i += NT) s2_s[i] = s2_g[i];
#endif
  __syncthreads();
  col_tile<N, T, RS>(panel, tw, corr_sh, s2, partials, P, f, c0, sp, tid, ColLoad<N, T>{P});
}

// One block per column tile.
template <int N, typename T, int RS = 0>
__global__ __attribute__((amdgpu_flat_work_group_size(1, ColCfg<N>::NT))) void k_col(
    const CallDesc* __restrict__ desc, cpx<T>* __restrict__ spec,
    const double* __restrict__ partials, const cpx<T>* __restrict__ tw_g,
    const double* __restrict__ s2_g, StepParams sp_arg) {
  using C = cpx<T>;
  constexpr int CT = ColCfg<N>::CT, BLK = ColCfg<N>::BLOCKS;
  __shared__ C panel[CT * ColPanel<N, T, RS>::value];
  __shared__ C tw_s[ColPanel<N, T, RS>::TWN];
#if PR_S2_LDS
  __shared__ double s2[N];
#else
  double* s2 = nullptr;
#endif
  __shared__ double corr_sh;
  const int64_t f = blockIdx.x / BLK;
  if (f >= desc->nfields) return;
  col_body<N, T, RS>(panel, tw_s, s2, &corr_sh, desc, spec, partials, tw_g, s2_g, sp_arg, f,
                     (int)(blockIdx.x % BLK), threadIdx.x);
}

// ------------------------------------------------ Crank-Nicolson + Picard
//
// The paper's fine scheme (Section 3.1, eq. fully-discrete) solved by
// Picard iteration from V_(0) = U_n.  In Fourier space, with
// q_k = (dt eps^2 / 2) mu_k, A_k = 1 - q_k, D_k = 1 + q_k and F^(m) the
// DFT of f(V_(m)), iteration m is
//     D V^_(m+1) = K + (dt/2) F^(m),   K = A U^_n + (dt/2) F^_n,
// with F^(0) = F^_n since V_(0) = U_n.  In the conservative model the
// nonlocal term dt g removes the means of f(U_n)/2 and f(V_(m))/2, i.e.
// exactly the DC bins of both F terms, so V keeps the DC of U_n.
//
// The row passes transform f(v) (RHS_F).  The column pass of Picard
// iteration m transforms those row spectra along the columns, forms
// V^_(m+1) from them and the field's second spectral buffer X, and
// stores V^_(m+1) / N^2 as row spectra for the next row pass.  X holds
// U^_n (2-D layout) between steps and K during a step's iterations:
//     m = 0:   K = A X + (dt/2) F^,  V^ = (K + (dt/2) F^) / D,  X <- K;
//     m > 0:   V^ = (X + (dt/2) F^) / D;
// and at the last m, X <- V^ (= U^_{n+1}).  Stage-in transforms U_0 into
// X (a row pass with RHS_U, then k_col_fwd) and f(U_0) into the row
// spectra.

enum { CN_FIRST = 1, CN_LAST = 2 };

// Forward column transform in place: row spectra -> 2-D spectrum.
template <int N, typename T>
__global__ __attribute__((amdgpu_flat_work_group_size(1, ColCfg<N>::NT))) void k_col_fwd(
    const CallDesc* __restrict__ desc, cpx<T>* __restrict__ xspec, const cpx<T>* __restrict__ tw_g) {
  using C = cpx<T>;
  constexpr int CT = ColCfg<N>::CT, NT = ColCfg<N>::NT, BLK = ColCfg<N>::BLOCKS;
  using CL = ColLS<N, T>;
  constexpr int LS = CL::value;
  using Lay = LinePanel<LS, CL::SH>;
  __shared__ C panel[CT * LS];
  __shared__ C tw_s[CL::TWN];
  const auto tw = twiddle_source<CL::TWP>((const C*)tw_s);
  const int tid = threadIdx.x;
  const int64_t f = blockIdx.x / BLK;
  if (f >= desc->nfields) return;
  const int c0 = (blockIdx.x % BLK) * CT;
  C* P = xspec + f * (int64_t)(N / 2) * N + (int64_t)c0 * N;
  load_twiddles<N, NT, CL::TWP>(tw_s, tw_g, tid);
  __syncthreads();
  fft_lines<N, -1, NT, T, 1, SpecLayout<N>::LF>(panel, tw, Lay{}, tid, ColLoad<N, T>{P},
                                                  ColStore<N, T>{P});
}

// Last forward stage of a Picard column pass, for every column but the
// packed one: combine with X, update X, scale by 1/N^2 for the inverse.
template <int N, typename T, int MODE> struct CnEpi {
  static constexpr bool kWritesLds = true;
  cpx<T>* X;           // column c0 of the field's X
  const double* s2;
  StepParams sp;
  int c0;
  __device__ __forceinline__ void apply(int line, int ky, cpx<T>& v) const {
    const int col = c0 + line;
    if (col == 0) return;  // the packed column is done after the transform
    const double q = 0.5 * sp.lam * (s2[col] + s2[ky]);
    const T h = (T)(0.5 * sp.dt);
    cpx<T>* xp = X + col_at<N>(line, ky);
    const cpx<T> x = *xp;
    cpx<T> K = x;
    if constexpr ((MODE & CN_FIRST) != 0) {
      const T A = (T)(1.0 - q);
      K = cpx<T>{A * x.x + h * v.x, A * x.y + h * v.y};
    }
    const T dinv = (T)(1.0 / (1.0 + q));
    const cpx<T> V{(K.x + h * v.x) * dinv, (K.y + h * v.y) * dinv};
    if constexpr ((MODE & CN_LAST) != 0) *xp = V;
    else if constexpr ((MODE & CN_FIRST) != 0) *xp = K;
    const T sc = (T)sp.inv_n2;
    v = cpx<T>{V.x * sc, V.y * sc};
  }
};

// a (m0 + mn)/2 + conj(b) (m0 - mn)/2: multiplies the kx = 0 part of a
// packed column value a by m0 and its kx = N/2 part by mn, for real
// multipliers even in ky, given b = the value at -ky.
template <typename T>
__device__ __forceinline__ cpx<T> packed_mul(cpx<T> a, cpx<T> b, double m0, double mn) {
  const T pp = (T)(0.5 * (m0 + mn)), mm = (T)(0.5 * (m0 - mn));
  return cpx<T>{a.x * pp + b.x * mm, a.y * pp - b.y * mm};
}

template <int N, typename T, int MODE>
__global__ __attribute__((amdgpu_flat_work_group_size(1, ColCfg<N>::NT))) void k_col_cn(
    const CallDesc* __restrict__ desc, cpx<T>* __restrict__ spec, cpx<T>* __restrict__ xspec,
    const cpx<T>* __restrict__ tw_g, const double* __restrict__ s2_g, StepParams sp_arg) {
  using C = cpx<T>;
  constexpr int CT = ColCfg<N>::CT, NT = ColCfg<N>::NT, BLK = ColCfg<N>::BLOCKS;
  using CL = ColLS<N, T, N * 8>;
  constexpr int LS = CL::value;
  constexpr int E0 = (N + NT - 1) / NT;
  using Lay = LinePanel<LS, CL::SH>;
  __shared__ C panel[CT * LS];
  __shared__ C tw_s[CL::TWN];
  __shared__ double s2[N];
  const auto tw = twiddle_source<CL::TWP>((const C*)tw_s);

  const int tid = threadIdx.x;
  const int64_t f = blockIdx.x / BLK;
  if (f >= desc->nfields) return;
  const StepParams sp = field_params(desc, f, sp_arg);
  const int c0 = (blockIdx.x % BLK) * CT;
  const Lay lay{};
  C* P = spec + f * (int64_t)(N / 2) * N + (int64_t)c0 * N;
  C* X = xspec + f * (int64_t)(N / 2) * N + (int64_t)c0 * N;
  load_twiddles<N, NT, CL::TWP>(tw_s, tw_g, tid);
  for (int i = tid; i < N; i += NT) s2[i] = s2_g[i];
  __syncthreads();
  fft_lines<N, -1, NT, T, 1, SpecLayout<N>::LF>(panel, tw, lay, tid, ColLoad<N, T>{P},
                                                  CnEpi<N, T, MODE>{X, s2, sp, c0});
  if (c0 == 0) {
    const double h = 0.5 * sp.dt;
    C vals[E0], xnew[E0];
#pragma unroll
    for (int q = 0; q < E0; ++q) {
      const int ky = tid + q * NT;
      if (ky < N) {
        const int kr = (N - ky) % N;
        C z = panel[lay(0, ky)], w = panel[lay(0, kr)];
        if (sp.conservative) {   // drop F^(0, 0)
          if (ky == 0) z.x = (T)0;
          if (kr == 0) w.x = (T)0;
        }
        const C x = X[col_at<N>(0, ky)], xr = X[col_at<N>(0, kr)];
        const double q0 = 0.5 * sp.lam * (s2[0] + s2[ky]), qn = 0.5 * sp.lam * (s2[N / 2] + s2[ky]);
        C K = x, Kr = xr;
        if constexpr ((MODE & CN_FIRST) != 0) {
          K = packed_mul<T>(x, xr, 1.0 - q0, 1.0 - qn);
          Kr = packed_mul<T>(xr, x, 1.0 - q0, 1.0 - qn);
          K = C{K.x + (T)h * z.x, K.y + (T)h * z.y};
          Kr = C{Kr.x + (T)h * w.x, Kr.y + (T)h * w.y};
        }
        const C Y{K.x + (T)h * z.x, K.y + (T)h * z.y}, Yr{Kr.x + (T)h * w.x, Kr.y + (T)h * w.y};
        const C V = packed_mul<T>(Y, Yr, 1.0 / (1.0 + q0), 1.0 / (1.0 + qn));
        xnew[q] = (MODE & CN_LAST) != 0 ? V : K;
        const T sc = (T)sp.inv_n2;
        vals[q] = C{V.x * sc, V.y * sc};
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < E0; ++q) {
      const int ky = tid + q * NT;
      if (ky < N) {
        panel[lay(0, ky)] = vals[q];
        if constexpr (MODE != 0) X[col_at<N>(0, ky)] = xnew[q];
      }
    }
    __syncthreads();
  }
  fft_lines<N, +1, NT, T, 1, SpecLayout<N>::LF>(panel, tw, lay, tid, NoPro{}, ColStore<N, T>{P});
}

// ---------------------------------------------------- on-chip resident step
//
// One block per field for all steps of the call, for N <= 128: the field's
// spectrum (N/2 x N complex, the same column-major layout as in HBM) stays
// in LDS.  The row pass runs in place on those slots: the complex row pair
// p (rows 2p, 2p+1) occupies the 2 x N/2 slots of rows 2p and 2p+1, with
// Z_p[kx] at slot (kx mod N/2, 2p + kx / (N/2)); packing into and splitting
// out of that form permutes only those slots.  Slot (c, r) lives at
// c * LS + c/8 + r + r/8 (LS odd), so unit and stride-8 walks along either
// index spread over the LDS banks.

template <int N> struct ResCfg {
  static constexpr int H = N / 2;
  static constexpr int G = N >= 128 ? 2 : 1;     // radix-8 groups per thread
  static constexpr int NT = N * N / (16 * G);    // 8 G complex elements per thread
  static constexpr int LS = N + N / 8 + 1;   // SlotAddr pads every 8 rows
  static constexpr int SLOTS = H * LS + H / 8 + 1;
};

template <int N> struct SlotAddr {
  __device__ __forceinline__ static int at(int c, int r) {
    return c * ResCfg<N>::LS + (c >> 3) + r + (r >> 3);
  }
};
template <int N> struct ResColLay {   // line = column c, element = row r
  __device__ __forceinline__ int operator()(int c, int r) const { return SlotAddr<N>::at(c, r); }
};
template <int N> struct ResRowLay {   // line = row pair p, element = kx
  __device__ __forceinline__ int operator()(int p, int kx) const {
    return SlotAddr<N>::at(kx & (N / 2 - 1), 2 * p + (kx >= N / 2 ? 1 : 0));
  }
};

// (c, p) work items of the pack / split permutations, four per thread
template <int N, typename T, bool PACK>
__device__ __forceinline__ void res_permute(cpx<T>* S, int tid) {
  using C = cpx<T>;
  constexpr int H = N / 2, NT = ResCfg<N>::NT, IT = H * H / NT;  // 4 G
  C a[IT], b[IT];
#pragma unroll
  for (int q = 0; q < IT; ++q) {
    const int item = tid + q * NT;
    const int c = item % H, p = item / H;
    if constexpr (PACK) {
      a[q] = S[SlotAddr<N>::at(c, 2 * p)];
      b[q] = S[SlotAddr<N>::at(c, 2 * p + 1)];
    } else {
      a[q] = S[SlotAddr<N>::at(c, 2 * p)];                         // Z[c] (Z[0] for c = 0)
      b[q] = S[SlotAddr<N>::at(c == 0 ? 0 : H - c, 2 * p + 1)];   // Z[N-c] (Z[N/2] for c = 0)
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < IT; ++q) {
    const int item = tid + q * NT;
    const int c = item % H, p = item / H;
    const C A = a[q], B = b[q];
    if constexpr (PACK) {
      if (c == 0) {
        S[SlotAddr<N>::at(0, 2 * p)] = C{A.x, B.x};        // Z[0]
        S[SlotAddr<N>::at(0, 2 * p + 1)] = C{A.y, B.y};    // Z[N/2]
      } else {
        S[SlotAddr<N>::at(c, 2 * p)] = C{A.x - B.y, A.y + B.x};          // Z[c]
        S[SlotAddr<N>::at(H - c, 2 * p + 1)] = C{A.x + B.y, B.x - A.y};  // Z[N-c]
      }
    } else {
      if (c == 0) {
        S[SlotAddr<N>::at(0, 2 * p)] = C{A.x, B.x};
        S[SlotAddr<N>::at(0, 2 * p + 1)] = C{A.y, B.y};
      } else {
        const T h = (T)0.5;
        S[SlotAddr<N>::at(c, 2 * p)] = C{h * (A.x + B.x), h * (A.y - B.y)};
        S[SlotAddr<N>::at(c, 2 * p + 1)] = C{h * (A.y + B.y), h * (B.x - A.x)};
      }
    }
  }
  __syncthreads();
}

template <int N, typename T>
__global__ __attribute__((amdgpu_flat_work_group_size(1, ResCfg<N>::NT))) void k_resident(
    const CallDesc* __restrict__ desc, const cpx<T>* __restrict__ tw_g,
    const double* __restrict__ s2_g, StepParams sp_arg, int steps) {
  using C = cpx<T>;
  using Cfg = ResCfg<N>;
  constexpr int NT = Cfg::NT, E0 = (N + NT - 1) / NT;
  __shared__ C S[Cfg::SLOTS];
  __shared__ C tw[TwSize<N>::value];
  __shared__ double s2[N];
  __shared__ double red[NT / 64 + 1];
  __shared__ double corr_sh;

  const int tid = threadIdx.x;
  const int64_t f = blockIdx.x;
  if (f >= desc->nfields) return;
  const StepParams sp = field_params(desc, f, sp_arg);
  load_stage_twiddles<N, NT>(tw, tw_g, tid);
  for (int t = tid; t < N; t += NT) s2[t] = s2_g[t];
  const T a = (T)sp.a, dt = (T)sp.dt;
  const ResRowLay<N> rlay{};
  const ResColLay<N> clay{};
  double fsum = 0.0;
  __syncthreads();

  // first right-hand side straight from the FP64 state
  const double* u = desc->in_base + (desc->in_offs ? desc->in_offs[f] : f * (int64_t)N * N);
  fft_lines<N, -1, NT, T, Cfg::G>(S, tw, rlay, tid, RealRowsPro<N, T>{u, 0, a, dt, &fsum});
  res_permute<N, T, false>(S, tid);

  for (int s = 0; s < steps; ++s) {
    const int tid = opaque_tid(threadIdx.x);
    if (sp.conservative) {
      const double tot = block_sum<NT>(fsum, red, tid);
      if (tid == 0) corr_sh = sp.dt * tot;
    } else if (tid == 0) {
      corr_sh = 0.0;
    }
    fsum = 0.0;
    // column pass
    fft_lines<N, -1, NT, T, Cfg::G>(S, tw, clay, tid, NoPro{}, DivideEpi<T>{s2, sp, 0});
    {
      const double corr = corr_sh;
      C vals[E0];
#pragma unroll
      for (int q = 0; q < E0; ++q) {
        const int ky = tid + q * NT;
        if (ky < N) {
          const int kr = (N - ky) % N;
          C z = S[clay(0, ky)], w = S[clay(0, kr)];
          if (ky == 0) z.x = (T)((double)z.x - corr);
          if (kr == 0) w.x = (T)((double)w.x - corr);
          const double d0 = inv_symbol(sp, s2, ky, 0), dn = inv_symbol(sp, s2, ky, N / 2);
          const T pp = (T)(0.5 * (d0 + dn)), mm = (T)(0.5 * (d0 - dn));
          vals[q] = C{z.x * pp + w.x * mm, z.y * pp - w.y * mm};
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < E0; ++q) {
        const int ky = tid + q * NT;
        if (ky < N) S[clay(0, ky)] = vals[q];
      }
      __syncthreads();
    }
    fft_lines<N, +1, NT, T, Cfg::G>(S, tw, clay, tid);
    // row pass
    res_permute<N, T, true>(S, tid);
    if (s + 1 < steps) {
      fft_lines<N, +1, NT, T, Cfg::G>(S, tw, rlay, tid, NoPro{}, RhsEpi<T>{a, dt, &fsum});
      fft_lines<N, -1, NT, T, Cfg::G>(S, tw, rlay, tid);
      res_permute<N, T, false>(S, tid);
    }
  }
  const int64_t ob = desc->out_offs ? desc->out_offs[f] : f * (int64_t)N * N;
  fft_lines<N, +1, NT, T, Cfg::G>(S, tw, rlay, tid, NoPro{},
                          RealRowsStore<N, T>{desc->out_base, ob, 0, desc->out_f32});
}

// ------------------------------------------------------------- launchers

__global__ void k_set_desc(CallDesc* d, CallDesc v) { *d = v; }

bool fine_radix_differs(int n) {
  switch (n) {
    case 16: return radix_split_differs<16>();
    case 32: return radix_split_differs<32>();
    case 64: return radix_split_differs<64>();
    case 128: return radix_split_differs<128>();
    case 256: return radix_split_differs<256>();
    case 512: return radix_split_differs<512>();
    case 1024: return radix_split_differs<1024>();
    default: return false;
  }
}

// The 2 * steps + 1 launches of one streaming F call, for a grid of
// `grid_fields` fields (blocks of fields beyond desc->nfields exit).
template <int N, typename T, int RS>
static void enqueue_stream_steps(const StepJob& job, int64_t grid_fields, hipStream_t st) {
  using RC = RowCfg<N, T>;
  using CC = ColCfg<N>;
  const cpx<T>* tw = (const cpx<T>*)(sizeof(T) == 8 ? (const void*)job.ws.tw64 : (const void*)job.ws.tw32);
  cpx<T>* spec = (cpx<T>*)job.ws.spec;
  const CallDesc* d = job.ws.desc;
  const int64_t row_tiles = grid_fields * RC::TILES, col_tiles = grid_fields * CC::BLOCKS;
  const dim3 gfirst((unsigned)row_tiles), brow(RC::NT), bcol(CC::NT);
  const dim3 grow((unsigned)row_tiles), glast((unsigned)row_tiles), gcol((unsigned)col_tiles);
  k_row_first<N, T, RHS_SSI, RS><<<gfirst, brow, 0, st>>>(d, spec, job.ws.partials, tw, job.sp);
  for (int s = 0; s < job.steps; ++s) {
    k_col<N, T, RS><<<gcol, bcol, 0, st>>>(d, spec, job.ws.partials, tw, job.ws.s2, job.sp);
    if (s + 1 < job.steps)
      k_row<N, T, ROW_MID, RHS_SSI, RS><<<grow, brow, 0, st>>>(d, spec, job.ws.partials, tw, job.sp);
  }
  k_row<N, T, ROW_LAST, RHS_SSI, RS><<<glast, brow, 0, st>>>(d, spec, job.ws.partials, tw, job.sp);
}

template <int N, typename T, int MODE>
static void launch_col_cn(const StepJob& job, dim3 g, dim3 b, hipStream_t st) {
  const cpx<T>* tw = (const cpx<T>*)(sizeof(T) == 8 ? (const void*)job.ws.tw64 : (const void*)job.ws.tw32);
  k_col_cn<N, T, MODE><<<g, b, 0, st>>>(job.ws.desc, (cpx<T>*)job.ws.spec, (cpx<T>*)job.ws.xspec,
                                        tw, job.ws.s2, job.sp);
}

// The launches of one Crank-Nicolson F call: stage-in (3), then per step
// and Picard iteration a column pass and (except at the very end) a row
// pass, then the final row pass that writes the state.
template <int N, typename T>
static void enqueue_cn_steps(const StepJob& job, int64_t grid_fields, hipStream_t st) {
  using RC = RowCfg<N, T>;
  using CC = ColCfg<N>;
  const cpx<T>* tw = (const cpx<T>*)(sizeof(T) == 8 ? (const void*)job.ws.tw64 : (const void*)job.ws.tw32);
  cpx<T>* spec = (cpx<T>*)job.ws.spec;
  cpx<T>* xs = (cpx<T>*)job.ws.xspec;
  const CallDesc* d = job.ws.desc;
  const dim3 grow((unsigned)(grid_fields * RC::TILES)), brow(RC::NT);
  const dim3 gcol((unsigned)(grid_fields * CC::BLOCKS)), bcol(CC::NT);
  k_row_first<N, T, RHS_U><<<grow, brow, 0, st>>>(d, xs, job.ws.partials, tw, job.sp);
  k_col_fwd<N, T><<<gcol, bcol, 0, st>>>(d, xs, tw);
  k_row_first<N, T, RHS_F><<<grow, brow, 0, st>>>(d, spec, job.ws.partials, tw, job.sp);
  const int M = job.picard;
  for (int s = 0; s < job.steps; ++s) {
    for (int m = 0; m < M; ++m) {
      const int mode = (m == 0 ? CN_FIRST : 0) | (m == M - 1 ? CN_LAST : 0);
      switch (mode) {
        case 0: launch_col_cn<N, T, 0>(job, gcol, bcol, st); break;
        case CN_FIRST: launch_col_cn<N, T, CN_FIRST>(job, gcol, bcol, st); break;
        case CN_LAST: launch_col_cn<N, T, CN_LAST>(job, gcol, bcol, st); break;
        default: launch_col_cn<N, T, CN_FIRST | CN_LAST>(job, gcol, bcol, st); break;
      }
      if (s + 1 < job.steps || m + 1 < M)
        k_row<N, T, ROW_MID, RHS_F><<<grow, brow, 0, st>>>(d, spec, job.ws.partials, tw, job.sp);
    }
  }
  k_row<N, T, ROW_LAST><<<grow, brow, 0, st>>>(d, spec, job.ws.partials, tw, job.sp);
}

template <int N, typename T>
static void enqueue_steps(const StepJob& job, int64_t grid_fields, hipStream_t st) {
  if (job.scheme == SCHEME_CN) {
    enqueue_cn_steps<N, T>(job, grid_fields, st);
  } else if constexpr (radix_split_differs<N>()) {
    if (job.radix == 1) enqueue_stream_steps<N, T, 1>(job, grid_fields, st);
    else enqueue_stream_steps<N, T, 0>(job, grid_fields, st);
  } else {
    enqueue_stream_steps<N, T, 0>(job, grid_fields, st);
  }
}

// ---- replay of captured launch sequences
//
// A streaming F call is 2c+1 launches whose arguments depend only on the
// problem, the step count and the workspace (everything else is read from
// the descriptor).  The sequence is captured once per such key and
// replayed; a replay serves any batch no larger than the captured grid.

struct GraphKey {
  int n, f32, steps, conservative, scheme, picard, radix;
  double a, dt, lam, inv_n2;
  const void *desc, *spec, *xspec, *partials, *tw, *s2;
  bool same(const GraphKey& o) const {
    return n == o.n && f32 == o.f32 && steps == o.steps && conservative == o.conservative &&
           scheme == o.scheme && picard == o.picard && radix == o.radix && a == o.a &&
           dt == o.dt && lam == o.lam &&
           inv_n2 == o.inv_n2 && desc == o.desc && spec == o.spec && xspec == o.xspec &&
           partials == o.partials && tw == o.tw && s2 == o.s2;
  }
};

struct GraphEntry {
  GraphKey key;
  int64_t grid_fields;
  hipGraph_t graph;
  hipGraphExec_t exec;
  hipEvent_t done;     // recorded after every launch of exec
  uint64_t last_use;
};

static std::mutex g_graph_mu;
static std::vector<GraphEntry> g_graphs;
static uint64_t g_graph_clock = 0;
static hipStream_t g_capture_stream = nullptr;
static std::atomic<bool> g_graphs_on{true};
constexpr size_t kMaxGraphs = 32;

void set_graphs_enabled(bool on) { g_graphs_on.store(on); }
bool graphs_enabled() { return g_graphs_on.load(); }

// Replays an entry on st and marks the launch with the entry's event.
// Called with g_graph_mu held.
static hipError_t replay(GraphEntry& e, hipStream_t st) {
  e.last_use = ++g_graph_clock;
  hipError_t err = hipGraphLaunch(e.exec, st);
  if (err != hipSuccess) return err;
  return hipEventRecord(e.done, st);
}

template <int N, typename T>
static hipError_t launch_stream_graph(const StepJob& job, hipStream_t st) {
  // with per-field parameters the launch argument is unused, and every
  // such sequence with the same shape and workspace is the same graph
  const StepParams sp = job.params ? StepParams{0, 0, 0, 0, -1} : job.sp;
  GraphKey key{job.n, job.f32 ? 1 : 0, job.steps, sp.conservative, job.scheme,
               job.scheme == SCHEME_CN ? job.picard : 0, job.scheme == SCHEME_CN ? 0 : job.radix,
               sp.a, sp.dt, sp.lam, sp.inv_n2,
               job.ws.desc, job.ws.spec, job.scheme == SCHEME_CN ? job.ws.xspec : nullptr,
               job.ws.partials, job.f32 ? (const void*)job.ws.tw32 : (const void*)job.ws.tw64,
               job.ws.s2};
  auto find = [&]() -> GraphEntry* {
    GraphEntry* hit = nullptr;
    for (auto& e : g_graphs)
      if (e.key.same(key) && e.grid_fields >= job.nfields &&
          (!hit || e.grid_fields < hit->grid_fields))
        hit = &e;
    return hit;
  };
  GraphEntry victim{};
  bool evict = false;
  {
    std::lock_guard<std::mutex> lock(g_graph_mu);
    if (GraphEntry* hit = find()) return replay(*hit, st);
    if (g_graphs.size() >= kMaxGraphs) {
      // take the least recently used entry out of the cache; it is
      // destroyed below, once its last launch has finished
      size_t lru = 0;
      for (size_t i = 1; i < g_graphs.size(); ++i)
        if (g_graphs[i].last_use < g_graphs[lru].last_use) lru = i;
      victim = g_graphs[lru];
      g_graphs.erase(g_graphs.begin() + lru);
      evict = true;
    }
  }
  if (evict) {
    // waits for that entry's work only (not the device), without the lock
    hipError_t err = hipEventSynchronize(victim.done);
    (void)hipGraphExecDestroy(victim.exec);
    (void)hipGraphDestroy(victim.graph);
    (void)hipEventDestroy(victim.done);
    if (err != hipSuccess) return err;
  }
  std::lock_guard<std::mutex> lock(g_graph_mu);
  if (GraphEntry* hit = find()) return replay(*hit, st);   // captured meanwhile
  hipError_t err;
  if (!g_capture_stream) {
    err = hipStreamCreateWithFlags(&g_capture_stream, hipStreamNonBlocking);
    if (err != hipSuccess) return err;
  }
  GraphEntry e{key, job.nfields, nullptr, nullptr, nullptr, 0};
  err = hipEventCreateWithFlags(&e.done, hipEventDisableTiming);
  if (err != hipSuccess) return err;
  err = hipStreamBeginCapture(g_capture_stream, hipStreamCaptureModeThreadLocal);
  if (err != hipSuccess) {
    (void)hipEventDestroy(e.done);
    return err;
  }
  enqueue_steps<N, T>(job, job.nfields, g_capture_stream);
  hipError_t lerr = hipGetLastError();
  err = hipStreamEndCapture(g_capture_stream, &e.graph);
  if (lerr == hipSuccess && err == hipSuccess)
    err = hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0);
  if (lerr != hipSuccess || err != hipSuccess) {
    if (e.graph) (void)hipGraphDestroy(e.graph);
    (void)hipEventDestroy(e.done);
    return lerr != hipSuccess ? lerr : err;
  }
  g_graphs.push_back(e);
  return replay(g_graphs.back(), st);
}

template <int N, typename T>
static hipError_t launch_steps_n(const StepJob& job, hipStream_t st) {
  if (graphs_enabled() && !job.eager) return launch_stream_graph<N, T>(job, st);
  enqueue_steps<N, T>(job, job.nfields, st);
  return hipGetLastError();
}

template <int N, typename T>
static hipError_t launch_resident_n(const StepJob& job, hipStream_t st) {
  if constexpr (N <= kResidentMaxN) {
    const cpx<T>* tw = (const cpx<T>*)(sizeof(T) == 8 ? (const void*)job.ws.tw64 : (const void*)job.ws.tw32);
    k_resident<N, T><<<dim3((unsigned)job.nfields), dim3(ResCfg<N>::NT), 0, st>>>(
        job.ws.desc, tw, job.ws.s2, job.sp, job.steps);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <typename T>
static hipError_t launch_resident_t(const StepJob& job, hipStream_t st) {
  switch (job.n) {
    case 16: return launch_resident_n<16, T>(job, st);
    case 32: return launch_resident_n<32, T>(job, st);
    case 64: return launch_resident_n<64, T>(job, st);
    case 128: return launch_resident_n<128, T>(job, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
static hipError_t launch_steps_t(const StepJob& job, hipStream_t st) {
  CallDesc v{job.nfields, job.in_base, job.in_offs, job.out_base, job.out_offs, job.out_f32,
             job.params, job.pidx};
  k_set_desc<<<dim3(1), dim3(1), 0, st>>>(job.ws.desc, v);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (job.resident && job.scheme == SCHEME_SSI) return launch_resident_t<T>(job, st);
  switch (job.n) {
    case 16: return launch_steps_n<16, T>(job, st);
    case 32: return launch_steps_n<32, T>(job, st);
    case 64: return launch_steps_n<64, T>(job, st);
    case 128: return launch_steps_n<128, T>(job, st);
    case 256: return launch_steps_n<256, T>(job, st);
    case 512: return launch_steps_n<512, T>(job, st);
    case 1024: return launch_steps_n<1024, T>(job, st);
    default: return hipErrorInvalidValue;
  }
}

// ---- the work-queue fine sweep: one persistent launch for many groups
//
// The semi-implicit F calls of several launch groups (fields of one size
// and precision each) run as one launch.  Its work items are the tiles of
// every pass of every field: for field f, phase 0 is the first row pass
// (RT row tiles), odd phases the column passes (CT column tiles) and even
// phases p > 0 the middle row passes, the last one (p = 2 steps) writing
// the state.  Items are numbered group by group; inside a group, working-
// set chunk by chunk (the same chunks as the launch-by-launch sweep), and
// inside a chunk phase by phase, field by field, tile by tile.  Blocks take
// the next item from a queue counter; an item of phase p of field f first
// waits until the field's counter shows every item of its phases < p done
// (the tiles of one pass depend only on the previous pass of the same
// field), then runs the same tile code as the per-pass kernels, then
// counts itself done.  An item only waits for items numbered before it,
// which blocks that are running have already taken, so every wait ends;
// blocks leave when the queue is empty.  Results are bitwise those of the
// per-pass launches.

__global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v);

constexpr int kQueueMaxGroups = 12;
constexpr int kQueueThreads = 256;
// One queue per XCD: the fields are split into kQueues contiguous ranges,
// and the blocks of the XCD whose index a queue carries take its items.
constexpr int kQueues = 8;

// Most tiles per work item: an item runs up to this many consecutive tiles
// of one pass of one field, so that the per-item synchronisation (a release
// before the field's counter is raised, an acquire after it is read) is
// paid once per group of tiles.  A launch halves it (down to 1) while a
// pass would give a queue fewer items than a quarter of its XCD's blocks
// (more, smaller items measured slower: with one field per queue every
// block then polls the same counter).
#ifndef PR_QUEUE_TILES
#define PR_QUEUE_TILES 8
#endif

struct QGroup {
  int n, f32, steps, rt, ct;    // tiles per row / column pass
  int tpi;                      // tiles per work item
  int rti, cti;                 // work items per row / column pass
  int64_t nfields, chunk, per_field, done0;
  int64_t lo[kQueues + 1];      // queue q takes fields [lo[q], lo[q + 1])
  int64_t item0[kQueues];       // first item of this group in queue q
  StepParams sp;
  FineWs ws;
};

struct QTotals {
  int64_t t[kQueues];           // items per queue
};

// Counter words (64-bit) in the queue workspace: the head of queue q at
// q * 16 and its mode at 128 + q * 16 (one 128-byte line each), then one
// completion counter per field.
constexpr int kQueueHeadWords = 256;
constexpr unsigned long long kModeLocal = 1, kModeShared = 2;

template <int N, typename T> struct QLds {
  using C = cpx<T>;
  static constexpr size_t al(size_t b) { return (b + 15) / 16 * 16; }
  static constexpr size_t ROW_PANEL = al(sizeof(C) * RowCfg<N, T>::PAIRS * RowLS<N, T>::value);
  static constexpr size_t ROW_TW = al(sizeof(C) * RowLS<N, T>::TWN);
  static constexpr size_t ROW = ROW_PANEL + ROW_TW + al(sizeof(double) * (RowCfg<N, T>::NT / 64 + 1));
  static constexpr size_t COL_PANEL = al(sizeof(C) * ColCfg<N>::CT * ColPanel<N, T>::value);
  static constexpr size_t COL_TW = al(sizeof(C) * ColPanel<N, T>::TWN);
  static constexpr size_t COL_S2 = PR_S2_LDS ? al(sizeof(double) * N) : 0;
  static constexpr size_t COL = COL_PANEL + COL_TW + COL_S2 + 16;
  static constexpr size_t BYTES = ROW > COL ? ROW : COL;
};

// Sizes and precisions whose row and column tiles both take 256 threads
// (FP32 tiles at 512^2 and 1024^2 take 512 and stay with per-pass launches).
template <int N, typename T> constexpr bool queue_item_ok() {
  return RowCfg<N, T>::NT == kQueueThreads && ColCfg<N>::NT == kQueueThreads;
}

template <int N, typename T>
__device__ __forceinline__ void q_item(unsigned char* lds, const QGroup& G, int p, int64_t f, int tile,
                                    int tid) {
  static_assert(queue_item_ok<N, T>(), "queue items are 256-thread tiles");
  using C = cpx<T>;
  using L = QLds<N, T>;
  const C* twg = (const C*)(sizeof(T) == 8 ? (const void*)G.ws.tw64 : (const void*)G.ws.tw32);
  C* spec = (C*)G.ws.spec;
  if (p & 1) {
    col_body<N, T>((C*)lds, (C*)(lds + L::COL_PANEL), (double*)(lds + L::COL_PANEL + L::COL_TW),
                   (double*)(lds + L::COL_PANEL + L::COL_TW + L::COL_S2), G.ws.desc, spec,
                   G.ws.partials, twg, G.ws.s2, G.sp, f, tile, tid);
  } else {
    C* panel = (C*)lds;
    C* tw_s = (C*)(lds + L::ROW_PANEL);
    double* red = (double*)(lds + L::ROW_PANEL + L::ROW_TW);
    if (p == 0)
      row_first_body<N, T>(panel, tw_s, red, G.ws.desc, spec, G.ws.partials, twg, G.sp, f, tile, tid);
    else if (p == 2 * G.steps)
      row_body<N, T, ROW_LAST>(panel, tw_s, red, G.ws.desc, spec, G.ws.partials, twg, G.sp, f, tile,
                               tid);
    else
      row_body<N, T, ROW_MID>(panel, tw_s, red, G.ws.desc, spec, G.ws.partials, twg, G.sp, f, tile,
                              tid);
  }
}

// Writes one entry of the launch's group table into device memory (a
// kernel rather than a copy, so that a captured graph replays it).
__global__ void k_set_group(QGroup g, QGroup* __restrict__ out) {
  if (threadIdx.x == 0) *out = g;
}

// Reads a value that thread 0 left in LDS into scalar registers: every
// decision taken on it is then a uniform branch.  (A loop whose exit the
// compiler takes for per-lane may be restructured so that lanes other than
// thread 0 re-enter its body without the update thread 0 made, and the
// block never leaves it.)
__device__ __forceinline__ int64_t q_uniform(const long long* sh) {
  const unsigned long long raw = (unsigned long long)*sh;
  return (int64_t)(((unsigned long long)__builtin_amdgcn_readfirstlane((int)(raw >> 32)) << 32) |
                   (unsigned)__builtin_amdgcn_readfirstlane((int)(raw & 0xffffffffu)));
}

// Runs the items of queue q until it is empty.  local: every block that
// takes items of q runs on one XCD, whose L2 all of them share; a tile's
// stores are then visible to the next pass's blocks once they have left
// the CU (waitcnt), and the reader only drops its CU's L1.  Otherwise the
// writer publishes with a device-scope release, which writes back the dirty
// lines of its L2.
template <int N, typename T>
__device__ __forceinline__ void q_drain(unsigned char* qlds, long long* sh, const QGroup* __restrict__ groups,
                                        int ngroups, int q, int64_t total,
                                        unsigned long long* __restrict__ qc, bool local, int tid) {
  unsigned long long* head = qc + q * 16;
  unsigned long long* done = qc + kQueueHeadWords;
  for (;;) {
    if (tid == 0) *sh = (long long)atomicAdd(head, 1ull);
    __syncthreads();
    const int64_t it = q_uniform(sh);
    __syncthreads();  // every thread has read sh before it is overwritten
    if (it >= total) break;
    int g = 0;
    while (g + 1 < ngroups && it >= groups[g + 1].item0[q]) ++g;
    const QGroup& G = groups[g];
    // a chunk holds fewer than 2^31 items (the host caps it), so past the
    // chunk index the decoding is 32-bit
    int64_t li = it - G.item0[q];
    const int64_t chunk_items = G.chunk * G.per_field;
    int64_t ck = 0;
    if (li >= chunk_items) {
      ck = li / chunk_items;
      li -= ck * chunk_items;
    }
    const int64_t lo = G.lo[q], hi = G.lo[q + 1];
    const int64_t f0 = lo + ck * G.chunk;
    const unsigned nf = (unsigned)(hi - f0 < G.chunk ? hi - f0 : G.chunk);
    const unsigned l = (unsigned)li;
    const unsigned pair = nf * (unsigned)(G.rti + G.cti);
    const unsigned ph = l / pair;
    unsigned rem = l - ph * pair;
    int p;
    unsigned per;
    int tiles;
    if (rem < nf * (unsigned)G.rti) {
      p = (int)(2 * ph);
      per = (unsigned)G.rti;
      tiles = G.rt;
    } else {
      p = (int)(2 * ph + 1);
      rem -= nf * (unsigned)G.rti;
      per = (unsigned)G.cti;
      tiles = G.ct;
    }
    const unsigned fi = rem / per;
    const int64_t f = f0 + fi;
    const int t0 = (int)(rem - fi * per) * G.tpi;
    const int t1 = t0 + G.tpi < tiles ? t0 + G.tpi : tiles;
    // items of this field in phases < p: (p + 1) / 2 row passes, p / 2 column passes
    const unsigned long long need =
        (unsigned long long)((p + 1) / 2) * G.rti + (unsigned long long)(p / 2) * G.cti;
    if (tid == 0 && need > 0) {
      // poll without cache maintenance; one acquire once the count is there
      while (__hip_atomic_load(&done[G.done0 + f], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need)
        __builtin_amdgcn_s_sleep(2);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    for (int tile = t0; tile < t1; ++tile) {
      q_item<N, T>(qlds, G, p, f, tile, tid);
      __syncthreads();  // the tile's LDS is free for the next one
    }
    if (local)
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this wave's stores are in the L2
    else
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // and written back from it
    __syncthreads();
    if (tid == 0) {
      if (local)
        __hip_atomic_fetch_add(&done[G.done0 + f], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      else
        __hip_atomic_fetch_add(&done[G.done0 + f], 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    // a barrier between this thread-0 region and the next iteration's:
    // without it the compiler may join the two into one path for thread 0
    // that bypasses the loop head the other threads return to
    __syncthreads();
  }
}

// The block's XCD, from the hardware register that names it (4 bits).
__device__ __forceinline__ int q_xcd() {
  return (int)(__builtin_amdgcn_s_getreg((3 << 11) | 20) & 15u);
}

// Persistent blocks; queue q holds the items of fields [lo[q], lo[q + 1])
// of every group.  A block first serves the queue of its own XCD, then
// helps with any queue that no block of its XCD has claimed.  Each queue's
// mode is fixed once, by whichever block comes first: local if a block of
// its XCD claims it (then only blocks of that XCD take its items), shared
// if a block of another XCD adopts it (every block that takes its items
// then publishes device-wide).  Every queue is drained whatever the
// placement of the blocks: a queue no block of its XCD reaches is adopted
// by the first block to run out of work (local_ok = 0 makes every queue
// adopted: the device-wide hand-over alone).  (Blocks are dealt out to the
// XCDs round-robin, but the deal carries on from one launch to the next,
// so block b is not on XCD b mod 8 in general: the register decides.)
// Registers bounded for 3 waves per SIMD (2 at 1024^2): the row and column
// bodies in one kernel need more registers than either per-pass kernel,
// and the bound, with a few spilled bytes, measured faster than the
// occupancy left unbounded (512^2 FP64, 2048 fields, 100 steps: 432 ->
// 398 ms; bounded to 4 waves it spills more and was slower).
template <int N, typename T>
__global__ __launch_bounds__(kQueueThreads) __attribute__((amdgpu_waves_per_eu(N >= 1024 ? 2 : 3))) void k_fine_queue(const QGroup* __restrict__ groups,
                                                              int ngroups, QTotals tot,
                                                              unsigned long long* __restrict__ qc,
                                                              int local_ok) {
  extern __shared__ __align__(16) unsigned char qlds[];
  __shared__ long long sh;
  const int tid = threadIdx.x;
  unsigned long long* mode = qc + 128;
  const int xcd = q_xcd();
  const int home = local_ok && xcd < kQueues ? xcd : -1;
  const int start = home >= 0 ? home + 1 : (int)(blockIdx.x % kQueues);
  // i = -1: the home queue; then every other queue, to adopt
  for (int i = home >= 0 ? -1 : 0; i < kQueues; ++i) {
    const int q = i < 0 ? home : (start + i) % kQueues;
    if (i >= 0 && q == home) continue;
    const int64_t total = tot.t[q];
    if (total == 0) continue;
    if (tid == 0) {
      unsigned long long m = 0;
      if (i < 0) {
        if (__hip_atomic_compare_exchange_strong(&mode[q * 16], &m, kModeLocal, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
          m = kModeLocal;
      } else {
        m = __hip_atomic_load(&mode[q * 16], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // give the blocks of q's own XCD time to claim it first (bounded)
        for (int w = 0; w < 16 && m == 0 && local_ok; ++w) {
          __builtin_amdgcn_s_sleep(127);
          m = __hip_atomic_load(&mode[q * 16], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (m == 0 && __hip_atomic_compare_exchange_strong(&mode[q * 16], &m, kModeShared,
                                                           __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT))
          m = kModeShared;
      }
      sh = (long long)m;
    }
    __syncthreads();
    const int64_t m = q_uniform(&sh);
    __syncthreads();
    // the home queue in either mode; another queue only once adopted
    if (i < 0 || m == (int64_t)kModeShared)
      q_drain<N, T>(qlds, &sh, groups, ngroups, q, total, qc, m == (int64_t)kModeLocal, tid);
  }
}

static std::atomic<int> g_fine_queue{0};   // 0 off, 1 on, 2 on with every queue adopted
void set_fine_queue(int mode) { g_fine_queue.store(mode); }
int fine_queue_mode() { return g_fine_queue.load(); }
bool fine_queue_enabled() { return g_fine_queue.load() != 0; }

// The autotuner's choice per (log2 N, FP32): 0 none, 1 pass by pass, 2 queue.
static std::atomic<int> g_queue_tuned[11][2];
static int qlog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}
void record_fine_queue(int n, bool f32, bool queue) {
  const int l = qlog2(n);
  if (l >= 0 && l <= 10) g_queue_tuned[l][f32 ? 1 : 0].store(queue ? 2 : 1);
}
bool fine_queue_tuned(int n, bool f32) {
  const int l = qlog2(n);
  return l >= 0 && l <= 10 && g_queue_tuned[l][f32 ? 1 : 0].load() == 2;
}
bool fine_queue_use(const StepJob& job) {
  if (!fine_queue_supports(job)) return false;
  return fine_queue_enabled() || fine_queue_tuned(job.n, job.f32);
}

static int col_blocks(int n);

bool fine_queue_supports(const StepJob& job) {
  if (job.scheme != SCHEME_SSI) return false;
  // one field's items are counted in 31 bits
  if ((int64_t)(job.steps + 1) * (row_tiles(job.n, job.f32) + col_blocks(job.n)) >= INT32_MAX) return false;
  switch (job.n) {
#define PR_CASE(NN) \
  case NN: return job.f32 ? queue_item_ok<NN, float>() : queue_item_ok<NN, double>();
    PR_CASE(64) PR_CASE(128) PR_CASE(256) PR_CASE(512) PR_CASE(1024)
#undef PR_CASE
    default: return false;
  }
}

size_t fine_queue_ws_bytes(int64_t total_fields) {
  return (size_t)(kQueueHeadWords + total_fields) * sizeof(unsigned long long) +
         sizeof(QGroup) * kQueueMaxGroups + 512;
}

static int col_blocks(int n) {
  switch (n) {
#define PR_CASE(NN) case NN: return ColCfg<NN>::BLOCKS;
    PR_CASE(16) PR_CASE(32) PR_CASE(64) PR_CASE(128) PR_CASE(256) PR_CASE(512) PR_CASE(1024)
#undef PR_CASE
    default: return 0;
  }
}

// Blocks of the queue kernel for (N, T) that fill the GPU once.
template <int N, typename T> static hipError_t queue_grid(int* grid) {
  static int g = 0;
  static hipError_t attr = hipSuccess;
  static std::once_flag once;
  std::call_once(once, [] {
    constexpr size_t lds = QLds<N, T>::BYTES;
    if (lds > 64 * 1024)
      attr = hipFuncSetAttribute((const void*)k_fine_queue<N, T>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    int dev = 0, cus = 0, per_cu = 0;
    if (attr == hipSuccess) attr = hipGetDevice(&dev);
    if (attr == hipSuccess)
      attr = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (attr == hipSuccess)
      attr = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fine_queue<N, T>, kQueueThreads,
                                                          lds);
    g = std::max(1, cus * std::max(1, per_cu));
  });
  *grid = g;
  return attr;
}

template <int N, typename T>
static hipError_t queue_launch(const QGroup* gtab, int ngroups, const QTotals& tot,
                               unsigned long long* qc, hipStream_t st) {
  if constexpr (queue_item_ok<N, T>()) {
    int grid = 0;
    hipError_t e = queue_grid<N, T>(&grid);
    if (e != hipSuccess) return e;
    k_fine_queue<N, T><<<dim3((unsigned)grid), dim3(kQueueThreads), QLds<N, T>::BYTES, st>>>(
        gtab, ngroups, tot, qc, fine_queue_mode() == 2 ? 0 : 1);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

// Blocks of the queue kernel for (n, precision) (0: no such kernel).
static int queue_blocks(int n, bool f32) {
  int grid = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (n) {
#define PR_QB(NN)                                                                                  \
  case NN:                                                                                         \
    if (f32) {                                                                                     \
      if constexpr (queue_item_ok<NN, float>()) e = queue_grid<NN, float>(&grid);                 \
    } else {                                                                                       \
      if constexpr (queue_item_ok<NN, double>()) e = queue_grid<NN, double>(&grid);               \
    }                                                                                              \
    break;
    PR_QB(64) PR_QB(128) PR_QB(256) PR_QB(512) PR_QB(1024)
#undef PR_QB
    default: break;
  }
  return e == hipSuccess ? grid : 0;
}

// One persistent launch per (N, precision) class of the jobs, in the order
// the classes first appear (a batch of one class: one launch).
hipError_t launch_fine_queue(const StepJob* jobs, int njobs, void* qws, hipStream_t st) {
  // workspace: the group table, then the counters
  QGroup* gtab = (QGroup*)((char*)qws + 256);
  unsigned long long* qc =
      (unsigned long long*)((char*)qws + 256 + (sizeof(QGroup) * kQueueMaxGroups + 255) / 256 * 256);
  std::vector<char> taken(njobs, 0);
  for (int i0 = 0; i0 < njobs; ++i0) {
    if (taken[i0]) continue;
    const int n = jobs[i0].n;
    const bool f32 = jobs[i0].f32;
    const int per_queue = std::max(1, queue_blocks(n, f32) / kQueues);   // blocks per XCD
    QGroup gs[kQueueMaxGroups];
    QTotals tot{};
    int ngroups = 0;
    int64_t fields = 0;
    for (int i = i0; i < njobs && ngroups < kQueueMaxGroups; ++i) {
      const StepJob& j = jobs[i];
      if (taken[i] || j.n != n || j.f32 != f32) continue;
      if (!fine_queue_supports(j)) return hipErrorInvalidValue;
      taken[i] = 1;
      if (j.nfields <= 0 || j.steps <= 0) continue;
      CallDesc v{j.nfields, j.in_base, j.in_offs, j.out_base, j.out_offs, j.out_f32, j.params, j.pidx};
      k_set_desc<<<dim3(1), dim3(1), 0, st>>>(j.ws.desc, v);
      QGroup& G = gs[ngroups++];
      G = QGroup{};
      G.n = j.n;
      G.f32 = j.f32 ? 1 : 0;
      G.steps = j.steps;
      G.rt = row_tiles(j.n, j.f32);
      G.ct = col_blocks(j.n);
      // tiles per item: the most that still give a quarter of a queue's
      // blocks an item of each pass
      const int64_t fq = (j.nfields + kQueues - 1) / kQueues;
      G.tpi = PR_QUEUE_TILES;
      while (G.tpi > 1 && 4 * fq * ((G.rt + G.tpi - 1) / G.tpi) < per_queue) G.tpi /= 2;
      G.rti = (G.rt + G.tpi - 1) / G.tpi;
      G.cti = (G.ct + G.tpi - 1) / G.tpi;
      G.nfields = j.nfields;
      StepJob sj = j;
      sj.resident = false;
      // the working-set chunk is shared out among the queues, which run
      // side by side
      G.chunk = std::max<int64_t>(1, (chunk_fields(sj) + kQueues - 1) / kQueues);
      G.per_field = (int64_t)(j.steps + 1) * G.rti + (int64_t)j.steps * G.cti;
      // a chunk's items are decoded in 32 bits
      G.chunk = std::min<int64_t>(G.chunk, std::max<int64_t>(1, INT32_MAX / G.per_field));
      G.done0 = fields;
      // contiguous field ranges of near-equal size; the queues that take
      // one field more rotate with the fields placed so far
      const int rot = (int)(fields % kQueues);
      G.lo[0] = 0;
      for (int q = 0; q < kQueues; ++q)
        G.lo[q + 1] = G.lo[q] + j.nfields / kQueues +
                      (((q - rot + kQueues) % kQueues) < j.nfields % kQueues ? 1 : 0);
      for (int q = 0; q < kQueues; ++q) {
        G.item0[q] = tot.t[q];
        tot.t[q] += (G.lo[q + 1] - G.lo[q]) * G.per_field;
      }
      G.sp = j.sp;
      G.ws = j.ws;
      fields += j.nfields;
    }
    if (ngroups == 0) continue;
    --i0;   // the same class may hold more groups than one launch takes
    // counters: the queue heads and modes, then one per field (kernels, so
    // that a captured graph replays the clearing)
    const int64_t nc = kQueueHeadWords + fields;
    k_fill_u64<<<dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st>>>(qc, nc, 0ull);
    for (int g = 0; g < ngroups; ++g) k_set_group<<<dim3(1), dim3(64), 0, st>>>(gs[g], gtab + g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (n) {
#define PR_QCASE(NN) \
  case NN:                                                                            \
    e = f32 ? queue_launch<NN, float>(gtab, ngroups, tot, qc, st)                       \
            : queue_launch<NN, double>(gtab, ngroups, tot, qc, st);                    \
    break;
      PR_QCASE(64) PR_QCASE(128) PR_QCASE(256) PR_QCASE(512) PR_QCASE(1024)
#undef PR_QCASE
      default: e = hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_tables(int n, int laplacian, const FineWs& ws, hipStream_t st) {
  k_tables<<<dim3((n + 255) / 256), dim3(256), 0, st>>>(n, laplacian, ws.tw64, ws.tw32, ws.s2);
  return hipGetLastError();
}

// ---- working-set chunking
//
// A streaming F call moves every field's spectrum through two passes per
// step.  While the spectra of the fields in flight fit in the GPU's last-
// level cache (the 256 MB MALL of an MI355X), much of each pass's input is
// still cached from the previous pass; measured at 512^2 in FP64, 128
// fields per call (268 MB of spectra) run at 5.5 TB/s and 512 at 4.4.  So
// a call with more fields runs them in consecutive chunks whose spectra
// fit the working-set budget, each chunk through all of its steps.  The
// fields' arithmetic does not depend on the chunking.

static std::atomic<int64_t> g_ws_budget{256ll << 20};   // bytes; 0 = no chunking
static std::atomic<int64_t> g_ws_tuned[11][2];           // per (log2 N, f32): -1 none

static int log2n(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

void set_working_set(int64_t bytes) { g_ws_budget.store(bytes); }

int64_t working_set(int n, bool f32) {
  const int l = log2n(n);
  if (l >= 0 && l <= 10) {
    const int64_t t = g_ws_tuned[l][f32 ? 1 : 0].load();
    if (t > 0) return t == 1 ? 0 : t;   // 1 records "no chunking"
  }
  return g_ws_budget.load();
}

void record_working_set(int n, bool f32, int64_t bytes) {
  const int l = log2n(n);
  if (l >= 0 && l <= 10) g_ws_tuned[l][f32 ? 1 : 0].store(bytes == 0 ? 1 : bytes);
}

int64_t chunk_fields(const StepJob& job) {
  if (job.resident && job.scheme == SCHEME_SSI) return job.nfields;   // nothing streams
  const int64_t budget = job.ws_override >= 0 ? job.ws_override : working_set(job.n, job.f32);
  if (budget <= 0) return job.nfields;
  const int64_t per = (int64_t)job.n * job.n * (job.f32 ? 4 : 8) * (job.scheme == SCHEME_CN ? 2 : 1);
  return std::max<int64_t>(1, std::min<int64_t>(job.nfields, budget / per));
}

hipError_t launch_steps(const StepJob& job, hipStream_t st) {
  if (job.nfields <= 0 || job.steps <= 0) return hipSuccess;
  const int64_t chunk = chunk_fields(job);
  const int64_t n2 = (int64_t)job.n * job.n;
  for (int64_t c0 = 0; c0 < job.nfields; c0 += chunk) {
    StepJob sub = job;
    sub.nfields = std::min(chunk, job.nfields - c0);
    if (c0 > 0) {
      if (job.in_offs) sub.in_offs = job.in_offs + c0;
      else sub.in_base = job.in_base + c0 * n2;
      if (job.out_offs) sub.out_offs = job.out_offs + c0;
      else sub.out_base = (char*)job.out_base + c0 * n2 * (job.out_f32 ? 4 : 8);
      if (job.pidx) sub.pidx = job.pidx + c0;
    }
    const hipError_t e = job.f32 ? launch_steps_t<float>(sub, st) : launch_steps_t<double>(sub, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int row_tiles(int n, bool f32) {
  switch (n) {
#define PR_CASE(NN) \
  case NN: return f32 ? RowCfg<NN, float>::TILES : RowCfg<NN, double>::TILES;
    PR_CASE(16) PR_CASE(32) PR_CASE(64) PR_CASE(128) PR_CASE(256) PR_CASE(512) PR_CASE(1024)
#undef PR_CASE
    default: return 0;
  }
}

// ------------------------------------------------- correction and norm

// Block b of field fld takes points b * 1024 + k * 256 + threadIdx.x,
// k < 4 (coalesced, four independent loads of each operand in flight);
// the block's maximum goes to upd with at most one atomic.
template <typename TF>
__global__ __launch_bounds__(256) void k_correct(
    int64_t n2, const TF* __restrict__ fb, const int64_t* __restrict__ f_offs,
    const double* __restrict__ gnb, const int64_t* __restrict__ gn_offs,
    double* __restrict__ gob, const int64_t* __restrict__ go_offs,
    double* __restrict__ ub, const int64_t* __restrict__ u_offs,
    unsigned long long* __restrict__ upd, const int32_t* __restrict__ upd_idx,
    int update_cache, int blocks_per_field) {
  constexpr int PPT = 4;
  __shared__ unsigned long long red[4];
  const int64_t fld = blockIdx.x / blocks_per_field;
  const int64_t part = blockIdx.x % blocks_per_field;
  const TF* fp = fb + (f_offs ? f_offs[fld] : fld * n2);
  const double* gn = gnb + (gn_offs ? gn_offs[fld] : fld * n2);
  double* go = gob + (go_offs ? go_offs[fld] : fld * n2);
  double* u = ub + (u_offs ? u_offs[fld] : fld * n2);
  unsigned long long m = 0;
  const int64_t i0 = part * (256 * PPT) + threadIdx.x;
  double g1[PPT], f[PPT], g0[PPT], u0[PPT];
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int64_t i = i0 + k * 256;
    if (i < n2) {
      g1[k] = gn[i];
      f[k] = (double)fp[i];
      g0[k] = go[i];
      u0[k] = u[i];
    }
  }
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int64_t i = i0 + k * 256;
    if (i < n2) {
      // U^k_{j+1} = F(U^{k-1}_j) + (G(U^k_j) - G(U^{k-1}_j)), in this order
      const double un = f[k] + (g1[k] - g0[k]);
      const double d = fabs(un - u0[k]);
      u[i] = un;
      if (update_cache) go[i] = g1[k];
      // |d| >= 0, so its bit pattern orders like its value; NaN (sign
      // cleared) sorts above +Inf and therefore survives the max
      const unsigned long long bits = (unsigned long long)__double_as_longlong(d);
      m = bits > m ? bits : m;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long t = __shfl_xor(m, o, 64);
    m = t > m ? t : m;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long r = red[0];
#pragma unroll
    for (int w = 1; w < 4; ++w) r = red[w] > r ? red[w] : r;
    // the norm only grows: a maximum not above the stored value cannot
    // change it, and skipping its atomic spares the contended address
    unsigned long long* dst = &upd[upd_idx ? upd_idx[fld] : fld];
    if (r > __atomic_load_n(dst, __ATOMIC_RELAXED)) atomicMax(dst, r);
  }
}

hipError_t launch_correct(const CorrectJob& j, hipStream_t st) {
  if (j.nfields <= 0) return hipSuccess;
  const int64_t n2 = (int64_t)j.n * j.n;
  const int bpf = (int)((n2 + 1023) / 1024);  // 256 threads x 4 points
  const dim3 grid((unsigned)(j.nfields * bpf)), block(256);
  if (j.f_f32)
    k_correct<float><<<grid, block, 0, st>>>(n2, (const float*)j.f, j.f_offs, j.g_new, j.gn_offs,
                                             j.g_old, j.go_offs, j.u, j.u_offs, j.upd, j.upd_idx,
                                             j.update_cache, bpf);
  else
    k_correct<double><<<grid, block, 0, st>>>(n2, (const double*)j.f, j.f_offs, j.g_new, j.gn_offs,
                                              j.g_old, j.go_offs, j.u, j.u_offs, j.upd, j.upd_idx,
                                              j.update_cache, bpf);
  return hipGetLastError();
}

// -------------------------------------------------------------- copies

__global__ __launch_bounds__(256) void k_copy_fields(int64_t n2, const double* __restrict__ src,
                                                     const int64_t* __restrict__ s_offs,
                                                     double* __restrict__ dst,
                                                     const int64_t* __restrict__ d_offs,
                                                     int blocks_per_field) {
  const int64_t fld = blockIdx.x / blocks_per_field;
  const int64_t part = blockIdx.x % blocks_per_field;
  const double* s = src + (s_offs ? s_offs[fld] : fld * n2);
  double* d = dst + (d_offs ? d_offs[fld] : fld * n2);
  // points part * 1024 + k * 256 + threadIdx.x, k < 4: loads issued together
  const int64_t i0 = part * 1024 + threadIdx.x;
  double v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (i0 + k * 256 < n2) v[k] = s[i0 + k * 256];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (i0 + k * 256 < n2) d[i0 + k * 256] = v[k];
}

hipError_t launch_copy(int64_t nfields, int n, const double* src, const int64_t* s_offs,
                       double* dst, const int64_t* d_offs, hipStream_t st) {
  if (nfields <= 0) return hipSuccess;
  const int64_t n2 = (int64_t)n * n;
  const int bpf = (int)((n2 + 1023) / 1024);  // 256 threads x 4 points
  k_copy_fields<<<dim3((unsigned)(nfields * bpf)), dim3(256), 0, st>>>(n2, src, s_offs, dst,
                                                                       d_offs, bpf);
  return hipGetLastError();
}

__global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_fill_u64<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(p, n, v);
  return hipGetLastError();
}

}  // namespace pr
