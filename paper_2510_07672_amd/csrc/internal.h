// Internal interface between the C ABI (api.hip) and the kernels
// (fine_kernels.hip).  Not installed; include/pr.h is the public header.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pr {

enum { ROW_FIRST = 0, ROW_MID = 1, ROW_LAST = 2 };

// Fine schemes and discrete Laplacians (same values as in include/pr.h).
enum { SCHEME_SSI = 0, SCHEME_CN = 1 };
enum { LAP_FD5 = 0, LAP_SPECTRAL = 1 };

// What a row pass transforms: the semi-implicit right-hand side
// (1 + S dt) v + dt f(v), f(v) alone, or v itself.
enum { RHS_SSI = 0, RHS_F = 1, RHS_U = 2 };

// Row pass tiling: TR rows (TR/2 complex row pairs) of one field per block,
// one radix-8 group of eight elements per thread per FFT stage.  TR is the
// smallest even count that gives >= 256 threads and >= 128-byte contiguous
// runs per spectral column, capped at N.
#ifndef PR_ROW_RUN_BYTES
#define PR_ROW_RUN_BYTES 128   // contiguous bytes per spectral column in a row tile
#endif
#ifndef PR_ROW_PANEL_BYTES
#define PR_ROW_PANEL_BYTES 40960   // cap on the row tile's LDS panel (bytes)
#endif
#ifndef PR_COL_THREADS
#define PR_COL_THREADS 256     // threads of a column-pass block (N <= 2048 / CT)
#endif

constexpr int pow2_floor(int v) {
  int p = 1;
  while (p * 2 <= v) p *= 2;
  return p;
}

template <int N, typename T> struct RowCfg {
  static constexpr int kThreads = 4096 / N;                                   // >= 256 threads
  static constexpr int kCoalesce = PR_ROW_RUN_BYTES / (2 * (int)sizeof(T));  // run length
  static constexpr int kMaxThreads = 16384 / N;                               // <= 1024 threads
  static constexpr int kMaxLds = 2 * (PR_ROW_PANEL_BYTES / ((N + N / 8 + 1) * 2 * (int)sizeof(T)));
  static constexpr int kT0 = kThreads > kCoalesce ? kThreads : kCoalesce;
  static constexpr int kT1 = kT0 < kMaxThreads ? kT0 : kMaxThreads;
  static constexpr int kT2 = pow2_floor(kT1 < kMaxLds ? kT1 : kMaxLds);
  static constexpr int TR = kT2 < N ? kT2 : N;
  static constexpr int PAIRS = TR / 2;
  static constexpr int NT = PAIRS * N / 8;
  static constexpr int TILES = N / TR;
};

// Column pass tiling: CT whole columns of one field per block.
template <int N> struct ColCfg {
  static constexpr int kC0 = PR_COL_THREADS * 8 / N;
  static constexpr int CT = kC0 < N / 2 ? kC0 : N / 2;
  static constexpr int NT = CT * N / 8;
  static constexpr int BLOCKS = (N / 2) / CT;
};

// Largest N whose whole spectrum one block keeps in LDS (FP64: 148 KB).
constexpr int kResidentMaxN = 128;

struct StepParams {
  double a;       // 1 + S dt
  double dt;      // step
  double lam;     // dt eps^2 4 / h^2
  double inv_n2;  // 1 / N^2
  int conservative;
};

// What changes from one call of the step kernels to the next, kept in
// device memory so that a captured launch sequence can be replayed for
// any batch that fits its grid.
struct CallDesc {
  int64_t nfields;          // live fields; blocks beyond them exit
  const double* in_base;    // field i at in_base + (in_offs ? in_offs[i] : i N^2)
  const int64_t* in_offs;
  void* out_base;           // field i at out_base + (out_offs ? out_offs[i] : i N^2)
  const int64_t* out_offs;
  int32_t out_f32;
  const StepParams* params;  // per-field step parameters params[pidx[i]] (null:
  const int32_t* pidx;       // the launch argument); lets one launch carry fields
                             // of problems with different eps, dt, S or model
};

// Per-call device workspace of the step kernels.
struct FineWs {
  CallDesc* desc;    // one descriptor
  double2* tw64;     // [N]  exp(-2 pi i t / N)
  float2* tw32;      // [N]  same, rounded
  double* s2;        // [N]  sin^2(pi t / N)
  double* partials;  // [nfields * row tiles] FP64 partial sums of f
  void* spec;        // [nfields][N/2][N] complex in the step precision
  void* xspec;       // Crank-Nicolson only: [nfields][N/2][N] 2-D spectra
                     // (U_n between steps, the fixed part K during Picard)
  void* queue;       // the work-queue sweep's table and counters
                     // (fine_queue_ws_bytes(nfields))
};

struct StepJob {
  int n;
  bool f32;
  int steps;
  int scheme = SCHEME_SSI;
  int picard = 1;            // Crank-Nicolson: Picard iterations per step
  int64_t nfields;
  StepParams sp;
  const double* in_base;     // field i at in_base + (in_offs ? in_offs[i] : i N^2)
  const int64_t* in_offs;    // device or null
  void* out_base;            // field i at out_base + (out_offs ? out_offs[i] : i N^2)
  const int64_t* out_offs;   // device or null
  int out_f32;
  const StepParams* params;  // device or null: per-field parameters (see CallDesc)
  const int32_t* pidx;       // device or null
  bool resident;             // one block per field, all steps in LDS (N <= 128)
  int64_t ws_override = -1;  // working-set budget in bytes for this call (-1: the setting)
  bool eager = false;        // launch kernel by kernel even with graphs on
  int radix = 0;             // FFT radix split of the streaming semi-implicit passes (0, 1)
  FineWs ws;
};

struct CorrectJob {
  int64_t nfields;
  int n;
  const void* f; const int64_t* f_offs; int f_f32;
  const double* g_new; const int64_t* gn_offs;
  double* g_old; const int64_t* go_offs;
  double* u; const int64_t* u_offs;
  unsigned long long* upd; const int32_t* upd_idx;
  int update_cache;
};

// ---- convolutional coarse propagator

enum { kActGelu = 0, kActTanh = 1 };
enum { kCnnF64 = 0, kCnnF32 = 1, kCnnBf16 = 2, kCnnBf16x2 = 3 };   // same values as pr_dtype
constexpr int kCnnF64MaxC = 32;   // widest FP64 network whose tiles fit in LDS

// Tile groups of the first stage of the weight-gradient reduction.
constexpr int kWGradGroups = 64;

struct CnnWs {
  void* wpack;       // bfloat16 [L-2][C][KP] packed hidden-layer weights, then
                     // the last layer's [KB][hi, lo][64 lanes][8] fragments
  void* act[2];      // ping-pong activations [nfields][N][N][C] (x2 for hi+lo)
  double* partials;  // [nfields][(N/16)^2] FP64 sums of G(u) - u
  // backward only
  void* acts;        // [L-1] activations of every layer but the last
  void* zs;          // [L-1] pre-activations
  double* o1;        // [nfields][N][N] forward output before the limiter
  double* wpart;     // [tiles][params] weight-gradient partial sums
  double* wpart2;    // [kWGradGroups][params] their sums over groups of tiles
  void* d[2];        // gradient buffers [nfields][N][N][C]
  double* fpart;     // per-field partial sums of the output-stage gradient
};

struct CnnJob {
  int n, n_layers, channels, prec, act, residual, mass_fix, limiter;
  double lim_lo, lim_hi;
  int64_t nfields;
  const void* W;             // concatenated torch Conv2d weights (double for F64, else float)
  const void* B;             // concatenated biases
  const double* in_base;     // field i at in_base + (in_offs ? in_offs[i] : i N^2)
  const int64_t* in_offs;
  double* out_base;
  const int64_t* out_offs;
  CnnWs ws;
  // Parareal correction to apply after the forward pass (inference), field
  // i of this job being field i of the correction, whose g_new addresses
  // the output; the folded plan's last kernel applies it without storing
  // the output (at C = 32, without mass fix or limiter), else launch_cnn
  // runs it on the stored output.  nullptr: none.
  const CorrectJob* corr;
  // a second destination of the output (field i at out2_base +
  // out2_offs[i]), written by the last kernel where it can, else copied
  // after the forward pass; nullptr: none.  Inference, without corr.
  double* out2_base;
  const int64_t* out2_offs;
};

// Inference plan of the network: one layer per launch, all layers in one
// fused kernel (bf16 kinds, shapes with a fused instantiation), or one
// layer per launch with the first layer inside the first hidden layer's
// launch (bf16 kinds with at least one hidden layer).
enum { CNN_PLAN_AUTO = 0, CNN_PLAN_LAYERED = 1, CNN_PLAN_FUSED = 2, CNN_PLAN_FOLDED = 3 };
bool cnn_fused_available(int C, int L, int prec);
bool cnn_folded_available(int C, int L, int prec);
int cnn_effective_plan(int C, int L, int prec);
void cnn_set_plan(int plan);
int cnn_get_plan();
void cnn_record_tuned(int C, int L, int prec, int plan);
// Output tile of the bf16 hidden layers (layered and folded plans): the
// pr_cnn_tile values; cnn_effective_tile returns 0 for 8 x 32, 1 for 16 x 16.
enum { CNN_TILE_AUTO = 0, CNN_TILE_8X32 = 1, CNN_TILE_16X16 = 2 };
int cnn_effective_tile(int C, int prec, int n);
void cnn_set_tile(int tile);
int cnn_get_tile();
void cnn_record_tile(int C, int prec, int n, int shape);

hipError_t launch_cnn_pack(const CnnJob& j, hipStream_t st);
hipError_t launch_cnn(const CnnJob& j, hipStream_t st);
hipError_t launch_cnn_backward(const CnnJob& j, const double* dG, double* du, void* gW, void* gB,
                               hipStream_t st);
int cnn_act_bytes(int prec);
int cnn_grad_bytes(int prec);
size_t cnn_lds_bytes(int C, bool split, bool first = false, int shape = 0);
hipError_t cnn_set_lds_limits();

hipError_t launch_tables(int n, int laplacian, const FineWs& ws, hipStream_t st);
// Process-wide switch for replaying captured launch sequences (default on).
void set_graphs_enabled(bool on);
bool graphs_enabled();
hipError_t launch_steps(const StepJob& job, hipStream_t st);

// The work-queue fine sweep: the semi-implicit F calls of several jobs as
// one persistent launch per (N, precision) class, bitwise equal to
// launch_steps of each.  Supported: N in 64..1024 in FP64, 64..256 in FP32,
// semi-implicit scheme.  qws: fine_queue_ws_bytes(sum of the jobs' fields).
bool fine_queue_supports(const StepJob& job);
size_t fine_queue_ws_bytes(int64_t total_fields);
hipError_t launch_fine_queue(const StepJob* jobs, int njobs, void* qws, hipStream_t st);
// Whether N has a second FFT radix split (StepJob::radix = 1: a trailing
// 8 x 2 as 4 x 4; N = 16, 128, 1024), built for the streaming
// semi-implicit passes.
bool fine_radix_differs(int n);
void set_fine_queue(int mode);   // 0 off, 1 on, 2 on with no XCD-local hand-over
int fine_queue_mode();
bool fine_queue_enabled();
// The autotuner's record for (n, precision), and whether a job takes the
// queue: supported, and the queue on or recorded faster for its class.
void record_fine_queue(int n, bool f32, bool queue);
bool fine_queue_tuned(int n, bool f32);
bool fine_queue_use(const StepJob& job);
// Working-set budget of streaming F calls (bytes of spectra in flight; 0 =
// all fields at once): the process-wide setting, the effective value for
// (N, precision) and the autotuner's record.
void set_working_set(int64_t bytes);
int64_t working_set(int n, bool f32);
void record_working_set(int n, bool f32, int64_t bytes);
int64_t chunk_fields(const StepJob& job);
hipError_t launch_correct(const CorrectJob& job, hipStream_t st);
hipError_t launch_copy(int64_t nfields, int n, const double* src, const int64_t* s_offs,
                       double* dst, const int64_t* d_offs, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v,
                           hipStream_t st);
int row_tiles(int n, bool f32);

}  // namespace pr
