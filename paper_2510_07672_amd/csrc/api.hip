// C ABI of libpr (declared in include/pr.h): argument checks, workspace
// carving and the Parareal driver of Algorithm 2 (Section 3.3) around the
// kernels of fine_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <mutex>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pr.h"
#include "internal.h"
#include "loss_kernels.h"

using namespace pr;

namespace {

thread_local std::string g_last_error;

pr_status fail(pr_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
pr_status fail(pr_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

#define PR_HIP(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      return fail(PR_ERR_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_));  \
  } while (0)

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

pr_status check_problem(const pr_problem* p) {
  if (!p) return fail(PR_ERR_INVALID_ARG, "problem is NULL");
  if (p->dim != 2) return fail(PR_ERR_UNSUPPORTED, "dim=%d: only 2-D is supported", p->dim);
  if (!is_pow2(p->n) || p->n < 16 || p->n > 1024)
    return fail(PR_ERR_UNSUPPORTED, "n=%d: must be a power of two in [16, 1024]", p->n);
  if (!(p->length > 0) || !std::isfinite(p->length))
    return fail(PR_ERR_INVALID_ARG, "length must be finite and > 0");
  if (!(p->eps > 0) || !std::isfinite(p->eps)) return fail(PR_ERR_INVALID_ARG, "eps must be finite and > 0");
  if (!(p->stab >= 0) || !std::isfinite(p->stab)) return fail(PR_ERR_INVALID_ARG, "stab must be finite and >= 0");
  if (!(p->dt > 0) || !std::isfinite(p->dt)) return fail(PR_ERR_INVALID_ARG, "dt must be finite and > 0");
  if (p->steps < 1) return fail(PR_ERR_INVALID_ARG, "steps must be >= 1");
  if (p->conservative != 0 && p->conservative != 1)
    return fail(PR_ERR_INVALID_ARG, "conservative must be 0 or 1");
  if (p->fine_prec != PR_F64 && p->fine_prec != PR_F32)
    return fail(PR_ERR_UNSUPPORTED, "fine_prec must be PR_F64 or PR_F32");
  if (p->scheme != PR_SCHEME_SSI && p->scheme != PR_SCHEME_CN)
    return fail(PR_ERR_INVALID_ARG, "scheme must be PR_SCHEME_SSI or PR_SCHEME_CN");
  if (p->scheme == PR_SCHEME_CN && (p->picard_iters < 1 || p->picard_iters > 64))
    return fail(PR_ERR_INVALID_ARG, "picard_iters must be in [1, 64] for PR_SCHEME_CN");
  if (p->laplacian != PR_LAP_FD5 && p->laplacian != PR_LAP_SPECTRAL)
    return fail(PR_ERR_INVALID_ARG, "laplacian must be PR_LAP_FD5 or PR_LAP_SPECTRAL");
  if (p->f32_iters < 0) return fail(PR_ERR_INVALID_ARG, "f32_iters must be >= 0");
  if (p->f32_iters > 0 && p->fine_prec != PR_F64)
    return fail(PR_ERR_INVALID_ARG, "f32_iters > 0 needs fine_prec = PR_F64");
  return PR_OK;
}

pr_status check_coarse(const pr_coarse* g, int n) {
  if (!g) return fail(PR_ERR_INVALID_ARG, "coarse is NULL");
  if (g->kind == PR_G_SCHEME) {
    if (!(g->dt > 0) || !std::isfinite(g->dt)) return fail(PR_ERR_INVALID_ARG, "coarse dt must be finite and > 0");
    if (g->steps < 1) return fail(PR_ERR_INVALID_ARG, "coarse steps must be >= 1");
    if (g->prec != PR_F64 && g->prec != PR_F32) return fail(PR_ERR_UNSUPPORTED, "coarse prec must be PR_F64 or PR_F32");
    return PR_OK;
  }
  if (g->kind != PR_G_CNN) return fail(PR_ERR_UNSUPPORTED, "coarse kind %d not supported", g->kind);
  if (n < 32) return fail(PR_ERR_UNSUPPORTED, "the CNN coarse propagator needs N >= 32");
  if (g->n_layers < 2 || g->n_layers > 64) return fail(PR_ERR_INVALID_ARG, "n_layers must be in [2, 64]");
  const int C = g->channels;
  if (C != 8 && C != 16 && C != 32 && C != 48 && C != 64)
    return fail(PR_ERR_UNSUPPORTED, "channels=%d: must be 8, 16, 32, 48 or 64", C);
  if (g->prec != PR_F64 && g->prec != PR_F32 && g->prec != PR_BF16 && g->prec != PR_BF16X2)
    return fail(PR_ERR_UNSUPPORTED, "CNN prec must be PR_F64, PR_F32, PR_BF16 or PR_BF16X2");
  const bool mfma = g->prec == PR_BF16 || g->prec == PR_BF16X2;
  if (mfma && g->n_layers > 2 && C % 16 != 0)
    return fail(PR_ERR_UNSUPPORTED, "bfloat16 hidden layers need channels to be a multiple of 16");
  if (g->prec == PR_F64 && C > kCnnF64MaxC)
    return fail(PR_ERR_UNSUPPORTED, "PR_F64 networks need channels <= %d", kCnnF64MaxC);
  if (g->prec == PR_BF16X2 && C > 48) return fail(PR_ERR_UNSUPPORTED, "PR_BF16X2 needs channels <= 48");
  if (!g->weights || !g->biases) return fail(PR_ERR_INVALID_ARG, "CNN weights / biases are NULL");
  if (g->act != PR_ACT_GELU && g->act != PR_ACT_TANH) return fail(PR_ERR_INVALID_ARG, "act must be PR_ACT_GELU or PR_ACT_TANH");
  if (g->limiter && !(g->lim_lo <= g->lim_hi)) return fail(PR_ERR_INVALID_ARG, "limiter needs lim_lo <= lim_hi");
  return PR_OK;
}

// Bump allocator over the caller's workspace (p == nullptr: sizing only).
struct Carver {
  char* base;
  size_t used = 0;
  explicit Carver(void* b) : base((char*)b) {}
  void* take(size_t bytes) {
    const size_t off = (used + 255) & ~(size_t)255;
    used = off + bytes;
    return base ? base + off : nullptr;
  }
};

FineWs carve_fine(Carver& c, int n, bool f32, int64_t nfields, bool cn = false) {
  FineWs w{};
  w.desc = (CallDesc*)c.take(sizeof(CallDesc));
  w.tw64 = (double2*)c.take((size_t)n * sizeof(double2));
  w.tw32 = (float2*)c.take((size_t)n * sizeof(float2));
  w.s2 = (double*)c.take((size_t)n * sizeof(double));
  w.partials = (double*)c.take((size_t)nfields * row_tiles(n, f32) * sizeof(double));
  w.spec = c.take((size_t)nfields * n * (n / 2) * (f32 ? 8 : 16));
  if (cn) w.xspec = c.take((size_t)nfields * n * (n / 2) * (f32 ? 8 : 16));
  w.queue = c.take(fine_queue_ws_bytes(nfields));
  return w;
}

bool is_cn(const pr_problem* p) { return p->scheme == PR_SCHEME_CN; }

StepParams step_params(const pr_problem* p, double dt) {
  StepParams sp;
  const double h = p->length / p->n;
  sp.a = 1.0 + p->stab * dt;
  sp.dt = dt;
  sp.lam = dt * p->eps * p->eps * 4.0 / (h * h);
  sp.inv_n2 = 1.0 / ((double)p->n * (double)p->n);
  sp.conservative = p->conservative;
  return sp;
}

// Process-wide plan per (N, precision): PR_PLAN_AUTO falls back to the
// default rule (resident for N <= 128) unless pr_autotune_fine recorded a
// measured choice.
// Chunks of the fine batch that overlap the sequential sweep (1 = none).
std::atomic<int> g_overlap_chunks{1};
constexpr int kMaxChunks = 16;

std::atomic<int> g_plan[11][2];     // [log2 N][f32], user setting
std::atomic<int> g_tuned[11][2];    // [log2 N][f32], autotuner result (0 = none)
std::atomic<int> g_split[11][2];    // [log2 N][f32], pr_fft_split setting
std::atomic<int> g_split_tuned[11][2];  // [log2 N][f32], autotuner result (0 = none)

int log2i(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

int effective_plan(int n, bool f32) {
  const int l = log2i(n);
  if (l < 0 || l > 10) return PR_PLAN_STREAM;
  int pl = g_plan[l][f32 ? 1 : 0].load();
  if (pl == PR_PLAN_AUTO) pl = g_tuned[l][f32 ? 1 : 0].load();
  if (pl == PR_PLAN_AUTO) pl = n <= kResidentMaxN ? PR_PLAN_RESIDENT : PR_PLAN_STREAM;
  if (pl == PR_PLAN_RESIDENT && n > kResidentMaxN) pl = PR_PLAN_STREAM;
  return pl;
}

// FFT radix split of the streaming semi-implicit passes for (N, precision):
// the setting, else the autotuner's measured choice, else radix 8 first
// with the leftover last; PR_FFT_SPLIT_* values.
int effective_split(int n, bool f32) {
  const int l = log2i(n);
  if (l < 0 || l > 10 || !fine_radix_differs(n)) return PR_FFT_SPLIT_R8;
  int sp = g_split[l][f32 ? 1 : 0].load();
  if (sp == PR_FFT_SPLIT_AUTO) sp = g_split_tuned[l][f32 ? 1 : 0].load();
  return sp == PR_FFT_SPLIT_R4_TAIL ? PR_FFT_SPLIT_R4_TAIL : PR_FFT_SPLIT_R8;
}

StepJob make_job(const pr_problem* p, double dt, int steps, bool f32, int64_t nfields,
                 const FineWs& ws) {
  StepJob j{};
  j.scheme = p->scheme;
  j.picard = p->picard_iters;
  j.resident = p->scheme == PR_SCHEME_SSI && effective_plan(p->n, f32) == PR_PLAN_RESIDENT;
  j.radix = effective_split(p->n, f32) == PR_FFT_SPLIT_R4_TAIL ? 1 : 0;
  j.n = p->n;
  j.f32 = f32;
  j.steps = steps;
  j.nfields = nfields;
  j.sp = step_params(p, dt);
  j.ws = ws;
  return j;
}

CnnWs carve_cnn(Carver& c, int n, const pr_coarse* g, int64_t nfields, bool train = false) {
  CnnWs w{};
  const int C = g->channels, L = g->n_layers;
  const int kp = (9 * C + 31) / 32 * 32;
  const bool mfma = g->prec == PR_BF16 || g->prec == PR_BF16X2;
  // hidden layers, then the last layer's hi / lo A-fragments per lane
  // (2 KB per 32-deep step)
  w.wpack = c.take(!mfma || L < 3 ? 16 : (size_t)(L - 2) * C * kp * 2 + (size_t)((C + 31) / 32) * 2048);
  const size_t act = (size_t)nfields * n * n * C * cnn_act_bytes(g->prec);
  const size_t tiles = (size_t)nfields * (n / 16) * (n / 16);
  w.partials = (double*)c.take(tiles * 8);
  if (!train) {
    w.act[0] = c.take(act);
    w.act[1] = c.take(act);
    return w;
  }
  const size_t grad = (size_t)nfields * n * n * C * cnn_grad_bytes(g->prec);
  w.acts = c.take((size_t)(L - 1) * act);
  w.zs = c.take((size_t)(L - 1) * grad);
  w.o1 = (double*)c.take((size_t)nfields * n * n * 8);
  w.wpart = (double*)c.take(tiles * (size_t)(C * C * 9 + C) * 8);
  w.wpart2 = (double*)c.take((size_t)kWGradGroups * (C * C * 9 + C) * 8);
  w.d[0] = c.take(grad);
  w.d[1] = c.take(grad);
  w.fpart = (double*)c.take((size_t)nfields * std::max<int64_t>(1, (int64_t)n * n / 2048) * 8);
  return w;
}

// Workspace of one coarse propagator call on up to `nfields` fields.
struct CoarseWs {
  FineWs fine;   // numerical coarse step
  CnnWs cnn;     // network
};

CoarseWs carve_coarse(Carver& c, const pr_problem* p, const pr_coarse* g, int64_t nfields) {
  CoarseWs w{};
  if (g->kind == PR_G_CNN) w.cnn = carve_cnn(c, p->n, g, nfields);
  else w.fine = carve_fine(c, p->n, g->prec == PR_F32, nfields, is_cn(p));
  return w;
}

pr_status cnn_lds_once() {
  static std::once_flag once;
  static hipError_t err = hipSuccess;
  std::call_once(once, [] { err = cnn_set_lds_limits(); });
  if (err != hipSuccess) return fail(PR_ERR_DEVICE, "hipFuncSetAttribute: %s", hipGetErrorString(err));
  return PR_OK;
}

CnnJob make_cnn_job(const pr_problem* p, const pr_coarse* g, const CnnWs& w) {
  CnnJob j{};
  j.n = p->n;
  j.n_layers = g->n_layers;
  j.channels = g->channels;
  j.prec = g->prec;
  j.act = g->act;
  j.residual = g->residual;
  j.mass_fix = g->mass_fix;
  j.limiter = g->limiter;
  j.lim_lo = g->lim_lo;
  j.lim_hi = g->lim_hi;
  j.W = g->weights;
  j.B = g->biases;
  j.ws = w;
  return j;
}

// Per-call set-up of a coarse propagator (tables or packed weights).
hipError_t coarse_setup(const pr_problem* p, const pr_coarse* g, const CoarseWs& w, hipStream_t s) {
  if (g->kind == PR_G_CNN) return launch_cnn_pack(make_cnn_job(p, g, w.cnn), s);
  return launch_tables(p->n, p->laplacian, w.fine, s);
}

// G on `nfields` fields addressed through optional offset tables; with
// corr, followed by that Parareal correction of the same fields (whose
// g_new addresses the output); with out2_base, the output also goes there.
hipError_t coarse_run(const pr_problem* p, const pr_coarse* g, const CoarseWs& w, int64_t nfields,
                      const double* in_base, const int64_t* in_offs, double* out_base,
                      const int64_t* out_offs, hipStream_t s, const CorrectJob* corr = nullptr,
                      double* out2_base = nullptr, const int64_t* out2_offs = nullptr);

float event_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.f;
  return ms;
}

struct Events {
  hipEvent_t e[3] = {nullptr, nullptr, nullptr};
  bool ok = false;
  Events() {
    ok = true;
    for (auto& x : e) ok = ok && hipEventCreate(&x) == hipSuccess;
  }
  ~Events() {
    for (auto& x : e)
      if (x) (void)hipEventDestroy(x);
  }
};

hipError_t coarse_run(const pr_problem* p, const pr_coarse* g, const CoarseWs& w, int64_t nfields,
                      const double* in_base, const int64_t* in_offs, double* out_base,
                      const int64_t* out_offs, hipStream_t s, const CorrectJob* corr,
                      double* out2_base, const int64_t* out2_offs) {
  if (g->kind == PR_G_CNN) {
    CnnJob j = make_cnn_job(p, g, w.cnn);
    j.nfields = nfields;
    j.in_base = in_base;
    j.in_offs = in_offs;
    j.out_base = out_base;
    j.out_offs = out_offs;
    j.corr = corr;
    j.out2_base = out2_base;
    j.out2_offs = out2_offs;
    return launch_cnn(j, s);
  }
  StepJob j = make_job(p, g->dt, g->steps, g->prec == PR_F32, nfields, w.fine);
  j.in_base = in_base;
  j.in_offs = in_offs;
  j.out_base = out_base;
  j.out_offs = out_offs;
  j.out_f32 = 0;
  hipError_t e = launch_steps(j, s);
  if (e == hipSuccess && corr) e = launch_correct(*corr, s);
  if (e == hipSuccess && out2_base) e = launch_copy(nfields, p->n, out_base, out_offs, out2_base, out2_offs, s);
  return e;
}

// ------------------------------------------------------ Parareal driver
//
// Algorithm 2 for a batch of jobs.  Fields of every job live in caller
// arrays (u0, U) or in the workspace (G cache, fine outputs, coarse
// outputs); kernels address them as element offsets from two bases, the
// lowest caller array and the workspace, through tables uploaded once per
// iteration.

// Second stream and events of the overlapped sweep (default priority).
struct Overlap {
  hipStream_t stream = nullptr;
  hipEvent_t ready = nullptr;
  hipEvent_t start[kMaxChunks] = {}, end[kMaxChunks] = {};
  bool init(bool with_stream) {
    for (auto* e : {&ready})
      if (hipEventCreate(e) != hipSuccess) return false;
    for (int c = 0; c < kMaxChunks; ++c)
      if (hipEventCreate(&start[c]) != hipSuccess || hipEventCreate(&end[c]) != hipSuccess)
        return false;
    return !with_stream || hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) == hipSuccess;
  }
  ~Overlap() {
    if (stream) {
      (void)hipStreamSynchronize(stream);
      (void)hipStreamDestroy(stream);
    }
    if (ready) (void)hipEventDestroy(ready);
    for (int c = 0; c < kMaxChunks; ++c) {
      if (start[c]) (void)hipEventDestroy(start[c]);
      if (end[c]) (void)hipEventDestroy(end[c]);
    }
  }
};

struct JobRun {
  pr_job* J = nullptr;
  int N = 0, s = 0, K32 = 0, cap = 0;
  int64_t B = 0, ic0 = 0, n2 = 0;
  bool f32_only = false;
  double* gcache = nullptr;   // [B][s][N^2]
  void* fbuf = nullptr;       // [B][s][N^2] in the iteration's fine precision
  int fine_grp[2] = {-1, -1}; // by FP32
  int coarse_grp = -1;
  int pfine = 0, pcoarse = 0; // parameter table entries
  // state
  std::vector<char> active;
  std::vector<int32_t> ic_iter;
  bool done = false;
  int iters = 0;
  pr_status status = PR_OK;
  bool f32_at(int k) const { return f32_only || k <= K32; }
  // first slice of the window of iteration k
  int win_at(int k) const { return f32_only || k <= K32 ? k - 1 : k - K32 - 1; }
  // an IC may freeze once the iteration's fine solves are in the job's own
  // precision (never in the FP32 iterations of an FP64 schedule)
  bool may_freeze(int k) const { return k > K32; }
};

struct FineGroup {
  int N;
  bool f32;
  int steps;
  int scheme, picard, lap;
  int64_t cap = 0;
  FineWs ws{};
};

struct CoarseGroup {
  const pr_problem* p;  // representative (N only)
  const pr_coarse* g;   // representative
  int64_t cap = 0;      // fields per sweep step (sum of member n_ics)
  CoarseWs ws{};
  double* gtmp = nullptr;  // [cap][N^2]
};

bool same_coarse(const pr_coarse& a, const pr_coarse& b, const pr_problem& pa,
                 const pr_problem& pb) {
  if (pa.n != pb.n || a.kind != b.kind) return false;
  if (a.kind == PR_G_SCHEME)
    return a.prec == b.prec && a.steps == b.steps && pa.scheme == pb.scheme &&
           pa.laplacian == pb.laplacian && (pa.scheme != PR_SCHEME_CN || pa.picard_iters == pb.picard_iters);
  return a.prec == b.prec && a.n_layers == b.n_layers && a.channels == b.channels &&
         a.weights == b.weights && a.biases == b.biases && a.act == b.act &&
         a.residual == b.residual && a.mass_fix == b.mass_fix && a.limiter == b.limiter &&
         (!a.limiter || (a.lim_lo == b.lim_lo && a.lim_hi == b.lim_hi));
}

struct SolvePlan {
  std::vector<JobRun> jobs;
  std::vector<FineGroup> fine;
  std::vector<CoarseGroup> coarse;
  StepParams* params = nullptr;         // [2 n_jobs]
  std::vector<StepParams> hparams;      // host copy
  unsigned long long* upd = nullptr;    // [sum B]
  int64_t* t64 = nullptr;               // index tables
  int32_t* t32 = nullptr;
  int64_t n64 = 0, n32 = 0;
  int64_t total_ics = 0;
  void* queue = nullptr;                // work-queue sweep over all fine groups
  size_t bytes = 0;
};

pr_status check_job(const pr_job& J, int i) {
  pr_status st = check_problem(&J.problem);
  if (st != PR_OK) return st;
  if ((st = check_coarse(&J.coarse, J.problem.n)) != PR_OK) return st;
  if (J.n_ics < 0) return fail(PR_ERR_INVALID_ARG, "job %d: n_ics < 0", i);
  if (J.n_slices < 1) return fail(PR_ERR_INVALID_ARG, "job %d: n_slices < 1", i);
  if (!(J.tol >= 0)) return fail(PR_ERR_INVALID_ARG, "job %d: tol must be >= 0", i);
  if (J.max_iter < 0) return fail(PR_ERR_INVALID_ARG, "job %d: max_iter < 0", i);
  if (J.problem.f32_iters >= J.n_slices && J.problem.f32_iters > 0)
    return fail(PR_ERR_INVALID_ARG, "job %d: f32_iters must be < n_slices", i);
  if (J.n_ics > 0) {
    if (!J.u0 || !J.U) return fail(PR_ERR_INVALID_ARG, "job %d: u0 / U is NULL", i);
    if (((uintptr_t)J.u0 | (uintptr_t)J.U) & 7)
      return fail(PR_ERR_INVALID_ARG, "job %d: u0 / U not 8-byte aligned", i);
  }
  return PR_OK;
}

// Sizes (base == nullptr) or carves the workspace of a batch.
pr_status plan_solve(int32_t n_jobs, pr_job* jobs, void* base, SolvePlan& P) {
  Carver c(base);
  P.jobs.assign(n_jobs, JobRun{});
  P.fine.clear();
  P.coarse.clear();
  int64_t ics = 0, fields = 0;
  for (int i = 0; i < n_jobs; ++i) {
    JobRun& r = P.jobs[i];
    pr_job& J = jobs[i];
    r.J = &J;
    r.N = J.problem.n;
    r.s = J.n_slices;
    r.B = J.n_ics;
    r.n2 = (int64_t)r.N * r.N;
    r.K32 = J.problem.f32_iters;
    r.f32_only = J.problem.fine_prec == PR_F32;
    r.cap = std::min<int64_t>(J.max_iter, (int64_t)r.K32 + r.s);
    r.ic0 = ics;
    r.pfine = 2 * i;
    r.pcoarse = 2 * i + 1;
    ics += r.B;
    fields += r.B * r.s;
    if (r.B == 0) continue;
    for (int f32 = 0; f32 < 2; ++f32) {
      const bool used = f32 ? (r.f32_only || r.K32 > 0) : !r.f32_only;
      if (!used) continue;
      int gi = -1;
      const int pic = is_cn(&J.problem) ? J.problem.picard_iters : 0;
      for (size_t q = 0; q < P.fine.size(); ++q)
        if (P.fine[q].N == r.N && P.fine[q].f32 == (bool)f32 && P.fine[q].steps == J.problem.steps &&
            P.fine[q].scheme == J.problem.scheme && P.fine[q].picard == pic &&
            P.fine[q].lap == J.problem.laplacian)
          gi = (int)q;
      if (gi < 0) {
        P.fine.push_back(FineGroup{r.N, (bool)f32, J.problem.steps, J.problem.scheme, pic,
                                   J.problem.laplacian});
        gi = (int)P.fine.size() - 1;
      }
      P.fine[gi].cap += r.B * r.s;
      r.fine_grp[f32] = gi;
    }
    int ci = -1;
    for (size_t q = 0; q < P.coarse.size(); ++q)
      if (same_coarse(*P.coarse[q].g, J.coarse, *P.coarse[q].p, J.problem)) ci = (int)q;
    if (ci < 0) {
      P.coarse.push_back(CoarseGroup{&J.problem, &J.coarse});
      ci = (int)P.coarse.size() - 1;
    }
    P.coarse[ci].cap += r.B;
    r.coarse_grp = ci;
  }
  P.total_ics = ics;
  P.params = (StepParams*)c.take((size_t)std::max(1, 2 * n_jobs) * sizeof(StepParams));
  P.upd = (unsigned long long*)c.take((size_t)std::max<int64_t>(1, ics) * 8);
  for (auto& r : P.jobs) {
    if (r.B == 0) continue;
    r.gcache = (double*)c.take((size_t)(r.B * r.s * r.n2) * 8);
    r.fbuf = c.take((size_t)(r.B * r.s * r.n2) * (r.f32_only ? 4 : 8));
  }
  int64_t fine_fields = 0;
  for (auto& g : P.fine) {
    g.ws = carve_fine(c, g.N, g.f32, g.cap, g.scheme == PR_SCHEME_CN);
    fine_fields += g.cap;
  }
  P.queue = c.take(fine_queue_ws_bytes(fine_fields));
  for (auto& g : P.coarse) {
    g.ws = carve_coarse(c, g.p, g.g, g.cap);
    g.gtmp = (double*)c.take((size_t)g.cap * g.p->n * g.p->n * 8);
  }
  // fine: in, out, pidx per field; sweep: coarse in/out/pidx + correct
  // f/gn/go/u/upd per field; initial sweep and u0 copy reuse that room
  P.n64 = 8 * fields + 2 * ics + 1;
  P.n32 = 3 * fields + 1;
  P.t64 = (int64_t*)c.take((size_t)P.n64 * 8);
  P.t32 = (int32_t*)c.take((size_t)P.n32 * 4);
  P.bytes = c.used;
  return PR_OK;
}

// Host-side builder of one upload of index tables.
struct Tables {
  std::vector<int64_t> v64;
  std::vector<int32_t> v32;
  size_t a64(int64_t x) { v64.push_back(x); return v64.size() - 1; }
};

struct Seg {
  int grp;          // fine / coarse group, or N for copies and corrections
  int f32;          // corrections: F precision
  int64_t count;
  size_t i64[6];    // table starts (element index into t64)
  size_t i32[2];
  int uni = -1;     // step launches: the parameter entry all fields share, or -1
};

bool same_params(const StepParams& a, const StepParams& b) {
  return a.a == b.a && a.dt == b.dt && a.lam == b.lam && a.inv_n2 == b.inv_n2 &&
         a.conservative == b.conservative;
}

// The parameter entry shared by every field of a launch, or -1: a shared
// one goes in as the launch argument, so that the blocks need not load
// their own before the first transform.
template <class Idx>
int shared_entry(const std::vector<StepParams>& hp, const std::vector<Idx>& idx) {
  if (idx.empty()) return -1;
  for (const Idx& i : idx)
    if (!same_params(hp[i], hp[idx[0]])) return -1;
  return (int)idx[0];
}

hipError_t run_coarse_group(const CoarseGroup& G, const SolvePlan& P, int64_t nfields,
                            const double* in_base, const int64_t* in_offs, double* out_base,
                            const int64_t* out_offs, const int32_t* pidx, int uni, hipStream_t s,
                            const CorrectJob* corr = nullptr, double* out2_base = nullptr,
                            const int64_t* out2_offs = nullptr) {
  if (G.g->kind == PR_G_CNN)
    return coarse_run(G.p, G.g, G.ws, nfields, in_base, in_offs, out_base, out_offs, s, corr,
                      out2_base, out2_offs);
  StepJob j = make_job(G.p, G.g->dt, G.g->steps, G.g->prec == PR_F32, nfields, G.ws.fine);
  j.in_base = in_base;
  j.in_offs = in_offs;
  j.out_base = out_base;
  j.out_offs = out_offs;
  j.out_f32 = 0;
  if (uni >= 0) {
    j.sp = P.hparams[uni];
  } else {
    j.params = P.params;
    j.pidx = pidx;
  }
  hipError_t e = launch_steps(j, s);
  if (e == hipSuccess && corr) e = launch_correct(*corr, s);
  if (e == hipSuccess && out2_base) e = launch_copy(nfields, G.p->n, out_base, out_offs, out2_base, out2_offs, s);
  return e;
}

pr_status solve_jobs(int32_t n_jobs, pr_job* jobs, void* ws, size_t ws_bytes, hipStream_t hs) {
  for (int i = 0; i < n_jobs; ++i) {
    jobs[i].status = PR_OK;
    pr_status st = check_job(jobs[i], i);
    if (st != PR_OK) return st;
  }
  // no job's U may overlap another's U or any u0
  for (int i = 0; i < n_jobs; ++i) {
    const pr_job& A = jobs[i];
    if (A.n_ics == 0) continue;
    const uintptr_t a0 = (uintptr_t)A.U,
                    a1 = a0 + (uintptr_t)(A.n_ics * (A.n_slices + 1)) * A.problem.n * A.problem.n * 8;
    for (int k = 0; k < n_jobs; ++k) {
      const pr_job& Bj = jobs[k];
      if (Bj.n_ics == 0) continue;
      const uintptr_t n2b = (uintptr_t)Bj.problem.n * Bj.problem.n * 8;
      const uintptr_t u0 = (uintptr_t)Bj.u0, u1 = u0 + (uintptr_t)Bj.n_ics * n2b;
      if (u0 < a1 && a0 < u1) return fail(PR_ERR_INVALID_ARG, "U of job %d overlaps u0 of job %d", i, k);
      if (k != i) {
        const uintptr_t b0 = (uintptr_t)Bj.U, b1 = b0 + (uintptr_t)(Bj.n_ics * (Bj.n_slices + 1)) * n2b;
        if (b0 < a1 && a0 < b1) return fail(PR_ERR_INVALID_ARG, "U of jobs %d and %d overlap", i, k);
      }
    }
  }
  SolvePlan P;
  plan_solve(n_jobs, jobs, nullptr, P);
  if (!ws || ws_bytes < P.bytes)
    return fail(PR_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws ? ws_bytes : (size_t)0, P.bytes);
  plan_solve(n_jobs, jobs, ws, P);
  for (auto& r : P.jobs) {
    pr_stats* st = r.J->stats;
    if (st) {
      st->iterations = 0;
      st->n_converged = 0;
      st->fine_ms = 0;
      st->sweep_ms = 0;
      if (st->ic_iterations)
        for (int64_t b = 0; b < r.B; ++b) st->ic_iterations[b] = 0;
      if (st->history)
        for (int64_t i = 0; i < (int64_t)r.J->max_iter * r.B; ++i) st->history[i] = 0.0;
    }
    r.active.assign(r.B, 1);
    r.ic_iter.assign(r.B, 0);
    r.done = r.B == 0;
  }
  if (P.total_ics == 0) return PR_OK;
  Events ev;
  if (!ev.ok) return fail(PR_ERR_DEVICE, "hipEventCreate failed");
  const int overlap_chunks = std::max(1, std::min(g_overlap_chunks.load(), kMaxChunks));
  Overlap ovl;
  if (!ovl.init(overlap_chunks > 1))
    return fail(PR_ERR_DEVICE, "stream / event creation for the overlapped sweep failed");

  // bases: the lowest caller array, and the workspace
  uintptr_t ubase = UINTPTR_MAX;
  for (auto& r : P.jobs)
    if (r.B > 0) ubase = std::min({ubase, (uintptr_t)r.J->U, (uintptr_t)r.J->u0});
  const uintptr_t wbase = (uintptr_t)ws;
  double* const UB = (double*)ubase;
  double* const WB = (double*)wbase;
  auto offU = [&](const JobRun& r, int64_t b, int64_t q) {
    return (int64_t)(((uintptr_t)r.J->U - ubase) / 8) + (b * (r.s + 1) + q) * r.n2;
  };
  auto offU0 = [&](const JobRun& r, int64_t b) {
    return (int64_t)(((uintptr_t)r.J->u0 - ubase) / 8) + b * r.n2;
  };
  auto offGC = [&](const JobRun& r, int64_t b, int64_t q) {
    return (int64_t)(((uintptr_t)r.gcache - wbase) / 8) + (b * r.s + q) * r.n2;
  };
  auto offF = [&](const JobRun& r, int64_t b, int64_t q, bool f32) {
    return (int64_t)(((uintptr_t)r.fbuf - wbase) / (f32 ? 4 : 8)) + (b * r.s + q) * r.n2;
  };
  auto offGT = [&](const CoarseGroup& g, int64_t i) {
    return (int64_t)(((uintptr_t)g.gtmp - wbase) / 8) + i * (int64_t)g.p->n * g.p->n;
  };

  // set-up: parameter table, twiddles, packed weights
  {
    std::vector<StepParams>& prm = P.hparams;
    prm.assign(2 * n_jobs, StepParams{});
    for (int i = 0; i < n_jobs; ++i) {
      prm[2 * i] = step_params(&jobs[i].problem, jobs[i].problem.dt);
      prm[2 * i + 1] = step_params(&jobs[i].problem, jobs[i].coarse.kind == PR_G_SCHEME ? jobs[i].coarse.dt : jobs[i].problem.dt);
    }
    PR_HIP(hipMemcpyAsync(P.params, prm.data(), prm.size() * sizeof(StepParams), hipMemcpyHostToDevice, hs));
    for (auto& g : P.fine) PR_HIP(launch_tables(g.N, g.lap, g.ws, hs));
    for (auto& g : P.coarse) {
      if (g.g->kind == PR_G_CNN) {
        pr_status st = cnn_lds_once();
        if (st != PR_OK) return st;
      }
      PR_HIP(coarse_setup(g.p, g.g, g.ws, hs));
    }
    PR_HIP(hipStreamSynchronize(hs));
  }
  int smax = 0;
  for (auto& r : P.jobs) smax = std::max(smax, r.s);

  Tables T;
  std::vector<Seg> segs;
  auto upload = [&]() -> pr_status {
    if ((int64_t)T.v64.size() > P.n64 || (int64_t)T.v32.size() > P.n32)
      return fail(PR_ERR_DEVICE, "internal: index tables exceed their workspace");
    if (!T.v64.empty())
      PR_HIP(hipMemcpyAsync(P.t64, T.v64.data(), T.v64.size() * 8, hipMemcpyHostToDevice, hs));
    if (!T.v32.empty())
      PR_HIP(hipMemcpyAsync(P.t32, T.v32.data(), T.v32.size() * 4, hipMemcpyHostToDevice, hs));
    return PR_OK;
  };

  // ---- k = 0: U_0 = u0, then U^0_{j+1} = G(U^0_j), kept as G(U^0_j)
  {
    T.v64.clear();
    T.v32.clear();
    segs.clear();
    // per distinct N: u0 copies
    std::vector<int> Ns;
    for (auto& r : P.jobs)
      if (r.B > 0 && std::find(Ns.begin(), Ns.end(), r.N) == Ns.end()) Ns.push_back(r.N);
    std::vector<Seg> copy0;
    for (int N : Ns) {
      Seg sg{N, 0, 0, {}, {}};
      sg.i64[0] = T.v64.size();
      for (auto& r : P.jobs)
        if (r.N == N)
          for (int64_t b = 0; b < r.B; ++b) T.v64.push_back(offU0(r, b));
      sg.i64[1] = T.v64.size();
      for (auto& r : P.jobs)
        if (r.N == N)
          for (int64_t b = 0; b < r.B; ++b) T.v64.push_back(offU(r, b, 0));
      sg.count = (int64_t)(sg.i64[1] - sg.i64[0]);
      copy0.push_back(sg);
    }
    pr_status st = upload();
    if (st != PR_OK) return st;
    for (auto& sg : copy0)
      PR_HIP(launch_copy(sg.count, sg.grp, UB, P.t64 + sg.i64[0], UB, P.t64 + sg.i64[1], hs));
    PR_HIP(hipStreamSynchronize(hs));
    // the sweep, one upload for all steps
    T.v64.clear();
    T.v32.clear();
    std::vector<std::vector<Seg>> csteps(smax), ksteps(smax);
    for (int j = 0; j < smax; ++j) {
      for (size_t gi = 0; gi < P.coarse.size(); ++gi) {
        Seg sg{(int)gi, 0, 0, {}, {}};
        std::vector<std::pair<const JobRun*, int64_t>> mem;
        for (auto& r : P.jobs)
          if (r.coarse_grp == (int)gi && j < r.s)
            for (int64_t b = 0; b < r.B; ++b) mem.push_back({&r, b});
        if (mem.empty()) continue;
        sg.count = (int64_t)mem.size();
        sg.i64[0] = T.v64.size();
        for (auto& m : mem) T.v64.push_back(offU(*m.first, m.second, j));
        sg.i64[1] = T.v64.size();
        for (auto& m : mem) T.v64.push_back(offGC(*m.first, m.second, j));
        sg.i32[0] = T.v32.size();
        for (auto& m : mem) T.v32.push_back(m.first->pcoarse);
        {
          std::vector<int> idx;
          for (auto& m : mem) idx.push_back(m.first->pcoarse);
          sg.uni = shared_entry(P.hparams, idx);
        }
        csteps[j].push_back(sg);
        Seg cp{P.coarse[gi].p->n, 0, sg.count, {}, {}};
        cp.i64[0] = sg.i64[1];
        cp.i64[1] = T.v64.size();
        for (auto& m : mem) T.v64.push_back(offU(*m.first, m.second, j + 1));
        ksteps[j].push_back(cp);
      }
    }
    st = upload();
    if (st != PR_OK) return st;
    // G(U_j) goes to the coarse cache and to U_{j+1} (cp lists the same
    // fields as sg, in the same order)
    for (int j = 0; j < smax; ++j)
      for (size_t c = 0; c < csteps[j].size(); ++c) {
        const Seg& sg = csteps[j][c];
        const Seg& cp = ksteps[j][c];
        PR_HIP(run_coarse_group(P.coarse[sg.grp], P, sg.count, UB, P.t64 + sg.i64[0], WB,
                                P.t64 + sg.i64[1], P.t32 + sg.i32[0], sg.uni, hs, nullptr, UB,
                                P.t64 + cp.i64[1]));
      }
    PR_HIP(hipStreamSynchronize(hs));
  }

  std::vector<unsigned long long> upd_h(P.total_ics);
  pr_status result = PR_OK;
  for (int k = 1;; ++k) {
    bool any = false;
    for (auto& r : P.jobs) {
      if (r.done) continue;
      int64_t act = 0;
      for (char a : r.active) act += a;
      if (act == 0 || k > r.cap) r.done = true;
      else any = true;
    }
    if (!any) break;
    T.v64.clear();
    T.v32.clear();
    // The fine batch is split into slice ranges [cb[c], cb[c+1]) that run
    // on a second stream while the sweep proceeds; the sweep waits for a
    // chunk before the first correction that needs its results or would
    // overwrite its inputs.
    int wmin = smax, send = 0;
    for (auto& r : P.jobs)
      if (!r.done) {
        wmin = std::min(wmin, r.win_at(k));
        send = std::max(send, r.s);
      }
    const int nchunk = std::max(1, std::min({overlap_chunks, send - wmin, kMaxChunks}));
    std::vector<int> cb(nchunk + 1);
    for (int c = 0; c <= nchunk; ++c) cb[c] = wmin + (int)((int64_t)(send - wmin) * c / nchunk);
    // fine solves: per chunk and group, every running job's active ICs x window
    std::vector<std::vector<Seg>> fsegs(nchunk);
    for (int c = 0; c < nchunk; ++c)
      for (size_t gi = 0; gi < P.fine.size(); ++gi) {
        const FineGroup& G = P.fine[gi];
        std::vector<const JobRun*> mem;
        for (auto& r : P.jobs)
          if (!r.done && r.fine_grp[r.f32_at(k) ? 1 : 0] == (int)gi) mem.push_back(&r);
        if (mem.empty()) continue;
        auto q0 = [&](const JobRun* r) { return std::max(r->win_at(k), cb[c]); };
        auto q1 = [&](const JobRun* r) { return std::min(r->s, cb[c + 1]); };
        Seg sg{(int)gi, G.f32 ? 1 : 0, 0, {}, {}};
        sg.i64[0] = T.v64.size();
        for (auto* r : mem)
          for (int64_t b = 0; b < r->B; ++b)
            if (r->active[b])
              for (int q = q0(r); q < q1(r); ++q) T.v64.push_back(offU(*r, b, q));
        sg.i64[1] = T.v64.size();
        sg.count = (int64_t)(sg.i64[1] - sg.i64[0]);
        for (auto* r : mem)
          for (int64_t b = 0; b < r->B; ++b)
            if (r->active[b])
              for (int q = q0(r); q < q1(r); ++q) T.v64.push_back(offF(*r, b, q, G.f32));
        sg.i32[0] = T.v32.size();
        for (auto* r : mem)
          for (int64_t b = 0; b < r->B; ++b)
            if (r->active[b])
              for (int q = q0(r); q < q1(r); ++q) T.v32.push_back(r->pfine);
        {
          std::vector<int> idx;
          for (auto* r : mem) idx.push_back(r->pfine);
          sg.uni = shared_entry(P.hparams, idx);
        }
        if (sg.count > 0) fsegs[c].push_back(sg);
      }
    // sweep: step j applies G (per coarse group) and corrects (per N, F precision)
    std::vector<std::vector<Seg>> csteps(smax), ksteps(smax);
    for (int j = 0; j < smax; ++j) {
      struct Ent { const JobRun* r; int64_t b; int64_t gt; };
      std::vector<Ent> ents;
      for (size_t gi = 0; gi < P.coarse.size(); ++gi) {
        std::vector<std::pair<const JobRun*, int64_t>> mem;
        for (auto& r : P.jobs)
          if (!r.done && r.coarse_grp == (int)gi && j >= r.win_at(k) && j < r.s)
            for (int64_t b = 0; b < r.B; ++b)
              if (r.active[b]) mem.push_back({&r, b});
        if (mem.empty()) continue;
        Seg sg{(int)gi, 0, (int64_t)mem.size(), {}, {}};
        sg.i64[0] = T.v64.size();
        for (auto& m : mem) T.v64.push_back(offU(*m.first, m.second, j));
        sg.i64[1] = T.v64.size();
        for (size_t i = 0; i < mem.size(); ++i) {
          T.v64.push_back(offGT(P.coarse[gi], (int64_t)i));
          ents.push_back({mem[i].first, mem[i].second, offGT(P.coarse[gi], (int64_t)i)});
        }
        sg.i32[0] = T.v32.size();
        for (auto& m : mem) T.v32.push_back(m.first->pcoarse);
        {
          std::vector<int> idx;
          for (auto& m : mem) idx.push_back(m.first->pcoarse);
          sg.uni = shared_entry(P.hparams, idx);
        }
        csteps[j].push_back(sg);
      }
      // corrections grouped by (N, F precision)
      std::vector<std::pair<int, int>> keys;
      for (auto& e : ents) {
        std::pair<int, int> key{e.r->N, e.r->f32_at(k) ? 1 : 0};
        if (std::find(keys.begin(), keys.end(), key) == keys.end()) keys.push_back(key);
      }
      for (auto& key : keys) {
        Seg sg{key.first, key.second, 0, {}, {}};
        std::vector<const Ent*> sel;
        for (auto& e : ents)
          if (e.r->N == key.first && (e.r->f32_at(k) ? 1 : 0) == key.second) sel.push_back(&e);
        sg.count = (int64_t)sel.size();
        sg.i64[0] = T.v64.size();
        for (auto* e : sel) T.v64.push_back(offF(*e->r, e->b, j, key.second != 0));
        sg.i64[1] = T.v64.size();
        for (auto* e : sel) T.v64.push_back(e->gt);
        sg.i64[2] = T.v64.size();
        for (auto* e : sel) T.v64.push_back(offGC(*e->r, e->b, j));
        sg.i64[3] = T.v64.size();
        for (auto* e : sel) T.v64.push_back(offU(*e->r, e->b, j + 1));
        sg.i32[0] = T.v32.size();
        for (auto* e : sel) T.v32.push_back((int32_t)(e->r->ic0 + e->b));
        ksteps[j].push_back(sg);
      }
    }
    pr_status st = upload();
    if (st != PR_OK) return st;
    PR_HIP(launch_fill_u64(P.upd, P.total_ics, 0ull, hs));
    hipStream_t sf = hs;
    if (nchunk > 1) {
      sf = ovl.stream;
      PR_HIP(hipEventRecord(ovl.ready, hs));
      PR_HIP(hipStreamWaitEvent(sf, ovl.ready, 0));
    }
    for (int c = 0; c < nchunk; ++c) {
      PR_HIP(hipEventRecord(ovl.start[c], sf));
      std::vector<StepJob> queued;   // the work-queue sweep's jobs, if it is on
      for (auto& sg : fsegs[c]) {
        const FineGroup& G = P.fine[sg.grp];
        StepJob fj{};
        fj.n = G.N;
        fj.f32 = G.f32;
        fj.steps = G.steps;
        fj.scheme = G.scheme;
        fj.picard = G.picard;
        fj.nfields = sg.count;
        fj.ws = G.ws;
        fj.resident = G.scheme == PR_SCHEME_SSI && effective_plan(G.N, G.f32) == PR_PLAN_RESIDENT;
        fj.radix = effective_split(G.N, G.f32) == PR_FFT_SPLIT_R4_TAIL ? 1 : 0;
        fj.in_base = UB;
        fj.in_offs = P.t64 + sg.i64[0];
        fj.out_base = WB;
        fj.out_offs = P.t64 + sg.i64[1];
        fj.out_f32 = G.f32;
        if (sg.uni >= 0) {
          fj.sp = P.hparams[sg.uni];
        } else {
          fj.params = P.params;
          fj.pidx = P.t32 + sg.i32[0];
        }
        if (fine_queue_use(fj))
          queued.push_back(fj);
        else
          PR_HIP(launch_steps(fj, sf));
      }
      if (!queued.empty())
        PR_HIP(launch_fine_queue(queued.data(), (int)queued.size(), P.queue, sf));
      PR_HIP(hipEventRecord(ovl.end[c], sf));
    }
    PR_HIP(hipEventRecord(ev.e[1], hs));
    int waited = 0;  // chunks the sweep has waited for
    auto correction = [&](const Seg& sg) {
      CorrectJob cj{};
      cj.nfields = sg.count;
      cj.n = sg.grp;
      cj.f = WB;
      cj.f_offs = P.t64 + sg.i64[0];
      cj.f_f32 = sg.f32;
      cj.g_new = WB;
      cj.gn_offs = P.t64 + sg.i64[1];
      cj.g_old = WB;
      cj.go_offs = P.t64 + sg.i64[2];
      cj.u = UB;
      cj.u_offs = P.t64 + sg.i64[3];
      cj.upd = P.upd;
      cj.upd_idx = P.t32 + sg.i32[0];
      cj.update_cache = 1;
      return cj;
    };
    for (int j = 0; j < smax; ++j) {
      // the correction of step j reads F_j and overwrites U_{j+1}, an input
      // of the chunk holding slice j + 1
      auto wait_chunks = [&]() -> hipError_t {
        while (waited < nchunk && cb[waited] <= j + 1) {
          if (nchunk > 1) {
            const hipError_t e = hipStreamWaitEvent(hs, ovl.end[waited], 0);
            if (e != hipSuccess) return e;
          }
          ++waited;
        }
        return hipSuccess;
      };
      // One coarse group and one correction group: the correction's fields
      // are the coarse call's, in the same order (both follow the group's
      // member list), so G hands its output straight to the correction
      // (the network's last kernel applies it where it can).
      if (csteps[j].size() == 1 && ksteps[j].size() == 1 &&
          csteps[j][0].count == ksteps[j][0].count) {
        const Seg& sg = csteps[j][0];
        const CorrectJob cj = correction(ksteps[j][0]);
        PR_HIP(wait_chunks());
        PR_HIP(run_coarse_group(P.coarse[sg.grp], P, sg.count, UB, P.t64 + sg.i64[0], WB,
                                P.t64 + sg.i64[1], P.t32 + sg.i32[0], sg.uni, hs, &cj));
        continue;
      }
      for (auto& sg : csteps[j])
        PR_HIP(run_coarse_group(P.coarse[sg.grp], P, sg.count, UB, P.t64 + sg.i64[0], WB,
                                P.t64 + sg.i64[1], P.t32 + sg.i32[0], sg.uni, hs));
      PR_HIP(wait_chunks());
      for (auto& sg : ksteps[j]) PR_HIP(launch_correct(correction(sg), hs));
    }
    for (; waited < nchunk; ++waited)
      if (nchunk > 1) PR_HIP(hipStreamWaitEvent(hs, ovl.end[waited], 0));
    PR_HIP(hipEventRecord(ev.e[2], hs));
    PR_HIP(hipMemcpyAsync(upd_h.data(), P.upd, P.total_ics * 8, hipMemcpyDeviceToHost, hs));
    PR_HIP(hipStreamSynchronize(hs));
    // fine time: the chunks' own spans; sweep time: from its first launch
    double fms = 0.0;
    for (int c = 0; c < nchunk; ++c) fms += event_ms(ovl.start[c], ovl.end[c]);
    const double sms = event_ms(ev.e[1], ev.e[2]);
    for (int ji = 0; ji < n_jobs; ++ji) {
      JobRun& r = P.jobs[ji];
      if (r.done) continue;
      pr_stats* stt = r.J->stats;
      if (stt) {
        stt->fine_ms += fms;
        stt->sweep_ms += sms;
      }
      r.iters = k;
      for (int64_t b = 0; b < r.B; ++b) {
        if (!r.active[b]) continue;
        double d;
        std::memcpy(&d, &upd_h[r.ic0 + b], 8);
        r.ic_iter[b] = k;
        if (stt && stt->history && k <= r.J->max_iter) stt->history[(int64_t)(k - 1) * r.B + b] = d;
        if (!std::isfinite(d)) {
          r.status = PR_ERR_NUMERIC;
          result = fail(PR_ERR_NUMERIC, "job %d: non-finite update norm for IC %lld at iteration %d",
                        ji, (long long)b, k);
        } else if (d <= r.J->tol && r.may_freeze(k)) {
          r.active[b] = 0;
        }
      }
      if (r.status == PR_ERR_NUMERIC) r.done = true;
    }
  }
  bool not_conv = false;
  for (int ji = 0; ji < n_jobs; ++ji) {
    JobRun& r = P.jobs[ji];
    // exact once the FP64 phase (or the FP32-only run) has covered every slice
    const int exact_at = r.f32_only ? r.s : r.K32 + r.s;
    int n_conv = 0;
    for (int64_t b = 0; b < r.B; ++b)
      if (!r.active[b] || r.ic_iter[b] >= exact_at) ++n_conv;
    if (pr_stats* stt = r.J->stats) {
      stt->iterations = r.iters;
      stt->n_converged = n_conv;
      if (stt->ic_iterations)
        for (int64_t b = 0; b < r.B; ++b) stt->ic_iterations[b] = r.ic_iter[b];
    }
    if (r.status == PR_OK && n_conv < r.B) {
      r.status = PR_NOT_CONVERGED;
      not_conv = true;
    }
    r.J->status = r.status;
  }
  if (result != PR_OK) return result;
  if (not_conv) {
    for (int ji = 0; ji < n_jobs; ++ji)
      if (jobs[ji].status == PR_NOT_CONVERGED) {
        const JobRun& r = P.jobs[ji];
        int64_t left = 0;
        for (char a : r.active) left += a;
        return fail(PR_NOT_CONVERGED, "job %d: %lld of %lld ICs above tol after %d iterations", ji,
                    (long long)left, (long long)r.B, r.iters);
      }
  }
  return PR_OK;
}

pr_job single_job(const pr_problem* p, const pr_coarse* g, int64_t n_ics, int32_t n_slices,
                  const double* u0, double* U, double tol, int32_t max_iter, pr_stats* stats) {
  pr_job J{};
  J.problem = *p;
  J.coarse = *g;
  J.n_ics = n_ics;
  J.n_slices = n_slices;
  J.max_iter = max_iter;
  J.tol = tol;
  J.u0 = u0;
  J.U = U;
  J.stats = stats;
  return J;
}

}  // namespace

extern "C" {

int pr_abi_version(void) { return PR_ABI_VERSION; }

const char* pr_last_error(void) { return g_last_error.c_str(); }

const char* pr_status_string(pr_status s) {
  switch (s) {
    case PR_OK: return "PR_OK";
    case PR_ERR_INVALID_ARG: return "PR_ERR_INVALID_ARG";
    case PR_ERR_UNSUPPORTED: return "PR_ERR_UNSUPPORTED";
    case PR_ERR_WORKSPACE: return "PR_ERR_WORKSPACE";
    case PR_ERR_DEVICE: return "PR_ERR_DEVICE";
    case PR_ERR_NUMERIC: return "PR_ERR_NUMERIC";
    case PR_NOT_CONVERGED: return "PR_NOT_CONVERGED";
  }
  return "unknown pr_status";
}

size_t pr_fine_workspace_bytes(const pr_problem* p, int64_t nfields) {
  if (check_problem(p) != PR_OK || nfields < 0) return 0;
  Carver c(nullptr);
  carve_fine(c, p->n, p->fine_prec == PR_F32, nfields, is_cn(p));
  return c.used;
}

static pr_status fine_propagate(const pr_problem* p, int64_t nfields, const double* u_in,
                                void* u_out, pr_dtype out_dtype, void* ws, size_t ws_bytes,
                                void* stream, bool eager) {
  pr_status st = check_problem(p);
  if (st != PR_OK) return st;
  if (nfields < 0) return fail(PR_ERR_INVALID_ARG, "nfields < 0");
  if (nfields == 0) return PR_OK;
  if (!u_in || !u_out) return fail(PR_ERR_INVALID_ARG, "u_in / u_out is NULL");
  if ((const void*)u_in == u_out) return fail(PR_ERR_INVALID_ARG, "u_out may not alias u_in");
  if (out_dtype != PR_F64 && out_dtype != PR_F32) return fail(PR_ERR_INVALID_ARG, "out_dtype must be PR_F64 or PR_F32");
  const bool f32 = p->fine_prec == PR_F32;
  Carver c(ws);
  FineWs w = carve_fine(c, p->n, f32, nfields, is_cn(p));
  if (!ws || ws_bytes < c.used)
    return fail(PR_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws ? ws_bytes : (size_t)0, c.used);
  hipStream_t s = (hipStream_t)stream;
  StepJob j = make_job(p, p->dt, p->steps, f32, nfields, w);
  j.in_base = u_in;
  j.out_base = u_out;
  j.out_f32 = out_dtype == PR_F32;
  j.eager = eager;
  PR_HIP(launch_tables(p->n, p->laplacian, w, s));
  if (fine_queue_use(j))
    PR_HIP(launch_fine_queue(&j, 1, w.queue, s));
  else
    PR_HIP(launch_steps(j, s));
  return PR_OK;
}

pr_status pr_fine_propagate(const pr_problem* p, int64_t nfields, const double* u_in, void* u_out,
                            pr_dtype out_dtype, void* ws, size_t ws_bytes, void* stream) {
  return fine_propagate(p, nfields, u_in, u_out, out_dtype, ws, ws_bytes, stream, false);
}

// ------------------------------------------------ F without allocation
//
// pr_fine_propagate_noalloc: the same launches as pr_fine_propagate, with
// the workspace in a file-scope device array instead of a caller buffer.
// Host code never passes the array's name to a kernel: each device's
// address is looked up once (hipGetSymbolAddress, with that device
// current) and kept.

static __device__ __align__(256) unsigned char scratch[PR_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;   // per device ordinal; null until looked up
}  // namespace

static pr_status scratch_address(void** out) {
  int dev = 0;
  PR_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(PR_ERR_DEVICE, "hipGetSymbolAddress(scratch) on device %d failed: %s", dev,
                  hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return PR_OK;
}

pr_status pr_fine_propagate_noalloc(const pr_problem* p, int64_t nfields, const double* u_in,
                                    void* u_out, pr_dtype out_dtype, void* stream) {
  pr_status st = check_problem(p);
  if (st != PR_OK) return st;
  if (nfields < 0) return fail(PR_ERR_INVALID_ARG, "nfields < 0");
  if (nfields == 0) return PR_OK;
  const size_t need = pr_fine_workspace_bytes(p, nfields);
  if (need > (size_t)PR_NOALLOC_SCRATCH_BYTES)
    return fail(PR_ERR_WORKSPACE,
                "pr_fine_propagate_noalloc: %lld fields of %d^2 need %zu bytes of scratch, more "
                "than its %zu; call pr_fine_propagate with a workspace, or fewer fields",
                (long long)nfields, p->n, need, (size_t)PR_NOALLOC_SCRATCH_BYTES);
  if (!u_in || !u_out) return fail(PR_ERR_INVALID_ARG, "u_in / u_out is NULL");
  void* ws = nullptr;
  if ((st = scratch_address(&ws)) != PR_OK) return st;
  // launched kernel by kernel: no graph of the library's own is captured or
  // instantiated (a caller may be capturing this stream)
  return fine_propagate(p, nfields, u_in, u_out, out_dtype, ws, PR_NOALLOC_SCRATCH_BYTES, stream,
                        true);
}

pr_status pr_set_fine_queue(int32_t on) {
  if (on < 0 || on > 2) return fail(PR_ERR_INVALID_ARG, "pr_set_fine_queue: on must be 0, 1 or 2");
  set_fine_queue(on);
  return PR_OK;
}

int32_t pr_get_fine_queue(void) { return fine_queue_mode(); }

int32_t pr_get_fine_queue_choice(int32_t n, pr_dtype prec) {
  if (n < 16 || n > 1024 || (n & (n - 1)) || (prec != PR_F64 && prec != PR_F32)) return -1;
  StepJob j{};
  j.scheme = SCHEME_SSI;
  j.n = n;
  j.f32 = prec == PR_F32;
  j.steps = 1;
  return fine_queue_use(j) ? 1 : 0;
}

size_t pr_coarse_workspace_bytes(const pr_problem* p, const pr_coarse* g, int64_t nfields) {
  if (check_problem(p) != PR_OK || check_coarse(g, p->n) != PR_OK || nfields < 0) return 0;
  Carver c(nullptr);
  carve_coarse(c, p, g, nfields);
  return c.used;
}

pr_status pr_coarse_apply(const pr_problem* p, const pr_coarse* g, int64_t nfields,
                          const double* u_in, double* g_out, void* ws, size_t ws_bytes,
                          void* stream) {
  pr_status st = check_problem(p);
  if (st != PR_OK) return st;
  if ((st = check_coarse(g, p->n)) != PR_OK) return st;
  if (nfields < 0) return fail(PR_ERR_INVALID_ARG, "nfields < 0");
  if (nfields == 0) return PR_OK;
  if (!u_in || !g_out) return fail(PR_ERR_INVALID_ARG, "u_in / g_out is NULL");
  if (u_in == g_out) return fail(PR_ERR_INVALID_ARG, "g_out may not alias u_in");
  Carver c(ws);
  CoarseWs w = carve_coarse(c, p, g, nfields);
  if (!ws || ws_bytes < c.used)
    return fail(PR_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws ? ws_bytes : (size_t)0, c.used);
  if (g->kind == PR_G_CNN && (st = cnn_lds_once()) != PR_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  PR_HIP(coarse_setup(p, g, w, s));
  PR_HIP(coarse_run(p, g, w, nfields, u_in, nullptr, g_out, nullptr, s));
  return PR_OK;
}

size_t pr_scheme_loss_workspace_bytes(const pr_problem* p, int64_t nfields) {
  if (check_problem(p) != PR_OK || nfields < 0) return 0;
  return scheme_loss_ws_bytes(p->n, nfields, true);
}

pr_status pr_scheme_loss(const pr_problem* p, double dt, int64_t nfields, const double* u_n,
                         const double* u_np1, double* loss, double* grad, double* resid,
                         void* ws, size_t ws_bytes, void* stream) {
  pr_status st = check_problem(p);
  if (st != PR_OK) return st;
  if (p->laplacian != PR_LAP_FD5)
    return fail(PR_ERR_UNSUPPORTED, "the scheme loss uses the 5-point Laplacian (PR_LAP_FD5)");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(PR_ERR_INVALID_ARG, "dt must be finite and > 0");
  if (nfields < 1) return fail(PR_ERR_INVALID_ARG, "nfields must be >= 1");
  if (!u_n || !u_np1 || !loss) return fail(PR_ERR_INVALID_ARG, "u_n / u_np1 / loss is NULL");
  const size_t fb = (size_t)nfields * p->n * p->n * sizeof(double);
  auto overlaps = [](const void* a, size_t na, const void* b, size_t nb) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return a && b && x < y + nb && y < x + na;
  };
  const void* outs[3] = {loss, grad, resid};
  const size_t osz[3] = {sizeof(double), fb, fb};
  for (int i = 0; i < 3; ++i) {
    if (overlaps(outs[i], osz[i], u_n, fb) || overlaps(outs[i], osz[i], u_np1, fb))
      return fail(PR_ERR_INVALID_ARG, "an output aliases an input");
    for (int k = i + 1; k < 3; ++k)
      if (overlaps(outs[i], osz[i], outs[k], osz[k]))
        return fail(PR_ERR_INVALID_ARG, "outputs alias each other");
  }
  const size_t need = scheme_loss_ws_bytes(p->n, nfields, resid == nullptr);
  if (!ws || ws_bytes < need)
    return fail(PR_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws ? ws_bytes : (size_t)0, need);
  const double h = p->length / p->n;
  SchemeLossJob j{p->n, nfields, u_n, u_np1, dt, p->eps * p->eps, 1.0 / (h * h),
                  p->conservative, loss, grad, resid, ws};
  PR_HIP(launch_scheme_loss(j, (hipStream_t)stream));
  return PR_OK;
}

size_t pr_cnn_backward_workspace_bytes(const pr_problem* p, const pr_coarse* g, int64_t nfields) {
  if (check_problem(p) != PR_OK || check_coarse(g, p->n) != PR_OK || g->kind != PR_G_CNN ||
      nfields < 0)
    return 0;
  Carver c(nullptr);
  carve_cnn(c, p->n, g, nfields, true);
  return c.used;
}

pr_status pr_cnn_backward(const pr_problem* p, const pr_coarse* g, int64_t nfields,
                          const double* u_in, const double* grad_out, double* grad_in,
                          void* grad_w, void* grad_b, void* ws, size_t ws_bytes, void* stream) {
  pr_status st = check_problem(p);
  if (st != PR_OK) return st;
  if ((st = check_coarse(g, p->n)) != PR_OK) return st;
  if (g->kind != PR_G_CNN) return fail(PR_ERR_INVALID_ARG, "pr_cnn_backward needs a PR_G_CNN coarse");
  if (nfields < 0) return fail(PR_ERR_INVALID_ARG, "nfields < 0");
  if (nfields == 0) return PR_OK;
  if (!u_in || !grad_out || !grad_in || !grad_w || !grad_b)
    return fail(PR_ERR_INVALID_ARG, "NULL array");
  const void* ptrs[5] = {u_in, grad_out, grad_in, grad_w, grad_b};
  for (int i = 0; i < 5; ++i)
    for (int k = i + 1; k < 5; ++k)
      if (ptrs[i] == ptrs[k]) return fail(PR_ERR_INVALID_ARG, "arrays must be distinct");
  Carver c(ws);
  CnnWs w = carve_cnn(c, p->n, g, nfields, true);
  if (!ws || ws_bytes < c.used)
    return fail(PR_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws ? ws_bytes : (size_t)0, c.used);
  if ((st = cnn_lds_once()) != PR_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  CoarseWs cw{};
  cw.cnn = w;
  PR_HIP(coarse_setup(p, g, cw, s));
  CnnJob j = make_cnn_job(p, g, w);
  j.nfields = nfields;
  j.in_base = u_in;
  j.in_offs = nullptr;
  j.out_base = nullptr;
  j.out_offs = nullptr;
  PR_HIP(launch_cnn_backward(j, grad_out, grad_in, grad_w, grad_b, s));
  return PR_OK;
}

pr_status pr_correct(int64_t nfields, int32_t n, const void* f, pr_dtype f_dtype,
                     const double* g_new, double* g_old, double* u, double* upd_max,
                     int32_t update_cache, void* stream) {
  if (nfields < 0) return fail(PR_ERR_INVALID_ARG, "nfields < 0");
  if (n < 1) return fail(PR_ERR_INVALID_ARG, "n < 1");
  if (nfields == 0) return PR_OK;
  if (!f || !g_new || !g_old || !u || !upd_max) return fail(PR_ERR_INVALID_ARG, "NULL array");
  if (f_dtype != PR_F64 && f_dtype != PR_F32) return fail(PR_ERR_INVALID_ARG, "f_dtype must be PR_F64 or PR_F32");
  const void* ptrs[4] = {f, g_new, g_old, u};
  for (int i = 0; i < 4; ++i)
    for (int k = i + 1; k < 4; ++k)
      if (ptrs[i] == ptrs[k]) return fail(PR_ERR_INVALID_ARG, "f, g_new, g_old, u must be distinct");
  CorrectJob j{};
  j.nfields = nfields;
  j.n = n;
  j.f = f;
  j.f_f32 = f_dtype == PR_F32;
  j.g_new = g_new;
  j.g_old = g_old;
  j.u = u;
  j.upd = (unsigned long long*)upd_max;
  j.update_cache = update_cache != 0;
  PR_HIP(launch_correct(j, (hipStream_t)stream));
  return PR_OK;
}

size_t pr_solve_workspace_bytes(const pr_problem* p, const pr_coarse* g, int64_t n_ics,
                                int32_t n_slices) {
  if (!p || !g) return 0;
  pr_job J = single_job(p, g, n_ics, n_slices, nullptr, nullptr, 0.0, 0, nullptr);
  return pr_solve_many_workspace_bytes(1, &J);
}

pr_status pr_solve(const pr_problem* p, const pr_coarse* g, int64_t n_ics, int32_t n_slices,
                   const double* u0, double* U, double tol, int32_t max_iter, pr_stats* stats,
                   void* ws, size_t ws_bytes, void* stream) {
  pr_status st = check_problem(p);
  if (st != PR_OK) return st;
  if ((st = check_coarse(g, p->n)) != PR_OK) return st;
  pr_job J = single_job(p, g, n_ics, n_slices, u0, U, tol, max_iter, stats);
  return solve_jobs(1, &J, ws, ws_bytes, (hipStream_t)stream);
}

size_t pr_solve_many_workspace_bytes(int32_t n_jobs, const pr_job* jobs) {
  if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return 0;
  // sizing needs a valid problem, coarse propagator and counts per job
  std::vector<pr_job> copy(jobs, jobs + n_jobs);
  for (const pr_job& J : copy)
    if (check_problem(&J.problem) != PR_OK || check_coarse(&J.coarse, J.problem.n) != PR_OK ||
        J.n_slices < 1 || J.n_ics < 0 || J.max_iter < 0)
      return 0;
  SolvePlan P;
  plan_solve(n_jobs, copy.data(), nullptr, P);
  return P.bytes;
}

pr_status pr_solve_many(int32_t n_jobs, pr_job* jobs, void* ws, size_t ws_bytes, void* stream) {
  if (n_jobs < 0) return fail(PR_ERR_INVALID_ARG, "n_jobs < 0");
  if (n_jobs == 0) return PR_OK;
  if (!jobs) return fail(PR_ERR_INVALID_ARG, "jobs is NULL");
  return solve_jobs(n_jobs, jobs, ws, ws_bytes, (hipStream_t)stream);
}

pr_status pr_set_fine_plan(int32_t n, pr_dtype prec, int32_t plan) {
  if (!is_pow2(n) || n < 16 || n > 1024) return fail(PR_ERR_UNSUPPORTED, "n=%d not supported", n);
  if (prec != PR_F64 && prec != PR_F32) return fail(PR_ERR_INVALID_ARG, "prec must be PR_F64 or PR_F32");
  if (plan != PR_PLAN_AUTO && plan != PR_PLAN_STREAM && plan != PR_PLAN_RESIDENT)
    return fail(PR_ERR_INVALID_ARG, "plan %d unknown", plan);
  if (plan == PR_PLAN_RESIDENT && n > kResidentMaxN)
    return fail(PR_ERR_UNSUPPORTED, "resident plan needs n <= %d", kResidentMaxN);
  g_plan[log2i(n)][prec == PR_F32 ? 1 : 0].store(plan);
  return PR_OK;
}

pr_status pr_set_coarse_plan(int32_t plan) {
  if (plan != PR_CNN_PLAN_AUTO && plan != PR_CNN_PLAN_LAYERED && plan != PR_CNN_PLAN_FUSED &&
      plan != PR_CNN_PLAN_FOLDED)
    return fail(PR_ERR_INVALID_ARG, "coarse plan %d unknown", plan);
  cnn_set_plan(plan);
  return PR_OK;
}

int32_t pr_get_coarse_plan(const pr_coarse* g, int32_t n) {
  if (!g || g->kind != PR_G_CNN || check_coarse(g, n) != PR_OK) return -1;
  return cnn_effective_plan(g->channels, g->n_layers, g->prec);
}

pr_status pr_set_coarse_tile(int32_t tile) {
  if (tile != PR_CNN_TILE_AUTO && tile != PR_CNN_TILE_8X32 && tile != PR_CNN_TILE_16X16)
    return fail(PR_ERR_INVALID_ARG, "coarse tile %d unknown", tile);
  cnn_set_tile(tile);
  return PR_OK;
}

int32_t pr_get_coarse_tile(const pr_coarse* g, int32_t n) {
  if (!g || g->kind != PR_G_CNN || !is_pow2(n) || n > 1024 || check_coarse(g, n) != PR_OK) return -1;
  if ((g->prec != PR_BF16 && g->prec != PR_BF16X2) || g->n_layers < 3) return 0;
  return cnn_effective_tile(g->channels, g->prec, n) ? PR_CNN_TILE_16X16 : PR_CNN_TILE_8X32;
}

pr_status pr_autotune_coarse(const pr_problem* p, const pr_coarse* g, int64_t nfields,
                             const double* u_in, double* g_out, void* ws, size_t ws_bytes,
                             void* stream, int32_t* chosen) {
  pr_status st = check_problem(p);
  if (st != PR_OK) return st;
  if ((st = check_coarse(g, p->n)) != PR_OK) return st;
  if (g->kind != PR_G_CNN) return fail(PR_ERR_INVALID_ARG, "pr_autotune_coarse needs a PR_G_CNN coarse");
  if (nfields < 1) return fail(PR_ERR_INVALID_ARG, "nfields must be >= 1");
  if (!u_in || !g_out || u_in == g_out) return fail(PR_ERR_INVALID_ARG, "bad u_in / g_out");
  Carver c(ws);
  CoarseWs w = carve_coarse(c, p, g, nfields);
  if (!ws || ws_bytes < c.used)
    return fail(PR_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws ? ws_bytes : (size_t)0, c.used);
  if ((st = cnn_lds_once()) != PR_OK) return st;
  // every (plan, hidden-layer tile) pair that exists for the shape; the
  // tile matters only to the plans with hidden-layer launches of 32 or 48
  // channels (LAYERED, FOLDED)
  // best_tile: the fastest tile among the plans that have tiles (a FUSED
  // win records no tile)
  int best = PR_CNN_PLAN_LAYERED, best_tile = -1;
  float best_tile_ms = -1.f;
  const bool bf16 = g->prec == PR_BF16 || g->prec == PR_BF16X2;
  const bool fused = cnn_fused_available(g->channels, g->n_layers, g->prec) && g->n_layers <= 10;
  const bool folded = cnn_folded_available(g->channels, g->n_layers, g->prec);
  const bool tiles = bf16 && g->n_layers >= 3 && (g->channels == 32 || g->channels == 48);
  if (fused || folded || tiles) {
    hipStream_t s = (hipStream_t)stream;
    Events ev;
    if (!ev.ok) return fail(PR_ERR_DEVICE, "hipEventCreate failed");
    const int saved = cnn_get_plan(), saved_tile = cnn_get_tile();
    PR_HIP(coarse_setup(p, g, w, s));
    float best_ms = -1.f;
    for (int plan = PR_CNN_PLAN_LAYERED; plan <= PR_CNN_PLAN_FOLDED; ++plan) {
      if ((plan == PR_CNN_PLAN_FUSED && !fused) || (plan == PR_CNN_PLAN_FOLDED && !folded)) continue;
      const int ntiles = tiles && plan != PR_CNN_PLAN_FUSED ? 2 : 1;
      for (int tile = 0; tile < ntiles; ++tile) {
        cnn_set_plan(plan);
        cnn_set_tile(tile ? PR_CNN_TILE_16X16 : PR_CNN_TILE_8X32);
        hipError_t e = coarse_run(p, g, w, nfields, u_in, nullptr, g_out, nullptr, s);  // warm-up
        if (e == hipSuccess) e = hipEventRecord(ev.e[0], s);
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep)
          e = coarse_run(p, g, w, nfields, u_in, nullptr, g_out, nullptr, s);
        if (e == hipSuccess) e = hipEventRecord(ev.e[1], s);
        if (e == hipSuccess) e = hipEventSynchronize(ev.e[1]);
        if (e != hipSuccess) {
          cnn_set_plan(saved);
          cnn_set_tile(saved_tile);
          return fail(PR_ERR_DEVICE, "autotune: %s", hipGetErrorString(e));
        }
        const float ms = event_ms(ev.e[0], ev.e[1]);
        if (best_ms < 0.f || ms < best_ms) {
          best_ms = ms;
          best = plan;
        }
        if (ntiles > 1 && (best_tile_ms < 0.f || ms < best_tile_ms)) {
          best_tile_ms = ms;
          best_tile = tile;
        }
      }
    }
    cnn_set_plan(saved);
    cnn_set_tile(saved_tile);
  }
  cnn_record_tuned(g->channels, g->n_layers, g->prec, best);
  if (tiles && best_tile >= 0) cnn_record_tile(g->channels, g->prec, p->n, best_tile);
  if (chosen) *chosen = best;
  return PR_OK;
}

pr_status pr_set_fine_working_set(int64_t bytes) {
  if (bytes < 0) return fail(PR_ERR_INVALID_ARG, "working-set budget must be >= 0");
  set_working_set(bytes);
  return PR_OK;
}

int64_t pr_get_fine_working_set(int32_t n, pr_dtype prec) {
  if (!is_pow2(n) || n < 16 || n > 1024 || (prec != PR_F64 && prec != PR_F32)) return -1;
  return working_set(n, prec == PR_F32);
}

pr_status pr_set_overlap(int32_t chunks) {
  if (chunks < 1 || chunks > kMaxChunks)
    return fail(PR_ERR_INVALID_ARG, "overlap chunks must be in [1, %d]", kMaxChunks);
  g_overlap_chunks.store(chunks);
  return PR_OK;
}

int32_t pr_get_overlap(void) { return g_overlap_chunks.load(); }

void pr_set_graphs(int32_t enabled) { set_graphs_enabled(enabled != 0); }

int32_t pr_get_graphs(void) { return graphs_enabled() ? 1 : 0; }

pr_status pr_set_fft_split(int32_t n, pr_dtype prec, int32_t split) {
  if (!is_pow2(n) || n < 16 || n > 1024) return fail(PR_ERR_UNSUPPORTED, "n=%d not supported", n);
  if (prec != PR_F64 && prec != PR_F32) return fail(PR_ERR_INVALID_ARG, "prec must be PR_F64 or PR_F32");
  if (split != PR_FFT_SPLIT_AUTO && split != PR_FFT_SPLIT_R8 && split != PR_FFT_SPLIT_R4_TAIL)
    return fail(PR_ERR_INVALID_ARG, "FFT split %d unknown", split);
  g_split[log2i(n)][prec == PR_F32 ? 1 : 0].store(split);
  return PR_OK;
}

int32_t pr_get_fft_split(int32_t n, pr_dtype prec) {
  if (!is_pow2(n) || n < 16 || n > 1024 || (prec != PR_F64 && prec != PR_F32)) return -1;
  return effective_split(n, prec == PR_F32);
}

int32_t pr_get_fine_plan(int32_t n, pr_dtype prec) {
  if (!is_pow2(n) || n < 16 || n > 1024 || (prec != PR_F64 && prec != PR_F32)) return -1;
  return effective_plan(n, prec == PR_F32);
}

pr_status pr_autotune_fine(const pr_problem* p, int64_t nfields, const double* u_in, void* u_out,
                           void* ws, size_t ws_bytes, void* stream, int32_t* chosen) {
  pr_status st = check_problem(p);
  if (st != PR_OK) return st;
  if (nfields < 1) return fail(PR_ERR_INVALID_ARG, "nfields must be >= 1");
  if (!u_in || !u_out || (const void*)u_in == u_out) return fail(PR_ERR_INVALID_ARG, "bad u_in / u_out");
  const bool f32 = p->fine_prec == PR_F32;
  Carver c(ws);
  FineWs w = carve_fine(c, p->n, f32, nfields, is_cn(p));
  if (!ws || ws_bytes < c.used)
    return fail(PR_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws ? ws_bytes : (size_t)0, c.used);
  hipStream_t s = (hipStream_t)stream;
  const int l = log2i(p->n);
  int best = PR_PLAN_STREAM;
  // the resident plan exists for the semi-implicit step only
  if (p->n <= kResidentMaxN && !is_cn(p)) {
    Events ev;
    if (!ev.ok) return fail(PR_ERR_DEVICE, "hipEventCreate failed");
    PR_HIP(launch_tables(p->n, p->laplacian, w, s));
    float ms[3] = {0, 0, 0};
    for (int plan = PR_PLAN_STREAM; plan <= PR_PLAN_RESIDENT; ++plan) {
      StepJob j = make_job(p, p->dt, p->steps, f32, nfields, w);
      j.resident = plan == PR_PLAN_RESIDENT;
      j.in_base = u_in;
      j.out_base = u_out;
      j.out_f32 = 0;
      PR_HIP(launch_steps(j, s));  // warm-up
      PR_HIP(hipEventRecord(ev.e[0], s));
      PR_HIP(launch_steps(j, s));
      PR_HIP(hipEventRecord(ev.e[1], s));
      PR_HIP(hipEventSynchronize(ev.e[1]));
      ms[plan] = event_ms(ev.e[0], ev.e[1]);
    }
    best = ms[PR_PLAN_RESIDENT] <= ms[PR_PLAN_STREAM] ? PR_PLAN_RESIDENT : PR_PLAN_STREAM;
  }
  if (!is_cn(p)) g_tuned[l][f32 ? 1 : 0].store(best);
  // working-set budget of the streaming plan: all fields at once, or
  // chunks whose spectra fit 256 / 128 MiB, timed on this batch
  if (best == PR_PLAN_STREAM || is_cn(p)) {
    Events ev;
    if (!ev.ok) return fail(PR_ERR_DEVICE, "hipEventCreate failed");
    PR_HIP(launch_tables(p->n, p->laplacian, w, s));
    const int64_t budgets[3] = {0, 256ll << 20, 128ll << 20};
    float bms = 0.f;
    int64_t bbest = -1;
    for (int64_t b : budgets) {
      StepJob j = make_job(p, p->dt, p->steps, f32, nfields, w);
      j.resident = false;
      j.ws_override = b;
      j.in_base = u_in;
      j.out_base = u_out;
      j.out_f32 = 0;
      PR_HIP(launch_steps(j, s));  // warm-up
      PR_HIP(hipEventRecord(ev.e[0], s));
      PR_HIP(launch_steps(j, s));
      PR_HIP(hipEventRecord(ev.e[1], s));
      PR_HIP(hipEventSynchronize(ev.e[1]));
      const float t = event_ms(ev.e[0], ev.e[1]);
      if (bbest < 0 || t < bms) {
        bms = t;
        bbest = b;
      }
    }
    record_working_set(p->n, f32, bbest);
  }
  // the radix split of the streaming semi-implicit passes, where N has two
  // (with the working set just recorded)
  if (best == PR_PLAN_STREAM && !is_cn(p) && fine_radix_differs(p->n)) {
    Events ev;
    if (!ev.ok) return fail(PR_ERR_DEVICE, "hipEventCreate failed");
    PR_HIP(launch_tables(p->n, p->laplacian, w, s));
    float t[2] = {0.f, 0.f};
    for (int r = 0; r < 2; ++r) {
      StepJob j = make_job(p, p->dt, p->steps, f32, nfields, w);
      j.resident = false;
      j.radix = r;
      j.in_base = u_in;
      j.out_base = u_out;
      j.out_f32 = 0;
      PR_HIP(launch_steps(j, s));  // warm-up
      PR_HIP(hipEventRecord(ev.e[0], s));
      PR_HIP(launch_steps(j, s));
      PR_HIP(hipEventRecord(ev.e[1], s));
      PR_HIP(hipEventSynchronize(ev.e[1]));
      t[r] = event_ms(ev.e[0], ev.e[1]);
    }
    g_split_tuned[l][f32 ? 1 : 0].store(t[1] < t[0] ? PR_FFT_SPLIT_R4_TAIL : PR_FFT_SPLIT_R8);
  }
  // the work queue against the per-pass launches (with the plan and the
  // working set just recorded), for the classes the queue covers
  {
    StepJob j = make_job(p, p->dt, p->steps, f32, nfields, w);
    j.in_base = u_in;
    j.out_base = u_out;
    j.out_f32 = 0;
    if (fine_queue_supports(j) && !j.resident) {
      Events ev;
      if (!ev.ok) return fail(PR_ERR_DEVICE, "hipEventCreate failed");
      PR_HIP(launch_tables(p->n, p->laplacian, w, s));
      float t[2] = {0.f, 0.f};
      for (int q = 0; q < 2; ++q) {
        for (int rep = 0; rep < 2; ++rep) {   // warm-up, then timed
          if (rep == 1) PR_HIP(hipEventRecord(ev.e[0], s));
          if (q) PR_HIP(launch_fine_queue(&j, 1, w.queue, s));
          else PR_HIP(launch_steps(j, s));
        }
        PR_HIP(hipEventRecord(ev.e[1], s));
        PR_HIP(hipEventSynchronize(ev.e[1]));
        t[q] = event_ms(ev.e[0], ev.e[1]);
      }
      record_fine_queue(p->n, f32, t[1] < t[0]);
    }
  }
  if (chosen) *chosen = best;
  return PR_OK;
}

size_t pr_serial_workspace_bytes(const pr_problem* p, int64_t n_ics) {
  if (check_problem(p) != PR_OK || n_ics < 0) return 0;
  Carver c(nullptr);
  carve_fine(c, p->n, p->fine_prec == PR_F32, n_ics, is_cn(p));
  c.take((size_t)n_ics * 8);
  return c.used;
}

pr_status pr_serial_fine(const pr_problem* p, int64_t n_ics, int32_t n_slices, const double* u0,
                         double* U, void* ws, size_t ws_bytes, void* stream) {
  pr_status st = check_problem(p);
  if (st != PR_OK) return st;
  if (n_ics < 0) return fail(PR_ERR_INVALID_ARG, "n_ics < 0");
  if (n_slices < 1) return fail(PR_ERR_INVALID_ARG, "n_slices < 1");
  if (n_ics == 0) return PR_OK;
  if (!u0 || !U) return fail(PR_ERR_INVALID_ARG, "u0 / U is NULL");
  const bool f32 = p->fine_prec == PR_F32;
  Carver c(ws);
  FineWs w = carve_fine(c, p->n, f32, n_ics, is_cn(p));
  int64_t* off_u = (int64_t*)c.take((size_t)n_ics * 8);
  if (!ws || ws_bytes < c.used)
    return fail(PR_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws ? ws_bytes : (size_t)0, c.used);
  hipStream_t hs = (hipStream_t)stream;
  const int64_t n2 = (int64_t)p->n * p->n;
  std::vector<int64_t> off(n_ics);
  for (int64_t b = 0; b < n_ics; ++b) off[b] = b * (int64_t)(n_slices + 1) * n2;
  PR_HIP(hipMemcpyAsync(off_u, off.data(), n_ics * 8, hipMemcpyHostToDevice, hs));
  PR_HIP(launch_tables(p->n, p->laplacian, w, hs));
  PR_HIP(launch_copy(n_ics, p->n, u0, nullptr, U, off_u, hs));
  StepJob j = make_job(p, p->dt, p->steps, f32, n_ics, w);
  for (int32_t q = 0; q < n_slices; ++q) {
    j.in_base = U + q * n2;
    j.in_offs = off_u;
    j.out_base = U + (q + 1) * n2;
    j.out_offs = off_u;
    j.out_f32 = 0;
    PR_HIP(launch_steps(j, hs));
  }
  PR_HIP(hipStreamSynchronize(hs));
  return PR_OK;
}

}  // extern "C"
