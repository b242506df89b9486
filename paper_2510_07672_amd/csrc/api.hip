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

FineWs carve_fine(Carver& c, int n, bool f32, int64_t nfields) {
  FineWs w;
  w.desc = (CallDesc*)c.take(sizeof(CallDesc));
  w.tw64 = (double2*)c.take((size_t)n * sizeof(double2));
  w.tw32 = (float2*)c.take((size_t)n * sizeof(float2));
  w.s2 = (double*)c.take((size_t)n * sizeof(double));
  w.partials = (double*)c.take((size_t)nfields * row_tiles(n, f32) * sizeof(double));
  w.spec = c.take((size_t)nfields * n * (n / 2) * (f32 ? 8 : 16));
  return w;
}

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
std::atomic<int> g_plan[11][2];     // [log2 N][f32], user setting
std::atomic<int> g_tuned[11][2];    // [log2 N][f32], autotuner result (0 = none)

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

StepJob make_job(const pr_problem* p, double dt, int steps, bool f32, int64_t nfields,
                 const FineWs& ws) {
  StepJob j{};
  j.resident = effective_plan(p->n, f32) == PR_PLAN_RESIDENT;
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
  w.wpack = c.take(!mfma || L < 3 ? 16 : (size_t)(L - 2) * C * kp * 2);
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
  else w.fine = carve_fine(c, p->n, g->prec == PR_F32, nfields);
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
  return launch_tables(p->n, w.fine, s);
}

// G on `nfields` fields addressed through optional offset tables.
hipError_t coarse_run(const pr_problem* p, const pr_coarse* g, const CoarseWs& w, int64_t nfields,
                      const double* in_base, const int64_t* in_offs, double* out_base,
                      const int64_t* out_offs, hipStream_t s);

struct SolveWs {
  FineWs fine;
  CoarseWs coarse;
  double* gcache;          // [B][s][N][N]
  void* fbuf;              // [B][s][N][N] fine precision
  double* gtmp;            // [B][N][N]
  unsigned long long* upd; // [B]
  int64_t* off_u;          // [B] IC offsets into U (elements)
  int64_t* off_s;          // [B] IC offsets into gcache / fbuf
  int64_t* win_in;         // [B*s] window offsets into U
  int64_t* win_out;        // [B*s] window offsets into fbuf
  int32_t* act;            // [B] active IC ids
  size_t bytes;
};

SolveWs carve_solve(void* base, const pr_problem* p, const pr_coarse* g, int64_t B, int32_t s) {
  Carver c(base);
  SolveWs w;
  const size_t n2 = (size_t)p->n * p->n;
  const bool f32 = p->fine_prec == PR_F32;
  w.fine = carve_fine(c, p->n, f32, B * s);
  w.coarse = carve_coarse(c, p, g, B);
  w.gcache = (double*)c.take((size_t)B * s * n2 * 8);
  w.fbuf = c.take((size_t)B * s * n2 * (f32 ? 4 : 8));
  w.gtmp = (double*)c.take((size_t)B * n2 * 8);
  w.upd = (unsigned long long*)c.take((size_t)B * 8);
  w.off_u = (int64_t*)c.take((size_t)B * 8);
  w.off_s = (int64_t*)c.take((size_t)B * 8);
  w.win_in = (int64_t*)c.take((size_t)B * s * 8);
  w.win_out = (int64_t*)c.take((size_t)B * s * 8);
  w.act = (int32_t*)c.take((size_t)B * 4);
  w.bytes = c.used;
  return w;
}

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
                      const int64_t* out_offs, hipStream_t s) {
  if (g->kind == PR_G_CNN) {
    CnnJob j = make_cnn_job(p, g, w.cnn);
    j.nfields = nfields;
    j.in_base = in_base;
    j.in_offs = in_offs;
    j.out_base = out_base;
    j.out_offs = out_offs;
    return launch_cnn(j, s);
  }
  StepJob j = make_job(p, g->dt, g->steps, g->prec == PR_F32, nfields, w.fine);
  j.in_base = in_base;
  j.in_offs = in_offs;
  j.out_base = out_base;
  j.out_offs = out_offs;
  j.out_f32 = 0;
  return launch_steps(j, s);
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
  carve_fine(c, p->n, p->fine_prec == PR_F32, nfields);
  return c.used;
}

pr_status pr_fine_propagate(const pr_problem* p, int64_t nfields, const double* u_in, void* u_out,
                            pr_dtype out_dtype, void* ws, size_t ws_bytes, void* stream) {
  pr_status st = check_problem(p);
  if (st != PR_OK) return st;
  if (nfields < 0) return fail(PR_ERR_INVALID_ARG, "nfields < 0");
  if (nfields == 0) return PR_OK;
  if (!u_in || !u_out) return fail(PR_ERR_INVALID_ARG, "u_in / u_out is NULL");
  if ((const void*)u_in == u_out) return fail(PR_ERR_INVALID_ARG, "u_out may not alias u_in");
  if (out_dtype != PR_F64 && out_dtype != PR_F32) return fail(PR_ERR_INVALID_ARG, "out_dtype must be PR_F64 or PR_F32");
  const bool f32 = p->fine_prec == PR_F32;
  Carver c(ws);
  FineWs w = carve_fine(c, p->n, f32, nfields);
  if (!ws || ws_bytes < c.used)
    return fail(PR_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws ? ws_bytes : (size_t)0, c.used);
  hipStream_t s = (hipStream_t)stream;
  StepJob j = make_job(p, p->dt, p->steps, f32, nfields, w);
  j.in_base = u_in;
  j.out_base = u_out;
  j.out_f32 = out_dtype == PR_F32;
  PR_HIP(launch_tables(p->n, w, s));
  PR_HIP(launch_steps(j, s));
  return PR_OK;
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
  if (check_problem(p) != PR_OK || check_coarse(g, p->n) != PR_OK || n_ics < 0 || n_slices < 1) return 0;
  return carve_solve(nullptr, p, g, n_ics, n_slices).bytes;
}

pr_status pr_solve(const pr_problem* p, const pr_coarse* g, int64_t n_ics, int32_t n_slices,
                   const double* u0, double* U, double tol, int32_t max_iter, pr_stats* stats,
                   void* ws, size_t ws_bytes, void* stream) {
  pr_status st = check_problem(p);
  if (st != PR_OK) return st;
  if ((st = check_coarse(g, p->n)) != PR_OK) return st;
  if (n_ics < 0) return fail(PR_ERR_INVALID_ARG, "n_ics < 0");
  if (n_slices < 1) return fail(PR_ERR_INVALID_ARG, "n_slices < 1");
  if (!(tol >= 0)) return fail(PR_ERR_INVALID_ARG, "tol must be >= 0");
  if (max_iter < 0) return fail(PR_ERR_INVALID_ARG, "max_iter < 0");
  if (n_ics == 0) return PR_OK;
  if (!u0 || !U) return fail(PR_ERR_INVALID_ARG, "u0 / U is NULL");
  const int64_t B = n_ics;
  const int32_t s = n_slices;
  SolveWs w = carve_solve(ws, p, g, B, s);
  if (!ws || ws_bytes < w.bytes)
    return fail(PR_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws ? ws_bytes : (size_t)0, w.bytes);
  const int K = max_iter < s ? max_iter : s;
  hipStream_t hs = (hipStream_t)stream;
  const int64_t n2 = (int64_t)p->n * p->n;
  const int N = p->n;
  const bool f32 = p->fine_prec == PR_F32;
  const size_t fesz = f32 ? 4 : 8;
  Events ev;
  if (!ev.ok) return fail(PR_ERR_DEVICE, "hipEventCreate failed");

  if (stats) {
    stats->iterations = 0;
    stats->n_converged = 0;
    stats->fine_ms = 0;
    stats->sweep_ms = 0;
    if (stats->ic_iterations)
      for (int64_t b = 0; b < B; ++b) stats->ic_iterations[b] = 0;
    if (stats->history)
      for (int64_t i = 0; i < (int64_t)max_iter * B; ++i) stats->history[i] = 0.0;
  }

  // host copies of the index tables, uploaded once per iteration
  std::vector<int64_t> off_u(B), off_s(B), win_in, win_out;
  std::vector<int32_t> act(B);
  for (int64_t b = 0; b < B; ++b) {
    act[b] = (int32_t)b;
    off_u[b] = b * (int64_t)(s + 1) * n2;
    off_s[b] = b * (int64_t)s * n2;
  }
  PR_HIP(hipMemcpyAsync(w.off_u, off_u.data(), B * 8, hipMemcpyHostToDevice, hs));
  PR_HIP(hipMemcpyAsync(w.off_s, off_s.data(), B * 8, hipMemcpyHostToDevice, hs));
  PR_HIP(hipMemcpyAsync(w.act, act.data(), B * 4, hipMemcpyHostToDevice, hs));
  PR_HIP(launch_tables(N, w.fine, hs));
  if (g->kind == PR_G_CNN && (st = cnn_lds_once()) != PR_OK) return st;
  PR_HIP(coarse_setup(p, g, w.coarse, hs));
  // U_0 = u0
  PR_HIP(launch_copy(B, N, u0, nullptr, U, w.off_u, hs));

  // initial coarse sweep: U^0_{j+1} = G(U^0_j), kept as the cache G(U^0_j)
  for (int32_t j = 0; j < s; ++j) {
    PR_HIP(coarse_run(p, g, w.coarse, B, U + j * n2, w.off_u, w.gcache + j * n2, w.off_s, hs));
    PR_HIP(launch_copy(B, N, w.gcache + j * n2, w.off_s, U + (j + 1) * n2, w.off_u, hs));
  }
  PR_HIP(hipStreamSynchronize(hs));

  std::vector<unsigned long long> upd_h(B);
  std::vector<char> active(B, 1);
  std::vector<int32_t> ic_iter(B, 0);
  int64_t n_act = B;
  int iters = 0;
  pr_status result = PR_OK;
  StepJob fj = make_job(p, p->dt, p->steps, f32, 0, w.fine);
  for (int k = 1; k <= K && n_act > 0; ++k) {
    const int32_t W = s - k + 1;
    int64_t i = 0;
    for (int64_t b = 0; b < B; ++b)
      if (active[b]) {
        act[i] = (int32_t)b;
        off_u[i] = b * (int64_t)(s + 1) * n2;
        off_s[i] = b * (int64_t)s * n2;
        ++i;
      }
    win_in.resize(n_act * W);
    win_out.resize(n_act * W);
    for (int64_t a = 0; a < n_act; ++a)
      for (int32_t q = 0; q < W; ++q) {
        win_in[a * W + q] = off_u[a] + (int64_t)(k - 1 + q) * n2;
        win_out[a * W + q] = off_s[a] + (int64_t)(k - 1 + q) * n2;
      }
    PR_HIP(hipMemcpyAsync(w.act, act.data(), n_act * 4, hipMemcpyHostToDevice, hs));
    PR_HIP(hipMemcpyAsync(w.off_u, off_u.data(), n_act * 8, hipMemcpyHostToDevice, hs));
    PR_HIP(hipMemcpyAsync(w.off_s, off_s.data(), n_act * 8, hipMemcpyHostToDevice, hs));
    PR_HIP(hipMemcpyAsync(w.win_in, win_in.data(), n_act * W * 8, hipMemcpyHostToDevice, hs));
    PR_HIP(hipMemcpyAsync(w.win_out, win_out.data(), n_act * W * 8, hipMemcpyHostToDevice, hs));
    PR_HIP(launch_fill_u64(w.upd, B, 0ull, hs));
    PR_HIP(hipEventRecord(ev.e[0], hs));
    // fine solves of slices k-1..s-1 of every active IC, one batch
    fj.nfields = n_act * W;
    fj.in_base = U;
    fj.in_offs = w.win_in;
    fj.out_base = w.fbuf;
    fj.out_offs = w.win_out;
    fj.out_f32 = f32;
    PR_HIP(launch_steps(fj, hs));
    PR_HIP(hipEventRecord(ev.e[1], hs));
    // sequential correction sweep
    for (int32_t j = k - 1; j < s; ++j) {
      PR_HIP(coarse_run(p, g, w.coarse, n_act, U + j * n2, w.off_u, w.gtmp, nullptr, hs));
      CorrectJob cj{};
      cj.nfields = n_act;
      cj.n = N;
      cj.f = (const char*)w.fbuf + (size_t)j * n2 * fesz;
      cj.f_offs = w.off_s;
      cj.f_f32 = f32;
      cj.g_new = w.gtmp;
      cj.gn_offs = nullptr;
      cj.g_old = w.gcache + j * n2;
      cj.go_offs = w.off_s;
      cj.u = U + (j + 1) * n2;
      cj.u_offs = w.off_u;
      cj.upd = w.upd;
      cj.upd_idx = w.act;
      cj.update_cache = 1;
      PR_HIP(launch_correct(cj, hs));
    }
    PR_HIP(hipEventRecord(ev.e[2], hs));
    PR_HIP(hipMemcpyAsync(upd_h.data(), w.upd, B * 8, hipMemcpyDeviceToHost, hs));
    PR_HIP(hipStreamSynchronize(hs));
    if (stats) {
      stats->fine_ms += event_ms(ev.e[0], ev.e[1]);
      stats->sweep_ms += event_ms(ev.e[1], ev.e[2]);
    }
    iters = k;
    for (int64_t a = 0; a < n_act; ++a) {
      const int32_t b = act[a];
      double d;
      std::memcpy(&d, &upd_h[b], 8);
      ic_iter[b] = k;
      if (stats && stats->history && k <= max_iter) stats->history[(int64_t)(k - 1) * B + b] = d;
      if (!std::isfinite(d)) {
        result = fail(PR_ERR_NUMERIC, "non-finite update norm for IC %d at iteration %d", b, k);
      } else if (d <= tol) {
        active[b] = 0;
      }
    }
    if (result != PR_OK) break;
    n_act = 0;
    for (int64_t b = 0; b < B; ++b) n_act += active[b];
  }
  int n_conv = 0;
  for (int64_t b = 0; b < B; ++b)
    if (!active[b] || ic_iter[b] >= s) ++n_conv;
  if (stats) {
    stats->iterations = iters;
    stats->n_converged = n_conv;
    if (stats->ic_iterations)
      for (int64_t b = 0; b < B; ++b) stats->ic_iterations[b] = ic_iter[b];
  }
  if (result != PR_OK) return result;
  if (n_conv < B) return fail(PR_NOT_CONVERGED, "%lld of %lld ICs above tol after %d iterations",
                              (long long)(B - n_conv), (long long)B, iters);
  return PR_OK;
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

void pr_set_graphs(int32_t enabled) { set_graphs_enabled(enabled != 0); }

int32_t pr_get_graphs(void) { return graphs_enabled() ? 1 : 0; }

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
  FineWs w = carve_fine(c, p->n, f32, nfields);
  if (!ws || ws_bytes < c.used)
    return fail(PR_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws ? ws_bytes : (size_t)0, c.used);
  hipStream_t s = (hipStream_t)stream;
  const int l = log2i(p->n);
  int best = PR_PLAN_STREAM;
  if (p->n <= kResidentMaxN) {
    Events ev;
    if (!ev.ok) return fail(PR_ERR_DEVICE, "hipEventCreate failed");
    PR_HIP(launch_tables(p->n, w, s));
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
  g_tuned[l][f32 ? 1 : 0].store(best);
  if (chosen) *chosen = best;
  return PR_OK;
}

size_t pr_serial_workspace_bytes(const pr_problem* p, int64_t n_ics) {
  if (check_problem(p) != PR_OK || n_ics < 0) return 0;
  Carver c(nullptr);
  carve_fine(c, p->n, p->fine_prec == PR_F32, n_ics);
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
  FineWs w = carve_fine(c, p->n, f32, n_ics);
  int64_t* off_u = (int64_t*)c.take((size_t)n_ics * 8);
  if (!ws || ws_bytes < c.used)
    return fail(PR_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws ? ws_bytes : (size_t)0, c.used);
  hipStream_t hs = (hipStream_t)stream;
  const int64_t n2 = (int64_t)p->n * p->n;
  std::vector<int64_t> off(n_ics);
  for (int64_t b = 0; b < n_ics; ++b) off[b] = b * (int64_t)(n_slices + 1) * n2;
  PR_HIP(hipMemcpyAsync(off_u, off.data(), n_ics * 8, hipMemcpyHostToDevice, hs));
  PR_HIP(launch_tables(p->n, w, hs));
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
