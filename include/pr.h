/*
 * pr.h -- C ABI of libpr: the Parareal fine propagator for the classic and
 * mass-conservative Allen-Cahn equations on one gfx950 GPU.
 *
 * Method: arXiv 2510.07672, "Parallel-in-Time Solution of Allen-Cahn
 * Equations by Integrating Operator Learning into the Parareal Method".
 *
 * The problem (Section 2) is the initial-value problem
 *     u_t = eps^2 Lap u + f(u) [- (1/|Omega|) int f(u)],   f(u) = u - u^3,
 * periodic on Omega = [0, L]^2 (Section 3.1), u(0) = u0.  The grid is
 * x_i = i h, i = 0..N-1, h = L/N.  One fine step of size dt is the
 * stabilised semi-implicit step with the central-difference Laplacian
 * (Section 3.1 allows finite differences; the stabilised semi-implicit
 * family is the one the introduction cites):
 *     ((1 + S dt) I - dt eps^2 Lap_h) u+ = (1 + S dt) u + dt (f(u) - m),
 * with m = 0 (classic) or the grid mean of f(u) (conservative, the
 * discrete nonlocal term of Section 3.1).  It is solved exactly by 2-D
 * real FFTs.  The fine propagator F (eq. fine_operator) is `steps` such
 * steps; Parareal is Algorithm 2 of Section 3.3.
 *
 * Conventions for every entry point:
 *   - Every array argument is a DEVICE pointer, owned by the caller, C-
 *     contiguous, with u[b][i][j] = u(x_i, y_j) and N*N elements per field.
 *     Arrays are expected 256-byte aligned (any torch allocation is).
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *     asynchronous on that stream except pr_solve and pr_serial_fine,
 *     which block (pr_solve reads one double per initial condition back
 *     after each iteration to test convergence).
 *   - `ws` is a device workspace of at least the size the matching
 *     *_workspace_bytes() call returns; the library allocates nothing.
 *   - Arguments are validated before any launch; on a validation error
 *     nothing is written and pr_last_error() says what was wrong.
 *   - Thread safety: calls on different streams with different
 *     workspaces may run concurrently; pr_last_error() is per thread.
 *   - Results are deterministic: no atomics take part in any floating-
 *     point sum, and no two fields share a transform, so a field's bits do
 *     not depend on what else is in the batch.
 */
#ifndef PR_H_
#define PR_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PR_ABI_VERSION 13

typedef enum {
  PR_OK = 0,
  PR_ERR_INVALID_ARG = 1,  /* null pointer, negative size, bad enum value  */
  PR_ERR_UNSUPPORTED = 2,  /* N not a power of two in [16, 1024], dim != 2 */
  PR_ERR_WORKSPACE = 3,    /* ws NULL or smaller than *_workspace_bytes()  */
  PR_ERR_DEVICE = 4,       /* a HIP call failed (message in last_error)    */
  PR_ERR_NUMERIC = 5,      /* NaN or Inf reached the convergence norm      */
  PR_NOT_CONVERGED = 6     /* max_iter < slices stopped Parareal above tol */
} pr_status;

typedef enum { PR_F64 = 0, PR_F32 = 1, PR_BF16 = 2, PR_BF16X2 = 3 } pr_dtype;

/* Fine schemes (Section 3.1).
 *   PR_SCHEME_SSI  the stabilised semi-implicit step above (S = stab).
 *   PR_SCHEME_CN   the paper's Crank-Nicolson scheme (eq. fully-discrete)
 *                  solved by picard_iters Picard iterations from
 *                  U_{n+1,(0)} = U_n, each an exact solve of
 *                    (I - dt/2 eps^2 Lap_h) V_(m+1) = U_n + dt/2 (eps^2
 *                    Lap_h U_n + f(U_n) + f(V_(m))) - dt g,
 *                  g = 0 (classic) or the grid mean of (f(U_n) +
 *                  f(V_(m)))/2 (conservative; with the factor dt, the
 *                  placement that keeps the mass).  stab is unused.
 *                  Runs on the streaming plan at every N.
 * Discrete Laplacians (Section 3.1 allows either):
 *   PR_LAP_FD5       the periodic 5-point stencil;
 *   PR_LAP_SPECTRAL  Fourier collocation, symbol -(2 pi / L)^2 |k|^2 with
 *                    wavenumbers wrapped to |k_i| <= N/2. */
typedef enum { PR_SCHEME_SSI = 0, PR_SCHEME_CN = 1 } pr_scheme;
typedef enum { PR_LAP_FD5 = 0, PR_LAP_SPECTRAL = 1 } pr_laplacian;

/* The fine problem: Section 2 (model), Section 3.1 (grid and scheme). */
typedef struct {
  int32_t dim;          /* 2 (3-D is not supported: PR_ERR_UNSUPPORTED)      */
  int32_t n;            /* N: power of two, 16 <= N <= 1024                  */
  double length;        /* L > 0, h = L / N                                  */
  double eps;           /* interfacial parameter epsilon > 0                 */
  int32_t conservative; /* 0: classic AC, 1: mass-conservative AC            */
  double stab;          /* stabiliser S >= 0                                 */
  double dt;            /* fine step dt* > 0                                 */
  int32_t steps;        /* fine steps per slice c >= 1                       */
  int32_t fine_prec;    /* PR_F64 or PR_F32: arithmetic of the fine FFTs.
                           PR_F32 rounds its input state to float once, at
                           stage-in, and carries a float state in between.  */
  int32_t f32_iters;    /* Parareal only (pr_solve, pr_solve_many), with
                           fine_prec = PR_F64: the first f32_iters
                           iterations use FP32 fine solves; the next one
                           restarts the prefix with FP64 fine solves over
                           every slice (see pr_solve).  0 <= f32_iters <
                           n_slices; must be 0 with PR_F32.  Other calls
                           ignore it.                                      */
  int32_t scheme;       /* pr_scheme                                        */
  int32_t picard_iters; /* PR_SCHEME_CN: Picard iterations per step, 1..64  */
  int32_t laplacian;    /* pr_laplacian                                     */
} pr_problem;

typedef enum { PR_G_SCHEME = 0, PR_G_CNN = 1 } pr_coarse_kind;
typedef enum { PR_ACT_GELU = 0, PR_ACT_TANH = 1 } pr_act;

/* The coarse propagator G of Section 3.3.
 *
 * PR_G_SCHEME: the numerical coarse step, `steps` semi-implicit steps of
 *   `dt` in precision `prec` (PR_F64 or PR_F32).
 *
 * PR_G_CNN: the convolutional network of Section 3.2, one application per
 *   slice: 3x3 convolutions with circular padding 1 (torch.nn.Conv2d
 *   cross-correlation), widths 1 -> C -> ... -> C -> 1 (`n_layers`
 *   convolutions, hidden width `channels`), the activation `act` after
 *   every convolution except the last, then
 *     G(u) = u + net(u)             if residual (else net(u)),
 *     G(u) += mean(u) - mean(G(u))  if mass_fix (the uniform shift that
 *                                   keeps the mass, Section 3.2),
 *     G(u) = clamp(G(u), lim_lo, lim_hi) if limiter (bound limiter).
 *   weights: device array of the layers' torch Conv2d weights
 *            [Cout][Cin][3][3] concatenated in layer order; biases: device
 *            array of [Cout] per layer, concatenated.  Both are double for
 *            prec PR_F64 and float otherwise.  Read on every call; the
 *            library keeps a packed copy in the workspace only during a call.
 *   prec: PR_F64 or PR_F32 (every layer in that precision on the vector
 *         ALU; PR_F64 needs channels <= 32), PR_BF16 (hidden layers on the
 *         bf16 matrix cores with FP32 accumulation; hidden weights and
 *         activations rounded to bfloat16), or PR_BF16X2 (the same with
 *         each activation carried as a hi + lo bfloat16 pair, two products
 *         per term; needs channels <= 48).  The first layer reads the FP64
 *         state unrounded and the last writes FP64.
 *   Needs N >= 32, channels in {8, 16, 32, 48, 64} and, for bfloat16 with
 *   n_layers > 2, a multiple of 16; PR_ERR_UNSUPPORTED otherwise. */
typedef struct {
  int32_t kind;         /* PR_G_SCHEME or PR_G_CNN                      */
  double dt;            /* scheme: coarse step > 0 (one slice: c * dt*)  */
  int32_t steps;        /* scheme: coarse steps per slice >= 1           */
  int32_t prec;         /* see above                                     */
  int32_t n_layers;     /* CNN: convolutions, >= 2                       */
  int32_t channels;     /* CNN: hidden width C                           */
  const void* weights;  /* CNN: device, concatenated Conv2d weights      */
  const void* biases;   /* CNN: device, concatenated biases              */
  int32_t act;          /* CNN: PR_ACT_GELU (erf form) or PR_ACT_TANH    */
  int32_t residual;     /* CNN: 1: G(u) = u + net(u)                     */
  int32_t mass_fix;     /* CNN: 1: restore the input's mean              */
  int32_t limiter;      /* CNN: 1: clamp to [lim_lo, lim_hi]             */
  double lim_lo, lim_hi;
} pr_coarse;

/* Host-side report of pr_solve.  Pointers may be NULL. */
typedef struct {
  int32_t iterations;     /* out: iterations run (max over ICs)            */
  int32_t n_converged;    /* out: ICs whose update norm reached <= tol,
                             or that ran k = slices iterations (exact)     */
  int32_t* ic_iterations; /* in: host int32[n_ics] or NULL; out: per IC    */
  double* history;        /* in: host double[max_iter * n_ics] or NULL;
                             out: history[(k-1)*n_ics + b] = sup-norm
                             update of IC b in iteration k (0 once frozen) */
  double fine_ms;         /* out: wall time spent in the fine sweeps       */
  double sweep_ms;        /* out: wall time in the coarse/correction sweeps*/
} pr_stats;

/* ---------------------------------------------------------------- F --- */

/* Bytes of workspace pr_fine_propagate needs for `nfields` fields. */
size_t pr_fine_workspace_bytes(const pr_problem* p, int64_t nfields);

/* F(t_n, t_{n+1}, U) of eq. fine_operator: p->steps fine steps applied to
 * each of `nfields` independent fields.
 *   u_in   device double[nfields][N][N], read only.
 *   u_out  device [nfields][N][N] of out_dtype (PR_F64 or PR_F32); may not
 *          alias u_in.
 * All fields advance in the same launches (Section 3.3 computes the fine
 * solves of all slices in parallel). */
pr_status pr_fine_propagate(const pr_problem* p, int64_t nfields,
                            const double* u_in, void* u_out, pr_dtype out_dtype,
                            void* ws, size_t ws_bytes, void* stream);

/* F as pr_fine_propagate, for callers that cannot allocate device memory
 * (code under graph capture, tight serving loops, harnesses that forbid
 * allocation): no workspace argument and no allocation of any kind.  The
 * workspace is a static device array of PR_NOALLOC_SCRATCH_BYTES that the
 * library holds on each GPU it runs on until the process ends; its address
 * on the current device is looked up on the first call there.  A call
 * whose pr_fine_workspace_bytes(p, nfields) exceeds that size is rejected
 * with PR_ERR_WORKSPACE (64 MiB: e.g. 120 FP64 fields of 256^2, 30 of
 * 512^2).  Every call on one GPU uses the same array, so calls that
 * overlap in time on one GPU (other streams, other threads) race: order
 * them on one stream.  Nothing in the array needs clearing between calls.
 * The kernels are launched one by one on `stream` (no graph of the
 * library's own), so a caller may capture the call into its own graph.
 * Results are bit for bit those of pr_fine_propagate. */
#define PR_NOALLOC_SCRATCH_BYTES (64u << 20)
pr_status pr_fine_propagate_noalloc(const pr_problem* p, int64_t nfields,
                                    const double* u_in, void* u_out,
                                    pr_dtype out_dtype, void* stream);

/* ---------------------------------------------------------------- G --- */

size_t pr_coarse_workspace_bytes(const pr_problem* p, const pr_coarse* g,
                                 int64_t nfields);

/* G(U) of Section 3.3 on `nfields` fields: u_in, g_out device
 * double[nfields][N][N] (g_out may not alias u_in).  The model, grid and
 * stabiliser come from p; the step, count and precision from g. */
pr_status pr_coarse_apply(const pr_problem* p, const pr_coarse* g,
                          int64_t nfields, const double* u_in, double* g_out,
                          void* ws, size_t ws_bytes, void* stream);

/* Backward of the convolutional G (Section 3.2), for training it on
 * trajectories of F (Algorithm 1).  Given the input u_in and dL/dG(u_in)
 * (grad_out), all device double[nfields][N][N] and contiguous, writes
 *   grad_in  device double[nfields][N][N]: dL/du_in (through the network,
 *            the residual, the mass fix and the limiter, whose derivative is
 *            0 where it clamps);
 *   grad_w, grad_b: dL/dweights and dL/dbiases, laid out like g->weights
 *            and g->biases (double for PR_F64, float otherwise), summed
 *            over all fields -- overwritten, not accumulated.
 * The forward pass is recomputed inside (only u_in is kept between the two
 * passes).  For the bfloat16 precisions the recomputed forward is the
 * bfloat16 one and the backward runs in FP32 with the FP32 weights (the
 * rounding of the hidden weights is passed straight through).  All
 * parameter-gradient sums are tile partials added in a fixed order, so
 * results are deterministic.  The arrays must be distinct. */
size_t pr_cnn_backward_workspace_bytes(const pr_problem* p, const pr_coarse* g,
                                       int64_t nfields);
pr_status pr_cnn_backward(const pr_problem* p, const pr_coarse* g, int64_t nfields,
                          const double* u_in, const double* grad_out, double* grad_in,
                          void* grad_w, void* grad_b, void* ws, size_t ws_bytes,
                          void* stream);

/* The scheme-residual training loss of Algorithm 1 (eq. loss_ACN): for
 * `nfields` pairs (U_n, U_{n+1}) = (u_n, u_np1), device
 * double[nfields][N][N], the residual of the Crank-Nicolson scheme
 * (Section 3.1, eq. fully-discrete) over one step dt with the 5-point
 * Laplacian and the mass-keeping placement of the nonlocal term,
 *   r = U1 - U0 - dt/2 (eps^2 (Lap_h U1 + Lap_h U0) + f(U1) + f(U0))
 *       + dt/2 (mean f(U1) + mean f(U0))   (conservative model only),
 * and the loss mean(r^2) over every point of every pair, written to
 * *loss (device, one double).  Optional outputs (NULL to skip):
 *   grad   device double[nfields][N][N]: dloss/du_np1 (the coarse
 *          propagator's output is u_np1 in training);
 *   resid  device double[nfields][N][N]: r.
 * eps, the model and N come from p (p->laplacian must be PR_LAP_FD5,
 * PR_ERR_UNSUPPORTED otherwise; p->dt, steps and scheme are not used).
 * FP64 throughout; every sum is per-block partials added in a fixed
 * order.  The output arrays must not alias the inputs or each other. */
size_t pr_scheme_loss_workspace_bytes(const pr_problem* p, int64_t nfields);
pr_status pr_scheme_loss(const pr_problem* p, double dt, int64_t nfields,
                         const double* u_n, const double* u_np1, double* loss,
                         double* grad, double* resid, void* ws, size_t ws_bytes,
                         void* stream);

/* ------------------------------------------------------- correction --- */

/* The Parareal correction of Section 3.3 / Algorithm 2, for `nfields`
 * fields of n*n points, evaluated as  u_new = f + (g_new - g_old):
 *   f       device [nfields][n][n] of f_dtype (PR_F64 or PR_F32): F(U^{k-1}_j)
 *   g_new   device double[nfields][n][n]: G(U^k_j)
 *   g_old   device double[nfields][n][n]: in  G(U^{k-1}_j);
 *           out G(U^k_j) when update_cache != 0 (the reused coarse value)
 *   u       device double[nfields][n][n]: in U^{k-1}_{j+1}, out U^k_{j+1}
 *   upd_max device double[nfields]: running sup norm, updated as
 *           upd_max[b] = max(upd_max[b], max_points |u_new - u_in|);
 *           entries must be >= 0 (or NaN) on entry; a NaN anywhere in a
 *           field's update makes its entry NaN.
 * f, g_new, g_old and u must be four distinct arrays (PR_ERR_INVALID_ARG
 * otherwise). */
pr_status pr_correct(int64_t nfields, int32_t n, const void* f,
                     pr_dtype f_dtype, const double* g_new, double* g_old,
                     double* u, double* upd_max, int32_t update_cache,
                     void* stream);

/* -------------------------------------------------------- Parareal --- */

size_t pr_solve_workspace_bytes(const pr_problem* p, const pr_coarse* g,
                                int64_t n_ics, int32_t n_slices);

/* Algorithm 2 for n_ics initial conditions at once (one pr_job of
 * pr_solve_many; the two give the same bits).
 *   u0  device double[n_ics][N][N]
 *   U   device double[n_ics][n_slices+1][N][N]: out, the final iterate
 *       [U_0, U^1_1, ..., U^k_k, ..., U^k_s] of each IC.
 * Initial coarse sweep U^0_{j+1} = G(U^0_j); then for k = 1..max_iter the
 * fine solves of slices k-1..s-1 of every active IC in one batch, and the
 * sequential sweep U^k_{j+1} = F(U^{k-1}_j) + (G(U^k_j) - G(U^{k-1}_j)).
 * An IC whose sup-norm update over all slices is <= tol is frozen (so a
 * batch gives the same bits as its members run alone).  max_iter is
 * clamped to n_slices; after k iterations slices 0..k equal the serial
 * fine solve exactly, so k = n_slices always returns PR_OK.
 * Returns PR_NOT_CONVERGED if max_iter < n_slices stopped an IC above tol
 * (U still holds the last iterate), PR_ERR_NUMERIC on NaN/Inf.
 *
 * Precision schedule (p->f32_iters = K > 0, fine_prec = PR_F64): iterations
 * 1..K run the fine solves in FP32 (16 instead of 32 bytes per point and
 * step) and never freeze an IC, since their fixed point is the FP32 serial
 * solve.  Iteration K+1 runs FP64 fine solves over slices 0..s-1 and so
 * restarts the exact prefix; FP64 iteration j = k - K covers slices
 * j-1..s-1, and after it slices 0..j equal the FP64 serial fine solve
 * exactly.  The FP32 iterations only give the FP64 phase a better start:
 * the converged result is the FP64 one, max_iter is clamped to K + s, and
 * k = K + s returns the FP64 serial solve bit for bit. */
pr_status pr_solve(const pr_problem* p, const pr_coarse* g, int64_t n_ics,
                   int32_t n_slices, const double* u0, double* U, double tol,
                   int32_t max_iter, pr_stats* stats, void* ws,
                   size_t ws_bytes, void* stream);

/* One Parareal solve of a heterogeneous batch: its own problem (any N, eps,
 * dt, S, model, fine precision and schedule), coarse propagator, initial
 * conditions, slice count, tolerance and iteration cap. */
typedef struct {
  pr_problem problem;
  pr_coarse coarse;
  int64_t n_ics;        /* >= 0                                          */
  int32_t n_slices;     /* s >= 1                                        */
  int32_t max_iter;     /* >= 0; clamped to f32_iters + s                */
  double tol;           /* >= 0, sup-norm update per IC                  */
  const double* u0;     /* device double[n_ics][N][N]                    */
  double* U;            /* device double[n_ics][s+1][N][N], out          */
  pr_stats* stats;      /* host, may be NULL (as for pr_solve; fine_ms and
                           sweep_ms add the whole batch's sweep times of
                           the iterations this job took part in)         */
  int32_t status;       /* out: PR_OK, PR_NOT_CONVERGED or PR_ERR_NUMERIC */
} pr_job;

size_t pr_solve_many_workspace_bytes(int32_t n_jobs, const pr_job* jobs);

/* Algorithm 2 (Section 3.3) for n_jobs independent solves at once: the
 * uneven batching of the method's data parallelism.  Every job runs
 * exactly what pr_solve would run for it (same bits), but in each
 * iteration the fine solves of all jobs that share (N, precision, steps
 * per slice) go into one launch sequence, whatever their eps, dt, S or
 * model (per-field step parameters), and the sequential sweeps of all
 * jobs advance together: step j of the sweep applies every job's G to its
 * slice j (one launch per coarse propagator and N) and corrects all of
 * them (one launch per N and fine precision).  Jobs converge, freeze and
 * stop independently; the call returns when every job has.
 * All arrays must be 8-byte aligned; no job's U may overlap another's U
 * or any u0 (PR_ERR_INVALID_ARG).  jobs[i].status receives each job's
 * result; the return value is PR_ERR_NUMERIC if any job hit NaN/Inf,
 * else PR_NOT_CONVERGED if any job stopped above tol, else PR_OK. */
pr_status pr_solve_many(int32_t n_jobs, pr_job* jobs, void* ws, size_t ws_bytes,
                        void* stream);

/* The serial fine solve U_{j+1} = F(U_j), j = 0..n_slices-1, for n_ics ICs
 * batched per slice (the reference Parareal converges to).
 *   u0 device double[n_ics][N][N]; U device double[n_ics][n_slices+1][N][N].
 * Workspace: pr_fine_workspace_bytes(p, n_ics) + n_ics*N*N*8 bytes. */
size_t pr_serial_workspace_bytes(const pr_problem* p, int64_t n_ics);
pr_status pr_serial_fine(const pr_problem* p, int64_t n_ics, int32_t n_slices,
                         const double* u0, double* U, void* ws,
                         size_t ws_bytes, void* stream);

/* ----------------------------------------------------- launch plans --- */

/* How the fine and coarse steps are launched for a given (N, precision),
 * process-wide.  Both plans compute the same arithmetic (the classic model
 * gives identical bits; the conservative one may differ in the last bit of
 * the mass-multiplier sum, whose reduction order differs).
 *   PR_PLAN_STREAM    each step is two launches (a column pass and a row
 *                     pass) streaming every field's spectrum through HBM;
 *   PR_PLAN_RESIDENT  one launch for all steps, one workgroup per field
 *                     with the field's whole spectrum in LDS (N <= 128);
 *   PR_PLAN_AUTO      the autotuner's measured choice if pr_autotune_fine
 *                     ran for this (N, precision), else RESIDENT for
 *                     N <= 128 and STREAM above. */
typedef enum { PR_PLAN_AUTO = 0, PR_PLAN_STREAM = 1, PR_PLAN_RESIDENT = 2 } pr_plan;

/* How a bfloat16 network (PR_BF16, PR_BF16X2) is evaluated for inference,
 * process-wide.  Both plans compute the same arithmetic; they differ in
 * where the activations live.
 *   PR_CNN_PLAN_LAYERED  one launch per layer, activations through HBM;
 *   PR_CNN_PLAN_FUSED    all layers in one launch per call, a 16 x 16
 *                        output tile per work-group with the activations
 *                        (and recomputed halos) in LDS and every hidden
 *                        layer's weights in registers; available for
 *                        C = 16 (1..4 hidden layers), C = 32 (1..2) and
 *                        C = 48 (1, PR_BF16 only); other shapes fall back
 *                        to LAYERED;
 *   PR_CNN_PLAN_FOLDED   one launch per hidden layer: the first convolution
 *                        (1 -> C) runs inside the first hidden layer's
 *                        launch, on that layer's input tile in LDS; at
 *                        C = 32 the last convolution's per-tap products are
 *                        formed in the last hidden layer's epilogue, and a
 *                        small kernel sums them over the 3 x 3 taps; the
 *                        first layer's output and the last hidden layer's
 *                        never go through HBM.  Bitwise the same result as
 *                        LAYERED; networks with at least one hidden layer,
 *                        other shapes fall back to LAYERED;
 *   PR_CNN_PLAN_AUTO     the autotuner's measured choice for the shape if
 *                        pr_autotune_coarse ran, else FOLDED for networks
 *                        with a hidden layer that are PR_BF16X2 or have 32
 *                        channels, else LAYERED.
 * Training (pr_cnn_backward) always runs layer by layer. */
typedef enum {
  PR_CNN_PLAN_AUTO = 0,
  PR_CNN_PLAN_LAYERED = 1,
  PR_CNN_PLAN_FUSED = 2,
  PR_CNN_PLAN_FOLDED = 3
} pr_cnn_plan;

pr_status pr_set_coarse_plan(int32_t plan);

/* The plan pr_coarse_apply will use for g on N x N fields (LAYERED, FUSED
 * or FOLDED), or -1 if g is not a valid network. */
int32_t pr_get_coarse_plan(const pr_coarse* g, int32_t n);

/* Output tile of each work-group in the hidden-layer launches of a
 * bfloat16 network (plans LAYERED and FOLDED), process-wide.  A tile is the
 * layer's outputs for a block of pixels, computed from the block's input
 * activations plus a one-pixel halo staged in LDS.
 *   PR_CNN_TILE_8X32   8 rows x 32 columns (340 staged pixels per 256);
 *   PR_CNN_TILE_16X16  16 x 16 (324 staged pixels per 256); built for 32
 *                      and 48 channels, other widths use 8 x 32;
 *   PR_CNN_TILE_AUTO   the autotuner's measured choice for (channels,
 *                      prec, N) if pr_autotune_coarse ran, else 16 x 16
 *                      at 48 channels and 8 x 32 at other widths.
 * Each output takes the same products in the same order under either
 * tile, so the result is the same bit for bit. */
typedef enum {
  PR_CNN_TILE_AUTO = 0,
  PR_CNN_TILE_8X32 = 1,
  PR_CNN_TILE_16X16 = 2
} pr_cnn_tile;

pr_status pr_set_coarse_tile(int32_t tile);

/* The tile pr_coarse_apply will use for g's hidden layers on N x N fields
 * (8X32 or 16X16), 0 for a network without bfloat16 hidden layers, or -1
 * if g is not a valid network or N is not a power of two in [32, 1024]. */
int32_t pr_get_coarse_tile(const pr_coarse* g, int32_t n);

/* Times every plan available for g on the caller's batch (u_in -> g_out,
 * workspace as for pr_coarse_apply), with LAYERED and FOLDED under both
 * hidden-layer tiles where both exist, and records the fastest pair: the
 * plan as the AUTO choice for the shape (channels, n_layers, prec), the
 * tile as the AUTO choice for (channels, prec, N).  *chosen receives the
 * plan; pr_get_coarse_tile reports the tile. */
pr_status pr_autotune_coarse(const pr_problem* p, const pr_coarse* g, int64_t nfields,
                             const double* u_in, double* g_out, void* ws, size_t ws_bytes,
                             void* stream, int32_t* chosen);

/* Working-set budget of streaming fine propagation, process-wide: a call
 * with more fields than fit runs them in consecutive chunks whose spectra
 * (N*N words per field, twice for PR_SCHEME_CN) total at most `bytes`,
 * each chunk through all of its steps, so that the data of the two passes
 * of a step stays in the GPU's last-level cache (MI355X: 256 MB).  The
 * results do not depend on it.  0 turns chunking off; the default is
 * 256 MiB.  pr_autotune_fine also times {off, 256 MiB, 128 MiB} on its
 * batch and keeps the fastest for that (N, precision).
 * pr_get_fine_working_set returns the budget in effect for (n, prec), or
 * -1 for an unsupported pair. */
pr_status pr_set_fine_working_set(int64_t bytes);
int64_t pr_get_fine_working_set(int32_t n, pr_dtype prec);

/* Overlap of the fine solves with the sequential sweep in pr_solve and
 * pr_solve_many, process-wide.  With chunks > 1 each iteration's fine batch
 * is split into that many slice ranges, run in order on a second stream
 * of the library's (default priority), and the sweep on the caller's
 * stream waits for a range only before the first correction that reads
 * its results or overwrites its inputs (step j waits for every range that
 * starts at or before slice j + 1).  The results are the same bits for
 * any setting; stats.fine_ms then sums the ranges' own spans.  chunks = 1
 * runs the fine batch, then the sweep, on the caller's stream.  Default 1:
 * on one GPU a batch that fills HBM bandwidth gains nothing from sharing
 * the device with the sweep, and splitting it costs launch efficiency.
 * PR_ERR_INVALID_ARG outside [1, 16]. */
pr_status pr_set_overlap(int32_t chunks);
int32_t pr_get_overlap(void);

/* Set the plan for (n, prec).  PR_ERR_UNSUPPORTED for RESIDENT with n > 128. */
pr_status pr_set_fine_plan(int32_t n, pr_dtype prec, int32_t plan);

/* The plan that will be used for (n, prec) (STREAM or RESIDENT), or -1 for
 * an unsupported (n, prec). */
int32_t pr_get_fine_plan(int32_t n, pr_dtype prec);

/* Radix split of the length-N transforms of the streaming semi-implicit
 * passes (Section 3.1's FFT-diagonalised step), per (N, precision),
 * process-wide.  Every stage of a transform is one round trip through LDS
 * with 8 elements per thread, so both splits take the fewest stages:
 *   PR_FFT_SPLIT_R8       radix 8 while it fits, the leftover radix 2 or 4
 *                         last (N = 8^a * {1, 2, 4});
 *   PR_FFT_SPLIT_R4_TAIL  the same, but a trailing 8 x 2 becomes 4 x 4, so
 *                         that N = 16, 128 and 1024 have no radix-2 stage;
 *                         other N have no such split and take R8;
 *   PR_FFT_SPLIT_AUTO     the autotuner's measured choice for (N,
 *                         precision) if pr_autotune_fine ran, else R8.
 * The two differ in rounding only (the same DFT, other operation order).
 * The resident plan, the Crank-Nicolson passes and the work queue keep R8.
 * Invalid n, prec or split: PR_ERR_UNSUPPORTED / PR_ERR_INVALID_ARG. */
typedef enum {
  PR_FFT_SPLIT_AUTO = 0,
  PR_FFT_SPLIT_R8 = 1,
  PR_FFT_SPLIT_R4_TAIL = 2
} pr_fft_split;

pr_status pr_set_fft_split(int32_t n, pr_dtype prec, int32_t split);

/* The split the streaming semi-implicit passes use for (n, prec): R8 or
 * R4_TAIL; -1 for an unsupported (n, prec). */
int32_t pr_get_fft_split(int32_t n, pr_dtype prec);

/* Autotuner: times one F call of p on `nfields` fields under each plan
 * available for p->n (u_in read, u_out overwritten with scratch results;
 * workspace as for pr_fine_propagate), records the faster one as the AUTO
 * choice for (p->n, p->fine_prec) and returns it in *chosen (may be NULL).
 * For the streaming plan it also times the working-set budgets, then (for
 * the semi-implicit step, where N has two) both FFT radix splits, then,
 * where the work queue covers the class, the queue against the per-pass
 * launches; the faster of each is recorded (see pr_set_fft_split,
 * pr_set_fine_queue).  Blocks until the timing runs finish. */
pr_status pr_autotune_fine(const pr_problem* p, int64_t nfields, const double* u_in,
                           void* u_out, void* ws, size_t ws_bytes, void* stream,
                           int32_t* chosen);

/* The work-queue fine sweep (Section 3.3's fine solves of all slices, as
 * one persistent launch).  With it on, the semi-implicit fine solves of a
 * pr_fine_propagate call, and those of every launch group of one Parareal
 * iteration of pr_solve / pr_solve_many, run as one persistent launch per
 * (N, fine precision) class instead of 2*steps + 1 launches per group: the
 * blocks take the tiles of every pass of every field from a queue, and a
 * tile waits only for the previous pass of its own field (per-field
 * counters), so passes of different fields and groups overlap.  The
 * results are bitwise those of the per-pass launches under the R8 radix
 * split (the queue's transforms always take R8; see pr_set_fft_split).  It covers N = 64 ..
 * 1024 in PR_F64 and N = 64 .. 256 in PR_F32 (other sizes, FP32 at 512 and
 * 1024, and Crank-Nicolson keep the per-pass launches).  The fields are
 * split among eight queues, one per XCD, and a queue's items run on the
 * blocks of its XCD, so that a pass hands its results to the next through
 * that XCD's L2 (a queue that no block of its XCD reaches is adopted by
 * other XCDs, which then publish device-wide).  Process-wide, default off:
 * on MI355X it stays slower than the replayed per-pass launches at every
 * size measured (2048 fields of 512^2, 100 steps: 1.18x; 512 fields of
 * 256^2, 200 steps: 1.04x; the 48-solve uneven batch of pr_solve_many:
 * 1.3x; one field of 512^2: 1.9x).  on: 0 pass by pass, except for the (N, precision)
 * classes for which pr_autotune_fine measured the queue faster; 1 on; 2 on
 * with every queue adopted (the device-wide hand-over alone, which a
 * placement of blocks that leaves an XCD without any would fall back to;
 * for tests).  Other values: PR_ERR_INVALID_ARG.  pr_get_fine_queue returns
 * the setting. */
pr_status pr_set_fine_queue(int32_t on);
int32_t pr_get_fine_queue(void);

/* Whether the semi-implicit fine solves of (n, prec) take the work queue
 * under the current setting and the autotuner's record: 1 yes, 0 no, -1
 * for an unsupported (n, prec). */
int32_t pr_get_fine_queue_choice(int32_t n, pr_dtype prec);

/* A streaming F (or numerical G) call is 2*steps + 1 launches.  With
 * graphs on (the default), that sequence is captured once per (problem,
 * steps, workspace) into a hipGraph and replayed; the batch size and the
 * input/output field addresses are read from a descriptor in the
 * workspace, so one capture serves every later call on the same
 * workspace whose batch is no larger (e.g. every Parareal iteration).
 * The library keeps at most 32 captures, evicting the least recently used
 * once that capture's last launch has finished (an event recorded after
 * each of its launches; no device-wide wait).  pr_set_graphs(0) launches
 * the kernels one by one instead; results are identical either way. */
void pr_set_graphs(int32_t enabled);
int32_t pr_get_graphs(void);

/* ---------------------------------------------------------- helpers --- */

const char* pr_status_string(pr_status s);
const char* pr_last_error(void);
int pr_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PR_H_ */
