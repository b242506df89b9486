// The scheme-residual training loss of Algorithm 1 (eq. loss_ACN): for
// pairs (U_n, U_{n+1}) the pointwise residual of the Crank-Nicolson scheme
// (eq. fully-discrete) with the 5-point Laplacian and the mass-keeping
// placement of the nonlocal term,
//
//   r = U1 - U0 - dt/2 (eps^2 (Lap_h U1 + Lap_h U0) + f(U1) + f(U0))
//       + dt/2 (mean f(U1) + mean f(U0))          [conservative model only]
//
// (f(u) = u - u^3), the loss mean(r^2) over every point of every pair, and
// its gradient with respect to U1 (the coarse propagator's output):
//
//   dL/dU1 = (2/M) [ r (1 - dt/2 f'(U1)) - dt/2 eps^2 Lap_h r
//                    + dt/2 f'(U1) mean(r) ]       (last term conservative)
//
// with M the number of points and Lap_h symmetric.  Everything in FP64;
// sums are per-block partials reduced in a fixed order, so a call is
// deterministic.
#include <hip/hip_runtime.h>

#include "loss_kernels.h"

namespace pr {

namespace {

constexpr int kLossThreads = 256;
constexpr int kLossPts = 4;                                // points per thread
constexpr int kLossBlockPts = kLossThreads * kLossPts;     // points per block

__device__ __forceinline__ double fdw(double u) { return u - u * u * u; }

// Fixed-order block sum of two values per thread (tree in LDS).
__device__ __forceinline__ double2 block_sum2(double a, double b, double2* sh) {
  const int t = threadIdx.x;
  sh[t] = double2{a, b};
  __syncthreads();
  for (int s = kLossThreads / 2; s > 0; s >>= 1) {
    if (t < s) {
      sh[t].x += sh[t + s].x;
      sh[t].y += sh[t + s].y;
    }
    __syncthreads();
  }
  const double2 r = sh[0];
  __syncthreads();
  return r;
}

// Point q of block blk of a field: block blk covers points
// [blk * kLossBlockPts, ...) of the field's n^2, thread t the points
// blk * kLossBlockPts + t + j * kLossThreads (j < kLossPts), coalesced.

// Partial sums of f(U1) and f(U0) per (field, block).
__global__ __launch_bounds__(kLossThreads) void k_loss_fsum(const double* __restrict__ u0,
                                                           const double* __restrict__ u1, int n,
                                                           int bpf, double2* __restrict__ part) {
  __shared__ double2 sh[kLossThreads];
  const int64_t f = blockIdx.x / bpf;
  const int blk = (int)(blockIdx.x % bpf);
  const int64_t n2 = (int64_t)n * n;
  double a = 0.0, b = 0.0;
#pragma unroll
  for (int j = 0; j < kLossPts; ++j) {
    const int64_t q = (int64_t)blk * kLossBlockPts + threadIdx.x + j * kLossThreads;
    if (q < n2) {
      a += fdw(u1[f * n2 + q]);
      b += fdw(u0[f * n2 + q]);
    }
  }
  const double2 s = block_sum2(a, b, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// One block per field: the field's partials summed in block order, times
// 1/n^2 (out[f] = {mean of the first, mean of the second}).
__global__ __launch_bounds__(kLossThreads) void k_loss_field_mean(const double2* __restrict__ part,
                                                                 int bpf, double inv_n2,
                                                                 double2* __restrict__ out) {
  __shared__ double2 sh[kLossThreads];
  const int64_t f = blockIdx.x;
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < bpf; i += kLossThreads) {
    a += part[f * bpf + i].x;
    b += part[f * bpf + i].y;
  }
  const double2 s = block_sum2(a, b, sh);
  if (threadIdx.x == 0) out[f] = double2{s.x * inv_n2, s.y * inv_n2};
}

__device__ __forceinline__ double lap5(const double* __restrict__ v, int n, int i, int j,
                                       double inv_h2) {
  const int m = n - 1;
  const double c = v[(int64_t)i * n + j];
  return (v[(int64_t)((i + 1) & m) * n + j] + v[(int64_t)((i - 1) & m) * n + j] +
          v[(int64_t)i * n + ((j + 1) & m)] + v[(int64_t)i * n + ((j - 1) & m)] - 4.0 * c) *
         inv_h2;
}

// The residual r (stored), with per-(field, block) partial sums of r^2
// and r.  fmean[f] = {mean f(U1), mean f(U0)} (conservative model only).
__global__ __launch_bounds__(kLossThreads) void k_loss_resid(
    const double* __restrict__ u0, const double* __restrict__ u1, int n, int bpf, double dt,
    double eps2, double inv_h2, int conservative, const double2* __restrict__ fmean,
    double* __restrict__ r, double2* __restrict__ part) {
  __shared__ double2 sh[kLossThreads];
  const int64_t f = blockIdx.x / bpf;
  const int blk = (int)(blockIdx.x % bpf);
  const int64_t n2 = (int64_t)n * n;
  const double* a = u0 + f * n2;
  const double* b = u1 + f * n2;
  const double g = conservative ? 0.5 * dt * (fmean[f].x + fmean[f].y) : 0.0;
  double s2 = 0.0, s1 = 0.0;
#pragma unroll
  for (int j = 0; j < kLossPts; ++j) {
    const int64_t q = (int64_t)blk * kLossBlockPts + threadIdx.x + j * kLossThreads;
    if (q < n2) {
      const int y = (int)(q / n), x = (int)(q % n);
      const double v1 = b[q], v0 = a[q];
      const double lap = lap5(b, n, y, x, inv_h2) + lap5(a, n, y, x, inv_h2);
      const double res = v1 - v0 - 0.5 * dt * (eps2 * lap + fdw(v1) + fdw(v0)) + g;
      r[f * n2 + q] = res;
      s2 += res * res;
      s1 += res;
    }
  }
  const double2 s = block_sum2(s2, s1, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// One block: loss = (sum over fields of their mean r^2, fixed order) * scale,
// scale = 1 / nfields.
__global__ __launch_bounds__(kLossThreads) void k_loss_total(const double2* __restrict__ fmean,
                                                            int64_t nfields, double scale,
                                                            double* __restrict__ loss) {
  __shared__ double2 sh[kLossThreads];
  double a = 0.0;
  for (int64_t i = threadIdx.x; i < nfields; i += kLossThreads) a += fmean[i].x;
  const double2 s = block_sum2(a, 0.0, sh);
  if (threadIdx.x == 0) *loss = s.x * scale;
}

// dL/dU1; rmean[f] = {mean r^2, mean r} over field f (only the mean of r
// is used here).
__global__ __launch_bounds__(kLossThreads) void k_loss_grad(
    const double* __restrict__ u1, const double* __restrict__ r, int n, int bpf, double dt,
    double eps2, double inv_h2, int conservative, const double2* __restrict__ rmean,
    double two_over_m, double* __restrict__ grad) {
  const int64_t f = blockIdx.x / bpf;
  const int blk = (int)(blockIdx.x % bpf);
  const int64_t n2 = (int64_t)n * n;
  const double* rf = r + f * n2;
  const double rbar = conservative ? rmean[f].y : 0.0;
#pragma unroll
  for (int j = 0; j < kLossPts; ++j) {
    const int64_t q = (int64_t)blk * kLossBlockPts + threadIdx.x + j * kLossThreads;
    if (q < n2) {
      const int y = (int)(q / n), x = (int)(q % n);
      const double v = u1[f * n2 + q];
      const double fp = 1.0 - 3.0 * v * v;
      const double rq = rf[q];
      double gq = rq * (1.0 - 0.5 * dt * fp) - 0.5 * dt * eps2 * lap5(rf, n, y, x, inv_h2);
      if (conservative) gq += 0.5 * dt * fp * rbar;
      grad[f * n2 + q] = two_over_m * gq;
    }
  }
}

}  // namespace

size_t scheme_loss_ws_bytes(int n, int64_t nfields, bool need_r) {
  const int64_t n2 = (int64_t)n * n;
  const int bpf = (int)((n2 + kLossBlockPts - 1) / kLossBlockPts);
  size_t b = 0;
  auto add = [&](size_t bytes) { b += (bytes + 255) / 256 * 256; };
  add(sizeof(double2) * (size_t)nfields * bpf);  // block partials
  add(sizeof(double2) * (size_t)nfields);        // field means of f
  add(sizeof(double2) * (size_t)nfields);        // field sums of r^2, r
  if (need_r) add(sizeof(double) * (size_t)nfields * n2);
  return b;
}

hipError_t launch_scheme_loss(const SchemeLossJob& j, hipStream_t st) {
  const int64_t n2 = (int64_t)j.n * j.n;
  const int bpf = (int)((n2 + kLossBlockPts - 1) / kLossBlockPts);
  unsigned char* w = (unsigned char*)j.ws;
  auto take = [&](size_t bytes) {
    unsigned char* p = w;
    w += (bytes + 255) / 256 * 256;
    return p;
  };
  double2* part = (double2*)take(sizeof(double2) * (size_t)j.nfields * bpf);
  double2* fmean = (double2*)take(sizeof(double2) * (size_t)j.nfields);
  double2* rsum = (double2*)take(sizeof(double2) * (size_t)j.nfields);
  double* r = j.resid ? j.resid : (double*)take(sizeof(double) * (size_t)j.nfields * n2);
  const dim3 grid((unsigned)(j.nfields * bpf)), blk(kLossThreads);
  const double inv_n2 = 1.0 / (double)n2;
  if (j.conservative) {
    k_loss_fsum<<<grid, blk, 0, st>>>(j.u0, j.u1, j.n, bpf, part);
    k_loss_field_mean<<<dim3((unsigned)j.nfields), blk, 0, st>>>(part, bpf, inv_n2, fmean);
  }
  k_loss_resid<<<grid, blk, 0, st>>>(j.u0, j.u1, j.n, bpf, j.dt, j.eps2, j.inv_h2,
                                     j.conservative, fmean, r, part);
  k_loss_field_mean<<<dim3((unsigned)j.nfields), blk, 0, st>>>(part, bpf, inv_n2, rsum);
  const double inv_m = 1.0 / ((double)j.nfields * (double)n2);
  k_loss_total<<<dim3(1), blk, 0, st>>>(rsum, j.nfields, 1.0 / (double)j.nfields, j.loss);
  if (j.grad)
    k_loss_grad<<<grid, blk, 0, st>>>(j.u1, r, j.n, bpf, j.dt, j.eps2, j.inv_h2, j.conservative,
                                      rsum, 2.0 * inv_m, j.grad);
  return hipGetLastError();
}

}  // namespace pr
