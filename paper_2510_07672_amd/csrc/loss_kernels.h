// Interface between the C ABI (api.hip) and the scheme-residual loss
// kernels (loss_kernels.hip).  Not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pr {

struct SchemeLossJob {
  int n;
  int64_t nfields;
  const double* u0;    // [nfields][n][n]  U_n
  const double* u1;    // [nfields][n][n]  U_{n+1}
  double dt, eps2, inv_h2;
  int conservative;
  double* loss;        // device, one double
  double* grad;        // [nfields][n][n] or null
  double* resid;       // [nfields][n][n] or null (then kept in ws)
  void* ws;            // scheme_loss_ws_bytes(n, nfields, resid == null)
};

size_t scheme_loss_ws_bytes(int n, int64_t nfields, bool need_r);
hipError_t launch_scheme_loss(const SchemeLossJob& j, hipStream_t st);

}  // namespace pr
