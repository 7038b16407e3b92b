// Explicit time integration of dU/dt = R(U) with the five-stage, fourth-order,
// two-register Runge-Kutta scheme of Carpenter and Kennedy (1994), the
// integrator the paper uses for its linear advection-diffusion experiments
// (section on numerical experiments, linear advection-diffusion; its
// amplification polynomial is the RK54 truncation of the exponential in the
// temporal stability section, with the z^5 / 200 term).
//
// Two registers: for each stage i,
//   dU <- a_i dU + dt R(U),   U <- U + b_i dU
// (a_1 = 0).  R is the library's residual; each stage's update is one
// elementwise kernel.
#include <hip/hip_runtime.h>

#include <string>

#include "fr.h"
#include "fr_ctx.hpp"

namespace {

// Coefficients of the (5,4) 2N-storage scheme, as published.
constexpr double kRkA[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                            -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
constexpr double kRkB[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                            1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                            2277821191437.0 / 14882151754819.0};

template <class T>
__global__ void __launch_bounds__(256) k_rk_stage(long n, double a, double b, double dt, const T* R, T* dU, T* U) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double d = (a != 0.0 ? a * (double)dU[i] : 0.0) + dt * (double)R[i];   // stage 1 ignores dU
    dU[i] = (T)d;
    U[i] = (T)((double)U[i] + b * d);
  }
}

}  // namespace

extern "C" {

fr_status fr_rk54(fr_ctx* c, void* U, void* work, double dt, int64_t nsteps) {
  if (!c) return FR_E_INVALID;
  const size_t a = c->prec == FR_F64 ? 8 : 4;
  if (!U || !work || ((uintptr_t)U % a) || ((uintptr_t)work % a) || nsteps < 0 || !(dt == dt)) {
    c->err = "fr_rk54: null or misaligned pointer, negative step count or NaN time step";
    return FR_E_INVALID;
  }
  const long n = (long)c->ndof;
  char* R = (char*)work;
  char* dU = R + (size_t)n * a;
  if ((char*)U >= R && (char*)U < R + 2 * (size_t)n * a) {
    c->err = "fr_rk54: U must not overlap the work array";
    return FR_E_INVALID;
  }
  long g = (n + 255) / 256;
  const unsigned grid = (unsigned)(g > 8192 ? 8192 : (g < 1 ? 1 : g));
  for (int64_t s = 0; s < nsteps; ++s)
    for (int i = 0; i < 5; ++i) {
      int rc = c->ks.rhs(c, U, R);
      if (rc) return (fr_status)rc;
      if (c->prec == FR_F64)
        hipLaunchKernelGGL(k_rk_stage<double>, dim3(grid), dim3(256), 0, c->stream, n, kRkA[i], kRkB[i], dt,
                           (const double*)R, (double*)dU, (double*)U);
      else
        hipLaunchKernelGGL(k_rk_stage<float>, dim3(grid), dim3(256), 0, c->stream, n, kRkA[i], kRkB[i], dt,
                           (const float*)R, (float*)dU, (float*)U);
      if (hipGetLastError() != hipSuccess) { c->err = "k_rk_stage launch"; return FR_E_DEVICE; }
    }
  return FR_OK;
}

}  // extern "C"
