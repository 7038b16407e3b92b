// Pointwise physics of the HIP path, generic over the scalar type so the same
// code yields values (float/double), tangents (Dual) and pointwise Jacobians
// (MDual).
//
//   advection        f = c u                       (eq. "linear_advection")
//                    upwind flux                   (eq. "flux_advection")
//   Euler            f = (rho v, rho v v + p I, (rho E + p) v)
//                                                  (eq. "fluxOperatorEuler")
//   Navier-Stokes    f_v = (0, -tau, -(mu cp/Pr) grad T - tau.v),
//                    tau = mu (grad v + grad v^T - 2/3 div v I)
//                                                  (eq. "fluxOperatorNavierStokes")
//                    with cp grad T = gamma/(gamma-1) grad(p/rho).
//   common flux      Rusanov convective part + LDG viscous part
//                    n.[(1/2+beta) f_v,L + (1/2-beta) f_v,R] + eta (u_L - u_R)
//                    (SDRT section; beta = eta = 0 is BR1).
// The gradients q are gradients of the conserved variables; velocity and
// p/rho gradients follow from the quotient rule.
#pragma once
#include "dual.hpp"

enum { SYS_ADV = 0, SYS_EULER = 1, SYS_NS = 2 };

struct PhysP {
  double c[3];
  double gamma, mu, prandtl, beta, eta;
};

template <int SYS> struct SysTraits;
template <> struct SysTraits<SYS_ADV> { static constexpr bool kVisc = true; };  // advection-diffusion when mu != 0
template <> struct SysTraits<SYS_EULER> { static constexpr bool kVisc = false; };
template <> struct SysTraits<SYS_NS> { static constexpr bool kVisc = true; };

// Inviscid flux f[d][a].
template <int SYS, int ND, int NV, class T>
FR_HD void flux_inviscid(const PhysP& P, const T* u, T (*f)[NV]) {
  typedef typename BaseOf<T>::type R;
  if constexpr (SYS == SYS_ADV) {
#pragma unroll
    for (int d = 0; d < ND; ++d) f[d][0] = R(P.c[d]) * u[0];
  } else {
    const R gm1 = R(P.gamma - 1.0);
    T rho = u[0], E = u[ND + 1];
    T ir = T(R(1)) / rho;
    T v[ND];
    T ke = T(R(0));
#pragma unroll
    for (int i = 0; i < ND; ++i) { v[i] = u[1 + i] * ir; ke += u[1 + i] * v[i]; }
    T p = gm1 * (E - R(0.5) * ke);
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      f[d][0] = u[1 + d];
#pragma unroll
      for (int i = 0; i < ND; ++i) f[d][1 + i] = (i == d) ? u[1 + d] * v[i] + p : u[1 + d] * v[i];
      f[d][ND + 1] = (E + p) * v[d];
    }
  }
}

// Viscous flux f_v[d][a] (without the inviscid part).
template <int SYS, int ND, int NV, class T>
FR_HD void flux_viscous(const PhysP& P, const T* u, const T (*q)[NV], T (*f)[NV]) {
  typedef typename BaseOf<T>::type R;
  if constexpr (SYS == SYS_ADV) {
#pragma unroll
    for (int d = 0; d < ND; ++d) f[d][0] = R(-P.mu) * q[d][0];
  } else if constexpr (SYS == SYS_EULER) {
#pragma unroll
    for (int d = 0; d < ND; ++d)
#pragma unroll
      for (int a = 0; a < NV; ++a) f[d][a] = T(R(0));
  } else {
    const R gm1 = R(P.gamma - 1.0);
    const R mu = R(P.mu);
    const R kap = R(P.mu * P.gamma / (P.prandtl * (P.gamma - 1.0)));
    T rho = u[0];
    T ir = T(R(1)) / rho;
    T v[ND];
#pragma unroll
    for (int i = 0; i < ND; ++i) v[i] = u[1 + i] * ir;
    T e = u[ND + 1] * ir;
    T dv[ND][ND];   // dv[i][d] = d v_i / d x_d
    T dpr[ND];      // d(p/rho)/d x_d
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      T dr = q[d][0];
      T vg = T(R(0));
#pragma unroll
      for (int i = 0; i < ND; ++i) { dv[i][d] = (q[d][1 + i] - v[i] * dr) * ir; vg += v[i] * dv[i][d]; }
      T de = (q[d][ND + 1] - e * dr) * ir;
      dpr[d] = gm1 * (de - vg);
    }
    T divv = dv[0][0];
#pragma unroll
    for (int i = 1; i < ND; ++i) divv += dv[i][i];
    const R two3 = R(2.0 / 3.0);
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      f[d][0] = T(R(0));
      T work = T(R(0));
#pragma unroll
      for (int i = 0; i < ND; ++i) {
        T tau = (i == d) ? mu * (dv[i][d] + dv[d][i] - two3 * divv) : mu * (dv[i][d] + dv[d][i]);
        f[d][1 + i] = -tau;
        work += tau * v[i];
      }
      f[d][ND + 1] = -(kap * dpr[d] + work);
    }
  }
}

// Convective common flux F[a] for unit normal n (advection: upwind;
// Euler/NS: Rusanov with phi = max over both sides of |v.n| + c).
template <int SYS, int ND, int NV, class T>
FR_HD void common_inviscid(const PhysP& P, const T* uL, const T* uR, const typename BaseOf<T>::type* n, T* F) {
  typedef typename BaseOf<T>::type R;
  if constexpr (SYS == SYS_ADV) {
    R cn = R(0);
#pragma unroll
    for (int d = 0; d < ND; ++d) cn += R(P.c[d]) * n[d];
    F[0] = (cn >= R(0)) ? cn * uL[0] : cn * uR[0];
  } else {
    T fL[ND][NV], fR[ND][NV];
    flux_inviscid<SYS, ND, NV, T>(P, uL, fL);
    flux_inviscid<SYS, ND, NV, T>(P, uR, fR);
    const R g = R(P.gamma), gm1 = R(P.gamma - 1.0);
    T s[2];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const T* u = side ? uR : uL;
      T ir = T(R(1)) / u[0];
      T vn = T(R(0)), ke = T(R(0));
#pragma unroll
      for (int i = 0; i < ND; ++i) { vn += n[i] * u[1 + i]; ke += u[1 + i] * u[1 + i]; }
      vn = vn * ir;
      T p = gm1 * (u[ND + 1] - R(0.5) * ke * ir);
      s[side] = fr_abs(vn) + fr_sqrt(g * p * ir);
    }
    T phi = fr_max(s[0], s[1]);
#pragma unroll
    for (int a = 0; a < NV; ++a) {
      T acc = T(R(0));
#pragma unroll
      for (int d = 0; d < ND; ++d) acc += n[d] * (fL[d][a] + fR[d][a]);
      F[a] = R(0.5) * acc + R(0.5) * phi * (uL[a] - uR[a]);
    }
  }
}
