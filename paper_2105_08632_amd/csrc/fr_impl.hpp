// __global__ kernels and their launchers for one (element type, degree,
// system, precision).  Included by the per-instantiation .hip files.
#pragma once
#include <type_traits>

#include "fr_ctx.hpp"
#include "fr_jac_mf.hpp"

constexpr int kThreads = 256;
constexpr int kMaxLds = 160 * 1024;   // LDS per workgroup on gfx950

template <class E, int NV, class T, class R, class IO>
__global__ void __launch_bounds__(kThreads) k_trace(OpsD<R> op, int ne, const IO* U, const IO* V, T* UF) {
  __shared__ __align__(16) char lds[trace_lds<E, NV, T, R>()];
  trace_body<E, NV, T, R, IO>(blockIdx.x, threadIdx.x, blockDim.x, lds, op, ne, U, V, UF, DevSync());
}

template <class E, int NV, class T, class R, class IO>
__global__ void __launch_bounds__(kThreads) k_grad(OpsD<R> op, GeoD<R> geo, double beta, const IO* U, const IO* V,
                                                   const T* UF, T* Q, T* QF) {
  constexpr int GT = grad_tile<E, T>();
  __shared__ __align__(16) char lds[grad_lds<E, NV, T, R, GT>()];
  grad_body<E, NV, T, R, IO, DevSync, GT>(blockIdx.x, threadIdx.x, blockDim.x, lds, op, geo, beta, U, V, UF, Q, QF,
                                          DevSync());
}

template <class E, int NV, int SYS, class T, class R, class IO>
__global__ void __launch_bounds__(kThreads) k_div(OpsD<R> op, GeoD<R> geo, PhysP ph, const IO* U, const IO* V,
                                                  const T* UF, const T* Q, const T* QF, IO* Rout, IO* Rtan, double ta,
                                                  double tb) {
  constexpr int TD = div_tile<E, NV, SYS, T, R>();
  __shared__ __align__(16) char lds[div_lds<E, NV, SYS, T, R, TD>()];
  div_body<E, NV, SYS, T, R, IO, DevSync, TD>(blockIdx.x, threadIdx.x, blockDim.x, lds, op, geo, ph, U, V, UF, Q, QF,
                                              Rout, Rtan, DevSync(), ta, tb);
}

template <class E, int NV, int SYS, class T, class R, class IO>
__global__ void __launch_bounds__(kThreads) k_sd_div(OpsD<R> op, GeoD<R> geo, PhysP ph, const IO* U, const IO* V,
                                                     const T* UF, const T* Q, const T* QF, IO* Rout, IO* Rtan) {
  __shared__ __align__(16) char lds[sd_div_lds<E, NV, SYS, T, R>()];
  sd_div_body<E, NV, SYS, T, R, IO>(blockIdx.x, threadIdx.x, blockDim.x, lds, op, geo, ph, U, V, UF, Q, QF, Rout,
                                    Rtan, DevSync());
}

template <class E, int NV, int SYS, class R, class OT>
__global__ void __launch_bounds__(kThreads) k_jac(OpsD<R> op, GeoD<R> geo, PhysP ph, const R* U, const R* Q,
                                                  const R* UF, const R* QF, OT* B, int nblk) {
  __shared__ __align__(16) char lds[jac_lds<E, NV, SYS, R>()];
  jac_body<E, NV, SYS, R, OT>(blockIdx.x, threadIdx.x, blockDim.x, lds, op, geo, ph, U, Q, UF, QF, B, nblk,
                              DevSync());
}

template <class E, int NV, int SYS, class R, class OT>
__global__ void __launch_bounds__((jac_tp_threads<E, NV, SYS, R>())) k_jac_tp(OpsD<R> op, Ops1D<R> o1, GeoD<R> geo, PhysP ph, const R* U,
                                                     const R* Q, const R* UF, const R* QF, OT* B, int nblk) {
  __shared__ __align__(16) char lds[jac_tp_lds<E, NV, SYS, R>()];
  jac_tp_body<E, NV, SYS, R, OT>(blockIdx.x, threadIdx.x, blockDim.x, lds, op, o1, geo, ph, U, Q, UF, QF, B, nblk,
                                 DevSync());
}

// Mixed meshes: each workgroup assembles every block of a contiguous range of
// `per` elements of the group.
template <class E, class EO, int NV, int SYS, class R, class OT>
__global__ void __launch_bounds__(kThreads) k_jac_mixed_inv(OpsD<R> op, GeoD<R> geo, MixD<R> mx, PhysP ph,
                                                            const R* U, const R* UF, OT* B, int ne, int per) {
  __shared__ __align__(16) char lds[jac_mixed_inv_lds<E, EO, NV, R>()];
  const int n0 = blockIdx.x * per, n1 = min(ne, n0 + per);
  jac_mixed_inv_body<E, EO, NV, SYS, R, OT>(n0, n1, threadIdx.x, blockDim.x, lds, op, geo, mx, ph, U, UF, B,
                                            DevSync());
}

// Matrix-core Jacobian (tensor-product elements, FP32): sensitivities once
// per mesh, tables per state, then one wavefront per (element, block, tile).
template <class E, int NV, int SYS, class R>
__global__ void __launch_bounds__(kThreads) k_jac_mf_sens(OpsD<R> op, Ops1D<R> o1, GeoD<R> geo, PhysP ph, R* out,
                                                          int nsb) {
  __shared__ __align__(16) char lds[jac_mf_sens_lds<E, NV, SYS, R>()];
  jac_mf_sens_body<E, NV, SYS, R>(blockIdx.x, threadIdx.x, blockDim.x, lds, op, o1, geo, ph, out, nsb);
}
template <class E, int NV, int SYS, class R>
__global__ void __launch_bounds__(kThreads) k_jac_mf_tab(GeoD<R> geo, PhysP ph, const R* U, const R* Q, const R* UF,
                                                         const R* QF, R* out) {
  __shared__ __align__(16) char lds[jac_mf_tables_lds<E, NV, SYS, R>()];
  jac_mf_tables_body<E, NV, SYS, R>(blockIdx.x, threadIdx.x, blockDim.x, lds, geo, ph, U, Q, UF, QF, out);
}
template <class E, int NV, int SYS, class R, class OT>
__global__ void __launch_bounds__((64 * jac_mf_wpb<E, NV, SYS, R>()))
__attribute__((amdgpu_waves_per_eu(jac_mf_min_waves<E, NV, SYS, R, OT>()))) k_jac_mf_asm(Ops1D<R> o1, const R* rdet,
                                                                                const R* tab, const R* sens,
                                                                                const R* sigtab, const int* sig,
                                                                                int nsb, int nblk, long ntasks, OT* B) {
  typedef MfSizes<E, NV, SYS> Y;
  constexpr int WPB = jac_mf_wpb<E, NV, SYS, R>(), STG = jac_mf_stage<E, NV, SYS, R>();
  __shared__ __align__(16) R stage[WPB * STG];
  __shared__ __align__(16) char xs[jac_mf_xs_bytes<E, NV, SYS, R, OT>()];
  const int wave = threadIdx.x >> 6;
  // Workgroups are dealt to the 8 XCDs in turn; renumber them so that each
  // XCD runs a contiguous range of tasks: the tasks of one (element, block)
  // and the blocks of one element then share that XCD's L2.
  const unsigned nwg = gridDim.x, q = nwg / 8u, rm = nwg % 8u, x = blockIdx.x % 8u, j = blockIdx.x / 8u;
  const unsigned wg = x < rm ? x * (q + 1u) + j : rm * (q + 1u) + (x - rm) * q + j;
  const long task = (long)wg * WPB + wave;
  const bool active = task < ntasks;        // every wave reaches the barrier inside the task
  const long t = active ? task : 0;
  const int sub = (int)(t % Y::TASKS);
  const int k = (int)((t / Y::TASKS) % nblk);
  const int n = (int)(t / ((long)Y::TASKS * nblk));
  const int slab = sub % Y::SL, nt = (sub / Y::SL) % Y::NT, mt = sub / (Y::SL * Y::NT);
  R* stg = stage + wave * STG;
  const int lane = threadIdx.x & 63;
  jac_mf_task<E, NV, SYS, R, OT>(n, k, mt, nt, slab, lane, o1, rdet, tab, sens, sigtab, sig, nsb, nblk, B, stg, xs,
                                 active);
}

template <class R> Ops1D<R>& ctx_o1(fr_ctx_s* c);
template <> inline Ops1D<float>& ctx_o1<float>(fr_ctx_s* c) { return c->o1f; }
template <> inline Ops1D<double>& ctx_o1<double>(fr_ctx_s* c) { return c->o1d; }

template <class R> OpsD<R>& ctx_ops(fr_ctx_s* c);
template <> inline OpsD<float>& ctx_ops<float>(fr_ctx_s* c) { return c->opsf; }
template <> inline OpsD<double>& ctx_ops<double>(fr_ctx_s* c) { return c->opsd; }
template <class R> GeoD<R>& ctx_geo(fr_ctx_s* c);
template <> inline GeoD<float>& ctx_geo<float>(fr_ctx_s* c) { return c->geof; }
template <> inline GeoD<double>& ctx_geo<double>(fr_ctx_s* c) { return c->geod; }

template <int ET, int P, int SYS, class R> struct Impl {
  typedef Elem<ET, P> E;
  static constexpr int NV = (SYS == SYS_ADV) ? 1 : E::ND + 2;
  static constexpr bool VISC = SysTraits<SYS>::kVisc;

  // T: scalar of the evaluation (real or dual), RC: its base precision
  // (operators and geometry), IO: precision of U, V and the outputs.
  // SDRT (tensor elements): the FR trace and gradient passes (the gradient
  // with the SD correction is the SDRT gradient), then the SDRT divergence.
  template <class T, class RC, class IO>
  static int residual_sd(fr_ctx_s* c, const IO* U, const IO* V, T* UF, T* Q, T* QF, IO* Rout, IO* Rtan) {
    if constexpr (!et_tensor(ET)) {
      c->err = "SDRT is provided for quadrilaterals and hexahedra";
      return -2;
    } else {
      OpsD<RC> op = ctx_ops<RC>(c);
      GeoD<RC> geo = ctx_geo<RC>(c);
      const int ne = (int)c->ne;
      const int TE = rhs_tile<E>();
      const int nt = (ne + TE - 1) / TE;
      hipLaunchKernelGGL((k_trace<E, NV, T, RC, IO>), dim3(nt), dim3(kThreads), 0, c->stream, op, ne, U, V, UF);
      FR_LAUNCH_CHECK(c);
      if (c->visc) {
        constexpr int GT = grad_tile<E, T>();
        hipLaunchKernelGGL((k_grad<E, NV, T, RC, IO>), dim3((ne + GT - 1) / GT), dim3(kThreads), 0, c->stream, op, geo,
                           c->ph.beta, U, V, (const T*)UF, Q, QF);
        FR_LAUNCH_CHECK(c);
      }
      if (c->timing) fr_time_begin(c, 1);
      hipLaunchKernelGGL((k_sd_div<E, NV, SYS, T, RC, IO>), dim3(nt), dim3(kThreads), 0, c->stream, op, geo, c->ph,
                         U, V, (const T*)UF, (const T*)Q, (const T*)QF, Rout, Rtan);
      FR_LAUNCH_CHECK(c);
      if (c->timing) fr_time_end(c, 1);
      return 0;
    }
  }
  static int rhs_sd(fr_ctx_s* c, const void* U, void* Rout) {
    return residual_sd<double, double, R>(c, (const R*)U, (const R*)nullptr, (double*)c->UF64, (double*)c->Q64,
                                          (double*)c->QF64, (R*)Rout, (R*)nullptr);
  }
  static int jvp_sd(fr_ctx_s* c, const void* U, const void* V, void* Jv, void* Rv) {
    return residual_sd<Dual<double>, double, R>(c, (const R*)U, (const R*)V, (Dual<double>*)c->UFd,
                                                (Dual<double>*)c->Qd, (Dual<double>*)c->QFd, (R*)Rv, (R*)Jv);
  }

  template <class T, class RC, class IO>
  static int residual(fr_ctx_s* c, const IO* U, const IO* V, T* UF, T* Q, T* QF, IO* Rout, IO* Rtan) {
    OpsD<RC> op = ctx_ops<RC>(c);
    GeoD<RC> geo = ctx_geo<RC>(c);
    const int ne = (int)c->ne;
    const int TE = rhs_tile<E>();
    const int nt = (ne + TE - 1) / TE;
    hipLaunchKernelGGL((k_trace<E, NV, T, RC, IO>), dim3(nt), dim3(kThreads), 0, c->stream, op, ne, U, V, UF);
    FR_LAUNCH_CHECK(c);
    if (c->visc) {
      constexpr int GT = grad_tile<E, T>();
      hipLaunchKernelGGL((k_grad<E, NV, T, RC, IO>), dim3((ne + GT - 1) / GT), dim3(kThreads), 0, c->stream, op, geo,
                         c->ph.beta, U, V, (const T*)UF, Q, QF);
      FR_LAUNCH_CHECK(c);
    }
    if (c->timing) fr_time_begin(c, 1);
    constexpr int TD = div_tile<E, NV, SYS, T, RC>();
    hipLaunchKernelGGL((k_div<E, NV, SYS, T, RC, IO>), dim3((ne + TD - 1) / TD), dim3(kThreads), 0, c->stream, op,
                       geo, c->ph, U, V, (const T*)UF, (const T*)Q, (const T*)QF, Rout, Rtan, c->jv_a, c->jv_b);
    FR_LAUNCH_CHECK(c);
    if (c->timing) fr_time_end(c, 1);
    return 0;
  }

  // The residual is always evaluated in FP64 (the FR divergence of a flux with
  // a large mean, e.g. the pressure at low Mach number, loses about
  // log10(|D| |F| / |R|) digits); FP32 contexts read and write FP32 states.
  static int rhs(fr_ctx_s* c, const void* U, void* Rout) {
    return residual<double, double, R>(c, (const R*)U, (const R*)nullptr, (double*)c->UF64, (double*)c->Q64,
                                       (double*)c->QF64, (R*)Rout, (R*)nullptr);
  }

  // The same evaluation with the FP64 traces and gradients in caller memory.
  static int rhs_ws(fr_ctx_s* c, const void* U, void* Rout, void* UF, void* Q, void* QF) {
    return residual<double, double, R>(c, (const R*)U, (const R*)nullptr, (double*)UF, (double*)Q, (double*)QF,
                                       (R*)Rout, (R*)nullptr);
  }

  // The JVP too: one FP64 dual-number evaluation (the tangent of a
  // low-Mach flux divergence cancels like the divergence itself).
  static int jvp(fr_ctx_s* c, const void* U, const void* V, void* Jv, void* Rv) {
    return residual<Dual<double>, double, R>(c, (const R*)U, (const R*)V, (Dual<double>*)c->UFd,
                                             (Dual<double>*)c->Qd, (Dual<double>*)c->QFd, (R*)Rv, (R*)Jv);
  }

  // One residual pass of an element group (mixed meshes run each pass over
  // every group before the next: the passes read the neighbours' traces).
  template <class T, class IO>
  static int phase_t(fr_ctx_s* c, int which, const IO* U, const IO* V, T* UF, T* Q, T* QF, IO* Rout, IO* Rtan) {
    OpsD<double> op = ctx_ops<double>(c);
    GeoD<double> geo = ctx_geo<double>(c);
    const int ne = (int)c->ne;
    if (ne == 0) return 0;
    const int TE = rhs_tile<E>();
    const int nt = (ne + TE - 1) / TE;
    if (which == 0) {
      hipLaunchKernelGGL((k_trace<E, NV, T, double, IO>), dim3(nt), dim3(kThreads), 0, c->stream, op, ne, U, V, UF);
    } else if (which == 1) {
      if (!c->visc) return 0;
      constexpr int GT = grad_tile<E, T>();
      hipLaunchKernelGGL((k_grad<E, NV, T, double, IO>), dim3((ne + GT - 1) / GT), dim3(kThreads), 0, c->stream, op,
                         geo, c->ph.beta, U, V, (const T*)UF, Q, QF);
    } else {
      constexpr int TD = div_tile<E, NV, SYS, T, double>();
      hipLaunchKernelGGL((k_div<E, NV, SYS, T, double, IO>), dim3((ne + TD - 1) / TD), dim3(kThreads), 0, c->stream,
                         op, geo, c->ph, U, V, (const T*)UF, (const T*)Q, (const T*)QF, Rout, Rtan, 0.0, 1.0);
    }
    FR_LAUNCH_CHECK(c);
    return 0;
  }
  static int phase(fr_ctx_s* c, int which, int dual, const void* U, const void* V, void* UF, void* Q, void* QF,
                   void* Rout, void* Rtan) {
    if (dual)
      return phase_t<Dual<double>, R>(c, which, (const R*)U, (const R*)V, (Dual<double>*)UF, (Dual<double>*)Q,
                                      (Dual<double>*)QF, (R*)Rout, (R*)Rtan);
    return phase_t<double, R>(c, which, (const R*)U, (const R*)nullptr, (double*)UF, (double*)Q, (double*)QF,
                              (R*)Rout, (R*)nullptr);
  }

  // Jacobian blocks of an element group of a mixed 2-D mesh (inviscid).
  static constexpr bool kMixedJac = (ET == ET_QUAD || ET == ET_TRI) && SYS != SYS_NS;
  template <class OT> static int jac_mixed_t(fr_ctx_s* c, int stage, const R* U, OT* B, const MixD<R>* mx) {
    if constexpr (!kMixedJac) {
      c->err = "Jacobian blocks of mixed meshes: 2-D inviscid systems only";
      return -2;
    } else {
      typedef Elem<(ET == ET_TRI ? ET_QUAD : ET_TRI), P> EO;
      if (c->visc) { c->err = "Jacobian blocks of mixed meshes: inviscid systems only"; return -2; }
      const int ne = (int)c->ne;
      if (ne == 0) return 0;
      OpsD<R> op = ctx_ops<R>(c);
      GeoD<R> geo = ctx_geo<R>(c);
      if (stage == 0) {
        const int TE = rhs_tile<E>();
        hipLaunchKernelGGL((k_trace<E, NV, R, R, R>), dim3((ne + TE - 1) / TE), dim3(kThreads), 0, c->stream, op, ne,
                           U, (const R*)nullptr, (R*)c->UF);
      } else if (stage == 1) {
        // a few tiles per workgroup: the operators are staged once for them
        constexpr int TE = mixed_tile<E>();
        const int per = TE * (ne >= 4096 * TE ? 4 : (ne >= 1024 * TE ? 2 : 1));
        hipLaunchKernelGGL((k_jac_mixed_inv<E, EO, NV, SYS, R, OT>), dim3((ne + per - 1) / per), dim3(kThreads), 0,
                           c->stream, op, geo, *mx, c->ph, U, (const R*)c->UF, B, ne, per);
      }
      FR_LAUNCH_CHECK(c);
      return 0;
    }
  }
  static int jac_mixed(fr_ctx_s* c, int stage, const void* U, void* B, int out_prec, const void* mix) {
    const MixD<R>* mx = (const MixD<R>*)mix;
    if constexpr (std::is_same<R, double>::value) {
      if (out_prec == 0) return jac_mixed_t<double>(c, stage, (const R*)U, (double*)B, mx);
    } else {
      if (out_prec == 1) return jac_mixed_t<float>(c, stage, (const R*)U, (float*)B, mx);
      if (out_prec == 2) return jac_mixed_t<bf16_t>(c, stage, (const R*)U, (bf16_t*)B, mx);
    }
    c->err = "unsupported block precision for this context precision";
    return -2;
  }

  static constexpr bool tensor_fits() {
    if constexpr (et_tensor(ET)) return jac_tp_lds<E, NV, SYS, R>() <= kMaxLds;
    else return false;
  }
  static constexpr bool mfma_fits() {
    if constexpr (et_tensor(ET) && std::is_same<R, float>::value)
      return jac_mf_sens_lds<E, NV, SYS, R>() <= kMaxLds && jac_mf_tables_lds<E, NV, SYS, R>() <= kMaxLds;
    else return false;
  }
  static constexpr bool kTensorPath = tensor_fits();
  // matrix-core path: FP32 quadrilaterals and hexahedra
  static constexpr bool kMfmaPath = mfma_fits();
  // the generic assembly needs faces of equal size (not prisms)
  static constexpr bool generic_fits() {
    if constexpr (ET == ET_PRI) return false;
    else return jac_lds<E, NV, SYS, R>() <= kMaxLds;
  }
  typedef MfSizes<E, NV, SYS> MF;

  template <class OT> static int jac_t(fr_ctx_s* c, const R* U, OT* B, int nblk) {
    if constexpr (!kMfmaPath && !kTensorPath && !generic_fits()) {
      c->err = ET == ET_PRI ? "Jacobian blocks are not provided for prisms"
                            : "Jacobian blocks of this element type / degree / precision do not fit one workgroup";
      return -2;
    } else {
    OpsD<R> op = ctx_ops<R>(c);
    GeoD<R> geo = ctx_geo<R>(c);
    const int ne = (int)c->ne;
    const int TE = rhs_tile<E>();
    const int nt = (ne + TE - 1) / TE;
    R* UF = (R*)c->UF;
    R* Q = (R*)c->Q;
    R* QF = (R*)c->QF;
    hipLaunchKernelGGL((k_trace<E, NV, R, R, R>), dim3(nt), dim3(kThreads), 0, c->stream, op, ne, U, (const R*)nullptr, UF);
    FR_LAUNCH_CHECK(c);
    if (c->visc) {
      constexpr int GT = grad_tile<E, R>();
      hipLaunchKernelGGL((k_grad<E, NV, R, R, R>), dim3((ne + GT - 1) / GT), dim3(kThreads), 0, c->stream, op, geo,
                         c->ph.beta, U, (const R*)nullptr, (const R*)UF, Q, QF);
      FR_LAUNCH_CHECK(c);
    }
    if constexpr (kMfmaPath) {
      if (!c->mf_sens || !c->mf_tab || !c->mf_sigtab || !c->mf_sig) { c->err = "Jacobian workspace missing"; return -4; }
      if (c->timing) fr_time_begin(c, 0);     // tables + assembly
      hipLaunchKernelGGL((k_jac_mf_tab<E, NV, SYS, R>), dim3(ne), dim3(kThreads), 0, c->stream, geo, c->ph, U,
                         (const R*)Q, (const R*)UF, (const R*)QF, (R*)c->mf_tab);
      FR_LAUNCH_CHECK(c);
      const long ntasks = (long)ne * nblk * MF::TASKS;
      constexpr int per = jac_mf_wpb<E, NV, SYS, R>();
      hipLaunchKernelGGL((k_jac_mf_asm<E, NV, SYS, R, OT>), dim3((unsigned)((ntasks + per - 1) / per)), dim3(64 * per),
                         0, c->stream, ctx_o1<R>(c), geo.rdet, (const R*)c->mf_tab, (const R*)c->mf_sens,
                         (const R*)c->mf_sigtab, (const int*)c->mf_sig, 1 + E::NFACE, nblk, ntasks, B);
      FR_LAUNCH_CHECK(c);
      if (c->timing) fr_time_end(c, 0);
      return 0;
    } else {
    if (c->timing) fr_time_begin(c, 0);
    if constexpr (kTensorPath)
      hipLaunchKernelGGL((k_jac_tp<E, NV, SYS, R, OT>), dim3(ne), dim3(jac_tp_threads<E, NV, SYS, R>()), 0, c->stream,
                         op, ctx_o1<R>(c), geo,
                         c->ph, U, (const R*)Q, (const R*)UF, (const R*)QF, B, nblk);
    else
      hipLaunchKernelGGL((k_jac<E, NV, SYS, R, OT>), dim3(ne), dim3(kThreads), 0, c->stream, op, geo, c->ph, U,
                         (const R*)Q, (const R*)UF, (const R*)QF, B, nblk);
    FR_LAUNCH_CHECK(c);
    if (c->timing) fr_time_end(c, 0);
    return 0;
    }
    }
  }

  // out_prec: 0 = f64, 1 = f32, 2 = bf16
  static int jac(fr_ctx_s* c, const void* U, void* B, int out_prec, int nblk) {
    if constexpr (std::is_same<R, double>::value) {
      if (out_prec == 0) return jac_t<double>(c, (const R*)U, (double*)B, nblk);
    } else {
      if (out_prec == 1) return jac_t<float>(c, (const R*)U, (float*)B, nblk);
      if (out_prec == 2) return jac_t<bf16_t>(c, (const R*)U, (bf16_t*)B, nblk);
    }
    c->err = "unsupported block precision for this context precision";
    return -2;
  }

  // bytes per element of the matrix-core path's sensitivity and table arrays (0: not used)
  // which: 0 sensitivities, 1 tables
  static size_t mf_bytes(int which) {
    if constexpr (kMfmaPath)
      return which == 0 ? (size_t)(1 + E::NFACE) * MF::BLK * sizeof(R) : (size_t)MF::TAB * sizeof(R);
    else return 0;
  }
  static int mf_setup(fr_ctx_s* c) {
    if constexpr (kMfmaPath) {
      hipLaunchKernelGGL((k_jac_mf_sens<E, NV, SYS, R>), dim3((unsigned)c->ne), dim3(kThreads), 0, c->stream,
                         ctx_ops<R>(c), ctx_o1<R>(c), ctx_geo<R>(c), c->ph, (R*)c->mf_sens, 1 + E::NFACE);
      FR_LAUNCH_CHECK(c);
    }
    return 0;
  }

  static KernelSet set() {
    KernelSet k{&rhs, &rhs_ws, &jvp, &jac, &mf_bytes, &mf_setup, nullptr, nullptr, &phase, nullptr};
    if constexpr (et_tensor(ET)) { k.rhs_sd = &rhs_sd; k.jvp_sd = &jvp_sd; }
    if constexpr (ET == ET_QUAD || ET == ET_TRI) k.jac_mixed = &jac_mixed;
    return k;
  }
};
