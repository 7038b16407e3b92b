// Library-internal context shared by the C ABI and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "fr_jac_tp.hpp"

struct fr_ctx_s;

// Type-erased launchers of one (element type, degree, system, precision).
struct KernelSet {
  int (*rhs)(fr_ctx_s*, const void* U, void* R);
  // the residual with caller-provided FP64 trace / gradient workspaces
  int (*rhs_ws)(fr_ctx_s*, const void* U, void* R, void* UF, void* Q, void* QF);
  int (*jvp)(fr_ctx_s*, const void* U, const void* V, void* Jv, void* Rv);
  int (*jac)(fr_ctx_s*, const void* U, void* B, int out_prec, int nblk);
  size_t (*mf_bytes)(int which);       // matrix-core Jacobian workspaces per element (0: sensitivities, 1: tables)
  int (*mf_setup)(fr_ctx_s*);          // computes the geometry-only sensitivities
  // SDRT residual and its tangent (tensor elements; null for triangles)
  int (*rhs_sd)(fr_ctx_s*, const void* U, void* R);
  int (*jvp_sd)(fr_ctx_s*, const void* U, const void* V, void* Jv, void* Rv);
  // one pass of the FR-DG residual (0 traces, 1 BR1 gradients, 2 divergence)
  // in FP64 on the given workspaces; dual = 1 carries the tangent direction V
  // (outputs: Rout = R, may be null; Rtan = Jv)
  int (*phase)(fr_ctx_s*, int which, int dual, const void* U, const void* V, void* UF, void* Q, void* QF, void* Rout,
               void* Rtan);
  // element group of a mixed mesh, inviscid systems: stage 0 traces (context
  // precision, into the group's UF), 1 every block; mix: a host MixD of the
  // context precision (2-D types only, null otherwise)
  int (*jac_mixed)(fr_ctx_s*, int stage, const void* U, void* B, int out_prec, const void* mix);
};

struct fr_ctx_s {
  int nd = 0, type = 0, p = 0, system = 0, nv = 0, prec = 0;
  int scheme = 0;              // 0 FR-DG, 1 FR-SDRT, 2 SDRT
  int64_t ne = 0;
  int ns = 0, nf = 0, nface = 0, nfp = 0, b = 0;
  bool visc = false;
  PhysP ph{};
  hipStream_t stream = nullptr;
  std::string err;
  KernelSet ks{};
  // The tangent output of the FR-DG JVP is jv_a V + jv_b J V (jv_fused: the
  // context's jvp honours them; the solver writes (I - dt J) v this way)
  double jv_a = 0.0, jv_b = 1.0;
  bool jv_fused = false;
  // device allocations owned by the context
  void* ops_mem = nullptr;
  void* geo_mem = nullptr;
  void* work_mem = nullptr;
  int* status = nullptr;       // device [2]: kinds of non-finite outputs (FR_NF_*), smallest element
  std::vector<double> face_off;  // host [ne][nface][nd]: face centroid - element centroid
  int64_t ndof = 0;            // state entries (sum of ns * nv over the elements)
  int64_t nf_tot = 0, ns_tot = 0;   // flux and solution points of the whole mesh
  // mixed meshes: one sub-context per element-type group (elements grouped
  // by type), sharing this context's workspaces and status word
  bool mixed = false, sub = false;
  std::vector<fr_ctx_s*> grp;
  std::vector<int64_t> grp_e0, grp_dof0, grp_fp0, grp_sp0;   // first element / state entry / flux / solution point
  std::vector<int64_t> blk_off;     // [ne + 1] first Jacobian-block entry of each element
  void* mix_mem = nullptr;          // group: MixInfo arrays and block offsets (device)
  const void* mixd = nullptr;       // group: host MixD<context precision> for jac_mixed
  void* mixd_host = nullptr;        // its storage
  int dev = 0;                 // device the context was created on
  OpsD<float> opsf{}; OpsD<double> opsd{};
  Ops1D<float> o1f{}; Ops1D<double> o1d{};
  GeoD<float> geof{}; GeoD<double> geod{};
  // workspaces: traces and gradients, real and dual
  void* UF = nullptr; void* Q = nullptr; void* QF = nullptr;        // context precision
  void* UF64 = nullptr; void* Q64 = nullptr; void* QF64 = nullptr;  // FP64 residual
  void* UFd = nullptr; void* Qd = nullptr; void* QFd = nullptr;
  void* mf_mem = nullptr; void* mf_sens = nullptr; void* mf_tab = nullptr;   // matrix-core Jacobian
  void* mf_sigtab = nullptr;   // shared reference sensitivities, one block per key
  int* mf_sig = nullptr;       // [ne][1 + nface] key of each block's reference part
  int mf_nsig = 0;
  // optional timing of the dominant kernels with HIP events on the context stream
  static constexpr int kEvPool = 64;
  bool timing = false;
  hipEvent_t ev[2][kEvPool][2] = {};
  int ev_n[2] = {0, 0};
  double ev_ms[2] = {0.0, 0.0};
  long ev_count[2] = {0, 0};
};

// Brackets a kernel launch with timing events (which: 0 = Jacobian assembly,
// 1 = residual divergence pass).  Pools are drained when full.
void fr_time_begin(fr_ctx_s* c, int which);
void fr_time_end(fr_ctx_s* c, int which);

// Clears the non-finite report (synchronous; not for capture).
int fr_status_reset(fr_ctx_s* c);

// Registry lookup implemented by the per-instantiation translation units.
bool fr_find_kernels(int type, int p, int system, int prec, KernelSet* out);

#define FR_LAUNCH_CHECK(ctx)                                         \
  do {                                                               \
    hipError_t e_ = hipGetLastError();                               \
    if (e_ != hipSuccess) {                                          \
      (ctx)->err = std::string("kernel launch: ") + hipGetErrorString(e_); \
      return -4;                                                     \
    }                                                                \
  } while (0)
