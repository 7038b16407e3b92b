// Batched residual and Jacobian blocks over many meshes in one launch per
// phase (mixed element types and degrees).
//
// A batch groups FP32 contexts of one system (2-D Euler or Navier-Stokes) on
// triangles and quadrilaterals of degree 1..4; a context whose mesh mixes
// triangles and quadrilaterals (Euler batches) enters as its two element
// groups, which share the mesh's trace workspace, so every phase covers every
// group before the next phase starts.  Each phase (traces, BR1
// gradients, divergence; or the Jacobian prelude and block assembly) is one
// persistent launch: workgroups walk a work list of (mesh, first tile,
// tile count) items, longest first, and switch on the mesh's (type, degree)
// to the same kernel bodies the single-mesh path uses, so every mesh's
// residual is bitwise identical to the mesh run alone.  Jacobian blocks of
// quadrilateral meshes have a faster single-mesh path (matrix-core tables and
// assembly): the default Jacobian strategy runs those meshes on it (bitwise
// identical again), the fully persistent strategies assemble them with the
// scalar bodies (FP32 parity).  The strategy, grid size and work-item
// granularity per (type, degree) come from a table that fr_batch_tune fills
// by timing candidates on the batch itself.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "fr.h"
#include "fr_impl.hpp"

namespace {

constexpr int kBT = 256;   // threads of the persistent workgroups
constexpr int kNV = 4;     // 2-D Euler / Navier-Stokes
constexpr FR_HD int bcode(int et, int p) { return et * 8 + p; }
constexpr int kMixCode = 16;   // added to the code of an element group of a mixed mesh

#define FR_BATCH_CASES(X) \
  X(ET_TRI, 1) X(ET_TRI, 2) X(ET_TRI, 3) X(ET_TRI, 4) X(ET_QUAD, 1) X(ET_QUAD, 2) X(ET_QUAD, 3) X(ET_QUAD, 4)

struct BDesc {
  OpsD<double> opd; GeoD<double> geod;        // FP64 residual
  OpsD<float> opr; GeoD<float> geor;          // FP32 Jacobian
  Ops1D<float> o1;
  MixD<float> md;                             // element group of a mixed mesh: cross-type data
  PhysP ph;
  int ne, code, visc, nblk;
  int mesh, mix;                              // mesh of the group; 1 for a group of a mixed mesh
  long uoff;                                  // first state entry of the group in its mesh
  double *UF64, *Q64, *QF64;
  float *UFr, *Qr, *QFr;
};
struct BItem { int desc, first, count, pad; };   // tiles (residual phases) or elements (assembly)
constexpr int kMaxMeshes = 64;
// per-call state / output pointers, passed by value as a kernel argument
struct BPtrs { const float* U[kMaxMeshes]; float* R[kMaxMeshes]; float* B[kMaxMeshes]; };

template <int ET, int P> constexpr int tile_of() { return rhs_tile<Elem<ET, P>>(); }
static int tile_rt(int code) {
  code %= kMixCode;
#define TCASE(ET, P) if (code == bcode(ET, P)) return tile_of<ET, P>();
  FR_BATCH_CASES(TCASE)
#undef TCASE
  return 1;
}
// elements per unit of the assembly work list: mixed-mesh groups are
// assembled in tiles
static int asm_unit_rt(int code) {
  if (code < kMixCode) return 1;
  code -= kMixCode;
#define ACASE(ET, P) if (code == bcode(ET, P)) return mixed_tile<Elem<ET, P>>();
  FR_BATCH_CASES(ACASE)
#undef ACASE
  return 1;
}

constexpr int cmax(int a, int b) { return a > b ? a : b; }
template <int SYS> constexpr int res_lds() {
  int m = 0;
#define LCASE(ET, P)                                                                                      \
  m = cmax(m, trace_lds<Elem<ET, P>, kNV, double, double>());                                             \
  m = cmax(m, grad_lds<Elem<ET, P>, kNV, double, double>());                                              \
  m = cmax(m, div_lds<Elem<ET, P>, kNV, SYS, double, double>());
  FR_BATCH_CASES(LCASE)
#undef LCASE
  return m;
}
template <int ET, int P> using OtherElem = Elem<(ET == ET_TRI ? ET_QUAD : ET_TRI), P>;
template <int ET, int P, int SYS> constexpr int asm_lds_one() {
  return cmax(ET == ET_TRI ? jac_lds<Elem<ET, P>, kNV, SYS, float>() : jac_tp_lds<Elem<ET, P>, kNV, SYS, float>(),
              jac_mixed_inv_lds<Elem<ET, P>, OtherElem<ET, P>, kNV, float>());
}
template <int SYS> constexpr int jac_lds_all() {
  int m = 0;
#define JCASE(ET, P)                                                                                      \
  m = cmax(m, trace_lds<Elem<ET, P>, kNV, float, float>());                                               \
  m = cmax(m, grad_lds<Elem<ET, P>, kNV, float, float>());                                                \
  m = cmax(m, asm_lds_one<ET, P, SYS>());
  FR_BATCH_CASES(JCASE)
#undef JCASE
  return m;
}

// One work item of a residual phase (PH: 0 traces, 1 gradients, 2
// divergence; FP64 residual of FP32 states) for one (type, degree).
// The descriptor is copied into locals first: the bodies store through float
// pointers, and operands read through a pointer into global memory would
// have to be reloaded after every such store.
template <int ET, int DEG, int SYS, int PH>
__device__ __forceinline__ void res_item(char* lds, const BDesc* D, const BPtrs& P, const BItem& w) {
  typedef Elem<ET, DEG> E;
  const OpsD<double> op = D[w.desc].opd;
  const GeoD<double> geo = D[w.desc].geod;
  const PhysP ph = D[w.desc].ph;
  const int ne = D[w.desc].ne;
  double* UF = D[w.desc].UF64;
  double* Q = D[w.desc].Q64;
  double* QF = D[w.desc].QF64;
  const long uoff = D[w.desc].uoff;
  const int mesh = D[w.desc].mesh;
  const float* U = P.U[mesh] + uoff;
  float* Rout = P.R[mesh] ? P.R[mesh] + uoff : nullptr;
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int t = w.first; t < w.first + w.count; ++t) {
    if constexpr (PH == 0)
      trace_body<E, kNV, double, double, float>(t, tid, nth, lds, op, ne, U, (const float*)nullptr, UF, DevSync());
    else if constexpr (PH == 1)
      grad_body<E, kNV, double, double, float>(t, tid, nth, lds, op, geo, ph.beta, U, (const float*)nullptr,
                                               (const double*)UF, Q, QF, DevSync());
    else
      div_body<E, kNV, SYS, double, double, float>(t, tid, nth, lds, op, geo, ph, U, (const float*)nullptr,
                                                   (const double*)UF, (const double*)Q, (const double*)QF, Rout,
                                                   (float*)nullptr, DevSync());
    __syncthreads();
  }
}

// MIX: 1 the item is a group of a mixed mesh, 0 it is not, -1 decided per item.
template <int ET, int DEG, int SYS, int PH, int MIX>
__device__ __forceinline__ void jac_item(char* lds, const BDesc* D, const BPtrs& P, const BItem& w) {
  typedef Elem<ET, DEG> E;
  const OpsD<float> op = D[w.desc].opr;
  const GeoD<float> geo = D[w.desc].geor;
  const PhysP ph = D[w.desc].ph;
  const int ne = D[w.desc].ne, nblk = D[w.desc].nblk;
  float* UF = D[w.desc].UFr;
  float* Q = D[w.desc].Qr;
  float* QF = D[w.desc].QFr;
  const int mesh = D[w.desc].mesh;
  const float* U = P.U[mesh] + D[w.desc].uoff;
  float* B = P.B[mesh];
  const int tid = threadIdx.x, nth = blockDim.x;
  if constexpr (PH == 2 && SYS == SYS_EULER && MIX != 0) {
    if (MIX == 1 || D[w.desc].mix) {
      // a group of a mixed mesh (inviscid): self blocks, then the face
      // blocks through the neighbour's own interpolation; blocks at absolute
      // offsets in the mesh's array
      // items count tiles of mixed_tile<E>() elements
      constexpr int TE = mixed_tile<E>();
      const MixD<float> md = D[w.desc].md;
      const int n0 = w.first * TE, n1 = min(ne, (w.first + w.count) * TE);
      jac_mixed_inv_body<E, OtherElem<ET, DEG>, kNV, SYS, float, float>(n0, n1, tid, nth, lds, op, geo, md, ph, U,
                                                                        UF, B, DevSync());
      __syncthreads();
      return;
    }
  }
  if constexpr (PH == 2 && MIX == 1) {
    return;
  } else if constexpr (PH == 2 && ET != ET_TRI) {
    const Ops1D<float> o1 = D[w.desc].o1;
    for (int t = w.first; t < w.first + w.count; ++t) {
      jac_tp_body<E, kNV, SYS, float, float>(t, tid, nth, lds, op, o1, geo, ph, U, Q, UF, QF, B, nblk, DevSync());
      __syncthreads();
    }
  } else {
    for (int t = w.first; t < w.first + w.count; ++t) {
      if constexpr (PH == 0)
        trace_body<E, kNV, float, float, float>(t, tid, nth, lds, op, ne, U, (const float*)nullptr, UF, DevSync());
      else if constexpr (PH == 1)
        grad_body<E, kNV, float, float, float>(t, tid, nth, lds, op, geo, ph.beta, U, (const float*)nullptr,
                                               (const float*)UF, Q, QF, DevSync());
      else
        jac_body<E, kNV, SYS, float, float>(t, tid, nth, lds, op, geo, ph, U, Q, UF, QF, B, nblk, DevSync());
      __syncthreads();
    }
  }
}

// The mixed launch: one persistent grid over the whole work list, switching
// on each item's (type, degree).
template <int SYS, int PH>
__global__ void __launch_bounds__(kBT) k_batch_res(const BDesc* D, BPtrs P, const BItem* items, int nitems) {
  __shared__ __align__(16) char lds[res_lds<SYS>()];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const BItem w = items[it];
    const BDesc& d = D[w.desc];
    switch (d.code) {
#define RCASE(ET, DEG) \
  case bcode(ET, DEG): \
  case bcode(ET, DEG) + kMixCode: res_item<ET, DEG, SYS, PH>(lds, D, P, w); break;
      FR_BATCH_CASES(RCASE)
#undef RCASE
      default: break;
    }
  }
}
template <int SYS, int PH>
__global__ void __launch_bounds__(kBT) k_batch_jac(const BDesc* D, BPtrs P, const BItem* items, int nitems) {
  __shared__ __align__(16) char lds[jac_lds_all<SYS>()];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const BItem w = items[it];
    const BDesc& d = D[w.desc];
    switch (d.code) {
#define JCASE2(ET, DEG) \
  case bcode(ET, DEG): \
  case bcode(ET, DEG) + kMixCode: jac_item<ET, DEG, SYS, PH, -1>(lds, D, P, w); break;
      FR_BATCH_CASES(JCASE2)
#undef JCASE2
      default: break;
    }
  }
}

// Grouped launches: one persistent grid per (type, degree) with that
// group's own LDS and thread count.
template <int ET, int DEG, int SYS, int PH> constexpr int gres_lds() {
  typedef Elem<ET, DEG> E;
  return PH == 0 ? trace_lds<E, kNV, double, double>()
                 : (PH == 1 ? grad_lds<E, kNV, double, double>() : div_lds<E, kNV, SYS, double, double>());
}
// MIX: the groups of mixed meshes, whose assembly takes the mixed-mesh body
// only (its own LDS and thread count).
template <int ET, int DEG, int SYS, int PH, int MIX> constexpr int gjac_lds() {
  typedef Elem<ET, DEG> E;
  return PH == 0 ? trace_lds<E, kNV, float, float>()
                 : (PH == 1 ? grad_lds<E, kNV, float, float>()
                            : (MIX ? jac_mixed_inv_lds<E, OtherElem<ET, DEG>, kNV, float>()
                                   : asm_lds_one<ET, DEG, SYS>()));
}
template <int ET, int DEG, int SYS, int PH, int MIX> constexpr int gjac_threads() {
  return (PH == 2 && ET != ET_TRI && !MIX) ? jac_tp_threads<Elem<ET, DEG>, kNV, SYS, float>() : kThreads;
}
template <int ET, int DEG, int SYS, int PH>
__global__ void __launch_bounds__(kThreads) k_group_res(const BDesc* D, BPtrs P, const BItem* items, int nitems) {
  __shared__ __align__(16) char lds[gres_lds<ET, DEG, SYS, PH>()];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const BItem w = items[it];
    res_item<ET, DEG, SYS, PH>(lds, D, P, w);
  }
}
template <int ET, int DEG, int SYS, int PH, int MIX>
__global__ void __launch_bounds__((gjac_threads<ET, DEG, SYS, PH, MIX>())) k_group_jac(const BDesc* D, BPtrs P,
                                                                                      const BItem* items,
                                                                                      int nitems) {
  __shared__ __align__(16) char lds[gjac_lds<ET, DEG, SYS, PH, MIX>()];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const BItem w = items[it];
    jac_item<ET, DEG, SYS, PH, MIX>(lds, D, P, w);
  }
}

}  // namespace

struct fr_batch_s {
  std::vector<fr_ctx_s*> mesh;     // the contexts as given, one per mesh
  std::vector<fr_ctx_s*> ctx;      // one per descriptor: a single-type mesh, or a group of a mixed mesh
  int sys = 0, ncu = 1;
  hipStream_t stream = nullptr;
  BDesc* ddesc = nullptr;          // device
  BDesc* hdesc = nullptr;          // pinned
  // device work lists (all items longest first, then the same items grouped
  // by (type, degree)); seg_* give each group's range in the grouped half
  BItem* dres = nullptr;           // residual tiles
  BItem* djac = nullptr;           // assembly elements
  BItem* dtil = nullptr;           // tiles of the Jacobian prelude
  int nres = 0, njac = 0, ntil = 0;
  size_t cap_res = 0, cap_jac = 0, cap_til = 0;
  int seg_off[3][32], seg_cnt[3][32];
  std::vector<int> codes;          // (type, degree) codes present
  int res_mode = 0, jac_mode = 2;  // 0: one mixed launch per phase, 1: one launch per group,
                                   // 2 (Jacobian): as 1, quadrilateral meshes on the matrix-core path
  int k_res[32], k_jac[32];        // work-item granularity per (type, degree)
  int grid_res = 0, grid_jac = 0;  // persistent workgroups per launch
  hipEvent_t t0 = nullptr, t1 = nullptr;
  BPtrs ptrs{};
  std::string err;
};

static int desc_code(const fr_batch_s* b, size_t i) { return b->hdesc[i].code; }

static fr_status bfail(fr_batch_s* b, fr_status s, const std::string& m) {
  if (b) b->err = m;
  return s;
}

static int sec_cost(const fr_ctx_s* c) { return c->ns * (c->ns + c->nf); }
static int desc_code(const fr_batch_s* b, size_t i);

// work list: units (tiles or elements) in items of k[code] units, longest
// first; `seg` receives each group's range in the grouped copy (appended)
static void make_items(fr_batch_s* b, bool tiles, const int* k, std::vector<BItem>& out, int* seg_off,
                       int* seg_cnt) {
  out.clear();
  std::vector<std::pair<long, BItem>> v;
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    const fr_ctx_s* c = b->ctx[i];
    const int code = desc_code(b, i);
    const int te = tiles ? tile_rt(code) : asm_unit_rt(code);
    const int units = (int)((c->ne + te - 1) / te);
    const int per = std::max(1, k[code]);
    for (int u = 0; u < units; u += per) {
      BItem it{(int)i, u, std::min(per, units - u), 0};
      v.push_back({(long)it.count * te * sec_cost(c), it});
    }
  }
  std::stable_sort(v.begin(), v.end(), [](const auto& a, const auto& c) { return a.first > c.first; });
  for (auto& x : v) out.push_back(x.second);
  const size_t nall = out.size();
  for (int code = 0; code < 32; ++code) { seg_off[code] = 0; seg_cnt[code] = 0; }
  for (int code : b->codes) {
    seg_off[code] = (int)out.size();
    for (size_t j = 0; j < nall; ++j)
      if (desc_code(b, (size_t)out[j].desc) == code) out.push_back(out[j]);
    seg_cnt[code] = (int)out.size() - seg_off[code];
  }
}

static fr_status upload_items(fr_batch_s* b, const std::vector<BItem>& v, BItem** dst, size_t* cap, int* n) {
  if (v.size() > *cap) {
    if (*dst) (void)hipFree(*dst);
    *dst = nullptr;
    *cap = 0;
    if (hipMalloc(dst, v.size() * sizeof(BItem)) != hipSuccess) return bfail(b, FR_E_NOMEM, "batch work list");
    *cap = v.size();
  }
  if (hipMemcpy(*dst, v.data(), v.size() * sizeof(BItem), hipMemcpyHostToDevice) != hipSuccess)
    return bfail(b, FR_E_DEVICE, "batch work list upload");
  *n = (int)v.size() / 2;          // the mixed half
  return FR_OK;
}

static fr_status rebuild(fr_batch_s* b) {
  // launches already queued may still read the current lists
  if (hipStreamSynchronize(b->stream) != hipSuccess) return bfail(b, FR_E_DEVICE, "batch stream");
  std::vector<BItem> v;
  fr_status st;
  make_items(b, true, b->k_res, v, b->seg_off[0], b->seg_cnt[0]);
  if ((st = upload_items(b, v, &b->dres, &b->cap_res, &b->nres))) return st;
  int one[32];
  std::fill(one, one + 32, 1);
  make_items(b, true, one, v, b->seg_off[1], b->seg_cnt[1]);
  if ((st = upload_items(b, v, &b->dtil, &b->cap_til, &b->ntil))) return st;
  make_items(b, false, b->k_jac, v, b->seg_off[2], b->seg_cnt[2]);
  return upload_items(b, v, &b->djac, &b->cap_jac, &b->njac);
}

template <int SYS, int PH>
static void group_res(fr_batch_s* b, int code, const BItem* items, int n, int grid) {
  switch (code) {
#define GR(ET, DEG)                                                                                             \
  case bcode(ET, DEG):                                                                                          \
  case bcode(ET, DEG) + kMixCode:                                                                               \
    hipLaunchKernelGGL((k_group_res<ET, DEG, SYS, PH>), dim3(grid), dim3(kThreads), 0, b->stream, b->ddesc,      \
                       b->ptrs, items, n);                                                                      \
    break;
    FR_BATCH_CASES(GR)
#undef GR
    default: break;
  }
}
template <int SYS, int PH>
static void group_jac(fr_batch_s* b, int code, const BItem* items, int n, int grid) {
  switch (code) {
#define GJ(ET, DEG)                                                                                             \
  case bcode(ET, DEG):                                                                                          \
    hipLaunchKernelGGL((k_group_jac<ET, DEG, SYS, PH, 0>), dim3(grid), dim3(gjac_threads<ET, DEG, SYS, PH, 0>()), \
                       0, b->stream, b->ddesc, b->ptrs, items, n);                                              \
    break;                                                                                                      \
  case bcode(ET, DEG) + kMixCode:                                                                               \
    if constexpr (SYS == SYS_EULER)                                                                             \
      hipLaunchKernelGGL((k_group_jac<ET, DEG, SYS, PH, 1>), dim3(grid),                                        \
                         dim3(gjac_threads<ET, DEG, SYS, PH, 1>()), 0, b->stream, b->ddesc, b->ptrs, items, n); \
    break;
    FR_BATCH_CASES(GJ)
#undef GJ
    default: break;
  }
}
// grid <= 0: one workgroup per item (hardware scheduling, no persistent loop)
static int gsize(int grid, int n) { return grid <= 0 ? std::max(1, n) : std::max(1, std::min(grid, n)); }

template <int SYS>
static fr_status launch_res(fr_batch_s* b, bool visc) {
  if (b->res_mode == 0) {
    const dim3 g(gsize(b->grid_res, b->nres)), t(kBT);
    hipLaunchKernelGGL((k_batch_res<SYS, 0>), g, t, 0, b->stream, b->ddesc, b->ptrs, b->dres, b->nres);
    if (visc) hipLaunchKernelGGL((k_batch_res<SYS, 1>), g, t, 0, b->stream, b->ddesc, b->ptrs, b->dres, b->nres);
    hipLaunchKernelGGL((k_batch_res<SYS, 2>), g, t, 0, b->stream, b->ddesc, b->ptrs, b->dres, b->nres);
  } else {
    // phase by phase: a group of a mixed mesh reads the other group's traces
    for (int ph = 0; ph < 3; ++ph)
      for (int code : b->codes) {
        const BItem* it = b->dres + b->seg_off[0][code];
        const int n = b->seg_cnt[0][code], g = gsize(b->grid_res, n);
        if (ph == 0) group_res<SYS, 0>(b, code, it, n, g);
        else if (ph == 1) { if (visc) group_res<SYS, 1>(b, code, it, n, g); }
        else group_res<SYS, 2>(b, code, it, n, g);
      }
  }
  return hipGetLastError() == hipSuccess ? FR_OK : bfail(b, FR_E_DEVICE, "batch residual launch");
}
template <int SYS>
static fr_status launch_jac(fr_batch_s* b, bool visc) {
  if (b->jac_mode == 0) {
    const dim3 gt(gsize(b->grid_res, b->ntil)), t(kBT);
    hipLaunchKernelGGL((k_batch_jac<SYS, 0>), gt, t, 0, b->stream, b->ddesc, b->ptrs, b->dtil, b->ntil);
    if (visc) hipLaunchKernelGGL((k_batch_jac<SYS, 1>), gt, t, 0, b->stream, b->ddesc, b->ptrs, b->dtil, b->ntil);
    hipLaunchKernelGGL((k_batch_jac<SYS, 2>), dim3(gsize(b->grid_jac, b->njac)), t, 0, b->stream, b->ddesc, b->ptrs,
                       b->djac, b->njac);
  } else {
    // the single-mesh matrix-core path (tables + MFMA assembly) for
    // single-type quadrilateral meshes in mode 2, mesh by mesh on the batch
    // stream: the same kernels as the mesh run alone
    auto mf = [&](int code) { return b->jac_mode == 2 && code / 8 == ET_QUAD; };
    for (int code : b->codes) {
      if (!mf(code)) continue;
      for (size_t i = 0; i < b->ctx.size(); ++i) {
        if (b->hdesc[i].code != code) continue;
        fr_ctx_s* c = b->ctx[i];
        const int ms = b->hdesc[i].mesh;
        hipStream_t own = c->stream;
        c->stream = b->stream;
        const int rc = c->ks.jac(c, b->ptrs.U[ms], b->ptrs.B[ms], 1, b->hdesc[i].nblk);
        c->stream = own;
        if (rc) return bfail(b, (fr_status)rc, "mesh " + std::to_string(ms) + ": " + c->err);
      }
    }
    // the others phase by phase (a group of a mixed mesh reads the other
    // group's traces)
    for (int ph = 0; ph < 3; ++ph)
      for (int code : b->codes) {
        if (mf(code)) continue;
        const BItem* tl = b->dtil + b->seg_off[1][code];
        const int nt = b->seg_cnt[1][code], gt = gsize(b->grid_res, nt);
        if (ph == 0) group_jac<SYS, 0>(b, code, tl, nt, gt);
        else if (ph == 1) { if (visc) group_jac<SYS, 1>(b, code, tl, nt, gt); }
        else {
          const int na = b->seg_cnt[2][code];
          group_jac<SYS, 2>(b, code, b->djac + b->seg_off[2][code], na, gsize(b->grid_jac, na));
        }
      }
  }
  return hipGetLastError() == hipSuccess ? FR_OK : bfail(b, FR_E_DEVICE, "batch Jacobian launch");
}

static fr_status set_ptrs(fr_batch_s* b, const void* const* U, void* const* R, void* const* B) {
  BPtrs p{};
  for (size_t i = 0; i < b->mesh.size(); ++i) {
    if (!U[i] || (R && !R[i]) || (B && !B[i]))
      return bfail(b, FR_E_INVALID, "null pointer for mesh " + std::to_string(i));
    p.U[i] = (const float*)U[i];
    p.R[i] = R ? (float*)R[i] : nullptr;
    p.B[i] = B ? (float*)B[i] : nullptr;
  }
  b->ptrs = p;
  return FR_OK;
}

static fr_status run_rhs(fr_batch_s* b) {
  return b->sys == SYS_NS ? launch_res<SYS_NS>(b, true) : launch_res<SYS_EULER>(b, false);
}
static fr_status run_jac(fr_batch_s* b) {
  return b->sys == SYS_NS ? launch_jac<SYS_NS>(b, true) : launch_jac<SYS_EULER>(b, false);
}

static double time_ms(fr_batch_s* b, fr_status (*fn)(fr_batch_s*), int reps) {
  if (fn(b) != FR_OK) return 1e30;     // warm-up
  (void)hipEventRecord(b->t0, b->stream);
  for (int r = 0; r < reps; ++r)
    if (fn(b) != FR_OK) return 1e30;
  (void)hipEventRecord(b->t1, b->stream);
  (void)hipEventSynchronize(b->t1);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, b->t0, b->t1);
  return ms / reps;
}

extern "C" {

fr_status fr_batch_create(fr_ctx* const* ctxs, int n_ctx, fr_batch** out) {
  if (!ctxs || !out || n_ctx < 1 || n_ctx > kMaxMeshes) return FR_E_INVALID;
  *out = nullptr;
  fr_batch_s* b = new fr_batch_s();
  for (int i = 0; i < n_ctx; ++i) {
    fr_ctx_s* c = ctxs[i];
    if (!c) { fr_status s = bfail(nullptr, FR_E_INVALID, ""); delete b; return s; }
    const char* why = nullptr;
    if (c->prec != 1) why = "batched meshes must be FP32 contexts";
    else if (c->scheme == 2) why = "batched meshes must be FR (FR-DG or FR-SDRT) contexts";
    else if (c->mixed && c->system != SYS_EULER) why = "batched mixed meshes must be Euler (inviscid blocks)";
    else if (c->nd != 2 || (!c->mixed && c->type != ET_QUAD && c->type != ET_TRI))
      why = "batched meshes must be 2-D triangles or quadrilaterals";
    else if (c->system != SYS_EULER && c->system != SYS_NS) why = "batched meshes must be Euler or Navier-Stokes";
    else if (i > 0 && c->system != ctxs[0]->system) why = "batched meshes must share one system";
    else if (c->p < 1 || c->p > 4) why = "batched meshes must have degree 1..4";
    if (why) {
      c->err = std::string(why) + " (mesh " + std::to_string(i) + ")";
      delete b;
      return FR_E_UNSUPPORTED;
    }
    b->mesh.push_back(c);
  }
  std::vector<int> dmesh, dmix;
  std::vector<long> duoff;
  std::vector<const void*> dmd;
  for (size_t i = 0; i < b->mesh.size(); ++i) {
    fr_ctx_s* c = b->mesh[i];
    if (!c->mixed) {
      b->ctx.push_back(c); dmesh.push_back((int)i); dmix.push_back(0); duoff.push_back(0); dmd.push_back(nullptr);
      continue;
    }
    for (size_t g = 0; g < c->grp.size(); ++g) {
      b->ctx.push_back(c->grp[g]); dmesh.push_back((int)i); dmix.push_back(1);
      duoff.push_back((long)c->grp_dof0[g]); dmd.push_back(c->grp[g]->mixd);
    }
  }
  b->sys = ctxs[0]->system;
  b->stream = ctxs[0]->stream;
  for (size_t i = 0; i < b->ctx.size(); ++i)
    b->codes.push_back(bcode(b->ctx[i]->type, b->ctx[i]->p) + (dmix[i] ? kMixCode : 0));
  std::sort(b->codes.begin(), b->codes.end());
  b->codes.erase(std::unique(b->codes.begin(), b->codes.end()), b->codes.end());
  int dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, dev);
  b->grid_res = 4 * b->ncu;
  b->grid_jac = 2 * b->ncu;
  std::fill(b->k_res, b->k_res + 32, 1);
  std::fill(b->k_jac, b->k_jac + 32, 1);
  const size_t nd = b->ctx.size();
  if (hipMalloc(&b->ddesc, nd * sizeof(BDesc)) != hipSuccess ||
      hipHostMalloc((void**)&b->hdesc, nd * sizeof(BDesc), hipHostMallocDefault) != hipSuccess ||
      hipEventCreate(&b->t0) != hipSuccess || hipEventCreate(&b->t1) != hipSuccess) {
    fr_batch_destroy(b);
    return FR_E_NOMEM;
  }
  for (size_t i = 0; i < nd; ++i) {
    fr_ctx_s* c = b->ctx[i];
    BDesc& d = b->hdesc[i];
    d = BDesc{};
    d.opd = c->opsd; d.geod = c->geod; d.opr = c->opsf; d.geor = c->geof; d.o1 = c->o1f; d.ph = c->ph;
    d.ne = (int)c->ne; d.code = bcode(c->type, c->p); d.visc = c->visc ? 1 : 0; d.nblk = 1 + c->nface;
    d.UF64 = (double*)c->UF64; d.Q64 = (double*)c->Q64; d.QF64 = (double*)c->QF64;
    d.UFr = (float*)c->UF; d.Qr = (float*)c->Q; d.QFr = (float*)c->QF;
    d.mesh = dmesh[i]; d.mix = dmix[i]; d.uoff = duoff[i];
    if (dmix[i]) { d.md = *(const MixD<float>*)dmd[i]; d.code += kMixCode; }
  }
  if (hipMemcpy(b->ddesc, b->hdesc, nd * sizeof(BDesc), hipMemcpyHostToDevice) != hipSuccess) {
    fr_batch_destroy(b);
    return FR_E_DEVICE;
  }
  fr_status st = rebuild(b);
  if (st) { fr_batch_destroy(b); return st; }
  *out = b;
  return FR_OK;
}

fr_status fr_batch_destroy(fr_batch* b) {
  if (!b) return FR_E_INVALID;
  (void)hipStreamSynchronize(b->stream);
  (void)hipFree(b->ddesc);
  (void)hipFree(b->dres);
  (void)hipFree(b->djac);
  (void)hipFree(b->dtil);
  if (b->hdesc) (void)hipHostFree(b->hdesc);
  if (b->t0) (void)hipEventDestroy(b->t0);
  if (b->t1) (void)hipEventDestroy(b->t1);
  delete b;
  return FR_OK;
}

const char* fr_batch_last_error(const fr_batch* b) { return b ? b->err.c_str() : ""; }

fr_status fr_batch_rhs(fr_batch* b, const void* const* U, void* const* R) {
  if (!b || !U || !R) return FR_E_INVALID;
  fr_status st = set_ptrs(b, U, R, nullptr);
  return st ? st : run_rhs(b);
}

fr_status fr_batch_jacobian_blocks(fr_batch* b, const void* const* U, void* const* blocks) {
  if (!b || !U || !blocks) return FR_E_INVALID;
  fr_status st = set_ptrs(b, U, nullptr, blocks);
  return st ? st : run_jac(b);
}

fr_status fr_batch_tune(fr_batch* b, const void* const* U, void* const* R, void* const* blocks, int reps) {
  if (!b || !U || !R || !blocks || reps < 1) return FR_E_INVALID;
  fr_status st = set_ptrs(b, U, R, blocks);
  if (st) return st;
  // residual: grid size, then the tiles per work item of each (type, degree)
  // per phase: launch strategy, then grid size, then units per work item of
  // each (type, degree) (coordinate descent on measured times)
  auto tune_one = [&](int* mode, int nmodes, int* grid, int* k, fr_status (*fn)(fr_batch_s*),
                      const std::vector<int>& grids, const std::vector<int>& ks) -> fr_status {
    double best = 1e30;
    int bm = *mode;
    for (int md = 0; md < nmodes; ++md) {
      *mode = md;
      double t = time_ms(b, fn, reps);
      if (t < best) { best = t; bm = md; }
    }
    *mode = bm;
    int bg = *grid;
    for (int gm : grids) {
      *grid = gm * b->ncu;          // 0: uncapped
      double t = time_ms(b, fn, reps);
      if (t < best) { best = t; bg = *grid; }
    }
    *grid = bg;
    for (int code : b->codes) {
      int bk = k[code];
      for (int kk : ks) {
        k[code] = kk;
        fr_status s = rebuild(b);
        if (s) return s;
        double t = time_ms(b, fn, reps);
        if (t < best) { best = t; bk = kk; }
      }
      k[code] = bk;
      fr_status s = rebuild(b);
      if (s) return s;
    }
    return FR_OK;
  };
  if ((st = tune_one(&b->res_mode, 2, &b->grid_res, b->k_res, run_rhs, {1, 2, 4, 8, 0}, {1, 2, 4, 8}))) return st;
  if ((st = tune_one(&b->jac_mode, 3, &b->grid_jac, b->k_jac, run_jac, {1, 2, 4, 8, 0}, {1, 2, 4}))) return st;
  return hipStreamSynchronize(b->stream) == hipSuccess ? FR_OK : bfail(b, FR_E_DEVICE, "batch tuning");
}

fr_status fr_batch_tuning(const fr_batch* b, int* modes, int* grid_res, int* grid_jac, int* k_res, int* k_jac) {
  if (!b) return FR_E_INVALID;
  if (modes) { modes[0] = b->res_mode; modes[1] = b->jac_mode; }
  if (grid_res) *grid_res = b->grid_res;
  if (grid_jac) *grid_jac = b->grid_jac;
  if (k_res) std::copy(b->k_res, b->k_res + 32, k_res);
  if (k_jac) std::copy(b->k_jac, b->k_jac + 32, k_jac);
  return FR_OK;
}

fr_status fr_batch_set_tuning(fr_batch* b, const int* modes, int grid_res, int grid_jac, const int* k_res,
                              const int* k_jac) {
  if (!b || grid_res < 0 || grid_jac < 0) return FR_E_INVALID;
  if (modes) {
    if (modes[0] < 0 || modes[0] > 1 || modes[1] < 0 || modes[1] > 2) return bfail(b, FR_E_INVALID, "launch mode");
    b->res_mode = modes[0];
    b->jac_mode = modes[1];
  }
  b->grid_res = grid_res;
  b->grid_jac = grid_jac;
  for (int i = 0; i < 32; ++i) {
    if (k_res) b->k_res[i] = std::max(1, k_res[i]);
    if (k_jac) b->k_jac[i] = std::max(1, k_jac[i]);
  }
  return rebuild(b);
}

}  // extern "C"
