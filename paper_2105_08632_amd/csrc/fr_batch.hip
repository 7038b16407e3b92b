// Batched residual and Jacobian blocks over many meshes in one launch per
// phase (mixed element types and degrees).
//
// A batch groups FP32 contexts of one system (2-D Euler or Navier-Stokes) on
// triangles and quadrilaterals of degree 1..4.  Each phase (traces, BR1
// gradients, divergence; or the Jacobian prelude and block assembly) is one
// persistent launch: workgroups walk a work list of (mesh, first tile,
// tile count) items, longest first, and switch on the mesh's (type, degree)
// to the same kernel bodies the single-mesh path uses, so every mesh's result
// is bitwise identical to the mesh run alone.  The grid size and the work-item
// granularity per (type, degree) come from a table that fr_batch_tune fills by
// timing candidates on the batch itself.
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

#define FR_BATCH_CASES(X) \
  X(ET_TRI, 1) X(ET_TRI, 2) X(ET_TRI, 3) X(ET_TRI, 4) X(ET_QUAD, 1) X(ET_QUAD, 2) X(ET_QUAD, 3) X(ET_QUAD, 4)

struct BDesc {
  OpsD<double> opd; GeoD<double> geod;        // FP64 residual
  OpsD<float> opr; GeoD<float> geor;          // FP32 Jacobian
  Ops1D<float> o1;
  PhysP ph;
  int ne, code, visc, nblk;
  double *UF64, *Q64, *QF64;
  float *UFr, *Qr, *QFr;
};
struct BItem { int desc, first, count, pad; };   // tiles (residual phases) or elements (assembly)
constexpr int kMaxMeshes = 64;
// per-call state / output pointers, passed by value as a kernel argument
struct BPtrs { const float* U[kMaxMeshes]; float* R[kMaxMeshes]; float* B[kMaxMeshes]; };

template <int ET, int P> constexpr int tile_of() { return rhs_tile<Elem<ET, P>>(); }
static int tile_rt(int code) {
#define TCASE(ET, P) if (code == bcode(ET, P)) return tile_of<ET, P>();
  FR_BATCH_CASES(TCASE)
#undef TCASE
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
template <int ET, int P, int SYS> constexpr int asm_lds_one() {
  return ET == ET_TRI ? jac_lds<Elem<ET, P>, kNV, SYS, float>() : jac_tp_lds<Elem<ET, P>, kNV, SYS, float>();
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

// PH: 0 traces, 1 gradients, 2 divergence (FP64 residual of FP32 states)
template <int SYS, int PH>
__global__ void __launch_bounds__(kBT) k_batch_res(const BDesc* D, BPtrs P, const BItem* items, int nitems) {
  __shared__ __align__(16) char lds[res_lds<SYS>()];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const BItem w = items[it];
    const BDesc& d = D[w.desc];
    switch (d.code) {
#define RCASE(ET, DEG)                                                                                            \
  case bcode(ET, DEG): {                                                                                          \
    typedef Elem<ET, DEG> E;                                                                                      \
    const float* U = P.U[w.desc];                                                                                 \
    for (int t = w.first; t < w.first + w.count; ++t) {                                                           \
      if constexpr (PH == 0)                                                                                      \
        trace_body<E, kNV, double, double, float>(t, threadIdx.x, kBT, lds, d.opd, d.ne, U, (const float*)nullptr, \
                                                  d.UF64, DevSync());                                             \
      else if constexpr (PH == 1)                                                                                 \
        grad_body<E, kNV, double, double, float>(t, threadIdx.x, kBT, lds, d.opd, d.geod, d.ph.beta, U,           \
                                                 (const float*)nullptr, (const double*)d.UF64, d.Q64, d.QF64,     \
                                                 DevSync());                                                      \
      else                                                                                                        \
        div_body<E, kNV, SYS, double, double, float>(t, threadIdx.x, kBT, lds, d.opd, d.geod, d.ph, U,            \
                                                     (const float*)nullptr, (const double*)d.UF64,                \
                                                     (const double*)d.Q64, (const double*)d.QF64, P.R[w.desc],    \
                                                     (float*)nullptr, DevSync());                                 \
      __syncthreads();                                                                                            \
    }                                                                                                             \
  } break;
      FR_BATCH_CASES(RCASE)
#undef RCASE
      default: break;
    }
  }
}

// PH: 0 traces, 1 gradients (FP32, the assembly's inputs), 2 block assembly
template <int SYS, int PH>
__global__ void __launch_bounds__(kBT) k_batch_jac(const BDesc* D, BPtrs P, const BItem* items, int nitems) {
  __shared__ __align__(16) char lds[jac_lds_all<SYS>()];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const BItem w = items[it];
    const BDesc& d = D[w.desc];
    switch (d.code) {
#define JKCASE(ET, DEG)                                                                                           \
  case bcode(ET, DEG): {                                                                                          \
    typedef Elem<ET, DEG> E;                                                                                      \
    const float* U = P.U[w.desc];                                                                                 \
    for (int t = w.first; t < w.first + w.count; ++t) {                                                           \
      if constexpr (PH == 0)                                                                                      \
        trace_body<E, kNV, float, float, float>(t, threadIdx.x, kBT, lds, d.opr, d.ne, U, (const float*)nullptr,  \
                                                d.UFr, DevSync());                                                \
      else if constexpr (PH == 1)                                                                                 \
        grad_body<E, kNV, float, float, float>(t, threadIdx.x, kBT, lds, d.opr, d.geor, d.ph.beta, U,             \
                                               (const float*)nullptr, (const float*)d.UFr, d.Qr, d.QFr,           \
                                               DevSync());                                                        \
      else if constexpr (ET == ET_TRI)                                                                            \
        jac_body<E, kNV, SYS, float, float>(t, threadIdx.x, kBT, lds, d.opr, d.geor, d.ph, U, d.Qr, d.UFr,       \
                                            d.QFr, P.B[w.desc], d.nblk, DevSync());                               \
      else                                                                                                        \
        jac_tp_body<E, kNV, SYS, float, float>(t, threadIdx.x, kBT, lds, d.opr, d.o1, d.geor, d.ph, U, d.Qr,     \
                                               d.UFr, d.QFr, P.B[w.desc], d.nblk, DevSync());                     \
      __syncthreads();                                                                                            \
    }                                                                                                             \
  } break;
      FR_BATCH_CASES(JKCASE)
#undef JKCASE
      default: break;
    }
  }
}

}  // namespace

struct fr_batch_s {
  std::vector<fr_ctx_s*> ctx;
  int sys = 0, ncu = 1;
  hipStream_t stream = nullptr;
  BDesc* ddesc = nullptr;          // device
  BDesc* hdesc = nullptr;          // pinned
  BItem* dres = nullptr;           // device work lists
  BItem* djac = nullptr;
  BItem* dtil = nullptr;           // tiles of the Jacobian prelude
  int nres = 0, njac = 0, ntil = 0;
  size_t cap_res = 0, cap_jac = 0, cap_til = 0;
  int k_res[32], k_jac[32];        // work-item granularity per (type, degree)
  int grid_res = 0, grid_jac = 0;  // persistent workgroups per launch
  hipEvent_t t0 = nullptr, t1 = nullptr;
  BPtrs ptrs{};
  std::string err;
};

static fr_status bfail(fr_batch_s* b, fr_status s, const std::string& m) {
  if (b) b->err = m;
  return s;
}

static int sec_cost(const fr_ctx_s* c) { return c->ns * (c->ns + c->nf); }

// work list: `count` units (tiles or elements) of `per` each, longest first
static void make_items(fr_batch_s* b, bool tiles, const int* k, std::vector<BItem>& out) {
  out.clear();
  std::vector<std::pair<long, BItem>> v;
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    const fr_ctx_s* c = b->ctx[i];
    const int code = bcode(c->type, c->p);
    const int te = tiles ? tile_rt(code) : 1;
    const int units = (int)((c->ne + te - 1) / te);
    const int per = std::max(1, k[code]);
    for (int u = 0; u < units; u += per) {
      BItem it{(int)i, u, std::min(per, units - u), 0};
      v.push_back({(long)it.count * te * sec_cost(c), it});
    }
  }
  std::stable_sort(v.begin(), v.end(), [](const auto& a, const auto& c) { return a.first > c.first; });
  for (auto& x : v) out.push_back(x.second);
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
  *n = (int)v.size();
  return FR_OK;
}

static fr_status rebuild(fr_batch_s* b) {
  // launches already queued may still read the current lists
  if (hipStreamSynchronize(b->stream) != hipSuccess) return bfail(b, FR_E_DEVICE, "batch stream");
  std::vector<BItem> v;
  fr_status st;
  make_items(b, true, b->k_res, v);
  if ((st = upload_items(b, v, &b->dres, &b->cap_res, &b->nres))) return st;
  int one[32];
  std::fill(one, one + 32, 1);
  make_items(b, true, one, v);
  if ((st = upload_items(b, v, &b->dtil, &b->cap_til, &b->ntil))) return st;
  make_items(b, false, b->k_jac, v);
  return upload_items(b, v, &b->djac, &b->cap_jac, &b->njac);
}

template <int SYS>
static fr_status launch_res(fr_batch_s* b, bool visc) {
  const dim3 g(std::max(1, std::min(b->grid_res, b->nres))), t(kBT);
  hipLaunchKernelGGL((k_batch_res<SYS, 0>), g, t, 0, b->stream, b->ddesc, b->ptrs, b->dres, b->nres);
  if (visc) hipLaunchKernelGGL((k_batch_res<SYS, 1>), g, t, 0, b->stream, b->ddesc, b->ptrs, b->dres, b->nres);
  hipLaunchKernelGGL((k_batch_res<SYS, 2>), g, t, 0, b->stream, b->ddesc, b->ptrs, b->dres, b->nres);
  return hipGetLastError() == hipSuccess ? FR_OK : bfail(b, FR_E_DEVICE, "batch residual launch");
}
template <int SYS>
static fr_status launch_jac(fr_batch_s* b, bool visc) {
  const dim3 gt(std::max(1, std::min(b->grid_res, b->ntil))), t(kBT);
  hipLaunchKernelGGL((k_batch_jac<SYS, 0>), gt, t, 0, b->stream, b->ddesc, b->ptrs, b->dtil, b->ntil);
  if (visc) hipLaunchKernelGGL((k_batch_jac<SYS, 1>), gt, t, 0, b->stream, b->ddesc, b->ptrs, b->dtil, b->ntil);
  const dim3 gj(std::max(1, std::min(b->grid_jac, b->njac)));
  hipLaunchKernelGGL((k_batch_jac<SYS, 2>), gj, t, 0, b->stream, b->ddesc, b->ptrs, b->djac, b->njac);
  return hipGetLastError() == hipSuccess ? FR_OK : bfail(b, FR_E_DEVICE, "batch Jacobian launch");
}

static fr_status set_ptrs(fr_batch_s* b, const void* const* U, void* const* R, void* const* B) {
  BPtrs p{};
  for (size_t i = 0; i < b->ctx.size(); ++i) {
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
    else if (c->nd != 2 || (c->type != ET_QUAD && c->type != ET_TRI)) why = "batched meshes must be 2-D triangles or quadrilaterals";
    else if (c->system != SYS_EULER && c->system != SYS_NS) why = "batched meshes must be Euler or Navier-Stokes";
    else if (i > 0 && c->system != ctxs[0]->system) why = "batched meshes must share one system";
    else if (c->p < 1 || c->p > 4) why = "batched meshes must have degree 1..4";
    if (why) {
      c->err = std::string(why) + " (mesh " + std::to_string(i) + ")";
      delete b;
      return FR_E_UNSUPPORTED;
    }
    b->ctx.push_back(c);
  }
  b->sys = ctxs[0]->system;
  b->stream = ctxs[0]->stream;
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
  auto tune_one = [&](int* grid, int* k, fr_status (*fn)(fr_batch_s*), const std::vector<int>& grids,
                      const std::vector<int>& ks) -> fr_status {
    double best = 1e30;
    int bg = *grid;
    for (int gm : grids) {
      *grid = gm * b->ncu;
      double t = time_ms(b, fn, reps);
      if (t < best) { best = t; bg = *grid; }
    }
    *grid = bg;
    std::vector<int> codes;
    for (auto* c : b->ctx) codes.push_back(bcode(c->type, c->p));
    std::sort(codes.begin(), codes.end());
    codes.erase(std::unique(codes.begin(), codes.end()), codes.end());
    for (int code : codes) {
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
  if ((st = tune_one(&b->grid_res, b->k_res, run_rhs, {1, 2, 4, 8}, {1, 2, 4, 8}))) return st;
  if ((st = tune_one(&b->grid_jac, b->k_jac, run_jac, {1, 2, 4}, {1, 2, 4}))) return st;
  return hipStreamSynchronize(b->stream) == hipSuccess ? FR_OK : bfail(b, FR_E_DEVICE, "batch tuning");
}

fr_status fr_batch_tuning(const fr_batch* b, int* grid_res, int* grid_jac, int* k_res, int* k_jac) {
  if (!b) return FR_E_INVALID;
  if (grid_res) *grid_res = b->grid_res;
  if (grid_jac) *grid_jac = b->grid_jac;
  if (k_res) std::copy(b->k_res, b->k_res + 32, k_res);
  if (k_jac) std::copy(b->k_jac, b->k_jac + 32, k_jac);
  return FR_OK;
}

}  // extern "C"
