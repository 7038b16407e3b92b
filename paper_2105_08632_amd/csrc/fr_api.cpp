// C ABI of libfr.so (declared in include/fr.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <map>
#include <string>
#include <vector>

#include "fr.h"
#include "fr_ctx.hpp"
#include "fr_host.hpp"

// ------------------------------------------------------------ registry
#define FR_DECL(et, p) void fr_reg_##et##_##p(KernelSet*);
FR_DECL(quad, 1) FR_DECL(quad, 2) FR_DECL(quad, 3) FR_DECL(quad, 4)
FR_DECL(hex, 1) FR_DECL(hex, 2) FR_DECL(hex, 3) FR_DECL(hex, 4)
FR_DECL(tri, 1) FR_DECL(tri, 2) FR_DECL(tri, 3) FR_DECL(tri, 4)
FR_DECL(tet, 1) FR_DECL(tet, 2) FR_DECL(tet, 3) FR_DECL(tet, 4)
FR_DECL(pri, 1) FR_DECL(pri, 2) FR_DECL(pri, 3) FR_DECL(pri, 4)

static KernelSet g_table[5][5][6];
static std::once_flag g_once;

static void fill_table() {
  fr_reg_quad_1(g_table[ET_QUAD][1]); fr_reg_quad_2(g_table[ET_QUAD][2]);
  fr_reg_quad_3(g_table[ET_QUAD][3]); fr_reg_quad_4(g_table[ET_QUAD][4]);
  fr_reg_hex_1(g_table[ET_HEX][1]); fr_reg_hex_2(g_table[ET_HEX][2]);
  fr_reg_hex_3(g_table[ET_HEX][3]); fr_reg_hex_4(g_table[ET_HEX][4]);
  fr_reg_tri_1(g_table[ET_TRI][1]); fr_reg_tri_2(g_table[ET_TRI][2]);
  fr_reg_tri_3(g_table[ET_TRI][3]); fr_reg_tri_4(g_table[ET_TRI][4]);
  fr_reg_tet_1(g_table[ET_TET][1]); fr_reg_tet_2(g_table[ET_TET][2]);
  fr_reg_tet_3(g_table[ET_TET][3]); fr_reg_tet_4(g_table[ET_TET][4]);
  fr_reg_pri_1(g_table[ET_PRI][1]); fr_reg_pri_2(g_table[ET_PRI][2]);
  fr_reg_pri_3(g_table[ET_PRI][3]); fr_reg_pri_4(g_table[ET_PRI][4]);
}

bool fr_find_kernels(int type, int p, int system, int prec, KernelSet* out) {
  std::call_once(g_once, fill_table);
  if (type < 0 || type > 4 || p < 1 || p > 4 || system < 0 || system > 2 || prec < 0 || prec > 1) return false;
  *out = g_table[type][p][system * 2 + prec];
  return out->rhs != nullptr;
}

static thread_local std::string g_create_err;

// ------------------------------------------------------------ allocation-free residual
// fr_rhs_noalloc keeps the FP64 traces and gradients of the residual in this
// file-scope array instead of the context's workspaces.  Every device holds
// its own copy until the process ends.  In host code `scratch` names a host
// stand-in: kernels receive the device address from hipGetSymbolAddress,
// looked up once per device when the first context is created on it.
static constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];
static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};
static hipError_t g_scratch_rc[kMaxDevices] = {};

// Called with the context's device current.
static void scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev] || g_scratch_rc[dev] != hipSuccess) return;
  void* ptr = nullptr;
  hipError_t rc = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (rc == hipSuccess && ptr) g_scratch_ptr[dev] = ptr;
  else g_scratch_rc[dev] = rc != hipSuccess ? rc : hipErrorInvalidSymbol;
}

static void* scratch_ptr(int dev, hipError_t* rc) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (dev < 0 || dev >= kMaxDevices) { *rc = hipErrorInvalidDevice; return nullptr; }
  *rc = g_scratch_rc[dev];
  return g_scratch_ptr[dev];
}

// ------------------------------------------------------------ helpers
template <class R>
static void pack_ops(const frh::RefOps& ref, std::vector<char>& blob, std::vector<size_t>& offs) {
  auto put = [&](const void* src, size_t bytes) {
    size_t o = (blob.size() + 255) & ~(size_t)255;
    blob.resize(o + bytes);
    std::memcpy(blob.data() + o, src, bytes);
    offs.push_back(o);
  };
  auto putR = [&](const std::vector<double>& v) {
    std::vector<R> t(v.begin(), v.end());
    put(t.data(), t.size() * sizeof(R));
  };
  auto putI = [&](const std::vector<int>& v) { put(v.data(), v.size() * sizeof(int)); };
  putR(ref.M0); putR(ref.D); putR(ref.Cor); putR(ref.nref); putI(ref.fface);
  putI(ref.m0c); putR(ref.m0v); putI(ref.dcc); putR(ref.dcv); putI(ref.gc); putR(ref.gv);
  putI(ref.crc); putR(ref.crv); putI(ref.ddc); putR(ref.ddv);
  putR(ref.sdI); putR(ref.sdD); putI(ref.sdend);
}

template <class R> static OpsD<R> ops_view(char* base, const std::vector<size_t>& o) {
  OpsD<R> v;
  v.M0 = (const R*)(base + o[0]); v.D = (const R*)(base + o[1]); v.Cor = (const R*)(base + o[2]);
  v.nref = (const R*)(base + o[3]); v.fface = (const int*)(base + o[4]);
  v.m0c = (const int*)(base + o[5]); v.m0v = (const R*)(base + o[6]);
  v.dcc = (const int*)(base + o[7]); v.dcv = (const R*)(base + o[8]);
  v.gc = (const int*)(base + o[9]); v.gv = (const R*)(base + o[10]);
  v.crc = (const int*)(base + o[11]); v.crv = (const R*)(base + o[12]);
  v.ddc = (const int*)(base + o[13]); v.ddv = (const R*)(base + o[14]);
  v.sdI = (const R*)(base + o[15]); v.sdD = (const R*)(base + o[16]); v.sdend = (const int*)(base + o[17]);
  return v;
}

template <class R>
static void pack_geo(const frh::Geometry& g, std::vector<char>& blob, std::vector<size_t>& offs) {
  auto put = [&](const void* src, size_t bytes) {
    size_t o = (blob.size() + 255) & ~(size_t)255;
    blob.resize(o + bytes);
    std::memcpy(blob.data() + o, src, bytes);
    offs.push_back(o);
  };
  auto putR = [&](const std::vector<double>& v) {
    std::vector<R> t(v.begin(), v.end());
    put(t.data(), t.size() * sizeof(R));
  };
  putR(g.S); putR(g.Jinv); putR(g.rdet); putR(g.nrm); putR(g.magN);
  put(g.nbfp.data(), g.nbfp.size() * sizeof(int));
  put(g.nbr.data(), g.nbr.size() * sizeof(int));
  put(g.nbface.data(), g.nbface.size() * sizeof(int));
  put(g.back.data(), g.back.size() * sizeof(int));
  putR(g.Sint);
}

template <class R> static GeoD<R> geo_view(char* base, const std::vector<size_t>& o, int ne) {
  GeoD<R> v{};
  v.ne = ne;
  v.S = (const R*)(base + o[0]); v.Jinv = (const R*)(base + o[1]); v.rdet = (const R*)(base + o[2]);
  v.nrm = (const R*)(base + o[3]); v.magN = (const R*)(base + o[4]);
  v.nbfp = (const int*)(base + o[5]); v.nbr = (const int*)(base + o[6]);
  v.nbface = (const int*)(base + o[7]); v.back = (const int*)(base + o[8]);
  v.Sint = (const R*)(base + o[9]);
  return v;
}

template <class R> static const OpsD<R>& ctx_ops_c(const fr_ctx_s* c);
template <> const OpsD<double>& ctx_ops_c<double>(const fr_ctx_s* c) { return c->opsd; }
template <> const OpsD<float>& ctx_ops_c<float>(const fr_ctx_s* c) { return c->opsf; }

static fr_status fail(fr_ctx_s* c, fr_status s, const std::string& m) {
  if (c) c->err = m; else g_create_err = m;
  return s;
}

static void release(fr_ctx_s* c) {
  if (!c) return;
  for (fr_ctx_s* s : c->grp) release(s);
  if (c->mix_mem) (void)hipFree(c->mix_mem);
  if (c->mixd_host) {
    if (c->prec == FR_F64) delete (MixD<double>*)c->mixd_host;
    else delete (MixD<float>*)c->mixd_host;
  }
  if (c->ops_mem) (void)hipFree(c->ops_mem);
  if (c->geo_mem) (void)hipFree(c->geo_mem);
  if (c->work_mem) (void)hipFree(c->work_mem);
  if (c->mf_mem) (void)hipFree(c->mf_mem);
  for (int w = 0; w < 2; ++w)
    for (int k = 0; k < fr_ctx_s::kEvPool; ++k)
      for (int j = 0; j < 2; ++j)
        if (c->ev[w][k][j]) (void)hipEventDestroy(c->ev[w][k][j]);
  delete c;
}

static void drain(fr_ctx_s* c, int w) {
  if (c->ev_n[w] == 0) return;
  (void)hipEventSynchronize(c->ev[w][c->ev_n[w] - 1][1]);
  for (int k = 0; k < c->ev_n[w]; ++k) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev[w][k][0], c->ev[w][k][1]) == hipSuccess) c->ev_ms[w] += ms;
  }
  c->ev_count[w] += c->ev_n[w];
  c->ev_n[w] = 0;
}

void fr_time_begin(fr_ctx_s* c, int w) {
  if (c->ev_n[w] == fr_ctx_s::kEvPool) drain(c, w);
  (void)hipEventRecord(c->ev[w][c->ev_n[w]][0], c->stream);
}
void fr_time_end(fr_ctx_s* c, int w) {
  (void)hipEventRecord(c->ev[w][c->ev_n[w]][1], c->stream);
  ++c->ev_n[w];
}

int fr_status_reset(fr_ctx_s* c) {
  static const int clear[2] = {0, 0x7fffffff};
  return hipMemcpy(c->status, clear, sizeof(clear), hipMemcpyHostToDevice) == hipSuccess ? 0 : -4;
}

// Uploads one context's (or element group's) FP64 operators and geometry,
// and FP32 copies for FP32 contexts; fills the views and the 1-D factors of
// tensor elements.  On failure the caller releases the context.
static fr_status upload_ops_geo(fr_ctx_s* c, const frh::RefOps& ref, const frh::Geometry& geo, fr_precision prec,
                                double beta) {
  std::vector<char> ob, gb;
  std::vector<size_t> oo, go;
  // FP64 operators and geometry always (residual); FP32 copies for FP32 contexts
  pack_ops<double>(ref, ob, oo); pack_geo<double>(geo, gb, go);
  std::vector<size_t> oo32, go32;
  if (prec == FR_F32) {
    std::vector<char> o2, g2;
    pack_ops<float>(ref, o2, oo32); pack_geo<float>(geo, g2, go32);
    size_t obase = (ob.size() + 255) & ~(size_t)255, gbase = (gb.size() + 255) & ~(size_t)255;
    ob.resize(obase + o2.size()); std::memcpy(ob.data() + obase, o2.data(), o2.size());
    gb.resize(gbase + g2.size()); std::memcpy(gb.data() + gbase, g2.data(), g2.size());
    for (auto& v : oo32) v += obase;
    for (auto& v : go32) v += gbase;
  }

  if (hipMalloc(&c->ops_mem, ob.size()) != hipSuccess || hipMalloc(&c->geo_mem, gb.size()) != hipSuccess) {
    return fail(nullptr, FR_E_NOMEM, "device allocation failed (operators/geometry)");
  }
  if (hipMemcpy(c->ops_mem, ob.data(), ob.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->geo_mem, gb.data(), gb.size(), hipMemcpyHostToDevice) != hipSuccess) {
    return fail(nullptr, FR_E_DEVICE, "upload failed");
  }
  if (ref.type == FR_QUAD || ref.type == FR_HEX) {
    for (int i = 0; i <= ref.p; ++i) {
      for (int j = 0; j <= ref.p; ++j) {
        double d = ref.D1[i * (ref.p + 1) + j];
        double cm = ref.hp[i] * ref.lp[j] - ref.hm[i] * ref.lm[j];
        c->o1d.Dc1[i][j] = d - cm;
        c->o1d.G1[i][j] = d - (0.5 + beta) * cm;
        c->o1f.Dc1[i][j] = (float)(d - cm);
        c->o1f.G1[i][j] = (float)(d - (0.5 + beta) * cm);
      }
      c->o1d.hp[i] = ref.hp[i]; c->o1d.hm[i] = ref.hm[i]; c->o1d.lp[i] = ref.lp[i]; c->o1d.lm[i] = ref.lm[i];
      c->o1f.hp[i] = (float)ref.hp[i]; c->o1f.hm[i] = (float)ref.hm[i];
      c->o1f.lp[i] = (float)ref.lp[i]; c->o1f.lm[i] = (float)ref.lm[i];
    }
  }
  c->opsd = ops_view<double>((char*)c->ops_mem, oo);
  c->geod = geo_view<double>((char*)c->geo_mem, go, (int)c->ne);
  if (prec == FR_F32) {
    c->opsf = ops_view<float>((char*)c->ops_mem, oo32);
    c->geof = geo_view<float>((char*)c->geo_mem, go32, (int)c->ne);
  }
  return FR_OK;
}

// Workspaces: traces / gradients for the Jacobian assembly (context
// precision), their FP64 dual versions for the JVP and FP64 ones for the
// residual (both evaluated in FP64 whatever the context precision), sized by
// the mesh's flux and solution points; and the status word.  On failure the
// caller releases the context.
static fr_status alloc_work(fr_ctx_s* c) {
  const size_t nv = (size_t)c->nv, rs = (c->prec == FR_F64) ? 8 : 4;
  const bool visc = c->visc, f32 = c->prec == FR_F32;
  const size_t nuf = (size_t)c->nf_tot * nv, nq = (size_t)c->ns_tot * c->nd * nv, nqf = (size_t)c->nf_tot * c->nd * nv;
  size_t sizes[10] = {nuf * rs, visc ? nq * rs : 0, visc ? nqf * rs : 0,
                      2 * nuf * 8, visc ? 2 * nq * 8 : 0, visc ? 2 * nqf * 8 : 0,
                      f32 ? nuf * 8 : 0, (f32 && visc) ? nq * 8 : 0, (f32 && visc) ? nqf * 8 : 0,
                      2 * sizeof(int)};
  size_t off[10], tot = 0;
  for (int i = 0; i < 10; ++i) { off[i] = tot; tot += (sizes[i] + 255) & ~(size_t)255; }
  if (hipMalloc(&c->work_mem, tot) != hipSuccess) return fail(nullptr, FR_E_NOMEM, "device allocation failed (workspaces)");
  char* w = (char*)c->work_mem;
  c->UF = w + off[0]; c->Q = w + off[1]; c->QF = w + off[2];
  c->UFd = w + off[3]; c->Qd = w + off[4]; c->QFd = w + off[5];
  if (f32) { c->UF64 = w + off[6]; c->Q64 = w + off[7]; c->QF64 = w + off[8]; }
  else { c->UF64 = c->UF; c->Q64 = c->Q; c->QF64 = c->QF; }
  c->status = (int*)(w + off[9]);
  c->geod.status = c->status;
  c->geof.status = c->status;
  (void)hipGetDevice(&c->dev);
  scratch_setup(c->dev);
  if (fr_status_reset(c) != 0) return fail(nullptr, FR_E_DEVICE, "status word initialisation failed");
  return FR_OK;
}

// ------------------------------------------------------------ mixed meshes
// A 2-D mesh of triangles and quadrilaterals (of one degree) listed grouped
// by type is one context with a sub-context per group.  The groups share the
// context's trace and gradient workspaces, in a flux-point numbering that
// runs over the groups in order; each group's kernels see their slice, and
// reach the traces of a neighbour in the other group through partner indices
// relative to the slice (build_geometry_groups).  Each residual pass runs over
// every group before the next pass starts.

// Residual (dual = 0) or residual and tangent (dual = 1) of a mixed mesh on
// the given FP64 workspaces.
static int mixed_eval(fr_ctx_s* c, int dual, const void* U, const void* V, void* Rout, void* Rtan, void* UF, void* Q,
                      void* QF) {
  const size_t io = c->prec == FR_F64 ? 8 : 4, ts = dual ? 16 : 8;
  const size_t nv = (size_t)c->nv, nd = (size_t)c->nd;
  for (int pass = 0; pass < 3; ++pass)
    for (size_t g = 0; g < c->grp.size(); ++g) {
      fr_ctx_s* s = c->grp[g];
      const size_t du = (size_t)c->grp_dof0[g] * io;
      const size_t fo = (size_t)c->grp_fp0[g] * nv * ts, so = (size_t)c->grp_sp0[g] * nd * nv * ts;
      int rc = s->ks.phase(s, pass, dual, (const char*)U + du, V ? (const char*)V + du : nullptr, (char*)UF + fo,
                           Q ? (char*)Q + so : nullptr, QF ? (char*)QF + fo * nd : nullptr,
                           Rout ? (char*)Rout + du : nullptr, Rtan ? (char*)Rtan + du : nullptr);
      if (rc) { c->err = s->err; return rc; }
    }
  return 0;
}
static int mixed_rhs(fr_ctx_s* c, const void* U, void* R) {
  return mixed_eval(c, 0, U, nullptr, R, nullptr, c->UF64, c->Q64, c->QF64);
}
static int mixed_rhs_ws(fr_ctx_s* c, const void* U, void* R, void* UF, void* Q, void* QF) {
  return mixed_eval(c, 0, U, nullptr, R, nullptr, UF, Q, QF);
}
static int mixed_jvp(fr_ctx_s* c, const void* U, const void* V, void* Jv, void* Rv) {
  return mixed_eval(c, 1, U, V, Rv, Jv, c->UFd, c->Qd, c->QFd);
}
// Blocks of every element: traces of all groups, then the blocks (the face
// blocks read the traces of the neighbours in either group).
static int mixed_jac(fr_ctx_s* c, const void* U, void* B, int out_prec, int nblk) {
  (void)nblk;
  if (c->visc) { c->err = "Jacobian blocks of mixed meshes: inviscid systems only"; return FR_E_UNSUPPORTED; }
  const size_t io = c->prec == FR_F64 ? 8 : 4;
  for (int stage = 0; stage < 2; ++stage)
    for (size_t g = 0; g < c->grp.size(); ++g) {
      fr_ctx_s* s = c->grp[g];
      if (!s->ks.jac_mixed) { c->err = "no mixed-mesh Jacobian kernels for this element type"; return FR_E_UNSUPPORTED; }
      int rc = s->ks.jac_mixed(s, stage, (const char*)U + (size_t)c->grp_dof0[g] * io, B, out_prec, s->mixd);
      if (rc) { c->err = s->err; return rc; }
    }
  return 0;
}

template <class R> static void set_mixd(fr_ctx_s* s, const fr_ctx_s* other, const int* nbpt, const int* nbt,
                                        const long* fboff) {
  MixD<R>* h = new MixD<R>();
  h->nbpt = nbpt; h->nbt = nbt; h->fboff = fboff; h->M0o = ctx_ops_c<R>(other).M0;
  s->mixd_host = h;
  s->mixd = h;
}

static fr_status create_mixed(const fr_mesh_desc* m, const fr_physics* ph, fr_precision prec, void* stream, int nv,
                              bool visc, fr_ctx** out) {
  const int64_t ne = m->n_elem;
  if (m->ndim != 2) return fail(nullptr, FR_E_UNSUPPORTED, "mixed meshes: 2-D triangles and quadrilaterals only");
  if (ph->scheme != FR_SCHEME_FR_DG) return fail(nullptr, FR_E_UNSUPPORTED, "mixed meshes: FR-DG only");
  std::vector<int64_t> gs = {0};
  for (int64_t e = 1; e < ne; ++e)
    if (m->elem_type[e] != m->elem_type[e - 1]) gs.push_back(e);
  gs.push_back(ne);
  const int ngrp = (int)gs.size() - 1;
  for (int g = 0; g < ngrp; ++g) {
    const int t = m->elem_type[gs[g]];
    if (t != FR_TRI && t != FR_QUAD) return fail(nullptr, FR_E_UNSUPPORTED, "mixed meshes: 2-D triangles and quadrilaterals only");
  }
  if (ngrp != 2) return fail(nullptr, FR_E_INVALID, "mixed meshes must list their elements grouped by type");
  frh::RefOps refs[3];
  std::string err;
  for (int g = 0; g < ngrp; ++g) {
    const int t = m->elem_type[gs[g]];
    if (!frh::build_ref(t, m->degree, ph->ldg_beta, ph->scheme, m->tri_sol_pts, m->tet_sol_pts, refs[t], err))
      return fail(nullptr, FR_E_INVALID, err);
    if (m->max_vert < refs[t].nvert || m->max_face < refs[t].nface)
      return fail(nullptr, FR_E_INVALID, "max_vert/max_face too small");
  }
  const frh::RefOps* rp[3] = {&refs[0], &refs[1], &refs[2]};
  frh::Geometry geo[2];
  frh::MixInfo mix[2];
  if (!frh::build_geometry_groups(rp, 2, ne, m->elem_type, m->elem_xyz, m->max_vert, m->nbr, m->nbr_face, m->max_face,
                                  ngrp, gs.data(), geo, mix, err))
    return fail(nullptr, FR_E_INVALID, err);

  fr_ctx_s* c = new fr_ctx_s();
  c->mixed = true;
  c->nd = 2; c->type = -1; c->p = m->degree; c->system = ph->system; c->nv = nv; c->prec = prec; c->ne = ne;
  c->visc = visc;
  for (int i = 0; i < 3; ++i) c->ph.c[i] = ph->adv_vel[i];
  c->ph.gamma = ph->gamma; c->ph.mu = ph->mu; c->ph.prandtl = ph->prandtl;
  c->ph.beta = ph->ldg_beta; c->ph.eta = ph->ldg_penalty;
  c->stream = (hipStream_t)stream;
  c->scheme = ph->scheme;
  // block sizes and Jacobian-block offsets: per element its self block, then
  // one block per local face (b_n x b_m, m the neighbour), packed
  std::vector<int> bsz((size_t)ne);
  for (int64_t e = 0; e < ne; ++e) bsz[e] = refs[m->elem_type[e]].ns * nv;
  c->blk_off.assign((size_t)ne + 1, 0);
  for (int64_t e = 0; e < ne; ++e) {
    const frh::RefOps& R = refs[m->elem_type[e]];
    int64_t n = (int64_t)bsz[e] * bsz[e];
    for (int f = 0; f < R.nface; ++f) n += (int64_t)bsz[e] * bsz[m->nbr[e * m->max_face + f]];
    c->blk_off[e + 1] = c->blk_off[e] + n;
  }
  int64_t dof = 0, fp = 0, sp = 0;
  for (int g = 0; g < ngrp; ++g) {
    const frh::RefOps& R = refs[m->elem_type[gs[g]]];
    const int64_t ng = gs[g + 1] - gs[g];
    c->grp_e0.push_back(gs[g]); c->grp_dof0.push_back(dof); c->grp_fp0.push_back(fp); c->grp_sp0.push_back(sp);
    dof += ng * R.ns * nv; fp += ng * R.nf; sp += ng * R.ns;
    c->ns = std::max(c->ns, R.ns); c->nf = std::max(c->nf, R.nf); c->nface = std::max(c->nface, R.nface);
    c->nfp = R.nfp; c->b = std::max(c->b, R.ns * nv);
  }
  c->ndof = dof; c->nf_tot = fp; c->ns_tot = sp;
  c->ks = KernelSet{};
  c->ks.rhs = &mixed_rhs; c->ks.rhs_ws = &mixed_rhs_ws; c->ks.jvp = &mixed_jvp; c->ks.jac = &mixed_jac;
  if (fr_status ws = alloc_work(c)) { release(c); return ws; }
  for (int g = 0; g < ngrp; ++g) {
    const int t = m->elem_type[gs[g]];
    const frh::RefOps& R = refs[t];
    const int64_t ng = gs[g + 1] - gs[g];
    fr_ctx_s* s = new fr_ctx_s();
    c->grp.push_back(s);
    s->sub = true;
    s->nd = 2; s->type = t; s->p = m->degree; s->system = ph->system; s->nv = nv; s->prec = prec; s->scheme = c->scheme;
    s->ne = ng; s->ns = R.ns; s->nf = R.nf; s->nface = R.nface; s->nfp = R.nfp; s->b = R.ns * nv; s->visc = visc;
    s->ph = c->ph; s->stream = c->stream; s->dev = c->dev; s->status = c->status;
    s->ndof = ng * s->b; s->nf_tot = ng * R.nf; s->ns_tot = ng * R.ns;
    if (!fr_find_kernels(t, m->degree, ph->system, prec, &s->ks)) {
      release(c);
      return fail(nullptr, FR_E_UNSUPPORTED, "no kernels for this element type / degree / system / precision");
    }
    if (fr_status us = upload_ops_geo(s, R, geo[g], prec, ph->ldg_beta)) { release(c); return us; }
    // the group's slices of the shared workspaces
    const size_t rs = (prec == FR_F64) ? 8 : 4, nvs = (size_t)nv, nds = 2;
    const size_t fo = (size_t)c->grp_fp0[g] * nvs, so = (size_t)c->grp_sp0[g] * nds * nvs;
    s->UF = (char*)c->UF + fo * rs;
    s->Q = c->Q ? (char*)c->Q + so * rs : nullptr;
    s->QF = c->QF ? (char*)c->QF + fo * nds * rs : nullptr;
    s->UF64 = (char*)c->UF64 + fo * 8;
    s->Q64 = c->Q64 ? (char*)c->Q64 + so * 8 : nullptr;
    s->QF64 = c->QF64 ? (char*)c->QF64 + fo * nds * 8 : nullptr;
    s->UFd = (char*)c->UFd + fo * 16;
    s->Qd = c->Qd ? (char*)c->Qd + so * 16 : nullptr;
    s->QFd = c->QFd ? (char*)c->QFd + fo * nds * 16 : nullptr;
    // cross-type data and block offsets on the device
    std::vector<long> boff((size_t)ng), fboff((size_t)ng * R.nface);
    for (int64_t el = 0; el < ng; ++el) {
      const int64_t e = gs[g] + el;
      boff[el] = (long)c->blk_off[e];
      long o = (long)c->blk_off[e] + (long)bsz[e] * bsz[e];
      for (int f = 0; f < R.nface; ++f) {
        fboff[el * R.nface + f] = o;
        o += (long)bsz[e] * bsz[m->nbr[e * m->max_face + f]];
      }
    }
    const size_t b0 = 0, b1 = (b0 + boff.size() * sizeof(long) + 255) & ~(size_t)255;
    const size_t b2 = (b1 + fboff.size() * sizeof(long) + 255) & ~(size_t)255;
    const size_t b3 = (b2 + mix[g].nbpt.size() * sizeof(int) + 255) & ~(size_t)255;
    const size_t bt = b3 + mix[g].nbt.size() * sizeof(int);
    if (hipMalloc(&s->mix_mem, bt) != hipSuccess) { release(c); return fail(nullptr, FR_E_NOMEM, "device allocation failed (mixed mesh)"); }
    char* mm = (char*)s->mix_mem;
    if (hipMemcpy(mm + b0, boff.data(), boff.size() * sizeof(long), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(mm + b1, fboff.data(), fboff.size() * sizeof(long), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(mm + b2, mix[g].nbpt.data(), mix[g].nbpt.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(mm + b3, mix[g].nbt.data(), mix[g].nbt.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
      release(c);
      return fail(nullptr, FR_E_DEVICE, "upload failed (mixed mesh)");
    }
    s->geod.boff = (const long*)(mm + b0); s->geof.boff = (const long*)(mm + b0);
    s->geod.e0 = (long)gs[g]; s->geof.e0 = (long)gs[g];
    s->geod.status = c->status; s->geof.status = c->status;
  }
  for (int g = 0; g < ngrp; ++g) {
    fr_ctx_s* s = c->grp[g];
    char* mm = (char*)s->mix_mem;
    const size_t ng = (size_t)s->ne;
    const size_t b1 = (ng * sizeof(long) + 255) & ~(size_t)255;
    const size_t b2 = (b1 + ng * s->nface * sizeof(long) + 255) & ~(size_t)255;
    const size_t b3 = (b2 + ng * s->nf * sizeof(int) + 255) & ~(size_t)255;
    const fr_ctx_s* o = c->grp[1 - g];
    if (prec == FR_F64) set_mixd<double>(s, o, (const int*)(mm + b2), (const int*)(mm + b3), (const long*)(mm + b1));
    else set_mixd<float>(s, o, (const int*)(mm + b2), (const int*)(mm + b3), (const long*)(mm + b1));
  }
  *out = c;
  return FR_OK;
}

// ------------------------------------------------------------ ABI
extern "C" {

fr_status fr_ctx_create(const fr_mesh_desc* m, const fr_physics* ph, fr_precision prec, void* stream, fr_ctx** out) {
  if (!m || !ph || !out) return fail(nullptr, FR_E_INVALID, "null argument");
  *out = nullptr;
  if (m->ndim != 2 && m->ndim != 3) return fail(nullptr, FR_E_INVALID, "ndim must be 2 or 3");
  if (m->n_elem <= 0 || m->n_elem > (int64_t)1 << 26) return fail(nullptr, FR_E_INVALID, "n_elem out of range");
  if (!m->elem_type || !m->elem_xyz || !m->nbr || !m->nbr_face) return fail(nullptr, FR_E_INVALID, "null mesh array");
  if (m->degree < 1 || m->degree > 4) return fail(nullptr, FR_E_UNSUPPORTED, "degree must be in 1..4");
  if (prec != FR_F64 && prec != FR_F32) return fail(nullptr, FR_E_UNSUPPORTED, "state precision must be FR_F64 or FR_F32");
  const int type = m->elem_type[0];
  bool one_type = true;
  for (int64_t e = 0; e < m->n_elem; ++e) {
    if (m->elem_type[e] < 0 || m->elem_type[e] > 4) return fail(nullptr, FR_E_INVALID, "unknown element type");
    if (m->elem_type[e] != type) one_type = false;
  }
  for (int64_t e = 0; e < m->n_elem; ++e)
    if ((m->elem_type[e] == FR_QUAD || m->elem_type[e] == FR_TRI) != (m->ndim == 2))
      return fail(nullptr, FR_E_INVALID, "element type does not match ndim");
  if (ph->system < 0 || ph->system > 2) return fail(nullptr, FR_E_INVALID, "unknown system");
  const int nv = (ph->system == FR_ADVECTION) ? 1 : m->ndim + 2;
  if (ph->nvars != nv) return fail(nullptr, FR_E_INVALID, "nvars does not match the system");
  if (ph->system != FR_ADVECTION && !(ph->gamma > 1.0)) return fail(nullptr, FR_E_INVALID, "gamma must exceed 1");
  if (ph->system == FR_NAVIER_STOKES && !(ph->prandtl > 0.0)) return fail(nullptr, FR_E_INVALID, "prandtl must be positive");
  if (ph->ldg_beta != 0.0 || ph->ldg_penalty != 0.0)
    return fail(nullptr, FR_E_UNSUPPORTED, "only the BR1 scheme is provided: ldg_beta and ldg_penalty must be 0");
  if (ph->scheme < FR_SCHEME_FR_DG || ph->scheme > FR_SCHEME_SDRT)
    return fail(nullptr, FR_E_INVALID, "unknown scheme");
  if (ph->scheme != FR_SCHEME_FR_DG && type != FR_QUAD && type != FR_HEX)
    return fail(nullptr, FR_E_UNSUPPORTED, "FR-SDRT and SDRT are provided for quadrilaterals and hexahedra");
  if (!one_type)
    return create_mixed(m, ph, prec, stream, nv,
                        (ph->system == FR_NAVIER_STOKES) || (ph->system == FR_ADVECTION && ph->mu != 0.0), out);

  frh::RefOps ref;
  std::string err;
  if (!frh::build_ref(type, m->degree, ph->ldg_beta, ph->scheme, m->tri_sol_pts, m->tet_sol_pts, ref, err))
    return fail(nullptr, FR_E_INVALID, err);
  if (m->max_vert < ref.nvert || m->max_face < ref.nface) return fail(nullptr, FR_E_INVALID, "max_vert/max_face too small");
  frh::Geometry geo;
  if (!frh::build_geometry(ref, m->ndim, m->n_elem, m->elem_xyz, m->max_vert, m->nbr, m->nbr_face, m->max_face, geo, err))
    return fail(nullptr, FR_E_INVALID, err);
  if (ph->scheme == FR_SCHEME_SDRT)
    frh::build_sd_metric(ref, m->ndim, m->n_elem, m->elem_xyz, m->max_vert, geo.Sint);
  const bool visc = (ph->system == FR_NAVIER_STOKES) || (ph->system == FR_ADVECTION && ph->mu != 0.0);
  if (visc && !frh::check_stencil(m->n_elem, ref.nface, geo.nbr.data(), err)) return fail(nullptr, FR_E_UNSUPPORTED, err);
  if (m->n_elem * ref.nf > ((int64_t)1 << 31) - 1) return fail(nullptr, FR_E_UNSUPPORTED, "mesh too large for 32-bit face indices");

  fr_ctx_s* c = new fr_ctx_s();
  c->nd = m->ndim; c->type = type; c->p = m->degree; c->system = ph->system; c->nv = nv; c->prec = prec;
  c->ne = m->n_elem; c->ns = ref.ns; c->nf = ref.nf; c->nface = ref.nface; c->nfp = ref.nfp; c->b = ref.ns * nv;
  c->visc = visc;
  // face-centroid offsets (vertex averages), used by the Fourier analysis
  c->face_off.assign((size_t)c->ne * ref.nface * m->ndim, 0.0);
  for (int64_t e = 0; e < c->ne; ++e) {
    const double* X = m->elem_xyz + (size_t)e * m->max_vert * m->ndim;
    for (int d = 0; d < m->ndim; ++d) {
      double ctr = 0.0;
      for (int v = 0; v < ref.nvert; ++v) ctr += X[v * m->ndim + d];
      ctr /= ref.nvert;
      for (int f = 0; f < ref.nface; ++f) {
        double fc = 0.0;
        for (int v : ref.face_verts[f]) fc += X[v * m->ndim + d];
        fc /= (double)ref.face_verts[f].size();
        c->face_off[((size_t)e * ref.nface + f) * m->ndim + d] = fc - ctr;
      }
    }
  }
  for (int i = 0; i < 3; ++i) c->ph.c[i] = ph->adv_vel[i];
  c->ph.gamma = ph->gamma; c->ph.mu = ph->mu; c->ph.prandtl = ph->prandtl;
  c->ph.beta = ph->ldg_beta; c->ph.eta = ph->ldg_penalty;
  c->stream = (hipStream_t)stream;
  if (!fr_find_kernels(type, m->degree, ph->system, prec, &c->ks)) {
    release(c);
    return fail(nullptr, FR_E_UNSUPPORTED, "no kernels for this element type / degree / system / precision");
  }
  c->scheme = ph->scheme;
  if (c->scheme == FR_SCHEME_SDRT) {
    // the SDRT residual and tangent replace the FR ones; no Jacobian blocks
    if (!c->ks.rhs_sd || !c->ks.jvp_sd) {
      release(c);
      return fail(nullptr, FR_E_UNSUPPORTED, "no SDRT kernels for this element type");
    }
    c->ks.rhs = c->ks.rhs_sd;
    c->ks.jvp = c->ks.jvp_sd;
    c->ks.rhs_ws = nullptr;
    c->ks.jac = nullptr;
    c->ks.mf_bytes = nullptr;
    c->ks.mf_setup = nullptr;
  }
  c->jv_fused = c->scheme != FR_SCHEME_SDRT;   // the FR divergence pass takes the tangent shift
  if (fr_status us = upload_ops_geo(c, ref, geo, prec, ph->ldg_beta)) {
    release(c);
    return us;
  }
  c->nf_tot = c->ne * c->nf;
  c->ns_tot = c->ne * c->ns;
  c->ndof = c->ne * (int64_t)c->b;
  if (fr_status ws = alloc_work(c)) {
    release(c);
    return ws;
  }
  // matrix-core Jacobian: geometry-only sensitivities (computed here, once)
  // and the per-state tables
  const size_t mfs = c->ks.mf_bytes ? c->ks.mf_bytes(0) : 0, mft = c->ks.mf_bytes ? c->ks.mf_bytes(1) : 0;
  if (mfs) {
    // The reference part of a block's sensitivities (the corrected-gradient
    // rows and the face-value rows) involves no geometry: it depends on the
    // block (self, or the face) and on which neighbour flux point each of
    // the face's flux points pairs with.  Blocks with equal keys share one
    // copy, which the assembly reads instead of the element's own.
    const int nsb = 1 + c->nface, nf = c->nf, nfp = c->nf / c->nface;
    std::map<std::vector<int>, int> ids;
    std::vector<int> sig((size_t)c->ne * nsb);
    std::vector<std::pair<int64_t, int>> reps;     // representative (element, block) of each key
    std::vector<int> key;
    for (int64_t n = 0; n < c->ne; ++n)
      for (int k = 0; k < nsb; ++k) {
        key.assign(1, k);
        if (k > 0)
          for (int j = 0; j < nfp; ++j) key.push_back(geo.nbfp[(size_t)n * nf + (k - 1) * nfp + j] % nf);
        auto it = ids.find(key);
        int id;
        if (it == ids.end()) {
          id = (int)reps.size();
          ids.emplace(key, id);
          reps.emplace_back(n, k);
        } else {
          id = it->second;
        }
        sig[(size_t)n * nsb + k] = id;
      }
    const size_t blk = mfs / nsb;                     // bytes of one block's sensitivities
    const size_t a = ((size_t)c->ne * mfs + 255) & ~(size_t)255;
    const size_t t = ((size_t)c->ne * mft + 255) & ~(size_t)255;
    const size_t st = ((size_t)reps.size() * blk + 255) & ~(size_t)255;
    if (hipMalloc(&c->mf_mem, a + t + st + sig.size() * sizeof(int)) != hipSuccess) {
      release(c);
      return fail(nullptr, FR_E_NOMEM, "device allocation failed (Jacobian workspaces)");
    }
    c->mf_sens = c->mf_mem;
    c->mf_tab = (char*)c->mf_mem + a;
    c->mf_sigtab = (char*)c->mf_mem + a + t;
    c->mf_sig = (int*)((char*)c->mf_mem + a + t + st);
    c->mf_nsig = (int)reps.size();
    if (hipMemcpy(c->mf_sig, sig.data(), sig.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
      release(c);
      return fail(nullptr, FR_E_DEVICE, "upload of the sensitivity keys");
    }
    if (c->ks.mf_setup(c) != 0) {
      std::string e = c->err;
      release(c);
      return fail(nullptr, FR_E_DEVICE, "Jacobian sensitivities: " + e);
    }
    for (size_t i = 0; i < reps.size(); ++i)
      if (hipMemcpyAsync((char*)c->mf_sigtab + i * blk, (char*)c->mf_sens + ((size_t)reps[i].first * nsb + reps[i].second) * blk,
                         blk, hipMemcpyDeviceToDevice, c->stream) != hipSuccess) {
        release(c);
        return fail(nullptr, FR_E_DEVICE, "copy of the shared sensitivities");
      }
    if (hipStreamSynchronize(c->stream) != hipSuccess) {
      release(c);
      return fail(nullptr, FR_E_DEVICE, "Jacobian sensitivities");
    }
  }
  *out = c;
  return FR_OK;
}

fr_status fr_ctx_destroy(fr_ctx* c) {
  if (!c) return FR_E_INVALID;
  (void)hipStreamSynchronize(c->stream);
  release(c);
  return FR_OK;
}

fr_status fr_ctx_info(const fr_ctx* c, fr_info* info) {
  if (!c || !info) return FR_E_INVALID;
  info->ndim = c->nd; info->n_sol = c->ns; info->n_flux = c->nf; info->n_face = c->nface; info->nvars = c->nv;
  info->block_dim = c->b; info->n_elem = c->ne; info->n_dof = c->ndof;
  info->blocks_per_elem = 1 + c->nface; info->precision = c->prec;
  return FR_OK;
}

const char* fr_last_error(const fr_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }

fr_status fr_ctx_sync(fr_ctx* c) {
  if (!c) return FR_E_INVALID;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return fail(c, FR_E_DEVICE, std::string("device: ") + hipGetErrorString(e));
  int st[2] = {0, 0};
  if (hipMemcpy(st, c->status, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(c, FR_E_DEVICE, "reading the status word");
  if (st[0]) {
    std::string what;
    if (st[0] & FR_NF_RHS) what += " R";
    if (st[0] & FR_NF_JVP) what += " Jv";
    if (st[0] & FR_NF_BLOCKS) what += " Jacobian-blocks";
    if (fr_status_reset(c) != 0) return fail(c, FR_E_DEVICE, "clearing the status word");
    return fail(c, FR_E_NONFINITE,
                "non-finite value stored to" + what + "; first element " + std::to_string(st[1]));
  }
  return FR_OK;
}

fr_status fr_set_kernel_timing(fr_ctx* c, int enable) {
  if (!c) return FR_E_INVALID;
  if (enable && !c->ev[0][0][0])
    for (int w = 0; w < 2; ++w)
      for (int k = 0; k < fr_ctx_s::kEvPool; ++k)
        for (int j = 0; j < 2; ++j)
          if (hipEventCreate(&c->ev[w][k][j]) != hipSuccess) return fail(c, FR_E_DEVICE, "hipEventCreate failed");
  c->timing = enable != 0;
  return FR_OK;
}

fr_status fr_kernel_time(fr_ctx* c, int which, double* ms_total, int64_t* count) {
  if (!c || which < 0 || which > 1 || !ms_total || !count) return FR_E_INVALID;
  drain(c, which);
  *ms_total = c->ev_ms[which];
  *count = c->ev_count[which];
  c->ev_ms[which] = 0.0;
  c->ev_count[which] = 0;
  return FR_OK;
}

static bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

fr_status fr_rhs(fr_ctx* c, const void* U, void* R) {
  if (!c) return FR_E_INVALID;
  const size_t a = c->prec == FR_F64 ? 8 : 4;
  if (!U || !R || !aligned(U, a) || !aligned(R, a)) return fail(c, FR_E_INVALID, "fr_rhs: null or misaligned pointer");
  if (U == R) return fail(c, FR_E_INVALID, "fr_rhs: U and R must not alias");
  int rc = c->ks.rhs(c, U, R);
  return rc ? (fr_status)rc : FR_OK;
}

fr_status fr_rhs_noalloc(fr_ctx* c, const void* U, void* R) {
  if (!c) return FR_E_INVALID;
  const size_t a = c->prec == FR_F64 ? 8 : 4;
  if (!U || !R || !aligned(U, a) || !aligned(R, a))
    return fail(c, FR_E_INVALID, "fr_rhs_noalloc: null or misaligned pointer");
  if (U == R) return fail(c, FR_E_INVALID, "fr_rhs_noalloc: U and R must not alias");
  if (!c->ks.rhs_ws) return fail(c, FR_E_UNSUPPORTED, "fr_rhs_noalloc: not provided for SDRT contexts");
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t nuf = (size_t)c->nf_tot * c->nv * 8;
  const size_t nq = c->visc ? (size_t)c->ns_tot * c->nd * c->nv * 8 : 0;
  const size_t nqf = c->visc ? (size_t)c->nf_tot * c->nd * c->nv * 8 : 0;
  const size_t need = up(nuf) + up(nq) + up(nqf);
  if (need > kScratchBytes)
    return fail(c, FR_E_UNSUPPORTED, "fr_rhs_noalloc: this mesh needs " + std::to_string(need) +
                                         " bytes of scratch, more than the " + std::to_string(kScratchBytes) +
                                         " the library holds per device");
  hipError_t rc = hipSuccess;
  char* w = (char*)scratch_ptr(c->dev, &rc);
  if (!w)
    return fail(c, FR_E_DEVICE, std::string("fr_rhs_noalloc: scratch address unavailable: ") + hipGetErrorString(rc));
  int r = c->ks.rhs_ws(c, U, R, w, w + up(nuf), w + up(nuf) + up(nq));
  return r ? (fr_status)r : FR_OK;
}

fr_status fr_jvp(fr_ctx* c, const void* U, const void* v, void* Jv, void* Rout) {
  if (!c) return FR_E_INVALID;
  const size_t a = c->prec == FR_F64 ? 8 : 4;
  if (!U || !v || !Jv || !aligned(U, a) || !aligned(v, a) || !aligned(Jv, a) || (Rout && !aligned(Rout, a)))
    return fail(c, FR_E_INVALID, "fr_jvp: null or misaligned pointer");
  if (Jv == U || Jv == v || (Rout && (Rout == U || Rout == v || Rout == Jv)))
    return fail(c, FR_E_INVALID, "fr_jvp: outputs must not alias inputs");
  int rc = c->ks.jvp(c, U, v, Jv, Rout);
  return rc ? (fr_status)rc : FR_OK;
}

fr_status fr_block_offsets(const fr_ctx* c, int64_t* off) {
  if (!c || !off) return FR_E_INVALID;
  if (c->mixed) {
    std::memcpy(off, c->blk_off.data(), c->blk_off.size() * sizeof(int64_t));
  } else {
    const int64_t per = (int64_t)(1 + c->nface) * c->b * c->b;
    for (int64_t n = 0; n <= c->ne; ++n) off[n] = n * per;
  }
  return FR_OK;
}

fr_status fr_jacobian_blocks(fr_ctx* c, const void* U, void* blocks, fr_precision out_prec) {
  if (!c) return FR_E_INVALID;
  const size_t a = c->prec == FR_F64 ? 8 : 4;
  const size_t ob = out_prec == FR_F64 ? 8 : (out_prec == FR_F32 ? 4 : 2);
  if (!U || !blocks || !aligned(U, a) || !aligned(blocks, ob))
    return fail(c, FR_E_INVALID, "fr_jacobian_blocks: null or misaligned pointer");
  if (out_prec < FR_F64 || out_prec > FR_BF16) return fail(c, FR_E_INVALID, "fr_jacobian_blocks: bad precision");
  if (!c->ks.jac)
    return fail(c, FR_E_UNSUPPORTED, "fr_jacobian_blocks: not provided for SDRT contexts (for linear fluxes on "
                                     "affine elements FR-SDRT gives the same operator)");
  int rc = c->ks.jac(c, U, blocks, (int)out_prec, 1 + c->nface);
  return rc ? (fr_status)rc : FR_OK;
}

}  // extern "C"
