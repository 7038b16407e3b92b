// Device code of the FR-DG residual, its tangent (JVP) and the Jacobian-block
// assembly.  Kernel bodies are written against (tile, thread id, thread
// count, LDS pointer, barrier) so the same body serves every launch shape.
//
// Per element the residual follows the paper's FR formulation:
//   u^f  = M0 u                                   (eq. "interpolate_sol_to_flux")
//   C    = u^f + (1/2 + beta) (u^f_nbr - u^f)      (eq. "common_var_for_grad")
//   q~_d = D_d u + sum_f Cor_f nref_{f,d} (C_f - u^f_f),  q = J^{-T} q~
//   F~_d = sum_k S_dk f_k(u, q),  S = detJ J^{-1}  (eq. "transformed_quantities")
//   div  = sum_d D_d F~_d + sum_f Cor_f (|N_f| F(u_L,u_R,q_L,q_R,n_f) - nref_f.M0 F~)
//                                                  (eq. "divergence_fr")
//   R    = -div / detJ                             (method of lines)
// Cor_f is the divergence of the FR-DG correction function of flux point f.
#pragma once
#include <type_traits>

#include "dual.hpp"
#include "physics.hpp"

enum { ET_QUAD = 0, ET_TRI = 1, ET_HEX = 2, ET_TET = 3, ET_PRI = 4 };
// Tensor-product element types (line operators, matrix-core Jacobian, SDRT).
constexpr bool et_tensor(int et) { return et == ET_QUAD || et == ET_HEX; }

template <int ET, int P> struct Elem;
template <int P> struct Elem<ET_QUAD, P> {
  static constexpr int ET = ET_QUAD, DEG = P, ND = 2, NS = (P + 1) * (P + 1), NFACE = 4, NFP = P + 1,
                       NF = 4 * (P + 1), NVERT = 4;
  static constexpr int WL = P + 1;   // non-zeros per row of a line operator (M0, D_d, Dc_d, G_d)
  static constexpr int WC = 4;       // non-zeros per row of the correction matrix
};
template <int P> struct Elem<ET_HEX, P> {
  static constexpr int ET = ET_HEX, DEG = P, ND = 3, NS = (P + 1) * (P + 1) * (P + 1), NFACE = 6,
                       NFP = (P + 1) * (P + 1), NF = 6 * (P + 1) * (P + 1), NVERT = 8;
  static constexpr int WL = P + 1;
  static constexpr int WC = 6;
};
// Tetrahedra: four triangular faces of (p+1)(p+2)/2 points; dense operator rows.
template <int P> struct Elem<ET_TET, P> {
  static constexpr int ET = ET_TET, DEG = P, ND = 3, NS = (P + 1) * (P + 2) * (P + 3) / 6, NFACE = 4,
                       NFP = (P + 1) * (P + 2) / 2, NF = 4 * NFP, NVERT = 4;
  static constexpr int WL = NS;
  static constexpr int WC = NF;
};
// Prisms: two triangular faces of (p+1)(p+2)/2 points and three
// quadrilateral faces of (p+1)^2 (faces of unequal size: NFP is the largest;
// the residual kernels only use NF); dense operator rows.
template <int P> struct Elem<ET_PRI, P> {
  static constexpr int ET = ET_PRI, DEG = P, ND = 3, NS = (P + 1) * (P + 1) * (P + 2) / 2, NFACE = 5,
                       NFP = (P + 1) * (P + 1), NF = (P + 1) * (P + 2) + 3 * (P + 1) * (P + 1), NVERT = 6;
  static constexpr int WL = NS;
  static constexpr int WC = NF;
};
template <int P> struct Elem<ET_TRI, P> {
  static constexpr int ET = ET_TRI, DEG = P, ND = 2, NS = (P + 1) * (P + 2) / 2, NFACE = 3, NFP = P + 1,
                       NF = 3 * (P + 1), NVERT = 3;
  static constexpr int WL = (P + 1) * (P + 2) / 2;
  static constexpr int WC = 3 * (P + 1);
};

// Reference operators of one (element type, degree), row-major.  The
// compressed rows (col, val) list the non-zeros of each row padded to the
// fixed width of the element (zeros past the end).
template <class R> struct OpsD {
  const R* M0;      // [NF][NS]      l_sigma(x_f)
  const R* D;       // [ND][NS][NS]  d l_sigma/d xi_d (x_rho)
  const R* Cor;     // [NS][NF]      div g_f (x_rho)
  const R* nref;    // [NF][ND]      unit reference normals
  const int* fface; // [NF]          face of each flux point
  const int* m0c; const R* m0v;    // [NF][WL]
  const int* dcc; const R* dcv;    // [ND][NS][WL]  Dc_d = D_d - Cor diag(nref_d) M0
  const int* gc;  const R* gv;     // [ND][NS][WL]  G_d  = D_d - (1/2+beta) Cor diag(nref_d) M0
  const int* ddc; const R* ddv;    // [ND][NS][WL]  D_d
  const int* crc; const R* crv;    // [NS][WC]      Cor rows
  // SDRT (tensor elements): sdI [p][p+1] solution points -> interior SD flux
  // points of a line, sdD [p+1][p+2] flux-point Lagrange derivatives at the
  // solution points, sdend [ND][NL][2] external flux point at each line end
  const R* sdI; const R* sdD; const int* sdend;
};

// Per-element geometry of one group, element-major.
template <class R> struct GeoD {
  int ne;
  const R* S;       // [ne][NS][ND][ND]  detJ J^{-1}
  const R* Jinv;    // [ne][NS][ND][ND]  J^{-1}: (J^{-1})_{d e} = d xi_d / d x_e
  const R* rdet;    // [ne][NS]          1/detJ
  const R* nrm;     // [ne][NF][ND]      unit physical normal (outward)
  const R* magN;    // [ne][NF]          |S^T nref|
  const int* nbfp;  // [ne][NF]          m*NF + g' of the flux point paired with g
  const int* nbr;   // [ne][NFACE]       face neighbours
  const int* nbface;  // [ne][NFACE]     the neighbour's local index of the shared face
  const int* back;    // [ne][NFACE][NFP] this element's point paired with each point of that neighbour face
  int* status;        // [2] non-finite output report (device): [0] kinds, [1] smallest element
  const R* Sint;      // SDRT: [ne][ND][NL][p][ND] row d of detJ J^{-1} at the interior flux points of d-lines
  const long* boff;   // mixed meshes: [ne] first block entry of each element (null: element stride nblk b^2)
  long e0;            // mesh index of the group's first element (reports of non-finite values)
};

// Kinds of output a non-finite value was stored to.
enum { FR_NF_RHS = 1, FR_NF_JVP = 2, FR_NF_BLOCKS = 4 };
template <class R> FR_HD bool fr_finite(R x) { return __builtin_isfinite(x); }
// Records that element `elem` stored a non-finite value of kind `what`.
FR_HD void fr_flag_nonfinite(int* st, int what, long elem) {
  if (!st) return;
#if defined(__HIP_DEVICE_COMPILE__)
  atomicOr(&st[0], what);
  atomicMin(&st[1], (int)elem);
#else
  st[0] |= what;
  if ((int)elem < st[1]) st[1] = (int)elem;
#endif
}

struct DevSync {
  __device__ __forceinline__ void operator()() const { __syncthreads(); }
};

// LDS bump allocator (16-byte aligned slices).
struct Lds {
  char* p;
  template <class X> FR_HD X* take(int n) {
    X* r = reinterpret_cast<X*>(p);
    int bytes = (int)((sizeof(X) * (size_t)n + 15) & ~(size_t)15);
    p += bytes;
    return r;
  }
};
template <class X> constexpr int lds_bytes(int n) { return (int)((sizeof(X) * (size_t)n + 15) & ~(size_t)15); }

// Input element i of U (and of the tangent direction V for dual scalars),
// converted from the I/O type to the compute type.
template <class T, class R, class IO> struct MakeIn {
  static FR_HD T get(const IO* U, const IO*, long i) { return T(R(U[i])); }
};
template <class R, class IO> struct MakeIn<Dual<R>, R, IO> {
  static FR_HD Dual<R> get(const IO* U, const IO* V, long i) { return Dual<R>(R(U[i]), R(V[i])); }
};
template <class T, class R, class IO> FR_HD T make_in(const IO* U, const IO* V, long i) {
  return MakeIn<T, R, IO>::get(U, V, i);
}

template <class E> constexpr int rhs_tile() {
  // tetrahedra and prisms keep dense operator rows in LDS: fewer elements per tile
  if constexpr (E::ET == ET_TET || E::ET == ET_PRI) return E::NS >= 30 ? 1 : (E::NS >= 10 ? 2 : 4);
  else return E::NS >= 64 ? 2 : (E::NS >= 25 ? 4 : (E::NS >= 9 ? 8 : 16));
}

// --------------------------------------------------------------------------
// Pass 1: face traces u^f = M0 u for a tile of elements.
template <class E, int NV, class T, class R> constexpr int trace_lds() {
  return lds_bytes<int>(E::NF * E::WL) + lds_bytes<R>(E::NF * E::WL) + lds_bytes<T>(rhs_tile<E>() * E::NS * NV);
}
template <class E, int NV, class T, class R, class IO, class Sync>
FR_HD void trace_body(int tile, int tid, int nth, char* lds, const OpsD<R>& op, int ne, const IO* U, const IO* V,
                      T* UF, Sync sync) {
  constexpr int NS = E::NS, NF = E::NF, WL = E::WL, TE = rhs_tile<E>();
  Lds L{lds};
  int* m0c = L.take<int>(NF * WL);
  R* m0v = L.take<R>(NF * WL);
  T* su = L.take<T>(TE * NS * NV);
  const int e0 = tile * TE;
  const int nte = (ne - e0) < TE ? (ne - e0) : TE;
  for (int i = tid; i < NF * WL; i += nth) { m0c[i] = op.m0c[i]; m0v[i] = op.m0v[i]; }
  for (int i = tid; i < nte * NS * NV; i += nth) su[i] = make_in<T, R, IO>(U, V, (long)e0 * NS * NV + i);
  sync();
  for (int i = tid; i < nte * NF * NV; i += nth) {
    int e = i / (NF * NV), g = (i / NV) % NF, a = i % NV;
    T acc = T(R(0));
    for (int w = 0; w < WL; ++w) acc += m0v[g * WL + w] * su[(e * NS + m0c[g * WL + w]) * NV + a];
    UF[(long)e0 * NF * NV + i] = acc;
  }
}

// --------------------------------------------------------------------------
// Pass 2 (viscous systems): corrected physical gradient q at solution points
// and its face trace q^f = M0 q.
// Elements per gradient tile: 2-D dual-number tiles take half the residual
// tile (their LDS is twice as large; with more workgroups per CU the 2-D
// NS p=3 tangent pass ran 109 -> 96 us).
template <class E, class T> constexpr int grad_tile() {
  constexpr int t = rhs_tile<E>();
  return (E::ND == 2 && sizeof(T) > 8 && t > 1) ? t / 2 : t;
}
template <class E, int NV, class T, class R, int TE = rhs_tile<E>()> constexpr int grad_lds() {
  constexpr int NS = E::NS, NF = E::NF, ND = E::ND, WL = E::WL, WC = E::WC;
  return lds_bytes<int>(NF * WL) + lds_bytes<R>(NF * WL) + lds_bytes<int>(ND * NS * WL) + lds_bytes<R>(ND * NS * WL) +
         lds_bytes<int>(NS * WC) + lds_bytes<R>(NS * WC) + lds_bytes<R>(NF * ND) + lds_bytes<T>(TE * NS * NV) +
         lds_bytes<T>(TE * NF * NV) + lds_bytes<T>(TE * NS * ND * NV);
}
template <class E, int NV, class T, class R, class IO, class Sync, int TE = rhs_tile<E>()>
FR_HD void grad_body(int tile, int tid, int nth, char* lds, const OpsD<R>& op, const GeoD<R>& geo, double beta,
                     const IO* U, const IO* V, const T* UF, T* Q, T* QF, Sync sync) {
  constexpr int NS = E::NS, NF = E::NF, ND = E::ND, WL = E::WL, WC = E::WC;
  Lds L{lds};
  int* m0c = L.take<int>(NF * WL);
  R* m0v = L.take<R>(NF * WL);
  int* ddc = L.take<int>(ND * NS * WL);
  R* ddv = L.take<R>(ND * NS * WL);
  int* crc = L.take<int>(NS * WC);
  R* crv = L.take<R>(NS * WC);
  R* snr = L.take<R>(NF * ND);
  T* su = L.take<T>(TE * NS * NV);
  T* sdf = L.take<T>(TE * NF * NV);
  T* sq = L.take<T>(TE * NS * ND * NV);
  const int e0 = tile * TE;
  const int nte = (geo.ne - e0) < TE ? (geo.ne - e0) : TE;
  const R cb = R(0.5 + beta);
  for (int i = tid; i < NF * WL; i += nth) { m0c[i] = op.m0c[i]; m0v[i] = op.m0v[i]; }
  for (int i = tid; i < ND * NS * WL; i += nth) { ddc[i] = op.ddc[i]; ddv[i] = op.ddv[i]; }
  for (int i = tid; i < NS * WC; i += nth) { crc[i] = op.crc[i]; crv[i] = op.crv[i]; }
  for (int i = tid; i < NF * ND; i += nth) snr[i] = op.nref[i];
  for (int i = tid; i < nte * NS * NV; i += nth) su[i] = make_in<T, R, IO>(U, V, (long)e0 * NS * NV + i);
  // (C - u^f) = (1/2 + beta)(u^f_nbr - u^f)
  for (int i = tid; i < nte * NF * NV; i += nth) {
    int e = i / (NF * NV), g = (i / NV) % NF, a = i % NV;
    long n = e0 + e;
    long pg = geo.nbfp[n * NF + g];
    sdf[i] = cb * (UF[pg * NV + a] - UF[(n * NF + g) * NV + a]);
  }
  sync();
  for (int i = tid; i < nte * NS * NV; i += nth) {
    int e = i / (NS * NV), r = (i / NV) % NS, a = i % NV;
    long n = e0 + e;
    T qt[ND];
    for (int d = 0; d < ND; ++d) {
      T acc = T(R(0));
      for (int w = 0; w < WL; ++w) acc += ddv[(d * NS + r) * WL + w] * su[(e * NS + ddc[(d * NS + r) * WL + w]) * NV + a];
      for (int w = 0; w < WC; ++w) {
        int g = crc[r * WC + w];
        acc += (crv[r * WC + w] * snr[g * ND + d]) * sdf[(e * NF + g) * NV + a];
      }
      qt[d] = acc;
    }
    const R* Ji = geo.Jinv + (n * NS + r) * ND * ND;
    for (int d2 = 0; d2 < ND; ++d2) {
      T acc = T(R(0));
      for (int d = 0; d < ND; ++d) acc += Ji[d * ND + d2] * qt[d];
      sq[((e * NS + r) * ND + d2) * NV + a] = acc;
      Q[((n * NS + r) * ND + d2) * NV + a] = acc;
    }
  }
  sync();
  for (int i = tid; i < nte * NF * ND * NV; i += nth) {
    int e = i / (NF * ND * NV), g = (i / (ND * NV)) % NF, d = (i / NV) % ND, a = i % NV;
    T acc = T(R(0));
    for (int w = 0; w < WL; ++w) acc += m0v[g * WL + w] * sq[((e * NS + m0c[g * WL + w]) * ND + d) * NV + a];
    QF[(long)e0 * NF * ND * NV + i] = acc;
  }
}

// --------------------------------------------------------------------------
// Pass 3: transformed flux, common flux, FR divergence, R = -div/detJ.
template <class E, int NV, int SYS, class T, class R, int TE = rhs_tile<E>()> constexpr int div_lds() {
  constexpr int NS = E::NS, NF = E::NF, ND = E::ND, WL = E::WL, WC = E::WC;
  return lds_bytes<int>(NF * WL) + lds_bytes<R>(NF * WL) + lds_bytes<int>(ND * NS * WL) + lds_bytes<R>(ND * NS * WL) +
         lds_bytes<int>(NS * WC) + lds_bytes<R>(NS * WC) + lds_bytes<R>(NF * ND) + lds_bytes<T>(TE * NS * ND * NV) +
         lds_bytes<T>(TE * NF * NV);
}
// Elements per divergence tile: the flux and common-flux phases run one
// thread per solution point and per flux point, so the tile is doubled while
// those phases still fit the 256 threads and its LDS stays within 64 KB
// (two workgroups per CU).
template <class E, int NV, int SYS, class T, class R> constexpr int div_tile() {
  constexpr int t = rhs_tile<E>();
  constexpr int NP = E::NS > E::NF ? E::NS : E::NF;
  if constexpr (2 * t * NP <= 256 && div_lds<E, NV, SYS, T, R, 2 * t>() <= 64 * 1024) return 2 * t;
  else return t;
}
// Dual scalars: the tangent output is ta V + tb (J V).
template <class E, int NV, int SYS, class T, class R, class IO, class Sync, int TE = rhs_tile<E>()>
FR_HD void div_body(int tile, int tid, int nth, char* lds, const OpsD<R>& op, const GeoD<R>& geo, const PhysP& ph,
                    const IO* U, const IO* V, const T* UF, const T* Q, const T* QF, IO* Rout, IO* Rtan, Sync sync,
                    double ta = 0.0, double tb = 1.0) {
  constexpr int NS = E::NS, NF = E::NF, ND = E::ND, WL = E::WL, WC = E::WC;
  constexpr bool VISC = SysTraits<SYS>::kVisc;
  Lds L{lds};
  int* m0c = L.take<int>(NF * WL);
  R* m0v = L.take<R>(NF * WL);
  int* ddc = L.take<int>(ND * NS * WL);
  R* ddv = L.take<R>(ND * NS * WL);
  int* crc = L.take<int>(NS * WC);
  R* crv = L.take<R>(NS * WC);
  R* snr = L.take<R>(NF * ND);
  T* sFt = L.take<T>(TE * NS * ND * NV);
  T* sJ = L.take<T>(TE * NF * NV);
  const int e0 = tile * TE;
  const int nte = (geo.ne - e0) < TE ? (geo.ne - e0) : TE;
  const bool visc = VISC && (SYS != SYS_ADV || ph.mu != 0.0);
  for (int i = tid; i < NF * WL; i += nth) { m0c[i] = op.m0c[i]; m0v[i] = op.m0v[i]; }
  for (int i = tid; i < ND * NS * WL; i += nth) { ddc[i] = op.ddc[i]; ddv[i] = op.ddv[i]; }
  for (int i = tid; i < NS * WC; i += nth) { crc[i] = op.crc[i]; crv[i] = op.crv[i]; }
  for (int i = tid; i < NF * ND; i += nth) snr[i] = op.nref[i];
  // transformed flux at solution points
  for (int i = tid; i < nte * NS; i += nth) {
    int e = i / NS, r = i % NS;
    long n = e0 + e;
    T u[NV], f[ND][NV];
    for (int a = 0; a < NV; ++a) u[a] = make_in<T, R, IO>(U, V, (n * NS + r) * NV + a);
    flux_inviscid<SYS, ND, NV, T>(ph, u, f);
    if (visc) {
      T q[ND][NV], fv[ND][NV];
      for (int d = 0; d < ND; ++d)
        for (int a = 0; a < NV; ++a) q[d][a] = Q[((n * NS + r) * ND + d) * NV + a];
      flux_viscous<SYS, ND, NV, T>(ph, u, q, fv);
      for (int d = 0; d < ND; ++d)
        for (int a = 0; a < NV; ++a) f[d][a] += fv[d][a];
    }
    const R* Sm = geo.S + (n * NS + r) * ND * ND;
    for (int d = 0; d < ND; ++d)
      for (int a = 0; a < NV; ++a) {
        T acc = T(R(0));
        for (int k = 0; k < ND; ++k) acc += Sm[d * ND + k] * f[k][a];
        sFt[((e * NS + r) * ND + d) * NV + a] = acc;
      }
  }
  sync();
  // common flux minus interpolated normal flux at flux points
  const R cL = R(0.5 + ph.beta), cR = R(0.5 - ph.beta), eta = R(ph.eta);
  for (int i = tid; i < nte * NF; i += nth) {
    int e = i / NF, g = i % NF;
    long n = e0 + e;
    long pg = geo.nbfp[n * NF + g];
    T uL[NV], uR[NV], F[NV];
    for (int a = 0; a < NV; ++a) { uL[a] = UF[(n * NF + g) * NV + a]; uR[a] = UF[pg * NV + a]; }
    R nn[ND];
    for (int d = 0; d < ND; ++d) nn[d] = geo.nrm[(n * NF + g) * ND + d];
    common_inviscid<SYS, ND, NV, T>(ph, uL, uR, nn, F);
    if (visc) {
      T qL[ND][NV], qR[ND][NV], fL[ND][NV], fR[ND][NV];
      for (int d = 0; d < ND; ++d)
        for (int a = 0; a < NV; ++a) {
          qL[d][a] = QF[((n * NF + g) * ND + d) * NV + a];
          qR[d][a] = QF[(pg * ND + d) * NV + a];
        }
      flux_viscous<SYS, ND, NV, T>(ph, uL, qL, fL);
      flux_viscous<SYS, ND, NV, T>(ph, uR, qR, fR);
      for (int a = 0; a < NV; ++a) {
        T acc = eta * (uL[a] - uR[a]);
        for (int d = 0; d < ND; ++d) acc += nn[d] * (cL * fL[d][a] + cR * fR[d][a]);
        F[a] += acc;
      }
    }
    R mg = geo.magN[n * NF + g];
    for (int a = 0; a < NV; ++a) {
      T fn = T(R(0));
      for (int d = 0; d < ND; ++d) {
        T t = T(R(0));
        for (int w = 0; w < WL; ++w) t += m0v[g * WL + w] * sFt[((e * NS + m0c[g * WL + w]) * ND + d) * NV + a];
        fn += snr[g * ND + d] * t;
      }
      sJ[(e * NF + g) * NV + a] = mg * F[a] - fn;
    }
  }
  sync();
  for (int i = tid; i < nte * NS * NV; i += nth) {
    int e = i / (NS * NV), r = (i / NV) % NS, a = i % NV;
    long n = e0 + e;
    T acc = T(R(0));
    for (int d = 0; d < ND; ++d)
      for (int w = 0; w < WL; ++w)
        acc += ddv[(d * NS + r) * WL + w] * sFt[((e * NS + ddc[(d * NS + r) * WL + w]) * ND + d) * NV + a];
    for (int w = 0; w < WC; ++w) acc += crv[r * WC + w] * sJ[(e * NF + crc[r * WC + w]) * NV + a];
    T res = -(geo.rdet[n * NS + r] * acc);
    long o = (n * NS + r) * NV + a;
    if (Rout) {
      Rout[o] = IO(val(res));
      if (!fr_finite(val(res))) fr_flag_nonfinite(geo.status, FR_NF_RHS, geo.e0 + n);
    }
    if constexpr (!std::is_same<T, R>::value) {
      if (Rtan) {
        const R jv = (ta == 0.0 && tb == 1.0) ? res.d : R(ta * double(V[o]) + tb * double(res.d));
        Rtan[o] = IO(jv);
        if (!fr_finite(jv)) fr_flag_nonfinite(geo.status, FR_NF_JVP, geo.e0 + n);
      }
    }
  }
}

// --------------------------------------------------------------------------
// SDRT divergence (tensor elements, section "SDRT method"): on every line
// along axis d the flux is represented by the Lagrange basis psi_0..psi_{p+1}
// of the SD flux points {-1, z_1..z_p, +1}.  At the interior points the
// transformed normal flux (detJ J^{-1} f(u, q)) . e_d is evaluated from u and
// q interpolated along the line; at the two ends the |N|-scaled common flux
// (outward) stands in, with sign -1 at the -1 end.  The divergence at the
// solution points is the sum over axes of psi_j' along the point's line
// (eq. "divergence_sdrt"); R = -div / detJ.  The gradient pass is the FR one
// with the SD correction, which equals the SDRT gradient (u is of degree p).
template <class E> struct SdSizes {
  static constexpr int N1 = E::DEG + 1, P = E::DEG, NL = E::NS / (E::DEG + 1), NI = E::ND * NL * P;
};
template <class E, int NV, int SYS, class T, class R> constexpr int sd_div_lds() {
  typedef SdSizes<E> Q;
  constexpr int TE = rhs_tile<E>();
  return lds_bytes<R>(Q::P * Q::N1) + lds_bytes<R>(Q::N1 * (Q::P + 2)) + lds_bytes<int>(E::ND * Q::NL * 2) +
         lds_bytes<T>(TE * Q::NI * NV) + lds_bytes<T>(TE * E::NF * NV);
}
// index of the solution point at position m of line l along axis d (the
// other axes' indices taken from l in increasing axis order)
template <class E> FR_HD int sd_point(int d, int l, int m) {
  constexpr int N1 = E::DEG + 1;
  int idx[3] = {0, 0, 0}, rem = l;
  for (int a = 0; a < E::ND; ++a)
    if (a != d) { idx[a] = rem % N1; rem /= N1; }
  idx[d] = m;
  return idx[0] + N1 * (idx[1] + N1 * idx[2]);
}
template <class E> FR_HD void sd_line_of(int r, int d, int& l, int& m) {
  constexpr int N1 = E::DEG + 1;
  int idx[3] = {r % N1, (r / N1) % N1, r / (N1 * N1)};
  m = idx[d];
  l = 0;
  int mul = 1;
  for (int a = 0; a < E::ND; ++a)
    if (a != d) { l += idx[a] * mul; mul *= N1; }
}
template <class E, int NV, int SYS, class T, class R, class IO, class Sync>
FR_HD void sd_div_body(int tile, int tid, int nth, char* lds, const OpsD<R>& op, const GeoD<R>& geo, const PhysP& ph,
                       const IO* U, const IO* V, const T* UF, const T* Q, const T* QF, IO* Rout, IO* Rtan, Sync sync) {
  typedef SdSizes<E> Z;
  constexpr int NS = E::NS, NF = E::NF, ND = E::ND, N1 = Z::N1, P = Z::P, NL = Z::NL, NI = Z::NI;
  constexpr int TE = rhs_tile<E>();
  constexpr bool VISC = SysTraits<SYS>::kVisc;
  Lds L{lds};
  R* sI = L.take<R>(P * N1);
  R* sD = L.take<R>(N1 * (P + 2));
  int* send = L.take<int>(ND * NL * 2);
  T* sFi = L.take<T>(TE * NI * NV);
  T* sJ = L.take<T>(TE * NF * NV);
  const int e0 = tile * TE;
  const int nte = (geo.ne - e0) < TE ? (geo.ne - e0) : TE;
  const bool visc = VISC && (SYS != SYS_ADV || ph.mu != 0.0);
  for (int i = tid; i < P * N1; i += nth) sI[i] = op.sdI[i];
  for (int i = tid; i < N1 * (P + 2); i += nth) sD[i] = op.sdD[i];
  for (int i = tid; i < ND * NL * 2; i += nth) send[i] = op.sdend[i];
  sync();
  // transformed normal flux at the interior flux points
  for (int i = tid; i < nte * NI; i += nth) {
    const int e = i / NI, k = i % NI, d = k / (NL * P), l = (k / P) % NL, j = k % P;
    const long n = e0 + e;
    T u[NV], f[ND][NV];
    for (int a = 0; a < NV; ++a) u[a] = T(R(0));
    for (int m = 0; m < N1; ++m) {
      const long o = (n * NS + sd_point<E>(d, l, m)) * NV;
      for (int a = 0; a < NV; ++a) u[a] += sI[j * N1 + m] * make_in<T, R, IO>(U, V, o + a);
    }
    flux_inviscid<SYS, ND, NV, T>(ph, u, f);
    if (visc) {
      T q[ND][NV], fv[ND][NV];
      for (int dd = 0; dd < ND; ++dd)
        for (int a = 0; a < NV; ++a) q[dd][a] = T(R(0));
      for (int m = 0; m < N1; ++m) {
        const long o = (n * NS + sd_point<E>(d, l, m)) * ND * NV;
        for (int dd = 0; dd < ND; ++dd)
          for (int a = 0; a < NV; ++a) q[dd][a] += sI[j * N1 + m] * Q[o + dd * NV + a];
      }
      flux_viscous<SYS, ND, NV, T>(ph, u, q, fv);
      for (int dd = 0; dd < ND; ++dd)
        for (int a = 0; a < NV; ++a) f[dd][a] += fv[dd][a];
    }
    const R* Sr = geo.Sint + (((n * ND + d) * NL + l) * P + j) * ND;
    for (int a = 0; a < NV; ++a) {
      T acc = T(R(0));
      for (int kk = 0; kk < ND; ++kk) acc += Sr[kk] * f[kk][a];
      sFi[(e * NI + k) * NV + a] = acc;
    }
  }
  // |N| times the common flux at the external flux points
  const R cL = R(0.5 + ph.beta), cR = R(0.5 - ph.beta), eta = R(ph.eta);
  for (int i = tid; i < nte * NF; i += nth) {
    const int e = i / NF, g = i % NF;
    const long n = e0 + e;
    const long pg = geo.nbfp[n * NF + g];
    T uL[NV], uR[NV], F[NV];
    for (int a = 0; a < NV; ++a) { uL[a] = UF[(n * NF + g) * NV + a]; uR[a] = UF[pg * NV + a]; }
    R nn[ND];
    for (int d = 0; d < ND; ++d) nn[d] = geo.nrm[(n * NF + g) * ND + d];
    common_inviscid<SYS, ND, NV, T>(ph, uL, uR, nn, F);
    if (visc) {
      T qL[ND][NV], qR[ND][NV], fL[ND][NV], fR[ND][NV];
      for (int d = 0; d < ND; ++d)
        for (int a = 0; a < NV; ++a) {
          qL[d][a] = QF[((n * NF + g) * ND + d) * NV + a];
          qR[d][a] = QF[(pg * ND + d) * NV + a];
        }
      flux_viscous<SYS, ND, NV, T>(ph, uL, qL, fL);
      flux_viscous<SYS, ND, NV, T>(ph, uR, qR, fR);
      for (int a = 0; a < NV; ++a) {
        T acc = eta * (uL[a] - uR[a]);
        for (int d = 0; d < ND; ++d) acc += nn[d] * (cL * fL[d][a] + cR * fR[d][a]);
        F[a] += acc;
      }
    }
    const R mg = geo.magN[n * NF + g];
    for (int a = 0; a < NV; ++a) sJ[(e * NF + g) * NV + a] = mg * F[a];
  }
  sync();
  for (int i = tid; i < nte * NS * NV; i += nth) {
    const int e = i / (NS * NV), r = (i / NV) % NS, a = i % NV;
    const long n = e0 + e;
    T acc = T(R(0));
    for (int d = 0; d < ND; ++d) {
      int l, m;
      sd_line_of<E>(r, d, l, m);
      const R* Dm = sD + m * (P + 2);
      acc += Dm[P + 1] * sJ[(e * NF + send[(d * NL + l) * 2 + 1]) * NV + a];
      acc -= Dm[0] * sJ[(e * NF + send[(d * NL + l) * 2 + 0]) * NV + a];
      for (int j = 0; j < P; ++j) acc += Dm[j + 1] * sFi[(e * NI + (d * NL + l) * P + j) * NV + a];
    }
    T res = -(geo.rdet[n * NS + r] * acc);
    const long o = (n * NS + r) * NV + a;
    if (Rout) {
      Rout[o] = IO(val(res));
      if (!fr_finite(val(res))) fr_flag_nonfinite(geo.status, FR_NF_RHS, geo.e0 + n);
    }
    if constexpr (!std::is_same<T, R>::value) {
      if (Rtan) {
        Rtan[o] = IO(res.d);
        if (!fr_finite(res.d)) fr_flag_nonfinite(geo.status, FR_NF_JVP, geo.e0 + n);
      }
    }
  }
}

// --------------------------------------------------------------------------
// Jacobian blocks dR_n/dU_k for k in {n} U face-neighbours(n).
//
// Every step between U and R is either a linear reference operator acting on
// each conserved variable separately, or a pointwise map.  The chain rule
// therefore gives, for each pair (alpha, beta) of output/input variables,
// an independent product of scalar operators:
//   X_d[tau][sigma] = a_d(tau) delta_{tau sigma} [k = n] + sum_e b_de(tau) Gam_e[tau][sigma]
//   Y[g][sigma]     = fuL(g) DL[g][sigma] + fuR(g) DR[g][sigma]
//                     + sum_d' fqL_d'(g) SL_d'[g][sigma] + fqR_d'(g) SR_d'[g][sigma]
//   J[(rho,alpha),(sigma,beta)] = -rdet(rho) (sum_d Dc_d X_d + Cor Y)[rho][sigma]
// with a_d = dF~_d/du, b_de = dF~_d/dq~_e (solution points), fuL/fuR/fqL/fqR
// the |N|-scaled derivatives of the common flux (flux points), all taken at
// entry (alpha, beta); Gam_e = dq~_e/du_k (scalar), SL/SR = derivatives of
// the own / neighbour physical face gradient w.r.t. u_k, DL/DR the face
// interpolation of u_k, and Dc_d = D_d - Cor diag(nref_d) M0.  Second-layer
// blocks of the viscous stencil are not produced (their paths reach R_n only
// through the neighbour's gradient, with k outside the face stencil).
// Blocks are written column-major: B[n][k][c][r], r = rho*NV + alpha,
// c = sigma*NV + beta.

template <class E, int NV, int SYS> struct JacSizes {
  static constexpr int NS = E::NS, NF = E::NF, ND = E::ND, NFACE = E::NFACE, NFP = E::NFP, WL = E::WL, WC = E::WC;
  static constexpr int NV2 = NV * NV;
  static constexpr bool VISC = SysTraits<SYS>::kVisc;
  static constexpr int NQ = VISC ? ND : 0;
};

template <class E, int NV, int SYS, class R> constexpr int jac_lds() {
  typedef JacSizes<E, NV, SYS> Z;
  constexpr int NS = Z::NS, NF = Z::NF, ND = Z::ND, NFACE = Z::NFACE, NFP = Z::NFP, WL = Z::WL, WC = Z::WC,
                NV2 = Z::NV2;
  int b = 0;
  // operators
  b += lds_bytes<R>(NF * NS) + lds_bytes<R>(NS * NF) + lds_bytes<R>(NF * ND) + lds_bytes<int>(NF);
  b += lds_bytes<int>(NF * WL) + lds_bytes<R>(NF * WL);
  b += 2 * (lds_bytes<int>(ND * NS * WL) + lds_bytes<R>(ND * NS * WL));
  b += lds_bytes<int>(NS * WC) + lds_bytes<R>(NS * WC);
  // element data
  b += lds_bytes<R>(NS * NV) + lds_bytes<R>(NS * ND * NV) + 2 * lds_bytes<R>(NF * NV) + 2 * lds_bytes<R>(NF * ND * NV);
  b += 2 * lds_bytes<R>(NS * ND * ND) + lds_bytes<R>(NS) + lds_bytes<R>(NF * ND) + lds_bytes<R>(NF) + lds_bytes<int>(NF);
  b += lds_bytes<R>(NFACE * NFP * NFP * ND);
  b += lds_bytes<R>(NFACE * NS * ND * ND) + lds_bytes<int>(NFACE * NFP) + lds_bytes<int>(NFACE) + lds_bytes<int>(NFACE);
  // tables
  b += lds_bytes<R>(ND * NS * NV2) + lds_bytes<R>(ND * ND * NS * NV2) + 2 * lds_bytes<R>(NF * NV2) +
       2 * lds_bytes<R>(ND * NF * NV2);
  // scratch shared by the table build and the per-block sensitivities
  int t1 = lds_bytes<R>(ND * ND * NS * NV2) + 4 * lds_bytes<R>(NF * NV2);
  int t2 = 2 * lds_bytes<R>(ND * NS * NS) + 2 * lds_bytes<R>(ND * NF * NS) + 2 * lds_bytes<R>(NF * NS) +
           lds_bytes<R>(NV * ND * NS * NS) + lds_bytes<R>(NV * NF * NS);
  b += t1 > t2 ? t1 : t2;
  return b;
}

template <class OT> FR_HD OT to_out(float x);
template <> FR_HD float to_out<float>(float x) { return x; }
template <class OT> FR_HD OT to_out(double x);
template <> FR_HD double to_out<double>(double x) { return x; }
template <> FR_HD float to_out<float>(double x) { return (float)x; }
// bf16 storage: round-to-nearest-even of the fp32 value.
struct bf16_t { unsigned short bits; };
template <> FR_HD bf16_t to_out<bf16_t>(float x) {
  unsigned int u;
  __builtin_memcpy(&u, &x, 4);
  unsigned int lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  bf16_t r; r.bits = (unsigned short)(u >> 16);
  return r;
}
template <> FR_HD bf16_t to_out<bf16_t>(double x) { return to_out<bf16_t>((float)x); }

// nblk = 1 + NFACE writes every block; nblk = 1 only the diagonal block (for
// block-Jacobi preconditioners), element stride nblk * b * b.
template <class E, int NV, int SYS, class R, class OT, class Sync>
FR_HD void jac_body(int n, int tid, int nth, char* lds, const OpsD<R>& op, const GeoD<R>& geo, const PhysP& ph,
                    const R* U, const R* Q, const R* UF, const R* QF, OT* B, int nblk, Sync sync) {
  typedef JacSizes<E, NV, SYS> Z;
  constexpr int NS = Z::NS, NF = Z::NF, ND = Z::ND, NFACE = Z::NFACE, NFP = Z::NFP, WL = Z::WL, WC = Z::WC,
                NV2 = Z::NV2;
  constexpr int BB = NS * NV;                 // block dimension
  const bool visc = Z::VISC && (SYS != SYS_ADV || ph.mu != 0.0);
  const R cb = R(0.5 + ph.beta), cL = R(0.5 + ph.beta), cR = R(0.5 - ph.beta), eta = R(ph.eta);
  typedef MDual<R, NV> MD;

  Lds L{lds};
  R* sM0 = L.take<R>(NF * NS);
  R* sCor = L.take<R>(NS * NF);
  R* snr = L.take<R>(NF * ND);
  int* sff = L.take<int>(NF);
  int* m0c = L.take<int>(NF * WL);
  R* m0v = L.take<R>(NF * WL);
  int* dcc = L.take<int>(ND * NS * WL);
  R* dcv = L.take<R>(ND * NS * WL);
  int* gcc = L.take<int>(ND * NS * WL);
  R* gcv = L.take<R>(ND * NS * WL);
  int* crc = L.take<int>(NS * WC);
  R* crv = L.take<R>(NS * WC);
  R* su = L.take<R>(NS * NV);
  R* sq = L.take<R>(NS * ND * NV);
  R* suL = L.take<R>(NF * NV);
  R* suR = L.take<R>(NF * NV);
  R* sqL = L.take<R>(NF * ND * NV);
  R* sqR = L.take<R>(NF * ND * NV);
  R* sJi = L.take<R>(NS * ND * ND);
  R* sS = L.take<R>(NS * ND * ND);
  R* srd = L.take<R>(NS);
  R* snn = L.take<R>(NF * ND);
  R* smg = L.take<R>(NF);
  int* spg = L.take<int>(NF);
  R* sW = L.take<R>(NFACE * NFP * NFP * ND);
  R* sJm = L.take<R>(NFACE * NS * ND * ND);   // neighbours' J^{-1} at their solution points
  int* sback = L.take<int>(NFACE * NFP);     // partner in n of each point of the neighbour's shared face
  int* snb = L.take<int>(NFACE);             // neighbour element of each face
  int* snf = L.take<int>(NFACE);             // the neighbour's face index of the shared face
  R* ta = L.take<R>(ND * NS * NV2);        // a[d][tau][ab]
  R* tb = L.take<R>(ND * ND * NS * NV2);   // b[d][e][tau][ab]
  R* tuL = L.take<R>(NF * NV2);            // fuL[g][ab]
  R* tuR = L.take<R>(NF * NV2);
  R* tqL = L.take<R>(ND * NF * NV2);       // fqL[d'][g][ab]
  R* tqR = L.take<R>(ND * NF * NV2);
  char* scratch = L.p;
  // table-build scratch
  Lds L1{scratch};
  R* bh = L1.take<R>(ND * ND * NS * NV2);  // df_k/dq_d' [d'][k][tau][ab]
  R* rL = L1.take<R>(NF * NV2);
  R* rR = L1.take<R>(NF * NV2);
  R* vL = L1.take<R>(NF * NV2);
  R* vR = L1.take<R>(NF * NV2);
  // per-block scratch (aliases the table-build scratch)
  Lds L2{scratch};
  R* gam = L2.take<R>(ND * NS * NS);       // Gam_e[tau][sigma]
  R* gamp = L2.take<R>(ND * NS * NS);      // physical: sum_e Jinv[tau][e][d'] Gam_e
  R* SL = L2.take<R>(ND * NF * NS);
  R* SR = L2.take<R>(ND * NF * NS);
  R* DL = L2.take<R>(NF * NS);
  R* DR = L2.take<R>(NF * NS);
  R* X = L2.take<R>(NV * ND * NS * NS);    // [alpha][d][tau][sigma] for one beta
  R* Y = L2.take<R>(NV * NF * NS);         // [alpha][g][sigma]

  // ---- load operators and element data
  for (int i = tid; i < NF * NS; i += nth) sM0[i] = op.M0[i];
  for (int i = tid; i < NS * NF; i += nth) sCor[i] = op.Cor[i];
  for (int i = tid; i < NF * ND; i += nth) snr[i] = op.nref[i];
  for (int i = tid; i < NF; i += nth) sff[i] = op.fface[i];
  for (int i = tid; i < NF * WL; i += nth) { m0c[i] = op.m0c[i]; m0v[i] = op.m0v[i]; }
  for (int i = tid; i < ND * NS * WL; i += nth) { dcc[i] = op.dcc[i]; dcv[i] = op.dcv[i]; gcc[i] = op.gc[i]; gcv[i] = op.gv[i]; }
  for (int i = tid; i < NS * WC; i += nth) { crc[i] = op.crc[i]; crv[i] = op.crv[i]; }
  const long nl = n;
  for (int i = tid; i < NS * NV; i += nth) su[i] = U[nl * NS * NV + i];
  if (visc)
    for (int i = tid; i < NS * ND * NV; i += nth) sq[i] = Q[nl * NS * ND * NV + i];
  for (int i = tid; i < NF; i += nth) spg[i] = geo.nbfp[nl * NF + i];
  for (int i = tid; i < NS * ND * ND; i += nth) { sJi[i] = geo.Jinv[nl * NS * ND * ND + i]; sS[i] = geo.S[nl * NS * ND * ND + i]; }
  for (int i = tid; i < NS; i += nth) srd[i] = geo.rdet[nl * NS + i];
  for (int i = tid; i < NF * ND; i += nth) snn[i] = geo.nrm[nl * NF * ND + i];
  for (int i = tid; i < NF; i += nth) smg[i] = geo.magN[nl * NF + i];
  for (int i = tid; i < NFACE; i += nth) snb[i] = geo.nbr[nl * NFACE + i];
  sync();
  for (int i = tid; i < NF * NV; i += nth) {
    int g = i / NV, a = i % NV;
    suL[i] = UF[(nl * NF + g) * NV + a];
    suR[i] = UF[(long)spg[g] * NV + a];
  }
  if (visc)
    for (int i = tid; i < NF * ND * NV; i += nth) {
      int g = i / (ND * NV), r = i % (ND * NV);
      sqL[i] = QF[(nl * NF + g) * ND * NV + r];
      sqR[i] = QF[(long)spg[g] * ND * NV + r];
    }
  // the neighbours' faces, metric and pairing enter the viscous blocks only
  if (visc) {
    for (int i = tid; i < NFACE; i += nth) snf[i] = sff[spg[i * NFP] - snb[i] * NF];
    for (int i = tid; i < NFACE * NS * ND * ND; i += nth) {
      int f = i / (NS * ND * ND), r = i % (NS * ND * ND);
      sJm[i] = geo.Jinv[(long)snb[f] * NS * ND * ND + r];
    }
  }
  sync();
  if (visc)
    for (int i = tid; i < NFACE * NFP; i += nth) {
      int f = i / NFP, gj = i % NFP;
      sback[i] = geo.nbfp[(long)snb[f] * NF + snf[f] * NFP + gj] - n * NF;
    }
  // W_d'[f][g][g'] for the neighbour gradient's dependence on u_n (self block):
  // sum_tau' M0[g2][tau'] Cor[tau'][g'] sum_e Jinv_m[tau'][e][d'] nref[g'][e],
  // g on face f, g2 its partner in m, g' on the shared face f2 of m.
  if (visc)
    for (int i = tid; i < NFACE * NFP * NFP * ND; i += nth) {
      int f = i / (NFP * NFP * ND), gi = (i / (NFP * ND)) % NFP, gj = (i / ND) % NFP, d2 = i % ND;
      int g = f * NFP + gi;
      int m = snb[f];
      int g2 = spg[g] - m * NF;
      int gp = snf[f] * NFP + gj;
      R acc = R(0);
      for (int w = 0; w < WL; ++w) {
        int t = m0c[g2 * WL + w];
        R mv = m0v[g2 * WL + w];
        R je = R(0);
        for (int e = 0; e < ND; ++e) je += sJm[((f * NS + t) * ND + e) * ND + d2] * snr[gp * ND + e];
        acc += mv * sCor[t * NF + gp] * je;
      }
      sW[i] = cb * acc;
    }
  sync();

  // ---- pointwise Jacobian tables (forward mode, NV seeds per pass)
  {
    constexpr int NPS = 1 + Z::NQ;                       // passes per solution point
    constexpr int NPF = Z::VISC ? 4 + 2 * ND : 2;        // passes per flux point
    const int nsp = visc ? NPS : 1, nfp = visc ? NPF : 2;
    for (int it = tid; it < NS * nsp + NF * nfp; it += nth) {
      if (it < NS * nsp) {
        int t = it / nsp, ps = it % nsp;
        MD u[NV], f[ND][NV];
        MD q[ND][NV];
        for (int a = 0; a < NV; ++a) { u[a] = MD(su[t * NV + a]); if (ps == 0) u[a].d[a] = R(1); }
        for (int d = 0; d < ND; ++d)
          for (int a = 0; a < NV; ++a) {
            q[d][a] = MD(visc ? sq[(t * ND + d) * NV + a] : R(0));
            if (ps == 1 + d) q[d][a].d[a] = R(1);
          }
        if (ps == 0) {
          flux_inviscid<SYS, ND, NV, MD>(ph, u, f);
          if (visc) {
            MD fv[ND][NV];
            flux_viscous<SYS, ND, NV, MD>(ph, u, q, fv);
            for (int d = 0; d < ND; ++d)
              for (int a = 0; a < NV; ++a) f[d][a] += fv[d][a];
          }
          for (int d = 0; d < ND; ++d)
            for (int a = 0; a < NV; ++a)
              for (int c = 0; c < NV; ++c) {
                R acc = R(0);
                for (int k = 0; k < ND; ++k) acc += sS[(t * ND + d) * ND + k] * f[k][a].d[c];
                ta[(d * NS + t) * NV2 + a * NV + c] = acc;
              }
        } else {
          int d2 = ps - 1;
          flux_viscous<SYS, ND, NV, MD>(ph, u, q, f);
          for (int k = 0; k < ND; ++k)
            for (int a = 0; a < NV; ++a)
              for (int c = 0; c < NV; ++c) bh[((d2 * ND + k) * NS + t) * NV2 + a * NV + c] = f[k][a].d[c];
        }
      } else {
        int j = it - NS * nsp;
        int g = j / nfp, ps = j % nfp;
        R nn[ND];
        for (int d = 0; d < ND; ++d) nn[d] = snn[g * ND + d];
        if (ps < 2) {
          MD uL[NV], uR[NV], F[NV];
          for (int a = 0; a < NV; ++a) {
            uL[a] = MD(suL[g * NV + a]); uR[a] = MD(suR[g * NV + a]);
            if (ps == 0) uL[a].d[a] = R(1); else uR[a].d[a] = R(1);
          }
          common_inviscid<SYS, ND, NV, MD>(ph, uL, uR, nn, F);
          R* o = ps == 0 ? rL : rR;
          for (int a = 0; a < NV; ++a)
            for (int c = 0; c < NV; ++c) o[g * NV2 + a * NV + c] = F[a].d[c];
        } else {
          int pp = ps - 2;
          int side = (pp == 0 || (pp >= 2 && pp < 2 + ND)) ? 0 : 1;   // 0: L, 1: R
          int qd = (pp >= 2) ? ((pp - 2) % ND) : -1;                   // seeded gradient direction
          if (pp == 1) { side = 1; qd = -1; }
          if (pp >= 2 + ND) side = 1;
          const R* us = side ? suR : suL;
          const R* qs = side ? sqR : sqL;
          MD u[NV], q[ND][NV], fv[ND][NV];
          for (int a = 0; a < NV; ++a) { u[a] = MD(us[g * NV + a]); if (qd < 0) u[a].d[a] = R(1); }
          for (int d = 0; d < ND; ++d)
            for (int a = 0; a < NV; ++a) {
              q[d][a] = MD(qs[(g * ND + d) * NV + a]);
              if (qd == d) q[d][a].d[a] = R(1);
            }
          flux_viscous<SYS, ND, NV, MD>(ph, u, q, fv);
          R wgt = side ? cR : cL;
          R mg = smg[g];
          for (int a = 0; a < NV; ++a)
            for (int c = 0; c < NV; ++c) {
              R acc = R(0);
              for (int d = 0; d < ND; ++d) acc += nn[d] * fv[d][a].d[c];
              acc *= wgt;
              if (qd < 0) (side ? vR : vL)[g * NV2 + a * NV + c] = acc;
              else (side ? tqR : tqL)[(qd * NF + g) * NV2 + a * NV + c] = mg * acc;
            }
        }
      }
    }
    sync();
    // b_de = sum_k S_dk sum_d' (df_k/dq_d') Jinv[e][d']
    if (visc)
      for (int i = tid; i < ND * ND * NS * NV2; i += nth) {
        int d = i / (ND * NS * NV2), e = (i / (NS * NV2)) % ND, t = (i / NV2) % NS, ab = i % NV2;
        R acc = R(0);
        for (int k = 0; k < ND; ++k) {
          R s = sS[(t * ND + d) * ND + k];
          for (int d2 = 0; d2 < ND; ++d2) acc += s * bh[((d2 * ND + k) * NS + t) * NV2 + ab] * sJi[(t * ND + e) * ND + d2];
        }
        tb[i] = acc;
      }
    for (int i = tid; i < NF * NV2; i += nth) {
      int g = i / NV2, ab = i % NV2;
      int a = ab / NV, c = ab % NV;
      R mg = smg[g];
      R id = (a == c) ? eta : R(0);
      R l = rL[i] + (visc ? vL[i] + id : R(0));
      R r = rR[i] + (visc ? vR[i] - id : R(0));
      tuL[i] = mg * l;
      tuR[i] = mg * r;
    }
    sync();
  }

  // ---- blocks
  OT* Bn = B + nl * (long)nblk * BB * BB;
  for (int k = 0; k < nblk; ++k) {
    const int f = k - 1;                 // face of the neighbour block (k >= 1)
    const int m = (k == 0) ? n : snb[f];
    // Gam_e[tau][sigma] = d q~_e(tau) / d u_k(sigma)
    for (int i = tid; i < ND * NS * NS; i += nth) {
      int e = i / (NS * NS), t = (i / NS) % NS, s = i % NS;
      R v = R(0);
      if (visc) {
        if (k == 0) {
          for (int w = 0; w < WL; ++w)
            if (gcc[(e * NS + t) * WL + w] == s) v += gcv[(e * NS + t) * WL + w];
        } else {
          for (int gi = 0; gi < NFP; ++gi) {
            int g = f * NFP + gi;
            R c = sCor[t * NF + g] * snr[g * ND + e];
            if (c != R(0)) v += c * sM0[(spg[g] - m * NF) * NS + s];
          }
          v *= cb;
        }
      }
      gam[i] = v;
    }
    for (int i = tid; i < NF * NS; i += nth) {
      int g = i / NS, s = i % NS;
      DL[i] = (k == 0) ? sM0[i] : R(0);
      DR[i] = (k > 0 && sff[g] == f) ? sM0[(spg[g] - m * NF) * NS + s] : R(0);
    }
    sync();
    if (visc) {
      for (int i = tid; i < ND * NS * NS; i += nth) {
        int d2 = i / (NS * NS), t = (i / NS) % NS, s = i % NS;
        R acc = R(0);
        for (int e = 0; e < ND; ++e) acc += sJi[(t * ND + e) * ND + d2] * gam[(e * NS + t) * NS + s];
        gamp[i] = acc;
      }
      // SR: derivative of the neighbour's physical face gradient
      for (int i = tid; i < ND * NF * NS; i += nth) {
        int d2 = i / (NF * NS), g = (i / NS) % NF, s = i % NS;
        int fg = sff[g];
        R acc = R(0);
        if (k == 0) {
          int gi = g - fg * NFP;
          for (int gj = 0; gj < NFP; ++gj)
            acc += sW[((fg * NFP + gi) * NFP + gj) * ND + d2] * sM0[sback[fg * NFP + gj] * NS + s];
        } else if (fg == f) {
          int g2 = spg[g] - m * NF;
          for (int w = 0; w < WL; ++w) {
            int t = m0c[g2 * WL + w];
            R mv = m0v[g2 * WL + w];
            if (mv == R(0)) continue;
            R gsum = R(0);
            for (int e = 0; e < ND; ++e) {
              R ge = R(0);
              for (int w2 = 0; w2 < WL; ++w2)
                if (gcc[(e * NS + t) * WL + w2] == s) ge += gcv[(e * NS + t) * WL + w2];
              gsum += sJm[((f * NS + t) * ND + e) * ND + d2] * ge;
            }
            acc += mv * gsum;
          }
        }
        SR[i] = acc;
      }
      sync();
      for (int i = tid; i < ND * NF * NS; i += nth) {
        int d2 = i / (NF * NS), g = (i / NS) % NF, s = i % NS;
        R acc = R(0);
        for (int w = 0; w < WL; ++w) acc += m0v[g * WL + w] * gamp[(d2 * NS + m0c[g * WL + w]) * NS + s];
        SL[i] = acc;
      }
    }
    sync();
    OT* Bk = Bn + (long)k * BB * BB;
    for (int beta = 0; beta < NV; ++beta) {
      // X[alpha][d][tau][sigma], Y[alpha][g][sigma]
      for (int i = tid; i < NV * ND * NS * NS; i += nth) {
        int a = i / (ND * NS * NS), d = (i / (NS * NS)) % ND, t = (i / NS) % NS, s = i % NS;
        int ab = a * NV + beta;
        R v = (k == 0 && t == s) ? ta[(d * NS + t) * NV2 + ab] : R(0);
        if (visc)
          for (int e = 0; e < ND; ++e) v += tb[((d * ND + e) * NS + t) * NV2 + ab] * gam[(e * NS + t) * NS + s];
        X[i] = v;
      }
      for (int i = tid; i < NV * NF * NS; i += nth) {
        int a = i / (NF * NS), g = (i / NS) % NF, s = i % NS;
        int ab = a * NV + beta;
        R v = tuL[g * NV2 + ab] * DL[g * NS + s] + tuR[g * NV2 + ab] * DR[g * NS + s];
        if (visc)
          for (int d2 = 0; d2 < ND; ++d2)
            v += tqL[(d2 * NF + g) * NV2 + ab] * SL[(d2 * NF + g) * NS + s] +
                 tqR[(d2 * NF + g) * NV2 + ab] * SR[(d2 * NF + g) * NS + s];
        Y[i] = v;
      }
      sync();
      // columns c = sigma*NV + beta, rows r = rho*NV + alpha
      for (int i = tid; i < NS * NS * NV; i += nth) {
        int s = i / (NS * NV), r = (i / NV) % NS, a = i % NV;
        R acc = R(0);
        for (int d = 0; d < ND; ++d)
          for (int w = 0; w < WL; ++w)
            acc += dcv[(d * NS + r) * WL + w] * X[((a * ND + d) * NS + dcc[(d * NS + r) * WL + w]) * NS + s];
        for (int w = 0; w < WC; ++w) acc += crv[r * WC + w] * Y[(a * NF + crc[r * WC + w]) * NS + s];
        const R jv = -(srd[r] * acc);
        Bk[(long)(s * NV + beta) * BB + r * NV + a] = to_out<OT>(jv);
        if (!fr_finite(jv)) fr_flag_nonfinite(geo.status, FR_NF_BLOCKS, geo.e0 + n);
      }
      sync();
    }
  }
}

// ---------------------------------------------------------------- mixed meshes
// Face-neighbour blocks of an inviscid system on a conforming mesh that mixes
// element types: element n (type E) and its neighbour m across face f (type
// E or EO) meet only through the common flux at the face's points, so
//   dR_n(rho, alpha) / dU_m(sigma, beta) =
//     -(1/detJ_rho) sum_{g on f} Cor[rho][g] |N_g| dF_alpha/du_R,beta (g) M0_m[g'][sigma]
// with g' the point of m paired with g (eq. "divergence_fr"; the neighbour's
// trace u_R(g) = M0_m u_m, eq. "interpolate_sol_to_flux").  The block is
// b_n x b_m (rows rho*NV+alpha, columns sigma*NV+beta, column-major) at
// fboff[n][f].
template <class R> struct MixD {
  const int* nbpt;    // [ne][NF]: the paired point's local index in the neighbour
  const int* nbt;     // [ne][NFACE]: 1 when the neighbour is of the other type
  const long* fboff;  // [ne][NFACE]: first entry of each face block
  const R* M0o;       // [NFo][NSo]: the other type's solution-to-flux-point interpolation
};

// Stores the NV rows r*NV .. r*NV+NV-1 of one block column (contiguous).
template <int NV, class OT, class R> FR_HD void store_rows(OT* dst, const R* v) {
  if constexpr (NV == 4 && std::is_same<OT, float>::value && std::is_same<R, float>::value) {
    *reinterpret_cast<float4*>(dst) = make_float4(v[0], v[1], v[2], v[3]);
  } else {
    for (int a = 0; a < NV; ++a) dst[a] = to_out<OT>(v[a]);
  }
}

// All blocks of elements n0 .. n1-1 of one group of a mixed mesh, inviscid
// system.  Self block (at geo.boff[n]):
//   dR_n(rho, alpha) / dU_n(sigma, beta) = -(1/detJ_rho) [ sum_d Dc_d[rho][sigma] A_d(sigma)
//       + sum_g Cor[rho][g] M0[g][sigma] |N_g| dF/du_L (g) ]_{alpha beta}
// with A_d = sum_k S_dk df_k/du (eq. "transformed_quantities") and Dc_d =
// D_d - Cor diag(nref_d) M0 (the flux's own trace leaves through the
// correction, eq. "divergence_fr"); face blocks as described at MixD, with
// |N_g| dF/du_R.  The operators are staged once per call and the elements
// taken in tiles of mixed_tile<E>() (so that low degrees still occupy the
// workgroup); one thread per (element, rho, sigma) forms an NV x NV
// sub-block, so each operator coefficient is read once for NV^2 outputs, and
// zero coefficients (the sparse rows of tensor elements) are skipped.
template <class E> constexpr int mixed_tile() {
  return E::NS * E::NS >= 128 ? 1 : (E::NS * E::NS >= 64 ? 2 : (E::NS * E::NS >= 32 ? 4 : (E::NS * E::NS >= 16 ? 8 : 16)));
}
template <class E, class EO, int NV, class R> constexpr int jac_mixed_inv_lds() {
  constexpr int NS = E::NS, NF = E::NF, ND = E::ND, NFACE = E::NFACE, WC = E::WC, NV2 = NV * NV;
  constexpr int TE = mixed_tile<E>();
  return lds_bytes<R>(NF * NS) + lds_bytes<R>(NS * NF) + lds_bytes<R>(ND * NS * NS) + lds_bytes<int>(NS * WC) +
         lds_bytes<R>(NS * WC) + lds_bytes<R>(EO::NF * EO::NS) +
         TE * (lds_bytes<R>(ND * NS * NV2) + 2 * lds_bytes<R>(NF * NV2) + lds_bytes<R>(NS) +
               lds_bytes<R>(NS * ND * ND) + lds_bytes<R>(NS * NV) + 2 * lds_bytes<R>(NF * NV) +
               lds_bytes<R>(NF * ND) + lds_bytes<R>(NF) + lds_bytes<int>(NF) + lds_bytes<int>(NFACE) +
               lds_bytes<long>(NFACE + 1));
}

template <class E, class EO, int NV, int SYS, class R, class OT, class Sync>
FR_HD void jac_mixed_inv_body(int n0, int n1, int tid, int nth, char* lds, const OpsD<R>& op, const GeoD<R>& geo,
                              const MixD<R>& mx, const PhysP& ph, const R* U, const R* UF, OT* B, Sync sync) {
  constexpr int NS = E::NS, NF = E::NF, ND = E::ND, NFACE = E::NFACE, NFP = E::NFP, WL = E::WL, WC = E::WC;
  constexpr int NV2 = NV * NV, NSO = EO::NS, NFO = EO::NF, BB = NS * NV;
  constexpr int TE = mixed_tile<E>(), NSM = NS > NSO ? NS : NSO;
  typedef MDual<R, NV> MD;
  Lds L{lds};
  R* sM0 = L.take<R>(NF * NS);
  R* sCor = L.take<R>(NS * NF);
  R* sDc = L.take<R>(ND * NS * NS);     // Dc_d, dense
  int* scrc = L.take<int>(NS * WC);     // compressed rows of the correction
  R* scrv = L.take<R>(NS * WC);
  R* sM0o = L.take<R>(NFO * NSO);
  // per element of the tile
  R* ta = L.take<R>(TE * ND * NS * NV2);   // A_d(sigma)[alpha][beta]
  R* tL = L.take<R>(TE * NF * NV2);        // |N_g| dF/du_L (g)
  R* tR = L.take<R>(TE * NF * NV2);        // |N_g| dF/du_R (g)
  R* srd = L.take<R>(TE * NS);
  R* sS = L.take<R>(TE * NS * ND * ND);
  R* su = L.take<R>(TE * NS * NV);
  R* suL = L.take<R>(TE * NF * NV);
  R* suR = L.take<R>(TE * NF * NV);
  R* snn = L.take<R>(TE * NF * ND);
  R* smg = L.take<R>(TE * NF);
  int* spt = L.take<int>(TE * NF);
  int* snt = L.take<int>(TE * NFACE);
  long* sbo = L.take<long>(TE * (NFACE + 1));  // self block, then each face block
  for (int i = tid; i < NF * NS; i += nth) sM0[i] = op.M0[i];
  for (int i = tid; i < NS * NF; i += nth) sCor[i] = op.Cor[i];
  for (int i = tid; i < NFO * NSO; i += nth) sM0o[i] = mx.M0o[i];
  for (int i = tid; i < NS * WC; i += nth) { scrc[i] = op.crc[i]; scrv[i] = op.crv[i]; }
  for (int i = tid; i < ND * NS * NS; i += nth) sDc[i] = R(0);
  sync();
  // dense Dc_d from its compressed rows (one thread per row: no collisions)
  for (int i = tid; i < ND * NS; i += nth)
    for (int w = 0; w < WL; ++w) sDc[i * NS + op.dcc[i * WL + w]] += op.dcv[i * WL + w];
  for (long t0 = n0; t0 < n1; t0 += TE) {
    const int nte = (int)((n1 - t0) < TE ? (n1 - t0) : TE);
    for (int i = tid; i < nte * NS; i += nth) srd[i] = geo.rdet[t0 * NS + i];
    for (int i = tid; i < nte * NS * ND * ND; i += nth) sS[i] = geo.S[t0 * NS * ND * ND + i];
    for (int i = tid; i < nte * NS * NV; i += nth) su[i] = U[t0 * NS * NV + i];
    for (int i = tid; i < nte * NF * NV; i += nth) {
      const long fg = t0 * NF + i / NV;                 // the tile's flux points are contiguous
      const int a = i % NV;
      suL[i] = UF[fg * NV + a];
      suR[i] = UF[(long)geo.nbfp[fg] * NV + a];
    }
    for (int i = tid; i < nte * NF * ND; i += nth) snn[i] = geo.nrm[t0 * NF * ND + i];
    for (int i = tid; i < nte * NF; i += nth) { smg[i] = geo.magN[t0 * NF + i]; spt[i] = mx.nbpt[t0 * NF + i]; }
    for (int i = tid; i < nte * NFACE; i += nth) snt[i] = mx.nbt[t0 * NFACE + i];
    for (int i = tid; i < nte * (NFACE + 1); i += nth) {
      const int e = i / (NFACE + 1), k = i % (NFACE + 1);
      sbo[i] = k == 0 ? geo.boff[t0 + e] : mx.fboff[(t0 + e) * NFACE + k - 1];
    }
    sync();
    // pointwise flux derivatives: A_d at the solution points, the common
    // flux's derivatives with respect to either side at the flux points
#pragma unroll 1
    for (int it = tid; it < nte * (NS + 2 * NF); it += nth) {
      const int e = it / (NS + 2 * NF), j = it % (NS + 2 * NF);
      if (j < NS) {
        const int t = e * NS + j;
        MD u[NV], f[ND][NV];
        for (int a = 0; a < NV; ++a) { u[a] = MD(su[t * NV + a]); u[a].d[a] = R(1); }
        flux_inviscid<SYS, ND, NV, MD>(ph, u, f);
        for (int d = 0; d < ND; ++d)
          for (int a = 0; a < NV; ++a)
            for (int c = 0; c < NV; ++c) {
              R acc = R(0);
              for (int k = 0; k < ND; ++k) acc += sS[(t * ND + d) * ND + k] * f[k][a].d[c];
              ta[((e * ND + d) * NS + j) * NV2 + a * NV + c] = acc;
            }
      } else {
        const int g = e * NF + ((j - NS) >> 1), side = (j - NS) & 1;
        R nn[ND];
        for (int d = 0; d < ND; ++d) nn[d] = snn[g * ND + d];
        MD uL[NV], uR[NV], F[NV];
        for (int a = 0; a < NV; ++a) {
          uL[a] = MD(suL[g * NV + a]);
          uR[a] = MD(suR[g * NV + a]);
          (side ? uR : uL)[a].d[a] = R(1);
        }
        common_inviscid<SYS, ND, NV, MD>(ph, uL, uR, nn, F);
        R* o = side ? tR : tL;
        for (int a = 0; a < NV; ++a)
          for (int c = 0; c < NV; ++c) o[g * NV2 + a * NV + c] = smg[g] * F[a].d[c];
      }
    }
    sync();
    // self blocks
#pragma unroll 1
    for (int i = tid; i < nte * NS * NS; i += nth) {
      const int e = i / (NS * NS), r = i % NS, s = (i / NS) % NS;
      R acc[NV2];
      for (int k = 0; k < NV2; ++k) acc[k] = R(0);
      for (int d = 0; d < ND; ++d) {
        const R c = sDc[(d * NS + r) * NS + s];
        if (c != R(0))
          for (int k = 0; k < NV2; ++k) acc[k] += c * ta[((e * ND + d) * NS + s) * NV2 + k];
      }
#pragma unroll 1
      for (int w = 0; w < WC; ++w) {     // the non-zeros of row rho of the correction
        const int g = scrc[r * WC + w];
        const R c = scrv[r * WC + w] * sM0[g * NS + s];
        if (c != R(0))
          for (int k = 0; k < NV2; ++k) acc[k] += c * tL[(e * NF + g) * NV2 + k];
      }
      const R sc = -srd[e * NS + r];
      OT* Bn = B + sbo[e * (NFACE + 1)];
      for (int be = 0; be < NV; ++be) {
        R v[NV];
        for (int a = 0; a < NV; ++a) {
          v[a] = sc * acc[a * NV + be];
          if (!fr_finite(v[a])) fr_flag_nonfinite(geo.status, FR_NF_BLOCKS, geo.e0 + t0 + e);
        }
        store_rows<NV>(Bn + (long)(s * NV + be) * BB + r * NV, v);
      }
    }
    // face blocks, b_n x b_m
#pragma unroll 1
    for (int f = 0; f < NFACE; ++f) {
#pragma unroll 1
      for (int i = tid; i < nte * NS * NSM; i += nth) {
        const int e = i / (NS * NSM), r = i % NS, s = (i / NS) % NSM;
        const bool other = snt[e * NFACE + f] != 0;
        const int nsm = other ? NSO : NS;
        if (s >= nsm) continue;
        const R* M0m = other ? sM0o : sM0;
        R acc[NV2];
        for (int k = 0; k < NV2; ++k) acc[k] = R(0);
        for (int gi = 0; gi < NFP; ++gi) {
          const int g = f * NFP + gi;
          const R c = sCor[r * NF + g] * M0m[spt[e * NF + g] * nsm + s];
          if (c != R(0))
            for (int k = 0; k < NV2; ++k) acc[k] += c * tR[(e * NF + g) * NV2 + k];
        }
        const R sc = -srd[e * NS + r];
        OT* Bk = B + sbo[e * (NFACE + 1) + 1 + f];
        for (int be = 0; be < NV; ++be) {
          R v[NV];
          for (int a = 0; a < NV; ++a) {
            v[a] = sc * acc[a * NV + be];
            if (!fr_finite(v[a])) fr_flag_nonfinite(geo.status, FR_NF_BLOCKS, geo.e0 + t0 + e);
          }
          store_rows<NV>(Bk + (long)(s * NV + be) * BB + r * NV, v);
        }
      }
    }
    sync();      // the next tile's data overwrite the tables
  }
}
