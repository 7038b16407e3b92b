// Jacobian blocks of tensor-product elements on the matrix cores.
//
// For each variable pair (alpha, beta) the block is (FR method, eq.
// "divergence_fr", differentiated as in eq. "jacobian_rhs")
//   J = -rdet (.) ( sum_d Dc_d X_d + Cor Y ),
//   X_d[tau] = sum_k T_d[tau][k] G_k[tau]   (k: Gam_0 .. Gam_{ND-1}, delta),
//   Y[g]     = sum_j W[g][j] S_j[g]          (j: DL, DR, SL_d.., SR_d..),
// where T, W are the pointwise Jacobian tables (rows m: variable pairs) and
// G, S the sensitivities of the gradient and face states to U_k (columns
// sigma).  For fixed tau (or g) the contraction over k (or j) is a
// (pairs x k) . (k x sigma) product: one 16x16x4 MFMA per (tau, d) and one
// per group of four j at g.  The 1-D factors Dc1 (along the d-lines through
// tau) and h+- (along g's normal line) then scatter X and Y into 16x16
// accumulator tiles per solution point rho, as FMAs with compile-time
// indices (hexahedra: one slab of points per task; the factors of lines
// crossing the slab go into the A operand instead).
//
// Three kernels: the sensitivities G, S depend on the geometry only and are
// computed once per mesh (jac_mf_sens_body; their geometry-free rows are
// shared between blocks with the same face-point pairing); the tables T, W
// of a state are computed per element (jac_mf_tables_body); the assembly
// (jac_mf_task) runs one wavefront per (element, block, pair tile, sigma
// tile, slab) task, fetching four points' MFMA operands per 16-byte load
// and staging the finished tile through LDS for contiguous stores.
// BF16 blocks of degree-3 elements take BF16 operands instead
// (jac_mf_accum_bf16): each solution point's contributions of a family of
// lines are one 16x16x32 product with the 1-D weights folded into A.
#pragma once
#include <type_traits>

#include "fr_jac_tp.hpp"

template <class E, int NV, int SYS> struct MfSizes {
  static constexpr int ND = E::ND, NS = E::NS, NF = E::NF, NFACE = E::NFACE, NV2 = NV * NV;
  static constexpr int KV = ND + 1;                 // Gam_0 .. Gam_{ND-1}, delta
  static constexpr int JF = 2 + 2 * ND;             // DL, DR, SL_d.., SR_d..
  static constexpr int JC = (JF + 3) / 4;           // K chunks of the face product
  static constexpr int MT = (NV2 + 15) / 16, MP = 16 * MT;   // pair tiles
  static constexpr int NT = (NS + 15) / 16, NP = 16 * NT;    // sigma tiles
  static constexpr int NS4 = (NS + 3) / 4 * 4, NF4 = (NF + 3) / 4 * 4;   // padded to groups of four
  static constexpr int TBT = NS4 * ND * KV * MP;
  static constexpr int TFT = NF4 * JF * MP;
  static constexpr int GSZ = NS4 * KV * NP;         // per block: G
  static constexpr int SSZ = NF4 * JF * NP;         // per block: S
  // Operand layouts: the fragment element of four consecutive points (flux
  // points) is contiguous, so a lane fetches four MFMA operands with one
  // 16-byte load.  G[t][e][sigma], S[g][j][sigma], T[t][d][e][m], W[g][j][m]:
  static constexpr FR_HD int gi(int t, int e, int sg) { return ((t >> 2) * KV + e) * NP * 4 + sg * 4 + (t & 3); }
  static constexpr FR_HD int si(int g, int j, int sg) { return ((g >> 2) * JF + j) * NP * 4 + sg * 4 + (g & 3); }
  static constexpr FR_HD int ti(int t, int d, int e, int m) {
    return (((t >> 2) * ND + d) * KV + e) * MP * 4 + m * 4 + (t & 3);
  }
  static constexpr FR_HD int fi(int g, int j, int m) { return ((g >> 2) * JF + j) * MP * 4 + m * 4 + (g & 3); }
  static constexpr int BLK = GSZ + SSZ;             // sensitivities of one block
  static constexpr int TAB = TBT + TFT;             // tables of one element
  // Pair rows: a tile of 16 rows owns whole columns (every alpha of its
  // betas).  NV <= 4: m = alpha NV + beta, one tile; NV = 5: three betas per
  // tile, m = 16 (beta / 3) + 5 (beta % 3) + alpha.
  static constexpr int BT = NV <= 4 ? NV : 3;       // betas per pair tile
  static constexpr FR_HD int pidx(int a, int b) { return NV <= 4 ? a * NV + b : (b / 3) * 16 + (b % 3) * 5 + a; }
  static constexpr FR_HD bool pair(int m, int& a, int& b) {
    if (NV <= 4) { a = m / NV; b = m % NV; return m < NV2; }
    const int t = m / 16, l = m % 16;
    a = l % 5; b = 3 * t + l / 5;
    return l < 15 && b < NV;
  }
  // solution-point slabs of a task: hexahedra split along the third
  // coordinate (one accumulator tile per point of the slab)
  static constexpr int N1 = E::DEG + 1;
  static constexpr int SL = ND == 3 ? N1 : 1, SLS = NS / SL;
  static constexpr int TASKS = MT * NT * SL;       // tasks per (element, block)
  static constexpr int NR = SLS * NV;               // rows of a task's column segment
  // staged in NH passes of NRH rows (two where the halves stay whole points
  // and 16-byte multiples: half the LDS, more resident waves)
  static constexpr int NH = (SLS % 2 == 0 && (SLS / 2 * NV) % 4 == 0 && NR >= 32) ? 2 : 1, NRH = NR / NH;
};

template <class R> struct Mfma;
template <> struct Mfma<float> {
  typedef __attribute__((__vector_size__(4 * sizeof(float)))) float acc;
  static __device__ __forceinline__ acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // row of D held in accumulator r by lanes 16 q .. 16 q + 15
  static constexpr __device__ int row(int q, int r) { return 4 * q + r; }
};


// assembly tasks per workgroup and the LDS staging of one task's tile
template <class E, int NV, int SYS, class R> constexpr int jac_mf_stage() {
  typedef MfSizes<E, NV, SYS> Y;
  return 16 * Y::BT * (Y::NRH + 1);
}
// Resident waves per SIMD the register allocation aims for (degree 3: the
// largest counts these tasks reach without spilling; elsewhere the hint
// would only force spills).
template <class E, int NV, int SYS, class R, class OT> constexpr int jac_mf_min_waves() {
  if (std::is_same<OT, bf16_t>::value && E::DEG == 3) return 2;   // BF16 operands: two waves, no spills
  return E::DEG == 3 ? (E::ND == 3 ? 3 : 4) : 1;
}
// points (flux points) whose operands one load round trip fetches
template <class E, int NV, int SYS, class R> constexpr int jac_mf_chunk() {
  return (E::ND == 2 && E::DEG == 3) ? 8 : 16;   // quads p = 3: half the operand registers, a fourth wave
}
template <class E, int NV, int SYS, class R> constexpr int jac_mf_wpb() {
  return (4 * jac_mf_stage<E, NV, SYS, R>() * (int)sizeof(R) <= 72 * 1024) ? 4 : 2;
}

// LDS of the third-axis operands a workgroup of hexahedral BF16 tasks shares
template <class E, int NV, int SYS, class R, class OT> constexpr int jac_mf_xs_bytes() {
  return (std::is_same<OT, bf16_t>::value && std::is_same<R, float>::value && E::DEG == 3 && E::ND == 3)
             ? (4 * 4 * 4 * 16 * 4 + 2 * 2 * 4 * 4 * 16 * 4) * 4 + 4 * 4 * 4 * 16 * 16
             : 16;
}
template <class E, int NV, int SYS, class R> constexpr int jac_mf_sens_lds() {
  typedef TPSizes<E, NV, SYS> Z;
  typedef MfSizes<E, NV, SYS> Y;
  constexpr int NS = Z::NS, NF = Z::NF, ND = Z::ND, NFACE = Z::NFACE, NFP = Z::NFP;
  return lds_bytes<R>(NF * NS) + lds_bytes<R>(NS * NF) + lds_bytes<R>(NS * ND * ND) + lds_bytes<int>(NF) +
         lds_bytes<R>(NFACE * NS * ND * ND) + 2 * lds_bytes<int>(NFACE) + lds_bytes<R>(NFACE * NFP * ND) +
         lds_bytes<Ops1D<R>>(1) + (ND == 3 ? 0 : lds_bytes<R>((1 + NFACE) * Y::GSZ));
}
template <class E, int NV, int SYS, class R> constexpr int jac_mf_tables_lds() {
  typedef TPSizes<E, NV, SYS> Z;
  typedef MfSizes<E, NV, SYS> Y;
  constexpr int NS = Z::NS, NF = Z::NF, ND = Z::ND;
  return lds_bytes<R>(NS * NV) + lds_bytes<R>(NS * ND * NV) + 2 * lds_bytes<R>(NF * NV) +
         2 * lds_bytes<R>(NF * ND * NV) + 2 * lds_bytes<R>(NS * ND * ND) + lds_bytes<R>(NF * ND) + lds_bytes<R>(NF) +
         lds_bytes<int>(NF);
}

// Sensitivities of element n for all blocks (geometry only):
// out[k][G | S] (MfSizes::BLK values per block, operand layout).
template <class E, int NV, int SYS, class R>
__device__ void jac_mf_sens_body(int n, int tid, int nth, char* lds, const OpsD<R>& op, const Ops1D<R>& o1,
                                 const GeoD<R>& geo, const PhysP& ph, R* out, int nblk) {
  typedef TPSizes<E, NV, SYS> Z;
  typedef MfSizes<E, NV, SYS> Y;
  typedef TPIdx<E> X;
  constexpr int NS = Z::NS, NF = Z::NF, ND = Z::ND, NFACE = Z::NFACE, NFP = Z::NFP;
  constexpr int N1 = E::DEG + 1;
  constexpr int KV = Y::KV, JF = Y::JF, NP = Y::NP, BLK = Y::BLK;
  const bool visc = SysTraits<SYS>::kVisc && (SYS != SYS_ADV || ph.mu != 0.0);
  const R cb = R(0.5 + ph.beta);
  auto sync = []() { __syncthreads(); };
  Lds L{lds};
  R* sM0 = L.take<R>(NF * NS);
  R* sCor = L.take<R>(NS * NF);
  R* sJi = L.take<R>(NS * ND * ND);
  int* spg = L.take<int>(NF);
  R* sJm = L.take<R>(NFACE * NS * ND * ND);
  int* snb = L.take<int>(NFACE);
  int* snf = L.take<int>(NFACE);
  R* sW = L.take<R>(NFACE * NFP * ND);
  Ops1D<R>* sO1 = L.take<Ops1D<R>>(1);
  const long nl = n;
  R* gout = out + nl * nblk * BLK;
  // G of every block: in LDS where it fits, else read back from the output
  // (same workgroup, after a barrier)
  R* gamT = ND == 3 ? gout : L.take<R>((1 + NFACE) * Y::GSZ);
  constexpr int GST = ND == 3 ? BLK : Y::GSZ;
  for (int i = tid; i < NF * NS; i += nth) sM0[i] = op.M0[i];
  for (int i = tid; i < NS * NF; i += nth) sCor[i] = op.Cor[i];
  for (int i = tid; i < NF; i += nth) spg[i] = geo.nbfp[nl * NF + i];
  for (int i = tid; i < NS * ND * ND; i += nth) sJi[i] = geo.Jinv[nl * NS * ND * ND + i];
  for (int i = tid; i < NFACE; i += nth) { snb[i] = geo.nbr[nl * NFACE + i]; snf[i] = geo.nbface[nl * NFACE + i]; }
  for (int i = tid; i < (int)(sizeof(Ops1D<R>) / sizeof(R)); i += nth)
    reinterpret_cast<R*>(sO1)[i] = reinterpret_cast<const R*>(&o1)[i];
  sync();
  for (int i = tid; i < NFACE * NS * ND * ND; i += nth) {
    int f = i / (NS * ND * ND), r = i % (NS * ND * ND);
    sJm[i] = geo.Jinv[(long)snb[f] * NS * ND * ND + r];
  }
  sync();
  // W_d'(g): the neighbour's face gradient at g's partner w.r.t. u_n (same
  // face point only on tensor elements)
  if (visc)
    for (int i = tid; i < NFACE * NFP * ND; i += nth) {
      int f = i / (NFP * ND), gi = (i / ND) % NFP, d2 = i % ND;
      int g = f * NFP + gi;
      int g2 = spg[g] - snb[f] * NF;
      int f2 = g2 / NFP;
      int ax = X::fax(f2);
      R sg = R(X::fsg(f2));
      R acc = R(0);
      for (int w = 0; w < N1; ++w) {
        int t = X::fline(g2, w);
        acc += sM0[g2 * NS + t] * sCor[t * NF + g2] * sJm[((f * NS + t) * ND + ax) * ND + d2] * sg;
      }
      sW[i] = cb * acc;
    }
  sync();
  const int kb = 0, nbk = nblk;
    // G_e[tau][sigma] = d q~_e(tau) / d u_k(sigma); e = ND: delta (k = 0)
    for (int i = tid; i < nbk * NS * KV * NP; i += nth) {
      const int kk = i / (NS * KV * NP), t = (i / (KV * NP)) % NS, e = (i / NP) % KV, s = i % NP;
      const int k = kb + kk;
      R v = R(0);
      if (s < NS) {
        if (e == ND) {
          v = (k == 0 && t == s) ? R(1) : R(0);
        } else if (visc) {
          if (k == 0) {
            bool on = true;
            for (int d = 0; d < ND; ++d)
              if (d != e && X::co(t, d) != X::co(s, d)) on = false;
            if (on) v = sO1->G1[X::co(t, e)][X::co(s, e)];
          } else {
            const int f = k - 1, m = snb[f];
            if (X::fax(f) == e) {
              // cb sum_{g on f} Cor[tau][g] nref_e(g) M0_m[P(g)][sigma]
              for (int gi = 0; gi < NFP; ++gi) {
                const int g = f * NFP + gi;
                const R c = sCor[t * NF + g];
                if (c != R(0)) v += c * R(X::fsg(f)) * sM0[(spg[g] - m * NF) * NS + s];
              }
              v *= cb;
            }
          }
        }
      }
      if (ND != 3) gamT[kk * Y::GSZ + (t * KV + e) * NP + s] = v;
      gout[kk * BLK + Y::gi(t, e, s)] = v;
    }
    sync();
    // S_j[g][sigma]: DL, DR (face values), SL_d', SR_d' (own / neighbour
    // physical face gradients)
    for (int i = tid; i < nbk * NF * NP; i += nth) {
      const int kk = i / (NF * NP), g = (i / NP) % NF, s = i % NP;
      const int k = kb + kk;
      R* o = gout + kk * BLK + Y::GSZ;
      const int fg = g / NFP;
      R dl = R(0), dr = R(0);
      if (s < NS) {
        if (k == 0) dl = sM0[g * NS + s];
        else if (fg == k - 1) dr = sM0[(spg[g] - snb[fg] * NF) * NS + s];
      }
      o[Y::si(g, 0, s)] = dl;
      o[Y::si(g, 1, s)] = dr;
      for (int d2 = 0; d2 < ND; ++d2) {
        R sl = R(0), sr = R(0);
        if (visc && s < NS) {
          for (int w = 0; w < N1; ++w) {
            const int t = X::fline(g, w);
            R acc = R(0);
            for (int e = 0; e < ND; ++e)
              acc += sJi[(t * ND + e) * ND + d2] *
                     gamT[kk * GST + (ND == 3 ? Y::gi(t, e, s) : (t * KV + e) * NP + s)];
            sl += sM0[g * NS + t] * acc;
          }
          if (k == 0) {
            sr = sW[g * ND + d2] * sM0[g * NS + s];
          } else if (fg == k - 1) {
            const int g2 = spg[g] - snb[fg] * NF;
            for (int w = 0; w < N1; ++w) {
              const int t = X::fline(g2, w);
              R acc = R(0);
              for (int e = 0; e < ND; ++e) {
                bool on = true;
                for (int d = 0; d < ND; ++d)
                  if (d != e && X::co(t, d) != X::co(s, d)) on = false;
                if (on) acc += sJm[((fg * NS + t) * ND + e) * ND + d2] * sO1->G1[X::co(t, e)][X::co(s, e)];
              }
              sr += sM0[g2 * NS + t] * acc;
            }
          }
        }
        o[Y::si(g, 2 + d2, s)] = sl;
        o[Y::si(g, 2 + ND + d2, s)] = sr;
      }
    }
    sync();
}

// Pointwise Jacobian tables of element n at the state:
// out[n][T | W] (MfSizes::TAB values, operand layout).
template <class E, int NV, int SYS, class R>
__device__ void jac_mf_tables_body(int n, int tid, int nth, char* lds, const GeoD<R>& geo, const PhysP& ph,
                                   const R* U, const R* Q, const R* UF, const R* QF, R* out) {
  typedef TPSizes<E, NV, SYS> Z;
  typedef MfSizes<E, NV, SYS> Y;
  constexpr int NS = Z::NS, NF = Z::NF, ND = Z::ND, NV2 = Z::NV2;
  constexpr int KV = Y::KV, JF = Y::JF, MP = Y::MP;
  const bool visc = SysTraits<SYS>::kVisc && (SYS != SYS_ADV || ph.mu != 0.0);
  const R cL = R(0.5 + ph.beta), cR = R(0.5 - ph.beta), eta = R(ph.eta);
  auto sync = []() { __syncthreads(); };
  Lds L{lds};
  R* su = L.take<R>(NS * NV);
  R* sq = L.take<R>(NS * ND * NV);
  R* suL = L.take<R>(NF * NV);
  R* suR = L.take<R>(NF * NV);
  R* sqL = L.take<R>(NF * ND * NV);
  R* sqR = L.take<R>(NF * ND * NV);
  R* sJi = L.take<R>(NS * ND * ND);
  R* sS = L.take<R>(NS * ND * ND);
  R* snn = L.take<R>(NF * ND);
  R* smg = L.take<R>(NF);
  int* spg = L.take<int>(NF);
  const long nl = n;
  R* tbT = out + nl * Y::TAB;
  R* tfT = tbT + Y::TBT;
  // The blocks are sums of products of these tables with the finite
  // geometric sensitivities, so a non-finite block entry can only come from
  // a non-finite table entry: they are recorded here, once per element,
  // rather than at every block store.
  bool bad = false;
  for (int i = tid; i < NS * NV; i += nth) su[i] = U[nl * NS * NV + i];
  if (visc)
    for (int i = tid; i < NS * ND * NV; i += nth) sq[i] = Q[nl * NS * ND * NV + i];
  for (int i = tid; i < NF; i += nth) { spg[i] = geo.nbfp[nl * NF + i]; smg[i] = geo.magN[nl * NF + i]; }
  for (int i = tid; i < NS * ND * ND; i += nth) { sJi[i] = geo.Jinv[nl * NS * ND * ND + i]; sS[i] = geo.S[nl * NS * ND * ND + i]; }
  for (int i = tid; i < NF * ND; i += nth) snn[i] = geo.nrm[nl * NF * ND + i];
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
  sync();
  // ---------------------------------------------------------------- tables
  // Each item evaluates with single-tangent duals every seeded input that
  // its table entries combine, and writes them directly (no intermediates):
  //   solution point (tau, c), kind 0: u_c seeded: transformed inviscid +
  //     viscous flux derivatives -> T[tau][d][delta];
  //   kind 1 (viscous): q_{d2,c} seeded for each d2, contracted with S and
  //     J^-1 -> T[tau][d][Gam_e];
  //   flux point (g, c), kind 0 / 1: u_c seeded on side L / R: common
  //     convective flux + that side's viscous flux -> W[g][DL] / W[g][DR];
  //   kinds 2 .. 1 + 2 N_D (viscous): q_{d,c} seeded on side L, then R ->
  //     W[g][SL_d] / W[g][SR_d].
  // Items run kind-major (kind, point, c), so a wavefront takes one path.
  {
    typedef Dual<R> DT;
    const int nsk = visc ? 2 : 1, nfk = visc ? 2 + 2 * ND : 2;
    const int nsi = NS * NV * nsk, ntot = nsi + NF * NV * nfk;
    for (int it = tid; it < ntot; it += nth) {
      if (it < nsi) {
        const int kind = it / (NS * NV), r = it % (NS * NV), t = r / NV, c = r % NV;
        DT u[NV];
        for (int a = 0; a < NV; ++a) u[a] = DT(su[t * NV + a], (kind == 0 && a == c) ? R(1) : R(0));
        if (kind == 0) {
          DT f[ND][NV], q[ND][NV];
          for (int d = 0; d < ND; ++d)
            for (int a = 0; a < NV; ++a) q[d][a] = DT(visc ? sq[(t * ND + d) * NV + a] : R(0), R(0));
          flux_inviscid<SYS, ND, NV, DT>(ph, u, f);
          if (visc) {
            DT fv[ND][NV];
            flux_viscous<SYS, ND, NV, DT>(ph, u, q, fv);
            for (int d = 0; d < ND; ++d)
              for (int a = 0; a < NV; ++a) f[d][a] += fv[d][a];
          }
          for (int a = 0; a < NV; ++a)
            for (int d = 0; d < ND; ++d) {
              R acc = R(0);
              for (int k = 0; k < ND; ++k) acc += sS[(t * ND + d) * ND + k] * f[k][a].d;
              tbT[Y::ti(t, d, ND, Y::pidx(a, c))] = acc;
              bad |= !fr_finite(acc);
            }
        } else {
          R bq[ND][ND][NV];   // d f^k_a / d q_{d2,c}
          for (int d2 = 0; d2 < ND; ++d2) {
            DT q[ND][NV], f[ND][NV];
            for (int d = 0; d < ND; ++d)
              for (int a = 0; a < NV; ++a) q[d][a] = DT(sq[(t * ND + d) * NV + a], (d == d2 && a == c) ? R(1) : R(0));
            flux_viscous<SYS, ND, NV, DT>(ph, u, q, f);
            for (int k = 0; k < ND; ++k)
              for (int a = 0; a < NV; ++a) bq[d2][k][a] = f[k][a].d;
          }
          for (int a = 0; a < NV; ++a)
            for (int d = 0; d < ND; ++d)
              for (int e = 0; e < ND; ++e) {
                R acc = R(0);
                for (int k = 0; k < ND; ++k) {
                  R sk = sS[(t * ND + d) * ND + k];
                  for (int d2 = 0; d2 < ND; ++d2) acc += sk * bq[d2][k][a] * sJi[(t * ND + e) * ND + d2];
                }
                tbT[Y::ti(t, d, e, Y::pidx(a, c))] = acc;
                bad |= !fr_finite(acc);
              }
        }
      } else {
        const int j = it - nsi, kind = j / (NF * NV), r = j % (NF * NV), g = r / NV, c = r % NV;
        R nn[ND];
        for (int d = 0; d < ND; ++d) nn[d] = snn[g * ND + d];
        const R mg = smg[g];
        if (kind < 2) {
          const int side = kind;
          DT uL[NV], uR[NV], F[NV];
          for (int a = 0; a < NV; ++a) {
            uL[a] = DT(suL[g * NV + a], (side == 0 && a == c) ? R(1) : R(0));
            uR[a] = DT(suR[g * NV + a], (side == 1 && a == c) ? R(1) : R(0));
          }
          common_inviscid<SYS, ND, NV, DT>(ph, uL, uR, nn, F);
          R vs[NV];
          for (int a = 0; a < NV; ++a) vs[a] = R(0);
          if (visc) {
            const R* us = side ? suR : suL;
            const R* qs = side ? sqR : sqL;
            DT u[NV], q[ND][NV], fv[ND][NV];
            for (int a = 0; a < NV; ++a) u[a] = DT(us[g * NV + a], a == c ? R(1) : R(0));
            for (int d = 0; d < ND; ++d)
              for (int a = 0; a < NV; ++a) q[d][a] = DT(qs[(g * ND + d) * NV + a], R(0));
            flux_viscous<SYS, ND, NV, DT>(ph, u, q, fv);
            const R wgt = side ? cR : cL;
            for (int a = 0; a < NV; ++a) {
              R acc = R(0);
              for (int d = 0; d < ND; ++d) acc += nn[d] * fv[d][a].d;
              vs[a] = acc * wgt;
            }
          }
          for (int a = 0; a < NV; ++a) {
            const int m = Y::pidx(a, c);
            const R id = (a == c) ? eta : R(0);
            const R w = mg * (F[a].d + (visc ? (side == 0 ? vs[a] + id : vs[a] - id) : R(0)));
            tfT[Y::fi(g, side, m)] = w;
            bad |= !fr_finite(w);
            if (!visc)
              for (int d = 0; d < ND; ++d) tfT[Y::fi(g, 2 + side * ND + d, m)] = R(0);
          }
        } else {
          const int side = (kind - 2) / ND, qd = (kind - 2) % ND;
          const R* us = side ? suR : suL;
          const R* qs = side ? sqR : sqL;
          DT u[NV], q[ND][NV], fv[ND][NV];
          for (int a = 0; a < NV; ++a) u[a] = DT(us[g * NV + a], R(0));
          for (int d = 0; d < ND; ++d)
            for (int a = 0; a < NV; ++a) q[d][a] = DT(qs[(g * ND + d) * NV + a], (qd == d && a == c) ? R(1) : R(0));
          flux_viscous<SYS, ND, NV, DT>(ph, u, q, fv);
          const R wgt = side ? cR : cL;
          for (int a = 0; a < NV; ++a) {
            R acc = R(0);
            for (int d = 0; d < ND; ++d) acc += nn[d] * fv[d][a].d;
            acc *= wgt;
            tfT[Y::fi(g, 2 + side * ND + qd, Y::pidx(a, c))] = mg * acc;
            bad |= !fr_finite(mg * acc);
          }
        }
      }
    }
    if (!visc)
      for (int i = tid; i < NV2 * NS * ND; i += nth) {
        const int ab = i / (NS * ND), r = i % (NS * ND);
        for (int e = 0; e < ND; ++e) tbT[Y::ti(r / ND, r % ND, e, Y::pidx(ab / NV, ab % NV))] = R(0);
      }
    sync();
  }
  if (bad) fr_flag_nonfinite(geo.status, FR_NF_BLOCKS, geo.e0 + nl);
}

// Compile-time loop: f(std::integral_constant<int, i>) for i in [B, E).
template <int B, int E, class F> __device__ __forceinline__ void mf_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    mf_for<B + 1, E>(f);
  }
}

// Four consecutive operand values (16-byte aligned) in one load.
template <class R> __device__ __forceinline__ void mf_ld4(const R* p, R& a, R& b, R& c, R& d) {
  if constexpr (std::is_same<R, float>::value) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    a = v.x; b = v.y; c = v.z; d = v.w;
  } else {
    a = p[0]; b = p[1]; c = p[2]; d = p[3];
  }
}

// Loads of a chunk of CNT points whose first point is congruent to B4 mod 4
// (B4 < 0: unknown): a group of four that starts on a multiple of four and
// lies inside the chunk is one 16-byte load (four(i) for its first point i),
// every other point a scalar load (one(i)).
template <int CNT, int B4, class L1, class L4> __device__ __forceinline__ void mf_chunk(L1&& one, L4&& four) {
  mf_for<0, CNT>([&](auto I) __attribute__((always_inline)) {
    constexpr int i = decltype(I)::value;
    constexpr int ph = B4 < 0 ? -1 : (B4 + i) % 4;            // position in its group of four
    constexpr bool start = ph == 0 && i + 3 < CNT;
    constexpr bool inside = ph > 0 && i - ph >= 0 && i - ph + 3 < CNT;
    if constexpr (start) four(I);
    else if constexpr (!inside) one(I);
  });
}

// Marks v as read and rewritten here (no instruction): updates of v are
// computed before this point instead of being sunk towards their last use.
template <class A> __device__ __forceinline__ void mf_pin(A& v) { asm volatile("" : "+v"(v)); }

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 mf_bf16x8;

// BF16 blocks of degree-3 elements: BF16 operands on the 16x16x32 matrix
// instruction, FP32 accumulation.  Its K = 32 holds every term one solution
// point rho of the slab receives from a family of lines through it, with the
// 1-D weight folded into the A operand, so nothing is scattered afterwards:
//   1. the in-slab volume terms, sum_s Dc1[x][s] X_0[(s, y)] + Dc1[y][s] X_1[(x, s)];
//   2. the in-slab faces, h+-(x) Y at both ends of rho's first-axis normal
//      line and h+-(y) Y at both ends of its second-axis line;
//   3. (hexahedra) the third-axis volume terms sum_c Dc1[z0][c] X_2[(x, y, c)]
//      and both third-axis faces, h+-(z0) Y[(x, y)].
// Lane group q = lane / 16 holds K entries 8 q .. 8 q + 7: the operand index
// e = q of the 16x16x4 form (Gam_e / delta; face rows j = q and 4 + q) at
// eight points, so the lanes load exactly the values of the FP32 form.
template <class E, int NV, int SYS>
__device__ __forceinline__ void jac_mf_accum_bf16(int z0, int kq, int mo, int so, const float (&dc)[4][4],
                                                  const float (&hp)[4], const float (&hm)[4], const float* G,
                                                  const float* tbT, const float* tfT, const float* Sr,
                                                  const float* S, char* xs, typename Mfma<float>::acc* V) {
  typedef MfSizes<E, NV, SYS> Y;
  typedef TPIdx<E> X;
  constexpr int ND = Y::ND, N1 = 4, SLS = Y::SLS, KV = Y::KV, JF = Y::JF, NFP = E::NFP;
  static_assert(E::DEG == 3 && SLS == 16, "degree-3 elements, slabs of 16 points");
  const int R0 = z0 * SLS;
  const bool kin = kq < KV;
  auto sface = [](int ax, bool pos) constexpr {   // in-slab face of axis ax, side pos
    int f = 0;
    for (int q = 0; q < E::NFACE; ++q)
      if (X::fax(q) == ax && (X::fsg(q) > 0) == pos) f = q;
    return f;
  };
  // flux point (face-local, slab-relative) of face f on rho's ax-line
  auto ta_of = [](int f, int ax, int rho) constexpr {
    int r = -1;
    for (int ta = 0; ta < N1; ++ta)
      if (X::fline(f * NFP + ta, X::co(rho, ax)) == rho) r = ta;
    return r;
  };
  float gv[SLS], tv[2][SLS];                      // 1: G, T_0, T_1 of the slab points
  float fa[2][2][2][N1], fb[2][2][2][N1];         // 2: W, S at the in-slab faces [axis][side][chunk][ta]
  auto load1 = [&]() __attribute__((always_inline)) {
    mf_for<0, SLS / 4>([&](auto Q) __attribute__((always_inline)) {
      constexpr int i = 4 * decltype(Q)::value;
      const int t = R0 + i;
      if (kin) {
        mf_ld4(G + Y::gi(t, kq, so), gv[i], gv[i + 1], gv[i + 2], gv[i + 3]);
        mf_ld4(tbT + Y::ti(t, 0, kq, mo), tv[0][i], tv[0][i + 1], tv[0][i + 2], tv[0][i + 3]);
        mf_ld4(tbT + Y::ti(t, 1, kq, mo), tv[1][i], tv[1][i + 1], tv[1][i + 2], tv[1][i + 3]);
      } else {
        gv[i] = gv[i + 1] = gv[i + 2] = gv[i + 3] = 0.f;
        tv[0][i] = tv[0][i + 1] = tv[0][i + 2] = tv[0][i + 3] = 0.f;
        tv[1][i] = tv[1][i + 1] = tv[1][i + 2] = tv[1][i + 3] = 0.f;
      }
    });
  };
  auto load2 = [&]() __attribute__((always_inline)) {
    mf_for<0, 4>([&](auto AS) __attribute__((always_inline)) {
      constexpr int ax = decltype(AS)::value / 2, sd = decltype(AS)::value % 2, f = sface(ax, sd == 1);
      const int g = f * NFP + (ND == 3 ? N1 * z0 : 0);
      mf_for<0, 2>([&](auto CC) __attribute__((always_inline)) {
        constexpr int ch = decltype(CC)::value;
        const int j = ch * 4 + kq;
        if (j < JF) {
          mf_ld4(tfT + Y::fi(g, j, mo), fa[ax][sd][ch][0], fa[ax][sd][ch][1], fa[ax][sd][ch][2], fa[ax][sd][ch][3]);
          mf_ld4((j < 2 ? Sr : S) + Y::si(g, j, so), fb[ax][sd][ch][0], fb[ax][sd][ch][1], fb[ax][sd][ch][2],
                 fb[ax][sd][ch][3]);
        } else {
          fa[ax][sd][ch][0] = fa[ax][sd][ch][1] = fa[ax][sd][ch][2] = fa[ax][sd][ch][3] = 0.f;
          fb[ax][sd][ch][0] = fb[ax][sd][ch][1] = fb[ax][sd][ch][2] = fb[ax][sd][ch][3] = 0.f;
        }
      });
    });
  };
  // 1. volume, in-slab directions
  auto comp1 = [&]() __attribute__((always_inline)) {
    mf_for<0, SLS>([&](auto P) __attribute__((always_inline)) {
      constexpr int rho = decltype(P)::value, cx = X::co(rho, 0), cy = X::co(rho, 1);
      mf_bf16x8 a, b;
      mf_for<0, N1>([&](auto Sx) __attribute__((always_inline)) {
        constexpr int sx = decltype(Sx)::value, tx = X::line(rho, 0, sx), ty = X::line(rho, 1, sx);
        a[sx] = (__bf16)(dc[cx][sx] * tv[0][tx]);
        a[4 + sx] = (__bf16)(dc[cy][sx] * tv[1][ty]);
        b[sx] = (__bf16)gv[tx];
        b[4 + sx] = (__bf16)gv[ty];
      });
      V[rho] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, V[rho], 0, 0, 0);
    });
  };
  // 2. faces whose normal lines lie in the slab: both ends of rho's lines
  auto comp2 = [&]() __attribute__((always_inline)) {
    mf_for<0, SLS>([&](auto P) __attribute__((always_inline)) {
      constexpr int rho = decltype(P)::value;
      mf_bf16x8 a, b;
      mf_for<0, 8>([&](auto I) __attribute__((always_inline)) {
        constexpr int i = decltype(I)::value, ax = i / 4, sd = (i / 2) % 2, ch = i % 2;
        constexpr int f = sface(ax, sd == 1), ta = ta_of(f, ax, rho), w = X::co(rho, ax);
        static_assert(ta >= 0, "every slab point lies on a normal line of each in-slab face");
        a[i] = (__bf16)((sd == 1 ? hp[w] : hm[w]) * fa[ax][sd][ch][ta]);
        b[i] = (__bf16)fb[ax][sd][ch][ta];
      });
      V[rho] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, V[rho], 0, 0, 0);
    });
  };
  if constexpr (ND == 2) {
    load1();
    load2();
    fr_sched_fence();
    comp1();
    fr_sched_fence();
    comp2();
    fr_sched_fence();
  } else {
    // 3. third axis, volume and faces, one row of the slab (four points) at
    // a time
    float wz[N1], hzm = hm[0], hzp = hp[0];
    mf_for<0, N1>([&](auto Cc) __attribute__((always_inline)) {
      constexpr int c = decltype(Cc)::value;
      wz[c] = dc[0][c];
      mf_for<1, N1>([&](auto Z) __attribute__((always_inline)) {
        if (z0 == decltype(Z)::value) wz[c] = dc[decltype(Z)::value][c];
      });
    });
    mf_for<1, N1>([&](auto Z) __attribute__((always_inline)) {
      if (z0 == decltype(Z)::value) { hzp = hp[decltype(Z)::value]; hzm = hm[decltype(Z)::value]; }
    });
    constexpr int fzm = 0, fzp = 5;
    static_assert(X::fax(fzm) == 2 && X::fsg(fzm) < 0 && X::fax(fzp) == 2 && X::fsg(fzp) > 0, "third-axis faces");
    mf_for<0, SLS>([&](auto Tq) __attribute__((always_inline)) {
      constexpr int t = decltype(Tq)::value;
      static_assert(X::fline(fzm * NFP + t, 0) % SLS == t && X::fline(fzp * NFP + t, 0) % SLS == t,
                    "third-axis flux point t lies over slab point t");
    });
    // The four waves of a workgroup are the four slabs of one (element,
    // block, pair tile, sigma tile) and read the same third-axis operands:
    // each loads one row of them into LDS; A operands stay FP32 (their
    // weights depend on the slab), B operands are stored as packed BF16.
    static_assert(jac_mf_wpb<E, NV, SYS, float>() == Y::SL, "one workgroup = the slabs of one task column");
    static_assert(KV == 4 && JF == 8, "hexahedra: every lane group holds an operand index and face rows");
    float* xT = reinterpret_cast<float*>(xs);                 // [c][y][e][m][x]
    float* xW = xT + N1 * N1 * 4 * 16 * 4;                    // [side][chunk][y][e][m][x]
    mf_bf16x8* xB = reinterpret_cast<mf_bf16x8*>(xW + 2 * 2 * N1 * 4 * 16 * 4);   // [y][x][e][sigma]
    const int li = so & 15;
    load1();
    load2();
    fr_sched_fence();
    comp1();
    fr_sched_fence();
    {
      const int r0 = N1 * z0;                                  // this wave's row: slab points r0 .. r0 + 3
      float tz[N1][4], gz[N1][4], za[2][2][4], zb[2][2][4];
      mf_for<0, N1>([&](auto Cc) __attribute__((always_inline)) {
        constexpr int c = decltype(Cc)::value;
        const int t = c * SLS + r0;
        mf_ld4(G + Y::gi(t, kq, so), gz[c][0], gz[c][1], gz[c][2], gz[c][3]);
        mf_ld4(tbT + Y::ti(t, 2, kq, mo), tz[c][0], tz[c][1], tz[c][2], tz[c][3]);
      });
      mf_for<0, 4>([&](auto FC) __attribute__((always_inline)) {
        constexpr int sd = decltype(FC)::value / 2, ch = decltype(FC)::value % 2;
        const int g = (sd ? fzp : fzm) * NFP + r0;
        const int j = ch * 4 + kq;   // JF = 8: every j is a face row
        mf_ld4(tfT + Y::fi(g, j, mo), za[sd][ch][0], za[sd][ch][1], za[sd][ch][2], za[sd][ch][3]);
        mf_ld4((j < 2 ? Sr : S) + Y::si(g, j, so), zb[sd][ch][0], zb[sd][ch][1], zb[sd][ch][2], zb[sd][ch][3]);
      });
      fr_sched_fence();
      comp2();
      fr_sched_fence();
      mf_for<0, N1>([&](auto Cc) __attribute__((always_inline)) {
        constexpr int c = decltype(Cc)::value;
        *reinterpret_cast<float4*>(xT + (((c * N1 + z0) * 4 + kq) * 16 + li) * 4) =
            make_float4(tz[c][0], tz[c][1], tz[c][2], tz[c][3]);
      });
      mf_for<0, 4>([&](auto FC) __attribute__((always_inline)) {
        constexpr int sd = decltype(FC)::value / 2, ch = decltype(FC)::value % 2;
        *reinterpret_cast<float4*>(xW + ((((sd * 2 + ch) * N1 + z0) * 4 + kq) * 16 + li) * 4) =
            make_float4(za[sd][ch][0], za[sd][ch][1], za[sd][ch][2], za[sd][ch][3]);
      });
      mf_for<0, 4>([&](auto Xc) __attribute__((always_inline)) {
        constexpr int x = decltype(Xc)::value;
        mf_bf16x8 b;
        mf_for<0, N1>([&](auto Cc) __attribute__((always_inline)) {
          b[decltype(Cc)::value] = (__bf16)gz[decltype(Cc)::value][x];
        });
        mf_for<0, 4>([&](auto FC) __attribute__((always_inline)) {
          constexpr int sd = decltype(FC)::value / 2, ch = decltype(FC)::value % 2;
          b[4 + 2 * sd + ch] = (__bf16)zb[sd][ch][x];
        });
        xB[((z0 * 4 + x) * 4 + kq) * 16 + li] = b;
      });
    }
    __syncthreads();
    mf_for<0, N1>([&](auto Yr) __attribute__((always_inline)) {
      constexpr int y = decltype(Yr)::value, r0 = N1 * y;
      float tz[N1][4], za[2][2][4];
      mf_for<0, N1>([&](auto Cc) __attribute__((always_inline)) {
        constexpr int c = decltype(Cc)::value;
        const float4 v = *reinterpret_cast<const float4*>(xT + (((c * N1 + y) * 4 + kq) * 16 + li) * 4);
        tz[c][0] = v.x; tz[c][1] = v.y; tz[c][2] = v.z; tz[c][3] = v.w;
      });
      mf_for<0, 4>([&](auto FC) __attribute__((always_inline)) {
        constexpr int sd = decltype(FC)::value / 2, ch = decltype(FC)::value % 2;
        const float4 v = *reinterpret_cast<const float4*>(xW + ((((sd * 2 + ch) * N1 + y) * 4 + kq) * 16 + li) * 4);
        za[sd][ch][0] = v.x; za[sd][ch][1] = v.y; za[sd][ch][2] = v.z; za[sd][ch][3] = v.w;
      });
      mf_for<0, 4>([&](auto Xc) __attribute__((always_inline)) {
        constexpr int x = decltype(Xc)::value;
        const mf_bf16x8 b = xB[((y * 4 + x) * 4 + kq) * 16 + li];
        mf_bf16x8 a;
        mf_for<0, N1>([&](auto Cc) __attribute__((always_inline)) {
          constexpr int c = decltype(Cc)::value;
          a[c] = (__bf16)(wz[c] * tz[c][x]);
        });
        mf_for<0, 4>([&](auto FC) __attribute__((always_inline)) {
          constexpr int sd = decltype(FC)::value / 2, ch = decltype(FC)::value % 2;
          a[4 + 2 * sd + ch] = (__bf16)((sd ? hzp : hzm) * za[sd][ch][x]);
        });
        V[r0 + x] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, V[r0 + x], 0, 0, 0);
      });
      fr_sched_fence();
    });
  }
}

// One wavefront task: element n, block k, pair tile mt, sigma tile nt and
// solution-point slab z0 (points whose third coordinate is z0; the whole
// element for quadrilaterals).  MFMA fragments: A[m][k] from lane (m = lane %
// 16, k = lane / 16), B[k][n] from lane (k = lane / 16, n = lane % 16);
// D[i][lane % 16] in accumulator r with i = Mfma<R>::row(lane / 16, r)
// (FP32: 4 (lane / 16) + r, FP64: lane / 16 + 4 r).
//
// The slab is a run-time (wave-uniform) value: one code path serves every
// slab, so the unrolled task stays within the instruction cache.  Indices
// into the accumulators are compile-time throughout: slab-relative for the
// point sets that move with z0 (their operands are loaded at a uniform
// run-time offset), and slab-independent for the third-axis lines, whose
// slab-dependent weight goes into the A operand instead.
template <class E, int NV, int SYS, class R, class OT>
__device__ __forceinline__ void jac_mf_task(int n, int k, int mt, int nt, int z0, int lane, const Ops1D<R>& o1,
                                            const R* rdet, const R* tab, const R* sens, const R* sigtab,
                                            const int* sig, int nsb, int nblk, OT* B, R* stage, char* xs,
                                            bool active) {
  typedef MfSizes<E, NV, SYS> Y;
  typedef TPIdx<E> X;
  typedef Mfma<R> M;
  typedef typename M::acc acc;
  constexpr int NS = Y::NS, ND = Y::ND, NF = Y::NF, NFP = E::NFP, N1 = E::DEG + 1;
  constexpr int KV = Y::KV, JF = Y::JF, JC = Y::JC, MP = Y::MP, NP = Y::NP, BB = NS * NV;
  constexpr int SLS = Y::SLS;
  const int R0 = z0 * SLS;                 // the slab's points R0 .. R0 + SLS - 1
  const int li = lane & 15, kq = lane >> 4;
  const long nl = n;
  const R* tbT = tab + nl * Y::TAB;
  const R* tfT = tbT + Y::TBT;
  // the block's reference rows (G; face values DL, DR) from its shared
  // copy, the geometric rows (face gradients SL, SR) from its own
  const R* G = sigtab + (long)sig[nl * nsb + k] * Y::BLK;
  const R* Sr = G + Y::GSZ;
  const R* S = sens + (nl * nsb + k) * Y::BLK + Y::GSZ;
  const R* srd = rdet + nl * NS;
  // the few 1-D coefficients the task uses, as scalars (indexing the
  // by-value operator struct directly keeps a private copy of it alive)
  R dc[N1][N1], hp[N1], hm[N1];
  mf_for<0, N1>([&](auto W) __attribute__((always_inline)) {
    constexpr int w = decltype(W)::value;
    hp[w] = o1.hp[w];
    hm[w] = o1.hm[w];
    mf_for<0, N1>([&](auto C) __attribute__((always_inline)) { dc[w][decltype(C)::value] = o1.Dc1[w][decltype(C)::value]; });
  });
  const acc zero = {};
  acc V[SLS];
#pragma unroll
  for (int r = 0; r < SLS; ++r) V[r] = zero;
  // lane offsets of the A (pair) and B (sigma) fragments
  const int mo = mt * 16 + li, so = nt * 16 + li;   // this lane's pair row and sigma column
  const bool kin = kq < KV;
  constexpr bool kBf16Mfma = std::is_same<OT, bf16_t>::value && std::is_same<R, float>::value && E::DEG == 3;
  if constexpr (kBf16Mfma) {
    jac_mf_accum_bf16<E, NV, SYS>(z0, kq, mo, so, dc, hp, hm, G, tbT, tfT, Sr, S, xs, V);
  } else {
  // Operands come straight from global memory: each chunk of up to 16
  // points (or flux points) issues its fragment loads at once (one memory
  // round trip), then computes; chunks bound the live registers.  After each
  // point the updated accumulators are pinned: without that, instruction
  // selection sinks every update to the final store and keeps each product
  // of the task live.
  constexpr int CH = jac_mf_chunk<E, NV, SYS, R>();
  constexpr int NDS = ND == 3 ? 2 : ND;    // directions whose lines lie in the slab
  // volume, in-slab directions: X_d[tau] (tau in the slab) scattered along
  // the d-line through tau
  mf_for<0, (SLS + CH - 1) / CH>([&](auto C) __attribute__((always_inline)) {
    constexpr int t0 = decltype(C)::value * CH;
    R bv[CH], av[NDS][CH];
    constexpr int CNT = (SLS - t0) < CH ? (SLS - t0) : CH;
    mf_chunk<CNT, (ND == 2 || SLS % 4 == 0) ? 0 : -1>(
        [&](auto I) __attribute__((always_inline)) {
          constexpr int i = decltype(I)::value;
          const int t = R0 + t0 + i;
          bv[i] = kin ? G[Y::gi(t, kq, so)] : R(0);
          mf_for<0, NDS>([&](auto D) __attribute__((always_inline)) {
            constexpr int d = decltype(D)::value;
            av[d][i] = kin ? tbT[Y::ti(t, d, kq, mo)] : R(0);
          });
        },
        [&](auto I) __attribute__((always_inline)) {
          constexpr int i = decltype(I)::value;
          const int t = R0 + t0 + i;
          if (kin) mf_ld4(G + Y::gi(t, kq, so), bv[i], bv[i + 1], bv[i + 2], bv[i + 3]);
          else bv[i] = bv[i + 1] = bv[i + 2] = bv[i + 3] = R(0);
          mf_for<0, NDS>([&](auto D) __attribute__((always_inline)) {
            constexpr int d = decltype(D)::value;
            if (kin) mf_ld4(tbT + Y::ti(t, d, kq, mo), av[d][i], av[d][i + 1], av[d][i + 2], av[d][i + 3]);
            else av[d][i] = av[d][i + 1] = av[d][i + 2] = av[d][i + 3] = R(0);
          });
        });
    fr_sched_fence();
    mf_for<0, CH>([&](auto I) __attribute__((always_inline)) {
      constexpr int i = decltype(I)::value, tl = t0 + i;
      if constexpr (tl < SLS) {
        mf_for<0, NDS>([&](auto D) __attribute__((always_inline)) {
          constexpr int d = decltype(D)::value;
          const acc x = M::mma(av[d][i], bv[i], zero);
          mf_for<0, N1>([&](auto W) __attribute__((always_inline)) {
            constexpr int w = decltype(W)::value, rho = X::line(tl, d, w);
            V[rho] += dc[w][X::co(tl, d)] * x;
          });
          mf_for<0, N1>([&](auto W) __attribute__((always_inline)) { mf_pin(V[X::line(tl, d, decltype(W)::value)]); });
        });
        fr_sched_fence();
      }
    });
    fr_sched_fence();
  });
  if constexpr (ND == 3) {
    // volume, third direction: every point tau = (x, y, c) reaches the slab
    // at (x, y, z0) with weight Dc1[z0][c], folded into A so that the MFMA
    // accumulates in place
    R wz[N1];
    mf_for<0, N1>([&](auto Cc) __attribute__((always_inline)) {
      constexpr int c = decltype(Cc)::value;
      wz[c] = dc[0][c];
      mf_for<1, N1>([&](auto Z) __attribute__((always_inline)) {
        if (z0 == decltype(Z)::value) wz[c] = dc[decltype(Z)::value][c];
      });
    });
    // chunks of CH points within each level c of the third coordinate
    constexpr int QL = (SLS + CH - 1) / CH;
    mf_for<0, N1 * QL>([&](auto CQ) __attribute__((always_inline)) {
      constexpr int c = decltype(CQ)::value / QL, i0 = (decltype(CQ)::value % QL) * CH;
      constexpr int CNT = (SLS - i0) < CH ? (SLS - i0) : CH;
      R bv[CH], av[CH];
      mf_chunk<CNT, (c * SLS + i0) % 4>(
          [&](auto I) __attribute__((always_inline)) {
            constexpr int i = decltype(I)::value, t = c * SLS + i0 + i;
            bv[i] = kin ? G[Y::gi(t, kq, so)] : R(0);
            av[i] = kin ? tbT[Y::ti(t, 2, kq, mo)] : R(0);
          },
          [&](auto I) __attribute__((always_inline)) {
            constexpr int i = decltype(I)::value, t = c * SLS + i0 + i;
            if (kin) {
              mf_ld4(G + Y::gi(t, kq, so), bv[i], bv[i + 1], bv[i + 2], bv[i + 3]);
              mf_ld4(tbT + Y::ti(t, 2, kq, mo), av[i], av[i + 1], av[i + 2], av[i + 3]);
            } else {
              bv[i] = bv[i + 1] = bv[i + 2] = bv[i + 3] = R(0);
              av[i] = av[i + 1] = av[i + 2] = av[i + 3] = R(0);
            }
          });
      fr_sched_fence();
      mf_for<0, CNT>([&](auto I) __attribute__((always_inline)) {
        constexpr int i = decltype(I)::value;
        V[i0 + i] = M::mma(wz[c] * av[i], bv[i], V[i0 + i]);
      });
      fr_sched_fence();
    });
  }
  // faces whose normal lines lie in the slab: Y[g] scattered along g's
  // normal line (quadrilaterals: every face; hexahedra: the first- and
  // second-axis faces, flux points (ta, z0) of each)
  constexpr int FPS = ND == 3 ? N1 : NFP;          // in-slab flux points per such face
  constexpr int NFS = ND == 3 ? 4 : E::NFACE;       // such faces
  auto face_of = [](int j) constexpr {              // j-th such face
    if (ND == 2) return j;
    int f = 0, seen = 0;
    for (int q = 0; q < E::NFACE; ++q)
      if (X::fax(q) != 2) { if (seen == j) f = q; ++seen; }
    return f;
  };
  constexpr int NG = NFS * FPS;
  mf_for<0, (NG + CH - 1) / CH>([&](auto C) __attribute__((always_inline)) {
    constexpr int g0 = decltype(C)::value * CH;
    R fa[JC][CH], fb[JC][CH];
    constexpr int CNT = (NG - g0) < CH ? (NG - g0) : CH;
    // consecutive in-slab flux points are consecutive in memory within a
    // face: always for quadrilaterals, for hexahedra when N1 = 4 (aligned)
    constexpr int B4 = (ND == 2) ? 0 : (FPS == 4 ? 0 : -1);
    auto gof = [&](int gi) {
      const int f = face_of(gi / FPS), ta = gi % FPS;
      return f * NFP + ta + (ND == 3 ? N1 * z0 : 0);
    };
    mf_chunk<CNT, B4>(
        [&](auto I) __attribute__((always_inline)) {
          constexpr int i = decltype(I)::value;
          const int g = gof(g0 + i);
          mf_for<0, JC>([&](auto CC) __attribute__((always_inline)) {
            constexpr int ch = decltype(CC)::value;
            const int j = ch * 4 + kq;
            const bool use = j < JF;
            fa[ch][i] = use ? tfT[Y::fi(g, j, mo)] : R(0);
            fb[ch][i] = use ? (j < 2 ? Sr : S)[Y::si(g, j, so)] : R(0);
          });
        },
        [&](auto I) __attribute__((always_inline)) {
          constexpr int i = decltype(I)::value;
          const int g = gof(g0 + i);
          mf_for<0, JC>([&](auto CC) __attribute__((always_inline)) {
            constexpr int ch = decltype(CC)::value;
            const int j = ch * 4 + kq;
            if (j < JF) {
              mf_ld4(tfT + Y::fi(g, j, mo), fa[ch][i], fa[ch][i + 1], fa[ch][i + 2], fa[ch][i + 3]);
              mf_ld4((j < 2 ? Sr : S) + Y::si(g, j, so), fb[ch][i], fb[ch][i + 1], fb[ch][i + 2], fb[ch][i + 3]);
            } else {
              fa[ch][i] = fa[ch][i + 1] = fa[ch][i + 2] = fa[ch][i + 3] = R(0);
              fb[ch][i] = fb[ch][i + 1] = fb[ch][i + 2] = fb[ch][i + 3] = R(0);
            }
          });
        });
    fr_sched_fence();
    mf_for<0, CH>([&](auto I) __attribute__((always_inline)) {
      constexpr int i = decltype(I)::value, gi = g0 + i;
      if constexpr (gi < NG) {
        constexpr int f = face_of(gi / FPS), ta = gi % FPS, ax = X::fax(f);
        constexpr bool pos = X::fsg(f) > 0;
        acc y = zero;
        mf_for<0, JC>([&](auto CC) __attribute__((always_inline)) {
          y = M::mma(fa[decltype(CC)::value][i], fb[decltype(CC)::value][i], y);
        });
        // slab-relative target: the normal line through (ta, z0) of face f
        auto tgt = [](int w) constexpr {
          return ND == 2 ? X::fline(f * NFP + ta, w) : (ax == 0 ? w + N1 * ta : ta + N1 * w);
        };
        mf_for<0, N1>([&](auto W) __attribute__((always_inline)) {
          constexpr int w = decltype(W)::value;
          V[tgt(w)] += (pos ? hp[w] : hm[w]) * y;
        });
        mf_for<0, N1>([&](auto W) __attribute__((always_inline)) { mf_pin(V[tgt(decltype(W)::value)]); });
        fr_sched_fence();
      }
    });
    fr_sched_fence();
  });
  if constexpr (ND == 3) {
    // third-axis faces: flux point t = (x, y) of either face reaches the
    // slab at (x, y, z0) with weight h(z0), folded into A
    R hzp = hp[0], hzm = hm[0];
    mf_for<1, N1>([&](auto Z) __attribute__((always_inline)) {
      if (z0 == decltype(Z)::value) { hzp = hp[decltype(Z)::value]; hzm = hm[decltype(Z)::value]; }
    });
    auto zface = [](int j) constexpr {
      int f = 0, seen = 0;
      for (int q = 0; q < E::NFACE; ++q)
        if (X::fax(q) == 2) { if (seen == j) f = q; ++seen; }
      return f;
    };
    // chunks of CH flux points within each of the two faces
    constexpr int QF = (NFP + CH - 1) / CH;
    mf_for<0, 2 * QF>([&](auto FQ) __attribute__((always_inline)) {
      constexpr int f = zface(decltype(FQ)::value / QF), t0 = (decltype(FQ)::value % QF) * CH;
      constexpr int CNT = (NFP - t0) < CH ? (NFP - t0) : CH;
      const R hz = X::fsg(f) > 0 ? hzp : hzm;
      R fa[JC][CH], fb[JC][CH];
      mf_chunk<CNT, (f * NFP + t0) % 4>(
          [&](auto I) __attribute__((always_inline)) {
            constexpr int i = decltype(I)::value, g = f * NFP + t0 + i;
            mf_for<0, JC>([&](auto CC) __attribute__((always_inline)) {
              constexpr int ch = decltype(CC)::value;
              const int j = ch * 4 + kq;
              const bool use = j < JF;
              fa[ch][i] = use ? tfT[Y::fi(g, j, mo)] : R(0);
              fb[ch][i] = use ? (j < 2 ? Sr : S)[Y::si(g, j, so)] : R(0);
            });
          },
          [&](auto I) __attribute__((always_inline)) {
            constexpr int i = decltype(I)::value, g = f * NFP + t0 + i;
            mf_for<0, JC>([&](auto CC) __attribute__((always_inline)) {
              constexpr int ch = decltype(CC)::value;
              const int j = ch * 4 + kq;
              if (j < JF) {
                mf_ld4(tfT + Y::fi(g, j, mo), fa[ch][i], fa[ch][i + 1], fa[ch][i + 2], fa[ch][i + 3]);
                mf_ld4((j < 2 ? Sr : S) + Y::si(g, j, so), fb[ch][i], fb[ch][i + 1], fb[ch][i + 2], fb[ch][i + 3]);
              } else {
                fa[ch][i] = fa[ch][i + 1] = fa[ch][i + 2] = fa[ch][i + 3] = R(0);
                fb[ch][i] = fb[ch][i + 1] = fb[ch][i + 2] = fb[ch][i + 3] = R(0);
              }
            });
          });
      fr_sched_fence();
      mf_for<0, CNT>([&](auto I) __attribute__((always_inline)) {
        constexpr int i = decltype(I)::value, t = t0 + i;
        static_assert(X::fline(f * NFP + t, 0) % SLS == t, "third-axis flux point t lies over slab point t");
        mf_for<0, JC>([&](auto CC) __attribute__((always_inline)) {
          V[t] = M::mma(hz * fa[decltype(CC)::value][i], fb[decltype(CC)::value][i], V[t]);
        });
      });
      fr_sched_fence();
    });
  }
  }   // FP32 operands
  // D rows are pairs m, columns sigma.  The task owns the columns (sigma in
  // tile nt, beta in pair tile mt) of block k and, in each, the contiguous
  // row segment (rho in the slab, every alpha): the tile goes through LDS
  // (NH passes of NRH rows, stride NRH + 1) and leaves as contiguous 16-byte
  // (FP32) or 8-byte (BF16) stores.
  constexpr int NH = Y::NH, NRH = Y::NRH, SP = NRH + 1, BT = Y::BT, PR = SLS / NH;
  const int b0 = mt * BT, nbt = (NV - b0) < BT ? (NV - b0) : BT;
  const int nsg = (NS - nt * 16) < 16 ? (NS - nt * 16) : 16;
  const int ncol = nsg * nbt;
  OT* Bk = B + (nl * nblk + k) * (long)BB * BB + (long)R0 * NV;
  mf_for<0, NH>([&](auto H) __attribute__((always_inline)) {
    constexpr int h = decltype(H)::value;
    if constexpr (h > 0) __syncthreads();      // the previous pass has left the stage
    if (active) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int a, b;
        const bool ok = Y::pair(mt * 16 + M::row(kq, r), a, b);
        if (ok && nt * 16 + li < NS) {
          R* col = stage + (li * nbt + (b - b0)) * SP + a;
          mf_for<0, PR>([&](auto L) __attribute__((always_inline)) {
            constexpr int rl = h * PR + decltype(L)::value;
            col[decltype(L)::value * NV] = -(srd[R0 + rl] * V[rl][r]);
          });
        }
      }
    }
    __syncthreads();
    if (active) {
      OT* Bh = Bk + h * NRH;
      if constexpr (NRH % 4 == 0 && BB % 4 == 0) {
        for (int i = 4 * lane; i < ncol * NRH; i += 256) {
          const int cl = i / NRH, rr = i % NRH;
          const int c = (nt * 16 + cl / nbt) * NV + b0 + cl % nbt;
          const R* sp = stage + cl * SP + rr;
          if constexpr (std::is_same<OT, float>::value) {
            // nontemporal 16-byte stores: the blocks are written once and
            // not read back here (24^3 hexahedra, degree 3: 26.7 -> 25.4 ms);
            // the BF16 blocks' 8-byte stores were 7% slower that way and
            // stay plain
            typedef float f4v __attribute__((ext_vector_type(4)));
            const f4v v = {sp[0], sp[1], sp[2], sp[3]};
            __builtin_nontemporal_store(v, reinterpret_cast<f4v*>(Bh + (long)c * BB + rr));
          } else {
            const OT q[4] = {to_out<OT>(sp[0]), to_out<OT>(sp[1]), to_out<OT>(sp[2]), to_out<OT>(sp[3])};
            uint2 w;
            __builtin_memcpy(&w, q, sizeof(w));
            *reinterpret_cast<uint2*>(Bh + (long)c * BB + rr) = w;
          }
        }
      } else {
        for (int i = lane; i < ncol * NRH; i += 64) {
          const int cl = i / NRH, rr = i % NRH;
          const int c = (nt * 16 + cl / nbt) * NV + b0 + cl % nbt;
          Bh[(long)c * BB + rr] = to_out<OT>(stage[cl * SP + rr]);
        }
      }
    }
  });
}
