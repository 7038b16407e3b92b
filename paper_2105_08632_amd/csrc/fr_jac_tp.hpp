// Jacobian-block assembly for tensor-product elements (quads, hexes).
//
// Same mathematics as jac_body (fr_kernels.hpp): for each pair (alpha, beta)
// of output / input variables the block is a product of scalar operators,
//   J[(rho,alpha),(sigma,beta)] = -rdet(rho) ( sum_d Dc_d X_d + Cor Y )[rho][sigma],
//   X_d[tau][sigma] = a_d(tau) delta_{tau sigma} [k = n] + sum_e b_de(tau) Gam_e[tau][sigma],
//   Y[g][sigma]     = fuL(g) DL[g][sigma] + fuR(g) DR[g][sigma]
//                     + sum_d' fqL_d'(g) SL_d'[g][sigma] + fqR_d'(g) SR_d'[g][sigma],
// organised for the hardware:
//   * set-up (one barrier-separated pass per element): pointwise flux Jacobian
//     tables (forward mode) and the scalar sensitivity matrices of every
//     block at once, laid out so a lane reads its own column with wide loads;
//   * assembly without barriers: each wavefront owns a task (block k, input
//     variable beta, 64 lanes over (sigma, alpha)) and accumulates the whole
//     output column in registers.  On tensor elements Dc_d and Cor act along
//     lines only; their 1-D factors come in through kernel arguments and all
//     point/line index arithmetic is resolved at compile time.
#pragma once
#include "fr_kernels.hpp"

// 1-D factors of the tensor operators (degree p, n1 = p + 1 <= 5):
//   Dc_d = Dc1 along the d-lines, Cor on a face with outward sign s: h_s,
//   M0 on that face: l_s; G_d = G1 along the d-lines.
template <class R> struct Ops1D {
  R Dc1[5][5];
  R G1[5][5];
  R hp[5], hm[5], lp[5], lm[5];
};

// Keeps the scheduler from hoisting the loads of every unrolled iteration
// to the top (which would exhaust the registers); no run-time effect.
FR_HD void fr_sched_fence() {
#if defined(__HIP_DEVICE_COMPILE__)
  __builtin_amdgcn_sched_barrier(0);
#endif
}

template <class E> struct TPIdx {
  static constexpr int ND = E::ND, N1 = E::DEG + 1, NS = E::NS, NFP = E::NFP;
  // coordinate d of point r
  static constexpr FR_HD int co(int r, int d) { return d == 0 ? r % N1 : (d == 1 ? (r / N1) % N1 : r / (N1 * N1)); }
  static constexpr FR_HD int str(int d) { return d == 0 ? 1 : (d == 1 ? N1 : N1 * N1); }
  // point r with coordinate d replaced by w
  static constexpr FR_HD int line(int r, int d, int w) { return r + (w - co(r, d)) * str(d); }
  // face geometry (mesh convention): normal axis and outward sign
  static constexpr FR_HD int fax(int f) {
    return ND == 2 ? (f == 0 || f == 2 ? 1 : 0) : (f == 0 || f == 5 ? 2 : (f == 1 || f == 3 ? 1 : 0));
  }
  static constexpr FR_HD int fsg(int f) {
    return ND == 2 ? (f == 1 || f == 2 ? 1 : -1) : (f == 2 || f == 3 || f == 5 ? 1 : -1);
  }
  // the solution point on flux point g's normal line with normal coordinate w
  static constexpr FR_HD int fline(int g, int w) {
    int f = g / NFP, t = g % NFP, ax = fax(f);
    if (ND == 2) {
      int i = (f == 0 || f == 1) ? t : (N1 - 1 - t);   // counter-clockwise along the edge
      return ax == 0 ? (w + N1 * i) : (i + N1 * w);
    }
    int ta = t % N1, tb = t / N1, c[3] = {0, 0, 0}, k = 0;
    for (int d = 0; d < 3; ++d) c[d] = (d == ax) ? w : (k++ == 0 ? ta : tb);
    return c[0] + N1 * (c[1] + N1 * c[2]);
  }
};

template <class E, int NV, int SYS> struct TPSizes {
  static constexpr int ND = E::ND, NS = E::NS, NF = E::NF, NFACE = E::NFACE, NFP = E::NFP, NV2 = NV * NV;
  static constexpr int NB = 1 + E::NFACE;
  // per (pair, tau, d): (b_d0 .. b_d(ND-1), a_d), against per (k, sigma, tau):
  // (Gam_0 .. Gam_(ND-1), delta_{tau sigma} [k = n])
  static constexpr int GE = 4;
  static constexpr int BE = ND * GE;                       // tb row per (pair, tau)
  // per (pair, g): (fuL, fuR, fqL_d.., fqR_d..), against per (k, sigma, g):
  // (DL, DR, SL_d.., SR_d..)
  static constexpr int FE = ((2 + 2 * ND + 3) / 4) * 4;
  static constexpr int SE = FE;
  // row strides padded so that the 4-dword loads of the lanes of a wavefront
  // (different sigma: gam, slr; different alpha: tb, tf) fall in different
  // LDS banks (32 banks of 4 bytes)
  static constexpr int pad(int x, int r) { return x + ((r - x % 32) + 32) % 32; }
  static constexpr int GS = pad(NS * GE, 4);           // gam: per (k, sigma)
  static constexpr int SS = pad(NF * SE, 4);           // slr: per (k, sigma)
  static constexpr int TBS = pad(NV * NS * BE, 8);     // tb: per alpha
  static constexpr int TFS = pad(NV * NF * FE, 8);     // tf: per alpha
};

// LDS: a persistent part (operators, element data, tables) and a region
// shared by the table-build scratch and the sensitivities of NBS blocks.
template <class E, int NV, int SYS, class R> constexpr int jac_tp_fixed() {
  typedef TPSizes<E, NV, SYS> Z;
  constexpr int NS = Z::NS, NF = Z::NF, ND = Z::ND, NFACE = Z::NFACE, NFP = Z::NFP, NV2 = Z::NV2;
  int b = 0;
  b += lds_bytes<R>(NF * NS) + lds_bytes<R>(NS * NF);                          // M0, Cor
  b += lds_bytes<R>(NS * NV) + lds_bytes<R>(NS * ND * NV) + 2 * lds_bytes<R>(NF * NV) + 2 * lds_bytes<R>(NF * ND * NV);
  b += 2 * lds_bytes<R>(NS * ND * ND) + lds_bytes<R>(NS) + lds_bytes<R>(NF * ND) + lds_bytes<R>(NF) + lds_bytes<int>(NF);
  b += lds_bytes<R>(NFACE * NS * ND * ND) + lds_bytes<int>(NFACE * NFP) + 2 * lds_bytes<int>(NFACE);
  b += lds_bytes<R>(NFACE * NFP * ND);                                         // W (diagonal on tensor faces)
  b += lds_bytes<Ops1D<R>>(1);
  b += lds_bytes<R>(NV * Z::TBS) + lds_bytes<R>(NV * Z::TFS);
  return b;
}
template <class E, int NV, int SYS, class R> constexpr int jac_tp_scratch() {
  typedef TPSizes<E, NV, SYS> Z;
  return lds_bytes<R>(Z::ND * Z::ND * Z::NS * Z::NV2) + 4 * lds_bytes<R>(Z::NF * Z::NV2) +
         2 * lds_bytes<R>(Z::ND * Z::NF * Z::NV2);
}
template <class E, int NV, int SYS, class R> constexpr int jac_tp_sens(int nbs) {
  typedef TPSizes<E, NV, SYS> Z;
  return lds_bytes<R>(nbs * Z::NS * Z::GS) + lds_bytes<R>(nbs * Z::NS * Z::SS);
}
template <class E, int NV, int SYS, class R> constexpr int jac_tp_lds_nbs(int nbs) {
  int sc = jac_tp_scratch<E, NV, SYS, R>(), se = jac_tp_sens<E, NV, SYS, R>(nbs);
  return jac_tp_fixed<E, NV, SYS, R>() + (sc > se ? sc : se);
}
// blocks whose sensitivities are held at once: all when they fit, else one
template <class E, int NV, int SYS, class R> constexpr int jac_tp_nbs() {
  return jac_tp_lds_nbs<E, NV, SYS, R>(1 + E::NFACE) <= 160 * 1024 ? 1 + E::NFACE : 1;
}
// input variables accumulated per lane: as many as keep NBT*NS <= 64
template <class E, int NV> constexpr int jac_tp_nbt() {
  return (64 / E::NS) < 1 ? 1 : ((64 / E::NS) > NV ? NV : (64 / E::NS));
}
// threads of one workgroup: one wavefront per task, at most 512
template <class E, int NV, int SYS, class R> constexpr int jac_tp_threads() {
  constexpr int tasks = jac_tp_nbs<E, NV, SYS, R>() * ((E::NS * NV + 63) / 64) *
                        ((NV + jac_tp_nbt<E, NV>() - 1) / jac_tp_nbt<E, NV>());
  return tasks >= 8 ? 512 : (tasks < 4 ? 256 : 64 * tasks);
}
template <class E, int NV, int SYS, class R> constexpr int jac_tp_lds() {
  return jac_tp_lds_nbs<E, NV, SYS, R>(jac_tp_nbs<E, NV, SYS, R>());
}

// One assembly task (see jac_tp_body): kept out of line so its register
// live range ends with the task.
template <class E, int NV, int SYS, class R, class OT>
FR_HD __forceinline__ bool jac_tp_task(int item, int kb, const Ops1D<R>& o1, const R* srd, const R* tb,
                                       const R* tf, const R* gam, const R* slr, OT* Bn) {
  typedef TPSizes<E, NV, SYS> Z;
  typedef TPIdx<E> X;
  constexpr int NS = Z::NS, NF = Z::NF, ND = Z::ND, NFP = Z::NFP;
  constexpr int N1 = E::DEG + 1;
  constexpr int BE = Z::BE, FE = Z::FE, GE = Z::GE, SE = Z::SE;
  constexpr int GS = Z::GS, SS = Z::SS, TBS = Z::TBS, TFS = Z::TFS;
  constexpr int BB = NS * NV;
  constexpr int LANES = NS * NV;
  constexpr int CHUNKS = (LANES + 63) / 64;
  constexpr int NBT = jac_tp_nbt<E, NV>();
  constexpr int NBG = (NV + NBT - 1) / NBT;
  const int task = item / 64, lane = item % 64;
  const int kk = task / (CHUNKS * NBG), chunk = (task / NBG) % CHUNKS, bg = task % NBG;
  const int k = kb + kk;
  const int l = chunk * 64 + lane;
  const bool live = l < LANES;
  const int s = live ? l / NV : 0, a = live ? l % NV : 0;
  const int b0 = bg * NBT;
  R out[NBT][NS];
#pragma unroll
  for (int bb = 0; bb < NBT; ++bb)
#pragma unroll
    for (int r = 0; r < NS; ++r) out[bb][r] = R(0);
  // volume: X_d[tau] = (b_d., a_d) . (Gam_., delta), out += Dc_d X_d along d-lines
  const R* gcol = gam + (kk * NS + s) * GS;
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    R gv[GE];
#pragma unroll
    for (int z = 0; z < GE; ++z) gv[z] = gcol[t * GE + z];
#pragma unroll
    for (int bb = 0; bb < NBT; ++bb) {
      const int beta = b0 + bb < NV ? b0 + bb : NV - 1;
      const R* tbp = tb + a * TBS + (beta * NS + t) * BE;
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        R xd = R(0);
#pragma unroll
        for (int z = 0; z < GE; ++z) xd += tbp[d * GE + z] * gv[z];
#pragma unroll
        for (int w = 0; w < N1; ++w) out[bb][X::line(t, d, w)] += o1.Dc1[w][X::co(t, d)] * xd;
      }
    }
    fr_sched_fence();
  }
  // faces: Y[g] = (fuL, fuR, fqL., fqR.) . (DL, DR, SL., SR.), out += Cor Y
  const R* sp = slr + (kk * NS + s) * SS;
#pragma unroll
  for (int g = 0; g < NF; ++g) {
    R sv[SE];
#pragma unroll
    for (int z = 0; z < SE; ++z) sv[z] = sp[g * SE + z];
    const int sg = X::fsg(g / NFP);
#pragma unroll
    for (int bb = 0; bb < NBT; ++bb) {
      const int beta = b0 + bb < NV ? b0 + bb : NV - 1;
      const R* tfp = tf + a * TFS + (beta * NF + g) * FE;
      R y = R(0);
#pragma unroll
      for (int z = 0; z < SE; ++z) y += tfp[z] * sv[z];
#pragma unroll
      for (int w = 0; w < N1; ++w) out[bb][X::fline(g, w)] += (sg > 0 ? o1.hp[w] : o1.hm[w]) * y;
    }
    fr_sched_fence();
  }
  bool bad = false;
  if (live) {
#pragma unroll
    for (int bb = 0; bb < NBT; ++bb) {
      const int beta = b0 + bb;
      if (beta < NV) {
        OT* col = Bn + (long)k * BB * BB + (long)(s * NV + beta) * BB;
#pragma unroll
        for (int r = 0; r < NS; ++r) {
          const R jv = -(srd[r] * out[bb][r]);
          col[r * NV + a] = to_out<OT>(jv);
          bad |= !fr_finite(jv);
        }
      }
    }
  }
  return bad;
}

template <class E, int NV, int SYS, class R, class OT, class Sync>
FR_HD void jac_tp_body(int n, int tid, int nth, char* lds, const OpsD<R>& op, const Ops1D<R>& o1, const GeoD<R>& geo,
                       const PhysP& ph, const R* U, const R* Q, const R* UF, const R* QF, OT* B, int nblk,
                       Sync sync) {
  typedef TPSizes<E, NV, SYS> Z;
  typedef TPIdx<E> X;
  constexpr int NS = Z::NS, NF = Z::NF, ND = Z::ND, NFACE = Z::NFACE, NFP = Z::NFP, NV2 = Z::NV2, NB = Z::NB;
  constexpr int N1 = E::DEG + 1;
  constexpr int BE = Z::BE, FE = Z::FE, GE = Z::GE, SE = Z::SE;
  constexpr int BB = NS * NV;
  const bool visc = SysTraits<SYS>::kVisc && (SYS != SYS_ADV || ph.mu != 0.0);
  const R cb = R(0.5 + ph.beta), cL = R(0.5 + ph.beta), cR = R(0.5 - ph.beta), eta = R(ph.eta);
  typedef MDual<R, NV> MD;

  Lds L{lds};
  R* sM0 = L.take<R>(NF * NS);
  R* sCor = L.take<R>(NS * NF);
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
  R* sJm = L.take<R>(NFACE * NS * ND * ND);
  int* sback = L.take<int>(NFACE * NFP);
  int* snb = L.take<int>(NFACE);
  int* snf = L.take<int>(NFACE);
  R* sW = L.take<R>(NFACE * NFP * ND);
  Ops1D<R>* sO1 = L.take<Ops1D<R>>(1);     // 1-D factors for the per-thread indexed reads below
  constexpr int GS = Z::GS, SS = Z::SS, TBS = Z::TBS, TFS = Z::TFS;
  R* tb = L.take<R>(NV * TBS);             // [alpha] [beta][tau][d][b_d0.., a_d]
  R* tf = L.take<R>(NV * TFS);             // [alpha] [beta][g][fuL, fuR, fqL_d.., fqR_d..]
  constexpr int NBS = jac_tp_nbs<E, NV, SYS, R>();
  Lds L2{L.p};
  R* gam = L2.take<R>(NBS * NS * GS);     // [k - kb][sigma] [tau][Gam_e.., delta]
  R* slr = L2.take<R>(NBS * NS * SS);     // [k - kb][sigma] [g][DL, DR, SL_d.., SR_d..]
  Lds L1{L.p};                             // table-build scratch (used before gam / slr)
  R* bh = L1.take<R>(ND * ND * NS * NV2);  // df_k/dq_d' [d'][k][tau][ab]
  R* rL = L1.take<R>(NF * NV2);
  R* rR = L1.take<R>(NF * NV2);
  R* vL = L1.take<R>(NF * NV2);
  R* vR = L1.take<R>(NF * NV2);
  R* qLt = L1.take<R>(ND * NF * NV2);
  R* qRt = L1.take<R>(ND * NF * NV2);

  const long nl = n;
  // ---------------------------------------------------------------- loads
  for (int i = tid; i < NF * NS; i += nth) sM0[i] = op.M0[i];
  for (int i = tid; i < NS * NF; i += nth) sCor[i] = op.Cor[i];
  for (int i = tid; i < NS * NV; i += nth) su[i] = U[nl * NS * NV + i];
  if (visc)
    for (int i = tid; i < NS * ND * NV; i += nth) sq[i] = Q[nl * NS * ND * NV + i];
  for (int i = tid; i < NF; i += nth) { spg[i] = geo.nbfp[nl * NF + i]; smg[i] = geo.magN[nl * NF + i]; }
  for (int i = tid; i < NS * ND * ND; i += nth) { sJi[i] = geo.Jinv[nl * NS * ND * ND + i]; sS[i] = geo.S[nl * NS * ND * ND + i]; }
  for (int i = tid; i < NS; i += nth) srd[i] = geo.rdet[nl * NS + i];
  for (int i = tid; i < NF * ND; i += nth) snn[i] = geo.nrm[nl * NF * ND + i];
  for (int i = tid; i < NFACE; i += nth) { snb[i] = geo.nbr[nl * NFACE + i]; snf[i] = geo.nbface[nl * NFACE + i]; }
  for (int i = tid; i < NFACE * NFP; i += nth) sback[i] = geo.back[nl * NFACE * NFP + i];
  for (int i = tid; i < (int)(sizeof(Ops1D<R>) / sizeof(R)); i += nth)
    reinterpret_cast<R*>(sO1)[i] = reinterpret_cast<const R*>(&o1)[i];
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
  for (int i = tid; i < NFACE * NS * ND * ND; i += nth) {
    int f = i / (NS * ND * ND), r = i % (NS * ND * ND);
    sJm[i] = geo.Jinv[(long)snb[f] * NS * ND * ND + r];
  }
  sync();
  // W_d'(g) = (1/2+beta) sum_tau' M0[g2][tau'] Cor[tau'][g2] sum_e Jinv_m[tau'][e][d'] nref[g2][e]:
  // the neighbour's face gradient at g2 (partner of g) w.r.t. u_n, which on
  // tensor elements only reaches through the same face point.
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

  // ---------------------------------------------------------------- tables
  // one seeded input per item (single-tangent duals keep register use low):
  // solution points: (tau, pass, c), pass 0 seeds u_c, pass 1+d seeds q_{d,c};
  // flux points: (g, pass, c), passes 0/1 seed u_L,c / u_R,c in the
  // convective flux, 2/3 seed u_c in the viscous flux at L / R, then q_{d,c}
  // at L, then at R.
  {
    typedef Dual<R> DT;
    constexpr int NPS = SysTraits<SYS>::kVisc ? 1 + ND : 1;
    constexpr int NPF = SysTraits<SYS>::kVisc ? 4 + 2 * ND : 2;
    const int nsp = visc ? NPS : 1, nfp = visc ? NPF : 2;
    for (int it = tid; it < (NS * nsp + NF * nfp) * NV; it += nth) {
      const int c = it % NV, j0 = it / NV;
      if (j0 < NS * nsp) {
        int t = j0 / nsp, ps = j0 % nsp;
        DT u[NV], f[ND][NV], q[ND][NV];
        for (int a = 0; a < NV; ++a) u[a] = DT(su[t * NV + a], (ps == 0 && a == c) ? R(1) : R(0));
        for (int d = 0; d < ND; ++d)
          for (int a = 0; a < NV; ++a)
            q[d][a] = DT(visc ? sq[(t * ND + d) * NV + a] : R(0), (ps == 1 + d && a == c) ? R(1) : R(0));
        if (ps == 0) {
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
              tb[a * TBS + (c * NS + t) * BE + d * GE + ND] = acc;
            }
        } else {
          flux_viscous<SYS, ND, NV, DT>(ph, u, q, f);
          for (int k = 0; k < ND; ++k)
            for (int a = 0; a < NV; ++a) bh[(((ps - 1) * ND + k) * NS + t) * NV2 + a * NV + c] = f[k][a].d;
        }
      } else {
        int j = j0 - NS * nsp;
        int g = j / nfp, ps = j % nfp;
        R nn[ND];
        for (int d = 0; d < ND; ++d) nn[d] = snn[g * ND + d];
        if (ps < 2) {
          DT uL[NV], uR[NV], F[NV];
          for (int a = 0; a < NV; ++a) {
            uL[a] = DT(suL[g * NV + a], (ps == 0 && a == c) ? R(1) : R(0));
            uR[a] = DT(suR[g * NV + a], (ps == 1 && a == c) ? R(1) : R(0));
          }
          common_inviscid<SYS, ND, NV, DT>(ph, uL, uR, nn, F);
          R* o = ps == 0 ? rL : rR;
          for (int a = 0; a < NV; ++a) o[g * NV2 + a * NV + c] = F[a].d;
        } else {
          int pp = ps - 2;
          int side = (pp == 1 || pp >= 2 + ND) ? 1 : 0;
          int qd = pp < 2 ? -1 : (pp - 2) % ND;
          const R* us = side ? suR : suL;
          const R* qs = side ? sqR : sqL;
          DT u[NV], q[ND][NV], fv[ND][NV];
          for (int a = 0; a < NV; ++a) u[a] = DT(us[g * NV + a], (qd < 0 && a == c) ? R(1) : R(0));
          for (int d = 0; d < ND; ++d)
            for (int a = 0; a < NV; ++a) q[d][a] = DT(qs[(g * ND + d) * NV + a], (qd == d && a == c) ? R(1) : R(0));
          flux_viscous<SYS, ND, NV, DT>(ph, u, q, fv);
          R wgt = side ? cR : cL;
          for (int a = 0; a < NV; ++a) {
            R acc = R(0);
            for (int d = 0; d < ND; ++d) acc += nn[d] * fv[d][a].d;
            acc *= wgt;
            if (qd < 0) (side ? vR : vL)[g * NV2 + a * NV + c] = acc;
            else (side ? qRt : qLt)[(qd * NF + g) * NV2 + a * NV + c] = acc;
          }
        }
      }
    }
    sync();
    for (int i = tid; i < NV2 * NS * ND; i += nth) {
      const int ab = i / (NS * ND), r = i % (NS * ND);
      R* row = tb + (ab / NV) * TBS + ((ab % NV) * NS * ND + r) * GE;
      for (int z = ND + 1; z < GE; ++z) row[z] = R(0);
      if (!visc)
        for (int e = 0; e < ND; ++e) row[e] = R(0);
    }
    if (visc)
      for (int i = tid; i < NV2 * NS * ND * ND; i += nth) {
        int ab = i / (NS * ND * ND), t = (i / (ND * ND)) % NS, d = (i / ND) % ND, e = i % ND;
        R acc = R(0);
        for (int k = 0; k < ND; ++k) {
          R s = sS[(t * ND + d) * ND + k];
          for (int d2 = 0; d2 < ND; ++d2) acc += s * bh[((d2 * ND + k) * NS + t) * NV2 + ab] * sJi[(t * ND + e) * ND + d2];
        }
        tb[(ab / NV) * TBS + ((ab % NV) * NS + t) * BE + d * GE + e] = acc;
      }
    for (int i = tid; i < NV2 * NF; i += nth) {
      int ab = i / NF, g = i % NF;
      int a = ab / NV, c = ab % NV;
      R mg = smg[g];
      R id = (a == c) ? eta : R(0);
      R* o = tf + (ab / NV) * TFS + ((ab % NV) * NF + g) * FE;
      o[0] = mg * (rL[g * NV2 + ab] + (visc ? vL[g * NV2 + ab] + id : R(0)));
      o[1] = mg * (rR[g * NV2 + ab] + (visc ? vR[g * NV2 + ab] - id : R(0)));
      for (int d = 0; d < ND; ++d) {
        o[2 + d] = visc ? mg * qLt[(d * NF + g) * NV2 + ab] : R(0);
        o[2 + ND + d] = visc ? mg * qRt[(d * NF + g) * NV2 + ab] : R(0);
      }
      for (int z = 2 + 2 * ND; z < FE; ++z) o[z] = R(0);
    }
    sync();
  }

  OT* Bn = B + nl * (long)nblk * BB * BB;
  for (int kb = 0; kb < nblk; kb += NBS) {
  const int nbk = (nblk - kb) < NBS ? (nblk - kb) : NBS;
  // ------------------------------------------- sensitivities of blocks kb..
  // gam[k][sigma][tau][e] = d q~_e(tau) / d u_k(sigma)
  for (int i = tid; i < nbk * NS * NS * ND; i += nth) {
    int kk = i / (NS * NS * ND), s = (i / (NS * ND)) % NS, t = (i / ND) % NS, e = i % ND;
    int k = kb + kk;
    R v = R(0);
    if (visc) {
      if (k == 0) {
        // G_e along e-lines
        bool on = true;
        for (int d = 0; d < ND; ++d)
          if (d != e && X::co(t, d) != X::co(s, d)) on = false;
        if (on) v = sO1->G1[X::co(t, e)][X::co(s, e)];
      } else {
        int f = k - 1, m = snb[f];
        if (X::fax(f) == e) {
          // H_e^f[tau][sigma] = cb sum_{g on f} Cor[tau][g] nref_e(g) M0_m[P(g)][sigma]
          for (int gi = 0; gi < NFP; ++gi) {
            int g = f * NFP + gi;
            R c = sCor[t * NF + g];
            if (c != R(0)) v += c * R(X::fsg(f)) * sM0[(spg[g] - m * NF) * NS + s];
          }
          v *= cb;
        }
      }
    }
    R* gp = gam + (kk * NS + s) * GS + t * GE;
    gp[e] = v;
    if (e == 0) {
      gp[ND] = (k == 0 && t == s) ? R(1) : R(0);
      for (int z = ND + 1; z < GE; ++z) gp[z] = R(0);
    }
  }
  sync();
  // slr[k][sigma][g][SL_d.., SR_d..]: derivatives of the own / neighbour
  // physical face gradient at g w.r.t. u_k(sigma)
  for (int i = tid; i < nbk * NS * NF; i += nth) {
    int kk = i / (NS * NF), s = (i / NF) % NS, g = i % NF;
    int k = kb + kk;
    R* o = slr + (kk * NS + s) * SS + g * SE;
    int fg = g / NFP;
    for (int d2 = 0; d2 < ND; ++d2) {
      R sl = R(0), sr = R(0);
      if (visc) {
        // SL = sum_tau M0[g][tau] sum_e Jinv[tau][e][d2] gam_e[tau][sigma], tau on g's normal line
        for (int w = 0; w < N1; ++w) {
          int t = X::fline(g, w);
          R mv = sM0[g * NS + t];
          R acc = R(0);
          for (int e = 0; e < ND; ++e) acc += sJi[(t * ND + e) * ND + d2] * gam[(kk * NS + s) * GS + t * GE + e];
          sl += mv * acc;
        }
        if (k == 0) {
          sr = sW[(fg * NFP + (g - fg * NFP)) * ND + d2] * sM0[g * NS + s];
        } else if (fg == k - 1) {
          // neighbour's own gradient: sum_tau' M0[g2][tau'] sum_e Jinv_m[tau'][e][d2] G_e[tau'][sigma]
          int g2 = spg[g] - snb[fg] * NF;
          for (int w = 0; w < N1; ++w) {
            int t = X::fline(g2, w);
            R mv = sM0[g2 * NS + t];
            R acc = R(0);
            for (int e = 0; e < ND; ++e) {
              bool on = true;
              for (int d = 0; d < ND; ++d)
                if (d != e && X::co(t, d) != X::co(s, d)) on = false;
              if (on) acc += sJm[((fg * NS + t) * ND + e) * ND + d2] * sO1->G1[X::co(t, e)][X::co(s, e)];
            }
            sr += mv * acc;
          }
        }
      }
      o[2 + d2] = sl;
      o[2 + ND + d2] = sr;
    }
    o[0] = (k == 0) ? sM0[g * NS + s] : R(0);
    o[1] = (k > 0 && fg == k - 1) ? sM0[(spg[g] - snb[fg] * NF) * NS + s] : R(0);
    for (int z = 2 + 2 * ND; z < SE; ++z) o[z] = R(0);
  }
  sync();

  // ---------------------------------------------------------------- assembly
  // task = (block k, lane chunk, group of NBT input variables beta); lane
  // l = sigma*NV + alpha accumulates out[beta][rho] for its group in registers
  constexpr int LANES = NS * NV;
  constexpr int CHUNKS = (LANES + 63) / 64;
  constexpr int NBT = jac_tp_nbt<E, NV>();
  constexpr int NBG = (NV + NBT - 1) / NBT;
  const int nitems = nbk * CHUNKS * NBG * 64;
  bool bad = false;
  for (int item = tid; item < nitems; item += nth)
    bad |= jac_tp_task<E, NV, SYS, R, OT>(item, kb, o1, srd, tb, tf, gam, slr, Bn);
  if (bad) fr_flag_nonfinite(geo.status, FR_NF_BLOCKS, geo.e0 + nl);
  sync();
  }
}
