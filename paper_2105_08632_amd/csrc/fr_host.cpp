// Host-side set-up of the HIP path (see fr_host.hpp).
//
// Reference data are built here by a route of their own:
//   * Gauss-Legendre nodes and weights by the Golub-Welsch method (the
//     eigen-decomposition of the symmetric Jacobi matrix of the Legendre
//     recurrence, solved with cyclic Jacobi rotations);
//   * the nodal basis in barycentric form and its differentiation matrix;
//   * FR-DG correction functions through the nodal-DG lifting identity: on
//     Gauss-Legendre solution points the divergence of the correction
//     function of an end point is l_i(+-1)/w_i (the DG-recovering choice of
//     the paper's FR section), tensorised along the normal line.
//   * FR-SDRT / SDRT (tensor elements): the correction of an end point is the
//     derivative of the flux-point Lagrange polynomial that is 1 there, on the
//     SD flux points {-1, Gauss-Legendre points of order p, +1} (the
//     Raviart-Thomas basis of the external flux points), in barycentric form;
//   * triangles: orthonormal Dubiner basis from a Gauss-Jacobi quadrature mass
//     matrix, nodal basis by the inverse Vandermonde, lifting M^{-1} E;
//   * tetrahedra and prisms (FR-DG): products of Legendre polynomials of
//     total degree <= p (tetrahedra; the triangle part of prisms, times a
//     Legendre polynomial along the axis) as the modal basis, nodal basis by
//     the inverse Vandermonde, mass matrix and face integrals E by collapsed
//     Gauss-Legendre rules, lifting M^{-1} E.
#include "fr_host.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>

namespace frh {

// ---------------------------------------------------------------- 1-D
static void sym_eigen(int n, std::vector<double>& A, std::vector<double>& V) {
  V.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A[p * n + q] * A[p * n + q];
    if (off < 1e-34) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        double tau = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < n; ++k) {  // A <- A R
          double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // A <- R^T A
          double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
}

// Golub-Welsch for the Legendre weight on [-1, 1]: nodes ascending.
static void gl_golub_welsch(int n, std::vector<double>& x, std::vector<double>& w) {
  std::vector<double> A(n * n, 0.0), V;
  for (int k = 1; k < n; ++k) {
    double b = k / std::sqrt(4.0 * k * k - 1.0);
    A[(k - 1) * n + k] = b;
    A[k * n + k - 1] = b;
  }
  sym_eigen(n, A, V);
  std::vector<std::pair<double, double>> xw(n);
  for (int i = 0; i < n; ++i) xw[i] = {A[i * n + i], 2.0 * V[0 * n + i] * V[0 * n + i]};
  std::sort(xw.begin(), xw.end());
  x.resize(n); w.resize(n);
  for (int i = 0; i < n; ++i) {
    // symmetrise (the rule is exactly symmetric about 0)
    x[i] = 0.5 * (xw[i].first - xw[n - 1 - i].first);
    w[i] = 0.5 * (xw[i].second + xw[n - 1 - i].second);
  }
}

struct Bary {
  std::vector<double> x, bw;
  explicit Bary(const std::vector<double>& xs) : x(xs), bw(xs.size(), 1.0) {
    for (size_t j = 0; j < x.size(); ++j)
      for (size_t k = 0; k < x.size(); ++k)
        if (k != j) bw[j] /= (x[j] - x[k]);
  }
  // all basis values at t
  void eval(double t, std::vector<double>& l) const {
    const size_t n = x.size();
    l.assign(n, 0.0);
    for (size_t j = 0; j < n; ++j)
      if (t == x[j]) { l[j] = 1.0; return; }
    double den = 0.0;
    for (size_t j = 0; j < n; ++j) den += bw[j] / (t - x[j]);
    for (size_t j = 0; j < n; ++j) l[j] = bw[j] / (t - x[j]) / den;
  }
  // all basis derivatives at t (t not a node)
  void deriv(double t, std::vector<double>& d) const {
    const size_t n = x.size();
    std::vector<double> l;
    eval(t, l);
    double s = 0.0;
    for (size_t k = 0; k < n; ++k) s += 1.0 / (t - x[k]);
    d.assign(n, 0.0);
    for (size_t j = 0; j < n; ++j) d[j] = l[j] * (s - 1.0 / (t - x[j]));
  }
  // D_ij = l_j'(x_i)
  std::vector<double> diff() const {
    const size_t n = x.size();
    std::vector<double> D(n * n, 0.0);
    for (size_t i = 0; i < n; ++i) {
      double s = 0.0;
      for (size_t j = 0; j < n; ++j)
        if (j != i) { D[i * n + j] = (bw[j] / bw[i]) / (x[i] - x[j]); s += D[i * n + j]; }
      D[i * n + i] = -s;
    }
    return D;
  }
};

static bool compress(const std::vector<double>& M, int rows, int cols, int width, std::vector<int>& c,
                     std::vector<double>& v) {
  c.assign(rows * width, 0); v.assign(rows * width, 0.0);
  for (int r = 0; r < rows; ++r) {
    int k = 0;
    for (int j = 0; j < cols; ++j) {
      double a = M[(size_t)r * cols + j];
      if (a == 0.0) continue;
      if (k >= width) return false;
      c[r * width + k] = j; v[r * width + k] = a; ++k;
    }
  }
  return true;
}

static void finish_ops(RefOps& R, double beta) {
  const int nd = R.nd, ns = R.ns, nf = R.nf;
  R.Dc.assign(nd * ns * ns, 0.0);
  R.G.assign(nd * ns * ns, 0.0);
  for (int d = 0; d < nd; ++d)
    for (int r = 0; r < ns; ++r)
      for (int s = 0; s < ns; ++s) {
        double cm = 0.0;
        for (int g = 0; g < nf; ++g) cm += R.Cor[r * nf + g] * R.nref[g * nd + d] * R.M0[g * ns + s];
        double dd = R.D[(d * ns + r) * ns + s];
        R.Dc[(d * ns + r) * ns + s] = dd - cm;
        R.G[(d * ns + r) * ns + s] = dd - (0.5 + beta) * cm;
      }
}

static void build_tensor(RefOps& R, int type, int p, int scheme) {
  const int n1 = p + 1;
  const int nd = (type == QUAD) ? 2 : 3;
  R.type = type; R.p = p; R.nd = nd;
  R.ns = (nd == 2) ? n1 * n1 : n1 * n1 * n1;
  R.nface = 2 * nd;
  R.nfp = (nd == 2) ? n1 : n1 * n1;
  R.nf = R.nface * R.nfp;
  R.nvert = (nd == 2) ? 4 : 8;
  R.wl = n1; R.wc = 2 * nd;
  std::vector<double> x, w;
  gl_golub_welsch(n1, x, w);
  Bary B(x);
  std::vector<double> D1 = B.diff(), lp, lm;
  B.eval(1.0, lp); B.eval(-1.0, lm);
  std::vector<double> hp(n1), hm(n1);
  for (int i = 0; i < n1; ++i) { hp[i] = lp[i] / w[i]; hm[i] = lm[i] / w[i]; }
  R.scheme = scheme;
  if (scheme != 0) {
    // SD flux points: -1, the p Gauss-Legendre points of order p, +1
    std::vector<double> zi, wi;
    gl_golub_welsch(p, zi, wi);
    std::vector<double> z(1, -1.0);
    z.insert(z.end(), zi.begin(), zi.end());
    z.push_back(1.0);
    Bary Bz(z);
    R.sdz = z;
    R.sdD.assign(n1 * (p + 2), 0.0);
    std::vector<double> d;
    for (int i = 0; i < n1; ++i) {
      Bz.deriv(x[i], d);
      for (int j = 0; j < p + 2; ++j) R.sdD[i * (p + 2) + j] = d[j];
      hp[i] = d[p + 1];      // div of the +1 end's basis function
      hm[i] = -d[0];         // outward normal -1 at the other end
    }
    R.sdI.assign(p * n1, 0.0);
    std::vector<double> l;
    for (int j = 0; j < p; ++j) {
      B.eval(z[j + 1], l);
      for (int i = 0; i < n1; ++i) R.sdI[j * n1 + i] = l[i];
    }
  }
  R.D1 = D1; R.hp = hp; R.hm = hm; R.lp = lp; R.lm = lm;

  auto sidx = [&](int r, int d) { return d == 0 ? r % n1 : (d == 1 ? (r / n1) % n1 : r / (n1 * n1)); };
  R.sp.assign(R.ns * nd, 0.0); R.wsol.assign(R.ns, 1.0);
  for (int r = 0; r < R.ns; ++r)
    for (int d = 0; d < nd; ++d) { R.sp[r * nd + d] = x[sidx(r, d)]; R.wsol[r] *= w[sidx(r, d)]; }

  // faces: normal axis / sign, and per flux point the tangential node indices
  struct F { int ax, sg; };
  std::vector<F> faces;
  if (nd == 2) {
    faces = {{1, -1}, {0, +1}, {1, +1}, {0, -1}};
    R.face_verts = {{0, 1}, {1, 2}, {2, 3}, {3, 0}};
  } else {
    faces = {{2, -1}, {1, -1}, {0, +1}, {1, +1}, {0, -1}, {2, +1}};
    R.face_verts = {{0, 1, 2, 3}, {0, 1, 5, 4}, {1, 2, 6, 5}, {2, 3, 7, 6}, {3, 0, 4, 7}, {4, 5, 6, 7}};
  }
  R.fp.assign(R.nf * nd, 0.0); R.nref.assign(R.nf * nd, 0.0); R.fface.assign(R.nf, 0);
  std::vector<int> fidx(R.nf * 3, -1);  // node index per axis (-1 on the normal axis)
  for (int f = 0; f < R.nface; ++f) {
    int ax = faces[f].ax, sg = faces[f].sg;
    for (int t = 0; t < R.nfp; ++t) {
      int g = f * R.nfp + t;
      R.fface[g] = f;
      R.nref[g * nd + ax] = sg;
      int ta = t % n1, tb = t / n1;
      if (nd == 2) {
        int other = 1 - ax;
        int i = (f == 0 || f == 1) ? ta : (n1 - 1 - ta);   // counter-clockwise along the edge
        fidx[g * 3 + other] = i;
      } else {
        int k = 0;
        for (int d = 0; d < 3; ++d)
          if (d != ax) fidx[g * 3 + d] = (k++ == 0) ? ta : tb;
      }
      for (int d = 0; d < nd; ++d) R.fp[g * nd + d] = (d == ax) ? sg : x[fidx[g * 3 + d]];
    }
  }
  if (scheme != 0) {
    // external flux points at the ends of each line (tangential indices of
    // the other axes in increasing axis order, as the line numbering)
    const int nl = R.ns / n1;
    R.sdend.assign(nd * nl * 2, -1);
    for (int d = 0; d < nd; ++d)
      for (int l = 0; l < nl; ++l) {
        int tan[3] = {-1, -1, -1}, rem = l;
        for (int e = 0; e < nd; ++e)
          if (e != d) { tan[e] = rem % n1; rem /= n1; }
        for (int g = 0; g < R.nf; ++g) {
          const int f = R.fface[g];
          if (faces[f].ax != d) continue;
          bool on = true;
          for (int e = 0; e < nd; ++e)
            if (e != d && fidx[g * 3 + e] != tan[e]) on = false;
          if (on) R.sdend[(d * nl + l) * 2 + (faces[f].sg > 0 ? 1 : 0)] = g;
        }
      }
  }
  R.M0.assign(R.nf * R.ns, 0.0);
  R.Cor.assign(R.ns * R.nf, 0.0);
  for (int g = 0; g < R.nf; ++g) {
    int f = R.fface[g], ax = faces[f].ax, sg = faces[f].sg;
    const std::vector<double>& le = (sg > 0) ? lp : lm;
    const std::vector<double>& he = (sg > 0) ? hp : hm;
    for (int r = 0; r < R.ns; ++r) {
      bool on = true;
      for (int d = 0; d < nd; ++d)
        if (d != ax && sidx(r, d) != fidx[g * 3 + d]) on = false;
      if (!on) continue;
      R.M0[g * R.ns + r] = le[sidx(r, ax)];
      R.Cor[r * R.nf + g] = he[sidx(r, ax)];
    }
  }
  R.D.assign(nd * R.ns * R.ns, 0.0);
  for (int d = 0; d < nd; ++d)
    for (int r = 0; r < R.ns; ++r)
      for (int s = 0; s < R.ns; ++s) {
        bool on = true;
        for (int e = 0; e < nd; ++e)
          if (e != d && sidx(r, e) != sidx(s, e)) on = false;
        if (on) R.D[(d * R.ns + r) * R.ns + s] = D1[sidx(r, d) * n1 + sidx(s, d)];
      }
}

// ---------------------------------------------------------------- triangles
// Orthonormal Dubiner basis psi_ij(r,s) and its gradient, by the collapsed
// coordinates with the scaled recurrences (regular at the top vertex).
static void dubiner_tri(int i, int j, double r, double s, double& v, double& dr, double& ds) {
  // Q_k(x,t) = t^k P_k(x/t), x = (1+2r+s)/2, t = (1-s)/2; dQ/dx, dQ/dt
  double x = 0.5 * (1.0 + 2.0 * r + s), t = 0.5 * (1.0 - s);
  double q0 = 1.0, q1 = x, qx0 = 0.0, qx1 = 1.0, qt0 = 0.0, qt1 = 0.0;
  double Q = 1.0, Qx = 0.0, Qt = 0.0;
  if (i >= 1) { Q = q1; Qx = qx1; Qt = qt1; }
  for (int k = 2; k <= i; ++k) {
    double a = (2.0 * k - 1.0) / k, b = (k - 1.0) / k;
    double q2 = a * x * q1 - b * t * t * q0;
    double qx2 = a * (q1 + x * qx1) - b * t * t * qx0;
    double qt2 = a * x * qt1 - b * (2.0 * t * q0 + t * t * qt0);
    q0 = q1; q1 = q2; qx0 = qx1; qx1 = qx2; qt0 = qt1; qt1 = qt2;
    Q = q2; Qx = qx2; Qt = qt2;
  }
  // Jacobi P_j^{(al,0)}(s) and derivative
  const double al = 2.0 * i + 1.0;
  double p0 = 1.0, p1 = 0.5 * (al + 2.0) * s + 0.5 * al, d0 = 0.0, d1 = 0.5 * (al + 2.0);
  double Pj = 1.0, dPj = 0.0;
  if (j >= 1) { Pj = p1; dPj = d1; }
  for (int k = 2; k <= j; ++k) {
    double a1 = 2.0 * k * (k + al) * (2.0 * k + al - 2.0);
    double a2 = (2.0 * k + al - 1.0) * (al * al);
    double a3 = (2.0 * k + al - 2.0) * (2.0 * k + al - 1.0) * (2.0 * k + al);
    double a4 = 2.0 * (k + al - 1.0) * (k - 1.0) * (2.0 * k + al);
    double p2 = ((a2 + a3 * s) * p1 - a4 * p0) / a1;
    double dd2 = ((a2 + a3 * s) * d1 + a3 * p1 - a4 * d0) / a1;
    p0 = p1; p1 = p2; d0 = d1; d1 = dd2;
    Pj = p2; dPj = dd2;
  }
  double c = std::sqrt((2.0 * i + 1.0) * (i + j + 1.0) / 2.0);
  // dx/dr = 1, dx/ds = 1/2, dt/dr = 0, dt/ds = -1/2
  v = c * Q * Pj;
  dr = c * Qx * Pj;
  ds = c * ((0.5 * Qx - 0.5 * Qt) * Pj + Q * dPj);
}

static bool invert_dense(std::vector<double> A, int n, std::vector<double>& inv) {
  inv.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0.0) return false;
    for (int k = 0; k < n; ++k) { std::swap(A[c * n + k], A[piv * n + k]); std::swap(inv[c * n + k], inv[piv * n + k]); }
    double d = A[c * n + c];
    for (int k = 0; k < n; ++k) { A[c * n + k] /= d; inv[c * n + k] /= d; }
    for (int r = 0; r < n; ++r)
      if (r != c) {
        double f = A[r * n + c];
        if (f == 0.0) continue;
        for (int k = 0; k < n; ++k) { A[r * n + k] -= f * A[c * n + k]; inv[r * n + k] -= f * inv[c * n + k]; }
      }
  }
  return true;
}

static bool build_tri(RefOps& R, int p, const double* pts, std::string& err) {
  const int n1 = p + 1, ns = (p + 1) * (p + 2) / 2;
  R.type = TRI; R.p = p; R.nd = 2; R.ns = ns; R.nface = 3; R.nfp = n1; R.nf = 3 * n1; R.nvert = 3;
  R.wl = ns; R.wc = R.nf;
  R.face_verts = {{0, 1}, {1, 2}, {2, 0}};
  R.sp.assign(pts, pts + 2 * ns);
  std::vector<std::pair<int, int>> modes;
  for (int i = 0; i <= p; ++i)
    for (int j = 0; i + j <= p; ++j) modes.push_back({i, j});
  // V[r][m] = psi_m(x_r); nodal l_s = sum_m Vinv[m][s] psi_m
  std::vector<double> V(ns * ns), Vr(ns * ns), Vs(ns * ns), Vinv;
  for (int r = 0; r < ns; ++r)
    for (int m = 0; m < ns; ++m)
      dubiner_tri(modes[m].first, modes[m].second, pts[2 * r], pts[2 * r + 1], V[r * ns + m], Vr[r * ns + m], Vs[r * ns + m]);
  if (!invert_dense(V, ns, Vinv)) { err = "triangle solution points are not unisolvent"; return false; }
  auto nodal = [&](double r, double s, std::vector<double>& l) {
    l.assign(ns, 0.0);
    for (int m = 0; m < ns; ++m) {
      double v, a, b;
      dubiner_tri(modes[m].first, modes[m].second, r, s, v, a, b);
      for (int q = 0; q < ns; ++q) l[q] += Vinv[m * ns + q] * v;
    }
  };
  // derivative matrices D_d[r][s] = sum_m dpsi_m/dxi_d(x_r) Vinv[m][s]
  R.D.assign(2 * ns * ns, 0.0);
  for (int r = 0; r < ns; ++r)
    for (int s = 0; s < ns; ++s) {
      double a = 0.0, b = 0.0;
      for (int m = 0; m < ns; ++m) { a += Vr[r * ns + m] * Vinv[m * ns + s]; b += Vs[r * ns + m] * Vinv[m * ns + s]; }
      R.D[(0 * ns + r) * ns + s] = a;
      R.D[(1 * ns + r) * ns + s] = b;
    }
  // mass matrix by a collapsed Gauss-Jacobi rule of degree >= 2p
  std::vector<double> ga, wa;
  gl_golub_welsch(p + 2, ga, wa);
  std::vector<double> Mm(ns * ns, 0.0), l;
  for (int ia = 0; ia < p + 2; ++ia)
    for (int ib = 0; ib < p + 2; ++ib) {
      double a = ga[ia], b = ga[ib];
      double r = 0.5 * (1.0 + a) * (1.0 - b) - 1.0, s = b;
      double wt = wa[ia] * wa[ib] * 0.5 * (1.0 - b);
      nodal(r, s, l);
      for (int i = 0; i < ns; ++i)
        for (int j = 0; j < ns; ++j) Mm[i * ns + j] += wt * l[i] * l[j];
    }
  std::vector<double> Minv;
  if (!invert_dense(Mm, ns, Minv)) { err = "singular triangle mass matrix"; return false; }
  std::vector<double> x, w;
  gl_golub_welsch(n1, x, w);
  const double E[3][2][2] = {{{-1, -1}, {1, -1}}, {{1, -1}, {-1, 1}}, {{-1, 1}, {-1, -1}}};
  const double nr[3][2] = {{0, -1}, {M_SQRT1_2, M_SQRT1_2}, {-1, 0}};
  const double elen[3] = {2.0, 2.0 * M_SQRT2, 2.0};
  R.fp.assign(R.nf * 2, 0.0); R.nref.assign(R.nf * 2, 0.0); R.fface.assign(R.nf, 0);
  std::vector<double> fw(R.nf);
  R.M0.assign(R.nf * ns, 0.0);
  for (int f = 0; f < 3; ++f)
    for (int t = 0; t < n1; ++t) {
      int g = f * n1 + t;
      double sp = 0.5 * (x[t] + 1.0);
      R.fp[g * 2] = E[f][0][0] + sp * (E[f][1][0] - E[f][0][0]);
      R.fp[g * 2 + 1] = E[f][0][1] + sp * (E[f][1][1] - E[f][0][1]);
      R.nref[g * 2] = nr[f][0]; R.nref[g * 2 + 1] = nr[f][1];
      R.fface[g] = f;
      fw[g] = w[t] * elen[f] / 2.0;
      nodal(R.fp[g * 2], R.fp[g * 2 + 1], l);
      for (int s = 0; s < ns; ++s) R.M0[g * ns + s] = l[s];
    }
  R.Cor.assign(ns * R.nf, 0.0);
  for (int r = 0; r < ns; ++r)
    for (int g = 0; g < R.nf; ++g) {
      double acc = 0.0;
      for (int j = 0; j < ns; ++j) acc += Minv[r * ns + j] * R.M0[g * ns + j] * fw[g];
      R.Cor[r * R.nf + g] = acc;
    }
  R.wsol.assign(ns, 0.0);
  for (int r = 0; r < ns; ++r)
    for (int j = 0; j < ns; ++j) R.wsol[r] += Mm[r * ns + j];
  return true;
}

// ---------------------------------------------------- tetrahedra and prisms
// Legendre P_n and its derivative at x.
static void legendre_pd(int n, double x, double& P, double& dP) {
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  if (n == 0) { P = 1.0; dP = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    const double d2 = d0 + (2.0 * k - 1.0) * p1;
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  P = p1; dP = d1;
}

// A 3-D face: flux points, unit outward normal, a quadrature rule (reference
// surface measure) and the face's nodal basis at the rule's points.
struct Face3 {
  std::vector<double> fp, qx, qw, phi;
  double n[3];
};

// Triangle nodal basis on the caller's points: 2-D Legendre products of total
// degree <= p through the inverse Vandermonde.
struct TriNodal {
  int nt = 0;
  std::vector<std::pair<int, int>> modes;
  std::vector<double> Vinv;
  bool init(int p, const double* pts) {
    nt = (p + 1) * (p + 2) / 2;
    for (int a = 0; a <= p; ++a)
      for (int b = 0; a + b <= p; ++b) modes.push_back({a, b});
    std::vector<double> V(nt * nt);
    for (int r = 0; r < nt; ++r)
      for (int m = 0; m < nt; ++m) V[r * nt + m] = mode(m, pts[2 * r], pts[2 * r + 1]);
    return invert_dense(V, nt, Vinv);
  }
  double mode(int m, double a, double b) const {
    double Pa, dPa, Pb, dPb;
    legendre_pd(modes[m].first, a, Pa, dPa);
    legendre_pd(modes[m].second, b, Pb, dPb);
    return Pa * Pb;
  }
  void eval(double a, double b, std::vector<double>& l) const {
    l.assign(nt, 0.0);
    for (int m = 0; m < nt; ++m) {
      const double v = mode(m, a, b);
      for (int q = 0; q < nt; ++q) l[q] += Vinv[m * nt + q] * v;
    }
  }
};

static void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1]; c[1] = a[2] * b[0] - a[0] * b[2]; c[2] = a[0] * b[1] - a[1] * b[0];
}

// Triangular face with vertices A, B, C; points and rule mapped through the
// barycentric coordinates of the 2-D reference triangle.
static Face3 face_tri(const double* A, const double* B, const double* C, const double* n, int p, const double* pts,
                      const TriNodal& tn) {
  Face3 F;
  for (int k = 0; k < 3; ++k) F.n[k] = n[k];
  auto map = [&](double a, double b, double* X) {
    const double l0 = -0.5 * (a + b), l1 = 0.5 * (1 + a), l2 = 0.5 * (1 + b);
    for (int k = 0; k < 3; ++k) X[k] = l0 * A[k] + l1 * B[k] + l2 * C[k];
  };
  for (int i = 0; i < tn.nt; ++i) {
    double X[3]; map(pts[2 * i], pts[2 * i + 1], X);
    F.fp.insert(F.fp.end(), X, X + 3);
  }
  double e1[3], e2[3], cr[3];
  for (int k = 0; k < 3; ++k) { e1[k] = B[k] - A[k]; e2[k] = C[k] - A[k]; }
  cross3(e1, e2, cr);
  const double area = 0.5 * std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
  std::vector<double> g, w, l;
  gl_golub_welsch(p + 2, g, w);
  for (int i = 0; i < p + 2; ++i)
    for (int j = 0; j < p + 2; ++j) {
      const double a = 0.5 * (1 + g[i]) * (1 - g[j]) - 1, b = g[j];
      double X[3]; map(a, b, X);
      F.qx.insert(F.qx.end(), X, X + 3);
      F.qw.push_back(w[i] * w[j] * 0.5 * (1 - g[j]) * area / 2.0);   // the 2-D reference triangle has area 2
      tn.eval(a, b, l);
      F.phi.insert(F.phi.end(), l.begin(), l.end());
    }
  return F;
}

// Parallelogram face A + u (B - A) + v (D - A), u, v in [0, 1]: Gauss-Legendre
// points (the rule of its own nodal basis).
static Face3 face_quad(const double* A, const double* B, const double* D, const double* n, int p) {
  Face3 F;
  for (int k = 0; k < 3; ++k) F.n[k] = n[k];
  const int n1 = p + 1;
  std::vector<double> g, w;
  gl_golub_welsch(n1, g, w);
  double e1[3], e2[3], cr[3];
  for (int k = 0; k < 3; ++k) { e1[k] = B[k] - A[k]; e2[k] = D[k] - A[k]; }
  cross3(e1, e2, cr);
  const double area = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
  for (int j = 0; j < n1; ++j)
    for (int i = 0; i < n1; ++i) {
      double X[3];
      for (int k = 0; k < 3; ++k) X[k] = A[k] + 0.5 * (1 + g[i]) * e1[k] + 0.5 * (1 + g[j]) * e2[k];
      F.fp.insert(F.fp.end(), X, X + 3);
      F.qx.insert(F.qx.end(), X, X + 3);
      F.qw.push_back(w[i] * w[j] * area / 4.0);
    }
  const int nq = n1 * n1;
  F.phi.assign(nq * nq, 0.0);
  for (int a = 0; a < nq; ++a) F.phi[a * nq + a] = 1.0;
  return F;
}

// Operators of a 3-D element from a modal basis (values and gradients),
// solution points, a volume rule and its faces.  The modal basis is first
// made orthonormal on the element (Cholesky factor of its Gram matrix under
// the volume rule), which keeps the Vandermonde matrix well conditioned.
template <class Modal0>
static bool build_3d(RefOps& R, int nm, const Modal0& modal0, const std::vector<double>& sp,
                     const std::vector<double>& vq, const std::vector<double>& vw, const std::vector<Face3>& faces,
                     std::string& err) {
  const int ns = (int)sp.size() / 3;
  R.nd = 3; R.ns = ns; R.sp = sp;
  if (nm != ns) { err = "solution point count does not match the polynomial space"; return false; }
  // Gram matrix and its Cholesky factor G = L L^T; psi = L^{-1} phi
  std::vector<double> Gm(nm * nm, 0.0), Lc(nm * nm, 0.0), Li(nm * nm, 0.0), phv(nm);
  for (size_t a = 0; a < vw.size(); ++a) {
    double g[3];
    for (int m = 0; m < nm; ++m) phv[m] = modal0(m, &vq[3 * a], g);
    for (int i = 0; i < nm; ++i)
      for (int j = 0; j < nm; ++j) Gm[i * nm + j] += vw[a] * phv[i] * phv[j];
  }
  for (int j = 0; j < nm; ++j) {
    double d = Gm[j * nm + j];
    for (int k = 0; k < j; ++k) d -= Lc[j * nm + k] * Lc[j * nm + k];
    if (!(d > 0.0)) { err = "modal basis is not independent on the element"; return false; }
    Lc[j * nm + j] = std::sqrt(d);
    for (int i = j + 1; i < nm; ++i) {
      double v = Gm[i * nm + j];
      for (int k = 0; k < j; ++k) v -= Lc[i * nm + k] * Lc[j * nm + k];
      Lc[i * nm + j] = v / Lc[j * nm + j];
    }
  }
  for (int c = 0; c < nm; ++c)          // L^{-1} by forward substitution, column by column
    for (int i = 0; i < nm; ++i) {
      double v = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) v -= Lc[i * nm + k] * Li[k * nm + c];
      Li[i * nm + c] = v / Lc[i * nm + i];
    }
  auto modal = [&](int m, const double* X, double* g) {
    double v = 0.0, gk[3];
    g[0] = g[1] = g[2] = 0.0;
    for (int k = 0; k <= m; ++k) {
      const double c = Li[m * nm + k];
      if (c == 0.0) continue;
      v += c * modal0(k, X, gk);
      for (int d = 0; d < 3; ++d) g[d] += c * gk[d];
    }
    return v;
  };
  std::vector<double> V(ns * ns), Vg(3 * ns * ns), Vinv;
  for (int r = 0; r < ns; ++r)
    for (int m = 0; m < ns; ++m) {
      double g[3];
      V[r * ns + m] = modal(m, &sp[3 * r], g);
      for (int d = 0; d < 3; ++d) Vg[(d * ns + r) * ns + m] = g[d];
    }
  if (!invert_dense(V, ns, Vinv)) { err = "solution points are not unisolvent"; return false; }
  auto nodal = [&](const double* X, std::vector<double>& l) {
    l.assign(ns, 0.0);
    double g[3];
    for (int m = 0; m < ns; ++m) {
      const double v = modal(m, X, g);
      for (int q = 0; q < ns; ++q) l[q] += Vinv[m * ns + q] * v;
    }
  };
  R.D.assign(3 * ns * ns, 0.0);
  for (int d = 0; d < 3; ++d)
    for (int r = 0; r < ns; ++r)
      for (int s = 0; s < ns; ++s) {
        double acc = 0.0;
        for (int m = 0; m < ns; ++m) acc += Vg[(d * ns + r) * ns + m] * Vinv[m * ns + s];
        R.D[(d * ns + r) * ns + s] = acc;
      }
  R.nface = (int)faces.size();
  R.face_off.assign(1, 0);
  R.fp.clear(); R.nref.clear(); R.fface.clear();
  R.nfp = 0;
  for (int f = 0; f < R.nface; ++f) {
    const int nfp = (int)faces[f].fp.size() / 3;
    R.nfp = std::max(R.nfp, nfp);
    R.face_off.push_back(R.face_off.back() + nfp);
    R.fp.insert(R.fp.end(), faces[f].fp.begin(), faces[f].fp.end());
    for (int g = 0; g < nfp; ++g) {
      R.nref.insert(R.nref.end(), faces[f].n, faces[f].n + 3);
      R.fface.push_back(f);
    }
  }
  R.nf = R.face_off.back();
  std::vector<double> l;
  R.M0.assign(R.nf * ns, 0.0);
  for (int g = 0; g < R.nf; ++g) {
    nodal(&R.fp[3 * g], l);
    for (int s = 0; s < ns; ++s) R.M0[g * ns + s] = l[s];
  }
  std::vector<double> Mm(ns * ns, 0.0), Minv;
  for (size_t a = 0; a < vw.size(); ++a) {
    nodal(&vq[3 * a], l);
    for (int i = 0; i < ns; ++i)
      for (int j = 0; j < ns; ++j) Mm[i * ns + j] += vw[a] * l[i] * l[j];
  }
  if (!invert_dense(Mm, ns, Minv)) { err = "singular mass matrix"; return false; }
  std::vector<double> E(ns * R.nf, 0.0);
  for (int f = 0; f < R.nface; ++f) {
    const Face3& F = faces[f];
    const int nfp = R.face_off[f + 1] - R.face_off[f];
    for (size_t a = 0; a < F.qw.size(); ++a) {
      nodal(&F.qx[3 * a], l);
      for (int j = 0; j < ns; ++j)
        for (int g = 0; g < nfp; ++g) E[j * R.nf + R.face_off[f] + g] += F.qw[a] * l[j] * F.phi[a * nfp + g];
    }
  }
  R.Cor.assign(ns * R.nf, 0.0);
  for (int r = 0; r < ns; ++r)
    for (int g = 0; g < R.nf; ++g) {
      double acc = 0.0;
      for (int j = 0; j < ns; ++j) acc += Minv[r * ns + j] * E[j * R.nf + g];
      R.Cor[r * R.nf + g] = acc;
    }
  R.wsol.assign(ns, 0.0);
  for (int r = 0; r < ns; ++r)
    for (int j = 0; j < ns; ++j) R.wsol[r] += Mm[r * ns + j];
  R.wl = ns; R.wc = R.nf;
  return true;
}

static bool build_tet(RefOps& R, int p, const double* tet_pts, const double* tri_pts, std::string& err) {
  R.type = TET; R.p = p; R.nvert = 4;
  const double v[4][3] = {{-1, -1, -1}, {1, -1, -1}, {-1, 1, -1}, {-1, -1, 1}};
  R.face_verts = {{0, 1, 2}, {0, 1, 3}, {1, 2, 3}, {0, 2, 3}};
  const double q3 = 1.0 / std::sqrt(3.0);
  const double nrm[4][3] = {{0, 0, -1}, {0, -1, 0}, {q3, q3, q3}, {-1, 0, 0}};
  TriNodal tn;
  if (!tn.init(p, tri_pts)) { err = "face points are not unisolvent"; return false; }
  std::vector<Face3> faces;
  for (int f = 0; f < 4; ++f)
    faces.push_back(face_tri(v[R.face_verts[f][0]], v[R.face_verts[f][1]], v[R.face_verts[f][2]], nrm[f], p, tri_pts, tn));
  std::vector<std::array<int, 3>> modes;
  for (int a = 0; a <= p; ++a)
    for (int b = 0; a + b <= p; ++b)
      for (int c = 0; a + b + c <= p; ++c) modes.push_back({a, b, c});
  const int ns = (int)modes.size();
  auto modal = [&](int m, const double* X, double* g) {
    double P[3], dP[3];
    for (int d = 0; d < 3; ++d) legendre_pd(modes[m][d], X[d], P[d], dP[d]);
    g[0] = dP[0] * P[1] * P[2]; g[1] = P[0] * dP[1] * P[2]; g[2] = P[0] * P[1] * dP[2];
    return P[0] * P[1] * P[2];
  };
  // collapsed Gauss-Legendre rule on the tetrahedron (volume 4/3)
  std::vector<double> gq, gw, vq, vw;
  gl_golub_welsch(p + 3, gq, gw);
  for (int i = 0; i < p + 3; ++i)
    for (int j = 0; j < p + 3; ++j)
      for (int k = 0; k < p + 3; ++k) {
        const double a = gq[i], b = gq[j], c = gq[k];
        vq.push_back(0.25 * (1 + a) * (1 - b) * (1 - c) - 1);
        vq.push_back(0.5 * (1 + b) * (1 - c) - 1);
        vq.push_back(c);
        vw.push_back(gw[i] * gw[j] * gw[k] * (1 - b) * (1 - c) * (1 - c) / 8.0);
      }
  std::vector<double> sp(tet_pts, tet_pts + 3 * ns);
  return build_3d(R, ns, modal, sp, vq, vw, faces, err);
}

static bool build_pri(RefOps& R, int p, const double* tri_pts, std::string& err) {
  R.type = PRI; R.p = p; R.nvert = 6;
  const double v[6][3] = {{-1, -1, -1}, {1, -1, -1}, {-1, 1, -1}, {-1, -1, 1}, {1, -1, 1}, {-1, 1, 1}};
  R.face_verts = {{0, 1, 2}, {3, 4, 5}, {0, 1, 4, 3}, {1, 2, 5, 4}, {2, 0, 3, 5}};
  const double h = M_SQRT1_2;
  const double nrm[5][3] = {{0, 0, -1}, {0, 0, 1}, {0, -1, 0}, {h, h, 0}, {-1, 0, 0}};
  TriNodal tn;
  if (!tn.init(p, tri_pts)) { err = "triangle points are not unisolvent"; return false; }
  std::vector<Face3> faces;
  faces.push_back(face_tri(v[0], v[1], v[2], nrm[0], p, tri_pts, tn));
  faces.push_back(face_tri(v[3], v[4], v[5], nrm[1], p, tri_pts, tn));
  faces.push_back(face_quad(v[0], v[1], v[3], nrm[2], p));
  faces.push_back(face_quad(v[1], v[2], v[4], nrm[3], p));
  faces.push_back(face_quad(v[2], v[0], v[5], nrm[4], p));
  const int nt = (p + 1) * (p + 2) / 2, n1 = p + 1;
  std::vector<std::array<int, 3>> modes;
  for (int c = 0; c <= p; ++c)
    for (int a = 0; a <= p; ++a)
      for (int b = 0; a + b <= p; ++b) modes.push_back({a, b, c});
  auto modal = [&](int m, const double* X, double* g) {
    double P[3], dP[3];
    for (int d = 0; d < 3; ++d) legendre_pd(modes[m][d], X[d], P[d], dP[d]);
    g[0] = dP[0] * P[1] * P[2]; g[1] = P[0] * dP[1] * P[2]; g[2] = P[0] * P[1] * dP[2];
    return P[0] * P[1] * P[2];
  };
  std::vector<double> gx, gwx;
  gl_golub_welsch(n1, gx, gwx);
  std::vector<double> sp;                    // triangle point i at axis point k: index i + nt k
  for (int k = 0; k < n1; ++k)
    for (int i = 0; i < nt; ++i) { sp.push_back(tri_pts[2 * i]); sp.push_back(tri_pts[2 * i + 1]); sp.push_back(gx[k]); }
  std::vector<double> gq, gw, vq, vw;
  gl_golub_welsch(p + 2, gq, gw);
  for (int i = 0; i < p + 2; ++i)
    for (int j = 0; j < p + 2; ++j)
      for (int k = 0; k < p + 2; ++k) {
        vq.push_back(0.5 * (1 + gq[i]) * (1 - gq[j]) - 1);
        vq.push_back(gq[j]);
        vq.push_back(gq[k]);
        vw.push_back(gw[i] * gw[j] * gw[k] * 0.5 * (1 - gq[j]));
      }
  return build_3d(R, (int)modes.size(), modal, sp, vq, vw, faces, err);
}

bool build_ref(int type, int p, double beta, int scheme, const double* tri_pts, const double* tet_pts, RefOps& R,
               std::string& err) {
  if (p < 1 || p > 4) { err = "degree must be in 1..4"; return false; }
  if (scheme < 0 || scheme > 2) { err = "unknown scheme"; return false; }
  if (scheme != 0 && type != QUAD && type != HEX) {
    err = "FR-SDRT and SDRT are provided for quadrilaterals and hexahedra";
    return false;
  }
  if (type == QUAD || type == HEX) build_tensor(R, type, p, scheme);
  else if (type == TRI) {
    if (!tri_pts) { err = "triangles need tri_sol_pts"; return false; }
    if (!build_tri(R, p, tri_pts, err)) return false;
  } else if (type == TET) {
    if (!tri_pts || !tet_pts) { err = "tetrahedra need tri_sol_pts (faces) and tet_sol_pts"; return false; }
    if (!build_tet(R, p, tet_pts, tri_pts, err)) return false;
  } else if (type == PRI) {
    if (!tri_pts) { err = "prisms need tri_sol_pts"; return false; }
    if (!build_pri(R, p, tri_pts, err)) return false;
  } else { err = "unknown element type"; return false; }
  if (R.face_off.empty()) {
    R.face_off.assign(R.nface + 1, 0);
    for (int f = 0; f <= R.nface; ++f) R.face_off[f] = f * R.nfp;
  }
  finish_ops(R, beta);
  bool ok = compress(R.M0, R.nf, R.ns, R.wl, R.m0c, R.m0v) &&
            compress(R.Dc, R.nd * R.ns, R.ns, R.wl, R.dcc, R.dcv) &&
            compress(R.G, R.nd * R.ns, R.ns, R.wl, R.gc, R.gv) &&
            compress(R.Cor, R.ns, R.nf, R.wc, R.crc, R.crv) &&
            compress(R.D, R.nd * R.ns, R.ns, R.wl, R.ddc, R.ddv);
  if (!ok) { err = "operator sparsity exceeds the element's row width"; return false; }
  return true;
}

// ---------------------------------------------------------------- geometry
static void shape(int type, const double* xi, double* N, double* dN) {
  if (type == QUAD) {
    static const double V[4][2] = {{-1, -1}, {1, -1}, {1, 1}, {-1, 1}};
    for (int v = 0; v < 4; ++v) {
      N[v] = 0.25 * (1 + V[v][0] * xi[0]) * (1 + V[v][1] * xi[1]);
      dN[v * 2] = 0.25 * V[v][0] * (1 + V[v][1] * xi[1]);
      dN[v * 2 + 1] = 0.25 * (1 + V[v][0] * xi[0]) * V[v][1];
    }
  } else if (type == HEX) {
    static const double V[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                                   {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};
    for (int v = 0; v < 8; ++v) {
      double a = 1 + V[v][0] * xi[0], b = 1 + V[v][1] * xi[1], c = 1 + V[v][2] * xi[2];
      N[v] = 0.125 * a * b * c;
      dN[v * 3] = 0.125 * V[v][0] * b * c;
      dN[v * 3 + 1] = 0.125 * a * V[v][1] * c;
      dN[v * 3 + 2] = 0.125 * a * b * V[v][2];
    }
  } else if (type == TET) {
    N[0] = -0.5 * (1 + xi[0] + xi[1] + xi[2]); N[1] = 0.5 * (1 + xi[0]); N[2] = 0.5 * (1 + xi[1]);
    N[3] = 0.5 * (1 + xi[2]);
    for (int k = 0; k < 12; ++k) dN[k] = 0.0;
    dN[0] = dN[1] = dN[2] = -0.5;
    dN[3] = 0.5; dN[7] = 0.5; dN[11] = 0.5;
  } else if (type == PRI) {
    const double L[3] = {-0.5 * (xi[0] + xi[1]), 0.5 * (1 + xi[0]), 0.5 * (1 + xi[1])};
    const double Lr[3] = {-0.5, 0.5, 0.0}, Ls[3] = {-0.5, 0.0, 0.5};
    for (int a = 0; a < 3; ++a) {
      const double zb = 0.5 * (1 - xi[2]), zt = 0.5 * (1 + xi[2]);
      N[a] = L[a] * zb; N[a + 3] = L[a] * zt;
      dN[a * 3] = Lr[a] * zb; dN[a * 3 + 1] = Ls[a] * zb; dN[a * 3 + 2] = -0.5 * L[a];
      dN[(a + 3) * 3] = Lr[a] * zt; dN[(a + 3) * 3 + 1] = Ls[a] * zt; dN[(a + 3) * 3 + 2] = 0.5 * L[a];
    }
  } else {
    N[0] = -0.5 * (xi[0] + xi[1]); N[1] = 0.5 * (1 + xi[0]); N[2] = 0.5 * (1 + xi[1]);
    dN[0] = -0.5; dN[1] = -0.5; dN[2] = 0.5; dN[3] = 0; dN[4] = 0; dN[5] = 0.5;
  }
}

static void mapping(const RefOps& R, int nd, const double* X /*[nvert][nd]*/, const double* xi, double* x, double* J) {
  double N[8], dN[24];
  shape(R.type, xi, N, dN);
  for (int i = 0; i < nd; ++i) {
    x[i] = 0.0;
    for (int j = 0; j < nd; ++j) J[i * nd + j] = 0.0;
  }
  for (int v = 0; v < R.nvert; ++v)
    for (int i = 0; i < nd; ++i) {
      x[i] += N[v] * X[v * nd + i];
      for (int j = 0; j < nd; ++j) J[i * nd + j] += X[v * nd + i] * dN[v * nd + j];
    }
}

static double adj(int nd, const double* J, double* S) {
  if (nd == 2) {
    S[0] = J[3]; S[1] = -J[1]; S[2] = -J[2]; S[3] = J[0];
    return J[0] * J[3] - J[1] * J[2];
  }
  S[0] = J[4] * J[8] - J[5] * J[7]; S[1] = J[2] * J[7] - J[1] * J[8]; S[2] = J[1] * J[5] - J[2] * J[4];
  S[3] = J[5] * J[6] - J[3] * J[8]; S[4] = J[0] * J[8] - J[2] * J[6]; S[5] = J[2] * J[3] - J[0] * J[5];
  S[6] = J[3] * J[7] - J[4] * J[6]; S[7] = J[1] * J[6] - J[0] * J[7]; S[8] = J[0] * J[4] - J[1] * J[3];
  return J[0] * S[0] + J[1] * S[3] + J[2] * S[6];
}

void build_sd_metric(const RefOps& R, int nd, int64_t ne, const double* xyz, int max_vert, std::vector<double>& Sint) {
  const int p = R.p, n1 = p + 1, nl = R.ns / n1;
  Sint.assign((size_t)ne * nd * nl * p * nd, 0.0);
  std::vector<double> X((size_t)R.nvert * nd);
  for (int64_t e = 0; e < ne; ++e) {
    for (int v = 0; v < R.nvert; ++v)
      for (int i = 0; i < nd; ++i) X[v * nd + i] = xyz[((size_t)e * max_vert + v) * nd + i];
    for (int d = 0; d < nd; ++d)
      for (int l = 0; l < nl; ++l) {
        int tan[3] = {0, 0, 0}, rem = l;
        for (int a = 0; a < nd; ++a)
          if (a != d) { tan[a] = rem % n1; rem /= n1; }
        for (int j = 0; j < p; ++j) {
          double xi[3], x[3], J[9], S[9];
          // 1-D node i is the first coordinate of solution point i
          for (int a = 0; a < nd; ++a) xi[a] = (a == d) ? R.sdz[j + 1] : R.sp[tan[a] * nd + 0];
          mapping(R, nd, X.data(), xi, x, J);
          adj(nd, J, S);
          for (int k = 0; k < nd; ++k)
            Sint[((((size_t)e * nd + d) * nl + l) * p + j) * nd + k] = S[d * nd + k];
        }
      }
  }
}

bool build_geometry_groups(const RefOps* const* refs, int nd, int64_t ne, const int8_t* etype, const double* xyz,
                           int max_vert, const int64_t* nbr, const int8_t* nbr_face, int max_face, int ngrp,
                           const int64_t* gstart, Geometry* G, MixInfo* mix, std::string& err) {
  char buf[256];
  // group of each element, and the first global flux point of each group
  std::vector<int> grp((size_t)ne, -1);
  std::vector<int64_t> fbase((size_t)ngrp + 1, 0);
  for (int g = 0; g < ngrp; ++g) {
    const RefOps& R = *refs[etype[gstart[g]]];
    for (int64_t e = gstart[g]; e < gstart[g + 1]; ++e) {
      if (etype[e] != etype[gstart[g]]) { err = "element types are not grouped"; return false; }
      grp[e] = g;
    }
    fbase[g + 1] = fbase[g] + (gstart[g + 1] - gstart[g]) * R.nf;
  }
  if (fbase[ngrp] > ((int64_t)1 << 31) - 1) { err = "mesh too large for 32-bit face indices"; return false; }
  auto ref_of = [&](int64_t e) -> const RefOps& { return *refs[etype[e]]; };
  auto gfp = [&](int64_t e, int j) -> int64_t {   // global flux point index
    const int g = grp[e];
    return fbase[g] + (e - gstart[g]) * ref_of(e).nf + j;
  };
  // physical flux-point positions, global numbering
  std::vector<double> fx((size_t)fbase[ngrp] * nd);
  for (int g = 0; g < ngrp; ++g) {
    const RefOps& R = *refs[etype[gstart[g]]];
    const int64_t ng = gstart[g + 1] - gstart[g];
    const int ns = R.ns, nf = R.nf;
    Geometry& Gg = G[g];
    Gg = Geometry();
    Gg.nd = nd; Gg.ns = ns; Gg.nf = nf; Gg.nface = R.nface; Gg.ne = ng;
    Gg.S.assign((size_t)ng * ns * nd * nd, 0.0);
    Gg.Jinv.assign((size_t)ng * ns * nd * nd, 0.0);
    Gg.rdet.assign((size_t)ng * ns, 0.0);
    Gg.nrm.assign((size_t)ng * nf * nd, 0.0);
    Gg.magN.assign((size_t)ng * nf, 0.0);
    Gg.nbfp.assign((size_t)ng * nf, -1);
    Gg.nbr.assign((size_t)ng * R.nface, -1);
    for (int64_t el = 0; el < ng; ++el) {
      const int64_t e = gstart[g] + el;
      const double* X = xyz + (size_t)e * max_vert * nd;
      double x[3], J[9], S[9];
      for (int r = 0; r < ns; ++r) {
        mapping(R, nd, X, &R.sp[r * nd], x, J);
        double dj = adj(nd, J, S);
        if (!(dj > 0.0)) {
          std::snprintf(buf, sizeof buf, "element %lld: non-positive Jacobian determinant", (long long)e);
          err = buf; return false;
        }
        size_t k = (size_t)el * ns + r;
        Gg.rdet[k] = 1.0 / dj;
        for (int i = 0; i < nd * nd; ++i) { Gg.S[k * nd * nd + i] = S[i]; Gg.Jinv[k * nd * nd + i] = S[i] / dj; }
      }
      for (int j = 0; j < nf; ++j) {
        mapping(R, nd, X, &R.fp[j * nd], x, J);
        adj(nd, J, S);
        double N[3] = {0, 0, 0}, mg = 0.0;
        for (int i = 0; i < nd; ++i) {
          for (int d = 0; d < nd; ++d) N[i] += S[d * nd + i] * R.nref[j * nd + d];
          mg += N[i] * N[i];
        }
        mg = std::sqrt(mg);
        size_t k = (size_t)el * nf + j;
        Gg.magN[k] = mg;
        for (int i = 0; i < nd; ++i) { Gg.nrm[k * nd + i] = N[i] / mg; fx[(size_t)gfp(e, j) * nd + i] = x[i]; }
      }
      for (int f = 0; f < R.nface; ++f) {
        int64_t m = nbr[e * max_face + f];
        if (m < 0 || m >= ne) {
          std::snprintf(buf, sizeof buf, "element %lld face %d: neighbour out of range", (long long)e, f);
          err = buf; return false;
        }
        // group-local index when the neighbour shares the group, else the
        // element itself (the kernels that read it run on single-type meshes)
        Gg.nbr[el * R.nface + f] = grp[m] == g ? (int)(m - gstart[g]) : (int)el;
      }
    }
  }
  // flux-point pairing across faces by position relative to the face centroid
  std::vector<int64_t> pair((size_t)fbase[ngrp], -1);
  for (int64_t e = 0; e < ne; ++e) {
    const RefOps& R = ref_of(e);
    for (int f = 0; f < R.nface; ++f) {
      int64_t m = nbr[e * max_face + f];
      const RefOps& Rm = ref_of(m);
      int f2 = nbr_face[e * max_face + f];
      if (f2 < 0 || f2 >= Rm.nface) { err = "neighbour face index out of range"; return false; }
      const int na = R.face_off[f + 1] - R.face_off[f], nb = Rm.face_off[f2 + 1] - Rm.face_off[f2];
      if (na != nb) { err = "faces of different point counts meet"; return false; }
      double c1[3] = {0, 0, 0}, c2[3] = {0, 0, 0}, sz = 0.0;
      const std::vector<int>& v1 = R.face_verts[f];
      const std::vector<int>& v2 = Rm.face_verts[f2];
      for (int v : v1)
        for (int i = 0; i < nd; ++i) c1[i] += xyz[((size_t)e * max_vert + v) * nd + i] / v1.size();
      for (int v : v2)
        for (int i = 0; i < nd; ++i) c2[i] += xyz[((size_t)m * max_vert + v) * nd + i] / v2.size();
      for (int i = 0; i < nd; ++i) {
        double d = xyz[((size_t)e * max_vert + v1[0]) * nd + i] - c1[i];
        sz += d * d;
      }
      sz = std::sqrt(sz);
      for (int a = 0; a < na; ++a) {
        const int64_t ga = gfp(e, R.face_off[f] + a);
        int64_t best = -1; double bd = 1e300;
        for (int b = 0; b < nb; ++b) {
          const int64_t gb = gfp(m, Rm.face_off[f2] + b);
          double d2 = 0.0;
          for (int i = 0; i < nd; ++i) {
            double t = (fx[(size_t)ga * nd + i] - c1[i]) - (fx[(size_t)gb * nd + i] - c2[i]);
            d2 += t * t;
          }
          if (d2 < bd) { bd = d2; best = gb; }
        }
        if (std::sqrt(bd) > 1e-8 * sz) {
          std::snprintf(buf, sizeof buf, "element %lld face %d: neighbour face points do not coincide", (long long)e, f);
          err = buf; return false;
        }
        pair[(size_t)ga] = best;
      }
    }
  }
  // the pairing must be an involution
  for (int64_t i = 0; i < fbase[ngrp]; ++i)
    if (pair[(size_t)i] < 0 || pair[(size_t)pair[(size_t)i]] != i) { err = "face-point pairing is not symmetric"; return false; }
  // per group: partner indices relative to the group's first flux point
  // (negative or past the group for partners in other groups)
  for (int g = 0; g < ngrp; ++g) {
    const RefOps& R = *refs[etype[gstart[g]]];
    const int64_t ng = gstart[g + 1] - gstart[g];
    for (int64_t i = 0; i < ng * R.nf; ++i) G[g].nbfp[(size_t)i] = (int)(pair[(size_t)(fbase[g] + i)] - fbase[g]);
  }
  // per face: the neighbour's local face index and, for each point of that
  // neighbour face, the partner point in this element (single groups: used by
  // the viscous Jacobian paths)
  for (int g = 0; g < ngrp; ++g) {
    const RefOps& R = *refs[etype[gstart[g]]];
    const int64_t ng = gstart[g + 1] - gstart[g];
    const int nf = R.nf;
    G[g].nbface.assign((size_t)ng * R.nface, 0);
    G[g].back.assign((size_t)ng * R.nface * R.nfp, 0);
    if (ngrp == 1 && R.nf == R.nface * R.nfp)
      for (int64_t e = 0; e < ng; ++e)
        for (int f = 0; f < R.nface; ++f) {
          int pg = G[g].nbfp[(size_t)e * nf + f * R.nfp];
          int64_t m = pg / nf;
          int f2 = R.fface[pg - m * nf];
          G[g].nbface[e * R.nface + f] = f2;
          for (int j = 0; j < R.nfp; ++j)
            G[g].back[((size_t)e * R.nface + f) * R.nfp + j] = (int)(G[g].nbfp[(size_t)m * nf + f2 * R.nfp + j] - e * nf);
        }
  }
  if (mix) {
    for (int g = 0; g < ngrp; ++g) {
      const int gt = etype[gstart[g]];
      const RefOps& R = *refs[gt];
      const int64_t ng = gstart[g + 1] - gstart[g];
      MixInfo& M = mix[g];
      M.nbpt.assign((size_t)ng * R.nf, 0);
      M.nbt.assign((size_t)ng * R.nface, 0);
      M.nbg.assign((size_t)ng * R.nface, 0);
      for (int64_t el = 0; el < ng; ++el) {
        const int64_t e = gstart[g] + el;
        for (int f = 0; f < R.nface; ++f) {
          const int64_t m = nbr[e * max_face + f];
          M.nbg[el * R.nface + f] = m;
          M.nbt[el * R.nface + f] = etype[m] != gt ? 1 : 0;
          for (int a = 0; a < R.face_off[f + 1] - R.face_off[f]; ++a) {
            const int j = R.face_off[f] + a;
            const int64_t pg = pair[(size_t)gfp(e, j)];
            M.nbpt[(size_t)el * R.nf + j] = (int)(pg - gfp(m, 0));
          }
        }
      }
    }
  }
  return true;
}

bool build_geometry(const RefOps& R, int nd, int64_t ne, const double* xyz, int max_vert, const int64_t* nbr,
                    const int8_t* nbr_face, int max_face, Geometry& G, std::string& err) {
  const RefOps* refs[5] = {&R, &R, &R, &R, &R};
  std::vector<int8_t> et((size_t)ne, (int8_t)R.type);
  const int64_t gs[2] = {0, ne};
  return build_geometry_groups(refs, nd, ne, et.data(), xyz, max_vert, nbr, nbr_face, max_face, 1, gs, &G, nullptr,
                               err);
}

bool check_stencil(int64_t ne, int nface, const int* nbr, std::string& err) {
  char buf[256];
  for (int64_t n = 0; n < ne; ++n) {
    std::vector<int> first = {(int)n};
    for (int f = 0; f < nface; ++f) first.push_back(nbr[n * nface + f]);
    for (size_t i = 0; i < first.size(); ++i)
      for (size_t j = i + 1; j < first.size(); ++j)
        if (first[i] == first[j]) {
          std::snprintf(buf, sizeof buf, "element %lld: face neighbours are not distinct", (long long)n);
          err = buf; return false;
        }
    for (int f = 0; f < nface; ++f) {
      int m = nbr[n * nface + f];
      int back = 0;
      for (int f2 = 0; f2 < nface; ++f2) {
        int k = nbr[(int64_t)m * nface + f2];
        if (k == (int)n) { ++back; continue; }
        for (int x : first)
          if (k == x) {
            std::snprintf(buf, sizeof buf, "element %lld: second face layer folds onto the first", (long long)n);
            err = buf; return false;
          }
      }
      if (back != 1) { err = "neighbour relation is not symmetric"; return false; }
    }
  }
  return true;
}

}  // namespace frh
