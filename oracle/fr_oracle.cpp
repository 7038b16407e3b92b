// FP64 CPU oracle for the FR-DG residual R(U), its Jacobian dR/dU and
// Jacobian-vector products.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
// call this file; only the tests, the smoke check and the CPU-baseline leg of
// the benchmark do.  It shares no source with the HIP library.
//
// The code is deliberately plain: one element at a time, dense loops, no
// blocking or fusion, every step in the order the paper states it.
//
//   * Reference data: Gauss-Legendre solution and flux points (appendix A),
//     Lagrange nodal basis, FR-DG correction functions taken as the Radau
//     polynomials g_R = (P_{p+1} + P_p)/2 and g_L(x) = g_R(-x) (the DG
//     recovering choice the FR section refers to).
//   * Geometry: analytic bilinear / trilinear / affine maps, J, detJ,
//     S = detJ J^{-1}, transformed quantities (section 2, eq.
//     "transformed_quantities"); at flux points N = S^T n_ref,
//     common transformed normal flux = |N| * common flux (SDRT section).
//   * Common solution (eq. "common_var_for_grad") with beta, corrected
//     gradient q~ = grad~ u + sum_f (C_f - u_f) n_f div g_f (FR gradient,
//     remark after eq. "divergence_equivalence"), physical q = J^{-T} q~.
//   * Fluxes: linear advection (eq. "linear_advection") with the upwind
//     flux (eq. "flux_advection"); Euler (eq. "fluxOperatorEuler") and
//     Navier-Stokes (eq. "fluxOperatorNavierStokes") with the Rusanov
//     convective flux and the LDG viscous common flux of the SDRT section.
//   * Divergence: eq. "divergence_fr"; method of lines dU/dt = -J^{-1} div.
//
// Derivatives are computed by complex-step differentiation of the very same
// residual code instantiated with std::complex<double>: for a real-analytic
// map, Im R(U + i h e_j)/h equals dR/dU_j up to O(h^2) with no cancellation,
// so with h = 1e-30 the Jacobian column is exact to rounding.  The only
// non-analytic operations (|.|, max, sign) branch on the real part, which is
// the derivative of the active branch (ties go to the left state).
//
// Schemes (tensor elements): FR-DG (the Radau corrections above), FR-SDRT
// (FR whose correction functions are the Raviart-Thomas flux basis functions
// of the external flux points: along the normal line, the Lagrange
// polynomial of degree p+1 on the SD flux points {-1, zeros of P_p, +1} that
// is 1 at the face; section "Connections between the SDRT and FR formalisms")
// and SDRT itself (section "SDRT method"): u and the gradient interpolated to
// the internal flux points, the transformed normal flux evaluated there, the
// common flux at the external ones, and the divergence of the flux nodal
// basis at the solution points (eq. "divergence_sdrt"); the gradient from
// the internal values and the common solution with the same basis.
//
// Triangles: the solution point set is supplied by the caller (the paper's
// Williams-Shunn tables are not reproduced in the text); the nodal basis is
// built from the orthonormal Dubiner (PKD) modal basis through the
// Vandermonde matrix, edge flux points are Gauss-Legendre, and the FR-DG
// correction is the nodal-DG lifting M^{-1} E.
//
// Tetrahedra and prisms (FR-DG only): the solution points of tetrahedra are
// supplied by the caller (the paper's Shunn-Ham tables are not reproduced
// either); prisms take the triangle points times Gauss-Legendre points along
// the prism axis.  Triangular faces carry the caller's triangle point set,
// quadrilateral faces Gauss-Legendre points.  The nodal basis comes from the
// collapsed-coordinate PKD basis (tetrahedra) or the triangle PKD basis times
// Legendre polynomials (prisms) through the Vandermonde matrix; the mass
// matrix and the face integrals E_jf = int_face l_j phi_f dS (phi_f the
// face's nodal basis on its flux points) use collapsed Gauss-Legendre rules
// exact for the integrands, and the correction is again M^{-1} E.

#include <array>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

typedef std::complex<double> cd;

static inline double re(double x) { return x; }
static inline double re(const cd& z) { return z.real(); }
template <class T> static inline T tabs(const T& x) { return re(x) >= 0 ? x : -x; }
template <class T> static inline T tmax(const T& a, const T& b) { return re(a) >= re(b) ? a : b; }

enum { QUAD = 0, TRI = 1, HEX = 2, TET = 3, PRI = 4 };
enum { ADVECTION = 0, EULER = 1, NAVIER_STOKES = 2 };

// ---------------------------------------------------------------- 1-D data
// Legendre polynomial P_n and its derivative by the three-term recurrence.
static void legendre(int n, double x, double* P, double* dP) {
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  if (n == 0) { *P = 1.0; *dP = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    double d2 = d0 + (2.0 * k - 1.0) * p1;
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  *P = p1; *dP = d1;
}

// Gauss-Legendre nodes (ascending) and weights, Newton on P_n.
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0); w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = -std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double P, dP; legendre(n, z, &P, &dP);
      double dz = P / dP; z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double P, dP; legendre(n, z, &P, &dP);
    x[i] = z; w[i] = 2.0 / ((1.0 - z * z) * dP * dP);
  }
}

// Lagrange basis l_j on nodes x, evaluated at t.
static double lagrange(const std::vector<double>& x, int j, double t) {
  double v = 1.0;
  for (size_t k = 0; k < x.size(); ++k)
    if ((int)k != j) v *= (t - x[k]) / (x[j] - x[k]);
  return v;
}
static double lagrange_d(const std::vector<double>& x, int j, double t) {
  double s = 0.0;
  for (size_t m = 0; m < x.size(); ++m) {
    if ((int)m == j) continue;
    double v = 1.0 / (x[j] - x[m]);
    for (size_t k = 0; k < x.size(); ++k)
      if ((int)k != j && k != m) v *= (t - x[k]) / (x[j] - x[k]);
    s += v;
  }
  return s;
}
// Derivative of the right Radau correction g_R = (P_{p+1} + P_p)/2.
static double radau_right_d(int p, double t) {
  double P, dP1, dP0; legendre(p + 1, t, &P, &dP1); legendre(p, t, &P, &dP0);
  return 0.5 * (dP1 + dP0);
}

// SD flux points on a line: -1, the p zeros of P_p, +1 (ascending).
static std::vector<double> sd_points(int p) {
  std::vector<double> z, w;
  gauss_legendre(p, z, w);
  std::vector<double> out;
  out.push_back(-1.0);
  for (double v : z) out.push_back(v);
  out.push_back(1.0);
  return out;
}
// Derivative of the right SD correction: the Lagrange polynomial on the SD
// flux points that is 1 at +1.
static double sd_right_d(int p, double t) {
  std::vector<double> z = sd_points(p);
  return lagrange_d(z, p + 1, t);
}

// ------------------------------------------------------ triangle basis (PKD)
// Orthonormal Dubiner (PKD) basis on the reference triangle (v0=(-1,-1),
// v1=(1,-1), v2=(-1,1)): psi_ij = c_ij ((1-s)/2)^i P_i(a) P_j^{(2i+1,0)}(s)
// with the collapsed coordinate a = 2(1+r)/(1-s) - 1.  The factor
// t^i P_i(a), t = (1-s)/2, is evaluated by the scaled Legendre recurrence
// Q_k = ((2k-1) x Q_{k-1} - (k-1) t^2 Q_{k-2}) / k with x = a t, which has
// no singularity at the top vertex.  c_ij = sqrt((2i+1)(i+j+1)/2) makes the
// basis orthonormal on the triangle of area 2.
template <class T>
static T dubiner(int i, int j, const T& r, const T& s) {
  T t = (T(1.0) - s) * T(0.5);
  T x = (T(1.0) + T(2.0) * r + s) * T(0.5);
  T q0 = T(1.0), q1 = x;
  T qi = (i == 0) ? q0 : q1;
  for (int k = 2; k <= i; ++k) {
    T q2 = (T(2.0 * k - 1.0) * x * q1 - T(k - 1.0) * t * t * q0) / T((double)k);
    q0 = q1; q1 = q2; qi = q2;
  }
  // Jacobi P_j^{(al,0)}(s) by its three-term recurrence
  const double al = 2.0 * i + 1.0;
  T p0 = T(1.0), p1 = T(0.5 * (al + 2.0)) * s + T(0.5 * al);
  T pj = (j == 0) ? p0 : p1;
  for (int k = 2; k <= j; ++k) {
    double a1 = 2.0 * k * (k + al) * (2.0 * k + al - 2.0);
    double a2 = (2.0 * k + al - 1.0) * (al * al);
    double a3 = (2.0 * k + al - 2.0) * (2.0 * k + al - 1.0) * (2.0 * k + al);
    double a4 = 2.0 * (k + al - 1.0) * (k - 1.0) * (2.0 * k + al);
    T p2 = ((T(a2) + T(a3) * s) * p1 - T(a4) * p0) / T(a1);
    p0 = p1; p1 = p2; pj = p2;
  }
  return T(std::sqrt((2.0 * i + 1.0) * (i + j + 1.0) / 2.0)) * qi * pj;
}

// ------------------------------------------------------- reference element
struct RefElem {
  int type = -1, p = 0, nd = 0, ns = 0, nf = 0, nface = 0, nvert = 0;
  std::vector<double> sp;     // [ns][nd] reference solution points
  std::vector<double> fp;     // [nf][nd] reference flux points
  std::vector<int> fface;     // [nf] face of each flux point
  std::vector<int> face_off;  // [nface+1] first flux point of each face
  std::vector<double> nref;   // [nf][nd] unit reference outward normal
  std::vector<double> M0;     // [nf][ns] l_sigma(x_f)
  std::vector<double> Dm;     // [nd][ns][ns] d l_sigma / d xi_d at x_rho
  std::vector<double> Cor;    // [ns][nf] div g_f at x_rho
  std::vector<double> wq;     // [ns] quadrature weights at solution points (mass lumping for conservation checks)
  std::vector<std::vector<int>> face_verts;
  int scheme = 0;             // 0 FR-DG, 1 FR-SDRT, 2 SDRT
  // SDRT internal flux points (tensor elements)
  int nint = 0;
  std::vector<double> ip;     // [nint][nd] reference position
  std::vector<int> idir;      // [nint] axis d of the degree of freedom (normal e_d)
  std::vector<double> Mint;   // [nint][ns] solution basis at the point
  std::vector<double> Dint;   // [ns][nint] divergence of the point's flux basis function at x_rho
};

static void shape_fn(int type, const double* xi, double* N, double* dN /*[nvert][nd]*/) {
  if (type == QUAD) {
    static const double V[4][2] = {{-1, -1}, {1, -1}, {1, 1}, {-1, 1}};
    for (int v = 0; v < 4; ++v) {
      N[v] = (1 + V[v][0] * xi[0]) * (1 + V[v][1] * xi[1]) / 4;
      dN[v * 2 + 0] = V[v][0] * (1 + V[v][1] * xi[1]) / 4;
      dN[v * 2 + 1] = (1 + V[v][0] * xi[0]) * V[v][1] / 4;
    }
  } else if (type == HEX) {
    static const double V[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                                   {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};
    for (int v = 0; v < 8; ++v) {
      double a = 1 + V[v][0] * xi[0], b = 1 + V[v][1] * xi[1], c = 1 + V[v][2] * xi[2];
      N[v] = a * b * c / 8;
      dN[v * 3 + 0] = V[v][0] * b * c / 8;
      dN[v * 3 + 1] = a * V[v][1] * c / 8;
      dN[v * 3 + 2] = a * b * V[v][2] / 8;
    }
  } else if (type == TET) {  // affine, v0=(-1,-1,-1) v1=(1,-1,-1) v2=(-1,1,-1) v3=(-1,-1,1)
    N[0] = -(1 + xi[0] + xi[1] + xi[2]) / 2; N[1] = (1 + xi[0]) / 2; N[2] = (1 + xi[1]) / 2; N[3] = (1 + xi[2]) / 2;
    const double d[4][3] = {{-0.5, -0.5, -0.5}, {0.5, 0, 0}, {0, 0.5, 0}, {0, 0, 0.5}};
    for (int v = 0; v < 4; ++v)
      for (int k = 0; k < 3; ++k) dN[v * 3 + k] = d[v][k];
  } else if (type == PRI) {  // triangle (r, s) x [-1, 1] (t); v0..v2 at t = -1, v3..v5 at t = +1
    const double L[3] = {-(xi[0] + xi[1]) / 2, (1 + xi[0]) / 2, (1 + xi[1]) / 2};
    const double dL[3][2] = {{-0.5, -0.5}, {0.5, 0.0}, {0.0, 0.5}};
    for (int h = 0; h < 2; ++h) {
      const double z = h == 0 ? (1 - xi[2]) / 2 : (1 + xi[2]) / 2, dz = h == 0 ? -0.5 : 0.5;
      for (int a = 0; a < 3; ++a) {
        const int v = 3 * h + a;
        N[v] = L[a] * z;
        dN[v * 3 + 0] = dL[a][0] * z;
        dN[v * 3 + 1] = dL[a][1] * z;
        dN[v * 3 + 2] = L[a] * dz;
      }
    }
  } else {  // TRI affine
    N[0] = -(xi[0] + xi[1]) / 2; N[1] = (1 + xi[0]) / 2; N[2] = (1 + xi[1]) / 2;
    dN[0] = -0.5; dN[1] = -0.5; dN[2] = 0.5; dN[3] = 0.0; dN[4] = 0.0; dN[5] = 0.5;
  }
}

// Dense Gauss-Jordan inverse (row-major, small matrices only).
static bool invert(std::vector<double> A, int n, std::vector<double>& inv) {
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
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = A[r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) { A[r * n + k] -= f * A[c * n + k]; inv[r * n + k] -= f * inv[c * n + k]; }
    }
  }
  return true;
}

static void build_tensor(RefElem& R, int type, int p, int scheme) {
  R.type = type; R.p = p; R.scheme = scheme;
  R.nd = (type == QUAD) ? 2 : 3;
  const int n1 = p + 1, nd = R.nd;
  std::vector<double> x, w; gauss_legendre(n1, x, w);
  R.ns = (nd == 2) ? n1 * n1 : n1 * n1 * n1;
  R.nface = 2 * nd; R.nvert = (nd == 2) ? 4 : 8;
  R.sp.assign(R.ns * nd, 0.0); R.wq.assign(R.ns, 0.0);
  for (int r = 0; r < R.ns; ++r) {
    int idx[3] = {r % n1, (r / n1) % n1, r / (n1 * n1)};
    double wr = 1.0;
    for (int d = 0; d < nd; ++d) { R.sp[r * nd + d] = x[idx[d]]; wr *= w[idx[d]]; }
    R.wq[r] = wr;
  }
  // faces: (axis, sign) in the local face order of the mesh convention
  std::vector<std::pair<int, int>> faces;
  if (nd == 2) {
    faces = {{1, -1}, {0, +1}, {1, +1}, {0, -1}};
    R.face_verts = {{0, 1}, {1, 2}, {2, 3}, {3, 0}};
  } else {
    faces = {{2, -1}, {1, -1}, {0, +1}, {1, +1}, {0, -1}, {2, +1}};
    R.face_verts = {{0, 1, 2, 3}, {0, 1, 5, 4}, {1, 2, 6, 5}, {2, 3, 7, 6}, {3, 0, 4, 7}, {4, 5, 6, 7}};
  }
  int npf = (nd == 2) ? n1 : n1 * n1;
  R.nf = R.nface * npf;
  R.fp.assign(R.nf * nd, 0.0); R.nref.assign(R.nf * nd, 0.0); R.fface.assign(R.nf, 0);
  R.face_off.assign(R.nface + 1, 0);
  for (int f = 0; f < R.nface; ++f) {
    R.face_off[f] = f * npf;
    int ax = faces[f].first, sg = faces[f].second;
    for (int t = 0; t < npf; ++t) {
      int g = f * npf + t;
      R.fface[g] = f;
      int tan[2] = {t % n1, t / n1};
      int k = 0;
      for (int d = 0; d < nd; ++d) {
        if (d == ax) R.fp[g * nd + d] = sg;
        else R.fp[g * nd + d] = x[tan[k++]];
      }
      R.nref[g * nd + ax] = sg;
    }
  }
  R.face_off[R.nface] = R.nf;
  // M0: tensor Lagrange basis at flux points
  R.M0.assign(R.nf * R.ns, 0.0);
  for (int g = 0; g < R.nf; ++g)
    for (int s = 0; s < R.ns; ++s) {
      int idx[3] = {s % n1, (s / n1) % n1, s / (n1 * n1)};
      double v = 1.0;
      for (int d = 0; d < nd; ++d) v *= lagrange(x, idx[d], R.fp[g * nd + d]);
      R.M0[g * R.ns + s] = v;
    }
  // D_d: derivative of the tensor basis at solution points
  R.Dm.assign(nd * R.ns * R.ns, 0.0);
  for (int d = 0; d < nd; ++d)
    for (int r = 0; r < R.ns; ++r)
      for (int s = 0; s < R.ns; ++s) {
        int is[3] = {s % n1, (s / n1) % n1, s / (n1 * n1)};
        double v = 1.0;
        for (int e = 0; e < nd; ++e) {
          double t = R.sp[r * nd + e];
          v *= (e == d) ? lagrange_d(x, is[e], t) : lagrange(x, is[e], t);
        }
        R.Dm[(d * R.ns + r) * R.ns + s] = v;
      }
  // Correction: div g_f at solution points.  g_f = s * g_1D(xi_ax) * prod of
  // tangential Lagrange functions of the flux point's line, g_1D = g_R on the
  // +1 face and g_L(x) = g_R(-x) on the -1 face; the outward sign s makes
  // g_f . n_f = 1 at the flux point.
  R.Cor.assign(R.ns * R.nf, 0.0);
  for (int g = 0; g < R.nf; ++g) {
    int f = R.fface[g], ax = faces[f].first, sg = faces[f].second;
    for (int r = 0; r < R.ns; ++r) {
      double t = R.sp[r * nd + ax];
      // s * d/dt g_L(t) = (-1)(-g_R'(-t)) for g_L(t) = g_R(-t)
      double dg = (scheme == 0) ? ((sg > 0) ? radau_right_d(p, t) : radau_right_d(p, -t))
                                : ((sg > 0) ? sd_right_d(p, t) : sd_right_d(p, -t));
      double tv = 1.0;
      int ir[3] = {r % n1, (r / n1) % n1, r / (n1 * n1)};
      for (int d = 0; d < nd; ++d)
        if (d != ax) tv *= lagrange(x, ir[d], R.fp[g * nd + d]);
      R.Cor[r * R.nf + g] = dg * tv;
    }
  }
  if (scheme != 2) return;
  // SDRT internal flux points: on each line along axis d, the p interior SD
  // points z_1..z_p of that axis at the solution-point positions of the
  // other axes; degree of freedom e_d, flux basis function
  // e_d psi_j(xi_d) prod_{e != d} l_{i_e}(xi_e) with psi_j the Lagrange
  // polynomial on the SD points.
  std::vector<double> z = sd_points(p);
  const int nl = R.ns / n1;                        // lines per axis
  R.nint = nd * nl * p;
  R.ip.assign(R.nint * nd, 0.0); R.idir.assign(R.nint, 0);
  R.Mint.assign(R.nint * R.ns, 0.0); R.Dint.assign(R.ns * R.nint, 0.0);
  int k = 0;
  for (int d = 0; d < nd; ++d)
    for (int l = 0; l < nl; ++l)
      for (int j = 1; j <= p; ++j, ++k) {
        // tangential solution-point indices of line l (the other axes in order)
        int tan[3] = {0, 0, 0}, rem = l;
        for (int e = 0; e < nd; ++e)
          if (e != d) { tan[e] = rem % n1; rem /= n1; }
        R.idir[k] = d;
        for (int e = 0; e < nd; ++e) R.ip[k * nd + e] = (e == d) ? z[j] : x[tan[e]];
        for (int s2 = 0; s2 < R.ns; ++s2) {
          int is[3] = {s2 % n1, (s2 / n1) % n1, s2 / (n1 * n1)};
          double v = 1.0;
          for (int e = 0; e < nd; ++e) v *= lagrange(x, is[e], R.ip[k * nd + e]);
          R.Mint[k * R.ns + s2] = v;
        }
        for (int r = 0; r < R.ns; ++r) {
          double v = lagrange_d(z, j, R.sp[r * nd + d]);
          for (int e = 0; e < nd; ++e)
            if (e != d) v *= lagrange(x, tan[e], R.sp[r * nd + e]);
          R.Dint[r * R.nint + k] = v;
        }
      }
}

static void build_tri(RefElem& R, int p, const double* pts /*[ns][2]*/) {
  R.type = TRI; R.p = p; R.nd = 2; R.nface = 3; R.nvert = 3;
  const int ns = (p + 1) * (p + 2) / 2, n1 = p + 1;
  R.ns = ns;
  R.sp.assign(pts, pts + 2 * ns);
  R.face_verts = {{0, 1}, {1, 2}, {2, 0}};
  // Vandermonde V[r][m] = psi_m(x_r)
  std::vector<std::pair<int, int>> modes;
  for (int i = 0; i <= p; ++i)
    for (int j = 0; i + j <= p; ++j) modes.push_back({i, j});
  std::vector<double> V(ns * ns), Vinv;
  for (int r = 0; r < ns; ++r)
    for (int m = 0; m < ns; ++m)
      V[r * ns + m] = dubiner<double>(modes[m].first, modes[m].second, pts[2 * r], pts[2 * r + 1]);
  invert(V, ns, Vinv);
  // nodal basis l_s(x) = sum_m Vinv[m][s] psi_m(x)
  auto lval = [&](int s, double r, double t) {
    double v = 0.0;
    for (int m = 0; m < ns; ++m) v += Vinv[m * ns + s] * dubiner<double>(modes[m].first, modes[m].second, r, t);
    return v;
  };
  // derivative via complex step on the modal basis
  auto lgrad = [&](int s, double r, double t, int d) {
    const double hh = 1e-30;
    double v = 0.0;
    for (int m = 0; m < ns; ++m) {
      cd rr = (d == 0) ? cd(r, hh) : cd(r, 0.0), tt = (d == 1) ? cd(t, hh) : cd(t, 0.0);
      v += Vinv[m * ns + s] * dubiner<cd>(modes[m].first, modes[m].second, rr, tt).imag() / hh;
    }
    return v;
  };
  std::vector<double> x, w; gauss_legendre(n1, x, w);
  // edge flux points: GL on each edge, ordered along the edge direction
  const double E[3][2][2] = {{{-1, -1}, {1, -1}}, {{1, -1}, {-1, 1}}, {{-1, 1}, {-1, -1}}};
  const double nr[3][2] = {{0, -1}, {M_SQRT1_2, M_SQRT1_2}, {-1, 0}};
  const double elen[3] = {2.0, 2.0 * M_SQRT2, 2.0};
  R.nf = 3 * n1;
  R.fp.assign(R.nf * 2, 0.0); R.nref.assign(R.nf * 2, 0.0); R.fface.assign(R.nf, 0);
  R.face_off = {0, n1, 2 * n1, 3 * n1};
  std::vector<double> fw(R.nf);
  for (int f = 0; f < 3; ++f)
    for (int t = 0; t < n1; ++t) {
      int g = f * n1 + t;
      double s = 0.5 * (x[t] + 1.0);
      R.fp[g * 2 + 0] = E[f][0][0] + s * (E[f][1][0] - E[f][0][0]);
      R.fp[g * 2 + 1] = E[f][0][1] + s * (E[f][1][1] - E[f][0][1]);
      R.nref[g * 2 + 0] = nr[f][0]; R.nref[g * 2 + 1] = nr[f][1];
      R.fface[g] = f;
      fw[g] = w[t] * elen[f] / 2.0;  // GL weight scaled to reference arc length
    }
  R.M0.assign(R.nf * ns, 0.0);
  for (int g = 0; g < R.nf; ++g)
    for (int s = 0; s < ns; ++s) R.M0[g * ns + s] = lval(s, R.fp[g * 2], R.fp[g * 2 + 1]);
  R.Dm.assign(2 * ns * ns, 0.0);
  for (int d = 0; d < 2; ++d)
    for (int r = 0; r < ns; ++r)
      for (int s = 0; s < ns; ++s) R.Dm[(d * ns + r) * ns + s] = lgrad(s, pts[2 * r], pts[2 * r + 1], d);
  // Mass matrix M = (V V^T)^{-1} for an orthonormal modal basis.
  std::vector<double> VVt(ns * ns, 0.0), Mmass, Minv;
  for (int a = 0; a < ns; ++a)
    for (int b = 0; b < ns; ++b)
      for (int m = 0; m < ns; ++m) VVt[a * ns + b] += Vinv[m * ns + a] * Vinv[m * ns + b];
  // VVt here is Vinv^T Vinv = (V V^T)^{-1} = M
  Mmass = VVt;
  invert(Mmass, ns, Minv);
  // lifting: div g_f(x_r) = sum_j Minv[r][j] E[j][f], E[j][f] = int_edge l_j phi_f ds
  // with phi_f the edge GL Lagrange function, exact by the edge GL rule.
  R.Cor.assign(ns * R.nf, 0.0);
  for (int r = 0; r < ns; ++r)
    for (int g = 0; g < R.nf; ++g) {
      double v = 0.0;
      for (int j = 0; j < ns; ++j) v += Minv[r * ns + j] * R.M0[g * ns + j] * fw[g];
      R.Cor[r * R.nf + g] = v;
    }
  R.wq.assign(ns, 0.0);
  for (int r = 0; r < ns; ++r)
    for (int j = 0; j < ns; ++j) R.wq[r] += Mmass[r * ns + j];
}

// ---------------------------------------------- tetrahedra and prisms (FR-DG)
// PKD basis on the reference tetrahedron (v0=(-1,-1,-1), v1=(1,-1,-1),
// v2=(-1,1,-1), v3=(-1,-1,1)), collapsed coordinates a = 2(1+r)/(-s-t) - 1,
// b = 2(1+s)/(1-t) - 1, c = t:
//   psi_ijk = P_i(a) ((1-b)/2)^i P_j^{(2i+1,0)}(b) ((1-c)/2)^{i+j} P_k^{(2i+2j+2,0)}(c),
// written as a polynomial: tau^i P_i(x / tau) with tau = (-s-t)/2, x = 1 + r +
// (s+t)/2, and sigma^j P_j^{(2i+1,0)}(y / sigma) with sigma = (1-t)/2, y =
// (1+2s+t)/2, each by its scaled recurrence (no singular points).  Not
// normalised: the mass matrix is integrated.
template <class T> static T scaled_jacobi(int n, double al, const T& y, const T& sg) {
  T p0 = T(1.0);
  if (n == 0) return p0;
  T p1 = T(0.5 * (al + 2.0)) * y + T(0.5 * al) * sg;
  for (int k = 2; k <= n; ++k) {
    double a1 = 2.0 * k * (k + al) * (2.0 * k + al - 2.0);
    double a2 = (2.0 * k + al - 1.0) * (al * al);
    double a3 = (2.0 * k + al - 2.0) * (2.0 * k + al - 1.0) * (2.0 * k + al);
    double a4 = 2.0 * (k + al - 1.0) * (k - 1.0) * (2.0 * k + al);
    T p2 = ((T(a2) * sg + T(a3) * y) * p1 - T(a4) * sg * sg * p0) / T(a1);
    p0 = p1; p1 = p2;
  }
  return p1;
}
template <class T> static T pkd_tet(int i, int j, int k, const T& r, const T& s, const T& t) {
  const T tau = (-s - t) * T(0.5), x = T(1.0) + r + (s + t) * T(0.5);
  T q0 = T(1.0), q1 = x, qi = (i == 0) ? q0 : q1;
  for (int m = 2; m <= i; ++m) {
    T q2 = (T(2.0 * m - 1.0) * x * q1 - T(m - 1.0) * tau * tau * q0) / T((double)m);
    q0 = q1; q1 = q2; qi = q2;
  }
  const T sg = (T(1.0) - t) * T(0.5), y = (T(1.0) + T(2.0) * s + t) * T(0.5);
  const T pj = scaled_jacobi(j, 2.0 * i + 1.0, y, sg);
  const T pk = scaled_jacobi(k, 2.0 * i + 2.0 * j + 2.0, t, T(1.0));
  return qi * pj * pk;
}
// Legendre P_n(t) (complex-capable).
template <class T> static T leg(int n, const T& t) {
  T p0 = T(1.0), p1 = t;
  if (n == 0) return p0;
  for (int k = 2; k <= n; ++k) {
    T p2 = (T(2.0 * k - 1.0) * t * p1 - T(k - 1.0) * p0) / T((double)k);
    p0 = p1; p1 = p2;
  }
  return p1;
}

// Collapsed Gauss-Legendre rule on the reference triangle (area 2), exact for
// degree 2n - 2: (a, b) in [-1,1]^2, r = (1+a)(1-b)/2 - 1, s = b, dA =
// (1-b)/2 da db.
static void tri_rule(int n, std::vector<double>& q, std::vector<double>& w) {
  std::vector<double> x, wx; gauss_legendre(n, x, wx);
  q.clear(); w.clear();
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      q.push_back((1 + x[i]) * (1 - x[j]) / 2 - 1);
      q.push_back(x[j]);
      w.push_back(wx[i] * wx[j] * (1 - x[j]) / 2);
    }
}
// Collapsed rule on the reference tetrahedron (volume 4/3): t = c, s = (1+b)(1-c)/2 - 1,
// r = (1+a)(1-b)(1-c)/4 - 1, dV = (1-b)(1-c)^2/8 da db dc.
static void tet_rule(int n, std::vector<double>& q, std::vector<double>& w) {
  std::vector<double> x, wx; gauss_legendre(n, x, wx);
  q.clear(); w.clear();
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int k = 0; k < n; ++k) {
        const double a = x[i], b = x[j], c = x[k];
        q.push_back((1 + a) * (1 - b) * (1 - c) / 4 - 1);
        q.push_back((1 + b) * (1 - c) / 2 - 1);
        q.push_back(c);
        w.push_back(wx[i] * wx[j] * wx[k] * (1 - b) * (1 - c) * (1 - c) / 8);
      }
}

// One face of a 3-D reference element: its flux points, unit outward
// normal, and a quadrature rule with the face's nodal basis at its points.
struct FaceData {
  std::vector<double> fp;      // [nfp][3]
  double n[3];
  std::vector<double> qx, qw;  // quadrature points [nq][3], weights (reference surface measure)
  std::vector<double> phi;     // [nq][nfp] face nodal basis at the quadrature points
};

// Triangular face with vertices A, B, C: the caller's triangle points mapped
// through the barycentric coordinates of the 2-D reference triangle.
static FaceData tri_face(const double* A, const double* B, const double* C, const double* n, int p,
                         const double* tri_pts) {
  FaceData F;
  const int nt = (p + 1) * (p + 2) / 2;
  auto map = [&](double a, double b, double* X) {
    const double l0 = -(a + b) / 2, l1 = (1 + a) / 2, l2 = (1 + b) / 2;
    for (int k = 0; k < 3; ++k) X[k] = l0 * A[k] + l1 * B[k] + l2 * C[k];
  };
  for (int i = 0; i < nt; ++i) {
    double X[3]; map(tri_pts[2 * i], tri_pts[2 * i + 1], X);
    F.fp.insert(F.fp.end(), X, X + 3);
  }
  for (int k = 0; k < 3; ++k) F.n[k] = n[k];
  // area of the face / area of the 2-D reference triangle
  double e1[3], e2[3], cr[3];
  for (int k = 0; k < 3; ++k) { e1[k] = B[k] - A[k]; e2[k] = C[k] - A[k]; }
  cr[0] = e1[1] * e2[2] - e1[2] * e2[1]; cr[1] = e1[2] * e2[0] - e1[0] * e2[2]; cr[2] = e1[0] * e2[1] - e1[1] * e2[0];
  const double scale = 0.5 * std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]) / 2.0;
  // face nodal basis: 2-D PKD Vandermonde on the triangle points
  std::vector<std::pair<int, int>> modes;
  for (int i = 0; i <= p; ++i)
    for (int j = 0; i + j <= p; ++j) modes.push_back({i, j});
  std::vector<double> V(nt * nt), Vinv;
  for (int r = 0; r < nt; ++r)
    for (int m = 0; m < nt; ++m) V[r * nt + m] = dubiner<double>(modes[m].first, modes[m].second, tri_pts[2 * r], tri_pts[2 * r + 1]);
  invert(V, nt, Vinv);
  std::vector<double> q, w; tri_rule(p + 2, q, w);
  const int nq = (int)w.size();
  F.phi.assign(nq * nt, 0.0);
  for (int a = 0; a < nq; ++a) {
    double X[3]; map(q[2 * a], q[2 * a + 1], X);
    F.qx.insert(F.qx.end(), X, X + 3);
    F.qw.push_back(w[a] * scale);
    for (int g = 0; g < nt; ++g) {
      double v = 0.0;
      for (int m = 0; m < nt; ++m) v += Vinv[m * nt + g] * dubiner<double>(modes[m].first, modes[m].second, q[2 * a], q[2 * a + 1]);
      F.phi[a * nt + g] = v;
    }
  }
  return F;
}
// Quadrilateral face with vertices A, B, C, D (a planar parallelogram):
// Gauss-Legendre points, point (i, j) at A + (1+x_i)/2 (B - A) + (1+x_j)/2 (D - A);
// the rule is the same points (exact for the products of two face
// polynomials of degree p in each direction).
static FaceData quad_face(const double* A, const double* B, const double* D, const double* n, int p) {
  FaceData F;
  const int n1 = p + 1;
  std::vector<double> x, w; gauss_legendre(n1, x, w);
  double e1[3], e2[3], cr[3];
  for (int k = 0; k < 3; ++k) { e1[k] = B[k] - A[k]; e2[k] = D[k] - A[k]; }
  cr[0] = e1[1] * e2[2] - e1[2] * e2[1]; cr[1] = e1[2] * e2[0] - e1[0] * e2[2]; cr[2] = e1[0] * e2[1] - e1[1] * e2[0];
  const double scale = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]) / 4.0;
  for (int j = 0; j < n1; ++j)
    for (int i = 0; i < n1; ++i) {
      double X[3];
      for (int k = 0; k < 3; ++k) X[k] = A[k] + 0.5 * (1 + x[i]) * e1[k] + 0.5 * (1 + x[j]) * e2[k];
      F.fp.insert(F.fp.end(), X, X + 3);
      F.qx.insert(F.qx.end(), X, X + 3);
      F.qw.push_back(w[i] * w[j] * scale);
    }
  const int nf = n1 * n1;
  F.phi.assign(nf * nf, 0.0);
  for (int a = 0; a < nf; ++a) F.phi[a * nf + a] = 1.0;
  for (int k = 0; k < 3; ++k) F.n[k] = n[k];
  return F;
}

// Operators of a 3-D element from its modal basis (value through T = double,
// derivatives by complex step), solution points, volume rule and faces.
template <class Basis>
static void build_3d(RefElem& R, int nm, Basis basis, const std::vector<double>& sp, const std::vector<double>& vq,
                     const std::vector<double>& vw, const std::vector<FaceData>& faces) {
  const int ns = (int)sp.size() / 3;
  R.nd = 3; R.ns = ns; R.sp = sp;
  std::vector<double> V(ns * nm), Vinv;
  for (int r = 0; r < ns; ++r)
    for (int m = 0; m < nm; ++m) V[r * nm + m] = basis(m, cd(sp[3 * r]), cd(sp[3 * r + 1]), cd(sp[3 * r + 2])).real();
  invert(V, ns, Vinv);
  auto lval = [&](int j, double r, double s, double t) {
    double v = 0.0;
    for (int m = 0; m < nm; ++m) v += Vinv[m * ns + j] * basis(m, cd(r), cd(s), cd(t)).real();
    return v;
  };
  auto lgrad = [&](int j, const double* X, int d) {
    const double hh = 1e-30;
    double v = 0.0;
    for (int m = 0; m < nm; ++m) {
      cd a(X[0], d == 0 ? hh : 0.0), b(X[1], d == 1 ? hh : 0.0), c(X[2], d == 2 ? hh : 0.0);
      v += Vinv[m * ns + j] * basis(m, a, b, c).imag() / hh;
    }
    return v;
  };
  R.nface = (int)faces.size();
  R.face_off.assign(1, 0);
  R.fp.clear(); R.nref.clear(); R.fface.clear();
  for (int f = 0; f < R.nface; ++f) {
    const int nfp = (int)faces[f].fp.size() / 3;
    R.face_off.push_back(R.face_off.back() + nfp);
    R.fp.insert(R.fp.end(), faces[f].fp.begin(), faces[f].fp.end());
    for (int g = 0; g < nfp; ++g) {
      R.nref.insert(R.nref.end(), faces[f].n, faces[f].n + 3);
      R.fface.push_back(f);
    }
  }
  R.nf = R.face_off.back();
  R.M0.assign(R.nf * ns, 0.0);
  for (int g = 0; g < R.nf; ++g)
    for (int j = 0; j < ns; ++j) R.M0[g * ns + j] = lval(j, R.fp[3 * g], R.fp[3 * g + 1], R.fp[3 * g + 2]);
  R.Dm.assign(3 * ns * ns, 0.0);
  for (int d = 0; d < 3; ++d)
    for (int r = 0; r < ns; ++r)
      for (int j = 0; j < ns; ++j) R.Dm[(d * ns + r) * ns + j] = lgrad(j, &sp[3 * r], d);
  // mass matrix by the volume rule
  const int nq = (int)vw.size();
  std::vector<double> L(nq * ns);
  for (int a = 0; a < nq; ++a)
    for (int j = 0; j < ns; ++j) L[a * ns + j] = lval(j, vq[3 * a], vq[3 * a + 1], vq[3 * a + 2]);
  std::vector<double> Mm(ns * ns, 0.0), Minv;
  for (int a = 0; a < nq; ++a)
    for (int i = 0; i < ns; ++i)
      for (int j = 0; j < ns; ++j) Mm[i * ns + j] += vw[a] * L[a * ns + i] * L[a * ns + j];
  invert(Mm, ns, Minv);
  // E[j][g] = int_face l_j phi_g dS, then the lifting M^{-1} E
  std::vector<double> E(ns * R.nf, 0.0);
  for (int f = 0; f < R.nface; ++f) {
    const FaceData& F = faces[f];
    const int nfp = R.face_off[f + 1] - R.face_off[f], nqf = (int)F.qw.size();
    for (int a = 0; a < nqf; ++a)
      for (int j = 0; j < ns; ++j) {
        const double lj = lval(j, F.qx[3 * a], F.qx[3 * a + 1], F.qx[3 * a + 2]);
        for (int g = 0; g < nfp; ++g) E[j * R.nf + R.face_off[f] + g] += F.qw[a] * lj * F.phi[a * nfp + g];
      }
  }
  R.Cor.assign(ns * R.nf, 0.0);
  for (int r = 0; r < ns; ++r)
    for (int g = 0; g < R.nf; ++g) {
      double v = 0.0;
      for (int j = 0; j < ns; ++j) v += Minv[r * ns + j] * E[j * R.nf + g];
      R.Cor[r * R.nf + g] = v;
    }
  R.wq.assign(ns, 0.0);
  for (int r = 0; r < ns; ++r)
    for (int j = 0; j < ns; ++j) R.wq[r] += Mm[r * ns + j];
}

static void build_tet(RefElem& R, int p, const double* tet_pts, const double* tri_pts) {
  R.type = TET; R.p = p; R.nvert = 4;
  const double v[4][3] = {{-1, -1, -1}, {1, -1, -1}, {-1, 1, -1}, {-1, -1, 1}};
  R.face_verts = {{0, 1, 2}, {0, 1, 3}, {1, 2, 3}, {0, 2, 3}};
  const double q3 = 1.0 / std::sqrt(3.0);
  const double nrm[4][3] = {{0, 0, -1}, {0, -1, 0}, {q3, q3, q3}, {-1, 0, 0}};
  std::vector<FaceData> faces;
  for (int f = 0; f < 4; ++f)
    faces.push_back(tri_face(v[R.face_verts[f][0]], v[R.face_verts[f][1]], v[R.face_verts[f][2]], nrm[f], p, tri_pts));
  std::vector<std::array<int, 3>> modes;
  for (int i = 0; i <= p; ++i)
    for (int j = 0; i + j <= p; ++j)
      for (int k = 0; i + j + k <= p; ++k) modes.push_back({i, j, k});
  const int ns = (int)modes.size();
  std::vector<double> sp(tet_pts, tet_pts + 3 * ns), q, w;
  tet_rule(p + 2, q, w);
  build_3d(R, ns, [&](int m, const cd& r, const cd& s, const cd& t) { return pkd_tet<cd>(modes[m][0], modes[m][1], modes[m][2], r, s, t); },
           sp, q, w, faces);
}

static void build_prism(RefElem& R, int p, const double* tri_pts) {
  R.type = PRI; R.p = p; R.nvert = 6;
  const double v[6][3] = {{-1, -1, -1}, {1, -1, -1}, {-1, 1, -1}, {-1, -1, 1}, {1, -1, 1}, {-1, 1, 1}};
  // faces: bottom, top (triangles), then the sides s = -1, r + s = 0, r = -1
  R.face_verts = {{0, 1, 2}, {3, 4, 5}, {0, 1, 4, 3}, {1, 2, 5, 4}, {2, 0, 3, 5}};
  const double h = 1.0 / std::sqrt(2.0);
  const double nrm[5][3] = {{0, 0, -1}, {0, 0, 1}, {0, -1, 0}, {h, h, 0}, {-1, 0, 0}};
  std::vector<FaceData> faces;
  faces.push_back(tri_face(v[0], v[1], v[2], nrm[0], p, tri_pts));
  faces.push_back(tri_face(v[3], v[4], v[5], nrm[1], p, tri_pts));
  faces.push_back(quad_face(v[0], v[1], v[3], nrm[2], p));
  faces.push_back(quad_face(v[1], v[2], v[4], nrm[3], p));
  faces.push_back(quad_face(v[2], v[0], v[5], nrm[4], p));
  const int nt = (p + 1) * (p + 2) / 2, n1 = p + 1;
  std::vector<std::array<int, 3>> modes;
  for (int k = 0; k <= p; ++k)
    for (int i = 0; i <= p; ++i)
      for (int j = 0; i + j <= p; ++j) modes.push_back({i, j, k});
  std::vector<double> x, wx; gauss_legendre(n1, x, wx);
  std::vector<double> sp;                     // triangle point i at axis point k: index i + nt k
  for (int k = 0; k < n1; ++k)
    for (int i = 0; i < nt; ++i) { sp.push_back(tri_pts[2 * i]); sp.push_back(tri_pts[2 * i + 1]); sp.push_back(x[k]); }
  std::vector<double> tq, tw, q, w;
  tri_rule(p + 2, tq, tw);
  std::vector<double> lx, lw; gauss_legendre(p + 2, lx, lw);
  for (size_t a = 0; a < tw.size(); ++a)
    for (size_t b = 0; b < lw.size(); ++b) {
      q.push_back(tq[2 * a]); q.push_back(tq[2 * a + 1]); q.push_back(lx[b]);
      w.push_back(tw[a] * lw[b]);
    }
  build_3d(R, (int)modes.size(), [&](int m, const cd& r, const cd& s, const cd& t) {
    return dubiner<cd>(modes[m][0], modes[m][1], r, s) * leg<cd>(modes[m][2], t);
  }, sp, q, w, faces);
}

// ------------------------------------------------------------- the problem
struct Phys {
  int system, nv;
  double c[3], gamma, mu, prandtl, beta, eta;
};

struct Oracle {
  int nd = 0;
  int64_t ne = 0;
  int maxv = 0, maxf = 0;
  Phys ph{};
  RefElem ref[5];
  std::vector<int8_t> etype;
  std::vector<double> xyz;
  std::vector<int64_t> nbr;
  std::vector<int8_t> nbrf;
  std::vector<int64_t> off;      // DOF offset of each element
  // geometry per element (stored flat, offsets by element)
  std::vector<int64_t> goff_s, goff_f;
  std::vector<double> detJ, Smat, Jinv;   // at solution points: [ns], [ns][nd][nd], [ns][nd][nd]
  std::vector<double> nrm, magN, fxyz;    // at flux points: [nf][nd], [nf], [nf][nd]
  std::vector<int> pair;                  // [elem][nf] neighbour flux point index
  std::vector<int64_t> goff_i;            // SDRT: first internal flux point of each element
  std::vector<double> Sint;               // SDRT: detJ J^{-1} at internal flux points [nint][nd][nd]
  int64_t ndof = 0;
  const RefElem& R(int64_t e) const { return ref[etype[e]]; }
};

static void map_eval(const Oracle& O, int64_t e, const double* xi, double* x, double* J) {
  const RefElem& R = O.R(e);
  const int nd = O.nd;
  double N[8], dN[24];
  shape_fn(R.type, xi, N, dN);
  for (int i = 0; i < nd; ++i) {
    x[i] = 0.0;
    for (int j = 0; j < nd; ++j) J[i * nd + j] = 0.0;
  }
  for (int v = 0; v < R.nvert; ++v) {
    const double* X = &O.xyz[(e * O.maxv + v) * nd];
    for (int i = 0; i < nd; ++i) {
      x[i] += N[v] * X[i];
      for (int j = 0; j < nd; ++j) J[i * nd + j] += X[i] * dN[v * nd + j];
    }
  }
}

// adj(J) = detJ * J^{-1}
static double adjugate(int nd, const double* J, double* S) {
  if (nd == 2) {
    S[0] = J[3]; S[1] = -J[1]; S[2] = -J[2]; S[3] = J[0];
    return J[0] * J[3] - J[1] * J[2];
  }
  S[0] = J[4] * J[8] - J[5] * J[7]; S[1] = J[2] * J[7] - J[1] * J[8]; S[2] = J[1] * J[5] - J[2] * J[4];
  S[3] = J[5] * J[6] - J[3] * J[8]; S[4] = J[0] * J[8] - J[2] * J[6]; S[5] = J[2] * J[3] - J[0] * J[5];
  S[6] = J[3] * J[7] - J[4] * J[6]; S[7] = J[1] * J[6] - J[0] * J[7]; S[8] = J[0] * J[4] - J[1] * J[3];
  return J[0] * S[0] + J[1] * S[3] + J[2] * S[6];
}

// --------------------------------------------------------------- physics
template <class T>
static void flux_phys(const Phys& P, int nd, const T* u, const T* q /*[nd][nv]*/, T* f /*[nd][nv]*/) {
  const int nv = P.nv;
  if (P.system == ADVECTION) {
    for (int d = 0; d < nd; ++d) f[d * nv] = P.c[d] * u[0];
    if (P.mu != 0.0)
      for (int d = 0; d < nd; ++d) f[d * nv] -= P.mu * q[d * nv];
    return;
  }
  const double g = P.gamma;
  T rho = u[0], E = u[nd + 1];
  T v[3], ke = T(0.0);
  for (int i = 0; i < nd; ++i) { v[i] = u[1 + i] / rho; ke += u[1 + i] * v[i]; }
  T p = (g - 1.0) * (E - 0.5 * ke);
  for (int d = 0; d < nd; ++d) {
    f[d * nv + 0] = u[1 + d];
    for (int i = 0; i < nd; ++i) f[d * nv + 1 + i] = u[1 + d] * v[i] + (i == d ? p : T(0.0));
    f[d * nv + nd + 1] = (E + p) * v[d];
  }
  if (P.system != NAVIER_STOKES || q == nullptr) return;
  // velocity gradient dv[i][d] = d v_i / d x_d and gradient of p/rho
  T dv[3][3], dpr[3];
  for (int d = 0; d < nd; ++d) {
    T drho = q[d * nv + 0];
    T vgv = T(0.0);
    for (int i = 0; i < nd; ++i) { dv[i][d] = (q[d * nv + 1 + i] - v[i] * drho) / rho; vgv += v[i] * dv[i][d]; }
    T dE = (q[d * nv + nd + 1] - (E / rho) * drho) / rho;
    dpr[d] = (g - 1.0) * (dE - vgv);
  }
  T divv = T(0.0);
  for (int i = 0; i < nd; ++i) divv += dv[i][i];
  const double mu = P.mu, kap = P.mu * g / (P.prandtl * (g - 1.0));
  for (int d = 0; d < nd; ++d) {
    T tv = T(0.0);
    for (int i = 0; i < nd; ++i) {
      T tau = mu * (dv[i][d] + dv[d][i] - (i == d ? (2.0 / 3.0) * divv : T(0.0)));
      f[d * nv + 1 + i] -= tau;
      tv += tau * v[i];
    }
    f[d * nv + nd + 1] -= kap * dpr[d] + tv;
  }
}

template <class T>
static void common_flux(const Phys& P, int nd, const T* uL, const T* uR, const T* qL, const T* qR,
                        const double* n, T* F) {
  const int nv = P.nv;
  if (P.system == ADVECTION) {
    double cn = 0.0;
    for (int d = 0; d < nd; ++d) cn += P.c[d] * n[d];
    F[0] = 0.5 * cn * (uL[0] + uR[0]) + 0.5 * std::fabs(cn) * (uL[0] - uR[0]);
    if (P.mu != 0.0) {
      for (int d = 0; d < nd; ++d)
        F[0] += n[d] * (-P.mu) * ((0.5 + P.beta) * qL[d * nv] + (0.5 - P.beta) * qR[d * nv]);
      F[0] += P.eta * (uL[0] - uR[0]);
    }
    return;
  }
  // Rusanov: n/2 (f_L + f_R) + |phi|/2 (u_L - u_R), phi = largest |v.n| + c
  T fL[3 * 5], fR[3 * 5];
  flux_phys<T>(P, nd, uL, nullptr, fL);
  flux_phys<T>(P, nd, uR, nullptr, fR);
  auto speed = [&](const T* u) {
    T rho = u[0], ke = T(0.0), vn = T(0.0);
    for (int i = 0; i < nd; ++i) { ke += u[1 + i] * u[1 + i] / rho; vn += n[i] * u[1 + i] / rho; }
    T p = (P.gamma - 1.0) * (u[nd + 1] - 0.5 * ke);
    return tabs(vn) + std::sqrt(P.gamma * p / rho);
  };
  T phi = tmax(speed(uL), speed(uR));
  for (int a = 0; a < nv; ++a) {
    T s = T(0.0);
    for (int d = 0; d < nd; ++d) s += n[d] * (fL[d * nv + a] + fR[d * nv + a]);
    F[a] = 0.5 * s + 0.5 * phi * (uL[a] - uR[a]);
  }
  if (P.system != NAVIER_STOKES) return;
  // viscous: n.[(1/2+beta) f^v_L + (1/2-beta) f^v_R] + eta (u_L - u_R)
  T zq[3 * 5];
  for (int i = 0; i < nd * nv; ++i) zq[i] = T(0.0);
  T vL[3 * 5], vR[3 * 5], cL[3 * 5], cR[3 * 5];
  flux_phys<T>(P, nd, uL, qL, vL); flux_phys<T>(P, nd, uL, zq, cL);
  flux_phys<T>(P, nd, uR, qR, vR); flux_phys<T>(P, nd, uR, zq, cR);
  for (int a = 0; a < nv; ++a) {
    T s = T(0.0);
    for (int d = 0; d < nd; ++d)
      s += n[d] * ((0.5 + P.beta) * (vL[d * nv + a] - cL[d * nv + a]) + (0.5 - P.beta) * (vR[d * nv + a] - cR[d * nv + a]));
    F[a] += s + P.eta * (uL[a] - uR[a]);
  }
}

// --------------------------------------------------------- state access
template <class T> struct State {
  const double* U;
  const double* dir = nullptr;   // full-mesh direction (JVP)
  int64_t pe = -1;               // single perturbed entry (element, row)
  int pr = -1;
  double h = 1e-30;
  const Oracle* O;
  T get(int64_t e, int r) const;
};
template <> double State<double>::get(int64_t e, int r) const { return U[O->off[e] + r]; }
template <> cd State<cd>::get(int64_t e, int r) const {
  double im = 0.0;
  if (dir) im += h * dir[O->off[e] + r];
  if (e == pe && r == pr) im += h;
  return cd(U[O->off[e] + r], im);
}

static bool viscous(const Phys& P) {
  return P.system == NAVIER_STOKES || (P.system == ADVECTION && P.mu != 0.0);
}

// u of element e at its flux point g
template <class T> static T face_value(const Oracle& O, const State<T>& S, int64_t e, int g, int a) {
  const RefElem& R = O.R(e);
  T v = T(0.0);
  for (int s = 0; s < R.ns; ++s) v += R.M0[g * R.ns + s] * S.get(e, s * O.ph.nv + a);
  return v;
}

// Physical corrected gradient q[ns][nd][nv] of element e.
template <class T> static void elem_grad(const Oracle& O, const State<T>& S, int64_t e, T* q) {
  const RefElem& R = O.R(e);
  const int nd = O.nd, nv = O.ph.nv, ns = R.ns, nf = R.nf;
  std::vector<T> u(ns * nv), uf(nf * nv), C(nf * nv), qt(ns * nd * nv);
  for (int s = 0; s < ns; ++s)
    for (int a = 0; a < nv; ++a) u[s * nv + a] = S.get(e, s * nv + a);
  for (int g = 0; g < nf; ++g)
    for (int a = 0; a < nv; ++a) {
      T v = T(0.0);
      for (int s = 0; s < ns; ++s) v += R.M0[g * ns + s] * u[s * nv + a];
      uf[g * nv + a] = v;
    }
  // common solution (eq. common_var_for_grad)
  for (int g = 0; g < nf; ++g) {
    int64_t m = O.nbr[e * O.maxf + R.fface[g]];
    int g2 = O.pair[O.goff_f[e] + g];
    for (int a = 0; a < nv; ++a) {
      T uR = face_value(O, S, m, g2, a);
      C[g * nv + a] = (0.5 - O.ph.beta) * uf[g * nv + a] + (0.5 + O.ph.beta) * uR;
    }
  }
  if (R.scheme == 2) {
    // SDRT: q~(x_rho) = sum_int u_int n_int div psi_int(x_rho) + sum_ext C n_ext div psi_ext(x_rho)
    std::vector<T> ui(R.nint * nv);
    for (int k = 0; k < R.nint; ++k)
      for (int a = 0; a < nv; ++a) {
        T v = T(0.0);
        for (int s = 0; s < ns; ++s) v += R.Mint[k * ns + s] * u[s * nv + a];
        ui[k * nv + a] = v;
      }
    for (int r = 0; r < ns; ++r)
      for (int d = 0; d < nd; ++d)
        for (int a = 0; a < nv; ++a) {
          T v = T(0.0);
          for (int k = 0; k < R.nint; ++k)
            if (R.idir[k] == d) v += R.Dint[r * R.nint + k] * ui[k * nv + a];
          for (int g = 0; g < nf; ++g) v += R.Cor[r * nf + g] * R.nref[g * nd + d] * C[g * nv + a];
          qt[(r * nd + d) * nv + a] = v;
        }
  } else {
  for (int r = 0; r < ns; ++r)
    for (int d = 0; d < nd; ++d)
      for (int a = 0; a < nv; ++a) {
        T v = T(0.0);
        for (int s = 0; s < ns; ++s) v += R.Dm[(d * ns + r) * ns + s] * u[s * nv + a];
        for (int g = 0; g < nf; ++g)
          v += R.Cor[r * nf + g] * R.nref[g * nd + d] * (C[g * nv + a] - uf[g * nv + a]);
        qt[(r * nd + d) * nv + a] = v;
      }
  }
  const double* Ji = &O.Jinv[O.goff_s[e] * nd * nd];
  for (int r = 0; r < ns; ++r)
    for (int d2 = 0; d2 < nd; ++d2)
      for (int a = 0; a < nv; ++a) {
        T v = T(0.0);
        for (int d = 0; d < nd; ++d) v += Ji[(r * nd + d) * nd + d2] * qt[(r * nd + d) * nv + a];
        q[(r * nd + d2) * nv + a] = v;
      }
}

// Residual of element n given its gradient and its face neighbours' gradients.
template <class T>
static void elem_residual(const Oracle& O, const State<T>& S, int64_t n, const T* qn,
                          const T* const* qnb /*[nface]*/, T* Rout) {
  const RefElem& R = O.R(n);
  const int nd = O.nd, nv = O.ph.nv, ns = R.ns, nf = R.nf;
  const bool visc = viscous(O.ph);
  std::vector<T> u(ns * nv), Ft(ns * nd * nv), div(ns * nv);
  for (int s = 0; s < ns; ++s)
    for (int a = 0; a < nv; ++a) u[s * nv + a] = S.get(n, s * nv + a);
  const double* Sm = &O.Smat[O.goff_s[n] * nd * nd];
  // transformed flux at solution points F~_d = sum_k S_dk f_k
  for (int s = 0; s < ns; ++s) {
    T f[3 * 5];
    flux_phys<T>(O.ph, nd, &u[s * nv], visc ? &qn[s * nd * nv] : nullptr, f);
    for (int d = 0; d < nd; ++d)
      for (int a = 0; a < nv; ++a) {
        T v = T(0.0);
        for (int k = 0; k < nd; ++k) v += Sm[(s * nd + d) * nd + k] * f[k * nv + a];
        Ft[(s * nd + d) * nv + a] = v;
      }
  }
  if (R.scheme == 2) {
    // SDRT volume part: transformed normal flux at the internal flux points,
    // F~n = (detJ J^{-1} f(u_int, q_int)) . e_d, times div psi_int
    for (int r = 0; r < ns * nv; ++r) div[r] = T(0.0);
    for (int k = 0; k < R.nint; ++k) {
      T ui[5], qi[3 * 5], f[3 * 5];
      for (int a = 0; a < nv; ++a) {
        T v = T(0.0);
        for (int s = 0; s < ns; ++s) v += R.Mint[k * ns + s] * u[s * nv + a];
        ui[a] = v;
      }
      if (visc)
        for (int d = 0; d < nd; ++d)
          for (int a = 0; a < nv; ++a) {
            T v = T(0.0);
            for (int s = 0; s < ns; ++s) v += R.Mint[k * ns + s] * qn[(s * nd + d) * nv + a];
            qi[d * nv + a] = v;
          }
      flux_phys<T>(O.ph, nd, ui, visc ? qi : nullptr, f);
      const double* Si = &O.Sint[(O.goff_i[n] + k) * nd * nd];
      const int d = R.idir[k];
      for (int a = 0; a < nv; ++a) {
        T fn = T(0.0);
        for (int kk = 0; kk < nd; ++kk) fn += Si[d * nd + kk] * f[kk * nv + a];
        for (int r = 0; r < ns; ++r) div[r * nv + a] += R.Dint[r * R.nint + k] * fn;
      }
    }
  } else {
  // volume part: sum_d D_d F~_d
  for (int r = 0; r < ns; ++r)
    for (int a = 0; a < nv; ++a) {
      T v = T(0.0);
      for (int d = 0; d < nd; ++d)
        for (int s = 0; s < ns; ++s) v += R.Dm[(d * ns + r) * ns + s] * Ft[(s * nd + d) * nv + a];
      div[r * nv + a] = v;
    }
  }
  // flux points: interpolated discontinuous normal flux and common flux
  for (int g = 0; g < nf; ++g) {
    int f = R.fface[g];
    int64_t m = O.nbr[n * O.maxf + f];
    int g2 = O.pair[O.goff_f[n] + g];
    const RefElem& Rm = O.R(m);
    T uL[5], uR[5], qL[3 * 5], qR[3 * 5], Fn[5], Fc[5];
    for (int a = 0; a < nv; ++a) {
      T vl = T(0.0);
      for (int s = 0; s < ns; ++s) vl += R.M0[g * ns + s] * u[s * nv + a];
      uL[a] = vl;
      uR[a] = face_value(O, S, m, g2, a);
      T fnv = T(0.0);
      for (int d = 0; d < nd; ++d) {
        T t = T(0.0);
        for (int s = 0; s < ns; ++s) t += R.M0[g * ns + s] * Ft[(s * nd + d) * nv + a];
        fnv += R.nref[g * nd + d] * t;
      }
      Fn[a] = fnv;
    }
    if (visc) {
      for (int d = 0; d < nd; ++d)
        for (int a = 0; a < nv; ++a) {
          T l = T(0.0), rr = T(0.0);
          for (int s = 0; s < ns; ++s) l += R.M0[g * ns + s] * qn[(s * nd + d) * nv + a];
          for (int s = 0; s < Rm.ns; ++s) rr += Rm.M0[g2 * Rm.ns + s] * qnb[f][(s * nd + d) * nv + a];
          qL[d * nv + a] = l; qR[d * nv + a] = rr;
        }
    }
    const double* nn = &O.nrm[(O.goff_f[n] + g) * nd];
    common_flux<T>(O.ph, nd, uL, uR, qL, qR, nn, Fc);
    double mg = O.magN[O.goff_f[n] + g];
    for (int a = 0; a < nv; ++a) {
      // SDRT: the common flux times the external basis divergence; FR: the
      // correction of the interpolated normal flux to the common flux
      T jump = (R.scheme == 2) ? mg * Fc[a] : mg * Fc[a] - Fn[a];
      for (int r = 0; r < ns; ++r) div[r * nv + a] += R.Cor[r * nf + g] * jump;
    }
  }
  const double* dj = &O.detJ[O.goff_s[n]];
  for (int r = 0; r < ns; ++r)
    for (int a = 0; a < nv; ++a) Rout[r * nv + a] = -div[r * nv + a] / dj[r];
}

// Residual of element n computing every gradient it needs on the fly.
template <class T> static void elem_residual_local(const Oracle& O, const State<T>& S, int64_t n, T* Rout) {
  const RefElem& R = O.R(n);
  const int nd = O.nd, nv = O.ph.nv;
  if (!viscous(O.ph)) {
    elem_residual<T>(O, S, n, nullptr, nullptr, Rout);
    return;
  }
  std::vector<T> qn(R.ns * nd * nv);
  elem_grad<T>(O, S, n, qn.data());
  std::vector<std::vector<T>> qb(R.nface);
  std::vector<const T*> qp(R.nface);
  for (int f = 0; f < R.nface; ++f) {
    int64_t m = O.nbr[n * O.maxf + f];
    qb[f].resize(O.R(m).ns * nd * nv);
    elem_grad<T>(O, S, m, qb[f].data());
    qp[f] = qb[f].data();
  }
  elem_residual<T>(O, S, n, qn.data(), qp.data(), Rout);
}

// Full-mesh residual: gradients of every element first, then residuals.
template <class T> static void full_residual(const Oracle& O, const State<T>& S, T* Rall) {
  const int nd = O.nd, nv = O.ph.nv;
  const bool visc = viscous(O.ph);
  std::vector<int64_t> qoff(O.ne + 1, 0);
  for (int64_t e = 0; e < O.ne; ++e) qoff[e + 1] = qoff[e] + (visc ? O.R(e).ns * nd * nv : 0);
  std::vector<T> q(qoff[O.ne]);
  if (visc) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t e = 0; e < O.ne; ++e) elem_grad<T>(O, S, e, &q[qoff[e]]);
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t n = 0; n < O.ne; ++n) {
    const T* qp[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    if (visc)
      for (int f = 0; f < O.R(n).nface; ++f) qp[f] = &q[qoff[O.nbr[n * O.maxf + f]]];
    elem_residual<T>(O, S, n, visc ? &q[qoff[n]] : nullptr, qp, &Rall[O.off[n]]);
  }
}

// ------------------------------------------------------------- set-up
static int setup(Oracle& O, std::vector<std::string>& err) {
  (void)err;
  const int nd = O.nd;
  O.off.assign(O.ne + 1, 0);
  O.goff_s.assign(O.ne + 1, 0);
  O.goff_f.assign(O.ne + 1, 0);
  for (int64_t e = 0; e < O.ne; ++e) {
    const RefElem& R = O.R(e);
    O.off[e + 1] = O.off[e] + (int64_t)R.ns * O.ph.nv;
    O.goff_s[e + 1] = O.goff_s[e] + R.ns;
    O.goff_f[e + 1] = O.goff_f[e] + R.nf;
  }
  O.ndof = O.off[O.ne];
  O.detJ.assign(O.goff_s[O.ne], 0.0);
  O.Smat.assign(O.goff_s[O.ne] * nd * nd, 0.0);
  O.Jinv.assign(O.goff_s[O.ne] * nd * nd, 0.0);
  O.nrm.assign(O.goff_f[O.ne] * nd, 0.0);
  O.magN.assign(O.goff_f[O.ne], 0.0);
  O.fxyz.assign(O.goff_f[O.ne] * nd, 0.0);
  O.pair.assign(O.goff_f[O.ne], -1);
  for (int64_t e = 0; e < O.ne; ++e) {
    const RefElem& R = O.R(e);
    double x[3], J[9], S[9];
    for (int r = 0; r < R.ns; ++r) {
      map_eval(O, e, &R.sp[r * nd], x, J);
      double dj = adjugate(nd, J, S);
      if (!(dj > 0.0)) return -1;
      int64_t k = O.goff_s[e] + r;
      O.detJ[k] = dj;
      for (int i = 0; i < nd * nd; ++i) { O.Smat[k * nd * nd + i] = S[i]; O.Jinv[k * nd * nd + i] = S[i] / dj; }
    }
    for (int g = 0; g < R.nf; ++g) {
      map_eval(O, e, &R.fp[g * nd], x, J);
      adjugate(nd, J, S);
      int64_t k = O.goff_f[e] + g;
      double N[3] = {0, 0, 0}, mg = 0.0;
      for (int i = 0; i < nd; ++i) {
        for (int d = 0; d < nd; ++d) N[i] += S[d * nd + i] * R.nref[g * nd + d];  // N = S^T n_ref
        mg += N[i] * N[i];
      }
      mg = std::sqrt(mg);
      O.magN[k] = mg;
      for (int i = 0; i < nd; ++i) { O.nrm[k * nd + i] = N[i] / mg; O.fxyz[k * nd + i] = x[i]; }
    }
  }
  // SDRT: metric terms at the internal flux points
  O.goff_i.assign(O.ne + 1, 0);
  for (int64_t e = 0; e < O.ne; ++e) O.goff_i[e + 1] = O.goff_i[e] + O.R(e).nint;
  O.Sint.assign(O.goff_i[O.ne] * nd * nd, 0.0);
  for (int64_t e = 0; e < O.ne; ++e) {
    const RefElem& R = O.R(e);
    double x[3], J[9], S[9];
    for (int k = 0; k < R.nint; ++k) {
      map_eval(O, e, &R.ip[k * nd], x, J);
      adjugate(nd, J, S);
      for (int i = 0; i < nd * nd; ++i) O.Sint[(O.goff_i[e] + k) * nd * nd + i] = S[i];
    }
  }
  // Pair flux points across faces by physical position relative to the
  // face centroid (translation invariant, so periodic wraps pair too).
  for (int64_t e = 0; e < O.ne; ++e) {
    const RefElem& R = O.R(e);
    for (int f = 0; f < R.nface; ++f) {
      int64_t m = O.nbr[e * O.maxf + f];
      int f2 = O.nbrf[e * O.maxf + f];
      if (m < 0 || m >= O.ne) return -2;
      const RefElem& Rm = O.R(m);
      double c1[3] = {0, 0, 0}, c2[3] = {0, 0, 0}, hsz = 0.0;
      for (int v : R.face_verts[f])
        for (int i = 0; i < nd; ++i) c1[i] += O.xyz[(e * O.maxv + v) * nd + i] / R.face_verts[f].size();
      for (int v : Rm.face_verts[f2])
        for (int i = 0; i < nd; ++i) c2[i] += O.xyz[(m * O.maxv + v) * nd + i] / Rm.face_verts[f2].size();
      for (int i = 0; i < nd; ++i) {
        double d = O.xyz[(e * O.maxv + R.face_verts[f][0]) * nd + i] - c1[i];
        hsz += d * d;
      }
      hsz = std::sqrt(hsz);
      for (int g = R.face_off[f]; g < R.face_off[f + 1]; ++g) {
        int best = -1; double bd = 1e300;
        for (int g2 = Rm.face_off[f2]; g2 < Rm.face_off[f2 + 1]; ++g2) {
          double d2 = 0.0;
          for (int i = 0; i < nd; ++i) {
            double a = (O.fxyz[(O.goff_f[e] + g) * nd + i] - c1[i]) - (O.fxyz[(O.goff_f[m] + g2) * nd + i] - c2[i]);
            d2 += a * a;
          }
          if (d2 < bd) { bd = d2; best = g2; }
        }
        if (std::sqrt(bd) > 1e-8 * hsz) return -3;
        O.pair[O.goff_f[e] + g] = best;
      }
    }
  }
  return 0;
}

// ============================================================== C entry points
extern "C" {

// Create an oracle for a mesh.  Tensor elements use Gauss-Legendre points;
// triangles use tri_pts[ns][2] (may be NULL when there are none).
int oracle_create(int nd, int64_t ne, const int8_t* etype, int p, const double* xyz, int maxv,
                  const int64_t* nbr, const int8_t* nbrf, int maxf, int system, int nv,
                  const double* c, double gamma, double mu, double prandtl, double beta, double eta,
                  int scheme, const double* tri_pts, const double* tet_pts, void** out) {
  // BR1 only: beta = 0 and no penalty (the von Neumann analysis with
  // diffusion identifies BR1 with beta = 0).  A single scalar beta taken
  // from each element's own side would make the common solution and the
  // viscous common flux two-valued across a face.
  if (beta != 0.0 || eta != 0.0) return -11;
  Oracle* O = new Oracle();
  O->nd = nd; O->ne = ne; O->maxv = maxv; O->maxf = maxf;
  O->ph.system = system; O->ph.nv = nv;
  for (int i = 0; i < 3; ++i) O->ph.c[i] = c ? c[i] : 0.0;
  O->ph.gamma = gamma; O->ph.mu = mu; O->ph.prandtl = prandtl; O->ph.beta = beta; O->ph.eta = eta;
  O->etype.assign(etype, etype + ne);
  O->xyz.assign(xyz, xyz + ne * maxv * nd);
  O->nbr.assign(nbr, nbr + ne * maxf);
  O->nbrf.assign(nbrf, nbrf + ne * maxf);
  bool has[5] = {false, false, false, false, false};
  for (int64_t e = 0; e < ne; ++e) {
    if (etype[e] < 0 || etype[e] > 4) { delete O; return -13; }
    has[etype[e]] = true;
  }
  if (scheme < 0 || scheme > 2 || (scheme != 0 && (has[TRI] || has[TET] || has[PRI]))) { delete O; return -12; }
  if (has[QUAD]) build_tensor(O->ref[QUAD], QUAD, p, scheme);
  if (has[HEX]) build_tensor(O->ref[HEX], HEX, p, scheme);
  if (has[TRI]) {
    if (!tri_pts) { delete O; return -10; }
    build_tri(O->ref[TRI], p, tri_pts);
  }
  if (has[TET]) {
    if (!tri_pts || !tet_pts) { delete O; return -10; }
    build_tet(O->ref[TET], p, tet_pts, tri_pts);
  }
  if (has[PRI]) {
    if (!tri_pts) { delete O; return -10; }
    build_prism(O->ref[PRI], p, tri_pts);
  }
  std::vector<std::string> err;
  int rc = setup(*O, err);
  if (rc != 0) { delete O; return rc; }
  *out = O;
  return 0;
}

void oracle_destroy(void* h) { delete (Oracle*)h; }
int64_t oracle_ndof(void* h) { return ((Oracle*)h)->ndof; }

// R(U), FP64.
void oracle_rhs(void* h, const double* U, double* R) {
  Oracle& O = *(Oracle*)h;
  State<double> S; S.U = U; S.O = &O;
  full_residual<double>(O, S, R);
}

// Jv = dR/dU(U) v by complex step over the whole mesh.
void oracle_jvp(void* h, const double* U, const double* v, double* Jv) {
  Oracle& O = *(Oracle*)h;
  State<cd> S; S.U = U; S.O = &O; S.dir = v;
  std::vector<cd> R(O.ndof);
  full_residual<cd>(O, S, R.data());
  for (int64_t i = 0; i < O.ndof; ++i) Jv[i] = R[i].imag() / S.h;
}

// Block dR_n/dU_k, row-major [rows of n][cols of k].
void oracle_jac_block(void* h, const double* U, int64_t n, int64_t k, double* out) {
  Oracle& O = *(Oracle*)h;
  int bn = O.R(n).ns * O.ph.nv, bk = O.R(k).ns * O.ph.nv;
  std::vector<cd> R(bn);
  for (int c = 0; c < bk; ++c) {
    State<cd> S; S.U = U; S.O = &O; S.pe = k; S.pr = c;
    elem_residual_local<cd>(O, S, n, R.data());
    for (int r = 0; r < bn; ++r) out[(int64_t)r * bk + c] = R[r].imag() / S.h;
  }
}

// For each listed element n: the self block and one block per local face
// (dR_n/dU_{nbr(n,f)}), each row-major bn x bk, concatenated per element in
// the order (self, face 0, face 1, ...).  Element blocks are packed with
// stride `stride` doubles.
void oracle_jac_blocks(void* h, const double* U, const int64_t* elems, int64_t count, double* out, int64_t stride) {
  Oracle& O = *(Oracle*)h;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < count; ++i) {
    int64_t n = elems[i];
    const RefElem& R = O.R(n);
    double* o = out + i * stride;
    int bn = R.ns * O.ph.nv;
    oracle_jac_block(h, U, n, n, o);
    o += (int64_t)bn * bn;
    for (int f = 0; f < R.nface; ++f) {
      int64_t m = O.nbr[n * O.maxf + f];
      int bk = O.R(m).ns * O.ph.nv;
      oracle_jac_block(h, U, n, m, o);
      o += (int64_t)bn * bk;
    }
  }
}

// Dense Jacobian, row-major ndof x ndof (tiny meshes only).
void oracle_jac_full(void* h, const double* U, double* out) {
  Oracle& O = *(Oracle*)h;
  const int64_t N = O.ndof;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t j = 0; j < N; ++j) {
    int64_t e = 0;
    while (O.off[e + 1] <= j) ++e;
    State<cd> S; S.U = U; S.O = &O; S.pe = e; S.pr = (int)(j - O.off[e]);
    std::vector<cd> R(N);
    full_residual<cd>(O, S, R.data());
    for (int64_t i = 0; i < N; ++i) out[i * N + j] = R[i].imag() / S.h;
  }
}

// Geometry of element e: detJ at solution points, flux-point coordinates,
// N = S^T n_ref (= magN * unit normal) and the neighbour pairing.
int oracle_elem_geom(void* h, int64_t e, double* detJ, double* fx, double* N, int* pair, double* sx) {
  Oracle& O = *(Oracle*)h;
  const RefElem& R = O.R(e);
  const int nd = O.nd;
  for (int r = 0; r < R.ns; ++r) {
    detJ[r] = O.detJ[O.goff_s[e] + r];
    if (sx) {
      double x[3], J[9];
      map_eval(O, e, &R.sp[r * nd], x, J);
      for (int i = 0; i < nd; ++i) sx[r * nd + i] = x[i];
    }
  }
  for (int g = 0; g < R.nf; ++g) {
    int64_t k = O.goff_f[e] + g;
    for (int i = 0; i < nd; ++i) {
      fx[g * nd + i] = O.fxyz[k * nd + i];
      N[g * nd + i] = O.nrm[k * nd + i] * O.magN[k];
    }
    pair[g] = O.pair[k];
  }
  return R.nf;
}

// Reference data of an element type (row-major dense matrices).
int oracle_ref(void* h, int type, int* dims, double* sp, double* fp, double* nref, double* M0, double* Dm,
               double* Cor, double* wq, int* fface) {
  Oracle& O = *(Oracle*)h;
  const RefElem& R = O.ref[type];
  if (R.type < 0) return -1;
  dims[0] = R.ns; dims[1] = R.nf; dims[2] = R.nd; dims[3] = R.nface;
  if (!sp) return 0;
  std::memcpy(sp, R.sp.data(), R.sp.size() * 8);
  std::memcpy(fp, R.fp.data(), R.fp.size() * 8);
  std::memcpy(nref, R.nref.data(), R.nref.size() * 8);
  std::memcpy(M0, R.M0.data(), R.M0.size() * 8);
  std::memcpy(Dm, R.Dm.data(), R.Dm.size() * 8);
  std::memcpy(Cor, R.Cor.data(), R.Cor.size() * 8);
  std::memcpy(wq, R.wq.data(), R.wq.size() * 8);
  for (int g = 0; g < R.nf; ++g) fface[g] = R.fface[g];
  return 0;
}

// 1-D data: GL nodes/weights, D1[i][j] = l_j'(x_i), l_j(+-1), and the Radau
// correction derivatives hp_i = g_R'(x_i), hm_i = -g_L'(x_i).
void oracle_ref1d(int p, double* x, double* w, double* D, double* lp, double* lm, double* hp, double* hm) {
  std::vector<double> X, W; gauss_legendre(p + 1, X, W);
  for (int i = 0; i <= p; ++i) {
    x[i] = X[i]; w[i] = W[i];
    lp[i] = lagrange(X, i, 1.0); lm[i] = lagrange(X, i, -1.0);
    hp[i] = radau_right_d(p, X[i]); hm[i] = radau_right_d(p, -X[i]);
    for (int j = 0; j <= p; ++j) D[i * (p + 1) + j] = lagrange_d(X, j, X[i]);
  }
}

// Pointwise physics for tests: physical flux f[nd][nv] of (u, q) and the
// common flux at one point pair.
void oracle_flux(int system, int nd, int nv, const double* c, double gamma, double mu, double prandtl,
                 const double* u, const double* q, double* f) {
  Phys P{}; P.system = system; P.nv = nv; P.gamma = gamma; P.mu = mu; P.prandtl = prandtl;
  for (int i = 0; i < 3; ++i) P.c[i] = c ? c[i] : 0.0;
  flux_phys<double>(P, nd, u, q, f);
}
void oracle_common_flux(int system, int nd, int nv, const double* c, double gamma, double mu, double prandtl,
                        double beta, double eta, const double* uL, const double* uR, const double* qL,
                        const double* qR, const double* n, double* F) {
  Phys P{}; P.system = system; P.nv = nv; P.gamma = gamma; P.mu = mu; P.prandtl = prandtl;
  P.beta = beta; P.eta = eta;
  for (int i = 0; i < 3; ++i) P.c[i] = c ? c[i] : 0.0;
  common_flux<double>(P, nd, uL, uR, qL, qR, n, F);
}

// Plain partial-pivot LU solve of a dense row-major n x n system (A copied).
int oracle_lu_solve(int n, const double* A, const double* b, double* x) {
  std::vector<double> M(A, A + (size_t)n * n);
  std::vector<double> y(b, b + n);
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(M[(size_t)r * n + c]) > std::fabs(M[(size_t)piv * n + c])) piv = r;
    if (M[(size_t)piv * n + c] == 0.0) return -1;
    if (piv != c) {
      for (int k = 0; k < n; ++k) std::swap(M[(size_t)c * n + k], M[(size_t)piv * n + k]);
      std::swap(y[c], y[piv]);
    }
    for (int r = c + 1; r < n; ++r) {
      double l = M[(size_t)r * n + c] / M[(size_t)c * n + c];
      M[(size_t)r * n + c] = l;
      for (int k = c + 1; k < n; ++k) M[(size_t)r * n + k] -= l * M[(size_t)c * n + k];
      y[r] -= l * y[c];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    double s = y[r];
    for (int k = r + 1; k < n; ++k) s -= M[(size_t)r * n + k] * x[k];
    x[r] = s / M[(size_t)r * n + r];
  }
  return 0;
}

}  // extern "C"
