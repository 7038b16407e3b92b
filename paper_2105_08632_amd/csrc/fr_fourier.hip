// Fourier (von Neumann) analysis of the FR semi-discretisation dU/dt = J U on
// uniform periodic meshes, from the library's own Jacobian blocks.
//
// On a uniform periodic mesh the Jacobian is block-circulant: every element
// sees the same blocks B_k of its face stencil.  A Bloch wave
// U_m = U_hat exp(i kappa . x_m) turns dU/dt = J U into dU_hat/dt = G(kappa)
// U_hat with G(kappa) = sum_k B_k exp(i kappa . d_k), d_k the offset of block
// k's element (section on temporal linear stability: the semi-discrete
// pattern of the Fourier analysis).  An explicit Runge-Kutta scheme with
// amplification polynomial P is stable for the time step tau when
// |P(tau lambda)| <= 1 for every eigenvalue lambda of every G(kappa) (the
// exponential's truncations of the same section); CFL_MAX is the largest
// such tau for eigenvalues of the Jacobian scaled by h / |c|.
//
// k_fourier_eigs: one wavefront per wavenumber.  G (complex, b <= 64) is
// formed in LDS, reduced to upper Hessenberg form by Householder reflections
// and its eigenvalues found by the shifted QR algorithm (Wilkinson shifts,
// Givens rotations, deflation at negligible subdiagonals), all in FP64.
// k_cfl_max: bisection on tau over all eigenvalues (one workgroup).
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "fr.h"
#include "fr_ctx.hpp"

namespace {

struct cplx {
  double re, im;
};
__device__ inline cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ inline cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ inline cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline cplx cconj(cplx a) { return {a.re, -a.im}; }
__device__ inline cplx cscale(cplx a, double s) { return {a.re * s, a.im * s}; }
__device__ inline double cabs2(cplx a) { return a.re * a.re + a.im * a.im; }
__device__ inline double cabs(cplx a) { return hypot(a.re, a.im); }
__device__ inline cplx csqrt(cplx a) {
  const double r = cabs(a);
  double x = sqrt(0.5 * (r + fabs(a.re)));
  if (x == 0.0) return {0.0, 0.0};
  double y = a.im / (2.0 * x);
  if (a.re >= 0.0) return {x, y};
  return {fabs(y), a.im >= 0.0 ? x : -x};
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

constexpr int kFB = 64;        // largest block order
constexpr int kFS = kFB + 1;   // LDS row stride (complex entries)
constexpr int kMaxBlk = 7;     // blocks of the face stencil (hexahedra: self + 6)

struct FourierArgs {
  int b, nblk, nd;
  double scale;
  double d[kMaxBlk][3];        // offsets of the blocks' elements
  long blk_off[kMaxBlk];       // offset of block k in the block array (entries)
};

}  // namespace

template <class IT>
__global__ void __launch_bounds__(64) k_fourier_eigs(FourierArgs a, const IT* B, const double* kappa, long nk,
                                                     double* eigs) {
  __shared__ cplx H[kFB * kFS];
  __shared__ cplx v[kFB];
  __shared__ cplx cs_s[kFB];
  __shared__ double cc_s[kFB];
  const long q = blockIdx.x;
  const int lane = threadIdx.x, b = a.b;
  // G = scale sum_k B_k exp(i kappa . d_k); lane = column
  cplx ph[kMaxBlk];
  for (int k = 0; k < a.nblk; ++k) {
    double t = 0.0;
    for (int d = 0; d < a.nd; ++d) t += kappa[q * a.nd + d] * a.d[k][d];
    ph[k] = {a.scale * cos(t), a.scale * sin(t)};
  }
  if (lane < b)
    for (int r = 0; r < b; ++r) {
      cplx g = {0.0, 0.0};
      for (int k = 0; k < a.nblk; ++k) g = cadd(g, cscale(ph[k], (double)B[a.blk_off[k] + (long)lane * b + r]));
      H[r * kFS + lane] = g;
    }
  __syncthreads();
  // Householder reduction to upper Hessenberg form: for column j, the
  // reflection I - tau v v^H maps H[j+1..][j] onto a multiple of e_1
  for (int j = 0; j + 2 < b; ++j) {
    const bool in = lane > j && lane < b;
    const cplx x = in ? H[lane * kFS + j] : cplx{0.0, 0.0};
    const double alpha = sqrt(wave_sum(cabs2(x)));
    const cplx x0 = H[(j + 1) * kFS + j];
    const double ax0 = cabs(x0);
    const double tail = alpha * alpha - ax0 * ax0;
    if (!(alpha > 0.0) || !(tail > 1e-300 * alpha * alpha)) { __syncthreads(); continue; }
    const cplx phase = ax0 > 0.0 ? cscale(x0, 1.0 / ax0) : cplx{1.0, 0.0};
    cplx vr = x;
    if (lane == j + 1) vr = cadd(x, cscale(phase, alpha));
    v[lane] = in ? vr : cplx{0.0, 0.0};
    const double vn2 = wave_sum(in ? cabs2(vr) : 0.0);
    const double tau = 2.0 / vn2;
    __syncthreads();
    // H <- (I - tau v v^H) H: column c = lane
    if (lane >= j && lane < b) {
      cplx w = {0.0, 0.0};
      for (int r = j + 1; r < b; ++r) w = cadd(w, cmul(cconj(v[r]), H[r * kFS + lane]));
      w = cscale(w, tau);
      for (int r = j + 1; r < b; ++r) H[r * kFS + lane] = csub(H[r * kFS + lane], cmul(v[r], w));
    }
    __syncthreads();
    // H <- H (I - tau v v^H): row r = lane
    if (lane < b) {
      cplx w = {0.0, 0.0};
      for (int c = j + 1; c < b; ++c) w = cadd(w, cmul(H[lane * kFS + c], v[c]));
      w = cscale(w, tau);
      for (int c = j + 1; c < b; ++c) H[lane * kFS + c] = csub(H[lane * kFS + c], cmul(w, cconj(v[c])));
    }
    __syncthreads();
    if (lane > j + 1 && lane < b) H[lane * kFS + j] = {0.0, 0.0};
    __syncthreads();
  }
  // shifted QR on the Hessenberg matrix; only the active block [lo, hi]
  // is transformed (eigenvalues only, no Schur vectors)
  double* out = eigs + q * 2 * b;
  int hi = b - 1, iter = 0, total = 0;
  bool failed = false;
  while (hi >= 0) {
    if (hi == 0) {
      if (lane == 0) { out[0] = H[0].re; out[1] = H[0].im; }
      break;
    }
    // lowest row of the active block: the nearest negligible subdiagonal
    int lo = 0;
    for (int k = hi; k >= 1; --k) {
      const double sd = cabs(H[k * kFS + k - 1]);
      const double dn = cabs(H[k * kFS + k]) + cabs(H[(k - 1) * kFS + k - 1]);
      if (sd <= 1e-15 * dn || sd < 1e-300) { lo = k; break; }
    }
    if (lo == hi) {
      if (lane == 0) { out[2 * hi] = H[hi * kFS + hi].re; out[2 * hi + 1] = H[hi * kFS + hi].im; }
      __syncthreads();
      if (lane == 0) H[hi * kFS + hi - 1] = {0.0, 0.0};
      __syncthreads();
      --hi;
      iter = 0;
      continue;
    }
    if (++total > 40 * b) { failed = true; break; }
    ++iter;
    // Wilkinson shift: the eigenvalue of the trailing 2 x 2 nearer H[hi][hi];
    // an exceptional shift after 10 steps without deflation
    const cplx aa = H[(hi - 1) * kFS + hi - 1], bb = H[(hi - 1) * kFS + hi];
    const cplx c2 = H[hi * kFS + hi - 1], dd = H[hi * kFS + hi];
    cplx mu;
    if (iter % 11 == 10) {
      mu = cadd(dd, {0.75 * cabs(c2), 0.0});
    } else {
      const cplx hm = cscale(csub(aa, dd), 0.5);
      const cplx disc = csqrt(cadd(cmul(hm, hm), cmul(bb, c2)));
      const cplx m0 = cadd(cscale(cadd(aa, dd), 0.5), disc), m1 = csub(cscale(cadd(aa, dd), 0.5), disc);
      mu = cabs2(csub(m0, dd)) <= cabs2(csub(m1, dd)) ? m0 : m1;
    }
    // H - mu I = Q R by rotations on rows lo..hi, then R Q + mu I
    if (lane >= lo && lane <= hi) H[lane * kFS + lane] = csub(H[lane * kFS + lane], mu);
    __syncthreads();
    for (int k = lo; k < hi; ++k) {
      const cplx x = H[k * kFS + k], y = H[(k + 1) * kFS + k];
      const double ax = cabs(x), r = hypot(ax, cabs(y));
      double c;
      cplx s;
      if (ax == 0.0) { c = 0.0; s = {1.0, 0.0}; }
      else if (r == 0.0) { c = 1.0; s = {0.0, 0.0}; }
      else { c = ax / r; s = cscale(cmul(cscale(x, 1.0 / ax), cconj(y)), 1.0 / r); }
      if (lane == 0) { cc_s[k] = c; cs_s[k] = s; }
      if (lane >= k && lane <= hi) {
        const cplx u = H[k * kFS + lane], w = H[(k + 1) * kFS + lane];
        H[k * kFS + lane] = cadd(cscale(u, c), cmul(s, w));
        H[(k + 1) * kFS + lane] = csub(cscale(w, c), cmul(cconj(s), u));
      }
      __syncthreads();
    }
    for (int k = lo; k < hi; ++k) {
      const double c = cc_s[k];
      const cplx s = cs_s[k];
      const int rend = min(k + 1, hi);
      if (lane >= lo && lane <= rend) {
        const cplx u = H[lane * kFS + k], w = H[lane * kFS + k + 1];
        H[lane * kFS + k] = cadd(cscale(u, c), cmul(w, cconj(s)));
        H[lane * kFS + k + 1] = csub(cscale(w, c), cmul(u, s));
      }
      __syncthreads();
    }
    if (lane >= lo && lane <= hi) H[lane * kFS + lane] = cadd(H[lane * kFS + lane], mu);
    __syncthreads();
  }
  if (failed)
    for (int i = lane; i <= hi; i += 64) { out[2 * i] = NAN; out[2 * i + 1] = NAN; }
}

// The largest tau in [0, tau_max] with |P(tau lambda)| <= 1 + tol for all n
// eigenvalues, by bisection (60 halvings); NaN if any eigenvalue is not finite.
struct PolyArgs {
  int deg;
  double coef[9];
  double tau_max, tol;
};

__global__ void __launch_bounds__(256) k_cfl_max(PolyArgs pa, const double* eigs, long n, double* cfl) {
  __shared__ double red[4];
  __shared__ int bad_s;
  const int tid = threadIdx.x;
  if (tid == 0) bad_s = 0;
  __syncthreads();
  int bad = 0;
  for (long i = tid; i < n; i += 256)
    if (!isfinite(eigs[2 * i]) || !isfinite(eigs[2 * i + 1])) bad = 1;
  if (bad) atomicOr(&bad_s, 1);
  __syncthreads();
  if (bad_s) {
    if (tid == 0) *cfl = NAN;
    return;
  }
  double lo = 0.0, hi = pa.tau_max;
  const double lim = (1.0 + pa.tol) * (1.0 + pa.tol);
  for (int it = 0; it < 60; ++it) {
    const double mid = 0.5 * (lo + hi);
    double mx = 0.0;
    for (long i = tid; i < n; i += 256) {
      const double zr = mid * eigs[2 * i], zi = mid * eigs[2 * i + 1];
      double pr = pa.coef[pa.deg], pi = 0.0;        // Horner
      for (int j = pa.deg - 1; j >= 0; --j) {
        const double t = pr * zr - pi * zi + pa.coef[j];
        pi = pr * zi + pi * zr;
        pr = t;
      }
      mx = fmax(mx, pr * pr + pi * pi);
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) mx = fmax(mx, __shfl_xor(mx, m, 64));
    if ((tid & 63) == 0) red[tid >> 6] = mx;
    __syncthreads();
    mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    __syncthreads();
    if (mx <= lim) lo = mid;
    else hi = mid;
  }
  if (tid == 0) *cfl = lo;
}

extern "C" {

fr_status fr_fourier_eigs(fr_ctx* c, const void* blocks, int64_t elem, const double* kappa, int64_t nk, double scale,
                          double* eigs) {
  if (!c) return FR_E_INVALID;
  if (!blocks || !kappa || !eigs || nk < 0 || elem < 0 || elem >= c->ne) {
    c->err = "fr_fourier_eigs: null pointer or element / count out of range";
    return FR_E_INVALID;
  }
  if (c->type == FR_TRI || c->mixed) {
    c->err = "fr_fourier_eigs: meshes with triangles are not translation-invariant element by element";
    return FR_E_UNSUPPORTED;
  }
  if (c->b > kFB) {
    c->err = "fr_fourier_eigs: blocks up to 64 x 64";
    return FR_E_UNSUPPORTED;
  }
  if (nk == 0) return FR_OK;
  FourierArgs a{};
  a.b = c->b;
  a.nblk = 1 + c->nface;
  a.nd = c->nd;
  a.scale = scale;
  const long bb = (long)c->b * c->b;
  for (int k = 0; k < a.nblk; ++k) {
    a.blk_off[k] = ((long)elem * a.nblk + k) * bb;
    for (int d = 0; d < 3; ++d)
      a.d[k][d] = (k == 0 || d >= c->nd) ? 0.0 : 2.0 * c->face_off[((size_t)elem * c->nface + (k - 1)) * c->nd + d];
  }
  if (c->prec == FR_F64)
    hipLaunchKernelGGL(k_fourier_eigs<double>, dim3((unsigned)nk), dim3(64), 0, c->stream, a, (const double*)blocks,
                       kappa, (long)nk, eigs);
  else
    hipLaunchKernelGGL(k_fourier_eigs<float>, dim3((unsigned)nk), dim3(64), 0, c->stream, a, (const float*)blocks,
                       kappa, (long)nk, eigs);
  if (hipGetLastError() != hipSuccess) { c->err = "k_fourier_eigs launch"; return FR_E_DEVICE; }
  return FR_OK;
}

fr_status fr_cfl_max(fr_ctx* c, const double* eigs, int64_t n, const double* coef, int degree, double tau_max,
                     double tol, double* cfl) {
  if (!c) return FR_E_INVALID;
  if (!eigs || !coef || !cfl || n <= 0 || degree < 1 || degree > 8 || !(tau_max > 0.0) || !(tol >= 0.0)) {
    c->err = "fr_cfl_max: null pointer, n <= 0, degree outside 1..8, tau_max <= 0 or tol < 0";
    return FR_E_INVALID;
  }
  PolyArgs pa{};
  pa.deg = degree;
  for (int j = 0; j <= degree; ++j) pa.coef[j] = coef[j];
  pa.tau_max = tau_max;
  pa.tol = tol;
  hipLaunchKernelGGL(k_cfl_max, dim3(1), dim3(256), 0, c->stream, pa, eigs, (long)n, cfl);
  if (hipGetLastError() != hipSuccess) { c->err = "k_cfl_max launch"; return FR_E_DEVICE; }
  return FR_OK;
}

}  // extern "C"
