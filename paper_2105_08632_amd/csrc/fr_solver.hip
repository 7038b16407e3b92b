// Block-Jacobi preconditioner, Krylov vector kernels and the backward-Euler
// Newton-GMRES step.
//
// The preconditioner inverts the diagonal Jacobian blocks A_n = shift I +
// scale dR_n/dU_n in FP64: blocks up to 128 by Gauss-Jordan elimination with
// partial pivoting (one workgroup per element, the block resident in LDS),
// applied as explicit inverses in a batched matrix-vector product; larger
// blocks by a blocked LU factorization in global memory, applied by
// substitution.  The Newton step
// solves U - U^n - dt R(U) = 0 with restarted, right-preconditioned GMRES
// (classical Gram-Schmidt applied twice, Givens rotations on the host),
// Jacobian-vector products from the exact tangent kernels, and the true
// linear residual recomputed at every restart.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "fr.h"
#include "fr_ctx.hpp"
#include "fr_solver.hpp"

// ------------------------------------------------------------ LU / inverse
constexpr int kInvThreads = 256;

// A = shift I + scale J (J column-major b x b, input type IT), inverted in
// place by Gauss-Jordan elimination with row pivoting; the inverse (column-
// major) is written to Ainv.  bad[n] = 1 when a pivot is zero or not finite.
template <class IT, int BMAX>
__global__ void __launch_bounds__(kInvThreads) k_block_inverse(const IT* J, long jstride, int b, double shift,
                                                               double scale, double* Ainv, int* bad, const int* list) {
  __shared__ double A[BMAX * BMAX];   // row-major in LDS: A[r*b + c]
  __shared__ int perm[BMAX];
  __shared__ double red_v[kInvThreads];
  __shared__ int red_i[kInvThreads];
  __shared__ int s_bad;
  const int n = list ? list[blockIdx.x] : (int)blockIdx.x, tid = threadIdx.x;
  const IT* Jn = J + (long)n * jstride;
  for (int i = tid; i < b * b; i += kInvThreads) {
    int c = i / b, r = i % b;                       // source is column-major
    double v = scale * (double)Jn[i];
    if (r == c) v += shift;
    A[r * b + c] = v;
  }
  if (tid == 0) s_bad = 0;
  __syncthreads();
  for (int k = 0; k < b; ++k) {
    // pivot: largest |A[i][k]|, i >= k
    double best = -1.0;
    int bi = k;
    for (int i = k + tid; i < b; i += kInvThreads) {
      double v = fabs(A[i * b + k]);
      if (v > best) { best = v; bi = i; }
    }
    red_v[tid] = best; red_i[tid] = bi;
    __syncthreads();
    for (int s = kInvThreads / 2; s > 0; s >>= 1) {
      if (tid < s) {
        double o = red_v[tid + s];
        int oi = red_i[tid + s];
        if (o > red_v[tid] || (o == red_v[tid] && oi < red_i[tid])) { red_v[tid] = o; red_i[tid] = oi; }
      }
      __syncthreads();
    }
    const int p = red_i[0];
    if (tid == 0) {
      perm[k] = p;
      double pv = A[p * b + k];
      if (!(fabs(pv) > 0.0) || !isfinite(pv)) s_bad = 1;
    }
    __syncthreads();
    if (p != k)
      for (int c = tid; c < b; c += kInvThreads) {
        double t = A[k * b + c]; A[k * b + c] = A[p * b + c]; A[p * b + c] = t;
      }
    __syncthreads();
    const double piv = A[k * b + k];
    const double ip = (s_bad || piv == 0.0) ? 0.0 : 1.0 / piv;
    __syncthreads();
    // row k <- row k / pivot, with A[k][k] replaced by 1 before scaling
    for (int c = tid; c < b; c += kInvThreads) A[k * b + c] = (c == k ? 1.0 : A[k * b + c]) * ip;
    __syncthreads();
    // eliminate column k from every other row
    for (int i = tid; i < b * b; i += kInvThreads) {
      int r = i / b, c = i % b;
      if (r == k) continue;
      double f = A[r * b + k];
      if (c == k) continue;
      A[r * b + c] -= f * A[k * b + c];
    }
    __syncthreads();
    for (int r = tid; r < b; r += kInvThreads)
      if (r != k) A[r * b + k] = -A[r * b + k] * A[k * b + k];
    __syncthreads();
  }
  // undo the row interchanges as column interchanges, last first
  for (int k = b - 1; k >= 0; --k) {
    int p = perm[k];
    if (p != k)
      for (int r = tid; r < b; r += kInvThreads) {
        double t = A[r * b + k]; A[r * b + k] = A[r * b + p]; A[r * b + p] = t;
      }
    __syncthreads();
  }
  double* out = Ainv + (long)n * b * b;
  for (int i = tid; i < b * b; i += kInvThreads) {
    int c = i / b, r = i % b;
    out[i] = A[r * b + c];                           // column-major
  }
  if (tid == 0) bad[n] = s_bad;
}

// Wave-uniform lane l's value of v.
__device__ __forceinline__ double fr_readlane(double v, int l) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)u, l), hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Lane l's value of x[s] for wave-uniform s and l: every slot is read with
// readlane and the slot chosen among the scalars (selecting the register
// first would turn into an indexed access to scratch memory).
template <int N>
__device__ __forceinline__ double fr_lane_slot(const double (&x)[N], int s, int l) {
  double v = fr_readlane(x[0], l);
#pragma unroll
  for (int i = 1; i < N; ++i) {
    const double o = fr_readlane(x[i], l);
    v = s == i ? o : v;
  }
  return v;
}

template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned long long fr_max_dpp(unsigned long long v) {
  const int lo = (int)(unsigned)v, hi = (int)(unsigned)(v >> 32);
  const unsigned lo2 = (unsigned)__builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWS, 0xF, false);
  const unsigned hi2 = (unsigned)__builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWS, 0xF, false);
  const unsigned long long o = ((unsigned long long)hi2 << 32) | lo2;
  return o > v ? o : v;
}

// Maximum over the wavefront by DPP: quad swaps, half-row and row mirrors
// (every row of 16 lanes then holds its maximum), then the row broadcasts
// 15 and 31 (lane 63 ends with the maximum of all four rows).
__device__ __forceinline__ unsigned long long fr_wave_max_u64(unsigned long long v) {
  v = fr_max_dpp<0xB1, 0xF>(v);
  v = fr_max_dpp<0x4E, 0xF>(v);
  v = fr_max_dpp<0x141, 0xF>(v);
  v = fr_max_dpp<0x140, 0xF>(v);
  v = fr_max_dpp<0x142, 0xA>(v);
  v = fr_max_dpp<0x143, 0xC>(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, 63);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), 63);
  return ((unsigned long long)hi << 32) | lo;
}

// Blocks up to 64 x 64: one wavefront per element, row r of A_n held in the
// registers of lane r.  Gauss-Jordan exchange steps without row
// interchanges: step k takes as pivot the unused row p_k with the largest
// |A[r][k]| (ties: the lowest row), scales it by 1/pivot and eliminates
// column k from every other row; the final tableau T then holds the inverse
// with permuted rows and columns, inv[k][p_j] = T[p_k][j].  After each step
// every row moves one register down (the new column k goes to the last
// register), so the pivot column always sits in register 0 and every
// register index is a compile-time constant; after b steps register i holds
// column (i + b) mod 64.  The normalised pivot row reaches the other lanes
// through LDS.  Rows b..63 are identity rows that are never pivots.
template <class IT>
__global__ void __launch_bounds__(256) k_block_inverse_w64(const IT* J, long jstride, int b, double shift,
                                                          double scale, double* Ainv, int* bad, const int* list,
                                                          long count) {
  __shared__ double prow_s[4][64];
  __shared__ int perm_s[4][64];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long item = (long)blockIdx.x * 4 + w;
  if (item >= count) return;                  // per-wave work, no workgroup barriers
  const long n = list ? (long)list[item] : item;
  const IT* Jn = J + n * jstride;
  double* prow = prow_s[w];
  double a[64];
#pragma unroll
  for (int c = 0; c < 64; ++c) {
    double v = (lane == c) ? 1.0 : 0.0;
    if (lane < b && c < b) v = scale * (double)Jn[(long)c * b + lane] + (lane == c ? shift : 0.0);
    a[c] = v;
  }
  bool used = lane >= b;
  int kstep = 0, sbad = 0;
  for (int k = 0; k < b; ++k) {
    const double a0 = a[0];
    const double av = fabs(a0);
    // pivot search as one DPP maximum over 64-bit keys, 63 - row in the
    // lowest 6 bits (ties go to the lowest row): rows already used 0,
    // not-a-number rows 0x40 | .. (below zero rows), others the bits of
    // |value| above the lowest 8 (ties to 2^-44 relative) | 0x80 | ..
    const unsigned long long lo6 = (unsigned long long)(63 - lane);
    const unsigned long long key =
        used ? 0ull
             : (av == av ? ((unsigned long long)__double_as_longlong(av) & ~0xFFull) | 0x80ull | lo6 : 0x40ull | lo6);
    const unsigned long long kmax = fr_wave_max_u64(key);
    const int p = 63 - (int)(kmax & 0x3Full);
    const double pv = fr_readlane(a0, p);
    const bool ok = kmax >= 0x80ull && fabs(pv) > 0.0 && isfinite(pv);
    sbad |= !ok;
    // 1 / pv: hardware reciprocal and two Newton steps
    double ip = __builtin_amdgcn_rcp(pv);
    ip = fma(ip, fma(-pv, ip, 1.0), ip);
    ip = fma(ip, fma(-pv, ip, 1.0), ip);
    ip = ok ? ip : 0.0;
    const bool is_p = lane == p;
    if (is_p) {
#pragma unroll
      for (int i = 0; i < 63; ++i) prow[i] = a[i + 1] * ip;
      used = true;
      kstep = k;
    }
    if (lane == 0) perm_s[w][k] = p;
    __builtin_amdgcn_wave_barrier();
    // pivot row: T'[p][.] = T[p][.] / pivot, T'[p][k] = 1 / pivot;
    // other rows: T'[r][.] = T[r][.] - T[r][k] T'[p][.], T'[r][k] = -T[r][k] / pivot
    const double f = is_p ? -1.0 : a0;
    const double keep = is_p ? 0.0 : 1.0;
#pragma unroll
    for (int i = 0; i < 63; ++i) a[i] = fma(-f, prow[i], a[i + 1] * keep);
    a[63] = is_p ? ip : -a0 * ip;
    __builtin_amdgcn_wave_barrier();
  }
  if (lane < b) {
    double* out = Ainv + n * (long)b * b;
#pragma unroll
    for (int i = 0; i < 64; ++i) {
      const int j = (i + b) & 63;
      if (j < b) out[(long)perm_s[w][j] * b + kstep] = a[i];
    }
  }
  if (lane == 0) bad[n] = sbad;
}

// z_n = Ainv_n r_n, one wavefront per element, lanes over rows, columns
// streamed (column-major inverse: each column is a contiguous run).
template <class VT>
__global__ void __launch_bounds__(256) k_block_apply(long ne, int b, const double* Ainv, const VT* r, VT* z) {
  const int lane = threadIdx.x & 63;
  const long n = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (n >= ne) return;
  block_matvec<double, VT>(b, Ainv + n * b * b, r + n * b, 1.0, z + n * b, lane);
}

// ------------------------------------------------------------ vector kernels
// out = a x + b y
__global__ void k_axpby(long n, double a, const double* x, double b, const double* y, double* out) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    out[i] = a * x[i] + (y ? b * y[i] : 0.0);
}

constexpr int kDotBlocks = 1024;
constexpr int kAugMax = 3;          // stored corrections of loose GMRES
constexpr int kDotThreads = 256;

// partial[blk][j] = sum over the block's slice of V_j . w, j < k (V_j = V + j*ld)
__global__ void __launch_bounds__(kDotThreads) k_multi_dot(long n, int k, const double* V, long ld, const double* w,
                                                           double* partial) {
  __shared__ double red[kDotThreads];
  for (int j = 0; j < k; ++j) {
    double acc = 0.0;
    const double* Vj = V + (long)j * ld;
    for (long i = (long)blockIdx.x * kDotThreads + threadIdx.x; i < n; i += (long)gridDim.x * kDotThreads)
      acc += Vj[i] * w[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kDotThreads / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[(long)blockIdx.x * 32 + j] = red[0];
    __syncthreads();
  }
}

// out[j] = sum over blocks of partial[blk][j]
__global__ void k_reduce_partials(int k, int nblk, const double* partial, double* out) {
  __shared__ double red[256];
  for (int j = 0; j < k; ++j) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) acc += partial[(long)b * 32 + j];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = red[0];
    __syncthreads();
  }
}

// ---- Arnoldi orthogonalisation: classical Gram-Schmidt with selective
// re-orthogonalisation, in up to three sweeps over the basis V_0 .. V_{K-1}:
//   0: partial sums of V^T w and of w.w
//   1: h1 = the sum of sweep 0's partials; w <- w - V h1, then partial sums of
//      V^T w and w.w (each entry projected right after its update, so the
//      basis is read once for both)
//   2: the second pass, run only where the first one cancelled: one pass
//      leaves the new vector orthogonal to the basis up to about
//      eps |w| / |w - V h1|, so with |w - V h1| >= |w| / 8 (the test of
//      Daniel, Gragg, Kaufman and Stewart, with a looser bound) the sweep
//      ends at once with h2 = 0 and the norm of sweep 1; otherwise h2 likewise,
//      w <- w - V h2, partial sums of w.w.
// Each workgroup of a sweep adds the previous sweep's per-workgroup partials
// itself, in a fixed order (stream order guarantees they are complete), so
// the results, and the decision to re-orthogonalise, are the same in every
// workgroup, need no separate reduction launch and stay on the device
// (graph-capturable).  Workgroup 0 stores h1 / h2.
constexpr int kOrthBlocks = 512, kOrthThreads = 512, kMaxK = 32;
constexpr double kReorthRatio2 = 1.0 / 64.0;   // (1/8)^2: re-orthogonalise when |w - V h1|^2 < |w|^2 / 64

// out[q] = sum over workgroups b < nblk of p[b][q], q < nq; every thread of
// the workgroup gets the sums (through red, [waves][kMaxK] plus [kMaxK]).
// NQ (>= nq) bounds the unrolled loads: all of a thread's loads are issued
// before the first reduction.
template <int NQ = kMaxK>
__device__ __forceinline__ void orth_sum_partials(const double* p, int nblk, int nq, double (*red)[kMaxK],
                                                  double* sums) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double v[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) v[q] = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kOrthThreads) {
    const double* pb = p + (long)b * kMaxK;
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      if (q < nq) v[q] += pb[q];
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    if (q < nq) {
      double x = v[q];
      for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
      if (lane == 0) red[wave][q] = x;
    }
  }
  __syncthreads();
  if (threadIdx.x < nq) {
    double x = 0.0;
    for (int wv = 0; wv < kOrthThreads / 64; ++wv) x += red[wv][threadIdx.x];
    sums[threadIdx.x] = x;
  }
  __syncthreads();
}

// K = the basis size, a template argument: the K loads of an entry are issued
// back to back without guards.
// pw (sweep 2): sweep 0's partials, whose slot K holds w.w before the first
// projection.  The first sweep of a large basis is given the register budget
// of four waves per SIMD: under the default occupancy target the compiler
// keeps only part of an entry's K loads in flight (K = 24: 205 -> 139 us on
// 4.2 M entries).
template <int MODE, int K> constexpr int orth_waves() { return MODE == 0 && K >= 20 ? 4 : 0; }
template <int MODE, int K>
__global__ void __launch_bounds__(kOrthThreads)
__attribute__((amdgpu_waves_per_eu(orth_waves<MODE, K>() ? orth_waves<MODE, K>() : 1,
                                   orth_waves<MODE, K>() ? orth_waves<MODE, K>() : 8)))
k_orth(long n, const double* V, long ld, double* w, const double* pin, const double* pw, double* pout, double* hout) {
  static_assert(K >= 1 && K < kMaxK, "basis size (slot K of the partials holds w.w)");
  __shared__ double red[kOrthThreads / 64][kMaxK];
  __shared__ double hs[kMaxK];
  __shared__ double nw[2];
  constexpr int NA = MODE == 2 ? 1 : K + 1;
  double acc[NA];
  if constexpr (MODE == 1) {
    orth_sum_partials<K>(pin, gridDim.x, K, red, hs);
    if (blockIdx.x == 0 && threadIdx.x < K) hout[threadIdx.x] = hs[threadIdx.x];
  } else if constexpr (MODE == 2) {
    // the two norms first: the K coefficients are summed only for a second pass
    orth_sum_partials<1>(pin + K, gridDim.x, 1, red, nw);       // |w - V h1|^2
    orth_sum_partials<1>(pw + K, gridDim.x, 1, red, nw + 1);    // |w|^2
    const bool once = nw[0] >= kReorthRatio2 * nw[1];
    if (once) {
      if (blockIdx.x == 0 && threadIdx.x < K) hout[threadIdx.x] = 0.0;
      if (threadIdx.x == 0) pout[(long)blockIdx.x * kMaxK] = blockIdx.x == 0 ? nw[0] : 0.0;
      return;
    }
    orth_sum_partials<K>(pin, gridDim.x, K, red, hs);           // h2
    if (blockIdx.x == 0 && threadIdx.x < K) hout[threadIdx.x] = hs[threadIdx.x];
  }
#pragma unroll
  for (int q = 0; q < NA; ++q) acc[q] = 0.0;
  for (long i = (long)blockIdx.x * kOrthThreads + threadIdx.x; i < n; i += (long)gridDim.x * kOrthThreads) {
    double vv[K];
    const double* Vi = V + i;
    // the basis is streamed (it does not fit the caches between sweeps)
#pragma unroll
    for (int q = 0; q < K; ++q) vv[q] = __builtin_nontemporal_load(Vi + (long)q * ld);
    double wi = w[i];
    if constexpr (MODE >= 1) {
      // the coefficients are read from LDS (broadcast) in every iteration
      // (an opaque offset keeps the loads in the loop) rather than held in
      // registers: K of them would cost 2 K registers and occupancy
      int ho = 0;
      asm volatile("" : "+v"(ho));
#pragma unroll
      for (int q = 0; q < K; ++q) wi -= hs[q + ho] * vv[q];
      w[i] = wi;
    }
    if constexpr (MODE <= 1) {
#pragma unroll
      for (int q = 0; q < K; ++q) acc[q] += vv[q] * wi;
      acc[K] += wi * wi;
    } else {
      acc[0] += wi * wi;
    }
  }
  __syncthreads();                    // red is reused
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NA; ++q) {
    double v = acc[q];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[wave][q] = v;
  }
  __syncthreads();
  if (threadIdx.x < NA) {
    double v = 0.0;
    for (int wv = 0; wv < kOrthThreads / 64; ++wv) v += red[wv][threadIdx.x];
    pout[(long)blockIdx.x * kMaxK + threadIdx.x] = v;
  }
}

template <int MODE, int K>
static void launch_orth_k(hipStream_t st, int k, long n, const double* V, long ld, double* w, const double* pin,
                          const double* pw, double* pout, double* hout) {
  if constexpr (K < kMaxK) {
    if (k == K)
      hipLaunchKernelGGL((k_orth<MODE, K>), dim3(kOrthBlocks), dim3(kOrthThreads), 0, st, n, V, ld, w, pin, pw, pout,
                         hout);
    else
      launch_orth_k<MODE, K + 1>(st, k, n, V, ld, w, pin, pw, pout, hout);
  }
}
template <int MODE>
static void launch_orth(hipStream_t st, int k, long n, const double* V, long ld, double* w, const double* pin,
                        const double* pw, double* pout, double* hout) {
  launch_orth_k<MODE, 1>(st, k, n, V, ld, w, pin, pw, pout, hout);
}

// The end of an Arnoldi step (graph-capturable: every scalar stays on the
// device): |w| from the last sweep's partials and v_{j+1} = w / |w| (0 on
// breakdown).  Workgroup 0 also completes the Hessenberg column, h[i] =
// h1[i] + h2[i] (i <= j), h[j+1] = |w| (dn = w.w), and rotates it: the
// previous Givens rotations, then the new one, which also rotates the
// right-hand side g (est[j] = |g[j+1]|, the residual estimate).  The column
// and the previous rotations are staged in LDS, so the one thread that
// applies the rotations in sequence waits on LDS, not on memory.
__global__ void __launch_bounds__(kOrthThreads) k_orth_finish(long n, int j, int m, const double* p2, int nblk,
                                                              const double* h1, const double* h2, const double* w,
                                                              double* v, double* H, double* dn, double* cs,
                                                              double* sn, double* g, double* est) {
  __shared__ double red[kOrthThreads / 64][kMaxK];
  __shared__ double nn[1];
  __shared__ double col[kMaxK + 1], rc[kMaxK], rs[kMaxK];
  orth_sum_partials<1>(p2, nblk, 1, red, nn);
  const double hn = sqrt(fmax(nn[0], 0.0));
  if (blockIdx.x == 0) {
    const int t = threadIdx.x;
    if (t <= j) col[t] = h1[t] + h2[t];
    if (t == j + 1) col[t] = hn;
    if (t < j) { rc[t] = cs[t]; rs[t] = sn[t]; }
    if (t == 0) *dn = nn[0];
    __syncthreads();
    if (t == 0) {
      for (int i = 0; i < j; ++i) {
        const double a = col[i], b = col[i + 1];
        col[i] = rc[i] * a + rs[i] * b;
        col[i + 1] = -rs[i] * a + rc[i] * b;
      }
      const double a = col[j], b = col[j + 1];
      const double r = hypot(a, b);
      const double c = r > 0.0 ? a / r : 1.0, sv = r > 0.0 ? b / r : 0.0;
      cs[j] = c;
      sn[j] = sv;
      col[j] = r;
      col[j + 1] = 0.0;
      const double gj = g[j];
      g[j + 1] = -sv * gj;
      g[j] = c * gj;
      est[j] = fabs(sv * gj);
    }
    __syncthreads();
    if (t <= j + 1) H[t * m + j] = col[t];
  }
  const double inv = hn > 0.0 ? 1.0 / hn : 0.0;
  for (long i = (long)blockIdx.x * kOrthThreads + threadIdx.x; i < n; i += (long)gridDim.x * kOrthThreads)
    v[i] = w[i] * inv;
}

__global__ void k_fill(long n, double v, double* x) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) x[i] = v;
}

// x += sum_j y[j] Z_j
__global__ void k_multi_axpy_add(long n, int k, const double* y, const double* Z, long ld, double* x) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    double acc = x[i];
    for (int j = 0; j < k; ++j) acc += y[j] * Z[(long)j * ld + i];
    x[i] = acc;
  }
}

// ------------------------------------------------------------ large blocks
// Blocks above 128 (hexahedra of degree 3: b = 320) do not fit one
// workgroup's LDS.  Blocked right-looking LU with partial pivoting, one
// 512-thread workgroup per element (two resident per CU, so that one
// block's chain of pivot steps overlaps another's trailing update), in
// 32-column panels:
//  1. the panel (every row, 32 columns) is held in registers: wave w owns
//     columns 4w .. 4w+3, lane l rows l + 64 s.  A pivot step is one
//     barrier: the wave owning the column picks the pivot (a DPP maximum of
//     |value| keyed with the row), forms the multipliers and publishes them
//     in LDS; every wave then updates its own columns, reading the pivot
//     row's values from its own registers (readlane);
//  2. rows never move in memory.  A chosen pivot row receives its rank (its
//     logical row index); the trailing columns keep physical row order, and
//     each panel is stored with its pivot rows at their ranks followed by
//     the rows still to pivot in increasing physical order, so that the
//     panel's multipliers below its first row are one contiguous range;
//  3. the trailing columns are updated in slabs of 32: every row not
//     pivoted before this panel (its pivot rows first, in pivot order) is
//     updated by 16-column chunks of the multipliers, each chunk's pivot
//     rows being finished first by the inverse of its 16 x 16 diagonal
//     block of L11 (the inverses formed once per panel).  So
//     U12 = L11^-1 A12 and A22 -= L21 U12 are one pass of 5 x 4 register
//     tiles, with no long sequential solve.
// The first panel reads A = shift I + scale J straight from J (no separate
// conversion pass).  The substitution recovers each panel's row positions
// from the ranks.
constexpr int kLuThreads = 512, kLuNB = 32, kLuMaxB = 320, kLuQM = (kLuMaxB + 63) / 64;
constexpr int kLuFree = 1 << 20;          // rank of a row not yet chosen as pivot
constexpr int kLuSlab = 32;               // trailing columns per slab
static_assert(kLuNB == 4 * (kLuThreads / 64) && kLuSlab == 4 * (kLuThreads / 64), "four columns per wavefront");
static_assert(kLuThreads == 16 * kLuSlab && kLuNB % 16 == 0, "chunk product: one thread per (row, column)");

// A = shift I + scale J (column-major, input type IT) factorized with partial
// pivoting.  perm[i] = the row (of A) chosen as pivot at step i.  Storage
// (column-major LU): column c of panel P (columns K .. K+w-1) holds at
// position i < K+w the entry of row perm[i] (U above the diagonal, the unit
// lower L's multipliers below it, the diagonal of U on it), and at position
// K+w+m the multiplier of the m-th row, in increasing row order, among those
// not pivoted by the end of panel P.  bad[n] = 1 when a pivot is zero or not
// finite.
template <class IT>
__global__ void __launch_bounds__(kLuThreads) __attribute__((amdgpu_waves_per_eu(4)))
k_block_lu(const IT* J, long jstride, int b, double shift, double scale,
                                                         double* LU, int* perm, int* bad, const int* list) {
  __shared__ int s_rank[kLuMaxB];
  __shared__ int s_perm[kLuMaxB];
  __shared__ int s_act[kLuMaxB];                  // rows still to pivot, increasing
  __shared__ int s_apos[kLuMaxB];                 // a row's position in s_act
  __shared__ double s_l[2][kLuQM * 64];           // multipliers of a pivot step (double-buffered)
  __shared__ int s_p[2];
  __shared__ int s_bad;
  __shared__ double s_ls[16][kLuMaxB];            // a chunk of multipliers, rows in stored order
  __shared__ double s_us[16][kLuSlab];            // a chunk's pivot rows over the slab, as updated so far
  __shared__ double s_uf[16][kLuSlab];            // the same rows finished (U)
  __shared__ double s_li[kLuNB / 16][16][16];     // inverses of L11's 16 x 16 diagonal blocks
  const int n = list ? list[blockIdx.x] : (int)blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const IT* Jn = J + (long)n * jstride;
  double* A = LU + (long)n * b * b;
  for (int i = tid; i < kLuMaxB; i += kLuThreads) s_rank[i] = kLuFree;
  if (tid == 0) s_bad = 0;
  __syncthreads();
  for (int K = 0; K < b; K += kLuNB) {
    const bool first = K == 0;                    // read A from J
    auto src = [&](int r, int c) -> double {
      return first ? scale * (double)Jn[(long)c * b + r] + (r == c ? shift : 0.0) : A[(long)c * b + r];
    };
    const int w = min(kLuNB, b - K);
    // ---- 1. the panel in registers
    double pa[kLuQM][4];
    unsigned act = 0;                             // bit s: row lane + 64 s not pivoted yet
#pragma unroll
    for (int s = 0; s < kLuQM; ++s) {
      const int r = lane + 64 * s;
      if (r < b && s_rank[r] == kLuFree) act |= 1u << s;
#pragma unroll
      for (int c = 0; c < 4; ++c) pa[s][c] = (r < b && 4 * wv + c < w) ? src(r, K + 4 * wv + c) : 0.0;
    }
    for (int j4 = 0; j4 < w; j4 += 4)
#pragma unroll
    for (int cj = 0; cj < 4; ++cj) {
      const int j = j4 + cj;                      // the column within the panel (cj: within its wave)
      if (j >= w) break;
      const int buf = j & 1;
      if (wv == (j >> 2)) {
        double colv[kLuQM];
#pragma unroll
        for (int s = 0; s < kLuQM; ++s) colv[s] = pa[s][cj];
        // pivot: the largest |value| among rows not pivoted; the key is the
        // bit pattern of |value| (ordered like the value) with its lowest 9
        // bits replaced by 511 - row (ties, to 2^-43 relative: the lowest
        // row); not-a-number ranks first and is flagged below
        unsigned long long key = 0;
#pragma unroll
        for (int s = 0; s < kLuQM; ++s)
          if (act >> s & 1) {
            const unsigned long long k = ((unsigned long long)__double_as_longlong(fabs(colv[s])) & ~0x1FFull) |
                                         (unsigned long long)(511 - (lane + 64 * s));
            key = k > key ? k : key;
          }
        key = fr_wave_max_u64(key);
        const int p = 511 - (int)(key & 0x1FFull);
        const double pv = fr_lane_slot(colv, p >> 6, p & 63);
        const bool ok = fabs(pv) > 0.0 && isfinite(pv);
        // 1 / pv: hardware reciprocal and two Newton steps
        double ip = __builtin_amdgcn_rcp(pv);
        ip = fma(ip, fma(-pv, ip, 1.0), ip);
        ip = fma(ip, fma(-pv, ip, 1.0), ip);
        ip = ok ? ip : 0.0;
#pragma unroll
        for (int s = 0; s < kLuQM; ++s) {
          const int r = lane + 64 * s;
          double l = 0.0;
          if ((act >> s & 1) && r != p) {
            l = colv[s] * ip;
            pa[s][cj] = l;
          }
          s_l[buf][r] = l;
        }
        if (lane == 0) {
          s_p[buf] = p;
          if (!ok) s_bad = 1;
        }
      }
      __syncthreads();
      const int p = __builtin_amdgcn_readfirstlane(s_p[buf]);
      if (tid == 0) {
        s_perm[K + j] = p;
        s_rank[p] = K + j;
      }
      if ((p & 63) == lane) act &= ~(1u << (p >> 6));
      if (4 * wv + 3 > j) {
        double u[4], l[kLuQM];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          double col[kLuQM];
#pragma unroll
          for (int s = 0; s < kLuQM; ++s) col[s] = pa[s][c];
          u[c] = fr_lane_slot(col, p >> 6, p & 63);
        }
#pragma unroll
        for (int s = 0; s < kLuQM; ++s) l[s] = s_l[buf][lane + 64 * s];
#pragma unroll
        for (int c = 0; c < 4; ++c)
          if (4 * wv + c > j)
#pragma unroll
            for (int s = 0; s < kLuQM; ++s) pa[s][c] -= l[s] * u[c];
      }
    }
    __syncthreads();                              // the panel's ranks are complete
    if (wv == 0) {
      // rows still to pivot, in increasing order
      int base = 0;
#pragma unroll
      for (int s = 0; s < kLuQM; ++s) {
        const int r = lane + 64 * s;
        const bool f = r < b && s_rank[r] == kLuFree;
        const unsigned long long m = __ballot(f);
        const int pos = base + __popcll(m & ((1ull << lane) - 1ull));
        if (f) {
          s_act[pos] = r;
          s_apos[r] = pos;
        }
        base += __popcll(m);
      }
    }
    __syncthreads();
    const int na = b - K - w;                     // rows still to pivot = trailing columns
#pragma unroll
    for (int s = 0; s < kLuQM; ++s) {
      const int r = lane + 64 * s;
      if (r < b) {
        const int rk = s_rank[r];
        const int pos = rk != kLuFree ? rk : K + w + s_apos[r];
#pragma unroll
        for (int c = 0; c < 4; ++c)
          if (4 * wv + c < w) A[(long)(K + 4 * wv + c) * b + pos] = pa[s][c];
      }
    }
    if (na == 0) break;
    // ---- 3. the trailing columns, slab by slab: rows in stored order (the
    // panel's pivot rows, then the rows still to pivot), 5 x 4 tiles: lane
    // rows rg + 64 a, wave columns 4 wv .. 4 wv + 3 of the slab
    const int nr = w + na;                        // rows updated (w = 64 here)
    const int rg = lane;
    __syncthreads();                              // the stored panel is read below
    if (tid < kLuNB) {
      // inverse of diagonal block tid / 16 of the unit-lower L11, column
      // tid % 16, by forward substitution
      const int d = tid >> 4, c = tid & 15;
      double x[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) x[i] = i == c ? 1.0 : 0.0;
#pragma unroll
      for (int q = 0; q < 15; ++q) {
        // the column's address is made opaque and tied to x[q], so its loads
        // wait for x[q] instead of all 120 being hoisted into registers
        const double xq = x[q];
        long co = (long)(K + 16 * d + q) * b + K + 16 * d;
        asm volatile("" : "+v"(co) : "v"(xq));
#pragma unroll
        for (int i = q + 1; i < 16; ++i) x[i] -= A[co + i] * xq;
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) s_li[d][i][c] = x[i];
    }
    for (int c0 = K + w; c0 < b; c0 += kLuSlab) {
      __syncthreads();                            // the stored panel / the previous slab
      int phys[kLuQM];
#pragma unroll
      for (int a = 0; a < kLuQM; ++a) {
        const int i = rg + 64 * a;
        phys[a] = i < w ? s_perm[K + i] : (i < nr ? s_act[i - w] : -1);
      }
      double acc[kLuQM][4];
#pragma unroll
      for (int a = 0; a < kLuQM; ++a)
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
          const int col = c0 + 4 * wv + cc;
          acc[a][cc] = (phys[a] >= 0 && col < b) ? src(phys[a], col) : 0.0;
        }
      for (int q0 = 0; q0 < w; q0 += 16) {
        // multipliers of columns K+q0 .. K+q0+15 for the rows after this
        // chunk's pivot rows (zero for the pivot rows up to the chunk's
        // last: the chunk's own are solved below, the earlier ones are done)
        for (int e = tid; e < 16 * kLuMaxB; e += kLuThreads) {
          const int q = e / kLuMaxB, i = e % kLuMaxB;
          s_ls[q][i] = (i >= q0 + 16 && i < nr) ? A[(long)(K + q0 + q) * b + K + i] : 0.0;
        }
        if (rg >= q0 && rg < q0 + 16)
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) s_us[rg - q0][4 * wv + cc] = acc[0][cc];
        __syncthreads();
        {
          // the chunk's pivot rows finished: U = (diagonal block)^-1 x rows
          const int i = tid / kLuSlab, c = tid % kLuSlab;
          const double(*li)[16] = s_li[q0 >> 4];
          double v = 0.0;
#pragma unroll
          for (int q = 0; q < 16; ++q) v += li[i][q] * s_us[q][c];
          s_uf[i][c] = v;
        }
        __syncthreads();
        if (rg >= q0 && rg < q0 + 16)
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) acc[0][cc] = s_uf[rg - q0][4 * wv + cc];
#pragma unroll 4
        for (int q = 0; q < 16; ++q) {
          double l[kLuQM], u[4];
#pragma unroll
          for (int a = 0; a < kLuQM; ++a) l[a] = s_ls[q][rg + 64 * a];
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) u[cc] = s_uf[q][4 * wv + cc];
#pragma unroll
          for (int a = 0; a < kLuQM; ++a)
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) acc[a][cc] -= l[a] * u[cc];
        }
        __syncthreads();                          // s_ls / s_us / s_uf are rewritten next
      }
#pragma unroll
      for (int a = 0; a < kLuQM; ++a)
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
          const int col = c0 + 4 * wv + cc;
          if (phys[a] >= 0 && col < b) A[(long)col * b + phys[a]] = acc[a][cc];
        }
    }
    __syncthreads();
  }
  if (tid == 0) bad[n] = s_bad;
  for (int i = tid; i < b; i += kLuThreads) perm[(long)n * b + i] = s_perm[i];
}

// z_n = A_n^-1 r_n from the factors: one wavefront per element, the vector in
// registers in the rows' own order (lane l holds rows l + 64 s), each
// substitution step's value read from the lane holding the pivot row.  Rows
// still to pivot at the end of a panel sit after its pivot rows in
// increasing order (their positions from a ballot prefix count), so the
// forward sweep reads only positions below the diagonal and the backward
// sweep only those above.
template <class VT>
__global__ void __launch_bounds__(256) k_block_lu_apply(long ne, int b, const double* LU, const int* perm, const VT* r,
                                                        VT* z) {
  __shared__ int s_perm[4][kLuMaxB];
  __shared__ int s_rank[4][kLuMaxB];
  const int lane = threadIdx.x & 63, wl = threadIdx.x >> 6;
  const long n = (long)blockIdx.x * 4 + wl;
  if (n >= ne) return;
  const double* A = LU + n * b * b;
  int* sp = s_perm[wl];
  int* sr = s_rank[wl];
  for (int i = lane; i < b; i += 64) {
    const int p = perm[n * b + i];
    sp[i] = p;
    sr[p] = i;
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  const VT* rn = r + n * b;
  double y[kLuQM];
  int rk[kLuQM];
#pragma unroll
  for (int s = 0; s < kLuQM; ++s) {
    const int row = lane + 64 * s;
    y[s] = row < b ? (double)rn[row] : 0.0;
    rk[s] = row < b ? sr[row] : -1;
  }
  // forward: L y' = P r
  for (int K = 0; K < b; K += kLuNB) {
    const int w = min(kLuNB, b - K);
    int pos[kLuQM];
    int base = 0;
#pragma unroll
    for (int s = 0; s < kLuQM; ++s) {
      const bool f = rk[s] >= K + w;
      const unsigned long long m = __ballot(f);
      pos[s] = f ? K + w + base + __popcll(m & ((1ull << lane) - 1ull)) : rk[s];
      base += __popcll(m);
    }
    for (int j = K; j < K + w; ++j) {
      const int p = __builtin_amdgcn_readfirstlane(sp[j]);
      const double yj = fr_lane_slot(y, p >> 6, p & 63);
      const double* Lc = A + (long)j * b;
#pragma unroll
      for (int s = 0; s < kLuQM; ++s)
        if (rk[s] > j) y[s] -= Lc[pos[s]] * yj;
    }
  }
  // backward: U x = y'
  for (int j = b - 1; j >= 0; --j) {
    const int p = __builtin_amdgcn_readfirstlane(sp[j]);
    const double* Uc = A + (long)j * b;
    const double xj = fr_lane_slot(y, p >> 6, p & 63) / Uc[j];
#pragma unroll
    for (int s = 0; s < kLuQM; ++s) {
      if (s == (p >> 6) && lane == (p & 63)) y[s] = xj;
      if (rk[s] >= 0 && rk[s] < j) y[s] -= Uc[rk[s]] * xj;
    }
  }
#pragma unroll
  for (int s = 0; s < kLuQM; ++s)
    if (rk[s] >= 0) z[n * b + rk[s]] = (VT)y[s];
}

// ------------------------------------------------------------ helpers
static fr_status sfail(fr_ctx_s* c, fr_status s, const std::string& m) {
  c->err = m;
  return s;
}
#define HIPCHK(ctx, x)                                                              \
  do {                                                                              \
    hipError_t e_ = (x);                                                            \
    if (e_ != hipSuccess) return sfail((ctx), FR_E_DEVICE, std::string(#x ": ") + hipGetErrorString(e_)); \
  } while (0)

static int grid_for(long n, int threads) {
  long g = (n + threads - 1) / threads;
  return (int)(g > 4096 ? 4096 : (g < 1 ? 1 : g));
}

// Inverts A_n = shift I + scale J_n for the listed elements (all when list
// is null) from the diagonal blocks in pc->jbuf; flags land in pc->bad.
fr_status pc_invert(fr_precond_s* pc, double shift, double scale, const int* list, long count) {
  fr_ctx_s* c = pc->ctx;
  const int b = c->b;
  const long bb = (long)b * b;
  if (count <= 0) return FR_OK;
  const void* J = pc->jbuf;
  if (b <= 64) {
    const unsigned grid = (unsigned)((count + 3) / 4);
    if (c->prec == 0)
      hipLaunchKernelGGL((k_block_inverse_w64<double>), dim3(grid), dim3(256), 0, c->stream, (const double*)J, bb, b,
                         shift, scale, pc->inv, pc->bad, list, count);
    else
      hipLaunchKernelGGL((k_block_inverse_w64<float>), dim3(grid), dim3(256), 0, c->stream, (const float*)J, bb, b,
                         shift, scale, pc->inv, pc->bad, list, count);
  } else if (b <= 128) {
    if (c->prec == 0)
      hipLaunchKernelGGL((k_block_inverse<double, 128>), dim3(count), dim3(kInvThreads), 0, c->stream,
                         (const double*)J, bb, b, shift, scale, pc->inv, pc->bad, list);
    else
      hipLaunchKernelGGL((k_block_inverse<float, 128>), dim3(count), dim3(kInvThreads), 0, c->stream,
                         (const float*)J, bb, b, shift, scale, pc->inv, pc->bad, list);
  } else if (b <= kLuMaxB) {
    if (!pc->piv) return sfail(c, FR_E_INVALID, "preconditioner without pivot storage");
    if (c->prec == 0)
      hipLaunchKernelGGL((k_block_lu<double>), dim3(count), dim3(kLuThreads), 0, c->stream, (const double*)J, bb, b,
                         shift, scale, pc->inv, pc->piv, pc->bad, list);
    else
      hipLaunchKernelGGL((k_block_lu<float>), dim3(count), dim3(kLuThreads), 0, c->stream, (const float*)J, bb, b,
                         shift, scale, pc->inv, pc->piv, pc->bad, list);
  } else {
    return sfail(c, FR_E_UNSUPPORTED, "block-Jacobi preconditioner supports blocks up to 320 x 320");
  }
  HIPCHK(c, hipGetLastError());
  return FR_OK;
}

fr_status pc_lu_setup(fr_precond_s* pc, const void* U, double shift, double scale) {
  fr_ctx_s* c = pc->ctx;
  const long ne = c->ne;
  // diagonal blocks in the context precision, then FP64 inversion
  int rc = c->ks.jac(c, U, pc->jbuf, c->prec == 0 ? 0 : 1, 1);
  if (rc) return (fr_status)rc;
  fr_status st = pc_invert(pc, shift, scale, nullptr, ne);
  if (st) return st;
  HIPCHK(c, hipMemcpyAsync(pc->bad_host, pc->bad, ne * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (long n = 0; n < ne; ++n)
    if (pc->bad_host[n]) {
      c->err = "diagonal block of element " + std::to_string(n) + " is singular";
      return FR_E_SINGULAR;
    }
  return FR_OK;
}

fr_status pc_lu_apply(fr_precond_s* pc, const void* r, void* z) {
  fr_ctx_s* c = pc->ctx;
  const long ne = c->ne;
  const int grid = (int)((ne + 3) / 4);
  if (c->b > 128) {
    if (c->prec == 0)
      hipLaunchKernelGGL((k_block_lu_apply<double>), dim3(grid), dim3(256), 0, c->stream, ne, c->b, pc->inv, pc->piv,
                         (const double*)r, (double*)z);
    else
      hipLaunchKernelGGL((k_block_lu_apply<float>), dim3(grid), dim3(256), 0, c->stream, ne, c->b, pc->inv, pc->piv,
                         (const float*)r, (float*)z);
  } else if (c->prec == 0)
    hipLaunchKernelGGL((k_block_apply<double>), dim3(grid), dim3(256), 0, c->stream, ne, c->b, pc->inv,
                       (const double*)r, (double*)z);
  else
    hipLaunchKernelGGL((k_block_apply<float>), dim3(grid), dim3(256), 0, c->stream, ne, c->b, pc->inv,
                       (const float*)r, (float*)z);
  HIPCHK(c, hipGetLastError());
  return FR_OK;
}

// ------------------------------------------------------------ solver
struct fr_solver_s {
  fr_ctx_s* ctx = nullptr;
  int m = 30;
  long N = 0;
  void* mem = nullptr;
  double *V = nullptr, *Z = nullptr, *w = nullptr, *x = nullptr, *F = nullptr, *R = nullptr, *tmp = nullptr;
  double* Aug = nullptr;   // kAugMax + 1 stored cycle corrections (loose GMRES)
  int stall = 4;           // stagnation window in restart cycles
  double *partial = nullptr, *dots = nullptr, *hcol = nullptr;
  double* host = nullptr;   // pinned scalars
  hipEvent_t e0 = nullptr, e1 = nullptr;
  // captured restart cycle: Hessenberg state on the device, [H | cs | sn | g | est]
  double *dH = nullptr, *dcs = nullptr, *dsn = nullptr, *dg = nullptr, *dest = nullptr;
  double *dh1 = nullptr, *dh2 = nullptr, *dn = nullptr;
  double* hstate = nullptr;      // pinned copy of the state block
  hipStream_t cs = nullptr;      // the solver's own (capturable) stream
  hipEvent_t join0 = nullptr, join1 = nullptr;
  double* opart = nullptr;       // per-workgroup partial sums of the three Gram-Schmidt sweeps
  static constexpr int kChunk = 5, kMaxChunks = (31 + kChunk - 1) / kChunk;
  hipGraphExec_t chunk[kMaxChunks] = {};   // captured Arnoldi steps [c kChunk, (c+1) kChunk)
  hipGraphExec_t single[31] = {};          // captured Arnoldi step j
  const void* key_U = nullptr; const void* key_pc = nullptr; double key_dt = 0.0;
};

static fr_status dots(fr_solver_s* s, int k, const double* V, const double* w, double* out_host) {
  fr_ctx_s* c = s->ctx;
  hipLaunchKernelGGL(k_multi_dot, dim3(kDotBlocks), dim3(kDotThreads), 0, c->stream, s->N, k, V, s->N, w, s->partial);
  hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, c->stream, k, kDotBlocks, s->partial, s->dots);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(s->host, s->dots, k * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::memcpy(out_host, s->host, k * sizeof(double));
  return FR_OK;
}

static fr_status axpby(fr_solver_s* s, double a, const double* x, double b, const double* y, double* out) {
  hipLaunchKernelGGL(k_axpby, dim3(grid_for(s->N, 256)), dim3(256), 0, s->ctx->stream, s->N, a, x, b, y, out);
  HIPCHK(s->ctx, hipGetLastError());
  return FR_OK;
}

// out = A v = v - dt J(U) v (R(U) written to R_out when not null)
static fr_status apply_A(fr_solver_s* s, const double* U, double dt, const double* v, double* out, double* R_out) {
  fr_ctx_s* c = s->ctx;
  if (c->jv_fused) {   // the divergence pass writes v - dt J v itself
    c->jv_a = 1.0;
    c->jv_b = -dt;
    const int rc = c->ks.jvp(c, U, v, out, R_out);
    c->jv_a = 0.0;
    c->jv_b = 1.0;
    return (fr_status)rc;
  }
  int rc = c->ks.jvp(c, U, v, s->tmp, R_out);
  if (rc) return (fr_status)rc;
  return axpby(s, 1.0, v, -dt, s->tmp, out);
}

static fr_status precond(fr_solver_s* s, fr_precond_s* pc, const double* v, double* z) {
  if (!pc) {
    HIPCHK(s->ctx, hipMemcpyAsync(z, v, s->N * sizeof(double), hipMemcpyDeviceToDevice, s->ctx->stream));
    return FR_OK;
  }
  return fr_apply_precond(pc, v, z);
}

// One Arnoldi step j with every scalar on the device: z_j = M^-1 v_j (or,
// with zsrc, z_j = zscale zsrc), w = A z_j, two classical Gram-Schmidt
// passes, the Hessenberg column, v_{j+1} = w / |w| and the Givens rotation
// of column j (est[j] = the residual estimate).  Graph-capturable.
static fr_status arnoldi_step(fr_solver_s* s, fr_precond_s* pc, const double* U, double dt, int j, const double* zsrc,
                              double zscale) {
  fr_ctx_s* c = s->ctx;
  const int m = s->m;
  const long N = s->N;
  const int grid = grid_for(N, 256);
  double* vj = s->V + (long)j * N;
  double* zj = s->Z + (long)j * N;
  fr_status st = FR_OK;
  if (zsrc) hipLaunchKernelGGL(k_axpby, dim3(grid), dim3(256), 0, c->stream, N, zscale, zsrc, 0.0, nullptr, zj);
  else if (pc) st = fr_apply_precond(pc, vj, zj);
  else hipLaunchKernelGGL(k_axpby, dim3(grid), dim3(256), 0, c->stream, N, 1.0, vj, 0.0, nullptr, zj);
  if (st == FR_OK) st = apply_A(s, U, dt, zj, s->w, nullptr);
  if (st) return st;
  double* p0 = s->opart;
  double* p1 = p0 + kOrthBlocks * kMaxK;
  double* p2 = p1 + kOrthBlocks * kMaxK;
  launch_orth<0>(c->stream, j + 1, N, s->V, N, s->w, nullptr, nullptr, p0, nullptr);
  launch_orth<1>(c->stream, j + 1, N, s->V, N, s->w, p0, nullptr, p1, s->dh1);
  launch_orth<2>(c->stream, j + 1, N, s->V, N, s->w, p1, p0, p2, s->dh2);
  hipLaunchKernelGGL(k_orth_finish, dim3(kOrthBlocks), dim3(kOrthThreads), 0, c->stream, N, j, m, (const double*)p2,
                     kOrthBlocks, (const double*)s->dh1, (const double*)s->dh2, (const double*)s->w,
                     s->V + (long)(j + 1) * N, s->dH, s->dn, s->dcs, s->dsn, s->dg, s->dest);
  HIPCHK(c, hipGetLastError());
  return FR_OK;
}

// Reads the Hessenberg state after jj steps (H, g, est) and solves the
// triangular system; returns the number of steps that enter the update (the
// first whose estimate meets the tolerance, or the breakdown).
static fr_status cycle_solution(fr_solver_s* s, int jj, double tol, std::vector<double>& y, int* used) {
  fr_ctx_s* c = s->ctx;
  const int m = s->m;
  const size_t nstate = (size_t)(m + 1) * m + (m + 1) + m;    // H, g, est
  HIPCHK(c, hipMemcpyAsync(s->hstate, s->dH, nstate * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const double* H = s->hstate;
  const double* g = H + (size_t)(m + 1) * m;
  const double* est = g + (m + 1);
  int n = jj;
  for (int j = 0; j < jj; ++j) {
    if (H[j * m + j] == 0.0) { n = j; break; }          // breakdown: the Krylov space is exhausted
    if (est[j] <= tol) { n = j + 1; break; }
  }
  for (int i = n - 1; i >= 0; --i) {
    double acc = g[i];
    for (int k = i + 1; k < n; ++k) acc -= H[i * m + k] * y[k];
    y[i] = acc / H[i * m + i];
  }
  *used = n;
  return FR_OK;
}

// GMRES(m) on A x = rhs from x = 0; returns iterations, true residual norm.
// The Arnoldi steps run on the device (arnoldi_step); the host reads the
// residual estimate after each step to stop at the tolerance.
// With aug = k > 0 this is loose GMRES, LGMRES(m - k, k) (Baker, Jessup and
// Manteuffel, SIAM J. Matrix Anal. Appl. 26, 2005): the last k directions of
// every cycle are the corrections x_i - x_{i-1} of the k previous cycles,
// newest first, in place of preconditioned Arnoldi vectors.  The flexible
// form A Z = V H stays exact for any choice of Z's columns, so the cycle's
// minimisation and update are unchanged; the subspace is still m wide.
static fr_status gmres(fr_solver_s* s, fr_precond_s* pc, const double* U, double dt, const double* rhs, double rtol,
                       int maxit, int aug, double* x, int* iters, double* res_true, double* res0_out) {
  fr_ctx_s* c = s->ctx;
  const int m = s->m;
  const long N = s->N;
  std::vector<double> g0(m + 1, 0.0), y(m);
  aug = std::min(aug, m - 1);
  std::vector<int> order;              // slots of the stored corrections, newest first
  double aug_norm[kAugMax + 1] = {};
  int ring = 0;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(N, 256)), dim3(256), 0, c->stream, N, 0.0, x);
  // r0 = rhs (x = 0)
  HIPCHK(c, hipMemcpyAsync(s->w, rhs, N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  double nrm;
  fr_status st = dots(s, 1, s->w, s->w, &nrm);
  if (st) return st;
  const double b0 = std::sqrt(nrm);
  *res0_out = b0;
  *iters = 0;
  *res_true = 0.0;
  if (b0 == 0.0) { *res_true = 0.0; return FR_OK; }
  double beta = b0;
  int total = 0;
  std::vector<double> hist{b0};   // true residual at the start of each cycle
  while (true) {
    // v_0 = r / beta
    if ((st = axpby(s, 1.0 / beta, s->w, 0.0, nullptr, s->V))) return st;
    g0[0] = beta;
    HIPCHK(c, hipMemcpyAsync(s->dg, g0.data(), (m + 1) * sizeof(double), hipMemcpyHostToDevice, c->stream));
    int j = 0;
    const int mk = m - (int)order.size();   // directions from the preconditioned Arnoldi vectors
    for (; j < m && total < maxit; ++j, ++total) {
      const double* zsrc = nullptr;
      double zscale = 1.0;
      if (j >= mk) {
        const int slot = order[j - mk];
        zsrc = s->Aug + (long)slot * N;
        zscale = 1.0 / aug_norm[slot];
      }
      if ((st = arnoldi_step(s, pc, U, dt, j, zsrc, zscale))) return st;
      HIPCHK(c, hipMemcpyAsync(s->host, s->dest + j, sizeof(double), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipMemcpyAsync(s->host + 1, s->dn, sizeof(double), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      if (s->host[0] <= rtol * b0 || !(s->host[1] > 0.0)) { ++j; ++total; break; }
    }
    int used = 0;
    if ((st = cycle_solution(s, j, rtol * b0, y, &used))) return st;
    if (used > 0) HIPCHK(c, hipMemcpyAsync(s->hcol, y.data(), used * sizeof(double), hipMemcpyHostToDevice, c->stream));
    if (aug > 0) {
      // the cycle's correction d = Z y is kept for the next cycles (the ring
      // has k + 1 slots, so the slot written is never one this cycle used)
      double* d = s->Aug + (long)ring * N;
      hipLaunchKernelGGL(k_fill, dim3(grid_for(N, 256)), dim3(256), 0, c->stream, N, 0.0, d);
      if (used > 0)
        hipLaunchKernelGGL(k_multi_axpy_add, dim3(grid_for(N, 256)), dim3(256), 0, c->stream, N, used, s->hcol, s->Z,
                           N, d);
      HIPCHK(c, hipGetLastError());
      if ((st = axpby(s, 1.0, x, 1.0, d, x))) return st;
      double dn;
      if ((st = dots(s, 1, d, d, &dn))) return st;
      dn = std::sqrt(dn);
      if (dn > 0.0 && std::isfinite(dn)) {
        aug_norm[ring] = dn;
        order.insert(order.begin(), ring);
        if ((int)order.size() > aug) order.pop_back();
        ring = (ring + 1) % (aug + 1);
      }
    } else if (used > 0) {
      hipLaunchKernelGGL(k_multi_axpy_add, dim3(grid_for(N, 256)), dim3(256), 0, c->stream, N, used, s->hcol, s->Z, N, x);
      HIPCHK(c, hipGetLastError());
    }
    // true residual r = rhs - A x
    if ((st = apply_A(s, U, dt, x, s->w, nullptr))) return st;
    if ((st = axpby(s, 1.0, rhs, -1.0, s->w, s->w))) return st;
    if ((st = dots(s, 1, s->w, s->w, &nrm))) return st;
    beta = std::sqrt(nrm);
    *iters = total;
    *res_true = beta;
    // stagnation: less than 1% reduction over the last s->stall restart cycles
    hist.push_back(beta);
    const size_t nh = hist.size();
    const bool stalled = (int)nh > s->stall && beta > 0.99 * hist[nh - 1 - s->stall];
    if (beta <= rtol * b0 || total >= maxit || stalled || used == 0) break;
  }
  return FR_OK;
}

// ---- GMRES with captured Arnoldi steps
// The steps of a restart cycle are captured once per (iterate buffer,
// preconditioner, dt) twice over: in chunks of kChunk steps and one step per
// graph.  The host replays a chunk while the residual estimate, extrapolated
// at the last chunk's rate of decrease, stays above the tolerance for all of
// it, and single steps near the tolerance; it reads the estimates after each
// replay, so few steps run past the tolerance and a host round trip is paid
// once per chunk far from it.
static void drop_chunks(fr_solver_s* s) {
  for (auto& g : s->chunk)
    if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
  for (auto& g : s->single)
    if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
}

static fr_status capture_steps(fr_solver_s* s, fr_precond_s* pc, const double* U, double dt, int j0, int j1,
                               hipGraphExec_t* out) {
  fr_ctx_s* c = s->ctx;
  HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  fr_status st = FR_OK;
  for (int j = j0; j < j1 && st == FR_OK; ++j) st = arnoldi_step(s, pc, U, dt, j, nullptr, 1.0);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(c->stream, &g);
  if (st == FR_OK && e != hipSuccess) st = sfail(c, FR_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  if (st == FR_OK && hipGraphInstantiate(out, g, nullptr, nullptr, 0) != hipSuccess) {
    *out = nullptr;
    st = sfail(c, FR_E_DEVICE, "hipGraphInstantiate of the Arnoldi steps");
  }
  if (g) (void)hipGraphDestroy(g);
  return st;
}

static fr_status ensure_chunks(fr_solver_s* s, fr_precond_s* pc, const double* U, double dt) {
  fr_ctx_s* c = s->ctx;
  if (s->chunk[0] && s->key_U == U && s->key_pc == pc && s->key_dt == dt) return FR_OK;
  drop_chunks(s);
  const bool timing = c->timing;
  c->timing = false;
  fr_status st = FR_OK;
  const int K = fr_solver_s::kChunk;
  for (int ch = 0; (ch + 1) * K <= s->m && st == FR_OK; ++ch)
    st = capture_steps(s, pc, U, dt, ch * K, (ch + 1) * K, &s->chunk[ch]);
  for (int j = 0; j < s->m && st == FR_OK; ++j) st = capture_steps(s, pc, U, dt, j, j + 1, &s->single[j]);
  c->timing = timing;
  if (st) { drop_chunks(s); return st; }
  s->key_U = U; s->key_pc = pc; s->key_dt = dt;
  return FR_OK;
}

static fr_status gmres_graph(fr_solver_s* s, fr_precond_s* pc, const double* U, double dt, const double* rhs,
                             double rtol, int maxit, double* x, int* iters, double* res_true, double* res0_out,
                             int* cycles) {
  fr_ctx_s* c = s->ctx;
  const int m = s->m;
  const long N = s->N;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(N, 256)), dim3(256), 0, c->stream, N, 0.0, x);
  HIPCHK(c, hipMemcpyAsync(s->w, rhs, N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  double nrm;
  fr_status st = dots(s, 1, s->w, s->w, &nrm);
  if (st) return st;
  const double b0 = std::sqrt(nrm);
  *res0_out = b0;
  *iters = 0;
  *res_true = 0.0;
  if (b0 == 0.0) return FR_OK;
  if ((st = ensure_chunks(s, pc, U, dt))) return st;
  double beta = b0;
  int total = 0, work = 0;
  std::vector<double> hist{b0}, g0(m + 1, 0.0), y(m);
  const int K = fr_solver_s::kChunk;
  while (true) {
    if ((st = axpby(s, 1.0 / beta, s->w, 0.0, nullptr, s->V))) return st;
    g0[0] = beta;
    HIPCHK(c, hipMemcpyAsync(s->dg, g0.data(), (m + 1) * sizeof(double), hipMemcpyHostToDevice, c->stream));
    *cycles += 1;
    int jj = 0;
    double est = beta, rate = 0.0;     // rate: per-step decrease of the estimate (0: unknown)
    while (jj < m) {
      // a chunk while the extrapolated estimate stays above the tolerance
      const bool chunk = jj % K == 0 && s->chunk[jj / K] &&
                         (rate <= 0.0 || est * std::pow(rate, (double)K) > rtol * b0);
      const int n = chunk ? K : 1;
      HIPCHK(c, hipGraphLaunch(chunk ? s->chunk[jj / K] : s->single[jj], c->stream));
      work += n;
      HIPCHK(c, hipMemcpyAsync(s->host, s->dest + jj, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      bool stop = false;
      for (int q = 0; q < n; ++q)
        if (s->host[q] <= rtol * b0) { stop = true; break; }
      const double e1 = s->host[n - 1];
      if (est > 0.0 && e1 > 0.0 && e1 < est) rate = std::pow(e1 / est, 1.0 / n);
      est = e1;
      jj += n;
      if (stop || work >= maxit) break;
    }
    int used = 0;
    if ((st = cycle_solution(s, jj, rtol * b0, y, &used))) return st;
    total += used;
    if (used > 0) {
      HIPCHK(c, hipMemcpyAsync(s->hcol, y.data(), used * sizeof(double), hipMemcpyHostToDevice, c->stream));
      hipLaunchKernelGGL(k_multi_axpy_add, dim3(grid_for(N, 256)), dim3(256), 0, c->stream, N, used, s->hcol, s->Z, N, x);
      HIPCHK(c, hipGetLastError());
    }
    if ((st = apply_A(s, U, dt, x, s->w, nullptr))) return st;
    if ((st = axpby(s, 1.0, rhs, -1.0, s->w, s->w))) return st;
    if ((st = dots(s, 1, s->w, s->w, &nrm))) return st;
    beta = std::sqrt(nrm);
    *iters = total;
    *res_true = beta;
    hist.push_back(beta);
    const size_t nh = hist.size();
    const bool stalled = (int)nh > s->stall && beta > 0.99 * hist[nh - 1 - s->stall];
    if (beta <= rtol * b0 || work >= maxit || stalled || used == 0) break;
  }
  return FR_OK;
}

extern "C" {

fr_status fr_precond_create(fr_ctx* c, fr_pc_kind kind, fr_precond** out) {
  if (!c || !out) return FR_E_INVALID;
  *out = nullptr;
  if (kind != FR_PC_BLOCK_JACOBI && kind != FR_PC_MLP) return sfail(c, FR_E_INVALID, "unknown preconditioner kind");
  if (!c->ks.jac) return sfail(c, FR_E_UNSUPPORTED, "block preconditioners need Jacobian blocks (not for SDRT contexts)");
  if (c->mixed) return sfail(c, FR_E_UNSUPPORTED, "block preconditioners need one block size (not for mixed meshes)");
  if (c->b > kLuMaxB) return sfail(c, FR_E_UNSUPPORTED, "block-Jacobi preconditioner supports blocks up to 320 x 320");
  if (kind == FR_PC_MLP && c->b > 64) return sfail(c, FR_E_UNSUPPORTED, "learned preconditioner blocks up to 64 x 64");
  fr_precond_s* pc = new fr_precond_s();
  pc->ctx = c; pc->kind = kind;
  const size_t bb = (size_t)c->b * c->b, ne = (size_t)c->ne;
  const size_t rs = c->prec == 0 ? 8 : 4;
  const bool lu = c->b > 128;     // LU factors and row order instead of explicit inverses
  size_t off_inv = (ne * bb * rs + 255) & ~(size_t)255;
  size_t off_bad = off_inv + ((ne * bb * 8 + 255) & ~(size_t)255);
  size_t off_perm = off_bad + ((ne * sizeof(int) + 255) & ~(size_t)255);
  size_t tot = off_perm + (lu ? ne * (size_t)c->b * sizeof(int) : 0);
  if (hipMalloc(&pc->mem, tot) != hipSuccess) { delete pc; return sfail(c, FR_E_NOMEM, "preconditioner storage"); }
  pc->jbuf = pc->mem;
  pc->inv = (double*)((char*)pc->mem + off_inv);
  pc->bad = (int*)((char*)pc->mem + off_bad);
  pc->piv = lu ? (int*)((char*)pc->mem + off_perm) : nullptr;
  if (hipHostMalloc((void**)&pc->bad_host, ne * sizeof(int), hipHostMallocDefault) != hipSuccess) {
    (void)hipFree(pc->mem); delete pc; return sfail(c, FR_E_NOMEM, "pinned flags");
  }
  if (kind == FR_PC_MLP) {
    fr_status st = pc_mlp_create(pc);
    if (st) { (void)hipFree(pc->mem); (void)hipHostFree(pc->bad_host); delete pc; return st; }
  }
  *out = pc;
  return FR_OK;
}

fr_status fr_precond_setup(fr_precond* pc, const void* U, double shift, double scale) {
  if (!pc || !U) return FR_E_INVALID;
  fr_status st = (pc->kind == FR_PC_MLP) ? pc_mlp_setup(pc, U, shift, scale) : pc_lu_setup(pc, U, shift, scale);
  pc->ready = (st == FR_OK);
  return st;
}

fr_status fr_apply_precond(fr_precond* pc, const void* r, void* z) {
  if (!pc || !r || !z || r == z) return FR_E_INVALID;
  if (!pc->ready) return sfail(pc->ctx, FR_E_INVALID, "fr_apply_precond before a successful fr_precond_setup");
  return (pc->kind == FR_PC_MLP) ? pc_mlp_apply(pc, r, z) : pc_lu_apply(pc, r, z);
}

fr_status fr_precond_destroy(fr_precond* pc) {
  if (!pc) return FR_E_INVALID;
  (void)hipStreamSynchronize(pc->ctx->stream);
  if (pc->mlp) pc_mlp_destroy(pc);
  (void)hipFree(pc->mem);
  (void)hipHostFree(pc->bad_host);
  delete pc;
  return FR_OK;
}

fr_status fr_solver_create(fr_ctx* c, int restart, fr_solver** out) {
  if (!c || !out || restart < 1 || restart > 31) return FR_E_INVALID;
  if (c->prec != 0) return sfail(c, FR_E_UNSUPPORTED, "Newton-GMRES runs on FP64 contexts");
  if (c->mixed) return sfail(c, FR_E_UNSUPPORTED, "Newton-GMRES runs on single-type meshes");
  fr_solver_s* s = new fr_solver_s();
  s->ctx = c; s->m = restart; s->N = c->ne * (long)c->b;
  const long N = s->N;
  size_t doubles = (size_t)N * (2 * (restart + 1) + 5 + kAugMax + 1) + kDotBlocks * 32 + 64 + 64;
  if (hipMalloc(&s->mem, doubles * sizeof(double)) != hipSuccess) { delete s; return sfail(c, FR_E_NOMEM, "solver workspace"); }
  double* p = (double*)s->mem;
  s->V = p; p += N * (restart + 1);
  s->Z = p; p += N * (restart + 1);
  s->w = p; p += N; s->x = p; p += N; s->F = p; p += N; s->R = p; p += N; s->tmp = p; p += N;
  s->Aug = p; p += N * (kAugMax + 1);
  s->partial = p; p += kDotBlocks * 32;
  s->dots = p; p += 64;
  s->hcol = p; p += 64;
  if (hipHostMalloc((void**)&s->host, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    (void)hipFree(s->mem); delete s; return sfail(c, FR_E_NOMEM, "pinned host scalars");
  }
  if (hipEventCreate(&s->e0) != hipSuccess || hipEventCreate(&s->e1) != hipSuccess) {
    (void)hipFree(s->mem); (void)hipHostFree(s->host); delete s; return sfail(c, FR_E_DEVICE, "events");
  }
  const int m = restart;
  const size_t nstate = (size_t)(m + 1) * m + (m + 1) + m + 2 * m + 3 * 32;
  if (hipMalloc(&s->dH, nstate * sizeof(double)) != hipSuccess ||
      hipHostMalloc((void**)&s->hstate, nstate * sizeof(double), hipHostMallocDefault) != hipSuccess ||
      hipStreamCreateWithFlags(&s->cs, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&s->join0, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&s->join1, hipEventDisableTiming) != hipSuccess) {
    fr_solver_destroy(s);
    return sfail(c, FR_E_NOMEM, "solver cycle state");
  }
  if (hipMalloc(&s->opart, 3 * kOrthBlocks * kMaxK * sizeof(double)) != hipSuccess) {
    fr_solver_destroy(s);
    return sfail(c, FR_E_NOMEM, "solver partial sums");
  }
  s->dg = s->dH + (size_t)(m + 1) * m;
  s->dest = s->dg + (m + 1);
  s->dcs = s->dest + m;
  s->dsn = s->dcs + m;
  s->dh1 = s->dsn + m;
  s->dh2 = s->dh1 + 32;
  s->dn = s->dh2 + 32;
  *out = s;
  return FR_OK;
}

fr_status fr_solver_destroy(fr_solver* s) {
  if (!s) return FR_E_INVALID;
  (void)hipStreamSynchronize(s->ctx->stream);
  if (s->cs) (void)hipStreamSynchronize(s->cs);
  drop_chunks(s);
  (void)hipFree(s->mem);
  if (s->opart) (void)hipFree(s->opart);
  (void)hipFree(s->dH);
  (void)hipHostFree(s->host);
  (void)hipHostFree(s->hstate);
  (void)hipEventDestroy(s->e0);
  (void)hipEventDestroy(s->e1);
  if (s->join0) (void)hipEventDestroy(s->join0);
  if (s->join1) (void)hipEventDestroy(s->join1);
  if (s->cs) (void)hipStreamDestroy(s->cs);
  delete s;
  return FR_OK;
}

static fr_status newton_body(fr_solver_s* s, fr_precond_s* pc, const void* Un_, void* U_, const fr_newton_opts* o,
                             fr_newton_stats* st) {
  fr_ctx_s* c = s->ctx;
  if (pc && pc->ctx != c) return sfail(c, FR_E_INVALID, "preconditioner belongs to another context");
  const double* Un = (const double*)Un_;
  double* U = (double*)U_;
  const long N = s->N;
  std::memset(st, 0, sizeof(*st));
  hipEvent_t e0 = s->e0, e1 = s->e1;
  HIPCHK(c, hipEventRecord(e0, c->stream));
  HIPCHK(c, hipMemcpyAsync(U, Un, N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  fr_status rs;
  if (pc) {
    if ((rs = fr_precond_setup(pc, Un, 1.0, -o->dt))) return rs;
    st->pc_setups = 1;
  }
  double f0 = 0.0;
  for (int it = 0; it <= o->newton_maxit; ++it) {
    // F = U - Un - dt R(U)
    int rc = c->ks.rhs(c, U, s->R);
    if (rc) return (fr_status)rc;
    HIPCHK(c, hipGetLastError());
    hipLaunchKernelGGL(k_axpby, dim3(grid_for(N, 256)), dim3(256), 0, c->stream, N, 1.0, U, -1.0, Un, s->F);
    if ((rs = axpby(s, 1.0, s->F, -o->dt, s->R, s->F))) return rs;
    double fn;
    if ((rs = dots(s, 1, s->F, s->F, &fn))) return rs;
    fn = std::sqrt(fn);
    if (!std::isfinite(fn)) return sfail(c, FR_E_NONFINITE, "Newton: the residual of the iterate is not finite");
    if (it == 0) f0 = fn;
    if (it < 32) st->res_hist[it] = fn;
    st->res0 = f0;
    st->res = fn;
    st->newton_iters = it;
    if (fn <= o->newton_rtol * f0 || f0 == 0.0) { st->converged = 1; break; }
    if (it == o->newton_maxit) break;
    if (pc && o->pc_refresh && it > 0) {
      if ((rs = fr_precond_setup(pc, U, 1.0, -o->dt))) return rs;
      st->pc_setups += 1;
    }
    // solve (I - dt J) dU = -F
    if ((rs = axpby(s, -1.0, s->F, 0.0, nullptr, s->F))) return rs;
    int gi = 0;
    double rt = 0.0, r0 = 0.0;
    if (o->use_graph && o->gmres_augment == 0)
      rs = gmres_graph(s, pc, U, o->dt, s->F, o->gmres_rtol, o->gmres_maxit, s->x, &gi, &rt, &r0, &st->cycles);
    else
      rs = gmres(s, pc, U, o->dt, s->F, o->gmres_rtol, o->gmres_maxit, o->gmres_augment, s->x, &gi, &rt, &r0);
    if (rs) return rs;
    st->gmres_iters += gi;
    if (it < 32) st->gmres_hist[it] = gi;
    st->last_linear_rel = r0 > 0 ? rt / r0 : 0.0;
    // backtracking on |F|: U + lambda dU, lambda = 1, 1/2, ... (at most 5 halvings)
    double lam = 1.0;
    bool found = false;
    for (int ls = 0; ls < 6; ++ls) {
      if ((rs = axpby(s, 1.0, U, lam, s->x, s->tmp))) return rs;
      rc = c->ks.rhs(c, s->tmp, s->R);
      if (rc) return (fr_status)rc;
      hipLaunchKernelGGL(k_axpby, dim3(grid_for(N, 256)), dim3(256), 0, c->stream, N, 1.0, s->tmp, -1.0, Un, s->w);
      if ((rs = axpby(s, 1.0, s->w, -o->dt, s->R, s->w))) return rs;
      double ft;
      if ((rs = dots(s, 1, s->w, s->w, &ft))) return rs;
      ft = std::sqrt(ft);
      if (std::isfinite(ft) && (ft < fn || ls == 5)) { found = true; break; }
      lam *= 0.5;
    }
    // no finite trial: the iterate is left as it is
    if (!found) return sfail(c, FR_E_NONFINITE, "Newton: no line-search trial has a finite residual");
    if ((rs = axpby(s, 1.0, U, lam, s->x, U))) return rs;
  }
  HIPCHK(c, hipEventRecord(e1, c->stream));
  HIPCHK(c, hipEventSynchronize(e1));
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  st->ms = ms;
  return st->converged ? FR_OK : sfail(c, FR_E_NOT_CONVERGED, "Newton did not reach its tolerance");
}

// The step runs on the solver's own stream (capturable), joined to the
// context stream by events at entry and exit.
fr_status fr_newton_step(fr_solver* s, fr_precond* pc, const void* Un_, void* U_, const fr_newton_opts* o,
                         fr_newton_stats* st) {
  if (!s || !Un_ || !U_ || !o || !st) return FR_E_INVALID;
  fr_ctx_s* c = s->ctx;
  if (o->gmres_augment < 0 || o->gmres_augment > kAugMax)
    return sfail(c, FR_E_INVALID, "gmres_augment must be in 0..3");
  if (o->gmres_stall < 0) return sfail(c, FR_E_INVALID, "gmres_stall must be >= 0");
  s->stall = o->gmres_stall > 0 ? o->gmres_stall : 4;
  if (pc && pc->ctx != c) return sfail(c, FR_E_INVALID, "preconditioner belongs to another context");
  const hipStream_t orig = c->stream;
  HIPCHK(c, hipEventRecord(s->join0, orig));
  HIPCHK(c, hipStreamWaitEvent(s->cs, s->join0, 0));
  c->stream = s->cs;
  fr_status r = newton_body(s, pc, Un_, U_, o, st);
  // the captured steps refer to this call's buffers and preconditioner
  if (s->chunk[0]) {
    (void)hipStreamSynchronize(s->cs);
    drop_chunks(s);
  }
  // rejected line-search trials may have recorded non-finite residuals:
  // the step reports its own outcome, so the word is cleared
  (void)hipStreamSynchronize(s->cs);
  if (fr_status_reset(c) != 0 && r == FR_OK) r = sfail(c, FR_E_DEVICE, "clearing the status word");
  c->stream = orig;
  (void)hipEventRecord(s->join1, s->cs);
  (void)hipStreamWaitEvent(orig, s->join1, 0);
  return r;
}

}  // extern "C"
