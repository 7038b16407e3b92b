// Learned block preconditioner: a multilayer perceptron mapping a normalised
// diagonal block A^ = A / s (s = max |A_ij|) to an approximate inverse
// M ~ A^^-1, applied as z = M r / s.  Layers b^2 -> H -> H -> b^2 with ReLU
// after the two hidden layers; BF16 weights and activations, FP32
// accumulation on the gfx950 matrix cores (v_mfma_f32_16x16x32_bf16).
//
// Training minimises L = (1/B) sum_n ||A^_n M_n - I||_F^2 (the quantity the
// safeguard tests), so it needs no precomputed inverses: dL/dM_n =
// (2/B) A^_n^T (A^_n M_n - I).  Blocks and network outputs are stored as
// vec() of the column-major b x b matrix, the layout of the Jacobian blocks.
//
// Parameter vector (FP32 master copy, BF16 shadow for the matrix cores):
//   W1 [H][b^2], b1 [H], W2 [H][H], b2 [H], W3 [b^2][H], b3 [b^2]
// (row o of W holds the weights into output o).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "fr.h"
#include "fr_ctx.hpp"
#include "fr_solver.hpp"

typedef uint16_t bfu;   // raw BF16 bits
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__host__ __device__ inline bfu f2bf(float x) {    // round to nearest even
  uint32_t u = __builtin_bit_cast(uint32_t, x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (bfu)((u >> 16) | ((u & 0x7fffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bfu)(u >> 16);
}
__host__ __device__ inline float bf2f(bfu h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }

// ------------------------------------------------------------------ GEMM
// C[m][n] = sum_k opA(m,k) opB(n,k), BF16 operands, FP32 accumulation.
// opA(m,k) = AT ? A[k*lda + m] : A[m*lda + k]   (same for B with n).
// 128x128 output tile per workgroup (4 wavefronts of 64x64), K step 32,
// operands staged through LDS as [row][k] so each lane's MFMA fragment is
// one 16-byte read; the next K tile is fetched into registers while the
// current one is multiplied.
constexpr int kGT = 128, kGK = 32, kLDK = kGK + 8;
enum { EPI_BIAS_RELU = 0, EPI_BIAS = 1, EPI_MASK = 2, EPI_F32_ATOMIC = 3, EPI_F32_SLICE = 4 };

struct GemmArgs {
  int M, N, K, kchunk;
  const bfu* A; long lda;
  const bfu* B; long ldb;
  const float* bias;                    // [N]            EPI_BIAS_RELU, EPI_BIAS
  const bfu* mask; long ldm;         // C *= (mask > 0) EPI_MASK
  void* C; long ldc;                    // BF16, or FP32 accumulated atomically
  long slice;                           // EPI_F32_SLICE: FP32 partial sums of k-chunk z at C + z * slice
};

template <bool TR>
__device__ __forceinline__ void gemm_gload(const bfu* P, long ld, int row0, int rows, int k0, int kend, int tid,
                                           uint4 (&r)[2]) {
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int idx = tid + 256 * i;
    int row, k;
    if (!TR) { row = idx >> 2; k = (idx & 3) * 8; }
    else { k = idx >> 4; row = (idx & 15) * 8; }
    const int gr = row0 + row, gk = k0 + k;
    uint4 v = make_uint4(0, 0, 0, 0);
    if (gr < rows && gk < kend) v = *(const uint4*)(TR ? P + (long)gk * ld + gr : P + (long)gr * ld + gk);
    r[i] = v;
  }
}
template <bool TR>
__device__ __forceinline__ void gemm_lstore(bfu* S, int tid, const uint4 (&r)[2]) {
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int idx = tid + 256 * i;
    if (!TR) {
      *(uint4*)(S + (idx >> 2) * kLDK + (idx & 3) * 8) = r[i];
    } else {
      const int k = idx >> 4, row = (idx & 15) * 8;
      const bfu* h = (const bfu*)&r[i];
#pragma unroll
      for (int j = 0; j < 8; ++j) S[(row + j) * kLDK + k] = h[j];
    }
  }
}

template <bool AT, bool BT, int EPI>
__global__ void __launch_bounds__(256) k_gemm(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) bfu sA[kGT * kLDK];
  __shared__ __attribute__((aligned(16))) bfu sB[kGT * kLDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * kGT, n0 = blockIdx.x * kGT;
  const int kbeg = blockIdx.z * g.kchunk;
  const int kend = min(g.K, kbeg + g.kchunk);
  const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;
  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  uint4 ra[2], rb[2];
  if (kbeg < kend) {
    gemm_gload<AT>(g.A, g.lda, m0, g.M, kbeg, kend, tid, ra);
    gemm_gload<BT>(g.B, g.ldb, n0, g.N, kbeg, kend, tid, rb);
  }
  const int fr = lane & 15, fk = (lane >> 4) * 8;
  for (int k0 = kbeg; k0 < kend; k0 += kGK) {
    __syncthreads();
    gemm_lstore<AT>(sA, tid, ra);
    gemm_lstore<BT>(sB, tid, rb);
    __syncthreads();
    if (k0 + kGK < kend) {
      gemm_gload<AT>(g.A, g.lda, m0, g.M, k0 + kGK, kend, tid, ra);
      gemm_gload<BT>(g.B, g.ldb, n0, g.N, k0 + kGK, kend, tid, rb);
    }
    bf16x8 a[4], b[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      a[t] = __builtin_bit_cast(bf16x8, *(const uint4*)(sA + (wm + t * 16 + fr) * kLDK + fk));
      b[t] = __builtin_bit_cast(bf16x8, *(const uint4*)(sB + (wn + t * 16 + fr) * kLDK + fk));
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  }
  // lane holds D[4*(lane/16) + r][lane%16] of each 16x16 tile
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + i * 16 + (lane >> 4) * 4 + r;
        const int n = n0 + wn + j * 16 + fr;
        if (m >= g.M || n >= g.N) continue;
        float v = acc[i][j][r];
        if (EPI == EPI_F32_ATOMIC) {
          atomicAdd((float*)g.C + (long)m * g.ldc + n, v);
        } else if (EPI == EPI_F32_SLICE) {
          ((float*)g.C)[blockIdx.z * g.slice + (long)m * g.ldc + n] = v;
        } else {
          if (EPI == EPI_BIAS_RELU || EPI == EPI_BIAS) v += g.bias[n];
          if (EPI == EPI_BIAS_RELU) v = v > 0.f ? v : 0.f;
          if (EPI == EPI_MASK) v = bf2f(g.mask[(long)m * g.ldm + n]) > 0.f ? v : 0.f;
          ((bfu*)g.C)[(long)m * g.ldc + n] = f2bf(v);
        }
      }
}

// ------------------------------------------------------------------ residual
// Per sample n (one workgroup): E = A^ M - I; res[n] = ||E||_F; with grad,
// dM = gscale A^^T E written as BF16 (column-major).  b <= 64; the blocks are
// zero-padded to 64 x 64 in LDS.
constexpr int kRB = 64, kRP = 65;
__global__ void __launch_bounds__(256) k_mlp_resid(int b, const bfu* X, const bfu* Y, float gscale, float* res,
                                                   bfu* dY) {
  __shared__ __attribute__((aligned(16))) float sA[kRB * kRB];   // A^[r][k] at k*64 + r
  __shared__ float sAt[kRB * kRP];                               // A^[r][k] at r*65 + k
  __shared__ float sM[kRB * kRP];                                // M[k][c]  at c*65 + k
  __shared__ float sE[kRB * kRP];                                // E[k][c]  at c*65 + k
  __shared__ float red[256];
  const long n = blockIdx.x;
  const int tid = threadIdx.x;
  const long bb = (long)b * b;
  for (int i = tid; i < kRB * kRB; i += 256) {
    const int c = i / kRB, r = i % kRB;
    float a = 0.f, m = 0.f;
    if (r < b && c < b) { a = bf2f(X[n * bb + c * b + r]); m = bf2f(Y[n * bb + c * b + r]); }
    sA[c * kRB + r] = a;
    sAt[r * kRP + c] = a;
    sM[c * kRP + r] = m;
  }
  __syncthreads();
  const int r0 = 4 * (tid & 15), c0 = 4 * (tid >> 4);
  float e[4][4] = {};
  for (int k = 0; k < kRB; ++k) {
    const float4 av = *(const float4*)(sA + k * kRB + r0);
    const float a4[4] = {av.x, av.y, av.z, av.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float mv = sM[(c0 + j) * kRP + k];
#pragma unroll
      for (int i = 0; i < 4; ++i) e[i][j] += a4[i] * mv;
    }
  }
  float ss = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = r0 + i, c = c0 + j;
      float v = e[i][j] - ((r == c && r < b) ? 1.f : 0.f);
      if (r >= b || c >= b) v = 0.f;
      e[i][j] = v;
      ss += v * v;
      sE[c * kRP + r] = v;
    }
  red[tid] = ss;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) res[n] = sqrtf(red[0]);
  if (!dY) return;
  float d[4][4] = {};
  for (int k = 0; k < kRB; ++k) {
    float a4[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a4[i] = sAt[k * kRP + r0 + i];     // A^[k][r0+i]
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float ev = sE[(c0 + j) * kRP + k];
#pragma unroll
      for (int i = 0; i < 4; ++i) d[i][j] += a4[i] * ev;
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = r0 + i, c = c0 + j;
      if (r < b && c < b) dY[n * bb + c * b + r] = f2bf(gscale * d[i][j]);
    }
}

// ------------------------------------------------------------------ small kernels
// out[c] += sum over rows [y*chunk, (y+1)*chunk) of X[r][c] (bias gradients)
__global__ void __launch_bounds__(256) k_colsum(const bfu* X, int rows, int cols, long ld, int chunk, float* out) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= cols) return;
  const int r0 = blockIdx.y * chunk, r1 = min(rows, r0 + chunk);
  float s = 0.f;
  for (int r = r0; r < r1; ++r) s += bf2f(X[(long)r * ld + c]);
  atomicAdd(out + c, s);
}

// C = epilogue(sum over the nz k-chunk slices of P, in slice order): the
// split-K GEMM's deterministic reduction (P [nz][M][N] FP32, C BF16)
template <int EPI>
__global__ void __launch_bounds__(256) k_split_epi(int M, int N, int nz, const float* P, long slice, const float* bias,
                                                   const bfu* mask, long ldm, bfu* C, long ldc) {
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < (long)M * N; i += (long)gridDim.x * 256) {
    const int m = (int)(i / N), n = (int)(i % N);
    float v = 0.f;
    for (int z = 0; z < nz; ++z) v += P[z * slice + i];
    if (EPI == EPI_BIAS_RELU || EPI == EPI_BIAS) v += bias[n];
    if (EPI == EPI_BIAS_RELU) v = v > 0.f ? v : 0.f;
    if (EPI == EPI_MASK) v = bf2f(mask[(long)m * ldm + n]) > 0.f ? v : 0.f;
    C[(long)m * ldc + n] = f2bf(v);
  }
}

__global__ void k_fill_f32(long n, float v, float* x) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) x[i] = v;
}

// sum of per-sample squared residuals, times gscale (the training loss)
__global__ void __launch_bounds__(256) k_loss_sum(long nb, const float* res, float gscale, float* loss) {
  __shared__ float red[256];
  float s = 0.f;
  for (long i = threadIdx.x; i < nb; i += 256) s += res[i] * res[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = gscale * red[0];
}

// Adam (Kingma & Ba) on the FP32 master weights; refreshes the BF16 shadow.
__global__ void k_adam(long n, float* w, const float* g, float* m, float* v, bfu* wbf, float lr, float b1, float b2,
                       float eps, float bc1, float bc2) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi; v[i] = vi;
    const float wi = w[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    w[i] = wi;
    wbf[i] = f2bf(wi);
  }
}

__global__ void k_to_bf16(long n, const float* w, bfu* wbf) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    wbf[i] = f2bf(w[i]);
}

// A = shift I + scale J_nn (column-major), s_n = max |A_ij|, X_n = bf16(A / s_n)
template <class IT>
__global__ void __launch_bounds__(256) k_mlp_inputs(long ne, int b, const IT* J, double shift, double scale, bfu* X,
                                                    float* s) {
  __shared__ double red[256];
  const long n = blockIdx.x;
  const long bb = (long)b * b;
  double mx = 0.0;
  for (long i = threadIdx.x; i < bb; i += 256) {
    double a = scale * (double)J[n * bb + i] + ((i / b == i % b) ? shift : 0.0);
    mx = fmax(mx, fabs(a));
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + k]);
    __syncthreads();
  }
  const double sc = red[0] > 0.0 ? red[0] : 1.0;
  for (long i = threadIdx.x; i < bb; i += 256) {
    double a = scale * (double)J[n * bb + i] + ((i / b == i % b) ? shift : 0.0);
    X[n * bb + i] = f2bf((float)(a / sc));
  }
  if (threadIdx.x == 0) s[n] = (float)sc;
}

// z_n = M_n r_n / s_n (network), or Ainv_n r_n where the safeguard rejected
// the network (use_lu[n] != 0).  One wavefront per element, lanes over rows.
template <class VT, class MT>
__global__ void __launch_bounds__(256) k_mlp_apply(long ne, int b, const MT* M, const float* s, const int* use_lu,
                                                   const double* Ainv, const VT* r, VT* z) {
  const int lane = threadIdx.x & 63;
  const long n = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (n >= ne) return;
  const long bb = (long)b * b;
  if (use_lu[n]) block_matvec<double, VT>(b, Ainv + n * bb, r + n * b, 1.0, z + n * b, lane);
  else block_matvec<MT, VT>(b, M + n * bb, r + n * b, 1.0 / (double)s[n], z + n * b, lane);
}

// ------------------------------------------------------------------ refinement
// Newton-Schulz refinement of an approximate inverse M of A^ = (shift I +
// scale J_n) / s_n, one workgroup of four wavefronts per element (b <= 64,
// padded to 64 with identity rows and columns):
//   E = I - A^ M,   M <- M + M E      (the new residual is E^2)
// until ||E||_F <= tol, max_it steps, or divergence (||E||_F > 1e6 or not
// finite).  A^ is rounded to FP32 from the assembled block (not from the
// network's BF16 input), so res[n] is the residual the safeguard needs.
// start 0: M from the network output (BF16); start 1: the scaled transpose
// A^T / (|A^|_1 |A^|_inf), for which rho(I - A^ M) < 1 for any nonsingular
// block (the refinement without the network).  Products on
// v_mfma_f32_16x16x4f32: wave w owns rows 16w..16w+15 of each product.
constexpr int kNS = 64, kNSS = 68;   // padded order; LDS row stride (16-byte aligned rows)
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float ns_acc;

// C rows 16w..16w+15, columns 0..63: C[r][c] = sum_k A[r][k] B[k][c], A and B
// row-major with stride kNSS.  Matrix instruction kk takes k = 16 g + kk in
// the slot of lane group g (the order of a sum over k is free as long as A
// and B agree), so each lane reads its sixteen A values as four 16-byte runs.
__device__ __forceinline__ void ns_gemm(const float* A, const float* B, int w, int lane, ns_acc (&acc)[4]) {
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = ns_acc{0.f, 0.f, 0.f, 0.f};
  const int i = lane & 15, g = lane >> 4;
  const float4* ar = (const float4*)(A + (16 * w + i) * kNSS + 16 * g);
  float av[16];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float4 v = ar[q];
    av[4 * q] = v.x; av[4 * q + 1] = v.y; av[4 * q + 2] = v.z; av[4 * q + 3] = v.w;
  }
  const float* bcol = B + 16 * g * kNSS + i;
#pragma unroll
  for (int kk = 0; kk < 16; ++kk)
#pragma unroll
    for (int t = 0; t < 4; ++t)
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[kk], bcol[kk * kNSS + 16 * t], acc[t], 0, 0, 0);
}

template <class IT>
__global__ void __launch_bounds__(256) k_ns_refine(long ne, int b, const IT* J, double shift, double scale,
                                                   const float* s, const bfu* M0, int start, int max_it, float tol,
                                                   float* Mout, float* res, int* iters) {
  __shared__ __attribute__((aligned(16))) float Ar[kNS * kNSS];   // A^ row-major
  __shared__ __attribute__((aligned(16))) float Mr[kNS * kNSS];   // M row-major
  __shared__ __attribute__((aligned(16))) float Er[kNS * kNSS];   // E row-major
  __shared__ float red[8];
  const long n = blockIdx.x;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const long bb = (long)b * b;
  const double is = 1.0 / (double)s[n];
  for (int i = tid; i < kNS * kNS; i += 256) {
    const int c = i >> 6, r = i & 63;
    float a = (r == c) ? 1.f : 0.f;
    if (r < b && c < b) a = (float)((scale * (double)J[n * bb + (long)c * b + r] + (r == c ? shift : 0.0)) * is);
    Ar[r * kNSS + c] = a;
  }
  __syncthreads();
  if (start == 1) {
    // alpha = 1 / (largest column sum * largest row sum) of |A^|
    float cs = 0.f;
    if (tid < 64) {
      for (int r = 0; r < kNS; ++r) cs += fabsf(Ar[r * kNSS + tid]);
    } else if (tid < 128) {
      for (int c = 0; c < kNS; ++c) cs += fabsf(Ar[(tid - 64) * kNSS + c]);
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) cs = fmaxf(cs, __shfl_xor(cs, m, 64));
    if (lane == 0) red[w] = cs;
    __syncthreads();
    const float alpha = 1.f / (red[0] * red[1]);
    for (int i = tid; i < kNS * kNS; i += 256) {
      const int c = i >> 6, r = i & 63;
      Mr[r * kNSS + c] = alpha * Ar[c * kNSS + r];        // M[r][c] = alpha A^[c][r]
    }
  } else {
    for (int i = tid; i < kNS * kNS; i += 256) {
      const int c = i >> 6, r = i & 63;
      float v = (r == c) ? 1.f : 0.f;
      if (r < b && c < b) v = bf2f(M0[n * bb + (long)c * b + r]);
      Mr[r * kNSS + c] = v;
    }
  }
  __syncthreads();
  // output fragment of this lane: rows rq..rq+3, column 16 t + col of tile t
  const int col = lane & 15, rq = 16 * w + 4 * (lane >> 4);
  int it = 0;
  float nrm = 0.f;
  for (;;) {
    ns_acc acc[4];
    ns_gemm(Ar, Mr, w, lane, acc);                         // T = A^ M
    float ss = 0.f;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = rq + v, c = 16 * t + col;
        const float e = ((r == c) ? 1.f : 0.f) - acc[t][v];
        Er[r * kNSS + c] = e;
        ss += e * e;
      }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) ss += __shfl_xor(ss, m, 64);
    if (lane == 0) red[4 + w] = ss;
    __syncthreads();
    nrm = sqrtf(red[4] + red[5] + red[6] + red[7]);
    if (!(nrm > tol) || it >= max_it || !(nrm <= 1e6f)) break;   // uniform over the workgroup
    ns_gemm(Mr, Er, w, lane, acc);                         // P = M E
    __syncthreads();                                       // every wave has read M
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) Mr[(rq + v) * kNSS + 16 * t + col] += acc[t][v];
    __syncthreads();
    ++it;
  }
  float* out = Mout + n * bb;
  for (int i = tid; i < b * b; i += 256) {
    const int c = i / b, r = i % b;
    out[i] = Mr[r * kNSS + c];
  }
  if (tid == 0) { res[n] = nrm; iters[n] = it; }
}

// ------------------------------------------------------------------ host object
struct fr_mlp_s {
  int b = 0, nin = 0, H = 0, max_batch = 0;
  long np = 0;
  long oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0;
  hipStream_t stream = nullptr;
  void* mem = nullptr;
  float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  bfu* wbf = nullptr;
  bfu *H1 = nullptr, *H2 = nullptr, *Y = nullptr, *dY = nullptr, *dZ2 = nullptr, *dZ1 = nullptr;
  float *res = nullptr, *loss = nullptr;
  float* part = nullptr;                // split-K partial sums, [kSplit][max_batch][H]
  int step = 0;
  std::string err;
};

static fr_status mfail(fr_mlp_s* m, fr_status s, const std::string& e) {
  if (m) m->err = e;
  return s;
}
#define MCHK(mm, x)                                                                     \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess) return mfail((mm), FR_E_DEVICE, std::string(#x ": ") + hipGetErrorString(e_)); \
  } while (0)

static int egrid(long n) {
  long g = (n + 255) / 256;
  return (int)(g > 8192 ? 8192 : (g < 1 ? 1 : g));
}

template <bool AT, bool BT, int EPI>
static fr_status gemm(fr_mlp_s* mm, hipStream_t st, int M, int N, int K, const bfu* A, long lda, const bfu* B,
                      long ldb, void* C, long ldc, const float* bias = nullptr, const bfu* mask = nullptr,
                      long ldm = 0, int ksplit = 1, long slice = 0) {
  if (M <= 0) return FR_OK;
  // 16-byte operand rows: the contiguous dimension of each operand is a multiple of 8
  if (N % kGT || ((!AT || !BT) && K % 8) || lda % 8 || ldb % 8 || (AT && M % 8))
    return mfail(mm, FR_E_INVALID, "gemm shape not supported");
  GemmArgs g{};
  g.M = M; g.N = N; g.K = K;
  int kc = (K + ksplit - 1) / ksplit;
  kc = (kc + kGK - 1) / kGK * kGK;
  g.kchunk = kc;
  g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.bias = bias; g.mask = mask; g.ldm = ldm; g.C = C; g.ldc = ldc;
  g.slice = slice;
  dim3 grid(N / kGT, (M + kGT - 1) / kGT, (K + kc - 1) / kc);
  hipLaunchKernelGGL((k_gemm<AT, BT, EPI>), grid, dim3(256), 0, st, g);
  MCHK(mm, hipGetLastError());
  return FR_OK;
}

// A GEMM with a BF16 result of N = H columns: when its output has few
// 128 x 128 tiles (a training batch) and K is long, the k range is split
// over up to kSplit workgroups per tile, each writing FP32 partial sums to
// its own slice, and k_split_epi adds the slices in order and applies the
// epilogue (deterministic, unlike atomic accumulation).
constexpr int kSplit = 16;
template <bool AT, bool BT, int EPI>
static fr_status gemm_narrow(fr_mlp_s* mm, hipStream_t st, int M, int N, int K, const bfu* A, long lda, const bfu* B,
                             long ldb, bfu* C, long ldc, const float* bias = nullptr, const bfu* mask = nullptr,
                             long ldm = 0) {
  const long tiles = (long)((M + kGT - 1) / kGT) * (N / kGT);
  int ks = (int)std::min<long>(kSplit, (256 + tiles - 1) / tiles);
  ks = std::min(ks, std::max(1, K / (4 * kGK)));
  if (ks <= 1 || M > mm->max_batch || N > mm->H)
    return gemm<AT, BT, EPI>(mm, st, M, N, K, A, lda, B, ldb, C, ldc, bias, mask, ldm);
  int kc = (K + ks - 1) / ks;
  kc = (kc + kGK - 1) / kGK * kGK;
  const int nz = (K + kc - 1) / kc;
  const long slice = (long)M * N;
  fr_status r = gemm<AT, BT, EPI_F32_SLICE>(mm, st, M, N, K, A, lda, B, ldb, mm->part, N, nullptr, nullptr, 0, ks,
                                            slice);
  if (r) return r;
  hipLaunchKernelGGL((k_split_epi<EPI>), dim3(egrid(slice)), dim3(256), 0, st, M, N, nz, mm->part, slice, bias, mask,
                     ldm, C, ldc);
  MCHK(mm, hipGetLastError());
  return FR_OK;
}

// forward of nb samples X [nb][nin] -> Y [nb][nin] (BF16), hidden layers kept
static fr_status mlp_forward(fr_mlp_s* mm, hipStream_t st, const bfu* X, long nb, bfu* Y) {
  const int H = mm->H, nin = mm->nin;
  fr_status r;
  if ((r = gemm_narrow<false, false, EPI_BIAS_RELU>(mm, st, (int)nb, H, nin, X, nin, mm->wbf + mm->oW1, nin, mm->H1,
                                                    H, mm->w + mm->ob1)))
    return r;
  if ((r = gemm_narrow<false, false, EPI_BIAS_RELU>(mm, st, (int)nb, H, H, mm->H1, H, mm->wbf + mm->oW2, H, mm->H2, H,
                                                    mm->w + mm->ob2)))
    return r;
  return gemm<false, false, EPI_BIAS>(mm, st, (int)nb, nin, H, mm->H2, H, mm->wbf + mm->oW3, H, Y, nin,
                                      mm->w + mm->ob3);
}

// loss and gradient of one batch (nb <= max_batch); grad [np] is overwritten
static fr_status mlp_loss_grad(fr_mlp_s* mm, hipStream_t st, const bfu* X, long nb, float* grad, float* loss,
                               float* res) {
  const int H = mm->H, nin = mm->nin;
  fr_status r;
  if ((r = mlp_forward(mm, st, X, nb, mm->Y))) return r;
  const float gs = 2.0f / (float)nb;
  hipLaunchKernelGGL(k_mlp_resid, dim3(nb), dim3(256), 0, st, mm->b, X, mm->Y, gs, res, mm->dY);
  MCHK(mm, hipGetLastError());
  hipLaunchKernelGGL(k_loss_sum, dim3(1), dim3(256), 0, st, nb, res, 1.0f / (float)nb, loss);
  hipLaunchKernelGGL(k_fill_f32, dim3(egrid(mm->np)), dim3(256), 0, st, mm->np, 0.f, grad);
  const int ks = (int)((nb + 255) / 256);
  const int rchunk = 16;                        // rows per column-sum workgroup
  const int kr = (int)((nb + rchunk - 1) / rchunk);
  const dim3 cg_in((nin + 255) / 256, kr), cg_h((H + 255) / 256, kr);
  // layer 3: dW3 = dY^T H2, db3 = sum dY, dZ2 = (dY W3) * (H2 > 0)
  if ((r = gemm<true, true, EPI_F32_ATOMIC>(mm, st, nin, H, (int)nb, mm->dY, nin, mm->H2, H, grad + mm->oW3, H,
                                            nullptr, nullptr, 0, ks)))
    return r;
  hipLaunchKernelGGL(k_colsum, cg_in, dim3(256), 0, st, mm->dY, (int)nb, nin, (long)nin, rchunk, grad + mm->ob3);
  if ((r = gemm_narrow<false, true, EPI_MASK>(mm, st, (int)nb, H, nin, mm->dY, nin, mm->wbf + mm->oW3, H, mm->dZ2,
                                              H, nullptr, mm->H2, H)))
    return r;
  // layer 2
  if ((r = gemm<true, true, EPI_F32_ATOMIC>(mm, st, H, H, (int)nb, mm->dZ2, H, mm->H1, H, grad + mm->oW2, H, nullptr,
                                            nullptr, 0, ks)))
    return r;
  hipLaunchKernelGGL(k_colsum, cg_h, dim3(256), 0, st, mm->dZ2, (int)nb, H, (long)H, rchunk, grad + mm->ob2);
  if ((r = gemm_narrow<false, true, EPI_MASK>(mm, st, (int)nb, H, H, mm->dZ2, H, mm->wbf + mm->oW2, H, mm->dZ1, H,
                                              nullptr, mm->H1, H)))
    return r;
  // layer 1
  if ((r = gemm<true, true, EPI_F32_ATOMIC>(mm, st, H, nin, (int)nb, mm->dZ1, H, X, nin, grad + mm->oW1, nin,
                                            nullptr, nullptr, 0, ks)))
    return r;
  hipLaunchKernelGGL(k_colsum, cg_h, dim3(256), 0, st, mm->dZ1, (int)nb, H, (long)H, rchunk, grad + mm->ob1);
  MCHK(mm, hipGetLastError());
  return FR_OK;
}

// seeded initial weights (splitmix64 + Box-Muller): He-normal for the hidden
// layers, a small normal for the output layer, zero biases
static uint64_t splitmix(uint64_t& x) {
  uint64_t z = (x += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
static double unif(uint64_t& x) { return ((splitmix(x) >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
static double gauss(uint64_t& x) {
  double u = unif(x), v = unif(x);
  return std::sqrt(-2.0 * std::log(u)) * std::cos(6.283185307179586 * v);
}

// ------------------------------------------------------------------ preconditioner
struct PcMlp {
  fr_mlp_s* net = nullptr;
  double theta = 0.0;
  void* mem = nullptr;
  bfu* X = nullptr;    // [ne][b*b] normalised blocks
  bfu* M = nullptr;    // [ne][b*b] network outputs
  float* s = nullptr;     // [ne]
  float* res = nullptr;   // [ne] ||A^ M - I||_F
  int* use_lu = nullptr;  // [ne]
  int* list = nullptr;    // [ne] elements that fall back to LU
  float* M32 = nullptr;   // [ne][b*b] refined inverses (FP32)
  int* iters = nullptr;   // [ne] refinement steps taken
  float* res_host = nullptr;
  int* flag_host = nullptr;
  int* iters_host = nullptr;
  long n_fallback = 0;
  // Newton-Schulz refinement: steps, tolerance, start (0 network, 1 scaled transpose)
  int refine = 0;
  float refine_tol = 0.f;
  int start = 0;
  double mean_iters = 0.0, mean_res = 0.0, max_res = 0.0;
};

static fr_status sfail_pc(fr_precond_s* pc, fr_status s, const std::string& m) {
  pc->ctx->err = m;
  return s;
}

fr_status pc_mlp_create(fr_precond_s* pc) {
  fr_ctx_s* c = pc->ctx;
  PcMlp* p = new PcMlp();
  const size_t ne = (size_t)c->ne, bb = (size_t)c->b * c->b;
  size_t o1 = (ne * bb * 2 + 255) & ~(size_t)255;
  size_t o2 = o1 + ((ne * bb * 2 + 255) & ~(size_t)255);
  size_t o3 = o2 + ((ne * 4 + 255) & ~(size_t)255);
  size_t o4 = o3 + ((ne * 4 + 255) & ~(size_t)255);
  size_t o5 = o4 + ((ne * 4 + 255) & ~(size_t)255);
  size_t o6 = o5 + ((ne * 4 + 255) & ~(size_t)255);
  size_t o7 = o6 + ((ne * bb * 4 + 255) & ~(size_t)255);
  size_t tot = o7 + ne * 4;
  if (hipMalloc(&p->mem, tot) != hipSuccess) { delete p; c->err = "learned-preconditioner storage"; return FR_E_NOMEM; }
  char* base = (char*)p->mem;
  p->X = (bfu*)base; p->M = (bfu*)(base + o1); p->s = (float*)(base + o2); p->res = (float*)(base + o3);
  p->use_lu = (int*)(base + o4); p->list = (int*)(base + o5); p->M32 = (float*)(base + o6);
  p->iters = (int*)(base + o7);
  if (hipHostMalloc((void**)&p->res_host, ne * 4, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&p->flag_host, ne * 4, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&p->iters_host, ne * 4, hipHostMallocDefault) != hipSuccess) {
    (void)hipFree(p->mem);
    if (p->res_host) (void)hipHostFree(p->res_host);
    if (p->flag_host) (void)hipHostFree(p->flag_host);
    delete p; c->err = "pinned buffers"; return FR_E_NOMEM;
  }
  pc->mlp = p;
  return FR_OK;
}

void pc_mlp_destroy(fr_precond_s* pc) {
  PcMlp* p = (PcMlp*)pc->mlp;
  if (!p) return;
  (void)hipFree(p->mem);
  (void)hipHostFree(p->res_host);
  (void)hipHostFree(p->flag_host);
  (void)hipHostFree(p->iters_host);
  delete p;
  pc->mlp = nullptr;
}

static fr_status pc_mlp_normalise(fr_precond_s* pc, const void* U, double shift, double scale, bfu* X, float* s) {
  fr_ctx_s* c = pc->ctx;
  int rc = c->ks.jac(c, U, pc->jbuf, c->prec == 0 ? 0 : 1, 1);
  if (rc) return (fr_status)rc;
  if (c->prec == 0)
    hipLaunchKernelGGL(k_mlp_inputs<double>, dim3(c->ne), dim3(256), 0, c->stream, (long)c->ne, c->b,
                       (const double*)pc->jbuf, shift, scale, X, s);
  else
    hipLaunchKernelGGL(k_mlp_inputs<float>, dim3(c->ne), dim3(256), 0, c->stream, (long)c->ne, c->b,
                       (const float*)pc->jbuf, shift, scale, X, s);
  if (hipGetLastError() != hipSuccess) { c->err = "k_mlp_inputs launch"; return FR_E_DEVICE; }
  return FR_OK;
}

static bool b_too_large(const fr_ctx_s* c) { return c->b > kNS; }

fr_status pc_mlp_setup(fr_precond_s* pc, const void* U, double shift, double scale) {
  fr_ctx_s* c = pc->ctx;
  PcMlp* p = (PcMlp*)pc->mlp;
  const bool use_net = p->start == 0;
  if (use_net && !p->net) {
    c->err = "learned preconditioner has no network (fr_precond_set_mlp)"; return FR_E_INVALID;
  }
  if (b_too_large(c)) { c->err = "learned preconditioner: blocks up to 64 x 64"; return FR_E_UNSUPPORTED; }
  fr_mlp_s* mm = p->net;
  const long ne = c->ne;
  const int b = c->b;
  fr_status st = pc_mlp_normalise(pc, U, shift, scale, p->X, p->s);
  if (st) return st;
  // network outputs in chunks of the network's batch capacity
  if (use_net)
    for (long n0 = 0; n0 < ne; n0 += mm->max_batch) {
      long nb = std::min<long>(mm->max_batch, ne - n0);
      if ((st = mlp_forward(mm, c->stream, p->X + n0 * mm->nin, nb, p->M + n0 * mm->nin))) {
        c->err = mm->err; return st;
      }
    }
  // refinement (none: 0 steps) and the safeguard residual ||I - A^ M||_F
  // against the assembled block in FP32
  if (c->prec == 0)
    hipLaunchKernelGGL(k_ns_refine<double>, dim3(ne), dim3(256), 0, c->stream, ne, b, (const double*)pc->jbuf, shift,
                       scale, (const float*)p->s, (const bfu*)p->M, p->start, p->refine, p->refine_tol, p->M32,
                       p->res, p->iters);
  else
    hipLaunchKernelGGL(k_ns_refine<float>, dim3(ne), dim3(256), 0, c->stream, ne, b, (const float*)pc->jbuf, shift,
                       scale, (const float*)p->s, (const bfu*)p->M, p->start, p->refine, p->refine_tol, p->M32,
                       p->res, p->iters);
  if (hipGetLastError() != hipSuccess) { c->err = "k_ns_refine launch"; return FR_E_DEVICE; }
  if (hipMemcpyAsync(p->res_host, p->res, ne * 4, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipMemcpyAsync(p->iters_host, p->iters, ne * 4, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    c->err = "safeguard residual copy"; return FR_E_DEVICE;
  }
  std::vector<int> lst;
  double sum_it = 0.0, sum_res = 0.0, max_res = 0.0;
  for (long n = 0; n < ne; ++n) {
    const float r = p->res_host[n];
    const int fb = !(r <= (float)p->theta);          // also catches NaN
    p->flag_host[n] = fb;
    if (fb) lst.push_back((int)n);
    sum_it += p->iters_host[n];
    sum_res += std::isfinite(r) ? r : 1e30;
    max_res = std::max(max_res, std::isfinite(r) ? (double)r : 1e30);
  }
  p->mean_iters = sum_it / (double)ne;
  p->mean_res = sum_res / (double)ne;
  p->max_res = max_res;
  p->n_fallback = (long)lst.size();
  if (hipMemcpyAsync(p->use_lu, p->flag_host, ne * 4, hipMemcpyHostToDevice, c->stream) != hipSuccess) {
    c->err = "fallback flags copy"; return FR_E_DEVICE;
  }
  if (!lst.empty()) {
    if (hipMemcpyAsync(p->list, lst.data(), lst.size() * 4, hipMemcpyHostToDevice, c->stream) != hipSuccess) {
      c->err = "fallback list copy"; return FR_E_DEVICE;
    }
    if ((st = pc_invert(pc, shift, scale, p->list, (long)lst.size()))) return st;
    if (hipMemcpyAsync(pc->bad_host, pc->bad, ne * sizeof(int), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
      c->err = "fallback flags"; return FR_E_DEVICE;
    }
    for (int n : lst)
      if (pc->bad_host[n]) {
        c->err = "diagonal block of element " + std::to_string(n) + " is singular";
        return FR_E_SINGULAR;
      }
  }
  return FR_OK;
}

fr_status pc_mlp_apply(fr_precond_s* pc, const void* r, void* z) {
  fr_ctx_s* c = pc->ctx;
  PcMlp* p = (PcMlp*)pc->mlp;
  const long ne = c->ne;
  const int grid = (int)((ne + 3) / 4);
  // the network's BF16 output when it is used as is, else the refined FP32 inverse
  if (p->refine == 0 && p->start == 0) {
    if (c->prec == 0)
      hipLaunchKernelGGL((k_mlp_apply<double, bfu>), dim3(grid), dim3(256), 0, c->stream, ne, c->b,
                         (const bfu*)p->M, p->s, p->use_lu, pc->inv, (const double*)r, (double*)z);
    else
      hipLaunchKernelGGL((k_mlp_apply<float, bfu>), dim3(grid), dim3(256), 0, c->stream, ne, c->b,
                         (const bfu*)p->M, p->s, p->use_lu, pc->inv, (const float*)r, (float*)z);
  } else {
    if (c->prec == 0)
      hipLaunchKernelGGL((k_mlp_apply<double, float>), dim3(grid), dim3(256), 0, c->stream, ne, c->b,
                         (const float*)p->M32, p->s, p->use_lu, pc->inv, (const double*)r, (double*)z);
    else
      hipLaunchKernelGGL((k_mlp_apply<float, float>), dim3(grid), dim3(256), 0, c->stream, ne, c->b,
                         (const float*)p->M32, p->s, p->use_lu, pc->inv, (const float*)r, (float*)z);
  }
  if (hipGetLastError() != hipSuccess) { c->err = "k_mlp_apply launch"; return FR_E_DEVICE; }
  return FR_OK;
}

// ------------------------------------------------------------------ ABI
extern "C" {

fr_status fr_mlp_create(int b, int hidden, uint64_t seed, int max_batch, void* hip_stream, fr_mlp** out) {
  if (!out) return FR_E_INVALID;
  *out = nullptr;
  if (b < 1 || b > 64 || hidden < kGT || hidden % kGT || max_batch < 1 || (b * b) % kGT) return FR_E_INVALID;
  fr_mlp_s* m = new fr_mlp_s();
  m->b = b; m->nin = b * b; m->H = hidden; m->max_batch = max_batch;
  m->stream = (hipStream_t)hip_stream;
  const long nin = m->nin, H = hidden;
  m->oW1 = 0; m->ob1 = m->oW1 + H * nin; m->oW2 = m->ob1 + H; m->ob2 = m->oW2 + H * H; m->oW3 = m->ob2 + H;
  m->ob3 = m->oW3 + nin * H; m->np = m->ob3 + nin;
  // oW* offsets are multiples of 8 (BF16 rows stay 16-byte aligned)
  const size_t np = (size_t)m->np, mb = (size_t)max_batch;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  size_t off = 0;
  std::vector<size_t> o;
  for (size_t bytes : {np * 4, np * 4, np * 4, np * 4, np * 2, mb * H * 2, mb * H * 2, mb * nin * 2, mb * nin * 2,
                       mb * H * 2, mb * H * 2, mb * 4, (size_t)256, (size_t)kSplit * mb * H * 4}) {
    o.push_back(off);
    off += al(bytes);
  }
  if (hipMalloc(&m->mem, off) != hipSuccess) { delete m; return FR_E_NOMEM; }
  char* p = (char*)m->mem;
  m->w = (float*)(p + o[0]); m->g = (float*)(p + o[1]); m->m = (float*)(p + o[2]); m->v = (float*)(p + o[3]);
  m->wbf = (bfu*)(p + o[4]); m->H1 = (bfu*)(p + o[5]); m->H2 = (bfu*)(p + o[6]); m->Y = (bfu*)(p + o[7]);
  m->dY = (bfu*)(p + o[8]); m->dZ2 = (bfu*)(p + o[9]); m->dZ1 = (bfu*)(p + o[10]);
  m->res = (float*)(p + o[11]); m->loss = (float*)(p + o[12]); m->part = (float*)(p + o[13]);
  std::vector<float> w(np, 0.f);
  uint64_t x = seed;
  const double s1 = std::sqrt(2.0 / nin), s2 = std::sqrt(2.0 / H), s3 = 0.1 / std::sqrt((double)H);
  for (long i = 0; i < H * nin; ++i) w[m->oW1 + i] = (float)(s1 * gauss(x));
  for (long i = 0; i < H * H; ++i) w[m->oW2 + i] = (float)(s2 * gauss(x));
  for (long i = 0; i < nin * H; ++i) w[m->oW3 + i] = (float)(s3 * gauss(x));
  if (hipMemcpy(m->w, w.data(), np * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(m->m, 0, np * 4) != hipSuccess || hipMemset(m->v, 0, np * 4) != hipSuccess) {
    (void)hipFree(m->mem); delete m; return FR_E_DEVICE;
  }
  hipLaunchKernelGGL(k_to_bf16, dim3(egrid(m->np)), dim3(256), 0, m->stream, m->np, m->w, m->wbf);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(m->stream) != hipSuccess) {
    (void)hipFree(m->mem); delete m; return FR_E_DEVICE;
  }
  *out = m;
  return FR_OK;
}

fr_status fr_mlp_destroy(fr_mlp* m) {
  if (!m) return FR_E_INVALID;
  (void)hipStreamSynchronize(m->stream);
  (void)hipFree(m->mem);
  delete m;
  return FR_OK;
}

const char* fr_mlp_last_error(const fr_mlp* m) { return m ? m->err.c_str() : ""; }

fr_status fr_mlp_info(const fr_mlp* m, int64_t* n_params, int* b, int* hidden, int* max_batch) {
  if (!m) return FR_E_INVALID;
  if (n_params) *n_params = m->np;
  if (b) *b = m->b;
  if (hidden) *hidden = m->H;
  if (max_batch) *max_batch = m->max_batch;
  return FR_OK;
}

fr_status fr_mlp_set_params(fr_mlp* m, const float* params) {
  if (!m || !params) return FR_E_INVALID;
  MCHK(m, hipMemcpyAsync(m->w, params, m->np * 4, hipMemcpyDeviceToDevice, m->stream));
  hipLaunchKernelGGL(k_to_bf16, dim3(egrid(m->np)), dim3(256), 0, m->stream, m->np, m->w, m->wbf);
  MCHK(m, hipGetLastError());
  return FR_OK;
}

fr_status fr_mlp_get_params(fr_mlp* m, float* params) {
  if (!m || !params) return FR_E_INVALID;
  MCHK(m, hipMemcpyAsync(params, m->w, m->np * 4, hipMemcpyDeviceToDevice, m->stream));
  return FR_OK;
}

fr_status fr_mlp_forward(fr_mlp* m, const void* X, int64_t nb, void* Y) {
  if (!m || !X || !Y || nb < 0) return FR_E_INVALID;
  for (int64_t n0 = 0; n0 < nb; n0 += m->max_batch) {
    long k = (long)std::min<int64_t>(m->max_batch, nb - n0);
    fr_status st = mlp_forward(m, m->stream, (const bfu*)X + n0 * m->nin, k, (bfu*)Y + n0 * m->nin);
    if (st) return st;
  }
  return FR_OK;
}

fr_status fr_mlp_loss_grad(fr_mlp* m, const void* X, int64_t nb, float* loss, float* grad, float* resid) {
  if (!m || !X || !loss || !grad || nb < 1) return FR_E_INVALID;
  if (nb > m->max_batch) return mfail(m, FR_E_INVALID, "batch larger than max_batch");
  fr_status st = mlp_loss_grad(m, m->stream, (const bfu*)X, nb, grad, loss, resid ? resid : m->res);
  return st;
}

fr_status fr_mlp_train_step(fr_mlp* m, const void* X, int64_t nb, float lr, float* loss) {
  if (!m || !X || nb < 1) return FR_E_INVALID;
  if (nb > m->max_batch) return mfail(m, FR_E_INVALID, "batch larger than max_batch");
  fr_status st = mlp_loss_grad(m, m->stream, (const bfu*)X, nb, m->g, loss ? loss : m->loss, m->res);
  if (st) return st;
  m->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float bc1 = 1.f - std::pow(b1, (float)m->step), bc2 = 1.f - std::pow(b2, (float)m->step);
  hipLaunchKernelGGL(k_adam, dim3(egrid(m->np)), dim3(256), 0, m->stream, m->np, m->w, m->g, m->m, m->v, m->wbf, lr,
                     b1, b2, 1e-8f, bc1, bc2);
  MCHK(m, hipGetLastError());
  return FR_OK;
}

fr_status fr_precond_set_mlp(fr_precond* pc, fr_mlp* m, double theta) {
  if (!pc) return FR_E_INVALID;
  if (pc->kind != FR_PC_MLP) return sfail_pc(pc, FR_E_INVALID, "fr_precond_set_mlp needs an FR_PC_MLP preconditioner");
  if (m && m->b != pc->ctx->b) return sfail_pc(pc, FR_E_INVALID, "network block size differs from the context's");
  PcMlp* p = (PcMlp*)pc->mlp;
  p->net = m;
  p->theta = theta;
  pc->ready = false;
  return FR_OK;
}

fr_status fr_precond_mlp_inputs(fr_precond* pc, const void* U, double shift, double scale, void* X, float* s) {
  if (!pc || !U || !X || !s) return FR_E_INVALID;
  return pc_mlp_normalise(pc, U, shift, scale, (bfu*)X, s);
}

fr_status fr_precond_set_refine(fr_precond* pc, int max_iters, double tol, int start) {
  if (!pc) return FR_E_INVALID;
  if (pc->kind != FR_PC_MLP) return sfail_pc(pc, FR_E_INVALID, "fr_precond_set_refine needs an FR_PC_MLP preconditioner");
  if (max_iters < 0 || max_iters > 64 || !(tol >= 0.0) || (start != 0 && start != 1))
    return sfail_pc(pc, FR_E_INVALID, "fr_precond_set_refine: max_iters in 0..64, tol >= 0, start 0 or 1");
  PcMlp* p = (PcMlp*)pc->mlp;
  p->refine = max_iters;
  p->refine_tol = (float)tol;
  p->start = start;
  pc->ready = false;
  return FR_OK;
}

fr_status fr_precond_stats(const fr_precond* pc, int64_t* n_fallback, double* mean_refine_iters, double* mean_resid,
                           double* max_resid) {
  if (!pc) return FR_E_INVALID;
  const PcMlp* p = (pc->kind == FR_PC_MLP) ? (const PcMlp*)pc->mlp : nullptr;
  if (n_fallback) *n_fallback = p ? p->n_fallback : 0;
  if (mean_refine_iters) *mean_refine_iters = p ? p->mean_iters : 0.0;
  if (mean_resid) *mean_resid = p ? p->mean_res : 0.0;
  if (max_resid) *max_resid = p ? p->max_res : 0.0;
  return FR_OK;
}

fr_status fr_precond_info(const fr_precond* pc, int64_t* n_fallback) {
  if (!pc || !n_fallback) return FR_E_INVALID;
  *n_fallback = (pc->kind == FR_PC_MLP && pc->mlp) ? ((const PcMlp*)pc->mlp)->n_fallback : 0;
  return FR_OK;
}

}  // extern "C"
