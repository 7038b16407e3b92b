// Preconditioner object shared by the solver and the ABI.
#pragma once
#include <hip/hip_runtime.h>

#include "fr.h"
#include "fr_ctx.hpp"

struct fr_precond_s {
  fr_ctx_s* ctx = nullptr;
  int kind = 0;              // fr_pc_kind
  void* mem = nullptr;
  void* jbuf = nullptr;      // diagonal blocks, context precision
  double* inv = nullptr;     // [ne][b][b] column-major inverses (FP64); LU factors when b > 128
  int* piv = nullptr;        // [ne][b] pivot rows of the LU factors (b > 128)
  int* bad = nullptr;        // [ne] singular-pivot flags
  int* bad_host = nullptr;   // pinned copy
  bool ready = false;
  void* mlp = nullptr;       // learned-preconditioner state (FR_PC_MLP)
};

// learned preconditioner (fr_mlp.hip)
fr_status pc_mlp_create(fr_precond_s* pc);
fr_status pc_mlp_setup(fr_precond_s* pc, const void* U, double shift, double scale);
fr_status pc_mlp_apply(fr_precond_s* pc, const void* r, void* z);
void pc_mlp_destroy(fr_precond_s* pc);

fr_status pc_invert(fr_precond_s* pc, double shift, double scale, const int* list, long count);

// Value of v in lane l of the wavefront (l wave-uniform).
__device__ inline double wave_bcast(double v, int l) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)x, l), hi = __builtin_amdgcn_readlane((int)(x >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}


// Stored matrix entries: FP64, FP32 or raw BF16 bits.
__device__ inline double mat_val(double x) { return x; }
__device__ inline double mat_val(float x) { return (double)x; }
__device__ inline double mat_val(uint16_t h) { return (double)__uint_as_float((unsigned)h << 16); }

// z = sc * M r for one b x b column-major block (b <= 128) and one
// wavefront: lane l computes rows l and l + 64.  r is read once (lane c holds
// r[c] and r[c + 64]) and broadcast per column, so the column loads of the
// wavefront (b contiguous values each) are independent of one another.
// The same for b <= 64 with b a multiple of V = 16 / sizeof(entry): each
// lane loads V consecutive rows of one column with one 16-byte load, so a
// wavefront instruction reads V whole columns (1 KB); the partial sums of the
// V column groups are then added across lanes.
template <class MT, class VT>
__device__ inline void block_matvec16(int b, const MT* M, const VT* r, double sc, VT* z, int lane) {
  constexpr int V = 16 / (int)sizeof(MT), L = 64 / V;   // rows per lane load, lanes per column
  const int row0 = V * (lane % L), cg = lane / L;
  double a[V];
#pragma unroll
  for (int i = 0; i < V; ++i) a[i] = 0.0;
  // unrolled so that every load of a 64-row block can be in flight (FP32
  // blocks: 65 536 applications 0.190 -> 0.172 ms; FP64 unchanged)
#pragma unroll 16
  for (int c0 = 0; c0 < b; c0 += V) {
    const int c = c0 + cg;
    if (c < b && row0 < b) {
      const double rc = (double)r[c] * sc;
      // the inverses are streamed once per application (nontemporal)
      typedef unsigned int u4v __attribute__((ext_vector_type(4)));
      const u4v raw = __builtin_nontemporal_load((const u4v*)(M + (long)c * b + row0));
      MT vals[V];
      __builtin_memcpy(vals, &raw, 16);
#pragma unroll
      for (int i = 0; i < V; ++i) a[i] += mat_val(vals[i]) * rc;
    }
  }
#pragma unroll
  for (int off = L; off < 64; off <<= 1)
#pragma unroll
    for (int i = 0; i < V; ++i) a[i] += __shfl_xor(a[i], off, 64);
  if (cg == 0 && row0 < b)
#pragma unroll
    for (int i = 0; i < V; ++i) z[row0 + i] = (VT)a[i];
}

template <class MT, class VT>
__device__ inline void block_matvec(int b, const MT* M, const VT* r, double sc, VT* z, int lane) {
  if (b <= 64 && b % (16 / (int)sizeof(MT)) == 0) {
    block_matvec16<MT, VT>(b, M, r, sc, z, lane);
    return;
  }
  const int r0 = lane, r1 = lane + 64;
  const double v0 = r0 < b ? (double)r[r0] * sc : 0.0;
  const double v1 = r1 < b ? (double)r[r1] * sc : 0.0;
  double a0 = 0.0, a1 = 0.0;
  const int b0 = b < 64 ? b : 64;
#pragma unroll 16
  for (int c = 0; c < b0; ++c) {
    const double rc = wave_bcast(v0, c);
    if (r0 < b) a0 += mat_val(M[(long)c * b + r0]) * rc;
    if (r1 < b) a1 += mat_val(M[(long)c * b + r1]) * rc;
  }
#pragma unroll 4
  for (int c = 64; c < b; ++c) {
    const double rc = wave_bcast(v1, c - 64);
    if (r0 < b) a0 += mat_val(M[(long)c * b + r0]) * rc;
    if (r1 < b) a1 += mat_val(M[(long)c * b + r1]) * rc;
  }
  if (r0 < b) z[r0] = (VT)a0;
  if (r1 < b) z[r1] = (VT)a1;
}

fr_status pc_lu_setup(fr_precond_s* pc, const void* U, double shift, double scale);
fr_status pc_lu_apply(fr_precond_s* pc, const void* r, void* z);
