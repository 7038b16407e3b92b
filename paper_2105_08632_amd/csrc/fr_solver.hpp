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
fr_status pc_lu_setup(fr_precond_s* pc, const void* U, double shift, double scale);
fr_status pc_lu_apply(fr_precond_s* pc, const void* r, void* z);
