// Prisms of degree 4: their dense operator rows exceed one workgroup's LDS,
// so no kernels are registered (fr_ctx_create returns FR_E_UNSUPPORTED).
#include "fr_impl.hpp"

void fr_reg_pri_4(KernelSet* t) {
  for (int i = 0; i < 6; ++i) t[i] = KernelSet{};
}
