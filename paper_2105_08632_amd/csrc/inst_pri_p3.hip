// Kernel instantiations for prism elements of degree 3.
#include "fr_impl.hpp"

void fr_reg_pri_3(KernelSet* t) {
  t[SYS_ADV * 2 + 0] = Impl<ET_PRI, 3, SYS_ADV, double>::set();
  t[SYS_ADV * 2 + 1] = Impl<ET_PRI, 3, SYS_ADV, float>::set();
  t[SYS_EULER * 2 + 0] = Impl<ET_PRI, 3, SYS_EULER, double>::set();
  t[SYS_EULER * 2 + 1] = Impl<ET_PRI, 3, SYS_EULER, float>::set();
  t[SYS_NS * 2 + 0] = Impl<ET_PRI, 3, SYS_NS, double>::set();
  t[SYS_NS * 2 + 1] = Impl<ET_PRI, 3, SYS_NS, float>::set();
}
