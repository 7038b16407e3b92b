// Kernel instantiations for tetrahedron elements of degree 2.
#include "fr_impl.hpp"

void fr_reg_tet_2(KernelSet* t) {
  t[SYS_ADV * 2 + 0] = Impl<ET_TET, 2, SYS_ADV, double>::set();
  t[SYS_ADV * 2 + 1] = Impl<ET_TET, 2, SYS_ADV, float>::set();
  t[SYS_EULER * 2 + 0] = Impl<ET_TET, 2, SYS_EULER, double>::set();
  t[SYS_EULER * 2 + 1] = Impl<ET_TET, 2, SYS_EULER, float>::set();
  t[SYS_NS * 2 + 0] = Impl<ET_TET, 2, SYS_NS, double>::set();
  t[SYS_NS * 2 + 1] = Impl<ET_TET, 2, SYS_NS, float>::set();
}
