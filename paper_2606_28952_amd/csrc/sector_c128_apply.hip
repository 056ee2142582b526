// Sector kernel variants for c128 storage, plain product (Section 2.4, Eq. sreverse_sum).
#include "sector.h"

namespace pbs {

void* sector_kernel_c128_apply(bool batch, bool r16, bool rowlds, bool realc) {
  return sector_variants<double2, false>(batch, r16, rowlds, realc);
}

}  // namespace pbs
