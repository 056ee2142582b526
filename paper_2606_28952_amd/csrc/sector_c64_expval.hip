// Sector kernel variants for c64 storage, fused energy (Section 2.4, Eq. sreverse_sum).
#include "sector.h"

namespace pbs {

void* sector_kernel_c64_expval(bool batch, bool r16, bool rowlds, bool realc) {
  return sector_variants<float2, true>(batch, r16, rowlds, realc);
}

}  // namespace pbs
