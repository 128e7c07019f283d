// FFT pass kernel instantiations: 5-smooth axis lengths 9..36 (those not in group a).
#include "rve_registry.h"

namespace rve {
void register_group_d() {
  static const LenEntry e[] = {
      RVE_LEN_ENTRY(9, 9, 1),   RVE_LEN_ENTRY(10, 10, 1), RVE_LEN_ENTRY(15, 15, 1), RVE_LEN_ENTRY(18, 6, 3),
      RVE_LEN_ENTRY(20, 5, 4),  RVE_LEN_ENTRY(25, 5, 5),  RVE_LEN_ENTRY(27, 9, 3),  RVE_LEN_ENTRY(30, 6, 5),
      RVE_LEN_ENTRY(36, 6, 6),
  };
  for (const auto& x : e) register_len(x);
}
}  // namespace rve
