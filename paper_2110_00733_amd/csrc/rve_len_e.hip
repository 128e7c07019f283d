// FFT pass kernel instantiations: 5-smooth axis lengths 40..81 (those not in group b).
#include "rve_registry.h"

namespace rve {
void register_group_e() {
  static const LenEntry e[] = {
      RVE_LEN_ENTRY(40, 8, 5), RVE_LEN_ENTRY(45, 9, 5),  RVE_LEN_ENTRY(50, 10, 5), RVE_LEN_ENTRY(54, 9, 6),
      RVE_LEN_ENTRY(60, 10, 6), RVE_LEN_ENTRY(72, 9, 8), RVE_LEN_ENTRY(75, 15, 5), RVE_LEN_ENTRY(80, 10, 8),
      RVE_LEN_ENTRY(81, 9, 9),
  };
  for (const auto& x : e) register_len(x);
}
}  // namespace rve
