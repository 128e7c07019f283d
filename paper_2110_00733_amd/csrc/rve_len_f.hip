// FFT pass kernel instantiations: 5-smooth axis lengths 90..160 (those not in groups b, c).
#include "rve_registry.h"

namespace rve {
void register_group_f() {
  static const LenEntry e[] = {
      RVE_LEN_ENTRY(90, 10, 9),   RVE_LEN_ENTRY(100, 10, 10), RVE_LEN_ENTRY(108, 12, 9),
      RVE_LEN_ENTRY(120, 12, 10), RVE_LEN_ENTRY(125, 25, 5),  RVE_LEN_ENTRY(135, 15, 9),
      RVE_LEN_ENTRY(144, 12, 12), RVE_LEN_ENTRY(150, 15, 10), RVE_LEN_ENTRY(160, 16, 10),
  };
  for (const auto& x : e) register_len(x);
}
}  // namespace rve
