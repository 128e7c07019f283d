// FFT pass kernel instantiations: 5-smooth axis lengths 162..250.
#include "rve_registry.h"

namespace rve {
void register_group_g() {
  static const LenEntry e[] = {
      RVE_LEN_ENTRY(162, 18, 9),  RVE_LEN_ENTRY(180, 15, 12), RVE_LEN_ENTRY(192, 16, 12),
      RVE_LEN_ENTRY(200, 20, 10), RVE_LEN_ENTRY(216, 18, 12), RVE_LEN_ENTRY(225, 15, 15),
      RVE_LEN_ENTRY(240, 16, 15), RVE_LEN_ENTRY(243, 27, 9),  RVE_LEN_ENTRY(250, 25, 10),
  };
  for (const auto& x : e) register_len(x);
}
}  // namespace rve
