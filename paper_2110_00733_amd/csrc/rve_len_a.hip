// FFT pass kernel instantiations: axis lengths 2..30.
#include "rve_registry.h"

namespace rve {
void register_group_a() {
  static const LenEntry e[] = {
      RVE_LEN_ENTRY(2, 2, 1),   RVE_LEN_ENTRY(3, 3, 1),   RVE_LEN_ENTRY(4, 4, 1),  RVE_LEN_ENTRY(5, 5, 1),
      RVE_LEN_ENTRY(6, 6, 1),   RVE_LEN_ENTRY(8, 8, 1),   RVE_LEN_ENTRY(12, 12, 1), RVE_LEN_ENTRY(16, 4, 4),
      RVE_LEN_ENTRY(24, 6, 4),
      // alternative factorisations the autotuner may choose (stage A radix >= threads per row)
      RVE_LEN_ENTRY(16, 8, 2),  RVE_LEN_ENTRY(24, 8, 3),  RVE_LEN_ENTRY(24, 12, 2),
  };
  for (const auto& x : e) register_len(x);
}
}  // namespace rve
