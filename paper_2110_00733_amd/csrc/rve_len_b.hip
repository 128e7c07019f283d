// FFT pass kernel instantiations: axis lengths 32..96.
#include "rve_registry.h"

namespace rve {
void register_group_b() {
  static const LenEntry e[] = {
      RVE_LEN_ENTRY(32, 8, 4), RVE_LEN_ENTRY(48, 12, 4), RVE_LEN_ENTRY(64, 8, 8), RVE_LEN_ENTRY(96, 12, 8),
      // alternative factorisations the autotuner may choose (stage A radix >= threads per row)
      RVE_LEN_ENTRY(32, 16, 2), RVE_LEN_ENTRY(48, 8, 6), RVE_LEN_ENTRY(48, 16, 3), RVE_LEN_ENTRY(64, 16, 4),
      RVE_LEN_ENTRY(96, 16, 6),
  };
  for (const auto& x : e) register_len(x);
}
}  // namespace rve
