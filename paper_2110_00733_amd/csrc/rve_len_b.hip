// FFT pass kernel instantiations: axis lengths 32..96.
#include "rve_registry.h"

namespace rve {
void register_group_b() {
  static const LenEntry e[] = {
      RVE_LEN_ENTRY(32, 8, 4), RVE_LEN_ENTRY(48, 12, 4), RVE_LEN_ENTRY(64, 8, 8), RVE_LEN_ENTRY(96, 12, 8),
  };
  for (const auto& x : e) register_len(x);
}
}  // namespace rve
