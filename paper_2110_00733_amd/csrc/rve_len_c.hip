// FFT pass kernel instantiations: axis lengths 128..256.
#include "rve_registry.h"

namespace rve {
void register_group_c() {
  static const LenEntry e[] = {
      RVE_LEN_ENTRY(128, 16, 8),
      RVE_LEN_ENTRY(256, 16, 16),
  };
  for (const auto& x : e) register_len(x);
}
}  // namespace rve
