// FFT pass kernel instantiations: alternative factorisations of the paper's discretisation lengths
// (54, 108, 162, 216) with fewer threads per row, so that the split P3 variants apply (NB | 64 or
// W*NB a multiple of 64); the autotuner chooses among them.
#include "rve_registry.h"

namespace rve {
void register_group_h() {
  static const LenEntry e[] = {
      RVE_LEN_ENTRY(54, 18, 3),  RVE_LEN_ENTRY(108, 27, 4), RVE_LEN_ENTRY(108, 18, 6),
      RVE_LEN_ENTRY(162, 27, 6), RVE_LEN_ENTRY(216, 27, 8), RVE_LEN_ENTRY(216, 24, 9),
  };
  for (const auto& x : e) register_len(x);
}
}  // namespace rve
