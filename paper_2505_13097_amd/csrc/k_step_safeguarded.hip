// k_step_safeguarded.hip -- single-lattice step kernels (one and two steps per
// launch) with the safeguarded Newton update (Algorithm 3).
#include "launch.hpp"

IREBM_INSTANTIATE_STEP(irebm::kSafeguarded);
