// k_step_plain.hip -- single-lattice step kernels (one and two steps per
// launch) with the printed Newton update (Algorithm 3).
#include "launch.hpp"

IREBM_INSTANTIATE_STEP(irebm::kPlain);
