// k_step_eebm.hip -- single-lattice step kernels (one and two steps per
// launch) with the explicit enthalpy based method (Algorithm 2).
#include "launch.hpp"

IREBM_INSTANTIATE_STEP(irebm::kEebm);
