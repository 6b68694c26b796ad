// k_step_eebm_neumann.hip -- one-step kernels with the Neumann closure
// (eq. Neu_on_q) for lattices that have a Neumann wall.
#include "launch.hpp"

IREBM_INSTANTIATE_STEP1(irebm::kEebm | irebm::kNeumann);
