// k_step_safeguarded_neumann.hip -- one-step kernels with the Neumann closure
// (eq. Neu_on_q) for lattices that have a Neumann wall.
#include "launch.hpp"

IREBM_INSTANTIATE_STEP1(irebm::kSafeguarded | irebm::kNeumann);
