// k_batch_eebm.hip -- batch step kernels with the explicit enthalpy based
// method (Algorithm 2).
#include "launch.hpp"

IREBM_INSTANTIATE_BATCH(irebm::kEebm);
