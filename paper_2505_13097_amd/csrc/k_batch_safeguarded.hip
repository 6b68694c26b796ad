// k_batch_safeguarded.hip -- batch step kernels with the safeguarded
// Newton update (Algorithm 3).
#include "launch.hpp"

IREBM_INSTANTIATE_BATCH(irebm::kSafeguarded);
