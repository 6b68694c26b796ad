// k_batch_plain.hip -- batch step kernels with the printed Newton update
// (Algorithm 3).
#include "launch.hpp"

IREBM_INSTANTIATE_BATCH(irebm::kPlain);
