// 3D step kernels, safeguarded node update with the Neumann closure (see
// launch3.hpp)
#include "launch3.hpp"

IREBM_INSTANTIATE_STEP3(irebm::kSafeguarded | irebm::kNeumann);
