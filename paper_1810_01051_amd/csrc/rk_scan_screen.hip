// Scan kernels of the two screen families (one register target per bucket;
// any screen bucket), every tile geometry, both kernels.
#include "rk_scan.h"

namespace rk {
RK_INSTANTIATE_SCAN(kFamScreen1, 0)
RK_INSTANTIATE_SCAN(kFamScreen1, 1)
RK_INSTANTIATE_SCAN(kFamScreen1, 2)
RK_INSTANTIATE_SCAN(kFamScreen1, 3)
RK_INSTANTIATE_LIST(kFamScreen1, 0)
RK_INSTANTIATE_LIST(kFamScreen1, 1)
RK_INSTANTIATE_LIST(kFamScreen1, 2)
RK_INSTANTIATE_LIST(kFamScreen1, 3)
RK_INSTANTIATE_SCAN(kFamScreen, 0)
RK_INSTANTIATE_SCAN(kFamScreen, 1)
RK_INSTANTIATE_SCAN(kFamScreen, 2)
RK_INSTANTIATE_SCAN(kFamScreen, 3)
RK_INSTANTIATE_LIST(kFamScreen, 0)
RK_INSTANTIATE_LIST(kFamScreen, 1)
RK_INSTANTIATE_LIST(kFamScreen, 2)
RK_INSTANTIATE_LIST(kFamScreen, 3)
}  // namespace rk
