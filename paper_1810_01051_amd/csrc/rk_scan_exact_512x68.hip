// Exact family (d = 256, q = 2^61 - 1; hash dump), general scan kernel, tile geometry
// 512x68 (workgroup size x windows per thread): one kernel per translation unit,
// so that the exact kernels compile in parallel.
#include "rk_scan.h"

namespace rk {
RK_INSTANTIATE_SCAN(kFamExact, 2)
}  // namespace rk
