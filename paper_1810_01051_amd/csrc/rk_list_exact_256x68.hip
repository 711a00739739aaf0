// Exact family (d = 256, q = 2^61 - 1; hash dump), single-bucket kernel, tile geometry
// 256x68 (workgroup size x windows per thread): one kernel per translation unit,
// so that the exact kernels compile in parallel.
#include "rk_scan.h"

namespace rk {
RK_INSTANTIATE_LIST(kFamExact, 0)
}  // namespace rk
