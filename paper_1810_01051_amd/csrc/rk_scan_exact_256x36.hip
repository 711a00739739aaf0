// Scan kernels of the exact family (d = 256, q = 2^61 - 1; hash dump) for the
// 256x36 tile geometry (workgroup size x windows per thread); one geometry per
// translation unit, so that the exact kernels compile in parallel.
#include "rk_scan.h"

namespace rk {
template struct ScanGeom<kFamExact, 3>;
}  // namespace rk
