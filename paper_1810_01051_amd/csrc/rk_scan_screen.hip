// Scan kernels of the two screen families (one register target per bucket;
// any screen bucket), every tile geometry.
#include "rk_scan.h"

namespace rk {
template struct ScanGeom<kFamScreen1, 0>;
template struct ScanGeom<kFamScreen1, 1>;
template struct ScanGeom<kFamScreen1, 2>;
template struct ScanGeom<kFamScreen1, 3>;
template struct ScanGeom<kFamScreen, 0>;
template struct ScanGeom<kFamScreen, 1>;
template struct ScanGeom<kFamScreen, 2>;
template struct ScanGeom<kFamScreen, 3>;
}  // namespace rk
