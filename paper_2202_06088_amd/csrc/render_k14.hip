// Compiled shapes of the global-hyperangle form: K = 14 (Table 3's N = 14:
// every HH function with n <= 2), C = 8 and 31.
#include "render_kernels.h"

namespace neuvv {

NEUVV_RENDER_SHAPE(14, 8)
NEUVV_RENDER_SHAPE(14, 31)

}  // namespace neuvv
