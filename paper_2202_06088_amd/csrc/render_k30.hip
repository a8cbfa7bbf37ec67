// Compiled shape of the global-hyperangle form: K = 30 (Table 3's N = 30:
// every HH function with n <= 3), C = 8.
#include "render_kernels.h"

namespace neuvv {

NEUVV_RENDER_SHAPE(30, 8)

}  // namespace neuvv
