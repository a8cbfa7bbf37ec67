// Compiled shapes of the global-hyperangle form: K = 16 and 30 with the
// paper's C = 31 density weights.
#include "render_kernels.h"

namespace neuvv {

NEUVV_RENDER_SHAPE(16, 31)
NEUVV_RENDER_SHAPE(30, 31)

}  // namespace neuvv
