// Compiled shape of the global-hyperangle form: the workloads' leaf (K = 16,
// C = 8), with the appearance-edit variants.
#include "render_kernels.h"

namespace neuvv {

NEUVV_RENDER_SHAPE(16, 8)

}  // namespace neuvv
