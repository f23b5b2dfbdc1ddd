// float32 instantiations of the line-transform passes (inner solves of the
// mixed-precision defect correction).
#include "fsd_passes.hpp"

namespace fsd {
FSD_DEFINE_LAUNCHERS2(float)
}  // namespace fsd
