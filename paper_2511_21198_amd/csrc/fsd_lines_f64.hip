// float64 instantiations of the line-transform passes.
#include "fsd_passes.hpp"

namespace fsd {
FSD_DEFINE_LAUNCHERS2(double)
}  // namespace fsd
