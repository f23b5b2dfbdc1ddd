// float64 instantiations of the line-transform passes.
#include "fsd_lines.hpp"

namespace fsd {
FSD_DEFINE_LAUNCHERS(double)
}  // namespace fsd
