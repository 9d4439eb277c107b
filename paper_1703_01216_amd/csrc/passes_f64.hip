// FP64 instances of the pass launchers.
#include "passes_impl.hpp"

namespace fr3d {
FR3D_INST(double)
}  // namespace fr3d
