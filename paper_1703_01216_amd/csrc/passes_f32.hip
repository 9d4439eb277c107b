// FP32 instances of the pass launchers.
#include "passes_impl.hpp"

namespace fr3d {
FR3D_INST(float)
bool supported_length(int P) { return supported_length_impl(P); }
}  // namespace fr3d
