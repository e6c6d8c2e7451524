// Instances of the fused x-update kernel for s-lengths 16, 24, 32, 48.
#include "solve_s_core.h"

namespace sr3d {
SR3D_SOLVE_S_DEFINE(16)
SR3D_SOLVE_S_DEFINE(24)
SR3D_SOLVE_S_DEFINE(32)
SR3D_SOLVE_S_DEFINE(48)
}  // namespace sr3d
