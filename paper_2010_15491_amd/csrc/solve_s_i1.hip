// Instances of the fused x-update kernel for s-lengths 64, 96, 128.
#include "solve_s_core.h"

namespace sr3d {
SR3D_SOLVE_S_DEFINE(64)
SR3D_SOLVE_S_DEFINE(96)
SR3D_SOLVE_S_DEFINE(128)
}  // namespace sr3d
