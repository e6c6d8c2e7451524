// Instances of the fused x-update kernel for s-lengths 192, 256.
#include "solve_s_core.h"

namespace sr3d {
SR3D_SOLVE_S_DEFINE(192)
SR3D_SOLVE_S_DEFINE(256)
}  // namespace sr3d
