// Instances of the fused x-update kernel for s-lengths 384, 512.
#include "solve_s_core.h"

namespace sr3d {
SR3D_SOLVE_S_DEFINE(384)
SR3D_SOLVE_S_DEFINE(512)
}  // namespace sr3d
