// Row-marching 2D kernels with float state (see k_march2d.inc).
#include "k_march2d.inc"

namespace mgx {
hipError_t launch_march2d_f32(int mode, bool vc, int nsweeps, int G, const MarchArgs &a, int grid, hipStream_t s)
{
    return march_launch_state<float, float>(mode, vc, nsweeps, G, a, grid, s);
}
}  // namespace mgx
