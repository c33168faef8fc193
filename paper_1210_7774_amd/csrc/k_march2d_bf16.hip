// Row-marching 2D kernels with bf16_t state (see k_march2d.inc).
#include "k_march2d.inc"

namespace mgx {
hipError_t launch_march2d_bf16(int mode, bool vc, int nsweeps, int G, const MarchArgs &a, int grid, hipStream_t s)
{
    return march_launch_state<bf16_t, float>(mode, vc, nsweeps, G, a, grid, s);
}
}  // namespace mgx
