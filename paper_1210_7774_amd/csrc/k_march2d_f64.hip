// Row-marching 2D kernels with double state (see k_march2d.inc).
#include "k_march2d.inc"

namespace mgx {
hipError_t launch_march2d_f64(int mode, bool vc, int nsweeps, int G, const MarchArgs &a, int grid, hipStream_t s)
{
    return march_launch_state<double, double>(mode, vc, nsweeps, G, a, grid, s);
}
}  // namespace mgx
