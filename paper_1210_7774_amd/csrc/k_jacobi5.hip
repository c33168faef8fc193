// The paper's fixed-iteration Jacobi benchmark ("Performance Study":
// n x n array, a fixed number of iterations): every interior point becomes
// one fifth of the sum of itself and its four neighbours (the five-view
// stencil of the "NumPy" section, read as an average: a coefficient of one
// on the centre would not converge), the outermost ring of the array is a
// fixed boundary.
//
// Temporal blocking in registers: one wave owns a 64 x 64 region (a 56 x 56
// core plus four points of halo), one column per lane, loads it once, takes
// up to four iterations on it and stores the core, so several iterations
// cost one read and one write of the array (the paper's blocking rule,
// applied across iterations by recomputing the halo).  Horizontal
// neighbours come across lanes (DPP wave shifts), vertical ones from the
// lane's own registers; the rows are updated in place in order, keeping the
// old value of the row above.  Waves are independent: no LDS, no barriers.
// Only the array's fixed boundary needs a test: a point near the region's
// edge may be computed from stale or clamped neighbours, but such errors
// move inwards by one point per iteration and never reach the core.
#include "dev_common.h"

namespace mgx {

constexpr int kJR = 64;                // region edge (rows; columns = lanes)
constexpr int kJH = 4;                 // halo = most iterations per pass
constexpr int kJC = kJR - 2 * kJH;     // core edge
constexpr int kJThreads = 256;         // four independent waves

__global__ __launch_bounds__(kJThreads) void k_jacobi5(const double *in, double *out, int rows, int cols, int steps,
                                                        int tiles_x, int ntiles, int nblocks)
{
    const int lane = threadIdx.x & 63;
    // consecutive workgroups go to different XCDs: give each XCD a contiguous
    // range of tiles so neighbouring tiles share its L2 (halo rows/columns)
    int b = blockIdx.x;
    if ((nblocks & 7) == 0) b = (b & 7) * (nblocks >> 3) + (b >> 3);
    // the wave's region index is uniform: keep it (and every row condition
    // derived from it) in scalar registers
    const int t = __builtin_amdgcn_readfirstlane(b * (kJThreads / 64) + (int)(threadIdx.x >> 6));
    if (t >= ntiles) return;  // whole waves only
    const int tx = t % tiles_x, ty = t / tiles_x;
    const int gx = tx * kJC - kJH + lane;
    const int gy0 = ty * kJC - kJH;
    // rows and columns outside the array read a clamped copy: only boundary
    // points neighbour them, and those are never updated
    const int gxc = min(max(gx, 0), cols - 1);
    double v[kJR];
#pragma unroll
    for (int q = 0; q < kJR; ++q) {
        const int gy = min(max(gy0 + q, 0), rows - 1);
        v[q] = (in + (long long)gy * cols)[gxc];
    }
    const bool colint = gx >= 1 && gx <= cols - 2;
#pragma unroll 1
    for (int s = 1; s <= steps; ++s) {
        double prev = v[0];
#pragma unroll
        for (int q = 1; q < kJR - 1; ++q) {
            const double old = v[q];
            const double lf = from_prev(old, old), rt = from_next(old, old);
            const double sum = (((old + prev) + v[q + 1]) + lf) + rt;
            const bool rowint = (unsigned)(gy0 + q - 1) < (unsigned)(rows - 2);
            v[q] = (colint && rowint) ? 0.2 * sum : old;
            prev = old;
        }
    }
    if (lane >= kJH && lane < kJH + kJC && gx < cols) {
#pragma unroll
        for (int q = kJH; q < kJH + kJC; ++q) {
            const int gy = gy0 + q;
            if (gy < rows) (out + (long long)gy * cols)[gx] = v[q];
        }
    }
}

int jacobi5_max_steps() { return kJH; }

hipError_t launch_jacobi5(const double *in, double *out, int rows, int cols, int steps, hipStream_t s)
{
    if (steps < 0 || steps > kJH || rows < 1 || cols < 1) return hipErrorInvalidValue;
    const long long tx = (cols + kJC - 1) / kJC, ty = (rows + kJC - 1) / kJC;
    const long long nt = tx * ty, nb = (nt + kJThreads / 64 - 1) / (kJThreads / 64);
    if (nt > 0x7fffff00LL) return hipErrorInvalidValue;  // the tile index b * 4 + wave stays an int
    hipLaunchKernelGGL(k_jacobi5, dim3((unsigned)nb), dim3(kJThreads), 0, s, in, out, rows, cols, steps, (int)tx,
                       (int)nt, (int)nb);
    return hipGetLastError();
}

}  // namespace mgx
