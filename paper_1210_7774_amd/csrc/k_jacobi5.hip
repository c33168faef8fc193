// The paper's fixed-iteration Jacobi benchmark ("Performance Study":
// n x n array, a fixed number of iterations): every interior point becomes
// one fifth of the sum of itself and its four neighbours (the five-view
// stencil of the "NumPy" section, read as an average: a coefficient of one
// on the centre would not converge), the outermost ring of the array is a
// fixed boundary.
//
// Temporal blocking: a workgroup loads a 64 x 64 region (a 56 x 56 core plus
// four points of halo) into LDS once, takes up to four iterations there (step
// s updates the region shrunk by s, which only reads values that step s - 1
// made valid) and stores the core, so several iterations cost one read and
// one write of the array: the paper's blocking rule, applied across
// iterations by recomputing the halo.  Each wave owns 16 rows of the
// region's 64 columns (one column per lane) and keeps its own points in
// registers: the vertical neighbours come from registers except at the
// segment ends; the horizontal ones from LDS.
#include "dev_common.h"

namespace mgx {

constexpr int kJR = 64;                // region edge
constexpr int kJH = 4;                 // halo = most iterations per pass
constexpr int kJC = kJR - 2 * kJH;     // core edge
constexpr int kJThreads = 256;         // 4 waves x 16 rows
constexpr int kJSeg = kJR / (kJThreads / 64);

__global__ __launch_bounds__(kJThreads) void k_jacobi5(const double *in, double *out, int rows, int cols, int steps,
                                                        int tiles_x, int nblocks)
{
    __shared__ double U[kJR * kJR];
    const int c = threadIdx.x & 63, seg = threadIdx.x >> 6;
    // consecutive workgroups go to different XCDs: give each XCD a contiguous
    // range of tiles so neighbouring tiles share its L2 (halo rows/columns)
    int b = blockIdx.x;
    if ((nblocks & 7) == 0) b = (b & 7) * (nblocks >> 3) + (b >> 3);
    const int tx = b % tiles_x, ty = b / tiles_x;
    const int gx = tx * kJC - kJH + c;
    const int r0 = seg * kJSeg;
    const int gy0 = ty * kJC - kJH + r0;
    const bool colok = gx >= 0 && gx < cols;
    double v[kJSeg];
#pragma unroll
    for (int q = 0; q < kJSeg; ++q) {
        const int gy = gy0 + q;
        const bool ok = colok && gy >= 0 && gy < rows;
        const double t = in[ok ? (long long)gy * cols + gx : 0];
        v[q] = ok ? t : 0.0;
    }
    const bool colint = gx >= 1 && gx <= cols - 2;
    const int cl = c > 0 ? c - 1 : 0, cr = c < kJR - 1 ? c + 1 : kJR - 1;
    for (int s = 1; s <= steps; ++s) {
        // the previous step's values (or the loads) into LDS
#pragma unroll
        for (int q = 0; q < kJSeg; ++q) U[(r0 + q) * kJR + c] = v[q];
        __syncthreads();
        const bool colupd = colint && c >= s && c <= kJR - 1 - s;
        const double above = U[(r0 > 0 ? r0 - 1 : 0) * kJR + c];
        const double below = U[(r0 + kJSeg < kJR ? r0 + kJSeg : kJR - 1) * kJR + c];
        double nv[kJSeg];
#pragma unroll
        for (int q = 0; q < kJSeg; ++q) {
            const int r = r0 + q, gy = gy0 + q;
            const double up = q > 0 ? v[q - 1] : above;
            const double dn = q < kJSeg - 1 ? v[q + 1] : below;
            const double lf = U[r * kJR + cl], rt = U[r * kJR + cr];
            const double sum = (((v[q] + up) + dn) + lf) + rt;
            const bool upd = colupd && r >= s && r <= kJR - 1 - s && gy >= 1 && gy <= rows - 2;
            nv[q] = upd ? 0.2 * sum : v[q];
        }
#pragma unroll
        for (int q = 0; q < kJSeg; ++q) v[q] = nv[q];
        __syncthreads();  // every read of this step is done before the next writes
    }
    if (c >= kJH && c < kJH + kJC && gx < cols) {
#pragma unroll
        for (int q = 0; q < kJSeg; ++q) {
            const int r = r0 + q, gy = gy0 + q;
            if (r >= kJH && r < kJH + kJC && gy < rows) out[(long long)gy * cols + gx] = v[q];
        }
    }
}

int jacobi5_max_steps() { return kJH; }

hipError_t launch_jacobi5(const double *in, double *out, int rows, int cols, int steps, hipStream_t s)
{
    if (steps < 0 || steps > kJH || rows < 1 || cols < 1) return hipErrorInvalidValue;
    const long long tx = (cols + kJC - 1) / kJC, ty = (rows + kJC - 1) / kJC;
    if (tx * ty > 0x7fffffffLL) return hipErrorInvalidValue;
    const int nb = (int)(tx * ty);
    hipLaunchKernelGGL(k_jacobi5, dim3(nb), dim3(kJThreads), 0, s, in, out, rows, cols, steps, (int)tx, nb);
    return hipGetLastError();
}

}  // namespace mgx
