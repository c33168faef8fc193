// LDS-tiled fused level kernels for the small 2D levels of the cycle.
//
// The row-marching kernels walk a chain of row steps whose length is set by
// the block height plus the halo; on a level of a few hundred rows that chain
// is pure memory latency.  Here one workgroup owns a 32 x 32 tile: it loads
// the tile plus a halo of R = 2 nu + 2 points into LDS in one round, runs the
// fused stages there with a barrier between stages, and writes its owned
// points back.  The stages and their arithmetic are those of the marching
// kernels (same update, residual, full weighting and bilinear correction
// formulas); the halo shrinks by one ring per stage, so every value kept
// depends only on data the workgroup loaded itself (the fusion that the
// paper's blockable rule, "Vector Engine" section, forbids for elementwise
// kernels is legal through the recomputed halo).
//
// PRE  (mode 0): from u (or zero), nu red-black sweeps, residual, full
//   weighting onto the coarse points the tile owns; writes A and f_c.
// POST (mode 1): A + P u_c (bilinear), nu red-black sweeps; writes B.
// Levels that hold a system's finest level keep the marching kernels (they
// add into the FP64 iterate and measure the residual norm).
#include "dev_common.h"

namespace mgx {

constexpr int kTile = 32;                            // owned points per side
constexpr int kTileRMax = 8;                         // halo for nu <= 3
constexpr int kTileNR = kTile + 2 * kTileRMax;       // largest region side
constexpr int kTileThreads = 1024;

template <class C>
__device__ __forceinline__ C tharmonic(C a, C b)
{
    return (C)2 * a * b / (a + b);
}

template <class S, class F, bool VC, int MODE, int NS>
__global__ __launch_bounds__(kTileThreads) void k_tile2d(MarchArgs args)
{
    using T = Traits<S>;
    using C = typename T::C;
    constexpr int NIT = (kTileNR * kTileNR + kTileThreads - 1) / kTileThreads;  // region passes
    constexpr int NA = NIT * kTileThreads;
    constexpr int kCN = kTileNR / 2 + 2;                                         // coarse region side
    constexpr int NCIT = (kCN * kCN + kTileThreads - 1) / kTileThreads;
    __shared__ C U[NA];
    __shared__ C Fv[NA];  // rhs, then (PRE) the residual
    __shared__ C WE[VC ? NA : 1], WN[VC ? NA : 1], ID[VC ? NA : 1];
    __shared__ C CV[MODE == 1 ? NCIT * kTileThreads : 1];  // coarse correction values
    constexpr int R = 2 * NS + 2, NR = kTile + 2 * R, NP = NR * NR;  // compile-time: index math by constants
    // items == null: one level (args.levels[0]) whose tiles follow the
    // workgroup index, which saves the dependent load of a work-item record
    const bool direct = args.items == nullptr;
    for (int item = blockIdx.x; item < args.nitems; item += gridDim.x) {
        MarchItem wi;
        LevelDesc L;
        if (direct) {
            L = args.levels[0];
            const int tiles_x = (L.n + kTile - 1) / kTile;
            wi.lvl = 0;
            wi.ia = 1 + kTile * (item % tiles_x);
            wi.ja = 1 + kTile * (item / tiles_x);
            wi.part = 0;
        } else {
            wi = args.items[item];
            L = args.levels[wi.lvl];
        }
        // the stop flag is tested after the region's loads are issued (the
        // same value for the whole workgroup)
        const int done = args.states[L.sys].done;
        const int n = L.n, nc = L.nc;
        const long long pitch = L.pitch, cpitch = L.cpitch;
        const int i0 = wi.ia - R, j0 = wi.ja - R;  // region origin (1-based)
        const int ia1 = wi.ia + kTile - 1, ja1 = wi.ja + kTile - 1;
        const C h2 = (C)L.h2, ih2 = (C)L.inv_h2;
        const S *uin = (MODE == 0) ? (L.uzero ? nullptr : (const S *)L.B) : (const S *)L.A;
        const F *fin = (const F *)L.f;
        const C *acoef = (const C *)L.a;
        // ---- load the region (and the faces touching it).  Fixed trip
        // count and clamped addresses, values selected afterwards: every
        // thread has all its loads in flight at once.
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int p = threadIdx.x + it * kTileThreads;
            const int gi = i0 + p % NR, gj = j0 + p / NR;
            const bool inside = p < NP && gi >= 1 && gi <= n && gj >= 1 && gj <= n;
            const long long o = inside ? (long long)(gj - 1) * pitch + (gi - 1) : 0;
            const C uv = uin ? (C)T::ld(uin + o) : (C)0;
            const C fv = (C)gld(fin + o);
            U[p] = inside ? uv : (C)0;
            Fv[p] = inside ? fv : (C)0;
            if constexpr (VC) {
                // east / north face of node (gi, gj) for nodes 0 .. n (faces
                // against boundary nodes use the boundary's coefficient)
                const bool fe = p < NP && gi >= 0 && gi <= n && gj >= 0 && gj <= n + 1;
                const bool fn = p < NP && gi >= 0 && gi <= n + 1 && gj >= 0 && gj <= n;
                const long long an = (fe || fn) ? (long long)gj * (n + 2) + gi : 0;
                const C ac = gld(acoef + an);
                const C ae = gld(acoef + (fe ? an + 1 : an));
                const C anb = gld(acoef + (fn ? an + (n + 2) : an));
                WE[p] = fe ? tharmonic(ac, ae) : (C)1;
                WN[p] = fn ? tharmonic(ac, anb) : (C)1;
            }
        }
        // ---- POST: the coarse values under the region, staged in LDS
        // (coarse I covers fine 2I; index 0 and nc + 1 are the zero boundary)
        const int ci0 = (i0 >= 1 ? (i0 - 1) / 2 : -((1 - i0 + 1) / 2)), cj0 = (j0 >= 1 ? (j0 - 1) / 2 : -((1 - j0 + 1) / 2));
        if constexpr (MODE == 1) {
            const S *bc = (const S *)L.Bc;
#pragma unroll
            for (int it = 0; it < NCIT; ++it) {
                const int q = threadIdx.x + it * kTileThreads;
                const int I = ci0 + q % kCN, J = cj0 + q / kCN;
                const bool ok = q < kCN * kCN && I >= 1 && I <= nc && J >= 1 && J <= nc;
                const C v = (C)T::ld(bc + (ok ? (long long)(J - 1) * cpitch + (I - 1) : 0));
                CV[q] = ok ? v : (C)0;
            }
        }
        if (done) continue;  // before the first barrier of the item
        __syncthreads();
        if constexpr (VC) {
            for (int p = threadIdx.x; p < NP; p += kTileThreads) {
                const int x = p % NR, y = p / NR;
                C v = (C)0.25;
                if (x >= 1 && y >= 1) v = (C)1 / (((WE[p - 1] + WE[p]) + WN[p - NR]) + WN[p]);
                ID[p] = v;
            }
        }
        // ---- POST: bilinear coarse-grid correction on the region
        if constexpr (MODE == 1) {
            auto cv = [&](int I, int J) -> C { return CV[(J - cj0) * kCN + (I - ci0)]; };
            for (int p = threadIdx.x; p < NP; p += kTileThreads) {
                const int gi = i0 + p % NR, gj = j0 + p / NR;
                if (!(gi >= 1 && gi <= n && gj >= 1 && gj <= n)) continue;
                auto hx = [&](int J) -> C {
                    if ((gi & 1) == 0) return cv(gi / 2, J);
                    return (cv((gi - 1) / 2, J) + cv((gi + 1) / 2, J)) * (C)0.5;
                };
                const C corr = ((gj & 1) == 0) ? hx(gj / 2) : (hx((gj - 1) / 2) + hx((gj + 1) / 2)) * (C)0.5;
                U[p] = T::rnd(U[p] + corr);
            }
        }
        __syncthreads();
        // ---- the red-black stages; stage m updates the points within R - m
        // of the tile (red: 1-based index sum even)
        for (int m = 1; m <= 2 * NS; ++m) {
            const int colour = (m & 1) ? 0 : 1;
            const int lim = R - m;
            for (int p = threadIdx.x; p < NP; p += kTileThreads) {
                const int x = p % NR, y = p / NR;
                const int gi = i0 + x, gj = j0 + y;
                const int d = max(max(wi.ia - gi, gi - ia1), max(wi.ja - gj, gj - ja1));
                if (!(gi >= 1 && gi <= n && gj >= 1 && gj <= n) || ((gi + gj) & 1) != colour || d > lim) continue;
                const C w = U[p - 1], e = U[p + 1], up = U[p - NR], dn = U[p + NR];
                C v;
                if constexpr (!VC) {
                    v = ((((h2 * Fv[p] + w) + e) + up) + dn) * (C)0.25;
                } else {
                    v = ((((h2 * Fv[p] + WE[p - 1] * w) + WE[p] * e) + WN[p - NR] * up) + WN[p] * dn) * ID[p];
                }
                U[p] = T::rnd(v);
            }
            __syncthreads();
        }
        if constexpr (MODE == 0) {
            // ---- residual on the tile + 1 (into Fv), then full weighting
            for (int p = threadIdx.x; p < NP; p += kTileThreads) {
                const int x = p % NR, y = p / NR;
                const int gi = i0 + x, gj = j0 + y;
                const int d = max(max(wi.ia - gi, gi - ia1), max(wi.ja - gj, gj - ja1));
                if (d > 1) continue;
                C r = (C)0;
                if (gi >= 1 && gi <= n && gj >= 1 && gj <= n) {
                    const C u = U[p], w = U[p - 1], e = U[p + 1], up = U[p - NR], dn = U[p + NR];
                    C Au;
                    if constexpr (!VC) {
                        Au = ((((u - w) + (u - e)) + (u - up)) + (u - dn)) * ih2;
                    } else {
                        Au = (((WE[p - 1] * (u - w) + WE[p] * (u - e)) + WN[p - NR] * (u - up)) + WN[p] * (u - dn)) *
                             ih2;
                    }
                    r = Fv[p] - Au;
                }
                Fv[p] = r;
            }
            __syncthreads();
            F *fc = (F *)L.fc;
            for (int q = threadIdx.x; q < (kTile / 2) * (kTile / 2); q += kTileThreads) {
                // coarse (I, J) sits on fine (2I, 2J); the tile owns it when that
                // fine point is owned (ia, ja odd, so 2I = ia + 1 + 2 qx)
                const int fi = wi.ia + 1 + 2 * (q % (kTile / 2)), fj = wi.ja + 1 + 2 * (q / (kTile / 2));
                const int I = fi / 2, J = fj / 2;
                if (I > nc || J > nc) continue;
                const int x = fi - i0, y = fj - j0;
                auto rx = [&](int yy) {
                    const int b = yy * NR + x;
                    return (Fv[b - 1] + (C)2 * Fv[b]) + Fv[b + 1];
                };
                const C v = ((rx(y - 1) + (C)2 * rx(y)) + rx(y + 1)) * (C)0.0625;
                fc[(long long)(J - 1) * cpitch + (I - 1)] = (F)v;
            }
        }
        // ---- store the owned points
        S *uout = (MODE == 0) ? (S *)L.A : (S *)L.B;
        for (int q = threadIdx.x; q < kTile * kTile; q += kTileThreads) {
            const int gi = wi.ia + q % kTile, gj = wi.ja + q / kTile;
            if (gi > n || gj > n) continue;
            const int p = (gj - j0) * NR + (gi - i0);
            T::st(uout + (long long)(gj - 1) * pitch + (gi - 1), U[p]);
        }
        __syncthreads();  // the next item reuses the LDS arrays
    }
}

template <class S, class F, bool VC, int NS>
static hipError_t tile_ns(int mode, const MarchArgs &a, int grid, hipStream_t s)
{
    if (mode == 0) hipLaunchKernelGGL((k_tile2d<S, F, VC, 0, NS>), dim3(grid), dim3(kTileThreads), 0, s, a);
    else hipLaunchKernelGGL((k_tile2d<S, F, VC, 1, NS>), dim3(grid), dim3(kTileThreads), 0, s, a);
    return hipGetLastError();
}

template <class S, class F, bool VC>
static hipError_t tile_typed(int mode, const MarchArgs &a, int NS, int grid, hipStream_t s)
{
    switch (NS) {
    case 1: return tile_ns<S, F, VC, 1>(mode, a, grid, s);
    case 2: return tile_ns<S, F, VC, 2>(mode, a, grid, s);
    default: return tile_ns<S, F, VC, 3>(mode, a, grid, s);
    }
}

hipError_t launch_tile2d(int mode, int st, bool vc, int nsweeps, const MarchArgs &a, hipStream_t s)
{
    if (a.W != kTile || a.Hb != kTile || nsweeps < 1 || 2 * nsweeps + 2 > kTileRMax) return hipErrorInvalidValue;
    const int grid = std::max(1, std::min(a.nitems, 65535));
    switch (st) {
    case ST_F64: return vc ? tile_typed<double, double, true>(mode, a, nsweeps, grid, s)
                           : tile_typed<double, double, false>(mode, a, nsweeps, grid, s);
    case ST_F32: return vc ? tile_typed<float, float, true>(mode, a, nsweeps, grid, s)
                           : tile_typed<float, float, false>(mode, a, nsweeps, grid, s);
    default: return vc ? tile_typed<bf16_t, float, true>(mode, a, nsweeps, grid, s)
                       : tile_typed<bf16_t, float, false>(mode, a, nsweeps, grid, s);
    }
}

}  // namespace mgx
