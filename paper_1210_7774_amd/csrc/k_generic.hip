// Per-point level kernels for any dimension (1, 2, 3): red-black half
// sweeps, weighted Jacobi, residual + full-weighting restriction, bilinear /
// trilinear prolongation + correction, and the FP64 residual norm with the
// device-side stop test.  They serve the 3D levels, the Jacobi smoother and
// the outer residual of iterative refinement; the 2D Gauss-Seidel levels use
// the fused row-marching kernels.
//
// Grid convention: 1-based interior index (i, j, k), x fastest, element at
// (i-1) + (j-1) pitch + (k-1) ppitch; values outside [1, n] are the Dirichlet
// zeros.  Nodal coefficients (2D) cover (n+2)^2 nodes.
#include "dev_common.h"

namespace mgx {

template <int DIM>
struct Idx {
    int n;
    long long pitch, ppitch;
    __device__ __forceinline__ long long off(int i, int j, int k) const
    {
        return (long long)(i - 1) + (DIM > 1 ? (long long)(j - 1) * pitch : 0) +
               (DIM > 2 ? (long long)(k - 1) * ppitch : 0);
    }
    __device__ __forceinline__ bool in(int i, int j, int k) const
    {
        return i >= 1 && i <= n && (DIM < 2 || (j >= 1 && j <= n)) && (DIM < 3 || (k >= 1 && k <= n));
    }
};

template <class S, int DIM>
__device__ __forceinline__ typename Traits<S>::C getu(const S *u, const Idx<DIM> &x, int i, int j, int k)
{
    using C = typename Traits<S>::C;
    if (!u || !x.in(i, j, k)) return (C)0;
    return Traits<S>::ld(u + x.off(i, j, k));
}

template <class C>
__device__ __forceinline__ C harm(C a, C b)
{
    return (C)2 * a * b / (a + b);
}

// Faces of the 2D variable-coefficient operator at node (i, j):
// west, east, south (row j-1), north (row j+1).
template <class C>
__device__ __forceinline__ void faces2d(const C *a, int n, int i, int j, C &ww, C &we, C &ws, C &wn)
{
    const long long s = n + 2;
    const C ac = a[i + s * j];
    ww = harm(ac, a[(i - 1) + s * j]);
    we = harm(ac, a[(i + 1) + s * j]);
    ws = harm(ac, a[i + s * (j - 1)]);
    wn = harm(ac, a[i + s * (j + 1)]);
}

// Gauss-Seidel point value from the current neighbours.
template <class S, class F, int DIM, bool VC>
__device__ __forceinline__ typename Traits<S>::C relax_pt(const S *u, const F *f, const typename Traits<S>::C *a,
                                                          const Idx<DIM> &x, double h2d, int i, int j, int k)
{
    using C = typename Traits<S>::C;
    const C h2 = (C)h2d;
    const C fv = (C)f[x.off(i, j, k)];
    if constexpr (!VC) {
        C s = h2 * fv;
        s = s + getu(u, x, i - 1, j, k);
        s = s + getu(u, x, i + 1, j, k);
        if (DIM > 1) {
            s = s + getu(u, x, i, j - 1, k);
            s = s + getu(u, x, i, j + 1, k);
        }
        if (DIM > 2) {
            s = s + getu(u, x, i, j, k - 1);
            s = s + getu(u, x, i, j, k + 1);
        }
        return s * (C)(DIM == 1 ? 0.5 : DIM == 2 ? 0.25 : 1.0 / 6.0);
    } else {
        C ww, we, ws, wn;
        faces2d(a, x.n, i, j, ww, we, ws, wn);
        C s = h2 * fv;
        s = s + ww * getu(u, x, i - 1, j, k);
        s = s + we * getu(u, x, i + 1, j, k);
        s = s + ws * getu(u, x, i, j - 1, k);
        s = s + wn * getu(u, x, i, j + 1, k);
        return s / (((ww + we) + ws) + wn);
    }
}

// (A u) at one point.
template <class S, int DIM, bool VC>
__device__ __forceinline__ typename Traits<S>::C apply_pt(const S *u, const typename Traits<S>::C *a,
                                                          const Idx<DIM> &x, double ih2d, int i, int j, int k)
{
    using C = typename Traits<S>::C;
    const C uc = getu(u, x, i, j, k);
    C s;
    if constexpr (!VC) {
        s = (uc - getu(u, x, i - 1, j, k)) + (uc - getu(u, x, i + 1, j, k));
        if (DIM > 1) s = (s + (uc - getu(u, x, i, j - 1, k))) + (uc - getu(u, x, i, j + 1, k));
        if (DIM > 2) s = (s + (uc - getu(u, x, i, j, k - 1))) + (uc - getu(u, x, i, j, k + 1));
    } else {
        C ww, we, ws, wn;
        faces2d(a, x.n, i, j, ww, we, ws, wn);
        s = ((ww * (uc - getu(u, x, i - 1, j, k)) + we * (uc - getu(u, x, i + 1, j, k))) +
             ws * (uc - getu(u, x, i, j - 1, k))) +
            wn * (uc - getu(u, x, i, j + 1, k));
    }
    return s * (C)ih2d;
}

__device__ __forceinline__ void coords(long long p, int n, int dim, int &i, int &j, int &k)
{
    i = (int)(p % n) + 1;
    p /= n;
    j = 1;
    k = 1;
    if (dim > 1) {
        j = (int)(p % n) + 1;
        p /= n;
    }
    if (dim > 2) k = (int)p + 1;
}

__host__ __device__ __forceinline__ long long npts(int n, int dim)
{
    long long m = n;
    if (dim > 1) m *= n;
    if (dim > 2) m *= n;
    return m;
}

// ---- red-black half sweep (in place on B; colours are disjoint) -------------
template <class S, class F, int DIM, bool VC>
__global__ __launch_bounds__(256) void k_rb_half(GenArgs g)
{
    using C = typename Traits<S>::C;
    if (g.state && g.state->done) return;
    const LevelDesc &L = g.L;
    Idx<DIM> x{L.n, L.pitch, L.ppitch};
    S *u = (S *)L.B;
    const F *f = (const F *)L.f;
    const C *a = (const C *)L.a;
    // thread p handles the pair of x-points (2m+1, 2m+2) and updates the one of the colour
    const int half = (L.n + 1) / 2;
    long long total = (long long)half * (DIM > 1 ? L.n : 1) * (DIM > 2 ? L.n : 1);
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < total;
         p += (long long)gridDim.x * blockDim.x) {
        long long t = p;
        const int m = (int)(t % half);
        t /= half;
        int j = 1, k = 1;
        if (DIM > 1) {
            j = (int)(t % L.n) + 1;
            t /= L.n;
        }
        if (DIM > 2) k = (int)t + 1;
        int i = 2 * m + 1;
        if (((i + (DIM > 1 ? j : 0) + (DIM > 2 ? k : 0)) & 1) != g.colour) i += 1;
        if (i > L.n) continue;
        C v = relax_pt<S, F, DIM, VC>(u, f, a, x, L.h2, i, j, k);
        Traits<S>::st(u + x.off(i, j, k), Traits<S>::rnd(v));
    }
}

// ---- weighted Jacobi (out of place): dst = src + omega D^-1 (f - A src) -------
template <class S, class F, int DIM, bool VC>
__global__ __launch_bounds__(256) void k_jacobi(GenArgs g)
{
    using C = typename Traits<S>::C;
    if (g.state && g.state->done) return;
    const LevelDesc &L = g.L;
    Idx<DIM> x{L.n, L.pitch, L.ppitch};
    const S *src = g.u_zero ? nullptr : (const S *)g.src;
    S *dst = (S *)g.dst;
    const F *f = (const F *)L.f;
    const C *a = (const C *)L.a;
    const long long m = npts(L.n, DIM);
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < m; p += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        coords(p, L.n, DIM, i, j, k);
        const C uc = getu(src, x, i, j, k);
        const C r = (C)f[x.off(i, j, k)] - apply_pt<S, DIM, VC>(src, a, x, L.inv_h2, i, j, k);
        C diag;
        if constexpr (!VC) {
            diag = (C)(2 * DIM) * (C)L.inv_h2;
        } else {
            C ww, we, ws, wn;
            faces2d(a, L.n, i, j, ww, we, ws, wn);
            diag = (((ww + we) + ws) + wn) * (C)L.inv_h2;
        }
        Traits<S>::st(dst + x.off(i, j, k), Traits<S>::rnd(uc + (C)g.omega * r / diag));
    }
}

// ---- residual + full weighting: fc(I) = sum_o w(o) r(2I + o) / 4^d ---------------
template <class S, class F, int DIM, bool VC>
__global__ __launch_bounds__(256) void k_resid_restrict(GenArgs g)
{
    using C = typename Traits<S>::C;
    if (g.state && g.state->done) return;
    const LevelDesc &L = g.L;
    Idx<DIM> x{L.n, L.pitch, L.ppitch};
    Idx<DIM> xc{L.nc, L.cpitch, L.cppitch};
    const S *u = (const S *)L.B;
    const F *f = (const F *)L.f;
    const C *a = (const C *)L.a;
    F *fc = (F *)L.fc;
    const long long mc = npts(L.nc, DIM);
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < mc;
         p += (long long)gridDim.x * blockDim.x) {
        int I, J, K;
        coords(p, L.nc, DIM, I, J, K);
        C s = (C)0;
        for (int oz = (DIM > 2 ? -1 : 0); oz <= (DIM > 2 ? 1 : 0); ++oz)
            for (int oy = (DIM > 1 ? -1 : 0); oy <= (DIM > 1 ? 1 : 0); ++oy)
                for (int ox = -1; ox <= 1; ++ox) {
                    const int i = 2 * I + ox, j = DIM > 1 ? 2 * J + oy : 1, k = DIM > 2 ? 2 * K + oz : 1;
                    const int wt = (2 - (ox < 0 ? -ox : ox)) * (DIM > 1 ? (2 - (oy < 0 ? -oy : oy)) : 1) *
                                   (DIM > 2 ? (2 - (oz < 0 ? -oz : oz)) : 1);
                    const C r = (C)f[x.off(i, j, k)] - apply_pt<S, DIM, VC>(u, a, x, L.inv_h2, i, j, k);
                    s = s + (C)wt * r;
                }
        fc[xc.off(I, J, K)] = (F)(s * (C)(DIM == 1 ? 0.25 : DIM == 2 ? 0.0625 : 0.015625));
    }
}

// 3D in two streaming passes: the fused form recomputes 27 fine residuals of
// 7 points each per coarse point.  Pass 1 writes r = f - A u (compute type,
// contiguous) into the level's spare state buffer A; pass 2 applies the
// same weights in the same order, so the coarse values are unchanged.
template <class S, class F, int DIM, bool VC>
__global__ __launch_bounds__(256) void k_residual_to_a(GenArgs g)
{
    using C = typename Traits<S>::C;
    if (g.state && g.state->done) return;
    const LevelDesc &L = g.L;
    Idx<DIM> x{L.n, L.pitch, L.ppitch};
    const S *u = (const S *)L.B;
    const F *f = (const F *)L.f;
    const C *a = (const C *)L.a;
    C *r = (C *)L.A;
    const long long m = npts(L.n, DIM);
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < m; p += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        coords(p, L.n, DIM, i, j, k);
        r[p] = (C)f[x.off(i, j, k)] - apply_pt<S, DIM, VC>(u, a, x, L.inv_h2, i, j, k);
    }
}

// 3D pass 1 as column marches (the vertical neighbours stay in registers)
template <class S, class F>
__global__ __launch_bounds__(256) void k_residual_to_a3(GenArgs g)
{
    using T = Traits<S>;
    using C = typename T::C;
    if (g.state && g.state->done) return;
    const LevelDesc &L = g.L;
    Idx<3> x{L.n, L.pitch, L.ppitch};
    const int n = L.n;
    const S *u = (const S *)L.B;
    const F *f = (const F *)L.f;
    C *r = (C *)L.A;
    const C ih2 = (C)L.inv_h2;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int ntx = (n + 63) / 64, nty = (n + 3) / 4, ntz = (n + 31) / 32;
    const long long nunits = (long long)ntx * nty * ntz;
    auto U = [&](int i, int j, int k) -> C {
        return (i >= 1 && i <= n && j >= 1 && j <= n && k >= 1 && k <= n) ? (C)T::ld(u + x.off(i, j, k)) : (C)0;
    };
    for (long long un = blockIdx.x; un < nunits; un += gridDim.x) {
        const int i = (int)(un % ntx) * 64 + tx + 1, j = (int)((un / ntx) % nty) * 4 + ty + 1;
        const int k0 = (int)(un / ((long long)ntx * nty)) * 32 + 1, k1 = min(k0 + 32, n + 1);
        if (i > n || j > n) continue;
        C dn = U(i, j, k0 - 1), c = U(i, j, k0);
#pragma unroll 4
        for (int k = k0; k < k1; ++k) {
            const C up = U(i, j, k + 1);
            C sa = (c - U(i - 1, j, k)) + (c - U(i + 1, j, k));
            sa = (sa + (c - U(i, j - 1, k))) + (c - U(i, j + 1, k));
            sa = (sa + (c - dn)) + (c - up);
            r[(long long)(i - 1) + (long long)n * ((j - 1) + (long long)n * (k - 1))] =
                (C)f[x.off(i, j, k)] - sa * ih2;
            dn = c;
            c = up;
        }
    }
}

template <class S, class F, int DIM>
__global__ __launch_bounds__(256) void k_restrict_from_a(GenArgs g)
{
    using C = typename Traits<S>::C;
    if (g.state && g.state->done) return;
    const LevelDesc &L = g.L;
    Idx<DIM> xc{L.nc, L.cpitch, L.cppitch};
    const C *r = (const C *)L.A;
    F *fc = (F *)L.fc;
    const int n = L.n;
    const long long mc = npts(L.nc, DIM);
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < mc;
         p += (long long)gridDim.x * blockDim.x) {
        int I, J, K;
        coords(p, L.nc, DIM, I, J, K);
        C s = (C)0;
        for (int oz = (DIM > 2 ? -1 : 0); oz <= (DIM > 2 ? 1 : 0); ++oz)
            for (int oy = (DIM > 1 ? -1 : 0); oy <= (DIM > 1 ? 1 : 0); ++oy)
                for (int ox = -1; ox <= 1; ++ox) {
                    const int i = 2 * I + ox, j = DIM > 1 ? 2 * J + oy : 1, k = DIM > 2 ? 2 * K + oz : 1;
                    const int wt = (2 - (ox < 0 ? -ox : ox)) * (DIM > 1 ? (2 - (oy < 0 ? -oy : oy)) : 1) *
                                   (DIM > 2 ? (2 - (oz < 0 ? -oz : oz)) : 1);
                    const C rv = r[(long long)(i - 1) + (long long)n * ((j - 1) + (long long)n * (k - 1))];
                    s = s + (C)wt * rv;
                }
        fc[xc.off(I, J, K)] = (F)(s * (C)(DIM == 1 ? 0.25 : DIM == 2 ? 0.0625 : 0.015625));
    }
}

// 3D prolongation + correction as column marches: a thread keeps the
// bilinear (x, y) interpolation of the coarse planes K and K + 1 of its column
// in registers, so each coarse plane is interpolated once per fine column
// instead of once per fine point; the interpolation order is the generic
// kernel's (x, then y, then z)
template <class S>
__global__ __launch_bounds__(256) void k_prolong_correct3(GenArgs g)
{
    using T = Traits<S>;
    using C = typename T::C;
    if (g.state && g.state->done) return;
    const LevelDesc &L = g.L;
    Idx<3> x{L.n, L.pitch, L.ppitch};
    Idx<3> xc{L.nc, L.cpitch, L.cppitch};
    const int n = L.n;
    S *u = (S *)L.B;
    const S *uc = (const S *)L.Bc;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int ntx = (n + 63) / 64, nty = (n + 3) / 4, ntz = (n + 31) / 32;
    const long long nunits = (long long)ntx * nty * ntz;
    for (long long un = blockIdx.x; un < nunits; un += gridDim.x) {
        const int i = (int)(un % ntx) * 64 + tx + 1, j = (int)((un / ntx) % nty) * 4 + ty + 1;
        const int k0 = (int)(un / ((long long)ntx * nty)) * 32 + 1, k1 = min(k0 + 32, n + 1);
        if (i > n || j > n) continue;
        const int i0 = i / 2, i1 = (i & 1) ? i0 + 1 : i0;
        const int j0 = j / 2, j1 = (j & 1) ? j0 + 1 : j0;
        auto plane = [&](int kk) -> C {
            auto line = [&](int jj) -> C {
                const C a0 = getu(uc, xc, i0, jj, kk);
                return (i & 1) ? (a0 + getu(uc, xc, i1, jj, kk)) * (C)0.5 : a0;
            };
            const C b0 = line(j0);
            return (j & 1) ? (b0 + line(j1)) * (C)0.5 : b0;
        };
        int K = k0 / 2;
        C pk = plane(K), pk1 = plane(K + 1);
        for (int k = k0; k < k1; ++k) {
            if (k / 2 != K) {  // advance one coarse plane
                K = k / 2;
                pk = pk1;
                pk1 = plane(K + 1);
            }
            const C corr = (k & 1) ? (pk + pk1) * (C)0.5 : pk;
            S *p = u + x.off(i, j, k);
            T::st(p, T::rnd((C)T::ld(p) + corr));
        }
    }
}

// ---- prolongation + correction: B += P Bc ------------------------------------
template <class S, int DIM>
__global__ __launch_bounds__(256) void k_prolong_correct(GenArgs g)
{
    using C = typename Traits<S>::C;
    if (g.state && g.state->done) return;
    const LevelDesc &L = g.L;
    Idx<DIM> x{L.n, L.pitch, L.ppitch};
    Idx<DIM> xc{L.nc, L.cpitch, L.cppitch};
    S *u = (S *)L.B;
    const S *uc = (const S *)L.Bc;
    const long long m = npts(L.n, DIM);
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < m; p += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        coords(p, L.n, DIM, i, j, k);
        // parents along each axis: even index -> one parent (weight 1), odd -> two (1/2 each)
        const int i0 = i / 2, i1 = (i & 1) ? i0 + 1 : i0;
        const int j0 = j / 2, j1 = (j & 1) ? j0 + 1 : j0;
        const int k0 = k / 2, k1 = (k & 1) ? k0 + 1 : k0;
        auto line = [&](int jj, int kk) -> C {
            const C a0 = getu(uc, xc, i0, jj, kk);
            return (i & 1) ? (a0 + getu(uc, xc, i1, jj, kk)) * (C)0.5 : a0;
        };
        auto plane = [&](int kk) -> C {
            if (DIM < 2) return line(1, kk);
            const C b0 = line(j0, kk);
            return (j & 1) ? (b0 + line(j1, kk)) * (C)0.5 : b0;
        };
        C corr;
        if (DIM < 3) {
            corr = plane(1);
        } else {
            const C c0 = plane(k0);
            corr = (k & 1) ? (c0 + plane(k1)) * (C)0.5 : c0;
        }
        S *pu = u + x.off(i, j, k);
        Traits<S>::st(pu, Traits<S>::rnd(Traits<S>::ld(pu) + corr));
    }
}

// ---- full multigrid: fc = R f (the rhs carried down by full weighting) -------
template <class F, int DIM>
__global__ __launch_bounds__(256) void k_restrict_rhs(GenArgs g)
{
    if (g.state && g.state->done) return;
    const LevelDesc &L = g.L;
    Idx<DIM> x{L.n, L.pitch, L.ppitch};
    Idx<DIM> xc{L.nc, L.cpitch, L.cppitch};
    const F *f = (const F *)L.f;
    F *fc = (F *)L.fc;
    const long long mc = npts(L.nc, DIM);
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < mc;
         p += (long long)gridDim.x * blockDim.x) {
        int I, J, K;
        coords(p, L.nc, DIM, I, J, K);
        F s = (F)0;
        for (int oz = (DIM > 2 ? -1 : 0); oz <= (DIM > 2 ? 1 : 0); ++oz)
            for (int oy = (DIM > 1 ? -1 : 0); oy <= (DIM > 1 ? 1 : 0); ++oy)
                for (int ox = -1; ox <= 1; ++ox) {
                    const int i = 2 * I + ox, j = DIM > 1 ? 2 * J + oy : 1, k = DIM > 2 ? 2 * K + oz : 1;
                    const int wt = (2 - (ox < 0 ? -ox : ox)) * (DIM > 1 ? (2 - (oy < 0 ? -oy : oy)) : 1) *
                                   (DIM > 2 ? (2 - (oz < 0 ? -oz : oz)) : 1);
                    s = s + (F)wt * f[x.off(i, j, k)];
                }
        fc[xc.off(I, J, K)] = s * (F)(DIM == 1 ? 0.25 : DIM == 2 ? 0.0625 : 0.015625);
    }
}

// ---- full multigrid: B = P Bc (the coarse solution interpolated) ---------------
template <class S, int DIM>
__global__ __launch_bounds__(256) void k_interp(GenArgs g)
{
    using C = typename Traits<S>::C;
    if (g.state && g.state->done) return;
    const LevelDesc &L = g.L;
    Idx<DIM> x{L.n, L.pitch, L.ppitch};
    Idx<DIM> xc{L.nc, L.cpitch, L.cppitch};
    S *u = (S *)L.B;
    const S *uc = (const S *)L.Bc;
    const long long m = npts(L.n, DIM);
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < m; p += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        coords(p, L.n, DIM, i, j, k);
        const int i0 = i / 2, i1 = (i & 1) ? i0 + 1 : i0;
        const int j0 = j / 2, j1 = (j & 1) ? j0 + 1 : j0;
        const int k0 = k / 2, k1 = (k & 1) ? k0 + 1 : k0;
        auto line = [&](int jj, int kk) -> C {
            const C a0 = getu(uc, xc, i0, jj, kk);
            return (i & 1) ? (a0 + getu(uc, xc, i1, jj, kk)) * (C)0.5 : a0;
        };
        auto plane = [&](int kk) -> C {
            if (DIM < 2) return line(1, kk);
            const C b0 = line(j0, kk);
            return (j & 1) ? (b0 + line(j1, kk)) * (C)0.5 : b0;
        };
        C v;
        if (DIM < 3) {
            v = plane(1);
        } else {
            const C c0 = plane(k0);
            v = (k & 1) ? (c0 + plane(k1)) * (C)0.5 : c0;
        }
        Traits<S>::st(u + x.off(i, j, k), Traits<S>::rnd(v));
    }
}

__global__ void k_fill_zero(uint32_t *p, long long nwords)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < nwords; q += (long long)gridDim.x * blockDim.x)
        p[q] = 0u;
}

template <class S, int DIM>
__global__ __launch_bounds__(256) void k_copy_state(GenArgs g, const S *src, S *dst)
{
    if (g.state && g.state->done) return;
    const LevelDesc &L = g.L;
    Idx<DIM> x{L.n, L.pitch, L.ppitch};
    const long long m = npts(L.n, DIM);
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < m; p += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        coords(p, L.n, DIM, i, j, k);
        dst[x.off(i, j, k)] = src[x.off(i, j, k)];
    }
}

// ---- FP64 residual norm (+ optional r32 / r64 output) and stop test ------------
template <int DIM, bool VC>
__global__ __launch_bounds__(256) void k_norm(NormArgs g)
{
    if (!g.first && g.state->done) return;
    Idx<DIM> x{g.n, g.pitch, g.ppitch};
    // (the finish kernel that follows reduces the block partials)
    const long long m = npts(g.n, DIM);
    double rr = 0.0, ff = 0.0;
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < m; p += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        coords(p, g.n, DIM, i, j, k);
        const long long o = x.off(i, j, k);
        const double fv = g.f[o];
        const double r = fv - apply_pt<double, DIM, VC>(g.u, g.a, x, g.inv_h2, i, j, k);
        rr += r * r;
        ff += fv * fv;
        // contiguous interior outputs
        if (g.r32) g.r32[p] = (float)r;
        if (g.r64) g.r64[p] = r;
    }
    __shared__ double srr[4], sff[4];
    rr = wave_sum(rr);
    ff = wave_sum(ff);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        srr[w] = rr;
        sff[w] = ff;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        double a = 0.0, b = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
            a += srr[q];
            b += sff[q];
        }
        put_partial(g.partials, blockIdx.x, a, b);
    }
}

// ---- 3D FP64 residual norm: each thread marches one column up a run of 32
// planes keeping u(k - 1), u(k), u(k + 1) in registers, so every array is
// streamed once (the in-plane neighbours come from the cache); work units of
// 64 x 4 columns x 32 planes are dealt to the blocks in a fixed order
template <int RUN>
__global__ __launch_bounds__(256) void k_norm3(NormArgs g)
{
    if (!g.first && g.state->done) return;
    Idx<3> x{g.n, g.pitch, g.ppitch};
    const int n = g.n;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int ntx = (n + 63) / 64, nty = (n + 3) / 4, ntz = (n + RUN - 1) / RUN;
    const long long nunits = (long long)ntx * nty * ntz;
    const double ih2 = g.inv_h2;
    const double *u = g.u;
    double rr = 0.0, ff = 0.0;
    auto U = [&](int i, int j, int k) -> double {
        return (u && i >= 1 && i <= n && j >= 1 && j <= n && k >= 1 && k <= n) ? u[x.off(i, j, k)] : 0.0;
    };
    for (long long un = blockIdx.x; un < nunits; un += gridDim.x) {
        const int i = (int)(un % ntx) * 64 + tx + 1, j = (int)((un / ntx) % nty) * 4 + ty + 1;
        const int k0 = (int)(un / ((long long)ntx * nty)) * RUN + 1, k1 = min(k0 + RUN, n + 1);
        if (i > n || j > n) continue;
        double dn = U(i, j, k0 - 1), c = U(i, j, k0);
#pragma unroll 4
        for (int k = k0; k < k1; ++k) {
            const double up = U(i, j, k + 1);
            const long long o = x.off(i, j, k);
            const double fv = g.f[o];
            double sa = (c - U(i - 1, j, k)) + (c - U(i + 1, j, k));
            sa = (sa + (c - U(i, j - 1, k))) + (c - U(i, j + 1, k));
            sa = (sa + (c - dn)) + (c - up);
            const double r = fv - sa * ih2;
            rr += r * r;
            ff += fv * fv;
            const long long pc = (long long)(i - 1) + (long long)n * ((j - 1) + (long long)n * (k - 1));
            if (g.r32) g.r32[pc] = (float)r;
            if (g.r64) g.r64[pc] = r;
            dn = c;
            c = up;
        }
    }
    __shared__ double srr[4], sff[4];
    rr = wave_sum(rr);
    ff = wave_sum(ff);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        srr[w] = rr;
        sff[w] = ff;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        double a = 0.0, b = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
            a += srr[q];
            b += sff[q];
        }
        put_partial(g.partials, blockIdx.x, a, b);
    }
}

// ---- batched FP64 residual (2D), one block per chunk of rows of one system ----
__global__ __launch_bounds__(256) void k_norm_batch(const NormItem *items, const NormSys *sys, SolveState *states,
                                                    double *partials, int flags)
{
    const NormItem it = items[blockIdx.x];
    const NormSys S = sys[it.sys];
    const int first = flags & 1;
    if (!first && states[it.sys].done) return;
    Idx<2> x{S.n, S.pitch, 0};
    double rr = 0.0, ff = 0.0;
    const long long cnt = (long long)(it.j1 - it.j0) * S.n;
    for (long long q = threadIdx.x; q < cnt; q += blockDim.x) {
        const int i = (int)(q % S.n) + 1, j = it.j0 + (int)(q / S.n);
        const long long o = x.off(i, j, 1);
        const double fv = S.f[o];
        const double au = S.a ? apply_pt<double, 2, true>(S.u, S.a, x, S.inv_h2, i, j, 1)
                              : apply_pt<double, 2, false>(S.u, S.a, x, S.inv_h2, i, j, 1);
        const double r = fv - au;
        rr += r * r;
        ff += fv * fv;
        if (flags & 2) S.r32[(long long)(j - 1) * S.n + (i - 1)] = (float)r;
    }
    __shared__ double srr[4], sff[4];
    rr = wave_sum(rr);
    ff = wave_sum(ff);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        srr[w] = rr;
        sff[w] = ff;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        double a = 0.0, b = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
            a += srr[q];
            b += sff[q];
        }
        put_partial(partials, it.slot, a, b);
    }
}

hipError_t launch_norm_batch(const NormItem *items, int nitems, const NormSys *sys, SolveState *states,
                             double *partials, int flags, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_norm_batch, dim3(nitems), dim3(256), 0, s, items, sys, states, partials, flags);
    return hipGetLastError();
}

// ---- reduction of the partial sums + stop test: one wavefront per system ----
// part0 / nparts: per-system slot ranges (device), or null for one system
// whose slots are [slot0, slot0 + nslots).
__global__ __launch_bounds__(64) void k_norm_finish(SolveState *states, const double *partials, const int *part0,
                                                    const int *nparts, int slot0, int nslots, int first)
{
    const int sys = blockIdx.x;
    SolveState *st = states + sys;
    if (!first && st->done) return;
    const int lane = threadIdx.x;
    const int p0 = part0 ? part0[sys] : slot0;
    const int np = nparts ? nparts[sys] : nslots;
    double srr = 0.0, sff = 0.0;
    // eight loads in flight per lane; the sums keep the order k, k + 64, ...
    for (int k0 = lane; k0 < np; k0 += 64 * 8) {
        double vr[8], vf[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = k0 + 64 * j;
            const int kk = k < np ? k : k0;
            vr[j] = partials[2 * (p0 + kk)];
            vf[j] = partials[2 * (p0 + kk) + 1];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (k0 + 64 * j < np) {
                srr += vr[j];
                sff += vf[j];
            }
        }
    }
    srr = wave_sum(srr);
    sff = wave_sum(sff);
    if (lane != 0) return;
    if (first) {
        st->ff = sff;
        st->nres = 0;
    }
    const double rel = sqrt(srr) / sqrt(st->ff);
    const int k = st->nres;
    if (k <= 200) st->hist[k] = rel;
    st->rel = rel;
    st->nres = k + 1;
    int done = 0;
    if (!isfinite(rel)) done = 2;
    else if (rel <= st->tol) done = 1;
    else if (k >= 1 && st->watch > 0.0 && !(rel <= st->watch * st->hist[k - 1])) done = 4;
    else if (k <= 200) {
        const int rule = history_rule(st->hist, k + 1, st->stall);
        if (rule == 2) done = 6;
        else if (rule == 1) done = 5;
    }
    if (done == 0 && k >= st->maxc) done = 3;
    st->done = done;
}

hipError_t launch_norm_finish(SolveState *states, int nsys, const double *partials, const int *part0,
                              const int *nparts, int slot0, int nslots, int first, hipStream_t s)
{
    hipLaunchKernelGGL(k_norm_finish, dim3(nsys), dim3(64), 0, s, states, partials, part0, nparts, slot0, nslots,
                       first);
    return hipGetLastError();
}

// ---- FP64 correction u += e (state type S) -----------------------------------
template <class S>
__global__ __launch_bounds__(256) void k_ir_correct(double *u, long long pitch, long long ppitch, const S *e,
                                                    int n, int dim, SolveState *st)
{
    if (st && st->done) return;
    const long long m = npts(n, dim);
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < m; p += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        coords(p, n, dim, i, j, k);
        const long long o = (long long)(i - 1) + (long long)(j - 1) * pitch + (long long)(k - 1) * ppitch;
        u[o] = u[o] + (double)Traits<S>::ld(e + p);
    }
}

// ---- setup: nodal coefficient hierarchy by injection ---------------------------
// Injection composes, so level l takes node (2^l I, 2^l J) of the finest array.
__global__ void k_coef_inject(const double *af, int nf, void *ac, int ncn, int stride, int as_float)
{
    const long long s = ncn + 2;
    const long long m = s * s;
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < m; p += (long long)gridDim.x * blockDim.x) {
        const int I = (int)(p % s), J = (int)(p / s);
        const double v = af[(long long)stride * I + (long long)(nf + 2) * ((long long)stride * J)];
        if (as_float) ((float *)ac)[p] = (float)v;
        else ((double *)ac)[p] = v;
    }
}

__global__ void k_coef_check(const double *a, long long m, int *bad)
{
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < m; p += (long long)gridDim.x * blockDim.x) {
        const double v = a[p];
        if (!(v > 0.0) || !isfinite(v)) atomicOr(bad, 1);
    }
}

// ---- s = D^-1 (f - A u) in FP64 (2D; a null = Poisson) --------------------------
__global__ __launch_bounds__(256) void k_scaled_residual64(const double *u, const double *f, const double *a, int n,
                                                           long long pitch, double *s)
{
    Idx<2> x{n, pitch, 0};
    const double ih2 = (double)(n + 1) * (n + 1);
    const long long m = (long long)n * n;
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < m; p += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(p % n) + 1, j = (int)(p / n) + 1;
        const long long o = x.off(i, j, 1);
        double r, dsum;
        if (a) {
            r = f[o] - apply_pt<double, 2, true>(u, a, x, ih2, i, j, 1);
            double ww, we, ws, wn;
            faces2d(a, n, i, j, ww, we, ws, wn);
            dsum = (((ww + we) + ws) + wn) * ih2;
        } else {
            r = f[o] - apply_pt<double, 2, false>(u, a, x, ih2, i, j, 1);
            dsum = 4.0 * ih2;
        }
        s[p] = r / dsum;
    }
}

hipError_t launch_scaled_residual64(const double *u, const double *f, const double *a, int n, long long pitch,
                                    double *s, hipStream_t st)
{
    const long long m = (long long)n * n;
    hipLaunchKernelGGL(k_scaled_residual64, dim3((int)std::min<long long>((m + 255) / 256, 65536)), dim3(256), 0, st,
                       u, f, a, n, pitch, s);
    return hipGetLastError();
}

// ---- launchers ---------------------------------------------------------------
static int grid_for(long long work, int block = 256)
{
    long long g = (work + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (int)g;
}

template <class S, class F, bool VC>
static hipError_t rb_dim(const GenArgs &g, hipStream_t s)
{
    const long long half = (g.L.n + 1) / 2;
    const long long work = half * (g.L.dim > 1 ? g.L.n : 1) * (g.L.dim > 2 ? g.L.n : 1);
    const int grid = grid_for(work);
    switch (g.L.dim) {
    case 1: hipLaunchKernelGGL((k_rb_half<S, F, 1, false>), dim3(grid), dim3(256), 0, s, g); break;
    case 2: hipLaunchKernelGGL((k_rb_half<S, F, 2, VC>), dim3(grid), dim3(256), 0, s, g); break;
    case 3: hipLaunchKernelGGL((k_rb_half<S, F, 3, false>), dim3(grid), dim3(256), 0, s, g); break;
    }
    return hipGetLastError();
}

hipError_t launch_rb_half(int st, bool vc, const GenArgs &g, hipStream_t s)
{
    switch (st) {
    case ST_F64: return vc ? rb_dim<double, double, true>(g, s) : rb_dim<double, double, false>(g, s);
    case ST_F32: return vc ? rb_dim<float, float, true>(g, s) : rb_dim<float, float, false>(g, s);
    case ST_BF16: return vc ? rb_dim<bf16_t, float, true>(g, s) : rb_dim<bf16_t, float, false>(g, s);
    }
    return hipErrorInvalidValue;
}

template <class S, class F, bool VC>
static hipError_t jac_dim(const GenArgs &g, hipStream_t s)
{
    const int grid = grid_for(npts(g.L.n, g.L.dim));
    switch (g.L.dim) {
    case 1: hipLaunchKernelGGL((k_jacobi<S, F, 1, false>), dim3(grid), dim3(256), 0, s, g); break;
    case 2: hipLaunchKernelGGL((k_jacobi<S, F, 2, VC>), dim3(grid), dim3(256), 0, s, g); break;
    case 3: hipLaunchKernelGGL((k_jacobi<S, F, 3, false>), dim3(grid), dim3(256), 0, s, g); break;
    }
    return hipGetLastError();
}

hipError_t launch_jacobi(int st, bool vc, const GenArgs &g, hipStream_t s)
{
    switch (st) {
    case ST_F64: return vc ? jac_dim<double, double, true>(g, s) : jac_dim<double, double, false>(g, s);
    case ST_F32: return vc ? jac_dim<float, float, true>(g, s) : jac_dim<float, float, false>(g, s);
    case ST_BF16: return vc ? jac_dim<bf16_t, float, true>(g, s) : jac_dim<bf16_t, float, false>(g, s);
    }
    return hipErrorInvalidValue;
}

template <class S, class F, bool VC>
static hipError_t rr_dim(const GenArgs &g, hipStream_t s)
{
    const int grid = grid_for(npts(g.L.nc, g.L.dim));
    switch (g.L.dim) {
    case 1: hipLaunchKernelGGL((k_resid_restrict<S, F, 1, false>), dim3(grid), dim3(256), 0, s, g); break;
    case 2: hipLaunchKernelGGL((k_resid_restrict<S, F, 2, VC>), dim3(grid), dim3(256), 0, s, g); break;
    case 3:
        hipLaunchKernelGGL((k_residual_to_a3<S, F>), dim3(grid_for(((long long)(g.L.n + 63) / 64) * ((g.L.n + 3) / 4) *
                                                               ((g.L.n + 31) / 32) * 256)),
                           dim3(256), 0, s, g);
        hipLaunchKernelGGL((k_restrict_from_a<S, F, 3>), dim3(grid), dim3(256), 0, s, g);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_resid_restrict(int st, bool vc, const GenArgs &g, hipStream_t s)
{
    switch (st) {
    case ST_F64: return vc ? rr_dim<double, double, true>(g, s) : rr_dim<double, double, false>(g, s);
    case ST_F32: return vc ? rr_dim<float, float, true>(g, s) : rr_dim<float, float, false>(g, s);
    case ST_BF16: return vc ? rr_dim<bf16_t, float, true>(g, s) : rr_dim<bf16_t, float, false>(g, s);
    }
    return hipErrorInvalidValue;
}

template <class S>
static hipError_t pc_dim(const GenArgs &g, hipStream_t s)
{
    const int grid = grid_for(npts(g.L.n, g.L.dim));
    switch (g.L.dim) {
    case 1: hipLaunchKernelGGL((k_prolong_correct<S, 1>), dim3(grid), dim3(256), 0, s, g); break;
    case 2: hipLaunchKernelGGL((k_prolong_correct<S, 2>), dim3(grid), dim3(256), 0, s, g); break;
    case 3:
        hipLaunchKernelGGL((k_prolong_correct3<S>), dim3(grid_for(((long long)(g.L.n + 63) / 64) * ((g.L.n + 3) / 4) *
                                                                ((g.L.n + 31) / 32) * 256)),
                           dim3(256), 0, s, g);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_prolong_correct(int st, const GenArgs &g, hipStream_t s)
{
    switch (st) {
    case ST_F64: return pc_dim<double>(g, s);
    case ST_F32: return pc_dim<float>(g, s);
    case ST_BF16: return pc_dim<bf16_t>(g, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_restrict_rhs(int st, const GenArgs &g, hipStream_t s)
{
    const int grid = grid_for(npts(g.L.nc, g.L.dim));
#define MGX_RR(F)                                                                                   \
    switch (g.L.dim) {                                                                              \
    case 1: hipLaunchKernelGGL((k_restrict_rhs<F, 1>), dim3(grid), dim3(256), 0, s, g); break;      \
    case 2: hipLaunchKernelGGL((k_restrict_rhs<F, 2>), dim3(grid), dim3(256), 0, s, g); break;      \
    case 3: hipLaunchKernelGGL((k_restrict_rhs<F, 3>), dim3(grid), dim3(256), 0, s, g); break;      \
    }
    if (st == ST_F64) { MGX_RR(double) } else { MGX_RR(float) }
#undef MGX_RR
    return hipGetLastError();
}

hipError_t launch_interp(int st, const GenArgs &g, hipStream_t s)
{
    const int grid = grid_for(npts(g.L.n, g.L.dim));
#define MGX_IP(S)                                                                              \
    switch (g.L.dim) {                                                                         \
    case 1: hipLaunchKernelGGL((k_interp<S, 1>), dim3(grid), dim3(256), 0, s, g); break;       \
    case 2: hipLaunchKernelGGL((k_interp<S, 2>), dim3(grid), dim3(256), 0, s, g); break;       \
    case 3: hipLaunchKernelGGL((k_interp<S, 3>), dim3(grid), dim3(256), 0, s, g); break;       \
    }
    switch (st) {
    case ST_F64: MGX_IP(double) break;
    case ST_F32: MGX_IP(float) break;
    case ST_BF16: MGX_IP(bf16_t) break;
    }
#undef MGX_IP
    return hipGetLastError();
}

hipError_t launch_fill_zero(void *p, long long bytes, hipStream_t s)
{
    const long long nw = bytes / 4;
    hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(nw)), dim3(256), 0, s, (uint32_t *)p, nw);
    return hipGetLastError();
}

hipError_t launch_copy_state(int st, const GenArgs &g, const void *src, void *dst, hipStream_t s)
{
    const int grid = grid_for(npts(g.L.n, g.L.dim));
#define MGX_COPY(S)                                                                                                   \
    switch (g.L.dim) {                                                                                                \
    case 1: hipLaunchKernelGGL((k_copy_state<S, 1>), dim3(grid), dim3(256), 0, s, g, (const S *)src, (S *)dst); break; \
    case 2: hipLaunchKernelGGL((k_copy_state<S, 2>), dim3(grid), dim3(256), 0, s, g, (const S *)src, (S *)dst); break; \
    case 3: hipLaunchKernelGGL((k_copy_state<S, 3>), dim3(grid), dim3(256), 0, s, g, (const S *)src, (S *)dst); break; \
    }
    switch (st) {
    case ST_F64: MGX_COPY(double) break;
    case ST_F32: MGX_COPY(float) break;
    case ST_BF16: MGX_COPY(bf16_t) break;
    }
#undef MGX_COPY
    return hipGetLastError();
}

hipError_t launch_norm(const NormArgs &a, hipStream_t s)
{
    const int grid = a.nblocks;
    const bool vc = a.a != nullptr;
    switch (a.dim) {
    case 1: hipLaunchKernelGGL((k_norm<1, false>), dim3(grid), dim3(256), 0, s, a); break;
    case 2:
        if (vc) hipLaunchKernelGGL((k_norm<2, true>), dim3(grid), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_norm<2, false>), dim3(grid), dim3(256), 0, s, a);
        break;
    case 3: hipLaunchKernelGGL((k_norm3<32>), dim3(grid), dim3(256), 0, s, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_ir_correct(int st, double *u, long long pitch, long long ppitch, const void *e, int n, int dim,
                             SolveState *state, hipStream_t s)
{
    const int grid = grid_for(npts(n, dim));
    switch (st) {
    case ST_F64: hipLaunchKernelGGL((k_ir_correct<double>), dim3(grid), dim3(256), 0, s, u, pitch, ppitch, (const double *)e, n, dim, state); break;
    case ST_F32: hipLaunchKernelGGL((k_ir_correct<float>), dim3(grid), dim3(256), 0, s, u, pitch, ppitch, (const float *)e, n, dim, state); break;
    case ST_BF16: hipLaunchKernelGGL((k_ir_correct<bf16_t>), dim3(grid), dim3(256), 0, s, u, pitch, ppitch, (const bf16_t *)e, n, dim, state); break;
    }
    return hipGetLastError();
}

hipError_t launch_coef_inject(const double *af, int nf, void *ac, int ncn, int stride, int as_float, hipStream_t s)
{
    const long long m = (long long)(ncn + 2) * (ncn + 2);
    hipLaunchKernelGGL(k_coef_inject, dim3(grid_for(m)), dim3(256), 0, s, af, nf, ac, ncn, stride, as_float);
    return hipGetLastError();
}

hipError_t launch_coef_check(const double *a, long long count, int *bad, hipStream_t s)
{
    hipLaunchKernelGGL(k_coef_check, dim3(grid_for(count)), dim3(256), 0, s, a, count, bad);
    return hipGetLastError();
}

}  // namespace mgx
