// Coarse-level tail of the V-cycle: one workgroup per system runs every level
// from the tail's top level down to the coarsest and back up, entirely in LDS:
//   down:  nu1 smoothing sweeps, residual + full-weighting restriction
//   bottom: x = A_c^-1 f_c in FP64 with the host-computed inverse
//   up:    bilinear/trilinear prolongation + correction, nu2 sweeps
// It reads the top level's rhs and writes its final state.  These levels are
// far too small to fill the GPU, so they run back to back in one launch
// instead of a dozen latency-bound ones.
#include "dev_common.h"

namespace mgx {

static constexpr int kTailMaxLevels = 12;
// 160 KB of LDS per workgroup minus the staged level descriptors
static constexpr int kTailMaxDynLds = 160 * 1024 - 8192;  // static LDS: descriptors, coarsest inverse

template <int DIM>
struct LIdx {
    int n;
    __device__ __forceinline__ int off(int i, int j, int k) const
    {
        return (i - 1) + (DIM > 1 ? (j - 1) * n : 0) + (DIM > 2 ? (k - 1) * n * n : 0);
    }
    __device__ __forceinline__ bool in(int i, int j, int k) const
    {
        return i >= 1 && i <= n && (DIM < 2 || (j >= 1 && j <= n)) && (DIM < 3 || (k >= 1 && k <= n));
    }
    __device__ __forceinline__ int npts() const { return n * (DIM > 1 ? n : 1) * (DIM > 2 ? n : 1); }
    __device__ __forceinline__ void coords(int p, int &i, int &j, int &k) const
    {
        i = p % n + 1;
        p /= n;
        j = 1;
        k = 1;
        if (DIM > 1) {
            j = p % n + 1;
            p /= n;
        }
        if (DIM > 2) k = p + 1;
    }
};

// Visit every interior point of an n^DIM level without integer division:
// 2D levels have n <= 63 (64 threads per row), 3D levels n <= 15 (16 x 16
// threads per plane); 1D levels stride by the block size.
template <int DIM, class Fn>
__device__ __forceinline__ void for_points(int n, int tid, int nt, Fn &&fn)
{
    if constexpr (DIM == 1) {
        for (int i = tid + 1; i <= n; i += nt) fn(i, 1, 1, i - 1);
    } else if constexpr (DIM == 2) {
        const int i = (tid & 63) + 1;
        if (i > n) return;
        for (int j = (tid >> 6) + 1; j <= n; j += nt >> 6) fn(i, j, 1, (i - 1) + (j - 1) * n);
    } else {
        const int i = (tid & 15) + 1, j = ((tid >> 4) & 15) + 1;
        if (i > n || j > n) return;
        for (int k = (tid >> 8) + 1; k <= n; k += nt >> 8) fn(i, j, k, (i - 1) + (j - 1) * n + (k - 1) * n * n);
    }
}

template <class C, int DIM>
__device__ __forceinline__ C lget(const C *u, const LIdx<DIM> &x, int i, int j, int k)
{
    return x.in(i, j, k) ? u[x.off(i, j, k)] : (C)0;
}

template <class C>
__device__ __forceinline__ C tharm(C a, C b)
{
    return (C)2 * a * b / (a + b);
}

template <class C, int DIM, bool VC>
__device__ __forceinline__ void tfaces(const C *a, int n, int i, int j, C &ww, C &we, C &ws, C &wn)
{
    if constexpr (VC) {
        const int s = n + 2;
        const C ac = a[i + s * j];
        ww = tharm(ac, a[(i - 1) + s * j]);
        we = tharm(ac, a[(i + 1) + s * j]);
        ws = tharm(ac, a[i + s * (j - 1)]);
        wn = tharm(ac, a[i + s * (j + 1)]);
    } else {
        ww = we = ws = wn = (C)1;
    }
}

template <class C, int DIM, bool VC>
__device__ __forceinline__ C t_relax(const C *u, const C *f, const C *a, const LIdx<DIM> &x, C h2, int i, int j, int k)
{
    const C fv = f[x.off(i, j, k)];
    if constexpr (!VC) {
        C s = h2 * fv;
        s = s + lget(u, x, i - 1, j, k);
        s = s + lget(u, x, i + 1, j, k);
        if (DIM > 1) {
            s = s + lget(u, x, i, j - 1, k);
            s = s + lget(u, x, i, j + 1, k);
        }
        if (DIM > 2) {
            s = s + lget(u, x, i, j, k - 1);
            s = s + lget(u, x, i, j, k + 1);
        }
        return s * (C)(DIM == 1 ? 0.5 : DIM == 2 ? 0.25 : 1.0 / 6.0);
    } else {
        C ww, we, ws, wn;
        tfaces<C, DIM, VC>(a, x.n, i, j, ww, we, ws, wn);
        C s = h2 * fv;
        s = s + ww * lget(u, x, i - 1, j, k);
        s = s + we * lget(u, x, i + 1, j, k);
        s = s + ws * lget(u, x, i, j - 1, k);
        s = s + wn * lget(u, x, i, j + 1, k);
        return s / (((ww + we) + ws) + wn);
    }
}

template <class C, int DIM, bool VC>
__device__ __forceinline__ C t_apply(const C *u, const C *a, const LIdx<DIM> &x, C ih2, int i, int j, int k)
{
    const C uc = lget(u, x, i, j, k);
    C s;
    if constexpr (!VC) {
        s = (uc - lget(u, x, i - 1, j, k)) + (uc - lget(u, x, i + 1, j, k));
        if (DIM > 1) s = (s + (uc - lget(u, x, i, j - 1, k))) + (uc - lget(u, x, i, j + 1, k));
        if (DIM > 2) s = (s + (uc - lget(u, x, i, j, k - 1))) + (uc - lget(u, x, i, j, k + 1));
    } else {
        C ww, we, ws, wn;
        tfaces<C, DIM, VC>(a, x.n, i, j, ww, we, ws, wn);
        s = ((ww * (uc - lget(u, x, i - 1, j, k)) + we * (uc - lget(u, x, i + 1, j, k))) +
             ws * (uc - lget(u, x, i, j - 1, k))) +
            wn * (uc - lget(u, x, i, j + 1, k));
    }
    return s * ih2;
}

// Padded LDS level: (n+2)^DIM values with a zero border, so neighbours need
// no bounds checks; index of (i,j,k), 0 <= i,j,k <= n+1.
template <int DIM>
struct PIdx {
    int n, s1, s2;  // n, row stride n+2, plane stride (n+2)^2
    __device__ __forceinline__ PIdx(int n_) : n(n_), s1(n_ + 2), s2((n_ + 2) * (n_ + 2)) {}
    __device__ __forceinline__ int at(int i, int j, int k) const
    {
        return i + (DIM > 1 ? j * s1 : 0) + (DIM > 2 ? k * s2 : 0);
    }
    __device__ __forceinline__ int size() const { return DIM == 1 ? s1 : DIM == 2 ? s2 : s2 * s1; }
};

// Visit the points of one colour (1-based index sum even = red = 0) without
// division: pairs of x-points per thread.  2D: 32 pairs per row (n <= 63);
// 3D: 8 pairs per row, 16 rows per plane (n <= 15); 1D: strided.
template <int DIM, class Fn>
__device__ __forceinline__ void for_colour(int n, int colour, int tid, int nt, Fn &&fn)
{
    if constexpr (DIM == 1) {
        for (int p = tid; 2 * p + 1 <= n; p += nt) {
            const int i = 2 * p + 1 + ((colour + 1) & 1);
            if (i <= n) fn(i, 1, 1);
        }
    } else if constexpr (DIM == 2) {
        const int p = tid & 31;
        for (int j = (tid >> 5) + 1; j <= n; j += nt >> 5) {
            const int i = 2 * p + 1 + ((j + colour + 1) & 1);
            if (i <= n) fn(i, j, 1);
        }
    } else {
        const int p = tid & 7, j = ((tid >> 3) & 15) + 1;
        if (j > n) return;
        for (int k = (tid >> 7) + 1; k <= n; k += nt >> 7) {
            const int i = 2 * p + 1 + ((j + k + colour + 1) & 1);
            if (i <= n) fn(i, j, k);
        }
    }
}

template <class C, int DIM, bool VC>
__device__ __forceinline__ void pfaces(const C *a, int n, int i, int j, C &ww, C &we, C &ws, C &wn)
{
    tfaces<C, DIM, VC>(a, n, i, j, ww, we, ws, wn);
}

// GS point value from padded neighbours
template <class C, int DIM, bool VC>
__device__ __forceinline__ C p_relax(const C *u, C fv, const C *a, const PIdx<DIM> &x, C h2, int i, int j, int k)
{
    const int c = x.at(i, j, k);
    if constexpr (!VC) {
        C s = h2 * fv;
        s = s + u[c - 1];
        s = s + u[c + 1];
        if (DIM > 1) {
            s = s + u[c - x.s1];
            s = s + u[c + x.s1];
        }
        if (DIM > 2) {
            s = s + u[c - x.s2];
            s = s + u[c + x.s2];
        }
        return s * (C)(DIM == 1 ? 0.5 : DIM == 2 ? 0.25 : 1.0 / 6.0);
    } else {
        C ww, we, ws, wn;
        pfaces<C, DIM, VC>(a, x.n, i, j, ww, we, ws, wn);
        C s = h2 * fv;
        s = s + ww * u[c - 1];
        s = s + we * u[c + 1];
        s = s + ws * u[c - x.s1];
        s = s + wn * u[c + x.s1];
        return s / (((ww + we) + ws) + wn);
    }
}

template <class C, int DIM, bool VC>
__device__ __forceinline__ C p_apply(const C *u, const C *a, const PIdx<DIM> &x, C ih2, int i, int j, int k)
{
    const int c = x.at(i, j, k);
    const C uc = u[c];
    C s;
    if constexpr (!VC) {
        s = (uc - u[c - 1]) + (uc - u[c + 1]);
        if (DIM > 1) s = (s + (uc - u[c - x.s1])) + (uc - u[c + x.s1]);
        if (DIM > 2) s = (s + (uc - u[c - x.s2])) + (uc - u[c + x.s2]);
    } else {
        C ww, we, ws, wn;
        pfaces<C, DIM, VC>(a, x.n, i, j, ww, we, ws, wn);
        s = ((ww * (uc - u[c - 1]) + we * (uc - u[c + 1])) + ws * (uc - u[c - x.s1])) + wn * (uc - u[c + x.s1]);
    }
    return s * ih2;
}

// The same two operations with the faces read from the precomputed tables
// (2D diffusion): identical operands and order.
template <class C>
__device__ __forceinline__ C pf_relax(const C *u, C fv, const C *fe, const C *fn, const C *dg, int s1, C h2, int c)
{
    C s = h2 * fv;
    s = s + fe[c - 1] * u[c - 1];
    s = s + fe[c] * u[c + 1];
    s = s + fn[c - s1] * u[c - s1];
    s = s + fn[c] * u[c + s1];
    return s / dg[c];
}

template <class C>
__device__ __forceinline__ C pf_apply(const C *u, const C *fe, const C *fn, int s1, C ih2, int c)
{
    const C uc = u[c];
    const C s = ((fe[c - 1] * (uc - u[c - 1]) + fe[c] * (uc - u[c + 1])) + fn[c - s1] * (uc - u[c - s1])) +
                fn[c] * (uc - u[c + s1]);
    return s * ih2;
}

template <class S, class F, int DIM, bool VC>
__global__ __launch_bounds__(1024) void k_tail(TailArgs args)
{
    using T = Traits<S>;
    using C = typename T::C;
    extern __shared__ __align__(16) unsigned char smem[];
    const int sys = blockIdx.x;
    const int nl = args.nlev;
    const int tid = threadIdx.x, nt = blockDim.x;
    // stage this system's level descriptors and its coarsest inverse in LDS
    // once (they are read in every phase below); the stop flag is loaded in
    // the same round
    __shared__ LevelDesc Ls[kTailMaxLevels];
    constexpr int kCinvCap = DIM == 3 ? 27 * 27 : DIM == 2 ? 9 * 9 : 1;  // the default coarsest sizes
    __shared__ double Cinv[kCinvCap];
    const int done = args.states[sys].done;
    const int mm = args.m * args.m;
    const double *ci = args.cinv + (long long)sys * mm;
    const bool cinv_lds = mm <= kCinvCap;
    {
        const LevelDesc *src = args.levels + (long long)sys * args.nlev;
        const int words = (int)(sizeof(LevelDesc) / 4) * nl;
        for (int w = tid; w < words; w += nt) ((uint32_t *)Ls)[w] = ((const uint32_t *)src)[w];
        if (cinv_lds)
            for (int q = tid; q < mm; q += nt) Cinv[q] = ci[q];
    }
    if (done) return;
    __syncthreads();

    // The dynamic LDS holds the padded u_k and f_k per level, then the Jacobi
    // copy of the top level, then (2D diffusion) the face tables.  Their
    // offsets (in elements) sit in a small LDS table and every array below is
    // smem plus an offset, so each access is an LDS instruction: pointers kept
    // in per-thread arrays indexed by the level would live in scratch memory
    // and turn every access into a generic (flat) one.
    __shared__ int loff[kTailMaxLevels][5];  // u, f, east face, north face, face sum
    __shared__ int ltmp;
    C *const lds = (C *)smem;
    if (tid == 0) {
        int q = 0;
        for (int k = 0; k < nl; ++k) {
            const int m = PIdx<DIM>(Ls[k].n).size();
            loff[k][0] = q;
            loff[k][1] = q + m;
            q += 2 * m;
        }
        ltmp = q;
        q += PIdx<DIM>(Ls[0].n).size();
        for (int k = 0; k < nl; ++k) {
            const int m = PIdx<DIM>(Ls[k].n).size();
            loff[k][2] = q;
            loff[k][3] = q + m;
            loff[k][4] = q + 2 * m;
            q += 3 * m;
        }
    }
    __syncthreads();
    auto uk = [&](int k) { return lds + loff[k][0]; };
    auto fk = [&](int k) { return lds + loff[k][1]; };
    auto fe = [&](int k) { return lds + loff[k][2]; };
    auto fn = [&](int k) { return lds + loff[k][3]; };
    auto dg = [&](int k) { return lds + loff[k][4]; };
    C *tmp = lds + ltmp;
    for (int q = tid; q < ltmp; q += nt) lds[q] = (C)0;
    // 2D diffusion: per level the east face fe (nodes 0..n on rows 1..n), the
    // north face fn (rows 0..n on columns 1..n) and the face sum dg of every
    // interior node, computed once from the nodal coefficient with the same
    // operations the on-the-fly form uses (harmonic means of the same pair)
    const bool faces = VC && DIM == 2 && args.faces;
    if constexpr (VC && DIM == 2) {
        if (faces) {
            for (int k = 0; k < nl; ++k) {
                const int n = Ls[k].n, s1 = n + 2, m = s1 * s1;
                const C *a = (const C *)Ls[k].a;
                for (int q = tid; q < m; q += nt) {
                    const int i = q % s1, j = q / s1;
                    // the nodal array has the padded layout: node (i, j) at q
                    fe(k)[q] = (i <= n && j >= 1 && j <= n) ? tharm(a[q], a[q + 1]) : (C)0;
                    fn(k)[q] = (j <= n && i >= 1 && i <= n) ? tharm(a[q], a[q + s1]) : (C)0;
                }
            }
            __syncthreads();
            for (int k = 0; k < nl; ++k) {
                const int n = Ls[k].n, s1 = n + 2, m = s1 * s1;
                for (int q = tid; q < m; q += nt) {
                    const int i = q % s1, j = q / s1;
                    if (i >= 1 && i <= n && j >= 1 && j <= n)
                        dg(k)[q] = ((fe(k)[q - 1] + fe(k)[q]) + fn(k)[q - s1]) + fn(k)[q];
                }
            }
        }
    }
    __syncthreads();
    // load the top level: rhs from global, state zero or from B
    {
        const LevelDesc &L = Ls[0];
        const PIdx<DIM> x(L.n);
        const F *f = (const F *)L.f;
        const S *b = (const S *)L.B;
        if (DIM == 2 && nt == 1024 && L.n <= 64) {
            // one 64-column x 16-row pass per 1024 threads, unrolled so that
            // all of a thread's loads are in flight together
            const int i = (tid & 63) + 1;
#pragma unroll
            for (int it = 0; it < 4; ++it) {
                const int j = (tid >> 6) + 1 + 16 * it;
                const bool ok = i <= L.n && j <= L.n;
                const long long go = ok ? (long long)(i - 1) + (long long)(j - 1) * L.pitch : 0;
                const C fv = (C)gld(f + go);
                const C bv = L.uzero ? (C)0 : (C)T::ld(b + go);
                if (ok) {
                    fk(0)[x.at(i, j, 1)] = fv;
                    if (!L.uzero) uk(0)[x.at(i, j, 1)] = bv;
                }
            }
        } else {
            for_points<DIM>(L.n, tid, nt, [&](int i, int j, int k, int q) {
                (void)q;
                const long long go = (long long)(i - 1) + (long long)(j - 1) * L.pitch + (long long)(k - 1) * L.ppitch;
                fk(0)[x.at(i, j, k)] = (C)gld(f + go);
                if (!L.uzero) uk(0)[x.at(i, j, k)] = T::ld(b + go);
            });
        }
    }
    __syncthreads();

    auto smooth = [&](int lv, int nsweeps) {
        const LevelDesc &L = Ls[lv];
        const PIdx<DIM> x(L.n);
        const C *a = (const C *)L.a;
        const C h2 = (C)L.h2, ih2 = (C)L.inv_h2;
        C *u = uk(lv);
        const C *f = fk(lv);
        for (int sw = 0; sw < nsweeps; ++sw) {
            if (args.smoother == 1) {
                for (int q = tid; q < x.size(); q += nt) tmp[q] = u[q];
                __syncthreads();
                for_points<DIM>(L.n, tid, nt, [&](int i, int j, int k, int q) {
                    (void)q;
                    const int c = x.at(i, j, k);
                    const C r = f[c] - p_apply<C, DIM, VC>(tmp, a, x, ih2, i, j, k);
                    C ww, we, ws, wn;
                    pfaces<C, DIM, VC>(a, L.n, i, j, ww, we, ws, wn);
                    const C diag = VC ? (((ww + we) + ws) + wn) * ih2 : (C)(2 * DIM) * ih2;
                    u[c] = T::rnd(tmp[c] + (C)args.omega * r / diag);
                });
                __syncthreads();
            } else {
                for (int colour = 0; colour < 2; ++colour) {
                    for_colour<DIM>(L.n, colour, tid, nt, [&](int i, int j, int k) {
                        const int c = x.at(i, j, k);
                        if constexpr (VC && DIM == 2) {
                            if (faces) {
                                u[c] = T::rnd(pf_relax<C>(u, f[c], fe(lv), fn(lv), dg(lv), x.s1, h2, c));
                                return;
                            }
                        }
                        u[c] = T::rnd(p_relax<C, DIM, VC>(u, f[c], a, x, h2, i, j, k));
                    });
                    __syncthreads();
                }
            }
        }
    };

    // residual (or, for full multigrid, the rhs itself) restricted to level
    // lv + 1 by full weighting; the coarse state starts from zero
    auto restrict_to = [&](int lv, bool rhs_only) {
        const LevelDesc &L = Ls[lv];
        const PIdx<DIM> x(L.n), xc(Ls[lv + 1].n);
        const C *a = (const C *)L.a;
        const C ih2 = (C)L.inv_h2;
        for_points<DIM>(xc.n, tid, nt, [&](int I, int J, int K, int q) {
            (void)q;
            C s = (C)0;
            for (int oz = (DIM > 2 ? -1 : 0); oz <= (DIM > 2 ? 1 : 0); ++oz)
                for (int oy = (DIM > 1 ? -1 : 0); oy <= (DIM > 1 ? 1 : 0); ++oy)
                    for (int ox = -1; ox <= 1; ++ox) {
                        const int i = 2 * I + ox, j = DIM > 1 ? 2 * J + oy : 1, k = DIM > 2 ? 2 * K + oz : 1;
                        const int wt = (2 - (ox < 0 ? -ox : ox)) * (DIM > 1 ? (2 - (oy < 0 ? -oy : oy)) : 1) *
                                       (DIM > 2 ? (2 - (oz < 0 ? -oz : oz)) : 1);
                        C r = fk(lv)[x.at(i, j, k)];
                        if (!rhs_only) {
                            C Au;
                            if constexpr (VC && DIM == 2) {
                                Au = faces ? pf_apply<C>(uk(lv), fe(lv), fn(lv), x.s1, ih2, x.at(i, j, k))
                                           : p_apply<C, DIM, VC>(uk(lv), a, x, ih2, i, j, k);
                            } else {
                                Au = p_apply<C, DIM, VC>(uk(lv), a, x, ih2, i, j, k);
                            }
                            r = r - Au;
                        }
                        s = s + (C)wt * r;
                    }
            const int cq = xc.at(I, J, K);
            fk(lv + 1)[cq] = s * (C)(DIM == 1 ? 0.25 : DIM == 2 ? 0.0625 : 0.015625);
            uk(lv + 1)[cq] = (C)0;
        });
        __syncthreads();
    };
    // coarsest: FP64 inverse times rhs
    auto solve_coarsest = [&]() {
        const int m = args.m;
        const int nc = Ls[nl - 1].n;
        const PIdx<DIM> xc(nc);
        double xv = 0.0;
        if (tid < m) {
            for (int q = 0; q < m; ++q) {
                const int i = q % nc + 1, j = DIM > 1 ? (q / nc) % nc + 1 : 1, k = DIM > 2 ? q / (nc * nc) + 1 : 1;
                const double cv = cinv_lds ? Cinv[tid * m + q] : ci[(long long)tid * m + q];
                xv += cv * (double)fk(nl - 1)[xc.at(i, j, k)];
            }
        }
        __syncthreads();
        if (tid < m) {
            const int i = tid % nc + 1, j = DIM > 1 ? (tid / nc) % nc + 1 : 1, k = DIM > 2 ? tid / (nc * nc) + 1 : 1;
            uk(nl - 1)[xc.at(i, j, k)] = T::rnd((C)xv);
        }
        __syncthreads();
    };
    // u_lv += P u_{lv+1} (or, for full multigrid, u_lv = P u_{lv+1})
    auto prolong = [&](int lv, bool set) {
        const PIdx<DIM> x(Ls[lv].n), xc(Ls[lv + 1].n);
        const C *uc = uk(lv + 1);
        C *u = uk(lv);
        for_points<DIM>(x.n, tid, nt, [&](int i, int j, int k, int q) {
            (void)q;
            // parents along each axis: even index -> one (weight 1), odd -> two (1/2 each);
            // coarse index 0 / nc+1 are the zero border
            const int i0 = i / 2, i1 = (i & 1) ? i0 + 1 : i0;
            const int j0 = j / 2, j1 = (j & 1) ? j0 + 1 : j0;
            const int k0 = k / 2, k1 = (k & 1) ? k0 + 1 : k0;
            auto line = [&](int jj, int kk) -> C {
                const C a0 = uc[xc.at(i0, jj, kk)];
                return (i & 1) ? (a0 + uc[xc.at(i1, jj, kk)]) * (C)0.5 : a0;
            };
            auto plane = [&](int kk) -> C {
                if (DIM < 2) return line(0, kk);
                const C b0 = line(j0, kk);
                return (j & 1) ? (b0 + line(j1, kk)) * (C)0.5 : b0;
            };
            C corr;
            if (DIM < 3) {
                corr = plane(0);
            } else {
                const C c0 = plane(k0);
                corr = (k & 1) ? (c0 + plane(k1)) * (C)0.5 : c0;
            }
            const int c = x.at(i, j, k);
            u[c] = T::rnd(set ? corr : u[c] + corr);
        });
        __syncthreads();
    };

    if (args.ops) {
        // a schedule of level operations built on the host (W- and F-cycles,
        // full multigrid): op = kind | level << 4 | sweeps << 12
        for (int q = 0; q < args.nops; ++q) {
            const int op = args.ops[q];
            const int kind = op & 15, lv = (op >> 4) & 255, arg = op >> 12;
            switch (kind) {
            case TAIL_OP_SMOOTH: smooth(lv, arg); break;
            case TAIL_OP_RESTRICT: restrict_to(lv, false); break;
            case TAIL_OP_SOLVE: solve_coarsest(); break;
            case TAIL_OP_PROLONG: prolong(lv, false); break;
            case TAIL_OP_RESTRICT_RHS: restrict_to(lv, true); break;
            case TAIL_OP_INTERP: prolong(lv, true); break;
            }
        }
    } else {
        // the V-cycle
        for (int lv = 0; lv + 1 < nl; ++lv) {
            smooth(lv, args.nu1);
            restrict_to(lv, false);
        }
        solve_coarsest();
        for (int lv = nl - 2; lv >= 0; --lv) {
            prolong(lv, false);
            smooth(lv, args.nu2);
        }
    }
    // write the top level's final state
    {
        const LevelDesc &L = Ls[0];
        const PIdx<DIM> x(L.n);
        S *b = (S *)L.B;
        for_points<DIM>(L.n, tid, nt, [&](int i, int j, int k, int q) {
            (void)q;
            const long long go = (long long)(i - 1) + (long long)(j - 1) * L.pitch + (long long)(k - 1) * L.ppitch;
            T::st(b + go, uk(0)[x.at(i, j, k)]);
        });
    }
}

size_t tail_lds_bytes(int st, int dim, int n_top, bool jacobi, bool faces)
{
    const size_t cs = (st == ST_F64) ? 8 : 4;
    size_t tot = 0, top = 0;
    for (int n = n_top; n >= 1; n = (n - 1) / 2) {
        const size_t e = (size_t)n + 2;
        const size_t m = dim == 1 ? e : dim == 2 ? e * e : e * e * e;
        if (!top) top = m;
        tot += 2 * m;
        if (n == 1) break;
    }
    (void)jacobi;
    // faces: east, north and the diagonal sum per level (3 arrays like u, f, u)
    return (tot + top + (faces ? tot / 2 * 3 : 0)) * cs;
}

size_t tail_max_lds() { return kTailMaxDynLds; }

template <class S, class F, bool VC>
static hipError_t tail_dim(int dim, const TailArgs &a, size_t lds, int threads, hipStream_t s)
{
    switch (dim) {
    case 1: hipLaunchKernelGGL((k_tail<S, F, 1, false>), dim3(a.nsys), dim3(threads), lds, s, a); break;
    case 2: hipLaunchKernelGGL((k_tail<S, F, 2, VC>), dim3(a.nsys), dim3(threads), lds, s, a); break;
    case 3: hipLaunchKernelGGL((k_tail<S, F, 3, false>), dim3(a.nsys), dim3(threads), lds, s, a); break;
    }
    return hipGetLastError();
}

template <class S, class F, bool VC>
static int tail_attr(int dim)
{
    switch (dim) {
    case 1: (void)hipFuncSetAttribute((const void *)k_tail<S, F, 1, false>, hipFuncAttributeMaxDynamicSharedMemorySize, kTailMaxDynLds); break;
    case 2: (void)hipFuncSetAttribute((const void *)k_tail<S, F, 2, VC>, hipFuncAttributeMaxDynamicSharedMemorySize, kTailMaxDynLds); break;
    case 3: (void)hipFuncSetAttribute((const void *)k_tail<S, F, 3, false>, hipFuncAttributeMaxDynamicSharedMemorySize, kTailMaxDynLds); break;
    }
    return 0;
}

// Allow the tail kernels up to 160 KB of dynamic LDS (called once at setup,
// outside any graph capture).
hipError_t tail_prepare(int st, bool vc, int dim)
{
    switch (st) {
    case ST_F64: vc ? tail_attr<double, double, true>(dim) : tail_attr<double, double, false>(dim); break;
    case ST_F32: vc ? tail_attr<float, float, true>(dim) : tail_attr<float, float, false>(dim); break;
    case ST_BF16: vc ? tail_attr<bf16_t, float, true>(dim) : tail_attr<bf16_t, float, false>(dim); break;
    }
    return hipGetLastError();
}

// lds: bytes of dynamic LDS (tail_lds_bytes of the top level); threads <= 1024
hipError_t launch_tail_sized(int st, bool vc, int dim, const TailArgs &a, size_t lds, int threads, hipStream_t s)
{
    if (a.nlev > kTailMaxLevels) return hipErrorInvalidValue;
    switch (st) {
    case ST_F64: return vc ? tail_dim<double, double, true>(dim, a, lds, threads, s)
                           : tail_dim<double, double, false>(dim, a, lds, threads, s);
    case ST_F32: return vc ? tail_dim<float, float, true>(dim, a, lds, threads, s)
                           : tail_dim<float, float, false>(dim, a, lds, threads, s);
    case ST_BF16: return vc ? tail_dim<bf16_t, float, true>(dim, a, lds, threads, s)
                            : tail_dim<bf16_t, float, false>(dim, a, lds, threads, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace mgx
