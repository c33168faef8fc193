// Fused 3D plane-marching level kernels: one red-black Gauss-Seidel sweep of
// the 7-point Poisson operator per pass, with the neighbouring operations of
// the V-cycle fused in front of it (a zero start, or the trilinear coarse-grid
// correction) and behind it (residual + full-weighting restriction, or the
// residual's squared norm, or adding the result into an FP64 iterate).
//
// A workgroup owns a TX x TY tile of columns and a run of planes and marches
// up the planes.  At the step that brings plane z + 1 into the LDS ring it
// updates the red points of plane z, then the black points of plane z - 1
// (which is then final and is stored), and the residual of plane z - 3 (whose
// neighbour planes are all final by then).  That is the red-black order: red
// at z reads black values that are still old, black at z - 1 reads red values
// that are all new.  In the plane, each stage reads the four in-plane
// neighbours of the previous one, so the tile is loaded with a halo of R
// points (2 for the sweep, plus 2 for residual + restriction, plus 1 for the
// norm) and the ring is recomputed: every value the workgroup keeps depends
// only on data it loaded itself.  This is how the paper's blockable rule
// ("Vector Engine" section: an operation may join a kernel only if it does
// not read shifted views of what the kernel writes) is met for stages that
// do read shifted views: the halo makes each tile self-contained.
//
// Threads work on pairs of x-adjacent points, of which exactly one is red,
// so every lane does one update per pair and colour.  Two barriers per step:
// [store plane z+1] | red z, residual z-3 | black z-1, store, restriction.
// The sum orders are those of the unfused kernels (half sweeps, column-march
// residual, restriction, prolongation), so both paths give the same values.
#include <cstdlib>
#include <utility>

#include "dev_common.h"
#include "mg_m3.h"

// Tile shapes (owned columns TX x TY, threads NT) per pass kind: the
// residual + restriction tail needs a halo of 4 and gets its own shape, which
// for an FP64 state is narrower (its LDS ring is twice as large).  Measured
// at 511^3 (FP64 / FP32 state): 64 x 16 with 512 threads for the other
// passes; the restriction pass 32 x 16 (FP64) and 64 x 16 (FP32).
#ifndef MGX_M3_TX
#define MGX_M3_TX 64
#endif
#ifndef MGX_M3_TY
#define MGX_M3_TY 16
#endif
#ifndef MGX_M3_NT
#define MGX_M3_NT 512
#endif
#ifndef MGX_M3_RR_TX
#define MGX_M3_RR_TX 64
#endif
#ifndef MGX_M3_NORM_TX
#define MGX_M3_NORM_TX 64
#endif
#ifndef MGX_M3_RR_TX64
#define MGX_M3_RR_TX64 32
#endif
#ifndef MGX_M3_RR_TY
#define MGX_M3_RR_TY 16
#endif
#ifndef MGX_M3_RR_NT
#define MGX_M3_RR_NT 512
#endif
#ifndef MGX_M3_PD
#define MGX_M3_PD 3  // planes of loads in flight per workgroup
#endif

namespace mgx {

struct M3Shape {
    int tx, ty, nt;
};
__host__ __device__ constexpr M3Shape m3_shape(int tail, bool f64)
{
    return tail == M3_TAIL_RR     ? M3Shape{f64 ? MGX_M3_RR_TX64 : MGX_M3_RR_TX, MGX_M3_RR_TY, MGX_M3_RR_NT}
           : tail == M3_TAIL_NORM ? M3Shape{MGX_M3_NORM_TX, MGX_M3_TY, MGX_M3_NT}
                                  : M3Shape{MGX_M3_TX, MGX_M3_TY, MGX_M3_NT};
}

template <int... Q, class Fn>
__device__ __forceinline__ void m3_static_for_impl(std::integer_sequence<int, Q...>, Fn &&fn)
{
    (fn(std::integral_constant<int, Q>{}), ...);
}
template <int N, class Fn>
__device__ __forceinline__ void m3_static_for(Fn &&fn)
{
    m3_static_for_impl(std::make_integer_sequence<int, N>{}, fn);
}

__host__ __device__ constexpr int m3_halo(int tail) { return tail == M3_TAIL_RR ? 4 : tail == M3_TAIL_NORM ? 3 : 2; }

template <class S, class F, int HEAD, int TAIL, int TX, int TY, int NT, int PD>
__global__ __launch_bounds__(NT) void k_march3d(M3Args a)
{
    using T = Traits<S>;
    using C = typename T::C;
    constexpr int R = m3_halo(TAIL);
    // black (final) planes recomputed below / above the run: the residual of
    // plane k needs final planes k - 1 and k + 1, and the restriction of the
    // top coarse plane needs the residual of the first plane above the run
    constexpr int ER = TAIL == M3_TAIL_RR ? 1 : 0;
    constexpr int EL = TAIL == M3_TAIL_NONE ? 0 : 1;
    constexpr int EH = TAIL == M3_TAIL_NONE ? 0 : 1 + ER;
    constexpr int LX = TX + 2 * R, LY = TY + 2 * R, NU = LX * LY;
    constexpr int FR = R - 1, FX = TX + 2 * FR, FY = TY + 2 * FR, NF = FX * FY;
    constexpr int D = TAIL == M3_TAIL_NONE ? 5 : 6;     // planes of u in the ring
    // the residual of plane z - 3 reads f from the ring when a fifth plane
    // fits (the norm pass; the restriction pass with 4-byte values), else
    // from memory again
    constexpr bool FRES = TAIL == M3_TAIL_NORM || (TAIL == M3_TAIL_RR && sizeof(C) == 4);
    constexpr int DF = FRES ? 5 : 4;                    // planes of f in the ring
    constexpr int QU = (NU + NT - 1) / NT, QF = (NF + NT - 1) / NT;
    // residual region: the tile plus one (RR) or the tile (NORM)
    constexpr int RRing = TAIL == M3_TAIL_RR ? 1 : 0;
    constexpr int RXN = TX + 2 * RRing, RYN = TY + 2 * RRing, NR = TAIL == M3_TAIL_NONE ? 1 : RXN * RYN;
    constexpr int QR = (NR + NT - 1) / NT;
    constexpr int CXN = TX / 2, CYN = TY / 2;           // coarse points of a tile plane (RR)
    // coarse region of the correction: coarse index from floor((i0 - R) / 2)
    constexpr int KCX = LX / 2 + 3, KCY = LY / 2 + 3, NKC = HEAD == M3_HEAD_CORR ? KCX * KCY : 1;
    constexpr int QC = (NKC + NT - 1) / NT;
    constexpr int PX = LX / 2;                          // pairs per row
    constexpr int NRED = (LY - 2) * PX;                 // pairs of the red stage (rows 1 .. LY-2)
    constexpr int NBLK = (LY - 4) * (PX - 2);           // pairs of the black stage (rows, pairs 2 .. -2)
    constexpr int IR = (NRED + NT - 1) / NT, IB = (NBLK + NT - 1) / NT;
    constexpr uint32_t SB = sizeof(S), FB = sizeof(F);
    static_assert(TX % 2 == 0 && TY % 2 == 0, "even tiles");
    static_assert(TAIL != M3_TAIL_RR || CXN * CYN <= NT, "one coarse point per thread");

    __shared__ C U[D][NU];
    __shared__ C Fs[DF][NF];
    __shared__ C Rp[TAIL == M3_TAIL_RR ? NR : 1];
    __shared__ C Kc[HEAD == M3_HEAD_CORR ? 2 : 1][NKC];
    __shared__ double wsum[NT / 64];

    if (a.state && a.state->done) return;
    // tiles: x fastest, then y, then the plane run; workgroups are dealt to
    // the 8 XCDs round-robin, so give each XCD a contiguous range of tiles
    // (neighbouring tiles share halo lines in one L2)
    const int nb = a.ntx * a.nty * a.ntz;
    const int per = (nb + 7) / 8;
    const int t = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (t >= nb) return;
    const int n = a.n;
    const int i0 = (t % a.ntx) * TX + 1, j0 = ((t / a.ntx) % a.nty) * TY + 1;
    const int k0 = (t / (a.ntx * a.nty)) * a.kz + 1, k1 = min(k0 + a.kz, n + 1);
    const int tid = threadIdx.x;
    const C h2 = (C)a.h2, ih2 = (C)a.ih2;

    // plane schedule: red on [zr0, k1 + EH], black on [k0 - EL, k1 - 1 + EH],
    // residual on [k0, k1 - 1 + ER]; step z does red z, black z - 1, residual z - 3
    const int zr0 = k0 - 1 - EL;
    const int zred1 = k1 + EH;
    const int zres1 = k1 - 1 + ER;
    const int zend = TAIL == M3_TAIL_NONE ? zred1 : zres1 + 3;
    const int zload1 = zred1 + 1;  // last plane of u / f the sweep reads
    const int zb = zr0 - 1;        // ring slots count from here (p >= zb always)
    auto slot = [&](int p) { return (p - zb) % D; };
    auto fslot = [&](int p) { return (p - zb) % DF; };
    auto xy_in = [&](int i, int j) { return i >= 1 && i <= n && j >= 1 && j <= n; };

    // Memory goes through one buffer descriptor per plane: a byte offset
    // inside the plane per lane (precomputed once), records = the plane's
    // extent, or none for a plane outside the domain -- loads then return 0
    // and stores are dropped, so masked lanes and planes need no branch.
    auto extent = [&](long long pitch, uint32_t es) -> uint32_t {
        return (uint32_t)(((long long)(n - 1) * pitch + n) * es);
    };
    auto plane_rsrc = [&](const void *base, long long ppitch, uint32_t es, int k, uint32_t ext, bool ok) {
        const int kk = min(max(k, 1), n);
        return make_rsrc((const char *)base + (long long)(kk - 1) * ppitch * es, ok ? ext : 0u);
    };
    const uint32_t ext_u = extent(a.ip, SB), ext_f = extent(a.fp, FB);

    // ---- per-thread offsets and masks (fixed for the whole run) ------------
    uint32_t uo[QU], fo[QF];
#pragma unroll
    for (int q = 0; q < QU; ++q) {
        const int p = tid + q * NT;
        const int i = i0 - R + p % LX, j = j0 - R + p / LX;
        uo[q] = (p < NU && xy_in(i, j)) ? (uint32_t)((i - 1) + (long long)(j - 1) * a.ip) * SB : kOOB;
    }
#pragma unroll
    for (int q = 0; q < QF; ++q) {
        const int p = tid + q * NT;
        const int i = i0 - FR + p % FX, j = j0 - FR + p / FX;
        fo[q] = (p < NF && xy_in(i, j)) ? (uint32_t)((i - 1) + (long long)(j - 1) * a.fp) * FB : kOOB;
    }
    // red stage: LDS index of the pair's even point, its f index, and
    // bits 0/1 = even/odd point updatable, bit 2 = parity of (i + j) there
    int rp[IR], rf[IR], rm[IR];
#pragma unroll
    for (int it = 0; it < IR; ++it) {
        const int pp = tid + it * NT;
        const int y = 1 + (pp < NRED ? pp / PX : 0), x0 = pp < NRED ? 2 * (pp % PX) : 2;
        const int j = j0 - R + y, ix0 = i0 - R + x0;
        const bool v0 = pp < NRED && x0 >= 1 && xy_in(ix0, j);
        const bool v1 = pp < NRED && x0 + 1 < LX - 1 && xy_in(ix0 + 1, j);
        rp[it] = y * LX + x0;
        rf[it] = (y - 1) * FX + x0 - 1;
        rm[it] = (v0 ? 1 : 0) | (v1 ? 2 : 0) | (((ix0 + j) & 1) << 2);
    }
    // black stage: the same, bits 3/4 = even/odd point owned (stored), and
    // the byte offsets of the even point in the output plane
    const bool use_acc = a.acc != nullptr;
    const long long opitch = use_acc ? a.accp : a.op;
    const uint32_t OB = use_acc ? 8u : SB;
    int bp[IB], bf[IB], bm[IB];
    uint32_t bo[IB];
#pragma unroll
    for (int it = 0; it < IB; ++it) {
        const int pp = tid + it * NT;
        const int y = 2 + (pp < NBLK ? pp / (PX - 2) : 0), x0 = pp < NBLK ? 2 + 2 * (pp % (PX - 2)) : 2;
        const int j = j0 - R + y, ix0 = i0 - R + x0;
        const bool v0 = pp < NBLK && xy_in(ix0, j), v1 = pp < NBLK && xy_in(ix0 + 1, j);
        const bool yown = y >= R && y < R + TY;
        const bool o0 = v0 && yown && x0 >= R && x0 < R + TX, o1 = v1 && yown && x0 + 1 >= R && x0 + 1 < R + TX;
        bp[it] = y * LX + x0;
        bf[it] = (y - 1) * FX + x0 - 1;
        bm[it] = (v0 ? 1 : 0) | (v1 ? 2 : 0) | (((ix0 + j) & 1) << 2) | (o0 ? 8 : 0) | (o1 ? 16 : 0);
        bo[it] = (v0 || v1) ? (uint32_t)((ix0 - 1) + (long long)(j - 1) * opitch) * OB : 0u;
    }
    // residual stage: LDS index, bit 0 = in the domain, bit 1 = owned; f offsets
    int rsp[QR], rsm[QR], rsf[QR];
    uint32_t ro[QR];
#pragma unroll
    for (int q = 0; q < QR; ++q) {
        const int pq = tid + q * NT;
        const int xr = pq < NR ? pq % RXN : 0, yr = pq < NR ? pq / RXN : 0;
        const int x = xr + R - RRing, y = yr + R - RRing;
        const int i = i0 - R + x, j = j0 - R + y;
        const bool ok = pq < NR && xy_in(i, j);
        const bool own = ok && i >= i0 && i < i0 + TX && j >= j0 && j < j0 + TY;
        rsp[q] = y * LX + x;
        rsf[q] = (y - 1) * FX + x - 1;  // the same point in the f ring (origin one point further in)
        rsm[q] = (ok ? 1 : 0) | (own ? 2 : 0);
        ro[q] = ok ? (uint32_t)((i - 1) + (long long)(j - 1) * a.fp) * FB : kOOB;
    }

    // ---- coarse correction --------------------------------------------------
    // Coarse planes are staged in LDS (two slots); each thread keeps, for each
    // point of the u region it loads, the bilinear (x, y) interpolation of the
    // two coarse planes around its current fine plane p (Pa: plane p / 2,
    // Pb: plane p / 2 + 1); the correction is Pa (p even) or (Pa + Pb) / 2 (p
    // odd) -- the order of the unfused prolongation kernel (x, y, then z).
    const int ci0 = (i0 - R) >> 1, cj0 = (j0 - R) >> 1;  // floor
    C pk[HEAD == M3_HEAD_CORR ? QC : 1];
    C Pa[HEAD == M3_HEAD_CORR ? QU : 1], Pb[HEAD == M3_HEAD_CORR ? QU : 1];
    uint32_t co[HEAD == M3_HEAD_CORR ? QC : 1];
    int kci[HEAD == M3_HEAD_CORR ? QU : 1], kpar[HEAD == M3_HEAD_CORR ? QU : 1];
    const uint32_t ext_c = HEAD == M3_HEAD_CORR ? (uint32_t)(((long long)(a.nc - 1) * a.ucp + a.nc) * SB) : 0u;
    if constexpr (HEAD == M3_HEAD_CORR) {
#pragma unroll
        for (int q = 0; q < QC; ++q) {
            const int p = tid + q * NT;
            const int I = ci0 + p % KCX, J = cj0 + p / KCX;
            co[q] = (p < NKC && I >= 1 && I <= a.nc && J >= 1 && J <= a.nc)
                        ? (uint32_t)((I - 1) + (long long)(J - 1) * a.ucp) * SB : kOOB;
        }
#pragma unroll
        for (int q = 0; q < QU; ++q) {
            const int p = min(tid + q * NT, NU - 1);
            const int i = i0 - R + p % LX, j = j0 - R + p / LX;
            kci[q] = ((j >> 1) - cj0) * KCX + (i >> 1) - ci0;
            kpar[q] = (i & 1) | ((j & 1) << 1);
        }
    }
    auto load_coarse = [&](int K) {
        if constexpr (HEAD == M3_HEAD_CORR) {
            const rsrc_t rc = plane_rsrc(a.uc, a.ucpp, SB, K, ext_c, K >= 1 && K <= a.nc);
#pragma unroll
            for (int q = 0; q < QC; ++q) pk[q] = T::bload(rc, co[q]);
        }
    };
    auto put_coarse = [&](int K) {
        if constexpr (HEAD == M3_HEAD_CORR) {
#pragma unroll
            for (int q = 0; q < QC; ++q) {
                const int p = tid + q * NT;
                if (p < NKC) Kc[K & 1][p] = pk[q];
            }
        }
    };
    // bilinear interpolation of staged coarse plane K at the thread's points
    auto bilin = [&](int K, C (&P)[HEAD == M3_HEAD_CORR ? QU : 1]) {
        if constexpr (HEAD == M3_HEAD_CORR) {
            const C *pl = Kc[K & 1];
#pragma unroll
            for (int q = 0; q < QU; ++q) {
                const int b = kci[q];
                const bool xo = kpar[q] & 1, yo = kpar[q] & 2;
                const C a00 = pl[b], a01 = pl[b + 1], a10 = pl[b + KCX], a11 = pl[b + KCX + 1];
                const C l0 = xo ? (a00 + a01) * (C)0.5 : a00;
                const C l1 = xo ? (a10 + a11) * (C)0.5 : a10;
                P[q] = yo ? (l0 + l1) * (C)0.5 : l0;
            }
        }
    };

    // ---- plane loads: a ring of PD planes of registers in flight -----------
    C pu[PD][QU], pf[PD][QF];
    auto load_u = [&](int k, C (&ru)[QU]) {
        if constexpr (HEAD == M3_HEAD_ZERO) {
#pragma unroll
            for (int q = 0; q < QU; ++q) ru[q] = (C)0;
        } else {
            const rsrc_t r = plane_rsrc(a.uin, a.ipp, SB, k, ext_u, k >= 1 && k <= n && k <= zload1);
#pragma unroll
            for (int q = 0; q < QU; ++q) ru[q] = T::bload(r, uo[q]);
        }
    };
    auto load_f = [&](int k, C (&rf_)[QF]) {
        const rsrc_t r = plane_rsrc(a.f, a.fpp, FB, k, ext_f, k >= 1 && k <= n && k <= zload1);
#pragma unroll
        for (int q = 0; q < QF; ++q) rf_[q] = (C)bld<F>(r, fo[q]);
    };
    auto put_u = [&](int k, const C (&ru)[QU]) {
        C *dst = U[slot(k)];
        const bool kin = k >= 1 && k <= n;
#pragma unroll
        for (int q = 0; q < QU; ++q) {
            const int p = tid + q * NT;
            if (p >= NU) continue;
            C v = ru[q];
            if constexpr (HEAD == M3_HEAD_CORR) {
                const C corr = (k & 1) ? (Pa[q] + Pb[q]) * (C)0.5 : Pa[q];
                if (kin && uo[q] != kOOB) v = T::rnd(v + corr);
            }
            dst[p] = v;
        }
    };
    auto put_f = [&](int k, const C (&rf_)[QF]) {
        C *dst = Fs[fslot(k)];
#pragma unroll
        for (int q = 0; q < QF; ++q) {
            const int p = tid + q * NT;
            if (p < NF) dst[p] = rf_[q];
        }
    };
    // f of the residual region, straight from memory PD steps ahead
    C pr[PD][QR];
    auto load_fr = [&](int k, C (&rr)[QR]) {
        if constexpr (TAIL != M3_TAIL_NONE && !FRES) {
            const rsrc_t r = plane_rsrc(a.f, a.fpp, FB, k, ext_f, k >= k0 && k <= zres1 && k >= 1 && k <= n);
#pragma unroll
            for (int q = 0; q < QR; ++q) rr[q] = (C)bld<F>(r, ro[q]);
        }
    };

    // Coarse pair for fine plane p, called for every plane in order: at an
    // even p the pair moves up one coarse plane (Pb from the plane staged
    // at p - 1); at an odd p the plane the next even p needs is staged.
    auto coarse_step = [&](int p) {
        if constexpr (HEAD == M3_HEAD_CORR) {
            if (p & 1) {
                put_coarse((p >> 1) + 2);
            } else {
#pragma unroll
                for (int q = 0; q < QU; ++q) Pa[q] = Pb[q];
                bilin((p >> 1) + 1, Pb);
                load_coarse((p >> 1) + 2);
            }
        }
    };

    // ---- prologue --------------------------------------------------------------
    {
        const int p0 = zr0 - 1;
        if constexpr (HEAD == M3_HEAD_CORR) {
            const int K0 = p0 >> 1;
            load_coarse(K0);
            put_coarse(K0);
            load_coarse(K0 + 1);
            put_coarse(K0 + 1);
            __syncthreads();
            bilin(K0, Pa);
            bilin(K0 + 1, Pb);
            load_coarse(K0 + 2);
            __syncthreads();
            if (p0 & 1) put_coarse(K0 + 2);  // what coarse_step(p0) stages
            __syncthreads();
        }
        C ru[QU], rf_[QF];
        load_u(p0, ru);
        put_u(p0, ru);
        if constexpr (HEAD == M3_HEAD_CORR) {
            __syncthreads();
            coarse_step(zr0);
            __syncthreads();
        }
        load_u(zr0, ru);
        load_f(zr0, rf_);
        put_u(zr0, ru);
        put_f(zr0, rf_);
    }
#pragma unroll
    for (int d = 0; d < PD; ++d) {
        load_u(zr0 + 1 + d, pu[d]);
        load_f(zr0 + 1 + d, pf[d]);
        load_fr(zr0 - 3 + d, pr[d]);
    }

    double nacc = 0.0;                 // NORM: this thread's sum of r^2
    C cacc0 = (C)0, cacc1 = (C)0;      // RR: running sums of the coarse point for even / odd coarse planes
    const int cxi = tid % CXN, cyi = tid / CXN;
    const bool has_coarse = TAIL == M3_TAIL_RR && tid < CXN * CYN;
    const int Ic = (i0 + 1) / 2 + cxi, Jc = (j0 + 1) / 2 + cyi;
    const uint32_t ext_fc =
        TAIL == M3_TAIL_RR ? (uint32_t)(((long long)(a.nc - 1) * a.fcp + a.nc) * FB) : 0u;
    const uint32_t fco = (has_coarse && Ic <= a.nc && Jc <= a.nc)
                             ? (uint32_t)((Ic - 1) + (long long)(Jc - 1) * a.fcp) * FB : kOOB;
    const uint32_t ext_o = use_acc ? extent(a.accp, 8u) : extent(a.op, SB);

    for (int zbase = zr0; zbase <= zend; zbase += PD) {
      m3_static_for<PD>([&](auto dc) {
        constexpr int d = dc;
        const int z = zbase + d;
        if (z > zend) return;
        // ---- L: plane z + 1 into the ring, plane z + 1 + PD into flight
        if (z + 1 <= zload1) {
            coarse_step(z + 1);
            put_u(z + 1, pu[d]);
            put_f(z + 1, pf[d]);
            load_u(z + 1 + PD, pu[d]);
            load_f(z + 1 + PD, pf[d]);
        }
        __syncthreads();
        // ---- A: red of plane z on the tile + (R - 1); residual of plane z - 3
        if (z <= zred1 && z >= 1 && z <= n) {
            const C *um = U[slot(z - 1)], *up = U[slot(z + 1)];
            C *uc = U[slot(z)];
            const C *fz = Fs[fslot(z)];
#pragma unroll
            for (int it = 0; it < IR; ++it) {
                const int c = ((rm[it] >> 2) + z) & 1;  // the red one of the pair
                if (!((rm[it] >> c) & 1)) continue;
                const int p = rp[it] + c;
                C s = h2 * fz[rf[it] + c];
                s = s + uc[p - 1];
                s = s + uc[p + 1];
                s = s + uc[p - LX];
                s = s + uc[p + LX];
                s = s + um[p];
                s = s + up[p];
                uc[p] = T::rnd(s * (C)(1.0 / 6.0));
            }
        }
        if constexpr (TAIL != M3_TAIL_NONE) {
            const int zr = z - 3;
            C frc[QR];
            if constexpr (!FRES) {
#pragma unroll
                for (int q = 0; q < QR; ++q) frc[q] = pr[d][q];
                load_fr(z - 3 + PD, pr[d]);
            }
            if (zr >= k0 && zr <= zres1 && zr >= 1 && zr <= n) {
                if constexpr (FRES) {
                    // zr >= k0 > zb: a plane the ring still holds
                    const C *fr = Fs[fslot(zr)];
#pragma unroll
                    for (int q = 0; q < QR; ++q) frc[q] = fr[tid + q * NT < NR ? rsf[q] : 0];
                }
                const C *um = U[slot(zr - 1)], *uc = U[slot(zr)], *up = U[slot(zr + 1)];
#pragma unroll
                for (int q = 0; q < QR; ++q) {
                    if (tid + q * NT >= NR) continue;
                    const int p = rsp[q];
                    const C c = uc[p];
                    C sa = (c - uc[p - 1]) + (c - uc[p + 1]);
                    sa = (sa + (c - uc[p - LX])) + (c - uc[p + LX]);
                    sa = (sa + (c - um[p])) + (c - up[p]);
                    const C r = (rsm[q] & 1) ? frc[q] - sa * ih2 : (C)0;
                    if constexpr (TAIL == M3_TAIL_RR) {
                        Rp[tid + q * NT] = r;
                    } else {
                        const double rd = (double)r;
                        nacc += ((rsm[q] & 2) && zr < k1) ? rd * rd : 0.0;
                    }
                }
            }
        }
        __syncthreads();
        // ---- B: black of plane z - 1 on the tile + (R - 2), store the tile;
        // restriction of the residual plane z - 3
        {
            const int zk = z - 1;
            if (zk >= k0 - EL && zk <= k1 - 1 + EH && zk >= 1 && zk <= n) {
                const C *um = U[slot(zk - 1)], *up = U[slot(zk + 1)];
                C *uc = U[slot(zk)];
                const C *fz = Fs[fslot(zk)];
                const bool st_plane = zk >= k0 && zk < k1;
                const rsrc_t ro_ = use_acc ? plane_rsrc(a.acc, a.accpp, 8u, zk, ext_o, st_plane)
                                           : plane_rsrc(a.uout, a.opp, SB, zk, ext_o, st_plane);
#pragma unroll
                for (int it = 0; it < IB; ++it) {
                    const int c = 1 - (((bm[it] >> 2) + zk) & 1);  // the black one of the pair
                    C vb = (C)0;
                    if ((bm[it] >> c) & 1) {
                        const int p = bp[it] + c;
                        C s = h2 * fz[bf[it] + c];
                        s = s + uc[p - 1];
                        s = s + uc[p + 1];
                        s = s + uc[p - LX];
                        s = s + uc[p + LX];
                        s = s + um[p];
                        s = s + up[p];
                        vb = T::rnd(s * (C)(1.0 / 6.0));
                        uc[p] = vb;
                    }
                    if (bm[it] & 24) {
#pragma unroll
                        for (int e2 = 0; e2 < 2; ++e2) {
                            const C v = (e2 == c) ? vb : uc[bp[it] + e2];
                            const uint32_t off = ((bm[it] >> (3 + e2)) & 1) ? bo[it] + (uint32_t)e2 * OB : kOOB;
                            if (use_acc) bst(ro_, off, bld<double>(ro_, off) + (double)v);
                            else T::bstore(ro_, off, v);
                        }
                    }
                }
            }
        }
        if constexpr (TAIL == M3_TAIL_RR) {
            const int zr = z - 3;
            if (has_coarse && zr >= k0 && zr <= zres1) {
                // residual plane zr is oz = 0 of coarse plane zr / 2 (even zr), or
                // oz = +1 of (zr - 1) / 2 and oz = -1 of (zr + 1) / 2 (odd zr);
                // the coarse point's fine point 2I is residual-plane x = 2 + 2 cxi
                const int rx = 2 + 2 * cxi, ry = 2 + 2 * cyi;
                auto partial = [&](C s, int oz) -> C {
#pragma unroll
                    for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
                        for (int ox = -1; ox <= 1; ++ox) {
                            const int wt = (2 - (ox < 0 ? -ox : ox)) * (2 - (oy < 0 ? -oy : oy)) * (2 - (oz < 0 ? -oz : oz));
                            s = s + (C)wt * Rp[(ry + oy) * RXN + (rx + ox)];
                        }
                    return s;
                };
                // (the coarse-plane parity is uniform over the workgroup)
                if ((zr & 1) == 0) {
                    const int Z = zr >> 1;
                    if (Z & 1) cacc1 = partial(cacc1, 0);
                    else cacc0 = partial(cacc0, 0);
                } else {
                    const int Z = (zr - 1) >> 1;
                    const C sz = partial((Z & 1) ? cacc1 : cacc0, 1);
                    const bool zown = Z >= 1 && Z <= a.nc && 2 * Z >= k0 && 2 * Z < k1;
                    const rsrc_t rc = plane_rsrc(a.fc, a.fcpp, FB, Z, ext_fc, zown);
                    bst(rc, fco, (F)(sz * (C)0.015625));
                    if (Z & 1) cacc0 = partial((C)0, -1);
                    else cacc1 = partial((C)0, -1);
                }
            }
        }
      });
    }

    if constexpr (TAIL == M3_TAIL_NORM) {
        const double w = wave_sum(nacc);
        if ((tid & 63) == 0) wsum[tid >> 6] = w;
        __syncthreads();
        if (tid < 64) {
            double s = 0.0;
            for (int q = 0; q < NT / 64; ++q) s += wsum[q];
            put_partial(a.partials, t, s, 0.0);
        }
    }
}

static int m3_kz(int n, int tail, bool f64)
{
    // planes per workgroup: 64, fewer on small levels so that a launch has
    // at least MGX_M3_MINWG workgroups (default 256, one per CU); each run
    // recomputes one or two planes below and above it, so shorter runs cost
    // redundant work (measured at 255^3: 0.62 ms per cycle for the level's
    // four passes with at least 2048 workgroups, 0.43 ms with 256)
    static const int minwg = [] {
        const char *v = getenv("MGX_M3_MINWG");
        const int x = v && *v ? atoi(v) : 256;
        return x > 0 ? x : 256;
    }();
    const M3Shape sh = m3_shape(tail, f64);
    const int ntx = (n + sh.tx - 1) / sh.tx, nty = (n + sh.ty - 1) / sh.ty;
    int kz = 64;
    while (kz > 8 && (long long)ntx * nty * ((n + kz - 1) / kz) < minwg) kz /= 2;
    return kz;
}

int march3d_blocks(int n, int tail, int st)
{
    const M3Shape sh = m3_shape(tail, st == ST_F64);
    const int kz = m3_kz(n, tail, st == ST_F64);
    return ((n + sh.tx - 1) / sh.tx) * ((n + sh.ty - 1) / sh.ty) * ((n + kz - 1) / kz);
}

template <class S, class F, int HEAD, int TAIL>
static void m3_go(const M3Args &a, dim3 grid, hipStream_t s)
{
    constexpr M3Shape sh = m3_shape(TAIL, sizeof(S) == 8);
    hipLaunchKernelGGL((k_march3d<S, F, HEAD, TAIL, sh.tx, sh.ty, sh.nt, MGX_M3_PD>), grid, dim3(sh.nt), 0, s, a);
}

template <class S, class F, int HEAD>
static hipError_t m3_tail(int tail, const M3Args &a, dim3 grid, hipStream_t s)
{
    switch (tail) {
    case M3_TAIL_NONE: m3_go<S, F, HEAD, M3_TAIL_NONE>(a, grid, s); break;
    case M3_TAIL_RR: m3_go<S, F, HEAD, M3_TAIL_RR>(a, grid, s); break;
    case M3_TAIL_NORM:
        if constexpr (sizeof(S) == 8) {
            m3_go<S, F, HEAD, M3_TAIL_NORM>(a, grid, s);
            break;
        }
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class S, class F>
static hipError_t m3_head(int head, int tail, const M3Args &a, dim3 grid, hipStream_t s)
{
    switch (head) {
    case M3_HEAD_U: return m3_tail<S, F, M3_HEAD_U>(tail, a, grid, s);
    case M3_HEAD_ZERO: return m3_tail<S, F, M3_HEAD_ZERO>(tail, a, grid, s);
    case M3_HEAD_CORR: return m3_tail<S, F, M3_HEAD_CORR>(tail, a, grid, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_march3d(int st, int head, int tail, const M3Args &in, hipStream_t s)
{
    M3Args a = in;
    a.kz = m3_kz(a.n, tail, st == ST_F64);
    const M3Shape sh = m3_shape(tail, st == ST_F64);
    a.ntx = (a.n + sh.tx - 1) / sh.tx;
    a.nty = (a.n + sh.ty - 1) / sh.ty;
    a.ntz = (a.n + a.kz - 1) / a.kz;
    const long long nb = (long long)a.ntx * a.nty * a.ntz;
    if (nb < 1 || nb > 0x7fffffffLL - 8) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((nb + 7) / 8 * 8));
    switch (st) {
    case ST_F64: return m3_head<double, double>(head, tail, a, grid, s);
    case ST_F32: return m3_head<float, float>(head, tail, a, grid, s);
    case ST_BF16: return m3_head<bf16_t, float>(head, tail, a, grid, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace mgx
