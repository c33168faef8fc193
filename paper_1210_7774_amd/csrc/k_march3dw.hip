// Wavefront 3D level passes: one or two red-black Gauss-Seidel sweeps of the
// 7-point Poisson operator per pass over a 32 x 32 column tile, with the
// operations next to them in the cycle fused in front (zero start, trilinear
// coarse-grid correction) and behind (residual + full-weighting restriction,
// or the residual's squared norm, or adding the result into an FP64 iterate).
//
// Every thread owns a pair of x-adjacent columns of the tile's loaded region
// (the tile plus a halo of R points) for the whole march up the planes.  The
// two columns hold one point of each colour class ((i + j) even / odd), so in
// every plane exactly one of them is red.  A thread keeps its columns' values
// of the last eight planes, and their right-hand side, in registers: the
// vertical neighbours of every update and of the residual never leave the
// thread.  Only in-plane neighbours go through LDS, in a ring of planes stored
// by colour class (all class-0 points row by row, then all class-1 points),
// so the three in-plane neighbours a point does not own are one LDS read and
// one two-address read, and the lanes of a wave read consecutive elements
// (no bank conflicts).
//
// At step z the march brings plane z into LDS and updates, with two barriers
// per step (phase A | phase B):
//   A: red of sweep 1 on plane z, red of sweep 2 on plane z - 3, and the
//      restriction of the residual plane finished in the previous step;
//   B: black of sweep 1 on plane z - 1, black of sweep 2 on plane z - 4 (the
//      plane is then final and is stored), and the residual of plane z - 5.
// (One sweep: red z | black z - 1, store, residual z - 2.)  These lags are the
// red-black order: each update reads neighbour values of exactly the half
// sweep the unfused sweeps would give it.  Each stage works on the loaded
// region shrunk by one point more than the stage before it (the halo is
// recomputed, as in the paper's blockable rule -- "Vector Engine" section --
// a kernel must not read shifted views of what it writes unless every tile is
// self-contained), and in z on the planes of the run grown by the same
// margins.  Sum orders are those of the unfused kernels except where noted
// (rounding-level differences).
#include <algorithm>
#include <cstdlib>
#include <utility>

#include "dev_common.h"
#include "mg_m3.h"

#ifndef MGX_W3_PD
#define MGX_W3_PD 1
#endif
#ifndef MGX_W3_PD_CORR
#define MGX_W3_PD_CORR 1
#endif
#ifndef MGX_W3_ONEBAR
#define MGX_W3_ONEBAR 1  // one barrier per step (every stage's LDS inputs come from earlier steps)
#endif
#ifndef MGX_W3_RESREG
#define MGX_W3_RESREG 1  // two sweeps: the residual's plane and the one below from registers (1) or LDS (0)
#endif

namespace mgx {

template <int... Q, class Fn>
__device__ __forceinline__ void w3_static_for_impl(std::integer_sequence<int, Q...>, Fn &&fn)
{
    (fn(std::integral_constant<int, Q>{}), ...);
}
template <int N, class Fn>
__device__ __forceinline__ void w3_static_for(Fn &&fn)
{
    w3_static_for_impl(std::make_integer_sequence<int, N>{}, fn);
}

// Geometry of a pass with NS sweeps and the given tail.
template <int NS, int TAIL>
struct W3Geo {
    static constexpr int T = 32;  // owned tile edge (columns)
    // halo: 2 per sweep, + 2 for residual + restriction (the restriction reads
    // the residual one point around the tile), + 1 for the norm
    static constexpr int R = 2 * NS + (TAIL == M3_TAIL_RR ? 2 : TAIL == M3_TAIL_NORM ? 1 : 0);
    static constexpr int LX = T + 2 * R, LY = LX, PX = LX / 2, NP = PX * LY;
    static constexpr int NT = (NP + 63) / 64 * 64;
    static constexpr int DL = NS == 2 ? 8 : 4;      // LDS ring planes
    static constexpr int LB = 3 * (NS - 1) + 1;     // lag of the last black stage
    static constexpr int LR = LB + 1;               // lag of the residual
    static_assert(LX % 2 == 0, "pairs of columns");
};

template <class S, class F, int NS, int HEAD, int TAIL>
__global__ __launch_bounds__((W3Geo<NS, TAIL>::NT)) void k_march3dw(M3Args a)
{
    using G = W3Geo<NS, TAIL>;
    using Tr = Traits<S>;
    using C = typename Tr::C;
    constexpr int TT = G::T, R = G::R, LX = G::LX, LY = G::LY, PX = G::PX, NP = G::NP, NT = G::NT;
    constexpr int DL = G::DL, LB = G::LB, LR = G::LR;
    constexpr int PLN = 2 * PX * LY + 2;            // one LDS plane (+ a spare pair for idle threads)
    constexpr int RX = TT + 2;                      // residual region edge (RR)
    constexpr int NRP = TAIL == M3_TAIL_RR ? RX * RX + 1 : 1;  // + a spare element
    constexpr int KCX = LX / 2 + 3, NKC = HEAD == M3_HEAD_CORR ? KCX * KCX : 1;
    constexpr int QC = (NKC + NT - 1) / NT;
    // planes of loads in flight (one with the correction's registers)
    constexpr int PD = HEAD == M3_HEAD_CORR ? MGX_W3_PD_CORR : MGX_W3_PD;
    constexpr int CN = TT / 2;                      // coarse points per tile edge (RR)
    constexpr uint32_t SB = sizeof(S), FB = sizeof(F);
    // residual margin: the tile + 1 (RR) or the tile (NORM)
    constexpr int MRES = TAIL == M3_TAIL_RR ? R - 1 : R;
    static_assert(TAIL != M3_TAIL_RR || CN * CN <= NT, "one coarse point per thread");

    __shared__ C U[DL * PLN];
    __shared__ C Rp[MGX_W3_ONEBAR ? 2 : 1][NRP];  // (two planes: written and read in one phase)
    __shared__ C Kc[HEAD == M3_HEAD_CORR ? 3 * NKC : 1];
    __shared__ double wsum[NT / 64];

    if (a.state && a.state->done) return;
    // Tiles are dealt to the 8 XCDs round-robin; each XCD gets a contiguous
    // range of the tile order, and the order runs through bands of four tile
    // rows column by column, so an XCD's tiles form a compact block whose
    // shared halo lines meet in its L2 while they march up the same planes.
    const int ntt = a.ntx * a.nty, nb = ntt * a.ntz;
    const int per = (nb + 7) / 8;
    const int t = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (t >= nb) return;
    const int run = t / ntt, tu = t % ntt;
    const int band = tu / (4 * a.ntx), brem = tu % (4 * a.ntx);
    const int bh = min(4, a.nty - 4 * band);
    const int i0 = (brem / bh) * TT + 1, j0 = (4 * band + brem % bh) * TT + 1;
    const int n = a.n;
    const int k0 = run * a.kz + 1, k1 = min(k0 + a.kz, n + 1);
    const int tid = threadIdx.x;
    const C h2 = (C)a.h2, ih2 = (C)a.ih2;

    // ---- the thread's pair of columns ---------------------------------------
    const bool act = NP == NT || tid < NP;
    const int y = act ? tid / PX : 0, kp = act ? tid % PX : 0;
    const int j = j0 - R + y;
    const bool jin = j >= 1 && j <= n;
    int ex[2], xc[2], dm[2];
    ex[0] = (i0 - R + j) & 1;  // x offset in the pair of the class-0 point
    ex[1] = 1 - ex[0];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        xc[c] = 2 * kp + ex[c];
        const int i = i0 - R + xc[c];
        const int dist = min(min(xc[c], LX - 1 - xc[c]), min(y, LY - 1 - y));
        // stage test: a stage of margin m updates the point when dm >= m
        dm[c] = (act && jin && i >= 1 && i <= n) ? dist : -1;
    }
    const bool rreg[2] = {act && min(min(xc[0], LX - 1 - xc[0]), min(y, LY - 1 - y)) >= R - 1,
                          act && min(min(xc[1], LX - 1 - xc[1]), min(y, LY - 1 - y)) >= R - 1};

    // memory: one buffer descriptor per plane, a byte offset per point
    auto off = [&](int c, long long pitch, uint32_t es, bool ok) -> uint32_t {
        const int i = i0 - R + xc[c];
        return ok ? (uint32_t)((long long)(i - 1) + (long long)(j - 1) * pitch) * es : kOOB;
    };
    // (adding into an FP64 iterate is the refinement's, whose inner cycles
    // keep a 4- or 2-byte state; the launcher rejects it for an FP64 state)
    const bool use_acc = sizeof(S) < 8 && a.acc != nullptr;
    const uint32_t OB = use_acc ? 8u : SB;
    const long long opitch = use_acc ? a.accp : a.op, oppitch = use_acc ? a.accpp : a.opp;
    uint32_t uo[2], fo[2], so[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        uo[c] = off(c, a.ip, SB, dm[c] >= 0);
        fo[c] = off(c, a.fp, FB, dm[c] >= 0);
        so[c] = off(c, opitch, OB, dm[c] >= R);  // owned points only
    }
    auto extent = [&](long long pitch, uint32_t es) -> uint32_t {
        return (uint32_t)(((long long)(n - 1) * pitch + n) * es);
    };
    auto plane_rsrc = [&](const void *base, long long ppitch, uint32_t es, int k, uint32_t ext, bool ok) {
        const int kk = min(max(k, 1), n);
        return make_rsrc((const char *)base + (long long)(kk - 1) * ppitch * es, ok ? ext : 0u);
    };
    const uint32_t ext_u = extent(a.ip, SB), ext_f = extent(a.fp, FB), ext_o = extent(opitch, OB);

    // LDS element indices inside a plane: my class-c point, the neighbour in
    // x of the class-c point that the partner is not, the point above (y - 1)
    // of the class-c point (the one below is 2 PX further)
    int me[2], xn[2], yb[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        me[c] = act ? c * PX * LY + y * PX + kp : 2 * PX * LY + c;
        const int kx = min(max(kp + (ex[c] ? 1 : -1), 0), PX - 1);
        xn[c] = (1 - c) * PX * LY + y * PX + kx;
        yb[c] = (1 - c) * PX * LY + min(max(y - 1, 0), LY - 3) * PX + kp;
    }
    // residual region index (RR), or the spare element: rows of the region,
    // each split by x parity (even x, then odd x), so that the coarse points'
    // reads (x = 2I - 1, 2I, 2I + 1 across consecutive I) are consecutive
    auto rp_index = [](int xr, int yr) { return yr * RX + (xr & 1) * (RX / 2) + (xr >> 1); };
    int rpi[2];
#pragma unroll
    for (int c = 0; c < 2; ++c)
        rpi[c] = (TAIL == M3_TAIL_RR && rreg[c]) ? rp_index(xc[c] - (R - 1), y - (R - 1)) : NRP - 1;

    // ---- plane schedule -----------------------------------------------------
    // stage of margin m works on planes [k0 - R + m, k1 - 1 + R - m] in the
    // domain; loads cover [k0 - R, k1 - 1 + R]; the first step is even so
    // that a plane's red class is known at compile time in the unrolled loop
    const int z0 = max(k0 - R, 0) & ~1;
    const int zl1 = min(k1 - 1 + R, n + 1);
    auto lo = [&](int m) { return max(1, k0 - R + m); };
    auto hi = [&](int m) { return min(n, k1 - 1 + R - m); };
    const int rlo = k0, rhi = TAIL == M3_TAIL_RR ? min(k1, n) : k1 - 1;  // residual planes
    const int zend = TAIL == M3_TAIL_RR ? rhi + LR + 1 : TAIL == M3_TAIL_NORM ? rhi + LR : k1 - 1 + LB;

    // ---- registers: the pair's last 8 planes of u and f, loads in flight -----
    C ur[8][2], fr[8][2], pu[PD][2], pf[PD][2];
#pragma unroll
    for (int p = 0; p < 8; ++p) ur[p][0] = ur[p][1] = fr[p][0] = fr[p][1] = (C)0;

    auto load_u = [&](int k, C (&ru)[2]) {
        if constexpr (HEAD == M3_HEAD_ZERO) {
            ru[0] = ru[1] = (C)0;
        } else {
            const rsrc_t r = plane_rsrc(a.uin, a.ipp, SB, k, ext_u, k >= 1 && k <= n && k <= zl1);
            ru[0] = Tr::bload(r, uo[0]);
            ru[1] = Tr::bload(r, uo[1]);
        }
    };
    auto load_f = [&](int k, C (&rf)[2]) {
        const rsrc_t r = plane_rsrc(a.f, a.fpp, FB, k, ext_f, k >= 1 && k <= n && k <= zl1);
        rf[0] = (C)bld<F>(r, fo[0]);
        rf[1] = (C)bld<F>(r, fo[1]);
    };

    // ---- coarse correction (HEAD_CORR) ----------------------------------------
    // Coarse planes are staged in LDS, three slots (plane K in slot K % 3):
    // fine plane p needs coarse plane p / 2, and p / 2 + 1 when p is odd.  The
    // correction of a point is the bilinear (x, y) interpolation Pa of plane
    // p / 2 (p even) or (Pa + Pb) / 2 with Pb that of p / 2 + 1 (p odd) -- the
    // order of the unfused prolongation kernel (x, y, then z); it is computed
    // when the plane enters the registers.  Coarse plane K + 2 is loaded when
    // fine plane 2K enters and staged when 2K + 1 does, two steps (four
    // barriers) before fine plane 2K + 3 first reads it and after the last
    // reader of the slot's previous plane.
    const int ci0 = (i0 - R) >> 1, cj0 = (j0 - R) >> 1;  // floor
    C pk[QC];
    uint32_t co[QC];
    const uint32_t ext_c = HEAD == M3_HEAD_CORR ? (uint32_t)(((long long)(a.nc - 1) * a.ucp + a.nc) * SB) : 0u;
    if constexpr (HEAD == M3_HEAD_CORR) {
#pragma unroll
        for (int q = 0; q < QC; ++q) {
            const int p = tid + q * NT;
            const int I = ci0 + p % KCX, J = cj0 + p / KCX;
            co[q] = (p < NKC && I >= 1 && I <= a.nc && J >= 1 && J <= a.nc)
                        ? (uint32_t)((I - 1) + (long long)(J - 1) * a.ucp) * SB : kOOB;
        }
    }
    auto load_coarse = [&](int K) {
        if constexpr (HEAD == M3_HEAD_CORR) {
            const rsrc_t rc = plane_rsrc(a.uc, a.ucpp, SB, K, ext_c, K >= 1 && K <= a.nc);
#pragma unroll
            for (int q = 0; q < QC; ++q) pk[q] = Tr::bload(rc, co[q]);
        }
    };
    auto put_coarse = [&](int K) {
        if constexpr (HEAD == M3_HEAD_CORR) {
            C *dst = Kc + (K % 3) * NKC;
#pragma unroll
            for (int q = 0; q < QC; ++q) {
                const int p = tid + q * NT;
                if (p < NKC) dst[p] = pk[q];
            }
        }
    };
    // bilinear interpolation of staged coarse plane K at my class-c point
    // (per class of the pair: both columns lie between coarse columns I and
    // I + 1, I = floor of the left column / 2, so the pair reads four values)
    const int il = i0 - R + 2 * (act ? xc[0] >> 1 : 0);     // the pair's left column
    const bool lodd = (i0 - R) & 1;                         // (the same for every pair)
    const int kb = act ? ((j >> 1) - cj0) * KCX + (il >> 1) - ci0 : 0;
    auto bilin = [&](int K, C (&out)[2]) {
        const C *pl = Kc + (K % 3) * NKC;
        const C a00 = pl[kb], a01 = pl[kb + 1], a10 = pl[kb + KCX], a11 = pl[kb + KCX + 1];
        const C m0 = (a00 + a01) * (C)0.5, m1 = (a10 + a11) * (C)0.5;
        // left column: on coarse column I (even) or between I and I + 1 (odd);
        // right column: between them (left even) or on I + 1 (left odd)
        const C l0L = lodd ? m0 : a00, l1L = lodd ? m1 : a10;
        const C l0R = lodd ? a01 : m0, l1R = lodd ? a11 : m1;
        const bool yo = j & 1;
        const C vL = yo ? (l0L + l1L) * (C)0.5 : l0L, vR = yo ? (l0R + l1R) * (C)0.5 : l0R;
        out[0] = ex[0] ? vR : vL;
        out[1] = ex[0] ? vL : vR;
    };
    // staging for the plane p that enters next (p in order)
    auto coarse_step = [&](int p) {
        if constexpr (HEAD == M3_HEAD_CORR) {
            if (p & 1) put_coarse((p >> 1) + 2);
            else load_coarse((p >> 1) + 2);
        }
    };
    // the plane's values as they enter the registers (correction added)
    auto enter = [&](int p, const C (&ru)[2], C (&dst)[2]) {
        dst[0] = ru[0];
        dst[1] = ru[1];
        if constexpr (HEAD == M3_HEAD_CORR) {
            if (p >= 1 && p <= n) {
                const int K = p >> 1;
                C pa[2], pb[2];
                bilin(K, pa);
                if (p & 1) bilin(K + 1, pb);
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const C corr = (p & 1) ? (pa[c] + pb[c]) * (C)0.5 : pa[c];
                    if (dm[c] >= 0) dst[c] = Tr::rnd(ru[c] + corr);
                }
            }
        }
    };

    // ---- prologue: plane z0 into the registers, z0 + 1 .. z0 + PD in flight ---
    {
        if constexpr (HEAD == M3_HEAD_CORR) {
            const int K0 = z0 >> 1;  // z0 is even
            load_coarse(K0);
            put_coarse(K0);
            load_coarse(K0 + 1);
            put_coarse(K0 + 1);
            load_coarse(K0 + 2);     // staged when z0 + 1 enters
            __syncthreads();
        }
        C ru[2];
        load_u(z0, ru);
        load_f(z0, fr[0]);
        enter(z0, ru, ur[0]);
    }
#pragma unroll
    for (int d = 0; d < PD; ++d) {
        load_u(z0 + 1 + d, pu[(1 + d) % PD]);
        load_f(z0 + 1 + d, pf[(1 + d) % PD]);
    }

    // one Gauss-Seidel update of the class-c point of the plane in LDS slot
    // `pl`, its vertical neighbours zm / zp and partner from the registers
    // (in x the partner is added first: the order of the two x neighbours
    // then differs from the unfused kernels' by the point's side in the pair,
    // a rounding-level difference)
    auto gs = [&](const C *pl, int c, C fv, C partner, C zm, C zp) -> C {
        const C xo = pl[xn[c]];
        const C ym = pl[yb[c]], yp = pl[yb[c] + 2 * PX];
        C s = h2 * fv;
        s = s + partner;
        s = s + xo;
        s = s + ym;
        s = s + yp;
        s = s + zm;
        s = s + zp;
        return Tr::rnd(s * (C)(1.0 / 6.0));
    };
    auto resid = [&](const C *pl, int c, C fv, C cen, C partner, C zm, C zp) -> C {
        const C xo = pl[xn[c]];
        const C ym = pl[yb[c]], yp = pl[yb[c] + 2 * PX];
        C sa = (cen - partner) + (cen - xo);
        sa = (sa + (cen - ym)) + (cen - yp);
        sa = (sa + (cen - zm)) + (cen - zp);
        return fv - sa * ih2;
    };

    double nacc = 0.0;             // NORM: this thread's sum of r^2
    C cacc0 = (C)0, cacc1 = (C)0;  // RR: running sums of the coarse point for even / odd coarse planes
    const int cxi = tid % CN, cyi = tid / CN;
    const bool has_coarse = TAIL == M3_TAIL_RR && tid < CN * CN;
    const int Ic = (i0 + 1) / 2 + cxi, Jc = (j0 + 1) / 2 + cyi;
    const uint32_t ext_fc =
        TAIL == M3_TAIL_RR ? (uint32_t)(((long long)(a.nc - 1) * a.fcp + a.nc) * FB) : 0u;
    const uint32_t fco = (has_coarse && Ic <= a.nc && Jc <= a.nc)
                             ? (uint32_t)((Ic - 1) + (long long)(Jc - 1) * a.fcp) * FB : kOOB;

    // planes the loop loads next (z + 1 + PD at step z)
    const long long upb = a.ipp * SB, fpb = a.fpp * FB;
    const char *unext = (const char *)a.uin + (long long)(z0 + PD) * upb;
    const char *fnext = (const char *)a.f + (long long)(z0 + PD) * fpb;

    // FP64 iterate (refinement): its values at the owned points of the next
    // plane to be stored, loaded one step ahead of the read-add-write
    double ap[2] = {0.0, 0.0};
    auto load_acc = [&](int q) {
        const bool ok = q >= k0 && q < k1 && q >= 1 && q <= n;
        const rsrc_t r = plane_rsrc(a.acc, oppitch, 8u, q, ext_o, ok);
        ap[0] = bld<double>(r, so[0]);
        ap[1] = bld<double>(r, so[1]);
    };
    if (use_acc) load_acc(z0 - LB);
    // the plane the loop stores next (z - LB at step z; out of range: no records)
    const long long opb = oppitch * OB;
    const char *onext = (const char *)(use_acc ? (const void *)a.acc : a.uout) + (long long)(z0 - LB - 1) * opb;

    for (int zb = z0; zb <= zend; zb += 8) {
      w3_static_for<8>([&](auto dc) {
        constexpr int d = dc;
        // register ring index of plane z + o, LDS slot of plane z + o
        constexpr auto ri = [](int o) { return ((d + o) % 8 + 8) % 8; };
        constexpr auto ls = [](int o) { return ((d + o) % DL + DL) % DL; };
        const int z = zb + d;
        if (z > zend) return;
        // ---- L: plane z into LDS; plane z + 1 into the registers; plane
        // z + 1 + PD into flight
        {
            C *dst = U + ls(0) * PLN;
            dst[me[0]] = ur[ri(0)][0];
            dst[me[1]] = ur[ri(0)][1];
            constexpr int fs = (d + 1) % PD;
            coarse_step(z + 1);
            enter(z + 1, pu[fs], ur[ri(1)]);
            fr[ri(1)][0] = pf[fs][0];
            fr[ri(1)][1] = pf[fs][1];
            // (the march's loads are in plane order: running plane addresses,
            // no product per descriptor; k >= 1 here)
            {
                const bool okk = z + 1 + PD <= min(n, zl1);
                if constexpr (HEAD == M3_HEAD_ZERO) {
                    pu[fs][0] = pu[fs][1] = (C)0;
                } else {
                    const rsrc_t r = make_rsrc(unext, okk ? ext_u : 0u);
                    pu[fs][0] = Tr::bload(r, uo[0]);
                    pu[fs][1] = Tr::bload(r, uo[1]);
                }
                const rsrc_t rf_ = make_rsrc(fnext, okk ? ext_f : 0u);
                pf[fs][0] = (C)bld<F>(rf_, fo[0]);
                pf[fs][1] = (C)bld<F>(rf_, fo[1]);
                unext += upb;
                fnext += fpb;
            }
        }
        __syncthreads();
        // ---- A: red stages; restriction of the residual plane of the last step
        {
            constexpr int c = d & 1;  // the red class of plane z (z0 is even)
            const int ok = z >= lo(1) && z <= hi(1) ? 1 : LX;  // (a margin no point has)
            C *pl = U + ls(0) * PLN;
            const C v = gs(pl, c, fr[ri(0)][c], ur[ri(0)][1 - c], ur[ri(-1)][c], ur[ri(1)][c]);
            ur[ri(0)][c] = dm[c] >= ok ? v : ur[ri(0)][c];
            pl[me[c]] = ur[ri(0)][c];
        }
        if constexpr (NS == 2) {
            constexpr int c = (d + 1) & 1;  // the red class of plane z - 3
            const int q = z - 3;
            const int ok = q >= lo(3) && q <= hi(3) ? 3 : LX;
            C *pl = U + ls(-3) * PLN;
            const C zm = U[ls(-4) * PLN + me[c]];  // (plane z - 4 from LDS: fewer live registers)
            const C v = gs(pl, c, fr[ri(-3)][c], ur[ri(-3)][1 - c], zm, ur[ri(-2)][c]);
            ur[ri(-3)][c] = dm[c] >= ok ? v : ur[ri(-3)][c];
            pl[me[c]] = ur[ri(-3)][c];
        }
        if constexpr (TAIL == M3_TAIL_RR) {
            const int zr = z - LR - 1;
            if (has_coarse && zr >= rlo && zr <= rhi) {
                // residual plane zr is oz = 0 of coarse plane zr / 2 (even zr), or
                // oz = +1 of (zr - 1) / 2 and oz = -1 of (zr + 1) / 2 (odd zr);
                // the coarse point's fine point 2I is residual-region x = 2 + 2 cxi
                const int rx = 2 + 2 * cxi, ry = 2 + 2 * cyi;
                // 3 x 3 weighted sum of residual plane zr around the coarse
                // point, weight (2 - |ox|)(2 - |oy|) wz, in a fixed order
                auto partial = [&](C s, C wz) -> C {
#pragma unroll
                    for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
                        for (int ox = -1; ox <= 1; ++ox) {
                            const int wt = (2 - (ox < 0 ? -ox : ox)) * (2 - (oy < 0 ? -oy : oy));
                            s = s + ((C)wt * wz) * Rp[MGX_W3_ONEBAR ? (d + 1) & 1 : 0][rp_index(rx + ox, ry + oy)];
                        }
                    return s;
                };
                // (the coarse-plane parity is uniform over the workgroup)
                if constexpr (((d - LR - 1) & 1) == 0) {  // zr even (zr - d is even)
                    const int Z = zr >> 1;
                    if (Z & 1) cacc1 = partial(cacc1, (C)2);
                    else cacc0 = partial(cacc0, (C)2);
                } else {
                    // weight 1 for both coarse planes: one sum, added to the
                    // plane below (which is then complete) and starting the one
                    // above (the unfused kernel adds the taps to the running
                    // sum one by one: a rounding-level difference)
                    const int Z = (zr - 1) >> 1;
                    const C tz = partial((C)0, (C)1);
                    const C sz = ((Z & 1) ? cacc1 : cacc0) + tz;
                    const bool zown = Z >= 1 && Z <= a.nc && 2 * Z >= k0 && 2 * Z < k1;
                    const rsrc_t rc = plane_rsrc(a.fc, a.fcpp, FB, Z, ext_fc, zown);
                    bst(rc, fco, (F)(sz * (C)0.015625));
                    if (Z & 1) cacc0 = tz;
                    else cacc1 = tz;
                }
            }
        }
        if constexpr (!MGX_W3_ONEBAR) __syncthreads();
        // ---- B: black stages, the store of the final plane, the residual
        {
            constexpr int c = d & 1;  // the black class of plane z - 1
            const int q = z - 1;
            const int ok = q >= lo(2) && q <= hi(2) ? 2 : LX;
            C *pl = U + ls(-1) * PLN;
            const C v = gs(pl, c, fr[ri(-1)][c], ur[ri(-1)][1 - c], ur[ri(-2)][c], ur[ri(0)][c]);
            ur[ri(-1)][c] = dm[c] >= ok ? v : ur[ri(-1)][c];
            pl[me[c]] = ur[ri(-1)][c];
        }
        if constexpr (NS == 2) {
            constexpr int c = (d + 1) & 1;  // the black class of plane z - 4
            const int q = z - 4;
            const int ok = q >= lo(4) && q <= hi(4) ? 4 : LX;
            C *pl = U + ls(-4) * PLN;
            const C zm = U[ls(-5) * PLN + me[c]];
            const C v = gs(pl, c, fr[ri(-4)][c], ur[ri(-4)][1 - c], zm, ur[ri(-3)][c]);
            ur[ri(-4)][c] = dm[c] >= ok ? v : ur[ri(-4)][c];
            pl[me[c]] = ur[ri(-4)][c];
        }
        {
            // plane z - LB is final: store the owned points
            const int q = z - LB;
            // (a plane outside the run gets no records: the stores are dropped)
            const bool ok = q >= k0 && q < k1 && q >= 1 && q <= n;
            const rsrc_t ro = make_rsrc(onext, ok ? ext_o : 0u);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const C v = ur[ri(-LB)][c];
                if (use_acc) bst(ro, so[c], ap[c] + (double)v);
                else Tr::bstore(ro, so[c], v);
            }
            onext += opb;
            if (use_acc) {
                const bool ok1 = q + 1 >= k0 && q + 1 < k1 && q + 1 >= 1 && q + 1 <= n;
                const rsrc_t r1 = make_rsrc(onext, ok1 ? ext_o : 0u);
                ap[0] = bld<double>(r1, so[0]);
                ap[1] = bld<double>(r1, so[1]);
            }
        }
        if constexpr (TAIL != M3_TAIL_NONE) {
            const int q = z - LR;
            const int ok = q >= rlo && q <= rhi ? MRES : LX;
            {
                const C *pl = U + ls(-LR) * PLN;
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    // two sweeps: the plane and the one below from LDS, or the
                    // one below only (the correction pass: fewest spilled
                    // registers), or neither (from the registers)
                    constexpr bool lds = NS == 2 && !MGX_W3_RESREG;
                    constexpr bool lzm = NS == 2 && (lds || HEAD == M3_HEAD_CORR);
                    const C cen = lds ? pl[me[c]] : ur[ri(-LR)][c];
                    const C prt = lds ? pl[me[1 - c]] : ur[ri(-LR)][1 - c];
                    const C zm = lzm ? U[ls(-LR - 1) * PLN + me[c]] : ur[ri(-LR - 1)][c];
                    const C r = resid(pl, c, fr[ri(-LR)][c], cen, prt, zm, ur[ri(-LR + 1)][c]);
                    if constexpr (TAIL == M3_TAIL_RR) {
                        Rp[MGX_W3_ONEBAR ? d & 1 : 0][rpi[c]] = dm[c] >= ok ? r : (C)0;
                    } else {
                        const double rd = (double)r;
                        nacc += dm[c] >= ok ? rd * rd : 0.0;
                    }
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

// planes per run: one run per tile column when the level has at least 256
// tiles (one workgroup per CU), else shorter runs so that a launch has about
// 256 workgroups; runs are an even number of planes (coarse planes then never
// straddle two runs' restriction ownership)
static int w3_kz(int n)
{
    const int nt = (n + 31) / 32;
    const int tiles = nt * nt;
    const int runs = std::max(1, 256 / tiles);
    int kz = (n + runs - 1) / runs;
    kz += kz & 1;
    return kz;
}

int march3dw_blocks(int n)
{
    const int nt = (n + 31) / 32;
    const int kz = w3_kz(n);
    return nt * nt * ((n + kz - 1) / kz);
}

template <class S, class F, int NS, int HEAD, int TAIL>
static void w3_go(const M3Args &a, dim3 grid, hipStream_t s)
{
    hipLaunchKernelGGL((k_march3dw<S, F, NS, HEAD, TAIL>), grid, dim3(W3Geo<NS, TAIL>::NT), 0, s, a);
}

template <class S, class F, int NS, int HEAD>
static hipError_t w3_tail(int tail, const M3Args &a, dim3 grid, hipStream_t s)
{
    switch (tail) {
    case M3_TAIL_NONE: w3_go<S, F, NS, HEAD, M3_TAIL_NONE>(a, grid, s); break;
    case M3_TAIL_RR:
        // (the cycle never restricts right after a correction)
        if constexpr (HEAD != M3_HEAD_CORR) {
            w3_go<S, F, NS, HEAD, M3_TAIL_RR>(a, grid, s);
            break;
        }
        return hipErrorInvalidValue;
    case M3_TAIL_NORM:
        if constexpr (sizeof(S) == 8) {
            w3_go<S, F, NS, HEAD, M3_TAIL_NORM>(a, grid, s);
            break;
        }
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class S, class F, int NS>
static hipError_t w3_head(int head, int tail, const M3Args &a, dim3 grid, hipStream_t s)
{
    switch (head) {
    case M3_HEAD_U: return w3_tail<S, F, NS, M3_HEAD_U>(tail, a, grid, s);
    case M3_HEAD_ZERO: return w3_tail<S, F, NS, M3_HEAD_ZERO>(tail, a, grid, s);
    case M3_HEAD_CORR: return w3_tail<S, F, NS, M3_HEAD_CORR>(tail, a, grid, s);
    }
    return hipErrorInvalidValue;
}

template <class S, class F>
static hipError_t w3_ns(int ns, int head, int tail, const M3Args &a, dim3 grid, hipStream_t s)
{
    if (ns == 1) return w3_head<S, F, 1>(head, tail, a, grid, s);
    if (ns == 2) return w3_head<S, F, 2>(head, tail, a, grid, s);
    return hipErrorInvalidValue;
}

hipError_t launch_march3dw(int st, int ns, int head, int tail, const M3Args &in, hipStream_t s)
{
    M3Args a = in;
    if (st == ST_F64 && a.acc) return hipErrorInvalidValue;
    a.kz = w3_kz(a.n);
    a.ntx = a.nty = (a.n + 31) / 32;
    a.ntz = (a.n + a.kz - 1) / a.kz;
    const long long nb = (long long)a.ntx * a.nty * a.ntz;
    if (nb < 1 || nb > 0x7fffffffLL - 8) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((nb + 7) / 8 * 8));
    switch (st) {
    case ST_F64: return w3_ns<double, double>(ns, head, tail, a, grid, s);
    case ST_F32: return w3_ns<float, float>(ns, head, tail, a, grid, s);
    case ST_BF16: return w3_ns<bf16_t, float>(ns, head, tail, a, grid, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace mgx
