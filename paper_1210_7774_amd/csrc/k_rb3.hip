// One full red-black Gauss-Seidel sweep of the 3D 7-point Poisson operator in
// one pass (out of place: uin -> uout).
//
// A red-black sweep is two half sweeps; run separately each one streams the
// whole state (the colours interleave within every cache line).  Here a
// workgroup owns a 32 x 16 column tile and a run of planes and marches
// up the planes with a lag of one: at step z it updates the red points of
// plane z, then the black points of plane z - 1, which then is final and is
// stored.  This is the red-black order exactly: red at plane z reads black
// values that are still old (black z - 1 and z + 1 are updated later), black
// at z - 1 reads red values that are all new.  In the plane, black on the
// tile needs red on a one-point ring and red there needs old black on a
// two-point ring, so the workgroup loads its tile plus two points of halo and
// recomputes the ring (the fusion the paper's blockable rule, "Vector
// Engine" section, forbids for elementwise kernels, made legal by the
// recomputed halo).  Four planes of u and two of f live in LDS; the next
// plane's loads are issued into registers before the current plane's
// updates, so memory latency overlaps the arithmetic.
#include "dev_common.h"

namespace mgx {

constexpr int kRX = 32, kRY = 16;                   // owned column tile
constexpr int kUX = kRX + 4, kUY = kRY + 4;          // u region: tile + 2
constexpr int kFX = kRX + 2, kFY = kRY + 2;          // f region: tile + 1
constexpr int kR3Threads = 256;
constexpr int kNU = (kUX * kUY + kR3Threads - 1) / kR3Threads;
constexpr int kNF = (kFX * kFY + kR3Threads - 1) / kR3Threads;

template <class S, class F>
__global__ __launch_bounds__(kR3Threads) void k_rb3_sweep(const S *uin, long long ip, long long ipp, S *uout,
                                                           long long op, long long opp, const F *f, long long fp,
                                                           long long fpp, int n, int kz, double h2d,
                                                           const SolveState *state)
{
    using T = Traits<S>;
    using C = typename T::C;
    if (state && state->done) return;
    __shared__ C U[4][kUX * kUY];
    __shared__ C Fs[2][kFX * kFY];
    const int ntx = (n + kRX - 1) / kRX, nty = (n + kRY - 1) / kRY;
    const int b = blockIdx.x;
    const int i0 = (b % ntx) * kRX + 1, j0 = ((b / ntx) % nty) * kRY + 1, k0 = (b / (ntx * nty)) * kz + 1;
    const int k1 = min(k0 + kz, n + 1);  // planes k0 .. k1 - 1 are owned
    const C h2 = (C)h2d;
    const int tid = threadIdx.x;
    // one plane of the u region into registers (zero outside the domain);
    // addresses are clamped in range so the loads carry no branches
    auto load_u = [&](int k, C (&r)[kNU]) {
#pragma unroll
        for (int q = 0; q < kNU; ++q) {
            const int p = tid + q * kR3Threads;
            const int i = i0 - 2 + p % kUX, j = j0 - 2 + p / kUX;
            const bool ok = p < kUX * kUY && i >= 1 && i <= n && j >= 1 && j <= n && k >= 1 && k <= n;
            const C v = (C)T::ld(uin + (ok ? (long long)(i - 1) + (j - 1) * ip + (long long)(k - 1) * ipp : 0));
            r[q] = ok ? v : (C)0;
        }
    };
    auto load_f = [&](int k, C (&r)[kNF]) {
#pragma unroll
        for (int q = 0; q < kNF; ++q) {
            const int p = tid + q * kR3Threads;
            const int i = i0 - 1 + p % kFX, j = j0 - 1 + p / kFX;
            const bool ok = p < kFX * kFY && i >= 1 && i <= n && j >= 1 && j <= n && k >= 1 && k <= n;
            const C v = (C)gld(f + (ok ? (long long)(i - 1) + (j - 1) * fp + (long long)(k - 1) * fpp : 0));
            r[q] = ok ? v : (C)0;
        }
    };
    auto put_u = [&](int slot, const C (&r)[kNU]) {
#pragma unroll
        for (int q = 0; q < kNU; ++q) {
            const int p = tid + q * kR3Threads;
            if (p < kUX * kUY) U[slot][p] = r[q];
        }
    };
    auto put_f = [&](int slot, const C (&r)[kNF]) {
#pragma unroll
        for (int q = 0; q < kNF; ++q) {
            const int p = tid + q * kR3Threads;
            if (p < kFX * kFY) Fs[slot][p] = r[q];
        }
    };
    // relax one point of plane k (slot sc, neighbours in slots sm / sp), u
    // region coordinates (x, y); the same sum order as the half-sweep kernel
    auto relax = [&](int sm, int sc, int sp, int fs, int x, int y) -> C {
        const int p = y * kUX + x;
        C s = h2 * Fs[fs][(y - 1) * kFX + (x - 1)];
        s = s + U[sc][p - 1];
        s = s + U[sc][p + 1];
        s = s + U[sc][p - kUX];
        s = s + U[sc][p + kUX];
        s = s + U[sm][p];
        s = s + U[sp][p];
        return T::rnd(s * (C)(1.0 / 6.0));
    };

    // prologue: planes k0 - 2 and k0 - 1 in their slots; plane k0 and f of
    // plane k0 - 1 in registers for the first step
    C ru[kNU], rf[kNF];
    load_u(k0 - 2, ru);
    put_u((k0 - 2) & 3, ru);
    load_u(k0 - 1, ru);
    put_u((k0 - 1) & 3, ru);
    load_u(k0, ru);
    load_f(k0 - 1, rf);
    for (int z = k0 - 1; z <= k1; ++z) {
        // step z needs u of planes z - 2 .. z + 1 and f of planes z - 1, z:
        // the prefetched plane z + 1 and f of plane z go to their slots
        // (after the previous step's last barrier), then the next ones are
        // issued
        put_u((z + 1) & 3, ru);
        put_f(z & 1, rf);
        load_u(z + 2, ru);
        load_f(z + 1, rf);
        __syncthreads();
        // red of plane z on the tile + 1 (1-based index sum even)
        if (z >= 1 && z <= n) {
            const int sm = (z - 1) & 3, sc = z & 3, sp = (z + 1) & 3, fs = z & 1;
            for (int q = tid; q < kFX * kFY; q += kR3Threads) {
                const int x = 1 + q % kFX, y = 1 + q / kFX;
                const int i = i0 - 2 + x, j = j0 - 2 + y;
                if (i < 1 || i > n || j < 1 || j > n || ((i + j + z) & 1) != 0) continue;
                U[sc][y * kUX + x] = relax(sm, sc, sp, fs, x, y);
            }
        }
        __syncthreads();
        // black of plane z - 1 on the tile; the plane is then final
        const int zb = z - 1;
        if (zb >= k0 && zb < k1) {
            const int sm = (zb - 1) & 3, sc = zb & 3, sp = z & 3, fs = zb & 1;
            for (int q = tid; q < kRX * kRY; q += kR3Threads) {
                const int x = 2 + q % kRX, y = 2 + q / kRX;
                const int i = i0 - 2 + x, j = j0 - 2 + y;
                if (i > n || j > n) continue;
                C v = U[sc][y * kUX + x];
                if (((i + j + zb) & 1) != 0) {
                    v = relax(sm, sc, sp, fs, x, y);
                    U[sc][y * kUX + x] = v;
                }
                T::st(uout + (long long)(i - 1) + (j - 1) * op + (long long)(zb - 1) * opp, v);
            }
        }
        __syncthreads();
    }
}

hipError_t launch_rb3_sweep(int st, const void *uin, long long ip, long long ipp, void *uout, long long op,
                            long long opp, const void *f, long long fp, long long fpp, int n, double h2,
                            const SolveState *state, hipStream_t s)
{
    // planes per workgroup: 64 on large levels; fewer on small ones so that
    // there are enough workgroups (at least 8) to fill the device
    const int ntx = (n + kRX - 1) / kRX, nty = (n + kRY - 1) / kRY;
    int kz = 64;
    while (kz > 8 && (long long)ntx * nty * ((n + kz - 1) / kz) < 2048) kz /= 2;
    const int ntz = (n + kz - 1) / kz;
    const long long blocks = (long long)ntx * nty * ntz;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks);
    switch (st) {
    case ST_F64:
        hipLaunchKernelGGL((k_rb3_sweep<double, double>), grid, dim3(kR3Threads), 0, s, (const double *)uin, ip, ipp,
                           (double *)uout, op, opp, (const double *)f, fp, fpp, n, kz, h2, state);
        break;
    case ST_F32:
        hipLaunchKernelGGL((k_rb3_sweep<float, float>), grid, dim3(kR3Threads), 0, s, (const float *)uin, ip, ipp,
                           (float *)uout, op, opp, (const float *)f, fp, fpp, n, kz, h2, state);
        break;
    default:
        hipLaunchKernelGGL((k_rb3_sweep<bf16_t, float>), grid, dim3(kR3Threads), 0, s, (const bf16_t *)uin, ip, ipp,
                           (bf16_t *)uout, op, opp, (const float *)f, fp, fpp, n, kz, h2, state);
        break;
    }
    return hipGetLastError();
}

}  // namespace mgx
