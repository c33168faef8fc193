// Internal types shared by the host runtime and the kernels of libmgx.so.
// Nothing here is part of the C-ABI (include/mg.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef uint16_t bf16_t;  // bfloat16 storage (upper half of an IEEE binary32)

namespace mgx {

enum StateType { ST_F64 = 0, ST_F32 = 1, ST_BF16 = 2 };

// Per-system solver state that lives in device memory, so that the stop test
// runs on the device and the host can enqueue cycles ahead of it.
struct SolveState {
    int done;           // 0 running, 1 converged, 2 non-finite, 3 cycle limit,
                        // 4 a cycle reduced the residual by less than `watch`,
                        // 5 bf16-state steps stalled (history_rule), 6 diverged
    int nres;           // residual norms recorded so far (hist[0..nres-1])
    unsigned counter;   // finished work items of the current reduction
    int maxc;           // cycle limit
    double tol;         // relative residual target
    double watch;       // > 0: stop (done = 4) when rel > watch * previous rel
    double ff;          // ||f||_2^2 (set by the first norm of a solve)
    double rel;         // last relative residual
    double stall;       // > 0: the bf16-state stall ratio of history_rule (0: off)
    double hist[201];
};

// The solver's rules on a residual history hist[0 .. nres-1] (relative
// residuals after 0, 1, ... cycles), applied by the device-side stop test
// after every norm and exported on the host as mg_monitor:
//   2 (diverged): the last value is not finite, or above kDivergeGrowth
//     times the smallest so far, or it rose in each of the last three cycles
//     past the first (a converging FP64 / FP32 cycle lowers the residual
//     every cycle; a bf16-state step may raise it once, on the first step,
//     by up to ~100x for smooth data);
//   1 (fall back, when stall > 0, i.e. bf16 state): after the first step,
//     the last two steps each reduced the residual by less than 1 / stall;
//   0 otherwise.
constexpr double kDivergeGrowth = 1e3;
__host__ __device__ inline int history_rule(const double *hist, int nres, double stall)
{
    if (!hist || nres < 1) return 0;
    const int k = nres - 1;
    const double last = hist[k];
    if (!(last - last == 0.0)) return 2;  // NaN or infinite
    double mn = hist[0];
    for (int i = 1; i <= k; ++i) mn = hist[i] < mn ? hist[i] : mn;
    if (last > kDivergeGrowth * mn) return 2;
    if (k >= 4 && hist[k] > hist[k - 1] && hist[k - 1] > hist[k - 2] && hist[k - 2] > hist[k - 3]) return 2;
    if (stall > 0.0 && k >= 3 && hist[k] > stall * hist[k - 1] && hist[k - 1] > stall * hist[k - 2]) return 1;
    return 0;
}

// One grid level of one system as the kernels see it.  Arrays are
// interior-only with row pitch `pitch` (elements) and plane pitch `ppitch`;
// the nodal coefficient covers (n+2)^d nodes, contiguous.
struct LevelDesc {
    int n;              // interior points per axis
    int dim;
    int sys;            // system index (SolveState slot)
    int pad0;
    long long pitch, ppitch;
    double h2, inv_h2;  // h^2 and 1/h^2 of this level
    const void *a;      // nodal coefficient (compute type of the level) or null
    void *A;            // pre-smoothed state (march kernels)
    void *B;            // final state of the cycle on this level
    void *f;            // right-hand side
    // the next coarser level (for restriction output / prolongation input)
    int nc;
    int pad1;
    long long cpitch, cppitch;
    void *fc;           // coarse rhs
    const void *Bc;     // coarse final state
    // per-call flags of this level
    int uzero;          // the cycle starts from a zero state on this level
    int norm;           // POST on this level measures ||f - A u|| and runs the stop test
    double *acc;        // POST: if set, acc += final state instead of storing B (FP64 iterate)
    long long acc_pitch, acc_ppitch;
};

// A work item of the 2D row-marching kernels: one strip of columns of one
// block of rows of one level.
struct MarchItem {
    int lvl;            // index into the LevelDesc array of the launch
    int ia, ja;         // first owned column / row (1-based, odd)
    int part;           // norm partial slot of this item (global index)
};

struct MarchArgs {
    const LevelDesc *levels;
    const MarchItem *items;
    int nitems;
    int W, Hb;          // owned strip width / block height
    SolveState *states;
    double *partials;   // one per item (norm)
    const int *part0;   // per system: first partial slot
    const int *nparts;  // per system: number of partial slots
};

// ---- launchers (defined in the kernel translation units) -----------------
// LDS-tiled PRE (mode 0) / POST (mode 1) for small non-finest 2D levels:
// items are 32 x 32 tiles (args.W == args.Hb == 32), nsweeps <= 3.
// One full red-black sweep of the 3D Poisson operator, out of place (uin ->
// uout; pitches in elements); the state and rhs types follow st.
hipError_t launch_rb3_sweep(int st, const void *uin, long long ip, long long ipp, void *uout, long long op,
                            long long opp, const void *f, long long fp, long long fpp, int n, double h2,
                            const SolveState *state, hipStream_t s);
hipError_t launch_tile2d(int mode, int st, bool vc, int nsweeps, const MarchArgs &a, hipStream_t s);
struct Launch {
    hipStream_t stream;
};

// 2D row-marching fused kernels.  mode bit 0 = 0: nu1 sweeps + residual +
// full-weighting restriction; = 1: bilinear prolongation + correction + nu2
// sweeps (+ norm).  mode bit 1: the finest level (a separately named
// instantiation of the same code); bit 2: skew-1 stage schedule; bit 3: the
// POST adds into an FP64 iterate (refinement).  st: ST_*; vc: variable
// coefficient.
hipError_t launch_march2d_f64(int mode, bool vc, int nsweeps, int G, const MarchArgs &a, int grid, hipStream_t s);
hipError_t launch_march2d_f32(int mode, bool vc, int nsweeps, int G, const MarchArgs &a, int grid, hipStream_t s);
hipError_t launch_march2d_bf16(int mode, bool vc, int nsweeps, int G, const MarchArgs &a, int grid, hipStream_t s);
inline hipError_t launch_march2d(int mode, int st, bool vc, int nsweeps, int G, const MarchArgs &a, int grid,
                                 hipStream_t s)
{
    if (grid <= 0) return hipSuccess;
    switch (st) {
    case ST_F64: return launch_march2d_f64(mode, vc, nsweeps, G, a, grid, s);
    case ST_F32: return launch_march2d_f32(mode, vc, nsweeps, G, a, grid, s);
    case ST_BF16: return launch_march2d_bf16(mode, vc, nsweeps, G, a, grid, s);
    }
    return hipErrorInvalidValue;
}
// Owned columns of one strip: 128 G loaded minus a halo of 2 nu + 2 per side.
inline int march_strip_width(int G, int nsweeps) { return 128 * G - 2 * (2 * nsweeps + 2); }

// Geometry of the row-marching pipeline (shared by host and kernels):
// stage m of 2 nu works SK (m-1) + 1 rows behind the newest row; OL/OR/OX are
// the offsets of the finished row, the residual row and the restricted row;
// R = 2 nu + 2 the halo; P the register-ring period; D the rows in flight.
#ifndef MGX_MARCH_D1
#define MGX_MARCH_D1 3  // rows in flight per wave (skew-1 schedule)
#endif
struct MarchGeom {
    int NS, SK, R, OL, OR, OX, D, P;
};
constexpr int march_prefetch(int SK) { return SK == 1 ? MGX_MARCH_D1 : 5; }
constexpr MarchGeom march_geom(int NS, int SK)
{
    return MarchGeom{NS,
                     SK,
                     2 * NS + 2,
                     1 + SK * (2 * NS - 1),
                     1 + SK * (2 * NS - 1) + SK,
                     1 + SK * (2 * NS - 1) + 2 * SK,
                     march_prefetch(SK),
                     // smallest even ring that holds the window plus the rows in flight
                     ((march_prefetch(SK) + 1 + SK * (2 * NS - 1) + SK + 2) + 1) / 2 * 2};
}
// Row steps of one work item (a multiple of P; the host picks block heights
// that make the padding small): PRE runs Hb + OX + R steps, POST Hb + OR + R.
__host__ __device__ inline int march_steps(int mode, int Hb, int NS, int SK)
{
    const MarchGeom g = march_geom(NS, SK);
    const int raw = Hb + ((mode & 1) ? g.OR : g.OX) + g.R;
    return (raw + g.P - 1) / g.P * g.P;
}

// Generic per-point kernels (any dim).
struct GenArgs {
    LevelDesc L;
    SolveState *state;  // early exit when state->done (may be null)
    int colour;         // red-black half sweep colour
    double omega;       // Jacobi weight
    const void *src;    // Jacobi: source state
    void *dst;          // Jacobi: destination state
    int u_zero;
};
hipError_t launch_rb_half(int st, bool vc, const GenArgs &g, hipStream_t s);
hipError_t launch_jacobi(int st, bool vc, const GenArgs &g, hipStream_t s);
hipError_t launch_resid_restrict(int st, bool vc, const GenArgs &g, hipStream_t s);
hipError_t launch_prolong_correct(int st, const GenArgs &g, hipStream_t s);
hipError_t launch_fill_zero(void *p, long long bytes, hipStream_t s);
// full multigrid: fc = R f on a level (rhs type by st), B = P Bc (set)
hipError_t launch_restrict_rhs(int st, const GenArgs &g, hipStream_t s);
hipError_t launch_interp(int st, const GenArgs &g, hipStream_t s);
hipError_t launch_copy_state(int st, const GenArgs &g, const void *src, void *dst, hipStream_t s);

// FP64 residual-norm kernels with a device-side stop test.
struct NormArgs {
    int dim, n;
    long long pitch, ppitch;
    double inv_h2;
    const double *u;    // FP64 iterate (null = 0)
    const double *f;
    const double *a;    // FP64 nodal coefficient or null
    float *r32;         // optional: write (float)(f - A u) (interior-only, contiguous)
    double *r64;        // optional: write f - A u
    SolveState *state;
    double *partials;   // 2 per block
    int nblocks;
    int first;          // 1: this norm also measures ||f||^2 and resets the history
};
hipError_t launch_norm(const NormArgs &a, hipStream_t s);
// Reduce partials + stop test (must follow every norm-producing launch).
hipError_t launch_norm_finish(SolveState *states, int nsys, const double *partials, const int *part0,
                              const int *nparts, int slot0, int nslots, int first, hipStream_t s);

// Coarse-level tail: one workgroup per system runs the whole V-cycle on the
// levels [lt, L) in LDS, reading f_lt and writing B_lt.
struct TailArgs {
    const LevelDesc *levels;  // device: levels lt .. L-1 of every system (stride nlev)
    int nlev;                 // levels per system in this tail
    int nsys;
    const double *cinv;       // per system: (m x m) FP64 inverse of the coarsest matrix
    int m;                    // unknowns on the coarsest level
    int nu1, nu2, smoother;
    double omega;
    SolveState *states;
    int faces;                // 2D diffusion: face weights precomputed in LDS (the LDS holds them)
    const int *ops;           // device: a schedule of level operations (W / F cycles, full
    int nops;                 //   multigrid), or null for the V-cycle
};
// Operations of a tail schedule: op = kind | level << 4 | sweeps << 12 (level
// relative to the tail's top level)
enum TailOp {
    TAIL_OP_SMOOTH = 1,        // `sweeps` smoothing sweeps on the level
    TAIL_OP_RESTRICT = 2,      // f_{l+1} = R (f_l - A u_l), u_{l+1} = 0
    TAIL_OP_SOLVE = 3,         // coarsest level: u = A^-1 f (FP64 inverse)
    TAIL_OP_PROLONG = 4,       // u_l += P u_{l+1}
    TAIL_OP_RESTRICT_RHS = 5,  // f_{l+1} = R f_l, u_{l+1} = 0 (full multigrid)
    TAIL_OP_INTERP = 6,        // u_l = P u_{l+1} (full multigrid)
};
hipError_t tail_prepare(int st, bool vc, int dim);
hipError_t launch_tail_sized(int st, bool vc, int dim, const TailArgs &a, size_t lds, int threads, hipStream_t s);
// Dynamic LDS of the tail (levels n_top and below); faces adds the face tables.
size_t tail_lds_bytes(int st, int dim, int n_top, bool jacobi, bool faces);
size_t tail_max_lds();  // the largest dynamic LDS a tail launch may use

hipError_t launch_ir_correct(int st, double *u, long long pitch, long long ppitch, const void *e, int n, int dim,
                             SolveState *state, hipStream_t s);

// Batched FP64 residual (2D): work items are row chunks of one system.
struct NormSys {
    int n;
    int part0, nparts;
    int pad;
    long long pitch;
    double inv_h2;
    const double *u, *f, *a;
    float *r32;
};
struct NormItem {
    int sys, j0, j1, slot;
};
// flags: bit 0 = first norm of a solve (also measures ||f||), bit 1 = write r32
hipError_t launch_norm_batch(const NormItem *items, int nitems, const NormSys *sys, SolveState *states,
                             double *partials, int flags, hipStream_t s);

// Setup helpers
hipError_t launch_coef_inject(const double *af, int nf, void *ac, int ncn, int stride, int as_float, hipStream_t s);
hipError_t launch_coef_check(const double *a, long long count, int *bad, hipStream_t s);

// ---- learned smoother (k_learned.hip) -------------------------------------
struct LearnedW {       // device weight copies (bf16 / bf16-rounded)
    float *w1;          // [16][9]
    bf16_t *wf2, *wd2;  // [9][16][16]: forward [t][co][ci], data gradient [t][ci][co]
    bf16_t *wf3, *wd3;
    float *w4;          // [16][9]
    bf16_t *w1m;        // [16][16]: MFMA operand of layer 1, [co][tap] (taps 9..15 zero)
    // K = 32 MFMA operands, [b][row][k]: tap 2b + k / 16, channel k % 16 (tap 9 zero)
    bf16_t *w2k, *w3k;  // rows = output channels of layers 2, 3
    bf16_t *w4k;        // row 0 = layer 4, rows 1..15 zero
};
struct TrainBufs {
    bf16_t *x1, *x2, *x3, *dz3, *dz2, *dz1;
    float *y, *dy, *lossb, *E0, *part, *g, *m, *v;
    double *lacc;
    LearnedW d;
};
hipError_t learned_prep(const float *w, const LearnedW &d, hipStream_t s);
hipError_t learned_forward(const float *s, const int *idx, int B, int H, int W, const LearnedW &d, bf16_t *x1,
                           bf16_t *x2, bf16_t *x3, float *y, hipStream_t st);
hipError_t learned_step_fused(int st, const void *ein, void *eout, const float *f, const float *a, int n, double h2,
                              const LearnedW &d, hipStream_t s);
hipError_t learned_step(int st, void *e, const float *f, const float *a, int n, double h2, const LearnedW &d,
                        float *sbuf, bf16_t *x1, bf16_t *x2, bf16_t *x3, hipStream_t s);
size_t learned_train_scratch(int B, int P);
TrainBufs learned_carve(void *scratch, int B, int P);
hipError_t learned_loss_grad(const float *S, const float *E, const float *A, const int *idx, int B, int P, int border,
                             TrainBufs &t, float *g, hipStream_t st);
hipError_t learned_check_order(const int *order, long long cnt, int npairs, const TrainBufs &t, hipStream_t st);
hipError_t learned_loss_accumulate(const TrainBufs &t, int B, bool reset, hipStream_t st);
hipError_t learned_adam(float *w, const float *g, float *m, float *v, int t, float lr, float b1, float b2, float eps,
                        hipStream_t st);
hipError_t learned_crop(const double *s, const double *ustar, const double *uk, const double *a, int n, const int *y0,
                        const int *x0, int ncrops, int P, float *S, float *E, float *A, hipStream_t st);
hipError_t launch_scaled_residual64(const double *u, const double *f, const double *a, int n, long long pitch,
                                    double *s, hipStream_t st);

}  // namespace mgx
