/*
 * mg.h -- C-ABI of the MI355X geometric multigrid library (libmgx.so).
 *
 * Problem: -div(a grad u) = f on the unit square/cube [0,1]^d, d = 1..3, with
 * u = 0 on the boundary, discretised on a vertex-centred grid with n = 2^k - 1
 * interior points per axis, h = 1/(n+1):
 *   Poisson   (a == NULL): (A u)_c = (2d u_c - sum of the 2d neighbours) / h^2
 *   Diffusion (d == 2)   : (A u)_c = sum over the 4 faces f of w_f (u_c - u_nbr) / h^2,
 *                          w_f the harmonic mean of the nodal a at the face's ends.
 * Solver: V(nu1,nu2)-cycles with red-black Gauss-Seidel (or weighted Jacobi,
 * the simultaneous five-point update of the paper's "Numerical Python"
 * section) smoothing, full-weighting restriction, (bi/tri)linear prolongation,
 * coarse operators rediscretised on 2h (diffusion: nodal a injected), and an
 * FP64 direct solve on the coarsest level.  Optional FP64 iterative
 * refinement around FP32 cycles, with the cycle's iterate stored as bfloat16.
 *
 * Memory and ownership (the data-ownership protocol of the paper's "Vector
 * Engine Manager" section, specialised to one device):
 *  - u, f, a and the workspace are caller-owned DEVICE buffers (e.g. torch
 *    tensors).  The library writes only u and the workspace; f and a are
 *    read-only and must not alias u (MG_ERR_ARG).
 *  - Interior-only arrays, x fastest: element (i,j,k) (1-based) at offset
 *    (i-1) + (j-1)*pitch[1] + (k-1)*pitch[2]; pitch 0 means contiguous
 *    (pitch[1] = n, pitch[2] = n*pitch[1]).  The nodal coefficient covers the
 *    (n+2)^2 nodes including the boundary, contiguous, node (i,j) at
 *    i + (n+2)*j, 0 <= i,j <= n+1.
 *  - The workspace (size from mg_workspace_size) belongs to the handle from
 *    mg_setup until mg_destroy; the library keeps no copy of u, f or a between
 *    calls (a is read at setup and at every FP64 residual).
 *  - All device work goes to options.stream (a hipStream_t; NULL = the null
 *    stream).  Results are visible once that stream has completed.  u on
 *    entry is the initial guess.
 *  - A handle is not thread-safe; separate handles are independent.
 * Errors: no function aborts, throws or prints.  Negative status = error,
 * positive = informational.  After MG_ERR_HIP the handle must be destroyed;
 * mg_last_error gives the HIP message.
 */
#ifndef MG_H
#define MG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int mg_status;
#define MG_OK 0
#define MG_NOT_CONVERGED 1      /* max_cycles reached; u holds the last iterate */
#define MG_FELL_BACK 2          /* converged after switching to the fallback smoother/precision */
#define MG_ERR_ARG (-1)
#define MG_ERR_UNSUPPORTED (-2)
#define MG_ERR_HIP (-3)
#define MG_ERR_NONFINITE (-4)   /* a residual norm was NaN/Inf; stats hold the finite history */
#define MG_ERR_DIVERGED (-5)    /* the residual grew (see mg_monitor); u holds the last iterate */
#define MG_ERR_WORKSPACE (-6)   /* workspace NULL, too small or misaligned (256 B) */

#define MG_OP_POISSON 0
#define MG_OP_DIFFUSION 1

#define MG_SM_RBGS 0            /* red (1-based index sum even) first, then black */
#define MG_SM_JACOBI 1          /* weighted Jacobi, omega (0 -> 2d/(2d+1)) */
#define MG_SM_LEARNED 2         /* learned convolutional smoother on the finest level */

#define MG_P_F64 0              /* every level operation in FP64 */
#define MG_P_F32_IR 1           /* FP64 outer residual + update, FP32 inner V-cycle */
#define MG_P_F32_BF16_IR 2      /* as MG_P_F32_IR, inner iterate stored as bfloat16 (RNE) */

/* Cycle types (standard multigrid; the paper gives only the smoother): on
 * every level above the coarsest, the coarse problem is visited
 *   MG_CYCLE_V: once (a V-cycle);
 *   MG_CYCLE_W: twice, the second visit starting from the first's result;
 *   MG_CYCLE_F: by an F-cycle, then by a V-cycle from its result.
 * Every first visit starts from a zero correction. */
#define MG_CYCLE_V 0
#define MG_CYCLE_W 1
#define MG_CYCLE_F 2

#define MG_MAX_CYCLES 200

typedef struct mg_handle_s *mg_handle;

typedef struct {
    int dim;                    /* 1, 2 or 3 */
    int n[3];                   /* interior points per axis, equal, each 2^k - 1; unused axes 1 */
    long long pitch[3];         /* elements; pitch[0] unused; 0 = contiguous */
} mg_grid;

typedef struct {
    int kind;                   /* MG_OP_POISSON or MG_OP_DIFFUSION (dim 2 only) */
    const double *a;            /* device, nodal coefficient, (n+2)^2, finite and > 0; NULL for Poisson */
} mg_operator;

typedef struct {
    int nu1, nu2;               /* pre/post sweeps per level (default 2, 2; fused path: 1..3) */
    int smoother;               /* MG_SM_* */
    int precision;              /* MG_P_* */
    int ncoarse;                /* coarsest points per axis: 1 or 3 (0 = 1 for dim 1, else 3) */
    int max_cycles;             /* cycle (or outer step) limit, <= MG_MAX_CYCLES (0 = 100) */
    int inner_cycles;           /* inner V-cycles per refinement step (0 = 1) */
    int use_graph;              /* capture one cycle as a hipGraph and replay it */
    double omega;               /* Jacobi weight (0 = 2d/(2d+1)) */
    const void *learned;        /* mg_learned weights for MG_SM_LEARNED, else NULL */
    void *stream;               /* hipStream_t */
    int cycle;                  /* MG_CYCLE_* (0 = V); W and F: single systems, RB-GS or Jacobi */
    int fmg;                    /* 1: mg_solve's first step is one full-multigrid pass (nested
                                 * iteration: f carried down by full weighting, the coarsest
                                 * level solved, on each finer level u = P u_c then one cycle);
                                 * MG_P_F64 only, the u passed in is overwritten */
    int zero_start;             /* 1: mg_solve starts from u = 0 without reading the u passed in
                                 * (the initial residual norm reads f alone; on the fused 3D path
                                 * the first cycle's finest pre-smoothing starts from zero, other
                                 * paths zero u first, which needs a contiguous array); single
                                 * systems only; mg_vcycle ignores it */
} mg_options;

typedef struct {
    int cycles;                 /* V-cycles (plain) or outer steps (refinement) done */
    double rel_res;             /* final ||f - A u||_2 / ||f||_2 (FP64) */
    double rho_avg;             /* (rel_res / hist[0])^(1/cycles) */
    double rho_asym;            /* geometric mean of the last three ratios */
    int fell_back;              /* 1 if the fallback smoother or precision was used */
    double hist[MG_MAX_CYCLES + 1]; /* hist[k] = relative residual after k cycles */
} mg_stats;

/* Fill *o with the defaults above (V(2,2), RB-GS, FP64, null stream). */
void mg_options_default(mg_options *o);

/* Bytes of device workspace mg_setup needs for this problem.
 * MG_ERR_ARG for an invalid grid/operator/options, MG_ERR_UNSUPPORTED for a
 * combination the library does not implement (e.g. diffusion in 3D). */
mg_status mg_workspace_size(const mg_grid *g, const mg_operator *op, const mg_options *o, size_t *bytes);

/* Build the level hierarchy in the caller's workspace (device, >= bytes from
 * mg_workspace_size, 256-byte aligned): level sizes n_{l+1} = (n_l - 1)/2
 * down to ncoarse, coarse coefficients by injection, the FP64 inverse of the
 * coarsest matrix.  Checks a > 0 and finite (MG_ERR_ARG).  Synchronises the
 * stream once.  The handle keeps pointers to the options' learned weights. */
mg_status mg_setup(const mg_grid *g, const mg_operator *op, const mg_options *o, void *workspace,
                   size_t bytes, mg_handle *out);

/* One cycle of the configured type (MG_P_F64) or one refinement step (other
 * precisions) on (u, f), enqueued on the stream; no host synchronisation. */
mg_status mg_vcycle(mg_handle h, double *u, const double *f);

/* *rel = ||f - A u||_2 / ||f||_2 in FP64 (synchronises the stream). */
mg_status mg_residual_norm(mg_handle h, const double *u, const double *f, double *rel);

/* Solve from the initial guess in u until the relative residual <= rtol,
 * tested after every complete cycle (first k with rho_k <= rtol), or
 * max_cycles.  Blocks until done.  st may be NULL.  Returns MG_OK,
 * MG_FELL_BACK, MG_NOT_CONVERGED or an error. */
mg_status mg_solve(mg_handle h, double *u, const double *f, double rtol, mg_stats *st);

/* Level operations on the finest level in the handle's precision (MG_P_F64
 * handles; others MG_ERR_UNSUPPORTED).  They run the same kernels as the
 * cycle and are exported for parity checks and composition:
 *   mg_smooth_restrict: u_out = nu1 smoothing sweeps from u;
 *                       fc = R (f - A u_out) on the next coarser level
 *                       (interior-only, contiguous, n_c = (n-1)/2).
 *   mg_correct_smooth:  u_out = nu2 sweeps from u + P uc.
 *   mg_residual:        r = f - A u.
 * u_out must not alias u, f or uc. */
mg_status mg_smooth_restrict(mg_handle h, const double *u, const double *f, double *u_out, double *fc);
mg_status mg_correct_smooth(mg_handle h, const double *u, const double *uc, const double *f, double *u_out);
mg_status mg_residual(mg_handle h, const double *u, const double *f, double *r);

/* ---- per-kernel timing ----------------------------------------------------
 * While profiling is on, every launch that mg_solve / mg_vcycle makes for a
 * level operation is bracketed by HIP events on the handle's stream (graph
 * replay is suspended meanwhile).  mg_profile_read returns one record per
 * kernel class ("pre n=4095", "post n=4095", "tail", "norm", ...), averaged
 * over the launches that did work: launches enqueued after the device-side
 * stop test fired are not counted.  bytes_per_launch is the algorithmic
 * traffic of one launch (every array it touches read once / written once).
 * mg_profile(h, 1) clears the records and starts, mg_profile(h, 2) does the
 * same for the finest level's launches only (two events per launch cost
 * about a microsecond each; this keeps them off the small levels), and
 * mg_profile(h, 0) stops. */
typedef struct {
    char name[48];
    int launches;
    double total_ms;
    double avg_ms;
    double bytes_per_launch;
} mg_kernel_timing;
mg_status mg_profile(mg_handle h, int on);
mg_status mg_profile_read(mg_handle h, mg_kernel_timing *out, int max, int *count);

/* The solver's rules on a residual history, on the host (no device work),
 * the same function the solve loop applies after every chunk of cycles:
 * hist[0 .. nres-1] are relative residuals after 0, 1, ... cycles.
 *   MG_MONITOR_DIVERGED: the last value is not finite, or it exceeds 1e3
 *     times the smallest so far, or it rose in each of the last three cycles
 *     (past the first) -- the solve stops with MG_ERR_DIVERGED and the last
 *     iterate in u;
 *   MG_MONITOR_FALLBACK (precision MG_P_F32_BF16_IR only): after the first
 *     step, the last two steps each reduced the residual by less than a
 *     factor 1 / stall_ratio (the solver uses 0.5, i.e. 2x) -- the solve
 *     continues with an FP32-stored iterate and reports MG_FELL_BACK;
 *   MG_MONITOR_CONTINUE otherwise. */
#define MG_MONITOR_CONTINUE 0
#define MG_MONITOR_FALLBACK 1
#define MG_MONITOR_DIVERGED 2
int mg_monitor(const double *hist, int nres, int precision, double stall_ratio);

mg_status mg_destroy(mg_handle h);
const char *mg_status_str(mg_status s);
const char *mg_last_error(mg_handle h);  /* h NULL: the last failed setup, or handle-free
                                           * (learned) call, of this thread */

/* ---- batches of independent systems -------------------------------------
 * nsys systems, each with its own grid (dim 2, n_s in any mix of 2^k - 1),
 * operator and device arrays; one options struct for all.  Levels of equal
 * size across systems run in one launch per level size and phase (a work
 * list of tiles of every system at that size); the cycle is
 * captured once as a hipGraph when use_graph is set.  Converged systems are
 * masked out of later launches. */
mg_status mg_workspace_size_batch(int nsys, const mg_grid *g, const mg_operator *op, const mg_options *o,
                                  size_t *bytes);
mg_status mg_setup_batch(int nsys, const mg_grid *g, const mg_operator *op, const mg_options *o,
                         void *workspace, size_t bytes, mg_handle *out);
/* u[s], f[s]: device pointers (host array of nsys pointers).  st: nsys
 * entries or NULL.  Returns the worst status over the systems. */
mg_status mg_solve_batch(mg_handle h, double *const *u, const double *const *f, double rtol, mg_stats *st);

/* ---- the paper's fixed-iteration Jacobi benchmark ----------------------------
 * The "Performance Study" runs a Jacobi iteration a fixed number of times on
 * a square array, built in the "NumPy" section from five views of one array
 * (centre and four shifted neighbours).  Read as an average: each interior
 * point becomes 0.2 * (centre + up + down + left + right), summed in that
 * order, all five taken from the previous iteration; the outermost ring of
 * the array is a fixed boundary and is copied unchanged.
 * in, out: rows x cols FP64 device arrays, row-major and contiguous
 * (up/down = previous/next row).  in is read only; out receives the result
 * after `iters` (>= 0) iterations.  work: a third rows x cols device array,
 * scratch, needed only when iters > 4 (NULL otherwise allowed); its contents
 * on return are unspecified.  The three arrays must not overlap
 * (MG_ERR_ARG), nor may rows or cols be < 1.  Enqueued on `stream` (a
 * hipStream_t; NULL: the default stream), asynchronous; HIP failures:
 * MG_ERR_HIP with mg_last_error(NULL). */
mg_status mg_jacobi5(const double *in, double *out, double *work, int rows, int cols, int iters, void *stream);

/* mg_jacobi5 for callers that cannot allocate device memory -- code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc --
 * and so cannot pass a work array.  Same arguments and results as
 * mg_jacobi5 without `work`: when iters > 4 the library uses its own static
 * work array, a file-scope device array of MG_JACOBI5_STATIC_MAX doubles
 * (32 MiB) that each device the library runs on holds until the process
 * ends.  rows * cols above that maximum (with iters > 4) gives
 * MG_ERR_WORKSPACE before any launch, with the reason in mg_last_error(NULL).
 * Nothing is allocated or freed.  Every call on one device shares that
 * device's array: calls that overlap in time on one device (other streams,
 * other threads) race and give undefined results; calls in one stream are
 * ordered and safe.  The array's contents between calls are unspecified. */
#define MG_JACOBI5_STATIC_MAX 4194304
mg_status mg_jacobi5_static(const double *in, double *out, int rows, int cols, int iters, void *stream);

/* ---- autotuner --------------------------------------------------------------
 * The paper's benchmarks use the best block size per experiment (its
 * "Performance Study": block counts tuned per workload); here the library
 * measures launch shapes on the device.  For every 2D level size that runs
 * the fused PRE/POST kernels, mg_autotune times the PRE launch with block
 * heights 4 .. 256 and, on sizes that hold no system's finest level, LDS
 * tiles, on the bound arrays (u[s], f[s]: nsys device pointers, as for a
 * solve), `reps` (1 .. 50) timed launches per candidate, and keeps the
 * fastest; the choice lasts for the handle's life.  The finest level's
 * smoother runs in place, so u[s] comes back smoothed (a better iterate of
 * the same system), not unchanged.  3D handles: MG_OK, nothing tuned.
 * Synchronises; not inside a graph capture.
 * mg_tune_get lists the choices (level size n, block height hb, tiled
 * 0/1; count = how many there are, of which min(count, max) are written to
 * the caller's arrays); mg_tune_set applies one (e.g. read back from a
 * cache): MG_ERR_ARG for n < 1 or hb outside 2 .. 256; odd hb is rounded
 * down; a tile request on a size that holds a finest level, or on a 3D
 * handle, is kept but that size marches. */
mg_status mg_autotune(mg_handle h, double *const *u, const double *const *f, int reps);
mg_status mg_tune_get(mg_handle h, int *n, int *hb, int *tiled, int max, int *count);
mg_status mg_tune_set(mg_handle h, int n, int hb, int tiled);

/* ---- learned smoother ------------------------------------------------------
 * Not in the paper (which has no multigrid): an extension of the solver in
 * which the finest-level sweeps are replaced by a learned step; the paper's
 * component interface (its "Vector Engine Manager" section: register a
 * user-defined operation, then execute) shapes it as weights registered at
 * mg_setup and training / inference entry points beside the solver.
 * A bias-free 3x3 convolutional network N (1 -> 16 -> 16 -> 16 -> 1 channels,
 * ReLU after the first three layers, zero padding) replaces the finest-level
 * sweeps of the cycle: each sweep becomes u <- u + N(s), s = D^-1 (f - A u),
 * D the operator's diagonal.  Weights are caller-owned device FP32 arrays of
 * MG_LEARNED_NWEIGHTS numbers, the four layers' W[c_out][c_in][ky][kx]
 * C-ordered one after another (output pixel (y, x) reads input
 * (y + ky - 1, x + kx - 1)); the kernels use bfloat16 copies of the weights
 * and activations with FP32 accumulation (16 -> 16 layers on MFMA).
 * The solver uses it with options.smoother = MG_SM_LEARNED, options.learned =
 * the weights (read at mg_setup), dim 2, the diffusion operator and an FP32 /
 * bf16-state refinement precision (else MG_ERR_UNSUPPORTED; batches too).  If a learned cycle reduces the residual by less than a factor
 * 0.9, or produces non-finite values (then u restarts from 0), the rest of the
 * solve uses red-black Gauss-Seidel and the status is MG_FELL_BACK.
 * Training minimises the energy-norm loss over P x P patches (s, e, a):
 *   L = mean_b E_V(e_b - N(s_b)) / E_V(e_b),
 *   E_V(w) = sum over faces with both ends in the window V (the patch minus
 *   `border` pixels) of a_f (w_1 - w_2)^2, a_f the harmonic mean of the nodal
 *   coefficient at the face's ends,
 * with Adam on the FP32 master weights.  Patch arrays are device float
 * [npairs][P][P] (a: the nodal coefficient at the patch's nodes). */
#define MG_LEARNED_NWEIGHTS 4896

typedef struct {
    int epochs, batch, patch, border;   /* e.g. 30, 32, 64, 5 */
    double lr, beta1, beta2, eps;       /* Adam, e.g. 1e-3, 0.9, 0.999, 1e-8 */
} mg_train_options;

typedef struct {
    int steps;                /* Adam steps taken */
    double loss_first_epoch;  /* mean batch loss of the first epoch */
    double loss_last_epoch;   /* and of the last */
    double ms;                /* device time of the training loop */
} mg_train_stats;

/* Bytes of device scratch the training / gradient / apply entry points need
 * for batches of `batch` maps of `patch` x `patch` (apply: patch = max(H, W));
 * 0 for batch < 1 or patch < 3.  The scratch is caller-owned device memory
 * of at least this size (any alignment; it is carved on 256-byte
 * boundaries inside); its contents are not kept between calls. */
size_t mg_learned_scratch_bytes(int batch, int patch);

/* Loss (host double) and gradient dL/dw (device FP32 [MG_LEARNED_NWEIGHTS])
 * of the first B pairs at the weights w (device FP32); s, e, a are device
 * float [B][P][P].  MG_ERR_ARG for NULL pointers, P < 3 or 2 border >= P;
 * MG_ERR_WORKSPACE if bytes < mg_learned_scratch_bytes(B, P).  Synchronises;
 * HIP failures give MG_ERR_HIP with the message in mg_last_error(NULL). */
mg_status mg_learned_loss_grad(const float *s, const float *e, const float *a, int B, int P, int border,
                               const float *w, double *loss, float *grad, void *scratch, size_t bytes, void *stream);

/* y = N(s) for B maps of H x W (device float [B][H][W] each; y must not
 * alias s).  Errors as for mg_learned_loss_grad.  Synchronises. */
mg_status mg_learned_apply(const float *s, int B, int H, int W, const float *w, float *y, void *scratch,
                           size_t bytes, void *stream);

/* Adam training of the FP32 master weights w (device, in/out) over npairs
 * patches.  order: device int [epochs * npairs], the pair visited at each
 * position of each epoch (the caller's shuffle); batches take consecutive
 * runs of `batch` entries (a short last batch is dropped); an entry outside
 * [0, npairs) gives MG_ERR_ARG before any training.  loss_hist:
 * host double [epochs] mean batch loss per epoch, or NULL.  Synchronises. */
mg_status mg_learned_train(const float *s, const float *e, const float *a, int npairs, const int *order,
                           const mg_train_options *o, float *w, double *loss_hist, mg_train_stats *st,
                           void *scratch, size_t bytes, void *stream);

/* One learned step exactly as the solver takes it on the finest level of
 * the inner cycle (the fused kernel the solver launches):
 *   e_out = e + N(s),  s = D^-1 (f - A e),
 * on an n x n grid, h = 1/(n+1), A the diffusion operator of the float nodal
 * coefficient a ((n+2)^2 nodes, device), D its diagonal, f float (device).
 * e and e_out are device [n][n] arrays of the inner state type: precision =
 * MG_P_F32_IR (float) or MG_P_F32_BF16_IR (bfloat16; e_out rounded to
 * nearest even).  s is computed in FP32 and rounded to bf16 before the
 * network; w: the FP32 master weights (device).  scratch: device memory of at
 * least mg_learned_scratch_bytes(1, 3) bytes (the weights' bf16 copies).
 * e_out must not overlap e, f, a or the scratch (MG_ERR_ARG); (n+2)^2 * 4
 * bytes of 4 GiB or more give MG_ERR_UNSUPPORTED.  Synchronises the stream. */
mg_status mg_learned_step(const void *e, void *e_out, const float *f, const float *a, int n, int precision,
                          const float *w, void *scratch, size_t bytes, void *stream);

/* Training-pair gather: for each crop c, the P x P patch at interior offset
 * (y0[c], x0[c]) (0-based; device int arrays) of s, e = ustar - uk and the
 * nodal coefficient a ((n+2)^2, FP64), written as float [ncrops][P][P].
 * s, ustar, uk are device FP64 n x n contiguous.  A crop that does not fit
 * in the grid is written as NaN (nothing outside the arrays is read).
 * Enqueued on `stream`; does not synchronise. */
mg_status mg_learned_crop(const double *s, const double *ustar, const double *uk, const double *a, int n,
                          const int *y0, const int *x0, int ncrops, int P, float *S, float *E, float *A,
                          void *stream);

/* s = D^-1 (f - A u) in FP64 on the finest level of a 2D handle (D the
 * diagonal of A; u, f with the handle's pitch, device); s is interior-only
 * and contiguous.  MG_ERR_ARG for a batch or non-2D handle.  Synchronises. */
mg_status mg_scaled_residual(mg_handle h, const double *u, const double *f, double *s);

#ifdef __cplusplus
}
#endif

#endif /* MG_H */
