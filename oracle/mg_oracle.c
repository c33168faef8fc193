/*
 * mg_oracle.c -- the correctness oracle: a plain, slow CPU geometric multigrid
 * for -div(a grad u) = f on [0,1]^d with u = 0 on the boundary (d = 1, 2, 3;
 * a == NULL is the Poisson problem).
 *
 * TEST INFRASTRUCTURE ONLY.  It is loaded by the tests, by the smoke check and
 * by the benchmark's CPU-baseline leg; the product library never calls it, and
 * it shares no source with the HIP path.
 *
 * Exported (suffix _f64 for the FP64 build, _f32 for the float build of the
 * same level operations, see mg_core.inc):
 *   orc_apply, orc_residual, orc_sweep, orc_restrict, orc_prolong_add,
 *   orc_coarsen_coef, orc_dot, orc_assemble, orc_vcycle, orc_cycle (V, W or
 *   F cycle), orc_fmg (full multigrid)
 * plus, in FP64 only:
 *   orc_lu_solve     dense LU with partial pivoting (the coarsest solve)
 *   orc_solve        V-cycles until ||f - A u||_2 / ||f||_2 <= tol
 *   orc_solve_cycles the same with V, W or F cycles, optionally starting
 *                    with one full-multigrid pass
 *   orc_solve_ir     iterative refinement: FP64 outer residual and update,
 *                    one (or more) V-cycle(s) per step in FP64, FP32, or FP32
 *                    arithmetic with the iterate stored as bfloat16
 *   orc_solve_ir_cycles  the same with V, W or F inner cycles
 *   orc_bf16_round   the bfloat16 rounding used for the stored state
 *
 * The paper (cphVB, SciPy 2012) contributes the five-point stencil as five
 * shifted views and its simultaneous (weighted Jacobi) update, section
 * "Numerical Python"; the rest is standard multigrid as defined at each
 * function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int nu1, nu2;     /* pre- and post-smoothing sweeps per level */
    int smoother;     /* 0 red-black GS, 1 weighted Jacobi, 2 lexicographic GS */
    int ncoarse;      /* a level with n <= ncoarse is solved directly */
    int bf16;         /* float build: store every iterate value as bfloat16 */
    double omega;     /* Jacobi weight */
} orc_opts;

/* Round a float to the nearest bfloat16 (the upper 16 bits of the IEEE
 * binary32 pattern), ties to even on the 16 dropped bits; NaN stays NaN,
 * overflow goes to infinity as round-to-nearest requires. */
float orc_bf16_round(float x)
{
    uint32_t b;
    memcpy(&b, &x, 4);
    if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu)) {
        b = (b | 0x00400000u) & 0xffff0000u;
    } else {
        uint32_t lsb = (b >> 16) & 1u;
        b = (b + 0x7fffu + lsb) & 0xffff0000u;
    }
    memcpy(&x, &b, 4);
    return x;
}
static float bf16_round(float x) { return orc_bf16_round(x); }

/* Solve M x = b (M row-major m x m, copied) by Gaussian elimination with
 * partial pivoting.  Returns 0, or -1 for a singular matrix. */
int orc_lu_solve(int m, const double *Min, const double *b, double *x)
{
    double *M = (double *)malloc(sizeof(double) * (size_t)m * (size_t)m);
    double *y = (double *)malloc(sizeof(double) * (size_t)m);
    memcpy(M, Min, sizeof(double) * (size_t)m * (size_t)m);
    memcpy(y, b, sizeof(double) * (size_t)m);
    int rc = 0;
    for (int k = 0; k < m; ++k) {
        int piv = k;
        for (int i = k + 1; i < m; ++i)
            if (fabs(M[(size_t)i * m + k]) > fabs(M[(size_t)piv * m + k])) piv = i;
        if (M[(size_t)piv * m + k] == 0.0) { rc = -1; break; }
        if (piv != k) {
            for (int j = 0; j < m; ++j) {
                double t = M[(size_t)k * m + j];
                M[(size_t)k * m + j] = M[(size_t)piv * m + j];
                M[(size_t)piv * m + j] = t;
            }
            double t = y[k]; y[k] = y[piv]; y[piv] = t;
        }
        for (int i = k + 1; i < m; ++i) {
            double l = M[(size_t)i * m + k] / M[(size_t)k * m + k];
            M[(size_t)i * m + k] = l;
            for (int j = k + 1; j < m; ++j) M[(size_t)i * m + j] -= l * M[(size_t)k * m + j];
            y[i] -= l * y[k];
        }
    }
    if (rc == 0) {
        for (int i = m - 1; i >= 0; --i) {
            double s = y[i];
            for (int j = i + 1; j < m; ++j) s -= M[(size_t)i * m + j] * x[j];
            x[i] = s / M[(size_t)i * m + i];
        }
    }
    free(M);
    free(y);
    return rc;
}

#define REAL double
#define REAL_IS_FLOAT 0
#define SFX(name) name##_f64
#include "mg_core.inc"
#undef REAL
#undef REAL_IS_FLOAT
#undef SFX

#define REAL float
#define REAL_IS_FLOAT 1
#define SFX(name) name##_f32
#include "mg_core.inc"
#undef REAL
#undef REAL_IS_FLOAT
#undef SFX

static long npts(int d, int n)
{
    long m = 1;
    for (int ax = 0; ax < d; ++ax) m *= n;
    return m;
}

/* Relative residual ||f - A u||_2 / ||f||_2 in FP64, sequential sums. */
static double rel_residual(int d, int n, const double *a, const double *u, const double *f, double *r)
{
    long m = npts(d, n);
    double h = 1.0 / (n + 1);
    orc_residual_f64(d, n, h, a, u, f, r);
    return sqrt(orc_dot_f64(m, r, r)) / sqrt(orc_dot_f64(m, f, f));
}

/* Plain FP64 solve: starting from the u passed in, run V-cycles until the
 * relative residual rho_k <= tol (tested after each complete cycle, <=) or
 * maxc cycles.  hist[0..cycles] receives rho_0 .. rho_cycles.  Returns 0 when
 * converged, 1 when not, -4 on a non-finite residual. */
int orc_solve_cycles(int d, int n, const double *a, double *u, const double *f, const orc_opts *o,
                     int type, int fmg, double tol, int maxc, double *hist, int *cycles);

int orc_solve(int d, int n, const double *a, double *u, const double *f, const orc_opts *o,
              double tol, int maxc, double *hist, int *cycles)
{
    return orc_solve_cycles(d, n, a, u, f, o, 0, 0, tol, maxc, hist, cycles);
}

/* As orc_solve with cycles of type `type` (0 V, 1 W, 2 F); with fmg = 1 the
 * first step is one full-multigrid pass (one cycle of that type per level,
 * orc_fmg) from scratch instead of a cycle from u. */
int orc_solve_cycles(int d, int n, const double *a, double *u, const double *f, const orc_opts *o,
                     int type, int fmg, double tol, int maxc, double *hist, int *cycles)
{
    long m = npts(d, n);
    double h = 1.0 / (n + 1);
    double *r = (double *)malloc(sizeof(double) * (size_t)m);
    int k = 0, rc = 1;
    hist[0] = rel_residual(d, n, a, u, f, r);
    if (!isfinite(hist[0])) rc = -4;
    else if (hist[0] <= tol) rc = 0;
    while (rc == 1 && k < maxc) {
        if (fmg && k == 0) orc_fmg_f64(d, n, h, a, u, f, o, type, 1);
        else orc_cycle_f64(d, n, h, a, u, f, o, type);
        ++k;
        hist[k] = rel_residual(d, n, a, u, f, r);
        if (!isfinite(hist[k])) rc = -4;
        else if (hist[k] <= tol) rc = 0;
    }
    *cycles = k;
    free(r);
    return rc;
}

/* Iterative refinement.  Each outer step: r = f - A u in FP64 and the stop
 * test on ||r||/||f||; then e = V-cycle(s) from e = 0 on (A, r) in the working
 * precision; then u += e in FP64.
 *   prec 0: the V-cycle in FP64 (reproduces orc_solve step for step);
 *   prec 1: the V-cycle in float, r rounded to float, a rounded to float;
 *   prec 2: as 1 with every stored iterate value rounded to bfloat16.
 * The coarsest solve is FP64 in every case (float data widened to double). */
int orc_solve_ir_cycles(int d, int n, const double *a, double *u, const double *f, const orc_opts *o,
                        int prec, int inner, int type, double tol, int maxc, double *hist, int *cycles);

int orc_solve_ir(int d, int n, const double *a, double *u, const double *f, const orc_opts *o,
                 int prec, int inner, double tol, int maxc, double *hist, int *cycles)
{
    return orc_solve_ir_cycles(d, n, a, u, f, o, prec, inner, 0, tol, maxc, hist, cycles);
}

/* As orc_solve_ir with inner cycles of type `type` (0 V, 1 W, 2 F). */
int orc_solve_ir_cycles(int d, int n, const double *a, double *u, const double *f, const orc_opts *o,
                        int prec, int inner, int type, double tol, int maxc, double *hist, int *cycles)
{
    long m = npts(d, n);
    double h = 1.0 / (n + 1);
    double *r = (double *)malloc(sizeof(double) * (size_t)m);
    double *e = (double *)malloc(sizeof(double) * (size_t)m);
    float *rf = (float *)malloc(sizeof(float) * (size_t)m);
    float *ef = (float *)malloc(sizeof(float) * (size_t)m);
    float *af = NULL;
    if (a && prec != 0) {
        long ma = 1;
        for (int ax = 0; ax < d; ++ax) ma *= (n + 2);
        af = (float *)malloc(sizeof(float) * (size_t)ma);
        for (long p = 0; p < ma; ++p) af[p] = (float)a[p];
    }
    orc_opts oi = *o;
    oi.bf16 = (prec == 2);
    int k = 0, rc = 1;
    for (;;) {
        hist[k] = rel_residual(d, n, a, u, f, r);
        if (!isfinite(hist[k])) { rc = -4; break; }
        if (hist[k] <= tol) { rc = 0; break; }
        if (k >= maxc) break;
        if (prec == 0) {
            memset(e, 0, sizeof(double) * (size_t)m);
            for (int c = 0; c < inner; ++c) orc_cycle_f64(d, n, h, a, e, r, &oi, type);
            for (long p = 0; p < m; ++p) u[p] += e[p];
        } else {
            for (long p = 0; p < m; ++p) rf[p] = (float)r[p];
            memset(ef, 0, sizeof(float) * (size_t)m);
            for (int c = 0; c < inner; ++c) orc_cycle_f32(d, n, (float)h, af, ef, rf, &oi, type);
            for (long p = 0; p < m; ++p) u[p] += (double)ef[p];
        }
        ++k;
    }
    *cycles = k;
    free(r); free(e); free(rf); free(ef); free(af);
    return rc;
}
