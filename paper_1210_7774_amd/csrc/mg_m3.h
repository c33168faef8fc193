// Fused 3D plane-marching level kernels (k_march3d.hip): one red-black
// Gauss-Seidel sweep of the 7-point Poisson operator per pass, with the
// operations next to it in the cycle fused in front of and behind it.
#pragma once

#include <hip/hip_runtime.h>

#include "mg_internal.h"

namespace mgx {

// What the pass does to the state before its sweep.
enum M3Head {
    M3_HEAD_U = 0,     // sweep from the state in uin
    M3_HEAD_ZERO = 1,  // sweep from a zero state (uin not read)
    M3_HEAD_CORR = 2,  // sweep from uin + P uc (trilinear coarse-grid correction)
};
// What the pass does after its sweep (the swept state is always stored).
enum M3Tail {
    M3_TAIL_NONE = 0,
    M3_TAIL_RR = 1,    // residual r = f - A u and full weighting fc = R r
    M3_TAIL_NORM = 2,  // FP64: sum of r^2 over the owned points, one partial per workgroup
};

struct M3Args {
    int n;                    // interior points per axis of this level
    int nc;                   // the next coarser level's n (RR, CORR)
    double h2, ih2;           // h^2 and 1/h^2
    const void *uin;          // input state (HEAD_U, HEAD_CORR)
    long long ip, ipp;        // its row / plane pitch (elements)
    void *uout;               // output state (never aliases uin)
    long long op, opp;
    const void *f;            // right-hand side
    long long fp, fpp;
    void *fc;                 // RR: coarse right-hand side
    long long fcp, fcpp;
    const void *uc;           // CORR: coarse correction (state type)
    long long ucp, ucpp;
    double *partials;         // NORM: 2 doubles per workgroup (rr, 0)
    double *acc;              // non-null: the swept state is added into this FP64
    long long accp, accpp;    //   iterate (refinement) instead of being stored in uout
    const SolveState *state;  // every workgroup returns at once when state->done
    int kz, ntx, nty, ntz;    // tiling (filled in by launch_march3d)
};

// Workgroups a launch of this level makes (NORM: the partial slots it fills).
int march3d_blocks(int n, int tail, int st);
hipError_t launch_march3d(int st, int head, int tail, const M3Args &a, hipStream_t s);

// The wavefront passes (k_march3dw.hip): ns = 1 or 2 sweeps per pass over
// 32 x 32 column tiles, each thread owning a pair of columns; one workgroup
// per tile column and run of planes (march3dw_blocks of them, also the NORM
// partial slots).  Same arguments as launch_march3d (the tiling fields are
// filled in here).
int march3dw_blocks(int n);
hipError_t launch_march3dw(int st, int ns, int head, int tail, const M3Args &a, hipStream_t s);

}  // namespace mgx
