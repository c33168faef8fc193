/*
 * ve.h -- the vector-bytecode engine of libmgx.so: the paper's vector engine
 * and vector engine manager (cphVB, sections "Bytecode", "Interface",
 * "Vector Engine Manager" and "Vector Engine") on one MI355X.
 *
 * A front end records array operations as vector bytecode: one opcode per
 * instruction, every operand an array-view (a strided window of an
 * array-base, section "Numerical Python") or a constant.  ve_execute takes a
 * batch, forms kernels by scanning it in order and adding each instruction
 * to the current kernel while it is *blockable* with it (section "Vector
 * Engine": the new instruction's inputs and the kernel's outputs, and its
 * output and the kernel's inputs and outputs, share no element or are
 * precisely the same view), and runs every kernel as one generated HIP
 * kernel over its index space: each work-group takes contiguous blocks of
 * the space, each thread runs all of the kernel's instructions on its
 * elements, values pass between instructions in registers, and outputs that
 * a later free or discard makes dead are never stored.  Kernels are
 * generated as HIP source and compiled at run time (hipRTC) for the device's
 * architecture, once per distinct kernel shape; strides, offsets, sizes and
 * constants are launch arguments.
 *
 * Readings where the paper is silent:
 *  - "precisely the same data" is the same view (offset, shape, strides;
 *    strides of unit axes ignored);
 *  - a kernel is one index space: all its instructions have one shape;
 *  - a reduction's output exists only when its kernel ends: an instruction
 *    that reads or writes it starts a new kernel;
 *  - an instruction whose output shares elements with one of its own inputs
 *    without being that view reads a copy of the input staged before it
 *    (whole-array meaning: every input is read before the output is written);
 *  - a kernel also ends when it would exceed 64 instructions, 48 distinct
 *    memory operands or 32 constants (the size of its launch arguments).
 * Errors: every call returns VE_OK or a negative status and records a
 * message for ve_last_error.  Arithmetic follows IEEE-754 in the operands'
 * type with no contraction: add, subtract, multiply, divide and sqrt are
 * correctly rounded; exp, log, sin, cos, tanh and power use the device
 * math library (a few ulp).
 */
#ifndef VE_H
#define VE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int ve_status;
#define VE_OK 0
#define VE_ERR_ARG (-1)          /* invalid argument, view or batch */
#define VE_ERR_UNSUPPORTED (-2)  /* valid but not implemented (e.g. a self-overlapping output view) */
#define VE_ERR_HIP (-3)          /* a HIP runtime call failed */
#define VE_ERR_COMPILE (-4)      /* run-time compilation failed (log in ve_last_error) */

#define VE_MAX_NDIM 4
#define VE_MAX_IN 3

/* element types of an array-base */
#define VE_F64 0
#define VE_F32 1

/* opcodes (numpy names) */
#define VE_SYNC 1                /* out.base's data must be in memory (counts as a read) */
#define VE_DISCARD 2             /* out.base's contents are no longer needed */
#define VE_FREE 3                /* out.base is released (engine-owned memory freed) */
#define VE_COPY 10               /* out = in0 (converts between element types) */
#define VE_NEGATIVE 11
#define VE_ABSOLUTE 12
#define VE_SQRT 13
#define VE_EXP 14
#define VE_LOG 15
#define VE_SIN 16
#define VE_COS 17
#define VE_TANH 18
#define VE_ADD 30
#define VE_SUBTRACT 31
#define VE_MULTIPLY 32
#define VE_DIVIDE 33
#define VE_MAXIMUM 34            /* NaN-propagating, as numpy.maximum */
#define VE_MINIMUM 35
#define VE_POWER 36
#define VE_GREATER 37            /* comparisons give 1 or 0 in the output's type */
#define VE_GREATER_EQUAL 38
#define VE_LESS 39
#define VE_LESS_EQUAL 40
#define VE_EQUAL 41
#define VE_NOT_EQUAL 42
#define VE_WHERE 50              /* out = in0 != 0 ? in1 : in2 */
#define VE_ADD_REDUCE 60         /* out (one element) = sum of all elements of in0 */
#define VE_MAXIMUM_REDUCE 61     /* out (one element) = maximum of all elements of in0 */
#define VE_USER 100              /* first opcode of user-defined operations */

/* An array-view: elements base[offset + sum_d i_d * stride[d]], 0 <= i_d <
 * shape[d] (element units).  As an input, base < 0 means the constant
 * cst[k] of the instruction (or an unused slot). */
typedef struct {
    int base;
    int ndim;                          /* 1 .. VE_MAX_NDIM */
    long long offset;
    long long shape[VE_MAX_NDIM];
    long long stride[VE_MAX_NDIM];     /* may be negative; 0 only in inputs */
} ve_view;

typedef struct {
    int opcode;
    ve_view out;                       /* system instructions: out.base names the array-base */
    ve_view in[VE_MAX_IN];
    double cst[VE_MAX_IN];
} ve_instr;

typedef struct {
    long long instructions;            /* computation instructions executed */
    long long kernels;                 /* kernels launched */
    long long compiled;                /* distinct kernels compiled */
    long long cache_hits;              /* kernels found already compiled */
    long long stores_elided;           /* output views never stored (dead after a free / discard) */
    long long staged;                  /* inputs staged through a copy */
    double compile_ms;                 /* wall time spent in run-time compilation */
} ve_stats;

typedef struct {
    char name[32];                     /* "k<id>:<instructions>" */
    int launches;
    double total_ms, avg_ms;
    double bytes_per_launch;           /* algorithmic: elements loaded + stored, each once */
} ve_kernel_timing;

typedef struct ve_engine_s *ve_engine;

/* Initialise an engine on the current device; work is enqueued on `stream`
 * (hipStream_t, NULL = the null stream). */
ve_status ve_create(void *stream, ve_engine *out);

/* Finalise: frees the engine-owned array-bases (after the stream drains) and
 * the compiled kernels. */
ve_status ve_destroy(ve_engine e);

/* The vector engine manager's "define a new array": an array-base of nelem
 * elements of `dtype`.  device_ptr != NULL binds caller-owned device memory
 * (never freed by the engine); NULL lets the engine allocate it when it is
 * first used (late allocation, stream-ordered). */
ve_status ve_base_new(ve_engine e, int dtype, long long nelem, void *device_ptr, int *id);

/* The device address of an array-base (allocating it now if it has none). */
ve_status ve_base_ptr(ve_engine e, int id, void **ptr);

/* Execute a batch of n instructions (stream-ordered, no host
 * synchronisation; the batch array is not kept). */
ve_status ve_execute(ve_engine e, const ve_instr *batch, int n);

/* Kernel formation only, on the host: kernel_of[i] = the kernel of
 * instruction i (-1 for system and empty instructions), *nkernels = the
 * count (staging copies may form kernels of their own). */
ve_status ve_plan(const ve_instr *batch, int n, int *kernel_of, int *nkernels);

/* The generated HIP source of kernel k of a batch (base_dtype[b] the type
 * of base b); *need = bytes including the terminating zero. */
ve_status ve_kernel_source(const ve_instr *batch, int n, const int *base_dtype, int nbases, int k, char *buf,
                           size_t len, size_t *need);

/* The interface's "register a user-defined operation": an element-wise
 * expression in x0 .. x(nin-1) of the output's type T (HIP C++, e.g.
 * "x0 * x1 + x2"); *opcode receives its opcode (VE_USER + k). */
ve_status ve_register(ve_engine e, const char *expr, int nin, int *opcode);

ve_status ve_stats_get(ve_engine e, ve_stats *st);

/* Per-kernel HIP-event timing (on = 1) or off; ve_profile_read returns one
 * record per distinct kernel in first-launch order. */
ve_status ve_profile(ve_engine e, int on);
ve_status ve_profile_read(ve_engine e, ve_kernel_timing *out, int max, int *count);

const char *ve_last_error(ve_engine e);

#ifdef __cplusplus
}
#endif
#endif
