/*
 * stencil5d -- temporally blocked Jacobi-style stencil sweeps on MI355X (gfx950).
 *
 * C ABI of libstencil5d.so.  Plain C types only; no exception, abort or exit
 * ever crosses it: every entry point returns a status code and leaves a
 * detail string for s5d_last_error().
 *
 * The operation (AN5D, Background "Stencil Computation"; Table 3 for the
 * star/box stencils; Fig. 4 and "Host Code" under "Code Generation" for the
 * double-buffered time loop):
 *
 *   A[2] are two padded grids of ndim axes.  Axis 0 is the outermost
 *   (slowest-varying, C order) axis; it is also the axis the kernels stream
 *   along ("Implementation": the loop after the time loop is the streaming
 *   dimension).  Extents are interior[a] + 2*radius: the border of width
 *   `radius` on every face, both faces of axis 0 included, holds the fixed
 *   boundary values and is never written.  For t = 0 .. steps-1 every interior
 *   cell p receives
 *
 *       A[(t+1) % 2][p] = sum_k coeffs[k] * A[t % 2][p + o_k]
 *
 *   and the result is A[steps % 2], exactly where the modulo double buffer of
 *   the C program leaves it ("Host Code").
 *
 *   Offsets o_k come in ONE canonical order: lexicographic in (d0, d1[, d2]),
 *   each component in [-radius, radius], axis 0 first.  A box stencil keeps
 *   all (2r+1)^ndim offsets; a star stencil keeps the 2*r*ndim + 1 offsets
 *   with at most one non-zero component.  coeffs[k] belongs to offset o_k.
 *
 * How it is computed (AN5D, "Execution Model" and "Optimizations"): each GPU
 * launch advances b_T time steps at once.  A tile of the plane normal to axis
 * 0 streams along axis 0 and keeps, per fused time level, a window of
 * 2*radius+1 planes in registers; the tile overlaps its neighbours by
 * b_T*radius cells on each side and only its compute region is stored.  The
 * result equals the plain loop up to the rounding of the fused multiply-adds
 * the kernels use (float64: relative error far below 1e-12 for the workloads
 * in the test-suite).
 */
#ifndef STENCIL5D_H
#define STENCIL5D_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
typedef int32_t s5d_status;
#define S5D_OK 0           /* success */
#define S5D_EINVAL 1       /* an argument is invalid (null, out of range, aliased) */
#define S5D_EUNSUPPORTED 2 /* valid, but no kernel of this library covers it */
#define S5D_ENOMEM 3       /* host allocation failed */
#define S5D_EDEVICE 4      /* a HIP runtime call failed; see s5d_last_error() */
#define S5D_EBUDGET 5      /* a memory budget would be exceeded */

/* Stencil shape (Background "Stencil Computation"). */
#define S5D_STAR 0
#define S5D_BOX 1

/* Storage and arithmetic type of the grids. */
#define S5D_F32 0
#define S5D_F64 1

/* Accumulation of the stencil terms. */
#define S5D_ACC_PLAIN 0       /* one fused multiply-add per term, working precision */
#define S5D_ACC_COMPENSATED 1 /* float32 only: error-free products and sums
                                 (compensated dot product), one final rounding */

/* Problem descriptor.  Set struct_size = sizeof(s5d_desc). */
typedef struct s5d_desc {
    uint32_t struct_size;
    int32_t ndim;        /* 2 or 3 */
    int32_t radius;      /* stencil radius r >= 1 */
    int32_t shape;       /* S5D_STAR or S5D_BOX */
    int32_t dtype;       /* S5D_F32 or S5D_F64 */
    int32_t accum;       /* S5D_ACC_PLAIN or S5D_ACC_COMPENSATED */
    int64_t interior[3]; /* interior extents, axis 0 first; entries beyond ndim ignored */
    int64_t steps;       /* number of time steps T >= 0 */
    const double *coeffs;/* host pointer, n_coeffs values in canonical offset order;
                            copied by s5d_plan_create, not retained */
    int64_t n_coeffs;    /* star: 2*radius*ndim + 1, box: (2*radius + 1)^ndim */
} s5d_desc;

/* Blocking parameters (AN5D "Execution Model", "Division of Streaming
 * Dimension"; Table 5 header).  A zero field lets the library choose.
 * Set struct_size = sizeof(s5d_tuning). */
typedef struct s5d_tuning {
    uint32_t struct_size;
    int32_t bt;             /* temporal blocking degree b_T: time steps fused per launch */
    int32_t tile0;          /* 2D: b_S along axis 1; 3D: b_S along axis 1 (rows) */
    int32_t tile1;          /* 3D: b_S along axis 2 (columns); 2D: unused */
    int32_t stream_chunk;   /* h_SN: axis-0 length of one stream block */
    int32_t cells_per_lane; /* consecutive cells of the last axis owned by one lane */
    int32_t rows_per_wave;  /* 3D: consecutive axis-1 rows held by one wave */
    int32_t waves_per_eu;   /* reserved, 0 */
} s5d_tuning;

typedef struct s5d_plan s5d_plan; /* opaque; immutable once created */

/* Validate `desc`, copy its coefficients and fix the blocking parameters.
 * `tuning` may be NULL (all fields chosen by the library).  On success *out
 * receives a plan that the caller releases with s5d_plan_destroy.  Errors:
 * S5D_EINVAL for malformed descriptors or tunings, S5D_EUNSUPPORTED for
 * stencils or tunings without a kernel, S5D_EDEVICE if no HIP device is
 * usable.  Nothing is enqueued. */
s5d_status s5d_plan_create(const s5d_desc *desc, const s5d_tuning *tuning, s5d_plan **out);

/* Release a plan (NULL is accepted). */
void s5d_plan_destroy(s5d_plan *plan);

/* The blocking parameters the plan uses (`chosen`, may be NULL) and the
 * size in bytes of one padded grid buffer (`bytes_per_buffer`, may be NULL). */
s5d_status s5d_plan_query(const s5d_plan *plan, s5d_tuning *chosen, int64_t *bytes_per_buffer);

/* Run the whole sweep of `plan` on device buffers.
 *   buf0: device pointer, padded grid in C order (dtype of the plan), holding
 *         the initial state including the boundary.
 *   buf1: device pointer, same size, distinct and not overlapping buf0; its
 *         contents are ignored.  The library first copies buf0's boundary
 *         cells into it.
 *   stream: a hipStream_t (NULL = the null stream).  Work is enqueued
 *         asynchronously; a kernel fault surfaces at the caller's next
 *         synchronisation with that stream.
 *   result_index: may be NULL; receives steps % 2, the buffer that holds the
 *         result once the stream has drained (steps = 0 enqueues nothing and
 *         leaves buf0 untouched).
 * The caller owns both buffers and must keep them alive until the stream has
 * drained.  Errors are detected before anything is enqueued (S5D_EINVAL),
 * except launch failures (S5D_EDEVICE), which may leave a partial sweep. */
s5d_status s5d_run(const s5d_plan *plan, void *buf0, void *buf1, void *stream,
                   int32_t *result_index);

/* Error and norm reductions in float64 between a computed grid and a
 * reference, for checking a sweep against an independent result on the GPU
 * (the relative error measure of the accuracy evaluation).  Over the n
 * elements g = got[i], o = ref[i], with d = |g - o| formed in float64, `out`
 * receives S5D_NORMS_COUNT doubles:
 *   out[0] = max d,   out[1] = max |o|,
 *   out[2] = max (d / |o|), taking d itself where o = 0,
 *   out[3] = sqrt(sum d^2 / n),   out[4] = sqrt(sum o^2 / n).
 * A NaN in g or o propagates into out[0], out[2] and out[3].  n = 0 gives zeros.
 *   got, ref: device pointers, n elements of got_dtype / ref_dtype (S5D_F32 or
 *             S5D_F64), 16-byte aligned (any torch allocation is).
 *   out: device pointer, S5D_NORMS_COUNT doubles, 8-byte aligned; every value
 *        is written, so it needs no clearing.
 *   workspace: device memory of at least s5d_error_norms_workspace_bytes(n)
 *        bytes (at most 80 KiB), not overlapping out; the caller owns it and
 *        must not reuse it before the stream has passed this call.
 * Asynchronous on `stream` (a hipStream_t; NULL = null stream); two kernel
 * launches, no allocation and no host synchronisation, so the call may be
 * captured in a HIP graph.  The result is a deterministic function of the
 * inputs and n.  Errors: S5D_EINVAL before anything is enqueued,
 * S5D_EDEVICE if a launch fails. */
#define S5D_NORMS_COUNT 5
int64_t s5d_error_norms_workspace_bytes(int64_t n); /* -1 if n < 0 */
s5d_status s5d_error_norms(const void *got, int32_t got_dtype, const void *ref, int32_t ref_dtype,
                           int64_t n, double *out, void *workspace, int64_t workspace_bytes,
                           void *stream);

/* Human-readable name of a status code (static storage). */
const char *s5d_status_string(s5d_status status);

/* Detail of the last error raised on the calling thread ("" if none). */
const char *s5d_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* STENCIL5D_H */
