/*
 * CPU oracle for the Jacobi-style stencil sweep.  TEST INFRASTRUCTURE ONLY:
 * it is used by the test-suite, by the smoke check and by the CPU-baseline leg
 * of the benchmark, never by the GPU library.  It shares no code, header or
 * table with the GPU path.
 *
 * What it computes (AN5D, Background "Stencil Computation"; Fig. 4 and the
 * host-code description in "Code Generation"; Table 3 for the star/box
 * synthetic stencils):
 *
 *   A is a double-buffered, padded grid A[2][P0][P1] (2D) or A[2][P0][P1][P2]
 *   (3D), P_i = I_i + 2*radius.  The border of width `radius` on every face is
 *   the fixed boundary: it is read but never written.  For t = 0..T-1 every
 *   interior cell p of A[(t+1)%2] receives
 *
 *       A[(t+1)%2][p] = sum_k c_k * A[t%2][p + o_k]
 *
 *   and the result of the whole sweep is A[T%2].
 *
 * The offsets o_k are enumerated in ONE canonical order: lexicographic in
 * (d0, d1[, d2]), each component in [-radius, radius], axis 0 (the outermost,
 * slowest-varying axis) first.  A box stencil keeps every offset; a star
 * stencil keeps the offsets with at most one non-zero component.  For the 2D
 * 5-point star this order is exactly the term order printed in Fig. 4.
 *
 * Arithmetic: the sum is formed left to right in that order in the working
 * precision, product then add, with no fused multiply-add (this file must be
 * built with -ffp-contract=off and without fast-math).  Cells are
 * independent, so the OpenMP split over axis 0 gives the same bits as a
 * serial run.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_MAX_POINTS 729 /* (2*4+1)^3: box, radius 4, 3D */

/* Canonical offsets; returns their count, or -1 for an unsupported stencil.
 * out[3*k + a] is component a of offset k (unused components are 0). */
int oracle_offsets(int ndim, int radius, int box, int32_t *out)
{
    if ((ndim != 2 && ndim != 3) || radius < 1 || radius > 4)
        return -1;
    int n = 0;
    int r = radius;
    int lo2 = (ndim == 3) ? -r : 0, hi2 = (ndim == 3) ? r : 0;
    for (int d0 = -r; d0 <= r; ++d0)
        for (int d1 = -r; d1 <= r; ++d1)
            for (int d2 = lo2; d2 <= hi2; ++d2) {
                int nonzero = (d0 != 0) + (d1 != 0) + (d2 != 0);
                if (!box && nonzero > 1)
                    continue;
                if (out) {
                    out[3 * n + 0] = d0;
                    out[3 * n + 1] = d1;
                    out[3 * n + 2] = d2;
                }
                ++n;
            }
    return n;
}

/* One definition of the sweep per working precision.  `buf0` holds the
 * initial padded grid (boundary included); `buf1` receives a copy of it so
 * both buffers carry the same boundary; on return the result is in
 * buf[T % 2].  Returns T % 2, or a negative value on bad arguments. */
#define ORACLE_SWEEP(NAME, REAL)                                                  \
    int NAME(int ndim, int radius, int box, const int64_t *interior,              \
             int64_t steps, const REAL *coeffs, int64_t n_coeffs,                 \
             REAL *buf0, REAL *buf1, int threads)                                 \
    {                                                                             \
        int32_t off3[3 * ORACLE_MAX_POINTS];                                      \
        int n = oracle_offsets(ndim, radius, box, off3);                          \
        if (n < 0 || n != n_coeffs || steps < 0 || !buf0 || !buf1 || !coeffs)     \
            return -1;                                                            \
        int64_t I0 = interior[0], I1 = interior[1];                               \
        int64_t I2 = (ndim == 3) ? interior[2] : 1;                               \
        if (I0 < 1 || I1 < 1 || I2 < 1)                                           \
            return -1;                                                            \
        int64_t r = radius;                                                       \
        int64_t P0 = I0 + 2 * r, P1 = I1 + 2 * r;                                 \
        int64_t P2 = (ndim == 3) ? I2 + 2 * r : 1;                                \
        int64_t r2 = (ndim == 3) ? r : 0;                                         \
        int64_t total = P0 * P1 * P2;                                             \
        int64_t lin[ORACLE_MAX_POINTS];                                           \
        for (int k = 0; k < n; ++k)                                               \
            lin[k] = (int64_t)off3[3 * k] * P1 * P2 +                             \
                     (int64_t)off3[3 * k + 1] * P2 + (int64_t)off3[3 * k + 2];    \
        memcpy(buf1, buf0, (size_t)total * sizeof(REAL));                         \
        if (threads > 0) {                                                        \
            OMP_SET(threads);                                                     \
        }                                                                         \
        for (int64_t t = 0; t < steps; ++t) {                                     \
            const REAL *src = (t % 2 == 0) ? buf0 : buf1;                         \
            REAL *dst = (t % 2 == 0) ? buf1 : buf0;                               \
            OMP_FOR                                                               \
            for (int64_t i0 = r; i0 < r + I0; ++i0)                               \
                for (int64_t i1 = r; i1 < r + I1; ++i1)                           \
                    for (int64_t i2 = r2; i2 < r2 + I2; ++i2) {                   \
                        int64_t p = (i0 * P1 + i1) * P2 + i2;                     \
                        REAL acc = coeffs[0] * src[p + lin[0]];                   \
                        for (int k = 1; k < n; ++k)                               \
                            acc = acc + coeffs[k] * src[p + lin[k]];              \
                        dst[p] = acc;                                             \
                    }                                                             \
        }                                                                         \
        return (int)(steps % 2);                                                  \
    }

#ifdef _OPENMP
#define OMP_SET(n) omp_set_num_threads(n)
#define OMP_FOR _Pragma("omp parallel for schedule(static)")
#else
#define OMP_SET(n) ((void)(n))
#define OMP_FOR
#endif

ORACLE_SWEEP(oracle_sweep_f64, double)
ORACLE_SWEEP(oracle_sweep_f32, float)

/*
 * Compensated float32 accumulation (the float32 "Kahan" variant of the
 * library): each cell's terms are summed with the compensated dot product of
 * Ogita, Rump and Oishi (SIAM J. Sci. Comput. 26(6), 2005, Dot2): every
 * product c*x is split exactly into its rounded value h and error e by a
 * fused multiply-add, h is added to the running sum s with the error-free
 * two-sum of Knuth (s' = s + h, error t), the errors are gathered in a second
 * float32 accumulator q = q + (e + t), and the cell receives s + q rounded
 * once.  The first term sets s = h, q = e.  Same canonical term order as the
 * plain sweep.
 */
#include <math.h>

static float dot2_cell(const float *coeffs, const float *src, int64_t p, const int64_t *lin, int n)
{
    float h = coeffs[0] * src[p + lin[0]];
    float s = h;
    float q = fmaf(coeffs[0], src[p + lin[0]], -h);
    for (int k = 1; k < n; ++k) {
        float x = src[p + lin[k]];
        h = coeffs[k] * x;
        float e = fmaf(coeffs[k], x, -h);
        float t1 = s + h;
        float z = t1 - s;
        float t = (s - (t1 - z)) + (h - z);
        s = t1;
        q = q + (e + t);
    }
    return s + q;
}

int oracle_sweep_f32_dot2(int ndim, int radius, int box, const int64_t *interior, int64_t steps,
                          const float *coeffs, int64_t n_coeffs, float *buf0, float *buf1,
                          int threads)
{
    int32_t off3[3 * ORACLE_MAX_POINTS];
    int n = oracle_offsets(ndim, radius, box, off3);
    if (n < 0 || n != n_coeffs || steps < 0 || !buf0 || !buf1 || !coeffs)
        return -1;
    int64_t I0 = interior[0], I1 = interior[1];
    int64_t I2 = (ndim == 3) ? interior[2] : 1;
    if (I0 < 1 || I1 < 1 || I2 < 1)
        return -1;
    int64_t r = radius;
    int64_t P0 = I0 + 2 * r, P1 = I1 + 2 * r;
    int64_t P2 = (ndim == 3) ? I2 + 2 * r : 1;
    int64_t r2 = (ndim == 3) ? r : 0;
    int64_t lin[ORACLE_MAX_POINTS];
    for (int k = 0; k < n; ++k)
        lin[k] = (int64_t)off3[3 * k] * P1 * P2 + (int64_t)off3[3 * k + 1] * P2 + (int64_t)off3[3 * k + 2];
    memcpy(buf1, buf0, (size_t)(P0 * P1 * P2) * sizeof(float));
    if (threads > 0) {
        OMP_SET(threads);
    }
    for (int64_t t = 0; t < steps; ++t) {
        const float *src = (t % 2 == 0) ? buf0 : buf1;
        float *dst = (t % 2 == 0) ? buf1 : buf0;
        OMP_FOR
        for (int64_t i0 = r; i0 < r + I0; ++i0)
            for (int64_t i1 = r; i1 < r + I1; ++i1)
                for (int64_t i2 = r2; i2 < r2 + I2; ++i2) {
                    int64_t p = (i0 * P1 + i1) * P2 + i2;
                    dst[p] = dot2_cell(coeffs, src, p, lin, n);
                }
    }
    return (int)(steps % 2);
}

/*
 * Expression stencils of the paper's general benchmarks (Table 3,
 * "Benchmarks"), each written as its plain definition in the working
 * precision, product then add, no fused multiply-add.
 *
 * DIV: the weighted sum of a star or box stencil, divided by one constant c0
 *   A[(t+1)%2][p] = (sum_k c_k * A[t%2][p + o_k]) / c0
 * (j2d5pt: 2D star radius 1, printed in Fig. 4 with divisor 118; j2d9pt: 2D
 * star radius 2; j2d9pt-gol: 2D box radius 1; j3d27pt: 3D box radius 1).
 * The sum is formed left to right in canonical offset order, then divided
 * once.
 */
#define ORACLE_SWEEP_DIV(NAME, REAL)                                              \
    int NAME(int ndim, int radius, int box, const int64_t *interior,              \
             int64_t steps, const REAL *coeffs, int64_t n_coeffs, REAL c0,        \
             REAL *buf0, REAL *buf1, int threads)                                 \
    {                                                                             \
        int32_t off3[3 * ORACLE_MAX_POINTS];                                      \
        int n = oracle_offsets(ndim, radius, box, off3);                          \
        if (n < 0 || n != n_coeffs || steps < 0 || !buf0 || !buf1 || !coeffs)     \
            return -1;                                                            \
        int64_t I0 = interior[0], I1 = interior[1];                               \
        int64_t I2 = (ndim == 3) ? interior[2] : 1;                               \
        if (I0 < 1 || I1 < 1 || I2 < 1)                                           \
            return -1;                                                            \
        int64_t r = radius;                                                       \
        int64_t P0 = I0 + 2 * r, P1 = I1 + 2 * r;                                 \
        int64_t P2 = (ndim == 3) ? I2 + 2 * r : 1;                                \
        int64_t r2 = (ndim == 3) ? r : 0;                                         \
        int64_t lin[ORACLE_MAX_POINTS];                                           \
        for (int k = 0; k < n; ++k)                                               \
            lin[k] = (int64_t)off3[3 * k] * P1 * P2 +                             \
                     (int64_t)off3[3 * k + 1] * P2 + (int64_t)off3[3 * k + 2];    \
        memcpy(buf1, buf0, (size_t)(P0 * P1 * P2) * sizeof(REAL));               \
        if (threads > 0) {                                                        \
            OMP_SET(threads);                                                     \
        }                                                                         \
        for (int64_t t = 0; t < steps; ++t) {                                     \
            const REAL *src = (t % 2 == 0) ? buf0 : buf1;                         \
            REAL *dst = (t % 2 == 0) ? buf1 : buf0;                               \
            OMP_FOR                                                               \
            for (int64_t i0 = r; i0 < r + I0; ++i0)                               \
                for (int64_t i1 = r; i1 < r + I1; ++i1)                           \
                    for (int64_t i2 = r2; i2 < r2 + I2; ++i2) {                   \
                        int64_t p = (i0 * P1 + i1) * P2 + i2;                     \
                        REAL acc = coeffs[0] * src[p + lin[0]];                   \
                        for (int k = 1; k < n; ++k)                               \
                            acc = acc + coeffs[k] * src[p + lin[k]];              \
                        dst[p] = acc / c0;                                        \
                    }                                                             \
        }                                                                         \
        return (int)(steps % 2);                                                  \
    }

ORACLE_SWEEP_DIV(oracle_sweep_div_f64, double)
ORACLE_SWEEP_DIV(oracle_sweep_div_f32, float)

/*
 * gradient2d (Table 3): 2D, radius 1, non-linear in the cell values:
 *   A'[p] = cc * A[p] + 1 / sqrt(c0 + sum_n (A[p] - A[n]) * (A[p] - A[n]))
 * over the four axis neighbours n of p.  The sum starts from c0 and adds the
 * squared differences in canonical offset order, (-1,0), (0,-1), (0,1),
 * (1,0); then the square root (correctly rounded), the quotient 1 / root and
 * finally the product cc * A[p] plus that quotient.
 */
#define ORACLE_SWEEP_GRADIENT(NAME, REAL, SQRT)                                   \
    int NAME(const int64_t *interior, int64_t steps, REAL cc, REAL c0,            \
             REAL *buf0, REAL *buf1, int threads)                                 \
    {                                                                             \
        if (steps < 0 || !buf0 || !buf1)                                          \
            return -1;                                                            \
        int64_t I0 = interior[0], I1 = interior[1];                               \
        if (I0 < 1 || I1 < 1)                                                     \
            return -1;                                                            \
        int64_t P0 = I0 + 2, P1 = I1 + 2;                                         \
        const int64_t nb[4] = {-P1, -1, 1, P1};                                   \
        memcpy(buf1, buf0, (size_t)(P0 * P1) * sizeof(REAL));                     \
        if (threads > 0) {                                                        \
            OMP_SET(threads);                                                     \
        }                                                                         \
        for (int64_t t = 0; t < steps; ++t) {                                     \
            const REAL *src = (t % 2 == 0) ? buf0 : buf1;                         \
            REAL *dst = (t % 2 == 0) ? buf1 : buf0;                               \
            OMP_FOR                                                               \
            for (int64_t i0 = 1; i0 < 1 + I0; ++i0)                               \
                for (int64_t i1 = 1; i1 < 1 + I1; ++i1) {                         \
                    int64_t p = i0 * P1 + i1;                                     \
                    REAL s = c0;                                                  \
                    for (int k = 0; k < 4; ++k) {                                 \
                        REAL d = src[p] - src[p + nb[k]];                         \
                        s = s + d * d;                                            \
                    }                                                             \
                    REAL root = SQRT(s);                                          \
                    REAL q = (REAL)1 / root;                                      \
                    dst[p] = cc * src[p] + q;                                     \
                }                                                                 \
        }                                                                         \
        return (int)(steps % 2);                                                  \
    }

ORACLE_SWEEP_GRADIENT(oracle_sweep_gradient_f64, double, sqrt)
ORACLE_SWEEP_GRADIENT(oracle_sweep_gradient_f32, float, sqrtf)

/*
 * Variable coefficients (multi-array input): every interior cell has its own
 * weights,
 *   A'[p] = sum_k C[k][p] * A[p + o_k]
 * in canonical offset order.  C holds n_points arrays of the interior's
 * extents (I0 x I1 [x I2], C order), weight k of all cells first: C[k][q] is
 * weight k of the interior cell with 0-based interior index q.
 */
#define ORACLE_SWEEP_VARCOEF(NAME, REAL)                                          \
    int NAME(int ndim, int radius, int box, const int64_t *interior,              \
             int64_t steps, const REAL *cfield, REAL *buf0, REAL *buf1,           \
             int threads)                                                         \
    {                                                                             \
        int32_t off3[3 * ORACLE_MAX_POINTS];                                      \
        int n = oracle_offsets(ndim, radius, box, off3);                          \
        if (n < 0 || steps < 0 || !buf0 || !buf1 || !cfield)                      \
            return -1;                                                            \
        int64_t I0 = interior[0], I1 = interior[1];                               \
        int64_t I2 = (ndim == 3) ? interior[2] : 1;                               \
        if (I0 < 1 || I1 < 1 || I2 < 1)                                           \
            return -1;                                                            \
        int64_t r = radius;                                                       \
        int64_t P0 = I0 + 2 * r, P1 = I1 + 2 * r;                                 \
        int64_t P2 = (ndim == 3) ? I2 + 2 * r : 1;                                \
        int64_t r2 = (ndim == 3) ? r : 0;                                         \
        int64_t cells = I0 * I1 * I2;                                             \
        int64_t lin[ORACLE_MAX_POINTS];                                           \
        for (int k = 0; k < n; ++k)                                               \
            lin[k] = (int64_t)off3[3 * k] * P1 * P2 +                             \
                     (int64_t)off3[3 * k + 1] * P2 + (int64_t)off3[3 * k + 2];    \
        memcpy(buf1, buf0, (size_t)(P0 * P1 * P2) * sizeof(REAL));               \
        if (threads > 0) {                                                        \
            OMP_SET(threads);                                                     \
        }                                                                         \
        for (int64_t t = 0; t < steps; ++t) {                                     \
            const REAL *src = (t % 2 == 0) ? buf0 : buf1;                         \
            REAL *dst = (t % 2 == 0) ? buf1 : buf0;                               \
            OMP_FOR                                                               \
            for (int64_t i0 = r; i0 < r + I0; ++i0)                               \
                for (int64_t i1 = r; i1 < r + I1; ++i1)                           \
                    for (int64_t i2 = r2; i2 < r2 + I2; ++i2) {                   \
                        int64_t p = (i0 * P1 + i1) * P2 + i2;                     \
                        int64_t q = ((i0 - r) * I1 + (i1 - r)) * I2 + (i2 - r2);  \
                        REAL acc = cfield[q] * src[p + lin[0]];                   \
                        for (int k = 1; k < n; ++k)                               \
                            acc = acc + cfield[k * cells + q] * src[p + lin[k]];  \
                        dst[p] = acc;                                             \
                    }                                                             \
        }                                                                         \
        return (int)(steps % 2);                                                  \
    }

ORACLE_SWEEP_VARCOEF(oracle_sweep_varcoef_f64, double)
ORACLE_SWEEP_VARCOEF(oracle_sweep_varcoef_f32, float)

/* Number of OpenMP threads a parallel region would use (1 without OpenMP). */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
