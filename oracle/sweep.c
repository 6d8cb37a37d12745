/*
 * Oracle sweeps for Laplacian mesh smoothing -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow-on-purpose C99 in float64, built with -O2 -ffp-contract=off so
 * that every sum and quotient below is exactly the IEEE operation written.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * call this file; the library never does.
 *
 * Neighbour lists (nbr_ptr/nbr) come from the oracle's own Python topology
 * code: for each vertex, its distinct edge-adjacent vertices in ascending
 * label order.  fixed[v] != 0 marks a vertex that never moves.
 *
 * Update rule (Eq. 1, Section 3.2): a free vertex moves to the arithmetic
 * mean of its N neighbours, p_v <- (1/N) sum_i p_i, applied to x and y
 * separately.  The sum runs over the neighbours in ascending label order
 * starting from 0.0 and is then divided by N (one IEEE division).
 *
 * Three sweep schedules:
 *  - oracle_jacobi:     every free vertex reads the previous sweep's values
 *                       (double buffered).  Optional OpenMP static schedule
 *                       over evenly divided vertices, as in the paper's
 *                       parallel runs (Section 5.1).
 *  - oracle_multicolor: vertices grouped by colour (no two neighbours share
 *                       a colour); colour c = 0..C-1 is updated in place in
 *                       turn, each vertex reading the current values.
 *  - oracle_gauss_seidel: Algorithm 1 read literally: free vertices updated
 *                       in place in storage order.  A reference only: its
 *                       result depends on the storage order.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static void mean_of_neighbours(int64_t b, int64_t e, const int32_t *nbr,
                               const double *x, const double *y,
                               double *ox, double *oy)
{
    double sx = 0.0, sy = 0.0;
    for (int64_t j = b; j < e; ++j) {
        sx += x[nbr[j]];
        sy += y[nbr[j]];
    }
    double cnt = (double)(e - b);
    *ox = sx / cnt;
    *oy = sy / cnt;
}

/* K Jacobi sweeps in place on (x, y).  Returns 0, or -1 on allocation failure. */
int oracle_jacobi(int32_t n, const int64_t *nbr_ptr, const int32_t *nbr,
                  const uint8_t *fixed, double *x, double *y, int32_t K,
                  int32_t nthreads)
{
    double *bx = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *by = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!bx || !by) { free(bx); free(by); return -1; }
    double *sx = x, *sy = y, *dx = bx, *dy = by;
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#else
    (void)nthreads;
#endif
    for (int32_t k = 0; k < K; ++k) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(nthreads)
#endif
        for (int32_t v = 0; v < n; ++v) {
            if (fixed[v]) {
                dx[v] = sx[v];
                dy[v] = sy[v];
            } else {
                mean_of_neighbours(nbr_ptr[v], nbr_ptr[v + 1], nbr, sx, sy, &dx[v], &dy[v]);
            }
        }
        double *t;
        t = sx; sx = dx; dx = t;
        t = sy; sy = dy; dy = t;
    }
    if (sx != x) {
        memcpy(x, sx, sizeof(double) * (size_t)n);
        memcpy(y, sy, sizeof(double) * (size_t)n);
    }
    free(bx);
    free(by);
    return 0;
}

/* K multicolour sweeps in place.  colour_ptr[c]..colour_ptr[c+1] indexes the
 * vertices of colour c in colour_list; only free vertices appear there. */
int oracle_multicolor(int32_t n, const int64_t *nbr_ptr, const int32_t *nbr,
                      int32_t ncolors, const int64_t *colour_ptr,
                      const int32_t *colour_list, double *x, double *y, int32_t K)
{
    (void)n;
    for (int32_t k = 0; k < K; ++k) {
        for (int32_t c = 0; c < ncolors; ++c) {
            for (int64_t i = colour_ptr[c]; i < colour_ptr[c + 1]; ++i) {
                int32_t v = colour_list[i];
                mean_of_neighbours(nbr_ptr[v], nbr_ptr[v + 1], nbr, x, y, &x[v], &y[v]);
            }
        }
    }
    return 0;
}

/* K sweeps of Algorithm 1 read literally: in place, storage order. */
int oracle_gauss_seidel(int32_t n, const int64_t *nbr_ptr, const int32_t *nbr,
                        const uint8_t *fixed, double *x, double *y, int32_t K)
{
    for (int32_t k = 0; k < K; ++k) {
        for (int32_t v = 0; v < n; ++v) {
            if (!fixed[v])
                mean_of_neighbours(nbr_ptr[v], nbr_ptr[v + 1], nbr, x, y, &x[v], &y[v]);
        }
    }
    return 0;
}
