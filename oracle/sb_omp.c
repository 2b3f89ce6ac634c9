/* Test infrastructure, not product code: the FP64 simulated-bifurcation
 * oracle (oracle/sb.py) as plain C, with the independent agents spread over
 * host threads by OpenMP.  Only the tests and the benchmark's CPU-baseline
 * leg load it.
 *
 * Paper section "Simulated Bifurcation": bSB (Eq. 5-8), dSB (Eq. 9-12) and
 * aSB (Eq. 1-4), symplectic Euler, all spins updated at once.  The steps,
 * their order and every operation are those of oracle/sb.py, in FP64 with
 * separate multiplies and adds (built with -ffp-contract=off), so a run is
 * bit-identical to the Python oracle for the same inputs:
 *   a_k = (a0 k) / K,
 *   F_i = (sum over row i in CSR order of J_ij v_j, from 0) + h_i,
 *         v = x (bSB, aSB) or sgn x with sgn(0) = +1 (dSB),
 *   bSB/dSB: y += dt (c0 F - (a0 - a_k) x);  x += (dt a0) y;
 *            |x| > 1 -> x = sgn x, y = 0,
 *   aSB:     y += dt (c0 F - ((x x) + (a0 - a_k)) x);  x += (dt a0) y.
 * The start (x0, y0) is an input (oracle/philox.py draws it).
 *
 * State arrays are [n][agents] (agents contiguous), as in the Python oracle.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

enum { SBO_BSB = 0, SBO_DSB = 1, SBO_ASB = 2 };

static double sgn(double v) { return v >= 0.0 ? 1.0 : -1.0; }

/* One agent, all steps.  xa, ya: that agent's positions and momenta
 * (length n, contiguous); F, v: scratch of length n. */
static void run_agent(int n, const int64_t *row_ptr, const int32_t *col, const double *J,
                      const double *h, double c0, int mode, int steps, double dt, double a0,
                      double *xa, double *ya, double *F, double *v) {
    const double dta0 = dt * a0;
    for (int k = 0; k < steps; ++k) {
        const double a_k = a0 * (double)k / (double)steps;
        const double g = a0 - a_k;
        for (int i = 0; i < n; ++i) v[i] = mode == SBO_DSB ? sgn(xa[i]) : xa[i];
        for (int i = 0; i < n; ++i) {
            double s = 0.0;
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) s = s + J[p] * v[col[p]];
            F[i] = s + h[i];
        }
        for (int i = 0; i < n; ++i) {
            double x = xa[i], y = ya[i];
            if (mode == SBO_ASB) {
                y = y + dt * (c0 * F[i] - (x * x + g) * x);
                x = x + dta0 * y;
            } else {
                y = y + dt * (c0 * F[i] - g * x);
                x = x + dta0 * y;
                if (x > 1.0 || x < -1.0) {
                    x = sgn(x);
                    y = 0.0;
                }
            }
            xa[i] = x;
            ya[i] = y;
        }
    }
}

/* Runs `agents` independent shots for `steps` steps on `threads` host
 * threads (0: OpenMP's default).  x, y: [n][agents], in: start, out: final.
 * Returns 0, or -1 on bad arguments / no memory.  *threads_used receives the
 * thread count of the parallel region. */
int sbo_run(int n, const int64_t *row_ptr, const int32_t *col, const double *J, const double *h,
            double c0, int mode, int agents, int steps, double dt, double a0, double *x,
            double *y, int threads, int *threads_used) {
    if (n < 1 || agents < 1 || steps < 0 || !row_ptr || !h || !x || !y) return -1;
    if (mode != SBO_BSB && mode != SBO_DSB && mode != SBO_ASB) return -1;
    int bad = 0, used = 1;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#endif
#pragma omp parallel reduction(| : bad)
    {
#ifdef _OPENMP
#pragma omp single
        used = omp_get_num_threads();
#endif
        /* every thread meets the worksharing loop, with or without memory */
        double *buf = (double *)malloc(sizeof(double) * 4 * (size_t)n);
#pragma omp for schedule(dynamic, 1)
        for (int m = 0; m < agents; ++m) {
            if (!buf) {
                bad = 1;
                continue;
            }
            double *xa = buf, *ya = buf + n, *F = buf + 2 * (size_t)n, *v = buf + 3 * (size_t)n;
            for (int i = 0; i < n; ++i) {
                xa[i] = x[(size_t)i * agents + m];
                ya[i] = y[(size_t)i * agents + m];
            }
            run_agent(n, row_ptr, col, J, h, c0, mode, steps, dt, a0, xa, ya, F, v);
            for (int i = 0; i < n; ++i) {
                x[(size_t)i * agents + m] = xa[i];
                y[(size_t)i * agents + m] = ya[i];
            }
        }
        free(buf);
    }
    if (threads_used) *threads_used = used;
    return bad ? -1 : 0;
}
