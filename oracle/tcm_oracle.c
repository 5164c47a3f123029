/*
 * tcm_oracle.c -- plain, slow, obviously-correct CPU oracle for the
 * Triggered Cells Method (TCM) hot path.
 *
 * THIS IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it.  The GPU library shares no
 * code, header, table or helper with it, and never calls it.
 *
 *   O1  oracle_dense_{f32,f64}: eq.(3) over the whole grid (two arrays,
 *       phi^{n+1} overwrites phi^{n-1}); 1-D/2-D variants of the same
 *       central-difference operator for closed-form pins.
 *   O2  otcm_*_{f32,f64}: TCM with the paper's cell bookkeeping (Table 1:
 *       Triggered_cells, Triggered_hist, Max_cell_val, Cell2box, Box2cell,
 *       Shutdown_log, Trig_level), boxes padded with the neighbours'
 *       boundaries before the basic calculation ("Time stepping"), and the
 *       activation process of "Updating active cells" (items 1-4, 6-8) run
 *       every step, or every k <= 8 steps (eq.(5)) with the diagonal
 *       neighbourhood of item 5 / Figure 3; optional shutdown decay
 *       (eq.(6)) and levels relative to the domain maximum.
 *   O3  oracle_adjoint_f64: discrete adjoint of O1 (FP64) with
 *       checkpoint-and-recompute, gradient with respect to c.
 *   eq.(4), eq.(5), eq.(6): the paper's closed forms.
 *
 * Readings of points the paper leaves open (each restated where used):
 *   - boundary: zero field outside the domain;
 *   - neighbour-sum order ((x+ + x-) + (y+ + y-)) + (z+ + z-), no FMA;
 *   - source: additive, applied after the stencil and before the
 *     activation process; its cell stays active while samples remain;
 *   - activation: a cell stays active while any |phi^{n+1}| or |phi^n| in
 *     it exceeds `retire`; a face whose |phi^{n+1}| exceeds `trigger`
 *     activates the cell across it; a cell that stops is unboxed at once,
 *     or after `shutdown_steps` steps scaled by alpha (eq.(6));
 *   - update every k > 1 steps: a cell with any |phi| of either level above
 *     `trigger` (or a source still inserting) activates and keeps its 26
 *     neighbours, and a source's 26 neighbours are boxed with it.
 *
 * Build: gcc -O3 -fopenmp -ffp-contract=off -fno-fast-math (no FTZ/DAZ).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define REAL float
#define SFX(name) name##_f32
#define SFX_IS_F64 0
#include "tcm_oracle_impl.h"
#undef REAL
#undef SFX
#undef SFX_IS_F64

#define REAL double
#define SFX(name) name##_f64
#define SFX_IS_F64 1
#include "tcm_oracle_impl.h"
#undef REAL
#undef SFX
#undef SFX_IS_F64

/* eq.(4): c dt sqrt(sum_d 1/dx_d^2) <= 1 with equal spacing in `ndim`
 * dimensions, i.e. (c dt / dx)^2 * ndim <= 1.  Returns 1 if satisfied. */
int oracle_cfl_ok(double cmax, double dt, double dx, int ndim)
{
    const double r = cmax * dt / dx;
    return r * r * (double)ndim <= 1.0 + 4.0 * 2.220446049250313e-16;
}

/* eq.(5): activation-update interval n = dx * (cell length) / (2 c dt). */
double oracle_update_interval(double dx, double cell_len, double c, double dt)
{
    return dx * cell_len / (2.0 * c * dt);
}

/* eq.(6): total attenuation of the shutdown decay, A = alpha^n. */
double oracle_decay_total(double alpha, int n)
{
    return pow(alpha, (double)n);
}

int oracle_openmp_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Host memory bandwidth beside the CPU baseline: the STREAM triad
 * a[i] = b[i] + s*c[i] over n doubles per array (24 bytes per element),
 * best of reps passes, in GB/s.  Arrays are first touched by the threads
 * that later use them.  Returns -1 when the arrays cannot be allocated. */
double oracle_stream_triad(long n, int reps)
{
    double *a = malloc((size_t)n * sizeof(double));
    double *b = malloc((size_t)n * sizeof(double));
    double *c = malloc((size_t)n * sizeof(double));
    double best = -1.0;
    if (!a || !b || !c) goto out;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; i++) { a[i] = 0.0; b[i] = 1.0; c[i] = 2.0; }
    for (int r = 0; r < reps; r++) {
        struct timespec t0, t1;
        clock_gettime(CLOCK_MONOTONIC, &t0);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; i++) a[i] = b[i] + 3.0 * c[i];
        clock_gettime(CLOCK_MONOTONIC, &t1);
        const double s = (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);
        const double gbs = 24.0 * (double)n / s / 1e9;
        if (a[n / 2] != 7.0) { best = -1.0; goto out; }
        if (gbs > best) best = gbs;
    }
out:
    free(a); free(b); free(c);
    return best;
}

/* Thread count of the following parallel loops (timing on one core). */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
