/*
 * Oracle (test infrastructure): plain C restatement of the coarse operator of
 * Eq. (3) in the general form the Galerkin product of Sec. 3.4 produces,
 * FP64, one loop per coarse site, OpenMP over sites:
 *
 *   y(x) = X(x) u(x) + sum_{mu=0..3} [ Y_{2mu}(x) u(x + mu) + Y_{2mu+1}(x) u(x - mu) ]
 *
 * with periodic wrap on the coarse lattice (the fine operator's boundary sign
 * already sits inside Y).  Summation order per output row: the N terms of X,
 * then direction d = 0..7, each over its N columns in order.
 *
 * Layouts (complex128 interleaved): X [V][N][N], Y [8][V][N][N] (row major),
 * u, y [V][N][nrhs] (right-hand sides fastest).  Lattice L[0..3], x fastest.
 *
 * oracle_coarse_apply_timed repeats the apply `reps` times with `threads`
 * OpenMP threads (0: the OpenMP default) after one untimed warm-up, and returns
 * the mean seconds per apply from CLOCK_MONOTONIC (the steady clock) and the
 * thread count that ran.  It is the host baseline the GPU kernel is set
 * against; it is not tuned.
 */
#include <complex.h>
#include <omp.h>
#include <stdint.h>
#include <time.h>

typedef double complex cplx;

static int64_t site_index(const int x[4], const int L[4]) {
    return x[0] + (int64_t)L[0] * (x[1] + (int64_t)L[1] * (x[2] + (int64_t)L[2] * x[3]));
}

void oracle_coarse_apply(const int L[4], int N, int nrhs, const cplx* X, const cplx* Y, const cplx* u, cplx* y) {
    const int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < V; ++i) {
        int x[4];
        int64_t r = i;
        for (int m = 0; m < 4; ++m) {
            x[m] = (int)(r % L[m]);
            r /= L[m];
        }
        int64_t nb[8];
        for (int d = 0; d < 8; ++d) {
            const int mu = d / 2, step = (d % 2 == 0) ? 1 : -1;
            int z[4] = {x[0], x[1], x[2], x[3]};
            z[mu] = (x[mu] + step + L[mu]) % L[mu];
            nb[d] = site_index(z, L);
        }
        for (int a = 0; a < N; ++a)
            for (int k = 0; k < nrhs; ++k) {
                cplx acc = 0;
                const cplx* Xr = X + (i * N + a) * N;
                for (int b = 0; b < N; ++b) acc += Xr[b] * u[(i * N + b) * nrhs + k];
                for (int d = 0; d < 8; ++d) {
                    const cplx* Yr = Y + (((int64_t)d * V + i) * N + a) * N;
                    for (int b = 0; b < N; ++b) acc += Yr[b] * u[(nb[d] * N + b) * nrhs + k];
                }
                y[(i * N + a) * nrhs + k] = acc;
            }
    }
}

double oracle_coarse_apply_timed(const int L[4], int N, int nrhs, const cplx* X, const cplx* Y, const cplx* u,
                                 cplx* y, int reps, int threads, int* threads_used) {
    const int before = omp_get_max_threads();
    if (threads > 0) omp_set_num_threads(threads);
    int used = 1;
#pragma omp parallel
    {
#pragma omp single
        used = omp_get_num_threads();
    }
    oracle_coarse_apply(L, N, nrhs, X, Y, u, y);   /* warm-up */
    struct timespec t0, t1;
    clock_gettime(CLOCK_MONOTONIC, &t0);
    for (int r = 0; r < reps; ++r) oracle_coarse_apply(L, N, nrhs, X, Y, u, y);
    clock_gettime(CLOCK_MONOTONIC, &t1);
    omp_set_num_threads(before);
    if (threads_used) *threads_used = used;
    return ((double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec)) / (reps > 0 ? reps : 1);
}
