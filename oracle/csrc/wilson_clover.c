/*
 * Oracle (test infrastructure): plain C restatement of the Wilson-clover
 * matrix of Eq. (2), FP64, one loop per site, OpenMP over sites.  Used where
 * the numpy restatement in wilson.py is too slow (eigenvalue searches on
 * 16^3x32).  Both are pinned by the same closed-form tests.
 *
 *   out(x) = (4 + m0) in(x) + A(x) in(x)
 *          - 1/2 sum_mu [ eta+ (1 - gamma_mu) (x) U_mu(x)       in(x + mu)
 *                        + eta- (1 + gamma_mu) (x) U_mu(x - mu)^+ in(x - mu) ]
 *
 * Layouts (complex128 interleaved): U [4][V][3][3], clover [V][12][12] or
 * NULL, gamma [4][4][4] (the caller's Dirac matrices), fields [V][4][3].
 * eta = -1 on hops across the time boundary when antiperiodic_t is set.
 */
#include <complex.h>
#include <stdint.h>

typedef double complex cplx;

static int64_t idx(const int x[4], const int L[4]) {
    return x[0] + (int64_t)L[0] * (x[1] + (int64_t)L[1] * (x[2] + (int64_t)L[2] * x[3]));
}

void oracle_wilson_clover(const int L[4], const cplx* U, const cplx* clover, double m0, int antiperiodic_t,
                          const cplx* gamma, const cplx* in, cplx* out) {
    const int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
    cplx Pm[4][4][4], Pp[4][4][4];
    for (int mu = 0; mu < 4; ++mu)
        for (int s = 0; s < 4; ++s)
            for (int t = 0; t < 4; ++t) {
                const cplx g = gamma[(mu * 4 + s) * 4 + t];
                Pm[mu][s][t] = (s == t ? 1.0 : 0.0) - g;
                Pp[mu][s][t] = (s == t ? 1.0 : 0.0) + g;
            }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < V; ++i) {
        int x[4];
        int64_t r = i;
        for (int m = 0; m < 4; ++m) { x[m] = (int)(r % L[m]); r /= L[m]; }
        const cplx* p = in + i * 12;
        cplx acc[12];
        for (int f = 0; f < 12; ++f) acc[f] = (4.0 + m0) * p[f];
        if (clover)
            for (int f = 0; f < 12; ++f)
                for (int g = 0; g < 12; ++g) acc[f] += clover[(i * 12 + f) * 12 + g] * p[g];
        for (int mu = 0; mu < 4; ++mu) {
            int y[4] = {x[0], x[1], x[2], x[3]};
            /* forward hop */
            y[mu] = (x[mu] + 1) % L[mu];
            const int64_t jf = idx(y, L);
            const double ef = (antiperiodic_t && mu == 3 && x[3] == L[3] - 1) ? -1.0 : 1.0;
            const cplx* Uf = U + ((int64_t)mu * V + i) * 9;
            /* backward hop */
            y[mu] = (x[mu] - 1 + L[mu]) % L[mu];
            const int64_t jb = idx(y, L);
            const double eb = (antiperiodic_t && mu == 3 && x[3] == 0) ? -1.0 : 1.0;
            const cplx* Ub = U + ((int64_t)mu * V + jb) * 9;
            for (int s = 0; s < 4; ++s)
                for (int a = 0; a < 3; ++a) {
                    cplx hf = 0, hb = 0;
                    for (int t = 0; t < 4; ++t)
                        for (int b = 0; b < 3; ++b) {
                            hf += Pm[mu][s][t] * Uf[a * 3 + b] * in[jf * 12 + t * 3 + b];
                            hb += Pp[mu][s][t] * conj(Ub[b * 3 + a]) * in[jb * 12 + t * 3 + b];
                        }
                    acc[s * 3 + a] -= 0.5 * (ef * hf + eb * hb);
                }
        }
        for (int f = 0; f < 12; ++f) out[i * 12 + f] = acc[f];
    }
}
