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

/*
 * The same operator with the clover term formed at each site from the links
 * (no stored [V][12][12] field, so lattices of millions of sites fit):
 *
 *   A(x) = (i c_sw / 2) sum_{mu<nu} sigma_{mu nu} (x) (Q_{mu nu}(x) - Q_{mu nu}(x)^+) / 8,
 *   sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu],
 *
 * Q the sum of the four plaquette leaves at x in the mu-nu plane, each walked
 * with the same orientation (first along +mu or its turn, then +nu ...):
 *   x -> x+mu -> x+mu+nu -> x+nu -> x,   x -> x+nu -> x-mu+nu -> x-mu -> x,
 *   x -> x-mu -> x-mu-nu -> x-nu -> x,   x -> x-nu -> x+mu-nu -> x+mu -> x.
 */
static int64_t shifted(const int x[4], const int L[4], int mu, int smu, int nu, int snu) {
    int y[4] = {x[0], x[1], x[2], x[3]};
    y[mu] = (y[mu] + smu + L[mu]) % L[mu];
    y[nu] = (y[nu] + snu + L[nu]) % L[nu];
    return idx(y, L);
}

/* c = a b (3x3); with da / db the adjoint of a / b is used */
static void mul3(const cplx* a, int da, const cplx* b, int db, cplx* c) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx s = 0;
            for (int k = 0; k < 3; ++k) {
                const cplx aik = da ? conj(a[k * 3 + i]) : a[i * 3 + k];
                const cplx bkj = db ? conj(b[j * 3 + k]) : b[k * 3 + j];
                s += aik * bkj;
            }
            c[i * 3 + j] = s;
        }
}

/* product of four links l0 l1 l2 l3, each possibly daggered */
static void leaf(const cplx* l0, int d0, const cplx* l1, int d1, const cplx* l2, int d2, const cplx* l3, int d3,
                 cplx* out) {
    cplx t1[9], t2[9];
    mul3(l0, d0, l1, d1, t1);
    mul3(t1, 0, l2, d2, t2);
    mul3(t2, 0, l3, d3, out);
}

void oracle_wilson_clover_csw(const int L[4], const cplx* U, double csw, double m0, int antiperiodic_t,
                              const cplx* gamma, const cplx* in, cplx* out) {
    const int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
    cplx sig[4][4][4][4];   /* sigma[mu][nu][s][t] */
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = 0; nu < 4; ++nu)
            for (int s = 0; s < 4; ++s)
                for (int t = 0; t < 4; ++t) {
                    cplx c = 0;
                    for (int k = 0; k < 4; ++k)
                        c += gamma[(mu * 4 + s) * 4 + k] * gamma[(nu * 4 + k) * 4 + t]
                           - gamma[(nu * 4 + s) * 4 + k] * gamma[(mu * 4 + k) * 4 + t];
                    sig[mu][nu][s][t] = 0.5 * I * c;
                }
    oracle_wilson_clover(L, U, 0, m0, antiperiodic_t, gamma, in, out);
    if (csw == 0.0) return;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < V; ++i) {
        int x[4];
        int64_t r = i;
        for (int m = 0; m < 4; ++m) { x[m] = (int)(r % L[m]); r /= L[m]; }
        cplx A[12][12];
        for (int f = 0; f < 12; ++f)
            for (int g = 0; g < 12; ++g) A[f][g] = 0;
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                const cplx* Um = U + (int64_t)mu * V * 9;
                const cplx* Un = U + (int64_t)nu * V * 9;
                const int64_t xpm = shifted(x, L, mu, 1, nu, 0), xpn = shifted(x, L, mu, 0, nu, 1);
                const int64_t xmm = shifted(x, L, mu, -1, nu, 0), xmn = shifted(x, L, mu, 0, nu, -1);
                const int64_t xmm_pn = shifted(x, L, mu, -1, nu, 1), xmm_mn = shifted(x, L, mu, -1, nu, -1);
                const int64_t xpm_mn = shifted(x, L, mu, 1, nu, -1);
                cplx Q[9], t[9];
                leaf(Um + i * 9, 0, Un + xpm * 9, 0, Um + xpn * 9, 1, Un + i * 9, 1, Q);
                leaf(Un + i * 9, 0, Um + xmm_pn * 9, 1, Un + xmm * 9, 1, Um + xmm * 9, 0, t);
                for (int k = 0; k < 9; ++k) Q[k] += t[k];
                leaf(Um + xmm * 9, 1, Un + xmm_mn * 9, 1, Um + xmm_mn * 9, 0, Un + xmn * 9, 0, t);
                for (int k = 0; k < 9; ++k) Q[k] += t[k];
                leaf(Un + xmn * 9, 1, Um + xmn * 9, 0, Un + xpm_mn * 9, 0, Um + i * 9, 1, t);
                for (int k = 0; k < 9; ++k) Q[k] += t[k];
                for (int s = 0; s < 4; ++s)
                    for (int tt = 0; tt < 4; ++tt) {
                        const cplx w = 0.5 * I * csw * sig[mu][nu][s][tt];
                        if (w == 0) continue;
                        for (int a = 0; a < 3; ++a)
                            for (int b = 0; b < 3; ++b)
                                A[s * 3 + a][tt * 3 + b] += w * (Q[a * 3 + b] - conj(Q[b * 3 + a])) / 8.0;
                    }
            }
        const cplx* p = in + i * 12;
        for (int f = 0; f < 12; ++f) {
            cplx acc = 0;
            for (int g = 0; g < 12; ++g) acc += A[f][g] * p[g];
            out[i * 12 + f] += acc;
        }
    }
}
