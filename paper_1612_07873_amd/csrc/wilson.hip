// Fine Wilson-clover operator, Eq. (2):
//   M psi(x) = (4 + m0 + A(x)) psi(x)
//              - 1/2 sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu) + (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu) ]
// in the chiral basis gamma_k = [[0, g_k], [g_k^+, 0]] with g_k = -i sigma_k (k = 1..3)
// and g_4 = 1, so gamma_5 = diag(1, 1, -1, -1).  Each hop is done on the
// two-spin projection: (1 - gamma) psi = [a; -g^+ a] with a = psi_up - g psi_dn,
// and (1 + gamma) psi = [b; g^+ b] with b = psi_up + g psi_dn, so only the
// projected half spinor is multiplied by the SU(3) link.
//
// The clover term A(x) (the Sheikholeslami-Wohlert form the paper names) is
// built on the device from the clover-leaf field strength:
//   A = (i c_sw / 2) sum_{mu<nu} sigma_{mu nu} (x) (Q_{mu nu} - Q_{mu nu}^+)/8,
// sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu].  sigma commutes with gamma_5, so A
// is two Hermitian 6x6 blocks (one per chirality), stored packed.
//
// Device layout (internal): links SoA [4][9][V] complex with the antiperiodic
// time sign folded into U_3 on the last time slice (it multiplies both the
// forward hop out of that slice and the backward hop into it); clover SoA
// [2][36][V] reals (6 diagonal reals, then the 15 upper off-diagonal complex
// entries row by row); spinors [V][4][3] complex (the canonical layout).
#include "handles.h"

#include <vector>

namespace qmg {

// ------------------------------------------------------------------ helpers
template <typename R> struct c3 { cpx<R> v[3]; };

template <typename R>
__device__ __forceinline__ cpx<R> cadd(cpx<R> a, cpx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cpx<R> csub(cpx<R> a, cpx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cpx<R> cmulc(cpx<R> a, cpx<R> b) {  // conj(a) * b
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename R> __device__ __forceinline__ cpx<R> ci(cpx<R> a) { return {-a.im, a.re}; }   // i a
template <typename R> __device__ __forceinline__ cpx<R> cmi(cpx<R> a) { return {a.im, -a.re}; }  // -i a
template <typename R> __device__ __forceinline__ cpx<R> cneg(cpx<R> a) { return {-a.re, -a.im}; }

// g_mu * (p, q) for the 2x2 off-diagonal block of gamma_mu
template <int MU, typename R>
__device__ __forceinline__ void gmul(cpx<R>& o0, cpx<R>& o1, cpx<R> p, cpx<R> q) {
    if (MU == 0) { o0 = cmi(q); o1 = cmi(p); }          // -i sigma_1
    else if (MU == 1) { o0 = cneg(q); o1 = p; }         // -i sigma_2 = [[0,-1],[1,0]]
    else if (MU == 2) { o0 = cmi(p); o1 = ci(q); }      // -i sigma_3 = diag(-i, i)
    else { o0 = p; o1 = q; }                            // 1
}
// g_mu^+ * (p, q)
template <int MU, typename R>
__device__ __forceinline__ void gdmul(cpx<R>& o0, cpx<R>& o1, cpx<R> p, cpx<R> q) {
    if (MU == 0) { o0 = ci(q); o1 = ci(p); }            // i sigma_1
    else if (MU == 1) { o0 = q; o1 = cneg(p); }         // i sigma_2 = [[0,1],[-1,0]]
    else if (MU == 2) { o0 = ci(p); o1 = cmi(q); }      // i sigma_3 = diag(i, -i)
    else { o0 = p; o1 = q; }
}

template <typename R>
__device__ __forceinline__ void load_link(cpx<R> u[9], const cpx<R>* __restrict__ U, int mu, int64_t site,
                                          int64_t V) {
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = U[((int64_t)mu * 9 + e) * V + site];
}

// A site's 12 spinor components, with 16-byte loads (6 in FP32, 12 in FP64).
template <typename R>
__device__ __forceinline__ void load_spinor(cpx<R> p[12], const cpx<R>* __restrict__ src) {
    if constexpr (sizeof(R) == 4) {
        const float4* s4 = reinterpret_cast<const float4*>(src);
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            const float4 v = s4[i];
            p[2 * i] = cpx<R>{v.x, v.y};
            p[2 * i + 1] = cpx<R>{v.z, v.w};
        }
    } else {
#pragma unroll
        for (int f = 0; f < 12; ++f) p[f] = src[f];
    }
}

template <typename R>
__device__ __forceinline__ void store_spinor(cpx<R>* __restrict__ dst, const cpx<R> p[12]) {
    if constexpr (sizeof(R) == 4) {
        float4* d4 = reinterpret_cast<float4*>(dst);
#pragma unroll
        for (int i = 0; i < 6; ++i) d4[i] = make_float4(p[2 * i].re, p[2 * i].im, p[2 * i + 1].re, p[2 * i + 1].im);
    } else {
#pragma unroll
        for (int f = 0; f < 12; ++f) dst[f] = p[f];
    }
}

// One hop in direction MU; BACK selects the backward hop.  acc += -1/2 * P (x) W psi(n).
template <int MU, bool BACK, typename R>
__device__ __forceinline__ void hop(cpx<R> acc[12], const cpx<R>* __restrict__ in,
                                    const cpx<R>* __restrict__ U, int64_t V, int64_t site, int64_t n) {
    cpx<R> p[12];
    load_spinor(p, in + n * 12);
    cpx<R> a[2][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cpx<R> g0, g1;
        gmul<MU>(g0, g1, p[6 + c], p[9 + c]);
        if (!BACK) { a[0][c] = csub(p[c], g0); a[1][c] = csub(p[3 + c], g1); }
        else { a[0][c] = cadd(p[c], g0); a[1][c] = cadd(p[3 + c], g1); }
    }
    cpx<R> u[9];
    load_link(u, U, MU, BACK ? n : site, V);
    cpx<R> w[2][3];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            cpx<R> t = {0, 0};
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (!BACK) t = cadd(t, cmul(u[r * 3 + c], a[s][c]));      // U a
                else t = cadd(t, cmulc(u[c * 3 + r], a[s][c]));           // U^+ a
            }
            w[s][r] = t;
        }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cpx<R> l0, l1;
        gdmul<MU>(l0, l1, w[0][c], w[1][c]);
        const R h = R(-0.5);
        acc[c].re += h * w[0][c].re; acc[c].im += h * w[0][c].im;
        acc[3 + c].re += h * w[1][c].re; acc[3 + c].im += h * w[1][c].im;
        if (!BACK) { l0 = cneg(l0); l1 = cneg(l1); }      // lower = -g^+ a (fwd), +g^+ b (bwd)
        acc[6 + c].re += h * l0.re; acc[6 + c].im += h * l0.im;
        acc[9 + c].re += h * l1.re; acc[9 + c].im += h * l1.im;
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_wilson_clover(const cpx<R>* __restrict__ U,
                                                       const R* __restrict__ clov,
                                                       const int* __restrict__ nbr,
                                                       const cpx<R>* __restrict__ in,
                                                       cpx<R>* __restrict__ out, int64_t V, R diag,
                                                       int use_clover) {
    const int64_t site = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (site >= V) return;
    cpx<R> acc[12];
    cpx<R> p[12];
    load_spinor(p, in + site * 12);
#pragma unroll
    for (int f = 0; f < 12; ++f) acc[f] = {diag * p[f].re, diag * p[f].im};
    if (use_clover) {
#pragma unroll
        for (int chi = 0; chi < 2; ++chi) {
            const R* A = clov + (int64_t)chi * 36 * V + site;
            R d[6];
            cpx<R> o[15];
#pragma unroll
            for (int i = 0; i < 6; ++i) d[i] = A[i * V];
#pragma unroll
            for (int k = 0; k < 15; ++k) o[k] = {A[(6 + 2 * k) * V], A[(7 + 2 * k) * V]};
            const cpx<R>* x = p + 6 * chi;
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                cpx<R> t = {d[i] * x[i].re, d[i] * x[i].im};
                int k = 0;
#pragma unroll
                for (int r = 0; r < 6; ++r)
#pragma unroll
                    for (int c = r + 1; c < 6; ++c, ++k) {
                        if (r == i) t = cadd(t, cmul(o[k], x[c]));
                        if (c == i) t = cadd(t, cmulc(o[k], x[r]));
                    }
                acc[6 * chi + i] = cadd(acc[6 * chi + i], t);
            }
        }
    }
    const int* nb = nbr + site * 8;
    hop<0, false>(acc, in, U, V, site, nb[0]);
    hop<0, true>(acc, in, U, V, site, nb[1]);
    hop<1, false>(acc, in, U, V, site, nb[2]);
    hop<1, true>(acc, in, U, V, site, nb[3]);
    hop<2, false>(acc, in, U, V, site, nb[4]);
    hop<2, true>(acc, in, U, V, site, nb[5]);
    hop<3, false>(acc, in, U, V, site, nb[6]);
    hop<3, true>(acc, in, U, V, site, nb[7]);
    store_spinor(out + site * 12, acc);
}

// ------------------------------------------------------------ clover build
struct SigmaBlocks {
    // i c_sw/2 * sigma_{mu nu} restricted to chirality chi: [plane][chi][2][2] (re, im)
    double v[6][2][2][2][2];
};

__device__ __forceinline__ void m3mul(cpx<double> o[9], const cpx<double> a[9], const cpx<double> b[9]) {
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            cpx<double> t = {0, 0};
            for (int k = 0; k < 3; ++k) t = cadd(t, cmul(a[r * 3 + k], b[k * 3 + c]));
            o[r * 3 + c] = t;
        }
}
__device__ __forceinline__ void m3dag(cpx<double> o[9], const cpx<double> a[9]) {
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) o[r * 3 + c] = {a[c * 3 + r].re, -a[c * 3 + r].im};
}
__device__ __forceinline__ void m3load(cpx<double> o[9], const double2* G, int mu, int64_t x, int64_t V) {
    const double2* p = G + ((int64_t)mu * V + x) * 9;
    for (int e = 0; e < 9; ++e) o[e] = {p[e].x, p[e].y};
}

// Product of four links, each optionally daggered.
__device__ void leaf(cpx<double> out[9], const double2* G, int64_t V, const int m[4], const int64_t x[4],
                     const bool dag[4]) {
    cpx<double> a[9], b[9], t[9], acc[9];
    m3load(a, G, m[0], x[0], V);
    if (dag[0]) { m3dag(t, a); for (int e = 0; e < 9; ++e) a[e] = t[e]; }
    for (int e = 0; e < 9; ++e) acc[e] = a[e];
    for (int l = 1; l < 4; ++l) {
        m3load(b, G, m[l], x[l], V);
        if (dag[l]) { m3dag(t, b); for (int e = 0; e < 9; ++e) b[e] = t[e]; }
        m3mul(t, acc, b);
        for (int e = 0; e < 9; ++e) acc[e] = t[e];
    }
    for (int e = 0; e < 9; ++e) out[e] = acc[e];
}

template <typename R>
__global__ void k_clover_build(R* __restrict__ clov, const double2* __restrict__ G,
                               const int* __restrict__ nbr, int64_t V, SigmaBlocks sb) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= V) return;
    cpx<double> A[2][6][6];
    for (int chi = 0; chi < 2; ++chi)
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) A[chi][i][j] = {0, 0};
    int plane = 0;
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = mu + 1; nu < 4; ++nu, ++plane) {
            auto N = [&](int64_t s, int d) -> int64_t { return nbr[s * 8 + d]; };
            const int64_t xpm = N(x, 2 * mu), xpn = N(x, 2 * nu), xmm = N(x, 2 * mu + 1), xmn = N(x, 2 * nu + 1);
            const int64_t xmm_pn = N(xmm, 2 * nu), xmm_mn = N(xmm, 2 * nu + 1), xpm_mn = N(xpm, 2 * nu + 1);
            cpx<double> Q[9], L[9];
            for (int e = 0; e < 9; ++e) Q[e] = {0, 0};
            {   // x -> x+mu -> x+mu+nu -> x+nu -> x
                const int m[4] = {mu, nu, mu, nu}; const int64_t s[4] = {x, xpm, xpn, x};
                const bool d[4] = {false, false, true, true};
                leaf(L, G, V, m, s, d); for (int e = 0; e < 9; ++e) Q[e] = cadd(Q[e], L[e]);
            }
            {   // x -> x+nu -> x-mu+nu -> x-mu -> x
                const int m[4] = {nu, mu, nu, mu}; const int64_t s[4] = {x, xmm_pn, xmm, xmm};
                const bool d[4] = {false, true, true, false};
                leaf(L, G, V, m, s, d); for (int e = 0; e < 9; ++e) Q[e] = cadd(Q[e], L[e]);
            }
            {   // x -> x-mu -> x-mu-nu -> x-nu -> x
                const int m[4] = {mu, nu, mu, nu}; const int64_t s[4] = {xmm, xmm_mn, xmm_mn, xmn};
                const bool d[4] = {true, true, false, false};
                leaf(L, G, V, m, s, d); for (int e = 0; e < 9; ++e) Q[e] = cadd(Q[e], L[e]);
            }
            {   // x -> x-nu -> x+mu-nu -> x+mu -> x
                const int m[4] = {nu, mu, nu, mu}; const int64_t s[4] = {xmn, xmn, xpm_mn, x};
                const bool d[4] = {true, false, false, true};
                leaf(L, G, V, m, s, d); for (int e = 0; e < 9; ++e) Q[e] = cadd(Q[e], L[e]);
            }
            cpx<double> F[9];
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c)
                    F[r * 3 + c] = {(Q[r * 3 + c].re - Q[c * 3 + r].re) / 8.0,
                                    (Q[r * 3 + c].im + Q[c * 3 + r].im) / 8.0};
            for (int chi = 0; chi < 2; ++chi)
                for (int s = 0; s < 2; ++s)
                    for (int t = 0; t < 2; ++t) {
                        const cpx<double> w = {sb.v[plane][chi][s][t][0], sb.v[plane][chi][s][t][1]};
                        for (int a = 0; a < 3; ++a)
                            for (int b = 0; b < 3; ++b)
                                A[chi][s * 3 + a][t * 3 + b] = cadd(A[chi][s * 3 + a][t * 3 + b], cmul(w, F[a * 3 + b]));
                    }
        }
    for (int chi = 0; chi < 2; ++chi) {
        R* o = clov + (int64_t)chi * 36 * V + x;
        for (int i = 0; i < 6; ++i) o[i * V] = (R)A[chi][i][i].re;
        int k = 0;
        for (int r = 0; r < 6; ++r)
            for (int c = r + 1; c < 6; ++c, ++k) {
                o[(6 + 2 * k) * V] = (R)A[chi][r][c].re;
                o[(7 + 2 * k) * V] = (R)A[chi][r][c].im;
            }
    }
}

template <typename R>
__global__ void k_clover_export(double2* __restrict__ out, const R* __restrict__ clov, int64_t V) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= V) return;
    double2* o = out + x * 144;
    for (int e = 0; e < 144; ++e) o[e] = make_double2(0, 0);
    for (int chi = 0; chi < 2; ++chi) {
        const R* A = clov + (int64_t)chi * 36 * V + x;
        for (int i = 0; i < 6; ++i) o[(6 * chi + i) * 12 + 6 * chi + i] = make_double2(A[i * V], 0);
        int k = 0;
        for (int r = 0; r < 6; ++r)
            for (int c = r + 1; c < 6; ++c, ++k) {
                const double re = A[(6 + 2 * k) * V], im = A[(7 + 2 * k) * V];
                o[(6 * chi + r) * 12 + 6 * chi + c] = make_double2(re, im);
                o[(6 * chi + c) * 12 + 6 * chi + r] = make_double2(re, -im);
            }
    }
}

// Canonical gauge [4][V][3][3] complex128 -> SoA [4][9][V] in R, time sign folded.
template <typename R>
__global__ void k_pack_gauge(cpx<R>* __restrict__ U, const double2* __restrict__ G, int64_t V,
                             int64_t last_slice_start, int anti) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= 4 * 9 * V) return;
    const int64_t site = g % V;
    const int e = (int)((g / V) % 9);
    const int mu = (int)(g / (9 * V));
    const double2 v = G[((int64_t)mu * V + site) * 9 + e];
    const double sgn = (anti && mu == 3 && site >= last_slice_start) ? -1.0 : 1.0;
    U[g] = cpx<R>{(R)(sgn * v.x), (R)(sgn * v.y)};
}

// sigma_{mu nu} chirality blocks, from the chiral-basis gamma matrices.
static SigmaBlocks sigma_blocks(double csw) {
    double g[4][4][4][2];
    for (int mu = 0; mu < 4; ++mu) gamma_matrix(mu, g[mu]);
    auto mm = [&](const double (*a)[4][2], const double (*b)[4][2], double (*o)[4][2]) {
        for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c) {
                double re = 0, im = 0;
                for (int k = 0; k < 4; ++k) {
                    re += a[r][k][0] * b[k][c][0] - a[r][k][1] * b[k][c][1];
                    im += a[r][k][0] * b[k][c][1] + a[r][k][1] * b[k][c][0];
                }
                o[r][c][0] = re;
                o[r][c][1] = im;
            }
    };
    SigmaBlocks sb{};
    int plane = 0;
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = mu + 1; nu < 4; ++nu, ++plane) {
            double ab[4][4][2], ba[4][4][2];
            mm(g[mu], g[nu], ab);
            mm(g[nu], g[mu], ba);
            for (int chi = 0; chi < 2; ++chi)
                for (int s = 0; s < 2; ++s)
                    for (int t = 0; t < 2; ++t) {
                        const int r = 2 * chi + s, c = 2 * chi + t;
                        // sigma = (i/2)(ab - ba); coefficient i c_sw / 2  =>  w = -(c_sw/4)(ab - ba)
                        const double dre = ab[r][c][0] - ba[r][c][0], dim = ab[r][c][1] - ba[r][c][1];
                        sb.v[plane][chi][s][t][0] = -0.25 * csw * dre;
                        sb.v[plane][chi][s][t][1] = -0.25 * csw * dim;
                    }
        }
    return sb;
}

template <typename R>
static qmg_status launch_wilson(const qmg_fine_op_s* op, const void* in, void* out, hipStream_t s) {
    const unsigned nb = (unsigned)((op->V + 255) / 256);
    hipLaunchKernelGGL(k_wilson_clover<R>, dim3(nb), dim3(256), 0, s, (const cpx<R>*)op->U,
                       (const R*)op->clov, op->nbr, (const cpx<R>*)in, (cpx<R>*)out, op->V,
                       (R)(4.0 + op->m0), op->csw != 0.0 ? 1 : 0);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

static size_t real_bytes(qmg_prec p) { return p == QMG_C128 ? 8 : 4; }

void gamma_matrix(int mu, double g[4][4][2]) {
    // off-diagonal block g_mu (upper right); the lower-left block is g_mu^+
    static const double G[4][2][2][2] = {
        {{{0, 0}, {0, -1}}, {{0, -1}, {0, 0}}},   // -i sigma_1
        {{{0, 0}, {-1, 0}}, {{1, 0}, {0, 0}}},    // -i sigma_2
        {{{0, -1}, {0, 0}}, {{0, 0}, {0, 1}}},    // -i sigma_3
        {{{1, 0}, {0, 0}}, {{0, 0}, {1, 0}}}};    // 1
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) g[r][c][0] = g[r][c][1] = 0;
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) {
            g[r][2 + c][0] = G[mu][r][c][0];
            g[r][2 + c][1] = G[mu][r][c][1];
            g[2 + c][r][0] = G[mu][r][c][0];     // (g^+)_{c r} = conj(g_{r c})
            g[2 + c][r][1] = -G[mu][r][c][1];
        }
}

}  // namespace qmg

using namespace qmg;

extern "C" void qmg_fine_op_destroy(qmg_fine_op op) {
    if (!op) return;
    if (op->U) (void)hipFree(op->U);
    if (op->clov) (void)hipFree(op->clov);
    if (op->nbr) (void)hipFree(op->nbr);
    delete op;
}

extern "C" qmg_status qmg_fine_op_create(const int dims[4], const void* gauge, double m0, double csw,
                                         int antiperiodic_t, qmg_prec storage, void* stream,
                                         qmg_fine_op* out) {
    if (!out) return fail(QMG_ERR_ARG, "fine_op_create: out is NULL");
    *out = nullptr;
    QMG_TRY(check_dims(dims, 2, "fine_op_create"));
    if (!gauge) return fail(QMG_ERR_ARG, "fine_op_create: gauge is NULL");
    if (storage != QMG_C128 && storage != QMG_C64)
        return fail(QMG_ERR_PREC, "fine_op_create: storage %d not supported", (int)storage);
    hipStream_t s = as_stream(stream);
    auto* op = new qmg_fine_op_s();
    for (int m = 0; m < 4; ++m) op->dims[m] = dims[m];
    op->V = volume(dims);
    op->m0 = m0;
    op->csw = csw;
    op->antiperiodic_t = antiperiodic_t ? 1 : 0;
    op->storage = storage;
    const size_t rb = real_bytes(storage);
    hipError_t e = hipMalloc(&op->U, 2 * rb * 36 * op->V);
    if (e == hipSuccess) e = hipMalloc(&op->clov, rb * 72 * op->V);
    if (e != hipSuccess) {
        qmg_fine_op_destroy(op);
        return fail(QMG_ERR_NOMEM, "fine_op_create: %s", hipGetErrorString(e));
    }
    qmg_status st = make_neighbour_table(dims, &op->nbr, s);
    if (st != QMG_OK) {
        qmg_fine_op_destroy(op);
        return st;
    }
    const int64_t last = op->V - op->V / dims[3];
    const unsigned nbU = (unsigned)((36 * op->V + 255) / 256), nbS = (unsigned)((op->V + 127) / 128);
    const SigmaBlocks sb = sigma_blocks(csw);
    if (storage == QMG_C128) {
        hipLaunchKernelGGL(k_pack_gauge<double>, dim3(nbU), dim3(256), 0, s, (cpx<double>*)op->U,
                           (const double2*)gauge, op->V, last, op->antiperiodic_t);
        hipLaunchKernelGGL(k_clover_build<double>, dim3(nbS), dim3(128), 0, s, (double*)op->clov,
                           (const double2*)gauge, op->nbr, op->V, sb);
    } else {
        hipLaunchKernelGGL(k_pack_gauge<float>, dim3(nbU), dim3(256), 0, s, (cpx<float>*)op->U,
                           (const double2*)gauge, op->V, last, op->antiperiodic_t);
        hipLaunchKernelGGL(k_clover_build<float>, dim3(nbS), dim3(128), 0, s, (float*)op->clov,
                           (const double2*)gauge, op->nbr, op->V, sb);
    }
    e = hipGetLastError();
    if (e != hipSuccess) {
        qmg_fine_op_destroy(op);
        return fail(QMG_ERR_HIP, "fine_op_create: launch: %s", hipGetErrorString(e));
    }
    *out = op;
    return QMG_OK;
}

extern "C" qmg_status qmg_fine_op_export_clover(qmg_fine_op op, void* A, void* stream) {
    if (!op || !A) return fail(QMG_ERR_ARG, "fine_op_export_clover: NULL argument");
    hipStream_t s = as_stream(stream);
    const unsigned nb = (unsigned)((op->V + 127) / 128);
    if (op->storage == QMG_C128)
        hipLaunchKernelGGL(k_clover_export<double>, dim3(nb), dim3(128), 0, s, (double2*)A,
                           (const double*)op->clov, op->V);
    else
        hipLaunchKernelGGL(k_clover_export<float>, dim3(nb), dim3(128), 0, s, (double2*)A,
                           (const float*)op->clov, op->V);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

extern "C" qmg_status qmg_wilson_clover_dslash(qmg_fine_op op, const void* in, void* out, qmg_prec prec,
                                               void* stream) {
    if (!op || !in || !out) return fail(QMG_ERR_ARG, "wilson_clover_dslash: NULL argument");
    if (prec != op->storage)
        return fail(QMG_ERR_PREC, "wilson_clover_dslash: vector precision %d != operator storage %d",
                    (int)prec, (int)op->storage);
    if (in == out) return fail(QMG_ERR_ARG, "wilson_clover_dslash: in and out alias");
    hipStream_t s = as_stream(stream);
    if (op->storage == QMG_C128) return launch_wilson<double>(op, in, out, s);
    return launch_wilson<float>(op, in, out, s);
}
