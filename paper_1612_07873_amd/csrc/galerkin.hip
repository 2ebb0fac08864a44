// Galerkin coarse operator Mhat = P^+ M P (Sec. 3.4 step 4), keeping the
// nearest-neighbour form of Eq. (3) at every level (the recursion of Sec. 3.4).
//
// With Pf(x) the dof x N slice of P at fine site x (nonzero only where the
// chirality of the row matches that of the column), D(x) the on-site block
// and H_d(x) the hop block of the parent towards x' = x + hop_d:
//   Y_d(xc) = sum over x in xc with x' outside xc of Pf(x)^+ H_d(x) Pf(x')
//   X(xc)   = sum over x in xc of Pf(x)^+ D(x) Pf(x)
//           + sum over hops x -> x' that stay inside xc of Pf(x)^+ H_d(x) Pf(x').
// The parent is the fine Wilson-clover operator (D = 4 + m0 + A, H_d from the
// spin projectors and links) or a coarse operator (D = X, H_d = Y_d).
//
// Work decomposition: one work-group per (coarse site, term), 17 terms: the
// eight Y_d, and X split into its eight inside-hop sums and the on-site sum
// (written to separate slots and added in a fixed order afterwards, so the
// build is deterministic and needs no atomics).  For every contributing fine
// site the work-group first forms the parent's block H (dof x dof) in LDS,
// then W = H Pf(x') in LDS, then each thread adds Pf(x)^+ W to the N x N
// entries it owns.  All arithmetic is FP64.  This is setup work, done once
// per hierarchy.
#include "handles.h"

#include <vector>

namespace qmg {

constexpr int GAL_MAXE = 16;  // output entries per thread

struct Proj {  // spin matrices (1 - gamma_mu) [fwd] and (1 + gamma_mu) [bwd], 4x4 complex
    double p[8][4][4][2];
};

template <typename R>
__device__ __forceinline__ cpx<double> fine_link(const cpx<R>* U, int mu, int e, int64_t x, int64_t V) {
    const cpx<R> u = U[((int64_t)mu * 9 + e) * V + x];
    return {(double)u.re, (double)u.im};
}

// H[f][g] of the fine parent for term (d or diag) at fine site x.
template <typename R>
__device__ cpx<double> fine_H(const qmg_fine_op_s& op, const cpx<R>* U, const R* clov, const Proj& P,
                              int term, int64_t x, int64_t xn, int f, int g) {
    const int s = f / 3, a = f % 3, t = g / 3, b = g % 3;
    if (term == 8) {  // 4 + m0 + A(x)
        cpx<double> v = {f == g ? 4.0 + op.m0 : 0.0, 0.0};
        if (op.csw != 0.0 && (s / 2) == (t / 2)) {
            const int chi = s / 2, i = f - 6 * chi, j = g - 6 * chi;
            const R* A = clov + (int64_t)chi * 36 * op.V + x;
            if (i == j) v.re += (double)A[i * op.V];
            else {
                const int r = i < j ? i : j, c = i < j ? j : i;
                const int k = r * 6 - r * (r + 1) / 2 + (c - r - 1);
                const double re = (double)A[(6 + 2 * k) * op.V], im = (double)A[(7 + 2 * k) * op.V];
                v.re += re;
                v.im += i < j ? im : -im;
            }
        }
        return v;
    }
    const int mu = term / 2;
    const double pr = P.p[term][s][t][0], pi = P.p[term][s][t][1];
    if (pr == 0.0 && pi == 0.0) return {0.0, 0.0};
    cpx<double> u;
    if ((term & 1) == 0) u = fine_link(U, mu, a * 3 + b, x, op.V);  // U_mu(x)
    else {                                                        // U_mu(x - mu)^+
        const cpx<double> w = fine_link(U, mu, b * 3 + a, xn, op.V);
        u = {w.re, -w.im};
    }
    return {-0.5 * (pr * u.re - pi * u.im), -0.5 * (pr * u.im + pi * u.re)};
}

template <typename R>
__device__ __forceinline__ cpx<double> coarse_H(const qmg_coarse_op_s& op, const R* L, int term, int64_t x,
                                                int f, int g) {
    // element (row f, col g) of X (term 8) or Y_term in the chunked layout
    constexpr int cpc = sizeof(R) == 8 ? 1 : 2;
    const int blk = term == 8 ? 0 : term + 1;
    const int e = blk * op.N + g;
    const int j = e / cpc, q = e % cpc;
    const R* c = L + (((int64_t)x * op.J + j) * op.N + f) * 2 * cpc;
    return {(double)c[2 * q], (double)c[2 * q + 1]};
}

template <bool FINE, typename R, bool ST>
__global__ __launch_bounds__(1024) void k_galerkin(double2* __restrict__ Yout, double2* __restrict__ Xpart,
                                                   qmg_fine_op_s fop, qmg_coarse_op_s cop,
                                                   const void* __restrict__ parent_a,
                                                   const void* __restrict__ parent_b,
                                                   const int* __restrict__ nbr, const double2* __restrict__ B,
                                                   const int* __restrict__ members, const int* __restrict__ owner,
                                                   int64_t Vc, int dof, int nvec, int bsites, Proj P) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = 2 * nvec, half = dof / 2;
    cpx<double>* W = reinterpret_cast<cpx<double>*>(smem);  // [dof][N]
    // ST: the parent's block and the two basis blocks are staged in LDS
    cpx<double>* H = W + dof * N;                           // [dof][dof]
    cpx<double>* Px = H + dof * dof;                        // Pf(x) [dof][nvec]
    cpx<double>* Pn = Px + dof * nvec;                      // Pf(x') [dof][nvec]
    const int64_t xc = blockIdx.x / 17;
    const int term = (int)(blockIdx.x % 17);
    const bool isY = term < 8;
    const int hterm = isY ? term : term - 8;  // 0..7 hops, 8 = on-site
    const int T = blockDim.x;
    cpx<double> acc[GAL_MAXE];
#pragma unroll
    for (int i = 0; i < GAL_MAXE; ++i) acc[i] = {0.0, 0.0};

    for (int b = 0; b < bsites; ++b) {
        const int64_t x = members[xc * bsites + b];
        int64_t xn = x;
        if (hterm < 8) {
            xn = nbr[x * 8 + hterm];
            const bool inside = owner[xn] == xc;
            if (isY == inside) continue;  // Y wants hops leaving the aggregate, X the ones inside
        }
        // the parent's block H[f][g] for this (x, term), once (when it fits
        // in LDS; otherwise each element is formed where it is used)
        auto Hfg = [&](int f, int g) {
            return FINE ? fine_H<R>(fop, (const cpx<R>*)parent_a, (const R*)parent_b, P, hterm, x, xn, f, g)
                        : coarse_H<R>(cop, (const R*)parent_a, hterm, x, f, g);
        };
        __syncthreads();
        if constexpr (ST) {
            for (int e = threadIdx.x; e < dof * dof; e += T) H[e] = Hfg(e / dof, e % dof);
            for (int e = threadIdx.x; e < dof * nvec; e += T) {   // coalesced loads of both basis blocks
                const double2 a = B[x * dof * nvec + e], c = B[xn * dof * nvec + e];
                Px[e] = cpx<double>{a.x, a.y};
                Pn[e] = cpx<double>{c.x, c.y};
            }
            __syncthreads();
        }
        // W[f][m] = sum_{g in chi(m)} H[f][g] Pf(xn)[g][m'] ; Pf(xn)[g][m'] = B[xn][g][m']
        for (int e = threadIdx.x; e < dof * N; e += T) {
            const int f = e / N, m = e % N;
            const int chi = m / nvec, mp = m - chi * nvec;
            cpx<double> w = {0.0, 0.0};
            for (int gg = 0; gg < half; ++gg) {
                const int g = chi * half + gg;
                cpx<double> h, bv;
                if constexpr (ST) {
                    h = H[f * dof + g];
                    bv = Pn[g * nvec + mp];
                } else {
                    h = Hfg(f, g);
                    const double2 b2 = B[(xn * dof + g) * nvec + mp];
                    bv = cpx<double>{b2.x, b2.y};
                }
                cmac(w.re, w.im, h.re, h.im, bv.re, bv.im);
            }
            W[e] = w;
        }
        __syncthreads();
        // acc[n][m] += sum_{f in chi(n)} conj(Pf(x)[f][n']) W[f][m]
#pragma unroll
        for (int i = 0; i < GAL_MAXE; ++i) {
            const int e = threadIdx.x + i * T;
            if (e >= N * N) break;
            const int n = e / N, m = e % N;
            const int chi = n / nvec, np = n - chi * nvec;
            for (int ff = 0; ff < half; ++ff) {
                const int f = chi * half + ff;
                cpx<double> bv;
                if constexpr (ST) bv = Px[f * nvec + np];
                else {
                    const double2 b2 = B[(x * dof + f) * nvec + np];
                    bv = cpx<double>{b2.x, b2.y};
                }
                const cpx<double> w = W[f * N + m];
                cmac_conj(acc[i].re, acc[i].im, bv.re, bv.im, w.re, w.im);
            }
        }
    }
    double2* out = isY ? Yout + ((int64_t)term * Vc + xc) * N * N : Xpart + ((int64_t)hterm * Vc + xc) * N * N;
#pragma unroll
    for (int i = 0; i < GAL_MAXE; ++i) {
        const int e = threadIdx.x + i * T;
        if (e >= N * N) break;
        out[e] = make_double2(acc[i].re, acc[i].im);
    }
}

__global__ void k_sum_xparts(double2* __restrict__ X, const double2* __restrict__ Xpart, int64_t n) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    double re = 0, im = 0;
    for (int t = 0; t < 9; ++t) {  // hops 0..7, then the on-site term
        re += Xpart[t * n + g].x;
        im += Xpart[t * n + g].y;
    }
    X[g] = make_double2(re, im);
}

static Proj projectors() {
    Proj P{};
    for (int mu = 0; mu < 4; ++mu) {
        double g[4][4][2];
        gamma_matrix(mu, g);
        for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c) {
                const double id = r == c ? 1.0 : 0.0;
                P.p[2 * mu][r][c][0] = id - g[r][c][0];
                P.p[2 * mu][r][c][1] = -g[r][c][1];
                P.p[2 * mu + 1][r][c][0] = id + g[r][c][0];
                P.p[2 * mu + 1][r][c][1] = g[r][c][1];
            }
    }
    return P;
}

}  // namespace qmg

using namespace qmg;

extern "C" qmg_status qmg_build_coarse_op(qmg_transfer t, qmg_fine_op fine, qmg_coarse_op parent,
                                          qmg_prec storage, void* stream, qmg_coarse_op* out) {
    if (!out) return fail(QMG_ERR_ARG, "build_coarse_op: out is NULL");
    *out = nullptr;
    if (!t) return fail(QMG_ERR_ARG, "build_coarse_op: transfer is NULL");
    if ((fine == nullptr) == (parent == nullptr))
        return fail(QMG_ERR_ARG, "build_coarse_op: give exactly one of fine / parent");
    const int* pdims = fine ? fine->dims : parent->dims;
    const int pdof = fine ? 12 : parent->N;
    for (int m = 0; m < 4; ++m)
        if (pdims[m] != t->fdims[m])
            return fail(QMG_ERR_SHAPE, "build_coarse_op: transfer lattice does not match the parent");
    if (pdof != t->dof) return fail(QMG_ERR_SHAPE, "build_coarse_op: transfer dof %d != parent dof %d", t->dof, pdof);
    const int N = 2 * t->nvec;
    if (pdof * N > 4096)
        return fail(QMG_ERR_SHAPE, "build_coarse_op: parent dof x N = %d exceeds 4096", pdof * N);
    if (storage != QMG_C128 && storage != QMG_C64)
        return fail(QMG_ERR_PREC, "build_coarse_op: storage %d not supported", (int)storage);
    const qmg_prec from = fine ? fine->storage : parent->storage;
    if (from != QMG_C128 && from != QMG_C64)
        return fail(QMG_ERR_PREC, "build_coarse_op: the parent operator must use complex128 or complex64 storage");
    if (fine && fine->link_reals != 18)
        return fail(QMG_ERR_PREC, "build_coarse_op: the fine operator must store all 18 link reals");
    hipStream_t s = as_stream(stream);
    const int64_t Vc = t->Vc;
    const size_t blk = (size_t)Vc * N * N;
    double2 *Y = nullptr, *Xp = nullptr, *X = nullptr;
    hipError_t e = hipMalloc(&Y, sizeof(double2) * 8 * blk);
    if (e == hipSuccess) e = hipMalloc(&Xp, sizeof(double2) * 9 * blk);
    if (e == hipSuccess) e = hipMalloc(&X, sizeof(double2) * blk);
    auto cleanup = [&]() {
        if (Y) (void)hipFree(Y);
        if (Xp) (void)hipFree(Xp);
        if (X) (void)hipFree(X);
    };
    if (e != hipSuccess) {
        cleanup();
        return fail(QMG_ERR_NOMEM, "build_coarse_op: %s", hipGetErrorString(e));
    }
    int threads = 256;
    while ((int64_t)threads * GAL_MAXE < (int64_t)N * N) threads += 64;
    if (threads > 1024) {
        cleanup();
        return fail(QMG_ERR_SHAPE, "build_coarse_op: N=%d too large", N);
    }
    // W [pdof][N]; with the parent's block H [pdof][pdof] and the two basis
    // blocks [pdof][nvec] staged too when all of it fits in 64 KiB (the fine
    // parent: 21 KiB).  A larger staging area would cost more in occupancy
    // than it saves (measured on a 48 -> 64 coarse parent: 2.2 ms unstaged,
    // 2.75 ms with H staged).
    const size_t lds_st = sizeof(cpx<double>) * ((size_t)pdof * N + (size_t)pdof * pdof + 2 * (size_t)pdof * t->nvec);
    const bool st_lds = lds_st <= 65536;
    const size_t lds = st_lds ? lds_st : sizeof(cpx<double>) * (size_t)pdof * N;
    const dim3 grid((unsigned)(Vc * 17));
    const Proj P = projectors();
    qmg_fine_op_s fop{};
    qmg_coarse_op_s cop{};
#define QMG_GAL(FINE, R, ST, A, B_)                                                                            \
    hipLaunchKernelGGL((k_galerkin<FINE, R, ST>), grid, dim3(threads), lds, s, Y, Xp, fop, cop, A, B_,           \
                       FINE ? fine->nbr : parent->nbr, t->basis64, t->members, t->owner, Vc, pdof, t->nvec,     \
                       t->bsites, P)
    if (fine) {
        fop = *fine;
        const bool d = fine->storage == QMG_C128;
        if (st_lds) {
            if (d) QMG_GAL(true, double, true, fine->U, fine->clov);
            else QMG_GAL(true, float, true, fine->U, fine->clov);
        } else {
            if (d) QMG_GAL(true, double, false, fine->U, fine->clov);
            else QMG_GAL(true, float, false, fine->U, fine->clov);
        }
    } else {
        cop = *parent;
        const bool d = parent->storage == QMG_C128;
        if (st_lds) {
            if (d) QMG_GAL(false, double, true, parent->links, nullptr);
            else QMG_GAL(false, float, true, parent->links, nullptr);
        } else {
            if (d) QMG_GAL(false, double, false, parent->links, nullptr);
            else QMG_GAL(false, float, false, parent->links, nullptr);
        }
    }
#undef QMG_GAL
    hipLaunchKernelGGL(k_sum_xparts, dim3((unsigned)((blk + 255) / 256)), dim3(256), 0, s, X, Xp, (int64_t)blk);
    e = hipGetLastError();
    if (e != hipSuccess) {
        cleanup();
        return fail(QMG_ERR_HIP, "build_coarse_op: launch: %s", hipGetErrorString(e));
    }
    qmg_status st = qmg_coarse_op_create(t->cdims, N, X, Y, storage, stream, out);
    // the create call packs X, Y on the same stream; wait before freeing them
    e = hipStreamSynchronize(s);
    cleanup();
    if (st != QMG_OK) return st;
    if (e != hipSuccess) {
        qmg_coarse_op_destroy(*out);
        *out = nullptr;
        return fail(QMG_ERR_HIP, "build_coarse_op: %s", hipGetErrorString(e));
    }
    return QMG_OK;
}
