// Schwarz alternating procedure (SAP) smoother for the fine Wilson-clover
// operator of Eq. (2): the domain-decomposition smoother that relaxes each
// block of the lattice on its own, with no global reduction (the paper names
// Schwarz-preconditioned smoothers as the way to cut the smoother's global
// communication; its coarse levels are latency-bound, Sec. 7.2).
//
// The lattice is cut into blocks of extent b (an even number of at least two
// blocks per dimension) coloured by the parity of their block coordinates, so
// blocks sharing a face have opposite colours.  One sweep from x = 0 for A x = r:
//   for colour c = 0, 1, every block B of colour c at once:
//       r_B = (r - A x) on B;  `iters` MR steps on A_BB d = r_B from d = 0
//       (A_BB: Eq. (2) restricted to B, the hops leaving B dropped; each block
//       its own step lengths);  x += d on B.
// One launch per colour: a work-group owns a block, one thread per site.  The
// block's forward links (decoded to FP32) and the running residual sit in
// LDS, the site's clover block in registers, so the MR steps touch no global
// memory; the block sums are fixed-order work-group reductions in FP64.  The
// colour-1 launch first subtracts from r the hops of the colour-0 result that
// enter its blocks.
#include "wilson_dev.h"

#include <vector>

namespace qmg {

namespace {

struct SapGeom {
    int L[4];      // lattice extents
    int b[4];      // block extents
    int nb[4];     // blocks per dimension
};

__device__ __forceinline__ void herm_mul(cpx<float> out[12], const cpx<float> x[12], const float d[2][6],
                                         const cpx<float> o[2][15], float diag) {
#pragma unroll
    for (int chi = 0; chi < 2; ++chi) {
        const cpx<float>* v = x + 6 * chi;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            cpx<float> t = {(diag + d[chi][i]) * v[i].re, (diag + d[chi][i]) * v[i].im};
            int k = 0;
#pragma unroll
            for (int r = 0; r < 6; ++r)
#pragma unroll
                for (int c = r + 1; c < 6; ++c, ++k) {
                    if (r == i) t = cadd(t, cmul(o[chi][k], v[c]));
                    if (c == i) t = cadd(t, cmulc(o[chi][k], v[r]));
                }
            out[6 * chi + i] = t;
        }
    }
}

// fixed-order work-group sum of three doubles (every thread gets the totals)
__device__ __forceinline__ void wg_sum3(double v[3], double* red) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
        for (int o = 32; o > 0; o >>= 1) v[i] += __shfl_down(v[i], o, 64);
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int i = 0; i < 3; ++i) red[i * 16 + w] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double s = 0;
        for (int k = 0; k < nw; ++k) s += red[i * 16 + k];
        v[i] = s;
    }
}

template <int LF, int LR>
__global__ __launch_bounds__(256) void k_sap_colour(const void* __restrict__ U, const void* __restrict__ clov,
                                                     const float* __restrict__ cscale, const int* __restrict__ nbr,
                                                     const int* __restrict__ blocks, SapGeom G,
                                                     const float2* __restrict__ rin, float2* __restrict__ x,
                                                     int colour, int iters, int64_t V, float diag, int use_clover,
                                                     int64_t last) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int Sb = G.b[0] * G.b[1] * G.b[2] * G.b[3];
    cpx<float>* lk = reinterpret_cast<cpx<float>*>(smem);                 // [4][9][Sb] forward links
    cpx<float>* sr = lk + 36 * Sb;                                         // [12][Sb] residual
    double* red = reinterpret_cast<double*>(sr + 12 * Sb);                 // [3][16] (at most 4 waves used)
    const int t = threadIdx.x;
    // block and site coordinates
    int bc[4], l[4], g[4];
    {
        int q = blocks[blockIdx.x];
#pragma unroll
        for (int m = 0; m < 4; ++m) { bc[m] = q % G.nb[m]; q /= G.nb[m]; }
        int u = t;
#pragma unroll
        for (int m = 0; m < 4; ++m) { l[m] = u % G.b[m]; u /= G.b[m]; }
#pragma unroll
        for (int m = 0; m < 4; ++m) g[m] = bc[m] * G.b[m] + l[m];
    }
    const int64_t site = g[0] + (int64_t)G.L[0] * (g[1] + (int64_t)G.L[1] * (g[2] + (int64_t)G.L[2] * g[3]));
    const int64_t vo = (int64_t)blockIdx.y * V;
    int stride[4];
    stride[0] = 1;
    stride[1] = G.b[0];
    stride[2] = G.b[0] * G.b[1];
    stride[3] = G.b[0] * G.b[1] * G.b[2];
    // the site's forward links to LDS (decoded, time sign included)
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        cpx<float> u[9];
        load_link<LF, LR>(u, U, mu, site, V, last);
#pragma unroll
        for (int e = 0; e < 9; ++e) lk[(mu * 9 + e) * Sb + t] = u[e];
    }
    // the site's clover block in registers
    float cd[2][6];
    cpx<float> co[2][15];
#pragma unroll
    for (int chi = 0; chi < 2; ++chi) {
        if (use_clover) {
            load_clover<LF>(cd[chi], co[chi], clov, cscale, chi, site, V);
        } else {
#pragma unroll
            for (int i = 0; i < 6; ++i) cd[chi][i] = 0.f;
#pragma unroll
            for (int i = 0; i < 15; ++i) co[chi][i] = {0.f, 0.f};
        }
    }
    // residual on the block: r, minus (for colour 1) the hops of the colour-0
    // result x that enter the block from outside
    cpx<float> r[12];
#pragma unroll
    for (int f = 0; f < 12; ++f) {
        const float2 v = rin[(site + vo) * 12 + f];
        r[f] = {v.x, v.y};
    }
    const int* nb = nbr + site * 8;
    if (colour == 1) {
        cpx<float> p[12], u[9];
#define QMG_SAP_OUT(MU, BACK, D)                                                                    \
        if (BACK ? l[MU] == 0 : l[MU] == G.b[MU] - 1) {                                             \
            load_spinor<FMT_F32>(p, x, nullptr, (int64_t)nb[D] + vo);                               \
            load_link<LF, LR>(u, U, MU, BACK ? (int64_t)nb[D] : site, V, last);                     \
            hop_apply<MU, BACK>(r, p, u, 0.5f);                                                     \
        }
        QMG_SAP_OUT(0, false, 0) QMG_SAP_OUT(0, true, 1) QMG_SAP_OUT(1, false, 2) QMG_SAP_OUT(1, true, 3)
        QMG_SAP_OUT(2, false, 4) QMG_SAP_OUT(2, true, 5) QMG_SAP_OUT(3, false, 6) QMG_SAP_OUT(3, true, 7)
#undef QMG_SAP_OUT
    }
#pragma unroll
    for (int f = 0; f < 12; ++f) sr[f * Sb + t] = r[f];
    cpx<float> d[12];
#pragma unroll
    for (int f = 0; f < 12; ++f) d[f] = {0.f, 0.f};
    __syncthreads();
    for (int it = 0; it < iters; ++it) {
        // Ar = A_BB r at this site
        cpx<float> Ar[12];
        herm_mul(Ar, r, cd, co, diag);
        cpx<float> p[12], u[9];
#define QMG_SAP_IN(MU, BACK)                                                                        \
        if (BACK ? l[MU] > 0 : l[MU] < G.b[MU] - 1) {                                               \
            const int nl = BACK ? t - stride[MU] : t + stride[MU];                                  \
            _Pragma("unroll") for (int f = 0; f < 12; ++f) p[f] = sr[f * Sb + nl];                  \
            const int ls = BACK ? nl : t;                                                           \
            _Pragma("unroll") for (int e = 0; e < 9; ++e) u[e] = lk[(MU * 9 + e) * Sb + ls];        \
            hop_apply<MU, BACK>(Ar, p, u, -0.5f);                                                   \
        }
        QMG_SAP_IN(0, false) QMG_SAP_IN(0, true) QMG_SAP_IN(1, false) QMG_SAP_IN(1, true)
        QMG_SAP_IN(2, false) QMG_SAP_IN(2, true) QMG_SAP_IN(3, false) QMG_SAP_IN(3, true)
#undef QMG_SAP_IN
        double s3[3] = {0, 0, 0};
#pragma unroll
        for (int f = 0; f < 12; ++f) {
            s3[0] += (double)Ar[f].re * Ar[f].re + (double)Ar[f].im * Ar[f].im;
            s3[1] += (double)Ar[f].re * r[f].re + (double)Ar[f].im * r[f].im;
            s3[2] += (double)Ar[f].re * r[f].im - (double)Ar[f].im * r[f].re;
        }
        wg_sum3(s3, red);   // also the barrier after every thread has read its neighbours
        const float ar = s3[0] > 0 ? (float)(s3[1] / s3[0]) : 0.f, ai = s3[0] > 0 ? (float)(s3[2] / s3[0]) : 0.f;
#pragma unroll
        for (int f = 0; f < 12; ++f) {
            d[f].re += ar * r[f].re - ai * r[f].im;
            d[f].im += ar * r[f].im + ai * r[f].re;
            r[f].re -= ar * Ar[f].re - ai * Ar[f].im;
            r[f].im -= ar * Ar[f].im + ai * Ar[f].re;
        }
#pragma unroll
        for (int f = 0; f < 12; ++f) sr[f * Sb + t] = r[f];
        __syncthreads();
    }
#pragma unroll
    for (int f = 0; f < 12; ++f) x[(site + vo) * 12 + f] = make_float2(d[f].re, d[f].im);
}

}  // namespace

// Host side: the block tables of a (lattice, block) pair, cached per operator call.
struct SapPlan {
    SapGeom G;
    int nblk = 0;
    int* blocks = nullptr;   // device [2][nblk/2]: block ids of colour 0, then colour 1
};

static qmg_status sap_plan(const qmg_fine_op_s* op, const int block[4], SapPlan* P, hipStream_t s) {
    int n = 1;
    for (int m = 0; m < 4; ++m) {
        if (block[m] < 1 || op->dims[m] % block[m]) return fail(QMG_ERR_SHAPE, "sap: block does not divide the lattice");
        const int k = op->dims[m] / block[m];
        if (k < 2 || k % 2) return fail(QMG_ERR_SHAPE, "sap: need an even number (>= 2) of blocks per dimension");
        P->G.L[m] = op->dims[m];
        P->G.b[m] = block[m];
        P->G.nb[m] = k;
        n *= k;
    }
    const int Sb = block[0] * block[1] * block[2] * block[3];
    if (Sb > 256) return fail(QMG_ERR_SHAPE, "sap: %d sites per block (at most 256)", Sb);
    std::vector<int> h;
    for (int c = 0; c < 2; ++c)
        for (int q = 0; q < n; ++q) {
            int r = q, par = 0;
            for (int m = 0; m < 4; ++m) { par += r % P->G.nb[m]; r /= P->G.nb[m]; }
            if (par % 2 == c) h.push_back(q);
        }
    P->nblk = n;
    QMG_HIP(hipMalloc(&P->blocks, sizeof(int) * n));
    hipError_t e = hipMemcpyAsync(P->blocks, h.data(), sizeof(int) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(P->blocks);
        P->blocks = nullptr;
        return fail(QMG_ERR_HIP, "sap: block table upload: %s", hipGetErrorString(e));
    }
    return QMG_OK;
}

template <int LF, int LR>
static qmg_status launch_sap(const qmg_fine_op_s* op, const SapPlan& P, const void* r, void* x, int iters, int m,
                             hipStream_t s) {
    const int Sb = P.G.b[0] * P.G.b[1] * P.G.b[2] * P.G.b[3];
    const size_t lds = sizeof(cpx<float>) * 48 * (size_t)Sb + sizeof(double) * 48;
    auto kern = k_sap_colour<LF, LR>;
    if (lds > 65536) QMG_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const dim3 grid((unsigned)(P.nblk / 2), (unsigned)m), block((unsigned)Sb);
    for (int c = 0; c < 2; ++c) {
        hipLaunchKernelGGL(kern, grid, block, lds, s, op->U, op->clov, op->cscale, op->nbr, P.blocks + c * (P.nblk / 2),
                           P.G, (const float2*)r, (float2*)x, c, iters, op->V, (float)(4.0 + op->m0),
                           op->csw != 0.0 ? 1 : 0, op->last);
        QMG_LAUNCH_CHECK();
    }
    return QMG_OK;
}

// x = one SAP sweep for A x = r (complex64 fields of m members).
qmg_status sap_sweep(const qmg_fine_op_s* op, const SapPlan& P, const void* r, void* x, int iters, int m,
                     hipStream_t s) {
    const bool c12 = op->link_reals == 12;
    switch (op->storage) {
        case QMG_C64: return c12 ? launch_sap<FMT_F32, 12>(op, P, r, x, iters, m, s) : launch_sap<FMT_F32, 18>(op, P, r, x, iters, m, s);
        case QMG_H16: return c12 ? launch_sap<FMT_H16, 12>(op, P, r, x, iters, m, s) : launch_sap<FMT_H16, 18>(op, P, r, x, iters, m, s);
        case QMG_B16: return c12 ? launch_sap<FMT_B16, 12>(op, P, r, x, iters, m, s) : launch_sap<FMT_B16, 18>(op, P, r, x, iters, m, s);
        default: return fail(QMG_ERR_PREC, "sap: the operator must use complex64 or 16-bit storage (FP32 arithmetic)");
    }
}

qmg_status sap_plan_create(const qmg_fine_op_s* op, const int block[4], SapPlan** out, hipStream_t s) {
    auto* P = new SapPlan();
    const qmg_status st = sap_plan(op, block, P, s);
    if (st != QMG_OK) {
        delete P;
        return st;
    }
    *out = P;
    return QMG_OK;
}

void sap_plan_destroy(SapPlan* P) {
    if (!P) return;
    if (P->blocks) (void)hipFree(P->blocks);
    delete P;
}

}  // namespace qmg

using namespace qmg;

extern "C" qmg_status qmg_wilson_clover_sap(qmg_fine_op op, const int block[4], int iters, const void* r, void* x,
                                            int nrhs, void* stream) {
    if (!op || !block || !r || !x) return fail(QMG_ERR_ARG, "wilson_clover_sap: NULL argument");
    if (r == x) return fail(QMG_ERR_ARG, "wilson_clover_sap: r and x alias");
    if (iters < 1 || iters > 64) return fail(QMG_ERR_ARG, "wilson_clover_sap: iters %d outside [1, 64]", iters);
    if (nrhs < 1 || nrhs > kMaxFieldBatch) return fail(QMG_ERR_ARG, "wilson_clover_sap: nrhs %d", nrhs);
    if (op->storage == QMG_C128) return fail(QMG_ERR_PREC, "wilson_clover_sap: needs complex64 or 16-bit storage");
    hipStream_t s = as_stream(stream);
    SapPlan* P = nullptr;
    QMG_TRY(sap_plan_create(op, block, &P, s));
    const qmg_status st = sap_sweep(op, *P, r, x, iters, nrhs, s);
    (void)hipStreamSynchronize(s);
    sap_plan_destroy(P);
    return st;
}
