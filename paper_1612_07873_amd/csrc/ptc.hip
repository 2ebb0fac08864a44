// Learned smoother: gauge-equivariant parallel-transport convolution (PTC)
// network, two linear layers 1 -> C -> 1 channels, trained by Adam on
// (residual, error) pairs.  The paper's smoother is MR (Sec. 7.1); this
// network is the learned replacement, with MR as its fallback.
//
//   (T_0 h)(x) = h(x), (T_{+mu} h)(x) = U_mu(x) h(x+mu), (T_{-mu} h)(x) = U_mu(x-mu)^+ h(x-mu)
//   (boundary signs folded into the links as in the Wilson-clover operator);
//   layer: h'_a(x) = sum_b sum_p W[p][a][b] (T_p h_b)(x), W[p][a][b] a complex 4x4 spin matrix;
//   loss:  L = sum_i |N(r_i) - e_i|^2 / |e_i|^2;
//   backward: with D = dL/dy*, G[p][a][b] = 2 sum_{x,colour} D_a(x) (T_p h_b)(x)^+,
//             dL/dh_b* = sum_p T_p^+ (sum_a W[p][a][b]^+ D_a), T_{+mu}^+ = T_{-mu}.
// G is reported as dL/dRe W + i dL/dIm W; Adam updates real and imaginary parts.
// Paths p: 0 = identity, 1 + 2 mu = +mu, 2 + 2 mu = -mu.  Fields [C][V][4][3]
// complex64, weights [9][Cout][Cin][4][4] complex64.  Weight-gradient sums over
// the lattice are two-phase (per-block partials, then a fixed-order sum).
#include "handles.h"

#include <vector>



namespace qmg {

constexpr int kPtcThreads = 256;
constexpr int kPtcMaxBlocks = 512;

// (T_p h)(x) for one channel h [V][12], links with folded signs.
__device__ __forceinline__ void transport(float2 t[12], const float2* __restrict__ h, const float2* __restrict__ U,
                                          const int* __restrict__ nbr, int64_t V, int64_t x, int p) {
    if (p == 0) {
#pragma unroll
        for (int f = 0; f < 12; ++f) t[f] = h[x * 12 + f];
        return;
    }
    const int mu = (p - 1) >> 1;
    const bool back = ((p - 1) & 1) != 0;
    const int64_t n = nbr[x * 8 + 2 * mu + (back ? 1 : 0)];
    const int64_t ls = back ? n : x;
    float2 u[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = U[((int64_t)mu * 9 + e) * V + ls];
    float2 s[12];
#pragma unroll
    for (int f = 0; f < 12; ++f) s[f] = h[n * 12 + f];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float re = 0, im = 0;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const float2 w = back ? make_float2(u[b * 3 + a].x, -u[b * 3 + a].y) : u[a * 3 + b];
                const float2 v = s[sp * 3 + b];
                re += w.x * v.x - w.y * v.y;
                im += w.x * v.y + w.y * v.x;
            }
            t[sp * 3 + a] = make_float2(re, im);
        }
}

__device__ __forceinline__ int rev_path(int p) { return p == 0 ? 0 : (((p - 1) & 1) ? p - 1 : p + 1); }

// out_a = sum_b sum_p W[p][a][b] T_p h_b ; grid (sites, Cout)
__global__ void k_ptc_layer(float2* __restrict__ out, const float2* __restrict__ h, const float2* __restrict__ W,
                            const float2* __restrict__ U, const int* __restrict__ nbr, int64_t V, int cin, int cout) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int a = blockIdx.y;
    if (x >= V) return;
    float2 acc[12];
#pragma unroll
    for (int f = 0; f < 12; ++f) acc[f] = make_float2(0, 0);
    for (int b = 0; b < cin; ++b)
        for (int p = 0; p < 9; ++p) {
            float2 t[12];
            transport(t, h + (int64_t)b * V * 12, U, nbr, V, x, p);
            const float2* w = W + (((int64_t)p * cout + a) * cin + b) * 16;
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float re = acc[s * 3 + c].x, im = acc[s * 3 + c].y;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const float2 m = w[s * 4 + q], v = t[q * 3 + c];
                        re += m.x * v.x - m.y * v.y;
                        im += m.x * v.y + m.y * v.x;
                    }
                    acc[s * 3 + c] = make_float2(re, im);
                }
        }
#pragma unroll
    for (int f = 0; f < 12; ++f) out[((int64_t)a * V + x) * 12 + f] = acc[f];
}

// dL/dh_b* = sum_p T_{rev p} ( sum_a W[p][a][b]^+ D_a ) ; grid (sites, Cin)
__global__ void k_ptc_back_data(float2* __restrict__ Dh, const float2* __restrict__ D, const float2* __restrict__ W,
                                const float2* __restrict__ U, const int* __restrict__ nbr, int64_t V, int cin,
                                int cout) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (x >= V) return;
    float2 acc[12];
#pragma unroll
    for (int f = 0; f < 12; ++f) acc[f] = make_float2(0, 0);
    for (int p = 0; p < 9; ++p) {
        const int rp = rev_path(p);
        for (int a = 0; a < cout; ++a) {
            // g = W[p][a][b]^+ D_a, then transported by T_{rev p}: transport first (it
            // acts on colour only), then the spin matrix
            float2 t[12];
            transport(t, D + (int64_t)a * V * 12, U, nbr, V, x, rp);
            const float2* w = W + (((int64_t)p * cout + a) * cin + b) * 16;
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float re = acc[s * 3 + c].x, im = acc[s * 3 + c].y;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const float2 m = w[q * 4 + s], v = t[q * 3 + c];   // conj(W[q][s]) * t[q]
                        re += m.x * v.x + m.y * v.y;
                        im += m.x * v.y - m.y * v.x;
                    }
                    acc[s * 3 + c] = make_float2(re, im);
                }
        }
    }
#pragma unroll
    for (int f = 0; f < 12; ++f) Dh[((int64_t)b * V + x) * 12 + f] = acc[f];
}

// partial[blk][combo][16] of 2 sum_x sum_c D_a(x)[s][c] conj(T_p h_b(x)[t][c]); grid (blocks, 9*cout*cin)
__global__ __launch_bounds__(256) void k_ptc_wgrad(double* __restrict__ part, const float2* __restrict__ D,
                                                   const float2* __restrict__ h, const float2* __restrict__ U,
                                                   const int* __restrict__ nbr, int64_t V, int cin, int cout) {
    __shared__ double red[4][32];
    const int combo = blockIdx.y;
    const int p = combo / (cout * cin), a = (combo / cin) % cout, b = combo % cin;
    double acc[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) acc[i] = 0;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < V; x += (int64_t)gridDim.x * blockDim.x) {
        float2 t[12];
        transport(t, h + (int64_t)b * V * 12, U, nbr, V, x, p);
        const float2* d = D + ((int64_t)a * V + x) * 12;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float2 dv = d[s * 3 + c], tv = t[q * 3 + c];
                    acc[2 * (s * 4 + q)] += (double)dv.x * tv.x + (double)dv.y * tv.y;
                    acc[2 * (s * 4 + q) + 1] += (double)dv.y * tv.x - (double)dv.x * tv.y;
                }
    }
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        double v = acc[i];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
        if (l == 0) red[w][i] = v;
    }
    __syncthreads();
    if (threadIdx.x < 32) {
        const double v = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
        part[((int64_t)blockIdx.x * gridDim.y + combo) * 32 + threadIdx.x] = 2.0 * v;
    }
}

// G[combo][16] += sum over blocks (fixed order)
__global__ void k_ptc_wgrad_final(float2* __restrict__ G, const double* __restrict__ part, int nblk, int ncombo) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ncombo * 16) return;
    double re = 0, im = 0;
    for (int k = 0; k < nblk; ++k) {
        re += part[((int64_t)k * ncombo) * 32 + 2 * i];
        im += part[((int64_t)k * ncombo) * 32 + 2 * i + 1];
    }
    G[i].x += (float)re;
    G[i].y += (float)im;
}

// per-block partials of |e|^2 (slot 0) and |y - e|^2 (slot 1)
__global__ __launch_bounds__(256) void k_ptc_loss_part(double* __restrict__ part, const float2* __restrict__ y,
                                                       const float2* __restrict__ e, int64_t n) {
    __shared__ double red[2][4];
    double ee = 0, dd = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float2 a = y[i], b = e[i];
        ee += (double)b.x * b.x + (double)b.y * b.y;
        const double dx = (double)a.x - b.x, dy = (double)a.y - b.y;
        dd += dx * dx + dy * dy;
    }
    for (int o = 32; o > 0; o >>= 1) {
        ee += __shfl_down(ee, o, 64);
        dd += __shfl_down(dd, o, 64);
    }
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) { red[0][w] = ee; red[1][w] = dd; }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[blockIdx.x * 2] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        part[blockIdx.x * 2 + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
}

// loss[0] += |y-e|^2/|e|^2 ; loss[1] = |e|^2
__global__ void k_ptc_loss_final(double* __restrict__ loss, const double* __restrict__ part, int nblk) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double ee = 0, dd = 0;
    for (int k = 0; k < nblk; ++k) {
        ee += part[2 * k];
        dd += part[2 * k + 1];
    }
    loss[1] = ee;
    loss[0] += ee > 0 ? dd / ee : 0.0;
}

// D = (y - e)/|e|^2
__global__ void k_ptc_dloss(float2* __restrict__ D, const float2* __restrict__ y, const float2* __restrict__ e,
                            const double* __restrict__ loss, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float inv = loss[1] > 0 ? (float)(1.0 / loss[1]) : 0.0f;
    D[i] = make_float2((y[i].x - e[i].x) * inv, (y[i].y - e[i].y) * inv);
}

__global__ void k_ptc_adam(float2* __restrict__ W, const float2* __restrict__ G, float2* __restrict__ m,
                           float2* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float2 g = G[i];
    float2 mm = m[i], vv = v[i];
    mm.x = b1 * mm.x + (1 - b1) * g.x;
    mm.y = b1 * mm.y + (1 - b1) * g.y;
    vv.x = b2 * vv.x + (1 - b2) * g.x * g.x;
    vv.y = b2 * vv.y + (1 - b2) * g.y * g.y;
    m[i] = mm;
    v[i] = vv;
    float2 w = W[i];
    w.x -= lr * (mm.x / c1) / (sqrtf(vv.x / c2) + eps);
    w.y -= lr * (mm.y / c1) / (sqrtf(vv.y / c2) + eps);
    W[i] = w;
}

// out = gamma5 in * scale  (chiral basis: spins 2, 3 change sign)
__global__ void k_gamma5_scale(float2* __restrict__ out, const float2* __restrict__ in, const double* __restrict__ nrm,
                               int use_norm, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float sc = 1.0f;
    if (use_norm) sc = nrm[1] > 0 ? (float)(1.0 / nrm[1]) : 0.0f;
    const int f = (int)(i % 12);
    if (f >= 6) sc = -sc;
    out[i] = make_float2(in[i].x * sc, in[i].y * sc);
}

static int ptc_blocks(int64_t V) {
    int64_t b = (V + kPtcThreads - 1) / kPtcThreads;
    return (int)(b > kPtcMaxBlocks ? kPtcMaxBlocks : b);
}

qmg_status ptc_forward(qmg_ptc t, const void* r, void* y, hipStream_t s) {
    const int64_t V = t->V;
    const dim3 blk(kPtcThreads);
    const unsigned gx = (unsigned)((V + kPtcThreads - 1) / kPtcThreads);
    const float2* U = (const float2*)t->op->U;
    hipLaunchKernelGGL(k_ptc_layer, dim3(gx, t->C), blk, 0, s, t->h1, (const float2*)r, t->W1, U, t->op->nbr, V, 1, t->C);
    hipLaunchKernelGGL(k_ptc_layer, dim3(gx, 1), blk, 0, s, (float2*)y, t->h1, t->W2, U, t->op->nbr, V, t->C, 1);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

qmg_status ptc_backward(qmg_ptc t, const void* r, hipStream_t s);

}  // namespace qmg

using namespace qmg;

extern "C" void qmg_ptc_destroy(qmg_ptc t) {
    if (!t) return;
    float2* bufs[] = {t->W1, t->W2, t->G1, t->G2, t->m1, t->v1, t->m2, t->v2, t->h1, t->D1, t->y, t->D2, t->t1, t->t2};
    for (float2* b : bufs)
        if (b) (void)hipFree(b);
    if (t->part) (void)hipFree(t->part);
    if (t->loss) (void)hipFree(t->loss);
    delete t;
}

extern "C" qmg_status qmg_ptc_create(qmg_fine_op links, int hidden, void* stream, qmg_ptc* out) {
    if (!out) return fail(QMG_ERR_ARG, "ptc_create: out is NULL");
    *out = nullptr;
    if (!links) return fail(QMG_ERR_ARG, "ptc_create: links is NULL");
    if (links->storage != QMG_C64) return fail(QMG_ERR_PREC, "ptc_create: the operator must use complex64 storage");
    if (hidden < 1 || hidden > 16) return fail(QMG_ERR_ARG, "ptc_create: hidden channels %d outside [1,16]", hidden);
    hipStream_t s = as_stream(stream);
    auto* t = new qmg_ptc_s();
    t->op = links;
    t->C = hidden;
    t->V = links->V;
    const size_t nw = (size_t)9 * hidden * 16;
    const size_t fv = (size_t)t->V * 12;
    hipError_t e = hipSuccess;
    float2** wb[] = {&t->W1, &t->W2, &t->G1, &t->G2, &t->m1, &t->v1, &t->m2, &t->v2};
    for (float2** p : wb)
        if (e == hipSuccess) e = hipMalloc(p, sizeof(float2) * nw);
    if (e == hipSuccess) e = hipMalloc(&t->h1, sizeof(float2) * fv * hidden);
    if (e == hipSuccess) e = hipMalloc(&t->D1, sizeof(float2) * fv * hidden);
    if (e == hipSuccess) e = hipMalloc(&t->y, sizeof(float2) * fv);
    if (e == hipSuccess) e = hipMalloc(&t->D2, sizeof(float2) * fv);
    if (e == hipSuccess) e = hipMalloc(&t->t1, sizeof(float2) * fv);
    if (e == hipSuccess) e = hipMalloc(&t->t2, sizeof(float2) * fv);
    if (e == hipSuccess) e = hipMalloc(&t->part, sizeof(double) * kPtcMaxBlocks * 9 * hidden * 32);
    if (e == hipSuccess) e = hipMalloc(&t->loss, sizeof(double) * 2);
    for (float2** p : wb)
        if (e == hipSuccess) e = hipMemsetAsync(*p, 0, sizeof(float2) * nw, s);
    if (e == hipSuccess) e = hipMemsetAsync(t->loss, 0, sizeof(double) * 2, s);
    if (e != hipSuccess) {
        qmg_ptc_destroy(t);
        return fail(QMG_ERR_NOMEM, "ptc_create: %s", hipGetErrorString(e));
    }
    *out = t;
    return QMG_OK;
}

extern "C" qmg_status qmg_ptc_set_weights(qmg_ptc t, const void* W1, const void* W2, void* stream) {
    if (!t || !W1 || !W2) return fail(QMG_ERR_ARG, "ptc_set_weights: NULL argument");
    const size_t nb = sizeof(float2) * 9 * t->C * 16;
    hipStream_t s = as_stream(stream);
    QMG_HIP(hipMemcpyAsync(t->W1, W1, nb, hipMemcpyDeviceToDevice, s));
    QMG_HIP(hipMemcpyAsync(t->W2, W2, nb, hipMemcpyDeviceToDevice, s));
    QMG_HIP(hipMemsetAsync(t->m1, 0, nb, s));
    QMG_HIP(hipMemsetAsync(t->v1, 0, nb, s));
    QMG_HIP(hipMemsetAsync(t->m2, 0, nb, s));
    QMG_HIP(hipMemsetAsync(t->v2, 0, nb, s));
    t->adam_t = 0;
    return QMG_OK;
}

extern "C" qmg_status qmg_ptc_get_weights(qmg_ptc t, void* W1, void* W2, void* stream) {
    if (!t || !W1 || !W2) return fail(QMG_ERR_ARG, "ptc_get_weights: NULL argument");
    const size_t nb = sizeof(float2) * 9 * t->C * 16;
    hipStream_t s = as_stream(stream);
    QMG_HIP(hipMemcpyAsync(W1, t->W1, nb, hipMemcpyDeviceToDevice, s));
    QMG_HIP(hipMemcpyAsync(W2, t->W2, nb, hipMemcpyDeviceToDevice, s));
    return QMG_OK;
}

extern "C" qmg_status qmg_ptc_forward(qmg_ptc t, const void* r, void* y, void* stream) {
    if (!t || !r || !y) return fail(QMG_ERR_ARG, "ptc_forward: NULL argument");
    if (r == y) return fail(QMG_ERR_ARG, "ptc_forward: r and y alias");
    return ptc_forward(t, r, y, as_stream(stream));
}

extern "C" qmg_status qmg_ptc_accumulate_grad(qmg_ptc t, const void* r, const void* e, void* stream) {
    if (!t || !r || !e) return fail(QMG_ERR_ARG, "ptc_accumulate_grad: NULL argument");
    hipStream_t s = as_stream(stream);
    const int64_t V = t->V, n = V * 12;
    QMG_TRY(ptc_forward(t, r, t->y, s));
    const int nb = ptc_blocks(n);
    hipLaunchKernelGGL(k_ptc_loss_part, dim3(nb), dim3(256), 0, s, t->part, t->y, (const float2*)e, n);
    hipLaunchKernelGGL(k_ptc_loss_final, dim3(1), dim3(64), 0, s, t->loss, t->part, nb);
    hipLaunchKernelGGL(k_ptc_dloss, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, t->D2, t->y,
                       (const float2*)e, t->loss, n);
    return ptc_backward(t, r, s);
}

extern "C" qmg_status qmg_ptc_accumulate_grad_residual(qmg_ptc t, const void* r, void* stream) {
    if (!t || !r) return fail(QMG_ERR_ARG, "ptc_accumulate_grad_residual: NULL argument");
    hipStream_t s = as_stream(stream);
    const int64_t n = t->V * 12;
    QMG_TRY(ptc_forward(t, r, t->y, s));
    // t1 = M y ; loss += |M y - r|^2/|r|^2 ; t2 = (M y - r)/|r|^2 = dL/d(My)*
    QMG_TRY(qmg_wilson_clover_dslash(t->op, t->y, t->t1, 1, QMG_C64, stream));
    const int nb = ptc_blocks(n);
    hipLaunchKernelGGL(k_ptc_loss_part, dim3(nb), dim3(256), 0, s, t->part, t->t1, (const float2*)r, n);
    hipLaunchKernelGGL(k_ptc_loss_final, dim3(1), dim3(64), 0, s, t->loss, t->part, nb);
    hipLaunchKernelGGL(k_ptc_dloss, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, t->t2, t->t1,
                       (const float2*)r, t->loss, n);
    // D2 = M^+ t2 = gamma5 M gamma5 t2
    const unsigned g = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_gamma5_scale, dim3(g), dim3(256), 0, s, t->t1, t->t2, t->loss, 0, n);
    QMG_LAUNCH_CHECK();
    QMG_TRY(qmg_wilson_clover_dslash(t->op, t->t1, t->t2, 1, QMG_C64, stream));
    hipLaunchKernelGGL(k_gamma5_scale, dim3(g), dim3(256), 0, s, t->D2, t->t2, t->loss, 0, n);
    QMG_LAUNCH_CHECK();
    return ptc_backward(t, r, s);
}

namespace qmg {
qmg_status ptc_backward(qmg_ptc t, const void* r, hipStream_t s) {
    const int64_t V = t->V;
    const float2* U = (const float2*)t->op->U;
    const int* nbr = t->op->nbr;
    const int C = t->C;
    const int gb = ptc_blocks(V);
    // layer 2 (C -> 1): weight gradient, then D1 = dL/dh1*
    hipLaunchKernelGGL(k_ptc_wgrad, dim3(gb, 9 * C), dim3(256), 0, s, t->part, t->D2, t->h1, U, nbr, V, C, 1);
    hipLaunchKernelGGL(k_ptc_wgrad_final, dim3((9 * C * 16 + 255) / 256), dim3(256), 0, s, t->G2, t->part, gb, 9 * C);
    const unsigned gx = (unsigned)((V + kPtcThreads - 1) / kPtcThreads);
    hipLaunchKernelGGL(k_ptc_back_data, dim3(gx, C), dim3(kPtcThreads), 0, s, t->D1, t->D2, t->W2, U, nbr, V, C, 1);
    // layer 1 (1 -> C): weight gradient against the input r
    hipLaunchKernelGGL(k_ptc_wgrad, dim3(gb, 9 * C), dim3(256), 0, s, t->part, t->D1, (const float2*)r, U, nbr, V, 1, C);
    hipLaunchKernelGGL(k_ptc_wgrad_final, dim3((9 * C * 16 + 255) / 256), dim3(256), 0, s, t->G1, t->part, gb, 9 * C);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}
}  // namespace qmg

extern "C" qmg_status qmg_ptc_zero_grad(qmg_ptc t, void* stream) {
    if (!t) return fail(QMG_ERR_ARG, "ptc_zero_grad: NULL argument");
    hipStream_t s = as_stream(stream);
    const size_t nb = sizeof(float2) * 9 * t->C * 16;
    QMG_HIP(hipMemsetAsync(t->G1, 0, nb, s));
    QMG_HIP(hipMemsetAsync(t->G2, 0, nb, s));
    QMG_HIP(hipMemsetAsync(t->loss, 0, sizeof(double) * 2, s));
    return QMG_OK;
}

extern "C" qmg_status qmg_ptc_get_grad(qmg_ptc t, void* G1, void* G2, double* loss, void* stream) {
    if (!t || !G1 || !G2 || !loss) return fail(QMG_ERR_ARG, "ptc_get_grad: NULL argument");
    hipStream_t s = as_stream(stream);
    const size_t nb = sizeof(float2) * 9 * t->C * 16;
    QMG_HIP(hipMemcpyAsync(G1, t->G1, nb, hipMemcpyDeviceToDevice, s));
    QMG_HIP(hipMemcpyAsync(G2, t->G2, nb, hipMemcpyDeviceToDevice, s));
    QMG_HIP(hipMemcpyAsync(loss, t->loss, sizeof(double), hipMemcpyDeviceToHost, s));
    QMG_HIP(hipStreamSynchronize(s));
    return QMG_OK;
}

extern "C" qmg_status qmg_ptc_adam_step(qmg_ptc t, float lr, float beta1, float beta2, float eps, void* stream) {
    if (!t) return fail(QMG_ERR_ARG, "ptc_adam_step: NULL argument");
    if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return fail(QMG_ERR_ARG, "ptc_adam_step: bad hyper-parameters");
    hipStream_t s = as_stream(stream);
    t->adam_t += 1;
    const float c1 = 1.0f - powf(beta1, (float)t->adam_t), c2 = 1.0f - powf(beta2, (float)t->adam_t);
    const int n = 9 * t->C * 16;
    hipLaunchKernelGGL(k_ptc_adam, dim3((n + 255) / 256), dim3(256), 0, s, t->W1, t->G1, t->m1, t->v1, n, lr, beta1, beta2, eps, c1, c2);
    hipLaunchKernelGGL(k_ptc_adam, dim3((n + 255) / 256), dim3(256), 0, s, t->W2, t->G2, t->m2, t->v2, n, lr, beta1, beta2, eps, c1, c2);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}
