// Learned smoother: gauge-equivariant parallel-transport convolution (PTC)
// network, two linear layers 1 -> C -> 1 channels, trained by Adam on
// (residual, error) pairs.  The paper's smoother is MR (Sec. 7.1); this
// network is the learned replacement, with MR as its fallback.
//
//   (T_0 h)(x) = h(x), (T_{+mu} h)(x) = U_mu(x) h(x+mu), (T_{-mu} h)(x) = U_mu(x-mu)^+ h(x-mu)
//   (boundary signs folded into the links as in the Wilson-clover operator);
//   layer: h'_a(x) = sum_b sum_p W[p][a][b] (T_p h_b)(x), W[p][a][b] a complex 4x4 spin matrix;
//   loss:  L = sum_i |N(r_i) - e_i|^2 / |e_i|^2;
//   backward: with D = dL/dy*, G[p][a][b] = 2 sum_{x,colour} D_a(x) (T_p h_b)(x)^+
//             = 2 sum_{x,colour} (T_p^+ D_a)(x) h_b(x)^+,
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

__device__ __forceinline__ int rev_path(int p) { return p == 0 ? 0 : (((p - 1) & 1) ? p - 1 : p + 1); }

// The spin weights act on spin and the transports on colour and site, so they
// commute: sum_b W[p][a][b] (T_p h_b) = T_p (sum_b W[p][a][b] h_b).  The
// kernels below use that to transport each field once per path: a layer with
// one input channel transports it nine times per site and shares the
// results among all output channels; a layer with one output channel mixes
// the input channels first and transports the mixture once per path.  Work-
// groups cover kPtcSites sites with one thread per (site, path).
constexpr int kPtcSites = 32;
constexpr int kPtcFanThreads = kPtcSites * 9;

// T_p applied to the spinor v already read at the neighbour n of x
__device__ __forceinline__ void transport_vals(float2 t[12], const float2 v[12], const float2* __restrict__ U,
                                               int64_t V, int64_t x, int64_t n, int p) {
    if (p == 0) {
#pragma unroll
        for (int f = 0; f < 12; ++f) t[f] = v[f];
        return;
    }
    const int mu = (p - 1) >> 1;
    const bool back = ((p - 1) & 1) != 0;
    const int64_t ls = back ? n : x;
    float2 u[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = U[((int64_t)mu * 9 + e) * V + ls];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float re = 0, im = 0;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const float2 w = back ? make_float2(u[b * 3 + a].x, -u[b * 3 + a].y) : u[a * 3 + b];
                const float2 q = v[sp * 3 + b];
                re += w.x * q.x - w.y * q.y;
                im += w.x * q.y + w.y * q.x;
            }
            t[sp * 3 + a] = make_float2(re, im);
        }
}

__device__ __forceinline__ int64_t path_site(const int* __restrict__ nbr, int64_t x, int p) {
    return p == 0 ? x : nbr[x * 8 + 2 * ((p - 1) >> 1) + ((p - 1) & 1)];
}

// One transported input channel h, C output channels:
//   forward (first layer):           out_a = sum_p W1[p][a][0] (T_p h)
//   ADJ (data gradient of the second): out_b = sum_p W2[p][0][b]^+ (T_{rev p} h)
// Both weight arrays index (p, channel) as (p*C + channel)*16.
template <bool ADJ>
__global__ __launch_bounds__(kPtcFanThreads) void k_ptc_fan_out(float2* __restrict__ out, const float2* __restrict__ h,
                                                                const float2* __restrict__ W,
                                                                const float2* __restrict__ U,
                                                                const int* __restrict__ nbr, int64_t V, int C) {
    __shared__ float2 tp[kPtcSites][9][12];
    const int64_t x0 = (int64_t)blockIdx.x * kPtcSites;
    const int t = threadIdx.x;
    {
        const int sl = t / 9, p = t - (t / 9) * 9;
        const int64_t x = x0 + sl;
        if (x < V) {
            const int q = ADJ ? rev_path(p) : p;
            const int64_t n = path_site(nbr, x, q);
            float2 v[12], w[12];
#pragma unroll
            for (int f = 0; f < 12; ++f) v[f] = h[n * 12 + f];
            transport_vals(w, v, U, V, x, n, q);
#pragma unroll
            for (int f = 0; f < 12; ++f) tp[sl][p][f] = w[f];
        }
    }
    __syncthreads();
    for (int idx = t; idx < kPtcSites * C; idx += kPtcFanThreads) {
        const int sl = idx % kPtcSites, a = idx / kPtcSites;
        const int64_t x = x0 + sl;
        if (x >= V) continue;
        float2 acc[12];
#pragma unroll
        for (int f = 0; f < 12; ++f) acc[f] = make_float2(0, 0);
        for (int p = 0; p < 9; ++p) {
            const float2* w = W + ((int64_t)p * C + a) * 16;
#pragma unroll
            for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float re = acc[sp * 3 + c].x, im = acc[sp * 3 + c].y;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const float2 v = tp[sl][p][q * 3 + c];
                        if (ADJ) {   // conj(W[q][sp]) v
                            const float2 m = w[q * 4 + sp];
                            re += m.x * v.x + m.y * v.y;
                            im += m.x * v.y - m.y * v.x;
                        } else {
                            const float2 m = w[sp * 4 + q];
                            re += m.x * v.x - m.y * v.y;
                            im += m.x * v.y + m.y * v.x;
                        }
                    }
                    acc[sp * 3 + c] = make_float2(re, im);
                }
        }
#pragma unroll
        for (int f = 0; f < 12; ++f) out[((int64_t)a * V + x) * 12 + f] = acc[f];
    }
}

// C input channels h [C][V][12], one output: out = sum_p T_p (sum_b W2[p][0][b] h_b)
__global__ __launch_bounds__(kPtcFanThreads) void k_ptc_fan_in(float2* __restrict__ out, const float2* __restrict__ h,
                                                               const float2* __restrict__ W,
                                                               const float2* __restrict__ U,
                                                               const int* __restrict__ nbr, int64_t V, int C) {
    __shared__ float2 cp[kPtcSites][9][12];
    const int64_t x0 = (int64_t)blockIdx.x * kPtcSites;
    const int t = threadIdx.x;
    {
        const int sl = t / 9, p = t - (t / 9) * 9;
        const int64_t x = x0 + sl;
        if (x < V) {
            const int64_t n = path_site(nbr, x, p);
            float2 g[12];
#pragma unroll
            for (int f = 0; f < 12; ++f) g[f] = make_float2(0, 0);
            for (int b = 0; b < C; ++b) {
                const float2* w = W + ((int64_t)p * C + b) * 16;
                float2 v[12];
#pragma unroll
                for (int f = 0; f < 12; ++f) v[f] = h[((int64_t)b * V + n) * 12 + f];
#pragma unroll
                for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        float re = g[sp * 3 + c].x, im = g[sp * 3 + c].y;
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const float2 m = w[sp * 4 + q], vv = v[q * 3 + c];
                            re += m.x * vv.x - m.y * vv.y;
                            im += m.x * vv.y + m.y * vv.x;
                        }
                        g[sp * 3 + c] = make_float2(re, im);
                    }
            }
            float2 w2[12];
            transport_vals(w2, g, U, V, x, n, p);
#pragma unroll
            for (int f = 0; f < 12; ++f) cp[sl][p][f] = w2[f];
        }
    }
    __syncthreads();
    for (int idx = t; idx < kPtcSites * 12; idx += kPtcFanThreads) {
        const int sl = idx / 12, f = idx - (idx / 12) * 12;
        const int64_t x = x0 + sl;
        if (x >= V) continue;
        float re = 0, im = 0;
#pragma unroll
        for (int p = 0; p < 9; ++p) {
            re += cp[sl][p][f].x;
            im += cp[sl][p][f].y;
        }
        out[x * 12 + f] = make_float2(re, im);
    }
}

// Weight gradient against one transported field (tr, 1 channel) and one
// C-channel field (mc), G[p][k](s,t) = 2 sum_{x,c} L(x)[s][c] conj(R(x)[t][c]):
//   TR_LEFT (second layer, G2[p][0][k]): L = T_{rev p} tr (tr = D), R = mc_k (h1);
//   else    (first layer,  G1[p][k][0]): L = mc_k (D1), R = T_p tr (tr = r).
// Each work-group walks chunks of kPtcSites sites: per chunk the nine
// transports per site and the C channels of the chunk's sites go to LDS.
// Thread (pair, quarter) owns the 4x4 block of one (p, k) pair over one
// of Q slices of the chunk's sites (Q * 9C <= threads): per site and colour
// it reads 4 + 4 operands for 16 products, sums the chunk in FP32 and adds
// the chunk sums to FP64 totals in registers.  At the end the Q slices are
// added in a fixed order in LDS and the work-group's sums go to
// part[blk][9C][32], which a second kernel sums over work-groups in a fixed
// order.
template <bool TR_LEFT>
__global__ __launch_bounds__(kPtcFanThreads) void k_ptc_wgrad_fan(double* __restrict__ part,
                                                                  const float2* __restrict__ tr,
                                                                  const float2* __restrict__ mc,
                                                                  const float2* __restrict__ U,
                                                                  const int* __restrict__ nbr, int64_t V, int C) {
    extern __shared__ __align__(16) unsigned char smem[];
    float2 (*tp)[9][12] = reinterpret_cast<float2 (*)[9][12]>(smem);
    float2* ms = reinterpret_cast<float2*>(smem + sizeof(float2) * kPtcSites * 9 * 12);   // [C][kPtcSites][12]
    const int t = threadIdx.x;
    int Q = kPtcSites;
    while (Q * C > kPtcSites) Q >>= 1;   // 9 C Q <= 9 kPtcSites = the work-group size
    const int S = kPtcSites / Q;           // sites per slice
    const bool active = t < 9 * C * Q;
    const int pair = t / Q, quarter = t - (t / Q) * Q;
    const int p = pair / C, k = pair - (pair / C) * C;
    double acc[16][2];
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[e][0] = acc[e][1] = 0;
    const int64_t nchunks = (V + kPtcSites - 1) / kPtcSites;
    for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int64_t x0 = ch * kPtcSites;
        __syncthreads();   // the previous chunk's LDS reads are done
        {
            const int sl = t / 9, q = t - (t / 9) * 9;
            const int64_t x = x0 + sl;
            float2 w[12];
            if (x < V) {
                const int qq = TR_LEFT ? rev_path(q) : q;
                const int64_t n = path_site(nbr, x, qq);
                float2 v[12];
#pragma unroll
                for (int f = 0; f < 12; ++f) v[f] = tr[n * 12 + f];
                transport_vals(w, v, U, V, x, n, qq);
            } else {
#pragma unroll
                for (int f = 0; f < 12; ++f) w[f] = make_float2(0, 0);
            }
#pragma unroll
            for (int f = 0; f < 12; ++f) tp[sl][q][f] = w[f];
        }
        for (int idx = t; idx < C * kPtcSites * 12; idx += kPtcFanThreads) {
            const int f = idx % 12, sl = (idx / 12) % kPtcSites, kk = idx / (12 * kPtcSites);
            const int64_t x = x0 + sl;
            ms[idx] = x < V ? mc[((int64_t)kk * V + x) * 12 + f] : make_float2(0, 0);
        }
        __syncthreads();
        if (active) {
            float sr[16], si[16];
#pragma unroll
            for (int e = 0; e < 16; ++e) sr[e] = si[e] = 0.0f;
            for (int i = 0; i < S; ++i) {
                const int sl = quarter * S + i;
                const float2* m = ms + ((int64_t)k * kPtcSites + sl) * 12;
                const float2* tq = tp[sl][p];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float2 L[4], R[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        L[u] = TR_LEFT ? tq[u * 3 + c] : m[u * 3 + c];
                        R[u] = TR_LEFT ? m[u * 3 + c] : tq[u * 3 + c];
                    }
#pragma unroll
                    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                        for (int tt = 0; tt < 4; ++tt) {
                            sr[sp * 4 + tt] += L[sp].x * R[tt].x + L[sp].y * R[tt].y;
                            si[sp * 4 + tt] += L[sp].y * R[tt].x - L[sp].x * R[tt].y;
                        }
                }
            }
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                acc[e][0] += (double)sr[e];
                acc[e][1] += (double)si[e];
            }
        }
    }
    // the Q slices of each pair, added in slice order, then the work-group's sums
    __syncthreads();
    double* red = reinterpret_cast<double*>(smem);   // [9C][32]
    for (int qd = 0; qd < Q; ++qd) {
        if (active && quarter == qd)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                double* d = red + pair * 32 + 2 * e;
                d[0] = qd ? d[0] + acc[e][0] : acc[e][0];
                d[1] = qd ? d[1] + acc[e][1] : acc[e][1];
            }
        __syncthreads();
    }
    for (int i = t; i < 9 * C * 32; i += kPtcFanThreads) part[(int64_t)blockIdx.x * (9 * C) * 32 + i] = 2.0 * red[i];
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

// Inference.  The two layers are linear, so N(r) = sum_p T_p sum_q K[p][q] T_q r
// with K[p][q] = sum_b W2[p][0][b] W1[q][b][0] (the spin weights commute with
// the transports).  First the 81 spin matrices K are formed, then
//   k_ptc_mix:  per site, the nine transports T_q r (once each, in LDS) and the
//               nine mixtures g_p = sum_q K[p][q] T_q r;
//   k_ptc_gather: N(r)(x) = sum_p (T_p g_p)(x).
// The hidden channels are never stored: per site 96 bytes in, 864 bytes of g
// out and back, instead of the hidden layer's 8 channels read nine times.
// g is laid out [9][12][V] (site fastest).
__global__ void k_ptc_collapse(float2* __restrict__ K, const float2* __restrict__ W1, const float2* __restrict__ W2,
                               int C) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;   // (p, q, s, t)
    if (i >= 81 * 16) return;
    const int p = i / (9 * 16), q = (i / 16) % 9, sp = (i / 4) % 4, tt = i % 4;
    float re = 0, im = 0;
    for (int b = 0; b < C; ++b) {
        const float2* w2 = W2 + ((int64_t)p * C + b) * 16;   // W2[p][0][b]
        const float2* w1 = W1 + ((int64_t)q * C + b) * 16;   // W1[q][b][0]
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const float2 a = w2[sp * 4 + u], c = w1[u * 4 + tt];
            re += a.x * c.x - a.y * c.y;
            im += a.x * c.y + a.y * c.x;
        }
    }
    K[i] = make_float2(re, im);
}

// Thread layout of the two inference kernels: thread t works on path
// t / kPtcSites and site t % kPtcSites of the work-group's kPtcSites sites, so
// the 32 lanes of a half-wave share a path and take consecutive sites: their
// neighbour and link loads and their stores of g (layout [9][12][V], site
// fastest) are contiguous, the LDS fields [9][12][kPtcSites] are read without
// bank conflicts and a half-wave's reads of K[p][q] are one broadcast.
__device__ __forceinline__ void transport_site(float2 w[12], const float2* __restrict__ r,
                                               const float2* __restrict__ U, const int* __restrict__ nbr,
                                               int64_t V, int64_t x, int q) {
    const int64_t n = path_site(nbr, x, q);
    float2 v[12];
    const float4* r4 = reinterpret_cast<const float4*>(r + n * 12);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        const float4 a = r4[i];
        v[2 * i] = make_float2(a.x, a.y);
        v[2 * i + 1] = make_float2(a.z, a.w);
    }
    transport_vals(w, v, U, V, x, n, q);
}

__global__ __launch_bounds__(kPtcFanThreads) void k_ptc_mix(float2* __restrict__ g, const float2* __restrict__ r,
                                                            const float2* __restrict__ K,
                                                            const float2* __restrict__ U,
                                                            const int* __restrict__ nbr, int64_t V) {
    __shared__ float2 tp[9][12][kPtcSites];
    __shared__ float2 ks[81 * 16];
    const int64_t x0 = (int64_t)blockIdx.x * kPtcSites;
    const int t = threadIdx.x;
    for (int i = t; i < 81 * 16; i += kPtcFanThreads) ks[i] = K[i];
    const int pq = t / kPtcSites, sl = t - pq * kPtcSites;
    const int64_t x = x0 + sl;
    {
        float2 w[12];
        if (x < V) {
            transport_site(w, r, U, nbr, V, x, pq);
        } else {
#pragma unroll
            for (int f = 0; f < 12; ++f) w[f] = make_float2(0, 0);
        }
#pragma unroll
        for (int f = 0; f < 12; ++f) tp[pq][f][sl] = w[f];
    }
    __syncthreads();
    if (x >= V) return;
    // thread (p, site): g_p = sum_q K[p][q] T_q r
    const int p = pq;
    float2 acc[12];
#pragma unroll
    for (int f = 0; f < 12; ++f) acc[f] = make_float2(0, 0);
    for (int q = 0; q < 9; ++q) {
        const float2* k = ks + (p * 9 + q) * 16;
        float2 v[12];
#pragma unroll
        for (int f = 0; f < 12; ++f) v[f] = tp[q][f][sl];
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float2 m = k[sp * 4 + u];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float2 w = v[u * 3 + c];
                    acc[sp * 3 + c].x += m.x * w.x - m.y * w.y;
                    acc[sp * 3 + c].y += m.x * w.y + m.y * w.x;
                }
            }
    }
#pragma unroll
    for (int f = 0; f < 12; ++f) g[((int64_t)p * 12 + f) * V + x] = acc[f];
}

__global__ __launch_bounds__(kPtcFanThreads) void k_ptc_gather(float2* __restrict__ out, const float2* __restrict__ g,
                                                               const float2* __restrict__ U,
                                                               const int* __restrict__ nbr, int64_t V) {
    __shared__ float2 cp[9][12][kPtcSites];
    const int64_t x0 = (int64_t)blockIdx.x * kPtcSites;
    const int t = threadIdx.x;
    {
        const int p = t / kPtcSites, sl = t - p * kPtcSites;
        const int64_t x = x0 + sl;
        float2 w[12];
        if (x < V) {
            const int64_t n = path_site(nbr, x, p);
            float2 v[12];
#pragma unroll
            for (int f = 0; f < 12; ++f) v[f] = g[((int64_t)p * 12 + f) * V + n];
            transport_vals(w, v, U, V, x, n, p);
        } else {
#pragma unroll
            for (int f = 0; f < 12; ++f) w[f] = make_float2(0, 0);
        }
#pragma unroll
        for (int f = 0; f < 12; ++f) cp[p][f][sl] = w[f];
    }
    __syncthreads();
    for (int idx = t; idx < kPtcSites * 12; idx += kPtcFanThreads) {
        const int sl = idx / 12, f = idx - (idx / 12) * 12;
        const int64_t x = x0 + sl;
        if (x >= V) continue;
        float re = 0, im = 0;
#pragma unroll
        for (int p = 0; p < 9; ++p) {
            re += cp[p][f][sl].x;
            im += cp[p][f][sl].y;
        }
        out[x * 12 + f] = make_float2(re, im);
    }
}

static int ptc_blocks(int64_t V) {
    int64_t b = (V + kPtcThreads - 1) / kPtcThreads;
    return (int)(b > kPtcMaxBlocks ? kPtcMaxBlocks : b);
}

// Layer by layer, keeping the hidden channels h1 (the training path: the
// gradients need them).
static qmg_status ptc_forward_layers(qmg_ptc t, const void* r, void* y, hipStream_t s) {
    const int64_t V = t->V;
    const unsigned gx = (unsigned)((V + kPtcSites - 1) / kPtcSites);
    const float2* U = (const float2*)t->op->U;
    hipLaunchKernelGGL(k_ptc_fan_out<false>, dim3(gx), dim3(kPtcFanThreads), 0, s, t->h1, (const float2*)r, t->W1, U,
                       t->op->nbr, V, t->C);
    hipLaunchKernelGGL(k_ptc_fan_in, dim3(gx), dim3(kPtcFanThreads), 0, s, (float2*)y, t->h1, t->W2, U, t->op->nbr, V,
                       t->C);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

// y = N(r) through the collapsed form (inference: the smoother and the forward entry point).
qmg_status ptc_forward(qmg_ptc t, const void* r, void* y, hipStream_t s) {
    const int64_t V = t->V;
    const unsigned gx = (unsigned)((V + kPtcSites - 1) / kPtcSites);
    const float2* U = (const float2*)t->op->U;
    if (t->k_stale) {
        hipLaunchKernelGGL(k_ptc_collapse, dim3((81 * 16 + 255) / 256), dim3(256), 0, s, t->K, t->W1, t->W2, t->C);
        t->k_stale = false;
    }
    hipLaunchKernelGGL(k_ptc_mix, dim3(gx), dim3(kPtcFanThreads), 0, s, t->g, (const float2*)r, t->K, U, t->op->nbr, V);
    hipLaunchKernelGGL(k_ptc_gather, dim3(gx), dim3(kPtcFanThreads), 0, s, (float2*)y, t->g, U, t->op->nbr, V);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

qmg_status ptc_backward(qmg_ptc t, const void* r, hipStream_t s);

}  // namespace qmg

using namespace qmg;

extern "C" void qmg_ptc_destroy(qmg_ptc t) {
    if (!t) return;
    float2* bufs[] = {t->W1, t->W2, t->G1, t->G2, t->m1, t->v1, t->m2, t->v2, t->h1, t->D1, t->y, t->D2, t->t1, t->t2,
                      t->K, t->g};
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
    if (links->storage != QMG_C64 || links->link_reals != 18)
        return fail(QMG_ERR_PREC, "ptc_create: the operator must use complex64 storage of all 18 link reals");
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
    if (e == hipSuccess) e = hipMalloc(&t->K, sizeof(float2) * 81 * 16);
    if (e == hipSuccess) e = hipMalloc(&t->g, sizeof(float2) * fv * 9);
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
    t->k_stale = true;
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

extern "C" qmg_status qmg_ptc_get_adam(qmg_ptc t, void* m1, void* v1, void* m2, void* v2, int* steps, void* stream) {
    if (!t || !m1 || !v1 || !m2 || !v2 || !steps) return fail(QMG_ERR_ARG, "ptc_get_adam: NULL argument");
    const size_t nb = sizeof(float2) * 9 * t->C * 16;
    hipStream_t s = as_stream(stream);
    QMG_HIP(hipMemcpyAsync(m1, t->m1, nb, hipMemcpyDeviceToDevice, s));
    QMG_HIP(hipMemcpyAsync(v1, t->v1, nb, hipMemcpyDeviceToDevice, s));
    QMG_HIP(hipMemcpyAsync(m2, t->m2, nb, hipMemcpyDeviceToDevice, s));
    QMG_HIP(hipMemcpyAsync(v2, t->v2, nb, hipMemcpyDeviceToDevice, s));
    *steps = t->adam_t;
    return QMG_OK;
}

extern "C" qmg_status qmg_ptc_set_adam(qmg_ptc t, const void* m1, const void* v1, const void* m2, const void* v2,
                                       int steps, void* stream) {
    if (!t || !m1 || !v1 || !m2 || !v2) return fail(QMG_ERR_ARG, "ptc_set_adam: NULL argument");
    if (steps < 0) return fail(QMG_ERR_ARG, "ptc_set_adam: steps %d < 0", steps);
    const size_t nb = sizeof(float2) * 9 * t->C * 16;
    hipStream_t s = as_stream(stream);
    QMG_HIP(hipMemcpyAsync(t->m1, m1, nb, hipMemcpyDeviceToDevice, s));
    QMG_HIP(hipMemcpyAsync(t->v1, v1, nb, hipMemcpyDeviceToDevice, s));
    QMG_HIP(hipMemcpyAsync(t->m2, m2, nb, hipMemcpyDeviceToDevice, s));
    QMG_HIP(hipMemcpyAsync(t->v2, v2, nb, hipMemcpyDeviceToDevice, s));
    t->adam_t = steps;
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
    QMG_TRY(ptc_forward_layers(t, r, t->y, s));
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
    QMG_TRY(ptc_forward_layers(t, r, t->y, s));
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
    const size_t lds = sizeof(float2) * kPtcSites * 12 * (9 + C);
    if (lds > 65536) {
        QMG_HIP(hipFuncSetAttribute((const void*)k_ptc_wgrad_fan<true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        QMG_HIP(hipFuncSetAttribute((const void*)k_ptc_wgrad_fan<false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    }
    // second layer (C -> 1): weight gradient, then D1 = dL/dh1*
    hipLaunchKernelGGL(k_ptc_wgrad_fan<true>, dim3(gb), dim3(kPtcFanThreads), lds, s, t->part, t->D2, t->h1, U, nbr, V,
                       C);
    hipLaunchKernelGGL(k_ptc_wgrad_final, dim3((9 * C * 16 + 255) / 256), dim3(256), 0, s, t->G2, t->part, gb, 9 * C);
    const unsigned gx = (unsigned)((V + kPtcSites - 1) / kPtcSites);
    hipLaunchKernelGGL(k_ptc_fan_out<true>, dim3(gx), dim3(kPtcFanThreads), 0, s, t->D1, t->D2, t->W2, U, nbr, V, C);
    // first layer (1 -> C): weight gradient against the input r
    hipLaunchKernelGGL(k_ptc_wgrad_fan<false>, dim3(gb), dim3(kPtcFanThreads), lds, s, t->part, (const float2*)r,
                       t->D1, U, nbr, V, C);
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
    t->k_stale = true;
    const float c1 = 1.0f - powf(beta1, (float)t->adam_t), c2 = 1.0f - powf(beta2, (float)t->adam_t);
    const int n = 9 * t->C * 16;
    hipLaunchKernelGGL(k_ptc_adam, dim3((n + 255) / 256), dim3(256), 0, s, t->W1, t->G1, t->m1, t->v1, n, lr, beta1, beta2, eps, c1, c2);
    hipLaunchKernelGGL(k_ptc_adam, dim3((n + 255) / 256), dim3(256), 0, s, t->W2, t->G2, t->m2, t->v2, n, lr, beta1, beta2, eps, c1, c2);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}
