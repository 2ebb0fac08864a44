// BLAS-1 kernels of the solvers (see blas.h).
#include "blas.h"
#include "codes16.h"

#include <algorithm>
#include <type_traits>

namespace qmg {

static constexpr int kThreads = 256;
static constexpr int64_t kOneBlock = 1 << 12;  // up to this many entries one 1024-thread block reduces alone

static int nblocks(int64_t n) {
    if (n <= kOneBlock) return 1;
    int64_t b = (n + kThreads - 1) / kThreads;
    if (b > Blas::kMaxBlocks) b = Blas::kMaxBlocks;
    return (int)b;
}
static int rthreads(int nb) { return nb == 1 ? 1024 : kThreads; }

// sum of v over the work-group, valid in thread 0
__device__ __forceinline__ double wg_sum(double v, double* lds) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) lds[w] = v;
    __syncthreads();
    double t = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += lds[i];
    return t;
}

// phase 2: out[v] = sum over blocks of the partials; thread t adds blocks t
// and t+256, then a fixed tree: the same order on every run.  The partials of
// one value are contiguous ([value][block]), so the loads coalesce, and four
// values are summed per round: their loads are issued together and share one
// pass through LDS.  Loads past the nb blocks (or the nv values) stay inside
// the table and are not used.
static_assert(Blas::kMaxBlocks == 512, "k_final: each of its 256 threads adds two blocks");
__global__ __launch_bounds__(256) void k_final(const double* __restrict__ partials, int nb, int nv,
                                               double* __restrict__ out, int ss) {
    __shared__ double lds[4][4];   // [value][wave]
    partials += (int64_t)blockIdx.y * Blas::kMaxBlocks * Blas::kMaxVals;
    out += (int64_t)blockIdx.y * ss;
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    for (int v0 = 0; v0 < nv; v0 += 4) {
        double sv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int v = v0 + i < Blas::kMaxVals ? v0 + i : 0;
            const double a = partials[v * Blas::kMaxBlocks + t], b = partials[v * Blas::kMaxBlocks + t + 256];
            sv[i] = (t < nb ? a : 0.0) + (t + 256 < nb ? b : 0.0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
            for (int o = 32; o > 0; o >>= 1) sv[i] += __shfl_down(sv[i], o, 64);
        __syncthreads();
        if (l == 0)
#pragma unroll
            for (int i = 0; i < 4; ++i) lds[i][w] = sv[i];
        __syncthreads();
        if (t < 4 && v0 + t < nv) {
            double r = 0;
            for (int j = 0; j < 4; ++j) r += lds[t][j];
            out[v0 + t] = r;
        }
    }
}

// this work-group's batch member: shift its vectors by member*n, its scalars
// by member*ss and its partial sums to the member's own table
#define QMG_MEMBER_SCAL(p) p += (int64_t)blockIdx.y * ss
#define QMG_MEMBER_VEC(p) p += (int64_t)blockIdx.y * n
#define QMG_MEMBER_PART(p) p += (int64_t)blockIdx.y * Blas::kMaxBlocks * Blas::kMaxVals

// a work-group's sums: to the partials, or straight to the result when the grid is one block
__device__ __forceinline__ void put(double* part, double* out, int v, double val) {
    if (gridDim.x == 1) out[v] = val;
    else part[v * Blas::kMaxBlocks + blockIdx.x] = val;
}

template <typename R>
__global__ __launch_bounds__(1024) void k_dot(const cpx<R>* __restrict__ a, const cpx<R>* __restrict__ b, int64_t n,
                      double* __restrict__ part, double* __restrict__ out, int ss) {
    __shared__ double lds[16];
    QMG_MEMBER_VEC(a); QMG_MEMBER_VEC(b); QMG_MEMBER_SCAL(out); QMG_MEMBER_PART(part);
    double re = 0, im = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const cpx<R> x = a[i], y = b[i];
        re += (double)x.re * y.re + (double)x.im * y.im;
        im += (double)x.re * y.im - (double)x.im * y.re;
    }
    re = wg_sum(re, lds);
    im = wg_sum(im, lds);
    if (threadIdx.x == 0) {
        put(part, out, 0, re);
        put(part, out, 1, im);
    }
}

template <typename R>
__global__ __launch_bounds__(1024) void k_norm2(const cpx<R>* __restrict__ a, int64_t n, double* __restrict__ part,
                                                double* __restrict__ out, int ss) {
    __shared__ double lds[16];
    QMG_MEMBER_VEC(a); QMG_MEMBER_SCAL(out); QMG_MEMBER_PART(part);
    double s = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const cpx<R> x = a[i];
        s += (double)x.re * x.re + (double)x.im * x.im;
    }
    s = wg_sum(s, lds);
    if (threadIdx.x == 0) put(part, out, 0, s);
}

template <typename R>
__global__ __launch_bounds__(1024) void k_dot_norm(const cpx<R>* __restrict__ q, const cpx<R>* __restrict__ r,
                                                   int64_t n, double* __restrict__ part, double* __restrict__ out,
                                                   int ss) {
    __shared__ double lds[16];
    QMG_MEMBER_VEC(q); QMG_MEMBER_VEC(r); QMG_MEMBER_SCAL(out); QMG_MEMBER_PART(part);
    double qq = 0, re = 0, im = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const cpx<R> x = q[i], y = r[i];
        qq += (double)x.re * x.re + (double)x.im * x.im;
        re += (double)x.re * y.re + (double)x.im * y.im;
        im += (double)x.re * y.im - (double)x.im * y.re;
    }
    qq = wg_sum(qq, lds);
    re = wg_sum(re, lds);
    im = wg_sum(im, lds);
    if (threadIdx.x == 0) {
        put(part, out, 0, qq);
        put(part, out, 1, re);
        put(part, out, 2, im);
    }
}

template <typename R>
__global__ __launch_bounds__(1024) void k_multi_dot(const cpx<R>* __restrict__ Q, int64_t ld, int k,
                                                    const cpx<R>* __restrict__ q, int64_t n,
                                                    double* __restrict__ part, double* __restrict__ out, int ss) {
    __shared__ double lds[16];
    QMG_MEMBER_VEC(Q); QMG_MEMBER_VEC(q); QMG_MEMBER_SCAL(out); QMG_MEMBER_PART(part);
    double re[16], im[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) re[j] = im[j] = 0;
    // unconditional loads in blocks of CW slots (slots past the last one
    // re-read it and are not used), so a block's loads are in flight together
    constexpr int CW = sizeof(R) == 8 ? 8 : 16;
    const int kc = k - 1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const cpx<R> y = q[i];
#pragma unroll
        for (int j0 = 0; j0 < 16; j0 += CW)
            if (j0 < k) {
                cpx<R> x[CW];
#pragma unroll
                for (int j = 0; j < CW; ++j) x[j] = Q[(int64_t)(j0 + j < k ? j0 + j : kc) * ld + i];
#pragma unroll
                for (int j = 0; j < CW; ++j)
                    if (j0 + j < k) {
                        re[j0 + j] += (double)x[j].re * y.re + (double)x[j].im * y.im;
                        im[j0 + j] += (double)x[j].re * y.im - (double)x[j].im * y.re;
                    }
            }
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        if (j < k) {
            const double a = wg_sum(re[j], lds);
            const double b = wg_sum(im[j], lds);
            if (threadIdx.x == 0) {
                put(part, out, 2 * j, a);
                put(part, out, 2 * j + 1, b);
            }
        }
    }
}

template <typename R>
__global__ void k_multi_axpy(const double* __restrict__ beta, const cpx<R>* __restrict__ Q,
                             const cpx<R>* __restrict__ Z, int64_t ld, int k, cpx<R>* __restrict__ q,
                             cpx<R>* __restrict__ z, int64_t n, int ss) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    QMG_MEMBER_SCAL(beta); QMG_MEMBER_VEC(Q); QMG_MEMBER_VEC(q);
    if (z) { QMG_MEMBER_VEC(Z); QMG_MEMBER_VEC(z); }
    R qr = q[i].re, qi = q[i].im;
    R zr = 0, zi = 0;
    if (z) { zr = z[i].re; zi = z[i].im; }
    for (int j = 0; j < k; ++j) {
        const R br = (R)beta[2 * j], bi = (R)beta[2 * j + 1];
        const cpx<R> a = Q[j * ld + i];
        qr -= br * a.re - bi * a.im;
        qi -= br * a.im + bi * a.re;
        if (z) {
            const cpx<R> c = Z[j * ld + i];
            zr -= br * c.re - bi * c.im;
            zi -= br * c.im + bi * c.re;
        }
    }
    q[i] = cpx<R>{qr, qi};
    if (z) z[i] = cpx<R>{zr, zi};
}

template <typename R>
__global__ void k_gcr_update(const double* __restrict__ s3, cpx<R>* __restrict__ q, cpx<R>* __restrict__ z,
                             cpx<R>* __restrict__ x, cpx<R>* __restrict__ r, int64_t n, int ss) {
    // z and x null: the deferred form (q normalised, r updated; the caller
    // forms x from the unnormalised directions at the end of the cycle)
    QMG_MEMBER_SCAL(s3); QMG_MEMBER_VEC(q); QMG_MEMBER_VEC(r);
    if (z) { QMG_MEMBER_VEC(z); QMG_MEMBER_VEC(x); }
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !(s3[0] > 0)) return;  // q = 0: no update (breakdown is reported by the caller)
    const double nq = sqrt(s3[0]);
    const R inv = (R)(1.0 / nq);
    const R ar = (R)(s3[1] / nq), ai = (R)(s3[2] / nq);
    cpx<R> qq = q[i];
    qq.re *= inv; qq.im *= inv;
    q[i] = qq;
    if (z) {
        cpx<R> zz = z[i];
        zz.re *= inv; zz.im *= inv;
        z[i] = zz;
        cpx<R> xx = x[i];
        xx.re += ar * zz.re - ai * zz.im;
        xx.im += ar * zz.im + ai * zz.re;
        x[i] = xx;
    }
    cpx<R> rr = r[i];
    rr.re -= ar * qq.re - ai * qq.im;
    rr.im -= ar * qq.im + ai * qq.re;
    r[i] = rr;
}

template <typename R>
__global__ void k_mr_update(const double* __restrict__ s3, const cpx<R>* rin, cpx<R>* r, const cpx<R>* __restrict__ Ar,
                            cpx<R>* __restrict__ x, int first, int64_t n, int ss) {
    // XCD-contiguous ranges (the grid is a multiple of 8), as in the fine
    // operator's kernel: each XCD updates the sites whose A r it just wrote
    const int64_t per = gridDim.x >> 3;
    const int64_t wg = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
    const int64_t i = wg * blockDim.x + threadIdx.x;
    if (i >= n) return;
    QMG_MEMBER_SCAL(s3); QMG_MEMBER_VEC(rin); QMG_MEMBER_VEC(r); QMG_MEMBER_VEC(Ar); QMG_MEMBER_VEC(x);
    const double den = s3[0];
    const R ar = den > 0 ? (R)(s3[1] / den) : (R)0, ai = den > 0 ? (R)(s3[2] / den) : (R)0;
    cpx<R> rr = rin[i];
    const cpx<R> a = Ar[i];
    cpx<R> xx = first ? cpx<R>{0, 0} : x[i];
    xx.re += ar * rr.re - ai * rr.im;
    xx.im += ar * rr.im + ai * rr.re;
    rr.re -= ar * a.re - ai * a.im;
    rr.im -= ar * a.im + ai * a.re;
    x[i] = xx;
    r[i] = rr;
}

// MR on 16-bit spinor fields (FP16 pairs [site][12], one FP32 scale per site);
// member b's fields start at b * nsites sites.  The inner products give four
// consecutive lanes a site, lane j of the four taking components j, j + 4 and
// j + 8 (measured faster here than consecutive words per lane, which need a
// scale load per word).
__global__ __launch_bounds__(1024) void k_dot_norm_h16(const uint32_t* __restrict__ q, const float* __restrict__ qs,
                                                       const uint32_t* __restrict__ r, const float* __restrict__ rs,
                                                       int64_t nsites, double* __restrict__ part,
                                                       double* __restrict__ out, int ss) {
    __shared__ double lds[16];
    const int64_t mo = (int64_t)blockIdx.y * nsites;
    q += mo * 12;
    r += mo * 12;
    qs += mo;
    rs += mo;
    QMG_MEMBER_SCAL(out); QMG_MEMBER_PART(part);
    double qq = 0, re = 0, im = 0;
    const int64_t nq = nsites * 4;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nq; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t site = i >> 2;
        const float ka = qs[site], kb = rs[site];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int64_t w = (i & ~int64_t(3)) * 3 + (i & 3) + 4 * c;
            const cpx<float> a = dec_pair<FMT_H16>(q[w]), b = dec_pair<FMT_H16>(r[w]);
            const double xr = ka * a.re, xi = ka * a.im, yr = kb * b.re, yi = kb * b.im;
            qq += xr * xr + xi * xi;
            re += xr * yr + xi * yi;
            im += xr * yi - xi * yr;
        }
    }
    qq = wg_sum(qq, lds);
    re = wg_sum(re, lds);
    im = wg_sum(im, lds);
    if (threadIdx.x == 0) {
        put(part, out, 0, qq);
        put(part, out, 1, re);
        put(part, out, 2, im);
    }
}

// The update: a work-group of 256 lanes takes 64 whole sites (768 words, three
// per lane at stride 256, so every load and store instruction of a wave covers
// 64 consecutive words); the new residual's per-site maximum goes through LDS
// (one lane per site reduces its 12 words).
constexpr int kMrSites = 64;
__global__ __launch_bounds__(256) void k_mr_update_h16(const double* __restrict__ s3, const uint32_t* rin,
                                                       const float* rins, uint32_t* r, float* rs,
                                                       const uint32_t* __restrict__ Ar, const float* __restrict__ Ars,
                                                       float2* __restrict__ x, int first, int64_t nsites, int ss) {
    __shared__ float wmax[kMrSites * 12];
    __shared__ float smax[kMrSites];
    const int64_t per = gridDim.x >> 3;   // XCD-contiguous ranges, as in k_mr_update
    const int64_t wg = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
    const int64_t s0 = wg * kMrSites;     // first site of the work-group (grid padded to whole groups of 8)
    const int64_t mo = (int64_t)blockIdx.y * nsites;
    s3 += (int64_t)blockIdx.y * ss;
    const double den = s3[0];
    const float ar = den > 0 ? (float)(s3[1] / den) : 0.f, ai = den > 0 ? (float)(s3[2] / den) : 0.f;
    const int64_t nw = (nsites - s0) * 12;   // words of this group's sites left in the member (may be <= 0)
    const int64_t base = (mo + s0) * 12;
    float2 nr[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int lw = c * 256 + threadIdx.x;   // word within the group
        float m = 0.f;
        nr[c] = make_float2(0.f, 0.f);
        if (lw < nw) {
            const int64_t site = mo + s0 + lw / 12, w = base + lw;
            const float kr = rins[site], ka = Ars[site];
            const cpx<float> u = dec_pair<FMT_H16>(rin[w]), v = dec_pair<FMT_H16>(Ar[w]);
            const float ur = kr * u.re, ui = kr * u.im, vr = ka * v.re, vi = ka * v.im;
            float2 xx = first ? make_float2(0.f, 0.f) : x[w];
            xx.x += ar * ur - ai * ui;
            xx.y += ar * ui + ai * ur;
            x[w] = xx;
            nr[c] = make_float2(ur - (ar * vr - ai * vi), ui - (ar * vi + ai * vr));
            m = fmaxf(fabsf(nr[c].x), fabsf(nr[c].y));
        }
        wmax[lw] = m;
    }
    __syncthreads();
    if (threadIdx.x < kMrSites) {
        float m = 0.f;
#pragma unroll
        for (int k = 0; k < 12; ++k) m = fmaxf(m, wmax[threadIdx.x * 12 + k]);
        smax[threadIdx.x] = m;
        if (s0 + threadIdx.x < nsites) rs[mo + s0 + threadIdx.x] = m;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int lw = c * 256 + threadIdx.x;
        if (lw < nw) {
            const float m = smax[lw / 12];
            const float inv = m > 0.f ? 1.0f / m : 0.f;
            r[base + lw] = enc_pair<FMT_H16>(nr[c].x * inv, nr[c].y * inv);
        }
    }
}

// complex64 spinors [site][12] -> FP16 pairs with one scale per site, four lanes per
// site in the interleaved order above (a NaN or Inf input is recorded in nf)
__global__ __launch_bounds__(256) void k_quantize_spinor(const float2* __restrict__ in, uint32_t* __restrict__ out,
                                                         float* __restrict__ scale, int64_t nsites,
                                                         unsigned* __restrict__ nf) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nsites * 4) return;
    const int64_t w0 = (i >> 2) * 12 + (i & 3);   // component c at w0 + 4 c
    float2 v[3];
    float m = 0.f;
    bool bad = false;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        v[c] = in[w0 + 4 * c];
        bad = bad || !(isfinite(v[c].x) && isfinite(v[c].y));
        m = fmaxf(m, fmaxf(fabsf(v[c].x), fabsf(v[c].y)));
    }
    note_nonfinite(nf, bad);
    m = fmaxf(m, __shfl_xor(m, 1, 64));
    m = fmaxf(m, __shfl_xor(m, 2, 64));
    const float inv = m > 0.f ? 1.0f / m : 0.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) out[w0 + 4 * c] = enc_pair<FMT_H16>(v[c].x * inv, v[c].y * inv);
    if ((i & 3) == 0) scale[i >> 2] = m;
}

// FP16 pairs with per-site scales on the half lattice -> complex64 whole-lattice
// fields: full[b][hp[h]] = decoded half[b][h], full[b][hq[h]] = 0 (the
// other parity); four lanes per site in the interleaved order above
__global__ __launch_bounds__(256) void k_scatter_dequantize(const uint32_t* __restrict__ in,
                                                            const float* __restrict__ scale,
                                                            const int* __restrict__ hp, const int* __restrict__ hq,
                                                            float2* __restrict__ full, int64_t nsites) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nsites * 4) return;
    const int64_t b = blockIdx.y, h = i >> 2, hb = b * nsites + h;
    const float k = scale[hb];
    const int64_t wi = hb * 12 + (i & 3);
    const int64_t wp = (b * 2 * nsites + hp[h]) * 12 + (i & 3), wq = (b * 2 * nsites + hq[h]) * 12 + (i & 3);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cpx<float> v = dec_pair<FMT_H16>(in[wi + 4 * c]);
        full[wp + 4 * c] = make_float2(k * v.re, k * v.im);
        full[wq + 4 * c] = make_float2(0.f, 0.f);
    }
}

// Minimal-residual step along a given direction d with Ad = A d, from
// s3 = dot_norm(Ad, r) = [<Ad,Ad>, <Ad,r>.re, <Ad,r>.im]: alpha = <Ad,r>/<Ad,Ad>,
// x = alpha d, rout = r - alpha Ad (alpha = 0 when <Ad,Ad> = 0).
template <typename R>
__global__ void k_dir_step(const double* __restrict__ s3, const cpx<R>* __restrict__ d, const cpx<R>* __restrict__ Ad,
                           const cpx<R>* __restrict__ r, cpx<R>* __restrict__ x, cpx<R>* __restrict__ rout, int64_t n,
                           int ss) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    QMG_MEMBER_SCAL(s3); QMG_MEMBER_VEC(d); QMG_MEMBER_VEC(Ad); QMG_MEMBER_VEC(r); QMG_MEMBER_VEC(x);
    QMG_MEMBER_VEC(rout);
    const double den = s3[0];
    const R ar = den > 0 ? (R)(s3[1] / den) : (R)0, ai = den > 0 ? (R)(s3[2] / den) : (R)0;
    const cpx<R> dd = d[i], a = Ad[i], rr = r[i];
    x[i] = cpx<R>{ar * dd.re - ai * dd.im, ar * dd.im + ai * dd.re};
    rout[i] = cpx<R>{rr.re - (ar * a.re - ai * a.im), rr.im - (ar * a.im + ai * a.re)};
}

// As k_dir_step for a step that may be refused: it is taken only where it
// lowers the residual (|r - Ad|^2 < |r|^2, i.e. <Ad,Ad> - 2 Re <Ad,r> < 0,
// every scalar finite); a refused step leaves x = 0 and rout = r and adds one
// to the member's counter s3[cnt].
template <typename R>
__global__ void k_dir_step_checked(double* __restrict__ s3, const cpx<R>* __restrict__ d,
                                   const cpx<R>* __restrict__ Ad, const cpx<R>* __restrict__ r,
                                   cpx<R>* __restrict__ x, cpx<R>* __restrict__ rout, int64_t n, int ss, int cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    QMG_MEMBER_SCAL(s3); QMG_MEMBER_VEC(d); QMG_MEMBER_VEC(Ad); QMG_MEMBER_VEC(r); QMG_MEMBER_VEC(x);
    QMG_MEMBER_VEC(rout);
    const double den = s3[0], re = s3[1], im = s3[2];
    const bool ok = den > 0 && isfinite(den) && isfinite(re) && isfinite(im) && den - 2 * re < 0;
    const cpx<R> rr = r[i];
    if (!ok) {
        x[i] = cpx<R>{0, 0};
        rout[i] = rr;
        if (i == 0) s3[cnt] += 1.0;
        return;
    }
    const R ar = (R)(re / den), ai = (R)(im / den);
    const cpx<R> dd = d[i], a = Ad[i];
    x[i] = cpx<R>{ar * dd.re - ai * dd.im, ar * dd.im + ai * dd.re};
    rout[i] = cpx<R>{rr.re - (ar * a.re - ai * a.im), rr.im - (ar * a.im + ai * a.re)};
}

template <typename R>
__global__ void k_axpy(R a, const cpx<R>* __restrict__ x, cpx<R>* __restrict__ y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    QMG_MEMBER_VEC(x); QMG_MEMBER_VEC(y);
    y[i].re += a * x[i].re;
    y[i].im += a * x[i].im;
}

template <typename R>
__global__ void k_xmy(const cpx<R>* __restrict__ b, const cpx<R>* __restrict__ ax, cpx<R>* __restrict__ r, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    QMG_MEMBER_VEC(b); QMG_MEMBER_VEC(ax); QMG_MEMBER_VEC(r);
    r[i] = cpx<R>{b[i].re - ax[i].re, b[i].im - ax[i].im};
}

template <typename Rs, typename Rd>
__global__ void k_convert(const cpx<Rs>* __restrict__ s, cpx<Rd>* __restrict__ d, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    QMG_MEMBER_VEC(s); QMG_MEMBER_VEC(d);
    d[i] = cpx<Rd>{(Rd)s[i].re, (Rd)s[i].im};
}

template <typename R>
__global__ void k_normalize(cpx<R>* __restrict__ x, const double* __restrict__ nrm2, int64_t n, int ss) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    QMG_MEMBER_VEC(x); QMG_MEMBER_SCAL(nrm2);
    const R inv = (R)(1.0 / sqrt(nrm2[0]));
    x[i].re *= inv;
    x[i].im *= inv;
}

// Sums of per-thread values over the work-group, in a fixed order: each wave
// reduces by shuffles, then thread v adds the waves' partials in wave order.
// Slots v < nv (and slot 32 when with32) are summed into sc[v], visible to
// every thread on return.
__device__ __forceinline__ void wg_sums(const double* acc, int nv, bool with32, double (*part)[36], double* sc) {
    const int t = threadIdx.x, w = t >> 6, lane = t & 63, nw = blockDim.x >> 6;
#pragma unroll
    for (int v = 0; v < 36; ++v) {
        if (v < nv || (with32 && v == 32)) {
            double x = acc[v];
            for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
            if (lane == 0) part[w][v] = x;
        }
    }
    __syncthreads();
    if (t < nv || (with32 && t == 32)) {
        double x = 0;
        for (int i = 0; i < nw; ++i) x += part[i][t];
        sc[t] = x;
    }
    __syncthreads();
}

// One whole GCR step after q = A z, for short vectors, in a single work-group:
// classical Gram-Schmidt of (q, z) against the k stored pairs, repeated only
// when it cancelled most of q (|q'|^2 < |q|^2 / 2, the Daniel-Gragg-Kaufman-
// Stewart test: one pass is then not enough for orthogonality to working
// precision); the norms and <q', r> needed next are summed in the same sweep
// that updates q and z.  Then normalisation, x += alpha z, r -= alpha q, and
// |r|^2.  out = [<q,q>, <q,r>.re, <q,r>.im, |r|^2] (the first three for the
// orthogonalised q before normalisation).  When znext is given it receives r
// (the next step's unpreconditioned direction).  Common case: three sweeps
// over the vectors.
//
// Stopping test on the device: the step also writes ok = (<q,q> <= 0 or
// |r| <= tol |b|) (|b|^2 is read from out[bnoff]) and counts itself in
// out[okoff + 2].  The flags alternate between two slots: a launch with
// parity par reads every member's flag from out[okoff + par] (written by the
// previous launch, which has completed) and writes its own to
// out[okoff + 1 - par].  A launch that finds the flag set for every one of
// the nbm members returns at once, after carrying its member's flag forward,
// so the host can queue several steps and read the scalars only now and then:
// the steps after convergence change nothing, and whether a step runs is
// decided by the same data in every member's work-group.
//
// The number K of stored pairs is a template parameter, so every loop over
// them is unrolled with unconditional loads and a sweep keeps all of its
// loads in flight (a load under a run-time condition waits for the ones
// before it).
template <typename R, int K>
__global__ __launch_bounds__(512) void k_gcr_step_small(const cpx<R>* __restrict__ Q, const cpx<R>* __restrict__ Z,
                                                        int64_t ld, cpx<R>* __restrict__ q,
                                                        cpx<R>* __restrict__ z, cpx<R>* __restrict__ x,
                                                        cpx<R>* __restrict__ r, int64_t n, double* __restrict__ out,
                                                        cpx<R>* __restrict__ znext, int ss, double tol, int okoff,
                                                        int bnoff, int nbm, int par) {
    __shared__ double sc[36];
    __shared__ double part[16][36];
    {
        bool all = true;
        for (int b = 0; b < nbm; ++b) all = all && out[(int64_t)b * ss + okoff + par] != 0.0;
        if (all) {
            if (threadIdx.x == 0) out[(int64_t)blockIdx.y * ss + okoff + 1 - par] = 1.0;
            return;
        }
    }
    QMG_MEMBER_VEC(Q); QMG_MEMBER_VEC(Z); QMG_MEMBER_VEC(q); QMG_MEMBER_VEC(z); QMG_MEMBER_VEC(x);
    QMG_MEMBER_VEC(r); QMG_MEMBER_SCAL(out);
    if (znext) QMG_MEMBER_VEC(znext);
    const int t = threadIdx.x, T = blockDim.x;
    double acc[36];
    // sweep A: <Q_j, q> (j < K) and |q|^2
#pragma unroll
    for (int v = 0; v < 36; ++v) acc[v] = 0;
    for (int64_t i = t; i < n; i += T) {
        const cpx<R> b = q[i];
        acc[32] += (double)b.re * b.re + (double)b.im * b.im;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const cpx<R> a = Q[j * ld + i];
            acc[2 * j] += (double)a.re * b.re + (double)a.im * b.im;
            acc[2 * j + 1] += (double)a.re * b.im - (double)a.im * b.re;
        }
    }
    wg_sums(acc, 2 * K, true, part, sc);
    double qq0 = sc[32];
    double qq = qq0, re = 0, im = 0;
    for (int pass = 0; pass < 2; ++pass) {
        // sweep B: q -= sum beta_j Q_j, z -= sum beta_j Z_j (beta in sc), with |q'|^2 and <q', r>
        double n2 = 0, dr = 0, di = 0;
        for (int64_t i = t; i < n; i += T) {
            R qr = q[i].re, qi = q[i].im, zr = z[i].re, zi = z[i].im;
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const R br = (R)sc[2 * j], bi = (R)sc[2 * j + 1];
                const cpx<R> a = Q[j * ld + i], c = Z[j * ld + i];
                qr -= br * a.re - bi * a.im;
                qi -= br * a.im + bi * a.re;
                zr -= br * c.re - bi * c.im;
                zi -= br * c.im + bi * c.re;
            }
            q[i] = cpx<R>{qr, qi};
            z[i] = cpx<R>{zr, zi};
            const cpx<R> b = r[i];
            n2 += (double)qr * qr + (double)qi * qi;
            dr += (double)qr * b.re + (double)qi * b.im;
            di += (double)qr * b.im - (double)qi * b.re;
        }
        double a3[36];
        a3[0] = n2; a3[1] = dr; a3[2] = di;
        __syncthreads();   // every thread has read sc (the betas) before it is overwritten
        wg_sums(a3, 3, false, part, sc);
        qq = sc[0]; re = sc[1]; im = sc[2];
        if (pass == 1 || K == 0 || !(qq < 0.5 * qq0)) break;
        // the projection cancelled most of q: orthogonalise once more (sweep A again, dots only)
        qq0 = qq;
#pragma unroll
        for (int v = 0; v < 36; ++v) acc[v] = 0;
        for (int64_t i = t; i < n; i += T) {
            const cpx<R> b = q[i];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const cpx<R> a = Q[j * ld + i];
                acc[2 * j] += (double)a.re * b.re + (double)a.im * b.im;
                acc[2 * j + 1] += (double)a.re * b.im - (double)a.im * b.re;
            }
        }
        __syncthreads();
        wg_sums(acc, 2 * K, false, part, sc);
    }
    double rr = 0;
    if (qq > 0) {
        const double nq = sqrt(qq);
        const R inv = (R)(1.0 / nq), ar = (R)(re / nq), ai = (R)(im / nq);
        for (int64_t i = t; i < n; i += T) {
            cpx<R> a = q[i], c = z[i], xx = x[i], b = r[i];
            a.re *= inv; a.im *= inv;
            c.re *= inv; c.im *= inv;
            xx.re += ar * c.re - ai * c.im;
            xx.im += ar * c.im + ai * c.re;
            b.re -= ar * a.re - ai * a.im;
            b.im -= ar * a.im + ai * a.re;
            q[i] = a;
            z[i] = c;
            x[i] = xx;
            r[i] = b;
            if (znext) znext[i] = b;
            rr += (double)b.re * b.re + (double)b.im * b.im;
        }
    } else {
        for (int64_t i = t; i < n; i += T) {
            const cpx<R> b = r[i];
            if (znext) znext[i] = b;
            rr += (double)b.re * b.re + (double)b.im * b.im;
        }
    }
    double a1[36];
    a1[0] = rr;
    __syncthreads();
    wg_sums(a1, 1, false, part, sc);
    if (t == 0) {
        out[0] = qq;
        out[1] = re;
        out[2] = im;
        out[3] = sc[0];
        const double bn = sqrt(out[bnoff]);
        out[okoff + 1 - par] = (qq <= 0.0 || (bn > 0 && sqrt(sc[0]) <= tol * bn)) ? 1.0 : 0.0;
        out[okoff + 2] += 1.0;
    }
}

// The same step with its operands held in registers, for FP32 vectors of at
// most E * 512 entries: thread t owns the E entries t + e T (e < E); its loads
// of q, z, x, r and the stored Q_j are issued together at the start and those
// of the Z_j together once q is projected, so the step waits on memory about
// twice rather than once per entry and sweep.  Lanes past n read entry n - 1,
// scaled to zero, so they add nothing to any sum and store nothing.  Each
// stored pair costs about 7 E registers: E = 2 takes up to 9 pairs (restart
// length 10) in 256 registers, E = 4 up to 4.
template <int K, int E>
__global__ __launch_bounds__(512) void k_gcr_step_reg(const cpx<float>* __restrict__ Q,
                                                      const cpx<float>* __restrict__ Z, int64_t ld,
                                                      cpx<float>* __restrict__ q, cpx<float>* __restrict__ z,
                                                      cpx<float>* __restrict__ x, cpx<float>* __restrict__ r,
                                                      int64_t n, double* __restrict__ out,
                                                      cpx<float>* __restrict__ znext, int ss, double tol, int okoff,
                                                      int bnoff, int nbm, int par) {
    constexpr int KA = K > 0 ? K : 1;
    __shared__ double sc[36];
    __shared__ double part[16][36];
    {
        bool all = true;
        for (int b = 0; b < nbm; ++b) all = all && out[(int64_t)b * ss + okoff + par] != 0.0;
        if (all) {
            if (threadIdx.x == 0) out[(int64_t)blockIdx.y * ss + okoff + 1 - par] = 1.0;
            return;
        }
    }
    QMG_MEMBER_VEC(Q); QMG_MEMBER_VEC(Z); QMG_MEMBER_VEC(q); QMG_MEMBER_VEC(z); QMG_MEMBER_VEC(x);
    QMG_MEMBER_VEC(r); QMG_MEMBER_SCAL(out);
    if (znext) QMG_MEMBER_VEC(znext);
    const int t = threadIdx.x, T = blockDim.x;
    int64_t id[E];
    float live[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int64_t i = t + (int64_t)e * T;
        live[e] = i < n ? 1.0f : 0.0f;
        id[e] = i < n ? i : n - 1;
    }
    cpx<float> qv[E], zv[E], xv[E], rv[E], Qv[KA][E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        qv[e] = q[id[e]];
        zv[e] = z[id[e]];
        rv[e] = r[id[e]];
        xv[e] = x[id[e]];
    }
#pragma unroll
    for (int j = 0; j < K; ++j)
#pragma unroll
        for (int e = 0; e < E; ++e) Qv[j][e] = Q[j * ld + id[e]];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        qv[e] = {qv[e].re * live[e], qv[e].im * live[e]};
        zv[e] = {zv[e].re * live[e], zv[e].im * live[e]};
        rv[e] = {rv[e].re * live[e], rv[e].im * live[e]};
#pragma unroll
        for (int j = 0; j < K; ++j) Qv[j][e] = {Qv[j][e].re * live[e], Qv[j][e].im * live[e]};
    }
    // sweep A: <Q_j, q> and |q|^2
    double acc[36];
#pragma unroll
    for (int v = 0; v < 36; ++v) acc[v] = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const cpx<float> b = qv[e];
        acc[32] += (double)b.re * b.re + (double)b.im * b.im;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const cpx<float> a = Qv[j][e];
            acc[2 * j] += (double)a.re * b.re + (double)a.im * b.im;
            acc[2 * j + 1] += (double)a.re * b.im - (double)a.im * b.re;
        }
    }
    wg_sums(acc, 2 * K, true, part, sc);
    double qq0 = sc[32];
    double qq = qq0, re = 0, im = 0;
    for (int pass = 0; pass < 2; ++pass) {
        // sweep B: q -= sum beta_j Q_j, z -= sum beta_j Z_j, with |q'|^2 and <q', r>
        // (every thread reads the betas before any thread enters the next sum)
        float br[KA], bi[KA];
#pragma unroll
        for (int j = 0; j < K; ++j) { br[j] = (float)sc[2 * j]; bi[j] = (float)sc[2 * j + 1]; }
        double n2 = 0, dr = 0, di = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            float qr = qv[e].re, qi = qv[e].im;
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const cpx<float> a = Qv[j][e];
                qr -= br[j] * a.re - bi[j] * a.im;
                qi -= br[j] * a.im + bi[j] * a.re;
            }
            qv[e] = {qr, qi};
            const cpx<float> b = rv[e];
            n2 += (double)qr * qr + (double)qi * qi;
            dr += (double)qr * b.re + (double)qi * b.im;
            di += (double)qr * b.im - (double)qi * b.re;
        }
        {
            cpx<float> Zv[KA][E];
#pragma unroll
            for (int j = 0; j < K; ++j)
#pragma unroll
                for (int e = 0; e < E; ++e) Zv[j][e] = Z[j * ld + id[e]];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                float zr = zv[e].re, zi = zv[e].im;
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    const cpx<float> c = {Zv[j][e].re * live[e], Zv[j][e].im * live[e]};
                    zr -= br[j] * c.re - bi[j] * c.im;
                    zi -= br[j] * c.im + bi[j] * c.re;
                }
                zv[e] = {zr, zi};
            }
        }
        double a3[36];
        a3[0] = n2; a3[1] = dr; a3[2] = di;
        wg_sums(a3, 3, false, part, sc);
        qq = sc[0]; re = sc[1]; im = sc[2];
        if (pass == 1 || K == 0 || !(qq < 0.5 * qq0)) break;
        // the projection cancelled most of q: orthogonalise once more (dots
        // only), with the stored Q_j read again rather than kept live
        qq0 = qq;
        asm volatile("" ::: "memory");
#pragma unroll
        for (int j = 0; j < K; ++j)
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const cpx<float> a = Q[j * ld + id[e]];
                Qv[j][e] = {a.re * live[e], a.im * live[e]};
            }
#pragma unroll
        for (int v = 0; v < 36; ++v) acc[v] = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const cpx<float> b = qv[e];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const cpx<float> a = Qv[j][e];
                acc[2 * j] += (double)a.re * b.re + (double)a.im * b.im;
                acc[2 * j + 1] += (double)a.re * b.im - (double)a.im * b.re;
            }
        }
        __syncthreads();   // every thread has read sc (qq, re, im) before it is overwritten
        wg_sums(acc, 2 * K, false, part, sc);
    }
    double rr = 0;
    if (qq > 0) {
        const double nq = sqrt(qq);
        const float inv = (float)(1.0 / nq), ar = (float)(re / nq), ai = (float)(im / nq);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            cpx<float> a = qv[e], c = zv[e], xx = xv[e], b = rv[e];
            a.re *= inv; a.im *= inv;
            c.re *= inv; c.im *= inv;
            xx.re += ar * c.re - ai * c.im;
            xx.im += ar * c.im + ai * c.re;
            b.re -= ar * a.re - ai * a.im;
            b.im -= ar * a.im + ai * a.re;
            if (live[e] != 0.0f) {
                q[id[e]] = a;
                z[id[e]] = c;
                x[id[e]] = xx;
                r[id[e]] = b;
                if (znext) znext[id[e]] = b;
            }
            rr += (double)b.re * b.re + (double)b.im * b.im;
        }
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const cpx<float> b = rv[e];
            if (live[e] != 0.0f && znext) znext[id[e]] = b;
            rr += (double)b.re * b.re + (double)b.im * b.im;
        }
    }
    double a1[36];
    a1[0] = rr;
    __syncthreads();
    wg_sums(a1, 1, false, part, sc);
    if (t == 0) {
        out[0] = qq;
        out[1] = re;
        out[2] = im;
        out[3] = sc[0];
        const double bn = sqrt(out[bnoff]);
        out[okoff + 1 - par] = (qq <= 0.0 || (bn > 0 && sqrt(sc[0]) <= tol * bn)) ? 1.0 : 0.0;
        out[okoff + 2] += 1.0;
    }
}

// 512 threads: faster than 1024 or 256 on the 2048-unknown coarsest level of
// 16^3x32 (42.5 vs 44.0 and 45.7 ms per MG solve)
template <typename R>
qmg_status Blas::gcr_step_small(const void* Q, const void* Z, int64_t ld, int k, void* q, void* z, void* x, void* r,
                                int64_t n, double* out, void* znext, double tol, int okoff, int bnoff, int par) {
    if (k < 0 || k > 15) return fail(QMG_ERR_ARG, "gcr_step_small: %d stored directions (at most 15)", k);
    if constexpr (std::is_same<R, float>::value) {
        const int E = n <= 1024 && k <= 9 ? 2 : n <= 2048 && k <= 4 ? 4 : 0;
        if (E) {
            // E entries per thread, whole waves, at most 512 threads
            const int T = (int)std::min<int64_t>(512, std::max<int64_t>(64, ((n + E - 1) / E + 63) / 64 * 64));
#define QMG_STEP_REG(KK, EE)                                                                                         \
    case KK:                                                                                                         \
        hipLaunchKernelGGL((k_gcr_step_reg<KK, EE>), dim3(1, nb), dim3(T), 0, s, (const cpx<float>*)Q,              \
                           (const cpx<float>*)Z, ld, (cpx<float>*)q, (cpx<float>*)z, (cpx<float>*)x, (cpx<float>*)r, \
                           n, out, (cpx<float>*)znext, ss, tol, okoff, bnoff, nb, par);                              \
        break;
            if (E == 2) {
                switch (k) {
                    QMG_STEP_REG(0, 2) QMG_STEP_REG(1, 2) QMG_STEP_REG(2, 2) QMG_STEP_REG(3, 2) QMG_STEP_REG(4, 2)
                    QMG_STEP_REG(5, 2) QMG_STEP_REG(6, 2) QMG_STEP_REG(7, 2) QMG_STEP_REG(8, 2) QMG_STEP_REG(9, 2)
                }
            } else {
                switch (k) {
                    QMG_STEP_REG(0, 4) QMG_STEP_REG(1, 4) QMG_STEP_REG(2, 4) QMG_STEP_REG(3, 4) QMG_STEP_REG(4, 4)
                }
            }
#undef QMG_STEP_REG
            QMG_LAUNCH_CHECK();
            return QMG_OK;
        }
    }
#define QMG_STEP(KK)                                                                                                 \
    case KK:                                                                                                         \
        hipLaunchKernelGGL((k_gcr_step_small<R, KK>), dim3(1, nb), dim3(512), 0, s, (const cpx<R>*)Q,               \
                           (const cpx<R>*)Z, ld, (cpx<R>*)q, (cpx<R>*)z, (cpx<R>*)x, (cpx<R>*)r, n, out,            \
                           (cpx<R>*)znext, ss, tol, okoff, bnoff, nb, par);                                         \
        break;
    switch (k) {
        QMG_STEP(0) QMG_STEP(1) QMG_STEP(2) QMG_STEP(3) QMG_STEP(4) QMG_STEP(5) QMG_STEP(6) QMG_STEP(7)
        QMG_STEP(8) QMG_STEP(9) QMG_STEP(10) QMG_STEP(11) QMG_STEP(12) QMG_STEP(13) QMG_STEP(14) QMG_STEP(15)
    }
#undef QMG_STEP
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

qmg_status Blas::init() {
    if (partials) return QMG_OK;
    QMG_HIP(hipMalloc(&partials, sizeof(double) * kMaxBatch * kMaxBlocks * kMaxVals));
    return QMG_OK;
}

void Blas::release() {
    if (partials) (void)hipFree(partials);
    partials = nullptr;
}

static unsigned grid1(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

static void finish(hipStream_t s, double* partials, int nblk, int nv, double* out, int members, int ss) {
    if (nblk > 1) hipLaunchKernelGGL(k_final, dim3(1, members), dim3(256), 0, s, partials, nblk, nv, out, ss);
}

qmg_status Blas::final_sum(int groups, int nv, double* out) {
    if (groups < 1 || groups > kMaxBlocks || nv < 1 || nv > kMaxVals)
        return fail(QMG_ERR_ARG, "final_sum: %d groups, %d values", groups, nv);
    hipLaunchKernelGGL(k_final, dim3(1, nb), dim3(256), 0, s, partials, groups, nv, out, ss);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

template <typename R> qmg_status Blas::dot(const void* a, const void* b, int64_t n, double* out) {
    const int nblk = nblocks(n);
    hipLaunchKernelGGL(k_dot<R>, dim3(nblk, nb), dim3(rthreads(nblk)), 0, s, (const cpx<R>*)a, (const cpx<R>*)b, n,
                       partials, out, ss);
    finish(s, partials, nblk, 2, out, nb, ss);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}
template <typename R> qmg_status Blas::norm2(const void* a, int64_t n, double* out) {
    const int nblk = nblocks(n);
    hipLaunchKernelGGL(k_norm2<R>, dim3(nblk, nb), dim3(rthreads(nblk)), 0, s, (const cpx<R>*)a, n, partials, out, ss);
    finish(s, partials, nblk, 1, out, nb, ss);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}
template <typename R> qmg_status Blas::dot_norm(const void* q, const void* r, int64_t n, double* out) {
    const int nblk = nblocks(n);
    hipLaunchKernelGGL(k_dot_norm<R>, dim3(nblk, nb), dim3(rthreads(nblk)), 0, s, (const cpx<R>*)q, (const cpx<R>*)r, n,
                       partials, out, ss);
    finish(s, partials, nblk, 3, out, nb, ss);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}
template <typename R>
qmg_status Blas::multi_dot(const void* Q, int64_t ld, int k, const void* q, int64_t n, double* out) {
    if (k <= 0) return QMG_OK;
    if (k > 16) return fail(QMG_ERR_ARG, "multi_dot: k=%d > 16", k);
    const int nblk = nblocks(n);
    hipLaunchKernelGGL(k_multi_dot<R>, dim3(nblk, nb), dim3(rthreads(nblk)), 0, s, (const cpx<R>*)Q, ld, k,
                       (const cpx<R>*)q, n, partials, out, ss);
    finish(s, partials, nblk, 2 * k, out, nb, ss);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}
template <typename R>
qmg_status Blas::multi_axpy(const double* beta, const void* Q, const void* Z, int64_t ld, int k, void* q, void* z,
                            int64_t n) {
    if (k <= 0) return QMG_OK;
    hipLaunchKernelGGL(k_multi_axpy<R>, dim3(grid1(n), nb), dim3(kThreads), 0, s, beta, (const cpx<R>*)Q,
                       (const cpx<R>*)Z, ld, k, (cpx<R>*)q, (cpx<R>*)z, n, ss);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}
template <typename R>
qmg_status Blas::gcr_update(const double* s3, void* q, void* z, void* x, void* r, int64_t n) {
    hipLaunchKernelGGL(k_gcr_update<R>, dim3(grid1(n), nb), dim3(kThreads), 0, s, s3, (cpx<R>*)q, (cpx<R>*)z,
                       (cpx<R>*)x, (cpx<R>*)r, n, ss);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}
template <typename R>
qmg_status Blas::mr_update(const double* s3, const void* rin, void* r, const void* Ar, void* x, int first, int64_t n) {
    hipLaunchKernelGGL(k_mr_update<R>, dim3((grid1(n) + 7) / 8 * 8, nb), dim3(kThreads), 0, s, s3, (const cpx<R>*)rin,
                       (cpx<R>*)r, (const cpx<R>*)Ar, (cpx<R>*)x, first, n, ss);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}
qmg_status Blas::dot_norm_h16(const void* q, const float* qs, const void* r, const float* rs, int64_t nsites,
                              double* out) {
    const int nblk = nblocks(nsites * 4);   // four lanes per site
    hipLaunchKernelGGL(k_dot_norm_h16, dim3(nblk, nb), dim3(rthreads(nblk)), 0, s, (const uint32_t*)q, qs,
                       (const uint32_t*)r, rs, nsites, partials, out, ss);
    finish(s, partials, nblk, 3, out, nb, ss);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}
qmg_status Blas::mr_update_h16(const double* s3, const void* rin, const float* rins, void* r, float* rs, const void* Ar,
                               const float* Ars, void* x, int first, int64_t nsites) {
    static_assert(kThreads == 256, "k_mr_update_h16 takes 64 sites per 256-lane work-group");
    const int64_t groups = (nsites + kMrSites - 1) / kMrSites;
    hipLaunchKernelGGL(k_mr_update_h16, dim3((unsigned)((groups + 7) / 8 * 8), nb), dim3(kThreads), 0, s, s3,
                       (const uint32_t*)rin, rins, (uint32_t*)r, rs, (const uint32_t*)Ar, Ars, (float2*)x, first, nsites,
                       ss);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

qmg_status Blas::quantize_spinors(const void* in, void* out, float* scale, int64_t nsites) {
    unsigned* nf = nullptr;
    QMG_TRY(nonfinite_flag(&nf));
    hipLaunchKernelGGL(k_quantize_spinor, dim3(grid1(nsites * 4)), dim3(kThreads), 0, s, (const float2*)in,
                       (uint32_t*)out, scale, nsites, nf);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}
qmg_status Blas::scatter_dequantize(const void* in, const float* scale, const int* hp, const int* hq, void* full,
                                    int64_t nsites) {
    hipLaunchKernelGGL(k_scatter_dequantize, dim3(grid1(nsites * 4), nb), dim3(kThreads), 0, s, (const uint32_t*)in,
                       scale, hp, hq, (float2*)full, nsites);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

template <typename R>
qmg_status Blas::dir_step(const double* s3, const void* d, const void* Ad, const void* r, void* x, void* rout,
                          int64_t n) {
    hipLaunchKernelGGL(k_dir_step<R>, dim3(grid1(n), nb), dim3(kThreads), 0, s, s3, (const cpx<R>*)d,
                       (const cpx<R>*)Ad, (const cpx<R>*)r, (cpx<R>*)x, (cpx<R>*)rout, n, ss);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

template <typename R>
qmg_status Blas::dir_step_checked(double* s3, const void* d, const void* Ad, const void* r, void* x, void* rout,
                                  int64_t n, int cnt) {
    hipLaunchKernelGGL(k_dir_step_checked<R>, dim3(grid1(n), nb), dim3(kThreads), 0, s, s3, (const cpx<R>*)d,
                       (const cpx<R>*)Ad, (const cpx<R>*)r, (cpx<R>*)x, (cpx<R>*)rout, n, ss, cnt);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

template <typename R> qmg_status Blas::axpy(double a, const void* x, void* y, int64_t n) {
    hipLaunchKernelGGL(k_axpy<R>, dim3(grid1(n), nb), dim3(kThreads), 0, s, (R)a, (const cpx<R>*)x, (cpx<R>*)y, n);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}
template <typename R> qmg_status Blas::xmy(const void* b, const void* ax, void* r, int64_t n) {
    hipLaunchKernelGGL(k_xmy<R>, dim3(grid1(n), nb), dim3(kThreads), 0, s, (const cpx<R>*)b, (const cpx<R>*)ax,
                       (cpx<R>*)r, n);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}
template <typename Rs, typename Rd> qmg_status Blas::convert(const void* src, void* dst, int64_t n) {
    hipLaunchKernelGGL((k_convert<Rs, Rd>), dim3(grid1(n), nb), dim3(kThreads), 0, s, (const cpx<Rs>*)src,
                       (cpx<Rd>*)dst, n);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}
template <typename R> qmg_status Blas::normalize(void* x, const double* nrm2, int64_t n) {
    hipLaunchKernelGGL(k_normalize<R>, dim3(grid1(n), nb), dim3(kThreads), 0, s, (cpx<R>*)x, nrm2, n, ss);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

#define QMG_BLAS_INST(R)                                                                                   \
    template qmg_status Blas::dot<R>(const void*, const void*, int64_t, double*);                          \
    template qmg_status Blas::norm2<R>(const void*, int64_t, double*);                                     \
    template qmg_status Blas::dot_norm<R>(const void*, const void*, int64_t, double*);                     \
    template qmg_status Blas::multi_dot<R>(const void*, int64_t, int, const void*, int64_t, double*);      \
    template qmg_status Blas::multi_axpy<R>(const double*, const void*, const void*, int64_t, int, void*, \
                                            void*, int64_t);                                               \
    template qmg_status Blas::gcr_update<R>(const double*, void*, void*, void*, void*, int64_t);           \
    template qmg_status Blas::mr_update<R>(const double*, const void*, void*, const void*, void*, int, int64_t); \
    template qmg_status Blas::axpy<R>(double, const void*, void*, int64_t);                                \
    template qmg_status Blas::dir_step<R>(const double*, const void*, const void*, const void*, void*, void*, \
                                          int64_t);                                                        \
    template qmg_status Blas::dir_step_checked<R>(double*, const void*, const void*, const void*, void*,     \
                                                  void*, int64_t, int);                                    \
    template qmg_status Blas::xmy<R>(const void*, const void*, void*, int64_t);                            \
    template qmg_status Blas::normalize<R>(void*, const double*, int64_t);                                 \
    template qmg_status Blas::gcr_step_small<R>(const void*, const void*, int64_t, int, void*, void*, void*,  \
                                                void*, int64_t, double*, void*, double, int, int, int);

QMG_BLAS_INST(double)
QMG_BLAS_INST(float)
template qmg_status Blas::convert<double, float>(const void*, void*, int64_t);
template qmg_status Blas::convert<float, double>(const void*, void*, int64_t);
template qmg_status Blas::convert<double, double>(const void*, void*, int64_t);
template qmg_status Blas::convert<float, float>(const void*, void*, int64_t);

}  // namespace qmg
