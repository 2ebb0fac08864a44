// Device helpers of the fine Wilson-clover operator, Eq. (2), shared by the
// whole-lattice and red-black kernels (wilson.hip) and the Schwarz smoother
// (sap.hip): complex arithmetic, the chiral-basis gamma blocks, link, clover
// and spinor loads in every storage format, and the projected hop.
#pragma once

#include "codes16.h"
#include "handles.h"

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

template <int LF> struct FineT { using R = float; };
template <> struct FineT<FMT_F64> { using R = double; };
template <int F> constexpr bool is16f() { return F == FMT_H16 || F == FMT_B16; }

// Link U_mu at lattice index ls.  LR = 18: all nine entries stored, [4][9][V];
// LR = 12 (compressed): rows 0 and 1 stored, [4][6][V], and row 2 rebuilt from
// them, since for an SU(3) matrix each row is the complex conjugate of the
// cross product of the other two: c = conj(a x b).  The antiperiodic time
// sign is folded into the stored rows, and the rebuilt row takes it from the
// link's position (mu = 3 on the last time slice, ls >= last).
// load_link_at reads the link stored at index `idx` of a [4][ne][V] array
// (lattice order, or the red-black copy in parity order) and takes the time
// sign of a rebuilt row from `neg`; NT marks a once-per-application read.
template <int LF, int LR = 18, bool NT = false, typename R>
__device__ __forceinline__ void load_link_at(cpx<R> u[9], const void* __restrict__ U, int mu, int64_t idx, int64_t V,
                                             bool neg) {
    constexpr int ne = LR == 12 ? 6 : 9;
    if constexpr (is16f<LF>()) {
        const uint32_t* W = static_cast<const uint32_t*>(U);
#pragma unroll
        for (int e = 0; e < ne; ++e) {
            const uint32_t* a = W + ((int64_t)mu * ne + e) * V + idx;
            u[e] = dec_pair<LF>(NT ? __builtin_nontemporal_load(a) : *a);
        }
    } else {
        const cpx<R>* P = static_cast<const cpx<R>*>(U);
#pragma unroll
        for (int e = 0; e < ne; ++e) {
            const cpx<R>* a = P + ((int64_t)mu * ne + e) * V + idx;
            if constexpr (NT) {
                typedef R v2 __attribute__((ext_vector_type(2)));   // one 8- or 16-byte load (elements are so aligned)
                const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(a));
                u[e] = cpx<R>{v.x, v.y};
            } else {
                u[e] = *a;
            }
        }
    }
    if constexpr (LR == 12) {
        const R sg = neg ? R(-1) : R(1);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int k = (j + 1) % 3, l = (j + 2) % 3;
            // conj(a_k b_l - a_l b_k)
            const R re = (u[k].re * u[3 + l].re - u[k].im * u[3 + l].im) - (u[l].re * u[3 + k].re - u[l].im * u[3 + k].im);
            const R im = (u[k].re * u[3 + l].im + u[k].im * u[3 + l].re) - (u[l].re * u[3 + k].im + u[l].im * u[3 + k].re);
            u[6 + j] = cpx<R>{sg * re, -sg * im};
        }
    }
}

template <int LF, int LR = 18, typename R>
__device__ __forceinline__ void load_link(cpx<R> u[9], const void* __restrict__ U, int mu, int64_t ls, int64_t V,
                                          int64_t last = 0) {
    load_link_at<LF, LR, false>(u, U, mu, ls, V, mu == 3 && ls >= last);
}

// One chirality block of the clover term: 6 diagonal reals, 15 upper entries.
// Each site's block is read once per application: non-temporal loads, so it
// does not push the spinors and links that neighbouring sites share out of
// the caches.
template <int LF, typename R>
__device__ __forceinline__ void load_clover(R d[6], cpx<R> o[15], const void* __restrict__ clov,
                                            const float* __restrict__ cscale, int chi, int64_t site, int64_t V) {
    if constexpr (is16f<LF>()) {
        const uint32_t* W = static_cast<const uint32_t*>(clov) + (int64_t)chi * 18 * V + site;
        const float k = cscale[(int64_t)chi * V + site];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const cpx<float> v = dec_pair<LF>(__builtin_nontemporal_load(W + q * V));
            d[2 * q] = k * v.re;
            d[2 * q + 1] = k * v.im;
        }
#pragma unroll
        for (int q = 0; q < 15; ++q) {
            const cpx<float> v = dec_pair<LF>(__builtin_nontemporal_load(W + (3 + q) * V));
            o[q] = {k * v.re, k * v.im};
        }
    } else {
        const R* A = static_cast<const R*>(clov) + (int64_t)chi * 36 * V + site;
#pragma unroll
        for (int i = 0; i < 6; ++i) d[i] = __builtin_nontemporal_load(A + i * V);
#pragma unroll
        for (int q = 0; q < 15; ++q)
            o[q] = {__builtin_nontemporal_load(A + (6 + 2 * q) * V), __builtin_nontemporal_load(A + (7 + 2 * q) * V)};
    }
}

// acc += H x for a site-local matrix H stored as two packed Hermitian 6x6
// chirality blocks (the clover term, or the inverse of the site-local block).
template <int LF, typename R>
__device__ __forceinline__ void herm_mul_add(cpx<R> acc[12], const cpx<R> x12[12], const void* __restrict__ H,
                                             const float* __restrict__ hscale, int64_t site, int64_t V) {
#pragma unroll
    for (int chi = 0; chi < 2; ++chi) {
        R d[6];
        cpx<R> o[15];
        load_clover<LF>(d, o, H, hscale, chi, site, V);
        const cpx<R>* x = x12 + 6 * chi;
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

// A site's 12 spinor components, with 16-byte loads (3 for 16-bit pairs, 6 in
// FP32, 12 in FP64).
template <int VF, typename R>
__device__ __forceinline__ void load_spinor(cpx<R> p[12], const void* __restrict__ src,
                                            const float* __restrict__ scale, int64_t site) {
    if constexpr (is16f<VF>()) {
        const uint4* s4 = static_cast<const uint4*>(src) + site * 3;
        const float k = scale[site];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const uint4 w = s4[i];
            const uint32_t q[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const cpx<float> v = dec_pair<VF>(q[j]);
                p[4 * i + j] = cpx<R>{k * v.re, k * v.im};
            }
        }
    } else if constexpr (VF == FMT_F32) {
        const float4* s4 = static_cast<const float4*>(src) + site * 6;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            const float4 v = s4[i];
            p[2 * i] = cpx<R>{v.x, v.y};
            p[2 * i + 1] = cpx<R>{v.z, v.w};
        }
    } else {
        const cpx<R>* s = static_cast<const cpx<R>*>(src) + site * 12;
#pragma unroll
        for (int f = 0; f < 12; ++f) p[f] = s[f];
    }
}

template <int VF, typename R>
__device__ __forceinline__ void store_spinor(void* __restrict__ dst, float* __restrict__ scale, int64_t site,
                                             const cpx<R> p[12]) {
    if constexpr (is16f<VF>()) {
        float m = 0.0f;
#pragma unroll
        for (int f = 0; f < 12; ++f) m = fmaxf(m, fmaxf(fabsf(p[f].re), fabsf(p[f].im)));
        const float inv = m > 0.0f ? 1.0f / m : 0.0f;
        uint4* d4 = static_cast<uint4*>(dst) + site * 3;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            uint32_t q[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) q[j] = enc_pair<VF>(p[4 * i + j].re * inv, p[4 * i + j].im * inv);
            d4[i] = make_uint4(q[0], q[1], q[2], q[3]);
        }
        scale[site] = m;
    } else if constexpr (VF == FMT_F32) {
        float4* d4 = static_cast<float4*>(dst) + site * 6;
#pragma unroll
        for (int i = 0; i < 6; ++i) d4[i] = make_float4(p[2 * i].re, p[2 * i].im, p[2 * i + 1].re, p[2 * i + 1].im);
    } else {
        cpx<R>* d = static_cast<cpx<R>*>(dst) + site * 12;
#pragma unroll
        for (int f = 0; f < 12; ++f) d[f] = p[f];
    }
}

// One hop in direction MU; BACK selects the backward hop: the operands of
// acc += -1/2 * P (x) W psi(n).  vo: offset (in sites) of the batch member's vectors
template <int MU, bool BACK, int LF, int VF, int LR = 18, typename R>
__device__ __forceinline__ void hop_load(cpx<R> p[12], cpx<R> u[9], const void* __restrict__ in,
                                         const float* __restrict__ in_scale, const void* __restrict__ U, int64_t V,
                                         int64_t site, int64_t n, int64_t vo, int64_t last) {
    load_spinor<VF>(p, in, in_scale, n + vo);
    load_link<LF, LR>(u, U, MU, BACK ? n : site, V, last);
}

// acc += h * P (x) W psi(n): h = -1/2 is the hop term of Eq. (2)
template <int MU, bool BACK, typename R>
__device__ __forceinline__ void hop_apply(cpx<R> acc[12], const cpx<R> p[12], const cpx<R> u[9], const R h = R(-0.5)) {
    cpx<R> a[2][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cpx<R> g0, g1;
        gmul<MU>(g0, g1, p[6 + c], p[9 + c]);
        if (!BACK) { a[0][c] = csub(p[c], g0); a[1][c] = csub(p[3 + c], g1); }
        else { a[0][c] = cadd(p[c], g0); a[1][c] = cadd(p[3 + c], g1); }
    }
    cpx<R> w[2][3];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            cpx<R> t = {0, 0};
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (!BACK) t = cadd(t, cmul(u[r * 3 + c], a[s][c]));
                else t = cadd(t, cmulc(u[c * 3 + r], a[s][c]));
            }
            w[s][r] = t;
        }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cpx<R> l0, l1;
        gdmul<MU>(l0, l1, w[0][c], w[1][c]);
        acc[c].re += h * w[0][c].re; acc[c].im += h * w[0][c].im;
        acc[3 + c].re += h * w[1][c].re; acc[3 + c].im += h * w[1][c].im;
        if (!BACK) { l0 = cneg(l0); l1 = cneg(l1); }
        acc[6 + c].re += h * l0.re; acc[6 + c].im += h * l0.im;
        acc[9 + c].re += h * l1.re; acc[9 + c].im += h * l1.im;
    }
}

}  // namespace qmg
