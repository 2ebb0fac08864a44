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
//
// 16-bit storage (FP16 or BF16 pairs, FP32 arithmetic): the links as one pair
// per complex entry, [4][9][V] words, with no scale (SU(3) entries are
// bounded by 1 in magnitude); the clover term as [2][18][V] words (pair q of
// a chirality block holds its reals 2q and 2q+1 of the layout above) with one
// FP32 scale per (chirality, site), value = scale * stored.  Vectors are then
// either complex64 or 16-bit pairs [V][12] words with one FP32 scale per site
// (the largest |re| or |im| of its 12 components).
#include "wilson_dev.h"

#include <mutex>
#include <vector>

namespace qmg {

// LF: storage of links and clover; VF: storage of the vectors (the same as LF
// for complex128 / complex64, complex64 or 16-bit pairs for 16-bit links).
// Grid dimension y runs over batch members: member b's fields follow the
// first at b*V sites.
// DOT: also the minimal-residual step's inner products of the result with
// the input, <out,out> and <out,in> (re, im), summed over the work-group in
// FP64 (fixed order) into part[member*pmember + value*pvalue + blockIdx.x].
// LR: stored reals per link (18, or 12 with the third row rebuilt).
//
// Order of the work and reuse of the input.  A work-group covers 256
// consecutive sites.  When they are whole x-y planes (NEAR = 2) it first reads
// their input spinors (decoded) into LDS, then takes the t and z hops, whose
// neighbours belong to other work-groups that read them as their own sites at
// the same time, so the second request finds them in L2; then the clover
// term; then the x and y hops, whose neighbours come from LDS.  Taken in
// lattice order, the z and t neighbours were fetched again once the clover
// and link streams had pushed them out of L2: on 16^3x32 the order above
// reads 829 instead of 942 bytes per site (1.20x instead of 1.35x the
// algorithmic bytes, counters), at the same time per launch (the kernel is
// one wave of work-groups there, bound by its memory latency).  Without
// whole planes the hops are taken in lattice order, two in flight (taking t
// and z first without the LDS copy was measured slower: 154 vs 136 us on
// 24^3x48).
constexpr int kWilsonSites = 256;

template <typename R>
__device__ __forceinline__ void lds_put(cpx<R>* sh, int t, const cpx<R> p[12]) {
#pragma unroll
    for (int f = 0; f < 12; ++f) sh[f * kWilsonSites + t] = p[f];
}
// The x and y hops of site n.  NEAR = 2: the work-group's range
// [base, base + kWilsonSites) holds whole x-y planes (L0 L1 divides
// kWilsonSites), so the x and y neighbours lie in it and their spinors are
// read from the LDS copy; otherwise from memory.
template <int NEAR, int MU, bool BACK, int LF, int VF, int LR, typename R>
__device__ __forceinline__ void hop_load_near(cpx<R> p[12], cpx<R> u[9], const cpx<R>* sh,
                                              const void* __restrict__ in, const float* __restrict__ in_scale,
                                              const void* __restrict__ U, int64_t V, int64_t site, int64_t n,
                                              int64_t base, int64_t vo, int64_t last) {
    if constexpr (NEAR > MU) {
        const int j = (int)(n - base);
#pragma unroll
        for (int f = 0; f < 12; ++f) p[f] = sh[f * kWilsonSites + j];
    } else {
        load_spinor<VF>(p, in, in_scale, n + vo);
    }
    load_link<LF, LR>(u, U, MU, BACK ? n : site, V, last);
}

template <int LF, int VF, bool DOT = false, int LR = 18, int NEAR = 0>
__global__ __launch_bounds__(256) void k_wilson_clover(const void* __restrict__ U, const void* __restrict__ clov,
                                                       const float* __restrict__ cscale,
                                                       const int* __restrict__ nbr, const void* __restrict__ in,
                                                       const float* __restrict__ in_scale, void* __restrict__ out,
                                                       float* __restrict__ out_scale, int64_t V,
                                                       typename FineT<LF>::R diag, int use_clover,
                                                       double* __restrict__ part, int64_t pmember, int pvalue,
                                                       int64_t last) {
    using R = typename FineT<LF>::R;
    __shared__ cpx<R> sh[12 * kWilsonSites];
    // Work-groups are dealt to the 8 XCDs round-robin; renumber them so that
    // each XCD sweeps one contiguous range of sites and the neighbours one
    // x2-plane away stay in that XCD's L2.  The grid is a multiple of 8.
    const int64_t per = gridDim.x >> 3;
    const int64_t wg = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
    const int t = threadIdx.x;
    const int64_t base = wg * kWilsonSites;
    const int64_t site0 = base + t;
    // every thread reaches the barrier: one past the last site computes the
    // last site again, stores nothing (and adds zero to the sums)
    const bool live = site0 < V;
    const int64_t site = live ? site0 : V - 1;
    const int64_t vo = (int64_t)blockIdx.y * V;
    const int* nb = nbr + site * 8;
    cpx<R> acc[12];
    if constexpr (NEAR < 2 && sizeof(R) == 4) {
        // x-y neighbours in memory: the site-local terms first, then the hops
        // in lattice order, two in flight, no LDS copy (where the work-group's
        // range does not hold whole x-y planes, taking t and z first was
        // measured slower: 154 vs 136 us on 24^3x48)
        if (!DOT && !live) return;   // no barrier on this path
        cpx<R> pa[12], ua[9], pb[12], ub[9];
        hop_load<0, false, LF, VF, LR>(pa, ua, in, in_scale, U, V, site, nb[0], vo, last);
        hop_load<0, true, LF, VF, LR>(pb, ub, in, in_scale, U, V, site, nb[1], vo, last);
        {
            cpx<R> p[12];
            load_spinor<VF>(p, in, in_scale, site + vo);
#pragma unroll
            for (int f = 0; f < 12; ++f) acc[f] = {diag * p[f].re, diag * p[f].im};
            if (use_clover) herm_mul_add<LF>(acc, p, clov, cscale, site, V);
        }
        hop_apply<0, false>(acc, pa, ua);
        hop_load<1, false, LF, VF, LR>(pa, ua, in, in_scale, U, V, site, nb[2], vo, last);
        hop_apply<0, true>(acc, pb, ub);
        hop_load<1, true, LF, VF, LR>(pb, ub, in, in_scale, U, V, site, nb[3], vo, last);
        hop_apply<1, false>(acc, pa, ua);
        hop_load<2, false, LF, VF, LR>(pa, ua, in, in_scale, U, V, site, nb[4], vo, last);
        hop_apply<1, true>(acc, pb, ub);
        hop_load<2, true, LF, VF, LR>(pb, ub, in, in_scale, U, V, site, nb[5], vo, last);
        hop_apply<2, false>(acc, pa, ua);
        hop_load<3, false, LF, VF, LR>(pa, ua, in, in_scale, U, V, site, nb[6], vo, last);
        hop_apply<2, true>(acc, pb, ub);
        hop_load<3, true, LF, VF, LR>(pb, ub, in, in_scale, U, V, site, nb[7], vo, last);
        hop_apply<3, false>(acc, pa, ua);
        hop_apply<3, true>(acc, pb, ub);
    } else if constexpr (NEAR < 2) {
        // FP64 with the x-y neighbours in memory: the site-local terms first,
        // then the hops one at a time in lattice order, no LDS copy (this
        // order needs the fewest registers: two waves per SIMD)
        if (!DOT && !live) return;   // no barrier on this path
        cpx<R> pa[12], ua[9];
        load_spinor<VF>(pa, in, in_scale, site + vo);
#pragma unroll
        for (int f = 0; f < 12; ++f) acc[f] = {diag * pa[f].re, diag * pa[f].im};
        if (use_clover) herm_mul_add<LF>(acc, pa, clov, cscale, site, V);
        hop_load<0, false, LF, VF, LR>(pa, ua, in, in_scale, U, V, site, nb[0], vo, last);
        hop_apply<0, false>(acc, pa, ua);
        hop_load<0, true, LF, VF, LR>(pa, ua, in, in_scale, U, V, site, nb[1], vo, last);
        hop_apply<0, true>(acc, pa, ua);
        hop_load<1, false, LF, VF, LR>(pa, ua, in, in_scale, U, V, site, nb[2], vo, last);
        hop_apply<1, false>(acc, pa, ua);
        hop_load<1, true, LF, VF, LR>(pa, ua, in, in_scale, U, V, site, nb[3], vo, last);
        hop_apply<1, true>(acc, pa, ua);
        hop_load<2, false, LF, VF, LR>(pa, ua, in, in_scale, U, V, site, nb[4], vo, last);
        hop_apply<2, false>(acc, pa, ua);
        hop_load<2, true, LF, VF, LR>(pa, ua, in, in_scale, U, V, site, nb[5], vo, last);
        hop_apply<2, true>(acc, pa, ua);
        hop_load<3, false, LF, VF, LR>(pa, ua, in, in_scale, U, V, site, nb[6], vo, last);
        hop_apply<3, false>(acc, pa, ua);
        hop_load<3, true, LF, VF, LR>(pa, ua, in, in_scale, U, V, site, nb[7], vo, last);
        hop_apply<3, true>(acc, pa, ua);
    } else {
#pragma unroll
    for (int f = 0; f < 12; ++f) acc[f] = {0, 0};
    {
        cpx<R> p[12];
        load_spinor<VF>(p, in, in_scale, site + vo);
        lds_put(sh, t, p);
    }
    if constexpr (sizeof(R) == 4) {
        // FP32 arithmetic: two hops' operands in flight while two are applied
        cpx<R> pa[12], ua[9], pb[12], ub[9];
        hop_load<3, false, LF, VF, LR>(pa, ua, in, in_scale, U, V, site, nb[6], vo, last);
        hop_load<3, true, LF, VF, LR>(pb, ub, in, in_scale, U, V, site, nb[7], vo, last);
        hop_apply<3, false>(acc, pa, ua);
        hop_load<2, false, LF, VF, LR>(pa, ua, in, in_scale, U, V, site, nb[4], vo, last);
        hop_apply<3, true>(acc, pb, ub);
        hop_load<2, true, LF, VF, LR>(pb, ub, in, in_scale, U, V, site, nb[5], vo, last);
        hop_apply<2, false>(acc, pa, ua);
        hop_apply<2, true>(acc, pb, ub);
        __syncthreads();   // the work-group's spinors are in LDS
        hop_load_near<NEAR, 1, false, LF, VF, LR>(pa, ua, sh, in, in_scale, U, V, site, nb[2], base, vo, last);
        hop_load_near<NEAR, 1, true, LF, VF, LR>(pb, ub, sh, in, in_scale, U, V, site, nb[3], base, vo, last);
        {
            cpx<R> p[12];
#pragma unroll
            for (int f = 0; f < 12; ++f) p[f] = sh[f * kWilsonSites + t];
#pragma unroll
            for (int f = 0; f < 12; ++f) acc[f] = {acc[f].re + diag * p[f].re, acc[f].im + diag * p[f].im};
            if (use_clover) herm_mul_add<LF>(acc, p, clov, cscale, site, V);
        }
        hop_apply<1, false>(acc, pa, ua);
        hop_load_near<NEAR, 0, false, LF, VF, LR>(pa, ua, sh, in, in_scale, U, V, site, nb[0], base, vo, last);
        hop_apply<1, true>(acc, pb, ub);
        hop_load_near<NEAR, 0, true, LF, VF, LR>(pb, ub, sh, in, in_scale, U, V, site, nb[1], base, vo, last);
        hop_apply<0, false>(acc, pa, ua);
        hop_apply<0, true>(acc, pb, ub);
    } else {
        // FP64: two hops in flight would need all 256 registers (one wave per SIMD)
        cpx<R> pa[12], ua[9];
        hop_load<3, false, LF, VF, LR>(pa, ua, in, in_scale, U, V, site, nb[6], vo, last);
        hop_apply<3, false>(acc, pa, ua);
        hop_load<3, true, LF, VF, LR>(pa, ua, in, in_scale, U, V, site, nb[7], vo, last);
        hop_apply<3, true>(acc, pa, ua);
        hop_load<2, false, LF, VF, LR>(pa, ua, in, in_scale, U, V, site, nb[4], vo, last);
        hop_apply<2, false>(acc, pa, ua);
        hop_load<2, true, LF, VF, LR>(pa, ua, in, in_scale, U, V, site, nb[5], vo, last);
        hop_apply<2, true>(acc, pa, ua);
        __syncthreads();   // the work-group's spinors are in LDS
#pragma unroll
        for (int f = 0; f < 12; ++f) pa[f] = sh[f * kWilsonSites + t];
#pragma unroll
        for (int f = 0; f < 12; ++f) acc[f] = {acc[f].re + diag * pa[f].re, acc[f].im + diag * pa[f].im};
        if (use_clover) herm_mul_add<LF>(acc, pa, clov, cscale, site, V);
        hop_load_near<NEAR, 1, false, LF, VF, LR>(pa, ua, sh, in, in_scale, U, V, site, nb[2], base, vo, last);
        hop_apply<1, false>(acc, pa, ua);
        hop_load_near<NEAR, 1, true, LF, VF, LR>(pa, ua, sh, in, in_scale, U, V, site, nb[3], base, vo, last);
        hop_apply<1, true>(acc, pa, ua);
        hop_load_near<NEAR, 0, false, LF, VF, LR>(pa, ua, sh, in, in_scale, U, V, site, nb[0], base, vo, last);
        hop_apply<0, false>(acc, pa, ua);
        hop_load_near<NEAR, 0, true, LF, VF, LR>(pa, ua, sh, in, in_scale, U, V, site, nb[1], base, vo, last);
        hop_apply<0, true>(acc, pa, ua);
    }
    }
    if (live) store_spinor<VF>(out, out_scale, site + vo, acc);
    if constexpr (DOT) {
        // the site's input from the LDS copy (read again from memory, a cache
        // hit normally, on the paths that keep none)
        cpx<R> p[12];
        if constexpr (NEAR < 2) {
            asm volatile("" ::: "memory");
            load_spinor<VF>(p, in, in_scale, site + vo);
        } else {
#pragma unroll
            for (int f = 0; f < 12; ++f) p[f] = sh[f * kWilsonSites + t];
        }
        double s3[3] = {0, 0, 0};
        if (live)
#pragma unroll
            for (int f = 0; f < 12; ++f) {
                s3[0] += (double)acc[f].re * acc[f].re + (double)acc[f].im * acc[f].im;
                s3[1] += (double)acc[f].re * p[f].re + (double)acc[f].im * p[f].im;
                s3[2] += (double)acc[f].re * p[f].im - (double)acc[f].im * p[f].re;
            }
        __shared__ double red[3][4];   // [value][wave]
#pragma unroll
        for (int i = 0; i < 3; ++i)
            for (int o = 32; o > 0; o >>= 1) s3[i] += __shfl_down(s3[i], o, 64);
        if ((t & 63) == 0)
#pragma unroll
            for (int i = 0; i < 3; ++i) red[i][t >> 6] = s3[i];
        __syncthreads();
        if (t < 3) {
            double r = 0;
            for (int j = 0; j < 4; ++j) r += red[t][j];
            part[(int64_t)blockIdx.y * pmember + t * pvalue + blockIdx.x] = r;
        }
    }
}

// ------------------------------------------------------------ red-black form
// Red-black (even-odd) preconditioning (Sec. 3.3, used on every level in
// Sec. 7.1): the hops of Eq. (2) join sites of opposite parity, so with the
// site-local block C(x) = 4 + m0 + A(x) and the hop term D (the sum over mu
// in Eq. 2, its -1/2 included) the Schur complement on the even sites is
//     S = C_ee - D_eo C_oo^-1 D_oe,
// and M x = b is solved by S x_e = b_e - D_eo C_oo^-1 b_o followed by
// x_o = C_oo^-1 (b_o - D_oe x_e).  Every piece is one launch of k_wilson_eo
// over the sites x of one parity (half-lattice index h, x = hsite[h]):
//     out(x) = L_out( L_self(self(x)) + coef * [sum of the eight hops of hin](x) )
// L_self: none (SELF 0), the identity (1) or C(x) (2); L_out: the identity or
// C(x)^-1 (INV).  coef = 1 gives D, coef = -1 gives -D.  hin is a half-lattice
// field of the other parity; the neighbour y of x has half index y >> 1,
// because x0 runs fastest and L0 is even.  self and out are half-lattice
// fields, or whole-lattice ones indexed by x (self_full, out_full).
// Member b of a batch (grid dimension y) finds its fields at b*V/2 (half) or
// b*V (whole) sites.  Links, clover, inverse and neighbour table are read in
// their parity-order copies: the thread of site x (parity p, half index h)
// finds its own entries at p*V/2 + h and a neighbour y's link at
// (1-p)*V/2 + (y >> 1), so every wave reads them contiguously, and each link
// is read once per launch (non-temporal: forward links of this parity,
// backward links of the other).
// The site-local part of a red-black piece: acc = 0 (SELF 0), self (1) or
// C(x) self (2); the clover term in parity order at index ie.
template <int LF, int VF, int SELF, typename R>
__device__ __forceinline__ void eo_self_terms(cpx<R> acc[12], const void* __restrict__ self,
                                              const float* __restrict__ self_sc, int64_t si, R diag,
                                              int use_clover, const void* __restrict__ clov,
                                              const float* __restrict__ cscale, int64_t ie, int64_t V) {
    if constexpr (SELF == 0) {
#pragma unroll
        for (int f = 0; f < 12; ++f) acc[f] = {R(0), R(0)};
    } else {
        cpx<R> p[12];
        load_spinor<VF>(p, self, self_sc, si);
        if constexpr (SELF == 1) {
#pragma unroll
            for (int f = 0; f < 12; ++f) acc[f] = p[f];
        } else {
#pragma unroll
            for (int f = 0; f < 12; ++f) acc[f] = {diag * p[f].re, diag * p[f].im};
            if (use_clover) herm_mul_add<LF>(acc, p, clov, cscale, ie, V);
        }
    }
}

// Per-site scales of 16-bit vector fields (VF = FMT_H16 / FMT_B16), indexed
// like the fields; unused for complex vectors.
struct EoScales {
    const float* self = nullptr;
    const float* hin = nullptr;
    float* out = nullptr;
};

template <int LF, int VF, int SELF, bool HOPS, bool INV, int LR = 18>
__global__ __launch_bounds__(256) void k_wilson_eo(const void* __restrict__ U, const void* __restrict__ clov,
                                                   const float* __restrict__ cscale, const void* __restrict__ cinv,
                                                   const float* __restrict__ ciscale, const int* __restrict__ hnb,
                                                   const int* __restrict__ hsite, const void* __restrict__ self,
                                                   const void* __restrict__ hin, void* __restrict__ out, int64_t Vh,
                                                   int64_t V, typename FineT<LF>::R diag, typename FineT<LF>::R coef,
                                                   int use_clover, int self_full, int out_full, int64_t last,
                                                   int parity, EoScales sc) {
    using R = typename FineT<LF>::R;
    // XCD-contiguous work-group numbering, as in k_wilson_clover (grid a multiple of 8)
    const int64_t per = gridDim.x >> 3;
    const int64_t wg = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
    const int64_t h = wg * blockDim.x + threadIdx.x;
    if (h >= Vh) return;
    const int64_t ie = (int64_t)parity * Vh + h;       // this site in parity order
    const int64_t io = (int64_t)(1 - parity) * Vh;     // start of the other parity
    const int64_t site = hsite[ie];
    const int64_t vh = (int64_t)blockIdx.y * Vh, vf = (int64_t)blockIdx.y * V;
    cpx<R> acc[12];
    if constexpr (HOPS) {
        const int4* nb4 = reinterpret_cast<const int4*>(hnb + ie * 8);
        const int4 na = nb4[0], nc = nb4[1];
        const int nb[8] = {na.x, na.y, na.z, na.w, nc.x, nc.y, nc.z, nc.w};
        const R c = R(-0.5) * coef;
#define QMG_EO_LOAD(P, UU, MU, BACK, D)                                                               \
        load_spinor<VF>(P, hin, sc.hin, (int64_t)(nb[D] >> 1) + vh);                                   \
        load_link_at<LF, LR, true>(UU, U, MU, BACK ? io + (nb[D] >> 1) : ie, V,                        \
                                   MU == 3 && (BACK ? (int64_t)nb[D] : site) >= last);
        if constexpr (sizeof(R) == 4) {
            // FP32 arithmetic: the next two hops' operands are in flight while
            // two are applied; the site-local part runs under the first loads
            // (9-10 % faster than one hop at a time on 16^3x32 and 32^3x64
            // with 18-real links, 1-2 % with 12-real ones; with a register cap
            // of four waves per SIMD both forms spill and are slower)
            cpx<R> pa[12], ua[9], pb[12], ub[9];
            QMG_EO_LOAD(pa, ua, 0, false, 0)
            QMG_EO_LOAD(pb, ub, 0, true, 1)
            eo_self_terms<LF, VF, SELF>(acc, self, sc.self, self_full ? site + vf : h + vh, diag, use_clover, clov, cscale,
                                        ie, V);
            hop_apply<0, false>(acc, pa, ua, c);
            QMG_EO_LOAD(pa, ua, 1, false, 2)
            hop_apply<0, true>(acc, pb, ub, c);
            QMG_EO_LOAD(pb, ub, 1, true, 3)
            hop_apply<1, false>(acc, pa, ua, c);
            QMG_EO_LOAD(pa, ua, 2, false, 4)
            hop_apply<1, true>(acc, pb, ub, c);
            QMG_EO_LOAD(pb, ub, 2, true, 5)
            hop_apply<2, false>(acc, pa, ua, c);
            QMG_EO_LOAD(pa, ua, 3, false, 6)
            hop_apply<2, true>(acc, pb, ub, c);
            QMG_EO_LOAD(pb, ub, 3, true, 7)
            hop_apply<3, false>(acc, pa, ua, c);
            hop_apply<3, true>(acc, pb, ub, c);
        } else {
            // FP64: one hop at a time (registers)
            eo_self_terms<LF, VF, SELF>(acc, self, sc.self, self_full ? site + vf : h + vh, diag, use_clover, clov, cscale,
                                        ie, V);
            cpx<R> p[12], u[9];
#define QMG_EO_HOP(MU, BACK, D) QMG_EO_LOAD(p, u, MU, BACK, D) hop_apply<MU, BACK>(acc, p, u, c);
            QMG_EO_HOP(0, false, 0)
            QMG_EO_HOP(0, true, 1)
            QMG_EO_HOP(1, false, 2)
            QMG_EO_HOP(1, true, 3)
            QMG_EO_HOP(2, false, 4)
            QMG_EO_HOP(2, true, 5)
            QMG_EO_HOP(3, false, 6)
            QMG_EO_HOP(3, true, 7)
#undef QMG_EO_HOP
        }
#undef QMG_EO_LOAD
    } else {
        eo_self_terms<LF, VF, SELF>(acc, self, sc.self, self_full ? site + vf : h + vh, diag, use_clover, clov, cscale,
                                        ie, V);
    }
    if constexpr (INV) {
        cpx<R> t[12];
#pragma unroll
        for (int f = 0; f < 12; ++f) t[f] = {R(0), R(0)};
        herm_mul_add<LF>(t, acc, cinv, ciscale, ie, V);
        store_spinor<VF>(out, sc.out, out_full ? site + vf : h + vh, t);
    } else {
        store_spinor<VF>(out, sc.out, out_full ? site + vf : h + vh, acc);
    }
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

// (diag + A(x))^-1 per site and chirality block, in FP64: Gauss-Jordan
// elimination with partial pivoting on the 6x6 block (Hermitian, so its
// inverse is too and is stored packed like the clover term, from the upper
// triangle).  A singular block gives non-finite entries, which the solvers
// report as QMG_ERR_NONFINITE.
__global__ void k_clover_invert(double* __restrict__ cinv, const double* __restrict__ clov, int64_t V, double diag) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= V) return;
    for (int chi = 0; chi < 2; ++chi) {
        const double* A = clov + (int64_t)chi * 36 * V + x;
        cpx<double> a[6][6], b[6][6];
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) b[i][j] = {i == j ? 1.0 : 0.0, 0.0};
        for (int i = 0; i < 6; ++i) a[i][i] = {diag + A[i * V], 0.0};
        int k = 0;
        for (int r = 0; r < 6; ++r)
            for (int c = r + 1; c < 6; ++c, ++k) {
                a[r][c] = {A[(6 + 2 * k) * V], A[(7 + 2 * k) * V]};
                a[c][r] = {a[r][c].re, -a[r][c].im};
            }
        for (int col = 0; col < 6; ++col) {
            int piv = col;
            double best = a[col][col].re * a[col][col].re + a[col][col].im * a[col][col].im;
            for (int i = col + 1; i < 6; ++i) {
                const double m = a[i][col].re * a[i][col].re + a[i][col].im * a[i][col].im;
                if (m > best) { best = m; piv = i; }
            }
            if (piv != col)
                for (int j = 0; j < 6; ++j) {
                    const cpx<double> t = a[col][j]; a[col][j] = a[piv][j]; a[piv][j] = t;
                    const cpx<double> u = b[col][j]; b[col][j] = b[piv][j]; b[piv][j] = u;
                }
            // 1 / a[col][col]
            const cpx<double> p = a[col][col];
            const double den = p.re * p.re + p.im * p.im;
            const cpx<double> ip = {p.re / den, -p.im / den};
            for (int j = 0; j < 6; ++j) { a[col][j] = cmul(ip, a[col][j]); b[col][j] = cmul(ip, b[col][j]); }
            for (int i = 0; i < 6; ++i) {
                if (i == col) continue;
                const cpx<double> f = a[i][col];
                for (int j = 0; j < 6; ++j) {
                    a[i][j] = csub(a[i][j], cmul(f, a[col][j]));
                    b[i][j] = csub(b[i][j], cmul(f, b[col][j]));
                }
            }
        }
        double* o = cinv + (int64_t)chi * 36 * V + x;
        for (int i = 0; i < 6; ++i) o[i * V] = b[i][i].re;
        k = 0;
        for (int r = 0; r < 6; ++r)
            for (int c = r + 1; c < 6; ++c, ++k) {
                o[(6 + 2 * k) * V] = b[r][c].re;
                o[(7 + 2 * k) * V] = b[r][c].im;
            }
    }
}

__global__ void k_real_to_f32(float* __restrict__ out, const double* __restrict__ in, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

// Parity-order copy of a [K][V] array of W-sized elements: dst[k][j] =
// src[k][hsite[j]], hsite [V] holding the lattice index of parity-order index j.
template <typename W>
__global__ void k_to_parity_order(W* __restrict__ dst, const W* __restrict__ src, const int* __restrict__ hsite,
                                  int64_t K, int64_t V) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= K * V) return;
    const int64_t k = i / V, j = i - k * V;
    dst[i] = src[k * V + hsite[j]];
}
// hnb[j][d] = nbr[hsite[j]][d]: the neighbour table in parity order
__global__ void k_nbr_parity_order(int* __restrict__ hnb, const int* __restrict__ nbr, const int* __restrict__ hsite,
                                   int64_t V) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V * 8) return;
    hnb[i] = nbr[(int64_t)hsite[i >> 3] * 8 + (i & 7)];
}

template <int LF>
__global__ void k_clover_export(double2* __restrict__ out, const void* __restrict__ clov,
                                const float* __restrict__ cscale, int64_t V) {
    using R = typename FineT<LF>::R;
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= V) return;
    double2* o = out + x * 144;
    for (int e = 0; e < 144; ++e) o[e] = make_double2(0, 0);
    for (int chi = 0; chi < 2; ++chi) {
        R d[6];
        cpx<R> u[15];
        load_clover<LF>(d, u, clov, cscale, chi, x, V);
        for (int i = 0; i < 6; ++i) o[(6 * chi + i) * 12 + 6 * chi + i] = make_double2(d[i], 0);
        int k = 0;
        for (int r = 0; r < 6; ++r)
            for (int c = r + 1; c < 6; ++c, ++k) {
                o[(6 * chi + r) * 12 + 6 * chi + c] = make_double2(u[k].re, u[k].im);
                o[(6 * chi + c) * 12 + 6 * chi + r] = make_double2(u[k].re, -u[k].im);
            }
    }
}

// The links as the operator holds them -> canonical [4][V][3][3] complex128,
// with the antiperiodic time sign taken back out (the third row rebuilt for
// compressed storage).  One thread per link.
template <int LF, int LR>
__global__ void k_links_export(double2* __restrict__ G, const void* __restrict__ U, int64_t V, int64_t last,
                               int anti) {
    using R = typename FineT<LF>::R;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= 4 * V) return;
    const int64_t site = g % V;
    const int mu = (int)(g / V);
    cpx<R> u[9];
    load_link<LF, LR>(u, U, mu, site, V, last);
    const double sgn = (anti && mu == 3 && site >= last) ? -1.0 : 1.0;
    for (int e = 0; e < 9; ++e) G[((int64_t)mu * V + site) * 9 + e] = make_double2(sgn * (double)u[e].re, sgn * (double)u[e].im);
}

// FP64 clover [2][36][V] -> 16-bit pairs [2][18][V] with one scale per (chirality, site).
template <int LF>
__global__ void k_clover_pack16(uint32_t* __restrict__ W, float* __restrict__ cscale,
                                const double* __restrict__ clov, int64_t V, unsigned* __restrict__ nf) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= V) return;
    for (int chi = 0; chi < 2; ++chi) {
        const double* A = clov + (int64_t)chi * 36 * V + x;
        float m = 0.0f;
        bool bad = false;
        for (int i = 0; i < 36; ++i) {
            const float a = (float)A[i * V];
            bad = bad || !isfinite(a);
            m = fmaxf(m, fabsf(a));
        }
        note_nonfinite(nf, bad);
        const float inv = m > 0.0f ? 1.0f / m : 0.0f;
        for (int q = 0; q < 18; ++q)
            W[((int64_t)chi * 18 + q) * V + x] = enc_pair<LF>((float)A[2 * q * V] * inv, (float)A[(2 * q + 1) * V] * inv);
        cscale[(int64_t)chi * V + x] = m;
    }
}

// Canonical gauge -> 16-bit pairs [4][ne][V] (ne = 9, or 6: rows 0 and 1 of a
// compressed link), time sign folded.
template <int LF>
__global__ void k_pack_gauge16(uint32_t* __restrict__ U, const double2* __restrict__ G, int64_t V,
                               int64_t last_slice_start, int anti, int ne, unsigned* __restrict__ nf) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= 4 * ne * V) return;
    const int64_t site = g % V;
    const int e = (int)((g / V) % ne);
    const int mu = (int)(g / (ne * V));
    const double2 v = G[((int64_t)mu * V + site) * 9 + e];
    note_nonfinite(nf, !(isfinite((float)v.x) && isfinite((float)v.y)));
    const double sgn = (anti && mu == 3 && site >= last_slice_start) ? -1.0 : 1.0;
    U[g] = enc_pair<LF>((float)(sgn * v.x), (float)(sgn * v.y));
}

// Canonical gauge [4][V][3][3] complex128 -> SoA [4][ne][V] in R (ne = 9, or 6
// for compressed links), time sign folded.
template <typename R>
__global__ void k_pack_gauge(cpx<R>* __restrict__ U, const double2* __restrict__ G, int64_t V,
                             int64_t last_slice_start, int anti, int ne) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= 4 * ne * V) return;
    const int64_t site = g % V;
    const int e = (int)((g / V) % ne);
    const int mu = (int)(g / (ne * V));
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

// work-groups of one member's launch (256 sites each, a multiple of 8)
int wilson_groups(const qmg_fine_op_s* op) { return (int)(((op->V + 255) / 256 + 7) / 8 * 8); }

template <int LF, int VF, bool DOT = false>
static qmg_status launch_wilson(const qmg_fine_op_s* op, const void* in, const float* in_scale, void* out,
                                float* out_scale, int members, hipStream_t s, double* part = nullptr,
                                int64_t pmember = 0, int pvalue = 0) {
    using R = typename FineT<LF>::R;
    const unsigned nb = (unsigned)wilson_groups(op);
    // x and y neighbours from LDS when a work-group's 256 sites are whole x-y
    // planes; not for 16-bit links with FP32 spinors, which were measured
    // slower that way (21.8 vs 20.6 us on 16^3x32; FP32 25.6 vs 25.7, all
    // 16-bit 18.6 vs 19.6)
    const bool mixed = is16f<LF>() && !is16f<VF>();
    const int near = !mixed && kWilsonSites % ((int64_t)op->dims[0] * op->dims[1]) == 0 ? 2 : 0;
#define QMG_WC_LAUNCH(LR, NEAR)                                                                                    \
    hipLaunchKernelGGL((k_wilson_clover<LF, VF, DOT, LR, NEAR>), dim3(nb, members), dim3(256), 0, s, op->U,       \
                       op->clov, op->cscale, op->nbr, in, in_scale, out, out_scale, op->V, (R)(4.0 + op->m0),    \
                       op->csw != 0.0 ? 1 : 0, part, pmember, pvalue, op->last)
#define QMG_WC_NEAR(LR)                                                                                            \
    if (near == 2) QMG_WC_LAUNCH(LR, 2);                                                                           \
    else QMG_WC_LAUNCH(LR, 0);
    if constexpr (LF != FMT_F64) {
        if (op->link_reals == 12) {
            QMG_WC_NEAR(12)
        } else {
            QMG_WC_NEAR(18)
        }
    } else {
        QMG_WC_NEAR(18)
    }
#undef QMG_WC_NEAR
#undef QMG_WC_LAUNCH
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

// vprec: the vector storage (checked by the callers against the operator's)
static qmg_status wilson_any(const qmg_fine_op_s* op, const void* in, const float* in_scale, void* out,
                             float* out_scale, qmg_prec vprec, int m, hipStream_t s) {
    switch (op->storage) {
        case QMG_C128: return launch_wilson<FMT_F64, FMT_F64>(op, in, nullptr, out, nullptr, m, s);
        case QMG_C64: return launch_wilson<FMT_F32, FMT_F32>(op, in, nullptr, out, nullptr, m, s);
        case QMG_H16:
            if (vprec == QMG_C64) return launch_wilson<FMT_H16, FMT_F32>(op, in, nullptr, out, nullptr, m, s);
            if (vprec == QMG_H16) return launch_wilson<FMT_H16, FMT_H16>(op, in, in_scale, out, out_scale, m, s);
            return launch_wilson<FMT_H16, FMT_B16>(op, in, in_scale, out, out_scale, m, s);
        default:
            if (vprec == QMG_C64) return launch_wilson<FMT_B16, FMT_F32>(op, in, nullptr, out, nullptr, m, s);
            if (vprec == QMG_H16) return launch_wilson<FMT_B16, FMT_H16>(op, in, in_scale, out, out_scale, m, s);
            return launch_wilson<FMT_B16, FMT_B16>(op, in, in_scale, out, out_scale, m, s);
    }
}

// Solver-side entry: `members` fields of V sites one after another (vectors
// in complex128 / complex64 as `vprec`, checked by the caller).
qmg_status wilson_apply(const qmg_fine_op_s* op, const void* in, void* out, qmg_prec vprec, int members,
                        hipStream_t s) {
    return wilson_any(op, in, nullptr, out, nullptr, vprec, members, s);
}

// wilson_apply with the minimal-residual inner products of every member:
// <out,out>, <out,in>.re, <out,in>.im per work-group, value v of work-group g
// of member b at part[b*pmember + v*pvalue + g] (wilson_groups(op) groups).
// Vectors in complex128 / complex64 only.
qmg_status wilson_apply_dot(const qmg_fine_op_s* op, const void* in, void* out, qmg_prec vprec, int members,
                            double* part, int64_t pmember, int pvalue, hipStream_t s) {
    if (vprec == QMG_C128 && op->storage == QMG_C128)
        return launch_wilson<FMT_F64, FMT_F64, true>(op, in, nullptr, out, nullptr, members, s, part, pmember, pvalue);
    if (vprec != QMG_C64 || op->storage == QMG_C128)
        return fail(QMG_ERR_PREC, "wilson_apply_dot: vectors must be in the operator's inner precision");
    switch (op->storage) {
        case QMG_C64:
            return launch_wilson<FMT_F32, FMT_F32, true>(op, in, nullptr, out, nullptr, members, s, part, pmember,
                                                        pvalue);
        case QMG_H16:
            return launch_wilson<FMT_H16, FMT_F32, true>(op, in, nullptr, out, nullptr, members, s, part, pmember,
                                                        pvalue);
        default:
            return launch_wilson<FMT_B16, FMT_F32, true>(op, in, nullptr, out, nullptr, members, s, part, pmember,
                                                        pvalue);
    }
}

// Pieces of the red-black form (k_wilson_eo instances).
enum EoPiece {
    EO_HOP_INV = 0,   // out_o = C^-1 D in_e                 (first half of S)
    EO_DIAG_HOP = 1,  // out_e = C self_e - D in_o           (second half of S)
    EO_INV = 2,       // out = C^-1 self
    EO_SELF_HOP = 3,  // out = self - D in
    EO_RECON = 4,     // out = C^-1 (self - D in)
    EO_COPY = 5       // out = self (re-indexing between half and whole lattice)
};

template <int LF, int VF>
static qmg_status launch_eo(const qmg_fine_op_s* op, int piece, int parity, const void* self, int self_full,
                            const void* hin, void* out, int out_full, int m, hipStream_t s) {
    using R = typename FineT<LF>::R;
    const int64_t Vh = op->V / 2;
    const unsigned nb = (unsigned)(((Vh + 255) / 256 + 7) / 8 * 8);
    const R diag = (R)(4.0 + op->m0);
    const int uc = op->csw != 0.0 ? 1 : 0;
    const dim3 grid(nb, (unsigned)m), block(256);
#define QMG_EO_LAUNCH_LR(SELF, HOPS, INV, COEF, LR)                                                              \
    hipLaunchKernelGGL((k_wilson_eo<LF, VF, SELF, HOPS, INV, LR>), grid, block, 0, s, op->U_eo, op->clov_eo,    \
                       op->cscale_eo, op->cinv, op->ciscale, op->hnb, op->hsite, self, hin, out, Vh, op->V, diag,  \
                       (R)(COEF), uc, self_full, out_full, op->last, parity, EoScales{})
#define QMG_EO_LAUNCH(SELF, HOPS, INV, COEF)                                                                    \
    do {                                                                                                        \
        if constexpr (LF != FMT_F64 && HOPS) {                                                                  \
            if (op->link_reals == 12) QMG_EO_LAUNCH_LR(SELF, HOPS, INV, COEF, 12);                               \
            else QMG_EO_LAUNCH_LR(SELF, HOPS, INV, COEF, 18);                                                    \
        } else {                                                                                                \
            QMG_EO_LAUNCH_LR(SELF, HOPS, INV, COEF, 18);                                                         \
        }                                                                                                       \
    } while (0)
    switch (piece) {
        case EO_HOP_INV: QMG_EO_LAUNCH(0, true, true, 1.0); break;
        case EO_DIAG_HOP: QMG_EO_LAUNCH(2, true, false, -1.0); break;
        case EO_INV: QMG_EO_LAUNCH(1, false, true, 0.0); break;
        case EO_SELF_HOP: QMG_EO_LAUNCH(1, true, false, -1.0); break;
        case EO_RECON: QMG_EO_LAUNCH(1, true, true, -1.0); break;
        default: QMG_EO_LAUNCH(1, false, false, 0.0);
    }
#undef QMG_EO_LAUNCH
#undef QMG_EO_LAUNCH_LR
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

// One red-black piece with vectors in `vprec` (complex128 for a complex128
// operator, complex64 for the others).
static qmg_status fine_eo(const qmg_fine_op_s* op, int piece, int parity, const void* self, int self_full,
                          const void* hin, void* out, int out_full, qmg_prec vprec, int m, hipStream_t s) {
    if (!op->hsite) return fail(QMG_ERR_SHAPE, "red-black form needs every lattice extent even");
    const bool ok = op->storage == QMG_C128 ? vprec == QMG_C128 : vprec == QMG_C64;
    if (!ok) return fail(QMG_ERR_PREC, "red-black form: vector precision %d for storage %d", (int)vprec, (int)op->storage);
    switch (op->storage) {
        case QMG_C128: return launch_eo<FMT_F64, FMT_F64>(op, piece, parity, self, self_full, hin, out, out_full, m, s);
        case QMG_C64: return launch_eo<FMT_F32, FMT_F32>(op, piece, parity, self, self_full, hin, out, out_full, m, s);
        case QMG_H16: return launch_eo<FMT_H16, FMT_F32>(op, piece, parity, self, self_full, hin, out, out_full, m, s);
        default: return launch_eo<FMT_B16, FMT_F32>(op, piece, parity, self, self_full, hin, out, out_full, m, s);
    }
}

// out_e = S in_e = C_ee in_e - D_eo C_oo^-1 D_oe in_e; tmp_o: odd half-lattice scratch (m members).
qmg_status fine_schur_apply(const qmg_fine_op_s* op, const void* in_e, void* out_e, void* tmp_o, qmg_prec vprec,
                            int m, hipStream_t s) {
    QMG_TRY(fine_eo(op, EO_HOP_INV, 1, nullptr, 0, in_e, tmp_o, 0, vprec, m, s));
    return fine_eo(op, EO_DIAG_HOP, 0, in_e, 0, tmp_o, out_e, 0, vprec, m, s);
}

// The Schur operator on 16-bit half-lattice vectors (FP16 pairs with one FP32
// scale per site, FP32 arithmetic), for an operator with 16-bit storage:
// tmp_o = C_oo^-1 D_oe in_e, then out_e = C_ee in_e - D_eo tmp_o, every
// intermediate rounded to 16 bits with its own per-site scale.
template <int LF>
static void launch_schur16(const qmg_fine_op_s* op, const void* in_e, const float* in_s, void* out_e, float* out_s,
                           void* tmp_o, float* tmp_s, int m, hipStream_t s) {
    const int64_t Vh = op->V / 2;
    const unsigned nb = (unsigned)(((Vh + 255) / 256 + 7) / 8 * 8);
    const float diag = (float)(4.0 + op->m0);
    const int uc = op->csw != 0.0 ? 1 : 0;
    const dim3 grid(nb, (unsigned)m), block(256);
    EoScales a, b;
    a.hin = in_s;
    a.out = tmp_s;
    b.self = in_s;
    b.hin = tmp_s;
    b.out = out_s;
#define QMG_S16(LR)                                                                                                 \
    do {                                                                                                            \
        hipLaunchKernelGGL((k_wilson_eo<LF, FMT_H16, 0, true, true, LR>), grid, block, 0, s, op->U_eo, op->clov_eo,  \
                           op->cscale_eo, op->cinv, op->ciscale, op->hnb, op->hsite, nullptr, in_e, tmp_o, Vh, op->V, \
                           diag, 1.0f, uc, 0, 0, op->last, 1, a);                                                   \
        hipLaunchKernelGGL((k_wilson_eo<LF, FMT_H16, 2, true, false, LR>), grid, block, 0, s, op->U_eo,             \
                           op->clov_eo, op->cscale_eo, op->cinv, op->ciscale, op->hnb, op->hsite, in_e, tmp_o, out_e, \
                           Vh, op->V, diag, -1.0f, uc, 0, 0, op->last, 0, b);                                        \
    } while (0)
    if (op->link_reals == 12) QMG_S16(12);
    else QMG_S16(18);
#undef QMG_S16
}

qmg_status fine_schur_apply16(const qmg_fine_op_s* op, const void* in_e, const float* in_s, void* out_e, float* out_s,
                              void* tmp_o, float* tmp_s, int m, hipStream_t s) {
    if (!op->hsite) return fail(QMG_ERR_SHAPE, "red-black form needs every lattice extent even");
    if (op->storage == QMG_H16) launch_schur16<FMT_H16>(op, in_e, in_s, out_e, out_s, tmp_o, tmp_s, m, s);
    else if (op->storage == QMG_B16) launch_schur16<FMT_B16>(op, in_e, in_s, out_e, out_s, tmp_o, tmp_s, m, s);
    else return fail(QMG_ERR_PREC, "Schur operator on 16-bit vectors: the operator needs 16-bit storage");
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

// bhat_e = b_e - D_eo C_oo^-1 b_o for whole-lattice b.
qmg_status fine_schur_source(const qmg_fine_op_s* op, const void* b, void* bhat_e, void* tmp_o, qmg_prec vprec,
                             int m, hipStream_t s) {
    QMG_TRY(fine_eo(op, EO_INV, 1, b, 1, nullptr, tmp_o, 0, vprec, m, s));
    return fine_eo(op, EO_SELF_HOP, 0, b, 1, tmp_o, bhat_e, 0, vprec, m, s);
}

// whole-lattice x: x_e from the Schur solution, x_o = C_oo^-1 (b_o - D_oe x_e).
qmg_status fine_schur_reconstruct(const qmg_fine_op_s* op, const void* x_e, const void* b, void* x, qmg_prec vprec,
                                  int m, hipStream_t s) {
    QMG_TRY(fine_eo(op, EO_RECON, 1, b, 1, x_e, x, 1, vprec, m, s));
    return fine_eo(op, EO_COPY, 0, x_e, 0, nullptr, x, 1, vprec, m, s);
}

static size_t real_bytes(qmg_prec p) { return p == QMG_C128 ? 8 : p == QMG_C64 ? 4 : 2; }
static bool is16p(qmg_prec p) { return p == QMG_H16 || p == QMG_B16; }

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
    if (op->cscale) (void)hipFree(op->cscale);
    if (op->nbr) (void)hipFree(op->nbr);
    if (op->cinv) (void)hipFree(op->cinv);
    if (op->ciscale) (void)hipFree(op->ciscale);
    if (op->hsite) (void)hipFree(op->hsite);
    if (op->U_eo) (void)hipFree(op->U_eo);
    if (op->clov_eo) (void)hipFree(op->clov_eo);
    if (op->cscale_eo) (void)hipFree(op->cscale_eo);
    if (op->hnb) (void)hipFree(op->hnb);
    if (op->eo_tmp) (void)hipFree(op->eo_tmp);
    delete op;
}

extern "C" qmg_status qmg_fine_op_create_ex(const int dims[4], const void* gauge, double m0, double csw,
                                            int antiperiodic_t, qmg_prec storage, int link_reals, void* stream,
                                            qmg_fine_op* out) {
    if (!out) return fail(QMG_ERR_ARG, "fine_op_create: out is NULL");
    *out = nullptr;
    QMG_TRY(check_dims(dims, 2, "fine_op_create"));
    if (!gauge) return fail(QMG_ERR_ARG, "fine_op_create: gauge is NULL");
    if (storage != QMG_C128 && storage != QMG_C64 && !is16p(storage))
        return fail(QMG_ERR_PREC, "fine_op_create: storage %d not supported", (int)storage);
    if (link_reals != 18 && link_reals != 12)
        return fail(QMG_ERR_ARG, "fine_op_create: link_reals %d (18 or 12)", link_reals);
    if (link_reals == 12 && storage == QMG_C128)
        return fail(QMG_ERR_PREC, "fine_op_create: compressed links are for the complex64 and 16-bit storages");
    hipStream_t s = as_stream(stream);
    auto* op = new qmg_fine_op_s();
    for (int m = 0; m < 4; ++m) op->dims[m] = dims[m];
    op->V = volume(dims);
    op->m0 = m0;
    op->csw = csw;
    op->antiperiodic_t = antiperiodic_t ? 1 : 0;
    op->storage = storage;
    op->link_reals = link_reals;
    op->last = op->V - op->V / dims[3];
    const int ne = link_reals == 12 ? 6 : 9;   // stored entries per link
    const size_t rb = real_bytes(storage);
    hipError_t e = hipMalloc(&op->U, 2 * rb * 4 * ne * op->V);
    if (e == hipSuccess) e = hipMalloc(&op->clov, rb * 72 * op->V);
    if (e == hipSuccess && is16p(storage)) e = hipMalloc(&op->cscale, sizeof(float) * 2 * op->V);
    if (e != hipSuccess) {
        qmg_fine_op_destroy(op);
        return fail(QMG_ERR_NOMEM, "fine_op_create: %s", hipGetErrorString(e));
    }
    qmg_status st = make_neighbour_table(dims, &op->nbr, s);
    if (st != QMG_OK) {
        qmg_fine_op_destroy(op);
        return st;
    }
    const int64_t last = op->last;
    const unsigned nbU = (unsigned)((4 * ne * op->V + 255) / 256), nbS = (unsigned)((op->V + 127) / 128);
    const SigmaBlocks sb = sigma_blocks(csw);
    // red-black form when every extent is even: the half-site table and the
    // inverse of the site-local block, built from the FP64 clover term
    const bool eo = dims[0] % 2 == 0 && dims[1] % 2 == 0 && dims[2] % 2 == 0 && dims[3] % 2 == 0;
    void* c64 = nullptr;   // FP64 clover temporary (16-bit storage, or the red-black inverse of a complex64 one)
    void* i64 = nullptr;   // FP64 inverse temporary (storages other than complex128)
    if (eo) {
        st = make_half_site_table(dims, &op->hsite, s);
        if (st != QMG_OK) {
            qmg_fine_op_destroy(op);
            return st;
        }
        e = hipMalloc(&op->cinv, rb * 72 * op->V);
        if (e == hipSuccess && is16p(storage)) e = hipMalloc(&op->ciscale, sizeof(float) * 2 * op->V);
        if (e == hipSuccess && storage != QMG_C128) e = hipMalloc(&i64, sizeof(double) * 72 * op->V);
    }
    if (e == hipSuccess && (is16p(storage) || (eo && storage == QMG_C64))) e = hipMalloc(&c64, sizeof(double) * 72 * op->V);
    if (e != hipSuccess) {
        if (c64) (void)hipFree(c64);
        if (i64) (void)hipFree(i64);
        qmg_fine_op_destroy(op);
        return fail(QMG_ERR_NOMEM, "fine_op_create: clover temporaries: %s", hipGetErrorString(e));
    }
    const double diag = 4.0 + m0;
    if (storage == QMG_C128) {
        hipLaunchKernelGGL(k_pack_gauge<double>, dim3(nbU), dim3(256), 0, s, (cpx<double>*)op->U,
                           (const double2*)gauge, op->V, last, op->antiperiodic_t, ne);
        hipLaunchKernelGGL(k_clover_build<double>, dim3(nbS), dim3(128), 0, s, (double*)op->clov,
                           (const double2*)gauge, op->nbr, op->V, sb);
        if (eo)
            hipLaunchKernelGGL(k_clover_invert, dim3(nbS), dim3(128), 0, s, (double*)op->cinv,
                               (const double*)op->clov, op->V, diag);
    } else if (storage == QMG_C64) {
        hipLaunchKernelGGL(k_pack_gauge<float>, dim3(nbU), dim3(256), 0, s, (cpx<float>*)op->U,
                           (const double2*)gauge, op->V, last, op->antiperiodic_t, ne);
        hipLaunchKernelGGL(k_clover_build<float>, dim3(nbS), dim3(128), 0, s, (float*)op->clov,
                           (const double2*)gauge, op->nbr, op->V, sb);
        if (eo) {
            hipLaunchKernelGGL(k_clover_build<double>, dim3(nbS), dim3(128), 0, s, (double*)c64,
                               (const double2*)gauge, op->nbr, op->V, sb);
            hipLaunchKernelGGL(k_clover_invert, dim3(nbS), dim3(128), 0, s, (double*)i64, (const double*)c64,
                               op->V, diag);
            hipLaunchKernelGGL(k_real_to_f32, dim3((unsigned)((72 * op->V + 255) / 256)), dim3(256), 0, s,
                               (float*)op->cinv, (const double*)i64, 72 * op->V);
        }
    } else {
        // the clover term is built in FP64 in a temporary, then scaled per
        // (chirality, site) and rounded to 16 bits (its inverse likewise);
        // a NaN or Inf met on the way is reported below
        unsigned* nf = nullptr;
        st = nonfinite_flag(&nf);
        if (st != QMG_OK) {
            if (c64) (void)hipFree(c64);
            if (i64) (void)hipFree(i64);
            qmg_fine_op_destroy(op);
            return st;
        }
        hipLaunchKernelGGL(k_clover_build<double>, dim3(nbS), dim3(128), 0, s, (double*)c64,
                           (const double2*)gauge, op->nbr, op->V, sb);
        if (eo)
            hipLaunchKernelGGL(k_clover_invert, dim3(nbS), dim3(128), 0, s, (double*)i64, (const double*)c64,
                               op->V, diag);
        if (storage == QMG_H16) {
            hipLaunchKernelGGL(k_pack_gauge16<FMT_H16>, dim3(nbU), dim3(256), 0, s, (uint32_t*)op->U,
                               (const double2*)gauge, op->V, last, op->antiperiodic_t, ne, nf);
            hipLaunchKernelGGL(k_clover_pack16<FMT_H16>, dim3(nbS), dim3(128), 0, s, (uint32_t*)op->clov,
                               op->cscale, (const double*)c64, op->V, nf);
            if (eo)
                hipLaunchKernelGGL(k_clover_pack16<FMT_H16>, dim3(nbS), dim3(128), 0, s, (uint32_t*)op->cinv,
                                   op->ciscale, (const double*)i64, op->V, nf);
        } else {
            hipLaunchKernelGGL(k_pack_gauge16<FMT_B16>, dim3(nbU), dim3(256), 0, s, (uint32_t*)op->U,
                               (const double2*)gauge, op->V, last, op->antiperiodic_t, ne, nf);
            hipLaunchKernelGGL(k_clover_pack16<FMT_B16>, dim3(nbS), dim3(128), 0, s, (uint32_t*)op->clov,
                               op->cscale, (const double*)c64, op->V, nf);
            if (eo)
                hipLaunchKernelGGL(k_clover_pack16<FMT_B16>, dim3(nbS), dim3(128), 0, s, (uint32_t*)op->cinv,
                                   op->ciscale, (const double*)i64, op->V, nf);
        }
    }
    if (c64 || i64) {
        (void)hipStreamSynchronize(s);
        if (c64) (void)hipFree(c64);
        if (i64) (void)hipFree(i64);
    }
    const hipError_t le = hipGetLastError();
    if (eo && le == hipSuccess) {
        // parity-order copies for the red-black kernels; the inverse of the
        // site-local block is kept in parity order only
        const int64_t V = op->V;
        const int lb = storage == QMG_C128 ? 16 : storage == QMG_C64 ? 8 : 4;   // bytes per stored link entry
        const int64_t lk = 4 * ne;                                              // link entries per site
        const int cb = is16p(storage) ? 4 : (int)rb;                            // bytes per clover element
        const int64_t ck = is16p(storage) ? 36 : 72;                            // clover elements per site
        void *ci = nullptr, *cis = nullptr;
        e = hipMalloc(&op->U_eo, (size_t)lb * lk * V);
        if (e == hipSuccess) e = hipMalloc(&op->clov_eo, (size_t)cb * ck * V);
        if (e == hipSuccess) e = hipMalloc(&op->hnb, sizeof(int) * 8 * V);
        if (e == hipSuccess) e = hipMalloc(&ci, (size_t)cb * ck * V);
        if (e == hipSuccess && is16p(storage)) e = hipMalloc(&op->cscale_eo, sizeof(float) * 2 * V);
        if (e == hipSuccess && is16p(storage)) e = hipMalloc(&cis, sizeof(float) * 2 * V);
        if (e != hipSuccess) {
            if (ci) (void)hipFree(ci);
            if (cis) (void)hipFree(cis);
            qmg_fine_op_destroy(op);
            return fail(QMG_ERR_NOMEM, "fine_op_create: red-black copies: %s", hipGetErrorString(e));
        }
        auto permute = [&](void* dst, const void* src, int64_t K, int eb) {
            const unsigned g = (unsigned)((K * V + 255) / 256);
            if (eb == 16)
                hipLaunchKernelGGL(k_to_parity_order<uint4>, dim3(g), dim3(256), 0, s, (uint4*)dst, (const uint4*)src,
                                   op->hsite, K, V);
            else if (eb == 8)
                hipLaunchKernelGGL(k_to_parity_order<uint2>, dim3(g), dim3(256), 0, s, (uint2*)dst, (const uint2*)src,
                                   op->hsite, K, V);
            else
                hipLaunchKernelGGL(k_to_parity_order<uint32_t>, dim3(g), dim3(256), 0, s, (uint32_t*)dst,
                                   (const uint32_t*)src, op->hsite, K, V);
        };
        permute(op->U_eo, op->U, lk, lb);
        permute(op->clov_eo, op->clov, ck, cb);
        permute(ci, op->cinv, ck, cb);
        if (is16p(storage)) {
            permute(op->cscale_eo, op->cscale, 2, 4);
            permute(cis, op->ciscale, 2, 4);
        }
        hipLaunchKernelGGL(k_nbr_parity_order, dim3((unsigned)((8 * V + 255) / 256)), dim3(256), 0, s, op->hnb,
                           op->nbr, op->hsite, V);
        (void)hipStreamSynchronize(s);
        (void)hipFree(op->cinv);
        op->cinv = ci;
        if (is16p(storage)) {
            (void)hipFree(op->ciscale);
            op->ciscale = (float*)cis;
        }
    }
    e = le != hipSuccess ? le : hipGetLastError();
    if (e != hipSuccess) {
        qmg_fine_op_destroy(op);
        return fail(QMG_ERR_HIP, "fine_op_create: launch: %s", hipGetErrorString(e));
    }
    if (is16p(storage)) {
        st = take_nonfinite(s, "fine_op_create");
        if (st != QMG_OK) {
            qmg_fine_op_destroy(op);
            return st;
        }
    }
    *out = op;
    return QMG_OK;
}

extern "C" qmg_status qmg_fine_op_create(const int dims[4], const void* gauge, double m0, double csw,
                                         int antiperiodic_t, qmg_prec storage, void* stream, qmg_fine_op* out) {
    return qmg_fine_op_create_ex(dims, gauge, m0, csw, antiperiodic_t, storage, 18, stream, out);
}

extern "C" qmg_status qmg_fine_op_export_clover(qmg_fine_op op, void* A, void* stream) {
    if (!op || !A) return fail(QMG_ERR_ARG, "fine_op_export_clover: NULL argument");
    hipStream_t s = as_stream(stream);
    const unsigned nb = (unsigned)((op->V + 127) / 128);
    switch (op->storage) {
        case QMG_C128: hipLaunchKernelGGL(k_clover_export<FMT_F64>, dim3(nb), dim3(128), 0, s, (double2*)A, op->clov, op->cscale, op->V); break;
        case QMG_C64: hipLaunchKernelGGL(k_clover_export<FMT_F32>, dim3(nb), dim3(128), 0, s, (double2*)A, op->clov, op->cscale, op->V); break;
        case QMG_H16: hipLaunchKernelGGL(k_clover_export<FMT_H16>, dim3(nb), dim3(128), 0, s, (double2*)A, op->clov, op->cscale, op->V); break;
        default: hipLaunchKernelGGL(k_clover_export<FMT_B16>, dim3(nb), dim3(128), 0, s, (double2*)A, op->clov, op->cscale, op->V);
    }
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

extern "C" qmg_status qmg_fine_op_export_links(qmg_fine_op op, void* gauge, void* stream) {
    if (!op || !gauge) return fail(QMG_ERR_ARG, "fine_op_export_links: NULL argument");
    hipStream_t s = as_stream(stream);
    const unsigned nb = (unsigned)((4 * op->V + 255) / 256);
    const int64_t last = op->last;
    double2* G = static_cast<double2*>(gauge);
    const bool c12 = op->link_reals == 12;
#define QMG_LX(F)                                                                                                  \
    do {                                                                                                           \
        if (c12) hipLaunchKernelGGL((k_links_export<F, 12>), dim3(nb), dim3(256), 0, s, G, op->U, op->V, last,     \
                                    op->antiperiodic_t);                                                           \
        else hipLaunchKernelGGL((k_links_export<F, 18>), dim3(nb), dim3(256), 0, s, G, op->U, op->V, last,         \
                                op->antiperiodic_t);                                                               \
    } while (0)
    switch (op->storage) {
        case QMG_C128: hipLaunchKernelGGL((k_links_export<FMT_F64, 18>), dim3(nb), dim3(256), 0, s, G, op->U, op->V, last, op->antiperiodic_t); break;
        case QMG_C64: QMG_LX(FMT_F32); break;
        case QMG_H16: QMG_LX(FMT_H16); break;
        default: QMG_LX(FMT_B16);
    }
#undef QMG_LX
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

extern "C" qmg_status qmg_wilson_clover_dslash(qmg_fine_op op, const void* in, void* out, int nrhs, qmg_prec prec,
                                               void* stream) {
    if (!op || !in || !out) return fail(QMG_ERR_ARG, "wilson_clover_dslash: NULL argument");
    if (nrhs < 1 || nrhs > kMaxFieldBatch)
        return fail(QMG_ERR_ARG, "wilson_clover_dslash: nrhs %d not in [1, %d]", nrhs, kMaxFieldBatch);
    const bool ok = prec == op->storage || (is16p(op->storage) && prec == QMG_C64);
    if (!ok)
        return fail(QMG_ERR_PREC, "wilson_clover_dslash: vector precision %d does not fit operator storage %d",
                    (int)prec, (int)op->storage);
    if (is16p(prec)) return fail(QMG_ERR_PREC, "wilson_clover_dslash: 16-bit vectors go through wilson_clover_dslash_scaled");
    if (in == out) return fail(QMG_ERR_ARG, "wilson_clover_dslash: in and out alias");
    return wilson_any(op, in, nullptr, out, nullptr, prec, nrhs, as_stream(stream));
}

extern "C" qmg_status qmg_wilson_clover_dslash_scaled(qmg_fine_op op, const void* in, const float* in_scale,
                                                      void* out, float* out_scale, qmg_prec prec, void* stream) {
    if (!op || !in || !in_scale || !out || !out_scale)
        return fail(QMG_ERR_ARG, "wilson_clover_dslash_scaled: NULL argument");
    if (!is16p(op->storage) || !is16p(prec))
        return fail(QMG_ERR_PREC, "wilson_clover_dslash_scaled: needs 16-bit operator storage and vectors");
    if (in == out || in_scale == out_scale) return fail(QMG_ERR_ARG, "wilson_clover_dslash_scaled: in and out alias");
    return wilson_any(op, in, in_scale, out, out_scale, prec, 1, as_stream(stream));
}

// ---------------------------------------------------------- red-black entry points
static qmg_status schur_checks(qmg_fine_op op, int nrhs, qmg_prec prec, const char* what) {
    if (!op) return fail(QMG_ERR_ARG, "%s: NULL operator", what);
    if (!op->hsite) return fail(QMG_ERR_SHAPE, "%s: the red-black form needs every lattice extent even", what);
    if (nrhs < 1 || nrhs > kMaxFieldBatch) return fail(QMG_ERR_ARG, "%s: nrhs %d not in [1, %d]", what, nrhs, kMaxFieldBatch);
    const bool ok = op->storage == QMG_C128 ? prec == QMG_C128 : prec == QMG_C64;
    if (!ok) return fail(QMG_ERR_PREC, "%s: vector precision %d does not fit operator storage %d", what, (int)prec,
                         (int)op->storage);
    return QMG_OK;
}

// the operator's odd half-lattice scratch for nrhs members
static qmg_status schur_tmp(qmg_fine_op op, int nrhs, qmg_prec prec, hipStream_t s) {
    const size_t need = (size_t)nrhs * (op->V / 2) * 12 * (prec == QMG_C128 ? 16 : 8);
    if (op->eo_tmp_bytes >= need) return QMG_OK;
    if (op->eo_tmp) {
        QMG_HIP(hipStreamSynchronize(s));
        (void)hipFree(op->eo_tmp);
        op->eo_tmp = nullptr;
        op->eo_tmp_bytes = 0;
    }
    QMG_HIP(hipMalloc(&op->eo_tmp, need));
    op->eo_tmp_bytes = need;
    return QMG_OK;
}

extern "C" qmg_status qmg_wilson_clover_schur(qmg_fine_op op, const void* in_e, void* out_e, int nrhs, qmg_prec prec,
                                              void* stream) {
    QMG_TRY(schur_checks(op, nrhs, prec, "wilson_clover_schur"));
    if (!in_e || !out_e) return fail(QMG_ERR_ARG, "wilson_clover_schur: NULL field");
    if (in_e == out_e) return fail(QMG_ERR_ARG, "wilson_clover_schur: in and out alias");
    hipStream_t s = as_stream(stream);
    QMG_TRY(schur_tmp(op, nrhs, prec, s));
    return fine_schur_apply(op, in_e, out_e, op->eo_tmp, prec, nrhs, s);
}

extern "C" qmg_status qmg_wilson_clover_schur_scaled(qmg_fine_op op, const void* in_e, const float* in_scale,
                                                     void* out_e, float* out_scale, int nrhs, void* stream) {
    if (!op) return fail(QMG_ERR_ARG, "wilson_clover_schur_scaled: NULL operator");
    if (op->storage != QMG_H16 && op->storage != QMG_B16)
        return fail(QMG_ERR_PREC, "wilson_clover_schur_scaled: needs an operator with 16-bit storage");
    QMG_TRY(schur_checks(op, nrhs, QMG_C64, "wilson_clover_schur_scaled"));
    if (!in_e || !in_scale || !out_e || !out_scale) return fail(QMG_ERR_ARG, "wilson_clover_schur_scaled: NULL field");
    if (in_e == out_e || in_scale == out_scale)
        return fail(QMG_ERR_ARG, "wilson_clover_schur_scaled: in and out alias");
    hipStream_t s = as_stream(stream);
    // the odd intermediate (48 bytes and a scale per site) in the operator's
    // scratch, which holds 96 bytes per site and member
    QMG_TRY(schur_tmp(op, nrhs, QMG_C64, s));
    const int64_t n16 = (int64_t)nrhs * (op->V / 2) * 48;
    float* ts = reinterpret_cast<float*>(static_cast<char*>(op->eo_tmp) + n16);
    return fine_schur_apply16(op, in_e, in_scale, out_e, out_scale, op->eo_tmp, ts, nrhs, s);
}

extern "C" qmg_status qmg_wilson_clover_schur_source(qmg_fine_op op, const void* b, void* bhat_e, int nrhs,
                                                     qmg_prec prec, void* stream) {
    QMG_TRY(schur_checks(op, nrhs, prec, "wilson_clover_schur_source"));
    if (!b || !bhat_e) return fail(QMG_ERR_ARG, "wilson_clover_schur_source: NULL field");
    if (b == bhat_e) return fail(QMG_ERR_ARG, "wilson_clover_schur_source: b and bhat alias");
    hipStream_t s = as_stream(stream);
    QMG_TRY(schur_tmp(op, nrhs, prec, s));
    return fine_schur_source(op, b, bhat_e, op->eo_tmp, prec, nrhs, s);
}

extern "C" qmg_status qmg_wilson_clover_schur_reconstruct(qmg_fine_op op, const void* x_e, const void* b, void* x,
                                                          int nrhs, qmg_prec prec, void* stream) {
    QMG_TRY(schur_checks(op, nrhs, prec, "wilson_clover_schur_reconstruct"));
    if (!x_e || !b || !x) return fail(QMG_ERR_ARG, "wilson_clover_schur_reconstruct: NULL field");
    if (x == b || x == x_e) return fail(QMG_ERR_ARG, "wilson_clover_schur_reconstruct: x aliases an input");
    return fine_schur_reconstruct(op, x_e, b, x, prec, nrhs, as_stream(stream));
}

// ------------------------------------------------------ allocation-free Schur
// For callers that cannot allocate (code under graph capture, tight serving
// loops): the odd half-lattice scratch of the Schur operator lives in a
// fixed device array instead of the operator's grown buffer.  Each device
// the library runs on holds its own copy for the life of the process; host
// code only ever uses its device address, looked up once per device.
namespace {
constexpr size_t kNoAllocScratchBytes = (size_t)16 << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;   // per device

qmg_status scratch_address(void** out) {
    int dev = 0;
    QMG_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(QMG_ERR_HIP, "wilson_clover_schur_noalloc: scratch address on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return QMG_OK;
}
}  // namespace

extern "C" qmg_status qmg_wilson_clover_schur_noalloc(qmg_fine_op op, const void* in_e, void* out_e, int nrhs,
                                                      qmg_prec prec, void* stream) {
    QMG_TRY(schur_checks(op, nrhs, prec, "wilson_clover_schur_noalloc"));
    if (!in_e || !out_e) return fail(QMG_ERR_ARG, "wilson_clover_schur_noalloc: NULL field");
    if (in_e == out_e) return fail(QMG_ERR_ARG, "wilson_clover_schur_noalloc: in and out alias");
    const size_t need = (size_t)nrhs * (op->V / 2) * 12 * (prec == QMG_C128 ? 16 : 8);
    if (need > kNoAllocScratchBytes)
        return fail(QMG_ERR_ARG, "wilson_clover_schur_noalloc: %zu bytes of scratch needed, the fixed scratch holds %zu",
                    need, kNoAllocScratchBytes);
    void* tmp = nullptr;
    QMG_TRY(scratch_address(&tmp));
    return fine_schur_apply(op, in_e, out_e, tmp, prec, nrhs, as_stream(stream));
}
