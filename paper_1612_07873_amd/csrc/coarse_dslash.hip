// Coarse-grid operator, Eq. (3), applied with the fine-grained split of
// Sec. 6.1-6.4 re-designed for CDNA4 wave64.
//
// Work decomposition.  Per coarse site the operator is one dense
// (N x 9N) * (9N) product: the concatenated row [X | Y_0 .. Y_7] times the
// stacked input [u(x); u(x+hop_0); ..; u(x+hop_7)].  A work-group owns one
// site (grid parallelism, Sec. 6.1) and a tile of `rows` output rows
// (colour-spin parallelism, Sec. 6.2).  The 9N-long row is cut into 16-byte
// chunks (1 complex in FP64, 2 in FP32, 4 in FP16/BF16) and chunk j goes to
// split-lane s = j mod split: this one split covers both the
// stencil-direction split (Sec. 6.3, chunks of different d) and the
// dot-product split (Sec. 6.4, chunks of the same d), and the partial sums
// meet once in LDS before the single store.  The site index and its 8
// neighbours come from a precomputed table, so no integer division by
// lattice extents is done in the kernel (the indexing cost Sec. 6.5 names as
// the Amdahl limiter on the smallest grids).
//
// Link layout.  Chunks are stored [site][j][row] (row fastest).  For a fixed
// chunk index the rows of a site are contiguous, and consecutive split-lanes
// read consecutive chunk indices, so the rows*split threads of a work-group
// read one contiguous span of rows*split*16 bytes per step whatever the split:
// every load is a fully coalesced 16-byte-per-lane load, and the layout does
// not depend on the launch shape.  The 9 input vectors of the site are staged
// once in LDS (decoded to the accumulation precision, with the 16-bit link
// scale of each direction folded in); the first link chunks of every thread
// are already in flight while the staging loads complete.  All lanes of a wave
// read the same one or two LDS addresses per step (an LDS broadcast).
//
// Precisions (the paper's 16-bit storage exists to relieve bandwidth,
// Sec. 4 and 7.1):
//   C128: complex128 links and vectors, FP64 arithmetic;
//   C64:  complex64 links and vectors, FP32 arithmetic;
//   H16 / B16: links as FP16 / BF16 pairs with one FP32 scale per (site,
//         direction block), value = scale * stored; FP32 arithmetic; vectors
//         either complex64 or 16-bit pairs with one FP32 scale per site
//         (scale = largest |re| or |im| of the site's N components).
#include "codes16.h"
#include "handles.h"

#include <algorithm>
#include <vector>

namespace qmg {

template <int F> struct Fmt;
template <> struct Fmt<FMT_F64> { using R = double; using C = double2; static constexpr int cpc = 1; };
template <> struct Fmt<FMT_F32> { using R = float; using C = float4; static constexpr int cpc = 2; };
template <> struct Fmt<FMT_H16> { using R = float; using C = uint4; static constexpr int cpc = 4; };
template <> struct Fmt<FMT_B16> { using R = float; using C = uint4; static constexpr int cpc = 4; };

// a += chunk * b[0..cpc)
__device__ __forceinline__ void chunk_mac(const double2 a, const cpx<double>* b, double& ar, double& ai) {
    cmac(ar, ai, a.x, a.y, b[0].re, b[0].im);
}
__device__ __forceinline__ void chunk_mac(const float4 a, const cpx<float>* b, float& ar, float& ai) {
    cmac(ar, ai, a.x, a.y, b[0].re, b[0].im);
    cmac(ar, ai, a.z, a.w, b[1].re, b[1].im);
}
template <int F>
__device__ __forceinline__ void chunk_mac16(const uint4 a, const cpx<float>* b, float& ar, float& ai) {
    const uint32_t w[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const cpx<float> v = dec_pair<F>(w[q]);
        cmac(ar, ai, v.re, v.im, b[q].re, b[q].im);
    }
}
template <int F, typename C, typename R>
__device__ __forceinline__ void mac(const C a, const cpx<R>* b, R& ar, R& ai) {
    if constexpr (F == FMT_H16 || F == FMT_B16) chunk_mac16<F>(a, b, ar, ai);
    else chunk_mac(a, b, ar, ai);
}

__device__ __forceinline__ const double2* link_src(const double2* X, const double2* Y, int64_t V, int N,
                                                   int64_t site, int r, int e) {
    const int d = e / N, c = e - (e / N) * N;
    return d == 0 ? X + (site * N + r) * N + c : Y + ((((int64_t)(d - 1)) * V + site) * N + r) * N + c;
}
__device__ __forceinline__ double2* link_dst(double2* X, double2* Y, int64_t V, int N, int64_t site, int r, int e) {
    const int d = e / N, c = e - (e / N) * N;
    return d == 0 ? X + (site * N + r) * N + c : Y + ((((int64_t)(d - 1)) * V + site) * N + r) * N + c;
}

// ---------------------------------------------------------------- packing
// Canonical complex128 X, Y -> chunk layout [site][j][row].  One thread per chunk.
template <int F>
__global__ void k_pack(typename Fmt<F>::C* __restrict__ L, const float* __restrict__ lscale,
                       const double2* __restrict__ X, const double2* __restrict__ Y, int64_t V, int N, int J) {
    constexpr int cpc = Fmt<F>::cpc;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= V * J * N) return;
    const int r = (int)(g % N);
    const int64_t t = g / N;
    const int j = (int)(t % J);
    const int64_t site = t / J;
    const double2* p = link_src(X, Y, V, N, site, r, j * cpc);
    if constexpr (F == FMT_F64) {
        L[g] = p[0];
    } else if constexpr (F == FMT_F32) {
        L[g] = make_float4((float)p[0].x, (float)p[0].y, (float)p[1].x, (float)p[1].y);
    } else {
        const float s = lscale[site * 9 + (j * cpc) / N];
        const float inv = s > 0 ? 1.0f / s : 0.0f;
        uint4 c;
        c.x = enc_pair<F>((float)p[0].x * inv, (float)p[0].y * inv);
        c.y = enc_pair<F>((float)p[1].x * inv, (float)p[1].y * inv);
        c.z = enc_pair<F>((float)p[2].x * inv, (float)p[2].y * inv);
        c.w = enc_pair<F>((float)p[3].x * inv, (float)p[3].y * inv);
        L[g] = c;
    }
}

template <int F>
__global__ void k_unpack(const typename Fmt<F>::C* __restrict__ L, const float* __restrict__ lscale,
                         double2* __restrict__ X, double2* __restrict__ Y, int64_t V, int N, int J) {
    constexpr int cpc = Fmt<F>::cpc;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= V * J * N) return;
    const int r = (int)(g % N);
    const int64_t t = g / N;
    const int j = (int)(t % J);
    const int64_t site = t / J;
    double2* p = link_dst(X, Y, V, N, site, r, j * cpc);
    const auto a = L[g];
    if constexpr (F == FMT_F64) {
        p[0] = a;
    } else if constexpr (F == FMT_F32) {
        p[0] = make_double2(a.x, a.y);
        p[1] = make_double2(a.z, a.w);
    } else {
        const double s = lscale[site * 9 + (j * cpc) / N];
        const uint32_t w[4] = {a.x, a.y, a.z, a.w};
        for (int q = 0; q < 4; ++q) {
            const cpx<float> v = dec_pair<F>(w[q]);
            p[q] = make_double2(s * v.re, s * v.im);
        }
    }
}

// Per (site, direction block) scale: largest |re| or |im| of the N x N block.
__global__ __launch_bounds__(256) void k_link_scales(float* __restrict__ lscale, const double2* __restrict__ X,
                                                     const double2* __restrict__ Y, int64_t V, int N,
                                                     unsigned* __restrict__ nf) {
    __shared__ double red[4];
    const int64_t site = blockIdx.x / 9;
    const int d = blockIdx.x % 9;
    const double2* B = d == 0 ? X + site * N * N : Y + (((int64_t)(d - 1)) * V + site) * N * N;
    double m = 0;
    bool bad = false;
    for (int i = threadIdx.x; i < N * N; i += blockDim.x) {
        bad = bad || !(isfinite(B[i].x) && isfinite(B[i].y));
        m = fmax(m, fmax(fabs(B[i].x), fabs(B[i].y)));
    }
    note_nonfinite(nf, bad);
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float sc = (float)fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
        note_nonfinite(nf, !isfinite(sc));
        lscale[blockIdx.x] = sc;
    }
}

// ------------------------------------------------------------------ stencil
// Red-black pieces (EO): the operator is one parity's half of a coarse
// operator (sites = half-lattice sites, nbr = half-lattice indices of the
// other parity), and only the directions d0 .. d0+nd-1 of the stacked row
// [X | Y_0 .. Y_7] are applied: d0 = 1 drops the site-local block, nd = 1
// keeps only it.  The site-local block multiplies `uself` (at sidx[site], or
// at site if sidx is NULL, member stride vself sites) and the output goes to
// oidx[site] (or site; member stride vout), so a piece can read and write
// whole-lattice fields.

// A link chunk, read once per application: a non-temporal load, so the
// link stream does not push the input vector's blocks (each read by nine
// sites) out of the caches.
template <typename C> __device__ __forceinline__ C ld_link(const C* p) {
    static_assert(sizeof(C) == 16, "16-byte link chunks");
    typedef int i4 __attribute__((ext_vector_type(4)));
    const i4 v = __builtin_nontemporal_load(reinterpret_cast<const i4*>(p));
    C r;
    __builtin_memcpy(&r, &v, sizeof(C));
    return r;
}

// VF: 0 = vectors in the accumulation precision, else 16-bit pairs (format VF) + per-site scale.
template <int F, int VF, int PRE, bool EO = false>
__global__ __launch_bounds__(1024) void k_coarse_dslash(const typename Fmt<F>::C* __restrict__ L,
                                                        const float* __restrict__ lscale,
                                                        const int* __restrict__ nbr, const void* __restrict__ uin,
                                                        const float* __restrict__ uscale, void* __restrict__ yout,
                                                        float* __restrict__ yscale, int N, int J, int rows, int split,
                                                        int ntiles, int64_t V, EoArgs ea) {
    using R = typename Fmt<F>::R;
    using C = typename Fmt<F>::C;
    constexpr int cpc = Fmt<F>::cpc;
    extern __shared__ __align__(16) unsigned char smem[];
    cpx<R>* ul = reinterpret_cast<cpx<R>*>(smem);  // [9N] stacked inputs
    cpx<R>* red = ul + 9 * N;                       // [split][rows] partial sums

    const int site = blockIdx.x / ntiles;
    const int tile = blockIdx.x - site * ntiles;
    const int64_t vo = (int64_t)blockIdx.y * V;      // batch member: its fields follow at member*V sites
    const int t = threadIdx.x;
    const int T = rows * split;
    const int rl = t % rows;
    const int s = t / rows;
    const int r = tile * rows + rl;
    const int d0 = EO ? ea.d0 : 0;
    const int nd = EO ? ea.nd : 9;
    const int K = (EO ? nd * N / cpc : J) / split;
    const C* Ls = L + ((int64_t)site * J + (EO ? d0 * N / cpc : 0)) * N + r;

    // first link chunks in flight before the staging barrier
    C a[PRE];
#pragma unroll
    for (int q = 0; q < PRE; ++q)
        if (q < K) a[q] = ld_link(Ls + (int64_t)(s + split * q) * N);

    for (int idx = t; idx < nd * N; idx += T) {
        const int dd = idx / N;
        const int d = dd + d0;
        const int c = idx - dd * N;
        cpx<R> v;
        if constexpr (EO) {
            const bool loc = d == 0;
            const int64_t src = loc ? (ea.sidx ? ea.sidx[site] : site) + (int64_t)blockIdx.y * ea.vself
                                    : nbr[site * 8 + d - 1] + vo;
            v = reinterpret_cast<const cpx<R>*>(loc ? ea.uself : uin)[src * N + c];
        } else if constexpr (VF == 0) {
            const int64_t src = (d == 0 ? site : nbr[site * 8 + d - 1]) + vo;
            v = reinterpret_cast<const cpx<R>*>(uin)[(int64_t)src * N + c];
        } else {
            const int64_t src = (d == 0 ? site : nbr[site * 8 + d - 1]) + vo;
            v = dec_pair<VF>(reinterpret_cast<const uint32_t*>(uin)[(int64_t)src * N + c]);
            const float su = uscale[src];
            v.re *= su;
            v.im *= su;
        }
        if constexpr (F == FMT_H16 || F == FMT_B16) {
            const float sl = lscale[site * 9 + d];
            v.re *= sl;
            v.im *= sl;
        }
        ul[idx] = v;
    }
    __syncthreads();

    R ar[4] = {0, 0, 0, 0}, ai[4] = {0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < PRE; ++q)
        if (q < K) mac<F>(a[q], ul + (s + split * q) * cpc, ar[q & 3], ai[q & 3]);
    int k = PRE;
    for (; k + 4 <= K; k += 4) {
        C b[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) b[q] = ld_link(Ls + (int64_t)(s + split * (k + q)) * N);
#pragma unroll
        for (int q = 0; q < 4; ++q) mac<F>(b[q], ul + (s + split * (k + q)) * cpc, ar[q], ai[q]);
    }
    for (; k < K; ++k) mac<F>(ld_link(Ls + (int64_t)(s + split * k) * N), ul + (s + split * k) * cpc, ar[0], ai[0]);
    R sr = (ar[0] + ar[1]) + (ar[2] + ar[3]);
    R si = (ai[0] + ai[1]) + (ai[2] + ai[3]);
    if (split > 1) {
        red[s * rows + rl] = cpx<R>{sr, si};
        __syncthreads();
        if (s == 0)
            for (int q = 1; q < split; ++q) {
                sr += red[q * rows + rl].re;
                si += red[q * rows + rl].im;
            }
    }
    if constexpr (EO) {
        const int64_t o = (ea.oidx ? ea.oidx[site] : site) + (int64_t)blockIdx.y * ea.vout;
        if (s == 0) reinterpret_cast<cpx<R>*>(yout)[o * N + r] = cpx<R>{sr, si};
    } else if constexpr (VF == 0) {
        if (s == 0) reinterpret_cast<cpx<R>*>(yout)[(site + vo) * N + r] = cpx<R>{sr, si};
    } else {
        // per-site output scale: all N rows of the site are in this work-group (ntiles == 1)
        __syncthreads();
        float* mx = reinterpret_cast<float*>(red);
        if (s == 0) mx[rl] = fmaxf(fabsf((float)sr), fabsf((float)si));
        __syncthreads();
        if (t == 0) {
            float m = 0.f;
            for (int i = 0; i < rows; ++i) m = fmaxf(m, mx[i]);
            mx[rows] = m;
            yscale[site + vo] = m;
        }
        __syncthreads();
        if (s == 0) {
            const float m = mx[rows];
            const float inv = m > 0 ? 1.0f / m : 0.0f;
            reinterpret_cast<uint32_t*>(yout)[(site + vo) * N + r] = enc_pair<VF>((float)sr * inv, (float)si * inv);
        }
    }
}

// -------------------------------------------------------- vector (de)quantise
template <int VF>
__global__ __launch_bounds__(64) void k_quantize(const float2* __restrict__ in, uint32_t* __restrict__ out,
                                                 float* __restrict__ scale, int N, unsigned* __restrict__ nf) {
    const int64_t site = blockIdx.x;
    float m = 0.f;
    bool bad = false;
    for (int c = threadIdx.x; c < N; c += 64) {
        const float2 v = in[site * N + c];
        bad = bad || !(isfinite(v.x) && isfinite(v.y));
        m = fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y)));
    }
    note_nonfinite(nf, bad);
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    const float inv = m > 0 ? 1.0f / m : 0.0f;
    for (int c = threadIdx.x; c < N; c += 64) {
        const float2 v = in[site * N + c];
        out[site * N + c] = enc_pair<VF>(v.x * inv, v.y * inv);
    }
    if (threadIdx.x == 0) scale[site] = m;
}

// [m][V][N] complex64 -> 16-bit [V][m][N] with one scale per (site, member) [V][m]
template <int VF>
__global__ __launch_bounds__(64) void k_quantize_perm(const float2* __restrict__ in, uint32_t* __restrict__ out,
                                                      float* __restrict__ scale, int64_t V, int m, int N,
                                                      unsigned* __restrict__ nf) {
    const int64_t g = blockIdx.x;           // input row: member g / V, site g % V
    const int64_t site = g % V, j = g / V;
    const int64_t o = site * m + j;         // output row
    float mx = 0.f;
    bool bad = false;
    for (int c = threadIdx.x; c < N; c += 64) {
        const float2 v = in[g * N + c];
        bad = bad || !(isfinite(v.x) && isfinite(v.y));
        mx = fmaxf(mx, fmaxf(fabsf(v.x), fabsf(v.y)));
    }
    note_nonfinite(nf, bad);
    for (int k = 32; k > 0; k >>= 1) mx = fmaxf(mx, __shfl_xor(mx, k, 64));
    const float inv = mx > 0 ? 1.0f / mx : 0.0f;
    for (int c = threadIdx.x; c < N; c += 64) {
        const float2 v = in[g * N + c];
        out[o * N + c] = enc_pair<VF>(v.x * inv, v.y * inv);
    }
    if (threadIdx.x == 0) scale[o] = mx;
}

template <int VF>
__global__ void k_dequantize(const uint32_t* __restrict__ in, const float* __restrict__ scale,
                             float2* __restrict__ out, int64_t V, int N) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= V * N) return;
    const cpx<float> v = dec_pair<VF>(in[g]);
    const float s = scale[g / N];
    out[g] = make_float2(v.re * s, v.im * s);
}

// ----------------------------------------------------------------- host side
static int fmt_of(qmg_prec p) {
    return p == QMG_C128 ? FMT_F64 : p == QMG_C64 ? FMT_F32 : p == QMG_H16 ? FMT_H16 : FMT_B16;
}
static int complex_per_chunk(qmg_prec p) { return p == QMG_C128 ? 1 : p == QMG_C64 ? 2 : 4; }
static bool is16(qmg_prec p) { return p == QMG_H16 || p == QMG_B16; }

// Built-in launch choice: all rows of a site per work-group; the smallest
// split (dividing J) that gives at least 2^18 threads in flight while
// keeping at least 4 chunks per thread; row tiles only when a work-group
// would exceed 1024 threads or the grid is very small.
static void default_launch(const qmg_coarse_op_s* op, int* rows, int* split) {
    const int J = op->J, N = op->N;
    const int64_t want = (int64_t)1 << 18;
    int best = 1;
    for (int s = 1; s <= J; ++s) {
        if (J % s) continue;
        if (J / s < 4) break;
        best = s;
        if (op->V * N * (int64_t)s >= want) break;
    }
    int rt = N;
    while (rt * best > 1024 || (rt % 2 == 0 && op->V * (N / rt) < 256 && rt > 8 && rt * best > 256)) {
        if (rt % 2) break;
        rt /= 2;
    }
    while (rt * best > 1024) {
        int s = best - 1;
        while (s > 1 && J % s) --s;
        best = s;
    }
    *rows = rt;
    *split = best;
}

static qmg_status validate_launch(const qmg_coarse_op_s* op, int rows, int split) {
    if (rows <= 0 || split <= 0 || op->N % rows || op->J % split || rows * split > 1024)
        return fail(QMG_ERR_ARG,
                    "coarse launch rows=%d split=%d invalid (need rows | N=%d, split | J=%d, rows*split <= 1024)",
                    rows, split, op->N, op->J);
    return QMG_OK;
}

template <int F, int VF>
static qmg_status launch_f(const qmg_coarse_op_s* op, int rows, int split, int pre, const void* in,
                           const float* in_scale, void* out, float* out_scale, int m, hipStream_t s) {
    using R = typename Fmt<F>::R;
    const int ntiles = op->N / rows;
    const size_t lds = sizeof(cpx<R>) * (9 * op->N + std::max(rows * split, rows + 1));
    const dim3 grid((unsigned)(op->V * ntiles), (unsigned)m), block((unsigned)(rows * split));
    const auto* L = reinterpret_cast<const typename Fmt<F>::C*>(op->links);
    const int K = op->J / split;
    if (pre <= 0) pre = K >= 16 ? 16 : 4;
#define QMG_CD_LAUNCH(P)                                                                                          \
    hipLaunchKernelGGL((k_coarse_dslash<F, VF, P>), grid, block, lds, s, L, op->lscale, op->nbr, in, in_scale, out, \
                       out_scale, op->N, op->J, rows, split, ntiles, op->V, EoArgs{})
    if (pre >= 16) QMG_CD_LAUNCH(16);
    else if (pre >= 8) QMG_CD_LAUNCH(8);
    else if (pre >= 4) QMG_CD_LAUNCH(4);
    else QMG_CD_LAUNCH(1);
#undef QMG_CD_LAUNCH
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

qmg_status coarse_dslash_launch(const qmg_coarse_op_s* op, int rows, int split, int pre, const void* in,
                                const float* in_scale, void* out, float* out_scale, qmg_prec vprec, hipStream_t s,
                                int m) {
    const bool v16 = is16(vprec);
    if (v16 && rows != op->N) {  // per-site output scale needs the whole site in one work-group
        rows = op->N;
        while (rows * split > 1024 || op->J % split) --split;
    }
    switch (op->storage) {
        case QMG_C128: return launch_f<FMT_F64, 0>(op, rows, split, pre, in, nullptr, out, nullptr, m, s);
        case QMG_C64: return launch_f<FMT_F32, 0>(op, rows, split, pre, in, nullptr, out, nullptr, m, s);
        case QMG_H16:
            if (vprec == QMG_C64) return launch_f<FMT_H16, 0>(op, rows, split, pre, in, nullptr, out, nullptr, m, s);
            if (vprec == QMG_H16)
                return launch_f<FMT_H16, FMT_H16>(op, rows, split, pre, in, in_scale, out, out_scale, m, s);
            return launch_f<FMT_H16, FMT_B16>(op, rows, split, pre, in, in_scale, out, out_scale, m, s);
        default:
            if (vprec == QMG_C64) return launch_f<FMT_B16, 0>(op, rows, split, pre, in, nullptr, out, nullptr, m, s);
            if (vprec == QMG_H16)
                return launch_f<FMT_B16, FMT_H16>(op, rows, split, pre, in, in_scale, out, out_scale, m, s);
            return launch_f<FMT_B16, FMT_B16>(op, rows, split, pre, in, in_scale, out, out_scale, m, s);
    }
}

// Built-in launch for a piece of nd directions: all rows of a site per
// work-group (as many as fit 1024 threads), the split the largest divisor of
// the piece's chunk count that leaves at least 4 chunks per thread and keeps
// about 2^18 threads in flight.
void eo_piece_launch(const qmg_coarse_op_s* op, int nd, int* rows, int* split) {
    const int cpc = complex_per_chunk(op->storage);
    const int J = nd * op->N / cpc, N = op->N;
    int best = 1;
    for (int sp = 1; sp <= J; ++sp) {
        if (J % sp) continue;
        if (J / sp < 4) break;
        if (N * sp > 1024) break;
        best = sp;
        if (op->V * N * (int64_t)sp >= ((int64_t)1 << 18)) break;
    }
    int rt = N;
    while (rt * best > 1024 && rt % 2 == 0) rt /= 2;
    *rows = rt;
    *split = best;
}

// One red-black piece on a half operator (vectors complex128 / complex64 as
// the storage: complex128 for complex128 storage, complex64 otherwise).
template <int F>
static qmg_status launch_eo_f(const qmg_coarse_op_s* op, const EoArgs& ea, const void* in, void* out, int m,
                              hipStream_t s) {
    using R = typename Fmt<F>::R;
    int rows, split;
    eo_piece_launch(op, ea.nd, &rows, &split);
    const int ntiles = op->N / rows;
    const size_t lds = sizeof(cpx<R>) * (9 * op->N + std::max(rows * split, rows + 1));
    const dim3 grid((unsigned)(op->V * ntiles), (unsigned)m), block((unsigned)(rows * split));
    const auto* L = reinterpret_cast<const typename Fmt<F>::C*>(op->links);
    const int K = ea.nd * op->N / Fmt<F>::cpc / split;
    if (K >= 16)
        hipLaunchKernelGGL((k_coarse_dslash<F, 0, 16, true>), grid, block, lds, s, L, op->lscale, op->nbr, in, nullptr,
                           out, nullptr, op->N, op->J, rows, split, ntiles, op->V, ea);
    else
        hipLaunchKernelGGL((k_coarse_dslash<F, 0, 4, true>), grid, block, lds, s, L, op->lscale, op->nbr, in, nullptr,
                           out, nullptr, op->N, op->J, rows, split, ntiles, op->V, ea);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

qmg_status coarse_eo_launch(const qmg_coarse_op_s* op, const EoArgs& ea, const void* in, void* out, qmg_prec vprec,
                            int m, hipStream_t s) {
    const bool ok = op->storage == QMG_C128 ? vprec == QMG_C128 : vprec == QMG_C64;
    if (!ok) return fail(QMG_ERR_PREC, "coarse red-black piece: vector precision %d for storage %d", (int)vprec,
                         (int)op->storage);
    switch (op->storage) {
        case QMG_C128: return launch_eo_f<FMT_F64>(op, ea, in, out, m, s);
        case QMG_C64: return launch_eo_f<FMT_F32>(op, ea, in, out, m, s);
        case QMG_H16: return launch_eo_f<FMT_H16>(op, ea, in, out, m, s);
        default: return launch_eo_f<FMT_B16>(op, ea, in, out, m, s);
    }
}

qmg_status coarse_dslash_any(const qmg_coarse_op_s* op, const void* in, const float* in_scale, void* out,
                             float* out_scale, qmg_prec vprec, hipStream_t s) {
    return coarse_dslash_launch(op, op->rows, op->split, op->pre, in, in_scale, out, out_scale, vprec, s, 1);
}

qmg_status coarse_mrhs(qmg_coarse_op_s* op, const void* in, const float* sc, void* out, int nrhs, int rpw,
                       hipStream_t s, int64_t ors);

bool coarse_batch_uses_mfma(const qmg_coarse_op_s* op, int m) {
    return is16(op->storage) && op->N % 16 == 0 && op->N <= 64 && (m == 8 || m == 16 || m == 32 || m == 64);
}

// Solver-side batched application, fields [m][V][N] in `vprec` (complex128 or
// complex64).  A 16-bit operator with m in {8, 16, 32, 64} runs on the matrix
// cores: the inputs are rounded to 16 bits with one scale per (site, member)
// into q16 [V][m][N] / qsc [V][m] (caller-provided), then one multi-RHS launch
// writes the complex64 outputs in place.  Otherwise one launch of the
// single-RHS kernel covers all members (grid dimension y).
qmg_status coarse_apply(qmg_coarse_op_s* op, const void* in, void* out, qmg_prec vprec, int m, void* q16,
                        float* qsc, hipStream_t s) {
    if (m > 1 && vprec == QMG_C64 && q16 && coarse_batch_uses_mfma(op, m)) {
        unsigned* nf = nullptr;
        QMG_TRY(nonfinite_flag(&nf));
        if (op->storage == QMG_H16)
            hipLaunchKernelGGL(k_quantize_perm<FMT_H16>, dim3((unsigned)(op->V * m)), dim3(64), 0, s, (const float2*)in,
                               (uint32_t*)q16, qsc, op->V, m, op->N, nf);
        else
            hipLaunchKernelGGL(k_quantize_perm<FMT_B16>, dim3((unsigned)(op->V * m)), dim3(64), 0, s, (const float2*)in,
                               (uint32_t*)q16, qsc, op->V, m, op->N, nf);
        QMG_LAUNCH_CHECK();
        return coarse_mrhs(op, q16, qsc, out, m, 0, s, op->V * op->N);
    }
    return coarse_dslash_launch(op, op->rows, op->split, op->pre, in, nullptr, out, nullptr, vprec, s, m);
}

}  // namespace qmg

using namespace qmg;

namespace qmg {
// The operator from canonical complex128 X [V][N][N], Y [8][V][N][N] on V
// sites; nbr: a device neighbour table [V][8] the operator takes over, or NULL
// to build the lattice's own from dims (V = volume(dims) then).
qmg_status coarse_op_build(const int dims[4], int64_t V, int N, const void* X, const void* Y, qmg_prec storage,
                           int* nbr, hipStream_t s, qmg_coarse_op* out) {
    auto* op = new qmg_coarse_op_s();
    op->nbr = nbr;   // owned from here on, also on failure
    for (int m = 0; m < 4; ++m) op->dims[m] = dims[m];
    op->V = V;
    op->N = N;
    op->storage = storage;
    op->J = 9 * N / complex_per_chunk(storage);
    const size_t bytes = (size_t)op->V * op->J * N * 16;
    hipError_t e = hipMalloc(&op->links, bytes);
    if (e == hipSuccess && is16(storage)) e = hipMalloc(&op->lscale, sizeof(float) * op->V * 9);
    if (e != hipSuccess) {
        qmg_coarse_op_destroy(op);
        return fail(QMG_ERR_NOMEM, "coarse_op_create: %zu bytes: %s", bytes, hipGetErrorString(e));
    }
    qmg_status st = QMG_OK;
    if (!nbr) st = make_neighbour_table(dims, &op->nbr, s);
    if (st != QMG_OK) {
        qmg_coarse_op_destroy(op);
        return st;
    }
    const int64_t total = op->V * op->J * N;
    const unsigned nb = (unsigned)((total + 255) / 256);
    const double2 *x = (const double2*)X, *y = (const double2*)Y;
    unsigned* nf = nullptr;
    if (is16(storage)) st = nonfinite_flag(&nf);
    if (st != QMG_OK) {
        qmg_coarse_op_destroy(op);
        return st;
    }
    switch (fmt_of(storage)) {
        case FMT_F64: hipLaunchKernelGGL(k_pack<FMT_F64>, dim3(nb), dim3(256), 0, s, (double2*)op->links, nullptr, x, y, op->V, N, op->J); break;
        case FMT_F32: hipLaunchKernelGGL(k_pack<FMT_F32>, dim3(nb), dim3(256), 0, s, (float4*)op->links, nullptr, x, y, op->V, N, op->J); break;
        case FMT_H16:
            hipLaunchKernelGGL(k_link_scales, dim3((unsigned)(op->V * 9)), dim3(256), 0, s, op->lscale, x, y, op->V, N, nf);
            hipLaunchKernelGGL(k_pack<FMT_H16>, dim3(nb), dim3(256), 0, s, (uint4*)op->links, op->lscale, x, y, op->V, N, op->J);
            break;
        default:
            hipLaunchKernelGGL(k_link_scales, dim3((unsigned)(op->V * 9)), dim3(256), 0, s, op->lscale, x, y, op->V, N, nf);
            hipLaunchKernelGGL(k_pack<FMT_B16>, dim3(nb), dim3(256), 0, s, (uint4*)op->links, op->lscale, x, y, op->V, N, op->J);
    }
    e = hipGetLastError();
    if (e != hipSuccess) {
        qmg_coarse_op_destroy(op);
        return fail(QMG_ERR_HIP, "coarse_op_create: pack launch: %s", hipGetErrorString(e));
    }
    default_launch(op, &op->rows, &op->split);
    *out = op;
    return QMG_OK;
}
}  // namespace qmg

extern "C" qmg_status qmg_coarse_op_create(const int dims[4], int N, const void* X, const void* Y,
                                           qmg_prec storage, void* stream, qmg_coarse_op* out) {
    if (!out) return fail(QMG_ERR_ARG, "coarse_op_create: out is NULL");
    *out = nullptr;
    QMG_TRY(check_dims(dims, 2, "coarse_op_create"));
    if (N < 2 || N > 128 || (N & 1)) return fail(QMG_ERR_SHAPE, "coarse_op_create: N=%d must be even in [2,128]", N);
    if (!X || !Y) return fail(QMG_ERR_ARG, "coarse_op_create: X or Y is NULL");
    if (storage != QMG_C128 && storage != QMG_C64 && storage != QMG_H16 && storage != QMG_B16)
        return fail(QMG_ERR_PREC, "coarse_op_create: storage %d not supported", (int)storage);
    if (is16(storage) && N % 4)
        return fail(QMG_ERR_SHAPE, "coarse_op_create: 16-bit storage needs N %% 4 == 0 (N=%d)", N);
    return coarse_op_build(dims, volume(dims), N, X, Y, storage, nullptr, as_stream(stream), out);
}

extern "C" qmg_status qmg_coarse_op_export(qmg_coarse_op op, void* X, void* Y, void* stream) {
    if (!op || !X || !Y) return fail(QMG_ERR_ARG, "coarse_op_export: NULL argument");
    hipStream_t s = as_stream(stream);
    const int64_t total = op->V * op->J * op->N;
    const unsigned nb = (unsigned)((total + 255) / 256);
    double2 *x = (double2*)X, *y = (double2*)Y;
    switch (fmt_of(op->storage)) {
        case FMT_F64: hipLaunchKernelGGL(k_unpack<FMT_F64>, dim3(nb), dim3(256), 0, s, (const double2*)op->links, nullptr, x, y, op->V, op->N, op->J); break;
        case FMT_F32: hipLaunchKernelGGL(k_unpack<FMT_F32>, dim3(nb), dim3(256), 0, s, (const float4*)op->links, nullptr, x, y, op->V, op->N, op->J); break;
        case FMT_H16: hipLaunchKernelGGL(k_unpack<FMT_H16>, dim3(nb), dim3(256), 0, s, (const uint4*)op->links, op->lscale, x, y, op->V, op->N, op->J); break;
        default: hipLaunchKernelGGL(k_unpack<FMT_B16>, dim3(nb), dim3(256), 0, s, (const uint4*)op->links, op->lscale, x, y, op->V, op->N, op->J);
    }
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

extern "C" qmg_status qmg_coarse_dslash(qmg_coarse_op op, const void* in, void* out, int nrhs, qmg_prec prec,
                                        void* stream) {
    if (!op || !in || !out) return fail(QMG_ERR_ARG, "coarse_dslash: NULL argument");
    if (nrhs < 1 || nrhs > kMaxFieldBatch) return fail(QMG_ERR_ARG, "coarse_dslash: nrhs %d not in [1, %d]", nrhs, kMaxFieldBatch);
    const bool ok = prec == op->storage || (is16(op->storage) && prec == QMG_C64);
    if (!ok)
        return fail(QMG_ERR_PREC, "coarse_dslash: vector precision %d does not fit operator storage %d", (int)prec,
                    (int)op->storage);
    if (is16(prec)) return fail(QMG_ERR_PREC, "coarse_dslash: 16-bit vectors go through qmg_coarse_dslash_scaled");
    if (in == out) return fail(QMG_ERR_ARG, "coarse_dslash: in and out alias");
    return coarse_dslash_launch(op, op->rows, op->split, op->pre, in, nullptr, out, nullptr, prec, as_stream(stream), nrhs);
}

// Staging bytes of a batch rounded to 16 bits: pairs [V][nrhs][N], then scales [V][nrhs].
static size_t mrhs_stage_bytes(const qmg_coarse_op_s* op, int nrhs) {
    const size_t pairs = (size_t)op->V * nrhs * op->N * sizeof(uint32_t);
    return pairs + (size_t)op->V * nrhs * sizeof(float);
}

static qmg_status check_mrhs_c64(const qmg_coarse_op_s* op, const void* in, const void* out, int nrhs,
                                 const char* what) {
    if (!op || !in || !out) return fail(QMG_ERR_ARG, "%s: NULL argument", what);
    if (!is16(op->storage)) return fail(QMG_ERR_PREC, "%s: needs an operator with 16-bit storage", what);
    if (nrhs != 8 && nrhs != 16 && nrhs != 32 && nrhs != 64)
        return fail(QMG_ERR_ARG, "%s: nrhs %d not in {8,16,32,64}", what, nrhs);
    if (op->N % 16 || op->N > 64) return fail(QMG_ERR_SHAPE, "%s: N=%d must be 16, 32, 48 or 64", what, op->N);
    if (in == out) return fail(QMG_ERR_ARG, "%s: in and out alias", what);
    return QMG_OK;
}

extern "C" qmg_status qmg_coarse_dslash_mrhs_c64(qmg_coarse_op op, const void* in, void* out, int nrhs,
                                                 void* stream) {
    QMG_TRY(check_mrhs_c64(op, in, out, nrhs, "coarse_dslash_mrhs_c64"));
    const size_t need = mrhs_stage_bytes(op, nrhs);
    if (op->stage_bytes < need) {   // grow the operator's staging (hipFree waits for work that used it)
        if (op->stage) (void)hipFree(op->stage);
        op->stage = nullptr;
        op->stage_bytes = 0;
        QMG_HIP(hipMalloc(&op->stage, need));
        op->stage_bytes = need;
    }
    float* qsc = (float*)((char*)op->stage + (size_t)op->V * nrhs * op->N * sizeof(uint32_t));
    return coarse_apply(op, in, out, QMG_C64, nrhs, op->stage, qsc, as_stream(stream));
}

extern "C" qmg_status qmg_coarse_dslash_scaled(qmg_coarse_op op, const void* in, const float* in_scale, void* out,
                                               float* out_scale, qmg_prec prec, void* stream) {
    if (!op || !in || !in_scale || !out || !out_scale) return fail(QMG_ERR_ARG, "coarse_dslash_scaled: NULL argument");
    if (!is16(op->storage) || !is16(prec))
        return fail(QMG_ERR_PREC, "coarse_dslash_scaled: needs a 16-bit operator and 16-bit vectors");
    if (in == out || (const void*)in_scale == (void*)out_scale)
        return fail(QMG_ERR_ARG, "coarse_dslash_scaled: input and output alias");
    return coarse_dslash_any(op, in, in_scale, out, out_scale, prec, as_stream(stream));
}

extern "C" qmg_status qmg_quantize_sites(const void* in, void* out, float* scale, long long V, int N, qmg_prec prec,
                                         void* stream) {
    if (!in || !out || !scale) return fail(QMG_ERR_ARG, "quantize_sites: NULL argument");
    if (V < 1 || N < 1) return fail(QMG_ERR_SHAPE, "quantize_sites: V=%lld N=%d", V, N);
    if (!is16(prec)) return fail(QMG_ERR_PREC, "quantize_sites: precision must be QMG_H16 or QMG_B16");
    hipStream_t s = as_stream(stream);
    unsigned* nf = nullptr;
    QMG_TRY(nonfinite_flag(&nf));
    if (prec == QMG_H16)
        hipLaunchKernelGGL(k_quantize<FMT_H16>, dim3((unsigned)V), dim3(64), 0, s, (const float2*)in, (uint32_t*)out, scale, N,
                           nf);
    else
        hipLaunchKernelGGL(k_quantize<FMT_B16>, dim3((unsigned)V), dim3(64), 0, s, (const float2*)in, (uint32_t*)out, scale, N,
                           nf);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

extern "C" qmg_status qmg_dequantize_sites(const void* in, const float* scale, void* out, long long V, int N,
                                           qmg_prec prec, void* stream) {
    if (!in || !out || !scale) return fail(QMG_ERR_ARG, "dequantize_sites: NULL argument");
    if (V < 1 || N < 1) return fail(QMG_ERR_SHAPE, "dequantize_sites: V=%lld N=%d", V, N);
    if (!is16(prec)) return fail(QMG_ERR_PREC, "dequantize_sites: precision must be QMG_H16 or QMG_B16");
    hipStream_t s = as_stream(stream);
    const unsigned nb = (unsigned)((V * N + 255) / 256);
    if (prec == QMG_H16)
        hipLaunchKernelGGL(k_dequantize<FMT_H16>, dim3(nb), dim3(256), 0, s, (const uint32_t*)in, scale, (float2*)out, (int64_t)V, N);
    else
        hipLaunchKernelGGL(k_dequantize<FMT_B16>, dim3(nb), dim3(256), 0, s, (const uint32_t*)in, scale, (float2*)out, (int64_t)V, N);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

extern "C" qmg_status qmg_coarse_op_set_launch(qmg_coarse_op op, int rows, int split) {
    if (!op) return fail(QMG_ERR_ARG, "coarse_op_set_launch: NULL op");
    if (rows == 0 && split == 0) {
        default_launch(op, &op->rows, &op->split);
        return QMG_OK;
    }
    QMG_TRY(validate_launch(op, rows, split));
    op->rows = rows;
    op->split = split;
    return QMG_OK;
}

extern "C" qmg_status qmg_coarse_op_get_launch(qmg_coarse_op op, int* rows, int* split) {
    if (!op || !rows || !split) return fail(QMG_ERR_ARG, "coarse_op_get_launch: NULL argument");
    *rows = op->rows;
    *split = op->split;
    return QMG_OK;
}

extern "C" void qmg_coarse_op_destroy(qmg_coarse_op op) {
    if (!op) return;
    if (op->links) (void)hipFree(op->links);
    if (op->lscale) (void)hipFree(op->lscale);
    if (op->mlinks) (void)hipFree(op->mlinks);
    if (op->stage) (void)hipFree(op->stage);
    if (op->nbr) (void)hipFree(op->nbr);
    if (op->eo_even) qmg_coarse_op_destroy(op->eo_even);
    if (op->eo_odd) qmg_coarse_op_destroy(op->eo_odd);
    if (op->hsite) (void)hipFree(op->hsite);
    if (op->eo_tmp) (void)hipFree(op->eo_tmp);
    delete op;
}
