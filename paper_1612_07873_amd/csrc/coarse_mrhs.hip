// Multi-right-hand-side coarse operator on the matrix cores (the multi-RHS
// reformulation the paper proposes as future work, Sec. 9).
//
// Per coarse site, for nrhs right-hand sides at once,
//     Y(N x nrhs) = sum_{d=0..8} A_d (N x N) * U_d (N x nrhs),
// A_0 = X(x), A_{1+d} = Y_d(x), U_0 = u(x), U_{1+d} = u(x + hop_d).  With links
// and vectors in 16-bit form, each complex product is two real products
// sharing the same B operand: with K running over (column c, re/im),
//     Re Y = [Ar, -Ai] [Ur; Ui],   Im Y = [Ai, Ar] [Ur; Ui],
// and both A operands come from the stored (re, im) pairs by flipping the
// sign bit of the imaginary half or swapping the halves.  The products run on
// v_mfma_f32_16x16x32_{f16,bf16} with FP32 accumulation; each direction is
// accumulated separately and then scaled by s_link(x, d) * s_u(x + hop_d, rhs)
// (the per-(site, block) link scale and per-(site, rhs) vector scale).
//
// Work decomposition: one work-group per coarse site; wave w owns row tile
// w mod (N/16) (16 output rows) and `rpw` tiles of 16 right-hand sides.  The
// wave's link operands are loaded straight from HBM into registers one
// direction ahead (the links are repacked once so every wave load is one
// contiguous 1 KB: [site][d][row tile][k step][lane] x 16 bytes), and the
// input blocks U_d ([nrhs][N] per site, contiguous) stream through two LDS
// buffers one direction ahead of the multiplication.  B operands are 16-byte
// LDS reads.
//
// Field layout: u, y [V][nrhs][N] (each right-hand side's N components
// contiguous within a site); 16-bit u with FP32 scales [V][nrhs]; y complex64.
#include "handles.h"

#include <hip/hip_runtime.h>

#include <vector>

namespace qmg {

typedef _Float16 h8v __attribute__((ext_vector_type(8)));
typedef __bf16 b8v __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));

enum { MF_H16 = 2, MF_B16 = 3 };

template <int F> __device__ __forceinline__ f4v mfma(uint4 a, uint4 b, f4v c) {
    if constexpr (F == MF_H16)
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8v, a), __builtin_bit_cast(h8v, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8v, a), __builtin_bit_cast(b8v, b), c, 0, 0, 0);
}

__device__ __forceinline__ uint32_t rot16(uint32_t w) { return (w >> 16) | (w << 16); }

// chunked 16-bit layout [site][j][row] -> MFMA operand layout
// [site][d][rt][ks][lane]: lane l holds row rt*16 + l%16, complex columns ks*16 + 4*(l/16) + 0..3.
__global__ void k_pack_mfma(uint4* __restrict__ M, const uint4* __restrict__ L, int64_t V, int N, int J) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int T = N / 16;
    if (g >= V * 9 * T * T * 64) return;
    const int l = (int)(g % 64);
    int64_t t = g / 64;
    const int ks = (int)(t % T);
    t /= T;
    const int rt = (int)(t % T);
    t /= T;
    const int d = (int)(t % 9);
    const int64_t site = t / 9;
    const int row = rt * 16 + (l % 16);
    const int e = d * N + ks * 16 + 4 * (l / 16);  // first of 4 complex in the 9N row
    M[g] = L[(site * J + e / 4) * N + row];
}

// A link operand chunk, read once per application: a non-temporal load, so
// the link stream does not push the input blocks -- each read by nine sites --
// out of L2 before their neighbours ask for them.
__device__ __forceinline__ uint4 ld_stream(const uint4* p) {
    typedef unsigned int u4v __attribute__((ext_vector_type(4)));
    const u4v v = __builtin_nontemporal_load(reinterpret_cast<const u4v*>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}

// Work of one coarse site; the work-group has `nthreads` threads, of which the
// first NW waves compute (all of them stage).  The nine input blocks pass
// through two LDS buffers: while direction d is multiplied, every thread
// holds its share of block d+1 in registers and writes it to the other buffer
// afterwards, so staging overlaps the matrix-core work and the LDS footprint is
// two blocks instead of nine.
template <int F, int N, int NRHS, int RPW>
__device__ __forceinline__ void mrhs_site(int site, int nthreads, const uint4* __restrict__ M,
                                          const float* __restrict__ lscale, const int* __restrict__ nbr,
                                          const uint32_t* __restrict__ u, const float* __restrict__ uscale,
                                          float2* __restrict__ y, int64_t oss, int64_t ors, unsigned char* smem) {
    constexpr int T = N / 16;                       // row tiles = k steps per direction
    constexpr int NT = NRHS >= 16 ? NRHS / 16 : 1;  // right-hand-side tiles
    constexpr int NW = T * (NT / RPW);              // computing waves
    constexpr int UW = NRHS * N;                    // dwords per input block in HBM
    constexpr int LD = N + 4;                       // LDS row stride (dwords), padded against bank conflicts
    constexpr int US = NRHS * LD;                   // dwords per staged block
    constexpr int PER = (UW / 4 + NW * 64 - 1) / (NW * 64);  // 16-byte pieces per thread per block
    uint32_t* Us = reinterpret_cast<uint32_t*>(smem);       // [2][NRHS][LD]
    float* Sc = reinterpret_cast<float*>(Us + 2 * US);       // [9][NRHS]

    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const bool computes = w < NW;
    const int rt = w % T, tg = w / T;
    const uint4* Ms = M + ((int64_t)site * 9 * T + rt) * T * 64 + l;

    uint4 Acur[T], Anext[T];
    if (computes) {
#pragma unroll
        for (int ks = 0; ks < T; ++ks) Acur[ks] = ld_stream(Ms + (int64_t)ks * 64);
    }
    // block 0 and all scales
    {
        const uint4* g = reinterpret_cast<const uint4*>(u + (int64_t)site * UW);
        for (int i = threadIdx.x; i < UW / 4; i += nthreads) {
            const int j = (4 * i) / N, c = (4 * i) % N;
            *reinterpret_cast<uint4*>(Us + j * LD + c) = g[i];
        }
        for (int e = threadIdx.x; e < 9 * NRHS; e += nthreads) {
            const int d = e / NRHS, j = e % NRHS;
            const int sd = d == 0 ? site : nbr[site * 8 + d - 1];
            Sc[e] = lscale[(int64_t)site * 9 + d] * uscale[(int64_t)sd * NRHS + j];
        }
    }
    __syncthreads();
    f4v tot[RPW][2];
#pragma unroll
    for (int t = 0; t < RPW; ++t) tot[t][0] = tot[t][1] = f4v{0, 0, 0, 0};
    const int jl = l % 16;
#pragma unroll
    for (int d = 0; d < 9; ++d) {
        const uint32_t* Ub = Us + (d & 1) * US;
        uint4 nxt[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) nxt[q] = make_uint4(0, 0, 0, 0);
        if (d < 8) {
            const uint4* g = reinterpret_cast<const uint4*>(u + (int64_t)nbr[site * 8 + d] * UW);
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const int i = threadIdx.x + q * nthreads;
                if (i < UW / 4) nxt[q] = g[i];
            }
            if (computes) {
#pragma unroll
                for (int ks = 0; ks < T; ++ks) Anext[ks] = ld_stream(Ms + ((int64_t)(d + 1) * T * T + ks) * 64);
            }
        }
        if (computes) {
            f4v acc[RPW][2];
#pragma unroll
            for (int t = 0; t < RPW; ++t) acc[t][0] = acc[t][1] = f4v{0, 0, 0, 0};
#pragma unroll
            for (int ks = 0; ks < T; ++ks) {
                const uint4 a = Acur[ks];
                const uint4 ar = make_uint4(a.x ^ 0x80000000u, a.y ^ 0x80000000u, a.z ^ 0x80000000u, a.w ^ 0x80000000u);
                const uint4 ai = make_uint4(rot16(a.x), rot16(a.y), rot16(a.z), rot16(a.w));
#pragma unroll
                for (int t = 0; t < RPW; ++t) {
                    const int j = (tg * RPW + t) * 16 + jl;
                    uint4 b = make_uint4(0, 0, 0, 0);
                    if (NRHS >= 16 || j < NRHS)
                        b = *reinterpret_cast<const uint4*>(Ub + j * LD + ks * 16 + 4 * (l / 16));
                    acc[t][0] = mfma<F>(ar, b, acc[t][0]);
                    acc[t][1] = mfma<F>(ai, b, acc[t][1]);
                }
            }
#pragma unroll
            for (int t = 0; t < RPW; ++t) {
                const int j = (tg * RPW + t) * 16 + jl;
                const float sc = (NRHS >= 16 || j < NRHS) ? Sc[d * NRHS + j] : 0.0f;
                tot[t][0] += sc * acc[t][0];
                tot[t][1] += sc * acc[t][1];
            }
            if (d < 8) {
#pragma unroll
                for (int ks = 0; ks < T; ++ks) Acur[ks] = Anext[ks];
            }
        }
        if (d < 8) {
            uint32_t* Un = Us + ((d + 1) & 1) * US;
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const int i = threadIdx.x + q * nthreads;
                if (i < UW / 4) {
                    const int j = (4 * i) / N, c = (4 * i) % N;
                    *reinterpret_cast<uint4*>(Un + j * LD + c) = nxt[q];
                }
            }
        }
        __syncthreads();
    }
    if (computes) {
#pragma unroll
        for (int t = 0; t < RPW; ++t) {
            const int j = (tg * RPW + t) * 16 + jl;
            if (NRHS < 16 && j >= NRHS) continue;
            float2* o = y + (int64_t)site * oss + (int64_t)j * ors + rt * 16 + 4 * (l / 16);
            float4* o4 = reinterpret_cast<float4*>(o);
            o4[0] = make_float4(tot[t][0][0], tot[t][1][0], tot[t][0][1], tot[t][1][1]);
            o4[1] = make_float4(tot[t][0][2], tot[t][1][2], tot[t][0][3], tot[t][1][3]);
        }
    }
}

// Site of this work-group.  Work-groups are dealt to the 8 XCDs round-robin;
// numbering the sites so that each XCD takes one contiguous range of ceil(V/8)
// sites keeps most of a site's neighbours -- whose input blocks it reads --
// in the same XCD's L2.  The grid is 8 ceil(V/8); -1 past the last site.
__device__ __forceinline__ int xcd_site(int64_t V) {
    const int64_t per = (V + 7) / 8;
    const int64_t s = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
    return s < V ? (int)s : -1;
}
static unsigned xcd_grid(int64_t V) { return (unsigned)(8 * ((V + 7) / 8)); }

template <int F, int N, int NRHS, int RPW>
__global__ __launch_bounds__((N / 16) * ((NRHS >= 16 ? NRHS / 16 : 1) / RPW) * 64) void k_coarse_mrhs(
    const uint4* __restrict__ M, const float* __restrict__ lscale, const int* __restrict__ nbr,
    const uint32_t* __restrict__ u, const float* __restrict__ uscale, float2* __restrict__ y, int64_t oss, int64_t ors,
    int64_t V) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int site = xcd_site(V);
    if (site < 0) return;   // the whole work-group
    mrhs_site<F, N, NRHS, RPW>(site, blockDim.x, M, lscale, nbr, u, uscale, y, oss, ors, smem);
}

// Whole-site form: one wave per row tile, each owning every right-hand-side
// tile; the link operands of all nine directions are requested into
// registers and all nine input blocks are copied into LDS by direct
// global->LDS loads (no registers) at the start, so a site waits for memory
// once instead of once per direction.  LDS: 9 padded blocks (159 KB at N = 64,
// 64 right-hand sides: one work-group per CU).  Chunk c of a padded row holds
// columns 4c..4c+3 for c < N/4; the last chunk of each row is padding (filled
// with a copy of the row's last data chunk, never read).
template <int F, int N, int NRHS>
__global__ __launch_bounds__((N / 16) * 64) void k_coarse_mrhs_all(
    const uint4* __restrict__ M, const float* __restrict__ lscale, const int* __restrict__ nbr,
    const uint32_t* __restrict__ u, const float* __restrict__ uscale, float2* __restrict__ y, int64_t oss, int64_t ors,
    int64_t V) {
    constexpr int T = N / 16;                       // row tiles = waves = k steps per direction
    constexpr int NT = NRHS >= 16 ? NRHS / 16 : 1;  // right-hand-side tiles
    constexpr int UW = NRHS * N;                    // dwords per input block in HBM
    constexpr int RL = N / 4 + 1;                   // 16-byte chunks per padded LDS row
    constexpr int LD = 4 * RL;                      // LDS row stride (dwords)
    constexpr int US = NRHS * LD;                   // dwords per staged block
    constexpr int CH = NRHS * RL;                   // 16-byte chunks per staged block
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t* Us = reinterpret_cast<uint32_t*>(smem);   // [9][NRHS][LD]
    float* Sc = reinterpret_cast<float*>(Us + 9 * US);   // [9][NRHS]
    const int site = xcd_site(V);
    if (site < 0) return;   // the whole work-group
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int rt = w;

    uint4 A[9][T];
    {
        const uint4* Ms = M + ((int64_t)site * 9 * T + rt) * T * 64 + l;
#pragma unroll
        for (int d = 0; d < 9; ++d)
#pragma unroll
            for (int ks = 0; ks < T; ++ks) A[d][ks] = ld_stream(Ms + ((int64_t)d * T * T + ks) * 64);
    }
#pragma unroll
    for (int d = 0; d < 9; ++d) {
        const int src = d == 0 ? site : nbr[site * 8 + d - 1];
        const uint4* g = reinterpret_cast<const uint4*>(u + (int64_t)src * UW);
        for (int c0 = w * 64; c0 < CH; c0 += T * 64) {
            const int c = c0 + l;
            if (c < CH) {
                const int row = c / RL, col = c - (c / RL) * RL;
                const int gc = row * (N / 4) + (col < N / 4 ? col : N / 4 - 1);
                __builtin_amdgcn_global_load_lds(g + gc, (__attribute__((address_space(3))) void*)(Us + d * US + 4 * c0),
                                                 16, 0, 0);
            }
        }
    }
    for (int e = threadIdx.x; e < 9 * NRHS; e += T * 64) {
        const int d = e / NRHS, j = e % NRHS;
        const int sd = d == 0 ? site : nbr[site * 8 + d - 1];
        Sc[e] = lscale[(int64_t)site * 9 + d] * uscale[(int64_t)sd * NRHS + j];
    }
    __builtin_amdgcn_s_waitcnt(0);   // the direct-to-LDS copies have landed
    __syncthreads();

    f4v tot[NT][2];
#pragma unroll
    for (int t = 0; t < NT; ++t) tot[t][0] = tot[t][1] = f4v{0, 0, 0, 0};
    const int jl = l % 16;
#pragma unroll
    for (int d = 0; d < 9; ++d) {
        const uint32_t* Ub = Us + d * US;
        f4v acc[NT][2];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t][0] = acc[t][1] = f4v{0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < T; ++ks) {
            const uint4 a = A[d][ks];
            const uint4 ar = make_uint4(a.x ^ 0x80000000u, a.y ^ 0x80000000u, a.z ^ 0x80000000u, a.w ^ 0x80000000u);
            const uint4 ai = make_uint4(rot16(a.x), rot16(a.y), rot16(a.z), rot16(a.w));
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int j = t * 16 + jl;
                uint4 b = make_uint4(0, 0, 0, 0);
                if (NRHS >= 16 || j < NRHS) b = *reinterpret_cast<const uint4*>(Ub + j * LD + ks * 16 + 4 * (l / 16));
                acc[t][0] = mfma<F>(ar, b, acc[t][0]);
                acc[t][1] = mfma<F>(ai, b, acc[t][1]);
            }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int j = t * 16 + jl;
            const float sc = (NRHS >= 16 || j < NRHS) ? Sc[d * NRHS + j] : 0.0f;
            tot[t][0] += sc * acc[t][0];
            tot[t][1] += sc * acc[t][1];
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int j = t * 16 + jl;
        if (NRHS < 16 && j >= NRHS) continue;
        float2* o = y + (int64_t)site * oss + (int64_t)j * ors + rt * 16 + 4 * (l / 16);
        float4* o4 = reinterpret_cast<float4*>(o);
        o4[0] = make_float4(tot[t][0][0], tot[t][1][0], tot[t][0][1], tot[t][1][1]);
        o4[1] = make_float4(tot[t][0][2], tot[t][1][2], tot[t][0][3], tot[t][1][3]);
    }
}

// Persistent form over several operators ("levels") of possibly different
// size and N in {48, 64}: work item i of the queue [level 0 sites, level 1
// sites, ...] is taken by work-group i mod gridDim.x; work-groups loop until
// the queue is exhausted (every work-group reaches the end).
struct MultiLevel {
    int nlev;
    int64_t start[5];  // prefix offsets of the queue, start[nlev] = total
    int N[4];
    const uint4* M[4];
    const float* lscale[4];
    const int* nbr[4];
    const uint32_t* u[4];
    const float* uscale[4];
    float2* y[4];
};

// RP right-hand-side tiles per wave (the widest the batch allows: the
// largest level, which dominates the queue, is fastest with it).
template <int F, int NRHS, int RP>
__global__ __launch_bounds__(4 * ((NRHS >= 16 ? NRHS / 16 : 1) / RP) * 64) void k_coarse_mrhs_multi(MultiLevel ml) {
    extern __shared__ __align__(16) unsigned char smem[];
    for (int64_t item = blockIdx.x; item < ml.start[ml.nlev]; item += gridDim.x) {
        int l = 0;
        while (l + 1 < ml.nlev && item >= ml.start[l + 1]) ++l;
        const int site = (int)(item - ml.start[l]);
        if (ml.N[l] == 48)
            mrhs_site<F, 48, NRHS, RP>(site, blockDim.x, ml.M[l], ml.lscale[l], ml.nbr[l], ml.u[l], ml.uscale[l], ml.y[l],
                                       (int64_t)NRHS * 48, 48, smem);
        else
            mrhs_site<F, 64, NRHS, RP>(site, blockDim.x, ml.M[l], ml.lscale[l], ml.nbr[l], ml.u[l], ml.uscale[l], ml.y[l],
                                       (int64_t)NRHS * 64, 64, smem);
        __syncthreads();  // LDS is reused by the next item
    }
}

template <int F, int N, int NRHS, int RPW>
static qmg_status launch_mrhs_t(const qmg_coarse_op_s* op, const void* in, const float* sc, void* out, int64_t ors,
                                hipStream_t s) {
    constexpr int T = N / 16;
    constexpr int NT = NRHS >= 16 ? NRHS / 16 : 1;
    constexpr int NW = T * (NT / RPW);
    const size_t lds = 2 * (size_t)NRHS * (N + 4) * 4 + 9 * NRHS * 4;
    auto kern = k_coarse_mrhs<F, N, NRHS, RPW>;
    if (lds > 65536) QMG_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kern, dim3(xcd_grid(op->V)), dim3(NW * 64), lds, s, (const uint4*)op->mlinks, op->lscale,
                       op->nbr, (const uint32_t*)in, sc, (float2*)out, ors ? (int64_t)N : (int64_t)NRHS * N,
                       ors ? ors : (int64_t)N, op->V);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

template <int F, int N, int NRHS>
static qmg_status launch_all_t(const qmg_coarse_op_s* op, const void* in, const float* sc, void* out, int64_t ors,
                               hipStream_t s) {
    const size_t lds = 9 * (size_t)NRHS * (N + 4) * 4 + 9 * NRHS * 4;
    auto kern = k_coarse_mrhs_all<F, N, NRHS>;
    if (lds > 65536) QMG_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kern, dim3(xcd_grid(op->V)), dim3((N / 16) * 64), lds, s, (const uint4*)op->mlinks,
                       op->lscale, op->nbr, (const uint32_t*)in, sc, (float2*)out, ors ? (int64_t)N : (int64_t)NRHS * N,
                       ors ? ors : (int64_t)N, op->V);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

template <int F, int N, int NRHS>
static qmg_status launch_rpw(const qmg_coarse_op_s* op, int rpw, const void* in, const float* sc, void* out, int64_t ors,
                             hipStream_t s) {
    constexpr int NT = NRHS >= 16 ? NRHS / 16 : 1;
    if (rpw == 8) return launch_all_t<F, N, NRHS>(op, in, sc, out, ors, s);
    if (rpw == 1) return launch_mrhs_t<F, N, NRHS, 1>(op, in, sc, out, ors, s);
    if constexpr (NT >= 2) if (rpw == 2) return launch_mrhs_t<F, N, NRHS, 2>(op, in, sc, out, ors, s);
    if constexpr (NT >= 4) if (rpw == 4) return launch_mrhs_t<F, N, NRHS, 4>(op, in, sc, out, ors, s);
    return fail(QMG_ERR_ARG, "coarse_dslash_mrhs: rpw %d not available for nrhs %d", rpw, NRHS);
}

template <int F, int N>
static qmg_status launch_n(const qmg_coarse_op_s* op, int nrhs, int rpw, const void* in, const float* sc, void* out,
                           int64_t ors, hipStream_t s) {
    switch (nrhs) {
        case 8: return launch_rpw<F, N, 8>(op, rpw, in, sc, out, ors, s);
        case 16: return launch_rpw<F, N, 16>(op, rpw, in, sc, out, ors, s);
        case 32: return launch_rpw<F, N, 32>(op, rpw, in, sc, out, ors, s);
        case 64: return launch_rpw<F, N, 64>(op, rpw, in, sc, out, ors, s);
    }
    return fail(QMG_ERR_ARG, "coarse_dslash_mrhs: nrhs %d not in {8,16,32,64}", nrhs);
}

static int log2i(int n) { int k = 0; while ((1 << k) < n) ++k; return k; }

static int max_rpw(int nrhs) { return nrhs >= 64 ? 4 : nrhs >= 32 ? 2 : 1; }

static int default_rpw(const qmg_coarse_op_s* op, int nrhs) {
    // enough waves per work-group to keep several link loads in flight per SIMD,
    // at most 16 waves; the autotuner refines this
    const int T = op->N / 16, NT = nrhs >= 16 ? nrhs / 16 : 1;
    int rpw = 1;
    while (T * (NT / rpw) > 16 && rpw < max_rpw(nrhs)) rpw *= 2;
    return rpw;
}

// ors = 0: output [V][nrhs][N]; otherwise right-hand side j of site x at
// out + j*ors + x*N (ors = V*N gives [nrhs][V][N])
qmg_status coarse_mrhs(qmg_coarse_op_s* op, const void* in, const float* sc, void* out, int nrhs, int rpw,
                       hipStream_t s, int64_t ors) {
    if (!op->mlinks) {
        const int T = op->N / 16;
        const int64_t n = op->V * 9 * T * T * 64;
        QMG_HIP(hipMalloc(&op->mlinks, (size_t)n * 16));
        hipLaunchKernelGGL(k_pack_mfma, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (uint4*)op->mlinks,
                           (const uint4*)op->links, op->V, op->N, op->J);
        QMG_LAUNCH_CHECK();
    }
    if (rpw <= 0) rpw = op->rpw[log2i(nrhs)] > 0 ? op->rpw[log2i(nrhs)] : default_rpw(op, nrhs);
    const bool h = op->storage == QMG_H16;
    if (op->N == 48) return h ? launch_n<MF_H16, 48>(op, nrhs, rpw, in, sc, out, ors, s) : launch_n<MF_B16, 48>(op, nrhs, rpw, in, sc, out, ors, s);
    if (op->N == 64) return h ? launch_n<MF_H16, 64>(op, nrhs, rpw, in, sc, out, ors, s) : launch_n<MF_B16, 64>(op, nrhs, rpw, in, sc, out, ors, s);
    if (op->N == 32) return h ? launch_n<MF_H16, 32>(op, nrhs, rpw, in, sc, out, ors, s) : launch_n<MF_B16, 32>(op, nrhs, rpw, in, sc, out, ors, s);
    if (op->N == 16) return h ? launch_n<MF_H16, 16>(op, nrhs, rpw, in, sc, out, ors, s) : launch_n<MF_B16, 16>(op, nrhs, rpw, in, sc, out, ors, s);
    return fail(QMG_ERR_SHAPE, "coarse_dslash_mrhs: N=%d not in {16,32,48,64}", op->N);
}

}  // namespace qmg

using namespace qmg;

extern "C" qmg_status qmg_coarse_dslash_mrhs(qmg_coarse_op op, const void* in, const float* in_scale, void* out,
                                             int nrhs, void* stream) {
    if (!op || !in || !in_scale || !out) return fail(QMG_ERR_ARG, "coarse_dslash_mrhs: NULL argument");
    if (op->storage != QMG_H16 && op->storage != QMG_B16)
        return fail(QMG_ERR_PREC, "coarse_dslash_mrhs: needs an operator with 16-bit storage");
    if (nrhs != 8 && nrhs != 16 && nrhs != 32 && nrhs != 64)
        return fail(QMG_ERR_ARG, "coarse_dslash_mrhs: nrhs %d not in {8,16,32,64}", nrhs);
    if (op->N % 16 || op->N > 64) return fail(QMG_ERR_SHAPE, "coarse_dslash_mrhs: N=%d must be 16, 32, 48 or 64", op->N);
    if (in == out) return fail(QMG_ERR_ARG, "coarse_dslash_mrhs: in and out alias");
    return coarse_mrhs(op, in, in_scale, out, nrhs, 0, as_stream(stream), 0);
}

extern "C" qmg_status qmg_coarse_op_set_mrhs_tiles(qmg_coarse_op op, int nrhs, int rhs_tiles_per_wave) {
    if (!op) return fail(QMG_ERR_ARG, "coarse_op_set_mrhs_tiles: NULL op");
    if (nrhs != 8 && nrhs != 16 && nrhs != 32 && nrhs != 64)
        return fail(QMG_ERR_ARG, "coarse_op_set_mrhs_tiles: nrhs %d not in {8,16,32,64}", nrhs);
    const int r = rhs_tiles_per_wave;
    if (r != 0 && r != 1 && r != 2 && r != 4 && r != 8)
        return fail(QMG_ERR_ARG, "coarse_op_set_mrhs_tiles: tiles %d not in {0,1,2,4,8}", r);
    if (r != 8 && r > max_rpw(nrhs)) return fail(QMG_ERR_ARG, "coarse_op_set_mrhs_tiles: %d tiles exceed nrhs %d", r, nrhs);
    op->rpw[log2i(nrhs)] = r;
    return QMG_OK;
}

extern "C" qmg_status qmg_coarse_op_get_mrhs_tiles(qmg_coarse_op op, int nrhs, int* tiles) {
    if (!op || !tiles) return fail(QMG_ERR_ARG, "coarse_op_get_mrhs_tiles: NULL argument");
    if (nrhs != 8 && nrhs != 16 && nrhs != 32 && nrhs != 64)
        return fail(QMG_ERR_ARG, "coarse_op_get_mrhs_tiles: nrhs %d not in {8,16,32,64}", nrhs);
    const int r = op->rpw[log2i(nrhs)];
    *tiles = r > 0 ? r : default_rpw(op, nrhs);
    return QMG_OK;
}

namespace qmg {
template <int F, int NRHS>
static qmg_status launch_multi(const MultiLevel& ml, size_t lds, int grid, hipStream_t s) {
    constexpr int NT = NRHS >= 16 ? NRHS / 16 : 1;
    constexpr int RP = NRHS >= 64 ? 4 : NRHS >= 32 ? 2 : 1;
    auto kern = k_coarse_mrhs_multi<F, NRHS, RP>;
    if (lds > 65536) QMG_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const int block = 4 * (NT / RP) * 64;
    if (grid == 0) {   // as many work-groups as are resident at once: each walks its share of the queue
        int per_cu = 0, dev = 0, cus = 0;
        QMG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kern, block, lds));
        QMG_HIP(hipGetDevice(&dev));
        QMG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        grid = per_cu * cus;
        if (grid < 1) grid = 1;
        if ((int64_t)grid > ml.start[ml.nlev]) grid = (int)ml.start[ml.nlev];
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, s, ml);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}
}  // namespace qmg

extern "C" qmg_status qmg_coarse_dslash_mrhs_multi(int nops, const qmg_coarse_op* ops, const void* const* in,
                                                   const float* const* in_scale, void* const* out, int nrhs,
                                                   int grid, void* stream) {
    if (nops < 1 || nops > 4 || !ops || !in || !in_scale || !out)
        return fail(QMG_ERR_ARG, "coarse_dslash_mrhs_multi: 1..4 operators with their fields");
    if (nrhs != 8 && nrhs != 16 && nrhs != 32 && nrhs != 64)
        return fail(QMG_ERR_ARG, "coarse_dslash_mrhs_multi: nrhs %d not in {8,16,32,64}", nrhs);
    if (grid < 0) return fail(QMG_ERR_ARG, "coarse_dslash_mrhs_multi: grid %d < 0", grid);
    hipStream_t s = as_stream(stream);
    MultiLevel ml{};
    ml.nlev = nops;
    int64_t tot = 0;
    size_t lds = 0;
    for (int i = 0; i < nops; ++i) {
        qmg_coarse_op op = ops[i];
        if (!op || !in[i] || !in_scale[i] || !out[i]) return fail(QMG_ERR_ARG, "coarse_dslash_mrhs_multi: NULL entry %d", i);
        if (op->storage != ops[0]->storage || (op->storage != QMG_H16 && op->storage != QMG_B16))
            return fail(QMG_ERR_PREC, "coarse_dslash_mrhs_multi: all operators need the same 16-bit storage");
        if (op->N != 48 && op->N != 64) return fail(QMG_ERR_SHAPE, "coarse_dslash_mrhs_multi: N=%d not 48 or 64", op->N);
        if (!op->mlinks) {  // operand-order links (not created inside a capture: call once beforehand)
            const int T = op->N / 16;
            const int64_t n = op->V * 9 * T * T * 64;
            QMG_HIP(hipMalloc(&op->mlinks, (size_t)n * 16));
            hipLaunchKernelGGL(k_pack_mfma, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (uint4*)op->mlinks,
                               (const uint4*)op->links, op->V, op->N, op->J);
            QMG_LAUNCH_CHECK();
        }
        ml.start[i] = tot;
        tot += op->V;
        ml.N[i] = op->N;
        ml.M[i] = (const uint4*)op->mlinks;
        ml.lscale[i] = op->lscale;
        ml.nbr[i] = op->nbr;
        ml.u[i] = (const uint32_t*)in[i];
        ml.uscale[i] = in_scale[i];
        ml.y[i] = (float2*)out[i];
        const size_t l = 2 * (size_t)nrhs * (op->N + 4) * 4 + 9 * nrhs * 4;
        if (l > lds) lds = l;
    }
    ml.start[nops] = tot;
    const bool h = ops[0]->storage == QMG_H16;
    switch (nrhs) {
        case 8: return h ? launch_multi<MF_H16, 8>(ml, lds, grid, s) : launch_multi<MF_B16, 8>(ml, lds, grid, s);
        case 16: return h ? launch_multi<MF_H16, 16>(ml, lds, grid, s) : launch_multi<MF_B16, 16>(ml, lds, grid, s);
        case 32: return h ? launch_multi<MF_H16, 32>(ml, lds, grid, s) : launch_multi<MF_B16, 32>(ml, lds, grid, s);
        default: return h ? launch_multi<MF_H16, 64>(ml, lds, grid, s) : launch_multi<MF_B16, 64>(ml, lds, grid, s);
    }
}
