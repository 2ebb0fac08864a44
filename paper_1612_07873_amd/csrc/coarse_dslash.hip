// Coarse-grid operator, Eq. (3), applied with the fine-grained split of
// Sec. 6.1-6.4 re-designed for CDNA4 wave64.
//
// Work decomposition.  Per coarse site the operator is one dense
// (N x 9N) * (9N) product: the concatenated row [X | Y_0 .. Y_7] times the
// stacked input [u(x); u(x+hop_0); ..; u(x+hop_7)].  A work-group owns one
// site (grid parallelism, Sec. 6.1) and a tile of `rows` output rows
// (colour-spin parallelism, Sec. 6.2).  The 9N-long row is cut into 16-byte
// chunks (1 complex in FP64, 2 in FP32) and chunk j goes to split-lane
// s = j mod split: this one split covers both the stencil-direction split
// (Sec. 6.3, chunks of different d) and the dot-product split (Sec. 6.4,
// chunks of the same d), and the partial sums meet once in LDS before the
// single store.  The site index and its 8 neighbours come from a
// precomputed table, so no integer division by lattice extents is done in
// the kernel (the indexing cost Sec. 6.5 names as the Amdahl limiter).
//
// Link layout.  Chunks are stored [site][j][row] (row fastest).  For a fixed
// chunk index the rows of a site are contiguous, and consecutive split-lanes
// read consecutive chunk indices, so the rows*split threads of a work-group
// read one contiguous span of rows*split*16 bytes per step whatever the split:
// every load is a fully coalesced 16-byte-per-lane load, and the layout does
// not depend on the launch shape.  The 9 input vectors of the site are staged
// once in LDS; all lanes of a wave read the same (or two) LDS addresses per
// step, which the LDS serves as a broadcast.
#include "handles.h"

#include <algorithm>
#include <vector>

namespace qmg {

template <typename R> struct Chunk;
template <> struct Chunk<double> { using T = double2; static constexpr int cpc = 1; };
template <> struct Chunk<float> { using T = float4; static constexpr int cpc = 2; };

__device__ __forceinline__ const double2* link_src(const double2* X, const double2* Y, int64_t V,
                                                   int N, int64_t site, int r, int e) {
    const int d = e / N, c = e - (e / N) * N;
    return d == 0 ? X + (site * N + r) * N + c : Y + ((((int64_t)(d - 1)) * V + site) * N + r) * N + c;
}

__device__ __forceinline__ double2* link_dst(double2* X, double2* Y, int64_t V, int N, int64_t site,
                                             int r, int e) {
    const int d = e / N, c = e - (e / N) * N;
    return d == 0 ? X + (site * N + r) * N + c : Y + ((((int64_t)(d - 1)) * V + site) * N + r) * N + c;
}

// Canonical complex128 X, Y -> chunked layout.  One thread per chunk.
__global__ void k_pack_c128(double2* __restrict__ L, const double2* __restrict__ X,
                            const double2* __restrict__ Y, int64_t V, int N, int J) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= V * J * N) return;
    const int r = (int)(g % N);
    const int64_t t = g / N;
    const int j = (int)(t % J);
    const int64_t site = t / J;
    L[g] = *link_src(X, Y, V, N, site, r, j);
}

__global__ void k_pack_c64(float4* __restrict__ L, const double2* __restrict__ X,
                           const double2* __restrict__ Y, int64_t V, int N, int J) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= V * J * N) return;
    const int r = (int)(g % N);
    const int64_t t = g / N;
    const int j = (int)(t % J);
    const int64_t site = t / J;
    const double2* p = link_src(X, Y, V, N, site, r, 2 * j);
    L[g] = make_float4((float)p[0].x, (float)p[0].y, (float)p[1].x, (float)p[1].y);
}

__global__ void k_unpack_c128(const double2* __restrict__ L, double2* __restrict__ X,
                              double2* __restrict__ Y, int64_t V, int N, int J) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= V * J * N) return;
    const int r = (int)(g % N);
    const int64_t t = g / N;
    const int j = (int)(t % J);
    const int64_t site = t / J;
    *link_dst(X, Y, V, N, site, r, j) = L[g];
}

__global__ void k_unpack_c64(const float4* __restrict__ L, double2* __restrict__ X,
                             double2* __restrict__ Y, int64_t V, int N, int J) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= V * J * N) return;
    const int r = (int)(g % N);
    const int64_t t = g / N;
    const int j = (int)(t % J);
    const int64_t site = t / J;
    double2* p = link_dst(X, Y, V, N, site, r, 2 * j);
    const float4 a = L[g];
    p[0] = make_double2(a.x, a.y);
    p[1] = make_double2(a.z, a.w);
}

__device__ __forceinline__ void chunk_mac(const double2 a, const cpx<double>* b, double& ar, double& ai) {
    cmac(ar, ai, a.x, a.y, b[0].re, b[0].im);
}

__device__ __forceinline__ void chunk_mac(const float4 a, const cpx<float>* b, float& ar, float& ai) {
    cmac(ar, ai, a.x, a.y, b[0].re, b[0].im);
    cmac(ar, ai, a.z, a.w, b[1].re, b[1].im);
}

// One work-group = (coarse site, tile of `rows` rows); rows*split threads.
template <typename R>
__global__ __launch_bounds__(1024) void k_coarse_dslash(const typename Chunk<R>::T* __restrict__ L,
                                                        const int* __restrict__ nbr,
                                                        const cpx<R>* __restrict__ u,
                                                        cpx<R>* __restrict__ y, int N, int J,
                                                        int rows, int split, int ntiles) {
    constexpr int cpc = Chunk<R>::cpc;
    extern __shared__ __align__(16) unsigned char smem[];
    cpx<R>* ul = reinterpret_cast<cpx<R>*>(smem);  // [9N] stacked inputs
    cpx<R>* red = ul + 9 * N;                       // [split][rows] partial sums

    const int site = blockIdx.x / ntiles;
    const int tile = blockIdx.x - site * ntiles;
    const int t = threadIdx.x;
    const int T = rows * split;

    for (int idx = t; idx < 9 * N; idx += T) {
        const int d = idx / N;
        const int c = idx - d * N;
        const int src = d == 0 ? site : nbr[site * 8 + d - 1];
        ul[idx] = u[(int64_t)src * N + c];
    }
    __syncthreads();

    const int rl = t % rows;
    const int s = t / rows;
    const int r = tile * rows + rl;
    const int K = J / split;
    const typename Chunk<R>::T* Ls = L + (int64_t)site * J * N + r;

    R ar[4] = {0, 0, 0, 0}, ai[4] = {0, 0, 0, 0};
    int k = 0;
    for (; k + 4 <= K; k += 4) {
        typename Chunk<R>::T a[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] = Ls[(int64_t)(s + split * (k + q)) * N];
#pragma unroll
        for (int q = 0; q < 4; ++q) chunk_mac(a[q], ul + (s + split * (k + q)) * cpc, ar[q], ai[q]);
    }
    for (; k < K; ++k) {
        const typename Chunk<R>::T a = Ls[(int64_t)(s + split * k) * N];
        chunk_mac(a, ul + (s + split * k) * cpc, ar[0], ai[0]);
    }
    R sr = (ar[0] + ar[1]) + (ar[2] + ar[3]);
    R si = (ai[0] + ai[1]) + (ai[2] + ai[3]);
    if (split > 1) {
        red[s * rows + rl] = cpx<R>{sr, si};
        __syncthreads();
        if (s != 0) return;
        for (int q = 1; q < split; ++q) {
            sr += red[q * rows + rl].re;
            si += red[q * rows + rl].im;
        }
    }
    y[(int64_t)site * N + r] = cpx<R>{sr, si};
}

static int complex_per_chunk(qmg_prec p) { return p == QMG_C128 ? 1 : 2; }
static size_t chunk_bytes() { return 16; }

// Built-in launch choice: all rows of a site per work-group; the smallest
// split (dividing J) that gives at least 2^18 threads in flight while
// keeping at least 4 chunks per thread; row tiles only when a work-group
// would exceed 1024 threads.
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
    while (rt * best > 1024) {  // N odd multiple: fall back to fewer split lanes
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
                    "coarse launch rows=%d split=%d invalid (need rows | N=%d, split | J=%d, "
                    "rows*split <= 1024)",
                    rows, split, op->N, op->J);
    return QMG_OK;
}

template <typename R>
static qmg_status launch_dslash(const qmg_coarse_op_s* op, const void* in, void* out, hipStream_t s) {
    const int ntiles = op->N / op->rows;
    const dim3 grid((unsigned)(op->V * ntiles));
    const dim3 block((unsigned)(op->rows * op->split));
    const size_t lds = sizeof(cpx<R>) * (9 * op->N + (op->split > 1 ? op->rows * op->split : 0));
    hipLaunchKernelGGL(k_coarse_dslash<R>, grid, block, lds, s,
                       reinterpret_cast<const typename Chunk<R>::T*>(op->links), op->nbr,
                       reinterpret_cast<const cpx<R>*>(in), reinterpret_cast<cpx<R>*>(out), op->N,
                       op->J, op->rows, op->split, ntiles);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

}  // namespace qmg

using namespace qmg;

extern "C" qmg_status qmg_coarse_op_create(const int dims[4], int N, const void* X, const void* Y,
                                           qmg_prec storage, void* stream, qmg_coarse_op* out) {
    if (!out) return fail(QMG_ERR_ARG, "coarse_op_create: out is NULL");
    *out = nullptr;
    QMG_TRY(check_dims(dims, 2, "coarse_op_create"));
    if (N < 2 || N > 128 || (N & 1)) return fail(QMG_ERR_SHAPE, "coarse_op_create: N=%d must be even in [2,128]", N);
    if (!X || !Y) return fail(QMG_ERR_ARG, "coarse_op_create: X or Y is NULL");
    if (storage != QMG_C128 && storage != QMG_C64)
        return fail(QMG_ERR_PREC, "coarse_op_create: storage %d not supported", (int)storage);
    hipStream_t s = as_stream(stream);
    auto* op = new qmg_coarse_op_s();
    for (int m = 0; m < 4; ++m) op->dims[m] = dims[m];
    op->V = volume(dims);
    op->N = N;
    op->storage = storage;
    op->J = 9 * N / complex_per_chunk(storage);
    const size_t bytes = (size_t)op->V * op->J * N * chunk_bytes();
    hipError_t e = hipMalloc(&op->links, bytes);
    if (e != hipSuccess) {
        delete op;
        return fail(QMG_ERR_NOMEM, "coarse_op_create: %zu bytes: %s", bytes, hipGetErrorString(e));
    }
    qmg_status st = make_neighbour_table(dims, &op->nbr, s);
    if (st != QMG_OK) {
        (void)hipFree(op->links);
        delete op;
        return st;
    }
    const int64_t total = op->V * op->J * N;
    const unsigned nb = (unsigned)((total + 255) / 256);
    if (storage == QMG_C128)
        hipLaunchKernelGGL(k_pack_c128, dim3(nb), dim3(256), 0, s, (double2*)op->links,
                           (const double2*)X, (const double2*)Y, op->V, N, op->J);
    else
        hipLaunchKernelGGL(k_pack_c64, dim3(nb), dim3(256), 0, s, (float4*)op->links,
                           (const double2*)X, (const double2*)Y, op->V, N, op->J);
    e = hipGetLastError();
    if (e != hipSuccess) {
        qmg_coarse_op_destroy(op);
        return fail(QMG_ERR_HIP, "coarse_op_create: pack launch: %s", hipGetErrorString(e));
    }
    default_launch(op, &op->rows, &op->split);
    *out = op;
    return QMG_OK;
}

extern "C" qmg_status qmg_coarse_op_export(qmg_coarse_op op, void* X, void* Y, void* stream) {
    if (!op || !X || !Y) return fail(QMG_ERR_ARG, "coarse_op_export: NULL argument");
    hipStream_t s = as_stream(stream);
    const int64_t total = op->V * op->J * op->N;
    const unsigned nb = (unsigned)((total + 255) / 256);
    if (op->storage == QMG_C128)
        hipLaunchKernelGGL(k_unpack_c128, dim3(nb), dim3(256), 0, s, (const double2*)op->links,
                           (double2*)X, (double2*)Y, op->V, op->N, op->J);
    else
        hipLaunchKernelGGL(k_unpack_c64, dim3(nb), dim3(256), 0, s, (const float4*)op->links,
                           (double2*)X, (double2*)Y, op->V, op->N, op->J);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

extern "C" qmg_status qmg_coarse_dslash(qmg_coarse_op op, const void* in, void* out, qmg_prec prec,
                                        void* stream) {
    if (!op || !in || !out) return fail(QMG_ERR_ARG, "coarse_dslash: NULL argument");
    if (prec != op->storage)
        return fail(QMG_ERR_PREC, "coarse_dslash: vector precision %d != operator storage %d",
                    (int)prec, (int)op->storage);
    if (in == out) return fail(QMG_ERR_ARG, "coarse_dslash: in and out alias");
    hipStream_t s = as_stream(stream);
    if (op->storage == QMG_C128) return launch_dslash<double>(op, in, out, s);
    return launch_dslash<float>(op, in, out, s);
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
    if (op->nbr) (void)hipFree(op->nbr);
    delete op;
}
