// Red-black (even-odd) preconditioning of the coarse operator (Sec. 3.3; the
// solver of Sec. 7.1 uses it on every level).  The hops of Eq. (3) join sites
// of opposite parity p(x) = (x0 + x1 + x2 + x3) mod 2 (every extent even), so
// with the site-local block X and the hops Y the Schur complement on the even
// sites is
//     S = X_ee - Y_eo X_oo^-1 Y_oe,
// and Mhat x = b is solved by S x_e = b_e - Y_eo X_oo^-1 b_o followed by
// x_o = X_oo^-1 (b_o - Y_oe x_e).
//
// The operator is split into two operators on V/2 sites each, in the stencil
// kernel's own link layout:
//   even half: [X_ee | Y_0 .. Y_7 of the even sites], neighbours = half-lattice
//              indices of the odd sites;
//   odd half:  [X_oo^-1 | -X_oo^-1 Y_0 .. -X_oo^-1 Y_7 of the odd sites],
//              neighbours = half-lattice indices of the even sites.
// Then (each line one stencil launch over V/2 sites, coarse_dslash.hip):
//   S u_e:          t_o = odd half, hops only (u_e);  y_e = even half, all (self u_e, hops t_o)
//   reconstruction: x_o = odd half, all (self b_o, hops x_e)
//   source:         t_o = odd half, local block only (b_o); s_e = even half, hops only (t_o);
//                   bhat_e = b_e - s_e
// so S costs 17 of the 18 half-site blocks one application of Mhat reads.
// X_oo^-1 and the products X_oo^-1 Y_d are formed once, in FP64 (Gauss-Jordan
// elimination with partial pivoting, one work-group per site).
#include "handles.h"

#include <vector>

namespace qmg {

qmg_status coarse_eo_launch(const qmg_coarse_op_s* op, const EoArgs& ea, const void* in, void* out, qmg_prec vprec,
                            int m, hipStream_t s);
qmg_status coarse_op_build(const int dims[4], int64_t V, int N, const void* X, const void* Y, qmg_prec storage,
                           int* nbr, hipStream_t s, qmg_coarse_op* out);

namespace {

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// dst[b][h][e] = src[b][hsite[h]][e] for nblk blocks of NN entries per site
__global__ void k_gather_blocks(double2* __restrict__ dst, const double2* __restrict__ src,
                                const int* __restrict__ hsite, int64_t Vh, int64_t V, int64_t NN, int nblk) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nblk * Vh * NN) return;
    const int64_t e = g % NN;
    const int64_t h = (g / NN) % Vh;
    const int64_t b = g / (NN * Vh);
    dst[g] = src[(b * V + hsite[h]) * NN + e];
}

// augmented [Vh][N][2N]: the site's block on the left, the identity on the right
__global__ void k_aug_init(double2* __restrict__ A, const double2* __restrict__ X, const int* __restrict__ hsite,
                           int64_t Vh, int N) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int W = 2 * N;
    if (g >= Vh * N * W) return;
    const int j = (int)(g % W);
    const int i = (int)((g / W) % N);
    const int64_t h = g / ((int64_t)N * W);
    A[g] = j < N ? X[((int64_t)hsite[h] * N + i) * N + j] : make_double2(j - N == i ? 1.0 : 0.0, 0.0);
}

// Gauss-Jordan elimination with partial pivoting on each site's augmented
// [N][2N] block (one work-group per site, the block in global memory, which
// stays in the caches); afterwards the right half holds the inverse.
__global__ __launch_bounds__(256) void k_batched_gauss_jordan(double2* __restrict__ A, int N) {
    double2* M = A + (int64_t)blockIdx.x * N * 2 * N;
    const int W = 2 * N;
    const int t = threadIdx.x, T = blockDim.x;
    __shared__ int piv_s;
    __shared__ double2 fcol[128];
    for (int col = 0; col < N; ++col) {
        if (t < 64) {   // pivot: the largest |M[i][col]|, i >= col (lowest index on ties)
            double best = -1.0;
            int bi = col;
            for (int i = col + t; i < N; i += 64) {
                const double2 v = M[i * W + col];
                const double mg = v.x * v.x + v.y * v.y;
                if (mg > best) { best = mg; bi = i; }
            }
            for (int o = 32; o > 0; o >>= 1) {
                const double ob = __shfl_xor(best, o, 64);
                const int oi = __shfl_xor(bi, o, 64);
                if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
            }
            if (t == 0) piv_s = bi;
        }
        __syncthreads();
        const int piv = piv_s;
        if (piv != col)
            for (int j = t; j < W; j += T) {
                const double2 a = M[col * W + j];
                M[col * W + j] = M[piv * W + j];
                M[piv * W + j] = a;
            }
        __syncthreads();
        const double2 p = M[col * W + col];
        const double den = p.x * p.x + p.y * p.y;
        const double2 ip = make_double2(p.x / den, -p.y / den);
        for (int i = t; i < N; i += T)
            if (i != col) fcol[i] = M[i * W + col];
        __syncthreads();   // every thread has read the pivot before its row is scaled
        for (int j = t; j < W; j += T) M[col * W + j] = zmul(ip, M[col * W + j]);
        __syncthreads();
        for (int idx = t; idx < N * W; idx += T) {
            const int i = idx / W, j = idx - (idx / W) * W;
            if (i == col) continue;
            const double2 f = fcol[i], a = M[col * W + j];
            double2 v = M[idx];
            v.x -= f.x * a.x - f.y * a.y;
            v.y -= f.x * a.y + f.y * a.x;
            M[idx] = v;
        }
        __syncthreads();
    }
}

// Xinv [Vh][N][N] = right half of the augmented blocks
__global__ void k_aug_extract(double2* __restrict__ Xinv, const double2* __restrict__ A, int64_t Vh, int N) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= Vh * N * N) return;
    const int j = (int)(g % N);
    const int i = (int)((g / N) % N);
    const int64_t h = g / ((int64_t)N * N);
    Xinv[g] = A[(h * N + i) * 2 * N + N + j];
}

// Yh[d][h] = -Xinv[h] Y_d(hsite[h]) (canonical layouts); one work-group per (d, h)
__global__ __launch_bounds__(256) void k_hop_times_inverse(double2* __restrict__ Yh, const double2* __restrict__ Xinv,
                                                           const double2* __restrict__ Y, const int* __restrict__ hsite,
                                                           int64_t Vh, int64_t V, int N) {
    const int64_t h = blockIdx.x % Vh;
    const int d = (int)(blockIdx.x / Vh);
    const double2* A = Xinv + h * N * N;
    const double2* B = Y + ((int64_t)d * V + hsite[h]) * N * N;
    double2* C = Yh + ((int64_t)d * Vh + h) * N * N;
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int r = e / N, c = e - (e / N) * N;
        double re = 0, im = 0;
        for (int k = 0; k < N; ++k) {
            const double2 a = A[r * N + k], b = B[k * N + c];
            re += a.x * b.x - a.y * b.y;
            im += a.x * b.y + a.y * b.x;
        }
        C[e] = make_double2(-re, -im);
    }
}

// half[b][h][c] = full[b][hsite[h]][c]   (SUB: half = full - half)
template <typename R, bool SUB>
__global__ void k_eo_gather(cpx<R>* __restrict__ half, const cpx<R>* __restrict__ full, const int* __restrict__ hsite,
                            int64_t Vh, int64_t V, int dof) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= Vh * dof) return;
    const int64_t h = g / dof;
    const int c = (int)(g - h * dof);
    const int64_t b = blockIdx.y;
    const cpx<R> v = full[(b * V + hsite[h]) * dof + c];
    cpx<R>& o = half[b * Vh * dof + g];
    if constexpr (SUB) o = cpx<R>{v.re - o.re, v.im - o.im};
    else o = v;
}

// full[b][hsite_p[h]] = half[b][h]; full[b][hsite_q[h]] = 0 when hsite_q is given
template <typename R>
__global__ void k_eo_scatter(cpx<R>* __restrict__ full, const cpx<R>* __restrict__ half,
                             const int* __restrict__ hsite_p, const int* __restrict__ hsite_q, int64_t Vh, int64_t V,
                             int dof) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= Vh * dof) return;
    const int64_t h = g / dof;
    const int c = (int)(g - h * dof);
    const int64_t b = blockIdx.y;
    full[(b * V + hsite_p[h]) * dof + c] = half[b * Vh * dof + g];
    if (hsite_q) full[(b * V + hsite_q[h]) * dof + c] = cpx<R>{R(0), R(0)};
}

// half-lattice neighbour tables [2][V/2][8] on the host: hnbr[p][h][d] = (neighbour d of
// the h-th site of parity p) >> 1
std::vector<int> half_neighbours(const int dims[4]) {
    const int64_t V = volume(dims), Vh = V / 2;
    std::vector<int> out(V * 8);
    for (int64_t i = 0; i < V; ++i) {
        int x[4];
        int64_t t = i;
        int par = 0;
        for (int m = 0; m < 4; ++m) { x[m] = (int)(t % dims[m]); t /= dims[m]; par += x[m]; }
        const int64_t h = i >> 1;
        for (int d = 0; d < 8; ++d) {
            const int mu = d / 2, step = (d & 1) ? -1 : 1;
            int y[4] = {x[0], x[1], x[2], x[3]};
            y[mu] = (y[mu] + step + dims[mu]) % dims[mu];
            const int64_t j = y[0] + (int64_t)dims[0] * (y[1] + (int64_t)dims[1] * (y[2] + (int64_t)dims[2] * y[3]));
            out[((par & 1) * Vh + h) * 8 + d] = (int)(j >> 1);
        }
    }
    return out;
}

qmg_status upload(const std::vector<int>& h, size_t first, size_t count, int** dev, hipStream_t s) {
    QMG_HIP(hipMalloc(dev, sizeof(int) * count));
    hipError_t e = hipMemcpyAsync(*dev, h.data() + first, sizeof(int) * count, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(*dev);
        *dev = nullptr;
        return fail(QMG_ERR_HIP, "half-lattice table upload: %s", hipGetErrorString(e));
    }
    return QMG_OK;
}

inline unsigned blocks(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

// Build op's two half operators in `storage` from canonical complex128
// X [V][N][N], Y [8][V][N][N] of the operator (device).  Blocks.
qmg_status coarse_schur_build(qmg_coarse_op_s* op, const void* Xc, const void* Yc, qmg_prec storage, hipStream_t s) {
    for (int m = 0; m < 4; ++m)
        if (op->dims[m] % 2)
            return fail(QMG_ERR_SHAPE, "coarse red-black form: extent %d of dimension %d is odd", op->dims[m], m);
    const int N = op->N;
    const int64_t V = op->V, Vh = V / 2, NN = (int64_t)N * N;
    const double2* X = static_cast<const double2*>(Xc);
    const double2* Y = static_cast<const double2*>(Yc);
    if (!op->hsite) QMG_TRY(make_half_site_table(op->dims, &op->hsite, s));
    const int* hs0 = op->hsite;
    const int* hs1 = op->hsite + Vh;
    const std::vector<int> hn = half_neighbours(op->dims);
    double2 *Xe = nullptr, *Ye = nullptr, *Aug = nullptr, *Xi = nullptr, *Yh = nullptr;
    hipError_t e = hipMalloc(&Xe, Vh * NN * 16);
    if (e == hipSuccess) e = hipMalloc(&Ye, 8 * Vh * NN * 16);
    if (e == hipSuccess) e = hipMalloc(&Aug, 2 * Vh * NN * 16);
    if (e == hipSuccess) e = hipMalloc(&Xi, Vh * NN * 16);
    if (e == hipSuccess) e = hipMalloc(&Yh, 8 * Vh * NN * 16);
    qmg_status st = e == hipSuccess ? QMG_OK : fail(QMG_ERR_NOMEM, "coarse red-black form: %s", hipGetErrorString(e));
    if (st == QMG_OK) {
        hipLaunchKernelGGL(k_gather_blocks, dim3(blocks(Vh * NN)), dim3(256), 0, s, Xe, X, hs0, Vh, V, NN, 1);
        hipLaunchKernelGGL(k_gather_blocks, dim3(blocks(8 * Vh * NN)), dim3(256), 0, s, Ye, Y, hs0, Vh, V, NN, 8);
        hipLaunchKernelGGL(k_aug_init, dim3(blocks(2 * Vh * NN)), dim3(256), 0, s, Aug, X, hs1, Vh, N);
        hipLaunchKernelGGL(k_batched_gauss_jordan, dim3((unsigned)Vh), dim3(256), 0, s, Aug, N);
        hipLaunchKernelGGL(k_aug_extract, dim3(blocks(Vh * NN)), dim3(256), 0, s, Xi, Aug, Vh, N);
        hipLaunchKernelGGL(k_hop_times_inverse, dim3((unsigned)(8 * Vh)), dim3(256), 0, s, Yh, Xi, Y, hs1, Vh, V, N);
        e = hipGetLastError();
        if (e != hipSuccess) st = fail(QMG_ERR_HIP, "coarse red-black form: launch: %s", hipGetErrorString(e));
    }
    int *ne = nullptr, *no = nullptr;
    if (st == QMG_OK) st = upload(hn, 0, Vh * 8, &ne, s);
    if (st == QMG_OK) st = upload(hn, Vh * 8, Vh * 8, &no, s);
    qmg_coarse_op_s *even = nullptr, *odd = nullptr;
    if (st == QMG_OK) {
        st = coarse_op_build(op->dims, Vh, N, Xe, Ye, storage, ne, s, &even);
        ne = nullptr;   // owned by the half operator (also on failure)
    }
    if (st == QMG_OK) {
        st = coarse_op_build(op->dims, Vh, N, Xi, Yh, storage, no, s, &odd);
        no = nullptr;
    }
    if (st == QMG_OK && hipStreamSynchronize(s) != hipSuccess) st = fail(QMG_ERR_HIP, "coarse red-black form: build");
    if (ne) (void)hipFree(ne);
    if (no) (void)hipFree(no);
    for (double2* p : {Xe, Ye, Aug, Xi, Yh})
        if (p) (void)hipFree(p);
    if (st != QMG_OK) {
        if (even) qmg_coarse_op_destroy(even);
        if (odd) qmg_coarse_op_destroy(odd);
        return st;
    }
    if (op->eo_even) qmg_coarse_op_destroy(op->eo_even);
    if (op->eo_odd) qmg_coarse_op_destroy(op->eo_odd);
    op->eo_even = even;
    op->eo_odd = odd;
    return QMG_OK;
}

static qmg_status need_schur(const qmg_coarse_op_s* op) {
    if (!op->eo_even || !op->eo_odd)
        return fail(QMG_ERR_STATE, "coarse red-black form not prepared (qmg_coarse_op_prepare_schur)");
    return QMG_OK;
}

// out_e = S in_e; tmp_o: odd half-lattice scratch of m members
qmg_status coarse_schur_apply(const qmg_coarse_op_s* op, const void* in_e, void* out_e, void* tmp_o, qmg_prec vprec,
                              int m, hipStream_t s) {
    QMG_TRY(need_schur(op));
    const int64_t Vh = op->V / 2;
    QMG_TRY(coarse_eo_launch(op->eo_odd, EoArgs{nullptr, nullptr, nullptr, 1, 8, 0, Vh}, in_e, tmp_o, vprec, m, s));
    return coarse_eo_launch(op->eo_even, EoArgs{in_e, nullptr, nullptr, 0, 9, Vh, Vh}, tmp_o, out_e, vprec, m, s);
}

// generic half/whole-lattice re-indexing (R = complex128 or complex64 components)
qmg_status eo_gather(const int* hsite, int64_t Vh, int dof, const void* full, void* half, bool sub, qmg_prec vprec,
                     int m, hipStream_t s) {
    const dim3 grid(blocks(Vh * dof), (unsigned)m);
    if (vprec == QMG_C128) {
        if (sub) hipLaunchKernelGGL((k_eo_gather<double, true>), grid, dim3(256), 0, s, (cpx<double>*)half, (const cpx<double>*)full, hsite, Vh, 2 * Vh, dof);
        else hipLaunchKernelGGL((k_eo_gather<double, false>), grid, dim3(256), 0, s, (cpx<double>*)half, (const cpx<double>*)full, hsite, Vh, 2 * Vh, dof);
    } else {
        if (sub) hipLaunchKernelGGL((k_eo_gather<float, true>), grid, dim3(256), 0, s, (cpx<float>*)half, (const cpx<float>*)full, hsite, Vh, 2 * Vh, dof);
        else hipLaunchKernelGGL((k_eo_gather<float, false>), grid, dim3(256), 0, s, (cpx<float>*)half, (const cpx<float>*)full, hsite, Vh, 2 * Vh, dof);
    }
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

qmg_status eo_scatter(const int* hsite_p, const int* hsite_q, int64_t Vh, int dof, const void* half, void* full,
                      qmg_prec vprec, int m, hipStream_t s) {
    const dim3 grid(blocks(Vh * dof), (unsigned)m);
    if (vprec == QMG_C128)
        hipLaunchKernelGGL(k_eo_scatter<double>, grid, dim3(256), 0, s, (cpx<double>*)full, (const cpx<double>*)half,
                           hsite_p, hsite_q, Vh, 2 * Vh, dof);
    else
        hipLaunchKernelGGL(k_eo_scatter<float>, grid, dim3(256), 0, s, (cpx<float>*)full, (const cpx<float>*)half,
                           hsite_p, hsite_q, Vh, 2 * Vh, dof);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

// bhat_e = b_e - Y_eo X_oo^-1 b_o for whole-lattice b
qmg_status coarse_schur_source(const qmg_coarse_op_s* op, const void* b, void* bhat_e, void* tmp_o, qmg_prec vprec,
                               int m, hipStream_t s) {
    QMG_TRY(need_schur(op));
    const int64_t Vh = op->V / 2;
    QMG_TRY(coarse_eo_launch(op->eo_odd, EoArgs{b, op->hsite + Vh, nullptr, 0, 1, op->V, Vh}, b, tmp_o, vprec, m, s));
    QMG_TRY(coarse_eo_launch(op->eo_even, EoArgs{nullptr, nullptr, nullptr, 1, 8, 0, Vh}, tmp_o, bhat_e, vprec, m, s));
    return eo_gather(op->hsite, Vh, op->N, b, bhat_e, true, vprec, m, s);
}

// whole-lattice x from x_e: x_o = X_oo^-1 b_o - X_oo^-1 Y_oe x_e
qmg_status coarse_schur_reconstruct(const qmg_coarse_op_s* op, const void* x_e, const void* b, void* x,
                                    qmg_prec vprec, int m, hipStream_t s) {
    QMG_TRY(need_schur(op));
    const int64_t Vh = op->V / 2;
    QMG_TRY(coarse_eo_launch(op->eo_odd, EoArgs{b, op->hsite + Vh, op->hsite + Vh, 0, 9, op->V, op->V}, x_e, x, vprec,
                             m, s));
    return eo_scatter(op->hsite, nullptr, Vh, op->N, x_e, x, vprec, m, s);
}

}  // namespace qmg

using namespace qmg;

extern "C" qmg_status qmg_coarse_op_prepare_schur(qmg_coarse_op op, void* stream) {
    if (!op) return fail(QMG_ERR_ARG, "coarse_op_prepare_schur: NULL operator");
    hipStream_t s = as_stream(stream);
    const size_t blk = (size_t)op->V * op->N * op->N * 16;
    void *X = nullptr, *Y = nullptr;
    hipError_t e = hipMalloc(&X, blk);
    if (e == hipSuccess) e = hipMalloc(&Y, 8 * blk);
    qmg_status st = e == hipSuccess ? QMG_OK : fail(QMG_ERR_NOMEM, "coarse_op_prepare_schur: %s", hipGetErrorString(e));
    if (st == QMG_OK) st = qmg_coarse_op_export(op, X, Y, stream);
    if (st == QMG_OK) st = coarse_schur_build(op, X, Y, op->storage, s);
    (void)hipStreamSynchronize(s);
    if (X) (void)hipFree(X);
    if (Y) (void)hipFree(Y);
    return st;
}

static qmg_status coarse_schur_checks(qmg_coarse_op op, int nrhs, qmg_prec prec, const char* what) {
    if (!op) return fail(QMG_ERR_ARG, "%s: NULL operator", what);
    QMG_TRY(need_schur(op));
    if (nrhs < 1 || nrhs > kMaxFieldBatch) return fail(QMG_ERR_ARG, "%s: nrhs %d not in [1, %d]", what, nrhs, kMaxFieldBatch);
    const bool ok = op->storage == QMG_C128 ? prec == QMG_C128 : prec == QMG_C64;
    if (!ok) return fail(QMG_ERR_PREC, "%s: vector precision %d does not fit operator storage %d", what, (int)prec,
                         (int)op->storage);
    return QMG_OK;
}

static qmg_status coarse_schur_tmp(qmg_coarse_op op, int nrhs, qmg_prec prec, hipStream_t s) {
    const size_t need = (size_t)nrhs * (op->V / 2) * op->N * (prec == QMG_C128 ? 16 : 8);
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

extern "C" qmg_status qmg_coarse_dslash_schur(qmg_coarse_op op, const void* in_e, void* out_e, int nrhs,
                                              qmg_prec prec, void* stream) {
    QMG_TRY(coarse_schur_checks(op, nrhs, prec, "coarse_dslash_schur"));
    if (!in_e || !out_e) return fail(QMG_ERR_ARG, "coarse_dslash_schur: NULL field");
    if (in_e == out_e) return fail(QMG_ERR_ARG, "coarse_dslash_schur: in and out alias");
    hipStream_t s = as_stream(stream);
    QMG_TRY(coarse_schur_tmp(op, nrhs, prec, s));
    return coarse_schur_apply(op, in_e, out_e, op->eo_tmp, prec, nrhs, s);
}

extern "C" qmg_status qmg_coarse_schur_source(qmg_coarse_op op, const void* b, void* bhat_e, int nrhs, qmg_prec prec,
                                              void* stream) {
    QMG_TRY(coarse_schur_checks(op, nrhs, prec, "coarse_schur_source"));
    if (!b || !bhat_e) return fail(QMG_ERR_ARG, "coarse_schur_source: NULL field");
    if (b == bhat_e) return fail(QMG_ERR_ARG, "coarse_schur_source: b and bhat alias");
    hipStream_t s = as_stream(stream);
    QMG_TRY(coarse_schur_tmp(op, nrhs, prec, s));
    return coarse_schur_source(op, b, bhat_e, op->eo_tmp, prec, nrhs, s);
}

extern "C" qmg_status qmg_coarse_schur_reconstruct(qmg_coarse_op op, const void* x_e, const void* b, void* x, int nrhs,
                                                   qmg_prec prec, void* stream) {
    QMG_TRY(coarse_schur_checks(op, nrhs, prec, "coarse_schur_reconstruct"));
    if (!x_e || !b || !x) return fail(QMG_ERR_ARG, "coarse_schur_reconstruct: NULL field");
    if (x == b || x == x_e) return fail(QMG_ERR_ARG, "coarse_schur_reconstruct: x aliases an input");
    return coarse_schur_reconstruct(op, x_e, b, x, prec, nrhs, as_stream(stream));
}
