// Exact solve of the coarsest level through an explicit inverse (an option of
// the multigrid solver; the paper's coarsest solve is GCR, Sec. 7.1).  The
// coarsest operator is small (n = V*N unknowns, at most 4096), so its dense
// matrix is assembled from X and Y, inverted once at setup by Gauss-Jordan
// elimination with partial pivoting in FP64, and stored in the solver's inner
// precision; every coarsest solve is then one matrix-vector product (one
// matrix-matrix product for a batch), a single launch with no global
// reductions -- the latency the coarsest GCR spends on synchronisations.
#include "handles.h"

#include <cmath>

namespace qmg {

// A[(x,i), (x,j)] = X(x)_{ij}; A[(x,i), (nbr_d(x), j)] += Y_d(x)_{ij}, into the
// left half of the n x 2n matrix M = [A | I] (row stride 2n).  One thread per
// (x, i, j), adding the nine blocks of its row in a fixed order (on extent-2
// lattices two directions reach the same neighbour).  M starts zeroed.
__global__ void k_assemble(double2* __restrict__ M, const double2* __restrict__ X, const double2* __restrict__ Y,
                           const int* __restrict__ nbr, int64_t V, int N) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= V * N * N) return;
    const int j = (int)(g % N);
    const int i = (int)((g / N) % N);
    const int64_t x = g / ((int64_t)N * N);
    const int64_t n = V * N;
    double2* row = M + (x * N + i) * 2 * n;
    double2 v = X[(x * N + i) * N + j];
    row[x * N + j].x += v.x;
    row[x * N + j].y += v.y;
    for (int d = 0; d < 8; ++d) {
        const int64_t y = nbr[x * 8 + d];
        v = Y[((int64_t)d * V + x) * N * N + (int64_t)i * N + j];
        row[y * N + j].x += v.x;
        row[y * N + j].y += v.y;
    }
}

// M is n x 2n ([A | I]).  Step k, part 1 (one work-group): the row p >= k of
// largest |M[p][k]|; stores p and M[p][k].
__global__ __launch_bounds__(1024) void k_pivot(const double2* __restrict__ M, int n, int k, int* __restrict__ piv,
                                                double2* __restrict__ pval) {
    __shared__ double best[1024];
    __shared__ int where[1024];
    double b = -1.0;
    int w = k;
    for (int i = k + threadIdx.x; i < n; i += blockDim.x) {
        const double2 a = M[(int64_t)i * 2 * n + k];
        const double m = a.x * a.x + a.y * a.y;
        if (m > b) { b = m; w = i; }
    }
    best[threadIdx.x] = b;
    where[threadIdx.x] = w;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            const double o = best[threadIdx.x + s];
            const int ow = where[threadIdx.x + s];
            if (o > best[threadIdx.x] || (o == best[threadIdx.x] && ow < where[threadIdx.x])) {
                best[threadIdx.x] = o;
                where[threadIdx.x] = ow;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *piv = where[0];
        *pval = M[(int64_t)where[0] * 2 * n + k];
    }
}

// Part 2: swap rows k and p, divide row k by the pivot; save column k of every
// row (the elimination factors) before part 3 overwrites it.
__global__ void k_swap_scale(double2* __restrict__ M, int n, int k, const int* __restrict__ piv,
                             const double2* __restrict__ pval, int* __restrict__ singular) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= 2 * n) return;
    const int p = *piv;
    const double2 pv = *pval;
    const double den = pv.x * pv.x + pv.y * pv.y;
    if (c == 0 && !(den > 0)) *singular = 1;
    const double2 inv = make_double2(pv.x / den, -pv.y / den);
    double2* rk = M + (int64_t)k * 2 * n;
    double2* rp = M + (int64_t)p * 2 * n;
    const double2 t = rp[c];
    if (p != k) rp[c] = rk[c];
    rk[c] = make_double2(t.x * inv.x - t.y * inv.y, t.x * inv.y + t.y * inv.x);
}

__global__ void k_save_col(const double2* __restrict__ M, int n, int k, double2* __restrict__ f) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) f[i] = M[(int64_t)i * 2 * n + k];
}

// Part 3: M[i][c] -= f_i M[k][c] for i != k, columns c >= k (left of k the
// pivot row is zero).  Grid: (columns, rows).
__global__ void k_eliminate(double2* __restrict__ M, int n, int k, const double2* __restrict__ f) {
    const int c = k + blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (c >= 2 * n || i == k) return;
    const double2 a = f[i];
    const double2 b = M[(int64_t)k * 2 * n + c];
    double2& m = M[(int64_t)i * 2 * n + c];
    m.x -= a.x * b.x - a.y * b.y;
    m.y -= a.x * b.y + a.y * b.x;
}

__global__ void k_identity_right(double2* __restrict__ M, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) M[(int64_t)i * 2 * n + n + i] = make_double2(1.0, 0.0);
}

template <typename R>
__global__ void k_take_inverse(cpx<R>* __restrict__ inv, const double2* __restrict__ M, int n) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)n * n) return;
    const int64_t i = g / n, j = g % n;
    const double2 v = M[i * 2 * n + n + j];
    inv[g] = cpx<R>{(R)v.x, (R)v.y};
}

// y_m = Ainv b_m for members m of a batch ([nb][n] fields).  One work-group
// per (row, group of up to M members): its 256 threads stride the row, VEC
// complex numbers per load, four loads issued before any arithmetic so that
// HBM latency is covered; each thread keeps one partial per member.  Members
// past the last of a group read the last member's data and are not stored.
// A shuffle tree per wave and then the four waves in order sum the partials
// (fixed order, repeatable).
template <typename R, int VEC, int M>
__global__ __launch_bounds__(256) void k_dense_apply(const cpx<R>* __restrict__ Ainv, const cpx<R>* __restrict__ b,
                                                     cpx<R>* __restrict__ y, int n, int nb) {
    constexpr int U = 4;
    __shared__ R red[2][M][4];
    const int groups = (nb + M - 1) / M;
    const int row = (int)blockIdx.x / groups, m0 = ((int)blockIdx.x % groups) * M;
    const int nm = nb - m0 < M ? nb - m0 : M;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    R ar[M], ai[M];
#pragma unroll
    for (int m = 0; m < M; ++m) ar[m] = ai[m] = 0;
    const cpx<R>* a = Ainv + (int64_t)row * n;
    for (int c0 = threadIdx.x * VEC; c0 < n; c0 += 256 * VEC * U) {
        cpx<R> v[U][VEC];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int c = c0 + j * 256 * VEC;
#pragma unroll
            for (int q = 0; q < VEC; ++q) v[j][q] = c < n ? a[c + q] : cpx<R>{0, 0};
        }
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int mm = m < nm ? m0 + m : m0 + nm - 1;
            const cpx<R>* bm = b + (int64_t)mm * n;
            cpx<R> u[U][VEC];
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int c = c0 + j * 256 * VEC;
#pragma unroll
                for (int q = 0; q < VEC; ++q) u[j][q] = c < n ? bm[c + q] : cpx<R>{0, 0};
            }
#pragma unroll
            for (int j = 0; j < U; ++j)
#pragma unroll
                for (int q = 0; q < VEC; ++q) {
                    ar[m] += v[j][q].re * u[j][q].re - v[j][q].im * u[j][q].im;
                    ai[m] += v[j][q].re * u[j][q].im + v[j][q].im * u[j][q].re;
                }
        }
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
        for (int o = 32; o > 0; o >>= 1) {
            ar[m] += __shfl_down(ar[m], o, 64);
            ai[m] += __shfl_down(ai[m], o, 64);
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int m = 0; m < M; ++m) {
            red[0][m][w] = ar[m];
            red[1][m][w] = ai[m];
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nm) {
        const int m = threadIdx.x;
        const R re = ((red[0][m][0] + red[0][m][1]) + red[0][m][2]) + red[0][m][3];
        const R im = ((red[1][m][0] + red[1][m][1]) + red[1][m][2]) + red[1][m][3];
        y[(int64_t)(m0 + m) * n + row] = cpx<R>{re, im};
    }
}

// Build the inverse of the coarse operator in precision `prec` (complex128 or
// complex64) into *out (allocated here, owned by the caller).  Blocks.
qmg_status dense_inverse(qmg_coarse_op_s* op, qmg_prec prec, void** out, hipStream_t s) {
    const int64_t n = op->V * op->N;
    if (n > 4096) return fail(QMG_ERR_SHAPE, "coarse direct solve: %lld unknowns exceed 4096", (long long)n);
    const size_t blk = (size_t)op->V * op->N * op->N;
    double2 *X = nullptr, *Y = nullptr, *M = nullptr, *f = nullptr, *pval = nullptr;
    int* piv = nullptr;   // piv[0]: pivot row; piv[1]: set when a pivot was zero
    void* inv = nullptr;
    const size_t eb = prec == QMG_C128 ? 16 : 8;
    hipError_t e = hipMalloc(&X, blk * 16);
    if (e == hipSuccess) e = hipMalloc(&Y, 8 * blk * 16);
    if (e == hipSuccess) e = hipMalloc(&M, (size_t)n * 2 * n * 16);
    if (e == hipSuccess) e = hipMalloc(&f, n * 16);
    if (e == hipSuccess) e = hipMalloc(&pval, 16);
    if (e == hipSuccess) e = hipMalloc(&piv, 2 * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&inv, (size_t)n * n * eb);
    auto cleanup = [&]() {
        for (void* p : {(void*)X, (void*)Y, (void*)M, (void*)f, (void*)pval, (void*)piv})
            if (p) (void)hipFree(p);
    };
    if (e != hipSuccess) {
        cleanup();
        if (inv) (void)hipFree(inv);
        return fail(QMG_ERR_NOMEM, "coarse direct solve: %s", hipGetErrorString(e));
    }
    qmg_status st = qmg_coarse_op_export(op, X, Y, s);
    if (st == QMG_OK) {
        (void)hipMemsetAsync(M, 0, (size_t)n * 2 * n * 16, s);
        (void)hipMemsetAsync(piv, 0, 2 * sizeof(int), s);
        const int64_t tot = op->V * op->N * op->N;
        hipLaunchKernelGGL(k_assemble, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, M, X, Y, op->nbr, op->V, op->N);
        hipLaunchKernelGGL(k_identity_right, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, M, (int)n);
    }
    for (int k = 0; k < n && st == QMG_OK; ++k) {
        hipLaunchKernelGGL(k_pivot, dim3(1), dim3(1024), 0, s, M, (int)n, k, piv, pval);
        hipLaunchKernelGGL(k_swap_scale, dim3((unsigned)((2 * n + 255) / 256)), dim3(256), 0, s, M, (int)n, k, piv, pval,
                           piv + 1);
        hipLaunchKernelGGL(k_save_col, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, M, (int)n, k, f);
        hipLaunchKernelGGL(k_eliminate, dim3((unsigned)((2 * n - k + 255) / 256), (unsigned)n), dim3(256), 0, s, M,
                           (int)n, k, f);
        if (hipGetLastError() != hipSuccess) st = fail(QMG_ERR_HIP, "coarse direct solve: launch failed at step %d", k);
    }
    if (st == QMG_OK) {
        const unsigned g = (unsigned)(((int64_t)n * n + 255) / 256);
        if (prec == QMG_C128) hipLaunchKernelGGL(k_take_inverse<double>, dim3(g), dim3(256), 0, s, (cpx<double>*)inv, M, (int)n);
        else hipLaunchKernelGGL(k_take_inverse<float>, dim3(g), dim3(256), 0, s, (cpx<float>*)inv, M, (int)n);
        int sing = 0;
        e = hipMemcpyAsync(&sing, piv + 1, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = fail(QMG_ERR_HIP, "coarse direct solve: %s", hipGetErrorString(e));
        else if (sing) st = fail(QMG_ERR_NONFINITE, "coarse direct solve: the coarsest operator is singular");
    }
    cleanup();
    if (st != QMG_OK) {
        (void)hipFree(inv);
        return st;
    }
    *out = inv;
    return QMG_OK;
}

template <typename R, int VEC>
static void dense_apply_t(const void* Ainv, const void* b, void* y, int64_t n, int nb, hipStream_t s) {
    if (nb == 1)
        hipLaunchKernelGGL((k_dense_apply<R, VEC, 1>), dim3((unsigned)n), dim3(256), 0, s, (const cpx<R>*)Ainv,
                           (const cpx<R>*)b, (cpx<R>*)y, (int)n, nb);
    else
        hipLaunchKernelGGL((k_dense_apply<R, VEC, 8>), dim3((unsigned)(n * ((nb + 7) / 8))), dim3(256), 0, s,
                           (const cpx<R>*)Ainv, (const cpx<R>*)b, (cpx<R>*)y, (int)n, nb);
}

qmg_status dense_apply(const void* Ainv, const void* b, void* y, int64_t n, int nb, qmg_prec prec, hipStream_t s) {
    if (prec == QMG_C128) dense_apply_t<double, 1>(Ainv, b, y, n, nb, s);
    else if (n % 2 == 0) dense_apply_t<float, 2>(Ainv, b, y, n, nb, s);
    else dense_apply_t<float, 1>(Ainv, b, y, n, nb, s);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

}  // namespace qmg
