// Transfer operators (Sec. 3.4 step 3 and Sec. 6.6).
//
// Setup: the near-null vectors are cut into hypercubic aggregates; within
// each aggregate the two chirality halves of every vector (fine level: spins
// {0,1} vs {2,3}; coarse parent: components n < N/2 vs n >= N/2) are
// orthonormalised separately by modified Gram-Schmidt in vector order, every
// projection done twice, normalised so that R has a real positive diagonal.
// One work-group per (aggregate, chirality), FP64, working set in global
// memory (it is read from L2).
//
// Apply:
//   prolong  (P u)(x)_f = sum_k V(x)_{f,k} u(xc(x))_{chi(f)*Nvec + k}
//            a gather, one thread per fine degree of freedom;
//   restrict (R psi)(xc)_{chi*Nvec + k} = sum_{x in xc, chi(f) = chi} conj(V(x)_{f,k}) psi(x)_f
//            one work-group per aggregate, each thread owning one coarse
//            component and a slice of the aggregate, partial sums combined in
//            LDS in a fixed order: no atomics, bitwise repeatable.
// The basis is kept as [V][dof][Nvec] (row f of site x holds the Nvec
// coefficients of its chirality) in the storage precision, plus an FP64 copy
// for the Galerkin build.  The 16-bit storage keeps each complex entry as an
// FP16 pair with no scale: the columns are orthonormal within an aggregate,
// so no entry exceeds 1 in modulus.
#include "codes16.h"
#include "handles.h"

#include <vector>

namespace qmg {

__device__ __forceinline__ double block_sum(double v, double* red) {
    // sum over the work-group; result returned to every thread
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    double t = 0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) t += red[i];
    return t;
}

// gather vecs [nvec][V][dof] -> W [Vc][2][nvec][Lb]  (Lb = bsites*dof/2)
__global__ void k_gather_blocks(double2* __restrict__ W, const double2* __restrict__ vecs,
                                const int* __restrict__ members, int64_t V, int64_t Vc, int dof,
                                int nvec, int bsites) {
    const int half = dof / 2;
    const int64_t Lb = (int64_t)bsites * half;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = Vc * 2 * nvec * Lb;
    if (g >= total) return;
    const int64_t p = g % Lb;
    int64_t t = g / Lb;
    const int k = (int)(t % nvec);
    t /= nvec;
    const int chi = (int)(t % 2);
    const int64_t xc = t / 2;
    const int64_t x = members[xc * bsites + p / half];
    const int f = chi * half + (int)(p % half);
    W[g] = vecs[((int64_t)k * V + x) * dof + f];
}

// MGS on one (aggregate, chirality) per work-group.
__global__ __launch_bounds__(256) void k_block_mgs(double2* __restrict__ W, int nvec, int64_t Lb,
                                                    double rank_tol, int* __restrict__ rank_fail) {
    __shared__ double red[8];
    double2* Wb = W + (int64_t)blockIdx.x * nvec * Lb;
    for (int k = 0; k < nvec; ++k) {
        double2* wk = Wb + (int64_t)k * Lb;
        double s = 0;
        for (int64_t i = threadIdx.x; i < Lb; i += blockDim.x) s += wk[i].x * wk[i].x + wk[i].y * wk[i].y;
        const double before = sqrt(block_sum(s, red));
        for (int pass = 0; pass < 2; ++pass)
            for (int j = 0; j < k; ++j) {
                const double2* wj = Wb + (int64_t)j * Lb;
                double cr = 0, cim = 0;
                for (int64_t i = threadIdx.x; i < Lb; i += blockDim.x) {
                    cr += wj[i].x * wk[i].x + wj[i].y * wk[i].y;    // conj(wj) * wk
                    cim += wj[i].x * wk[i].y - wj[i].y * wk[i].x;
                }
                cr = block_sum(cr, red);
                cim = block_sum(cim, red);
                for (int64_t i = threadIdx.x; i < Lb; i += blockDim.x) {
                    const double2 a = wj[i];
                    wk[i].x -= cr * a.x - cim * a.y;
                    wk[i].y -= cr * a.y + cim * a.x;
                }
                __syncthreads();
            }
        s = 0;
        for (int64_t i = threadIdx.x; i < Lb; i += blockDim.x) s += wk[i].x * wk[i].x + wk[i].y * wk[i].y;
        const double nrm = sqrt(block_sum(s, red));
        if (!(nrm >= rank_tol * before) || nrm == 0.0) {
            if (threadIdx.x == 0) rank_fail[0] = 1;
        }
        const double inv = nrm > 0 ? 1.0 / nrm : 0.0;
        for (int64_t i = threadIdx.x; i < Lb; i += blockDim.x) {
            wk[i].x *= inv;
            wk[i].y *= inv;
        }
        __syncthreads();
    }
}

// W [Vc][2][nvec][Lb] -> basis [V][dof][nvec]
__global__ void k_scatter_basis(double2* __restrict__ B, const double2* __restrict__ W,
                                const int* __restrict__ members, int64_t Vc, int dof, int nvec,
                                int bsites) {
    const int half = dof / 2;
    const int64_t Lb = (int64_t)bsites * half;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= Vc * 2 * nvec * Lb) return;
    const int64_t p = g % Lb;
    int64_t t = g / Lb;
    const int k = (int)(t % nvec);
    t /= nvec;
    const int chi = (int)(t % 2);
    const int64_t xc = t / 2;
    const int64_t x = members[xc * bsites + p / half];
    const int f = chi * half + (int)(p % half);
    B[(x * dof + f) * nvec + k] = W[g];
}

__global__ void k_to_c64(float2* __restrict__ o, const double2* __restrict__ i, int64_t n) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n) o[g] = make_float2((float)i[g].x, (float)i[g].y);
}
__global__ void k_to_h16(uint32_t* __restrict__ o, const double2* __restrict__ i, int64_t n, unsigned* __restrict__ nf) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    note_nonfinite(nf, !(isfinite(i[g].x) && isfinite(i[g].y)));
    o[g] = enc_pair<FMT_H16>((float)i[g].x, (float)i[g].y);
}

// A stored basis entry as a complex number of the arithmetic precision R:
// BT = cpx<R> (complex128 or complex64 storage) or a 32-bit FP16 pair.
template <typename R> __device__ __forceinline__ cpx<R> bval(const cpx<R>& b) { return b; }
template <typename R> __device__ __forceinline__ cpx<R> bval(const uint32_t& w) {
    const cpx<float> v = dec_pair<FMT_H16>(w);
    return cpx<R>{(R)v.re, (R)v.im};
}

// CPC consecutive basis entries, read once per application: non-temporal
// loads, so the basis stream does not push the fine vector being restricted
// out of the caches (restriction 52.6 -> 51.1 us on 16^3x32, Nvec 24; the
// prolongation, which reads the small coarse vector, was slower with them,
// 61.2 -> 62.8 us, and keeps plain loads).
template <typename BT, int CPC>
__device__ __forceinline__ void ld_basis(BT (&b)[CPC], const BT* p) {
    constexpr int bytes = (int)sizeof(BT) * CPC;
    if constexpr (bytes == 4) {
        b[0] = __builtin_nontemporal_load(reinterpret_cast<const BT*>(p));
    } else if constexpr (bytes == 8) {
        typedef int i2 __attribute__((ext_vector_type(2)));
        const i2 v = __builtin_nontemporal_load(reinterpret_cast<const i2*>(p));
        __builtin_memcpy(b, &v, 8);
    } else {
        static_assert(bytes % 16 == 0, "basis chunks of 4, 8 or a multiple of 16 bytes");
        typedef int i4 __attribute__((ext_vector_type(4)));
        i4 v[bytes / 16];
#pragma unroll
        for (int i = 0; i < bytes / 16; ++i) v[i] = __builtin_nontemporal_load(reinterpret_cast<const i4*>(p) + i);
        __builtin_memcpy(b, v, bytes);
    }
}

// Prolongation: one thread per 16-byte chunk of the basis ([x][f][k] row
// major, so a wave reads one contiguous span).  A work-group covers RPT
// consecutive spans of rows_per_wg rows; each thread issues its RPT chunk
// loads before any arithmetic so that enough bytes are in flight to cover
// HBM latency.  The `cpr` chunks of a row (x, f) are then summed in LDS in a
// fixed order, one thread per row.
template <typename R, typename BT, int CPC, int RPT>
__global__ __launch_bounds__(256) void k_prolong(cpx<R>* __restrict__ out, const BT* __restrict__ B,
                                                 const cpx<R>* __restrict__ uc, const int* __restrict__ owner,
                                                 int64_t V, int dof, int nvec, int rows_per_wg, int64_t cstride) {
    constexpr int cpc = CPC;
    __shared__ cpx<R> part[RPT][256];
    out += (int64_t)blockIdx.y * V * dof;          // batch member
    uc += (int64_t)blockIdx.y * cstride;
    const int cpr = nvec / cpc;                    // chunks per row
    const int t = threadIdx.x;
    const int lr = t / cpr, kc = t - (t / cpr) * cpr;
    const int64_t rows = V * dof;
    const int64_t base = (int64_t)blockIdx.x * rows_per_wg * RPT;
    BT b[RPT][cpc];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int64_t row = base + (int64_t)j * rows_per_wg + lr;
        if (lr < rows_per_wg && row < rows) {
#pragma unroll
            for (int q = 0; q < cpc; ++q) b[j][q] = B[row * nvec + kc * cpc + q];
        }
    }
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int64_t row = base + (int64_t)j * rows_per_wg + lr;
        R ar = 0, ai = 0;
        if (lr < rows_per_wg && row < rows) {
            const int64_t x = row / dof;
            const int f = (int)(row - x * dof);
            const int chi = f / (dof / 2);
            const cpx<R>* u = uc + (int64_t)owner[x] * 2 * nvec + chi * nvec + kc * cpc;
#pragma unroll
            for (int q = 0; q < cpc; ++q) {
                const cpx<R> bq = bval<R>(b[j][q]);
                cmac(ar, ai, bq.re, bq.im, u[q].re, u[q].im);
            }
        }
        part[j][t] = cpx<R>{ar, ai};
    }
    __syncthreads();
    for (int rr = t; rr < rows_per_wg * RPT; rr += 256) {
        const int j = rr / rows_per_wg, r = rr - j * rows_per_wg;
        const int64_t row = base + rr;
        if (row < rows) {
            R sr = 0, si = 0;
            for (int q = 0; q < cpr; ++q) {
                sr += part[j][r * cpr + q].re;
                si += part[j][r * cpr + q].im;
            }
            out[row] = cpx<R>{sr, si};
        }
    }
}

// Restriction: one work-group per aggregate.  Thread (slice, q) owns chunk q
// of the per-site basis block (dof x nvec, contiguous) and accumulates
// conj(V) psi over the aggregate's sites slice, slice + S, ...; the S slices
// and then the dof/2 rows of each chirality are summed in LDS in a fixed
// order.  No atomics; bitwise repeatable.  With S = 1 the threads stride over
// the chunks instead (blocks with more chunks than threads).
template <typename R, typename BT, int CPC>
__global__ __launch_bounds__(1024) void k_restrict(cpx<R>* __restrict__ out, const BT* __restrict__ B,
                                                   const cpx<R>* __restrict__ in, const int* __restrict__ members,
                                                   int dof, int nvec, int bsites, int64_t fstride, int S) {
    constexpr int cpc = CPC;
    extern __shared__ __align__(16) unsigned char smem[];
    in += (int64_t)blockIdx.y * fstride;           // batch member
    out += (int64_t)blockIdx.y * gridDim.x * 2 * nvec;
    cpx<R>* acc_l = reinterpret_cast<cpx<R>*>(smem);   // [S][dof][nvec]
    const int64_t xc = blockIdx.x;
    const int* mem = members + xc * bsites;
    const int cpr = nvec / cpc;
    const int nchunk = dof * cpr;
    const int slice = S > 1 ? (int)threadIdx.x / nchunk : 0;
    const int q0 = S > 1 ? (int)threadIdx.x - slice * nchunk : (int)threadIdx.x;
    const int qstep = S > 1 ? nchunk : (int)blockDim.x;
    if (slice < S) {
        cpx<R>* acc_s = acc_l + (int64_t)slice * dof * nvec;
        for (int q = q0; q < nchunk; q += qstep) {
            const int f = q / cpr, kc = q - (q / cpr) * cpr;
            R ar[cpc], ai[cpc];
#pragma unroll
            for (int c = 0; c < cpc; ++c) ar[c] = ai[c] = 0;
            int b = slice;
            for (; b + 3 * S < bsites; b += 4 * S) {
                int64_t x[4];
                cpx<R> v[4];
                BT bb[4][cpc];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    x[j] = mem[b + j * S];
                    v[j] = in[x[j] * dof + f];
                    ld_basis<BT, cpc>(bb[j], B + (x[j] * dof + f) * nvec + kc * cpc);
                }
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int c = 0; c < cpc; ++c) {
                        const cpx<R> bq = bval<R>(bb[j][c]);
                        cmac_conj(ar[c], ai[c], bq.re, bq.im, v[j].re, v[j].im);
                    }
            }
            for (; b < bsites; b += S) {
                const int64_t x = mem[b];
                const cpx<R> v = in[x * dof + f];
                BT bv[cpc];
                ld_basis<BT, cpc>(bv, B + (x * dof + f) * nvec + kc * cpc);
#pragma unroll
                for (int c = 0; c < cpc; ++c) {
                    const cpx<R> bq = bval<R>(bv[c]);
                    cmac_conj(ar[c], ai[c], bq.re, bq.im, v.re, v.im);
                }
            }
#pragma unroll
            for (int c = 0; c < cpc; ++c) acc_s[f * nvec + kc * cpc + c] = cpx<R>{ar[c], ai[c]};
        }
    }
    __syncthreads();
    const int half = dof / 2;
    const int64_t sstride = (int64_t)dof * nvec;
    for (int n = threadIdx.x; n < 2 * nvec; n += blockDim.x) {
        const int chi = n / nvec, k = n - chi * nvec;
        R sr = 0, si = 0;
        for (int ff = 0; ff < half; ++ff)
            for (int sl = 0; sl < S; ++sl) {
                const cpx<R> a = acc_l[sl * sstride + (chi * half + ff) * nvec + k];
                sr += a.re;
                si += a.im;
            }
        out[xc * 2 * nvec + n] = cpx<R>{sr, si};
    }
}

}  // namespace qmg

using namespace qmg;

extern "C" void qmg_transfer_destroy(qmg_transfer t) {
    if (!t) return;
    if (t->basis && t->basis != (void*)t->basis64) (void)hipFree(t->basis);
    if (t->basis64) (void)hipFree(t->basis64);
    if (t->members) (void)hipFree(t->members);
    if (t->owner) (void)hipFree(t->owner);
    delete t;
}

namespace {

// Validation, aggregate tables and the FP64 basis buffer shared by
// qmg_transfer_create and qmg_transfer_import; `what` prefixes the messages.
qmg_status transfer_shell(const char* what, const int fine_dims[4], int fine_dof, const int block[4], int nvec,
                          const void* vecs, qmg_prec storage, hipStream_t s, qmg_transfer_s** out) {
    QMG_TRY(check_dims(fine_dims, 2, what));
    if (!block || !vecs) return fail(QMG_ERR_ARG, "%s: NULL argument", what);
    if (fine_dof < 2 || (fine_dof & 1) || fine_dof > 128)
        return fail(QMG_ERR_SHAPE, "%s: fine_dof %d must be even in [2,128]", what, fine_dof);
    if (nvec < 1 || 2 * nvec > 128) return fail(QMG_ERR_SHAPE, "%s: nvec %d outside [1,64]", what, nvec);
    if (storage != QMG_C128 && storage != QMG_C64 && storage != QMG_H16)
        return fail(QMG_ERR_PREC, "%s: storage %d not supported", what, (int)storage);
    int cd[4];
    int64_t bs = 1;
    for (int m = 0; m < 4; ++m) {
        if (block[m] < 1 || fine_dims[m] % block[m])
            return fail(QMG_ERR_SHAPE, "%s: block %d does not divide extent %d (dim %d)", what, block[m],
                        fine_dims[m], m);
        cd[m] = fine_dims[m] / block[m];
        if (cd[m] < 2) return fail(QMG_ERR_SHAPE, "%s: coarse extent %d < 2 in dim %d", what, cd[m], m);
        bs *= block[m];
    }
    if ((int64_t)nvec > bs * (fine_dof / 2))
        return fail(QMG_ERR_SHAPE, "%s: nvec %d exceeds aggregate dimension %lld", what, nvec,
                    (long long)(bs * (fine_dof / 2)));
    auto* t = new qmg_transfer_s();
    for (int m = 0; m < 4; ++m) { t->fdims[m] = fine_dims[m]; t->block[m] = block[m]; t->cdims[m] = cd[m]; }
    t->V = volume(fine_dims);
    t->Vc = volume(cd);
    t->dof = fine_dof;
    t->nvec = nvec;
    t->bsites = (int)bs;
    t->storage = storage;

    // aggregate tables on the host
    std::vector<int> members(t->V), owner(t->V), fill(t->Vc, 0);
    for (int64_t i = 0; i < t->V; ++i) {
        int64_t r = i;
        int x[4];
        for (int m = 0; m < 4; ++m) { x[m] = (int)(r % fine_dims[m]); r /= fine_dims[m]; }
        const int64_t xc = x[0] / block[0] + (int64_t)cd[0] * (x[1] / block[1] + (int64_t)cd[1] * (x[2] / block[2] + (int64_t)cd[2] * (x[3] / block[3])));
        owner[i] = (int)xc;
        members[xc * bs + fill[xc]++] = (int)i;
    }
    const size_t nb = (size_t)t->V * fine_dof * nvec;
    hipError_t e = hipMalloc(&t->members, sizeof(int) * t->V);
    if (e == hipSuccess) e = hipMalloc(&t->owner, sizeof(int) * t->V);
    if (e == hipSuccess) e = hipMalloc(&t->basis64, sizeof(double2) * nb);
    if (e == hipSuccess) e = hipMemcpyAsync(t->members, members.data(), sizeof(int) * t->V, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(t->owner, owner.data(), sizeof(int) * t->V, hipMemcpyHostToDevice, s);
    // the host tables are released on return: the copies must have landed
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        qmg_transfer_destroy(t);
        return fail(e == hipErrorOutOfMemory ? QMG_ERR_NOMEM : QMG_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    }
    *out = t;
    return QMG_OK;
}

// The storage-precision copy of the FP64 basis (the same buffer for QMG_C128).
qmg_status transfer_finish(const char* what, qmg_transfer_s* t, hipStream_t s) {
    const size_t nb = (size_t)t->V * t->dof * t->nvec;
    if (t->storage == QMG_C128) {
        t->basis = t->basis64;
        return QMG_OK;
    }
    const bool h16 = t->storage == QMG_H16;
    const hipError_t e = hipMalloc(&t->basis, (h16 ? sizeof(uint32_t) : sizeof(float2)) * nb);
    if (e != hipSuccess) return fail(QMG_ERR_NOMEM, "%s: %s", what, hipGetErrorString(e));
    if (h16) {
        unsigned* nf = nullptr;
        QMG_TRY(nonfinite_flag(&nf));
        hipLaunchKernelGGL(k_to_h16, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, (uint32_t*)t->basis,
                           t->basis64, (int64_t)nb, nf);
        QMG_LAUNCH_CHECK();
        return take_nonfinite(s, what);
    } else
        hipLaunchKernelGGL(k_to_c64, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, (float2*)t->basis,
                           t->basis64, (int64_t)nb);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

}  // namespace

extern "C" qmg_status qmg_transfer_create(const int fine_dims[4], int fine_dof, const int block[4],
                                          int nvec, const void* nullvecs, qmg_prec storage,
                                          void* stream, qmg_transfer* out) {
    if (!out) return fail(QMG_ERR_ARG, "transfer_create: out is NULL");
    *out = nullptr;
    hipStream_t s = as_stream(stream);
    qmg_transfer_s* t = nullptr;
    QMG_TRY(transfer_shell("transfer_create", fine_dims, fine_dof, block, nvec, nullvecs, storage, s, &t));
    const int64_t Lb = (int64_t)t->bsites * (fine_dof / 2);
    const size_t wbytes = sizeof(double2) * (size_t)t->Vc * 2 * nvec * Lb;
    double2* W = nullptr;
    int* flag = nullptr;
    hipError_t e = hipMalloc(&W, wbytes);
    if (e == hipSuccess) e = hipMalloc(&flag, sizeof(int));
    if (e == hipSuccess) e = hipMemsetAsync(flag, 0, sizeof(int), s);
    if (e != hipSuccess) {
        if (W) (void)hipFree(W);
        if (flag) (void)hipFree(flag);
        qmg_transfer_destroy(t);
        return fail(e == hipErrorOutOfMemory ? QMG_ERR_NOMEM : QMG_ERR_HIP, "transfer_create: %s", hipGetErrorString(e));
    }
    const int64_t total = t->Vc * 2 * nvec * Lb;
    const unsigned g1 = (unsigned)((total + 255) / 256);
    hipLaunchKernelGGL(k_gather_blocks, dim3(g1), dim3(256), 0, s, W, (const double2*)nullvecs, t->members,
                       t->V, t->Vc, fine_dof, nvec, t->bsites);
    hipLaunchKernelGGL(k_block_mgs, dim3((unsigned)(t->Vc * 2)), dim3(256), 0, s, W, nvec, Lb, 1e-10, flag);
    hipLaunchKernelGGL(k_scatter_basis, dim3(g1), dim3(256), 0, s, t->basis64, W, t->members, t->Vc,
                       fine_dof, nvec, t->bsites);
    e = hipGetLastError();
    int hflag = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(W);
    (void)hipFree(flag);
    if (e != hipSuccess) {
        qmg_transfer_destroy(t);
        return fail(QMG_ERR_HIP, "transfer_create: %s", hipGetErrorString(e));
    }
    if (hflag) {
        qmg_transfer_destroy(t);
        return fail(QMG_ERR_ARG, "transfer_create: near-null vectors are linearly dependent within an aggregate");
    }
    const qmg_status st = transfer_finish("transfer_create", t, s);
    if (st != QMG_OK) {
        qmg_transfer_destroy(t);
        return st;
    }
    *out = t;
    return QMG_OK;
}

extern "C" qmg_status qmg_transfer_import(const int fine_dims[4], int fine_dof, const int block[4], int nvec,
                                          const void* basis, qmg_prec storage, void* stream, qmg_transfer* out) {
    if (!out) return fail(QMG_ERR_ARG, "transfer_import: out is NULL");
    *out = nullptr;
    hipStream_t s = as_stream(stream);
    qmg_transfer_s* t = nullptr;
    QMG_TRY(transfer_shell("transfer_import", fine_dims, fine_dof, block, nvec, basis, storage, s, &t));
    qmg_status st = QMG_OK;
    if (hipMemcpyAsync(t->basis64, basis, sizeof(double2) * (size_t)t->V * fine_dof * nvec, hipMemcpyDeviceToDevice,
                       s) != hipSuccess)
        st = fail(QMG_ERR_HIP, "transfer_import: basis copy failed");
    if (st == QMG_OK) st = transfer_finish("transfer_import", t, s);
    if (st == QMG_OK && hipStreamSynchronize(s) != hipSuccess) st = fail(QMG_ERR_HIP, "transfer_import: sync");
    if (st != QMG_OK) {
        qmg_transfer_destroy(t);
        return st;
    }
    *out = t;
    return QMG_OK;
}

extern "C" qmg_status qmg_transfer_coarse_dims(qmg_transfer t, int cdims[4], int* N) {
    if (!t || !cdims || !N) return fail(QMG_ERR_ARG, "transfer_coarse_dims: NULL argument");
    for (int m = 0; m < 4; ++m) cdims[m] = t->cdims[m];
    *N = 2 * t->nvec;
    return QMG_OK;
}

extern "C" qmg_status qmg_transfer_export(qmg_transfer t, void* basis, void* stream) {
    if (!t || !basis) return fail(QMG_ERR_ARG, "transfer_export: NULL argument");
    QMG_HIP(hipMemcpyAsync(basis, t->basis64, sizeof(double2) * (size_t)t->V * t->dof * t->nvec,
                           hipMemcpyDeviceToDevice, as_stream(stream)));
    return QMG_OK;
}

namespace qmg {
template <typename R, typename BT, int CPC>
static qmg_status prolong_t(qmg_transfer t, const void* B, const void* in, void* out, int nb, hipStream_t s) {
    constexpr int RPT = 4;
    const int cpr = t->nvec / CPC;
    const int rows_per_wg = 256 / cpr;
    const int64_t rows = t->V * t->dof;
    const int64_t per_wg = (int64_t)rows_per_wg * RPT;
    const unsigned nblk = (unsigned)((rows + per_wg - 1) / per_wg);
    hipLaunchKernelGGL((k_prolong<R, BT, CPC, RPT>), dim3(nblk, nb), dim3(256), 0, s, (cpx<R>*)out, (const BT*)B,
                       (const cpx<R>*)in, t->owner, t->V, t->dof, t->nvec, rows_per_wg, t->Vc * 2 * t->nvec);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

template <typename R, typename BT, int CPC>
static qmg_status restrict_t(qmg_transfer t, const void* B, const void* in, void* out, int nb, hipStream_t s) {
    const int nchunk = t->dof * (t->nvec / CPC);
    const size_t lds1 = sizeof(cpx<R>) * t->dof * t->nvec;
    // site slices per aggregate: as many as fit in 1024 threads and 64 KiB of
    // LDS, at most 8 and at most the aggregate's sites
    int S = 1024 / nchunk;
    if (S > 8) S = 8;
    if (S > t->bsites) S = t->bsites;
    while (S > 1 && (size_t)S * lds1 > 65536) --S;
    if (S < 1) S = 1;
    int threads = S > 1 ? S * nchunk : nchunk;
    threads = ((threads + 63) / 64) * 64;
    if (threads > 1024) threads = 1024;
    const size_t lds = lds1 * S;
    if (lds > 65536)
        QMG_HIP(hipFuncSetAttribute((const void*)k_restrict<R, BT, CPC>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lds));
    hipLaunchKernelGGL((k_restrict<R, BT, CPC>), dim3((unsigned)t->Vc, nb), dim3(threads), lds, s, (cpx<R>*)out,
                       (const BT*)B, (const cpx<R>*)in, t->members, t->dof, t->nvec, t->bsites, t->V * t->dof, S);
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}

// complex64 fields with a 16-bit basis: 16-byte chunks of four FP16 pairs
// where nvec allows, else 8 or 4 bytes
qmg_status transfer_prolong(qmg_transfer t, const void* in, void* out, qmg_prec p, int nb, hipStream_t s) {
    using C64 = cpx<float>;
    if (p == QMG_C128) return prolong_t<double, cpx<double>, 1>(t, t->basis64, in, out, nb, s);
    if (t->storage == QMG_H16) {
        if (t->nvec % 4 == 0) return prolong_t<float, uint32_t, 4>(t, t->basis, in, out, nb, s);
        if (t->nvec % 2 == 0) return prolong_t<float, uint32_t, 2>(t, t->basis, in, out, nb, s);
        return prolong_t<float, uint32_t, 1>(t, t->basis, in, out, nb, s);
    }
    if (t->nvec % 2) return prolong_t<float, C64, 1>(t, t->basis, in, out, nb, s);
    return prolong_t<float, C64, 2>(t, t->basis, in, out, nb, s);
}

qmg_status transfer_restrict(qmg_transfer t, const void* in, void* out, qmg_prec p, int nb, hipStream_t s) {
    using C64 = cpx<float>;
    if (p == QMG_C128) return restrict_t<double, cpx<double>, 1>(t, t->basis64, in, out, nb, s);
    if (t->storage == QMG_H16) {
        if (t->nvec % 4 == 0) return restrict_t<float, uint32_t, 4>(t, t->basis, in, out, nb, s);
        if (t->nvec % 2 == 0) return restrict_t<float, uint32_t, 2>(t, t->basis, in, out, nb, s);
        return restrict_t<float, uint32_t, 1>(t, t->basis, in, out, nb, s);
    }
    if (t->nvec % 2) return restrict_t<float, C64, 1>(t, t->basis, in, out, nb, s);
    return restrict_t<float, C64, 2>(t, t->basis, in, out, nb, s);
}
}  // namespace qmg

static qmg_status check_transfer_prec(qmg_transfer t, qmg_prec p, const char* what) {
    if (p != QMG_C128 && p != QMG_C64) return fail(QMG_ERR_PREC, "%s: precision %d not supported", what, (int)p);
    if (p == QMG_C64 && t->storage != QMG_C64 && t->storage != QMG_H16)
        return fail(QMG_ERR_PREC, "%s: complex64 fields need a transfer created with complex64 or FP16 storage", what);
    return QMG_OK;
}

extern "C" qmg_status qmg_prolong(qmg_transfer t, const void* coarse_in, void* fine_out, int nrhs, qmg_prec p,
                                  void* stream) {
    if (!t || !coarse_in || !fine_out) return fail(QMG_ERR_ARG, "prolong: NULL argument");
    if (nrhs < 1 || nrhs > kMaxFieldBatch) return fail(QMG_ERR_ARG, "prolong: nrhs %d not in [1, %d]", nrhs, kMaxFieldBatch);
    QMG_TRY(check_transfer_prec(t, p, "prolong"));
    return transfer_prolong(t, coarse_in, fine_out, p, nrhs, as_stream(stream));
}

extern "C" qmg_status qmg_restrict(qmg_transfer t, const void* fine_in, void* coarse_out, int nrhs, qmg_prec p,
                                   void* stream) {
    if (!t || !fine_in || !coarse_out) return fail(QMG_ERR_ARG, "restrict: NULL argument");
    if (nrhs < 1 || nrhs > kMaxFieldBatch) return fail(QMG_ERR_ARG, "restrict: nrhs %d not in [1, %d]", nrhs, kMaxFieldBatch);
    QMG_TRY(check_transfer_prec(t, p, "restrict"));
    return transfer_restrict(t, fine_in, coarse_out, p, nrhs, as_stream(stream));
}
