// Mixed-precision BiCGStab with reliable updates: the Krylov solver the paper
// compares its multigrid against (Sec. 3.3 names BiCGStab with red-black
// preconditioning as the state of the art; Sec. 7.1 runs it in 16-bit
// precision with FP64 reliable updates).
//
// BiCGStab (van der Vorst) on A x = b from x = 0, shadow residual r~ = b:
//   rho = <r~, r>;  beta = (rho / rho_old)(alpha / omega);  p = r + beta (p - omega v)
//   v = A p;  alpha = rho / <r~, v>;  s = r - alpha v
//   t = A s;  omega = <t, s> / <t, t>;  x += alpha p + omega s;  r = s - omega t
// The iteration runs with the low-precision operator (FP32 arithmetic on
// complex64, FP16 or BF16 storage) and accumulates into a low-precision
// correction x_lo.  Reliable update (after Sleijpen and van der Vorst, as used
// for lattice QCD mixed-precision solvers): when |r| falls below delta times
// the largest |r| since the last update, or reaches the target, the
// correction is added to the FP64 solution x_hi, x_lo is cleared and the true
// residual b - A x_hi is recomputed with the FP64 operator; the iteration
// continues from it with its search direction kept.  It stops when the true
// residual is at most tol |b|.
//
// With the red-black form the system is the fine Schur complement
// S x_e = b_e - D_eo C_oo^-1 b_o (wilson.hip) and x_o is back-substituted in
// FP64 at the end.  Every scalar of the recursion stays on the device; the
// host reads |r|^2 once per step for the stopping and update tests.
#include "blas.h"
#include "handles.h"

#include <chrono>
#include <cmath>

namespace qmg {
qmg_status wilson_apply(const qmg_fine_op_s* op, const void* in, void* out, qmg_prec vprec, int members,
                        hipStream_t s);
qmg_status fine_schur_apply(const qmg_fine_op_s* op, const void* in_e, void* out_e, void* tmp_o, qmg_prec vprec,
                            int m, hipStream_t s);
qmg_status fine_schur_source(const qmg_fine_op_s* op, const void* b, void* bhat_e, void* tmp_o, qmg_prec vprec,
                             int m, hipStream_t s);
qmg_status fine_schur_reconstruct(const qmg_fine_op_s* op, const void* x_e, const void* b, void* x, qmg_prec vprec,
                                  int m, hipStream_t s);
}  // namespace qmg

using namespace qmg;

struct qmg_bicgstab_s {
    qmg_fine_op hi = nullptr, lo = nullptr;   // borrowed
    int eo = 0;
    int64_t n = 0;           // complex entries of the iterated system (V*12, or V*6 red-black)
    qmg_prec lp = QMG_C64;   // vector precision of the low-precision iteration
    Blas blas;
    double* dsc = nullptr;   // device scalars
    double* hsc = nullptr;   // pinned host mirror
    void *r = nullptr, *rt = nullptr, *p = nullptr, *v = nullptr, *s = nullptr, *t = nullptr, *xl = nullptr;
    void *tmp_lo = nullptr;                                   // odd half-lattice scratch (low precision)
    void *xh = nullptr, *r64 = nullptr, *b64 = nullptr, *t64 = nullptr, *tmp_hi = nullptr;   // FP64
    hipStream_t st = nullptr;
};

namespace {

// scalar slots (doubles)
constexpr int B_RHO = 0;      // 2: <r~, r>
constexpr int B_RHO_OLD = 2;  // 2
constexpr int B_ALPHA = 4;    // 2
constexpr int B_OMEGA = 6;    // 2
constexpr int B_RTV = 8;      // 2: <r~, v>
constexpr int B_TS = 10;      // 3: <t,t>, <t,s>.re, <t,s>.im
constexpr int B_RN = 14;      // 1: |r|^2
constexpr int B_N = 16;

struct zc { double re, im; };
__device__ __forceinline__ zc zmul(zc a, zc b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ zc zdiv(zc a, zc b) {
    const double d = b.re * b.re + b.im * b.im;
    return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
__device__ __forceinline__ zc ld(const double* p) { return {p[0], p[1]}; }

// p = r + beta (p - omega v), beta = (rho / rho_old)(alpha / omega)
template <typename R>
__global__ void k_bicg_p(const double* __restrict__ sc, const cpx<R>* __restrict__ r, cpx<R>* __restrict__ p,
                         const cpx<R>* __restrict__ v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const zc beta = zmul(zdiv(ld(sc + B_RHO), ld(sc + B_RHO_OLD)), zdiv(ld(sc + B_ALPHA), ld(sc + B_OMEGA)));
    const zc om = ld(sc + B_OMEGA);
    const cpx<R> a = p[i], w = v[i], q = r[i];
    // d = p - omega v
    const R dr = a.re - (R)(om.re * w.re - om.im * w.im), di = a.im - (R)(om.re * w.im + om.im * w.re);
    p[i] = cpx<R>{q.re + (R)(beta.re * dr - beta.im * di), q.im + (R)(beta.re * di + beta.im * dr)};
}

// alpha = rho / <r~, v>;  s = r - alpha v   (thread 0 keeps alpha)
template <typename R>
__global__ void k_bicg_s(double* __restrict__ sc, const cpx<R>* __restrict__ r, const cpx<R>* __restrict__ v,
                         cpx<R>* __restrict__ s, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const zc al = zdiv(ld(sc + B_RHO), ld(sc + B_RTV));
    if (i == 0) { sc[B_ALPHA] = al.re; sc[B_ALPHA + 1] = al.im; }
    if (i >= n) return;
    const cpx<R> a = r[i], w = v[i];
    s[i] = cpx<R>{a.re - (R)(al.re * w.re - al.im * w.im), a.im - (R)(al.re * w.im + al.im * w.re)};
}

// omega = <t,s>/<t,t>;  x += alpha p + omega s;  r = s - omega t
// (thread 0 keeps omega and moves rho to rho_old)
template <typename R>
__global__ void k_bicg_xr(double* __restrict__ sc, cpx<R>* __restrict__ x, cpx<R>* __restrict__ r,
                          const cpx<R>* __restrict__ p, const cpx<R>* __restrict__ s, const cpx<R>* __restrict__ t,
                          int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double tt = sc[B_TS];
    const zc om = tt > 0 ? zc{sc[B_TS + 1] / tt, sc[B_TS + 2] / tt} : zc{0.0, 0.0};
    const zc al = zdiv(ld(sc + B_RHO), ld(sc + B_RTV));
    if (i == 0) {
        sc[B_OMEGA] = om.re; sc[B_OMEGA + 1] = om.im;
        sc[B_RHO_OLD] = sc[B_RHO]; sc[B_RHO_OLD + 1] = sc[B_RHO + 1];
    }
    if (i >= n) return;
    const cpx<R> a = p[i], b = s[i], c = t[i];
    cpx<R> xx = x[i];
    xx.re += (R)(al.re * a.re - al.im * a.im) + (R)(om.re * b.re - om.im * b.im);
    xx.im += (R)(al.re * a.im + al.im * a.re) + (R)(om.re * b.im + om.im * b.re);
    x[i] = xx;
    r[i] = cpx<R>{b.re - (R)(om.re * c.re - om.im * c.im), b.im - (R)(om.re * c.im + om.im * c.re)};
}

// start of a cycle: rho_old = alpha = omega = 1
__global__ void k_bicg_reset(double* sc) {
    sc[B_RHO_OLD] = 1; sc[B_RHO_OLD + 1] = 0;
    sc[B_ALPHA] = 1; sc[B_ALPHA + 1] = 0;
    sc[B_OMEGA] = 1; sc[B_OMEGA + 1] = 0;
}

// x_hi += x_lo (promoted)
template <typename R>
__global__ void k_accumulate(double2* __restrict__ xh, const cpx<R>* __restrict__ xl, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    xh[i].x += (double)xl[i].re;
    xh[i].y += (double)xl[i].im;
}

unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

template <typename R>
qmg_status apply_lo(qmg_bicgstab_s* h, const void* in, void* out) {
    if (h->eo) return fine_schur_apply(h->lo, in, out, h->tmp_lo, h->lp, 1, h->st);
    return wilson_apply(h->lo, in, out, h->lp, 1, h->st);
}
qmg_status apply_hi(qmg_bicgstab_s* h, const void* in, void* out) {
    if (h->eo) return fine_schur_apply(h->hi, in, out, h->tmp_hi, QMG_C128, 1, h->st);
    return wilson_apply(h->hi, in, out, QMG_C128, 1, h->st);
}

qmg_status read(qmg_bicgstab_s* h, int slot, int count) {
    QMG_HIP(hipMemcpyAsync(h->hsc + slot, h->dsc + slot, sizeof(double) * count, hipMemcpyDeviceToHost, h->st));
    QMG_HIP(hipStreamSynchronize(h->st));
    return QMG_OK;
}

// r64 = b64 - A x_hi, r = (R) r64, |r64|^2 -> host
template <typename R>
qmg_status true_residual(qmg_bicgstab_s* h, double* rn2) {
    QMG_TRY(apply_hi(h, h->xh, h->t64));
    QMG_TRY(h->blas.xmy<double>(h->b64, h->t64, h->r64, h->n));
    QMG_TRY(h->blas.norm2<double>(h->r64, h->n, h->dsc + B_RN));
    QMG_TRY(h->blas.convert<double, R>(h->r64, h->r, h->n));
    QMG_TRY(read(h, B_RN, 1));
    *rn2 = h->hsc[B_RN];
    return QMG_OK;
}

template <typename R>
qmg_status solve(qmg_bicgstab_s* h, const void* b, void* x, const qmg_bicgstab_params* prm, qmg_solve_info* info) {
    const int64_t n = h->n;
    const size_t vb = n * sizeof(cpx<R>), vb64 = n * 16;
    const int64_t Vf = h->hi->V;
    auto t0 = std::chrono::steady_clock::now();
    // |b| of the whole system and the iterated system's right-hand side
    QMG_TRY(h->blas.norm2<double>(b, Vf * 12, h->dsc + B_RN));
    QMG_TRY(read(h, B_RN, 1));
    const double bnorm = std::sqrt(h->hsc[B_RN]);
    const double target = prm->tol * bnorm;
    if (h->eo) QMG_TRY(fine_schur_source(h->hi, b, h->b64, h->tmp_hi, QMG_C128, 1, h->st));
    else QMG_HIP(hipMemcpyAsync(h->b64, b, vb64, hipMemcpyDeviceToDevice, h->st));
    QMG_HIP(hipMemsetAsync(h->xh, 0, vb64, h->st));
    QMG_HIP(hipMemsetAsync(h->xl, 0, vb, h->st));
    QMG_HIP(hipMemsetAsync(h->p, 0, vb, h->st));
    QMG_HIP(hipMemsetAsync(h->v, 0, vb, h->st));
    double rn2 = 0;
    QMG_TRY(true_residual<R>(h, &rn2));
    QMG_HIP(hipMemcpyAsync(h->rt, h->r, vb, hipMemcpyDeviceToDevice, h->st));
    hipLaunchKernelGGL(k_bicg_reset, dim3(1), dim3(1), 0, h->st, h->dsc);
    QMG_LAUNCH_CHECK();
    double rn = std::sqrt(rn2), maxr = rn, true_rn = rn;
    int iters = 0, updates = 0;
    bool converged = bnorm == 0.0 || rn <= target;
    const unsigned g = blocks(n);
    while (!converged && iters < prm->maxit) {
        QMG_TRY(h->blas.dot<R>(h->rt, h->r, n, h->dsc + B_RHO));
        hipLaunchKernelGGL(k_bicg_p<R>, dim3(g), dim3(256), 0, h->st, h->dsc, (const cpx<R>*)h->r, (cpx<R>*)h->p,
                           (const cpx<R>*)h->v, n);
        QMG_LAUNCH_CHECK();
        QMG_TRY(apply_lo<R>(h, h->p, h->v));
        QMG_TRY(h->blas.dot<R>(h->rt, h->v, n, h->dsc + B_RTV));
        hipLaunchKernelGGL(k_bicg_s<R>, dim3(g), dim3(256), 0, h->st, h->dsc, (const cpx<R>*)h->r,
                           (const cpx<R>*)h->v, (cpx<R>*)h->s, n);
        QMG_LAUNCH_CHECK();
        QMG_TRY(apply_lo<R>(h, h->s, h->t));
        QMG_TRY(h->blas.dot_norm<R>(h->t, h->s, n, h->dsc + B_TS));
        hipLaunchKernelGGL(k_bicg_xr<R>, dim3(g), dim3(256), 0, h->st, h->dsc, (cpx<R>*)h->xl, (cpx<R>*)h->r,
                           (const cpx<R>*)h->p, (const cpx<R>*)h->s, (const cpx<R>*)h->t, n);
        QMG_LAUNCH_CHECK();
        QMG_TRY(h->blas.norm2<R>(h->r, n, h->dsc + B_RN));
        QMG_TRY(read(h, B_RHO, B_N));
        ++iters;
        rn = std::sqrt(h->hsc[B_RN]);
        const bool breakdown = !(std::isfinite(rn)) || (h->hsc[B_RHO] == 0 && h->hsc[B_RHO + 1] == 0) ||
                               !(h->hsc[B_TS] > 0);
        if (!std::isfinite(rn) && !std::isfinite(h->hsc[B_TS]))
            return fail(QMG_ERR_NONFINITE, "bicgstab: non-finite residual at step %d", iters);
        maxr = rn > maxr ? rn : maxr;
        if (breakdown || rn < prm->delta * maxr || rn <= target || iters >= prm->maxit) {
            // reliable update: fold the correction into the FP64 solution, true residual in FP64
            hipLaunchKernelGGL(k_accumulate<R>, dim3(g), dim3(256), 0, h->st, (double2*)h->xh, (const cpx<R>*)h->xl, n);
            QMG_LAUNCH_CHECK();
            QMG_HIP(hipMemsetAsync(h->xl, 0, vb, h->st));
            QMG_TRY(true_residual<R>(h, &rn2));
            true_rn = std::sqrt(rn2);
            if (!std::isfinite(true_rn)) return fail(QMG_ERR_NONFINITE, "bicgstab: non-finite true residual");
            rn = maxr = true_rn;
            ++updates;
            converged = true_rn <= target;
            if (breakdown && !converged) {   // restart the recursion from the true residual
                QMG_HIP(hipMemcpyAsync(h->rt, h->r, vb, hipMemcpyDeviceToDevice, h->st));
                QMG_HIP(hipMemsetAsync(h->p, 0, vb, h->st));
                QMG_HIP(hipMemsetAsync(h->v, 0, vb, h->st));
                hipLaunchKernelGGL(k_bicg_reset, dim3(1), dim3(1), 0, h->st, h->dsc);
                QMG_LAUNCH_CHECK();
            }
        }
    }
    // the whole-lattice solution and its true residual
    if (h->eo) QMG_TRY(fine_schur_reconstruct(h->hi, h->xh, b, x, QMG_C128, 1, h->st));
    else QMG_HIP(hipMemcpyAsync(x, h->xh, vb64, hipMemcpyDeviceToDevice, h->st));
    const int64_t nf = Vf * 12;
    void* tf = h->eo ? h->s : h->t64;   // scratch of at least V*12 complex128 entries
    void* rf = h->eo ? h->t : h->r64;
    QMG_TRY(wilson_apply(h->hi, x, tf, QMG_C128, 1, h->st));
    QMG_TRY(h->blas.xmy<double>(b, tf, rf, nf));
    QMG_TRY(h->blas.norm2<double>(rf, nf, h->dsc + B_RN));
    QMG_TRY(read(h, B_RN, 1));
    const double final_rel = bnorm > 0 ? std::sqrt(h->hsc[B_RN]) / bnorm : 0.0;
    auto t1 = std::chrono::steady_clock::now();
    const bool ok = bnorm == 0.0 || final_rel <= prm->tol;
    if (info) {
        *info = qmg_solve_info{};
        info->outer_iters = iters;
        info->level_iters[0] = iters;
        info->restarts = updates;
        info->converged = ok ? 1 : 0;
        info->true_rel_residual = final_rel;
        info->seconds = std::chrono::duration<double>(t1 - t0).count();
    }
    if (!ok) return fail(QMG_ERR_NOCONV, "bicgstab: %d steps, relative residual %.3e", iters, final_rel);
    return QMG_OK;
}

}  // namespace

extern "C" void qmg_bicgstab_destroy(qmg_bicgstab h) {
    if (!h) return;
    for (void* p : {h->r, h->rt, h->p, h->v, h->s, h->t, h->xl, h->tmp_lo, h->xh, h->r64, h->b64, h->t64, h->tmp_hi,
                    (void*)h->dsc})
        if (p) (void)hipFree(p);
    if (h->hsc) (void)hipHostFree(h->hsc);
    h->blas.release();
    delete h;
}

extern "C" qmg_status qmg_bicgstab_create(qmg_fine_op hi, qmg_fine_op lo, int evenodd, void* stream,
                                          qmg_bicgstab* out) {
    if (!out) return fail(QMG_ERR_ARG, "bicgstab_create: out is NULL");
    *out = nullptr;
    if (!hi || !lo) return fail(QMG_ERR_ARG, "bicgstab_create: NULL operator");
    if (hi->storage != QMG_C128) return fail(QMG_ERR_PREC, "bicgstab_create: the reliable-update operator must be complex128");
    for (int m = 0; m < 4; ++m)
        if (hi->dims[m] != lo->dims[m]) return fail(QMG_ERR_SHAPE, "bicgstab_create: operators on different lattices");
    if (hi->m0 != lo->m0 || hi->csw != lo->csw || hi->antiperiodic_t != lo->antiperiodic_t)
        return fail(QMG_ERR_ARG, "bicgstab_create: the two operators differ in m0, c_sw or boundary");
    if (evenodd && (!hi->hsite || !lo->hsite))
        return fail(QMG_ERR_SHAPE, "bicgstab_create: the red-black form needs every extent even");
    auto* h = new qmg_bicgstab_s();
    h->hi = hi;
    h->lo = lo;
    h->eo = evenodd ? 1 : 0;
    h->st = as_stream(stream);
    h->lp = lo->storage == QMG_C128 ? QMG_C128 : QMG_C64;
    h->n = hi->V * 12 / (h->eo ? 2 : 1);
    const size_t vb = h->n * (h->lp == QMG_C128 ? 16 : 8), vb64 = h->n * 16, half_hi = hi->V / 2 * 12 * 16;
    h->blas.s = h->st;
    qmg_status st = h->blas.init();
    hipError_t e = hipSuccess;
    for (void** p : {&h->r, &h->rt, &h->p, &h->v, &h->xl})
        if (e == hipSuccess) e = hipMalloc(p, vb);
    // s and t double as whole-lattice FP64 scratch at the end of a red-black solve
    const size_t st_bytes = h->eo ? (vb > (size_t)hi->V * 12 * 16 ? vb : (size_t)hi->V * 12 * 16) : vb;
    if (e == hipSuccess) e = hipMalloc(&h->s, st_bytes);
    if (e == hipSuccess) e = hipMalloc(&h->t, st_bytes);
    for (void** p : {&h->xh, &h->r64, &h->b64, &h->t64})
        if (e == hipSuccess) e = hipMalloc(p, vb64);
    if (e == hipSuccess && h->eo) e = hipMalloc(&h->tmp_lo, vb);
    if (e == hipSuccess && h->eo) e = hipMalloc(&h->tmp_hi, half_hi);
    if (e == hipSuccess) e = hipMalloc(&h->dsc, sizeof(double) * B_N);
    if (e == hipSuccess) e = hipHostMalloc((void**)&h->hsc, sizeof(double) * B_N);
    if (st == QMG_OK && e != hipSuccess) st = fail(QMG_ERR_NOMEM, "bicgstab_create: %s", hipGetErrorString(e));
    if (st != QMG_OK) {
        qmg_bicgstab_destroy(h);
        return st;
    }
    *out = h;
    return QMG_OK;
}

extern "C" qmg_status qmg_bicgstab_solve(qmg_bicgstab h, const void* b, void* x, const qmg_bicgstab_params* p,
                                         qmg_solve_info* info, void* stream) {
    if (!h || !b || !x || !p) return fail(QMG_ERR_ARG, "bicgstab_solve: NULL argument");
    if (b == x) return fail(QMG_ERR_ARG, "bicgstab_solve: b and x alias");
    if (!(p->tol > 0) || p->maxit < 1 || !(p->delta > 0 && p->delta < 1))
        return fail(QMG_ERR_ARG, "bicgstab_solve: tol, maxit or delta invalid");
    h->st = as_stream(stream);
    h->blas.s = h->st;
    if (info) *info = qmg_solve_info{};
    return h->lp == QMG_C128 ? solve<double>(h, b, x, p, info) : solve<float>(h, b, x, p, info);
}
