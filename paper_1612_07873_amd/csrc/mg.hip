// Adaptive multigrid hierarchy and K-cycle GCR solver (Sec. 3.4 setup,
// Sec. 7.1 solver), driven from the host; every vector operation runs in the
// library's kernels and every solver scalar stays in device memory (the host
// only reads residual norms for the stopping tests).
//
// Setup, per level l below the coarsest: for k = 0..nvec-1 take the caller's
// random start, make it orthogonal to the earlier candidates, relax A x = 0 by
// GCR(10) for setup_iters steps from it, make the result orthogonal again and
// normalise it; then build P (transfer.hip) and Mhat = P^+ A P (galerkin.hip).
//
// Solve: flexible GCR(restart) on the fine level in FP64, preconditioned by
// the K-cycle K_0 run in the inner precision (FP32 or FP64):
//   K_l(r): z = MR_s(r); rc = R (r - A z); xc = GCR_{l+1}(rc) [preconditioned by
//           K_{l+1}, plain on the coarsest level]; z += P xc; z += MR_s(r - A z).
// Orthogonalisation in GCR is classical Gram-Schmidt done twice (equal to the
// modified Gram-Schmidt of the reference algorithm in exact arithmetic; two
// passes keep it as stable).  When the iterated residual reaches the
// tolerance, or after `restart` steps, the true residual b - A x is recomputed
// in FP64 (a reliable update) and the cycle restarts from it.
#include "blas.h"
#include "handles.h"

#include <chrono>
#include <cmath>
#include <vector>

struct qmg_mg_s;

namespace qmg {
qmg_status transfer_prolong(qmg_transfer t, const void* in, void* out, qmg_prec p, hipStream_t s);
qmg_status transfer_restrict(qmg_transfer t, const void* in, void* out, qmg_prec p, hipStream_t s);
qmg_status ptc_forward(qmg_ptc t, const void* r, void* y, hipStream_t s);
}

using namespace qmg;

namespace {

struct Level {
    int dims[4] = {0, 0, 0, 0};
    int64_t V = 0;
    int dof = 0;
    int64_t n = 0;                  // complex entries of a field on this level
    qmg_coarse_op op = nullptr;     // l >= 1 (inner precision)
    qmg_transfer T = nullptr;       // to level l+1
    qmg_level_params p{};           // parameters of this level (smoother, next-level solve)
    // GCR on this level
    void *Q = nullptr, *Z = nullptr, *r = nullptr, *x = nullptr, *b = nullptr, *t = nullptr;
    // K-cycle on this level
    void *mr_r = nullptr, *mr_Ar = nullptr, *kt = nullptr, *kr2 = nullptr, *kx2 = nullptr;
    void *kin = nullptr, *kout = nullptr;  // level 0 only: inner-precision copies
};

}  // namespace

struct qmg_mg_s {
    qmg_fine_op fine64 = nullptr, fine_in = nullptr;
    qmg_prec inner = QMG_C64;
    int restart = 10;
    std::vector<Level> lv;
    Blas blas;
    double* dsc = nullptr;   // device scalars
    double* hsc = nullptr;   // pinned host mirror
    // outer FP64 workspace (level 0)
    void *Q64 = nullptr, *Z64 = nullptr, *r64 = nullptr, *x64 = nullptr, *t64 = nullptr;
    std::vector<void*> allocs;
    hipStream_t s = nullptr;
    int level_iters[8] = {0};
    qmg_ptc ptc = nullptr;      // learned level-0 smoother (NULL: MR)
    int fallbacks = 0;          // smoother applications that fell back to MR
    void* rec = nullptr;        // recording of outer iterates (complex128 [maxrec][V][12])
    int rec_max = 0, rec_n = 0;
};

namespace {

constexpr int kScal = 64;  // device scalar slots
// slot map
constexpr int S_BETA = 0;     // 32 doubles (16 complex)
constexpr int S_GCR = 32;     // 3
constexpr int S_NRM = 36;     // 1
constexpr int S_MR = 40;      // 3
constexpr int S_BN = 44;      // 1
constexpr int S_SM = 48;      // 2: smoother residual norms

size_t cbytes(qmg_prec p) { return p == QMG_C128 ? 16 : 8; }

qmg_status alloc(qmg_mg_s* mg, void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return fail(QMG_ERR_NOMEM, "mg: allocation of %zu bytes: %s", bytes, hipGetErrorString(e));
    mg->allocs.push_back(*p);
    return QMG_OK;
}

template <typename R> qmg_status apply_op(qmg_mg_s* mg, int l, const void* in, void* out) {
    const qmg_prec p = sizeof(R) == 8 ? QMG_C128 : QMG_C64;
    if (l == 0) return qmg_wilson_clover_dslash(mg->fine_in, in, out, p, mg->s);
    return qmg_coarse_dslash(mg->lv[l].op, in, out, p, mg->s);
}

qmg_status read_scalars(qmg_mg_s* mg, int first, int count) {
    QMG_HIP(hipMemcpyAsync(mg->hsc + first, mg->dsc + first, sizeof(double) * count, hipMemcpyDeviceToHost, mg->s));
    QMG_HIP(hipStreamSynchronize(mg->s));
    return QMG_OK;
}

// classical Gram-Schmidt, two passes: q -= Q beta; z -= Z beta
template <typename R>
qmg_status orthogonalize(qmg_mg_s* mg, const void* Q, const void* Z, int64_t ld, int k, void* q, void* z, int64_t n) {
    for (int pass = 0; pass < 2; ++pass)
        for (int j0 = 0; j0 < k; j0 += 16) {
            const int kk = k - j0 < 16 ? k - j0 : 16;
            const size_t off = (size_t)j0 * ld * sizeof(cpx<R>);
            QMG_TRY(mg->blas.multi_dot<R>((const char*)Q + off, ld, kk, q, n, mg->dsc + S_BETA));
            QMG_TRY(mg->blas.multi_axpy<R>(mg->dsc + S_BETA, (const char*)Q + off,
                                           Z ? (const char*)Z + off : nullptr, ld, kk, q, z, n));
        }
    return QMG_OK;
}

template <typename R> qmg_status kcycle(qmg_mg_s* mg, int l, const void* rin, void* zout);

// x = MR_s(r) on level l; on exit lv.mr_r holds r - A x.
template <typename R> qmg_status mr(qmg_mg_s* mg, int l, const void* r, void* x) {
    Level& L = mg->lv[l];
    const int64_t n = L.n;
    for (int it = 0; it < L.p.smoother_steps; ++it) {
        const void* cur = it == 0 ? r : L.mr_r;   // the first step reads r itself
        QMG_TRY(apply_op<R>(mg, l, cur, L.mr_Ar));
        QMG_TRY(mg->blas.dot_norm<R>(L.mr_Ar, cur, n, mg->dsc + S_MR));
        QMG_TRY(mg->blas.mr_update<R>(mg->dsc + S_MR, cur, L.mr_r, L.mr_Ar, x, it == 0, n));
    }
    if (L.p.smoother_steps <= 0) {
        QMG_HIP(hipMemsetAsync(x, 0, n * sizeof(cpx<R>), mg->s));
        QMG_HIP(hipMemcpyAsync(L.mr_r, r, n * sizeof(cpx<R>), hipMemcpyDeviceToDevice, mg->s));
    }
    return QMG_OK;
}

// GCR on level l (l >= 1 uses the level's op; l == 0 with inner precision is
// used by the setup).  Solves A x = b from x (if x0) or from 0.
template <typename R>
qmg_status gcr(qmg_mg_s* mg, int l, const void* b, void* x, bool x0, double tol, int maxit, bool precond,
               int* iters_out) {
    Level& L = mg->lv[l];
    const int64_t n = L.n;
    const int m = mg->restart;
    const size_t vb = n * sizeof(cpx<R>);
    double bnorm;
    QMG_TRY(mg->blas.norm2<R>(b, n, mg->dsc + S_BN));
    QMG_TRY(read_scalars(mg, S_BN, 1));
    bnorm = std::sqrt(mg->hsc[S_BN]);
    if (x0) {
        QMG_TRY(apply_op<R>(mg, l, x, L.t));
        QMG_TRY(mg->blas.xmy<R>(b, L.t, L.r, n));
    } else {
        QMG_HIP(hipMemsetAsync(x, 0, vb, mg->s));
        QMG_HIP(hipMemcpyAsync(L.r, b, vb, hipMemcpyDeviceToDevice, mg->s));
    }
    const double target = tol * bnorm;
    int iters = 0;
    bool done = false;
    // short unpreconditioned systems (the coarsest level): the whole step's
    // vector work is one single-work-group kernel, so a step is two launches
    const bool small = !precond && n <= Blas::kSmall;
    while (!done && iters < maxit) {
        int j = 0;
        if (small) QMG_HIP(hipMemcpyAsync(L.Z, L.r, vb, hipMemcpyDeviceToDevice, mg->s));
        for (; j < m && iters < maxit; ++j) {
            void* z = (char*)L.Z + j * vb;
            void* q = (char*)L.Q + j * vb;
            if (small) {
                QMG_TRY(apply_op<R>(mg, l, z, q));
                void* znext = j + 1 < m ? (char*)L.Z + (j + 1) * vb : nullptr;
                QMG_TRY(mg->blas.gcr_step_small<R>(L.Q, L.Z, n, j, q, z, x, L.r, n, mg->dsc + S_GCR, znext));
                QMG_TRY(read_scalars(mg, S_GCR, 4));
                ++iters;
                const double rn = std::sqrt(mg->hsc[S_GCR + 3]);
                if (!std::isfinite(rn) || !std::isfinite(mg->hsc[S_GCR]))
                    return fail(QMG_ERR_NONFINITE, "gcr on level %d: non-finite residual after %d steps", l, iters);
                if (mg->hsc[S_GCR] <= 0.0) { done = true; ++j; break; }
                if (bnorm > 0 && rn <= target) { done = true; ++j; break; }
                continue;
            }
            if (precond) QMG_TRY(kcycle<R>(mg, l, L.r, z));
            else QMG_HIP(hipMemcpyAsync(z, L.r, vb, hipMemcpyDeviceToDevice, mg->s));
            QMG_TRY(apply_op<R>(mg, l, z, q));
            QMG_TRY(orthogonalize<R>(mg, L.Q, L.Z, n, j, q, z, n));
            QMG_TRY(mg->blas.dot_norm<R>(q, L.r, n, mg->dsc + S_GCR));
            QMG_TRY(mg->blas.gcr_update<R>(mg->dsc + S_GCR, q, z, x, L.r, n));
            QMG_TRY(mg->blas.norm2<R>(L.r, n, mg->dsc + S_NRM));
            QMG_TRY(read_scalars(mg, S_GCR, 5));
            ++iters;
            const double rn = std::sqrt(mg->hsc[S_NRM]);
            if (!std::isfinite(rn) || !std::isfinite(mg->hsc[S_GCR]))
                return fail(QMG_ERR_NONFINITE, "gcr on level %d: non-finite residual after %d steps", l, iters);
            if (mg->hsc[S_GCR] <= 0.0) { done = true; ++j; break; }  // breakdown: q = 0
            if (bnorm > 0 && rn <= target) { done = true; ++j; break; }
        }
        if (done || iters >= maxit) break;
        // restart from the true residual
        QMG_TRY(apply_op<R>(mg, l, x, L.t));
        QMG_TRY(mg->blas.xmy<R>(b, L.t, L.r, n));
    }
    if (iters_out) *iters_out += iters;
    return QMG_OK;
}

// Level smoother: MR, or on level 0 the learned network when one is attached.
// The network's result is kept only if it reduces the residual; otherwise
// (including NaN/Inf from bad weights) MR is used for this application.
// On exit lv.mr_r holds r - A x.
template <typename R> qmg_status smooth(qmg_mg_s* mg, int l, const void* r, void* x) {
    Level& L = mg->lv[l];
    if (l == 0 && mg->ptc && sizeof(R) == 4) {
        QMG_TRY(ptc_forward(mg->ptc, r, x, mg->s));
        QMG_TRY(apply_op<R>(mg, 0, x, L.mr_Ar));
        QMG_TRY(mg->blas.xmy<R>(r, L.mr_Ar, L.mr_r, L.n));
        QMG_TRY(mg->blas.norm2<R>(r, L.n, mg->dsc + S_SM));
        QMG_TRY(mg->blas.norm2<R>(L.mr_r, L.n, mg->dsc + S_SM + 1));
        QMG_TRY(read_scalars(mg, S_SM, 2));
        if (mg->hsc[S_SM + 1] < mg->hsc[S_SM]) return QMG_OK;
        ++mg->fallbacks;
    }
    return mr<R>(mg, l, r, x);
}

template <typename R> qmg_status kcycle(qmg_mg_s* mg, int l, const void* rin, void* zout) {
    Level& L = mg->lv[l];
    Level& C = mg->lv[l + 1];
    const int64_t n = L.n;
    const qmg_prec p = sizeof(R) == 8 ? QMG_C128 : QMG_C64;
    const int nl = (int)mg->lv.size();
    // pre-smoothing; L.mr_r = rin - A zout afterwards
    QMG_TRY(smooth<R>(mg, l, rin, zout));
    QMG_TRY(transfer_restrict(L.T, L.mr_r, C.b, p, mg->s));
    const bool coarsest = (l + 1 == nl - 1);
    int it = 0;
    QMG_TRY(gcr<R>(mg, l + 1, C.b, C.x, false, L.p.coarse_tol, L.p.coarse_maxit, !coarsest, &it));
    mg->level_iters[l + 1] += it;
    QMG_TRY(transfer_prolong(L.T, C.x, L.kt, p, mg->s));
    QMG_TRY(mg->blas.axpy<R>(1.0, L.kt, zout, n));
    // post-smoothing on r - A z
    QMG_TRY(apply_op<R>(mg, l, zout, L.kt));
    QMG_TRY(mg->blas.xmy<R>(rin, L.kt, L.kr2, n));
    QMG_TRY(smooth<R>(mg, l, L.kr2, L.kx2));
    QMG_TRY(mg->blas.axpy<R>(1.0, L.kx2, zout, n));
    return QMG_OK;
}

template <typename R> qmg_status level_buffers(qmg_mg_s* mg, int l) {
    Level& L = mg->lv[l];
    const size_t vb = L.n * sizeof(cpx<R>);
    void** one[] = {&L.r, &L.x, &L.b, &L.t, &L.mr_r, &L.mr_Ar, &L.kt, &L.kr2, &L.kx2, &L.kin, &L.kout};
    for (void** p : one) QMG_TRY(alloc(mg, p, vb));
    QMG_TRY(alloc(mg, &L.Q, vb * mg->restart));
    QMG_TRY(alloc(mg, &L.Z, vb * mg->restart));
    return QMG_OK;
}

// near-null vectors of level l -> transfer and next coarse operator
template <typename R>
qmg_status setup_level(qmg_mg_s* mg, int l, const void* starts, int setup_iters) {
    Level& L = mg->lv[l];
    const int nvec = L.p.nvec;
    const int64_t n = L.n;
    const size_t vb = n * sizeof(cpx<R>);
    void* NV = nullptr;
    void* NV64 = nullptr;
    hipError_t e = hipMalloc(&NV, vb * nvec);
    if (e == hipSuccess) e = hipMalloc(&NV64, n * 16 * nvec);
    if (e != hipSuccess) {
        if (NV) (void)hipFree(NV);
        return fail(QMG_ERR_NOMEM, "mg setup: %s", hipGetErrorString(e));
    }
    qmg_status st = QMG_OK;
    for (int k = 0; k < nvec && st == QMG_OK; ++k) {
        void* v = (char*)NV + k * vb;
        st = mg->blas.convert<double, R>((const char*)starts + (size_t)k * n * 16, v, n);
        if (st == QMG_OK) st = orthogonalize<R>(mg, NV, nullptr, n, k, v, nullptr, n);
        if (st == QMG_OK && setup_iters > 0) {
            // relax A x = 0 from x = v: b = 0
            st = hipMemsetAsync(L.b, 0, vb, mg->s) == hipSuccess ? QMG_OK : fail(QMG_ERR_HIP, "memset");
            if (st == QMG_OK) st = gcr<R>(mg, l, L.b, v, true, 0.0, setup_iters, false, nullptr);
            if (st == QMG_OK) st = orthogonalize<R>(mg, NV, nullptr, n, k, v, nullptr, n);
        }
        if (st == QMG_OK) st = mg->blas.norm2<R>(v, n, mg->dsc + S_NRM);
        if (st == QMG_OK) st = mg->blas.normalize<R>(v, mg->dsc + S_NRM, n);
    }
    if (st == QMG_OK) st = mg->blas.convert<R, double>(NV, NV64, n * nvec);
    if (st == QMG_OK)
        st = qmg_transfer_create(L.dims, L.dof, L.p.block, nvec, NV64, mg->inner, mg->s, &L.T);
    if (st == QMG_OK) {
        Level& C = mg->lv[l + 1];
        if (l == 0) st = qmg_build_coarse_op(L.T, mg->fine64, nullptr, mg->inner, mg->s, &C.op);
        else st = qmg_build_coarse_op(L.T, nullptr, L.op, mg->inner, mg->s, &C.op);
    }
    (void)hipStreamSynchronize(mg->s);
    (void)hipFree(NV);
    (void)hipFree(NV64);
    return st;
}

template <typename R>
qmg_status solve_impl(qmg_mg_s* mg, const void* b, void* x, const qmg_solve_params* sp, qmg_solve_info* info) {
    Level& L0 = mg->lv[0];
    const int64_t n = L0.n;
    const size_t vb64 = n * 16;
    const int m = mg->restart;
    const int nl = (int)mg->lv.size();
    for (int i = 0; i < 8; ++i) mg->level_iters[i] = 0;
    mg->fallbacks = 0;
    mg->rec_n = 0;
    auto t0 = std::chrono::steady_clock::now();
    QMG_TRY(mg->blas.norm2<double>(b, n, mg->dsc + S_BN));
    QMG_TRY(read_scalars(mg, S_BN, 1));
    const double bnorm = std::sqrt(mg->hsc[S_BN]);
    QMG_HIP(hipMemsetAsync(x, 0, vb64, mg->s));
    QMG_HIP(hipMemcpyAsync(mg->r64, b, vb64, hipMemcpyDeviceToDevice, mg->s));
    const double target = sp->tol * bnorm;
    int iters = 0, restarts = 0;
    double true_rel = bnorm > 0 ? 1.0 : 0.0;
    bool converged = bnorm == 0.0;
    while (!converged && iters < sp->maxit) {
        for (int j = 0; j < m && iters < sp->maxit; ++j) {
            void* z = (char*)mg->Z64 + j * vb64;
            void* q = (char*)mg->Q64 + j * vb64;
            if (nl > 1) {
                QMG_TRY(mg->blas.convert<double, R>(mg->r64, L0.kin, n));
                QMG_TRY(kcycle<R>(mg, 0, L0.kin, L0.kout));
                QMG_TRY(mg->blas.convert<R, double>(L0.kout, z, n));
            } else {
                QMG_HIP(hipMemcpyAsync(z, mg->r64, vb64, hipMemcpyDeviceToDevice, mg->s));
            }
            QMG_TRY(qmg_wilson_clover_dslash(mg->fine64, z, q, QMG_C128, mg->s));
            QMG_TRY(orthogonalize<double>(mg, mg->Q64, mg->Z64, n, j, q, z, n));
            QMG_TRY(mg->blas.dot_norm<double>(q, mg->r64, n, mg->dsc + S_GCR));
            QMG_TRY(mg->blas.gcr_update<double>(mg->dsc + S_GCR, q, z, x, mg->r64, n));
            QMG_TRY(mg->blas.norm2<double>(mg->r64, n, mg->dsc + S_NRM));
            QMG_TRY(read_scalars(mg, S_GCR, 5));
            ++iters;
            if (mg->rec && mg->rec_n < mg->rec_max) {
                QMG_HIP(hipMemcpyAsync((char*)mg->rec + (size_t)mg->rec_n * vb64, x, vb64, hipMemcpyDeviceToDevice, mg->s));
                ++mg->rec_n;
            }
            const double rn = std::sqrt(mg->hsc[S_NRM]);
            if (!std::isfinite(rn)) return fail(QMG_ERR_NONFINITE, "mg_gcr_solve: non-finite residual at step %d", iters);
            if (rn <= target || mg->hsc[S_GCR] <= 0.0) break;
        }
        // reliable update: true residual in FP64
        QMG_TRY(qmg_wilson_clover_dslash(mg->fine64, x, mg->t64, QMG_C128, mg->s));
        QMG_TRY(mg->blas.xmy<double>(b, mg->t64, mg->r64, n));
        QMG_TRY(mg->blas.norm2<double>(mg->r64, n, mg->dsc + S_NRM));
        QMG_TRY(read_scalars(mg, S_NRM, 1));
        const double tr = std::sqrt(mg->hsc[S_NRM]);
        true_rel = tr / bnorm;
        if (!std::isfinite(tr)) return fail(QMG_ERR_NONFINITE, "mg_gcr_solve: non-finite true residual");
        if (tr <= target) converged = true;
        else ++restarts;
    }
    auto t1 = std::chrono::steady_clock::now();
    if (info) {
        info->outer_iters = iters;
        for (int l = 0; l < 4; ++l) info->level_iters[l] = l < nl ? mg->level_iters[l] : 0;
        info->level_iters[0] = iters;
        info->restarts = restarts;
        info->true_rel_residual = true_rel;
        info->seconds = std::chrono::duration<double>(t1 - t0).count();
        info->converged = converged ? 1 : 0;
        info->smoother_fallbacks = mg->fallbacks;
    }
    if (!converged) return fail(QMG_ERR_NOCONV, "mg_gcr_solve: %d steps, relative residual %.3e", iters, true_rel);
    return QMG_OK;
}

}  // namespace

extern "C" void qmg_mg_destroy(qmg_mg mg) {
    if (!mg) return;
    for (auto& L : mg->lv) {
        if (L.op) qmg_coarse_op_destroy(L.op);
        if (L.T) qmg_transfer_destroy(L.T);
    }
    if (mg->fine64) qmg_fine_op_destroy(mg->fine64);
    if (mg->fine_in && mg->fine_in != mg->fine64) qmg_fine_op_destroy(mg->fine_in);
    for (void* p : mg->allocs) (void)hipFree(p);
    if (mg->hsc) (void)hipHostFree(mg->hsc);
    mg->blas.release();
    delete mg;
}

extern "C" qmg_status qmg_mg_create(const int dims[4], const void* gauge, double m0, double csw,
                                    int antiperiodic_t, int nlevels, const qmg_level_params* lp,
                                    const void* const* starts, qmg_prec inner, void* stream, qmg_mg* out) {
    if (!out) return fail(QMG_ERR_ARG, "mg_create: out is NULL");
    *out = nullptr;
    QMG_TRY(check_dims(dims, 2, "mg_create"));
    if (!gauge) return fail(QMG_ERR_ARG, "mg_create: gauge is NULL");
    if (nlevels < 1 || nlevels > 4) return fail(QMG_ERR_ARG, "mg_create: nlevels %d outside [1,4]", nlevels);
    if (nlevels > 1 && (!lp || !starts)) return fail(QMG_ERR_ARG, "mg_create: level params / starts missing");
    if (inner != QMG_C128 && inner != QMG_C64) return fail(QMG_ERR_PREC, "mg_create: inner precision %d", (int)inner);
    for (int l = 0; l + 1 < nlevels; ++l) {
        if (!starts[l]) return fail(QMG_ERR_ARG, "mg_create: starts[%d] is NULL", l);
        if (lp[l].nvec < 1 || lp[l].nvec > 64) return fail(QMG_ERR_ARG, "mg_create: nvec %d", lp[l].nvec);
        if (lp[l].smoother_steps < 0 || lp[l].coarse_maxit < 1 || lp[l].setup_iters < 0)
            return fail(QMG_ERR_ARG, "mg_create: bad level %d parameters", l);
    }
    auto* mg = new qmg_mg_s();
    mg->s = as_stream(stream);
    mg->inner = inner;
    mg->blas.s = mg->s;
    qmg_status st = mg->blas.init();
    if (st == QMG_OK && hipHostMalloc((void**)&mg->hsc, sizeof(double) * kScal) != hipSuccess)
        st = fail(QMG_ERR_NOMEM, "mg_create: pinned scalars");
    if (st == QMG_OK) st = alloc(mg, (void**)&mg->dsc, sizeof(double) * kScal);
    if (st == QMG_OK) st = qmg_fine_op_create(dims, gauge, m0, csw, antiperiodic_t, QMG_C128, stream, &mg->fine64);
    if (st == QMG_OK) {
        if (inner == QMG_C128) mg->fine_in = mg->fine64;
        else st = qmg_fine_op_create(dims, gauge, m0, csw, antiperiodic_t, QMG_C64, stream, &mg->fine_in);
    }
    if (st != QMG_OK) {
        qmg_mg_destroy(mg);
        return st;
    }
    mg->lv.resize(nlevels);
    int cur[4] = {dims[0], dims[1], dims[2], dims[3]};
    int dof = 12;
    for (int l = 0; l < nlevels && st == QMG_OK; ++l) {
        Level& L = mg->lv[l];
        for (int k = 0; k < 4; ++k) L.dims[k] = cur[k];
        L.V = volume(cur);
        L.dof = dof;
        L.n = L.V * dof;
        if (l + 1 < nlevels) {
            L.p = lp[l];
            for (int k = 0; k < 4; ++k) {
                if (L.p.block[k] < 1 || cur[k] % L.p.block[k] || cur[k] / L.p.block[k] < 2)
                    st = fail(QMG_ERR_SHAPE, "mg_create: level %d block does not fit the lattice", l);
                cur[k] = L.p.block[k] ? cur[k] / L.p.block[k] : 0;
            }
            dof = 2 * L.p.nvec;
        }
        if (st == QMG_OK) st = inner == QMG_C128 ? level_buffers<double>(mg, l) : level_buffers<float>(mg, l);
    }
    const size_t vb64 = mg->lv[0].n * 16;
    if (st == QMG_OK) st = alloc(mg, &mg->Q64, vb64 * mg->restart);
    if (st == QMG_OK) st = alloc(mg, &mg->Z64, vb64 * mg->restart);
    if (st == QMG_OK) st = alloc(mg, &mg->r64, vb64);
    if (st == QMG_OK) st = alloc(mg, &mg->t64, vb64);
    for (int l = 0; l + 1 < nlevels && st == QMG_OK; ++l)
        st = inner == QMG_C128 ? setup_level<double>(mg, l, starts[l], lp[l].setup_iters)
                               : setup_level<float>(mg, l, starts[l], lp[l].setup_iters);
    if (st != QMG_OK) {
        qmg_mg_destroy(mg);
        return st;
    }
    *out = mg;
    return QMG_OK;
}

extern "C" qmg_status qmg_mg_gcr_solve(qmg_mg mg, const void* b, void* x, const qmg_solve_params* p,
                                       qmg_solve_info* info, void* stream) {
    if (!mg || !b || !x || !p) return fail(QMG_ERR_ARG, "mg_gcr_solve: NULL argument");
    if (b == x) return fail(QMG_ERR_ARG, "mg_gcr_solve: b and x alias");
    if (!(p->tol > 0) || p->maxit < 1) return fail(QMG_ERR_ARG, "mg_gcr_solve: tol/maxit invalid");
    if (p->restart != 0 && p->restart != mg->restart)
        return fail(QMG_ERR_ARG, "mg_gcr_solve: restart must be 0 or %d", mg->restart);
    mg->s = as_stream(stream);
    mg->blas.s = mg->s;
    if (info) *info = qmg_solve_info{};
    if (mg->inner == QMG_C128) return solve_impl<double>(mg, b, x, p, info);
    return solve_impl<float>(mg, b, x, p, info);
}

extern "C" qmg_status qmg_mg_level(qmg_mg mg, int level, int dims[4], int* dof, qmg_coarse_op* op,
                                   qmg_transfer* to_next) {
    if (!mg || !dims || !dof) return fail(QMG_ERR_ARG, "mg_level: NULL argument");
    if (level < 0 || level >= (int)mg->lv.size()) return fail(QMG_ERR_ARG, "mg_level: level %d out of range", level);
    const Level& L = mg->lv[level];
    for (int k = 0; k < 4; ++k) dims[k] = L.dims[k];
    *dof = L.dof;
    if (op) *op = L.op;
    if (to_next) *to_next = L.T;
    return QMG_OK;
}

extern "C" qmg_status qmg_mg_fine_op(qmg_mg mg, qmg_fine_op* fine64) {
    if (!mg || !fine64) return fail(QMG_ERR_ARG, "mg_fine_op: NULL argument");
    *fine64 = mg->fine64;
    return QMG_OK;
}

extern "C" qmg_status qmg_mg_set_smoother(qmg_mg mg, qmg_ptc net) {
    if (!mg) return fail(QMG_ERR_ARG, "mg_set_smoother: NULL mg");
    if (net) {
        if (mg->inner != QMG_C64) return fail(QMG_ERR_PREC, "mg_set_smoother: the learned smoother runs in complex64");
        if (net->V != mg->lv[0].V) return fail(QMG_ERR_SHAPE, "mg_set_smoother: network lattice does not match");
        if (mg->lv.size() < 2) return fail(QMG_ERR_STATE, "mg_set_smoother: a single-level solver has no smoother");
    }
    mg->ptc = net;
    return QMG_OK;
}

extern "C" qmg_status qmg_mg_gcr_solve_record(qmg_mg mg, const void* b, void* x, const qmg_solve_params* p,
                                              qmg_solve_info* info, void* xhist, int maxrec, int* nrec,
                                              void* stream) {
    if (!xhist || maxrec < 1 || !nrec) return fail(QMG_ERR_ARG, "mg_gcr_solve_record: bad record buffer");
    if (!mg) return fail(QMG_ERR_ARG, "mg_gcr_solve_record: NULL mg");
    mg->rec = xhist;
    mg->rec_max = maxrec;
    const qmg_status st = qmg_mg_gcr_solve(mg, b, x, p, info, stream);
    *nrec = mg->rec_n;
    mg->rec = nullptr;
    mg->rec_max = 0;
    return st;
}

namespace {
// e = x* - x_k in FP64, stored as complex64
__global__ void k_pair_error(const double2* __restrict__ xs, const double2* __restrict__ xk, double2* __restrict__ e64,
                             float2* __restrict__ e32, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 d = make_double2(xs[i].x - xk[i].x, xs[i].y - xk[i].y);
    e64[i] = d;
    e32[i] = make_float2((float)d.x, (float)d.y);
}
__global__ void k_to32(const double2* __restrict__ a, float2* __restrict__ b, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = make_float2((float)a[i].x, (float)a[i].y);
}
}  // namespace

extern "C" qmg_status qmg_mg_make_pairs(qmg_mg mg, const void* xstar, const void* xhist, int n, void* r_out,
                                        void* e_out, void* stream) {
    if (!mg || !xstar || !xhist || !r_out || !e_out || n < 1) return fail(QMG_ERR_ARG, "mg_make_pairs: bad argument");
    hipStream_t s = as_stream(stream);
    const int64_t nv = mg->lv[0].n;
    const unsigned g = (unsigned)((nv + 255) / 256);
    for (int k = 0; k < n; ++k) {
        const double2* xk = (const double2*)xhist + (size_t)k * nv;
        float2* e32 = (float2*)e_out + (size_t)k * nv;
        float2* r32 = (float2*)r_out + (size_t)k * nv;
        hipLaunchKernelGGL(k_pair_error, dim3(g), dim3(256), 0, s, (const double2*)xstar, xk, (double2*)mg->t64, e32, nv);
        QMG_LAUNCH_CHECK();
        QMG_TRY(qmg_wilson_clover_dslash(mg->fine64, mg->t64, mg->r64, QMG_C128, stream));
        hipLaunchKernelGGL(k_to32, dim3(g), dim3(256), 0, s, (const double2*)mg->r64, r32, nv);
        QMG_LAUNCH_CHECK();
    }
    return QMG_OK;
}
