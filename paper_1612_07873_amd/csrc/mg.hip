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
//
// Several right-hand sides are solved together as a batch of nb members run
// in lock step: every field of the batch is [member][site][component], each
// kernel launch covers all members (grid dimension y), each member keeps its
// own scalars (its own Krylov space, step lengths and stopping test), and a
// level's GCR stops when every member has reached its tolerance.  With a
// 16-bit coarse operator and 8, 16, 32 or 64 members the coarse stencil runs
// as one multi-right-hand-side matrix-core product.
#include "blas.h"
#include "handles.h"

#include <chrono>
#include <cmath>
#include <complex>
#include <vector>

struct qmg_mg_s;

namespace qmg {
qmg_status transfer_prolong(qmg_transfer t, const void* in, void* out, qmg_prec p, int nb, hipStream_t s);
qmg_status transfer_restrict(qmg_transfer t, const void* in, void* out, qmg_prec p, int nb, hipStream_t s);
qmg_status ptc_forward(qmg_ptc t, const void* r, void* y, hipStream_t s);
qmg_status wilson_apply(const qmg_fine_op_s* op, const void* in, void* out, qmg_prec vprec, int members,
                        hipStream_t s);
qmg_status wilson_apply_dot(const qmg_fine_op_s* op, const void* in, void* out, qmg_prec vprec, int members,
                            double* part, int64_t pmember, int pvalue, hipStream_t s);
int wilson_groups(const qmg_fine_op_s* op);
qmg_status coarse_apply(qmg_coarse_op_s* op, const void* in, void* out, qmg_prec vprec, int m, void* q16,
                        float* qsc, hipStream_t s);
bool coarse_batch_uses_mfma(const qmg_coarse_op_s* op, int m);
qmg_status dense_inverse(qmg_coarse_op_s* op, qmg_prec prec, void** out, hipStream_t s);
qmg_status dense_apply(const void* Ainv, const void* b, void* y, int64_t n, int nb, qmg_prec prec, hipStream_t s);
qmg_status fine_schur_apply16(const qmg_fine_op_s* op, const void* in_e, const float* in_s, void* out_e, float* out_s,
                              void* tmp_o, float* tmp_s, int m, hipStream_t s);
qmg_status fine_schur_apply(const qmg_fine_op_s* op, const void* in_e, void* out_e, void* tmp_o, qmg_prec vprec,
                            int m, hipStream_t s);
qmg_status fine_schur_source(const qmg_fine_op_s* op, const void* b, void* bhat_e, void* tmp_o, qmg_prec vprec,
                             int m, hipStream_t s);
qmg_status fine_schur_reconstruct(const qmg_fine_op_s* op, const void* x_e, const void* b, void* x, qmg_prec vprec,
                                  int m, hipStream_t s);
qmg_status coarse_schur_apply(const qmg_coarse_op_s* op, const void* in_e, void* out_e, void* tmp_o, qmg_prec vprec,
                              int m, hipStream_t s);
qmg_status coarse_schur_source(const qmg_coarse_op_s* op, const void* b, void* bhat_e, void* tmp_o, qmg_prec vprec,
                               int m, hipStream_t s);
qmg_status coarse_schur_reconstruct(const qmg_coarse_op_s* op, const void* x_e, const void* b, void* x,
                                    qmg_prec vprec, int m, hipStream_t s);
qmg_status coarse_schur_build(qmg_coarse_op_s* op, const void* Xc, const void* Yc, qmg_prec storage, hipStream_t s);
qmg_status eo_gather(const int* hsite, int64_t Vh, int dof, const void* full, void* half, bool sub, qmg_prec vprec,
                     int m, hipStream_t s);
qmg_status eo_scatter(const int* hsite_p, const int* hsite_q, int64_t Vh, int dof, const void* half, void* full,
                      qmg_prec vprec, int m, hipStream_t s);
struct SapPlan;
qmg_status sap_plan_create(const qmg_fine_op_s* op, const int block[4], SapPlan** out, hipStream_t s);
void sap_plan_destroy(SapPlan* P);
qmg_status sap_sweep(const qmg_fine_op_s* op, const SapPlan& P, const void* r, void* x, int iters, int m,
                     hipStream_t s);
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
    void* Ainv = nullptr;           // coarsest level solved exactly: dense inverse [n][n] (inner precision)
    void* Sdense = nullptr;         // coarsest level, red-black: its Schur operator as a dense [n/2][n/2] matrix
    void* q16 = nullptr;            // batched 16-bit stencil input [V][nb][N] (multi-RHS matrix-core path)
    float* qsc = nullptr;           // its scales [V][nb]
    // red-black form: half-lattice fields (n/2 entries per member)
    void *eb = nullptr, *ex = nullptr, *er = nullptr, *et = nullptr;   // GCR on the Schur system
    void *eQ = nullptr, *eZ = nullptr;                                 // its Krylov directions
    void *sb = nullptr, *sx = nullptr, *sr = nullptr, *sAr = nullptr;  // Schur MR smoother
    void *etmp = nullptr;   // odd half-lattice scratch of the Schur operator
    void *ekin = nullptr;   // level 0: inner-precision half field of the outer solve
    int small_steps[2] = {0, 0};   // steps of the last single-work-group GCR solve (whole, Schur system)
    // level 0, red-black, 16-bit smoother vectors: the Schur system's source,
    // residual, odd intermediate and A r as FP16 pairs [site][12] with scales
    void *hb = nullptr, *hr = nullptr, *ht = nullptr, *hAr = nullptr;
    float *hbs = nullptr, *hrs = nullptr, *hts = nullptr, *hArs = nullptr;
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
    void *Q64 = nullptr, *Z64 = nullptr, *r64 = nullptr, *t64 = nullptr;
    std::vector<void*> allocs;   // setup-time and lifetime allocations
    std::vector<void*> sallocs;  // solve workspace, sized for `cap` batch members
    int cap = 0;                 // batch members the solve workspace holds
    int nb = 1;                  // members of the running solve
    hipStream_t s = nullptr;
    int level_iters[8] = {0};
    qmg_ptc ptc = nullptr;      // learned level-0 smoother (NULL: MR)
    int ptc_mr = 0;             // MR steps after an accepted network step
    int fallbacks = 0;          // smoother applications that fell back to MR
    void* rec = nullptr;        // recording of outer iterates (complex128 [maxrec][V][12])
    int rec_max = 0, rec_n = 0;
    void* srec = nullptr;       // recording of level-0 smoother inputs (complex64 [maxrec][V][12])
    int srec_max = 0, srec_n = 0;
    bool eo = false;            // red-black form on every level
    bool smooth16 = false;      // level-0 MR on the Schur system with 16-bit vectors (red-black form)
    void *eb64 = nullptr, *ex64 = nullptr, *etmp64 = nullptr;   // outer FP64 Schur source, iterate, scratch
    // per-level timing (qmg_mg_set_level_timing): HIP events around every
    // coarse-grid solve, read after the solve
    SapPlan* sap = nullptr;     // level-0 Schwarz smoother (NULL: MR)
    int sap_iters = 0;
    bool timing = false;
    std::vector<hipEvent_t> ev;           // pool, created on first use
    std::vector<int> span_level;          // level of span k: events 2k, 2k+1
    bool spans_overflow = false;
};

namespace {

constexpr int kScal = 64;  // device scalar slots per batch member (member b at b*kScal)

// the n x n identity, [n][n]
template <typename R> __global__ void k_identity(cpx<R>* __restrict__ m, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * n) return;
    m[i] = cpx<R>{(i / n == i % n) ? R(1) : R(0), R(0)};
}
// out[i][j] = in[j][i], n x n
template <typename R> __global__ void k_transpose(cpx<R>* __restrict__ out, const cpx<R>* __restrict__ in, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * n) return;
    out[i] = in[(i % n) * n + i / n];
}
// slot map
constexpr int S_BETA = 0;     // 32 doubles (16 complex)
constexpr int S_GCR = 32;     // 3
constexpr int S_NRM = 36;     // 1
constexpr int S_MR = 40;      // 3
constexpr int S_BN = 44;      // 4: |b|^2 of the GCR on level l in slot S_BN + l (nested solves keep theirs)
constexpr int S_SM = 48;      // 3: learned-smoother step scalars
constexpr int S_OK = 52;      // 3: single-work-group GCR steps: stopping-test flags (two parities), steps done
constexpr int S_QQ = 56;      // 1: outer GCR: |q|^2 before the projection
constexpr int S_FB = 57;      // 1: network steps refused on the device (learned smoother followed by MR)
constexpr int kCheck = 4;     // such steps queued before the first host read of the scalars (at least)
constexpr int kRecheck = 2;   // and between later reads

size_t cbytes(qmg_prec p) { return p == QMG_C128 ? 16 : 8; }

qmg_status alloc(qmg_mg_s* mg, void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return fail(QMG_ERR_NOMEM, "mg: allocation of %zu bytes: %s", bytes, hipGetErrorString(e));
    mg->allocs.push_back(*p);
    return QMG_OK;
}

qmg_status salloc(qmg_mg_s* mg, void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return fail(QMG_ERR_NOMEM, "mg: workspace of %zu bytes: %s", bytes, hipGetErrorString(e));
    mg->sallocs.push_back(*p);
    return QMG_OK;
}

// scalar slot `slot` of batch member b (host mirror)
inline double& hs(qmg_mg_s* mg, int b, int slot) { return mg->hsc[(size_t)b * kScal + slot]; }

template <typename R> qmg_status apply_op(qmg_mg_s* mg, int l, const void* in, void* out) {
    const qmg_prec p = sizeof(R) == 8 ? QMG_C128 : QMG_C64;
    if (l == 0) return wilson_apply(mg->fine_in, in, out, p, mg->nb, mg->s);
    Level& L = mg->lv[l];
    return coarse_apply(L.op, in, out, p, mg->nb, L.q16, L.qsc, mg->s);
}

// ---------------------------------------------------------------- red-black form
// On level l the Schur complement S of the level's operator acts on the even
// half of the lattice (Sec. 3.3): fine level C_ee - D_eo C_oo^-1 D_oe
// (wilson.hip), coarse levels X_ee - Y_eo X_oo^-1 Y_oe (evenodd.hip).
const int* level_hsite(qmg_mg_s* mg, int l) { return l == 0 ? mg->fine_in->hsite : mg->lv[l].op->hsite; }

template <typename R> qmg_status schur_apply(qmg_mg_s* mg, int l, const void* in_e, void* out_e) {
    const qmg_prec p = sizeof(R) == 8 ? QMG_C128 : QMG_C64;
    Level& L = mg->lv[l];
    if (l == 0) return fine_schur_apply(mg->fine_in, in_e, out_e, L.etmp, p, mg->nb, mg->s);
    if (L.Sdense) return dense_apply(L.Sdense, in_e, out_e, L.n / 2, mg->nb, p, mg->s);
    return coarse_schur_apply(L.op, in_e, out_e, L.etmp, p, mg->nb, mg->s);
}
template <typename R> qmg_status schur_source(qmg_mg_s* mg, int l, const void* b, void* bhat_e) {
    const qmg_prec p = sizeof(R) == 8 ? QMG_C128 : QMG_C64;
    Level& L = mg->lv[l];
    if (l == 0) return fine_schur_source(mg->fine_in, b, bhat_e, L.etmp, p, mg->nb, mg->s);
    return coarse_schur_source(L.op, b, bhat_e, L.etmp, p, mg->nb, mg->s);
}
template <typename R> qmg_status schur_reconstruct(qmg_mg_s* mg, int l, const void* x_e, const void* b, void* x) {
    const qmg_prec p = sizeof(R) == 8 ? QMG_C128 : QMG_C64;
    if (l == 0) return fine_schur_reconstruct(mg->fine_in, x_e, b, x, p, mg->nb, mg->s);
    return coarse_schur_reconstruct(mg->lv[l].op, x_e, b, x, p, mg->nb, mg->s);
}

// The system a GCR iterates on: level l's operator on the whole lattice, or
// (schur) its Schur complement on the even sites.
struct Sys {
    int l;
    bool schur;
    int64_t n;                 // complex entries of one member's field
    void *Q, *Z, *r, *t;       // Krylov directions, residual, scratch
};

Sys full_sys(qmg_mg_s* mg, int l) {
    Level& L = mg->lv[l];
    return Sys{l, false, L.n, L.Q, L.Z, L.r, L.t};
}
Sys schur_sys(qmg_mg_s* mg, int l) {
    Level& L = mg->lv[l];
    return Sys{l, true, L.n / 2, L.eQ, L.eZ, L.er, L.et};
}

template <typename R> qmg_status apply_sys(qmg_mg_s* mg, const Sys& sy, const void* in, void* out) {
    return sy.schur ? schur_apply<R>(mg, sy.l, in, out) : apply_op<R>(mg, sy.l, in, out);
}

// copy every member's slots [first, first+count) to the host and wait
qmg_status read_scalars(qmg_mg_s* mg, int first, int count) {
    if (mg->nb == 1)
        QMG_HIP(hipMemcpyAsync(mg->hsc + first, mg->dsc + first, sizeof(double) * count, hipMemcpyDeviceToHost, mg->s));
    else
        QMG_HIP(hipMemcpy2DAsync(mg->hsc + first, sizeof(double) * kScal, mg->dsc + first, sizeof(double) * kScal,
                                 sizeof(double) * count, mg->nb, hipMemcpyDeviceToHost, mg->s));
    QMG_HIP(hipStreamSynchronize(mg->s));
    return QMG_OK;
}

// classical Gram-Schmidt, `passes` passes (two by default): q -= Q beta; z -= Z beta
template <typename R>
qmg_status orthogonalize(qmg_mg_s* mg, const void* Q, const void* Z, int64_t ld, int k, void* q, void* z, int64_t n,
                         int passes = 2) {
    for (int pass = 0; pass < passes; ++pass)
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
    const int nb = mg->nb;
    for (int it = 0; it < L.p.smoother_steps; ++it) {
        const void* cur = it == 0 ? r : L.mr_r;   // the first step reads r itself
        const int groups = l == 0 ? wilson_groups(mg->fine_in) : 0;
        if (l == 0 && groups <= Blas::kMaxBlocks) {
            // the fine operator also sums <Ar,Ar>, <Ar,r> per work-group
            QMG_TRY(wilson_apply_dot(mg->fine_in, cur, L.mr_Ar, sizeof(R) == 8 ? QMG_C128 : QMG_C64, nb,
                                     mg->blas.partials, (int64_t)Blas::kMaxBlocks * Blas::kMaxVals, Blas::kMaxBlocks,
                                     mg->s));
            QMG_TRY(mg->blas.final_sum(groups, 3, mg->dsc + S_MR));
        } else {
            QMG_TRY(apply_op<R>(mg, l, cur, L.mr_Ar));
            QMG_TRY(mg->blas.dot_norm<R>(L.mr_Ar, cur, n, mg->dsc + S_MR));
        }
        QMG_TRY(mg->blas.mr_update<R>(mg->dsc + S_MR, cur, L.mr_r, L.mr_Ar, x, it == 0, n));
    }
    if (L.p.smoother_steps <= 0) {
        QMG_HIP(hipMemsetAsync(x, 0, nb * n * sizeof(cpx<R>), mg->s));
        QMG_HIP(hipMemcpyAsync(L.mr_r, r, nb * n * sizeof(cpx<R>), hipMemcpyDeviceToDevice, mg->s));
    }
    return QMG_OK;
}

// Per-level timing: span k brackets one coarse-grid solve on level l (which
// includes every coarser level's work) with events 2k and 2k+1 on the solve's
// stream.  A pool of kTimingEvents events; spans beyond it are not recorded.
constexpr int kTimingEvents = 8192;
int timing_begin(qmg_mg_s* mg, int l) {
    if (!mg->timing) return -1;
    const int k = (int)mg->span_level.size();
    if (2 * k + 2 > kTimingEvents) {
        mg->spans_overflow = true;
        return -1;
    }
    while ((int)mg->ev.size() < 2 * k + 2) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return -1;
        mg->ev.push_back(e);
    }
    if (hipEventRecord(mg->ev[2 * k], mg->s) != hipSuccess) return -1;
    mg->span_level.push_back(l);
    return k;
}
void timing_end(qmg_mg_s* mg, int k) {
    if (k >= 0) (void)hipEventRecord(mg->ev[2 * k + 1], mg->s);
}
// seconds spent on each level, exclusive of the coarser levels; level 0 is
// the rest of the solve (outer FGCR, fine-level smoothing and transfers)
void timing_collect(qmg_mg_s* mg, double total_s, double out[4]) {
    double incl[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    incl[0] = total_s;
    for (size_t k = 0; k < mg->span_level.size(); ++k) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, mg->ev[2 * k], mg->ev[2 * k + 1]) == hipSuccess)
            incl[mg->span_level[k]] += ms * 1e-3;
    }
    const int nl = (int)mg->lv.size();
    for (int l = 0; l < 4; ++l) out[l] = l < nl ? incl[l] - (l + 1 < nl ? incl[l + 1] : 0.0) : 0.0;
    mg->span_level.clear();
}

// K-cycle preconditioner of a system: K_l(r) on the whole lattice, or for
// the Schur system the even part of K_l applied to (r_e, 0), which is S^-1 r_e
// when K_l = A_l^-1.
template <typename R> qmg_status precond_sys(qmg_mg_s* mg, const Sys& sy, const void* r, void* z) {
    if (!sy.schur) return kcycle<R>(mg, sy.l, r, z);
    Level& L = mg->lv[sy.l];
    const qmg_prec p = sizeof(R) == 8 ? QMG_C128 : QMG_C64;
    const int* hs = level_hsite(mg, sy.l);
    const int64_t Vh = L.V / 2;
    QMG_TRY(eo_scatter(hs, hs + Vh, Vh, L.dof, r, L.kin, p, mg->nb, mg->s));
    QMG_TRY(kcycle<R>(mg, sy.l, L.kin, L.kout));
    return eo_gather(hs, Vh, L.dof, L.kout, z, false, p, mg->nb, mg->s);
}

// Red-black smoother: MR_s on the Schur system S x_e = r_e - M_eo M_oo^-1 r_o
// of level l, then x_o = M_oo^-1 (r_o - M_oe x_e).  The residual r - A x it
// leaves is zero on the odd sites (up to rounding) and the MR residual on the
// even ones; that is what lv.mr_r receives.
// Level 0: the same MR steps on the Schur system with 16-bit vectors (FP16
// pairs with a scale per site; FP32 arithmetic; the iterate x in complex64),
// the paper's half-precision fine-level smoother.
qmg_status mr_schur16(qmg_mg_s* mg, const void* r, void* x) {
    Level& L = mg->lv[0];
    const int64_t Vh = L.V / 2;
    const int nb = mg->nb;
    hipStream_t s = mg->s;
    QMG_TRY(schur_source<float>(mg, 0, r, L.sb));
    QMG_TRY(mg->blas.quantize_spinors(L.sb, L.hb, L.hbs, Vh * nb));
    for (int it = 0; it < L.p.smoother_steps; ++it) {
        const void* cur = it == 0 ? L.hb : L.hr;
        const float* curs = it == 0 ? L.hbs : L.hrs;
        QMG_TRY(fine_schur_apply16(mg->fine_in, cur, curs, L.hAr, L.hArs, L.ht, L.hts, nb, s));
        QMG_TRY(mg->blas.dot_norm_h16(L.hAr, L.hArs, cur, curs, Vh, mg->dsc + S_MR));
        QMG_TRY(mg->blas.mr_update_h16(mg->dsc + S_MR, cur, curs, L.hr, L.hrs, L.hAr, L.hArs, L.sx, it == 0, Vh));
    }
    if (L.p.smoother_steps <= 0) {
        QMG_HIP(hipMemsetAsync(L.sx, 0, nb * Vh * 12 * sizeof(cpx<float>), s));
        QMG_HIP(hipMemcpyAsync(L.hr, L.hb, nb * Vh * 48, hipMemcpyDeviceToDevice, s));
        QMG_HIP(hipMemcpyAsync(L.hrs, L.hbs, nb * Vh * sizeof(float), hipMemcpyDeviceToDevice, s));
    }
    QMG_TRY(schur_reconstruct<float>(mg, 0, L.sx, r, x));
    // the whole residual: the even sites' 16-bit residual decoded, zero on the odd sites
    const int* hs = level_hsite(mg, 0);
    return mg->blas.scatter_dequantize(L.hr, L.hrs, hs, hs + Vh, L.mr_r, Vh);
}

template <typename R> qmg_status mr_schur(qmg_mg_s* mg, int l, const void* r, void* x) {
    if constexpr (sizeof(R) == 4)
        if (l == 0 && mg->smooth16) return mr_schur16(mg, r, x);
    Level& L = mg->lv[l];
    const int64_t ne = L.n / 2;
    const int nb = mg->nb;
    const qmg_prec p = sizeof(R) == 8 ? QMG_C128 : QMG_C64;
    QMG_TRY(schur_source<R>(mg, l, r, L.sb));
    for (int it = 0; it < L.p.smoother_steps; ++it) {
        const void* cur = it == 0 ? L.sb : L.sr;
        QMG_TRY(schur_apply<R>(mg, l, cur, L.sAr));
        QMG_TRY(mg->blas.dot_norm<R>(L.sAr, cur, ne, mg->dsc + S_MR));
        QMG_TRY(mg->blas.mr_update<R>(mg->dsc + S_MR, cur, L.sr, L.sAr, L.sx, it == 0, ne));
    }
    if (L.p.smoother_steps <= 0) {
        QMG_HIP(hipMemsetAsync(L.sx, 0, nb * ne * sizeof(cpx<R>), mg->s));
        QMG_HIP(hipMemcpyAsync(L.sr, L.sb, nb * ne * sizeof(cpx<R>), hipMemcpyDeviceToDevice, mg->s));
    }
    QMG_TRY(schur_reconstruct<R>(mg, l, L.sx, r, x));
    const int* hs = level_hsite(mg, l);
    return eo_scatter(hs, hs + L.V / 2, L.V / 2, L.dof, L.sr, L.mr_r, p, nb, mg->s);
}

// GCR on a system of level l (l >= 1 uses the level's op; l == 0 with inner
// precision is used by the setup).  Solves A x = b from x (if x0) or from 0,
// for every batch member; stops when all members reach tol (or after maxit
// steps).
template <typename R>
qmg_status gcr(qmg_mg_s* mg, const Sys& sy, const void* b, void* x, bool x0, double tol, int maxit, bool precond,
               int* iters_out) {
    const int l = sy.l;
    Level& L = mg->lv[l];
    const int64_t n = sy.n;
    if (L.Ainv && !sy.schur) {   // the coarsest level with its dense inverse: x = A^-1 b, one launch
        QMG_TRY(dense_apply(L.Ainv, b, x, n, mg->nb, sizeof(R) == 8 ? QMG_C128 : QMG_C64, mg->s));
        if (iters_out) *iters_out += 1;
        return QMG_OK;
    }
    const int m = mg->restart;
    const int nb = mg->nb;
    const size_t vb = n * sizeof(cpx<R>);   // one member's field
    const size_t bb = nb * vb;              // the batch's field (one Krylov direction of all members)
    // |b|^2 stays on the device (the single-work-group step takes its stopping
    // test from it); the host reads it with the first step's scalars
    double bnorm[Blas::kMaxBatch];
    const int sbn = S_BN + l;
    QMG_TRY(mg->blas.norm2<R>(b, n, mg->dsc + sbn));
    if (x0) {
        QMG_TRY(apply_sys<R>(mg, sy, x, sy.t));
        QMG_TRY(mg->blas.xmy<R>(b, sy.t, sy.r, n));
    } else {
        QMG_HIP(hipMemsetAsync(x, 0, bb, mg->s));
        QMG_HIP(hipMemcpyAsync(sy.r, b, bb, hipMemcpyDeviceToDevice, mg->s));
    }
    // all members converged (or broken down: q = 0) after the scalars in slots
    // S_GCR (and rnorm2 at `rslot`) were read.  A member with b = 0 is not
    // done by itself: from a start x0 that is the relaxation A x = 0 of the
    // setup, which runs to maxit; from x = 0 its q is 0 and it breaks down.
    auto all_done = [&](int rslot, bool* fault) {
        bool done = true;
        for (int k = 0; k < nb; ++k) {
            const double rn = std::sqrt(hs(mg, k, rslot));
            if (!std::isfinite(rn) || !std::isfinite(hs(mg, k, S_GCR))) *fault = true;
            const bool ok = hs(mg, k, S_GCR) <= 0.0 || (bnorm[k] > 0 && rn <= tol * bnorm[k]);
            done = done && ok;
        }
        return done;
    };
    int iters = 0;
    bool done = false;
    const int64_t ld = (int64_t)nb * n;
    // With tol = 0 (the setup's relaxation) only a breakdown (q = 0) or a
    // non-finite value can end the iteration early.  After a breakdown every
    // later step of the cycle is a no-op (the update skips q = 0 and the next
    // q is 0 again), so reading the scalars only at the end of a cycle stops
    // with the same x while saving a host round trip per step.
    const bool defer = !(tol > 0.0);
    // short unpreconditioned systems (the coarsest level): the whole step's
    // vector work is one single-work-group kernel per member, so a step is two launches
    const bool small = !precond && n <= Blas::kSmall;
    if (small)   // stopping-test flags and step counters of every member
        QMG_HIP(hipMemset2DAsync(mg->dsc + S_OK, sizeof(double) * kScal, 0, 3 * sizeof(double), nb, mg->s));
    int launches = 0;   // single-work-group steps queued: the flags of the last one are in slot S_OK + (launches & 1)
    // Single-work-group steps: a step queued after every member has passed its
    // test does nothing, so steps are queued ahead of the host's reads of the
    // scalars, across restarts: the first read comes a few steps before the
    // step count of this level's previous solve, then one every kRecheck steps
    // (with tol = 0, only at maxit).  Reads never change the iterates.
    int& expect = L.small_steps[sy.schur ? 1 : 0];
    int next_read = defer ? maxit : std::max(kCheck, expect - 3);
    while (!done && iters < maxit) {
        int j = 0;
        if (small) QMG_HIP(hipMemcpyAsync(sy.Z, sy.r, bb, hipMemcpyDeviceToDevice, mg->s));
        for (; j < m && iters < maxit; ++j) {
            void* z = (char*)sy.Z + j * bb;
            void* q = (char*)sy.Q + j * bb;
            bool fault = false;
            if (small) {
                // the step evaluates the stopping test itself (a step queued
                // after every member has passed it does nothing), so the
                // scalars are read only when next_read is reached
                QMG_TRY(apply_sys<R>(mg, sy, z, q));
                void* znext = j + 1 < m ? (char*)sy.Z + (j + 1) * bb : nullptr;
                QMG_TRY(mg->blas.gcr_step_small<R>(sy.Q, sy.Z, ld, j, q, z, x, sy.r, n, mg->dsc + S_GCR, znext,
                                                   tol > 0.0 ? tol : 0.0, S_OK - S_GCR, sbn - S_GCR,
                                                   launches & 1));
                ++launches;
                ++iters;
                if (iters < next_read && iters < maxit) continue;
                QMG_TRY(read_scalars(mg, S_GCR, S_OK + 3 - S_GCR));
                iters = (int)hs(mg, 0, S_OK + 2);   // steps that ran (the same for every member)
                done = true;
                for (int b = 0; b < nb; ++b) {
                    if (!std::isfinite(hs(mg, b, S_GCR + 3)) || !std::isfinite(hs(mg, b, S_GCR))) fault = true;
                    done = done && hs(mg, b, S_OK + (launches & 1)) != 0.0;
                }
                if (fault) return fail(QMG_ERR_NONFINITE, "gcr on level %d: non-finite residual after %d steps", l, iters);
                if (done) { ++j; break; }
                next_read = iters + kRecheck;
                continue;
            }
            if (precond) QMG_TRY(precond_sys<R>(mg, sy, sy.r, z));
            else QMG_HIP(hipMemcpyAsync(z, sy.r, bb, hipMemcpyDeviceToDevice, mg->s));
            QMG_TRY(apply_sys<R>(mg, sy, z, q));
            QMG_TRY(orthogonalize<R>(mg, sy.Q, sy.Z, ld, j, q, z, n));
            QMG_TRY(mg->blas.dot_norm<R>(q, sy.r, n, mg->dsc + S_GCR));
            QMG_TRY(mg->blas.gcr_update<R>(mg->dsc + S_GCR, q, z, x, sy.r, n));
            ++iters;
            if (defer && j + 1 < m && iters < maxit) continue;
            QMG_TRY(mg->blas.norm2<R>(sy.r, n, mg->dsc + S_NRM));
            QMG_TRY(read_scalars(mg, S_GCR, sbn + 1 - S_GCR));
            for (int k = 0; k < nb; ++k) bnorm[k] = std::sqrt(hs(mg, k, sbn));
            done = all_done(S_NRM, &fault);
            if (fault) return fail(QMG_ERR_NONFINITE, "gcr on level %d: non-finite residual after %d steps", l, iters);
            if (done) { ++j; break; }
        }
        if (done || iters >= maxit) break;
        // restart from the true residual
        QMG_TRY(apply_sys<R>(mg, sy, x, sy.t));
        QMG_TRY(mg->blas.xmy<R>(b, sy.t, sy.r, n));
    }
    if (small && !defer) expect = iters;
    if (iters_out) *iters_out += iters;
    return QMG_OK;
}

// Level smoother: MR, or on level 0 the learned network when one is attached.
// The network's output d = N(r) is kept only if it lowers the residual
// (|r - A d| < |r|); it is then taken with the minimal-residual step length,
// x = alpha d with alpha = <A d, r>/|A d|^2, which lowers it further.
// Network alone: otherwise (including NaN/Inf from bad weights) MR is used for
// this application; in a batch the network runs on every member and is kept
// only if it passes for every member; each member that fails counts as a
// fallback.  Network followed by MR steps: the test is made on the device,
// per member, with no host round trip; a refused network step is skipped
// (x = 0, counted as a fallback) and the MR steps run either way.
// On exit lv.mr_r holds r - A x.
template <typename R> qmg_status smooth(qmg_mg_s* mg, int l, const void* r, void* x) {
    Level& L = mg->lv[l];
    if (l == 0 && mg->ptc && sizeof(R) == 4) {
        const size_t vb = L.n * sizeof(cpx<R>);
        for (int k = 0; k < mg->nb; ++k)
            QMG_TRY(ptc_forward(mg->ptc, (const char*)r + k * vb, (char*)L.kt + k * vb, mg->s));
        QMG_TRY(apply_op<R>(mg, 0, L.kt, L.mr_Ar));
        QMG_TRY(mg->blas.dot_norm<R>(L.mr_Ar, r, L.n, mg->dsc + S_SM));
        if (mg->ptc_mr > 0) {
            QMG_TRY(mg->blas.dir_step_checked<R>(mg->dsc + S_SM, L.kt, L.mr_Ar, r, x, L.mr_r, L.n, S_FB - S_SM));
            // then MR steps on the residual left: x += MR_k(r - A x)
            const int keep = L.p.smoother_steps;
            L.p.smoother_steps = mg->ptc_mr;
            const qmg_status st = mr<R>(mg, l, L.mr_r, L.kt);
            L.p.smoother_steps = keep;
            QMG_TRY(st);
            return mg->blas.axpy<R>(1.0, L.kt, x, L.n);
        }
        QMG_TRY(read_scalars(mg, S_SM, 3));
        int bad = 0;
        for (int k = 0; k < mg->nb; ++k) {
            // kept only if the network's own output lowers the residual:
            // |r - M d|^2 - |r|^2 = |M d|^2 - 2 Re <M d, r> < 0
            const double den = hs(mg, k, S_SM), re = hs(mg, k, S_SM + 1), im = hs(mg, k, S_SM + 2);
            const bool ok = den > 0 && std::isfinite(den) && std::isfinite(re) && std::isfinite(im) && den - 2 * re < 0;
            if (!ok) ++bad;
        }
        if (bad == 0) return mg->blas.dir_step<R>(mg->dsc + S_SM, L.kt, L.mr_Ar, r, x, L.mr_r, L.n);
        mg->fallbacks += bad;
    }
    if (l == 0 && mg->sap && sizeof(R) == 4) {
        // one SAP sweep, then the residual r - A x the K-cycle goes on with
        QMG_TRY(sap_sweep(mg->fine_in, *mg->sap, r, x, mg->sap_iters, mg->nb, mg->s));
        QMG_TRY(apply_op<R>(mg, 0, x, L.mr_Ar));
        return mg->blas.xmy<R>(r, L.mr_Ar, L.mr_r, L.n);
    }
    if (mg->eo) return mr_schur<R>(mg, l, r, x);
    return mr<R>(mg, l, r, x);
}

// keep a copy of a level-0 smoother input when recording (single solves, complex64)
template <typename R> qmg_status record_smoother_input(qmg_mg_s* mg, const void* v, int64_t n) {
    if (!mg->srec || mg->srec_n >= mg->srec_max || sizeof(R) != 4) return QMG_OK;
    const size_t vb = n * sizeof(cpx<float>);
    QMG_HIP(hipMemcpyAsync((char*)mg->srec + (size_t)mg->srec_n * vb, v, vb, hipMemcpyDeviceToDevice, mg->s));
    ++mg->srec_n;
    return QMG_OK;
}

template <typename R> qmg_status kcycle(qmg_mg_s* mg, int l, const void* rin, void* zout) {
    Level& L = mg->lv[l];
    Level& C = mg->lv[l + 1];
    const int64_t n = L.n;
    const qmg_prec p = sizeof(R) == 8 ? QMG_C128 : QMG_C64;
    const int nl = (int)mg->lv.size();
    if (l == 0) QMG_TRY(record_smoother_input<R>(mg, rin, n));
    // pre-smoothing; L.mr_r = rin - A zout afterwards
    QMG_TRY(smooth<R>(mg, l, rin, zout));
    QMG_TRY(transfer_restrict(L.T, L.mr_r, C.b, p, mg->nb, mg->s));
    const bool coarsest = (l + 1 == nl - 1);
    int it = 0;
    const int span = timing_begin(mg, l + 1);
    if (mg->eo && !C.Ainv) {
        // red-black: GCR on the next level's Schur system, odd sites back-substituted
        QMG_TRY(schur_source<R>(mg, l + 1, C.b, C.eb));
        QMG_TRY(gcr<R>(mg, schur_sys(mg, l + 1), C.eb, C.ex, false, L.p.coarse_tol, L.p.coarse_maxit, !coarsest, &it));
        QMG_TRY(schur_reconstruct<R>(mg, l + 1, C.ex, C.b, C.x));
    } else {
        QMG_TRY(gcr<R>(mg, full_sys(mg, l + 1), C.b, C.x, false, L.p.coarse_tol, L.p.coarse_maxit, !coarsest, &it));
    }
    timing_end(mg, span);
    mg->level_iters[l + 1] += it;
    QMG_TRY(transfer_prolong(L.T, C.x, L.kt, p, mg->nb, mg->s));
    QMG_TRY(mg->blas.axpy<R>(1.0, L.kt, zout, n));
    // post-smoothing on r - A z
    QMG_TRY(apply_op<R>(mg, l, zout, L.kt));
    QMG_TRY(mg->blas.xmy<R>(rin, L.kt, L.kr2, n));
    if (l == 0) QMG_TRY(record_smoother_input<R>(mg, L.kr2, n));
    QMG_TRY(smooth<R>(mg, l, L.kr2, L.kx2));
    QMG_TRY(mg->blas.axpy<R>(1.0, L.kx2, zout, n));
    return QMG_OK;
}

// Solve workspace of every level and of the FP64 outer solver for `cap`
// batch members (replacing any smaller one).
qmg_status workspace(qmg_mg_s* mg, int cap) {
    for (void* p : mg->sallocs) (void)hipFree(p);
    mg->sallocs.clear();
    mg->cap = 0;
    const size_t cb = mg->inner == QMG_C128 ? 16 : 8;
    for (size_t l = 0; l < mg->lv.size(); ++l) {
        Level& L = mg->lv[l];
        const size_t vb = L.n * cb * cap;
        void** one[] = {&L.r, &L.x, &L.b, &L.t, &L.mr_r, &L.mr_Ar, &L.kt, &L.kr2, &L.kx2, &L.kin, &L.kout};
        for (void** p : one) QMG_TRY(salloc(mg, p, vb));
        QMG_TRY(salloc(mg, &L.Q, vb * mg->restart));
        QMG_TRY(salloc(mg, &L.Z, vb * mg->restart));
        L.q16 = nullptr;
        L.qsc = nullptr;
        if (l >= 1 && L.op && cap >= 8 && coarse_batch_uses_mfma(L.op, 8)) {
            QMG_TRY(salloc(mg, &L.q16, (size_t)L.V * cap * L.dof * 4));
            QMG_TRY(salloc(mg, (void**)&L.qsc, (size_t)L.V * cap * 4));
        }
        void** half[] = {&L.eb, &L.ex, &L.er, &L.et, &L.sb, &L.sx, &L.sr, &L.sAr, &L.etmp, &L.ekin};
        for (void** p : half) *p = nullptr;
        L.eQ = L.eZ = nullptr;
        if (mg->eo) {
            for (void** p : half) QMG_TRY(salloc(mg, p, vb / 2));
            QMG_TRY(salloc(mg, &L.eQ, vb / 2 * mg->restart));
            QMG_TRY(salloc(mg, &L.eZ, vb / 2 * mg->restart));
        }
        void** h16[] = {&L.hb, &L.hr, &L.ht, &L.hAr};
        float** h16s[] = {&L.hbs, &L.hrs, &L.hts, &L.hArs};
        for (void** p : h16) *p = nullptr;
        for (float** p : h16s) *p = nullptr;
        if (l == 0 && mg->eo && mg->smooth16) {
            const size_t sites = (size_t)(L.V / 2) * cap;
            for (void** p : h16) QMG_TRY(salloc(mg, p, sites * 48));
            for (float** p : h16s) QMG_TRY(salloc(mg, (void**)p, sites * 4));
        }
    }
    const size_t vb64 = mg->lv[0].n * 16 * cap;
    QMG_TRY(salloc(mg, &mg->Q64, vb64 * mg->restart));
    QMG_TRY(salloc(mg, &mg->Z64, vb64 * mg->restart));
    QMG_TRY(salloc(mg, &mg->r64, vb64));
    QMG_TRY(salloc(mg, &mg->t64, vb64));
    mg->eb64 = mg->ex64 = mg->etmp64 = nullptr;
    if (mg->eo) {
        QMG_TRY(salloc(mg, &mg->eb64, vb64 / 2));
        QMG_TRY(salloc(mg, &mg->ex64, vb64 / 2));
        QMG_TRY(salloc(mg, &mg->etmp64, vb64 / 2));
    }
    mg->cap = cap;
    return QMG_OK;
}

// storage of level L's transfer basis in the solve
qmg_prec transfer_prec(const qmg_mg_s* mg, const Level& L) {
    return L.p.transfer_storage ? (qmg_prec)L.p.transfer_storage : mg->inner;
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
            if (st == QMG_OK) st = gcr<R>(mg, full_sys(mg, l), L.b, v, true, 0.0, setup_iters, false, nullptr);
            if (st == QMG_OK) st = orthogonalize<R>(mg, NV, nullptr, n, k, v, nullptr, n);
        }
        if (st == QMG_OK) st = mg->blas.norm2<R>(v, n, mg->dsc + S_NRM);
        if (st == QMG_OK) st = mg->blas.normalize<R>(v, mg->dsc + S_NRM, n);
    }
    if (st == QMG_OK) st = mg->blas.convert<R, double>(NV, NV64, n * nvec);
    if (st == QMG_OK)
        st = qmg_transfer_create(L.dims, L.dof, L.p.block, nvec, NV64, transfer_prec(mg, L), mg->s, &L.T);
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

// transfer of level l from a finished FP64 basis (checkpoint resume), then the
// next coarse operator exactly as setup_level builds it
qmg_status import_level(qmg_mg_s* mg, int l, const void* basis) {
    Level& L = mg->lv[l];
    QMG_TRY(qmg_transfer_import(L.dims, L.dof, L.p.block, L.p.nvec, basis, transfer_prec(mg, L), mg->s, &L.T));
    Level& C = mg->lv[l + 1];
    const qmg_status st = l == 0 ? qmg_build_coarse_op(L.T, mg->fine64, nullptr, mg->inner, mg->s, &C.op)
                                 : qmg_build_coarse_op(L.T, nullptr, L.op, mg->inner, mg->s, &C.op);
    (void)hipStreamSynchronize(mg->s);
    return st;
}

// b, x: nb members of [V][12] complex128; info: nb entries (or NULL)
template <typename R>
qmg_status solve_impl(qmg_mg_s* mg, const void* b, void* x, const qmg_solve_params* sp, qmg_solve_info* info) {
    Level& L0 = mg->lv[0];
    const int64_t n = L0.n;
    const int nb = mg->nb;
    const size_t vb64 = n * 16;       // one member
    const size_t bb64 = nb * vb64;    // the batch
    const int m = mg->restart;
    const int nl = (int)mg->lv.size();
    const qmg_prec pin = sizeof(R) == 8 ? QMG_C128 : QMG_C64;
    // Red-black form: the outer FGCR runs on the fine Schur system
    // S x_e = b_e - D_eo C_oo^-1 b_o (fields of n/2 entries), preconditioned by
    // the even part of K_0 applied to (r_e, 0); x_o is back-substituted at every
    // reliable update, whose true residual is that of the whole system.
    const bool eo = mg->eo;
    const int64_t ns = eo ? n / 2 : n;             // entries of one member's outer field
    const size_t bbs = nb * ns * 16;               // one outer field of the batch
    const int64_t ld = (int64_t)nb * ns;
    const int* hs0 = eo ? mg->fine_in->hsite : nullptr;
    const int64_t Vh = L0.V / 2;
    auto outer_apply = [&](const void* in, void* out) -> qmg_status {
        if (eo) return fine_schur_apply(mg->fine64, in, out, mg->etmp64, QMG_C128, nb, mg->s);
        return wilson_apply(mg->fine64, in, out, QMG_C128, nb, mg->s);
    };
    for (int i = 0; i < 8; ++i) mg->level_iters[i] = 0;
    mg->span_level.clear();
    mg->spans_overflow = false;
    mg->fallbacks = 0;
    if (mg->ptc) QMG_HIP(hipMemset2DAsync(mg->dsc + S_FB, sizeof(double) * kScal, 0, sizeof(double), nb, mg->s));
    mg->rec_n = 0;
    mg->srec_n = 0;
    auto t0 = std::chrono::steady_clock::now();
    QMG_TRY(mg->blas.norm2<double>(b, n, mg->dsc + S_BN));
    QMG_TRY(read_scalars(mg, S_BN, 1));
    double bnorm[Blas::kMaxBatch], true_rel[Blas::kMaxBatch];
    bool conv[Blas::kMaxBatch];
    bool all_conv = true;
    for (int k = 0; k < nb; ++k) {
        bnorm[k] = std::sqrt(hs(mg, k, S_BN));
        true_rel[k] = bnorm[k] > 0 ? 1.0 : 0.0;
        conv[k] = bnorm[k] == 0.0;
        all_conv = all_conv && conv[k];
    }
    const void* bs = b;   // the outer system's right-hand side and iterate
    void* xs = x;
    QMG_HIP(hipMemsetAsync(x, 0, bb64, mg->s));
    if (eo) {
        QMG_TRY(fine_schur_source(mg->fine64, b, mg->eb64, mg->etmp64, QMG_C128, nb, mg->s));
        bs = mg->eb64;
        xs = mg->ex64;
        QMG_HIP(hipMemsetAsync(xs, 0, bbs, mg->s));
    }
    QMG_HIP(hipMemcpyAsync(mg->r64, bs, bbs, hipMemcpyDeviceToDevice, mg->s));
    // Deferred solution update (unless iterates are recorded every step): the
    // preconditioned directions w_j stay as the K-cycle returned them and only
    // q_j is orthogonalised and normalised; with Z_j = (w_j - sum_i beta_ij Z_i)
    // / nu_j the cycle's correction sum_j alpha_j Z_j = sum_j gamma_j w_j, gamma
    // by back substitution, is added to x once at the end of the cycle.  The
    // residual recursion is the same as in the eager form.
    const bool deferred = !mg->rec && m <= 16;
    std::vector<std::complex<double>> cbeta, calpha;
    std::vector<double> cnu;
    if (deferred) {
        cbeta.assign((size_t)nb * m * m, 0.0);
        calpha.assign((size_t)nb * m, 0.0);
        cnu.assign((size_t)nb * m, 0.0);
    }
    auto add_beta = [&](int j) {   // the projection coefficients of q_j now in the mirror's S_BETA slots
        for (int b = 0; b < nb; ++b)
            for (int i = 0; i < j; ++i)
                cbeta[((size_t)b * m + i) * m + j] += std::complex<double>(hs(mg, b, S_BETA + 2 * i),
                                                                           hs(mg, b, S_BETA + 2 * i + 1));
    };
    int iters = 0, restarts = 0;
    while (!all_conv && iters < sp->maxit) {
        int kc = 0;   // steps of this cycle
        if (deferred) std::fill(cbeta.begin(), cbeta.end(), 0.0);
        for (int j = 0; j < m && iters < sp->maxit; ++j) {
            void* z = (char*)mg->Z64 + j * bbs;
            void* q = (char*)mg->Q64 + j * bbs;
            if (nl > 1 && eo) {
                QMG_TRY(mg->blas.convert<double, R>(mg->r64, L0.ekin, ns));
                QMG_TRY(eo_scatter(hs0, hs0 + Vh, Vh, 12, L0.ekin, L0.kin, pin, nb, mg->s));
                QMG_TRY(kcycle<R>(mg, 0, L0.kin, L0.kout));
                QMG_TRY(eo_gather(hs0, Vh, 12, L0.kout, L0.ekin, false, pin, nb, mg->s));
                QMG_TRY(mg->blas.convert<R, double>(L0.ekin, z, ns));
            } else if (nl > 1) {
                QMG_TRY(mg->blas.convert<double, R>(mg->r64, L0.kin, n));
                QMG_TRY(kcycle<R>(mg, 0, L0.kin, L0.kout));
                QMG_TRY(mg->blas.convert<R, double>(L0.kout, z, n));
            } else {
                QMG_HIP(hipMemcpyAsync(z, mg->r64, bbs, hipMemcpyDeviceToDevice, mg->s));
            }
            QMG_TRY(outer_apply(z, q));
            if (j == 0) {
                QMG_TRY(mg->blas.dot_norm<double>(q, mg->r64, ns, mg->dsc + S_GCR));
            } else {
                // one projection pass, and a second only if it cancelled more
                // than half of |q|^2 for some member (the Daniel-Gragg-Kaufman-
                // Stewart test; the preconditioned directions are nearly
                // orthogonal already, so the second pass is rarely needed)
                QMG_TRY(mg->blas.norm2<double>(q, ns, mg->dsc + S_QQ));
                const void* Zs = deferred ? nullptr : mg->Z64;
                void* zs = deferred ? nullptr : z;
                QMG_TRY(orthogonalize<double>(mg, mg->Q64, Zs, ld, j, q, zs, ns, 1));
                QMG_TRY(mg->blas.dot_norm<double>(q, mg->r64, ns, mg->dsc + S_GCR));
                const int first = deferred ? S_BETA : S_GCR;
                QMG_TRY(read_scalars(mg, first, S_QQ + 1 - first));
                if (deferred) add_beta(j);
                bool again = false;
                for (int b = 0; b < nb; ++b) again = again || !(hs(mg, b, S_GCR) >= 0.5 * hs(mg, b, S_QQ));
                if (again) {
                    QMG_TRY(orthogonalize<double>(mg, mg->Q64, Zs, ld, j, q, zs, ns, 1));
                    QMG_TRY(mg->blas.dot_norm<double>(q, mg->r64, ns, mg->dsc + S_GCR));
                    if (deferred) {   // the second pass's coefficients add to the first's
                        QMG_TRY(read_scalars(mg, S_BETA, 2 * j));
                        add_beta(j);
                    }
                }
            }
            QMG_TRY(mg->blas.gcr_update<double>(mg->dsc + S_GCR, q, deferred ? nullptr : z, deferred ? nullptr : xs,
                                                mg->r64, ns));
            QMG_TRY(mg->blas.norm2<double>(mg->r64, ns, mg->dsc + S_NRM));
            QMG_TRY(read_scalars(mg, S_GCR, 5));
            if (deferred) {
                for (int b = 0; b < nb; ++b) {
                    const double qq = hs(mg, b, S_GCR);
                    const double nu = qq > 0 ? std::sqrt(qq) : 0.0;
                    cnu[(size_t)b * m + j] = nu;
                    calpha[(size_t)b * m + j] =
                        nu > 0 ? std::complex<double>(hs(mg, b, S_GCR + 1), hs(mg, b, S_GCR + 2)) / nu : 0.0;
                }
            }
            ++kc;
            ++iters;
            if (mg->rec && mg->rec_n < mg->rec_max) {
                QMG_HIP(hipMemcpyAsync((char*)mg->rec + (size_t)mg->rec_n * vb64, x, vb64, hipMemcpyDeviceToDevice, mg->s));
                ++mg->rec_n;
            }
            bool stop = true;
            for (int k = 0; k < nb; ++k) {
                const double rn = std::sqrt(hs(mg, k, S_NRM));
                if (!std::isfinite(rn)) return fail(QMG_ERR_NONFINITE, "mg_gcr_solve: non-finite residual at step %d", iters);
                stop = stop && (rn <= sp->tol * bnorm[k] || hs(mg, k, S_GCR) <= 0.0);
            }
            if (stop) break;
        }
        if (deferred && kc > 0) {
            // x += sum_j gamma_j w_j: back substitution through Z_j = (w_j - sum_i beta_ij Z_i) / nu_j
            // (a broken-down step, nu_j = 0, contributes nothing and projected nothing away)
            for (int b = 0; b < nb; ++b) {
                std::complex<double> c[16];
                for (int j = 0; j < kc; ++j) c[j] = calpha[(size_t)b * m + j];
                for (int j = kc - 1; j >= 0; --j) {
                    const double nu = cnu[(size_t)b * m + j];
                    const std::complex<double> g = nu > 0 ? c[j] / nu : 0.0;
                    for (int i = 0; i < j; ++i) c[i] -= cbeta[((size_t)b * m + i) * m + j] * g;
                    hs(mg, b, S_BETA + 2 * j) = -g.real();   // multi_axpy subtracts
                    hs(mg, b, S_BETA + 2 * j + 1) = -g.imag();
                }
            }
            if (nb == 1)
                QMG_HIP(hipMemcpyAsync(mg->dsc + S_BETA, mg->hsc + S_BETA, sizeof(double) * 2 * kc,
                                       hipMemcpyHostToDevice, mg->s));
            else
                QMG_HIP(hipMemcpy2DAsync(mg->dsc + S_BETA, sizeof(double) * kScal, mg->hsc + S_BETA,
                                         sizeof(double) * kScal, sizeof(double) * 2 * kc, nb, hipMemcpyHostToDevice,
                                         mg->s));
            QMG_TRY(mg->blas.multi_axpy<double>(mg->dsc + S_BETA, mg->Z64, nullptr, ld, kc, xs, nullptr, ns));
        }
        // reliable update: true residual in FP64 (of the whole system, after
        // the odd sites are back-substituted in the red-black form)
        void* rfull = eo ? mg->Q64 : mg->r64;   // the Krylov space is restarted, so Q64 is free
        if (eo) QMG_TRY(fine_schur_reconstruct(mg->fine64, xs, b, x, QMG_C128, nb, mg->s));
        QMG_TRY(wilson_apply(mg->fine64, x, mg->t64, QMG_C128, nb, mg->s));
        QMG_TRY(mg->blas.xmy<double>(b, mg->t64, rfull, n));
        QMG_TRY(mg->blas.norm2<double>(rfull, n, mg->dsc + S_NRM));
        QMG_TRY(read_scalars(mg, S_NRM, 1));
        all_conv = true;
        for (int k = 0; k < nb; ++k) {
            const double tr = std::sqrt(hs(mg, k, S_NRM));
            if (!std::isfinite(tr)) return fail(QMG_ERR_NONFINITE, "mg_gcr_solve: non-finite true residual");
            true_rel[k] = bnorm[k] > 0 ? tr / bnorm[k] : 0.0;
            conv[k] = tr <= sp->tol * bnorm[k];
            all_conv = all_conv && conv[k];
        }
        if (!all_conv) {
            ++restarts;
            if (eo) {   // restart from the Schur system's true residual
                QMG_TRY(outer_apply(xs, mg->t64));
                QMG_TRY(mg->blas.xmy<double>(bs, mg->t64, mg->r64, ns));
            }
        }
    }
    auto t1 = std::chrono::steady_clock::now();
    if (mg->ptc && mg->ptc_mr > 0) {   // network steps refused on the device
        QMG_TRY(read_scalars(mg, S_FB, 1));
        for (int k = 0; k < nb; ++k) mg->fallbacks += (int)hs(mg, k, S_FB);
    }
    double worst = 0;
    for (int k = 0; k < nb; ++k) worst = true_rel[k] > worst ? true_rel[k] : worst;
    double lsec[4] = {0, 0, 0, 0};
    if (mg->timing) {
        QMG_HIP(hipStreamSynchronize(mg->s));
        timing_collect(mg, std::chrono::duration<double>(t1 - t0).count(), lsec);
        if (mg->spans_overflow) lsec[0] = -1.0;   // incomplete: too many coarse solves to time
    }
    if (info) {
        for (int k = 0; k < nb; ++k) {
            qmg_solve_info& I = info[k];
            I.outer_iters = iters;
            for (int l = 0; l < 4; ++l) I.level_iters[l] = l < nl ? mg->level_iters[l] : 0;
            I.level_iters[0] = iters;
            I.restarts = restarts;
            I.true_rel_residual = true_rel[k];
            I.seconds = std::chrono::duration<double>(t1 - t0).count();
            I.converged = conv[k] ? 1 : 0;
            I.smoother_fallbacks = mg->fallbacks;
            for (int l = 0; l < 4; ++l) I.level_seconds[l] = lsec[l];
        }
    }
    if (!all_conv) return fail(QMG_ERR_NOCONV, "mg_gcr_solve: %d steps, relative residual %.3e", iters, worst);
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
    for (void* p : mg->sallocs) (void)hipFree(p);
    if (mg->hsc) (void)hipHostFree(mg->hsc);
    for (hipEvent_t e : mg->ev) (void)hipEventDestroy(e);
    sap_plan_destroy(mg->sap);
    mg->blas.release();
    delete mg;
}

// qmg_mg_create (vecs = start vectors of the relaxation) and
// qmg_mg_create_from_bases (vecs = finished transfer bases, no relaxation)
static qmg_status mg_make(const int dims[4], const void* gauge, double m0, double csw, int antiperiodic_t,
                          int nlevels, const qmg_level_params* lp, const void* const* starts,
                          bool from_bases, qmg_prec inner, qmg_prec fine_storage, void* stream, qmg_mg* out) {
    if (!out) return fail(QMG_ERR_ARG, "mg_create: out is NULL");
    *out = nullptr;
    QMG_TRY(check_dims(dims, 2, "mg_create"));
    if (!gauge) return fail(QMG_ERR_ARG, "mg_create: gauge is NULL");
    if (nlevels < 1 || nlevels > 4) return fail(QMG_ERR_ARG, "mg_create: nlevels %d outside [1,4]", nlevels);
    if (nlevels > 1 && (!lp || !starts))
        return fail(QMG_ERR_ARG, "mg_create: level params / %s missing", from_bases ? "bases" : "starts");
    if (inner != QMG_C128 && inner != QMG_C64) return fail(QMG_ERR_PREC, "mg_create: inner precision %d", (int)inner);
    const bool fine16 = fine_storage == QMG_H16 || fine_storage == QMG_B16;
    if (fine_storage != 0 && fine_storage != inner && !fine16)
        return fail(QMG_ERR_PREC, "mg_create: fine storage %d", (int)fine_storage);
    if (fine16 && inner != QMG_C64)
        return fail(QMG_ERR_PREC, "mg_create: 16-bit fine storage needs complex64 inner precision");
    for (int l = 0; l + 1 < nlevels; ++l) {
        if (!starts[l]) return fail(QMG_ERR_ARG, "mg_create: %s[%d] is NULL", from_bases ? "bases" : "starts", l);
        if (lp[l].nvec < 1 || lp[l].nvec > 64) return fail(QMG_ERR_ARG, "mg_create: nvec %d", lp[l].nvec);
        if (lp[l].smoother_steps < 0 || lp[l].coarse_maxit < 1 || lp[l].setup_iters < 0)
            return fail(QMG_ERR_ARG, "mg_create: bad level %d parameters", l);
        const int cs = lp[l].coarse_storage;
        if (cs != 0 && cs != QMG_H16 && cs != QMG_B16)
            return fail(QMG_ERR_PREC, "mg_create: coarse_storage %d of level %d", cs, l);
        if (cs != 0 && (inner != QMG_C64 || (2 * lp[l].nvec) % 4))
            return fail(QMG_ERR_PREC, "mg_create: 16-bit coarse storage needs complex64 inner precision and N %% 4 == 0");
        if (lp[l].coarse_direct && l + 2 != nlevels)
            return fail(QMG_ERR_ARG, "mg_create: coarse_direct is for the last level entry only (level %d)", l);
        const int ts = lp[l].transfer_storage;
        if (ts != 0 && ts != QMG_H16)
            return fail(QMG_ERR_PREC, "mg_create: transfer_storage %d of level %d", ts, l);
        if (ts != 0 && inner != QMG_C64)
            return fail(QMG_ERR_PREC, "mg_create: a 16-bit transfer basis needs complex64 inner precision");
    }
    auto* mg = new qmg_mg_s();
    mg->s = as_stream(stream);
    mg->inner = inner;
    mg->blas.s = mg->s;
    qmg_status st = mg->blas.init();
    if (st == QMG_OK && hipHostMalloc((void**)&mg->hsc, sizeof(double) * kScal * Blas::kMaxBatch) != hipSuccess)
        st = fail(QMG_ERR_NOMEM, "mg_create: pinned scalars");
    if (st == QMG_OK) st = alloc(mg, (void**)&mg->dsc, sizeof(double) * kScal * Blas::kMaxBatch);
    mg->blas.ss = kScal;
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
    }
    if (st == QMG_OK) st = workspace(mg, 1);
    for (int l = 0; l + 1 < nlevels && st == QMG_OK; ++l)
        st = from_bases ? import_level(mg, l, starts[l])
             : inner == QMG_C128 ? setup_level<double>(mg, l, starts[l], lp[l].setup_iters)
                                 : setup_level<float>(mg, l, starts[l], lp[l].setup_iters);
    // exact coarsest solve: the dense inverse of the full-precision operator
    if (st == QMG_OK && nlevels > 1 && lp[nlevels - 2].coarse_direct) {
        Level& C = mg->lv[nlevels - 1];
        st = dense_inverse(C.op, inner, &C.Ainv, mg->s);
        if (st == QMG_OK) mg->allocs.push_back(C.Ainv);
    }
    // 16-bit storage of coarse operators for the solve: every level was built
    // from the full-precision parent above; now convert the flagged ones
    for (int l = 0; l + 1 < nlevels && st == QMG_OK; ++l) {
        const int cs = lp[l].coarse_storage;
        if (cs == 0) continue;
        Level& C = mg->lv[l + 1];
        const size_t blk = (size_t)C.V * C.dof * C.dof * 16;
        void *X = nullptr, *Y = nullptr;
        hipError_t e = hipMalloc(&X, blk);
        if (e == hipSuccess) e = hipMalloc(&Y, 8 * blk);
        qmg_coarse_op op16 = nullptr;
        if (e != hipSuccess) st = fail(QMG_ERR_NOMEM, "mg_create: 16-bit conversion: %s", hipGetErrorString(e));
        if (st == QMG_OK) st = qmg_coarse_op_export(C.op, X, Y, mg->s);
        if (st == QMG_OK) st = qmg_coarse_op_create(C.dims, C.dof, X, Y, (qmg_prec)cs, mg->s, &op16);
        (void)hipStreamSynchronize(mg->s);
        if (X) (void)hipFree(X);
        if (Y) (void)hipFree(Y);
        if (st == QMG_OK) {
            qmg_coarse_op_destroy(C.op);
            C.op = op16;
        }
    }
    if (st == QMG_OK && fine16) {
        qmg_fine_op f16 = nullptr;
        st = qmg_fine_op_create(dims, gauge, m0, csw, antiperiodic_t, fine_storage, stream, &f16);
        if (st == QMG_OK) {
            qmg_fine_op_destroy(mg->fine_in);
            mg->fine_in = f16;
        }
    }
    // autotune every coarse operator's stencil on the level's own buffers
    for (int l = 1; l < nlevels && st == QMG_OK; ++l) {
        Level& L = mg->lv[l];
        const qmg_prec vp = inner == QMG_C128 ? QMG_C128 : QMG_C64;
        st = qmg_coarse_op_tune(L.op, L.x, nullptr, L.t, nullptr, vp, 0, mg->s, nullptr);
    }
    if (st == QMG_OK) st = take_nonfinite(mg->s, "mg_create");   // the 16-bit conversions above
    if (st != QMG_OK) {
        qmg_mg_destroy(mg);
        return st;
    }
    *out = mg;
    return QMG_OK;
}

extern "C" qmg_status qmg_mg_create(const int dims[4], const void* gauge, double m0, double csw,
                                    int antiperiodic_t, int nlevels, const qmg_level_params* lp,
                                    const void* const* starts, qmg_prec inner, qmg_prec fine_storage,
                                    void* stream, qmg_mg* out) {
    return mg_make(dims, gauge, m0, csw, antiperiodic_t, nlevels, lp, starts, false, inner, fine_storage, stream,
                   out);
}

extern "C" qmg_status qmg_mg_create_from_bases(const int dims[4], const void* gauge, double m0, double csw,
                                               int antiperiodic_t, int nlevels, const qmg_level_params* lp,
                                               const void* const* bases, qmg_prec inner, qmg_prec fine_storage,
                                               void* stream, qmg_mg* out) {
    return mg_make(dims, gauge, m0, csw, antiperiodic_t, nlevels, lp, bases, true, inner, fine_storage, stream, out);
}

static qmg_status check_solve(qmg_mg mg, const void* b, void* x, const qmg_solve_params* p, const char* what) {
    if (!mg || !b || !x || !p) return fail(QMG_ERR_ARG, "%s: NULL argument", what);
    if (b == x) return fail(QMG_ERR_ARG, "%s: b and x alias", what);
    if (!(p->tol > 0) || p->maxit < 1) return fail(QMG_ERR_ARG, "%s: tol/maxit invalid", what);
    if (p->restart != 0 && p->restart != mg->restart)
        return fail(QMG_ERR_ARG, "%s: restart must be 0 or %d", what, mg->restart);
    return QMG_OK;
}

static qmg_status run_solve(qmg_mg mg, const void* b, void* x, int nrhs, const qmg_solve_params* p,
                            qmg_solve_info* info, void* stream) {
    mg->s = as_stream(stream);
    mg->blas.s = mg->s;
    if (info)
        for (int k = 0; k < nrhs; ++k) info[k] = qmg_solve_info{};
    if (nrhs > mg->cap) QMG_TRY(workspace(mg, nrhs));
    mg->nb = nrhs;
    mg->blas.nb = nrhs;
    qmg_status st = mg->inner == QMG_C128 ? solve_impl<double>(mg, b, x, p, info)
                                          : solve_impl<float>(mg, b, x, p, info);
    mg->nb = 1;
    mg->blas.nb = 1;
    // a NaN or Inf met by the batched path's 16-bit rounding of stencil inputs
    if (st == QMG_OK) {
        st = take_nonfinite(mg->s, "mg_gcr_solve");
    } else {   // the solve's own failure is the one reported; the flag is cleared all the same
        char msg[1024];
        snprintf(msg, sizeof msg, "%s", last_error());
        (void)take_nonfinite(mg->s, "mg_gcr_solve");
        st = fail(st, "%s", msg);
    }
    return st;
}

extern "C" qmg_status qmg_mg_gcr_solve(qmg_mg mg, const void* b, void* x, const qmg_solve_params* p,
                                       qmg_solve_info* info, void* stream) {
    QMG_TRY(check_solve(mg, b, x, p, "mg_gcr_solve"));
    return run_solve(mg, b, x, 1, p, info, stream);
}

extern "C" qmg_status qmg_mg_gcr_solve_multi(qmg_mg mg, const void* b, void* x, int nrhs, const qmg_solve_params* p,
                                             qmg_solve_info* info, void* stream) {
    QMG_TRY(check_solve(mg, b, x, p, "mg_gcr_solve_multi"));
    if (nrhs < 1 || nrhs > Blas::kMaxBatch)
        return fail(QMG_ERR_ARG, "mg_gcr_solve_multi: nrhs %d outside [1, %d]", nrhs, Blas::kMaxBatch);
    if (mg->rec || mg->srec) return fail(QMG_ERR_STATE, "mg_gcr_solve_multi: recording is for single solves");
    return run_solve(mg, b, x, nrhs, p, info, stream);
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

extern "C" qmg_status qmg_mg_set_fine_links(qmg_mg mg, int link_reals, void* stream) {
    if (!mg) return fail(QMG_ERR_ARG, "mg_set_fine_links: NULL mg");
    if (link_reals != 18 && link_reals != 12) return fail(QMG_ERR_ARG, "mg_set_fine_links: link_reals %d", link_reals);
    if (mg->fine_in == mg->fine64)
        return fail(QMG_ERR_PREC, "mg_set_fine_links: needs a complex64 or 16-bit fine operator in the K-cycle");
    if (mg->fine_in->link_reals == link_reals) return QMG_OK;
    hipStream_t s = as_stream(stream);
    const qmg_fine_op_s* f = mg->fine64;
    void* G = nullptr;
    QMG_HIP(hipMalloc(&G, (size_t)f->V * 36 * 16));
    qmg_fine_op nf = nullptr;
    qmg_status st = qmg_fine_op_export_links(mg->fine64, G, stream);
    if (st == QMG_OK)
        st = qmg_fine_op_create_ex(f->dims, G, f->m0, f->csw, f->antiperiodic_t, mg->fine_in->storage, link_reals,
                                   stream, &nf);
    (void)hipStreamSynchronize(s);
    (void)hipFree(G);
    if (st != QMG_OK) return st;
    qmg_fine_op_destroy(mg->fine_in);
    mg->fine_in = nf;
    return QMG_OK;
}

extern "C" qmg_status qmg_mg_set_smoother_mr_steps(qmg_mg mg, int steps) {
    if (!mg) return fail(QMG_ERR_ARG, "mg_set_smoother_mr_steps: NULL mg");
    if (steps < 0 || steps > 16) return fail(QMG_ERR_ARG, "mg_set_smoother_mr_steps: steps %d outside [0, 16]", steps);
    mg->ptc_mr = steps;
    return QMG_OK;
}

extern "C" qmg_status qmg_mg_set_sap(qmg_mg mg, const int block[4], int iters, void* stream) {
    if (!mg) return fail(QMG_ERR_ARG, "mg_set_sap: NULL mg");
    if (iters == 0) {
        sap_plan_destroy(mg->sap);
        mg->sap = nullptr;
        mg->sap_iters = 0;
        return QMG_OK;
    }
    if (!block || iters < 1 || iters > 64) return fail(QMG_ERR_ARG, "mg_set_sap: block NULL or iters %d", iters);
    if (mg->inner != QMG_C64) return fail(QMG_ERR_PREC, "mg_set_sap: the Schwarz smoother runs in FP32 (complex64 inner)");
    if (mg->lv.size() < 2) return fail(QMG_ERR_STATE, "mg_set_sap: a single-level solver has no smoother");
    SapPlan* P = nullptr;
    QMG_TRY(sap_plan_create(mg->fine_in, block, &P, as_stream(stream)));
    sap_plan_destroy(mg->sap);
    mg->sap = P;
    mg->sap_iters = iters;
    return QMG_OK;
}

extern "C" qmg_status qmg_mg_set_level_timing(qmg_mg mg, int on) {
    if (!mg) return fail(QMG_ERR_ARG, "mg_set_level_timing: NULL mg");
    mg->timing = on != 0;
    return QMG_OK;
}

// The coarsest level's Schur operator as a dense matrix, when it is small
// (at most kDenseSchur even-site entries): its columns are the Schur stencil
// applied to the unit vectors (one batched application, all columns as batch
// members), transposed to rows.  A coarsest GCR step then applies it with one
// matrix-vector launch instead of the two stencil launches of the Schur form,
// whose tiny grids leave the launches latency-bound.  Same operator, same
// precision; the summation order differs.
constexpr int64_t kDenseSchur = 2048;
qmg_status dense_schur_coarsest(qmg_mg_s* mg) {
    const int nl = (int)mg->lv.size();
    if (nl < 2) return QMG_OK;
    Level& L = mg->lv[nl - 1];
    const int64_t ne = L.n / 2;
    if (L.Ainv || L.Sdense || ne > kDenseSchur || !L.op->eo_even) return QMG_OK;
    const size_t cb = cbytes(mg->inner);
    void *I = nullptr, *C = nullptr, *T = nullptr, *S = nullptr;
    hipError_t e = hipMalloc(&I, cb * ne * ne);
    if (e == hipSuccess) e = hipMalloc(&C, cb * ne * ne);
    if (e == hipSuccess) e = hipMalloc(&T, cb * (L.n - ne) * ne);
    if (e == hipSuccess) e = hipMalloc(&S, cb * ne * ne);
    qmg_status st = e == hipSuccess ? QMG_OK : fail(QMG_ERR_NOMEM, "mg: dense coarsest Schur matrix: %s",
                                                     hipGetErrorString(e));
    const unsigned g = (unsigned)((ne * ne + 255) / 256);
    if (st == QMG_OK) {
        if (mg->inner == QMG_C128) hipLaunchKernelGGL(k_identity<double>, dim3(g), dim3(256), 0, mg->s, (cpx<double>*)I, ne);
        else hipLaunchKernelGGL(k_identity<float>, dim3(g), dim3(256), 0, mg->s, (cpx<float>*)I, ne);
        st = coarse_schur_apply(L.op, I, C, T, mg->inner, (int)ne, mg->s);
    }
    if (st == QMG_OK) {
        if (mg->inner == QMG_C128)
            hipLaunchKernelGGL(k_transpose<double>, dim3(g), dim3(256), 0, mg->s, (cpx<double>*)S, (const cpx<double>*)C, ne);
        else
            hipLaunchKernelGGL(k_transpose<float>, dim3(g), dim3(256), 0, mg->s, (cpx<float>*)S, (const cpx<float>*)C, ne);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(mg->s);
        if (e != hipSuccess) st = fail(QMG_ERR_HIP, "mg: dense coarsest Schur matrix: %s", hipGetErrorString(e));
    }
    for (void* p : {I, C, T})
        if (p) (void)hipFree(p);
    if (st != QMG_OK) {
        if (S) (void)hipFree(S);
        return st;
    }
    L.Sdense = S;
    mg->allocs.push_back(S);
    return QMG_OK;
}

extern "C" qmg_status qmg_mg_set_evenodd(qmg_mg mg, int on, void* stream) {
    if (!mg) return fail(QMG_ERR_ARG, "mg_set_evenodd: NULL mg");
    if (!on) {
        mg->eo = false;
        return QMG_OK;
    }
    if (!mg->fine_in->hsite || !mg->fine64->hsite)
        return fail(QMG_ERR_SHAPE, "mg_set_evenodd: the red-black form needs every fine extent even");
    // the Schur form of every coarse operator a GCR or a smoother runs on
    const int nl = (int)mg->lv.size();
    for (int l = 1; l < nl; ++l) {
        Level& L = mg->lv[l];
        if (L.Ainv || L.op->eo_even) continue;
        QMG_TRY(qmg_coarse_op_prepare_schur(L.op, stream));
    }
    QMG_TRY(dense_schur_coarsest(mg));
    mg->eo = true;
    const qmg_status st = workspace(mg, mg->cap > 0 ? mg->cap : 1);
    if (st != QMG_OK) mg->eo = false;
    return st;
}

extern "C" qmg_status qmg_mg_set_smoother_vectors(qmg_mg mg, int storage, void* stream) {
    (void)stream;
    if (!mg) return fail(QMG_ERR_ARG, "mg_set_smoother_vectors: NULL mg");
    if (storage != 0 && storage != QMG_H16)
        return fail(QMG_ERR_PREC, "mg_set_smoother_vectors: storage %d (0 or QMG_H16)", storage);
    if (storage && mg->fine_in->storage != QMG_H16 && mg->fine_in->storage != QMG_B16)
        return fail(QMG_ERR_PREC, "mg_set_smoother_vectors: 16-bit vectors need a 16-bit fine operator in the K-cycle");
    const bool on = storage != 0;
    if (on == mg->smooth16) return QMG_OK;
    mg->smooth16 = on;
    const qmg_status st = workspace(mg, mg->cap > 0 ? mg->cap : 1);
    if (st != QMG_OK) mg->smooth16 = false;
    return st;
}

extern "C" qmg_status qmg_mg_gcr_solve_record(qmg_mg mg, const void* b, void* x, const qmg_solve_params* p,
                                              qmg_solve_info* info, void* xhist, int maxrec, int* nrec,
                                              void* stream) {
    if (!xhist || maxrec < 1 || !nrec) return fail(QMG_ERR_ARG, "mg_gcr_solve_record: bad record buffer");
    if (!mg) return fail(QMG_ERR_ARG, "mg_gcr_solve_record: NULL mg");
    if (mg->eo) return fail(QMG_ERR_STATE, "mg_gcr_solve_record: records the whole-lattice iterates (red-black form off)");
    mg->rec = xhist;
    mg->rec_max = maxrec;
    const qmg_status st = qmg_mg_gcr_solve(mg, b, x, p, info, stream);
    *nrec = mg->rec_n;
    mg->rec = nullptr;
    mg->rec_max = 0;
    return st;
}

extern "C" qmg_status qmg_mg_gcr_solve_record_smoother(qmg_mg mg, const void* b, void* x, const qmg_solve_params* p,
                                                       qmg_solve_info* info, void* rhist, int maxrec, int* nrec,
                                                       void* stream) {
    if (!rhist || maxrec < 1 || !nrec) return fail(QMG_ERR_ARG, "mg_gcr_solve_record_smoother: bad record buffer");
    if (!mg) return fail(QMG_ERR_ARG, "mg_gcr_solve_record_smoother: NULL mg");
    if (mg->inner != QMG_C64) return fail(QMG_ERR_PREC, "mg_gcr_solve_record_smoother: needs complex64 inner precision");
    if (mg->lv.size() < 2) return fail(QMG_ERR_STATE, "mg_gcr_solve_record_smoother: a single level has no smoother");
    mg->srec = rhist;
    mg->srec_max = maxrec;
    const qmg_status st = qmg_mg_gcr_solve(mg, b, x, p, info, stream);
    *nrec = mg->srec_n;
    mg->srec = nullptr;
    mg->srec_max = 0;
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
        QMG_TRY(qmg_wilson_clover_dslash(mg->fine64, mg->t64, mg->r64, 1, QMG_C128, stream));
        hipLaunchKernelGGL(k_to32, dim3(g), dim3(256), 0, s, (const double2*)mg->r64, r32, nv);
        QMG_LAUNCH_CHECK();
    }
    return QMG_OK;
}
