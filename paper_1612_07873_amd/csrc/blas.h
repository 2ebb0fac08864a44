// BLAS-1 layer of the Krylov solvers: every scalar stays in device memory;
// reductions are two-phase (per-block partials, then one block sums them in a
// fixed order) so results are bitwise repeatable and need no atomics.
//
// Batches: with nb > 1 every call works on nb independent members at once
// (grid dimension y = member).  Member b of a vector argument of length n
// starts at element b*n; multi-vector arguments (Q, Z with stride ld) are
// offset the same way, so a Krylov space of nb members is laid out
// [direction][member][n] with ld = nb*n.  Member b's scalars (inputs and
// results) sit at b*ss doubles after the given pointer.
#pragma once

#include "qmg_internal.h"

namespace qmg {

struct Blas {
    hipStream_t s = nullptr;
    double* partials = nullptr;  // [kMaxBatch][kMaxVals][kMaxBlocks]
    static constexpr int kMaxBlocks = 512;
    static constexpr int kMaxVals = 40;
    static constexpr int kMaxBatch = 64;
    int nb = 1;    // members per call
    int ss = 64;   // doubles between consecutive members' scalars

    qmg_status init();
    void release();

    // Results are written to device doubles at `out`.
    template <typename R> qmg_status dot(const void* a, const void* b, int64_t n, double* out);   // <a,b> (2)
    template <typename R> qmg_status norm2(const void* a, int64_t n, double* out);                // |a|^2 (1)
    // out = [<q,q>, <q,r>.re, <q,r>.im]
    template <typename R> qmg_status dot_norm(const void* q, const void* r, int64_t n, double* out);
    // second phase alone: out[v] = sum of partials[v][g] over g < groups, v < nv
    // (for kernels that leave per-work-group sums in the partials table)
    qmg_status final_sum(int groups, int nv, double* out);
    // out[2i..2i+1] = <Q_i, q>, i < k; Q_i = Q + i*ld
    template <typename R> qmg_status multi_dot(const void* Q, int64_t ld, int k, const void* q, int64_t n, double* out);
    // q -= sum_i beta_i Q_i ; z -= sum_i beta_i Z_i (z may be NULL)
    template <typename R> qmg_status multi_axpy(const double* beta, const void* Q, const void* Z, int64_t ld, int k,
                                                void* q, void* z, int64_t n);
    // GCR step (no-op when s[0] = 0): nq = sqrt(s[0]); alpha = (s[1] + i s[2]) / nq; q /= nq; z /= nq; x += alpha z; r -= alpha q
    template <typename R> qmg_status gcr_update(const double* s3, void* q, void* z, void* x, void* r, int64_t n);
    // MR step with s = dot_norm(Ar, r) = [<Ar,Ar>, <Ar,r>.re, <Ar,r>.im]:
    // alpha = (s1 + i s2)/s0; x = alpha r (first) or x += alpha r; r -= alpha Ar
    // (r may equal rin; the result residual goes to r)
    template <typename R> qmg_status mr_update(const double* s3, const void* rin, void* r, const void* Ar, void* x,
                                               int first, int64_t n);
    // the same two on 16-bit spinor fields (FP16 pairs [site][12], one FP32 scale per
    // site; x stays complex64): q, r and Ar of nsites sites per member
    qmg_status dot_norm_h16(const void* q, const float* qs, const void* r, const float* rs, int64_t nsites,
                            double* out);
    qmg_status mr_update_h16(const double* s3, const void* rin, const float* rins, void* r, float* rs, const void* Ar,
                             const float* Ars, void* x, int first, int64_t nsites);
    // complex64 spinors [nsites][12] -> FP16 pairs with one scale per site (all
    // members' sites at once; a NaN or Inf input is recorded for qmg_sync)
    qmg_status quantize_spinors(const void* in, void* out, float* scale, int64_t nsites);
    // 16-bit half-lattice spinors of every member (nsites each) decoded into
    // whole-lattice complex64 fields [member][2 nsites][12]: site hp[h] takes
    // half-site h, site hq[h] is set to zero
    qmg_status scatter_dequantize(const void* in, const float* scale, const int* hp, const int* hq, void* full,
                                  int64_t nsites);
    // minimal-residual step along d with Ad = A d, s3 = dot_norm(Ad, r): alpha = <Ad,r>/<Ad,Ad>;
    // x = alpha d; rout = r - alpha Ad
    template <typename R> qmg_status dir_step(const double* s3, const void* d, const void* Ad, const void* r, void* x,
                                              void* rout, int64_t n);
    // the same step only where it lowers the residual (<Ad,Ad> - 2 Re <Ad,r> < 0, all
    // finite); elsewhere x = 0, rout = r and the member's s3[cnt] is incremented
    template <typename R> qmg_status dir_step_checked(double* s3, const void* d, const void* Ad, const void* r,
                                                      void* x, void* rout, int64_t n, int cnt);
    template <typename R> qmg_status axpy(double a, const void* x, void* y, int64_t n);       // y += a x
    template <typename R> qmg_status xmy(const void* b, const void* ax, void* r, int64_t n);  // r = b - ax
    template <typename Rs, typename Rd> qmg_status convert(const void* src, void* dst, int64_t n);
    // A whole GCR step after q = A z for vectors of at most kSmall entries, in one
    // work-group: Gram-Schmidt of (q, z) against the k stored pairs (a second
    // pass only when the first cancelled more than half of |q|^2), normalisation,
    // x += alpha z, r -= alpha q; out = [<q,q>, <q,r>.re, <q,r>.im, |r|^2];
    // znext (may be NULL) receives the new r.
    static constexpr int64_t kSmall = 1 << 13;
    // The step also evaluates the stopping test |r| <= tol |b| (|b|^2 at
    // out[bnoff]) into out[okoff + 1 - par], reading the previous launch's
    // flags from out[okoff + par], and counts itself in out[okoff + 2]; once a
    // step has passed it for every member, later launches do nothing.
    template <typename R> qmg_status gcr_step_small(const void* Q, const void* Z, int64_t ld, int k, void* q, void* z,
                                                    void* x, void* r, int64_t n, double* out, void* znext, double tol,
                                                    int okoff, int bnoff, int par);
    // x /= sqrt(nrm2[0])
    template <typename R> qmg_status normalize(void* x, const double* nrm2, int64_t n);
};

}  // namespace qmg
