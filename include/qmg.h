/*
 * qmg.h -- C ABI of the MI355X (gfx950) adaptive-multigrid Wilson-clover library.
 *
 * The method is that of Clark et al., "Accelerating Lattice QCD Multigrid on
 * GPUs Using Fine-Grained Parallelization" (arXiv:1612.07873): the
 * Wilson-clover matrix of Eq. (2), the adaptive geometric setup of Sec. 3.4,
 * the coarse operator of Eq. (3) applied with the fine-grained split of
 * Sec. 6.1-6.4, the transfer operators of Sec. 6.6 and the K-cycle GCR
 * solver of Sec. 7.1.
 *
 * Conventions shared by every entry point
 *  - Pointers to field data are DEVICE pointers owned by the caller, unless a
 *    comment says "host".  The library never frees caller memory; it owns
 *    the memory behind its handles and releases it in *_destroy.
 *  - Complex numbers are interleaved (re, im).  complex128 = 2 x double,
 *    complex64 = 2 x float.
 *  - Lattice dims[4] = {L0, L1, L2, L3}; site index i = x0 + L0*(x1 + L1*(x2 +
 *    L2*x3)); dimension 3 is time (the index decomposition of Sec. 6.1).
 *  - Coarse fields are [V][N] (N = 2*Nvec components per site, n = chi*Nvec + k);
 *    multi-RHS coarse fields are [V][nrhs][N] (each right-hand side's N
 *    components contiguous within a site).
 *  - Direction d = 2*mu (forward hop, multiplies u(x+mu)) or 2*mu+1 (backward).
 *  - Work is enqueued on `stream` (a hipStream_t passed as void*, NULL = the
 *    default stream) and is asynchronous unless stated otherwise.
 *  - Every entry point checks its arguments before enqueuing anything and
 *    returns a qmg_status; on failure qmg_last_error() describes it.  No C++
 *    exception crosses this boundary.  A fault inside an enqueued kernel is
 *    reported by the next synchronising call (qmg_sync).
 *  - Handles are not thread-safe; use one handle from one host thread.
 */
#ifndef QMG_H
#define QMG_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QMG_OK = 0,
    QMG_ERR_ARG = 1,        /* null pointer, bad enum, bad count           */
    QMG_ERR_SHAPE = 2,      /* lattice / block / N inconsistent             */
    QMG_ERR_PREC = 3,       /* precision not supported by this entry point  */
    QMG_ERR_HIP = 4,        /* a HIP runtime call failed                    */
    QMG_ERR_NOMEM = 5,      /* device allocation failed                     */
    QMG_ERR_NOCONV = 6,     /* solver hit its iteration limit               */
    QMG_ERR_NONFINITE = 7,  /* NaN/Inf met in a solver, or by a 16-bit encoder */
    QMG_ERR_STATE = 8       /* handle used in a state that does not allow it */
} qmg_status;

/* Storage / arithmetic precision of a field or operator. */
typedef enum {
    QMG_C128 = 0,   /* complex128, FP64 arithmetic                          */
    QMG_C64 = 1,    /* complex64, FP32 arithmetic                           */
    QMG_H16 = 2,    /* FP16 pairs + FP32 scale, FP32 arithmetic             */
    QMG_B16 = 3     /* BF16 pairs + FP32 scale, FP32 arithmetic             */
} qmg_prec;

typedef struct qmg_coarse_op_s* qmg_coarse_op;
typedef struct qmg_fine_op_s* qmg_fine_op;
typedef struct qmg_transfer_s* qmg_transfer;
typedef struct qmg_mg_s* qmg_mg;
typedef struct qmg_ptc_s* qmg_ptc;

/* Message describing the most recent failure on this host thread. */
const char* qmg_last_error(void);

/* ABI version (major*100 + minor). */
int qmg_version(void);

/* Wait for all work on `stream`; returns QMG_ERR_HIP if an enqueued kernel
 * failed, and QMG_ERR_NONFINITE if a 16-bit encoder (qmg_quantize_sites, the
 * 16-bit storages of qmg_coarse_op_create, or the batched solve's rounding of
 * stencil inputs) met a NaN or Inf input, or a block whose largest entry does
 * not fit FP32, since the last such report: those inputs are never encoded
 * silently.  The record is one word per device, shared by every stream and
 * handle on it, and is cleared when reported.  Blocking calls that encode
 * (qmg_fine_op_create with a 16-bit storage, qmg_transfer_create/import with
 * QMG_H16, qmg_mg_create, the MG solves) report it themselves. */
qmg_status qmg_sync(void* stream);

/* Measurement reference: read `bytes` (a multiple of 16) of the DEVICE buffer
 * once with a plain read-stream kernel (16 work-groups of 256 threads per
 * compute unit, eight 16-byte non-temporal loads in flight per thread),
 * writing one word per work-group to the DEVICE `sink` (sink_words >= 16 x
 * compute units; fewer returns QMG_ERR_ARG).
 * Timed by the caller, it gives the achievable HBM read bandwidth that the
 * read-dominated stencils are compared with. */
qmg_status qmg_stream_read(const void* buf, long long bytes, void* sink, int sink_words, void* stream);

/* ---------------------------------------------------------------------------
 * Coarse operator, Eq. (3) (Sec. 3.4):
 *     y(x) = X(x) u(x) + sum_{d=0..7} Y_d(x) u(x + hop_d),   periodic wrap,
 * with hop_{2mu} = +mu and hop_{2mu+1} = -mu.  X and the eight Y_d are dense
 * complex N x N blocks per coarse site, in the general form the Galerkin
 * product P^+ M P produces (the paper's printed unit diagonal and daggered
 * backward link are special cases of it).
 * ------------------------------------------------------------------------- */

/* Create an operator on a coarse lattice `dims` (every extent >= 2) with N
 * components per site (N even, 2 <= N <= 128) from canonical DEVICE arrays
 *     X [V][N][N] complex128,  Y [8][V][N][N] complex128  (row-major blocks).
 * The data is copied and converted to `storage` in the library's own link
 * layout; the caller may free X and Y once the stream has passed this call.
 * storage:
 *   QMG_C128, QMG_C64  complex128 / complex64 links;
 *   QMG_H16, QMG_B16   FP16 / BF16 (re, im) pairs with one FP32 scale per
 *                      (site, block), block = X or one Y_d, scale = largest
 *                      |re| or |im| in the block (needs N % 4 == 0); the
 *                      arithmetic is FP32 (the paper's 16-bit storage, which
 *                      trades precision for bandwidth).
 * On success *out owns device memory of about 9*V*N*N*(bytes per complex). */
qmg_status qmg_coarse_op_create(const int dims[4], int N, const void* X, const void* Y,
                                qmg_prec storage, void* stream, qmg_coarse_op* out);

/* Write the operator back as canonical complex128 DEVICE arrays X, Y (same
 * shapes as in create), converting from the storage precision. */
qmg_status qmg_coarse_op_export(qmg_coarse_op op, void* X, void* Y, void* stream);

/* Apply Eq. (3): out = Mhat in, for nrhs right-hand sides.  `in` and `out` are
 * DEVICE arrays [nrhs][V][N] (each right-hand side contiguous) in precision
 * `prec`: the operator's storage precision for QMG_C128 / QMG_C64 operators,
 * and QMG_C64 (FP32 vectors) for QMG_H16 / QMG_B16 operators.  One launch
 * covers every right-hand side (the single-RHS kernel; the matrix-core form
 * is qmg_coarse_dslash_mrhs*).  1 <= nrhs <= 1024 (QMG_ERR_ARG otherwise).
 * in and out must not overlap. */
qmg_status qmg_coarse_dslash(qmg_coarse_op op, const void* in, void* out, int nrhs, qmg_prec prec,
                             void* stream);

/* Apply Eq. (3) with 16-bit vectors (QMG_H16 or QMG_B16 operator; `prec` is
 * QMG_H16 or QMG_B16 for the vectors): in/out DEVICE [V][N] 16-bit (re, im)
 * pairs, in_scale/out_scale DEVICE float [V]; value = scale[x] * stored.  The
 * result is accumulated in FP32 and re-scaled per site (out_scale = largest
 * |re| or |im| of the site's N outputs).  Buffers must not overlap. */
qmg_status qmg_coarse_dslash_scaled(qmg_coarse_op op, const void* in, const float* in_scale, void* out,
                                    float* out_scale, qmg_prec prec, void* stream);

/* Eq. (3) for a batch of complex64 fields on the matrix cores: in/out DEVICE
 * complex64 [nrhs][V][N] (each right-hand side contiguous), operator storage
 * QMG_H16 or QMG_B16, N in {16, 32, 48, 64}, nrhs in {8, 16, 32, 64}.  The
 * inputs are rounded to the operator's 16-bit format with one FP32 scale per
 * (site, right-hand side) into staging the operator owns (allocated, or
 * grown, on the first call that needs more), then the multi-RHS kernel of
 * qmg_coarse_dslash_mrhs (FP32 accumulation) writes the complex64 outputs in
 * the same layout.  It is the batched coarse apply of the multi-RHS solve
 * (the paper's multi-RHS future work, Sec. 9).  in and out must not overlap;
 * QMG_ERR_PREC / QMG_ERR_ARG / QMG_ERR_SHAPE as the checks above say. */
qmg_status qmg_coarse_dslash_mrhs_c64(qmg_coarse_op op, const void* in, void* out, int nrhs, void* stream);

/* Convert a DEVICE complex64 field [V][N] to 16-bit pairs `out` [V][N] with
 * per-site scales `scale` [V] (prec QMG_H16 or QMG_B16), and back. */
qmg_status qmg_quantize_sites(const void* in, void* out, float* scale, long long V, int N, qmg_prec prec,
                              void* stream);
qmg_status qmg_dequantize_sites(const void* in, const float* scale, void* out, long long V, int N,
                                qmg_prec prec, void* stream);

/* Apply Eq. (3) to nrhs right-hand sides at once on the matrix cores (the
 * multi-RHS reformulation of Sec. 9): operator with QMG_H16 / QMG_B16
 * storage and N in {16, 32, 48, 64}; nrhs in {8, 16, 32, 64}.
 *   in        DEVICE [V][nrhs][N] 16-bit (re, im) pairs of the operator's format,
 *   in_scale  DEVICE float [V][nrhs] (value = scale * stored; qmg_quantize_sites
 *             with V*nrhs "sites" produces both),
 *   out       DEVICE complex64 [V][nrhs][N].
 * Products in FP16/BF16 on MFMA, FP32 accumulation.  The first call builds a
 * second copy of the links in matrix-core operand order (same size as the
 * 16-bit links). */
qmg_status qmg_coarse_dslash_mrhs(qmg_coarse_op op, const void* in, const float* in_scale, void* out,
                                  int nrhs, void* stream);

/* One persistent launch applying several operators (the levels of a
 * hierarchy, of different size; N in {48, 64}; all with the same 16-bit
 * storage) to nrhs right-hand sides each: the sites of all operators form one
 * work queue that `grid` work-groups (0: as many as are resident on the
 * device at once, at most the total number of sites) walk until it is
 * exhausted.  ops/in/in_scale/out are host arrays of nops (1..4)
 * entries with the same meaning as in qmg_coarse_dslash_mrhs.  Launches no
 * memset and allocates nothing once each operator has been applied in the
 * multi-RHS form before, so it can be captured into a HIP graph. */
qmg_status qmg_coarse_dslash_mrhs_multi(int nops, const qmg_coarse_op* ops, const void* const* in,
                                        const float* const* in_scale, void* const* out, int nrhs, int grid,
                                        void* stream);

/* Tile shape of the multi-RHS kernel: each wave computes 16 rows x
 * (16 * rhs_tiles_per_wave) right-hand sides (1, 2 or 4; 0 = built-in), the
 * nine directions in turn through two LDS buffers; 8 selects the whole-site
 * form instead (each wave 16 rows x all right-hand sides, the link operands
 * of all nine directions in registers and all nine input blocks in LDS at
 * once, so a site waits for memory once).  QMG_ERR_ARG for other values or
 * for 2 / 4 tiles beyond nrhs / 16. */
qmg_status qmg_coarse_op_set_mrhs_tiles(qmg_coarse_op op, int nrhs, int rhs_tiles_per_wave);
/* The tile code in use for nrhs (set, tuned or built-in default) into *tiles. */
qmg_status qmg_coarse_op_get_mrhs_tiles(qmg_coarse_op op, int nrhs, int* tiles);

/* Launch shape of the fine-grained stencil (Sec. 6.2-6.4): each work-group
 * covers `rows` output rows of one coarse site (rows divides N), and the
 * 9N-long row of [X | Y_0 .. Y_7] is split `split` ways across threads, with
 * split dividing the number of 16-byte link chunks in that row.  rows*split
 * must not exceed 1024.  Passing 0 for both restores the built-in choice. */
qmg_status qmg_coarse_op_set_launch(qmg_coarse_op op, int rows, int split);
qmg_status qmg_coarse_op_get_launch(qmg_coarse_op op, int* rows, int* split);

/* Prefetch depth installed by the autotuner (link chunks per thread loaded
 * before the LDS staging barrier; 0 = chosen from the chunks per thread). */
qmg_status qmg_coarse_op_get_prefetch(qmg_coarse_op op, int* pre);

/* Autotune the single-RHS launch (rows, split, prefetch depth) by timing every
 * candidate with HIP events on `stream` (cold != 0: the caches are evicted by
 * reading a 1 GiB buffer before each of nine timed launches, so links stream
 * from HBM; the buffer is allocated for the call), install the fastest (among
 * candidates within 3 % of it: most rows, smallest split, deepest prefetch)
 * on `op`, and remember it for operators of the same shape and precision in
 * this process.  in/out (and scales for 16-bit vectors, vprec
 * QMG_H16/QMG_B16) are valid DEVICE fields as for the apply calls; their
 * contents are overwritten.  Blocks; *best_ms (host, may be NULL) receives the
 * best average time. */
qmg_status qmg_coarse_op_tune(qmg_coarse_op op, const void* in, const float* in_scale, void* out,
                              float* out_scale, qmg_prec vprec, int cold, void* stream, float* best_ms);

/* The same for the multi-RHS kernel's tile shape at this nrhs (candidates 1,
 * 2, 4 right-hand-side tiles per wave as nrhs allows, then the whole-site
 * form 8; a later candidate must be 3 % faster to be taken). */
qmg_status qmg_coarse_op_tune_mrhs(qmg_coarse_op op, const void* in, const float* in_scale, void* out, int nrhs,
                                   int cold, void* stream, float* best_ms);

/* The tuner's choices as a file (the paper's autotuner, Sec. 4, keeps its
 * results; here they also outlive the process).  save writes every entry of
 * this process's cache to the text file at `path` (host string), headed by
 * the current device's architecture name and the HIP runtime version;
 * load merges the entries of such a file into the cache, and refuses
 * (QMG_ERR_STATE) a file written for another architecture or runtime, so a
 * later qmg_coarse_op_tune / _tune_mrhs on the same shape installs the stored
 * launch without timing.  *entries (host, may be NULL) receives the number of
 * entries written / read.  QMG_ERR_ARG if the file cannot be opened, written
 * or parsed.  clear empties the in-process cache. */
qmg_status qmg_tune_cache_save(const char* path, int* entries);
qmg_status qmg_tune_cache_load(const char* path, int* entries);
qmg_status qmg_tune_cache_clear(void);

void qmg_coarse_op_destroy(qmg_coarse_op op);

/* ---------------------------------------------------------------------------
 * Red-black (even-odd) form of Eq. (3) (Sec. 3.3, used on every level in
 * Sec. 7.1): with the site-local block X and the hops Y,
 *     S = X_ee - Y_eo X_oo^-1 Y_oe,   S x_e = b_e - Y_eo X_oo^-1 b_o,
 *     x_o = X_oo^-1 (b_o - Y_oe x_e).
 * qmg_coarse_op_prepare_schur builds it (blocks): X_oo^-1 per odd site and the
 * products X_oo^-1 Y_d in FP64 (Gauss-Jordan elimination with partial
 * pivoting), stored with the operator's storage as two operators on V/2 sites
 * (about the size of the operator itself).  Needs every extent even
 * (QMG_ERR_SHAPE); the other calls return QMG_ERR_STATE before it.
 * Half-lattice fields [nrhs][V/2][N] (sites of one parity in lattice order),
 * whole-lattice [nrhs][V][N]; vectors complex128 for QMG_C128 storage and
 * complex64 otherwise; 1 <= nrhs <= 1024; inputs and outputs must not overlap.
 * S is two launches over V/2 sites that read 17 of the 18 half-site link
 * blocks one application of Eq. (3) reads.
 * ------------------------------------------------------------------------- */
qmg_status qmg_coarse_op_prepare_schur(qmg_coarse_op op, void* stream);
/* out_e = S in_e. */
qmg_status qmg_coarse_dslash_schur(qmg_coarse_op op, const void* in_e, void* out_e, int nrhs, qmg_prec prec,
                                   void* stream);
/* bhat_e = b_e - Y_eo X_oo^-1 b_o for whole-lattice b. */
qmg_status qmg_coarse_schur_source(qmg_coarse_op op, const void* b, void* bhat_e, int nrhs, qmg_prec prec,
                                   void* stream);
/* Whole-lattice x: x_e copied, x_o = X_oo^-1 (b_o - Y_oe x_e). */
qmg_status qmg_coarse_schur_reconstruct(qmg_coarse_op op, const void* x_e, const void* b, void* x, int nrhs,
                                        qmg_prec prec, void* stream);

/* ---------------------------------------------------------------------------
 * Fine Wilson-clover operator, Eq. (2) (Sec. 3.2):
 *   M psi(x) = (4 + m0 + A(x)) psi(x)
 *       - 1/2 sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu) + (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu) ]
 * Chiral gamma basis (gamma_5 = diag(1,1,-1,-1)); periodic space and, when
 * antiperiodic_t != 0, antiperiodic time.  A(x) is the clover term
 * (i c_sw/2) sum_{mu<nu} sigma_{mu nu} (x) (Q_{mu nu} - Q_{mu nu}^+)/8 built
 * from the clover-leaf sum Q; c_sw = 0 gives the plain Wilson operator.
 * ------------------------------------------------------------------------- */

/* Create the operator from the canonical DEVICE gauge field
 *     gauge [4][V][3][3] complex128  (U_mu(x), row-major colour matrices),
 * every extent >= 2.  The clover term is computed on the device here.  The
 * gauge array may be freed once the stream has passed this call.
 * storage: QMG_C128, QMG_C64, or QMG_H16 / QMG_B16 (the 16-bit precision form
 * of Sec. 4: link entries as FP16 / BF16 pairs with no scale, which assumes
 * unitary links, |entry| <= 1; the clover term as 16-bit pairs with one FP32
 * scale per (chirality, site), built in FP64 first; FP32 arithmetic). */
qmg_status qmg_fine_op_create(const int dims[4], const void* gauge, double m0, double csw,
                              int antiperiodic_t, qmg_prec storage, void* stream, qmg_fine_op* out);

/* As qmg_fine_op_create, with the links stored as link_reals real numbers
 * each: 18 (all nine entries), or 12 (rows 0 and 1 only; the kernels rebuild
 * row 2 as the complex conjugate of the cross product of the other two, which
 * holds for SU(3) links -- the gauge compression of Sec. 4 and 7.1, here to 12
 * reals; 8-real compression is not provided).  12 needs QMG_C64, QMG_H16 or
 * QMG_B16 storage and cuts the link bytes by a third; the links must be
 * special unitary (det = 1) for the rebuilt row to be right. */
qmg_status qmg_fine_op_create_ex(const int dims[4], const void* gauge, double m0, double csw, int antiperiodic_t,
                                 qmg_prec storage, int link_reals, void* stream, qmg_fine_op* out);

/* out = M in for nrhs fields; in/out DEVICE [nrhs][V][4][3] in the operator's
 * storage precision (complex64 for the 16-bit storages); one launch covers
 * every field; 1 <= nrhs <= 1024; in and out must not overlap. */
qmg_status qmg_wilson_clover_dslash(qmg_fine_op op, const void* in, void* out, int nrhs, qmg_prec prec,
                                    void* stream);

/* The same with 16-bit vectors (operator storage QMG_H16 / QMG_B16; prec =
 * QMG_H16 or QMG_B16 names the vector format): in/out DEVICE [V][12] 32-bit
 * words, each an (re, im) pair of the 16-bit format, value = scale[site] *
 * stored; in_scale/out_scale DEVICE float [V].  The output scale of a site is
 * the largest |re| or |im| of its 12 components (0 for a zero spinor).
 * Arithmetic in FP32.  Buffers must not overlap. */
qmg_status qmg_wilson_clover_dslash_scaled(qmg_fine_op op, const void* in, const float* in_scale, void* out,
                                           float* out_scale, qmg_prec prec, void* stream);

/* Write the clover term as dense DEVICE complex128 [V][12][12] (row/column
 * index 3*spin + colour). */
qmg_status qmg_fine_op_export_clover(qmg_fine_op op, void* A, void* stream);

/* Write the links the operator holds (after rounding to its storage) as
 * DEVICE complex128 [4][V][3][3], in the layout of qmg_fine_op_create's
 * gauge argument (the antiperiodic time sign taken back out). */
qmg_status qmg_fine_op_export_links(qmg_fine_op op, void* gauge, void* stream);

void qmg_fine_op_destroy(qmg_fine_op op);

/* Schwarz alternating procedure (the domain-decomposition smoother whose
 * blocks relax independently, with no global reduction): x = one sweep from
 * x = 0 for M x = r.  The lattice is cut into blocks of extent block[4]
 * (each dimension an even number >= 2 of blocks; at most 256 sites per
 * block) coloured by the parity of their block coordinates; for colour 0,
 * then 1, every block B of that colour takes `iters` (1..64) minimal-residual
 * steps on M_BB d = (r - M x)_B from d = 0 (M_BB: Eq. (2) with the hops
 * leaving B dropped; each block its own step lengths) and x += d on B.  One
 * launch per colour; the block's links and residual stay in LDS.  r, x DEVICE
 * complex64 [nrhs][V][4][3]; operator storage QMG_C64, QMG_H16 or QMG_B16
 * (FP32 arithmetic).  Blocks (it builds the block tables). */
qmg_status qmg_wilson_clover_sap(qmg_fine_op op, const int block[4], int iters, const void* r, void* x, int nrhs,
                                 void* stream);

/* ---------------------------------------------------------------------------
 * Red-black (even-odd) form of Eq. (2) (Sec. 3.3; the solver of Sec. 7.1
 * uses it on every level).  Every hop joins sites of opposite parity
 * p(x) = (x0 + x1 + x2 + x3) mod 2, so with the site-local block
 * C(x) = 4 + m0 + A(x) and the hop term D (the sum over mu of Eq. 2, its
 * -1/2 included) M x = b is solved through the Schur complement on the even
 * sites,
 *     S = C_ee - D_eo C_oo^-1 D_oe,   S x_e = b_e - D_eo C_oo^-1 b_o,
 *     x_o = C_oo^-1 (b_o - D_oe x_e).
 * Available when every lattice extent is even (QMG_ERR_SHAPE otherwise); the
 * operator then holds C^-1 (inverted per site in FP64 at creation, stored as
 * the clover term is).  Half-lattice fields hold the sites of one parity in
 * lattice order, [nrhs][V/2][4][3] (the half-lattice index of site x is
 * x >> 1); whole-lattice fields are [nrhs][V][4][3].  Vectors are complex128
 * for a QMG_C128 operator and complex64 otherwise; 1 <= nrhs <= 1024.  The
 * calls use a half-lattice scratch the operator owns (grown on first need,
 * which synchronises the stream).  Inputs and outputs must not overlap.
 * ------------------------------------------------------------------------- */

/* out_e = S in_e. */
qmg_status qmg_wilson_clover_schur(qmg_fine_op op, const void* in_e, void* out_e, int nrhs, qmg_prec prec,
                                   void* stream);

/* out_e = S in_e on 16-bit half-lattice vectors (Sec. 7.1: the fine-level
 * smoother in half precision): in_e, out_e DEVICE [nrhs][V/2][12] FP16
 * (re, im) pairs with one FP32 scale per site (in_scale, out_scale
 * [nrhs][V/2], the layout of qmg_quantize_sites); FP32 arithmetic, the odd
 * intermediate also rounded to 16 bits.  Needs an operator with 16-bit
 * storage (QMG_ERR_PREC otherwise). */
qmg_status qmg_wilson_clover_schur_scaled(qmg_fine_op op, const void* in_e, const float* in_scale, void* out_e,
                                          float* out_scale, int nrhs, void* stream);
/* bhat_e = b_e - D_eo C_oo^-1 b_o for whole-lattice b. */
qmg_status qmg_wilson_clover_schur_source(qmg_fine_op op, const void* b, void* bhat_e, int nrhs, qmg_prec prec,
                                          void* stream);
/* Whole-lattice x: x_e copied from the half-lattice x_e, x_o = C_oo^-1 (b_o - D_oe x_e). */
qmg_status qmg_wilson_clover_schur_reconstruct(qmg_fine_op op, const void* x_e, const void* b, void* x, int nrhs,
                                               qmg_prec prec, void* stream);

/* qmg_wilson_clover_schur for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels, with the odd half-lattice intermediate in a
 * fixed 16 MiB device array the library holds on every device it runs on
 * until the process ends, instead of the operator's grown scratch.  The call
 * allocates and frees nothing.  QMG_ERR_ARG if nrhs * V/2 * 12 complex
 * entries (16 bytes each for QMG_C128, 8 otherwise) exceed 16 MiB (e.g. up to
 * 16^3x32 in complex128 with one right-hand side).  Every call on a device
 * shares that device's array: calls that overlap in time on one device (on
 * different streams or host threads) race and must be serialised by the
 * caller.  Arguments and other errors as for qmg_wilson_clover_schur. */
qmg_status qmg_wilson_clover_schur_noalloc(qmg_fine_op op, const void* in_e, void* out_e, int nrhs, qmg_prec prec,
                                           void* stream);

/* ---------------------------------------------------------------------------
 * Transfer operators (Sec. 3.4 step 3, Sec. 6.6).  The near-null vectors are
 * cut into hypercubic aggregates of extent block[4]; within each aggregate
 * the two chirality halves (fine level: spins {0,1} and {2,3}; coarse
 * parent: components n < dof/2 and n >= dof/2) of every vector are
 * orthonormalised separately by modified Gram-Schmidt in vector order (each
 * projection done twice; R with real positive diagonal).  This gives the
 * prolongator P, N = 2*nvec coarse components per aggregate, and the
 * restrictor R = P^+:
 *   (P u)(x)_f = sum_k V(x)_{f,k} u(xc(x))_{chi(f)*nvec + k}
 *   (R psi)(xc)_{chi*nvec + k} = sum_{x in xc} sum_{f: chi(f) = chi} conj(V(x)_{f,k}) psi(x)_f
 * ------------------------------------------------------------------------- */

/* Build P from DEVICE near-null vectors nullvecs [nvec][V][fine_dof]
 * complex128 (fine_dof = 12 on the fine lattice, the parent's N on a coarse
 * one).  block must divide fine_dims with every coarse extent >= 2.  The
 * orthonormalisation runs in FP64; storage (QMG_C128, QMG_C64, or QMG_H16:
 * FP16 pairs with no scale, the entries being at most 1 in modulus) is the
 * basis prolong/restrict use for complex64 fields (complex128 fields always
 * use the FP64 basis).  Blocks this call
 * until the basis is built (it checks the rank on the host): returns
 * QMG_ERR_ARG if a vector is linearly dependent (relative residual norm
 * < 1e-10) on some aggregate. */
qmg_status qmg_transfer_create(const int fine_dims[4], int fine_dof, const int block[4], int nvec,
                               const void* nullvecs, qmg_prec storage, void* stream,
                               qmg_transfer* out);

/* Rebuild a transfer from a basis that is already block-orthonormal, as
 * qmg_transfer_export writes it (DEVICE complex128 [V][fine_dof][nvec]):
 * no orthonormalisation, the FP64 basis is copied as given, so a transfer
 * exported and imported again prolongs and restricts bit for bit as the
 * original.  Checkpoint/resume of a hierarchy (setup amortised over solves,
 * Sec. 3.4).  Same shape checks and errors as qmg_transfer_create; a basis
 * that is not block-orthonormal is not detected (R P then differs from 1).
 * Blocks until the copy is done. */
qmg_status qmg_transfer_import(const int fine_dims[4], int fine_dof, const int block[4], int nvec,
                               const void* basis, qmg_prec storage, void* stream, qmg_transfer* out);

/* Coarse lattice extents and N = 2*nvec of the transfer (host outputs). */
qmg_status qmg_transfer_coarse_dims(qmg_transfer t, int cdims[4], int* N);

/* Write the FP64 basis V as a DEVICE complex128 array [V][fine_dof][nvec]. */
qmg_status qmg_transfer_export(qmg_transfer t, void* basis, void* stream);

/* fine_out [nrhs][V][fine_dof] = P coarse_in [nrhs][Vc][N]; DEVICE fields,
 * precision p (QMG_C128, or QMG_C64 when the transfer was created with
 * QMG_C64); one launch covers every right-hand side; 1 <= nrhs <= 1024. */
qmg_status qmg_prolong(qmg_transfer t, const void* coarse_in, void* fine_out, int nrhs, qmg_prec p,
                       void* stream);

/* coarse_out [nrhs][Vc][N] = R fine_in [nrhs][V][fine_dof]; same rules. */
qmg_status qmg_restrict(qmg_transfer t, const void* fine_in, void* coarse_out, int nrhs, qmg_prec p,
                        void* stream);

void qmg_transfer_destroy(qmg_transfer t);

/* ---------------------------------------------------------------------------
 * Galerkin coarse operator (Sec. 3.4 step 4): Mhat = P^+ M P, assembled in
 * FP64 by hop direction into the X / Y_d blocks of Eq. (3).  The parent is
 * either the fine Wilson-clover operator (`fine`) or a coarse operator
 * (`parent`) -- exactly one must be non-NULL -- defined on the transfer's
 * fine lattice.  Requires parent dof x N <= 4096.  Blocks until the
 * operator is built; *out is a new coarse operator in `storage`
 * (QMG_C128 or QMG_C64).
 * ------------------------------------------------------------------------- */
qmg_status qmg_build_coarse_op(qmg_transfer t, qmg_fine_op fine, qmg_coarse_op parent,
                               qmg_prec storage, void* stream, qmg_coarse_op* out);

/* ---------------------------------------------------------------------------
 * Multigrid hierarchy and K-cycle GCR solver (Sec. 3.4 setup, Sec. 7.1).
 * ------------------------------------------------------------------------- */

/* Parameters of level l (the level that is coarsened), caller-owned, copied. */
typedef struct {
    int block[4];        /* aggregate extents (must divide the level's lattice, coarse extents >= 2) */
    int nvec;            /* near-null vectors; the next level has N = 2*nvec (1..64) */
    int setup_iters;     /* GCR(10) steps relaxing A x = 0 per vector (0: use the starts as given) */
    int smoother_steps;  /* MR steps before and after the coarse correction (4) */
    double coarse_tol;   /* relative tolerance of the GCR solve on the next level (0.25) */
    int coarse_maxit;    /* its iteration cap (10 intermediate, 100 coarsest) */
    int coarse_storage;  /* storage of the next level's operator in the solve: 0 = the inner
                            precision, QMG_H16 / QMG_B16 = 16-bit links with FP32 scales
                            (FP32 vectors; inner precision must be QMG_C64) */
    int coarse_direct;   /* last level entry only: solve the coarsest level exactly with a dense
                            inverse of its operator, built at setup by Gauss-Jordan elimination
                            in FP64 (at most 4096 coarsest unknowns) and applied in the inner
                            precision, instead of the paper's GCR (coarse_tol/coarse_maxit are
                            then unused); 0 = GCR */
    int transfer_storage; /* storage of this level's transfer basis for the solve's prolongation and
                            restriction: 0 = the inner precision, QMG_H16 = FP16 pairs with no
                            scale (entries of a block-orthonormal basis are at most 1 in modulus;
                            inner precision must be QMG_C64); the Galerkin build always uses the
                            FP64 basis */
} qmg_level_params;

typedef struct {
    double tol;   /* stop when |b - M x| <= tol |b| (true residual, FP64) */
    int restart;  /* 0 or 10: outer GCR Krylov space */
    int maxit;    /* cap on outer steps */
} qmg_solve_params;

typedef struct {
    int outer_iters;          /* outer GCR steps */
    int level_iters[4];       /* [0] = outer steps, [l] = total GCR steps on level l */
    int restarts;             /* true-residual restarts that did not converge */
    int converged;
    double true_rel_residual; /* |b - M x| / |b| from the FP64 operator */
    double seconds;           /* host wall time of the solve */
    int smoother_fallbacks;   /* learned-smoother applications replaced by MR */
    double level_seconds[4];  /* with qmg_mg_set_level_timing on: device time spent on each level,
                                 exclusive of the coarser ones ([0]: the rest of the solve: outer
                                 GCR, fine-level smoothing, transfers); -1 in [0] if some coarse
                                 solves were not timed; 0 otherwise */
} qmg_solve_info;

/* Build the hierarchy on DEVICE gauge [4][V][3][3] complex128 (as in
 * qmg_fine_op_create): nlevels (1..4) levels, lp[l] for l < nlevels-1, and
 * starts[l] = DEVICE complex128 [nvec_l][V_l][dof_l] random start vectors of
 * the near-null relaxation on level l (dof_0 = 12, dof_l = 2*nvec_{l-1}).
 * `inner` (QMG_C64 or QMG_C128) is the precision of the K-cycle, the
 * relaxation and the coarse operators; the outer GCR and the true residual
 * always use FP64.  `fine_storage` is the storage of the fine operator used
 * inside the K-cycle (smoothing and the residual handed to level 1): 0 or
 * `inner` for the inner precision, QMG_H16 / QMG_B16 for 16-bit links and
 * clover with complex64 vectors (inner must then be QMG_C64).  The setup
 * (relaxation, Galerkin build) always runs on the inner-precision operators;
 * 16-bit storages are made from them afterwards.  Every coarse operator's
 * stencil launch is autotuned here.  Blocks until the setup is complete. */
qmg_status qmg_mg_create(const int dims[4], const void* gauge, double m0, double csw, int antiperiodic_t,
                         int nlevels, const qmg_level_params* lp, const void* const* starts,
                         qmg_prec inner, qmg_prec fine_storage, void* stream, qmg_mg* out);

/* Resume a hierarchy from a checkpoint: as qmg_mg_create, with bases[l] =
 * the FP64 transfer basis of level l as qmg_transfer_export writes it (DEVICE
 * complex128 [V_l][dof_l][nvec_l], from the transfer that qmg_mg_level
 * returns) in place of the start vectors.  The near-null relaxation is
 * skipped (setup_iters unused) and the Galerkin build, the 16-bit
 * conversions and the autotuning run as in qmg_mg_create, so the coarse
 * operators come out bit for bit as in the hierarchy the bases were taken
 * from (same gauge field, m0, csw, level parameters and precisions).  The
 * solver settings changed after creation (qmg_mg_set_*) are not part of the
 * hierarchy and are set again by the caller.  Blocks. */
qmg_status qmg_mg_create_from_bases(const int dims[4], const void* gauge, double m0, double csw,
                                    int antiperiodic_t, int nlevels, const qmg_level_params* lp,
                                    const void* const* bases, qmg_prec inner, qmg_prec fine_storage,
                                    void* stream, qmg_mg* out);

/* Solve M x = b: b, x DEVICE complex128 [V][4][3] (x is overwritten, start
 * x = 0).  Blocks; returns QMG_ERR_NOCONV if maxit is reached and
 * QMG_ERR_NONFINITE on NaN/Inf; *info (host, may be NULL) is filled in any case. */
qmg_status qmg_mg_gcr_solve(qmg_mg mg, const void* b, void* x, const qmg_solve_params* p,
                            qmg_solve_info* info, void* stream);

/* Solve M x_k = b_k for nrhs (1..64) right-hand sides together: b, x DEVICE
 * complex128 [nrhs][V][4][3]; info: host array of nrhs entries (may be NULL).
 * The members run in lock step (the multi-RHS form the paper names as future
 * work, Sec. 9): every launch covers all of them, each keeps its own Krylov
 * space, step lengths and FP64 stopping test, and a level's GCR ends when
 * every member meets its tolerance, so one member may take more inner steps
 * than it would alone.  With a 16-bit coarse operator (level params'
 * coarse_storage) and nrhs in {8, 16, 32, 64}, the coarse stencil of that
 * level runs on the matrix cores (qmg_coarse_dslash_mrhs) after rounding the
 * batch's vectors to 16 bits with one scale per (site, member).  A learned
 * smoother is applied to every member and kept only if it lowers every
 * member's residual (else MR for the batch; info's smoother_fallbacks counts
 * the members whose residual grew).  The solve workspace grows to nrhs members
 * on first use and is kept (about nrhs times the single-solve workspace).
 * outer_iters and level_iters are shared by the batch.  Blocks; returns
 * QMG_ERR_NOCONV unless every member converged. */
qmg_status qmg_mg_gcr_solve_multi(qmg_mg mg, const void* b, void* x, int nrhs, const qmg_solve_params* p,
                                  qmg_solve_info* info, void* stream);

/* Store the links of the fine operator the K-cycle uses (the smoother's and
 * the residual's, in the inner or 16-bit precision) with link_reals reals
 * each, 18 or 12 (qmg_fine_op_create_ex), rebuilding it from the hierarchy's
 * FP64 links; the FP64 operator of the outer solve keeps all 18.  Needs a
 * complex64 inner precision (QMG_ERR_PREC).  Blocks. */
qmg_status qmg_mg_set_fine_links(qmg_mg mg, int link_reals, void* stream);

/* Level-0 smoother: one sweep of the Schwarz alternating procedure (as
 * qmg_wilson_clover_sap, `iters` MR steps per block) in place of MR, followed
 * by the residual r - A x the K-cycle continues with; iters = 0 returns to MR.
 * The learned smoother, when attached, takes precedence.  Needs complex64
 * inner precision (QMG_ERR_PREC) and a block that fits the lattice
 * (QMG_ERR_SHAPE, as qmg_wilson_clover_sap). */
qmg_status qmg_mg_set_sap(qmg_mg mg, const int block[4], int iters, void* stream);

/* Level-0 MR smoother vectors in the red-black form: 0 = the inner precision,
 * QMG_H16 = the Schur system's source, residual and intermediates as FP16
 * pairs with one FP32 scale per site (the paper's half-precision fine-level
 * smoother, Sec. 7.1), the correction kept in complex64.  Needs a 16-bit fine
 * operator in the K-cycle (QMG_ERR_PREC); takes effect while the red-black
 * form is on (the whole-lattice MR is unchanged); regrows the solve
 * workspace. */
qmg_status qmg_mg_set_smoother_vectors(qmg_mg mg, int storage, void* stream);

/* Time every coarse-grid solve of the following solves with HIP events on
 * the solve's stream (on != 0) and report each level's share in
 * info.level_seconds: the time-per-level picture of the paper's strong-scaling
 * study (Sec. 7.2), on one GPU.  Adds two event records per coarse solve;
 * off by default. */
qmg_status qmg_mg_set_level_timing(qmg_mg mg, int on);

/* Red-black preconditioning on every level (Sec. 7.1, with the Schur
 * complements of Sec. 3.3), on != 0; 0 switches it off.  With it on: the
 * smoother of every level is MR on that level's Schur system (the odd sites
 * back-substituted), every coarse-grid GCR runs on the next level's Schur
 * system (preconditioned by the even part of its K-cycle applied to (r_e, 0);
 * an exact coarsest solve, coarse_direct, stays on the whole coarsest
 * lattice), and the outer FP64 FGCR runs on the fine Schur system, stopping
 * when that residual reaches tol |b|; x_o is back-substituted at every
 * reliable update, whose true residual is that of the whole system.  Needs
 * every extent even on every level (QMG_ERR_SHAPE).  The first call builds
 * the coarse operators' Schur form (qmg_coarse_op_prepare_schur) and grows
 * the solve workspace by about half; blocks.  The learned smoother, when
 * attached, keeps acting on the whole fine lattice. */
qmg_status qmg_mg_set_evenodd(qmg_mg mg, int on, void* stream);

/* Borrowed views of level l: lattice dims, components per site, its coarse
 * operator (NULL on level 0) and the transfer to level l+1 (NULL on the
 * coarsest).  The handles stay owned by the hierarchy. */
qmg_status qmg_mg_level(qmg_mg mg, int level, int dims[4], int* dof, qmg_coarse_op* op,
                        qmg_transfer* to_next);

/* Borrowed FP64 fine operator of the hierarchy. */
qmg_status qmg_mg_fine_op(qmg_mg mg, qmg_fine_op* fine64);

void qmg_mg_destroy(qmg_mg mg);

/* ---------------------------------------------------------------------------
 * Mixed-precision BiCGStab with reliable updates: the Krylov solver the paper
 * compares its multigrid with (Sec. 3.3: BiCGStab with red-black
 * preconditioning; Sec. 7.1: 16-bit precision with FP64 reliable updates).
 * BiCGStab (van der Vorst) runs with the low-precision operator `lo` and
 * accumulates a low-precision correction; when the iterated residual falls
 * below delta times its largest value since the last update (or reaches the
 * target), the correction is added to the FP64 solution and the true
 * residual is recomputed with the FP64 operator `hi` and the iteration goes
 * on from it, keeping its search direction.  It stops when the FP64 true
 * residual of the iterated system is at most tol |b|; with the red-black form
 * that system is the fine Schur complement S x_e = b_e - D_eo C_oo^-1 b_o and
 * x_o is back-substituted in FP64 at the end.  info: outer_iters = BiCGStab
 * steps (two operator applications each), restarts = reliable updates,
 * true_rel_residual = |b - M x| / |b| of the whole system (FP64).
 * ------------------------------------------------------------------------- */
typedef struct qmg_bicgstab_s* qmg_bicgstab;

typedef struct {
    double tol;     /* stop when the FP64 true residual <= tol |b| */
    int maxit;      /* cap on BiCGStab steps */
    double delta;   /* reliable-update threshold, 0 < delta < 1 (e.g. 0.1) */
} qmg_bicgstab_params;

/* hi: a QMG_C128 operator; lo: an operator on the same lattice, m0, c_sw and
 * boundary in any storage (QMG_C128 gives a plain FP64 BiCGStab); both
 * borrowed.  evenodd != 0 selects the red-black form (every extent even).
 * Allocates the solver's workspace (about 12 fields). */
qmg_status qmg_bicgstab_create(qmg_fine_op hi, qmg_fine_op lo, int evenodd, void* stream, qmg_bicgstab* out);
/* Solve M x = b: b, x DEVICE complex128 [V][4][3] (x overwritten).  Blocks;
 * QMG_ERR_NOCONV if maxit is reached first, QMG_ERR_NONFINITE on NaN/Inf;
 * *info (host, may be NULL) is filled in any case. */
qmg_status qmg_bicgstab_solve(qmg_bicgstab h, const void* b, void* x, const qmg_bicgstab_params* p,
                              qmg_solve_info* info, void* stream);
void qmg_bicgstab_destroy(qmg_bicgstab h);

/* ---------------------------------------------------------------------------
 * Learned smoother: a gauge-equivariant parallel-transport convolution
 * network, two linear layers 1 -> hidden -> 1 channels (the paper's smoother
 * is MR, Sec. 7.1; this network replaces it, with MR as the fallback):
 *   (T_0 h)(x) = h(x), (T_{+mu} h)(x) = U_mu(x) h(x+mu), (T_{-mu} h)(x) = U_mu(x-mu)^+ h(x-mu)
 *   (with the operator's time boundary sign), paths p = 0, 1+2mu (+mu), 2+2mu (-mu);
 *   h'_a(x) = sum_b sum_p W[p][a][b] (T_p h_b)(x), W[p][a][b] complex 4x4 on spin;
 *   loss L = sum_i |N(r_i) - e_i|^2 / |e_i|^2.
 * Weights W1 [9][hidden][1][4][4], W2 [9][1][hidden][4][4] complex64 (DEVICE).
 * Fields r, e, y are DEVICE complex64 [V][4][3].
 * ------------------------------------------------------------------------- */

/* Network on the lattice of `links` (a complex64-storage fine operator,
 * borrowed: it must outlive the network), 1 <= hidden <= 16; weights start at 0. */
qmg_status qmg_ptc_create(qmg_fine_op links, int hidden, void* stream, qmg_ptc* out);
/* Copy weights in (resets the Adam state) or out. */
qmg_status qmg_ptc_set_weights(qmg_ptc net, const void* W1, const void* W2, void* stream);
qmg_status qmg_ptc_get_weights(qmg_ptc net, void* W1, void* W2, void* stream);
/* Adam state for checkpointing training: first and second moments m1, v1
 * (layer 1) and m2, v2 (layer 2), DEVICE float32 pairs shaped like the
 * weights (real and imaginary parts are independent parameters), and the
 * number of Adam steps taken (its bias corrections).  Restore after
 * qmg_ptc_set_weights, which clears the state. */
qmg_status qmg_ptc_get_adam(qmg_ptc net, void* m1, void* v1, void* m2, void* v2, int* steps, void* stream);
qmg_status qmg_ptc_set_adam(qmg_ptc net, const void* m1, const void* v1, const void* m2, const void* v2, int steps,
                            void* stream);
/* y = N(r); r and y must not overlap. */
qmg_status qmg_ptc_forward(qmg_ptc net, const void* r, void* y, void* stream);
/* Add the loss |N(r) - e|^2/|e|^2 of one pair and its gradients
 * G = dL/dRe W + i dL/dIm W to the network's accumulators. */
qmg_status qmg_ptc_accumulate_grad(qmg_ptc net, const void* r, const void* e, void* stream);
/* Residual form of the loss for one residual r: add |r - M N(r)|^2/|r|^2
 * (M = the Wilson-clover operator the network was created on) and its
 * gradients, back-propagated through M^+ = gamma5 M gamma5. */
qmg_status qmg_ptc_accumulate_grad_residual(qmg_ptc net, const void* r, void* stream);
/* Clear the gradient and loss accumulators. */
qmg_status qmg_ptc_zero_grad(qmg_ptc net, void* stream);
/* Copy the accumulated gradients (DEVICE, same shapes as the weights) and the
 * accumulated loss (host double); blocks. */
qmg_status qmg_ptc_get_grad(qmg_ptc net, void* G1, void* G2, double* loss, void* stream);
/* One Adam step on the real and imaginary parts with the accumulated gradients. */
qmg_status qmg_ptc_adam_step(qmg_ptc net, float lr, float beta1, float beta2, float eps, void* stream);
void qmg_ptc_destroy(qmg_ptc net);

/* Use `net` (NULL: MR) as the level-0 smoother of an FP32-inner hierarchy.
 * Each application keeps the network's output d = N(r) only if
 * |r - M d| < |r|, and then takes it with the minimal-residual step length,
 * x = alpha d, alpha = <M d, r>/|M d|^2; otherwise (including NaN/Inf) the
 * application uses MR instead (counted in smoother_fallbacks).  The network
 * is borrowed and must outlive its use. */
qmg_status qmg_mg_set_smoother(qmg_mg mg, qmg_ptc net);

/* MR steps (0..16, default 0) the learned smoother takes after an accepted
 * network step, on the residual the network left: x = alpha N(r) + MR_k(r -
 * alpha M N(r)).  Its kr2/kt workspace is the post-smoothing scratch of
 * level 0, which is free while the smoother runs. */
qmg_status qmg_mg_set_smoother_mr_steps(qmg_mg mg, int steps);

/* As qmg_mg_gcr_solve, and also copy the iterate x_k after each of the first
 * maxrec outer steps into xhist (DEVICE complex128 [maxrec][V][4][3]);
 * *nrec (host) receives the number recorded.  QMG_ERR_STATE with the
 * red-black form on (its outer iterates live on the even sites only). */
qmg_status qmg_mg_gcr_solve_record(qmg_mg mg, const void* b, void* x, const qmg_solve_params* p,
                                   qmg_solve_info* info, void* xhist, int maxrec, int* nrec, void* stream);

/* Solve as qmg_mg_gcr_solve and keep a copy of every input of the level-0
 * smoother, in the order they occur: the K-cycle's input residual (before
 * pre-smoothing) and the residual left after the coarse-grid correction
 * (before post-smoothing), as DEVICE complex64 [maxrec][V][4][3]; *nrec
 * (host) receives the count kept (at most maxrec).  These are the residuals a
 * smoother is applied to, for training a learned smoother (residual form of
 * the loss).  Needs complex64 inner precision and at least two levels. */
qmg_status qmg_mg_gcr_solve_record_smoother(qmg_mg mg, const void* b, void* x, const qmg_solve_params* p,
                                            qmg_solve_info* info, void* rhist, int maxrec, int* nrec,
                                            void* stream);

/* Training pairs from recorded iterates: e_k = x* - x_k (computed in FP64),
 * r_k = M e_k (FP64 operator), both written as complex64 [n][V][4][3]
 * (r_out, e_out DEVICE). */
qmg_status qmg_mg_make_pairs(qmg_mg mg, const void* xstar, const void* xhist, int n, void* r_out, void* e_out,
                             void* stream);

#ifdef __cplusplus
}
#endif
#endif /* QMG_H */
