// Internal layout of the library's handles (not part of the public ABI).
#pragma once

#include "qmg_internal.h"

struct qmg_coarse_op_s {
    int dims[4];
    int64_t V;
    int N;
    qmg_prec storage;
    int J;        // 16-byte chunks per 9N-long row
    void* links;    // [V][J][N] chunks (see coarse_dslash.hip)
    float* lscale;  // [V][9] scales of the 16-bit storages (X, then Y_0..Y_7), else NULL
    int* nbr;       // [V][8]
    int rows, split;
    int pre;        // link chunks each thread loads before the LDS staging barrier (0 = by K)
    void* mlinks;   // 16-bit links in MFMA operand order (built on first multi-RHS use), else NULL
    int rpw[7];     // multi-RHS: right-hand-side tiles per wave for nrhs = 1,2,4,..,64 (0 = built-in)
    void* stage;    // staging of complex64 batches rounded to 16 bits ([V][nrhs][N] pairs, then [V][nrhs] scales)
    size_t stage_bytes;
    // red-black form (built by qmg_coarse_op_prepare_schur): the even half
    // [X_ee | Y_eo] and the odd half [X_oo^-1 | -X_oo^-1 Y_oe] as operators on
    // V/2 sites whose neighbour tables hold half-lattice indices, and the
    // lattice index of every half-lattice site of each parity [2][V/2]
    qmg_coarse_op_s* eo_even = nullptr;
    qmg_coarse_op_s* eo_odd = nullptr;
    int* hsite = nullptr;
    void* eo_tmp = nullptr;    // odd half-lattice scratch of the Schur entry points (grown on demand)
    size_t eo_tmp_bytes = 0;
};

struct qmg_fine_op_s {
    int dims[4];
    int64_t V;
    double m0, csw;
    int antiperiodic_t;
    qmg_prec storage;
    void* U;     // [4][9][V] complex, time sign folded into U_3 on the last slice
    void* clov;  // [2][36][V] reals: 6 diagonal, then 15 upper off-diagonal complex
                 // (16-bit storages: [2][18][V] pairs of those reals)
    float* cscale;  // [2][V] clover scales of the 16-bit storages, else NULL
    int* nbr;    // [V][8]
    // red-black form (every extent even): the lattice index of every
    // half-lattice site of each parity, hsite [2][V/2] ("parity order":
    // index p*V/2 + h is site hsite[p*V/2 + h]); the inverse of the site-local
    // block (4 + m0 + A(x))^-1 in the clover's packed layout and storage, in
    // parity order; parity-order copies of the links, the clover term and its
    // scales, and the neighbour table hnb [V][8] in parity order (lattice
    // indices of the neighbours), so that a red-black kernel over the sites of
    // one parity reads each of them contiguously
    void* cinv = nullptr;
    float* ciscale = nullptr;
    int* hsite = nullptr;
    void* U_eo = nullptr;
    void* clov_eo = nullptr;
    float* cscale_eo = nullptr;
    int* hnb = nullptr;
    void* eo_tmp = nullptr;    // half-lattice scratch of the Schur entry points (grown on demand)
    size_t eo_tmp_bytes = 0;
    int link_reals = 18;       // 18, or 12: links stored as rows 0 and 1, [4][6][V], row 2 rebuilt
    int64_t last = 0;          // first lattice index of the last time slice
};

struct qmg_transfer_s {
    int fdims[4], block[4], cdims[4];
    int64_t V, Vc;
    int dof, nvec, bsites;
    qmg_prec storage;
    double2* basis64;  // [V][dof][nvec] FP64
    void* basis;       // [V][dof][nvec] storage precision (== basis64 for C128)
    int* members;      // [Vc][bsites]
    int* owner;        // [V]
};

struct qmg_ptc_s {
    qmg_fine_op op;   // links (complex64 storage) and neighbour table, borrowed
    int C;            // hidden channels
    int64_t V;
    float2 *W1, *W2;  // [9][C][1][16], [9][1][C][16]
    float2 *G1, *G2;  // gradients (accumulated)
    float2 *m1, *v1, *m2, *v2;  // Adam moments (re, im as independent reals)
    float2* h1;       // [C][V][12] hidden activations
    float2* D1;       // [C][V][12] dL/dh1*
    float2* y;        // [V][12] output
    float2* D2;       // [V][12] dL/dy*
    float2 *t1, *t2;  // [V][12] scratch of the residual-form loss
    double* part;     // partial sums for reductions
    double* loss;     // [2]: accumulated loss, scratch
    int adam_t;
    // inference: the network collapsed to K[p][q] = sum_b W2[p][0][b] W1[q][b][0]
    // (81 spin matrices, rebuilt when the weights change) and the mixed fields
    // g_p = sum_q K[p][q] T_q r, [9][V][12]
    float2* K = nullptr;
    float2* g = nullptr;
    bool k_stale = true;
};

namespace qmg {
// Arguments of a red-black piece of the coarse stencil (coarse_dslash.hip):
// directions d0 .. d0+nd-1 of the stacked row [X | Y_0 .. Y_7]; the
// site-local block multiplies `uself` at sidx[site] (or site; member stride
// vself sites), and the output goes to oidx[site] (or site; stride vout).
struct EoArgs {
    const void* uself;
    const int* sidx;
    const int* oidx;
    int d0, nd;
    int64_t vself, vout;
};

// Chiral-basis Dirac matrices: gamma_mu = [[0, g_mu], [g_mu^+, 0]] with
// g_k = -i sigma_k (k = 1..3), g_4 = 1.  gamma(mu, r, c) as (re, im).
void gamma_matrix(int mu, double out[4][4][2]);
}
