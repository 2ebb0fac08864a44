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
};

namespace qmg {
// Chiral-basis Dirac matrices: gamma_mu = [[0, g_mu], [g_mu^+, 0]] with
// g_k = -i sigma_k (k = 1..3), g_4 = 1.  gamma(mu, r, c) as (re, im).
void gamma_matrix(int mu, double out[4][4][2]);
}
