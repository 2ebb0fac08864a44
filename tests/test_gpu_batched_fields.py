"""Several right-hand sides through one call of the field entry points
(qmg_coarse_dslash, qmg_wilson_clover_dslash, qmg_prolong, qmg_restrict with
nrhs > 1, fields [nrhs][...] member-major), each member against the oracle's
single-field result: FP64 1e-12, FP32 1e-5 (relative, max norm)."""
import numpy as np
import pytest
import torch

import synth
from oracle import coarse, lattice, transfer, wilson
from gpu_util import dev, host, rel_err

pytestmark = pytest.mark.gpu

TOL = {'c128': 1e-12, 'c64': 1e-5}
CDT = {'c128': torch.complex128, 'c64': torch.complex64}


@pytest.mark.parametrize('prec', ['c128', 'c64'])
@pytest.mark.parametrize('cd,N,nrhs', [((3, 2, 5, 2), 8, 5), ((4, 4, 4, 8), 48, 3), ((2, 2, 2, 2), 48, 7)])
def test_coarse_dslash_nrhs(prec, cd, N, nrhs):
    from paper_1612_07873_amd import CoarseOp
    V = lattice.volume(cd)
    X, Y = synth.gaussian((V, N, N), 0, 2), synth.gaussian((8, V, N, N), 1, 2)
    ref_op = coarse.CoarseOp(cd, X, Y)
    U = np.stack([synth.gaussian((V, N), 10 + k, 2) for k in range(nrhs)])
    op = CoarseOp(cd, dev(X), dev(Y), prec)
    y = host(op.apply(dev(U, CDT[prec])))
    errs = [rel_err(y[k], ref_op.apply(U[k])) for k in range(nrhs)]
    print(cd, N, nrhs, prec, 'max member err %.2e' % max(errs))
    assert max(errs) <= TOL[prec]
    # the batch equals the single calls bitwise (same kernel, member on grid y)
    y1 = host(op.apply(dev(U[nrhs - 1], CDT[prec])))
    assert np.array_equal(y1, y[nrhs - 1])


@pytest.mark.parametrize('prec', ['c128', 'c64'])
def test_wilson_clover_dslash_nrhs(prec):
    from paper_1612_07873_amd import FineOp
    dims, nrhs, m0 = (4, 4, 4, 8), 3, -0.2
    V = lattice.volume(dims)
    U = synth.gauge_field(dims, 0.4, 1)
    A = wilson.clover_field(U, dims, 1.0)
    P = np.stack([synth.gaussian((V, 4, 3), 20 + k, 2) for k in range(nrhs)])
    op = FineOp(dims, dev(U), m0, 1.0, True, prec)
    y = host(op.apply(dev(P, CDT[prec])))
    errs = [rel_err(y[k], wilson.apply_wilson_clover(P[k], U, A, m0, dims)) for k in range(nrhs)]
    print('wilson nrhs', nrhs, prec, 'max member err %.2e' % max(errs))
    assert max(errs) <= TOL[prec]


@pytest.mark.parametrize('storage', ['c128', 'c64'])
def test_prolong_restrict_nrhs(storage):
    from paper_1612_07873_amd import Transfer
    dims, dof, block, nvec, nrhs = (8, 4, 4, 8), 12, (4, 2, 2, 4), 6, 4
    V = lattice.volume(dims)
    vecs = synth.gaussian((nvec, V, dof), 3, 1)
    Vb = transfer.block_orthonormalize(vecs, dims, block)
    Vc = lattice.volume(transfer.coarse_dims(dims, block))
    UC = np.stack([synth.gaussian((Vc, 2 * nvec), 30 + k, 2) for k in range(nrhs)])
    F = np.stack([synth.gaussian((V, dof), 40 + k, 2) for k in range(nrhs)])
    t = Transfer(dims, dof, block, dev(vecs), storage)
    p = host(t.prolong(dev(UC, CDT[storage])))
    r = host(t.restrict(dev(F, CDT[storage])))
    assert p.shape == (nrhs, V, dof) and r.shape == (nrhs, Vc, 2 * nvec)
    ep = max(rel_err(p[k], transfer.prolong(Vb, UC[k], dims, block)) for k in range(nrhs))
    er = max(rel_err(r[k], transfer.restrict(Vb, F[k], dims, block)) for k in range(nrhs))
    print('transfer nrhs', nrhs, storage, 'prolong %.2e restrict %.2e' % (ep, er))
    assert ep <= TOL[storage] and er <= TOL[storage]


@pytest.mark.parametrize('storage,unit', [('h16', 2.0 ** -11), ('b16', 2.0 ** -8)])
@pytest.mark.parametrize('cd,N,nrhs', [((4, 4, 4, 8), 64, 16), ((2, 2, 2, 4), 48, 8), ((3, 2, 2, 2), 32, 64)])
def test_coarse_dslash_mrhs_from_complex64(storage, unit, cd, N, nrhs):
    """qmg_coarse_dslash_mrhs_c64: complex64 batches [nrhs][V][N] rounded to 16
    bits (one scale per site and right-hand side) in the operator's staging and
    applied on the matrix cores.  Against the oracle applied to the stored
    (16-bit) links and the unrounded inputs, the norm-wise error of each member
    is bounded by the rounding of its inputs (1.5 units of the format)."""
    from paper_1612_07873_amd import CoarseOp
    V = lattice.volume(cd)
    X, Y = synth.gaussian((V, N, N), 4, 2), synth.gaussian((8, V, N, N), 5, 2)
    op = CoarseOp(cd, dev(X), dev(Y), storage)
    Xq, Yq = (host(t) for t in op.export())
    ref_op = coarse.CoarseOp(cd, Xq, Yq)
    U = np.stack([synth.gaussian((V, N), 50 + k, 2) for k in range(nrhs)]).astype(np.complex64)
    y = host(op.apply_mrhs_c64(dev(U, torch.complex64)))
    errs = []
    for k in range(nrhs):
        r = ref_op.apply(U[k].astype(np.complex128))
        errs.append(float(np.linalg.norm(y[k] - r) / np.linalg.norm(r)))
    print(cd, N, nrhs, storage, 'max member err %.2e (unit %.2e)' % (max(errs), unit))
    assert max(errs) <= 1.5 * unit
    # a smaller batch after a larger one reuses the operator's staging
    y8 = host(op.apply_mrhs_c64(dev(U[:8], torch.complex64)))
    if nrhs == 8:
        assert np.array_equal(y8, y)
    assert max(float(np.linalg.norm(y8[k] - ref_op.apply(U[k].astype(np.complex128)))
                     / np.linalg.norm(ref_op.apply(U[k].astype(np.complex128)))) for k in range(8)) <= 1.5 * unit
