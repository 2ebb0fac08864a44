"""GPU parity of the Galerkin coarse-operator build (P^+ M P) against the
oracle, from the fine operator and from a coarse parent, and the Galerkin
identity coarse_dslash(u) = R M P u through the GPU kernels."""
import numpy as np
import pytest
import torch

import synth
from oracle import coarse, lattice, transfer, wilson
from gpu_util import dev, host, rel_err

pytestmark = pytest.mark.gpu


def fine_inputs(dims, eps, seed):
    U = synth.gauge_field(dims, eps, seed)
    return U, wilson.clover_field(U, dims, 1.0)


@pytest.mark.parametrize('storage,tol', [('c128', 1e-12), ('c64', 1e-5)])
def test_build_and_galerkin_identity_8x8x8x8(storage, tol):
    from paper_1612_07873_amd import FineOp, Transfer, build_coarse_op
    dims, block, nvec, m0 = (8, 8, 8, 8), (4, 4, 4, 4), 24, -0.2
    V = lattice.volume(dims)
    U, A = fine_inputs(dims, 0.4, 0)
    vecs = synth.gaussian((nvec, V, 12), 0, 1)
    Vb = transfer.block_orthonormalize(vecs, dims, block)
    ref = coarse.galerkin(coarse.FineParent(U, A, m0, dims), Vb, block)
    fop = FineOp(dims, dev(U), m0, 1.0, True, 'c128')
    t = Transfer(dims, 12, block, dev(vecs), 'c128')
    op = build_coarse_op(t, fine=fop, storage=storage)
    X, Y = op.export()
    ex = max(rel_err(host(X), ref.X), rel_err(host(Y), ref.Y))
    print('8^4 build %s rel err %.3e' % (storage, ex))
    assert ex <= tol
    # Galerkin identity through the GPU kernels: Mhat u == R M P u
    u = synth.gaussian((16, 48), 0, 2)
    dt = torch.complex128 if storage == 'c128' else torch.complex64
    y = host(op.apply(dev(u, dt)))
    rmp = host(t.restrict(fop.apply(t.prolong(dev(u)).reshape(V, 4, 3)).reshape(V, 12)))
    assert rel_err(y, rmp) <= tol


def test_fine_op_in_fp32_storage():
    from paper_1612_07873_amd import FineOp, Transfer, build_coarse_op
    dims, block, nvec, m0 = (8, 8, 8, 8), (4, 4, 4, 4), 12, -0.3
    V = lattice.volume(dims)
    U, A = fine_inputs(dims, 0.4, 3)
    vecs = synth.gaussian((nvec, V, 12), 3, 1)
    Vb = transfer.block_orthonormalize(vecs, dims, block)
    ref = coarse.galerkin(coarse.FineParent(U, A, m0, dims), Vb, block)
    op = build_coarse_op(Transfer(dims, 12, block, dev(vecs)), fine=FineOp(dims, dev(U), m0, 1.0, True, 'c64'))
    X, Y = op.export()
    assert max(rel_err(host(X), ref.X), rel_err(host(Y), ref.Y)) <= 1e-5


def test_coarse_parent_recursion():
    """Level 2 from level 1: 4^3x8, N 48 -> 2^3x4, N 64 (the 16^3x32 hierarchy shape)."""
    from paper_1612_07873_amd import CoarseOp, Transfer, build_coarse_op
    cd, N = (4, 4, 4, 8), 48
    Vc = lattice.volume(cd)
    X1 = synth.gaussian((Vc, N, N), 1, 2)
    Y1 = synth.gaussian((8, Vc, N, N), 2, 2)
    op1 = coarse.CoarseOp(cd, X1, Y1)
    vecs = synth.gaussian((32, Vc, N), 4, 1)
    Vb = transfer.block_orthonormalize(vecs, cd, (2, 2, 2, 2))
    ref = coarse.galerkin(coarse.CoarseParent(op1), Vb, (2, 2, 2, 2))
    for pst, tol in (('c128', 1e-12), ('c64', 1e-5)):
        g1 = CoarseOp(cd, dev(X1), dev(Y1), pst)
        op2 = build_coarse_op(Transfer(cd, N, (2, 2, 2, 2), dev(vecs)), parent=g1, storage='c128')
        X, Y = op2.export()
        err = max(rel_err(host(X), ref.X), rel_err(host(Y), ref.Y))
        print('recursion parent %s rel err %.3e' % (pst, err))
        assert err <= tol


def test_coarse_parent_block_too_large_for_lds():
    """A parent with N = 96 and 16 vectors (its block is formed element by
    element where it is used, not staged in LDS), a shape off the
    hierarchy's."""
    from paper_1612_07873_amd import CoarseOp, Transfer, build_coarse_op
    cd, N, block = (4, 4, 2, 2), 96, (2, 2, 1, 1)
    Vc = lattice.volume(cd)
    X1 = synth.gaussian((Vc, N, N), 11, 2)
    Y1 = synth.gaussian((8, Vc, N, N), 12, 2)
    op1 = coarse.CoarseOp(cd, X1, Y1)
    vecs = synth.gaussian((16, Vc, N), 13, 1)
    Vb = transfer.block_orthonormalize(vecs, cd, block)
    ref = coarse.galerkin(coarse.CoarseParent(op1), Vb, block)
    g1 = CoarseOp(cd, dev(X1), dev(Y1), 'c128')
    op2 = build_coarse_op(Transfer(cd, N, block, dev(vecs)), parent=g1, storage='c128')
    X, Y = op2.export()
    err = max(rel_err(host(X), ref.X), rel_err(host(Y), ref.Y))
    print('N=96 parent rel err %.3e' % err)
    assert err <= 1e-12


def test_16x16x16x32_full_size_sampled_sites():
    """16^3x32 -> 4^3x8 (Nvec 24): GPU build of all 512 coarse sites, eight of
    them recomputed one by one by the oracle."""
    from paper_1612_07873_amd import FineOp, Transfer, build_coarse_op
    dims, block, nvec, m0 = (16, 16, 16, 32), (4, 4, 4, 4), 24, -0.2
    V = lattice.volume(dims)
    U, A = fine_inputs(dims, 0.3, 0)
    vecs = synth.gaussian((nvec, V, 12), 0, 1)
    Vb = transfer.block_orthonormalize(vecs, dims, block)
    op = build_coarse_op(Transfer(dims, 12, block, dev(vecs)), fine=FineOp(dims, dev(U), m0, 1.0, True, 'c128'))
    X, Y = op.export()
    X, Y = host(X), host(Y)
    sites = [0, 1, 17, 100, 255, 300, 480, 511]
    Xr, Yr = coarse.galerkin(coarse.FineParent(U, A, m0, dims), Vb, block, coarse_sites=sites)
    assert max(rel_err(X[sites], Xr), rel_err(Y[:, sites], Yr)) <= 1e-12
    # property at full size: coarse gamma5-hermiticity X = g5 X^+ g5 per site
    g5 = np.diag([1.0] * nvec + [-1.0] * nvec)
    Xh = g5 @ np.conj(np.swapaxes(X, 1, 2)) @ g5
    assert np.abs(Xh - X).max() <= 1e-12 * np.abs(X).max()


def test_ragged_build():
    from paper_1612_07873_amd import FineOp, Transfer, build_coarse_op
    dims, block, nvec, m0 = (4, 6, 2, 4), (2, 3, 1, 2), 3, 0.1
    V = lattice.volume(dims)
    U, A = fine_inputs(dims, 0.5, 5)
    vecs = synth.gaussian((nvec, V, 12), 5, 1)
    Vb = transfer.block_orthonormalize(vecs, dims, block)
    ref = coarse.galerkin(coarse.FineParent(U, A, m0, dims), Vb, block)
    op = build_coarse_op(Transfer(dims, 12, block, dev(vecs)), fine=FineOp(dims, dev(U), m0, 1.0, True, 'c128'))
    X, Y = op.export()
    assert max(rel_err(host(X), ref.X), rel_err(host(Y), ref.Y)) <= 1e-12
