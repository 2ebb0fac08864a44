"""Pins of the oracle's Schwarz alternating procedure (SAP) smoother against
dense block solves: with enough MR steps every block solve is exact, so one
sweep equals block Gauss-Seidel built from index slices of the dense matrix
and LAPACK; a single step equals the minimal-residual formula on each dense
block; and the sweep is gauge covariant."""
import numpy as np
import pytest

import synth
from oracle import lattice, schwarz, wilson
from oracle_helpers import gauge_rotate


def setup(dims=(4, 4, 4, 4), m0=0.3, seed=2):
    U = synth.gauge_field(dims, 0.4, seed)
    A = wilson.clover_field(U, dims, 1.0)
    V = lattice.volume(dims)
    apply = lambda v: wilson.apply_wilson_clover(v.reshape(V, 4, 3), U, A, m0, dims).reshape(V, 12)
    return U, A, m0, dims, V, apply


def sites_of(bid, b):
    s = np.nonzero(bid == b)[0]
    return (s[:, None] * 12 + np.arange(12)[None]).reshape(-1)


def test_block_colours_alternate():
    bid, colour, nblk = schwarz.block_ids((4, 8, 4, 4), (2, 2, 2, 2))
    assert nblk == 2 * 4 * 2 * 2
    nb = lattice.neighbour
    for mu in range(4):
        n = nb((4, 8, 4, 4), mu, 1)
        cross = bid != bid[n]
        assert np.all(colour[cross] != colour[n][cross])
    with pytest.raises(ValueError):
        schwarz.block_ids((4, 4, 4, 6), (2, 2, 2, 2))   # 3 blocks in time


def test_exact_block_solves_are_block_gauss_seidel():
    U, A, m0, dims, V, apply = setup()
    block = (2, 2, 2, 2)
    M = wilson.dense_matrix(lambda v: apply(v).reshape(-1), V * 12)
    r = synth.gaussian((V, 12), 3, 2)
    x = schwarz.sap(apply, r, dims, block, iters=300)
    bid, colour, nblk = schwarz.block_ids(dims, block)
    ref = np.zeros(V * 12, dtype=np.complex128)
    rr = r.reshape(-1).copy()
    for c in (0, 1):
        res = rr - M @ ref
        upd = np.zeros_like(ref)
        for b in range(nblk):
            idx = sites_of(bid, b)
            if colour[idx[0] // 12] != c:
                continue
            upd[idx] = np.linalg.solve(M[np.ix_(idx, idx)], res[idx])
        ref = ref + upd
    err = np.abs(x.reshape(-1) - ref).max() / np.abs(ref).max()
    print('SAP(300) vs block Gauss-Seidel: %.2e' % err)
    assert err < 1e-10


def test_single_step_is_the_blockwise_minimal_residual_step():
    U, A, m0, dims, V, apply = setup(m0=-0.2)
    block = (2, 2, 2, 2)
    M = wilson.dense_matrix(lambda v: apply(v).reshape(-1), V * 12)
    r = synth.gaussian((V, 12), 4, 2)
    x = schwarz.sap(apply, r, dims, block, iters=1).reshape(-1)
    bid, colour, nblk = schwarz.block_ids(dims, block)
    ref = np.zeros(V * 12, dtype=np.complex128)
    for c in (0, 1):
        res = r.reshape(-1) - M @ ref
        upd = np.zeros_like(ref)
        for b in range(nblk):
            idx = sites_of(bid, b)
            if colour[idx[0] // 12] != c:
                continue
            s = res[idx]
            As = M[np.ix_(idx, idx)] @ s
            upd[idx] = (np.vdot(As, s) / np.vdot(As, As).real) * s
        ref = ref + upd
    assert np.abs(x - ref).max() < 1e-13 * np.abs(ref).max()


def test_sap_is_gauge_covariant():
    U, A, m0, dims, V, apply = setup(m0=-0.2)
    g = synth.gauge_rotation(dims, 9)
    Ug = gauge_rotate(U, g, dims)
    Ag = wilson.clover_field(Ug, dims, 1.0)
    apply_g = lambda v: wilson.apply_wilson_clover(v.reshape(V, 4, 3), Ug, Ag, m0, dims).reshape(V, 12)
    r = synth.gaussian((V, 4, 3), 5, 2)
    rot = lambda v: np.einsum('xab,xsb->xsa', g, v.reshape(V, 4, 3)).reshape(V, 12)
    x = schwarz.sap(apply, r.reshape(V, 12), dims, (2, 2, 2, 2), iters=4)
    xg = schwarz.sap(apply_g, rot(r), dims, (2, 2, 2, 2), iters=4)
    assert np.abs(xg - rot(x)).max() < 1e-12 * np.abs(x).max()


def test_sweep_lowers_the_residual():
    U, A, m0, dims, V, apply = setup(m0=-0.2)
    r = synth.gaussian((V, 12), 6, 2)
    for iters in (1, 2, 4):
        x = schwarz.sap(apply, r, dims, (2, 2, 2, 2), iters)
        assert np.linalg.norm(r - apply(x)) < np.linalg.norm(r)
