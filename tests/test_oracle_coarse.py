"""Pins of the oracle's transfer operators (Sec. 3.4, 6.6) and coarse operator
(Eq. 3): orthonormality, adjointness, the Galerkin identity against an
independent R.M.P chain, a coarse free-field closed form over one and two
levels, gauge invariance and coarse gamma5-hermiticity."""
import numpy as np
import pytest

import synth
from oracle import coarse, lattice, transfer, wilson
from oracle_helpers import gauge_rotate, unit_gauge


def fine_setup(dims, eps, seed, csw=1.0):
    U = synth.gauge_field(dims, eps, seed)
    return U, wilson.clover_field(U, dims, csw)


def test_block_basis_is_orthonormal_and_transfers_are_adjoint():
    dims, block, nvec = (8, 4, 4, 8), (4, 2, 2, 4), 6
    V = lattice.volume(dims)
    vecs = synth.gaussian((nvec, V, 12), 0, 1)
    Vb = transfer.block_orthonormalize(vecs, dims, block)
    members = transfer.sites_of_blocks(dims, block)
    for xc in range(members.shape[0]):
        for chi in range(2):
            W = Vb[members[xc], 6 * chi:6 * chi + 6, :].reshape(-1, nvec)
            assert np.abs(W.conj().T @ W - np.eye(nvec)).max() < 1e-13
            # span is that of the original vectors restricted to the block
            O = vecs[:, members[xc], 6 * chi:6 * chi + 6].reshape(nvec, -1).T
            proj = W @ (W.conj().T @ O)
            assert np.abs(proj - O).max() < 1e-12
            # R of the MGS factor is upper triangular with a real positive diagonal
            R = W.conj().T @ O
            assert np.abs(np.tril(R, -1)).max() < 1e-12
            assert np.all(np.diag(R).real > 0) and np.abs(np.diag(R).imag).max() < 1e-12
    Vc = members.shape[0]
    u = synth.gaussian((Vc, 2 * nvec), 1, 2)
    f = synth.gaussian((V, 12), 2, 2)
    # R P = 1
    assert np.abs(transfer.restrict(Vb, transfer.prolong(Vb, u, dims, block), dims, block) - u).max() < 1e-13
    # <R f, u> = <f, P u>
    a = np.vdot(transfer.restrict(Vb, f, dims, block), u)
    b = np.vdot(f, transfer.prolong(Vb, u, dims, block))
    assert abs(a - b) < 1e-12 * abs(b)
    # P R is a Hermitian projector: applying it twice changes nothing
    pr = lambda v: transfer.prolong(Vb, transfer.restrict(Vb, v, dims, block), dims, block)
    assert np.abs(pr(pr(f)) - pr(f)).max() < 1e-13


def test_rank_deficient_vectors_are_rejected():
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    V = lattice.volume(dims)
    vecs = synth.gaussian((3, V, 12), 0, 1)
    vecs[2] = 2.0 * vecs[0] - 1j * vecs[1]
    with pytest.raises(transfer.RankError):
        transfer.block_orthonormalize(vecs, dims, block)


def test_galerkin_identity_8to2_nvec24():
    """8^4 -> 2^4 (block 4^4, Nvec 24, N 48): Eq. 3 apply == R M P u exactly."""
    dims, block, nvec = (8, 8, 8, 8), (4, 4, 4, 4), 24
    V = lattice.volume(dims)
    U, A = fine_setup(dims, 0.4, 0)
    Vb = transfer.block_orthonormalize(synth.gaussian((nvec, V, 12), 0, 1), dims, block)
    op = coarse.galerkin(coarse.FineParent(U, A, -0.2, dims), Vb, block)
    assert op.dims == (2, 2, 2, 2) and op.N == 48
    u = synth.gaussian((16, 48), 0, 2)
    rmp = transfer.restrict(Vb, wilson.apply_wilson_clover(
        transfer.prolong(Vb, u, dims, block), U, A, -0.2, dims), dims, block)
    assert np.abs(op.apply(u) - rmp).max() < 1e-13 * np.abs(rmp).max()
    # the plain C loop holds the same identity
    assert np.abs(op.apply_c(u) - rmp).max() < 1e-13 * np.abs(rmp).max()


def test_dense_galerkin_matches_matrix_product():
    """4^4 -> 2^4, Nvec 4: the assembled Mhat equals P^+ M P built densely."""
    dims, block, nvec = (4, 4, 4, 4), (2, 2, 2, 2), 4
    V = lattice.volume(dims)
    U, A = fine_setup(dims, 0.4, 2)
    Vb = transfer.block_orthonormalize(synth.gaussian((nvec, V, 12), 3, 1), dims, block)
    op = coarse.galerkin(coarse.FineParent(U, A, -0.2, dims), Vb, block)
    M = wilson.dense_matrix(lambda v: wilson.apply_wilson_clover(v.reshape(V, 12), U, A, -0.2, dims).reshape(-1), V * 12)
    Vc = 16
    # P as a (V*12) x (Vc*N) matrix from prolonging unit vectors
    P = np.zeros((V * 12, Vc * 2 * nvec), dtype=np.complex128)
    e = np.zeros(Vc * 2 * nvec, dtype=np.complex128)
    for j in range(Vc * 2 * nvec):
        e[j] = 1
        P[:, j] = transfer.prolong(Vb, e.reshape(Vc, 2 * nvec), dims, block).reshape(-1)
        e[j] = 0
    assert np.abs(P.conj().T @ P - np.eye(P.shape[1])).max() < 1e-13
    Mhat = P.conj().T @ M @ P
    assert np.abs(op.dense() - Mhat).max() < 1e-13


def constant_vectors(dims, dof):
    """Nvec = dof/2 vectors e_j + e_{j+dof/2}, constant over the lattice."""
    V = lattice.volume(dims)
    h = dof // 2
    v = np.zeros((h, V, dof), dtype=np.complex128)
    for j in range(h):
        v[j, :, j] = 1
        v[j, :, j + h] = 1
    return v


def free_wilson_coarse_op(cdims, mass, scale, anti=True):
    """Closed form: scale * M_W(mass) on cdims with U = 1, as X and Y blocks."""
    Pm, Pp = lattice.projectors()
    Vc = lattice.volume(cdims)
    X = np.broadcast_to(scale * (4 + mass) * np.eye(12), (Vc, 12, 12)).copy()
    Y = np.zeros((8, Vc, 12, 12), dtype=np.complex128)
    for mu in range(4):
        for back, P in ((0, Pm[mu]), (1, Pp[mu])):
            eta = lattice.boundary_sign(cdims, mu, 1 - 2 * back, anti)
            Y[2 * mu + back] = scale * (-0.5) * eta[:, None, None] * np.kron(P, np.eye(3))[None]
    return X, Y


@pytest.mark.parametrize("block", [(2, 2, 2, 2), (4, 2, 2, 4)])
def test_coarse_free_field_closed_form_one_level(block):
    """U = 1 and block-constant vectors: Mhat = (1/b) M_W(m0 b) for a cubic block
    b (the anisotropic form is m0 + sum_mu (1/b_mu)[1 - (P^- T_+ + P^+ T_-)/2])."""
    dims, m0 = (8, 4, 4, 8), -0.3
    U = unit_gauge(dims)
    Vb = transfer.block_orthonormalize(constant_vectors(dims, 12), dims, block)
    op = coarse.galerkin(coarse.FineParent(U, None, m0, dims), Vb, block)
    cd = op.dims
    Pm, Pp = lattice.projectors()
    Xe = (m0 + sum(1.0 / b for b in block)) * np.eye(12)
    assert np.abs(op.X - Xe[None]).max() < 1e-14
    for mu in range(4):
        for back, P in ((0, Pm[mu]), (1, Pp[mu])):
            eta = lattice.boundary_sign(cd, mu, 1 - 2 * back, True)
            Ye = (-0.5 / block[mu]) * eta[:, None, None] * np.kron(P, np.eye(3))[None]
            assert np.abs(op.Y[2 * mu + back] - Ye).max() < 1e-14


def test_coarse_free_field_closed_form_two_levels():
    """Coarsening twice (b1 = b2 = 2): Mhat2 = (1/(b1 b2)) M_W(m0 b1 b2), the
    recursion of Sec. 3.4 keeping the form of Eq. (3)."""
    dims, m0 = (8, 8, 8, 8), -0.25
    U = unit_gauge(dims)
    b = (2, 2, 2, 2)
    Vb1 = transfer.block_orthonormalize(constant_vectors(dims, 12), dims, b)
    op1 = coarse.galerkin(coarse.FineParent(U, None, m0, dims), Vb1, b)
    Vb2 = transfer.block_orthonormalize(constant_vectors(op1.dims, 12), op1.dims, b)
    op2 = coarse.galerkin(coarse.CoarseParent(op1), Vb2, b)
    X, Y = free_wilson_coarse_op(op2.dims, m0 * 4, 0.25)
    assert np.abs(op2.X - X).max() < 1e-14
    assert np.abs(op2.Y - Y).max() < 1e-14
    # and the apply agrees with the fine formula evaluated on the coarse lattice
    u = synth.gaussian((lattice.volume(op2.dims), 4, 3), 0, 2)
    ref = 0.25 * wilson.apply_wilson_clover(u, unit_gauge(op2.dims), None, 4 * m0, op2.dims)
    assert np.abs(op2.apply(u.reshape(-1, 12)) - ref.reshape(-1, 12)).max() < 1e-14
    assert np.abs(op2.apply_c(u.reshape(-1, 12)) - ref.reshape(-1, 12)).max() < 1e-14


def test_coarse_operator_is_gauge_invariant():
    """Rotating U and the null vectors by the same g leaves X and Y unchanged."""
    dims, block, nvec = (4, 4, 4, 4), (2, 2, 2, 2), 5
    V = lattice.volume(dims)
    U, A = fine_setup(dims, 0.4, 4)
    g = synth.gauge_rotation(dims, 5)
    Ug = gauge_rotate(U, g, dims)
    vecs = synth.gaussian((nvec, V, 4, 3), 6, 1)
    vg = np.einsum('xab,kxsb->kxsa', g, vecs)
    op = coarse.galerkin(coarse.FineParent(U, A, -0.2, dims),
                         transfer.block_orthonormalize(vecs.reshape(nvec, V, 12), dims, block), block)
    opg = coarse.galerkin(coarse.FineParent(Ug, wilson.clover_field(Ug, dims, 1.0), -0.2, dims),
                          transfer.block_orthonormalize(vg.reshape(nvec, V, 12), dims, block), block)
    assert np.abs(op.X - opg.X).max() < 1e-13
    assert np.abs(op.Y - opg.Y).max() < 1e-13


def test_coarse_gamma5_hermiticity():
    """gamma5hat Mhat gamma5hat = Mhat^+ with gamma5hat = diag(+1_Nvec, -1_Nvec)."""
    dims, block, nvec = (4, 4, 4, 4), (2, 2, 2, 2), 4
    V = lattice.volume(dims)
    U, A = fine_setup(dims, 0.4, 8)
    Vb = transfer.block_orthonormalize(synth.gaussian((nvec, V, 12), 9, 1), dims, block)
    M = coarse.galerkin(coarse.FineParent(U, A, -0.2, dims), Vb, block).dense()
    g5 = np.kron(np.eye(16), np.diag([1.0] * nvec + [-1.0] * nvec))
    assert np.abs(g5 @ M @ g5 - M.conj().T).max() < 1e-13
    assert np.abs(M - M.conj().T).max() > 1e-2


def test_galerkin_of_a_coarse_parent_matches_dense_product():
    """Level 2 from level 1 (recursion): Mhat2 = P2^+ Mhat1 P2 densely."""
    dims = (8, 8, 8, 8)
    V = lattice.volume(dims)
    U, A = fine_setup(dims, 0.4, 0)
    Vb1 = transfer.block_orthonormalize(synth.gaussian((4, V, 12), 0, 1), dims, (2, 2, 2, 2))
    op1 = coarse.galerkin(coarse.FineParent(U, A, -0.2, dims), Vb1, (2, 2, 2, 2))
    V1 = lattice.volume(op1.dims)
    Vb2 = transfer.block_orthonormalize(synth.gaussian((3, V1, 8), 1, 1), op1.dims, (2, 2, 2, 2))
    op2 = coarse.galerkin(coarse.CoarseParent(op1), Vb2, (2, 2, 2, 2))
    M1 = op1.dense()
    V2 = lattice.volume(op2.dims)
    P = np.zeros((V1 * 8, V2 * 6), dtype=np.complex128)
    e = np.zeros(V2 * 6, dtype=np.complex128)
    for j in range(V2 * 6):
        e[j] = 1
        P[:, j] = transfer.prolong(Vb2, e.reshape(V2, 6), op1.dims, (2, 2, 2, 2)).reshape(-1)
        e[j] = 0
    assert np.abs(op2.dense() - P.conj().T @ M1 @ P).max() < 1e-13


def test_multi_rhs_apply_equals_columnwise_apply():
    cd = (2, 2, 2, 4)
    Vc, N = lattice.volume(cd), 8
    X = synth.gaussian((Vc, N, N), 0, 2)
    Y = synth.gaussian((8, Vc, N, N), 1, 2)
    op = coarse.CoarseOp(cd, X, Y)
    u = synth.gaussian((Vc, N, 5), 2, 2)
    y = op.apply(u)
    for r in range(5):
        assert np.abs(y[:, :, r] - op.apply(u[:, :, r].copy())).max() < 1e-14


def test_apply_at_sampled_sites_equals_full_apply():
    cd = (2, 4, 2, 4)
    Vc, N = lattice.volume(cd), 6
    op = coarse.CoarseOp(cd, synth.gaussian((Vc, N, N), 3, 2), synth.gaussian((8, Vc, N, N), 4, 2))
    u = synth.gaussian((Vc, N, 3), 5, 2)
    sites = [0, 5, 17, 63]
    assert np.abs(op.apply_sites(u, sites) - op.apply(u)[sites]).max() < 1e-14


@pytest.mark.parametrize('cd,N,nrhs', [((3, 2, 5, 2), 8, 3), ((2, 4, 2, 3), 6, 1), ((4, 4, 4, 8), 48, 2)])
def test_c_apply_matches_numpy_apply(cd, N, nrhs):
    """The plain C loop of Eq. (3) (the host baseline) and the numpy restatement
    agree on ragged lattices with several right-hand sides, with 1 and all threads."""
    V = lattice.volume(cd)
    op = coarse.CoarseOp(cd, synth.gaussian((V, N, N), 0, 2), synth.gaussian((8, V, N, N), 1, 2))
    u = synth.gaussian((V, N, nrhs), 2, 2)
    ref = op.apply(u)
    assert np.abs(op.apply_c(u) - ref).max() < 1e-13 * np.abs(ref).max()
    for th in (1, 0):
        sec, used, y = op.time_apply_c(u, 1, th)
        assert sec > 0 and used >= 1 and (th == 0 or used == th)
        assert np.abs(y - ref).max() < 1e-13 * np.abs(ref).max()
