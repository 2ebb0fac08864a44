"""Pins of the oracle's red-black (even-odd) preconditioning (Sec. 3.3) and
BiCGStab: the Schur operator equals the Schur complement taken from the dense
matrix by index slicing, and Schur solve + back-substitution equals the dense
LAPACK solve, for the fine operator (Eq. 2) and a Galerkin coarse operator
(Eq. 3); BiCGStab reaches the LAPACK solution within its tolerance."""
import numpy as np
import pytest

import synth
from oracle import coarse, evenodd, lattice, solvers, transfer, wilson


def dense(apply, n):
    return wilson.dense_matrix(apply, n)


def fine_case(dims=(4, 4, 2, 4), m0=-0.2, seed=3):
    U = synth.gauge_field(dims, 0.4, seed)
    A = wilson.clover_field(U, dims, 1.0)
    V = lattice.volume(dims)
    M = lambda v: wilson.apply_wilson_clover(v.reshape(V, 4, 3), U, A, m0, dims).reshape(-1)
    return U, A, m0, dims, V, M


def coarse_case():
    dims, block, nvec = (4, 4, 4, 4), (2, 2, 2, 2), 2
    V = lattice.volume(dims)
    U = synth.gauge_field(dims, 0.4, 5)
    A = wilson.clover_field(U, dims, 1.0)
    Vb = transfer.block_orthonormalize(synth.gaussian((nvec, V, 12), 6, 1), dims, block)
    return coarse.galerkin(coarse.FineParent(U, A, -0.2, dims), Vb, block)


def check_schur(S, Md, dof):
    """S against the dense Schur complement; Schur solve against LAPACK."""
    V = S.V
    idx = lambda s: (s[:, None] * dof + np.arange(dof)[None]).reshape(-1)
    e, o = idx(S.even), idx(S.odd)
    Sd = Md[np.ix_(e, e)] - Md[np.ix_(e, o)] @ np.linalg.solve(Md[np.ix_(o, o)], Md[np.ix_(o, e)])
    xe = synth.gaussian((len(S.even), dof), 11, 2)
    assert np.abs(S.apply(xe).reshape(-1) - Sd @ xe.reshape(-1)).max() < 1e-12 * np.abs(Sd @ xe.reshape(-1)).max()
    b = synth.gaussian((V, dof), 12, 2)
    x_ref = np.linalg.solve(Md, b.reshape(-1))
    xe_sol = np.linalg.solve(Sd, S.source(b).reshape(-1))
    x = S.reconstruct(xe_sol.reshape(-1, dof), b)
    assert np.abs(x.reshape(-1) - x_ref).max() < 1e-11 * np.abs(x_ref).max()
    # the odd/even split really is by parity: every hop joins opposite parities
    assert np.abs(Md[np.ix_(e, e)] - np.kron(np.eye(len(S.even)), np.ones((dof, dof))) * Md[np.ix_(e, e)]).max() == 0
    return Sd


def test_parity_sites():
    dims = (4, 2, 2, 6)
    p = evenodd.parity(dims)
    c = lattice.coords(dims)
    assert np.array_equal(p, (c[:, 0] + c[:, 1] + c[:, 2] + c[:, 3]) % 2)
    assert len(evenodd.sites(dims, 0)) == len(evenodd.sites(dims, 1)) == lattice.volume(dims) // 2
    for mu in range(4):  # every hop changes parity on even extents
        assert np.all(p[lattice.neighbour(dims, mu, 1)] != p)


def test_fine_schur_matches_dense_complement_and_solve():
    U, A, m0, dims, V, M = fine_case()
    S = evenodd.fine_schur(U, A, m0, dims)
    check_schur(S, dense(M, V * 12), 12)


def test_coarse_schur_matches_dense_complement_and_solve():
    op = coarse_case()
    S = evenodd.coarse_schur(op)
    check_schur(S, op.dense(), op.N)


def test_bicgstab_reaches_lapack_solution():
    U, A, m0, dims, V, M = fine_case(m0=0.1)
    Md = dense(M, V * 12)
    b = synth.gaussian((V * 12,), 13, 2)
    x_ref = np.linalg.solve(Md, b)
    x, info = solvers.bicgstab(lambda v: Md @ v, b, 1e-12, maxit=2000)
    assert info.converged
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) <= 1e-9
    # on the Schur system, then back-substituted
    S = evenodd.fine_schur(U, A, m0, dims)
    bw = b.reshape(V, 12)
    xe, ie = solvers.bicgstab(lambda v: S.apply(v.reshape(-1, 12)).reshape(-1), S.source(bw).reshape(-1), 1e-12,
                              maxit=2000)
    xs = S.reconstruct(xe.reshape(-1, 12), bw).reshape(-1)
    assert np.linalg.norm(xs - x_ref) / np.linalg.norm(x_ref) <= 1e-9
    # the red-black system converges in fewer steps
    assert ie.iters < info.iters
    print('BiCGStab steps: full', info.iters, 'red-black', ie.iters)
