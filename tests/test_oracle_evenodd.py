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


def small_fine(dims=(4, 4, 4, 4), m0=-0.3, seed=1):
    from oracle import mg
    U = synth.gauge_field(dims, 0.4, seed)
    A = wilson.clover_field(U, dims, 1.0)
    return mg.FineLevel(U, A, m0, dims)


def test_red_black_smoother_leaves_no_odd_residual():
    """The red-black smoother back-substitutes the odd sites exactly, so the
    residual it leaves is zero there; on the even sites it is the Schur MR
    residual b_e - M_eo M_oo^-1 r_o - S x_e."""
    from oracle import mg
    fine = small_fine((4, 4, 2, 4))
    h = mg.Hierarchy(fine, [], [], [])
    K = mg.KCycle(h, evenodd=True)
    S = K.schur(0)
    r = synth.gaussian(fine.V * 12, 21, 2)
    x = K.smooth(0, r)
    res = (r - fine.apply(x)).reshape(fine.V, 12)
    assert np.abs(res[S.odd]).max() <= 1e-13 * np.abs(r).max()
    xe = x.reshape(fine.V, 12)[S.even]
    schur_res = S.source(r) - S.apply(xe)
    assert np.abs(res[S.even] - schur_res).max() <= 1e-13 * np.abs(r).max()
    # four MR steps lower the Schur residual
    assert np.linalg.norm(schur_res) < 0.9 * np.linalg.norm(S.source(r))


def test_even_part_of_exact_inverse_is_schur_inverse():
    """The reading behind the red-black K-cycle preconditioner: the even part of
    A^-1 applied to (r_e, 0) is S^-1 r_e, because (A^-1)_ee = S^-1."""
    U, A, m0, dims, V, M = fine_case()
    S = evenodd.fine_schur(U, A, m0, dims)
    Md = dense(M, V * 12)
    re = synth.gaussian((V // 2) * 12, 22, 2)
    lhs = S.even_part(np.linalg.solve(Md, S.embed_even(re).reshape(-1)))
    Sd = wilson.dense_matrix(lambda v: S.apply(v.reshape(-1, 12)).reshape(-1), (V // 2) * 12)
    rhs = np.linalg.solve(Sd, re)
    assert np.abs(lhs - rhs).max() <= 1e-11 * np.abs(rhs).max()


def test_red_black_two_level_kcycle_matches_lapack():
    """Red-black on every level: MR on the Schur systems, Schur GCR on the
    coarsest level and in the outer FGCR; the solution reaches 1e-10 against
    the dense LAPACK solve and needs no more outer steps than the plain cycle."""
    from oracle import mg
    fine = small_fine()
    n = fine.V * 12
    h = mg.Hierarchy(fine, [(2, 2, 2, 2)], [6], [synth.gaussian((6, n), 0, 1)], setup_iters=20)
    b = synth.gaussian(n, 0, 2)
    x, info = mg.solve(h, b, tol=1e-10, evenodd=True)
    assert info.converged
    Md = wilson.dense_matrix(fine.apply, n)
    assert solvers.norm(b - Md @ x) <= 1e-10 * solvers.norm(b) * (1 + 1e-6)
    x_lu = np.linalg.solve(Md, b)
    assert solvers.norm(x - x_lu) <= np.linalg.cond(Md) * 1e-10 * solvers.norm(x_lu)
    _, plain = mg.solve(h, b, tol=1e-10)
    print('outer steps: red-black', info.iters, 'plain', plain.iters, 'coarse', info.inner_iters, plain.inner_iters)
    assert info.iters <= plain.iters


def test_red_black_three_level_kcycle_converges():
    from oracle import mg
    dims = (8, 8, 4, 4)
    fine = small_fine(dims, m0=-0.3, seed=2)
    n = fine.V * 12
    starts = [synth.gaussian((6, n), 0, 1), synth.gaussian((8, 64 * 12), 1, 1)]
    h = mg.Hierarchy(fine, [(2, 2, 2, 2), (2, 2, 1, 1)], [6, 8], starts, setup_iters=15)
    b = synth.gaussian(n, 1, 2)
    x, info = mg.solve(h, b, tol=1e-10, evenodd=True)
    assert info.converged
    assert solvers.norm(b - fine.apply(x)) <= 1e-10 * solvers.norm(b) * (1 + 1e-6)
    assert info.inner_iters[1] > 0 and info.inner_iters[2] > 0
