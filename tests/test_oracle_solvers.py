"""Pins of the oracle's solvers (MR, GCR) and K-cycle multigrid against dense
LAPACK solves and the defining properties of each iteration."""
import numpy as np

import synth
from oracle import lattice, mg, solvers, wilson


def small_problem(dims=(4, 4, 2, 4), m0=-0.2, seed=0):
    U = synth.gauge_field(dims, 0.4, seed)
    A = wilson.clover_field(U, dims, 1.0)
    return mg.FineLevel(U, A, m0, dims)


def test_mr_step_minimises_residual():
    """One MR step leaves a residual orthogonal to A r (the minimal-residual condition)."""
    fine = small_problem()
    b = synth.gaussian(fine.V * 12, 0, 2)
    x = solvers.mr(fine.apply, b, 1)
    r1 = b - fine.apply(x)
    Ar = fine.apply(b)
    assert abs(np.vdot(Ar, r1)) < 1e-12 * solvers.norm(Ar) * solvers.norm(r1)
    # more steps never increase the residual
    norms = [solvers.norm(b - fine.apply(solvers.mr(fine.apply, b, k))) for k in range(1, 6)]
    assert all(a >= b_ - 1e-12 for a, b_ in zip(norms, norms[1:]))


def test_gcr_matches_dense_lapack_solve():
    fine = small_problem()
    n = fine.V * 12
    M = wilson.dense_matrix(fine.apply, n)
    b = synth.gaussian(n, 1, 2)
    x_lu = np.linalg.solve(M, b)
    x, info = solvers.gcr(fine.apply, b, 1e-12, restart=10, maxit=2000)
    assert info.converged
    assert solvers.norm(b - M @ x) <= 1e-12 * solvers.norm(b) * 1.0001
    kappa = np.linalg.cond(M)
    assert solvers.norm(x - x_lu) <= kappa * 1e-12 * solvers.norm(x_lu)
    # the iterated residual it stops on agrees with the true one
    assert abs(info.history[-1] - solvers.norm(b - M @ x)) < 1e-3 * info.history[-1] + 1e-15


def test_gcr_residuals_are_monotone_within_a_cycle():
    fine = small_problem()
    b = synth.gaussian(fine.V * 12, 2, 2)
    _, info = solvers.gcr(fine.apply, b, 1e-8, restart=10, maxit=60)
    h = np.array(info.history)
    assert np.all(np.diff(h) <= 1e-12 * h[0])


def test_two_level_kcycle_solves_to_1e10_and_matches_lapack():
    dims = (4, 4, 4, 4)
    fine = small_problem(dims, m0=-0.3, seed=1)
    n = fine.V * 12
    starts = [synth.gaussian((6, n), 0, 1)]
    h = mg.Hierarchy(fine, [(2, 2, 2, 2)], [6], starts, setup_iters=20)
    b = synth.gaussian(n, 0, 2)
    x, info = mg.solve(h, b, tol=1e-10)
    assert info.converged
    M = wilson.dense_matrix(fine.apply, n)
    assert solvers.norm(b - M @ x) <= 1e-10 * solvers.norm(b)
    x_lu = np.linalg.solve(M, b)
    assert solvers.norm(x - x_lu) <= np.linalg.cond(M) * 1e-10 * solvers.norm(x_lu)
    # the preconditioner pays: fewer outer steps than unpreconditioned GCR(10)
    _, plain = solvers.gcr(fine.apply, b, 1e-10, 10, 5000)
    assert info.iters < plain.iters / 3


def test_null_vectors_are_rich_in_low_modes():
    """Relaxing A x = 0 lowers the Rayleigh quotient |Ax|/|x| far below that of a
    random vector (setup steps 1-2)."""
    fine = small_problem((4, 4, 4, 4), m0=-0.3, seed=1)
    n = fine.V * 12
    starts = synth.gaussian((3, n), 4, 1)
    v = mg.null_vectors(fine, starts, 30)
    q = lambda x: solvers.norm(fine.apply(x)) / solvers.norm(x)
    for k in range(3):
        assert q(v[k]) < 0.2 * q(starts[k])
        assert abs(solvers.norm(v[k]) - 1) < 1e-12
        for j in range(k):
            assert abs(np.vdot(v[j], v[k])) < 1e-12


def test_three_level_kcycle_converges():
    dims = (8, 8, 4, 4)
    fine = small_problem(dims, m0=-0.3, seed=2)
    n = fine.V * 12
    starts = [synth.gaussian((6, n), 0, 1), synth.gaussian((8, 64 * 12), 1, 1)]
    h = mg.Hierarchy(fine, [(2, 2, 2, 2), (2, 2, 1, 1)], [6, 8], starts, setup_iters=15)
    assert h.levels[2].dims == (2, 2, 2, 2) and h.levels[2].dof == 16
    b = synth.gaussian(n, 1, 2)
    x, info = mg.solve(h, b, tol=1e-10)
    assert info.converged
    assert solvers.norm(b - fine.apply(x)) <= 1e-10 * solvers.norm(b)
    assert info.inner_iters[1] > 0 and info.inner_iters[2] > 0


def test_exact_coarse_correction_zeroes_the_restricted_residual():
    """The direct coarsest solve is the exact coarse-grid correction: after
    x += P Mhat^-1 R r1 the restricted residual R (r1 - A P xc) vanishes,
    because Mhat = R A P (Galerkin).  A two-level K-cycle built on it
    converges to 1e-10 against the dense LAPACK solution, in no more outer
    steps than with the GCR coarsest solve."""
    fine = small_problem()
    starts = [synth.gaussian((6, fine.V * 12), 1, 1)]
    h = mg.Hierarchy(fine, [(2, 2, 2, 2)], [6], starts, setup_iters=20)
    K = mg.KCycle(h, coarsest_direct=True)
    r = synth.gaussian(fine.V * 12, 3, 2)
    xs = K.smooth(0, r)
    r1 = r - fine.apply(xs)
    rc = h.restrict(0, r1)
    xc = np.linalg.solve(h.levels[1].op.dense(), rc)
    after = h.restrict(0, r1 - fine.apply(h.prolong(0, xc)))
    assert solvers.norm(after) <= 1e-12 * solvers.norm(rc)
    b = synth.gaussian(fine.V * 12, 4, 2)
    x, info = mg.solve(h, b, tol=1e-10, coarsest_direct=True)
    assert solvers.norm(b - fine.apply(x)) <= 1e-10 * solvers.norm(b)
    M = wilson.dense_matrix(fine.apply, fine.V * 12)
    ref = np.linalg.solve(M, b)
    assert solvers.norm(x - ref) <= np.linalg.cond(M) * 1e-10 * solvers.norm(ref)
    _, info_gcr = mg.solve(h, b, tol=1e-10)
    assert info.iters <= info_gcr.iters
