"""Several right-hand sides solved together (qmg_mg_gcr_solve_multi).

Checks: a batch of identical copies of one right-hand side reproduces the
single solve bit for bit (the batched kernels do each member's arithmetic in
the single-solve order); a batch of distinct right-hand sides gives every
member a true residual of 1e-10 under the oracle's FP64 operator for its own
b (a member reading another member's data would fail this); the 16-bit
coarse storage with 8 or 16 members runs the coarse stencil on the matrix
cores and meets the same bar."""
import numpy as np
import pytest
import torch

import synth
from oracle import lattice, mg as omg, solvers, wilson
from gpu_util import dev, host

pytestmark = pytest.mark.gpu


def setup(dims, m0, blocks, nvecs, seed, coarse_storage=None, setup_iters=30):
    from paper_1612_07873_amd import Multigrid
    U = synth.gauge_field(dims, 0.3, seed)
    A = wilson.clover_field(U, dims, 1.0)
    fine = omg.FineLevel(U, A, m0, dims)
    starts, cur, dof = [], tuple(dims), 12
    for l, (b, n) in enumerate(zip(blocks, nvecs)):
        starts.append(dev(synth.gaussian((n, lattice.volume(cur), dof), 40 + l, 1)))
        cur = tuple(c // bb for c, bb in zip(cur, b))
        dof = 2 * n
    levels = [dict(block=b, nvec=n, setup_iters=setup_iters, smoother_steps=4, coarse_tol=0.25, coarse_maxit=c,
                   coarse_storage=coarse_storage)
              for b, n, c in zip(blocks, nvecs, [10] * (len(blocks) - 1) + [100])]
    mg = Multigrid(dims, dev(U), m0, 1.0, levels, starts, inner='c64')
    return mg, fine


def oracle_residuals(fine, B, X):
    out = []
    for b, x in zip(B, X):
        r = b.reshape(-1) - fine.apply(x.reshape(-1))
        out.append(solvers.norm(r) / solvers.norm(b.reshape(-1)))
    return out


def test_identical_members_reproduce_the_single_solve():
    dims, m0 = (8, 8, 8, 8), -0.3
    mg, fine = setup(dims, m0, [(2, 2, 2, 2), (2, 2, 2, 2)], [8, 12], 2)
    b = synth.gaussian((lattice.volume(dims), 4, 3), 3, 2)
    x1, i1 = mg.solve(dev(b))
    B = np.stack([b] * 4)
    X, infos = mg.solve_multi(dev(B))
    Xh, x1h = host(X), host(x1)
    print('single', i1, 'batch of 4 copies', infos[0])
    for k in range(4):
        assert np.array_equal(Xh[k], x1h)
        assert infos[k]['outer_iters'] == i1['outer_iters']
        assert infos[k]['level_iters'] == i1['level_iters']


@pytest.mark.parametrize('nrhs', [1, 3, 6])
def test_distinct_members_each_converge(nrhs):
    dims, m0 = (8, 8, 8, 8), -0.3
    mg, fine = setup(dims, m0, [(2, 2, 2, 2), (2, 2, 2, 2)], [8, 12], 2)
    V = lattice.volume(dims)
    B = np.stack([synth.gaussian((V, 4, 3), 100 + k, 2) for k in range(nrhs)])
    X, infos = mg.solve_multi(dev(B))
    res = oracle_residuals(fine, B, host(X))
    single = [mg.solve(dev(B[k]))[1]['outer_iters'] for k in range(nrhs)]
    print('nrhs', nrhs, 'batch outer', infos[0]['outer_iters'], infos[0]['level_iters'], 'single outer', single,
          'oracle residuals', ['%.2e' % r for r in res])
    assert all(i['converged'] for i in infos)
    assert max(res) <= 1e-10
    assert all(abs(i['true_rel_residual'] - r) <= 1e-12 for i, r in zip(infos, res))
    # lock step: the batch needs as many outer steps as its slowest member, give or take
    assert infos[0]['outer_iters'] <= max(single) + 2


def test_zero_member_in_a_batch():
    dims, m0 = (4, 4, 4, 8), -0.3
    mg, fine = setup(dims, m0, [(2, 2, 2, 2)], [6], 1, setup_iters=0)
    V = lattice.volume(dims)
    B = np.stack([synth.gaussian((V, 4, 3), 7, 2), np.zeros((V, 4, 3), dtype=np.complex128)])
    X, infos = mg.solve_multi(dev(B))
    Xh = host(X)
    assert np.abs(Xh[1]).max() == 0.0
    assert infos[1]['converged'] and infos[1]['true_rel_residual'] == 0.0
    assert oracle_residuals(fine, B[:1], Xh[:1])[0] <= 1e-10


@pytest.mark.parametrize('storage,nrhs', [('h16', 8), ('b16', 16)])
def test_matrix_core_coarse_stencil_in_the_batch(storage, nrhs):
    """16-bit coarse operators with N = 16 (level 1) and N = 32 (level 2) and 8
    or 16 members: both coarse stencils run as multi-right-hand-side
    matrix-core products."""
    dims, m0 = (8, 8, 8, 8), -0.3
    mg, fine = setup(dims, m0, [(2, 2, 2, 2), (2, 2, 2, 2)], [8, 16], 2, coarse_storage=storage)
    V = lattice.volume(dims)
    B = np.stack([synth.gaussian((V, 4, 3), 200 + k, 2) for k in range(nrhs)])
    X, infos = mg.solve_multi(dev(B))
    res = oracle_residuals(fine, B, host(X))
    _, i1 = mg.solve(dev(B[0]))
    print(storage, nrhs, 'batch', infos[0], 'single (member 0)', i1, 'worst oracle residual %.2e' % max(res))
    assert all(i['converged'] for i in infos)
    assert max(res) <= 1e-10
    assert infos[0]['outer_iters'] <= i1['outer_iters'] + 4


def test_largest_batch_of_64():
    """64 distinct members (the largest batch) with 16-bit coarse operators
    (N = 16 and 32): the coarse stencils run as 64-right-hand-side matrix-core
    products, and every member meets the 1e-10 bar under the oracle's M."""
    dims, m0 = (8, 8, 8, 8), -0.3
    mg, fine = setup(dims, m0, [(2, 2, 2, 2), (2, 2, 2, 2)], [8, 16], 3, coarse_storage='h16')
    V = lattice.volume(dims)
    B = np.stack([synth.gaussian((V, 4, 3), 300 + k, 2) for k in range(64)])
    X, infos = mg.solve_multi(dev(B))
    res = oracle_residuals(fine, B, host(X))
    print('64 members:', infos[0], 'worst oracle residual %.2e' % max(res))
    assert len(infos) == 64 and all(i['converged'] for i in infos)
    assert max(res) <= 1e-10


def test_bad_batch_arguments():
    from paper_1612_07873_amd import QmgError
    dims, m0 = (4, 4, 4, 8), -0.3
    mg, fine = setup(dims, m0, [(2, 2, 2, 2)], [6], 1, setup_iters=0)
    V = lattice.volume(dims)
    B = torch.zeros((65, V, 4, 3), dtype=torch.complex128, device='cuda')
    with pytest.raises(QmgError):
        mg.solve_multi(B)
