"""Checkpoint and resume: a transfer rebuilt from a finished basis (its own
export, or the oracle's basis taken as data), a hierarchy saved to an .npz
file and resumed without the near-null relaxation (bases, coarse operators and
solves bit for bit equal), and the learned smoother's weights with its Adam
state (training resumed from a checkpoint takes the same steps)."""
import numpy as np
import pytest
import torch

import synth
from oracle import lattice, mg as omg, solvers, transfer, wilson
from gpu_util import dev, host, rel_err

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize('storage', ['c128', 'c64'])
def test_transfer_import_reproduces_the_transfer(storage):
    from paper_1612_07873_amd import Transfer
    dims, dof, block, nvec = (4, 6, 2, 4), 12, (2, 3, 1, 2), 3
    V = lattice.volume(dims)
    vecs = synth.gaussian((nvec, V, dof), 7, 1)
    t = Transfer(dims, dof, block, dev(vecs), storage)
    B = t.basis()
    t2 = Transfer.from_basis(dims, dof, block, B, storage)
    assert t2.coarse_dims == t.coarse_dims and t2.N == t.N
    assert torch.equal(t2.basis(), B)
    cd = transfer.coarse_dims(dims, block)
    uc = dev(synth.gaussian((lattice.volume(cd), 2 * nvec), 8, 2))
    f = dev(synth.gaussian((V, dof), 9, 2))
    assert torch.equal(t2.prolong(uc), t.prolong(uc)) and torch.equal(t2.restrict(f), t.restrict(f))
    if storage == 'c64':
        u32, f32 = uc.to(torch.complex64), f.to(torch.complex64)
        assert torch.equal(t2.prolong(u32), t.prolong(u32)) and torch.equal(t2.restrict(f32), t.restrict(f32))


def test_transfer_import_of_the_oracle_basis():
    """The oracle's block-orthonormal basis, taken as data: prolong and restrict
    agree with the oracle's to FP64 rounding."""
    from paper_1612_07873_amd import Transfer
    dims, dof, block, nvec = (4, 4, 4, 8), 48, (2, 2, 2, 2), 8
    V = lattice.volume(dims)
    Vb = transfer.block_orthonormalize(synth.gaussian((nvec, V, dof), 3, 1), dims, block)
    t = Transfer.from_basis(dims, dof, block, dev(Vb))
    cd = transfer.coarse_dims(dims, block)
    uc = synth.gaussian((lattice.volume(cd), 2 * nvec), 4, 2)
    f = synth.gaussian((V, dof), 5, 2)
    assert np.array_equal(host(t.basis()), Vb)
    assert rel_err(host(t.prolong(dev(uc))), transfer.prolong(Vb, uc, dims, block)) <= 1e-12
    assert rel_err(host(t.restrict(dev(f))), transfer.restrict(Vb, f, dims, block)) <= 1e-12


def test_transfer_import_rejects_bad_shapes():
    from paper_1612_07873_amd import QmgError, Transfer
    dims = (4, 4, 4, 4)
    B = torch.zeros((lattice.volume(dims), 12, 4), dtype=torch.complex128, device='cuda')
    with pytest.raises(QmgError):
        Transfer.from_basis(dims, 12, (3, 2, 2, 2), B)      # block does not divide the lattice
    with pytest.raises(QmgError):
        Transfer.from_basis(dims, 12, (4, 2, 2, 2), B)      # coarse extent 1


def _hierarchy(inner, coarse_storage=None):
    from paper_1612_07873_amd import Multigrid
    dims, m0 = (8, 8, 8, 8), -0.3
    U = synth.gauge_field(dims, 0.3, 2)
    blocks, nvecs = [(2, 2, 2, 2), (2, 2, 2, 2)], [8, 12]
    levels = [dict(block=b, nvec=n, setup_iters=30, smoother_steps=4, coarse_tol=0.25, coarse_maxit=c)
              for b, n, c in zip(blocks, nvecs, [10, 100])]
    if coarse_storage:
        levels[0]['coarse_storage'] = coarse_storage
    starts, cur, dof = [], dims, 12
    for l, (b, n) in enumerate(zip(blocks, nvecs)):
        starts.append(dev(synth.gaussian((n, lattice.volume(cur), dof), 5 + l, 1)))
        cur = tuple(c // bb for c, bb in zip(cur, b))
        dof = 2 * n
    return dims, m0, U, Multigrid(dims, dev(U), m0, 1.0, levels, starts, inner=inner)


@pytest.mark.parametrize('inner,coarse_storage', [('c128', None), ('c64', None), ('c64', 'h16')])
def test_hierarchy_save_and_resume_bitwise(tmp_path, inner, coarse_storage):
    from paper_1612_07873_amd import Multigrid
    dims, m0, U, mg = _hierarchy(inner, coarse_storage)
    path = str(tmp_path / 'hier.npz')
    mg.save(path)
    mg2 = Multigrid.load(path)
    assert mg2.nlevels == mg.nlevels and mg2.dims == mg.dims
    for l in range(mg.nlevels):
        d, n, op, T = mg.level(l)
        d2, n2, op2, T2 = mg2.level(l)
        assert (d, n) == (d2, n2)
        if T is not None:
            assert torch.equal(T.basis(), T2.basis())
        if op is not None:
            X, Y = op.export()
            X2, Y2 = op2.export()
            assert torch.equal(X, X2) and torch.equal(Y, Y2), l
    b = synth.gaussian((lattice.volume(dims), 4, 3), 1, 2)
    x, info = mg.solve(dev(b), tol=1e-10)
    x2, info2 = mg2.solve(dev(b), tol=1e-10)
    print(inner, coarse_storage, info, info2)
    assert info['converged'] and info2['outer_iters'] == info['outer_iters']
    assert info2['level_iters'] == info['level_iters']
    assert torch.equal(x, x2)
    # the resumed hierarchy solves the oracle's system: true residual under its FP64 M
    A = wilson.clover_field(U, dims, 1.0)
    r = b - wilson.apply_wilson_clover_c(host(x2).reshape(b.shape), U, A, m0, dims)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-10
    # solver settings are not part of the checkpoint: red-black on both, still alike
    mg.set_evenodd(True)
    mg2.set_evenodd(True)
    x, info = mg.solve(dev(b), tol=1e-10)
    x2, info2 = mg2.solve(dev(b), tol=1e-10)
    assert info2['level_iters'] == info['level_iters'] and torch.equal(x, x2)


def test_hierarchy_from_oracle_bases_matches_oracle_galerkin():
    """Bases computed by the oracle, taken as data: the coarse operators the
    library builds from them equal the oracle's Galerkin products."""
    from paper_1612_07873_amd import Multigrid
    dims, m0 = (4, 4, 4, 8), -0.3
    blocks, nvecs = [(2, 2, 2, 2)], [6]
    U = synth.gauge_field(dims, 0.4, 1)
    A = wilson.clover_field(U, dims, 1.0)
    fine = omg.FineLevel(U, A, m0, dims)
    st = synth.gaussian((nvecs[0], lattice.volume(dims), 12), 0, 1)
    h = omg.Hierarchy(fine, blocks, nvecs, [st.reshape(nvecs[0], -1)], setup_iters=0)
    Vb = transfer.block_orthonormalize(st, dims, blocks[0])
    levels = [dict(block=blocks[0], nvec=nvecs[0], setup_iters=0, smoother_steps=4, coarse_tol=0.25,
                   coarse_maxit=100)]
    mg = Multigrid(dims, dev(U), m0, 1.0, levels, None, inner='c128', bases=[dev(Vb)])
    X, Y = mg.level(1)[2].export()
    assert max(rel_err(host(X), h.levels[1].op.X), rel_err(host(Y), h.levels[1].op.Y)) <= 1e-12
    b = synth.gaussian((fine.V, 4, 3), 0, 2)
    x, info = mg.solve(dev(b), tol=1e-10)
    tr = solvers.norm(b.reshape(-1) - fine.apply(host(x).reshape(-1))) / solvers.norm(b.reshape(-1))
    assert info['converged'] and tr <= 1e-10


def test_ptc_checkpoint_resumes_training(tmp_path):
    """Two Adam steps, a checkpoint, two more steps; a second network loaded from
    the checkpoint takes the same two steps to the same weights, bit for bit."""
    from paper_1612_07873_amd import PTC, FineOp
    dims, C = (4, 4, 4, 8), 4
    V = lattice.volume(dims)
    U = synth.gauge_field(dims, 0.4, 2)
    fine = FineOp(dims, dev(U), -0.2, 1.0, True, 'c64')
    W1 = 0.3 * synth.gaussian((9, C, 1, 4, 4), 3, synth.TRAINING)
    W2 = 0.3 * synth.gaussian((9, 1, C, 4, 4), 4, synth.TRAINING)
    pairs = [(dev(synth.gaussian((V, 4, 3), 10 + i, 2), torch.complex64),
              dev(synth.gaussian((V, 4, 3), 20 + i, 2), torch.complex64)) for i in range(2)]

    def step(net):
        net.zero_grad()
        for r, e in pairs:
            net.accumulate(r, e)
        net.adam_step(lr=1e-2)

    net = PTC(fine, C)
    net.set_weights(dev(W1, torch.complex64), dev(W2, torch.complex64))
    step(net)
    step(net)
    path = str(tmp_path / 'ptc.npz')
    net.save(path)
    *_, n = net.adam_state()
    assert n == 2
    step(net)
    step(net)
    net2 = PTC(fine, C)
    net2.load(path)
    m1, v1, m2, v2, n2 = net2.adam_state()
    assert n2 == 2 and float(v1.abs().max()) > 0
    step(net2)
    step(net2)
    for a, b in zip(net.weights(), net2.weights()):
        assert torch.equal(a, b)
    # set_weights clears the Adam state
    net2.set_weights(*net2.weights())
    m1, v1, m2, v2, n2 = net2.adam_state()
    assert n2 == 0 and float(m1.abs().max()) == 0 and float(v2.abs().max()) == 0
