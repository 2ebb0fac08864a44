"""GPU parity of the transfer operators (blockwise chirality-split MGS basis,
prolong, restrict) against the oracle."""
import numpy as np
import pytest
import torch

import synth
from oracle import lattice, transfer
from gpu_util import dev, host, rel_err

pytestmark = pytest.mark.gpu

CASES = [  # fine dims, dof, block, nvec
    ((8, 8, 8, 8), 12, (4, 4, 4, 4), 24),          # 8^4, level 0 -> 1
    ((16, 16, 16, 32), 12, (4, 4, 4, 4), 24),      # 16^3x32 level 0 -> 1
    ((4, 4, 4, 8), 48, (2, 2, 2, 2), 32),          # 4^3x8 level 1 -> 2
    ((4, 6, 2, 4), 12, (2, 3, 1, 2), 3),           # ragged blocks, extent-1 block dims
    ((6, 2, 4, 2), 8, (3, 1, 2, 1), 5),            # coarse parent with N = 8
    ((4, 4, 4, 6), 12, (2, 2, 2, 3), 1),           # one vector: a prolong work-group spans 1024 rows
]


@pytest.mark.parametrize('dims,dof,block,nvec', CASES)
def test_basis_prolong_restrict(dims, dof, block, nvec):
    from paper_1612_07873_amd import Transfer
    V = lattice.volume(dims)
    vecs = synth.gaussian((nvec, V, dof), 7, 1)
    Vb = transfer.block_orthonormalize(vecs, dims, block)
    cd = transfer.coarse_dims(dims, block)
    Vc = lattice.volume(cd)
    uc = synth.gaussian((Vc, 2 * nvec), 8, 2)
    f = synth.gaussian((V, dof), 9, 2)
    ref_p = transfer.prolong(Vb, uc, dims, block)
    ref_r = transfer.restrict(Vb, f, dims, block)
    for storage in ('c128', 'c64'):
        t = Transfer(dims, dof, block, dev(vecs), storage)
        assert t.coarse_dims == cd and t.N == 2 * nvec
        err_b = rel_err(host(t.basis()), Vb)
        assert err_b <= 1e-12, err_b
        e_p = rel_err(host(t.prolong(dev(uc))), ref_p)
        e_r = rel_err(host(t.restrict(dev(f))), ref_r)
        assert e_p <= 1e-12 and e_r <= 1e-12, (e_p, e_r)
        if storage == 'c64':
            e_p = rel_err(host(t.prolong(dev(uc, torch.complex64))), ref_p)
            e_r = rel_err(host(t.restrict(dev(f, torch.complex64))), ref_r)
            assert e_p <= 1e-5 and e_r <= 1e-5, (e_p, e_r)
        print(dims, dof, block, nvec, storage, 'basis %.2e' % err_b)


def test_restrict_is_repeatable_and_rank_failure_reported():
    from paper_1612_07873_amd import QmgError, Transfer
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    V = lattice.volume(dims)
    vecs = synth.gaussian((6, V, 12), 1, 1)
    t = Transfer(dims, 12, block, dev(vecs))
    f = dev(synth.gaussian((V, 12), 2, 2))
    a = host(t.restrict(f))
    assert np.array_equal(a, host(t.restrict(f)))
    bad = vecs.copy()
    bad[4] = 0.5 * vecs[1] - 2j * vecs[3]
    with pytest.raises(QmgError):
        Transfer(dims, 12, block, dev(bad))
    with pytest.raises(QmgError):
        Transfer(dims, 12, (3, 4, 4, 4), dev(vecs))      # block does not divide the lattice
    with pytest.raises(QmgError):
        Transfer(dims, 12, (8, 4, 4, 4), dev(vecs))      # coarse extent 1


def _fp16_basis(Vb):
    """The basis as the 16-bit storage holds it: FP64 -> FP32 -> FP16 (round to
    nearest even each time), per real and imaginary part."""
    q = lambda a: a.astype(np.float32).astype(np.float16).astype(np.float64)
    return q(Vb.real) + 1j * q(Vb.imag)


@pytest.mark.parametrize('dims,dof,block,nvec', [CASES[1], CASES[2], CASES[3], CASES[4]])
def test_fp16_basis_prolong_restrict(dims, dof, block, nvec):
    """FP16 basis storage (complex64 fields): the arithmetic against the oracle
    applied to the rounded basis (1e-5), and the storage error against the
    oracle's FP64 transfer within 4u, u = 2^-11 the FP16 unit roundoff."""
    from paper_1612_07873_amd import Transfer
    V = lattice.volume(dims)
    vecs = synth.gaussian((nvec, V, dof), 7, 1)
    Vb = transfer.block_orthonormalize(vecs, dims, block)
    assert np.abs(Vb).max() <= 1.0
    Vq = _fp16_basis(Vb)
    cd = transfer.coarse_dims(dims, block)
    uc = synth.gaussian((lattice.volume(cd), 2 * nvec), 8, 2)
    f = synth.gaussian((V, dof), 9, 2)
    t = Transfer(dims, dof, block, dev(vecs), 'h16')
    assert rel_err(host(t.basis()), Vb) <= 1e-12          # the FP64 basis is kept for the Galerkin build
    yp = host(t.prolong(dev(uc, torch.complex64)))
    yr = host(t.restrict(dev(f, torch.complex64)))
    e_pq = rel_err(yp, transfer.prolong(Vq, uc, dims, block))
    e_rq = rel_err(yr, transfer.restrict(Vq, f, dims, block))
    assert e_pq <= 1e-5 and e_rq <= 1e-5, (e_pq, e_rq)
    u = 2.0 ** -11
    e_p = rel_err(yp, transfer.prolong(Vb, uc, dims, block))
    e_r = rel_err(yr, transfer.restrict(Vb, f, dims, block))
    assert e_p <= 4 * u and e_r <= 4 * u, (e_p, e_r)
    print(dims, dof, block, nvec, 'fp16 basis: arithmetic %.1e %.1e, storage %.1e %.1e' % (e_pq, e_rq, e_p, e_r))
    # complex128 fields use the FP64 basis whatever the storage
    assert rel_err(host(t.prolong(dev(uc))), transfer.prolong(Vb, uc, dims, block)) <= 1e-12
