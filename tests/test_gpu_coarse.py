"""GPU parity of coarse_dslash (Eq. 3) against the oracle: FP64 to 1e-12 and
FP32 to 1e-5 relative (max norm), over the configuration-1 Galerkin operator,
the shapes of the 3-level hierarchy, every launch shape on small grids,
ragged sizes and the edge cases of the interface."""
import numpy as np
import pytest
import torch

import synth
from oracle import coarse, lattice, transfer, wilson
from gpu_util import dev, divisors, host, rel_err

pytestmark = pytest.mark.gpu

TOL = {'c128': 1e-12, 'c64': 1e-5}
CDT = {'c128': torch.complex128, 'c64': torch.complex64}


@pytest.fixture(scope='module')
def galerkin_8x8x8x8_op():
    """Fine 8^4, eps 0.4, seed 0, c_sw 1, m0 -0.2; Gaussian Nvec 24; block 4^4 -> 2^4, N 48."""
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    V = lattice.volume(dims)
    U = synth.gauge_field(dims, 0.4, 0)
    A = wilson.clover_field(U, dims, 1.0)
    Vb = transfer.block_orthonormalize(synth.gaussian((24, V, 12), 0, 1), dims, block)
    return coarse.galerkin(coarse.FineParent(U, A, -0.2, dims), Vb, block)


def random_op(cdims, N, seed):
    Vc = lattice.volume(cdims)
    return coarse.CoarseOp(cdims, synth.gaussian((Vc, N, N), seed, 2), synth.gaussian((8, Vc, N, N), seed + 1, 2))


def gpu_apply(op, u, prec, launch=None):
    from paper_1612_07873_amd import CoarseOp
    g = CoarseOp(op.dims, dev(op.X), dev(op.Y), prec)
    if launch is not None:
        g.set_launch(*launch)
    y = g.apply(dev(u, CDT[prec]))
    return host(y), g


@pytest.mark.parametrize('prec', ['c128', 'c64'])
def test_galerkin_operator_8x8x8x8(galerkin_8x8x8x8_op, prec):
    u = synth.gaussian((16, 48), 0, 2)
    ref = galerkin_8x8x8x8_op.apply(u)
    y, _ = gpu_apply(galerkin_8x8x8x8_op, u, prec)
    err = rel_err(y, ref)
    print('8^4 Galerkin 2^4 N48 %s rel err %.3e' % (prec, err))
    assert err <= TOL[prec]


@pytest.mark.parametrize('cdims,N', [((4, 4, 4, 8), 48), ((2, 2, 2, 4), 64), ((2, 2, 2, 2), 48),
                                     ((8, 8, 8, 16), 48)])
@pytest.mark.parametrize('prec', ['c128', 'c64'])
def test_hierarchy_shapes(cdims, N, prec):
    op = random_op(cdims, N, 10)
    u = synth.gaussian((lattice.volume(cdims), N), 3, 2)
    ref = op.apply(u)
    y, g = gpu_apply(op, u, prec)
    err = rel_err(y, ref)
    print('%s N%d %s launch %s rel err %.3e' % (cdims, N, prec, g.launch(), err))
    assert err <= TOL[prec]


@pytest.mark.parametrize('prec', ['c128', 'c64'])
@pytest.mark.parametrize('cdims,N', [((2, 2, 2, 2), 48), ((2, 2, 2, 4), 64)])
def test_every_launch_shape_agrees(cdims, N, prec):
    op = random_op(cdims, N, 20)
    u = synth.gaussian((lattice.volume(cdims), N), 4, 2)
    ref = op.apply(u)
    from paper_1612_07873_amd import CoarseOp
    g = CoarseOp(op.dims, dev(op.X), dev(op.Y), prec)
    ud = dev(u, CDT[prec])
    J = g.chunks_per_row
    n = 0
    for rows in divisors(N):
        for split in divisors(J):
            if rows * split > 1024:
                continue
            g.set_launch(rows, split)
            err = rel_err(host(g.apply(ud)), ref)
            assert err <= TOL[prec], (rows, split, err)
            n += 1
    assert n > 50


@pytest.mark.parametrize('cdims,N', [((3, 2, 5, 2), 2), ((2, 3, 2, 2), 128), ((5, 2, 2, 3), 30)])
def test_ragged_and_extreme_sizes(cdims, N):
    op = random_op(cdims, N, 30)
    u = synth.gaussian((lattice.volume(cdims), N), 5, 2)
    ref = op.apply(u)
    for prec in ('c128', 'c64'):
        y, _ = gpu_apply(op, u, prec)
        assert rel_err(y, ref) <= TOL[prec]


def test_export_round_trip_and_repeatability(galerkin_8x8x8x8_op):
    from paper_1612_07873_amd import CoarseOp
    g = CoarseOp(galerkin_8x8x8x8_op.dims, dev(galerkin_8x8x8x8_op.X), dev(galerkin_8x8x8x8_op.Y), 'c128')
    X, Y = g.export()
    assert np.array_equal(host(X), galerkin_8x8x8x8_op.X) and np.array_equal(host(Y), galerkin_8x8x8x8_op.Y)
    g32 = CoarseOp(galerkin_8x8x8x8_op.dims, dev(galerkin_8x8x8x8_op.X), dev(galerkin_8x8x8x8_op.Y), 'c64')
    X32, _ = g32.export()
    assert np.array_equal(host(X32), galerkin_8x8x8x8_op.X.astype(np.complex64).astype(np.complex128))
    u = dev(synth.gaussian((16, 48), 1, 2))
    a = host(g.apply(u))
    for _ in range(3):
        assert np.array_equal(host(g.apply(u)), a)     # no atomics: bitwise repeatable


def test_interface_errors(galerkin_8x8x8x8_op):
    from paper_1612_07873_amd import CoarseOp, QmgError
    g = CoarseOp(galerkin_8x8x8x8_op.dims, dev(galerkin_8x8x8x8_op.X), dev(galerkin_8x8x8x8_op.Y), 'c128')
    u = dev(synth.gaussian((16, 48), 1, 2))
    with pytest.raises(TypeError):
        g.apply(u.to(torch.complex64))
    with pytest.raises(QmgError):
        g.set_launch(5, 1)          # 5 does not divide N = 48
    with pytest.raises(QmgError):
        g.set_launch(48, 432)       # more than 1024 threads
    g.set_launch(0, 0)
    assert g.launch()[0] > 0
