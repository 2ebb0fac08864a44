"""12-real link compression of the fine operator (the gauge compression of
Sec. 4 and 7.1): links stored as rows 0 and 1, row 2 rebuilt in the kernels.
Against the FP64 oracle: complex64 storage within 1e-5 (max norm), 16-bit
storages within a few units of the format's rounding; the rebuilt links
exported equal the oracle's links to the storage rounding; the red-black
pieces and a multigrid solve to 1e-10 run on compressed links (with the
per-level timing of the solve switched on)."""
import numpy as np
import pytest
import torch

import synth
from oracle import evenodd, lattice, wilson
from gpu_util import dev, host, rel_err

pytestmark = pytest.mark.gpu

U_ROUND = {'c64': 2.0 ** -24, 'h16': 2.0 ** -11, 'b16': 2.0 ** -8}


@pytest.mark.parametrize('storage', ['c64', 'h16', 'b16'])
@pytest.mark.parametrize('dims', [(8, 8, 8, 8), (6, 2, 4, 6), (3, 5, 2, 7)])
def test_compressed_links_match_oracle(storage, dims):
    from paper_1612_07873_amd import FineOp
    m0 = -0.2
    U = synth.gauge_field(dims, 0.4, 2)
    A = wilson.clover_field(U, dims, 1.0)
    V = lattice.volume(dims)
    psi = synth.gaussian((V, 4, 3), 5, 2)
    ref = wilson.apply_wilson_clover(psi, U, A, m0, dims)
    full = FineOp(dims, dev(U), m0, 1.0, True, storage)
    comp = FineOp(dims, dev(U), m0, 1.0, True, storage, link_reals=12)
    x = dev(psi, torch.complex64)
    yf, yc = host(full.apply(x)), host(comp.apply(x))
    u = U_ROUND[storage]
    ef = np.linalg.norm(yf - ref) / np.linalg.norm(ref)
    ec = np.linalg.norm(yc - ref) / np.linalg.norm(ref)
    print(dims, storage, 'norm-wise rel err: 18 reals %.2e, 12 reals %.2e' % (ef, ec))
    if storage == 'c64':
        assert rel_err(yc, ref) <= 1e-5
    else:
        assert ec <= 8 * u
    # the rebuilt links: rows 0, 1 as stored, row 2 from the cross product
    Ug = host(comp.links())
    assert np.abs(Ug - U).max() <= 8 * u


@pytest.mark.parametrize('storage', ['c64', 'h16'])
def test_compressed_links_in_the_red_black_pieces(storage):
    from paper_1612_07873_amd import FineOp
    dims, m0 = (4, 4, 4, 8), -0.2
    U = synth.gauge_field(dims, 0.4, 3)
    A = wilson.clover_field(U, dims, 1.0)
    S = evenodd.fine_schur(U, A, m0, dims)
    Vh = lattice.volume(dims) // 2
    xe = synth.gaussian((Vh, 12), 4, 2)
    op = FineOp(dims, dev(U), m0, 1.0, True, storage, link_reals=12)
    y = host(op.schur(dev(xe.reshape(Vh, 4, 3), torch.complex64))).reshape(Vh, 12)
    ref = S.apply(xe)
    err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    print(storage, 'compressed Schur norm-wise rel err %.2e' % err)
    assert err <= (1e-6 if storage == 'c64' else 8 * U_ROUND[storage])


def test_compression_needs_low_precision_storage_and_valid_count():
    from paper_1612_07873_amd import FineOp, QmgError
    U = synth.gauge_field((2, 2, 2, 2), 0.4, 0)
    with pytest.raises(QmgError, match='QMG_ERR_PREC'):
        FineOp((2, 2, 2, 2), dev(U), -0.2, 1.0, True, 'c128', link_reals=12)
    with pytest.raises(QmgError, match='QMG_ERR_ARG'):
        FineOp((2, 2, 2, 2), dev(U), -0.2, 1.0, True, 'c64', link_reals=8)


def test_multigrid_with_compressed_16bit_fine_links():
    """The K-cycle's fine operator in FP16 with 12-real links (the paper's
    fine-level form), red-black on every level: true residual 1e-10 under the
    oracle's M, and the level timing adds up to the solve."""
    import bench
    mg, Ud, m0, _, _ = bench.build_mg_16x32(coarse_storage='h16', fine_storage='h16')
    mg.set_fine_links(12)
    mg.set_evenodd(True)
    mg.set_level_timing(True)
    dims = (16, 16, 16, 32)
    b = synth.gaussian((mg.V, 4, 3), 0, 2)
    x, info = mg.solve(torch.from_numpy(b).to('cuda'), tol=1e-10)
    U = host(Ud)
    r = b - wilson.apply_wilson_clover_csw_c(host(x).reshape(b.shape), U, 1.0, m0, dims)
    tr = float(np.linalg.norm(r) / np.linalg.norm(b))
    print('16^3x32 FP16 12-real fine links, red-black', info, 'oracle-M residual %.2e' % tr)
    assert info['converged'] and tr <= 1e-10
    # level timing: every level's exclusive share is positive and the coarse
    # levels (timed with events) fit inside the solve's wall time
    ls = info['level_seconds']
    assert all(t > 0 for t in ls) and ls[1] + ls[2] < info['seconds']
