"""The solves the benchmark times, re-checked under the oracle's FP64 M.

Each test builds the hierarchy exactly as bench.py does (its own builder:
the same gauge field, m0, level recipe, start vectors and storage) and solves
the right-hand side the benchmark solves first; the true residual
|b - M x| / |b| is then computed on the host by the oracle's plain C
restatement of Eq. (2), which forms the clover term from the links at each
site (no stored clover field, so 32^3x64 fits)."""
import numpy as np
import pytest
import torch

import bench
import synth
from oracle import wilson
from gpu_util import host

pytestmark = pytest.mark.gpu


def oracle_residual(U, m0, dims, b, x):
    r = b - wilson.apply_wilson_clover_csw_c(x.reshape(b.shape), U, 1.0, m0, dims)
    return float(np.linalg.norm(r) / np.linalg.norm(b))


@pytest.mark.parametrize('coarse_direct', [False, True])
def test_benchmarked_16x16x16x32_solve(coarse_direct):
    """The mg_gcr record: 16^3x32 at the tuned m0, FP32 inner, MR(4), GCR or
    exact coarsest solve, right-hand side seed 0."""
    mg, Ud, m0, m0_src, _ = bench.build_mg_16x32(coarse_direct=coarse_direct)
    assert m0_src.startswith('tests/golden')
    dims = (16, 16, 16, 32)
    b = synth.gaussian((mg.V, 4, 3), 0, 2)
    x, info = mg.solve(torch.from_numpy(b).to('cuda'), tol=1e-10)
    tr = oracle_residual(host(Ud), m0, dims, b, host(x))
    print('16^3x32 m0 %.4f direct %s' % (m0, coarse_direct), info, 'oracle-M residual %.3e' % tr)
    assert info['converged'] and tr <= 1e-10


def test_benchmarked_16x16x16x32_batch_fp16_coarse():
    """The multi-RHS record: FP16 coarse operators on the matrix cores, a batch
    of right-hand sides (seeds 5000..), every member checked."""
    mg, Ud, m0, _, _ = bench.build_mg_16x32(coarse_storage='h16')
    dims, nrhs = (16, 16, 16, 32), 8
    B = np.stack([synth.gaussian((mg.V, 4, 3), 5000 + k, 2) for k in range(nrhs)])
    X, infos = mg.solve_multi(torch.from_numpy(B).to('cuda'), tol=1e-10)
    Xh, U = host(X), host(Ud)
    res = [oracle_residual(U, m0, dims, B[k], Xh[k]) for k in range(nrhs)]
    print('batch of %d, fp16 coarse' % nrhs, infos[0], 'oracle-M residuals', ['%.2e' % r for r in res])
    assert all(i['converged'] for i in infos) and max(res) <= 1e-10


@pytest.mark.timeout(300)
def test_precision_form_32x32x32x64_solve():
    """The precision form: 32^3x64, FP16 fine links and clover and FP16 coarse
    operators with FP32 scales, FP32 vectors, FP64 outer GCR to 1e-10."""
    from paper_1612_07873_amd import Multigrid
    dims = (32, 32, 32, 64)
    V = int(np.prod(dims))
    m0 = bench.golden_m0()
    U = synth.gauge_field(dims, 0.3, 0)
    Ud = torch.from_numpy(U).to('cuda')
    levels, starts = bench.precision_form_levels(dims)
    mg = Multigrid(dims, Ud, m0, 1.0, [dict(L, coarse_storage='h16') for L in levels], starts, inner='c64',
                   fine_storage='h16')
    b = synth.gaussian((V, 4, 3), 0, 2)
    x, info = mg.solve(torch.from_numpy(b).to('cuda'), tol=1e-10)
    xh = host(x)
    del mg, starts, Ud
    torch.cuda.empty_cache()
    tr = oracle_residual(U, m0, dims, b, xh)
    print('32^3x64 precision form', info, 'oracle-M residual %.3e' % tr)
    assert info['converged'] and tr <= 1e-10
