"""The autotuner: every launch shape it may pick computes the same operator,
and the tuned launch (the one the benchmark times) matches the oracle at the
benchmark's full size."""
import numpy as np
import pytest
import torch

import synth
from oracle import coarse, lattice
from gpu_util import dev, host, rel_err

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize('cd,N,prec,tol', [((4, 4, 4, 8), 48, 'c64', 1e-5), ((2, 2, 2, 2), 48, 'c128', 1e-12),
                                           ((2, 2, 2, 4), 64, 'c64', 1e-5), ((2, 2, 2, 2), 2, 'c128', 1e-12)])
def test_tuned_launch_matches_oracle(cd, N, prec, tol):
    from paper_1612_07873_amd import CoarseOp
    V = lattice.volume(cd)
    X = synth.gaussian((V, N, N), 0, 2)
    Y = synth.gaussian((8, V, N, N), 1, 2)
    u = synth.gaussian((V, N), 2, 2)
    ref = coarse.CoarseOp(cd, X, Y).apply(u)
    dt = torch.complex128 if prec == 'c128' else torch.complex64
    g = CoarseOp(cd, dev(X), dev(Y), prec)
    ud, out = dev(u, dt), torch.empty((V, N), dtype=dt, device='cuda')
    for cold in (False, True):
        ms = g.tune(ud, out, cold=cold)
        y = host(g.apply(ud))
        print(cd, N, prec, 'cold' if cold else 'warm', 'tuned', g.launch(), 'prefetch', g.prefetch(), '%.4f ms' % ms)
        assert rel_err(y, ref) <= tol
        # a timed launch, also where no candidate passes the thread floor (2^4, N = 2)
        assert 0 < ms < 1e3
    # a second operator of the same shape takes the cached choice
    g2 = CoarseOp(cd, dev(X), dev(Y), prec)
    g2.tune(ud, out, cold=True)
    assert g2.launch() == g.launch() and g2.prefetch() == g.prefetch()


def test_tuned_mrhs_and_sixteen_bit():
    from paper_1612_07873_amd import CoarseOp, dequantize_sites, quantize_sites
    cd, N, nrhs = (4, 4, 4, 8), 64, 64
    V = lattice.volume(cd)
    X = synth.gaussian((V, N, N), 3, 2)
    Y = synth.gaussian((8, V, N, N), 4, 2)
    g = CoarseOp(cd, dev(X), dev(Y), 'h16')
    Xq, Yq = (host(t) for t in g.export())
    u = np.stack([synth.gaussian((V, N), j, 2) for j in range(nrhs)], axis=1)
    q, s = quantize_sites(dev(u.reshape(V * nrhs, N), torch.complex64), 'h16')
    q, s = q.reshape(V, nrhs, N), s.reshape(V, nrhs)
    y = torch.empty((V, nrhs, N), dtype=torch.complex64, device='cuda')
    g.tune_mrhs(q, s, y, cold=True)
    y = host(g.apply_mrhs(q, s))
    ud = host(dequantize_sites(q.reshape(V * nrhs, N), s.reshape(-1), 'h16')).reshape(V, nrhs, N)
    sites = np.arange(0, V, 37)
    ref = np.transpose(coarse.CoarseOp(cd, Xq, Yq).apply_sites(np.ascontiguousarray(np.transpose(ud, (0, 2, 1))), sites), (0, 2, 1))
    assert np.abs(y[sites] - ref).max() <= 1e-5 * np.abs(ref).max()
    # 16-bit single RHS tuned launch
    u1 = dev(synth.gaussian((V, N), 9, 2), torch.complex64)
    uq, us = quantize_sites(u1, 'h16')
    yq, ys = torch.empty_like(uq), torch.empty_like(us)
    g.tune(None, None, cold=True, u16=uq, uscale=us, o16=yq, oscale=ys)
    yq, ys = g.apply_scaled(uq, us)
    yd = host(dequantize_sites(yq, ys, 'h16'))
    ref1 = coarse.CoarseOp(cd, Xq, Yq).apply(host(dequantize_sites(uq, us, 'h16')))
    assert np.linalg.norm(yd - ref1) / np.linalg.norm(ref1) <= 1.5 * 2.0 ** -11


def test_tune_cache_persists(tmp_path):
    """The tuner's choices written to a file and read back by an emptied cache:
    a second tune of the same shape installs the stored launch and time without
    timing again; a file headed for another device is refused."""
    import paper_1612_07873_amd as qmg
    from paper_1612_07873_amd import CoarseOp, QmgError
    cd, N = (2, 2, 2, 4), 64
    V = lattice.volume(cd)
    X, Y = dev(synth.gaussian((V, N, N), 5, 2)), dev(synth.gaussian((8, V, N, N), 6, 2))
    ud = dev(synth.gaussian((V, N), 7, 2), torch.complex64)
    out = torch.empty((V, N), dtype=torch.complex64, device='cuda')
    qmg.tune_cache_clear()
    g = CoarseOp(cd, X, Y, 'c64')
    ms = g.tune(ud, out, cold=False)
    path = str(tmp_path / 'tune.txt')
    assert qmg.tune_cache_save(path) >= 1
    head = open(path).read().splitlines()[0]
    assert head.startswith('qmg-tune-1 gfx950') and ' hip' in head
    qmg.tune_cache_clear()
    assert qmg.tune_cache_load(path) >= 1
    g2 = CoarseOp(cd, X, Y, 'c64')
    g2.set_launch(0, 0)
    ms2 = g2.tune(ud, out, cold=False)
    assert g2.launch() == g.launch() and g2.prefetch() == g.prefetch()
    assert abs(ms2 - ms) <= 1e-6 * ms   # the stored time: nothing was timed
    bad = str(tmp_path / 'other.txt')
    with open(bad, 'w') as f:
        f.write('qmg-tune-1 gfx000 hip1\n')
    with pytest.raises(QmgError):
        qmg.tune_cache_load(bad)
    qmg.tune_cache_clear()
