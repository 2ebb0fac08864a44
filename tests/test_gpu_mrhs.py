"""Multi-RHS coarse operator on the matrix cores: parity against the oracle's
Eq. (3) applied column by column to the dequantised links and vectors (FP16
products are exact in FP32, so only the accumulation order differs: 1e-5), and
against nrhs separate applications of the single-RHS 16-bit kernel."""
import numpy as np
import pytest
import torch

import synth
from oracle import coarse, lattice
from gpu_util import dev, host

pytestmark = pytest.mark.gpu


def run_case(cd, N, nrhs, fmt, tiles=None, seed=0):
    from paper_1612_07873_amd import CoarseOp, dequantize_sites, quantize_sites
    V = lattice.volume(cd)
    X = synth.gaussian((V, N, N), seed, 2)
    Y = synth.gaussian((8, V, N, N), seed + 1, 2)
    g = CoarseOp(cd, dev(X), dev(Y), fmt)
    Xq, Yq = (host(t) for t in g.export())
    # nrhs right-hand sides with seeds 0..nrhs-1, layout [V][nrhs][N]
    u = np.stack([synth.gaussian((V, N), j, 2) for j in range(nrhs)], axis=1)
    uq, us = quantize_sites(dev(u.reshape(V * nrhs, N), torch.complex64), fmt)
    ud = host(dequantize_sites(uq, us, fmt)).reshape(V, nrhs, N)
    if tiles is not None:
        g.set_mrhs_tiles(nrhs, tiles)
    y = host(g.apply_mrhs(uq.reshape(V, nrhs, N), us.reshape(V, nrhs)))
    qop = coarse.CoarseOp(cd, Xq, Yq)
    # the oracle one site at a time on a sample of at most 64 sites (all on small lattices)
    sites = np.arange(V) if V <= 64 else np.random.default_rng(seed).choice(V, 64, replace=False)
    ref = qop.apply_sites(np.ascontiguousarray(np.transpose(ud, (0, 2, 1))), sites)   # [s][N][nrhs]
    ref = np.transpose(ref, (0, 2, 1))
    ys = y[sites]
    err = float(np.linalg.norm(ys - ref) / np.linalg.norm(ref))
    emax = float(np.abs(ys - ref).max() / np.abs(ref).max())
    return err, emax, g, uq, us, y


@pytest.mark.parametrize('cd,N', [((4, 4, 4, 8), 64), ((8, 8, 8, 16), 48), ((2, 2, 2, 2), 48)])
@pytest.mark.parametrize('nrhs', [8, 16, 32, 64])
def test_mrhs_parity(cd, N, nrhs):
    for fmt in ('h16', 'b16'):
        err, emax, *_ = run_case(cd, N, nrhs, fmt)
        print('%s N%d nrhs %d %s: rel err %.2e (max %.2e)' % (cd, N, nrhs, fmt, err, emax))
        assert emax <= 1e-5


@pytest.mark.parametrize('cd,N', [((3, 3, 2, 2), 32), ((3, 2, 3, 3), 16)])
def test_mrhs_site_count_not_a_multiple_of_8(cd, N):
    """36 and 54 sites, N = 32 and 16: site counts and operator sizes off
    the shapes of the other cases."""
    for nrhs in (16, 64):
        err, emax, *_ = run_case(cd, N, nrhs, 'h16', seed=5)
        assert emax <= 1e-5, (cd, N, nrhs, emax)


@pytest.mark.parametrize('cd,N', [((4, 4, 4, 8), 64), ((2, 2, 2, 4), 48), ((3, 3, 2, 2), 32), ((3, 2, 3, 3), 16)])
@pytest.mark.parametrize('nrhs', [8, 16, 32, 64])
def test_whole_site_form(cd, N, nrhs):
    """Tile code 8: every wave owns one row tile and all right-hand sides, the
    nine input blocks staged in LDS by direct global->LDS copies."""
    for fmt in ('h16', 'b16'):
        err, emax, *_ = run_case(cd, N, nrhs, fmt, tiles=8, seed=7)
        assert emax <= 1e-5, (cd, N, nrhs, fmt, emax)


@pytest.mark.parametrize('tiles', [1, 2, 4, 8])
def test_every_tile_shape(tiles):
    err, emax, *_ = run_case((2, 2, 2, 4), 64, 64, 'h16', tiles=tiles, seed=3)
    assert emax <= 1e-5


def test_mrhs_equals_single_rhs_kernel():
    """Column j of the batched result equals the single-RHS 16-bit kernel on
    column j with FP32 vectors holding the same dequantised values."""
    from paper_1612_07873_amd import dequantize_sites
    cd, N, nrhs = (2, 2, 2, 4), 48, 16
    V = lattice.volume(cd)
    err, emax, g, uq, us, y = run_case(cd, N, nrhs, 'h16', seed=5)
    ud = dequantize_sites(uq, us, 'h16').reshape(V, nrhs, N)
    for j in (0, 7, 15):
        yj = host(g.apply(ud[:, j, :].contiguous()))
        assert np.abs(yj - y[:, j, :]).max() <= 1e-5 * np.abs(yj).max()


def test_mrhs_rejects_bad_arguments():
    from paper_1612_07873_amd import CoarseOp, QmgError
    cd, N = (2, 2, 2, 2), 48
    V = 16
    X = synth.gaussian((V, N, N), 0, 2)
    Y = synth.gaussian((8, V, N, N), 1, 2)
    g32 = CoarseOp(cd, dev(X), dev(Y), 'c64')
    u = torch.zeros((V, 8, N), dtype=torch.int32, device='cuda')
    s = torch.ones((V, 8), dtype=torch.float32, device='cuda')
    with pytest.raises(QmgError):
        g32.apply_mrhs(u, s)                      # FP32 operator
    g16 = CoarseOp(cd, dev(X), dev(Y), 'h16')
    u12 = torch.zeros((V, 12, N), dtype=torch.int32, device='cuda')
    with pytest.raises(QmgError):
        g16.apply_mrhs(u12, torch.ones((V, 12), dtype=torch.float32, device='cuda'))   # nrhs 12
    with pytest.raises(QmgError):
        g16.set_mrhs_tiles(16, 2)                 # only one 16-wide tile at nrhs 16


def _level(cd, N, nrhs, seed):
    from paper_1612_07873_amd import CoarseOp, quantize_sites
    V = lattice.volume(cd)
    g = CoarseOp(cd, dev(synth.gaussian((V, N, N), seed, 2)), dev(synth.gaussian((8, V, N, N), seed + 1, 2)), 'h16')
    u = np.stack([synth.gaussian((V, N), seed + 10 + j, 2) for j in range(nrhs)], axis=1)
    q, s = quantize_sites(dev(u.reshape(V * nrhs, N), torch.complex64), 'h16')
    return g, q.reshape(V, nrhs, N), s.reshape(V, nrhs)


@pytest.mark.parametrize('nrhs', [16, 64])
def test_persistent_multi_level_launch_in_a_graph(nrhs):
    """8^3x16 (N 48), 4^3x8 (N 64) and 2^4 (N 48) in one persistent launch, captured
    in a HIP graph and replayed several times between eager work: every replay
    equals the per-level launches bitwise."""
    from paper_1612_07873_amd import apply_mrhs_multi
    levels = [_level((8, 8, 8, 16), 48, nrhs, 0), _level((4, 4, 4, 8), 64, nrhs, 100), _level((2, 2, 2, 2), 48, nrhs, 200)]
    ops = [l[0] for l in levels]
    ref = [op.apply_mrhs(q, s) for op, q, s in levels]          # also builds the operand-order links
    outs = [torch.empty_like(r) for r in ref]
    apply_mrhs_multi(ops, [l[1] for l in levels], [l[2] for l in levels], outs)
    torch.cuda.synchronize()
    for o, r in zip(outs, ref):
        assert torch.equal(o, r)
    for grid in (7, 256):      # any grid walks the whole queue
        outs2 = [torch.zeros_like(r) for r in ref]
        apply_mrhs_multi(ops, [l[1] for l in levels], [l[2] for l in levels], outs2, grid=grid)
        torch.cuda.synchronize()
        assert all(torch.equal(o, r) for o, r in zip(outs2, ref))
    gout = [torch.zeros_like(r) for r in ref]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            apply_mrhs_multi(ops, [l[1] for l in levels], [l[2] for l in levels], gout)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(4):
        for o in gout:
            o.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert all(torch.equal(o, r) for o, r in zip(gout, ref)), rep
        _ = [op.apply_mrhs(q, sc) for op, q, sc in levels]      # eager work between replays
    # parity of the coarsest level with the oracle (dequantised inputs)
    from paper_1612_07873_amd import dequantize_sites
    op, q, sc = levels[2]
    Xq, Yq = (host(t) for t in op.export())
    V = 16
    ud = host(dequantize_sites(q.reshape(V * nrhs, 48), sc.reshape(-1), 'h16')).reshape(V, nrhs, 48)
    refo = np.transpose(coarse.CoarseOp((2, 2, 2, 2), Xq, Yq).apply(np.ascontiguousarray(np.transpose(ud, (0, 2, 1)))), (0, 2, 1))
    assert np.abs(host(gout[2]) - refo).max() <= 1e-5 * np.abs(refo).max()
