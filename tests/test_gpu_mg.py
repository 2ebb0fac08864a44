"""GPU multigrid: hierarchy built on the device (null-vector relaxation,
transfers, Galerkin) and the K-cycle FGCR solve.  Checked against the oracle: the
true residual under the oracle's FP64 M, the oracle's iteration count for the
same hierarchy inputs, and the levels' operators against the oracle's
Galerkin build from the same vectors."""
import numpy as np
import pytest
import torch

import synth
from oracle import coarse, lattice, mg as omg, solvers, transfer, wilson
from gpu_util import dev, host, rel_err

pytestmark = pytest.mark.gpu


def problem(dims, eps, seed, m0):
    U = synth.gauge_field(dims, eps, seed)
    A = wilson.clover_field(U, dims, 1.0)
    return U, A, omg.FineLevel(U, A, m0, dims)


def level_list(blocks, nvecs, setup_iters, coarse_maxit):
    return [dict(block=b, nvec=n, setup_iters=setup_iters, smoother_steps=4, coarse_tol=0.25,
                 coarse_maxit=c) for b, n, c in zip(blocks, nvecs, coarse_maxit)]


def starts_for(dims, blocks, nvecs, seed):
    out, cur, dof = [], tuple(dims), 12
    for l, (b, n) in enumerate(zip(blocks, nvecs)):
        out.append(synth.gaussian((n, lattice.volume(cur), dof), seed + l, 1))
        cur = tuple(c // bb for c, bb in zip(cur, b))
        dof = 2 * n
    return out


@pytest.mark.parametrize('inner', ['c128', 'c64'])
def test_two_level_matches_oracle_iterations(inner):
    """Setup vectors given as data (setup_iters = 0): GPU and oracle build the
    same hierarchy; FP64 inner iteration counts must agree within 1."""
    from paper_1612_07873_amd import Multigrid
    dims, m0 = (4, 4, 4, 8), -0.3
    blocks, nvecs = [(2, 2, 2, 2)], [6]
    U, A, fine = problem(dims, 0.4, 1, m0)
    st = starts_for(dims, blocks, nvecs, 0)
    h = omg.Hierarchy(fine, blocks, nvecs, [s.reshape(nvecs[0], -1) for s in st], setup_iters=0)
    b = synth.gaussian((fine.V, 4, 3), 0, 2)
    xo, io = omg.solve(h, b.reshape(-1), tol=1e-10, coarsest_maxit=100)
    mg = Multigrid(dims, dev(U), m0, 1.0, level_list(blocks, nvecs, 0, [100]), [dev(s) for s in st], inner=inner)
    # the level-1 operator equals the oracle's Galerkin build from the same vectors
    _, N, op1, _ = mg.level(1)
    X, Y = op1.export()
    tol = 1e-12 if inner == 'c128' else 1e-5
    assert max(rel_err(host(X), h.levels[1].op.X), rel_err(host(Y), h.levels[1].op.Y)) <= tol
    x, info = mg.solve(dev(b), tol=1e-10)
    xh = host(x)
    tr = solvers.norm(b.reshape(-1) - fine.apply(xh.reshape(-1))) / solvers.norm(b.reshape(-1))
    print('inner', inner, 'gpu', info, 'oracle iters', io.iters, io.inner_iters, 'oracle-M residual %.2e' % tr)
    assert info['converged'] and tr <= 1e-10
    # the coarsest GCR (single-work-group steps: 192 entries) takes the
    # oracle's number of steps over the whole solve
    if inner == 'c128':
        assert abs(info['outer_iters'] - io.iters) <= 1
        assert abs(info['level_iters'][1] - io.inner_iters[1]) <= 1
    else:
        assert info['outer_iters'] <= io.iters + 2
        assert abs(info['level_iters'][1] - io.inner_iters[1]) <= 2


@pytest.mark.parametrize('inner', ['c128', 'c64'])
def test_coarsest_gcr_on_1536_entries_matches_oracle(inner):
    """A coarsest level of 4^4 sites x 6 (1536 entries per vector), solved to
    1e-6 so that a solve takes about six steps: in FP32 the single-work-group
    GCR step keeps its operands in registers for up to four stored directions
    and takes the loop form beyond; FP64 always the loop form.  Outer and
    coarsest step counts against the oracle's K-cycle (FP64: +-1; FP32: +-2
    outer, 5 % coarsest), true residual under the oracle's M."""
    from paper_1612_07873_amd import Multigrid
    dims, m0 = (8, 8, 8, 8), -0.3
    blocks, nvecs = [(2, 2, 2, 2)], [3]
    U, A, fine = problem(dims, 0.4, 5, m0)
    st = starts_for(dims, blocks, nvecs, 3)
    h = omg.Hierarchy(fine, blocks, nvecs, [s.reshape(nvecs[0], -1) for s in st], setup_iters=0)
    b = synth.gaussian((fine.V, 4, 3), 1, 2)
    _, io = omg.solve(h, b.reshape(-1), tol=1e-10, coarsest_tol=1e-6, coarsest_maxit=100)
    levels = level_list(blocks, nvecs, 0, [100])
    levels[0]['coarse_tol'] = 1e-6
    mg = Multigrid(dims, dev(U), m0, 1.0, levels, [dev(s) for s in st], inner=inner)
    d1, N1 = mg.level(1)[:2]
    assert lattice.volume(d1) * N1 == 1536
    x, info = mg.solve(dev(b), tol=1e-10)
    tr = solvers.norm(b.reshape(-1) - fine.apply(host(x).reshape(-1))) / solvers.norm(b.reshape(-1))
    print('inner', inner, 'gpu', info, 'oracle iters', io.iters, io.inner_iters, 'oracle-M residual %.2e' % tr)
    assert info['converged'] and tr <= 1e-10
    if inner == 'c128':
        assert abs(info['outer_iters'] - io.iters) <= 1
        assert abs(info['level_iters'][1] - io.inner_iters[1]) <= 1
    else:
        assert abs(info['outer_iters'] - io.iters) <= 2
        assert abs(info['level_iters'][1] - io.inner_iters[1]) <= max(2, 0.05 * io.inner_iters[1])


def test_three_level_with_relaxed_null_vectors():
    from paper_1612_07873_amd import Multigrid
    dims, m0 = (8, 8, 8, 8), -0.3
    blocks, nvecs = [(2, 2, 2, 2), (2, 2, 2, 2)], [8, 12]
    U, A, fine = problem(dims, 0.3, 2, m0)
    st = starts_for(dims, blocks, nvecs, 5)
    mg = Multigrid(dims, dev(U), m0, 1.0, level_list(blocks, nvecs, 30, [10, 100]), [dev(s) for s in st], inner='c64')
    b = synth.gaussian((fine.V, 4, 3), 1, 2)
    x, info = mg.solve(dev(b), tol=1e-10)
    tr = solvers.norm(b.reshape(-1) - fine.apply(host(x).reshape(-1))) / solvers.norm(b.reshape(-1))
    print('3-level 8^4', info, 'oracle-M residual %.2e' % tr)
    assert info['converged'] and tr <= 1e-10
    assert info['level_iters'][1] > 0 and info['level_iters'][2] > 0
    # the relaxed vectors are rich in low modes: the level-1 operator is much
    # better conditioned for the smooth error than plain GCR on the fine level
    x2, info2 = mg.solve(dev(b), tol=1e-10)
    assert info2['outer_iters'] == info['outer_iters']       # repeatable
    # the relaxation did its work: the same starts without it give a weaker hierarchy
    mg0 = Multigrid(dims, dev(U), m0, 1.0, level_list(blocks, nvecs, 0, [10, 100]), [dev(s) for s in st], inner='c64')
    _, info0 = mg0.solve(dev(b), tol=1e-10)
    print('unrelaxed start vectors', info0)
    assert info['outer_iters'] < info0['outer_iters']


def test_16x16x16x32_three_levels_to_1e10():
    """16^3x32, eps 0.3: block 4^4 / Nvec 24 -> 4^3x8 (N 48), block 2^4 / Nvec 32 -> 2^3x4 (N 64),
    FP32 inner, MR(4) smoothing, FP64 outer GCR(10) to 1e-10 (true residual under the oracle's M)."""
    from paper_1612_07873_amd import Multigrid
    dims, m0 = (16, 16, 16, 32), -0.25
    blocks, nvecs = [(4, 4, 4, 4), (2, 2, 2, 2)], [24, 32]
    U = synth.gauge_field(dims, 0.3, 0)
    A = wilson.clover_field(U, dims, 1.0)
    st = starts_for(dims, blocks, nvecs, 0)
    mg = Multigrid(dims, dev(U), m0, 1.0, level_list(blocks, nvecs, 100, [10, 100]), [dev(s) for s in st], inner='c64')
    b = synth.gaussian((lattice.volume(dims), 4, 3), 0, 2)
    x, info = mg.solve(dev(b), tol=1e-10)
    r = b - wilson.apply_wilson_clover_c(host(x).reshape(b.shape), U, A, m0, dims)
    tr = np.linalg.norm(r) / np.linalg.norm(b)
    print('16^3x32', info, 'oracle-M residual %.2e' % tr)
    assert info['converged'] and tr <= 1e-10


@pytest.mark.parametrize('storage', ['h16', 'b16'])
def test_three_level_16bit_coarse_storage(storage):
    """Coarse operators stored as 16-bit links with per-(site, direction)
    scales inside an FP32 K-cycle; the FP64 outer GCR still reaches 1e-10
    under the oracle's M, the stored level operators equal the full-precision
    build to 16-bit rounding, and the iteration count stays close to the
    FP32-storage solve of the same hierarchy."""
    from paper_1612_07873_amd import Multigrid
    dims, m0 = (8, 8, 8, 8), -0.3
    blocks, nvecs = [(2, 2, 2, 2), (2, 2, 2, 2)], [8, 12]
    U, A, fine = problem(dims, 0.3, 2, m0)
    st = [dev(s) for s in starts_for(dims, blocks, nvecs, 5)]
    ref_levels = level_list(blocks, nvecs, 30, [10, 100])
    mg32 = Multigrid(dims, dev(U), m0, 1.0, ref_levels, st, inner='c64')
    lv16 = [dict(L, coarse_storage=storage) for L in ref_levels]
    mg16 = Multigrid(dims, dev(U), m0, 1.0, lv16, st, inner='c64')
    unit = 2.0 ** -11 if storage == 'h16' else 2.0 ** -8
    for l in (1, 2):
        X32, Y32 = (host(a) for a in mg32.level(l)[2].export())
        X16, Y16 = (host(a) for a in mg16.level(l)[2].export())
        # per-entry error is bounded by half a unit of the block's largest component
        for a, b in ((X16, X32), (Y16, Y32)):
            bound = unit * np.abs(b).max() * 1.5
            assert np.abs(a - b).max() <= bound
    b = synth.gaussian((fine.V, 4, 3), 1, 2)
    x32, i32 = mg32.solve(dev(b), tol=1e-10)
    x16, i16 = mg16.solve(dev(b), tol=1e-10)
    tr = solvers.norm(b.reshape(-1) - fine.apply(host(x16).reshape(-1))) / solvers.norm(b.reshape(-1))
    print(storage, 'fp32 storage', i32, '16-bit coarse storage', i16, 'oracle-M residual %.2e' % tr)
    assert i16['converged'] and tr <= 1e-10
    assert i16['outer_iters'] <= i32['outer_iters'] + 3
    # and the fine operator of the K-cycle in 16 bits as well
    mgf = Multigrid(dims, dev(U), m0, 1.0, lv16, st, inner='c64', fine_storage=storage)
    xf, inf = mgf.solve(dev(b), tol=1e-10)
    tr = solvers.norm(b.reshape(-1) - fine.apply(host(xf).reshape(-1))) / solvers.norm(b.reshape(-1))
    print(storage, 'all 16-bit', inf, 'oracle-M residual %.2e' % tr)
    assert inf['converged'] and tr <= 1e-10
    assert inf['outer_iters'] <= i32['outer_iters'] + 4


def test_16bit_coarse_storage_needs_fp32_inner():
    from paper_1612_07873_amd import Multigrid
    from paper_1612_07873_amd._lib import QmgError
    dims, m0 = (4, 4, 4, 8), -0.3
    blocks, nvecs = [(2, 2, 2, 2)], [6]
    U, A, fine = problem(dims, 0.4, 1, m0)
    st = [dev(s) for s in starts_for(dims, blocks, nvecs, 0)]
    lv = [dict(L, coarse_storage='h16') for L in level_list(blocks, nvecs, 0, [100])]
    with pytest.raises(QmgError):
        Multigrid(dims, dev(U), m0, 1.0, lv, st, inner='c128')
    with pytest.raises(QmgError):
        Multigrid(dims, dev(U), m0, 1.0, level_list(blocks, nvecs, 0, [100]), st, inner='c128', fine_storage='b16')


@pytest.mark.parametrize('storage', ['h16', 'b16'])
def test_precision_form_error_at_every_level(storage):
    """Every level of a hierarchy in the 16-bit precision form against the
    FP64 oracle: the oracle rebuilds each level's Galerkin operator from the
    block bases the GPU setup produced (exported in FP64), and each stored
    operator, applied with FP32 vectors, must stay within 4u (norm-wise
    relative) of the oracle's operator; the fine level is compared with the
    oracle's M directly."""
    from paper_1612_07873_amd import Multigrid
    dims, m0 = (8, 8, 8, 8), -0.3
    blocks, nvecs = [(2, 2, 2, 2), (2, 2, 2, 2)], [8, 12]
    U, A, fine = problem(dims, 0.3, 2, m0)
    st = [dev(s) for s in starts_for(dims, blocks, nvecs, 5)]
    lv = [dict(L, coarse_storage=storage) for L in level_list(blocks, nvecs, 30, [10, 100])]
    mg = Multigrid(dims, dev(U), m0, 1.0, lv, st, inner='c64', fine_storage=storage)
    ur = 2.0 ** -11 if storage == 'h16' else 2.0 ** -8
    from paper_1612_07873_amd import FineOp
    f16 = FineOp(dims, dev(U), m0, 1.0, True, storage)
    psi = synth.gaussian((lattice.volume(dims), 4, 3), 9, 2)
    e0 = float(np.linalg.norm(host(f16.apply(dev(psi, torch.complex64))) - fine.apply(psi.reshape(-1)).reshape(psi.shape))
               / np.linalg.norm(fine.apply(psi.reshape(-1))))
    errs = [e0]
    parent = coarse.FineParent(U, A, m0, dims)
    for l in (1, 2):
        pdims, pdof, _, T = mg.level(l - 1)
        Vb = host(T.basis())          # [V][dof][Nvec], the oracle's basis layout
        ref = coarse.galerkin(parent, Vb, blocks[l - 1])
        _, N, op, _ = mg.level(l)
        u = synth.gaussian((ref.X.shape[0], N), 20 + l, 2)
        y = host(op.apply(dev(u, torch.complex64)))
        yr = ref.apply(u)
        errs.append(float(np.linalg.norm(y - yr) / np.linalg.norm(yr)))
        parent = coarse.CoarseParent(ref)
    print(storage, 'error against the FP64 oracle per level', ['%.2e' % e for e in errs], 'u=%.2e' % ur)
    assert all(e <= 4 * ur for e in errs)


def test_one_level_is_plain_gcr():
    """With no coarse level the solver is plain FP64 GCR(10) with reliable
    restarts; on a small well-conditioned system it reaches 1e-10 under the
    oracle's M, and the oracle's GCR(10) needs the same number of steps (+-2)."""
    from paper_1612_07873_amd import Multigrid
    dims, m0 = (4, 4, 4, 4), 0.2
    U, A, fine = problem(dims, 0.4, 3, m0)
    mg = Multigrid(dims, dev(U), m0, 1.0, [], [], inner='c64')
    b = synth.gaussian((fine.V, 4, 3), 4, 2)
    x, info = mg.solve(dev(b), tol=1e-10, maxit=2000)
    r = b.reshape(-1) - fine.apply(host(x).reshape(-1))
    tr = solvers.norm(r) / solvers.norm(b.reshape(-1))
    _, oi = solvers.gcr(fine.apply, b.reshape(-1), 1e-10, 10, 2000)
    print('plain GCR', info, 'oracle steps', oi.iters, 'oracle-M residual %.2e' % tr)
    assert info['converged'] and tr <= 1e-10
    assert abs(info['outer_iters'] - oi.iters) <= 2


def test_direct_coarsest_solve_matches_oracle():
    """Coarsest level solved exactly by the dense inverse built at setup: the
    FP64 two-level solve takes the oracle's outer step count (+-1) with its
    exact coarsest solve, and FP32 three levels reach 1e-10 under the
    oracle's M, in no more outer steps than with the GCR coarsest solve."""
    from paper_1612_07873_amd import Multigrid, QmgError
    dims, m0 = (4, 4, 4, 8), -0.3
    blocks, nvecs = [(2, 2, 2, 2)], [6]
    U, A, fine = problem(dims, 0.4, 1, m0)
    st = starts_for(dims, blocks, nvecs, 0)
    h = omg.Hierarchy(fine, blocks, nvecs, [s.reshape(nvecs[0], -1) for s in st], setup_iters=0)
    b = synth.gaussian((fine.V, 4, 3), 0, 2)
    _, io = omg.solve(h, b.reshape(-1), tol=1e-10, coarsest_direct=True)
    lv = [dict(L, coarse_direct=True) for L in level_list(blocks, nvecs, 0, [100])]
    mg = Multigrid(dims, dev(U), m0, 1.0, lv, [dev(s) for s in st], inner='c128')
    x, info = mg.solve(dev(b), tol=1e-10)
    tr = solvers.norm(b.reshape(-1) - fine.apply(host(x).reshape(-1))) / solvers.norm(b.reshape(-1))
    print('direct coarsest FP64', info, 'oracle', io.iters, 'oracle-M residual %.2e' % tr)
    assert info['converged'] and tr <= 1e-10
    assert abs(info['outer_iters'] - io.iters) <= 1
    # three levels in FP32, and a batch
    dims, m0 = (8, 8, 8, 8), -0.3
    blocks, nvecs = [(2, 2, 2, 2), (2, 2, 2, 2)], [8, 12]
    U, A, fine = problem(dims, 0.3, 2, m0)
    st = [dev(s) for s in starts_for(dims, blocks, nvecs, 5)]
    base = level_list(blocks, nvecs, 30, [10, 100])
    mg_gcr = Multigrid(dims, dev(U), m0, 1.0, base, st, inner='c64')
    mg_dir = Multigrid(dims, dev(U), m0, 1.0, base[:1] + [dict(base[1], coarse_direct=True)], st, inner='c64')
    b = synth.gaussian((fine.V, 4, 3), 1, 2)
    _, ig = mg_gcr.solve(dev(b), tol=1e-10)
    x, idr = mg_dir.solve(dev(b), tol=1e-10)
    tr = solvers.norm(b.reshape(-1) - fine.apply(host(x).reshape(-1))) / solvers.norm(b.reshape(-1))
    print('3 levels: GCR coarsest', ig, 'direct coarsest', idr, 'oracle-M residual %.2e' % tr)
    assert idr['converged'] and tr <= 1e-10
    assert idr['outer_iters'] <= ig['outer_iters']
    B = np.stack([synth.gaussian((fine.V, 4, 3), 50 + k, 2) for k in range(4)])
    X, infos = mg_dir.solve_multi(dev(B), tol=1e-10)
    for k in range(4):
        r = B[k].reshape(-1) - fine.apply(host(X)[k].reshape(-1))
        assert solvers.norm(r) <= 1e-10 * solvers.norm(B[k].reshape(-1))
    with pytest.raises(QmgError):
        Multigrid(dims, dev(U), m0, 1.0, [dict(base[0], coarse_direct=True), base[1]], st, inner='c64')


def test_three_level_fp16_transfer_bases():
    """Both levels' transfer bases stored as FP16 pairs for the solve (the
    Galerkin build keeps the FP64 bases, so the coarse operators are unchanged):
    the FP64 outer GCR reaches 1e-10 under the oracle's M in about the step
    count of the complex64-basis solve, whole lattice and red-black, and a
    16-bit basis is refused with complex128 inner precision."""
    from paper_1612_07873_amd import Multigrid, QmgError
    dims, m0 = (8, 8, 8, 8), -0.3
    blocks, nvecs = [(2, 2, 2, 2), (2, 2, 2, 2)], [8, 12]
    U, A, fine = problem(dims, 0.3, 2, m0)
    st = [dev(s) for s in starts_for(dims, blocks, nvecs, 5)]
    ref_levels = level_list(blocks, nvecs, 30, [10, 100])
    mg32 = Multigrid(dims, dev(U), m0, 1.0, ref_levels, st, inner='c64')
    mg16 = Multigrid(dims, dev(U), m0, 1.0, [dict(L, transfer_storage='h16') for L in ref_levels], st, inner='c64')
    for l in (1, 2):
        X32, Y32 = mg32.level(l)[2].export()
        X16, Y16 = mg16.level(l)[2].export()
        assert torch.equal(X32, X16) and torch.equal(Y32, Y16)
    b = synth.gaussian((fine.V, 4, 3), 1, 2)
    for rb in (False, True):
        mg32.set_evenodd(rb)
        mg16.set_evenodd(rb)
        _, i32 = mg32.solve(dev(b), tol=1e-10)
        x16, i16 = mg16.solve(dev(b), tol=1e-10)
        tr = solvers.norm(b.reshape(-1) - fine.apply(host(x16).reshape(-1))) / solvers.norm(b.reshape(-1))
        print('red-black' if rb else 'whole lattice', 'c64 bases', i32, 'fp16 bases', i16, 'oracle-M residual %.2e' % tr)
        assert i16['converged'] and tr <= 1e-10
        assert i16['outer_iters'] <= i32['outer_iters'] + 1
    with pytest.raises(QmgError):
        Multigrid(dims, dev(U), m0, 1.0, [dict(L, transfer_storage='h16') for L in ref_levels], st, inner='c128')
    # every 16-bit storage at once (fine, coarse, transfer bases), red-black, a batch of 8
    lv = [dict(L, transfer_storage='h16', coarse_storage='h16') for L in ref_levels]
    mga = Multigrid(dims, dev(U), m0, 1.0, lv, st, inner='c64', fine_storage='h16')
    mga.set_evenodd(True)
    B = np.stack([synth.gaussian((fine.V, 4, 3), 60 + k, 2) for k in range(8)])
    X, infos = mga.solve_multi(dev(B), tol=1e-10)
    Xh = host(X)
    for k in range(8):
        r = solvers.norm(B[k].reshape(-1) - fine.apply(Xh[k].reshape(-1))) / solvers.norm(B[k].reshape(-1))
        assert infos[k]['converged'] and r <= 1e-10, (k, r)


def test_fp16_smoother_vectors_red_black():
    """The level-0 MR smoother on the Schur system with 16-bit vectors (the
    paper's half-precision fine smoother), with 16-bit fine and coarse
    operators: the FP64 outer GCR reaches 1e-10 under the oracle's M in about
    the step count of the complex64-vector smoother, also for a batch; a
    complex64 fine operator refuses it."""
    from paper_1612_07873_amd import Multigrid, QmgError
    dims, m0 = (8, 8, 8, 8), -0.3
    blocks, nvecs = [(2, 2, 2, 2), (2, 2, 2, 2)], [8, 12]
    U, A, fine = problem(dims, 0.3, 2, m0)
    st = [dev(s) for s in starts_for(dims, blocks, nvecs, 5)]
    lv = [dict(L, coarse_storage='h16', transfer_storage='h16') for L in level_list(blocks, nvecs, 30, [10, 100])]
    mg = Multigrid(dims, dev(U), m0, 1.0, lv, st, inner='c64', fine_storage='h16')
    mg.set_evenodd(True)
    b = synth.gaussian((fine.V, 4, 3), 1, 2)
    _, i32 = mg.solve(dev(b), tol=1e-10)
    mg.set_smoother_vectors('h16')
    x, i16 = mg.solve(dev(b), tol=1e-10)
    tr = solvers.norm(b.reshape(-1) - fine.apply(host(x).reshape(-1))) / solvers.norm(b.reshape(-1))
    print('complex64 smoother vectors', i32, '16-bit smoother vectors', i16, 'oracle-M residual %.2e' % tr)
    assert i16['converged'] and tr <= 1e-10
    assert i16['outer_iters'] <= i32['outer_iters'] + 2
    B = np.stack([synth.gaussian((fine.V, 4, 3), 70 + k, 2) for k in range(3)])
    X, infos = mg.solve_multi(dev(B), tol=1e-10)
    Xh = host(X)
    for k in range(3):
        r = solvers.norm(B[k].reshape(-1) - fine.apply(Xh[k].reshape(-1))) / solvers.norm(B[k].reshape(-1))
        assert infos[k]['converged'] and r <= 1e-10, (k, r)
    mg.set_smoother_vectors(None)
    _, i32b = mg.solve(dev(b), tol=1e-10)
    assert i32b['outer_iters'] == i32['outer_iters']
    mgc = Multigrid(dims, dev(U), m0, 1.0, level_list(blocks, nvecs, 0, [10, 100]), st, inner='c64')
    with pytest.raises(QmgError):
        mgc.set_smoother_vectors('h16')


@pytest.mark.parametrize('nb', [1, 3])
def test_fp16_smoother_vectors_ragged_half_lattice(nb):
    """16-bit smoother vectors on 6x6x4x4 (288 half-lattice sites: four whole
    work-groups of the MR update and a partial fifth) with odd aggregates
    (3x3x2x2): the solve reaches 1e-10 under the oracle's M for every member,
    in about the step count of complex64 smoother vectors."""
    from paper_1612_07873_amd import Multigrid
    dims, m0 = (6, 6, 4, 4), -0.3
    blocks, nvecs = [(3, 3, 2, 2)], [6]
    U, A, fine = problem(dims, 0.3, 4, m0)
    st = [dev(s) for s in starts_for(dims, blocks, nvecs, 9)]
    lv = [dict(L, coarse_storage='h16') for L in level_list(blocks, nvecs, 10, [100])]
    mg = Multigrid(dims, dev(U), m0, 1.0, lv, st, inner='c64', fine_storage='h16')
    mg.set_evenodd(True)
    B = np.stack([synth.gaussian((fine.V, 4, 3), 90 + k, 2) for k in range(nb)])
    _, i32 = mg.solve_multi(dev(B), tol=1e-10)
    mg.set_smoother_vectors('h16')
    X, i16 = mg.solve_multi(dev(B), tol=1e-10)
    Xh = host(X)
    for k in range(nb):
        r = solvers.norm(B[k].reshape(-1) - fine.apply(Xh[k].reshape(-1))) / solvers.norm(B[k].reshape(-1))
        print(k, i32[k]['outer_iters'], i16[k]['outer_iters'], '%.2e' % r)
        assert i16[k]['converged'] and r <= 1e-10, (k, r)
        assert i16[k]['outer_iters'] <= i32[k]['outer_iters'] + 2


def test_outer_deferred_update_matches_eager():
    """The outer FGCR forms x once per cycle from the unprojected directions
    (deferred update); the recording solve, which needs x after every step,
    updates it eagerly.  Both run the same residual recursion, so after one
    cycle of ten steps their iterates agree to FP64 rounding, and the full
    solves take the same steps and meet 1e-10 under the oracle's M."""
    from paper_1612_07873_amd import Multigrid
    dims, m0 = (8, 8, 8, 8), -0.3
    blocks, nvecs = [(2, 2, 2, 2)], [8]
    U, A, fine = problem(dims, 0.3, 3, m0)
    st = [dev(s) for s in starts_for(dims, blocks, nvecs, 11)]
    mg = Multigrid(dims, dev(U), m0, 1.0, level_list(blocks, nvecs, 20, [50]), st, inner='c64')
    b = synth.gaussian((fine.V, 4, 3), 12, 2)
    xr, hist, ir = mg.solve_record(dev(b), 64)
    x1, i1 = mg.solve(dev(b), tol=1e-10, maxit=10, check=False)
    assert ir['outer_iters'] > 10 and not i1['converged']
    err = rel_err(host(x1), host(hist[9]))
    xd, idf = mg.solve(dev(b), tol=1e-10)
    print('after one cycle: deferred vs eager %.2e;' % err, 'steps', idf['outer_iters'], ir['outer_iters'])
    assert err <= 1e-11
    assert idf['outer_iters'] == ir['outer_iters']
    for x in (xr, xd):
        r = solvers.norm(b.reshape(-1) - fine.apply(host(x).reshape(-1))) / solvers.norm(b.reshape(-1))
        assert r <= 1e-10
