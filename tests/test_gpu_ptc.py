"""The learned smoother's kernels against the oracle (forward, gradients, Adam),
its exact reduction to the Wilson operator, training on solver-produced
pairs, and its use inside the multigrid solve (with the MR fallback)."""
import numpy as np
import pytest
import torch

import synth
from oracle import lattice, mg as omg, ptc as optc, solvers, wilson
from gpu_util import dev, host, rel_err

pytestmark = pytest.mark.gpu


def weights(C, seed, scale=0.3):
    return (scale * synth.gaussian((9, C, 1, 4, 4), seed, synth.TRAINING),
            scale * synth.gaussian((9, 1, C, 4, 4), seed + 1, synth.TRAINING))


def test_forward_and_gradients_match_oracle():
    from paper_1612_07873_amd import PTC, FineOp
    dims, C = (4, 4, 4, 8), 8
    V = lattice.volume(dims)
    U = synth.gauge_field(dims, 0.4, 2)
    net = PTC(FineOp(dims, dev(U), -0.2, 1.0, True, 'c64'), C)
    W1, W2 = weights(C, 3)
    net.set_weights(dev(W1, torch.complex64), dev(W2, torch.complex64))
    W1q, W2q = (W1.astype(np.complex64).astype(np.complex128), W2.astype(np.complex64).astype(np.complex128))
    r = synth.gaussian((V, 4, 3), 4, 2)
    y = host(net.forward(dev(r, torch.complex64)))
    yo, _ = optc.forward([W1q, W2q], r.astype(np.complex64).astype(np.complex128), U, dims)
    assert rel_err(y, yo) <= 1e-5
    pairs = [(synth.gaussian((V, 4, 3), 10 + i, 2), synth.gaussian((V, 4, 3), 20 + i, 2)) for i in range(3)]
    pq = [(a.astype(np.complex64).astype(np.complex128), b.astype(np.complex64).astype(np.complex128)) for a, b in pairs]
    net.zero_grad()
    for a, b in pairs:
        net.accumulate(dev(a, torch.complex64), dev(b, torch.complex64))
    G1, G2, L = net.grad()
    Lo, (G1o, G2o) = optc.loss_and_grads([W1q, W2q], pq, U, dims)
    print('loss gpu %.8f oracle %.8f; grad errs %.2e %.2e' % (L, Lo, rel_err(host(G1), G1o), rel_err(host(G2), G2o)))
    assert abs(L - Lo) <= 1e-5 * Lo
    assert rel_err(host(G1), G1o) <= 1e-5 and rel_err(host(G2), G2o) <= 1e-5
    # one Adam step from the same gradients
    net.adam_step(lr=1e-2)
    A1, A2 = (host(w) for w in net.weights())
    opt = optc.Adam([W1.shape, W2.shape], lr=1e-2)
    N1, N2 = opt.step([W1q, W2q], [host(G1), host(G2)])
    assert rel_err(A1, N1) <= 1e-5 and rel_err(A2, N2) <= 1e-5


def test_residual_loss_matches_oracle():
    from paper_1612_07873_amd import PTC, FineOp
    dims, C, m0 = (4, 4, 2, 8), 4, -0.2
    V = lattice.volume(dims)
    U = synth.gauge_field(dims, 0.4, 6)
    A = wilson.clover_field(U, dims, 1.0)
    net = PTC(FineOp(dims, dev(U), m0, 1.0, True, 'c64'), C)
    W1, W2 = weights(C, 7)
    net.set_weights(dev(W1, torch.complex64), dev(W2, torch.complex64))
    q = lambda a: a.astype(np.complex64).astype(np.complex128)
    rs = [synth.gaussian((V, 4, 3), 50 + i, 2) for i in range(2)]
    net.zero_grad()
    for r in rs:
        net.accumulate_residual(dev(r, torch.complex64))
    G1, G2, L = net.grad()
    M = lambda v: wilson.apply_wilson_clover(v, U, A, m0, dims)
    Lo, (G1o, G2o) = optc.loss_and_grads_residual([q(W1), q(W2)], [q(r) for r in rs], U, dims, M)
    print('residual loss gpu %.8f oracle %.8f; grad errs %.2e %.2e' % (L, Lo, rel_err(host(G1), G1o), rel_err(host(G2), G2o)))
    assert abs(L - Lo) <= 1e-5 * Lo
    assert rel_err(host(G1), G1o) <= 1e-5 and rel_err(host(G2), G2o) <= 1e-5


def test_wilson_weights_reproduce_the_wilson_kernel():
    """hidden = 1, W1 = identity, W2 = Wilson stencil weights: the network is M at c_sw = 0."""
    from paper_1612_07873_amd import PTC, FineOp
    dims, m0 = (4, 4, 2, 6), -0.25
    V = lattice.volume(dims)
    U = synth.gauge_field(dims, 0.4, 5)
    f = FineOp(dims, dev(U), m0, 0.0, True, 'c64')
    net = PTC(f, 1)
    Pm, Pp = lattice.projectors()
    W1 = np.zeros((9, 1, 1, 4, 4), dtype=np.complex64)
    W1[0, 0, 0] = np.eye(4)
    W2 = np.zeros((9, 1, 1, 4, 4), dtype=np.complex64)
    W2[0, 0, 0] = (4 + m0) * np.eye(4)
    for mu in range(4):
        W2[1 + 2 * mu, 0, 0] = -0.5 * Pm[mu]
        W2[2 + 2 * mu, 0, 0] = -0.5 * Pp[mu]
    net.set_weights(dev(W1, torch.complex64), dev(W2, torch.complex64))
    r = dev(synth.gaussian((V, 4, 3), 6, 2), torch.complex64)
    assert rel_err(host(net.forward(r)), host(f.apply(r))) <= 1e-6


def mg_problem(dims, m0, nvec=8, setup_iters=30):
    from paper_1612_07873_amd import Multigrid
    U = synth.gauge_field(dims, 0.3, 1)
    blocks = [(2, 2, 2, 2), (2, 2, 2, 2)]
    nv = [nvec, 12]
    starts, cur, dof = [], dims, 12
    for l, (bb, n) in enumerate(zip(blocks, nv)):
        starts.append(dev(synth.gaussian((n, lattice.volume(cur), dof), 40 + l, 1)))
        cur = tuple(c // x for c, x in zip(cur, bb))
        dof = 2 * n
    levels = [dict(block=bb, nvec=n, setup_iters=setup_iters, smoother_steps=4, coarse_tol=0.25, coarse_maxit=c)
              for bb, n, c in zip(blocks, nv, [10, 100])]
    return U, Multigrid(dims, dev(U), m0, 1.0, levels, starts, inner='c64')


def test_training_on_solver_pairs_and_mg_with_learned_smoother():
    from paper_1612_07873_amd import PTC, FineOp, learned
    dims, m0 = (8, 8, 8, 8), -0.3
    V = lattice.volume(dims)
    U, mg = mg_problem(dims, m0)
    rhs = [dev(synth.gaussian((V, 4, 3), 100 + i, 2)) for i in range(4)]
    R, E, infos = learned.generate_pairs(mg, rhs, maxrec=40)
    assert R.shape[0] >= 20
    # pairs are consistent: r = M e with the oracle's operator
    A = wilson.clover_field(U, dims, 1.0)
    e0 = host(E[3])
    assert rel_err(host(R[3]), wilson.apply_wilson_clover_c(e0, U, A, m0, dims)) <= 1e-5
    net = PTC(FineOp(dims, dev(U), m0, 1.0, True, 'c64'), 8)
    gen = np.random.default_rng(0)
    W1, W2 = learned.initial_weights(8, m0, gen)
    net.set_weights(dev(W1, torch.complex64), dev(W2, torch.complex64))
    L0 = learned.mean_loss(net, R, E)
    hist = learned.train(net, R, E, epochs=6, batch=8, lr=2e-3, gen=gen)
    L1 = learned.mean_loss(net, R, E)
    print('training loss %.4f -> %.4f' % (L0, L1), ['%.4f' % h for h in hist])
    assert L1 < L0
    # the residual form of the loss on the same residuals
    net_r = PTC(FineOp(dims, dev(U), m0, 1.0, True, 'c64'), 8)
    net_r.set_weights(dev(W1, torch.complex64), dev(W2, torch.complex64))
    Lr0 = learned.mean_loss(net_r, R, E, loss='residual')
    learned.train(net_r, R, E, epochs=6, batch=8, lr=2e-3, gen=gen, loss='residual')
    Lr1 = learned.mean_loss(net_r, R, E, loss='residual')
    print('residual-form training loss %.4f -> %.4f' % (Lr0, Lr1))
    assert Lr1 < Lr0
    b = synth.gaussian((V, 4, 3), 7, 2)
    x, base = mg.solve(dev(b))
    tr0 = np.linalg.norm(b - wilson.apply_wilson_clover_c(host(x), U, A, m0, dims)) / np.linalg.norm(b)
    mg.set_smoother(net)
    x, info = mg.solve(dev(b))
    tr = np.linalg.norm(b - wilson.apply_wilson_clover_c(host(x), U, A, m0, dims)) / np.linalg.norm(b)
    print('MR smoother', base, '\nlearned smoother', info, 'oracle-M residual %.2e' % tr)
    assert info['converged'] and tr <= 1e-10 and tr0 <= 1e-10
    # what the network gains over MR(4) on the same solve, both checked under
    # the oracle's operator (outer steps to 1e-10)
    cmp = {'MR(4)': base['outer_iters'], 'learned': info['outer_iters']}
    # poisoned weights: every application falls back to MR and the solve still converges
    bad = torch.full((9, 8, 1, 4, 4), float('nan'), dtype=torch.complex64, device='cuda')
    net.set_weights(bad, dev(W2, torch.complex64))
    x, info2 = mg.solve(dev(b))
    assert info2['converged'] and info2['smoother_fallbacks'] > 0
    assert info2['outer_iters'] == base['outer_iters']
    mg.set_smoother(net_r)
    x, info3 = mg.solve(dev(b))
    tr = np.linalg.norm(b - wilson.apply_wilson_clover_c(host(x), U, A, m0, dims)) / np.linalg.norm(b)
    print('residual-trained smoother', info3, 'oracle-M residual %.2e' % tr)
    assert info3['converged'] and tr <= 1e-10
    cmp['learned (residual loss)'] = info3['outer_iters']
    # the network followed by two MR steps on what it leaves
    mg.set_smoother(net_r, mr_steps=2)
    x, info4 = mg.solve(dev(b))
    tr = np.linalg.norm(b - wilson.apply_wilson_clover_c(host(x), U, A, m0, dims)) / np.linalg.norm(b)
    assert info4['converged'] and tr <= 1e-10
    cmp['learned (residual loss) + MR(2)'] = info4['outer_iters']
    # the same with the poisoned network: every network step is refused on the
    # device and counted, the MR steps still run and the solve converges
    mg.set_smoother(net, mr_steps=2)
    x, info5 = mg.solve(dev(b))
    tr = np.linalg.norm(b - wilson.apply_wilson_clover_c(host(x), U, A, m0, dims)) / np.linalg.norm(b)
    print('poisoned network + MR(2)', info5, 'oracle-M residual %.2e' % tr)
    assert info5['converged'] and tr <= 1e-10 and info5['smoother_fallbacks'] >= info5['outer_iters'] > 0
    mg.set_smoother(None)
    print('outer steps to 1e-10 by level-0 smoother:', cmp)
    # measured so far on this problem: the output-trained network ties MR(4)
    # and the residual-trained one needs about a sixth more outer steps; every
    # learned form is held to at most half again as many as MR(4)
    assert max(v for k, v in cmp.items() if k != 'MR(4)') <= 1.5 * cmp['MR(4)']


def test_recorded_smoother_inputs_match_the_oracle_kcycle():
    """The recorded level-0 smoother inputs of a 2-level solve: the first is
    the K-cycle's input b itself (x0 = 0), the second the residual after the
    pre-smoother and the coarse-grid correction, which the oracle's K-cycle
    steps reproduce from the same hierarchy (FP32 inner vs FP64: 1e-4)."""
    from paper_1612_07873_amd import Multigrid
    dims, m0 = (4, 4, 4, 8), -0.3
    V = lattice.volume(dims)
    U = synth.gauge_field(dims, 0.4, 1)
    A = wilson.clover_field(U, dims, 1.0)
    fine = omg.FineLevel(U, A, m0, dims)
    st = synth.gaussian((6, V, 12), 0, 1)
    h = omg.Hierarchy(fine, [(2, 2, 2, 2)], [6], [st.reshape(6, -1)], setup_iters=0)
    mg = Multigrid(dims, dev(U), m0, 1.0, [dict(block=(2, 2, 2, 2), nvec=6, setup_iters=0, smoother_steps=4,
                                                coarse_tol=0.25, coarse_maxit=100)], [dev(st)], inner='c64')
    b = synth.gaussian((V, 4, 3), 3, 2)
    x, R, info = mg.solve_record_smoother(dev(b), 16)
    assert info['converged'] and R.shape[0] == 16
    Rh = host(R).reshape(16, -1)
    assert np.array_equal(Rh[0], b.reshape(-1).astype(np.complex64).astype(np.complex128))
    K = omg.KCycle(h)
    r = b.reshape(-1)
    xs = K.smooth(0, r)
    rc = h.restrict(0, r - fine.apply(xs))
    xc, _ = solvers.gcr(h.levels[1].apply, rc, 0.25, 10, 100)
    xs = xs + h.prolong(0, xc)
    r2 = r - fine.apply(xs)
    err = np.linalg.norm(Rh[1] - r2) / np.linalg.norm(r2)
    print('post-smoother input vs oracle K-cycle: %.2e' % err)
    assert err <= 1e-4
