"""GPU mixed-precision BiCGStab with FP64 reliable updates (Sec. 3.3, 7.1):
the FP64 form takes about the oracle's BiCGStab step count on the same
system, and every form reaches a true residual of 1e-10 under the oracle's
FP64 M, on the whole lattice and in the red-black form (which needs fewer
steps)."""
import numpy as np
import pytest
import torch

import synth
from oracle import evenodd, lattice, solvers, wilson
from gpu_util import dev, host

pytestmark = pytest.mark.gpu


def oracle_residual(U, A, m0, dims, b, x):
    V = lattice.volume(dims)
    r = b.reshape(-1) - wilson.apply_wilson_clover(x.reshape(V, 4, 3), U, A, m0, dims).reshape(-1)
    return float(np.linalg.norm(r) / np.linalg.norm(b))


@pytest.mark.parametrize('evenodd_form', [False, True])
def test_fp64_bicgstab_step_count_matches_oracle(evenodd_form):
    from paper_1612_07873_amd import BiCGStab, FineOp
    dims, m0 = (4, 4, 2, 4), 0.1
    U = synth.gauge_field(dims, 0.4, 3)
    A = wilson.clover_field(U, dims, 1.0)
    V = lattice.volume(dims)
    b = synth.gaussian((V, 4, 3), 13, 2)
    if evenodd_form:
        S = evenodd.fine_schur(U, A, m0, dims)
        bw = b.reshape(V, 12)
        _, io = solvers.bicgstab(lambda v: S.apply(v.reshape(-1, 12)).reshape(-1), S.source(bw).reshape(-1),
                                 1e-10 * np.linalg.norm(b) / np.linalg.norm(S.source(bw)), maxit=2000)
    else:
        M = lambda v: wilson.apply_wilson_clover(v.reshape(V, 4, 3), U, A, m0, dims).reshape(-1)
        _, io = solvers.bicgstab(M, b.reshape(-1), 1e-10, maxit=2000)
    hi = FineOp(dims, dev(U), m0, 1.0, True, 'c128')
    solver = BiCGStab(hi, hi, evenodd=evenodd_form)
    x, info = solver.solve(dev(b), tol=1e-10, delta=1e-3)
    tr = oracle_residual(U, A, m0, dims, b, host(x))
    print('red-black' if evenodd_form else 'whole lattice', 'gpu', info, 'oracle steps', io.iters, 'oracle-M %.2e' % tr)
    assert info['converged'] and tr <= 1e-10
    assert abs(info['iters'] - io.iters) <= max(2, io.iters // 10)


@pytest.mark.parametrize('lo,link_reals', [('c64', 18), ('h16', 18), ('h16', 12)])
def test_mixed_precision_reliable_updates_reach_1e10(lo, link_reals):
    """Low-precision iteration (FP32, or the paper's half precision, with or
    without 12-real gauge compression) with FP64 reliable updates."""
    from paper_1612_07873_amd import BiCGStab, FineOp
    dims, m0 = (8, 8, 8, 8), -0.2
    U = synth.gauge_field(dims, 0.3, 1)
    A = wilson.clover_field(U, dims, 1.0)
    V = lattice.volume(dims)
    b = synth.gaussian((V, 4, 3), 3, 2)
    hi = FineOp(dims, dev(U), m0, 1.0, True, 'c128')
    low = FineOp(dims, dev(U), m0, 1.0, True, lo, link_reals=link_reals)
    steps = {}
    for eo in (False, True):
        solver = BiCGStab(hi, low, evenodd=eo)
        x, info = solver.solve(dev(b), tol=1e-10, delta=0.1)
        tr = oracle_residual(U, A, m0, dims, b, host(x))
        print(lo, link_reals, 'red-black' if eo else 'whole', info, 'oracle-M %.2e' % tr)
        assert info['converged'] and tr <= 1e-10
        assert info['reliable_updates'] >= 2      # the low-precision recursion alone stalls near its rounding
        steps[eo] = info['iters']
    assert steps[True] < steps[False]
