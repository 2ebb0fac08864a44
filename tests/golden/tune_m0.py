"""Choose the bare mass m0 of the 16^3x32 workload with the oracle only.

Target: the smallest singular value of M (= the smallest |eigenvalue| of the
Hermitian Q = gamma5 M) near 1e-2, m0 <= 0.  sigma_min is found by plain
Lanczos (no restarts; the smallest Ritz value of the tridiagonal matrix, which
approaches lambda_min(Q^2) from above) on Q^2 = M^+ M using the oracle's C
restatement of Eq. (2).  If
1e-2 lies below the minimum of sigma_min over m0 (the antiperiodic time
direction keeps the lowest mode's momentum away from zero), the m0 that
minimises sigma_min is taken instead, the closest the workload can come to the
target.  Writes m0_16x16x16x32.json next to this file.

Usage: python tests/golden/tune_m0.py [--dims 16 16 16 32] [--eps 0.3] [--seed 0]
"""
import argparse
import json
import os
import sys
import time

import numpy as np
import scipy.linalg as sl

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import lattice, wilson  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--dims', type=int, nargs=4, default=[16, 16, 16, 32])
    ap.add_argument('--eps', type=float, default=0.3)
    ap.add_argument('--seed', type=int, default=0)
    ap.add_argument('--csw', type=float, default=1.0)
    ap.add_argument('--target', type=float, default=1e-2)
    ap.add_argument('--tol', type=float, default=2e-3, help='relative change of the Ritz value per 50 steps')
    ap.add_argument('--maxit', type=int, default=3000)
    ap.add_argument('--steps', type=int, default=5, help='golden-section steps')
    ap.add_argument('--out', default=os.path.join(HERE, 'm0_16x16x16x32.json'))
    args = ap.parse_args()
    dims = tuple(args.dims)
    V = lattice.volume(dims)
    U = synth.gauge_field(dims, args.eps, args.seed)
    A = wilson.clover_field(U, dims, args.csw)
    g5 = np.kron(lattice.gamma5(), np.eye(3))
    log = []

    def sigma_min(m0):
        def mv(v):
            y = wilson.apply_wilson_clover_c(v.reshape(V, 12), U, A, m0, dims) @ g5.T
            return (wilson.apply_wilson_clover_c(y, U, A, m0, dims) @ g5.T).reshape(-1)

        t = time.time()
        v = synth.gaussian(V * 12, args.seed, synth.TRAINING + 1)
        v /= np.linalg.norm(v)
        v_prev = np.zeros_like(v)
        alphas, betas = [], []
        beta = 0.0
        lam, k = np.inf, 0
        for k in range(1, args.maxit + 1):
            w = mv(v) - beta * v_prev
            alpha = float(np.vdot(v, w).real)
            w -= alpha * v
            beta = float(np.linalg.norm(w))
            alphas.append(alpha)
            betas.append(beta)
            v_prev, v = v, w / beta
            if k % 50 == 0:
                new = sl.eigh_tridiagonal(np.array(alphas), np.array(betas[:-1]), eigvals_only=True,
                                          select='i', select_range=(0, 0))[0]
                done = abs(lam - new) <= args.tol * abs(new)
                lam = new
                if done:
                    break
        s = float(np.sqrt(max(lam, 0.0)))
        log.append({'m0': m0, 'sigma_min': s, 'lanczos_steps': k, 'seconds': round(time.time() - t, 1)})
        print(json.dumps(log[-1]), flush=True)
        return s

    # golden-section search for the minimum of sigma_min over m0 in [-0.6, 0]
    gr = (np.sqrt(5) - 1) / 2
    a, b = -0.5, 0.0
    c, d = b - gr * (b - a), a + gr * (b - a)
    fc, fd = sigma_min(c), sigma_min(d)
    for _ in range(args.steps):
        if fc < fd:
            b, d, fd = d, c, fc
            c = b - gr * (b - a)
            fc = sigma_min(c)
        else:
            a, c, fc = c, d, fd
            d = a + gr * (b - a)
            fd = sigma_min(d)
    m_best, s_best = (c, fc) if fc < fd else (d, fd)
    result = {'dims': list(dims), 'eps': args.eps, 'seed': args.seed, 'csw': args.csw,
              'target_sigma_min': args.target, 'search': log}
    if s_best > args.target * 1.25:
        result.update({'m0': round(m_best, 4), 'sigma_min': s_best, 'reached_target': False,
                       'note': 'target below the minimum of sigma_min(m0); m0 minimising sigma_min'})
    else:
        # bisect on the heavier side of the minimum (m0 > m_best) for sigma_min = target
        lo, hi = m_best, 0.0
        for _ in range(12):
            mid = 0.5 * (lo + hi)
            if sigma_min(mid) < args.target:
                lo = mid
            else:
                hi = mid
        m = 0.5 * (lo + hi)
        result.update({'m0': round(m, 5), 'sigma_min': sigma_min(m), 'reached_target': True})
    with open(args.out, 'w') as f:
        json.dump(result, f, indent=1)
    print('wrote', args.out, result['m0'], result['sigma_min'])


if __name__ == '__main__':
    main()
