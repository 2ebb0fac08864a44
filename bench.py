"""Benchmark of the coarse-grid operator (Eq. 3) on one MI355X.

Workload: the level-1 coarse grid of the 3-level hierarchy on a 16^3x32
fine lattice (block 4^4, Nvec 24): coarse lattice 4^3x8, N = 48, FP32
storage and arithmetic.  One step = one application of the operator to one
vector.  Links are Gaussian synthetic blocks of that shape (the values do not
change bytes or flops).  To measure HBM rather than the 256 MB Infinity
Cache, the steps cycle over R copies of the operator whose total size is far
above the cache; the `warm` record repeats one copy.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def algorithmic(V, N, nrhs, cbytes, scale_bytes=0):
    """Flops and bytes of one application: each link, the input vector and the
    output counted once (perfect neighbour reuse)."""
    flops = 72 * N * N * nrhs * V
    byts = V * (9 * N * N * cbytes + 9 * scale_bytes + 2 * N * nrhs * cbytes + 2 * nrhs * scale_bytes)
    return flops, byts


def cpu_baseline(cd, N, X, Y, u, budget_s=12.0):
    """The oracle's Eq. 3 apply (numpy einsum, complex128) on the same shape."""
    import numpy as np
    from oracle import coarse
    op = coarse.CoarseOp(cd, X.astype(np.complex128), Y.astype(np.complex128))
    ref = op.apply(u)
    n, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        op.apply(u)
        n += 1
    dt = (time.perf_counter() - t0) / n
    V = X.shape[0]
    flops, _ = algorithmic(V, N, 1, 16)
    return ref, {'value': round(flops / dt / 1e9, 3), 'unit': 'GFLOP/s', 'cores': 1, 'kind': 'oracle',
                 'sample': '%d applications of the oracle Eq. 3 apply (numpy, complex128, single thread) '
                           'on the same %dx%dx%dx%d N=%d operator, %.1f s' % (n, *cd, N, n * dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=2000)
    ap.add_argument('--warmup', type=int, default=200)
    ap.add_argument('--no-cpu', action='store_true', help='skip the CPU oracle leg')
    args = ap.parse_args()
    if args.gpus != 1:
        print('bench.py measures one GPU only: the coarse-operator path is built and timed on a '
              'single MI355X; --gpus %d is not supported' % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    from paper_1612_07873_amd import CoarseOp

    dev = torch.device('cuda')
    cd, N = (4, 4, 4, 8), 48
    V = int(np.prod(cd))
    X = synth.gaussian((V, N, N), 0, 2)
    Y = synth.gaussian((8, V, N, N), 1, 2)
    u = synth.gaussian((V, N), 2, 2)
    Xd, Yd = torch.from_numpy(X).to(dev), torch.from_numpy(Y).to(dev)
    flops, byts = algorithmic(V, N, 1, 8)
    R = max(2, int(np.ceil(3 * 256e6 / byts)))      # copies: total >= 3x the Infinity Cache
    ops = [CoarseOp(cd, Xd, Yd, 'c64') for _ in range(R)]
    del Xd, Yd
    ud = torch.from_numpy(u).to(dev).to(torch.complex64)
    out = torch.empty_like(ud)
    torch.cuda.synchronize()

    for i in range(args.warmup):
        ops[i % R].apply(ud, out)
    torch.cuda.synchronize()

    # timed region: exactly K steps
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for i in range(args.steps):
        ops[i % R].apply(ud, out)
    stop.record()
    torch.cuda.synchronize()
    ms_total = start.elapsed_time(stop)
    ms_step = ms_total / args.steps

    # per-launch kernel duration (events right around each launch)
    nper = min(args.steps, 400)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(nper)]
    for i, (a, b) in enumerate(evs):
        a.record()
        ops[i % R].apply(ud, out)
        b.record()
    torch.cuda.synchronize()
    per = np.array([a.elapsed_time(b) for a, b in evs])
    kern_ms = float(np.mean(per))

    # warm: one copy, Infinity-Cache resident
    for _ in range(50):
        ops[0].apply(ud, out)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(500):
        ops[0].apply(ud, out)
    b.record()
    torch.cuda.synchronize()
    warm_ms = a.elapsed_time(b) / 500

    y = out.cpu().numpy().astype(np.complex128)
    achieved = byts / (kern_ms * 1e-3) / 1e9
    rec = {
        'metric': 'coarse-Dslash GFLOP/s & %HBM roofline; MG-GCR time to 1e-10 vs plain',
        'value': round(flops / (ms_step * 1e-3) / 1e9, 2),
        'unit': 'GFLOP/s',
        'n_gpus': 1, 'steps': args.steps, 'warmup': args.warmup,
        'ms_per_step': round(ms_step, 6),
        'higher_is_better': True, 'scaling': 'weak', 'vs_baseline': None,
        'dtype': 'f32', 'data': 'synthetic',
        'config': {'workload': 'coarse_dslash on 4^3x8, N=48 (level 1 of 16^3x32, block 4^4, Nvec 24), '
                               'single RHS, complex64, %d operator copies cycled' % R,
                   'lattice': list(cd), 'N': N, 'nrhs': 1, 'launch': list(ops[0].launch())},
        'roofline': {'bound': 'hbm', 'achieved': round(achieved, 1), 'peak': HBM_PEAK_GBS, 'unit': 'GB/s',
                     'frac': round(achieved / HBM_PEAK_GBS, 4), 'traffic': None,
                     'algorithmic_bytes_per_launch': byts, 'kernel_ms': round(kern_ms, 6)},
        'warm_cache': {'ms_per_step': round(warm_ms, 6),
                       'GFLOP/s': round(flops / (warm_ms * 1e-3) / 1e9, 2),
                       'effective_GB/s': round(byts / (warm_ms * 1e-3) / 1e9, 1)},
    }
    if not args.no_cpu:
        ref, rec['cpu_baseline'] = cpu_baseline(cd, N, X, Y, u)
        rec['parity_rel_err'] = float(np.abs(y - ref).max() / np.abs(ref).max())
    print(json.dumps(rec), flush=True)


if __name__ == '__main__':
    main()
