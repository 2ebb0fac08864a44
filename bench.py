"""Benchmark of the adaptive-multigrid hot path on one MI355X.

Headline (value): the coarse-grid operator of Eq. (3) on the level-1 grid of
the 16^3x32 hierarchy (coarse lattice 4^3x8, N = 48, FP32), one step = one
application to one vector, GFLOP/s = 72 N^2 V / time.  Links are Gaussian
synthetic blocks of that shape (values do not change bytes or flops).  To
measure HBM rather than the 256 MB Infinity Cache the steps cycle over R
copies of the operator whose total size is well above the cache.

Further records on the same line:
  warm_cache  the same kernel repeated on one copy (cache resident);
  precision   16-bit storage (FP16 links + FP32 scales, 16-bit vectors) on
              8^3x16/N48 and 4^3x8/N64;
  multi_rhs   the MFMA multi-right-hand-side form, nrhs 8..64, same shapes;
  mg_gcr      MG-GCR time to a true residual of 1e-10 on 16^3x32 (3 levels,
              FP32 inner, FP64 outer, MR smoother): 12 solves, the first
              discarded, mean and standard deviation of the rest; the same
              with red-black preconditioning on every level; the paper's
              comparison solver (mixed-precision BiCGStab with reliable
              updates, red-black) on the same system;
  cpu_baseline the oracle's Eq. (3) apply timed on the host.
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
TRAFFIC_FILE = os.path.join(ROOT, 'profiles', 'coarse_dslash_4x4x4x8_N48_c64_traffic.json')


def measured_traffic(launch):
    """HBM bytes per launch of the headline kernel from the counter summary, if it
    was taken on this kernel source and the same launch family (whole-site
    work-groups, rows = N); else None."""
    import hashlib
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        rec = json.load(f)
    src = os.path.join(ROOT, 'paper_1612_07873_amd', 'csrc', 'coarse_dslash.hip')
    sha = hashlib.sha256(open(src, 'rb').read()).hexdigest()
    if rec.get('source_sha256') != sha or rec.get('rows') != launch[0]:
        return None
    return rec['traffic_bytes_per_launch']
MG_M0_FILE = os.path.join(ROOT, 'tests', 'golden', 'm0_16x16x16x32.json')


def algorithmic(V, N, nrhs, cbytes, scale_bytes=0, out_cbytes=None, out_scale_bytes=None):
    """Flops and bytes of one application: each link, the input vectors and the
    outputs counted once (perfect neighbour reuse)."""
    out_cbytes = cbytes if out_cbytes is None else out_cbytes
    out_scale_bytes = scale_bytes if out_scale_bytes is None else out_scale_bytes
    flops = 72 * N * N * nrhs * V
    byts = V * (9 * N * N * cbytes + 9 * scale_bytes + N * nrhs * cbytes + nrhs * scale_bytes
                + N * nrhs * out_cbytes + nrhs * out_scale_bytes)
    return flops, byts


def timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn(0)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for i in range(steps):
        fn(i)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def host_cpu():
    """The host's CPU model, logical CPU count and the CPUs this process may use."""
    model = 'unknown'
    try:
        with open('/proc/cpuinfo') as f:
            for line in f:
                if line.startswith('model name'):
                    model = line.split(':', 1)[1].strip()
                    break
    except OSError:
        pass
    return {'cpu_model': model, 'nproc': os.cpu_count(), 'affinity_cpus': len(os.sched_getaffinity(0)),
            'omp_num_threads_env': os.environ.get('OMP_NUM_THREADS')}


def cpu_baseline(cd, N, X, Y, u, budget_s=8.0):
    """The oracle's Eq. (3) apply on the same operator, on the host: the plain C
    loop (FP64, OpenMP) with one thread and with the OpenMP default thread count
    (OMP_NUM_THREADS, the CPU share given to this process), timed with the
    steady clock; and the numpy restatement on one thread.  Each leg runs about
    budget_s seconds."""
    import numpy as np
    from oracle import coarse
    op = coarse.CoarseOp(cd, X.astype(np.complex128), Y.astype(np.complex128))
    flops, byts = algorithmic(X.shape[0], N, 1, 16)
    legs = {}
    ref = None
    for name, th in (('c_1_thread', 1), ('c_all_threads', 0)):
        sec, used, y = op.time_apply_c(u, 1, th)             # probe the cost of one apply
        reps = max(3, int(budget_s / max(sec, 1e-6)))
        sec, used, y = op.time_apply_c(u, reps, th)
        ref = y if ref is None else ref
        legs[name] = {'GFLOP/s': round(flops / sec / 1e9, 3), 'GB/s': round(byts / sec / 1e9, 2),
                      'threads': used, 'applies': reps, 'ms_per_apply': round(sec * 1e3, 4)}
    n, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s / 2:
        op.apply(u)
        n += 1
    dt = (time.perf_counter() - t0) / n
    legs['numpy_1_thread'] = {'GFLOP/s': round(flops / dt / 1e9, 3), 'applies': n}
    best = legs['c_all_threads']
    return ref, {'value': best['GFLOP/s'], 'unit': 'GFLOP/s', 'cores': best['threads'], 'kind': 'oracle',
                 'sample': 'the oracle Eq. 3 apply (plain C loop, complex128, OpenMP, gcc -O2) on the same '
                           '%dx%dx%dx%d N=%d operator: %d applies on %d threads (value) and %d on 1 thread, '
                           'about %.0f s each; numpy einsum on 1 thread beside it'
                           % (*cd, N, best['applies'], best['threads'], legs['c_1_thread']['applies'], budget_s),
                 'legs': legs, 'host': host_cpu(), 'algorithmic_bytes_per_apply_fp64': byts}


def cold_ops(cd, N, storage, X, Y, byts):
    import numpy as np
    from paper_1612_07873_amd import CoarseOp
    R = max(2, int(np.ceil(3 * 256e6 / byts)))
    return [CoarseOp(cd, X, Y, storage) for _ in range(R)]


def precision_and_mrhs(steps):
    import numpy as np
    import torch
    import synth
    from paper_1612_07873_amd import quantize_sites
    dev = torch.device('cuda')
    out = {'precision': [], 'multi_rhs': []}
    for cd, N in (((8, 8, 8, 16), 48), ((4, 4, 4, 8), 64)):
        V = int(np.prod(cd))
        X = torch.from_numpy(synth.gaussian((V, N, N), 0, 2)).to(dev)
        Y = torch.from_numpy(synth.gaussian((8, V, N, N), 1, 2)).to(dev)
        # single RHS, 16-bit links and vectors
        flops, byts = algorithmic(V, N, 1, 4, 4)
        ops = cold_ops(cd, N, 'h16', X, Y, byts)
        u = torch.from_numpy(synth.gaussian((V, N), 2, 2)).to(dev).to(torch.complex64)
        uq, us = quantize_sites(u, 'h16')
        yq, ys = torch.empty_like(uq), torch.empty_like(us)
        for op in ops:
            op.tune(None, None, cold=True, u16=uq, uscale=us, o16=yq, oscale=ys)
        ms = timed(lambda i: ops[i % len(ops)].apply_scaled(uq, us, yq, ys), steps, 20)
        out['precision'].append({'lattice': list(cd), 'N': N, 'storage': 'fp16+fp32 scale', 'ms': round(ms, 5),
                                 'GFLOP/s': round(flops / ms / 1e6, 1), 'GB/s': round(byts / ms / 1e6, 1),
                                 'hbm_frac': round(byts / ms / 1e6 / HBM_PEAK_GBS, 4), 'copies': len(ops)})
        del ops
        for nrhs in (8, 16, 32, 64):
            flops, byts = algorithmic(V, N, nrhs, 4, 4, out_cbytes=8, out_scale_bytes=0)
            ops = cold_ops(cd, N, 'h16', X, Y, byts)
            um = torch.from_numpy(np.stack([synth.gaussian((V, N), j, 2) for j in range(nrhs)], axis=1)
                                  ).to(dev).to(torch.complex64)
            q, s = quantize_sites(um.reshape(V * nrhs, N), 'h16')
            q, s = q.reshape(V, nrhs, N), s.reshape(V, nrhs)
            y = torch.empty((V, nrhs, N), dtype=torch.complex64, device=dev)
            for op in ops:
                op.apply_mrhs(q, s, y)      # builds the operand-order copy outside the timing
                op.tune_mrhs(q, s, y, cold=True)
            ms = timed(lambda i: ops[i % len(ops)].apply_mrhs(q, s, y), max(20, steps // 4), 5)
            out['multi_rhs'].append({'lattice': list(cd), 'N': N, 'nrhs': nrhs, 'ms': round(ms, 5),
                                     'tiles_tuned': ops[0].mrhs_tiles(nrhs),
                                     'GFLOP/s': round(flops / ms / 1e6, 1), 'GB/s': round(byts / ms / 1e6, 1),
                                     'hbm_frac': round(byts / ms / 1e6 / HBM_PEAK_GBS, 4),
                                     'mfma_frac_fp16': round(flops / ms / 1e9 / 2500.0, 4)})
            del ops
    return out


def multi_level(nrhs_list=(16, 64), reps=50):
    """The multi-RHS stencil on the three batched levels of the hierarchy
    (8^3x16 N48, 4^3x8 N64, 2^4 N48, FP16): the three tuned per-level launches
    back to back, against one persistent launch that walks the sites of all
    three (qmg_coarse_dslash_mrhs_multi) captured in a HIP graph and replayed."""
    import numpy as np
    import torch
    import synth
    from paper_1612_07873_amd import CoarseOp, apply_mrhs_multi, quantize_sites
    dev = torch.device('cuda')
    shapes = (((8, 8, 8, 16), 48), ((4, 4, 4, 8), 64), ((2, 2, 2, 2), 48))
    ops = []
    for k, (cd, N) in enumerate(shapes):
        V = int(np.prod(cd))
        X = torch.from_numpy(synth.gaussian((V, N, N), 10 * k, 2)).to(dev)
        Y = torch.from_numpy(synth.gaussian((8, V, N, N), 10 * k + 1, 2)).to(dev)
        ops.append(CoarseOp(cd, X, Y, 'h16'))
        del X, Y
    out = []
    for nrhs in nrhs_list:
        qs, ss, ys, byts = [], [], [], 0
        for k, ((cd, N), op) in enumerate(zip(shapes, ops)):
            V = int(np.prod(cd))
            um = torch.from_numpy(np.stack([synth.gaussian((V, N), 100 * k + j, 2) for j in range(nrhs)], axis=1)
                                  ).to(dev).to(torch.complex64)
            q, sc = quantize_sites(um.reshape(V * nrhs, N), 'h16')
            qs.append(q.reshape(V, nrhs, N))
            ss.append(sc.reshape(V, nrhs))
            ys.append(torch.empty((V, nrhs, N), dtype=torch.complex64, device=dev))
            op.apply_mrhs(qs[-1], ss[-1], ys[-1])
            op.tune_mrhs(qs[-1], ss[-1], ys[-1], cold=True)
            byts += algorithmic(V, N, nrhs, 4, 4, out_cbytes=8, out_scale_bytes=0)[1]
        ms_sep = timed(lambda i: [op.apply_mrhs(q, sc, y) for op, q, sc, y in zip(ops, qs, ss, ys)], reps, 5)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(side):
            apply_mrhs_multi(ops, qs, ss, ys)
            with torch.cuda.graph(g, stream=side):
                apply_mrhs_multi(ops, qs, ss, ys)
        torch.cuda.current_stream().wait_stream(side)
        ms_graph = timed(lambda i: g.replay(), reps, 5)
        out.append({'nrhs': nrhs, 'levels': [list(cd) + [N] for cd, N in shapes],
                    'separate_launches_us': round(ms_sep * 1e3, 2), 'persistent_graph_us': round(ms_graph * 1e3, 2),
                    'hbm_frac_separate': round(byts / ms_sep / 1e6 / HBM_PEAK_GBS, 4),
                    'hbm_frac_persistent': round(byts / ms_graph / 1e6 / HBM_PEAK_GBS, 4),
                    'tiles_tuned': [op.mrhs_tiles(nrhs) for op in ops]})
        del qs, ss, ys, g
    return out


def small_grids(steps=2000):
    """The smallest coarse grids (the Amdahl limit the fine-grained split is
    for): 2^4 N48 in FP64 and FP32 (the 8^4 workload's coarse level) and
    2^3x4 N64 in FP32 (level 2 of 16^3x32), tuned, back-to-back launches.  The
    operators (5.3 / 2.7 / 9.5 MB) stay in the caches, so the figure is
    launch-to-launch time, reported against the algorithmic bytes.  The last
    entry, the same kernel on a 2^4 operator with N = 2 (10 KB), is the fixed
    cost of one launch that the others are to be read against.  `us_in_graph`
    replays 200 captured launches: the device time per launch without the
    host's submission rate."""
    import numpy as np
    import torch
    import synth
    from paper_1612_07873_amd import CoarseOp
    dev = torch.device('cuda')
    out = []
    for cd, N, prec, cb in (((2, 2, 2, 2), 48, 'c128', 16), ((2, 2, 2, 2), 48, 'c64', 8), ((2, 2, 2, 4), 64, 'c64', 8),
                            ((2, 2, 2, 2), 2, 'c128', 16)):
        V = int(np.prod(cd))
        X = torch.from_numpy(synth.gaussian((V, N, N), 0, 2)).to(dev)
        Y = torch.from_numpy(synth.gaussian((8, V, N, N), 1, 2)).to(dev)
        op = CoarseOp(cd, X, Y, prec)
        dt = torch.complex128 if prec == 'c128' else torch.complex64
        u = torch.from_numpy(synth.gaussian((V, N), 2, 2)).to(dev).to(dt)
        y = torch.empty_like(u)
        op.tune(u, y)
        ms = timed(lambda i: op.apply(u, y), steps, 200)
        # the same launches captured in a HIP graph and replayed: device time per
        # launch without the host's submission rate
        g, reps = torch.cuda.CUDAGraph(), 200
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            op.apply(u, y)
        torch.cuda.current_stream().wait_stream(side)
        with torch.cuda.graph(g):
            for _ in range(reps):
                op.apply(u, y)
        g.replay()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(10):
            g.replay()
        b.record()
        torch.cuda.synchronize()
        ms_graph = a.elapsed_time(b) / (10 * reps)
        flops, byts = algorithmic(V, N, 1, cb)
        out.append({'lattice': list(cd), 'N': N, 'prec': prec, 'us': round(ms * 1e3, 3),
                    'us_in_graph': round(ms_graph * 1e3, 3),
                    'GFLOP/s': round(flops / ms / 1e6, 1), 'GB/s_algorithmic': round(byts / ms / 1e6, 1),
                    'GB/s_algorithmic_in_graph': round(byts / ms_graph / 1e6, 1),
                    'launch': list(op.launch()) + [op.prefetch()]})
    return out


def golden_m0(with_source=False):
    """m0 of the 16^3x32 workload (searched with the oracle, stored under tests/golden)."""
    m0, src = -0.25, 'provisional'
    if os.path.exists(MG_M0_FILE):
        with open(MG_M0_FILE) as f:
            m0 = float(json.load(f)['m0'])
        src = 'tests/golden/m0_16x16x16x32.json'
    return (m0, src) if with_source else m0


def precision_form_levels(dims):
    """Level recipe and start vectors (on the device) of the 32^3x64 precision form:
    block 4^4 / Nvec 24, then block 2^4 / Nvec 32."""
    import numpy as np
    import torch
    import synth
    V = int(np.prod(dims))
    b1 = [d // 4 for d in dims]
    levels = [dict(block=(4, 4, 4, 4), nvec=24, setup_iters=100, smoother_steps=4, coarse_tol=0.25, coarse_maxit=10),
              dict(block=(2, 2, 2, 2), nvec=32, setup_iters=100, smoother_steps=4, coarse_tol=0.25, coarse_maxit=100)]
    starts = [torch.from_numpy(synth.gaussian((24, V, 12), 0, 1)).to('cuda'),
              torch.from_numpy(synth.gaussian((32, int(np.prod(b1)), 48), 1, 1)).to('cuda')]
    return levels, starts


def build_mg_16x32(coarse_storage=None, fine_storage=None, coarse_direct=False, transfer_storage=None):
    import numpy as np
    import torch
    import synth
    from paper_1612_07873_amd import Multigrid
    dev = torch.device('cuda')
    dims = (16, 16, 16, 32)
    m0, m0_src = golden_m0(True)
    V = int(np.prod(dims))
    U = torch.from_numpy(synth.gauge_field(dims, 0.3, 0)).to(dev)
    levels = [dict(block=(4, 4, 4, 4), nvec=24, setup_iters=100, smoother_steps=4, coarse_tol=0.25, coarse_maxit=10,
                   coarse_storage=coarse_storage, transfer_storage=transfer_storage),
              dict(block=(2, 2, 2, 2), nvec=32, setup_iters=100, smoother_steps=4, coarse_tol=0.25, coarse_maxit=100,
                   coarse_storage=coarse_storage, coarse_direct=coarse_direct, transfer_storage=transfer_storage)]
    starts = [torch.from_numpy(synth.gaussian((24, V, 12), 0, 1)).to(dev),
              torch.from_numpy(synth.gaussian((32, 512, 48), 1, 1)).to(dev)]
    t0 = time.perf_counter()
    mg = Multigrid(dims, U, m0, 1.0, levels, starts, inner='c64', fine_storage=fine_storage)
    torch.cuda.synchronize()
    return mg, U, m0, m0_src, time.perf_counter() - t0


def torch_sync():
    import torch
    torch.cuda.synchronize()


def timed_batches(mg, nrhs, nbatches, seed0):
    """Time-to-solution per right-hand side of batched solves (first batch untimed)."""
    import numpy as np
    import torch
    import synth
    times, iters, res, fb = [], [], [], []
    for i in range(nbatches + 1):
        B = torch.from_numpy(np.stack([synth.gaussian((mg.V, 4, 3), seed0 + i * nrhs + k, 2)
                                       for k in range(nrhs)])).to('cuda')
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, infos = mg.solve_multi(B, tol=1e-10)
        torch.cuda.synchronize()
        if i == 0:
            continue
        times.append(time.perf_counter() - t)
        iters.append(infos[0]['outer_iters'])
        res.append(max(x['true_rel_residual'] for x in infos))
        fb.append(infos[0]['smoother_fallbacks'])
    t = np.array(times)
    return {'nrhs': nrhs, 'batches': nbatches, 'batch_time_s': round(float(t.mean()), 4),
            'time_per_rhs_s': round(float(t.mean()) / nrhs, 5), 'outer_iters_mean': float(np.mean(iters)),
            'level_iters_last': infos[0]['level_iters'], 'max_true_rel_residual': float(max(res)),
            'smoother_fallbacks_mean': float(np.mean(fb))}


def timed_solves(mg, nsolves, seed0):
    import numpy as np
    import torch
    import synth
    times, iters, res, fb = [], [], [], []
    for i in range(nsolves):
        b = torch.from_numpy(synth.gaussian((mg.V, 4, 3), seed0 + i, 2)).to('cuda')
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, info = mg.solve(b, tol=1e-10)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
        iters.append(info['outer_iters'])
        res.append(info['true_rel_residual'])
        fb.append(info['smoother_fallbacks'])
    t = np.array(times[1:])
    return {'solves': nsolves, 'time_to_1e-10_s': round(float(t.mean()), 4), 'std_s': round(float(t.std()), 4),
            'outer_iters_mean': float(np.mean(iters[1:])), 'level_iters_last': info['level_iters'],
            'max_true_rel_residual': float(max(res)), 'smoother_fallbacks_mean': float(np.mean(fb[1:]))}


def learned(npairs, epochs, loss, source='smoother'):
    """Learned-smoother comparison on 16^3x32: training data from the solver
    (source 'smoother': the residuals the level-0 smoother is applied to, for
    the residual loss; 'iterates': error/residual pairs of the outer
    iterates), training on the GPU."""
    import numpy as np
    import torch
    import synth
    from paper_1612_07873_amd import PTC, FineOp, learned as L
    mg, U, m0, m0_src, setup = build_mg_16x32()
    dims = (16, 16, 16, 32)
    plain = timed_solves(mg, 12, 1000)
    t0 = time.perf_counter()
    R, E, n = [], [], 0
    seed = 2000
    while n < npairs:
        b = torch.from_numpy(synth.gaussian((mg.V, 4, 3), seed, 2)).to('cuda')
        if source == 'smoother':
            r, _ = L.generate_smoother_inputs(mg, [b], maxrec=64)
            e = r[:0]
        else:
            r, e, _ = L.generate_pairs(mg, [b], maxrec=40)
        if loss == 'residual':
            e = e[:0]
        R.append(r)
        E.append(e)
        n += r.shape[0]
        seed += 1
    R = torch.cat(R)[:npairs]
    E = torch.cat(E)[:npairs] if loss != 'residual' else R[:0]
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t0
    net = PTC(FineOp(dims, U, m0, 1.0, True, 'c64'), 8)
    gen = np.random.default_rng(0)
    W1, W2 = L.initial_weights(8, m0, gen)
    net.set_weights(torch.from_numpy(W1).cuda(), torch.from_numpy(W2).cuda())
    t0 = time.perf_counter()
    hist = L.train(net, R, E, epochs=epochs, batch=16, lr=2e-3, gen=gen, loss=loss)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    mg.set_smoother(net)
    withnet = timed_solves(mg, 12, 1000)
    # the network step followed by two MR steps on the residual it leaves
    mg.set_smoother(net, mr_steps=2)
    hybrid = timed_solves(mg, 12, 1000)
    mg.set_smoother(net, mr_steps=1)
    hybrid1 = timed_solves(mg, 12, 1000)
    mg.set_smoother(None)
    del mg
    # the comparison the method is judged by: 16-bit fine and coarse storage,
    # 16 right-hand sides at once (matrix-core coarse stencils) and the
    # learned smoother, against the plain FP32 single-right-hand-side solve
    mg16, _, _, _, _ = build_mg_16x32(coarse_storage='h16', fine_storage='h16')
    mg16.set_smoother(net)
    combo = timed_batches(mg16, 16, 2, 1000)
    mg16.set_smoother(net, mr_steps=2)
    combo_h = timed_batches(mg16, 16, 2, 1000)
    mg16.set_smoother(None)
    combo_mr = timed_batches(mg16, 16, 2, 1000)
    del mg16
    # and with every 16-bit storage the build has (transfer bases too) and
    # red-black preconditioning on every level (the network acts on the whole
    # fine lattice, the MR steps after it too)
    mgb, _, _, _, _ = build_mg_16x32(coarse_storage='h16', fine_storage='h16', transfer_storage='h16')
    mgb.set_evenodd(True)
    mgb.set_smoother(net)
    rb_l = timed_batches(mgb, 16, 2, 1000)
    mgb.set_smoother(net, mr_steps=2)
    rb_h = timed_batches(mgb, 16, 2, 1000)
    mgb.set_smoother(None)
    rb_mr = timed_batches(mgb, 16, 2, 1000)
    # the MR smoother of the Schur system on 16-bit vectors (half-precision fine smoother)
    mgb.set_smoother_vectors('h16')
    rb_mr16 = timed_batches(mgb, 16, 2, 1000)
    del mgb
    for c in (combo, combo_mr, combo_h, rb_l, rb_h, rb_mr, rb_mr16):
        c['speedup_per_rhs_vs_single_fp32_MR'] = round(plain['time_to_1e-10_s'] / c['time_per_rhs_s'], 3)
    return {'lattice': list(dims), 'm0': m0, 'training_data': source, 'pairs': int(R.shape[0]),
            'pair_seconds': round(t_pairs, 2),
            'loss': loss, 'epochs': epochs, 'loss_history': [round(h, 5) for h in hist],
            'train_seconds': round(t_train, 2), 'mg_with_MR': plain, 'mg_with_learned': withnet,
            'mg_with_learned_then_MR2': hybrid, 'mg_with_learned_then_MR1': hybrid1,
            'speedup_time': round(plain['time_to_1e-10_s'] / withnet['time_to_1e-10_s'], 3),
            'speedup_time_learned_then_MR2': round(plain['time_to_1e-10_s'] / hybrid['time_to_1e-10_s'], 3),
            'speedup_time_learned_then_MR1': round(plain['time_to_1e-10_s'] / hybrid1['time_to_1e-10_s'], 3),
            'mixed_vs_plain': {'plain': 'FP32 inner, FP64 outer, single right-hand side, MR(4) smoother',
                           'mixed': 'FP16 fine and coarse storage (FP32 scales, FP32 arithmetic), 16 right-hand '
                                    'sides per solve, matrix-core coarse stencils, learned level-0 smoother',
                           'plain_time_to_1e-10_s': plain['time_to_1e-10_s'],
                           'mixed_with_learned': combo, 'mixed_with_learned_then_MR2': combo_h,
                           'mixed_with_MR': combo_mr,
                           'mixed_red_black': 'the same with FP16 transfer bases and red-black preconditioning on '
                                              'every level',
                           'mixed_red_black_with_learned': rb_l, 'mixed_red_black_with_learned_then_MR2': rb_h,
                           'mixed_red_black_with_MR': rb_mr,
                           'mixed_red_black_with_MR_fp16_smoother_vectors': rb_mr16}}


def fine_and_transfer(steps=200):
    """Rows a8 and a9 on 16^3x32: the fine Wilson-clover apply (FP32 storage;
    16-bit links and clover with FP32 and with 16-bit spinors) and the
    level-0 prolongation / restriction (Nvec 24, block 4^4, FP32), each as
    achieved GB/s against 8 TB/s from algorithmic bytes per launch.  Operator
    copies are cycled so that one launch's data is not left in the 256 MB
    Infinity Cache by the previous launch."""
    import numpy as np
    import torch
    import synth
    from paper_1612_07873_amd import FineOp, Transfer, quantize_sites
    dev = torch.device('cuda')
    dims = (16, 16, 16, 32)
    V = int(np.prod(dims))
    U = torch.from_numpy(synth.gauge_field(dims, 0.3, 0)).to(dev)
    psi = [torch.from_numpy(synth.gaussian((V, 4, 3), 10 + k, 2)).to(dev).to(torch.complex64) for k in range(4)]
    out = {}
    # bytes per site: links (4 x 18 or 12 reals), clover (72 reals + 2 scales), spinor in and out
    site_bytes = {'c64': 768, 'h16_fp32_vectors': 144 + 152 + 192, 'h16_16bit_vectors': 144 + 152 + 2 * (48 + 4),
                  'c64_12real_links': 192 + 288 + 192, 'h16_12real_links_fp32_vectors': 96 + 152 + 192}
    for name, storage, reals in (('c64', 'c64', 18), ('h16_fp32_vectors', 'h16', 18), ('h16_16bit_vectors', 'h16', 18),
                                 ('c64_12real_links', 'c64', 12), ('h16_12real_links_fp32_vectors', 'h16', 12)):
        R = 4 if storage == 'c64' else 8
        ops = [FineOp(dims, U, -0.18, 1.0, True, storage, link_reals=reals) for _ in range(R)]
        if name == 'h16_16bit_vectors':
            qs = [quantize_sites(p.reshape(V, 12), 'h16') for p in psi]
            o16, osc = torch.empty_like(qs[0][0]), torch.empty_like(qs[0][1])
            fn = lambda i: ops[i % R].apply_scaled(qs[i % 4][0], qs[i % 4][1], o16, osc)
        else:
            y = torch.empty_like(psi[0])
            fn = lambda i: ops[i % R].apply(psi[i % 4], y)
        ms = timed(fn, steps, 20)
        gbs = site_bytes[name] * V / (ms * 1e-3) / 1e9
        out['wilson_clover_' + name] = {'lattice': list(dims), 'us_per_launch': round(ms * 1e3, 2),
                                        'algorithmic_bytes_per_site': site_bytes[name], 'GB/s': round(gbs, 1),
                                        'frac_of_hbm_peak': round(gbs / HBM_PEAK_GBS, 4), 'copies_cycled': R}
        del ops
    vecs = torch.from_numpy(synth.gaussian((24, V, 12), 0, 1)).to(dev)
    T = Transfer(dims, 12, (4, 4, 4, 4), vecs, 'c64')
    del vecs
    f = psi[0].reshape(V, 12)
    c = torch.empty((T.Vc, T.N), dtype=torch.complex64, device=dev)
    fo = torch.empty_like(f)
    basis = V * 12 * 24 * 8
    for name, fn, byts in (('restrict', lambda i: T.restrict(f, c), basis + V * 12 * 8 + T.Vc * T.N * 8),
                           ('prolong', lambda i: T.prolong(c, fo), basis + V * 12 * 8 + T.Vc * T.N * 8)):
        ms = timed(fn, steps, 20)
        gbs = byts / (ms * 1e-3) / 1e9
        out[name] = {'lattice': list(dims), 'nvec': 24, 'block': [4, 4, 4, 4], 'us_per_launch': round(ms * 1e3, 2),
                     'algorithmic_bytes_per_launch': byts, 'GB/s': round(gbs, 1),
                     'frac_of_hbm_peak': round(gbs / HBM_PEAK_GBS, 4),
                     'note': 'basis (302 MB) exceeds the Infinity Cache; the fine vector may stay cached'}
    return out


def plain_gcr(maxit=40000):
    """The same 16^3x32 system (right-hand side of the first MG solve) solved
    by plain restarted GCR(10) in FP64 on the fine operator alone (a one-level
    hierarchy: no preconditioner), to the same 1e-10 true residual."""
    import numpy as np
    import torch
    import synth
    from paper_1612_07873_amd import Multigrid
    dims = (16, 16, 16, 32)
    m0 = -0.25
    if os.path.exists(MG_M0_FILE):
        with open(MG_M0_FILE) as f:
            m0 = float(json.load(f)['m0'])
    U = torch.from_numpy(synth.gauge_field(dims, 0.3, 0)).to('cuda')
    mg = Multigrid(dims, U, m0, 1.0, [], [], inner='c64')
    b = torch.from_numpy(synth.gaussian((mg.V, 4, 3), 0, 2)).to('cuda')
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, info = mg.solve(b, tol=1e-10, maxit=maxit, check=False)
    torch.cuda.synchronize()
    return {'solver': 'GCR(10), FP64, no preconditioner', 'time_to_1e-10_s': round(time.perf_counter() - t, 3),
            'iterations': info['outer_iters'], 'converged': info['converged'],
            'true_rel_residual': info['true_rel_residual']}


def bicgstab(U, m0, nsolves=3, dims=(16, 16, 16, 32)):
    """The paper's comparison solver on the same system: BiCGStab with FP64
    reliable updates (delta 0.1) on the red-black (Schur) system, iterating
    with 16-bit links and clover (the paper's half precision), the same with
    12-real gauge compression, and with FP32 storage; the first solve
    discarded."""
    import numpy as np
    import torch
    import synth
    from paper_1612_07873_amd import BiCGStab, FineOp
    hi = FineOp(dims, U, m0, 1.0, True, 'c128')
    out = {}
    for name, lo_storage, reals in (('fp16_red_black', 'h16', 18), ('fp16_12real_red_black', 'h16', 12),
                                    ('fp32_red_black', 'c64', 18)):
        lo = FineOp(dims, U, m0, 1.0, True, lo_storage, link_reals=reals)
        solver = BiCGStab(hi, lo, evenodd=True)
        times, iters, upd, res = [], [], [], []
        for i in range(nsolves):
            b = torch.from_numpy(synth.gaussian((int(np.prod(dims)), 4, 3), i, 2)).to('cuda')
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, info = solver.solve(b, tol=1e-10, maxit=40000, delta=0.1)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t)
            iters.append(info['iters'])
            upd.append(info['reliable_updates'])
            res.append(info['true_rel_residual'])
        t = np.array(times[1:])
        out[name] = {'time_to_1e-10_s': round(float(t.mean()), 4), 'std_s': round(float(t.std()), 4),
                     'solves': nsolves, 'iters_mean': float(np.mean(iters[1:])),
                     'reliable_updates_mean': float(np.mean(upd[1:])), 'max_true_rel_residual': float(max(res))}
        del solver, lo
    return out


def mg_gcr(nsolves=12, nrhs=16):
    import torch
    import synth
    mg, U, m0, m0_src, setup = build_mg_16x32()
    out = {'lattice': [16, 16, 16, 32], 'm0': m0, 'm0_source': m0_src,
           'levels': '16^3x32 -(4^4,Nvec24)-> 4^3x8 N48 -(2^4,Nvec32)-> 2^3x4 N64', 'inner': 'fp32',
           'outer': 'fp64 GCR(10)', 'smoother': 'MR(4)', 'setup_s': round(setup, 2)}
    out.update(timed_solves(mg, nsolves, 0))
    # red-black preconditioning on every level (Sec. 7.1), same hierarchy
    t0 = time.perf_counter()
    mg.set_evenodd(True)
    torch_sync()
    rb = {'schur_setup_s': round(time.perf_counter() - t0, 3)}
    rb.update(timed_solves(mg, nsolves, 0))
    rb['speedup_vs_whole_lattice'] = round(out['time_to_1e-10_s'] / rb['time_to_1e-10_s'], 3)
    out['red_black'] = rb
    # where the time goes, level by level (device time from events around the
    # coarse-grid solves; one solve each, whole lattice and red-black)
    out['level_seconds'] = {}
    for name, eo in (('whole_lattice', False), ('red_black', True)):
        mg.set_evenodd(eo)
        mg.set_level_timing(True)
        mg.solve(torch.from_numpy(synth.gaussian((mg.V, 4, 3), 0, 2)).to('cuda'), tol=1e-10)
        _, info = mg.solve(torch.from_numpy(synth.gaussian((mg.V, 4, 3), 1, 2)).to('cuda'), tol=1e-10)
        mg.set_level_timing(False)
        out['level_seconds'][name] = {'total_s': round(info['seconds'], 5),
                                      'per_level_s': [round(t, 5) for t in info['level_seconds']],
                                      'level_iters': info['level_iters']}
    # the Schwarz (SAP) level-0 smoother: 4^4 blocks, 4 MR steps per block
    mg.set_evenodd(False)
    mg.set_sap((4, 4, 4, 4), 4)
    sap = timed_solves(mg, nsolves, 0)
    mg.set_evenodd(True)
    sap['with_red_black'] = timed_solves(mg, nsolves, 0)
    mg.set_sap(iters=0)
    mg.set_evenodd(False)
    out['sap_smoother'] = sap
    del mg
    out['bicgstab'] = bicgstab(U, m0)
    for k, v in out['bicgstab'].items():
        v['mg_red_black_speedup'] = round(v['time_to_1e-10_s'] / rb['time_to_1e-10_s'], 2)
    out['plain_gcr'] = plain_gcr()
    out['speedup_vs_plain_gcr'] = round(out['plain_gcr']['time_to_1e-10_s'] / out['time_to_1e-10_s'], 1)
    # mixed precision, several right-hand sides at once: FP16 coarse operators,
    # matrix-core coarse stencils, the same FP64 outer solver and tolerance
    mg16, _, _, _, setup16 = build_mg_16x32(coarse_storage='h16')
    out['multi_rhs_fp16_coarse'] = dict(setup_s=round(setup16, 2), **timed_batches(mg16, nrhs, 2, 5000))
    out['multi_rhs_fp16_coarse']['speedup_per_rhs_vs_single_fp32'] = round(
        out['time_to_1e-10_s'] / out['multi_rhs_fp16_coarse']['time_per_rhs_s'], 3)
    # the coarsest level solved exactly by its dense inverse (an option: the
    # paper's coarsest solve is GCR), single and batched
    mgd, _, _, _, setupd = build_mg_16x32(coarse_direct=True)
    d = {'setup_s': round(setupd, 2)}
    d.update(timed_solves(mgd, nsolves, 0))
    mgd.set_evenodd(True)
    d['red_black'] = timed_solves(mgd, nsolves, 0)
    del mgd
    mgd16, _, _, _, _ = build_mg_16x32(coarse_storage='h16', coarse_direct=True)
    d['multi_rhs_fp16_coarse'] = timed_batches(mgd16, nrhs, 2, 5000)
    del mgd16
    d['speedup_vs_plain_gcr'] = round(out['plain_gcr']['time_to_1e-10_s'] / d['time_to_1e-10_s'], 1)
    out['direct_coarsest'] = d
    # time per right-hand side against the batch size
    per = {}
    for m in (8, 32, 64):
        r = timed_batches(mg16, m, 1, 7000 + 100 * m)
        per[str(m)] = {'time_per_rhs_s': r['time_per_rhs_s'], 'outer_iters': r['outer_iters_mean'],
                       'max_true_rel_residual': r['max_true_rel_residual']}
    per[str(nrhs)] = {k: out['multi_rhs_fp16_coarse'][k] for k in ('time_per_rhs_s', 'max_true_rel_residual')}
    out['multi_rhs_fp16_coarse']['by_nrhs'] = per
    return out


def precision_form(nsolves=12, dims=(32, 32, 32, 64)):
    """The 16-bit precision form on 32^3x64 against the plain FP32 inner
    precision, same hierarchy recipe and start vectors: fine links and clover
    and every coarse operator in FP16 (per-(site, block) FP32 scales), FP32
    vectors and arithmetic, FP64 outer GCR.  The error of each level's stored
    operator is measured against the FP64 operators the library builds from
    the same block bases."""
    import numpy as np
    import torch
    import synth
    from paper_1612_07873_amd import FineOp, Multigrid, Transfer, build_coarse_op
    dev = torch.device('cuda')
    m0, m0_src = golden_m0(True)
    if m0_src != 'provisional':
        m0_src += ' (16^3x32 value, same gauge recipe)'
    V = int(np.prod(dims))
    t0 = time.perf_counter()
    U = torch.from_numpy(synth.gauge_field(dims, 0.3, 0)).to(dev)
    b1 = [d // 4 for d in dims]
    levels, starts = precision_form_levels(dims)
    print('precision form: inputs %.1f s' % (time.perf_counter() - t0), file=sys.stderr, flush=True)
    out = {'lattice': list(dims), 'm0': m0, 'm0_source': m0_src,
           'levels': '%s -(4^4,Nvec24)-> %s N48 -(2^4,Nvec32)-> %s N64'
                     % ('x'.join(map(str, dims)), 'x'.join(map(str, b1)), 'x'.join(str(d // 2) for d in b1))}
    runs = {}
    for name, fs, cs in (('fp32', None, None), ('fp16', 'h16', 'h16')):
        t0 = time.perf_counter()
        mg = Multigrid(dims, U, m0, 1.0, [dict(L, coarse_storage=cs) for L in levels], starts, inner='c64',
                       fine_storage=fs)
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        r = {'setup_s': round(setup, 2)}
        r.update(timed_solves(mg, nsolves, 0))
        print('precision form: %s %s' % (name, r), file=sys.stderr, flush=True)
        if name == 'fp16':   # with red-black preconditioning on every level as well (the paper's set-up)
            mg.set_evenodd(True)
            r['red_black'] = timed_solves(mg, nsolves, 0)
            print('precision form: fp16 red-black %s' % r['red_black'], file=sys.stderr, flush=True)
            # and the fine links compressed to 12 reals
            mg.set_fine_links(12)
            r['red_black_12real_links'] = timed_solves(mg, nsolves, 0)
            mg.set_fine_links(18)
            mg.set_evenodd(False)
            print('precision form: fp16 red-black 12-real %s' % r['red_black_12real_links'], file=sys.stderr,
                  flush=True)
            # and the transfer bases as FP16 pairs too: the same hierarchy resumed
            # from its FP64 bases (no relaxation), only the bases' storage differs
            t0 = time.perf_counter()
            bases = [mg.level(l)[3].basis() for l in range(len(levels))]
            mgt = Multigrid(dims, U, m0, 1.0, [dict(L, coarse_storage=cs, transfer_storage='h16') for L in levels],
                            None, inner='c64', fine_storage=fs, bases=bases)
            del bases
            mgt.set_evenodd(True)
            mgt.set_fine_links(12)
            torch.cuda.synchronize()
            r['red_black_12real_links_fp16_transfers'] = {'resume_s': round(time.perf_counter() - t0, 2)}
            r['red_black_12real_links_fp16_transfers'].update(timed_solves(mgt, nsolves, 0))
            print('precision form: fp16 red-black 12-real fp16 transfers %s'
                  % r['red_black_12real_links_fp16_transfers'], file=sys.stderr, flush=True)
            # and the level-0 MR smoother on 16-bit vectors (the paper's half-precision smoother)
            mgt.set_smoother_vectors('h16')
            r['red_black_12real_links_fp16_transfers_fp16_smoother'] = timed_solves(mgt, nsolves, 0)
            print('precision form: ... and fp16 smoother vectors %s'
                  % r['red_black_12real_links_fp16_transfers_fp16_smoother'], file=sys.stderr, flush=True)
            del mgt
        runs[name] = (mg, r)
    # FP64 operators from the same block bases, and each stored operator's error against them
    mg16 = runs['fp16'][0]
    mg32 = runs['fp32'][0]
    f64 = FineOp(dims, U, m0, 1.0, True, 'c128')
    f16 = FineOp(dims, U, m0, 1.0, True, 'h16')
    psi = torch.from_numpy(synth.gaussian((V, 4, 3), 77, 2)).to(dev)
    ref = f64.apply(psi)
    errs = {'fp16': [float((f16.apply(psi.to(torch.complex64)).to(torch.complex128) - ref).norm() / ref.norm())],
            'fp32': [float((FineOp(dims, U, m0, 1.0, True, 'c64').apply(psi.to(torch.complex64))
                            .to(torch.complex128) - ref).norm() / ref.norm())]}
    parent, fine = None, f64
    for l in (1, 2):
        pdims, pdof, _, T = mg16.level(l - 1)
        B = T.basis().permute(2, 0, 1).contiguous()
        t64 = Transfer(pdims, pdof, levels[l - 1]['block'], B, 'c128')
        op64 = build_coarse_op(t64, fine=fine, parent=parent, storage='c128')
        del B
        cdims, N, op16, _ = mg16.level(l)
        _, _, op32, _ = mg32.level(l)
        u = torch.from_numpy(synth.gaussian((op64.V, N), 80 + l, 2)).to(dev)
        y64 = op64.apply(u)
        for name, op in (('fp16', op16), ('fp32', op32)):
            y = op.apply(u.to(torch.complex64)).to(torch.complex128)
            errs[name].append(float((y - y64).norm() / y64.norm()))
        parent, fine = op64, None
    torch.cuda.synchronize()
    out['error_vs_fp64_per_level'] = {k: [float('%.3e' % e) for e in v] for k, v in errs.items()}
    out['fp32'] = runs['fp32'][1]
    out['fp16'] = runs['fp16'][1]
    out['speedup_time'] = round(runs['fp32'][1]['time_to_1e-10_s'] / runs['fp16'][1]['time_to_1e-10_s'], 3)
    out['speedup_time_red_black'] = round(runs['fp32'][1]['time_to_1e-10_s'] /
                                          runs['fp16'][1]['red_black']['time_to_1e-10_s'], 3)
    out['speedup_time_all_16bit'] = round(runs['fp32'][1]['time_to_1e-10_s'] /
                                          runs['fp16'][1]['red_black_12real_links_fp16_transfers_fp16_smoother']
                                          ['time_to_1e-10_s'], 3)
    return out


def pf_solves(nsolves, dims=(32, 32, 32, 64)):
    """The 32^3x64 precision form at its fastest (FP16 fine links with 12 reals and
    clover, FP16 coarse operators and transfer bases, 16-bit level-0 smoother
    vectors, red-black on every level),
    built as precision_form() builds it; one read-stream launch marks the end of
    the setup for a kernel trace, then `nsolves` solves."""
    import torch
    import synth
    from paper_1612_07873_amd import Multigrid, stream_read
    m0, _ = golden_m0(True)
    U = torch.from_numpy(synth.gauge_field(dims, 0.3, 0)).to('cuda')
    levels, starts = precision_form_levels(dims)
    mg = Multigrid(dims, U, m0, 1.0, [dict(L, coarse_storage='h16', transfer_storage='h16') for L in levels], starts,
                   inner='c64', fine_storage='h16')
    mg.set_evenodd(True)
    mg.set_fine_links(12)
    mg.set_smoother_vectors('h16')
    buf = torch.ones(1 << 20, dtype=torch.float32, device='cuda')
    sink = torch.empty(1 << 14, dtype=torch.int32, device='cuda')
    stream_read(buf, sink)
    torch.cuda.synchronize()
    return timed_solves(mg, nsolves, 0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=2000)
    ap.add_argument('--warmup', type=int, default=200)
    ap.add_argument('--no-cpu', action='store_true', help='skip the CPU oracle leg')
    ap.add_argument('--only-headline', action='store_true', help='time the headline kernel only')
    ap.add_argument('--learned', action='store_true', help='learned-smoother comparison on 16^3x32 instead')
    ap.add_argument('--only-fine', action='store_true',
                    help='only the Wilson-clover and transfer records (rows a8, a9) instead')
    ap.add_argument('--mg-solves', type=int, default=0,
                    help='only time this many MG-GCR solves on 16^3x32 (after the setup) instead')
    ap.add_argument('--coarse-direct', action='store_true', help='with --mg-solves: exact coarsest solve')
    ap.add_argument('--red-black', action='store_true', help='with --mg-solves: red-black form on every level')
    ap.add_argument('--only-small', action='store_true',
                    help='only the smallest-grid records (rows a1, a3-a5) instead')
    ap.add_argument('--only-16bit', action='store_true',
                    help='only the 16-bit single-RHS and multi-RHS matrix-core records (rows a6, a7) instead')
    ap.add_argument('--precision-form', action='store_true',
                    help='16-bit precision form vs FP32 inner precision on 32^3x64 instead')
    ap.add_argument('--pf-solves', type=int, default=0,
                    help='only N solves of the 32^3x64 precision form with every storage 16-bit and red-black '
                         '(a profiling driver: the end of the setup is marked by one read-stream launch)')
    ap.add_argument('--quick', action='store_true',
                    help='leave out the learned-smoother and 32^3x64 precision-form records')
    ap.add_argument('--pairs', type=int, default=4096)
    ap.add_argument('--epochs', type=int, default=2)
    ap.add_argument('--loss', choices=['error', 'residual'], default='residual')
    ap.add_argument('--pairs-from', choices=['smoother', 'iterates'], default='smoother')
    args = ap.parse_args()
    if args.gpus != 1:
        print('bench.py measures one GPU only: the multigrid hot path is built and timed on a single MI355X; '
              '--gpus %d is not supported' % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    from paper_1612_07873_amd import CoarseOp

    if args.learned:
        if args.pairs_from == 'smoother' and args.loss != 'residual':
            print('smoother inputs have no error partner: use --loss residual', file=sys.stderr)
            sys.exit(2)
        print(json.dumps({'learned_smoother': learned(args.pairs, args.epochs, args.loss, args.pairs_from)}),
              flush=True)
        return
    if args.only_fine:
        print(json.dumps({'fine_and_transfer': fine_and_transfer()}), flush=True)
        return
    if args.only_small:
        print(json.dumps({'small_grids': small_grids()}), flush=True)
        return
    if args.only_16bit:
        rec16 = precision_and_mrhs(args.steps)
        rec16['multi_level'] = multi_level()
        print(json.dumps(rec16), flush=True)
        return
    if args.mg_solves:
        mg, _, m0, _, setup = build_mg_16x32(coarse_direct=args.coarse_direct)
        r = {'lattice': [16, 16, 16, 32], 'm0': m0, 'coarse_direct': args.coarse_direct,
             'red_black': args.red_black, 'setup_s': round(setup, 2)}
        if args.red_black:
            mg.set_evenodd(True)
        r.update(timed_solves(mg, args.mg_solves, 0))
        mg.set_level_timing(True)
        _, info = mg.solve(torch.from_numpy(synth.gaussian((mg.V, 4, 3), 1, 2)).to('cuda'), tol=1e-10)
        mg.set_level_timing(False)
        r['level_seconds'] = {'total_s': round(info['seconds'], 5),
                              'per_level_s': [round(t, 5) for t in info['level_seconds']]}
        print(json.dumps({'mg_solves': r}), flush=True)
        return
    if args.precision_form:
        print(json.dumps({'precision_form': precision_form()}), flush=True)
        return
    if args.pf_solves > 0:
        print(json.dumps({'precision_form_all_16bit_red_black': pf_solves(args.pf_solves)}), flush=True)
        return
    dev = torch.device('cuda')
    # a plain device copy of known size (512 MiB read, 512 MiB written), outside
    # any timed region: under a counter run it calibrates FETCH_SIZE / WRITE_SIZE
    calib = torch.ones(1 << 26, dtype=torch.complex64, device=dev)
    dst = torch.empty_like(calib)
    dst.copy_(calib)
    copy_ms = timed(lambda i: dst.copy_(calib), 10, 2)      # achievable copy bandwidth on this machine
    copy_gbs = 2 * calib.numel() * 8 / (copy_ms * 1e-3) / 1e9
    del calib, dst
    # achievable read bandwidth: the library's read-stream kernel over 1 GiB
    from paper_1612_07873_amd import stream_read
    rbuf = torch.ones(1 << 27, dtype=torch.complex64, device=dev)
    sink = torch.empty(1 << 14, dtype=torch.int32, device=dev)
    stream_read(rbuf, sink)
    read_ms = timed(lambda i: stream_read(rbuf, sink), 10, 2)
    read_gbs = rbuf.numel() * 8 / (read_ms * 1e-3) / 1e9
    del rbuf, sink
    cd, N = (4, 4, 4, 8), 48
    V = int(np.prod(cd))
    X = synth.gaussian((V, N, N), 0, 2)
    Y = synth.gaussian((8, V, N, N), 1, 2)
    u = synth.gaussian((V, N), 2, 2)
    Xd, Yd = torch.from_numpy(X).to(dev), torch.from_numpy(Y).to(dev)
    flops, byts = algorithmic(V, N, 1, 8)
    ops = cold_ops(cd, N, 'c64', Xd, Yd, byts)
    R = len(ops)
    ud = torch.from_numpy(u).to(dev).to(torch.complex64)
    out = torch.empty_like(ud)
    tuned_ms = ops[0].tune(ud, out, cold=True)       # autotuner, cold caches; the copies reuse its choice
    for op in ops[1:]:
        op.tune(ud, out, cold=True)
    ms_step = timed(lambda i: ops[i % R].apply(ud, out), args.steps, args.warmup)
    y = out.cpu().numpy().astype(np.complex128)
    achieved = byts / (ms_step * 1e-3) / 1e9
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
                   'lattice': list(cd), 'N': N, 'nrhs': 1,
                   'launch': {'rows': ops[0].launch()[0], 'split': ops[0].launch()[1], 'prefetch': ops[0].prefetch(),
                              'tuned_cold_ms': round(tuned_ms, 5)}},
        'roofline': {'bound': 'hbm', 'achieved': round(achieved, 1), 'peak': HBM_PEAK_GBS, 'unit': 'GB/s',
                     'frac': round(achieved / HBM_PEAK_GBS, 4),
                     'traffic': measured_traffic([ops[0].launch()[0], ops[0].launch()[1], ops[0].prefetch()]),
                     'algorithmic_bytes_per_launch': byts, 'kernel': 'qmg::k_coarse_dslash (FP32 links)',
                     'achievable_copy_GB/s': round(copy_gbs, 1),
                     'frac_of_achievable_copy': round(achieved / copy_gbs, 4),
                     'achievable_read_GB/s': round(read_gbs, 1),
                     'frac_of_achievable_read': round(achieved / read_gbs, 4)},
    }
    warm_ms = timed(lambda i: ops[0].apply(ud, out), 500, 50)
    rec['warm_cache'] = {'ms_per_step': round(warm_ms, 6), 'GFLOP/s': round(flops / (warm_ms * 1e-3) / 1e9, 2),
                         'effective_GB/s': round(byts / (warm_ms * 1e-3) / 1e9, 1)}
    del ops, Xd, Yd
    if not args.only_headline:
        def step(name, fn):
            t0 = time.perf_counter()
            r = fn()
            print('bench: %s done in %.1f s' % (name, time.perf_counter() - t0), file=sys.stderr, flush=True)
            return r
        rec.update(step('precision and multi_rhs', lambda: precision_and_mrhs(max(100, args.steps // 4))))
        rec['small_grids'] = step('small_grids', small_grids)
        rec['multi_level'] = step('multi_level', multi_level)
        rec['fine_and_transfer'] = step('fine_and_transfer', fine_and_transfer)
        rec['mg_gcr'] = step('mg_gcr', mg_gcr)
        if not args.quick:
            rec['learned_smoother'] = step('learned_smoother',
                                           lambda: learned(args.pairs, args.epochs, args.loss, args.pairs_from))
            rec['precision_form'] = step('precision_form', lambda: precision_form(nsolves=12))
    if not args.no_cpu:
        ref, rec['cpu_baseline'] = cpu_baseline(cd, N, X, Y, u)
        rec['parity_rel_err'] = float(np.abs(y - ref).max() / np.abs(ref).max())
    print(json.dumps(rec), flush=True)


if __name__ == '__main__':
    main()
