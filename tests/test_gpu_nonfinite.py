"""Failure detection on the 16-bit paths: a NaN or Inf input to an encoder,
or a block whose largest entry does not fit FP32, is reported as
QMG_ERR_NONFINITE (by the next qmg_sync, or by the blocking call that encoded
it) instead of being stored silently; the report clears the record; an
all-zero site keeps scale 0 and zero codes; and the solver reports a
non-finite right-hand side."""
import numpy as np
import pytest
import torch

import synth
from oracle import lattice
from gpu_util import dev

pytestmark = pytest.mark.gpu

NONFINITE = 7


def _expect_nonfinite(fn):
    from paper_1612_07873_amd import QmgError
    with pytest.raises(QmgError) as e:
        fn()
    assert e.value.status == NONFINITE, str(e.value)


@pytest.mark.parametrize('prec', ['h16', 'b16'])
def test_quantize_reports_nan_and_inf(prec):
    from paper_1612_07873_amd import dequantize_sites, quantize_sites, sync
    v = dev(synth.gaussian((64, 48), 1, 2), torch.complex64)
    v[9] = 0                                           # an all-zero site: scale 0, zero codes
    q, sc = quantize_sites(v, prec)
    sync()                                             # nothing to report
    assert float(sc[9]) == 0.0 and int(q[9].abs().max()) == 0
    assert torch.equal(dequantize_sites(q, sc, prec)[9], v[9])
    for bad in (float('nan'), float('inf'), -float('inf')):
        w = v.clone()
        w[5, 7] = complex(1.0, bad)
        quantize_sites(w, prec)
        _expect_nonfinite(sync)
        sync()                                         # the report cleared the record


def test_coarse_op_16bit_reports_nonfinite_and_out_of_range_blocks():
    from paper_1612_07873_amd import CoarseOp, sync
    dims, N = (2, 2, 2, 2), 8
    V = lattice.volume(dims)
    X = synth.gaussian((V, N, N), 0, 2)
    Y = synth.gaussian((8, V, N, N), 1, 2)
    op = CoarseOp(dims, dev(X), dev(Y), 'h16')
    sync()
    for where, val in (('X', np.nan), ('Y', np.inf), ('Y', 1e300)):   # 1e300: its scale overflows FP32
        X2, Y2 = X.copy(), Y.copy()
        (X2 if where == 'X' else Y2).flat[17] = val
        op2 = CoarseOp(dims, dev(X2), dev(Y2), 'h16')
        _expect_nonfinite(sync)
        del op2
    sync()
    # complex64 storage keeps the values as they are: nothing to report
    X2 = X.copy()
    X2.flat[3] = 1e300
    CoarseOp(dims, dev(X2), dev(Y), 'c128')
    sync()


def test_fine_op_16bit_and_fp16_basis_report_nonfinite_at_creation():
    from paper_1612_07873_amd import FineOp, Transfer, sync
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.4, 3)
    FineOp(dims, dev(U), -0.2, 1.0, True, 'h16')
    sync()
    Ub = U.copy()
    Ub.reshape(-1)[100] = np.nan
    _expect_nonfinite(lambda: FineOp(dims, dev(Ub), -0.2, 1.0, True, 'h16'))
    sync()
    V = lattice.volume(dims)
    vecs = synth.gaussian((4, V, 12), 5, 1)
    Transfer(dims, 12, (2, 2, 2, 2), dev(vecs), 'h16')
    vb = vecs.copy()
    vb[1, 7, 3] = np.inf
    from paper_1612_07873_amd import QmgError
    with pytest.raises(QmgError):        # the orthonormalisation or the FP16 rounding refuses it
        Transfer(dims, 12, (2, 2, 2, 2), dev(vb), 'h16')
    sync()


def test_solve_reports_nonfinite_right_hand_side():
    from paper_1612_07873_amd import Multigrid, QmgError, sync
    dims, m0 = (4, 4, 4, 8), -0.3
    U = synth.gauge_field(dims, 0.4, 1)
    st = [dev(synth.gaussian((6, lattice.volume(dims), 12), 0, 1))]
    lv = [dict(block=(2, 2, 2, 2), nvec=6, setup_iters=0, smoother_steps=4, coarse_tol=0.25, coarse_maxit=100,
               coarse_storage='h16')]
    mg = Multigrid(dims, dev(U), m0, 1.0, lv, st, inner='c64', fine_storage='h16')
    b = synth.gaussian((lattice.volume(dims), 4, 3), 2, 2)
    mg.solve(dev(b), tol=1e-10)
    b[3, 1, 2] = np.nan
    x, info = mg.solve(dev(b), tol=1e-10, check=False)
    assert info['status'] == NONFINITE and not info['converged']
    # a batch through the matrix-core path (16-bit coarse operators, 8 members)
    B = np.stack([synth.gaussian((lattice.volume(dims), 4, 3), 10 + k, 2) for k in range(8)])
    B[5, 0, 0, 0] = np.inf
    X, infos = mg.solve_multi(dev(B), tol=1e-10, check=False)
    assert infos[0]['status'] == NONFINITE
    sync()                               # the solve consumed the encoders' record
    X, infos = mg.solve_multi(dev(np.nan_to_num(B, posinf=0.0)), tol=1e-10)
    assert all(i['converged'] for i in infos)
