"""Pins of the oracle's parallel-transport convolution smoother: exact
reduction to the Wilson operator, gauge equivariance, adjointness of the
transports, and central finite differences of the loss gradients."""
import numpy as np

import synth
from oracle import lattice, ptc, wilson
from oracle_helpers import gauge_rotate


def setup(dims=(4, 2, 2, 4), seed=0):
    U = synth.gauge_field(dims, 0.5, seed)
    return U, lattice.volume(dims)


def test_one_layer_with_wilson_weights_is_the_wilson_operator():
    """W_0 = (4+m0) 1, W_{+mu} = -1/2 (1-gamma_mu), W_{-mu} = -1/2 (1+gamma_mu)
    gives M at c_sw = 0 exactly."""
    dims = (4, 4, 2, 4)
    U, V = setup(dims, 1)
    m0 = -0.3
    Pm, Pp = lattice.projectors()
    W = np.zeros((9, 1, 1, 4, 4), dtype=np.complex128)
    W[0, 0, 0] = (4 + m0) * np.eye(4)
    for mu in range(4):
        W[1 + 2 * mu, 0, 0] = -0.5 * Pm[mu]
        W[2 + 2 * mu, 0, 0] = -0.5 * Pp[mu]
    r = synth.gaussian((V, 4, 3), 2, 2)
    y = ptc.layer(W, r[None], U, dims)[0]
    assert np.abs(y - wilson.apply_wilson_clover(r, U, None, m0, dims)).max() < 1e-13
    # W_0 = alpha 1 alone scales
    W2 = np.zeros_like(W)
    W2[0, 0, 0] = (0.7 - 0.2j) * np.eye(4)
    assert np.abs(ptc.layer(W2, r[None], U, dims)[0] - (0.7 - 0.2j) * r).max() < 1e-15


def test_transport_adjoint_and_gauge_equivariance():
    dims = (4, 2, 4, 2)
    U, V = setup(dims, 2)
    a = synth.gaussian((V, 4, 3), 3, 2)
    b = synth.gaussian((V, 4, 3), 4, 2)
    for p in range(9):
        lhs = np.vdot(a, ptc.transport(b, U, dims, p))
        rhs = np.vdot(ptc.transport(a, U, dims, ptc.reverse(p)), b)
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # network equivariance: N[gU](g r) = g N[U](r)
    Ws = [synth.gaussian((9, 3, 1, 4, 4), 5, 4), synth.gaussian((9, 1, 3, 4, 4), 6, 4)]
    g = synth.gauge_rotation(dims, 7)
    Ug = gauge_rotate(U, g, dims)
    rot = lambda h: np.einsum('xab,xsb->xsa', g, h)
    y1, _ = ptc.forward(Ws, rot(a), Ug, dims)
    y0, _ = ptc.forward(Ws, a, U, dims)
    assert np.abs(y1 - rot(y0)).max() < 1e-12 * np.abs(y0).max()


def test_gradients_match_central_finite_differences():
    dims = (2, 2, 2, 4)
    U, V = setup(dims, 3)
    Ws = [0.3 * synth.gaussian((9, 2, 1, 4, 4), 8, 4), 0.3 * synth.gaussian((9, 1, 2, 4, 4), 9, 4)]
    pairs = [(synth.gaussian((V, 4, 3), 10 + i, 2), synth.gaussian((V, 4, 3), 20 + i, 2)) for i in range(2)]
    L, Gs = ptc.loss_and_grads(Ws, pairs, U, dims)
    rng = np.random.default_rng(0)
    h = 1e-6
    for l in range(2):
        for _ in range(12):
            idx = tuple(int(rng.integers(0, s)) for s in Ws[l].shape)
            num = 0j
            for unit in (1.0, 1j):
                Wp = [w.copy() for w in Ws]
                Wm = [w.copy() for w in Ws]
                Wp[l][idx] += h * unit
                Wm[l][idx] -= h * unit
                Lp, _ = ptc.loss_and_grads(Wp, pairs, U, dims)
                Lm, _ = ptc.loss_and_grads(Wm, pairs, U, dims)
                num += unit * (Lp - Lm) / (2 * h)
            assert abs(num - Gs[l][idx]) <= 1e-6 * max(1.0, abs(Gs[l][idx])), (l, idx, num, Gs[l][idx])


def test_adam_decreases_the_loss():
    dims = (2, 2, 2, 4)
    U, V = setup(dims, 4)
    from oracle import wilson as w
    # pairs from the Wilson operator: e Gaussian, r = M e
    pairs = []
    for i in range(4):
        e = synth.gaussian((V, 4, 3), 30 + i, 4)
        pairs.append((w.apply_wilson_clover(e, U, None, 0.2, dims), e))
    Ws = [0.1 * synth.gaussian((9, 2, 1, 4, 4), 1, 4), 0.1 * synth.gaussian((9, 1, 2, 4, 4), 2, 4)]
    opt = ptc.Adam([W.shape for W in Ws], lr=1e-2)
    L0, _ = ptc.loss_and_grads(Ws, pairs, U, dims)
    for _ in range(30):
        L, G = ptc.loss_and_grads(Ws, pairs, U, dims)
        Ws = opt.step(Ws, G)
    L1, _ = ptc.loss_and_grads(Ws, pairs, U, dims)
    assert L1 < 0.5 * L0


def test_residual_loss_gradients_match_finite_differences():
    dims = (2, 2, 2, 4)
    U, V = setup(dims, 6)
    A = wilson.clover_field(U, dims, 1.0)
    M = lambda v: wilson.apply_wilson_clover(v, U, A, -0.1, dims)
    Ws = [0.3 * synth.gaussian((9, 2, 1, 4, 4), 11, 4), 0.3 * synth.gaussian((9, 1, 2, 4, 4), 12, 4)]
    rs = [synth.gaussian((V, 4, 3), 40 + i, 2) for i in range(2)]
    L, Gs = ptc.loss_and_grads_residual(Ws, rs, U, dims, M)
    rng = np.random.default_rng(1)
    h = 1e-6
    for l in range(2):
        for _ in range(10):
            idx = tuple(int(rng.integers(0, s)) for s in Ws[l].shape)
            num = 0j
            for unit in (1.0, 1j):
                Wp = [w.copy() for w in Ws]
                Wm = [w.copy() for w in Ws]
                Wp[l][idx] += h * unit
                Wm[l][idx] -= h * unit
                num += unit * (ptc.loss_and_grads_residual(Wp, rs, U, dims, M)[0]
                               - ptc.loss_and_grads_residual(Wm, rs, U, dims, M)[0]) / (2 * h)
            assert abs(num - Gs[l][idx]) <= 1e-6 * max(1.0, abs(Gs[l][idx])), (l, idx, num, Gs[l][idx])


# ---- Adam against its published closed form (Kingma & Ba, Algorithm 1) ----
#
# From zero moments, the bias-corrected first step is m_hat = g and
# v_hat = g^2 exactly, so each real component moves by lr*g/(|g| + eps),
# independently of beta1 and beta2.  A dropped bias correction (a step of
# lr*(1-b1)/sqrt(1-b2) ~ 3.16*lr), a missing square root (lr*g/(g^2+eps)) or a
# sign error fails it, since |g| != 1 below.

def _adam_one(W0, gs, lr=0.1, b1=0.9, b2=0.999, eps=1e-8):
    opt = ptc.Adam([W0.shape], lr=lr, beta1=b1, beta2=b2, eps=eps)
    Ws = [W0.copy()]
    out = []
    for g in gs:
        Ws = opt.step(Ws, [g])
        out.append(Ws[0].copy())
    return out


def test_adam_first_step_is_lr_times_sign_of_gradient():
    W0 = np.array([[0.3 - 0.7j, -1.1 + 0.2j]])
    g = np.array([[0.5 - 2.0j, -3.0 + 0.25j]])
    (W1,) = _adam_one(W0, [g])
    eps = 1e-8
    expect = W0 - 0.1 * (g.real / (np.abs(g.real) + eps) + 1j * g.imag / (np.abs(g.imag) + eps))
    assert np.abs(W1 - expect).max() <= 1e-15
    # the first step does not depend on the betas
    (W1b,) = _adam_one(W0, [g], b1=0.5, b2=0.9)
    assert np.abs(W1b - expect).max() <= 1e-15


def test_adam_second_step_hand_computed():
    """Two steps with lr = 0.1, beta1 = 0.9, beta2 = 0.999, eps = 1e-8.
    Real part: g1 = 1/2, g2 = -3/2:
      m2 = 0.9*0.1*(1/2) + 0.1*(-3/2) = -21/200,  m_hat = m2/(1 - 0.81) = -21/38,
      v2 = 0.999*0.001*(1/4) + 0.001*(9/4) = 9999/4000000,
      v_hat = v2/(1 - 0.998001) = 9999/7996,
      step = 0.1*m_hat/(sqrt(v_hat) + eps) = -0.04941898288778031.
    Imaginary part: g1 = -2, g2 = 1/4:
      m2 = -31/200, m_hat = -31/38, v2 = 8117/2000000, v_hat = 8117/3998,
      step = -0.05725345717104488.
    Swapping beta1 and beta2 gives a different second step, so it fails."""
    W0 = np.array([0.25 + 0.5j])
    g1 = np.array([0.5 - 2.0j])
    g2 = np.array([-1.5 + 0.25j])
    W1, W2 = _adam_one(W0, [g1, g2])
    step2 = -0.04941898288778031 - 0.05725345717104488j
    assert abs((W1 - W2)[0] - step2) <= 1e-15
    _, W2s = _adam_one(W0, [g1, g2], b1=0.999, b2=0.9)
    assert abs((W1 - W2s)[0] - step2) > 1e-3


def test_adam_constant_gradient_moves_by_lr_every_step():
    """With the same gradient g at every step the bias corrections make
    m_hat = g and v_hat = g^2 exactly at every t, so every step moves each
    component by lr*g/(|g| + eps); a bias correction with the wrong power of
    beta (t - 1 or t + 1) breaks it from the second step on."""
    W0 = np.array([1.0 - 1.0j, 0.0 + 0.0j, -2.0 + 3.0j])
    g = np.array([0.3 + 4.0j, -0.02 - 0.7j, 5.0 - 0.001j])
    Ws = _adam_one(W0, [g] * 6, lr=0.01)
    eps = 1e-8
    d = 0.01 * (g.real / (np.abs(g.real) + eps) + 1j * g.imag / (np.abs(g.imag) + eps))
    prev = W0
    for W in Ws:
        assert np.abs((prev - W) - d).max() <= 1e-13
        prev = W
