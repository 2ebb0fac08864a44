"""Training of the learned level-0 smoother on pairs the solver produces.

Pairs: for each right-hand side b the multigrid solve records its outer
iterates x_k; with the converged x*, e_k = x* - x_k and r_k = M e_k (both made
by the library, qmg_mg_make_pairs).  Alternatively the solve records the
residuals the level-0 smoother itself is applied to (the K-cycle's input and
the residual left after the coarse-grid correction), which carry the high
modes a smoother has to remove; these train the residual form of the loss.  Pairs whose error has fallen below
`min_rel_err` of |x*| are dropped (they carry little beyond rounding).
Training: Adam on the loss sum_i |N(r_i) - e_i|^2/|e_i|^2 (or its residual
form sum_i |r_i - M N(r_i)|^2/|r_i|^2, which asks the network for exactly what
the solver's fallback test checks) over mini-batches,
every forward, backward and update in the library's kernels; random numbers
(initial weights, batch order) come from the caller.
"""
import numpy as np
import torch

from . import PTC, Multigrid  # noqa: F401


def generate_pairs(mg, rhs, maxrec=32, min_rel_err=1e-6, tol=1e-10):
    """rhs: iterable of complex128 device fields [V][4][3]; returns (R, E) complex64
    [n][V][4][3] and the per-solve info records."""
    Rs, Es, infos = [], [], []
    for b in rhs:
        x, hist, info = mg.solve_record(b, maxrec, tol=tol)
        r, e = mg.make_pairs(x, hist)
        xn = float(torch.linalg.vector_norm(x))
        keep = [k for k in range(e.shape[0]) if float(torch.linalg.vector_norm(e[k])) > min_rel_err * xn]
        Rs.append(r[keep])
        Es.append(e[keep])
        infos.append(info)
        del hist
    return torch.cat(Rs), torch.cat(Es), infos


def generate_smoother_inputs(mg, rhs, maxrec=64, tol=1e-10):
    """The residuals the level-0 smoother is applied to during solves of `rhs`
    (K-cycle inputs and residuals after the coarse-grid correction), complex64
    [n][V][4][3], for the residual form of the loss (no error partner)."""
    Rs, infos = [], []
    for b in rhs:
        _, hist, info = mg.solve_record_smoother(b, maxrec, tol=tol)
        Rs.append(hist.clone())
        infos.append(info)
        del hist
    return torch.cat(Rs), infos


def initial_weights(hidden, m0, gen):
    """Start near a damped Jacobi step: channel 0 carries r, the output takes
    1/(4 + m0) of it; every other weight is small Gaussian noise from `gen`."""
    def noise(shape, scale):
        return scale * (gen.standard_normal(shape) + 1j * gen.standard_normal(shape)) / np.sqrt(2)
    W1 = noise((9, hidden, 1, 4, 4), 1e-3)
    W2 = noise((9, 1, hidden, 4, 4), 1e-3)
    W1[0, 0, 0] += np.eye(4)
    W2[0, 0, 0] += np.eye(4) / (4.0 + m0)
    return W1.astype(np.complex64), W2.astype(np.complex64)


def train(net, R, E, epochs, batch, lr, gen, log_every=1, loss='error'):
    """Adam over shuffled mini-batches; returns the mean loss per epoch.
    loss='error': |N(r) - e|^2/|e|^2; loss='residual': |r - M N(r)|^2/|r|^2."""
    n = R.shape[0]
    hist = []
    for ep in range(epochs):
        order = gen.permutation(n)
        tot = 0.0
        for s in range(0, n, batch):
            net.zero_grad()
            idx = order[s:s + batch]
            for i in idx:
                if loss == 'residual':
                    net.accumulate_residual(R[int(i)])
                else:
                    net.accumulate(R[int(i)], E[int(i)])
            if ep % log_every == 0 or ep == epochs - 1:
                tot += net.grad()[2]
            net.adam_step(lr=lr)
        hist.append(tot / n)
    return hist


def mean_loss(net, R, E, loss='error'):
    net.zero_grad()
    for i in range(R.shape[0]):
        if loss == 'residual':
            net.accumulate_residual(R[i])
        else:
            net.accumulate(R[i], E[i])
    return net.grad()[2] / R.shape[0]
