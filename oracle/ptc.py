"""Gauge-equivariant parallel-transport convolution (PTC) network used as a
fine-level smoother (oracle, FP64; test infrastructure).

Nothing in the paper defines this network (its smoother is MR, Sec. 7.1); it is
the learned component of the workload, specified here as:

  transports  T_0 h = h,
              (T_{+mu} h)(x) = eta+ U_mu(x)        h(x + mu),
              (T_{-mu} h)(x) = eta- U_mu(x - mu)^+ h(x - mu),
              with the operator's boundary sign eta; T_{+mu}^+ = T_{-mu};
  layer       h'_a(x) = sum_b sum_p W[p, a, b] (T_p h_b)(x),
              W[p, a, b] a complex 4x4 matrix on spin (commutes with T);
              paths p = 0, +x, -x, +y, -y, +z, -z, +t, -t  (index 0, 1+2mu, 2+2mu);
  network     two layers 1 -> C -> 1 channels, no activation (a fixed linear map);
  loss        L = sum_i |N(r_i) - e_i|^2 / |e_i|^2 over (residual, error) pairs.

Gradients treat Re W and Im W as independent reals and are returned as
G = dL/dRe W + i dL/dIm W.  With D = dL/dy* the backward pass is
  G[p, a, b] = 2 sum_{x, colour} D_a(x) (T_p h_b)(x)^+,
  dL/dh_b*   = sum_p T_p^+ ( sum_a W[p, a, b]^+ D_a ).
Adam updates the real and imaginary parts elementwise.
Fields: h [C][V][4][3] complex.
"""
import numpy as np

from . import lattice

NPATH = 9


def path_dir(p):
    """(mu, step) of path p >= 1."""
    return (p - 1) // 2, (1 if (p - 1) % 2 == 0 else -1)


def transport(h, U, dims, p, antiperiodic_t=True):
    """T_p h for one field h [V][4][3]."""
    if p == 0:
        return h.copy()
    mu, step = path_dir(p)
    n = lattice.neighbour(dims, mu, step)
    eta = lattice.boundary_sign(dims, mu, step, antiperiodic_t)
    if step > 0:
        t = np.einsum('xab,xsb->xsa', U[mu], h[n])
    else:
        t = np.einsum('xba,xsb->xsa', np.conj(U[mu][n]), h[n])
    return eta[:, None, None] * t


def reverse(p):
    return 0 if p == 0 else (p + 1 if (p - 1) % 2 == 0 else p - 1)


def layer(W, h, U, dims, antiperiodic_t=True):
    """W [9][Cout][Cin][4][4], h [Cin][V][4][3] -> [Cout][V][4][3]."""
    cout, cin = W.shape[1], W.shape[2]
    V = h.shape[1]
    out = np.zeros((cout, V, 4, 3), dtype=np.complex128)
    for b in range(cin):
        for p in range(NPATH):
            t = transport(h[b], U, dims, p, antiperiodic_t)
            out += np.einsum('ast,xtc->axsc', W[p, :, b], t)
    return out


def forward(Ws, r, U, dims, antiperiodic_t=True):
    """Network output for one residual r [V][4][3]; Ws = [W1, W2].  Returns
    the output and the list of layer inputs (for the backward pass)."""
    h = r[None]
    inputs = []
    for W in Ws:
        inputs.append(h)
        h = layer(W, h, U, dims, antiperiodic_t)
    return h[0], inputs


def layer_backward(W, h, D, U, dims, antiperiodic_t=True):
    """Given the layer input h [Cin][V][4][3] and D = dL/d(out)* [Cout][V][4][3],
    return (G [9][Cout][Cin][4][4], dL/dh* [Cin][V][4][3])."""
    cout, cin = W.shape[1], W.shape[2]
    G = np.zeros_like(W)
    Dh = np.zeros_like(h)
    for b in range(cin):
        for p in range(NPATH):
            t = transport(h[b], U, dims, p, antiperiodic_t)
            G[p, :, b] = 2.0 * np.einsum('axsc,xtc->ast', D, np.conj(t))
            g = np.einsum('ats,axtc->xsc', np.conj(W[p, :, b]), D)       # sum_a W^+ D_a
            Dh[b] += transport(g, U, dims, reverse(p), antiperiodic_t)  # T_p^+ = T_{reverse(p)}
    return G, Dh


def loss_and_grads(Ws, pairs, U, dims, antiperiodic_t=True):
    """L = sum_i |N(r_i) - e_i|^2/|e_i|^2 and its gradients for every layer."""
    L = 0.0
    Gs = [np.zeros_like(W) for W in Ws]
    for r, e in pairs:
        y, inputs = forward(Ws, r, U, dims, antiperiodic_t)
        ne = float(np.vdot(e, e).real)
        diff = y - e
        L += float(np.vdot(diff, diff).real) / ne
        D = (diff / ne)[None]
        for l in range(len(Ws) - 1, -1, -1):
            G, D = layer_backward(Ws[l], inputs[l], D, U, dims, antiperiodic_t)
            Gs[l] += G
    return L, Gs


class Adam:
    """Adam on the real and imaginary parts of each weight (lr, beta1, beta2, eps)."""

    def __init__(self, shapes, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = [np.zeros(s, dtype=np.complex128) for s in shapes]
        self.v = [np.zeros(s, dtype=np.complex128) for s in shapes]
        self.t = 0

    def step(self, Ws, Gs):
        self.t += 1
        out = []
        for i, (W, G) in enumerate(zip(Ws, Gs)):
            gr, gi = G.real, G.imag
            m, v = self.m[i], self.v[i]
            mr = self.b1 * m.real + (1 - self.b1) * gr
            mi = self.b1 * m.imag + (1 - self.b1) * gi
            vr = self.b2 * v.real + (1 - self.b2) * gr * gr
            vi = self.b2 * v.imag + (1 - self.b2) * gi * gi
            self.m[i] = mr + 1j * mi
            self.v[i] = vr + 1j * vi
            c1 = 1 - self.b1 ** self.t
            c2 = 1 - self.b2 ** self.t
            upd_r = self.lr * (mr / c1) / (np.sqrt(vr / c2) + self.eps)
            upd_i = self.lr * (mi / c1) / (np.sqrt(vi / c2) + self.eps)
            out.append(W - (upd_r + 1j * upd_i))
        return out


def loss_and_grads_residual(Ws, rs, U, dims, apply_M, antiperiodic_t=True):
    """Residual form of the loss, L = sum_i |r_i - M N(r_i)|^2 / |r_i|^2, with M
    given as a callable on [V][4][3] fields.  D = dL/dN* = M^+ (M N(r) - r)/|r|^2,
    M^+ = gamma5 M gamma5 (gamma5-hermiticity of Eq. (2))."""
    g5 = np.diag(lattice.gamma5()).real.astype(np.complex128)
    flip = lambda v: v * g5[None, :, None]
    L = 0.0
    Gs = [np.zeros_like(W) for W in Ws]
    for r in rs:
        y, inputs = forward(Ws, r, U, dims, antiperiodic_t)
        nr = float(np.vdot(r, r).real)
        t = apply_M(y) - r
        L += float(np.vdot(t, t).real) / nr
        D = flip(apply_M(flip(t / nr)))[None]
        for l in range(len(Ws) - 1, -1, -1):
            G, D = layer_backward(Ws[l], inputs[l], D, U, dims, antiperiodic_t)
            Gs[l] += G
    return L, Gs
