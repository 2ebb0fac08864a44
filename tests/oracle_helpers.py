"""Fixtures shared by the oracle pin tests (constructed inputs, no method code)."""
import numpy as np

import synth
from oracle import lattice


def unit_gauge(dims):
    V = lattice.volume(dims)
    return np.broadcast_to(np.eye(3, dtype=np.complex128), (4, V, 3, 3)).copy()


def pure_gauge(dims, seed):
    """U_mu(x) = g(x) g(x+mu)^+ for a random SU(3) rotation g."""
    g = synth.gauge_rotation(dims, seed)
    U = np.empty((4, lattice.volume(dims), 3, 3), dtype=np.complex128)
    for mu in range(4):
        gn = g[lattice.neighbour(dims, mu, 1)]
        U[mu] = g @ np.conj(np.swapaxes(gn, 1, 2))
    return U


def gauge_rotate(U, g, dims):
    """U'_mu(x) = g(x) U_mu(x) g(x+mu)^+."""
    out = np.empty_like(U)
    for mu in range(4):
        gn = g[lattice.neighbour(dims, mu, 1)]
        out[mu] = g @ U[mu] @ np.conj(np.swapaxes(gn, 1, 2))
    return out


def abelian_flux(dims, n, q=(1.0, -1.0, 0.0)):
    """Constant abelian field strength theta = 2 pi n / (L0 L1) in the 0-1 plane:
    every 0-1 plaquette equals diag(exp(i q theta)), all other plaquettes are 1."""
    L0, L1 = dims[0], dims[1]
    theta = 2 * np.pi * n / (L0 * L1)
    q = np.asarray(q)
    x = lattice.coords(dims)
    V = lattice.volume(dims)
    U = unit_gauge(dims)
    ph0 = np.exp(-1j * np.outer(x[:, 1], q) * theta)           # U_0(x) = diag(e^{-i q theta x1})
    U[0] = ph0[:, :, None] * np.eye(3)[None]
    ph1 = np.ones((V, 3), dtype=np.complex128)
    last = x[:, 1] == L1 - 1
    ph1[last] = np.exp(1j * np.outer(x[last, 0], q) * theta * L1)
    U[1] = ph1[:, :, None] * np.eye(3)[None]
    return U, theta, q


def free_spectrum(dims, m0, antiperiodic_t=True):
    """Closed-form eigenvalues of the free Wilson operator (each with multiplicity 6)."""
    ps = []
    for mu, L in enumerate(dims):
        n = np.arange(L)
        p = (2 * n + 1) * np.pi / L if (mu == 3 and antiperiodic_t) else 2 * np.pi * n / L
        ps.append(p)
    P = np.meshgrid(*ps, indexing='ij')
    a = m0 + sum(1 - np.cos(p) for p in P)
    b = np.sqrt(sum(np.sin(p) ** 2 for p in P))
    ev = np.concatenate([(a + 1j * b).ravel(), (a - 1j * b).ravel()])
    return np.repeat(ev, 6)      # each sign: 2 spin states x 3 colours


def match_multisets(a, b):
    """Largest distance between two multisets of complex numbers after a
    greedy nearest-neighbour pairing (both sorted the same way first)."""
    a = np.asarray(a)
    b = np.asarray(b)
    if len(a) != len(b):
        return np.inf
    used = np.zeros(len(b), bool)
    worst = 0.0
    for z in a:
        d = np.abs(b - z)
        d[used] = np.inf
        j = int(np.argmin(d))
        used[j] = True
        worst = max(worst, d[j])
    return worst
