"""Lattice geometry and Dirac-space constants (oracle, FP64; test infrastructure).

Site ordering follows the paper's index decomposition (Sec. 6.1): x0 runs
fastest, dimension 3 is time.
"""
import functools

import numpy as np


def volume(dims):
    return int(np.prod(dims))


def coords(dims):
    """Integer coordinates [V][4] of every site, x0 fastest."""
    L0, L1, L2, L3 = dims
    i = np.arange(volume(dims))
    x0 = i % L0
    x1 = (i // L0) % L1
    x2 = (i // (L0 * L1)) % L2
    x3 = i // (L0 * L1 * L2)
    return np.stack([x0, x1, x2, x3], axis=1)


def site_index(x, dims):
    L0, L1, L2, L3 = dims
    return x[..., 0] + L0 * (x[..., 1] + L1 * (x[..., 2] + L2 * x[..., 3]))


@functools.lru_cache(maxsize=64)
def _neighbour(dims, mu, step):
    x = coords(dims).copy()
    x[:, mu] = (x[:, mu] + step) % dims[mu]
    out = site_index(x, dims)
    out.setflags(write=False)
    return out


def neighbour(dims, mu, step):
    """Index of x + step*mu_hat (periodic wrap) for every site x."""
    return _neighbour(tuple(int(d) for d in dims), int(mu), int(step))


def boundary_sign(dims, mu, step, antiperiodic_t):
    """+1, or -1 on hops x -> x+step*mu_hat that cross the time boundary when
    time is antiperiodic (space is periodic)."""
    s = np.ones(volume(dims))
    if antiperiodic_t and mu == 3:
        x = coords(dims)[:, 3]
        cross = (x == dims[3] - 1) if step > 0 else (x == 0)
        s[cross] = -1.0
    return s


def gammas():
    """Euclidean gamma matrices gamma_1..gamma_4 in a chiral basis, returned as
    g[mu] for mu = 0..3 (mu = 3 is time).

    gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] (k = 1..3) and
    gamma_4 = [[0, 1], [1, 0]]; then gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4
    is diag(1, 1, -1, -1), so spins {0,1} and {2,3} are the two chiralities
    that the aggregation of Sec. 3.4 keeps apart.
    """
    s = [np.array([[0, 1], [1, 0]], dtype=complex),
         np.array([[0, -1j], [1j, 0]], dtype=complex),
         np.array([[1, 0], [0, -1]], dtype=complex)]
    z = np.zeros((2, 2), dtype=complex)
    g = [np.block([[z, -1j * sk], [1j * sk, z]]) for sk in s]
    g.append(np.block([[z, np.eye(2)], [np.eye(2), z]]))
    return np.array(g)


def gamma5():
    g = gammas()
    return g[0] @ g[1] @ g[2] @ g[3]


def projectors():
    """Spin matrices of Eq. (2): P^{-mu} = 1 - gamma_mu multiplies the forward
    hop (x -> x+mu), P^{+mu} = 1 + gamma_mu the backward hop."""
    g = gammas()
    one = np.eye(4)
    return np.array([one - g[m] for m in range(4)]), np.array([one + g[m] for m in range(4)])


def sigma(mu, nu):
    """sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu] (Hermitian)."""
    g = gammas()
    return 0.5j * (g[mu] @ g[nu] - g[nu] @ g[mu])
