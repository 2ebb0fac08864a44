"""Seeded synthetic inputs shared by the HIP path and the oracle.

This module only draws random numbers and shapes them into the lattice
fields a caller hands to either side (gauge links, Gaussian vectors, random
gauge rotations).  It holds none of the method's arithmetic: no Dirac
operator, projector, transfer or coarse-grid step lives here.

Seeding: every stream is ``numpy.random.Generator(PCG64(SeedSequence([seed,
purpose])))`` with purpose 0 = gauge links (draw order: direction, site,
Gell-Mann index), 1 = near-null / setup vectors, 2 = right-hand sides,
3 = gauge rotations, 4 = smoother training data.

Layouts (complex128, row-major, site index i = x0 + L0*(x1 + L1*(x2 + L2*x3)),
dimension 3 is time):
  gauge   [4][V][3][3]     U_mu(x), colour row, colour column
  fields  [..][V][dof]     dof = 12 (spin*3 + colour) on the fine grid
"""
import numpy as np

GAUGE, NULLVEC, RHS, ROTATION, TRAINING = 0, 1, 2, 3, 4


def rng(seed, purpose):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(purpose)])))


def volume(dims):
    v = 1
    for d in dims:
        v *= int(d)
    return v


def gell_mann():
    """The eight Gell-Mann matrices (Hermitian, traceless, tr(l_a l_b) = 2 delta_ab)."""
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1] = -1j; l[1][1, 0] = 1j
    l[2][0, 0] = 1; l[2][1, 1] = -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2] = -1j; l[4][2, 0] = 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2] = -1j; l[6][2, 1] = 1j
    l[7][0, 0] = l[7][1, 1] = 1 / np.sqrt(3); l[7][2, 2] = -2 / np.sqrt(3)
    return l


def _expi_hermitian(H, eps):
    """exp(i*eps*H) for a stack of Hermitian matrices via the eigendecomposition."""
    w, Q = np.linalg.eigh(H)
    return np.einsum('...ab,...b,...cb->...ac', Q, np.exp(1j * eps * w), Q.conj())


def random_su3(n, eps, gen):
    """n matrices U = exp(i eps H), H = sum_a h_a lambda_a / 2, h_a ~ N(0,1) i.i.d."""
    h = gen.standard_normal((n, 8))
    H = np.einsum('na,aij->nij', h, gell_mann() / 2)
    return _expi_hermitian(H, eps)


def gauge_field(dims, eps, seed, chunk=1 << 18):
    """Gauge links [4][V][3][3] drawn with the recipe U = exp(i eps H)."""
    V = volume(dims)
    gen = rng(seed, GAUGE)
    U = np.empty((4 * V, 3, 3), dtype=np.complex128)
    for s in range(0, 4 * V, chunk):
        n = min(chunk, 4 * V - s)
        U[s:s + n] = random_su3(n, eps, gen)
    return U.reshape(4, V, 3, 3)


def gaussian(shape, seed, purpose):
    """Complex Gaussian entries (N(0,1) + i N(0,1)) / sqrt(2)."""
    gen = rng(seed, purpose)
    re = gen.standard_normal(shape)
    im = gen.standard_normal(shape)
    return (re + 1j * im) / np.sqrt(2.0)


def gauge_rotation(dims, seed, eps=3.0):
    """A random SU(3) matrix per site [V][3][3] (for gauge-covariance checks)."""
    return random_su3(volume(dims), eps, rng(seed, ROTATION))
