"""Red-black (even-odd) preconditioning (oracle, FP64; test infrastructure).

Sec. 3.3 (and the solver set-up of Sec. 7.1, which uses it on every level):
both the fine operator of Eq. (2) and the coarse operator of Eq. (3) couple a
site only to itself and to its nearest neighbours, which have the other
parity p(x) = (x0 + x1 + x2 + x3) mod 2.  Ordering the even sites first,

    M = [[M_ee, M_eo],        M_ee, M_oo  site-local blocks
         [M_oe, M_oo]],       M_eo, M_oe  the hops,

and M x = b is solved through the Schur complement on the even sites

    S = M_ee - M_eo M_oo^-1 M_oe,
    S x_e = b_e - M_eo M_oo^-1 b_o,       x_o = M_oo^-1 (b_o - M_oe x_e).

Here the site-local block is (4 + m0) + A(x) for the fine operator and X(x)
for the coarse operator; everything else is the hops.  Every function below
evaluates this with whole-lattice applications of the operator itself:
for an even-only field E (odd entries zero) the hop part M_oe E is the odd
half of M E, because the site-local block keeps E even.

Half-lattice fields are indexed by the even (odd) sites in lattice order.
"""
import numpy as np

from . import lattice


def parity(dims):
    """p(x) for every site, lattice order."""
    return lattice.coords(dims).sum(axis=1) % 2


def sites(dims, p):
    """Sites of parity p in lattice order."""
    return np.nonzero(parity(dims) == p)[0]


class Schur:
    """Even-odd Schur complement of an operator given as
    apply(v [V][dof]) and its site-local blocks local [V][dof][dof]."""

    def __init__(self, apply, local, dims):
        self.apply_full = apply
        self.dims = tuple(dims)
        self.V = lattice.volume(dims)
        self.dof = local.shape[-1]
        self.even = sites(dims, 0)
        self.odd = sites(dims, 1)
        self.local_odd_inv = np.linalg.inv(local[self.odd])

    def _embed(self, half, p):
        v = np.zeros((self.V, self.dof), dtype=np.complex128)
        v[self.even if p == 0 else self.odd] = half.reshape(-1, self.dof)
        return v

    def embed_even(self, xe):
        """Whole-lattice field [V][dof] with x_e on the even sites, 0 on the odd."""
        return self._embed(xe, 0)

    def even_part(self, v):
        """The even-site half [V/2 * dof] of a whole-lattice field."""
        return v.reshape(self.V, self.dof)[self.even].reshape(-1)

    def _oo_inv(self, vo):
        return np.einsum('xij,xj->xi', self.local_odd_inv, vo.reshape(-1, self.dof))

    def apply(self, xe):
        """S x_e = M_ee x_e - M_eo M_oo^-1 M_oe x_e."""
        shape = xe.shape
        ME = self.apply_full(self._embed(xe, 0))
        t = self._oo_inv(ME[self.odd])                 # M_oo^-1 M_oe x_e
        MT = self.apply_full(self._embed(t, 1))
        return (ME[self.even] - MT[self.even]).reshape(shape)

    def source(self, b):
        """b_e - M_eo M_oo^-1 b_o for a whole-lattice b [V][dof]."""
        b = b.reshape(self.V, self.dof)
        t = self._oo_inv(b[self.odd])
        return b[self.even] - self.apply_full(self._embed(t, 1))[self.even]

    def reconstruct(self, xe, b):
        """The whole-lattice solution from x_e: x_o = M_oo^-1 (b_o - M_oe x_e)."""
        b = b.reshape(self.V, self.dof)
        ME = self.apply_full(self._embed(xe, 0))
        x = self._embed(xe, 0)
        x[self.odd] = self._oo_inv(b[self.odd] - ME[self.odd])
        return x


def fine_schur(U, clover, m0, dims, antiperiodic_t=True):
    """Schur complement of the Wilson-clover operator of Eq. (2)."""
    from . import wilson
    V = lattice.volume(dims)
    local = np.broadcast_to((4.0 + m0) * np.eye(12, dtype=np.complex128), (V, 12, 12)).copy()
    if clover is not None:
        local += clover
    apply = lambda v: wilson.apply_wilson_clover(v.reshape(V, 4, 3), U, clover, m0, dims,
                                                 antiperiodic_t).reshape(V, 12)
    return Schur(apply, local, dims)


def coarse_schur(op):
    """Schur complement X_ee - Y_eo X_oo^-1 Y_oe of a coarse operator (Eq. 3)."""
    return Schur(lambda v: op.apply(v.reshape(-1, op.N)), op.X, op.dims)
