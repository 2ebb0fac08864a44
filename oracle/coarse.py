"""Coarse-grid operator (oracle, FP64; test infrastructure).

Setup step 4 of Sec. 3.4 builds Mhat = P^+ M P.  Because M only couples
nearest neighbours, Mhat does too, and it takes the form of Eq. (3): a dense
N x N block per coarse site and hop, N = 2*Nvec.  Eq. (3) as printed shows a
unit diagonal and a daggered backward link; this oracle keeps the general
form that the Galerkin product actually produces (a full diagonal block X
and eight explicit hop blocks), which is what the stencil applies:

    y(xc) = X(xc) u(xc) + sum_mu [ Y_{2mu}(xc) u(xc + mu) + Y_{2mu+1}(xc) u(xc - mu) ]

with periodic wrap on the coarse lattice (boundary signs of the fine
operator end up inside Y).

Galerkin build by hop direction: with Pf(x) the dof x N slice of P at fine
site x, D(x) the on-site block of the parent operator and H_d(x) its hop
block towards x' = x +/- mu,
    X(xc)  = sum_{x in B} Pf(x)^+ D(x) Pf(x) + sum of hops that stay inside B
    Y_d(xc) = sum_{x in B, x' not in B} Pf(x)^+ H_d(x) Pf(x').
On a coarse extent of 2, xc + mu and xc - mu coincide; the split between
Y_{2mu} and Y_{2mu+1} is then by hop direction, and only their sum is fixed
by Mhat.  The parent is either the fine Wilson-clover operator (D = 4 + m0
+ A, H from Eq. (2)) or a coarse operator (D = X, H_d = Y_d), which is the
recursion of Sec. 3.4.
"""
import numpy as np

from . import lattice, transfer, wilson


class CoarseOp:
    """X [Vc][N][N], Y [8][Vc][N][N] on lattice dims."""

    def __init__(self, dims, X, Y):
        self.dims = tuple(dims)
        self.X = X
        self.Y = Y
        self.N = X.shape[-1]
        self.nbr = np.stack([lattice.neighbour(self.dims, d // 2, 1 - 2 * (d % 2)) for d in range(8)])

    def apply(self, u):
        """Eq. (3); u [Vc][N] or [Vc][N][nrhs].  Summation: X first, then d = 0..7."""
        shp = u.shape
        u = u.reshape(self.X.shape[0], self.N, -1)
        y = np.einsum('xij,xjr->xir', self.X, u)
        for d in range(8):
            y = y + np.einsum('xij,xjr->xir', self.Y[d], u[self.nbr[d]])
        return y.reshape(shp)

    def apply_sites(self, u, sites):
        """Eq. (3) at the listed coarse sites only; u [Vc][N] or [Vc][N][nrhs]."""
        sites = np.asarray(sites)
        u = u.reshape(self.X.shape[0], self.N, -1)
        y = np.einsum('xij,xjr->xir', self.X[sites], u[sites])
        for d in range(8):
            y = y + np.einsum('xij,xjr->xir', self.Y[d][sites], u[self.nbr[d][sites]])
        return y

    def _c_args(self, u):
        import ctypes
        Vc, N = self.X.shape[0], self.N
        uu = np.ascontiguousarray(u, dtype=np.complex128).reshape(Vc, N, -1)
        X = np.ascontiguousarray(self.X, dtype=np.complex128)
        Y = np.ascontiguousarray(self.Y, dtype=np.complex128)
        return (ctypes.c_int * 4)(*self.dims), X, Y, uu, np.empty_like(uu)

    def apply_c(self, u):
        """Eq. (3) from the plain C loop in csrc/coarse_apply.c (same summation order)."""
        from .wilson import _clib
        L, X, Y, uu, y = self._c_args(u)
        _clib().oracle_coarse_apply(L, self.N, uu.shape[2], X.ctypes.data, Y.ctypes.data, uu.ctypes.data,
                                    y.ctypes.data)
        return y.reshape(np.shape(u))

    def time_apply_c(self, u, reps, threads=0):
        """Mean seconds per C apply over `reps` repetitions after a warm-up, with
        `threads` OpenMP threads (0: the OpenMP default); returns (seconds, threads used, y)."""
        import ctypes
        from .wilson import _clib
        L, X, Y, uu, y = self._c_args(u)
        used = ctypes.c_int(0)
        sec = _clib().oracle_coarse_apply_timed(L, self.N, uu.shape[2], X.ctypes.data, Y.ctypes.data,
                                                uu.ctypes.data, y.ctypes.data, int(reps), int(threads),
                                                ctypes.addressof(used))
        return sec, used.value, y.reshape(np.shape(u))

    def dense(self):
        Vc, N = self.X.shape[0], self.N
        M = np.zeros((Vc, N, Vc, N), dtype=np.complex128)
        idx = np.arange(Vc)
        M[idx, :, idx, :] += self.X
        for d in range(8):
            for x in range(Vc):
                M[x, :, self.nbr[d][x], :] += self.Y[d][x]
        return M.reshape(Vc * N, Vc * N)


class FineParent:
    """The Wilson-clover operator seen as on-site block + eight hop blocks."""

    def __init__(self, U, clover, m0, dims, antiperiodic_t=True):
        self.U, self.clover, self.m0 = U, clover, m0
        self.dims = tuple(dims)
        self.anti = antiperiodic_t
        self.dof = 12

    def diag(self, sites):
        D = np.broadcast_to((4.0 + self.m0) * np.eye(12, dtype=np.complex128), (len(sites), 12, 12)).copy()
        if self.clover is not None:
            D += self.clover[sites]
        return D

    def hop(self, d):
        return wilson.hop_matrices(self.U, self.dims, d, self.anti)


class CoarseParent:
    def __init__(self, op):
        self.op = op
        self.dims = op.dims
        self.dof = op.N

    def diag(self, sites):
        return self.op.X[sites]

    def hop(self, d):
        return self.op.Y[d]


def galerkin(parent, Vb, block, coarse_sites=None):
    """Build X, Y of Mhat = P^+ M P for the given coarse sites (all by default).

    Returns (X [n][N][N], Y [8][n][N][N]) for the n requested coarse sites;
    with coarse_sites=None a CoarseOp is returned."""
    dims = parent.dims
    cdims = transfer.coarse_dims(dims, block)
    Vc = lattice.volume(cdims)
    members = transfer.sites_of_blocks(dims, block)
    owner = transfer.block_of_site(dims, block)
    Pf = transfer.full_basis(Vb)
    N = Pf.shape[-1]
    want = np.arange(Vc) if coarse_sites is None else np.asarray(coarse_sites)
    X = np.zeros((len(want), N, N), dtype=np.complex128)
    Y = np.zeros((8, len(want), N, N), dtype=np.complex128)
    hops = [parent.hop(d) for d in range(8)]
    nbrs = [lattice.neighbour(dims, d // 2, 1 - 2 * (d % 2)) for d in range(8)]
    for i, xc in enumerate(want):
        xs = members[xc]
        P = Pf[xs]
        PH = np.conj(np.swapaxes(P, 1, 2))
        X[i] += (PH @ (parent.diag(xs) @ P)).sum(axis=0)
        for d in range(8):
            xn = nbrs[d][xs]
            T = PH @ (hops[d][xs] @ Pf[xn])
            inside = owner[xn] == xc
            X[i] += T[inside].sum(axis=0)
            Y[d, i] += T[~inside].sum(axis=0)
    if coarse_sites is None:
        return CoarseOp(cdims, X, Y)
    return X, Y
