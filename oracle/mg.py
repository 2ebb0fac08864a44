"""Adaptive multigrid hierarchy and K-cycle (oracle, FP64; test infrastructure).

Setup (Sec. 3.4, steps 1-4), per level:
  1-2. for k = 0..Nvec-1: take a random start x0 (an input), make it
       orthogonal to the earlier candidates, relax the homogeneous system
       A x = 0 from it, make the result orthogonal to the earlier candidates
       again and normalise it.  The paper names neither the relaxation method
       nor k; the reading used here is GCR(10) for `setup_iters` steps.
  3.   blockwise chirality-split orthonormalisation -> P (transfer.py);
  4.   Galerkin product Mhat = P^+ A P -> next level (coarse.py).

Solve (Sec. 7.1): flexible GCR(10) on the fine level preconditioned by the
K-cycle K_0, where on level l
    K_l(r):  x  = MR_s(r)                    (pre-smoothing)
             r1 = r - A_l x
             xc = GCR_{l+1}(R r1)             (GCR(10) preconditioned by K_{l+1},
                                               plain GCR on the coarsest level)
             x += P xc
             x += MR_s(r - A_l x)             (post-smoothing)
Inner tolerances are not given in the paper; readings: relative 0.25 with
at most 10 steps on intermediate levels and 100 on the coarsest.

Red-black preconditioning on every level (Sec. 7.1, with the Schur
complement of Sec. 3.3, evenodd.py), option `evenodd`:
  * smoother: MR_s on the Schur system S x_e = b_e - M_eo M_oo^-1 r_o of the
    level, then the odd sites back-substituted, x_o = M_oo^-1 (r_o - M_oe x_e);
    the residual it leaves is zero on the odd sites;
  * every GCR (the coarse-grid solves and the outer FGCR) runs on the Schur
    system of its level; a K-cycle preconditioner of level l is applied to
    the even residual embedded in the whole lattice (odd part zero) and its
    even part is kept (exact when K_l = A_l^-1, since (A^-1)_ee = S^-1);
    the odd sites are back-substituted after the solve;
  * tolerances are relative to the norm of the Schur source; the outer solve
    stops when the Schur residual reaches tol |b|, which is the whole-lattice
    residual after the back-substitution.
"""
import numpy as np

from . import coarse, evenodd, lattice, solvers, transfer, wilson


class FineLevel:
    def __init__(self, U, clover, m0, dims, antiperiodic_t=True):
        self.U, self.clover, self.m0 = U, clover, m0
        self.dims = tuple(dims)
        self.anti = antiperiodic_t
        self.dof = 12
        self.V = lattice.volume(dims)

    def apply(self, v):
        return wilson.apply_wilson_clover(v.reshape(self.V, 4, 3), self.U, self.clover,
                                          self.m0, self.dims, self.anti).reshape(v.shape)

    def parent(self):
        return coarse.FineParent(self.U, self.clover, self.m0, self.dims, self.anti)

    def schur(self):
        return evenodd.fine_schur(self.U, self.clover, self.m0, self.dims, self.anti)


class CoarseLevel:
    def __init__(self, op):
        self.op = op
        self.dims = op.dims
        self.dof = op.N
        self.V = lattice.volume(op.dims)

    def apply(self, v):
        return self.op.apply(v.reshape(self.V, self.dof)).reshape(v.shape)

    def parent(self):
        return coarse.CoarseParent(self.op)

    def schur(self):
        return evenodd.coarse_schur(self.op)


def _orth_against(v, basis):
    for w in basis:
        v = v - solvers.dot(w, v) * w
    return v


def null_vectors(level, starts, setup_iters):
    """Near-null candidates from random starts [Nvec][V*dof] (steps 1-2)."""
    out = []
    zero = np.zeros(level.V * level.dof, dtype=np.complex128)
    for x0 in starts:
        x0 = _orth_against(x0.reshape(-1).astype(np.complex128), out)
        x, _ = solvers.gcr(level.apply, zero, tol=0.0, restart=10, maxit=setup_iters, x0=x0)
        x = _orth_against(x, out)
        out.append(x / solvers.norm(x))
    return np.array(out)


class Hierarchy:
    def __init__(self, fine, blocks, nvecs, starts, setup_iters=100,
                 given_vectors=None):
        """starts[l]: random starts [Nvec_l][V_l*dof_l] for level l;
        given_vectors[l] (optional) replaces the relaxation of level l."""
        self.levels = [fine]
        self.transfers = []
        for l, (block, nvec) in enumerate(zip(blocks, nvecs)):
            lev = self.levels[-1]
            if given_vectors is not None and given_vectors[l] is not None:
                vecs = given_vectors[l]
            else:
                vecs = null_vectors(lev, starts[l], setup_iters)
            vecs = vecs.reshape(nvec, lev.V, lev.dof)
            Vb = transfer.block_orthonormalize(vecs, lev.dims, block)
            self.transfers.append((Vb, lev.dims, tuple(block)))
            op = coarse.galerkin(lev.parent(), Vb, block)
            self.levels.append(CoarseLevel(op))

    def prolong(self, l, uc):
        Vb, dims, block = self.transfers[l]
        return transfer.prolong(Vb, uc.reshape(-1, Vb.shape[2] * 2), dims, block).reshape(-1)

    def restrict(self, l, v):
        Vb, dims, block = self.transfers[l]
        return transfer.restrict(Vb, v.reshape(-1, Vb.shape[1]), dims, block).reshape(-1)


class KCycle:
    def __init__(self, hier, smoother_steps=4, inner_tol=0.25, inner_maxit=10,
                 coarsest_tol=0.25, coarsest_maxit=100, smoother=None, coarsest_direct=False,
                 evenodd=False):
        self.h = hier
        self.evenodd = evenodd
        self._schur = {}
        self.s = smoother_steps
        # coarsest_direct: the exact coarse-grid correction on the coarsest
        # level, x = Mhat^-1 r (a dense LAPACK solve), instead of its GCR
        self.coarsest_direct = coarsest_direct
        self._dense = None
        self.inner_tol, self.inner_maxit = inner_tol, inner_maxit
        self.coarsest_tol, self.coarsest_maxit = coarsest_tol, coarsest_maxit
        self.smoother = smoother          # optional replacement for MR on level 0
        self.inner_iters = [0] * len(hier.levels)

    def schur(self, l):
        if l not in self._schur:
            self._schur[l] = self.h.levels[l].schur()
        return self._schur[l]

    def smooth(self, l, r):
        if l == 0 and self.smoother is not None:
            return self.smoother(r)
        if self.evenodd:
            S = self.schur(l)
            xe = solvers.mr(lambda v: S.apply(v.reshape(-1, S.dof)).reshape(-1), S.source(r).reshape(-1), self.s)
            return S.reconstruct(xe.reshape(-1, S.dof), r).reshape(r.shape)
        return solvers.mr(self.h.levels[l].apply, r, self.s)

    def schur_gcr(self, l, b, tol, maxit, precond=None, info=None):
        """GCR(10) on the Schur system of level l for the whole-lattice b,
        tolerance relative to |source|; returns the whole-lattice solution."""
        S = self.schur(l)
        be = S.source(b).reshape(-1)
        Sa = lambda v: S.apply(v.reshape(-1, S.dof)).reshape(-1)
        pre = None
        if precond is not None:
            pre = lambda re: S.even_part(precond(S.embed_even(re).reshape(-1)))
        xe, info = solvers.gcr(Sa, be, tol, 10, maxit, precond=pre, info=info)
        return S.reconstruct(xe.reshape(-1, S.dof), b).reshape(-1), info

    def __call__(self, r, l=0):
        A = self.h.levels[l].apply
        x = self.smooth(l, r)
        r1 = r - A(x)
        rc = self.h.restrict(l, r1)
        nl = l + 1
        last = nl == len(self.h.levels) - 1
        info = solvers.SolveInfo()
        if last and self.coarsest_direct:
            if self._dense is None:
                self._dense = self.h.levels[nl].op.dense()
            xc = np.linalg.solve(self._dense, rc)
            info.iters = 1
        elif last and self.evenodd:
            xc, info = self.schur_gcr(nl, rc, self.coarsest_tol, self.coarsest_maxit, info=info)
        elif last:
            xc, info = solvers.gcr(self.h.levels[nl].apply, rc, self.coarsest_tol, 10,
                                   self.coarsest_maxit, info=info)
        elif self.evenodd:
            xc, info = self.schur_gcr(nl, rc, self.inner_tol, self.inner_maxit, precond=lambda z: self(z, nl),
                                      info=info)
        else:
            xc, info = solvers.gcr(self.h.levels[nl].apply, rc, self.inner_tol, 10,
                                   self.inner_maxit, precond=lambda z: self(z, nl), info=info)
        self.inner_iters[nl] += info.iters
        x = x + self.h.prolong(l, xc)
        x = x + self.smooth(l, r - A(x))
        return x


def solve(hier, b, tol=1e-10, restart=10, maxit=500, **kcycle_args):
    K = KCycle(hier, **kcycle_args)
    if K.evenodd:
        # outer FGCR on the Schur system, stopping at |r_e| <= tol |b|
        S = K.schur(0)
        be = S.source(b).reshape(-1)
        tol_e = tol * solvers.norm(b) / solvers.norm(be)
        Sa = lambda v: S.apply(v.reshape(-1, S.dof)).reshape(-1)
        pre = lambda re: S.even_part(K(S.embed_even(re).reshape(-1)))
        xe, info = solvers.gcr(Sa, be, tol_e, restart, maxit, precond=pre)
        x = S.reconstruct(xe.reshape(-1, S.dof), b).reshape(b.shape)
        info.converged = solvers.norm(b - hier.levels[0].apply(x)) <= tol * solvers.norm(b) * (1 + 1e-6)
    else:
        x, info = solvers.gcr(hier.levels[0].apply, b, tol, restart, maxit, precond=K)
    info.inner_iters = K.inner_iters
    return x, info
