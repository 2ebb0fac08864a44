"""Schwarz alternating procedure (SAP) smoother (oracle, FP64; test infrastructure).

The paper names Schwarz-preconditioned domain-decomposition smoothers as the
way to cut the smoother's global communication (its introduction, and the
latency-bound coarse levels of Sec. 7.2 / the outlook of Sec. 9): each block of
the lattice is relaxed on its own, with no global reduction.  The form written
out here is the multiplicative two-colour sweep:

  * the lattice is cut into hypercubic blocks of extent `block` (dividing the
    lattice, at least two blocks per dimension, an even number of them), and a
    block's colour is the parity of the sum of its block coordinates, so two
    blocks that share a face have opposite colours;
  * A_BB is the operator restricted to block B: the hops that leave the block
    are dropped;
  * one sweep from x = 0 for the right-hand side r:
        for colour c = 0, 1: for every block B of colour c:
            r_B = (r - A x) on B;  solve A_BB d = r_B by `iters` MR steps from 0
            (the step lengths are the block's own: alpha_B = <A_BB s, s>/<A_BB s, A_BB s>);
            x += d on B.
Blocks of one colour do not touch each other, so all of them are relaxed at
once (blockwise sums for the MR scalars).
"""
import numpy as np

from . import lattice


def block_ids(dims, block):
    """Block index and block colour of every site, lattice order."""
    dims, block = tuple(dims), tuple(block)
    nb = [d // b for d, b in zip(dims, block)]
    for d, b, n in zip(dims, block, nb):
        if d % b or n < 2 or n % 2:
            raise ValueError('blocks of %s on %s: need an even number (>= 2) of blocks per dimension' % (block, dims))
    c = lattice.coords(dims) // np.asarray(block)
    bid = c[:, 0] + nb[0] * (c[:, 1] + nb[1] * (c[:, 2] + nb[2] * c[:, 3]))
    colour = c.sum(axis=1) % 2
    return bid, colour, int(np.prod(nb))


def sap(apply, r, dims, block, iters, dof=12):
    """One multiplicative two-colour SAP sweep from x = 0 for A x = r, with
    `iters` block MR steps per block; apply(v [V][dof]) is the whole-lattice
    operator.  Returns x [V][dof]."""
    V = lattice.volume(dims)
    r = np.asarray(r).reshape(V, dof)
    bid, colour, nblk = block_ids(dims, block)
    x = np.zeros_like(r)
    for c in (0, 1):
        m = (colour == c)[:, None]
        rb = np.where(m, r - apply(x), 0)
        d = np.zeros_like(r)
        for _ in range(iters):
            Ar = np.where(m, apply(rb), 0)          # A_BB rb: hops from outside the colour dropped
            num = np.bincount(bid, weights=np.sum(np.conj(Ar) * rb, axis=1).real, minlength=nblk) \
                + 1j * np.bincount(bid, weights=np.sum(np.conj(Ar) * rb, axis=1).imag, minlength=nblk)
            den = np.bincount(bid, weights=np.sum(np.abs(Ar) ** 2, axis=1), minlength=nblk)
            alpha = np.where(den > 0, num / np.where(den > 0, den, 1), 0)[bid][:, None]
            d = d + alpha * rb
            rb = rb - alpha * Ar
        x = x + d
    return x
