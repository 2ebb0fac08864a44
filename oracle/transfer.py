"""Transfer operators (oracle, FP64; test infrastructure).

Setup step 3 of Sec. 3.4: the near-null vectors are cut into disjoint
hypercubic aggregates, and each aggregate is orthonormalised on its own.
The upper and lower spin halves (the two chiralities) are aggregated
separately (Sec. 3.4, footnote on chirality), so every aggregate gives two
local bases and the coarse grid has 2*Nvec components per site.

Reading of "a QR decomposition on these blocks": modified Gram-Schmidt over
the vectors in their given order k = 0..Nvec-1, each projection pass done
twice, normalised so the diagonal of R is real and positive.

Prolongation and restriction follow Sec. 6.6:
    (P u)(x)_f       = sum_k V(x)_{f,k} u(xc(x))_{chi(f)*Nvec + k}
    (R psi)(xc)_n    = sum_{x in block(xc)} sum_{f: chi(f) = chi(n)} conj(V(x)_{f,k}) psi(x)_f
with R = P^+ (restriction is the adjoint of prolongation).

The basis is stored as V [V_fine][dof][Nvec]: row f of site x holds the
components of the Nvec basis vectors of chirality chi(f).
"""
import numpy as np

from . import lattice


class RankError(RuntimeError):
    pass


def coarse_dims(dims, block):
    for d, b in zip(dims, block):
        if d % b:
            raise ValueError('block %r does not divide lattice %r' % (block, dims))
    return tuple(d // b for d, b in zip(dims, block))


def block_of_site(dims, block):
    """Coarse site index of every fine site."""
    cd = coarse_dims(dims, block)
    x = lattice.coords(dims) // np.array(block)
    return lattice.site_index(x, cd)


def sites_of_blocks(dims, block):
    """[Vc][|B|] fine site indices of each aggregate, ordered by fine index."""
    owner = block_of_site(dims, block)
    order = np.argsort(owner, kind='stable')
    Vc = lattice.volume(coarse_dims(dims, block))
    return order.reshape(Vc, -1)


def block_orthonormalize(vecs, dims, block, rank_tol=1e-10):
    """vecs [Nvec][V][dof] -> basis V [V][dof][Nvec] (see module docstring)."""
    nvec, V, dof = vecs.shape
    half = dof // 2
    members = sites_of_blocks(dims, block)            # [Vc][B]
    Vc, B = members.shape
    # W[c, chi, k, :] = vector k restricted to aggregate c and chirality chi
    W = vecs[:, members, :]                            # [k][Vc][B][dof]
    W = W.reshape(nvec, Vc, B, 2, half)
    W = np.transpose(W, (1, 3, 0, 2, 4)).reshape(Vc, 2, nvec, B * half).copy()
    for k in range(nvec):
        before = np.linalg.norm(W[:, :, k, :], axis=-1)
        for _pass in range(2):
            for j in range(k):
                c = np.einsum('abi,abi->ab', W[:, :, j, :].conj(), W[:, :, k, :])
                W[:, :, k, :] -= c[..., None] * W[:, :, j, :]
        nrm = np.linalg.norm(W[:, :, k, :], axis=-1)
        if np.any(nrm < rank_tol * before):
            raise RankError('near-null vector %d is linearly dependent within an aggregate' % k)
        W[:, :, k, :] /= nrm[..., None]
    # scatter back to [V][dof][Nvec]
    W = W.reshape(Vc, 2, nvec, B, half)
    out = np.zeros((V, 2, half, nvec), dtype=np.complex128)
    out[members] = np.transpose(W, (0, 3, 1, 4, 2))    # [Vc][B][chi][half][k]
    return out.reshape(V, dof, nvec)


def prolong(Vb, uc, dims, block):
    """Fine field [V][dof] = P u for coarse u [Vc][2*Nvec]."""
    V, dof, nvec = Vb.shape
    owner = block_of_site(dims, block)
    chi = np.arange(dof) // (dof // 2)
    # coarse components seen by fine row f: u(xc)[chi(f)*nvec + k]
    uc = uc.reshape(-1, 2, nvec)
    return np.einsum('xfk,xfk->xf', Vb, uc[owner][:, chi, :])


def restrict(Vb, psi, dims, block):
    """Coarse field [Vc][2*Nvec] = P^+ psi for fine psi [V][dof]."""
    V, dof, nvec = Vb.shape
    psi = psi.reshape(V, dof)
    owner = block_of_site(dims, block)
    Vc = owner.max() + 1
    half = dof // 2
    out = np.zeros((Vc, 2, nvec), dtype=np.complex128)
    for chi in range(2):
        rows = slice(chi * half, (chi + 1) * half)
        contrib = np.einsum('xfk,xf->xk', Vb[:, rows, :].conj(), psi[:, rows])
        np.add.at(out[:, chi, :], owner, contrib)
    return out.reshape(Vc, 2 * nvec)


def full_basis(Vb):
    """The dense per-site slice of P, [V][dof][2*Nvec] (zero off-chirality)."""
    V, dof, nvec = Vb.shape
    half = dof // 2
    Pf = np.zeros((V, dof, 2 * nvec), dtype=np.complex128)
    Pf[:, :half, :nvec] = Vb[:, :half, :]
    Pf[:, half:, nvec:] = Vb[:, half:, :]
    return Pf
