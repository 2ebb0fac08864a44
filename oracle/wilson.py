"""Fine Wilson-clover operator, Eq. (2) (oracle, FP64; test infrastructure).

    M psi(x) = (4 + m0) psi(x) + A(x) psi(x)
               - 1/2 sum_mu [ (1 - gamma_mu) (x) U_mu(x)         eta+ psi(x + mu)
                            + (1 + gamma_mu) (x) U_mu(x - mu)^+   eta- psi(x - mu) ]

eta = -1 on hops across the time boundary when time is antiperiodic.
A(x) is the 12x12 clover term (Sheikholeslami-Wohlert form; the paper only
names it as a first-order correction, so its normalisation is a reading):

    A(x) = (i c_sw / 2) sum_{mu<nu} sigma_{mu nu} (x) Fhat_{mu nu}(x),
    Fhat = (Q - Q^+)/8,  Q = sum of the four plaquette leaves at x in the
    mu-nu plane, all with the same orientation.
"""
import numpy as np

from . import lattice


def _links_at(U, idx):
    return U[idx]


def clover_leaves(U, dims, mu, nu, sites=None):
    """Q_{mu nu}(x): sum of the four same-orientation plaquettes touching x
    (at every site, or at the given sites only)."""
    V = lattice.volume(dims)
    x = np.arange(V) if sites is None else np.asarray(sites)
    f = lambda m, s: lattice.neighbour(dims, m, s)[x]
    Um, Un = U[mu], U[nu]
    dag = lambda a: np.conj(np.swapaxes(a, -1, -2))
    mm = lambda *ms: _chain(ms)
    xpm, xpn = f(mu, 1), f(nu, 1)
    xmm, xmn = f(mu, -1), f(nu, -1)
    xmm_pn = lattice.neighbour(dims, nu, 1)[xmm]        # x - mu + nu
    xmm_mn = lattice.neighbour(dims, nu, -1)[xmm]       # x - mu - nu
    xpm_mn = lattice.neighbour(dims, nu, -1)[xpm]       # x + mu - nu
    # leaf 1: x -> x+mu -> x+mu+nu -> x+nu -> x
    q = mm(Um[x], Un[xpm], dag(Um[xpn]), dag(Un[x]))
    # leaf 2: x -> x+nu -> x-mu+nu -> x-mu -> x
    q = q + mm(Un[x], dag(Um[xmm_pn]), dag(Un[xmm]), Um[xmm])
    # leaf 3: x -> x-mu -> x-mu-nu -> x-nu -> x
    q = q + mm(dag(Um[xmm]), dag(Un[xmm_mn]), Um[xmm_mn], Un[xmn])
    # leaf 4: x -> x-nu -> x+mu-nu -> x+mu -> x
    q = q + mm(dag(Un[xmn]), Um[xmn], Un[xpm_mn], dag(Um[x]))
    return q


def _chain(ms):
    out = ms[0]
    for m in ms[1:]:
        out = np.einsum('xab,xbc->xac', out, m)
    return out


def clover_field(U, dims, csw, sites=None):
    """A(x) as dense 12x12 matrices [V][12][12] (row/column index 3*spin + colour);
    with `sites`, only at those sites ([len(sites)][12][12])."""
    V = lattice.volume(dims) if sites is None else len(sites)
    A = np.zeros((V, 4, 3, 4, 3), dtype=np.complex128)
    for mu in range(4):
        for nu in range(mu + 1, 4):
            Q = clover_leaves(U, dims, mu, nu, sites)
            F = (Q - np.conj(np.swapaxes(Q, -1, -2))) / 8.0
            A += (0.5j * csw) * np.einsum('st,xab->xsatb', lattice.sigma(mu, nu), F)
    return A.reshape(V, 12, 12)


def apply_wilson_clover(psi, U, clover, m0, dims, antiperiodic_t=True, sites=None):
    """M psi for psi of shape [V][4][3] (or [V][12]); clover may be None (c_sw = 0).

    With `sites`, (M psi)(x) at those sites only, [len(sites)][4][3], and
    `clover` holds the clover term at those sites."""
    V = lattice.volume(dims)
    shape = psi.shape
    psi = psi.reshape(V, 4, 3)
    x = np.arange(V) if sites is None else np.asarray(sites)
    Pm, Pp = lattice.projectors()
    out = (4.0 + m0) * psi[x]
    if clover is not None:
        out = out + np.einsum('xij,xj->xi', clover, psi[x].reshape(len(x), 12)).reshape(len(x), 4, 3)
    for mu in range(4):
        fwd = lattice.neighbour(dims, mu, +1)[x]
        bwd = lattice.neighbour(dims, mu, -1)[x]
        eta_f = lattice.boundary_sign(dims, mu, +1, antiperiodic_t)[x]
        eta_b = lattice.boundary_sign(dims, mu, -1, antiperiodic_t)[x]
        # forward hop: (1 - gamma_mu) (x) U_mu(x) psi(x + mu)
        h = np.einsum('st,xta->xsa', Pm[mu], np.einsum('xab,xtb->xta', U[mu][x], psi[fwd]))
        out = out - 0.5 * eta_f[:, None, None] * h
        # backward hop: (1 + gamma_mu) (x) U_mu(x - mu)^dagger psi(x - mu)
        Ub = U[mu][bwd]
        h = np.einsum('st,xta->xsa', Pp[mu], np.einsum('xba,xtb->xta', np.conj(Ub), psi[bwd]))
        out = out - 0.5 * eta_b[:, None, None] * h
    return out.reshape(shape) if sites is None else out


def apply_wilson_clover_sites(psi, U, csw, m0, dims, sites, antiperiodic_t=True):
    """(M psi)(x) at the given sites only, the clover term computed there from
    the links: spot checks on lattices too large for the whole-field oracle."""
    A = clover_field(U, dims, csw, sites) if csw != 0 else None
    return apply_wilson_clover(psi, U, A, m0, dims, antiperiodic_t, sites)


def hop_matrices(U, dims, d, antiperiodic_t=True):
    """The 12x12 matrix H_d(x) [V][12][12] that multiplies psi(x +/- mu) in
    Eq. (2): d = 2*mu is the forward hop, d = 2*mu + 1 the backward hop."""
    mu, back = d // 2, d % 2
    Pm, Pp = lattice.projectors()
    if back == 0:
        eta = lattice.boundary_sign(dims, mu, +1, antiperiodic_t)
        H = np.einsum('st,xab->xsatb', Pm[mu], U[mu])
    else:
        eta = lattice.boundary_sign(dims, mu, -1, antiperiodic_t)
        Ub = U[mu][lattice.neighbour(dims, mu, -1)]
        H = np.einsum('st,xba->xsatb', Pp[mu], np.conj(Ub))
    V = lattice.volume(dims)
    return (-0.5 * eta[:, None, None]) * H.reshape(V, 12, 12)


def dense_matrix(apply, n):
    """Materialise a linear map on C^n by applying it to the unit vectors."""
    M = np.zeros((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[j] = 1.0
        M[:, j] = apply(e)
        e[j] = 0.0
    return M


_C = None


def _clib():
    global _C
    if _C is None:
        import ctypes
        import os
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), '_oracle_c.so')
        if not os.path.exists(path):
            from . import build_c
            build_c.build(verbose=False)
        lib = ctypes.CDLL(path)
        lib.oracle_wilson_clover.restype = None
        lib.oracle_wilson_clover.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_double, ctypes.c_int] + [ctypes.c_void_p] * 3
        lib.oracle_wilson_clover_csw.restype = None
        lib.oracle_wilson_clover_csw.argtypes = ([ctypes.c_void_p] * 2 + [ctypes.c_double, ctypes.c_double, ctypes.c_int]
                                                 + [ctypes.c_void_p] * 3)
        lib.oracle_coarse_apply.restype = None
        lib.oracle_coarse_apply.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int] + [ctypes.c_void_p] * 4
        lib.oracle_coarse_apply_timed.restype = ctypes.c_double
        lib.oracle_coarse_apply_timed.argtypes = ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int] + [ctypes.c_void_p] * 4
                                                  + [ctypes.c_int, ctypes.c_int, ctypes.c_void_p])
        _C = lib
    return _C


def apply_wilson_clover_c(psi, U, clover, m0, dims, antiperiodic_t=True):
    """Same map as apply_wilson_clover, from the plain C loop in csrc/wilson_clover.c."""
    import ctypes
    V = lattice.volume(dims)
    shape = psi.shape
    psi = np.ascontiguousarray(psi, dtype=np.complex128).reshape(V, 12)
    U = np.ascontiguousarray(U, dtype=np.complex128)
    cl = None if clover is None else np.ascontiguousarray(clover, dtype=np.complex128)
    g = np.ascontiguousarray(lattice.gammas(), dtype=np.complex128)
    out = np.empty_like(psi)
    L = (ctypes.c_int * 4)(*dims)
    _clib().oracle_wilson_clover(L, U.ctypes.data, None if cl is None else cl.ctypes.data, float(m0),
                                 int(bool(antiperiodic_t)), g.ctypes.data, psi.ctypes.data, out.ctypes.data)
    return out.reshape(shape)


def apply_wilson_clover_csw_c(psi, U, csw, m0, dims, antiperiodic_t=True):
    """M psi with the clover term formed at each site from the links inside the
    plain C loop (csrc/wilson_clover.c): no stored clover field, so it serves
    as the true-residual check on lattices of millions of sites."""
    import ctypes
    V = lattice.volume(dims)
    shape = psi.shape
    psi = np.ascontiguousarray(psi, dtype=np.complex128).reshape(V, 12)
    U = np.ascontiguousarray(U, dtype=np.complex128)
    g = np.ascontiguousarray(lattice.gammas(), dtype=np.complex128)
    out = np.empty_like(psi)
    L = (ctypes.c_int * 4)(*dims)
    _clib().oracle_wilson_clover_csw(L, U.ctypes.data, float(csw), float(m0), int(bool(antiperiodic_t)),
                                     g.ctypes.data, psi.ctypes.data, out.ctypes.data)
    return out.reshape(shape)
