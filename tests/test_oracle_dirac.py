"""Pins of the oracle's fine operator (Eq. 2) and its inputs, against closed
forms and invariants that do not reuse the oracle's own formulas."""
import numpy as np
import pytest

import synth
from oracle import lattice, wilson
from oracle_helpers import (abelian_flux, free_spectrum, match_multisets, pure_gauge,
                            unit_gauge)


# both restatements of Eq. (2) in the oracle are held to the same pins
IMPLS = {'numpy': wilson.apply_wilson_clover, 'c': wilson.apply_wilson_clover_c}


@pytest.fixture(params=sorted(IMPLS))
def apply_M(request):
    return IMPLS[request.param]


def dense_M(U, clover, m0, dims, anti=True, apply=wilson.apply_wilson_clover):
    V = lattice.volume(dims)
    return wilson.dense_matrix(
        lambda v: apply(v.reshape(V, 4, 3), U, clover, m0, dims, anti).reshape(-1), V * 12)


def test_gauge_links_are_special_unitary():
    U = synth.gauge_field((4, 4, 4, 8), 0.4, 0).reshape(-1, 3, 3)
    uu = U @ np.conj(np.swapaxes(U, 1, 2))
    assert np.abs(uu - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14
    # the recipe is seeded: same seed, same field; other seed, other field
    assert np.array_equal(synth.gauge_field((2, 2, 2, 2), 0.4, 0), synth.gauge_field((2, 2, 2, 2), 0.4, 0))
    assert not np.allclose(synth.gauge_field((2, 2, 2, 2), 0.4, 0), synth.gauge_field((2, 2, 2, 2), 0.4, 1))


def test_special_unitary_rows_are_conjugate_cross_products():
    """The property 12-real link compression rests on: for U in SU(3) each row
    is the complex conjugate of the cross product of the other two (from
    U^+ U = 1 and det U = 1); it holds to rounding for the synthetic links and
    fails for a unitary matrix with det = -1 (the time-boundary sign)."""
    U = synth.gauge_field((4, 4, 2, 2), 0.4, 7).reshape(-1, 3, 3)
    c = np.conj(np.cross(U[:, 0], U[:, 1]))
    assert np.abs(c - U[:, 2]).max() < 1e-14
    assert np.abs(np.conj(np.cross(U[:, 1], U[:, 2])) - U[:, 0]).max() < 1e-14
    W = -U   # det = -1
    assert np.abs(np.conj(np.cross(W[:, 0], W[:, 1])) + W[:, 2]).max() < 1e-14


def test_gamma_clifford_algebra_and_chiral_basis():
    g = lattice.gammas()
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)
        for nu in range(4):
            assert np.allclose(g[mu] @ g[nu] + g[nu] @ g[mu], 2 * (mu == nu) * np.eye(4))
    assert np.allclose(lattice.gamma5(), np.diag([1, 1, -1, -1]))
    Pm, Pp = lattice.projectors()
    for mu in range(4):  # (1 -/+ gamma)/2 are complementary projectors
        assert np.allclose((Pm[mu] / 2) @ (Pm[mu] / 2), Pm[mu] / 2)
        assert np.allclose(Pm[mu] + Pp[mu], 2 * np.eye(4))


@pytest.mark.parametrize("anti", [True, False])
def test_free_field_spectrum_closed_form(anti, apply_M):
    """U = 1: eigenvalues m0 + sum(1 - cos p) +/- i sqrt(sum sin^2 p), 6-fold."""
    dims = (4, 2, 2, 4)
    m0 = -0.2
    ev = np.linalg.eigvals(dense_M(unit_gauge(dims), None, m0, dims, anti, apply_M))
    assert match_multisets(ev, free_spectrum(dims, m0, anti)) < 1e-12


def test_pure_gauge_spectrum_and_vanishing_clover(apply_M):
    """U_mu(x) = g(x) g(x+mu)^+ is a gauge copy of U = 1: same spectrum, zero clover."""
    dims = (4, 2, 2, 4)
    U = pure_gauge(dims, 7)
    A = wilson.clover_field(U, dims, 1.0)
    assert np.abs(A).max() < 1e-14
    ev = np.linalg.eigvals(dense_M(U, A, -0.2, dims, True, apply_M))
    assert match_multisets(ev, free_spectrum(dims, -0.2)) < 1e-12


def test_gamma5_hermiticity_random_links(apply_M):
    """gamma5 M gamma5 = M^+, checked through <phi, g5 M g5 psi> = <M phi, psi>."""
    dims = (4, 4, 4, 4)
    V = lattice.volume(dims)
    U = synth.gauge_field(dims, 0.4, 3)
    A = wilson.clover_field(U, dims, 1.0)
    g5 = np.kron(lattice.gamma5(), np.eye(3))
    phi = synth.gaussian((V, 12), 1, 2)
    psi = synth.gaussian((V, 12), 2, 2)
    M = lambda v: apply_M(v, U, A, -0.2, dims)
    lhs = np.vdot(phi, M(psi @ g5.T) @ g5.T)
    rhs = np.vdot(M(phi), psi)
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)
    # M itself is not Hermitian, so this is not a trivial identity
    assert abs(np.vdot(phi, M(psi)) - np.vdot(M(phi), psi)) > 1e-3 * abs(rhs)


def test_clover_structure():
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.4, 0)
    A = wilson.clover_field(U, dims, 1.0)
    assert np.abs(A - np.conj(np.swapaxes(A, 1, 2))).max() < 1e-14          # Hermitian
    assert np.abs(A[:, :6, 6:]).max() < 1e-15                                 # chirality blocks
    assert np.abs(np.trace(A, axis1=1, axis2=2)).max() < 1e-13                # traceless
    assert np.abs(A).max() > 1e-2
    assert np.abs(wilson.clover_field(unit_gauge(dims), dims, 1.0)).max() == 0.0


@pytest.mark.parametrize("n", [1, 3])
def test_clover_constant_abelian_flux_closed_form(n):
    """Every 0-1 plaquette = exp(i q theta): A = -(c_sw/2) sigma_01 (x) diag(sin q theta)."""
    dims = (4, 4, 2, 2)
    U, theta, q = abelian_flux(dims, n)
    for csw in (1.0, 1.7):
        A = wilson.clover_field(U, dims, csw)
        expect = -(csw / 2) * np.kron(lattice.sigma(0, 1), np.diag(np.sin(q * theta)))
        assert np.abs(A - expect[None]).max() < 1e-14


def test_gauge_covariance_of_M(apply_M):
    """M[gU](g psi) = g M[U](psi) for a random local rotation g."""
    from oracle_helpers import gauge_rotate
    dims = (4, 4, 2, 4)
    V = lattice.volume(dims)
    U = synth.gauge_field(dims, 0.4, 1)
    g = synth.gauge_rotation(dims, 2)
    Ug = gauge_rotate(U, g, dims)
    psi = synth.gaussian((V, 4, 3), 3, 2)
    rot = lambda p: np.einsum('xab,xsb->xsa', g, p)
    a = apply_M(rot(psi), Ug, wilson.clover_field(Ug, dims, 1.0), -0.3, dims)
    b = rot(apply_M(psi, U, wilson.clover_field(U, dims, 1.0), -0.3, dims))
    assert np.abs(a - b).max() < 1e-13


def test_clover_enters_the_operator_through_A(apply_M):
    """M with clover minus M without clover is exactly A(x) psi(x) (site-local)."""
    dims = (4, 2, 4, 2)
    V = lattice.volume(dims)
    U = synth.gauge_field(dims, 0.5, 9)
    A = wilson.clover_field(U, dims, 1.3)
    psi = synth.gaussian((V, 4, 3), 4, 2)
    d = apply_M(psi, U, A, 0.1, dims) - apply_M(psi, U, None, 0.1, dims)
    assert np.abs(d.reshape(V, 12) - np.einsum('xij,xj->xi', A, psi.reshape(V, 12))).max() < 1e-14


def test_sampled_sites_agree_with_whole_field():
    """The site-restricted forms (clover term and M at chosen sites) give the
    rows of the whole-field results."""
    dims = (4, 2, 6, 4)
    U = synth.gauge_field(dims, 0.5, 7)
    V = lattice.volume(dims)
    psi = synth.gaussian((V, 4, 3), 7, 2)
    A = wilson.clover_field(U, dims, 1.3)
    full = wilson.apply_wilson_clover(psi, U, A, -0.1, dims)
    sites = np.array([0, 5, 17, V - 1, 40, 41])
    assert np.allclose(wilson.clover_field(U, dims, 1.3, sites), A[sites], rtol=0, atol=1e-14)
    part = wilson.apply_wilson_clover_sites(psi, U, 1.3, -0.1, dims, sites)
    assert np.allclose(part, full[sites], rtol=0, atol=1e-13)


# ---- the C loop that forms the clover term from the links at each site ----

def test_csw_c_constant_abelian_flux_closed_form():
    """M(c_sw) - M(0) = -(c_sw/2) sigma_01 (x) diag(sin q theta) on every site
    for the constant abelian flux, from the links alone."""
    dims = (4, 4, 2, 2)
    V = lattice.volume(dims)
    psi = synth.gaussian((V, 4, 3), 5, 2)
    for n in (1, 3):
        U, theta, q = abelian_flux(dims, n)
        for csw in (1.0, 1.7):
            d = (wilson.apply_wilson_clover_csw_c(psi, U, csw, -0.1, dims)
                 - wilson.apply_wilson_clover_csw_c(psi, U, 0.0, -0.1, dims))
            A = -(csw / 2) * np.kron(lattice.sigma(0, 1), np.diag(np.sin(q * theta)))
            assert np.abs(d.reshape(V, 12) - psi.reshape(V, 12) @ A.T).max() < 1e-14


def test_csw_c_pure_gauge_spectrum_and_gamma5_hermiticity():
    dims = (4, 2, 2, 4)
    V = lattice.volume(dims)
    U = pure_gauge(dims, 7)
    M = lambda v: wilson.apply_wilson_clover_csw_c(v.reshape(V, 4, 3), U, 1.0, -0.2, dims).reshape(-1)
    ev = np.linalg.eigvals(wilson.dense_matrix(M, V * 12))
    assert match_multisets(ev, free_spectrum(dims, -0.2)) < 1e-12
    dims = (4, 4, 4, 4)
    V = lattice.volume(dims)
    U = synth.gauge_field(dims, 0.4, 3)
    g5 = np.kron(lattice.gamma5(), np.eye(3))
    phi, psi = synth.gaussian((V, 12), 1, 2), synth.gaussian((V, 12), 2, 2)
    M = lambda v: wilson.apply_wilson_clover_csw_c(v, U, 1.0, -0.2, dims)
    lhs = np.vdot(phi, M(psi @ g5.T) @ g5.T)
    rhs = np.vdot(M(phi), psi)
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)


def test_csw_c_gauge_covariance_and_agreement_with_stored_clover():
    from oracle_helpers import gauge_rotate
    dims = (4, 4, 2, 4)
    V = lattice.volume(dims)
    U = synth.gauge_field(dims, 0.4, 1)
    g = synth.gauge_rotation(dims, 2)
    Ug = gauge_rotate(U, g, dims)
    psi = synth.gaussian((V, 4, 3), 3, 2)
    rot = lambda p: np.einsum('xab,xsb->xsa', g, p)
    a = wilson.apply_wilson_clover_csw_c(rot(psi), Ug, 1.0, -0.3, dims)
    b = rot(wilson.apply_wilson_clover_csw_c(psi, U, 1.0, -0.3, dims))
    assert np.abs(a - b).max() < 1e-13
    for dims, csw, m0 in (((4, 4, 2, 6), 1.0, -0.2), ((2, 4, 3, 4), 0.7, 0.1)):
        U = synth.gauge_field(dims, 0.4, 3)
        V = lattice.volume(dims)
        psi = synth.gaussian((V, 4, 3), 1, 2)
        ref = wilson.apply_wilson_clover(psi, U, wilson.clover_field(U, dims, csw), m0, dims)
        assert np.abs(wilson.apply_wilson_clover_csw_c(psi, U, csw, m0, dims) - ref).max() < 1e-13
