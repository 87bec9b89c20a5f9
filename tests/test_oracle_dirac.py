"""Pins of the oracle's Wilson-Dirac operator to facts that do not come from the oracle.

* the closed-form free-field spectrum (momentum space, U = 1);
* gamma_5-hermiticity D^dagger = gamma_5 D gamma_5, with D^dagger coded separately;
* gauge covariance D[U^g](g psi) = g D[U] psi;
* the stencil against a dense matrix built entry by entry;
* the exact mass shift of the spectrum;
* the Clifford algebra of the gamma matrices.
"""
import numpy as np
import pytest

import synth
from oracle import dirac, lattice, mg


def _sorted(ev, nd=10):
    ev = np.round(ev, nd)
    return ev[np.lexsort((ev.imag, ev.real))]


def _u1(L1, L2, beta=3.0, sweeps=20, seed=0):
    th = synth.u1_heatbath(L1, L2, beta, sweeps, synth.rng_for(99, seed, L1, L2))
    return dirac.u1_field(th)


def _su3(dims, seed=0):
    shape = (4,) + tuple(reversed(dims))
    return synth.su3_haar(shape, synth.rng_for(98, seed, *dims))


@pytest.mark.parametrize("nd", [2, 4])
def test_clifford_algebra_and_gamma5(nd):
    g = lattice.gammas(nd)
    ns = g[0].shape[0]
    for a in range(nd):
        assert np.allclose(g[a], g[a].conj().T)
        for b in range(nd):
            assert np.allclose(g[a] @ g[b] + g[b] @ g[a], 2 * (a == b) * np.eye(ns))
    g5 = lattice.gamma5(nd)
    assert np.allclose(g5, np.diag(np.concatenate([np.ones(ns // 2), -np.ones(ns // 2)])))
    for a in range(nd):
        assert np.allclose(g5 @ g[a] + g[a] @ g5, 0)


@pytest.mark.parametrize("dims,m", [((8, 8), 0.3), ((6, 4), -0.2), ((4, 4), 0.0)])
def test_free_field_spectrum_2d(dims, m):
    U = np.ones((2, dims[1], dims[0], 1, 1), dtype=np.complex128)
    ev = np.linalg.eigvals(dirac.dense_D(U, m))
    ref = dirac.free_field_eigenvalues(dims, m, nc=1)
    assert np.abs(_sorted(ev) - _sorted(ref)).max() < 1e-9


def test_free_field_spectrum_4d():
    dims = (2, 2, 2, 4)
    U = np.broadcast_to(np.eye(3, dtype=np.complex128), (4,) + tuple(reversed(dims)) + (3, 3)).copy()
    ev = np.linalg.eigvals(dirac.dense_D(U, 0.1))
    ref = dirac.free_field_eigenvalues(dims, 0.1, nc=3)
    assert np.abs(_sorted(ev, 8) - _sorted(ref, 8)).max() < 1e-7


@pytest.mark.parametrize("L", [4, 8])
def test_stencil_matches_dense_matrix_2d(L):
    U = _u1(L, L)
    psi = synth.gaussian_field((L, L, 2, 1), synth.rng_for(5, L))
    M = dirac.dense_D(U, 0.17)
    for dag in (False, True):
        ref = (M.conj().T if dag else M) @ psi.ravel()
        out = dirac.apply_D(U, psi, 0.17, dagger=dag).ravel()
        assert np.abs(out - ref).max() < 1e-13


def test_stencil_matches_dense_matrix_4d():
    dims = (2, 2, 2, 2)
    U = _su3(dims)
    psi = synth.gaussian_field(tuple(reversed(dims)) + (4, 3), synth.rng_for(6))
    M = dirac.dense_D(U, -0.3)
    for dag in (False, True):
        ref = (M.conj().T if dag else M) @ psi.ravel()
        out = dirac.apply_D(U, psi, -0.3, dagger=dag).ravel()
        assert np.abs(out - ref).max() < 1e-12


@pytest.mark.parametrize("nd", [2, 4])
def test_gamma5_hermiticity(nd):
    if nd == 2:
        U = _u1(8, 6)
        shape = (6, 8, 2, 1)
    else:
        U = _su3((4, 2, 2, 4))
        shape = (4, 2, 2, 4, 4, 3)
    psi = synth.gaussian_field(shape, synth.rng_for(7, nd))
    g5 = lattice.gamma5(nd)
    g5psi = np.einsum("st,...tc->...sc", g5, psi)
    lhs = dirac.apply_D(U, psi, 0.05, dagger=True)
    rhs = np.einsum("st,...tc->...sc", g5, dirac.apply_D(U, g5psi, 0.05))
    assert np.abs(lhs - rhs).max() < 1e-13
    # adjointness <phi, D psi> = <D^dag phi, psi>
    phi = synth.gaussian_field(shape, synth.rng_for(8, nd))
    a = np.vdot(phi, dirac.apply_D(U, psi, 0.05))
    b = np.vdot(dirac.apply_D(U, phi, 0.05, dagger=True), psi)
    assert abs(a - b) < 1e-11 * abs(a)


@pytest.mark.parametrize("nd", [2, 4])
def test_gauge_covariance(nd):
    if nd == 2:
        U = _u1(8, 8)
        lat = (8, 8)
        g = np.exp(1j * synth.rng_for(11).uniform(-np.pi, np.pi, lat))[..., None, None]
        shape = lat + (2, 1)
    else:
        U = _su3((2, 4, 2, 4))
        lat = (4, 2, 4, 2)
        g = synth.su3_haar(lat, synth.rng_for(12))
        shape = lat + (4, 3)
    psi = synth.gaussian_field(shape, synth.rng_for(13, nd))
    Ug = dirac.gauge_transform(U, g)
    gpsi = np.einsum("...ab,...sb->...sa", g, psi)
    lhs = dirac.apply_D(Ug, gpsi, 0.2)
    rhs = np.einsum("...ab,...sb->...sa", g, dirac.apply_D(U, psi, 0.2))
    assert np.abs(lhs - rhs).max() < 1e-13


def test_mass_shift_of_spectrum():
    U = _u1(6, 6, beta=6.0)
    e0 = np.linalg.eigvals(dirac.dense_D(U, 0.0))
    e1 = np.linalg.eigvals(dirac.dense_D(U, 0.37))
    assert np.abs(_sorted(e0 + 0.37, 8) - _sorted(e1, 8)).max() < 1e-7


@pytest.mark.parametrize("nd", [2, 4])
def test_wilson_stencil_object_matches_formula(nd):
    if nd == 2:
        U = _u1(8, 4)
        shape = (4, 8, 2, 1)
    else:
        U = _su3((2, 2, 4, 2))
        shape = (2, 4, 2, 2, 4, 3)
    psi = synth.gaussian_field(shape, synth.rng_for(21, nd))
    S = mg.wilson_stencil(U, 0.11)
    V = int(np.prod(shape[:nd]))
    f = psi.reshape(V, -1)
    assert np.abs(S.apply(f) - dirac.apply_D(U, psi, 0.11).reshape(V, -1)).max() < 1e-13
    assert np.abs(S.apply_dagger(f) - dirac.apply_D(U, psi, 0.11, True).reshape(V, -1)).max() < 1e-13
    assert np.abs(S.to_sparse() @ f.ravel() - dirac.apply_D(U, psi, 0.11).ravel()).max() < 1e-13
