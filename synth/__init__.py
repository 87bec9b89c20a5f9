"""Seeded synthetic inputs shared by the GPU path and the CPU oracle.

This module draws the random inputs of the adaptive multigrid solve and nothing
else: gauge configurations, sources and the random starting vectors that the
adaptive setup relaxes.  It holds none of the solver's arithmetic (no Dirac
operator, no transfer operator, no Krylov step), so both sides can import it
without sharing any of the method.

Layouts (canonical, array-of-structures, lexicographic with x1 fastest):

* a 2d lattice of extent L1 x L2 is a numpy array of shape ``(L2, L1, ...)``;
* U(1) links are angles ``theta[mu, x2, x1]`` with ``U_mu(x) = exp(i theta)``;
  ``mu = 0`` is the x1 direction;
* a 4d lattice ``L1 x L2 x L3 x L4`` is ``(L4, L3, L2, L1, ...)``; SU(3) links
  are ``U[mu, x4, x3, x2, x1, a, b]``;
* fermion fields are ``psi[x..., spin, colour]`` complex.

Gauge ensembles follow the paper's numerical test: quenched U(1) in two
dimensions with the Wilson plaquette action at coupling beta and periodic
boundaries, updated by heat-bath (the paper's test section).  The Boltzmann
weight is ``exp(+beta * sum_P Re U_P)``, which favours ordered plaquettes.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng_for", "u1_cold", "u1_heatbath", "u1_links", "u1_plaquette_angles",
    "u1_mean_plaquette", "u1_topological_charge", "gaussian_field",
    "point_source", "random_vectors", "su3_haar", "su3_stout_smear",
    "su3_mean_plaquette", "tile_u1",
]


def rng_for(*seq: int) -> np.random.Generator:
    """A numpy Generator seeded by an integer sequence (e.g. cfg, beta, L1, L2, idx)."""
    return np.random.default_rng([int(s) for s in seq])


# ----------------------------------------------------------------------------
# U(1) gauge field in two dimensions
# ----------------------------------------------------------------------------

def u1_cold(L1: int, L2: int) -> np.ndarray:
    """Cold start: all link angles zero, shape (2, L2, L1)."""
    return np.zeros((2, L2, L1), dtype=np.float64)


def _staple_sum(theta: np.ndarray, mu: int) -> np.ndarray:
    """Sum of the two staples attached to every mu-link, as a complex number.

    For the link U_mu(x) the action terms containing it are
    Re(U_mu(x) * S(x)) with
    S = U_nu(x+mu) U_mu(x+nu)^* U_nu(x)^* + U_nu(x+mu-nu)^* U_mu(x-nu)^* U_nu(x-nu).
    """
    nu = 1 - mu
    ax_mu = 1 - mu          # numpy axis of direction mu (x1 is the last axis)
    ax_nu = 1 - nu
    t_mu, t_nu = theta[mu], theta[nu]
    up = (np.roll(t_nu, -1, axis=ax_mu) - np.roll(t_mu, -1, axis=ax_nu) - t_nu)
    t_nu_xm = np.roll(t_nu, 1, axis=ax_nu)                       # U_nu(x-nu)
    t_nu_xpm = np.roll(np.roll(t_nu, -1, axis=ax_mu), 1, axis=ax_nu)  # U_nu(x+mu-nu)
    t_mu_xm = np.roll(t_mu, 1, axis=ax_nu)                       # U_mu(x-nu)
    down = (-t_nu_xpm - t_mu_xm + t_nu_xm)
    return np.exp(1j * up) + np.exp(1j * down)


def u1_flux(L1: int, L2: int, Q: int) -> np.ndarray:
    """Link angles (2, L2, L1) of a constant magnetic flux 2 pi Q / (L1 L2)
    through every plaquette: theta_1 = -2 pi Q x2 / (L1 L2) everywhere, and
    on the last row x2 = L2 - 1 theta_2 = 2 pi Q x1 / L1 closes the flux
    around the torus.  Total charge Q (a start in the sector Q)."""
    x2, x1 = np.meshgrid(np.arange(L2), np.arange(L1), indexing="ij")
    th = np.zeros((2, L2, L1))
    th[0] = -2.0 * np.pi * Q * x2 / (L1 * L2)
    th[1][L2 - 1] = 2.0 * np.pi * Q * np.arange(L1) / L1
    return np.angle(np.exp(1j * th))


def u1_heatbath(L1: int, L2: int, beta: float, sweeps: int,
                rng: np.random.Generator, theta: np.ndarray | None = None) -> np.ndarray:
    """Quenched U(1) heat-bath with the Wilson plaquette action (paper's test section).

    One sweep visits (mu, parity of x1+x2) in order mu = 0, 1 and parity 0, 1.
    Same-parity mu-links share no plaquette, so they are drawn together from
    their exact conditional distribution: with staple sum S = |S| e^{i phi},
    the weight exp(beta |S| cos(theta + phi)) is a von Mises law with mean
    -phi and concentration beta |S|.  Requires even L1 and L2.
    Returns link angles of shape (2, L2, L1) wrapped to (-pi, pi].
    """
    if L1 % 2 or L2 % 2:
        raise ValueError("checkerboard heat-bath needs even extents")
    th = u1_cold(L1, L2) if theta is None else theta.copy()
    x2, x1 = np.meshgrid(np.arange(L2), np.arange(L1), indexing="ij")
    parity = (x1 + x2) % 2
    masks = [parity == 0, parity == 1]
    for _ in range(sweeps):
        for mu in (0, 1):
            for par in (0, 1):
                S = _staple_sum(th, mu)
                m = masks[par]
                kappa = beta * np.abs(S[m])
                mean = -np.angle(S[m])
                th[mu][m] = rng.vonmises(mean, kappa)
    return np.angle(np.exp(1j * th))


def u1_field_of(entry: dict) -> np.ndarray:
    """Link angles of a 2d workload-table entry: the seeded heat-bath from its
    start (cold, or the constant flux of charge start_flux_Q)."""
    L1, L2 = entry["L1"], entry["L2"]
    q = entry.get("start_flux_Q", 0)
    return u1_heatbath(L1, L2, entry["beta"], entry["sweeps"], rng_for(*entry["seed"]),
                       u1_flux(L1, L2, q) if q else None)


def u1_links(theta: np.ndarray) -> np.ndarray:
    """Complex links U = exp(i theta), canonical layout [mu][x2][x1] (n_c = 1)."""
    return np.exp(1j * theta)


def u1_plaquette_angles(theta: np.ndarray) -> np.ndarray:
    """Plaquette angle theta_1(x) + theta_2(x+1) - theta_1(x+2) - theta_2(x), shape (L2, L1)."""
    t1, t2 = theta[0], theta[1]
    return t1 + np.roll(t2, -1, axis=1) - np.roll(t1, -1, axis=0) - t2


def u1_mean_plaquette(theta: np.ndarray) -> float:
    """<Re U_P> averaged over all plaquettes."""
    return float(np.mean(np.cos(u1_plaquette_angles(theta))))


def u1_topological_charge(theta: np.ndarray) -> float:
    """Q = (1/2pi) sum_x arg U_P(x) with arg in (-pi, pi]; an integer on a torus."""
    a = np.angle(np.exp(1j * u1_plaquette_angles(theta)))
    return float(np.sum(a) / (2.0 * np.pi))


def tile_u1(theta: np.ndarray, n1: int, n2: int) -> np.ndarray:
    """Periodic tiling of a U(1) configuration to (n2*L2, n1*L1); still a valid periodic field."""
    return np.tile(theta, (1, n2, n1))


# ----------------------------------------------------------------------------
# Fermion-side random inputs
# ----------------------------------------------------------------------------

def gaussian_field(shape, rng: np.random.Generator) -> np.ndarray:
    """Complex Gaussian field (g0 + i g1)/sqrt(2) with g = rng.standard_normal((2,) + shape)."""
    g = rng.standard_normal((2,) + tuple(shape))
    return (g[0] + 1j * g[1]) / np.sqrt(2.0)


def point_source(lat_shape, ns: int, nc: int, spin: int, colour: int,
                 site=None) -> np.ndarray:
    """Unit point source at `site` (default the origin) in spin/colour component."""
    out = np.zeros(tuple(lat_shape) + (ns, nc), dtype=np.complex128)
    idx = (0,) * len(lat_shape) if site is None else tuple(site)
    out[idx + (spin, colour)] = 1.0
    return out


def random_vectors(n: int, lat_shape, ns: int, nc: int,
                   rng: np.random.Generator) -> np.ndarray:
    """n complex Gaussian fields, shape (n,) + lat_shape + (ns, nc): the random
    starting vectors of the adaptive setup."""
    return gaussian_field((n,) + tuple(lat_shape) + (ns, nc), rng)


# ----------------------------------------------------------------------------
# SU(3) gauge field in four dimensions
# ----------------------------------------------------------------------------

def su3_haar(shape, rng: np.random.Generator) -> np.ndarray:
    """Haar-random SU(3) matrices of the given batch shape (+ (3, 3)).

    QR of a complex Ginibre matrix with the diagonal phases of R moved into Q
    (Mezzadri's construction) gives Haar U(3); dividing by a cube root of the
    determinant lands in SU(3) up to a centre element, which leaves Haar
    measure invariant.
    """
    z = gaussian_field(tuple(shape) + (3, 3), rng)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    ph = d / np.abs(d)
    q = q * ph[..., None, :]
    det = np.linalg.det(q)
    return q / (det ** (1.0 / 3.0))[..., None, None]


def _dagger(m: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(m, -1, -2))


def _su3_staples(U: np.ndarray, mu: int) -> np.ndarray:
    """Sum over nu != mu of the forward and backward staples of U_mu(x)."""
    nd = U.shape[0]
    ax = lambda m: nd - 1 - m  # noqa: E731  numpy axis (0-based within the lattice dims)
    S = np.zeros_like(U[mu])
    for nu in range(nd):
        if nu == mu:
            continue
        Unu_xpmu = np.roll(U[nu], -1, axis=ax(mu))
        Umu_xpnu = np.roll(U[mu], -1, axis=ax(nu))
        S += U[nu] @ Umu_xpnu @ _dagger(Unu_xpmu)
        Unu_xmnu = np.roll(U[nu], 1, axis=ax(nu))
        Umu_xmnu = np.roll(U[mu], 1, axis=ax(nu))
        Unu_xpmu_mnu = np.roll(Unu_xpmu, 1, axis=ax(nu))
        S += _dagger(Unu_xmnu) @ Umu_xmnu @ Unu_xpmu_mnu
    return S


def _expi_hermitian(Q: np.ndarray) -> np.ndarray:
    """exp(iQ) for Hermitian Q via a batched eigendecomposition."""
    w, v = np.linalg.eigh(Q)
    return (v * np.exp(1j * w)[..., None, :]) @ _dagger(v)


def su3_stout_smear(U: np.ndarray, rho: float, steps: int) -> np.ndarray:
    """Simultaneous stout smearing: U' = exp(iQ) U with
    Omega = rho * C U^dagger (C the staple sum), Q = (i/2)(Omega^dag - Omega)
    - (i/6) tr(Omega^dag - Omega).  Input and output shape (nd, lat..., 3, 3)."""
    U = U.copy()
    nd = U.shape[0]
    eye = np.eye(3)
    for _ in range(steps):
        new = np.empty_like(U)
        for mu in range(nd):
            om = rho * _su3_staples(U, mu) @ _dagger(U[mu])
            a = _dagger(om) - om
            tr = np.trace(a, axis1=-2, axis2=-1)[..., None, None]
            Q = 0.5j * a - (1j / 6.0) * tr * eye
            Q = 0.5 * (Q + _dagger(Q))
            new[mu] = _expi_hermitian(Q) @ U[mu]
        U = new
    return U


def su3_mean_plaquette(U: np.ndarray) -> float:
    """<(1/3) Re tr U_P> over all sites and planes."""
    nd = U.shape[0]
    ax = lambda m: nd - 1 - m  # noqa: E731
    tot, cnt = 0.0, 0
    for mu in range(nd):
        for nu in range(mu + 1, nd):
            P = (U[mu] @ np.roll(U[nu], -1, axis=ax(mu))
                 @ _dagger(np.roll(U[mu], -1, axis=ax(nu))) @ _dagger(U[nu]))
            tot += float(np.mean(np.real(np.trace(P, axis1=-2, axis2=-1)))) / 3.0
            cnt += 1
    return tot / cnt
