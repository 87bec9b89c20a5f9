"""Lattice geometry and spin matrices (oracle; test infrastructure only).

Conventions: a lattice of extents (L_1, ..., L_d) is stored as a numpy array
of shape (L_d, ..., L_1, ...), lexicographic with x_1 fastest.  Direction mu
(0-based) is coordinate x_{mu+1}; its numpy axis is d-1-mu.  Boundaries are
periodic in every direction (the paper states periodic boundaries for its
test lattices).
"""
from __future__ import annotations

import numpy as np

SIGMA = [
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
]


def gammas(nd: int) -> list[np.ndarray]:
    """Euclidean Hermitian gamma matrices gamma_mu, mu = 0..nd-1.

    2d: gamma_1 = sigma_1, gamma_2 = sigma_2 (so gamma_5 = sigma_3).
    4d: chiral basis gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] (k = 1..3)
        and gamma_4 = [[0, 1], [1, 0]], so gamma_5 = diag(1, 1, -1, -1).
    """
    if nd == 2:
        return [SIGMA[0], SIGMA[1]]
    if nd == 4:
        z = np.zeros((2, 2), dtype=np.complex128)
        e = np.eye(2, dtype=np.complex128)
        out = [np.block([[z, -1j * s], [1j * s, z]]) for s in SIGMA]
        out.append(np.block([[z, e], [e, z]]))
        return out
    raise ValueError("nd must be 2 or 4")


def gamma5(nd: int) -> np.ndarray:
    """gamma_5 built as a product of the gamma matrices.

    2d: -i gamma_1 gamma_2;  4d: gamma_1 gamma_2 gamma_3 gamma_4.
    """
    g = gammas(nd)
    if nd == 2:
        return -1j * g[0] @ g[1]
    return g[0] @ g[1] @ g[2] @ g[3]


def axis_of(mu: int, nd: int) -> int:
    return nd - 1 - mu


def shift(field: np.ndarray, mu: int, sign: int, nd: int) -> np.ndarray:
    """Return f(x + sign * mu_hat) for a field whose leading nd axes are the lattice."""
    return np.roll(field, -sign, axis=axis_of(mu, nd))


def site_coords(dims) -> np.ndarray:
    """Coordinates (V, nd) of every site in lexicographic order (x_1 fastest)."""
    nd = len(dims)
    grids = np.meshgrid(*[np.arange(L) for L in reversed(dims)], indexing="ij")
    # grids[k] is coordinate x_{nd-k}; flatten in C order = x_1 fastest
    return np.stack([grids[nd - 1 - mu].ravel() for mu in range(nd)], axis=1)


def site_index(coords: np.ndarray, dims) -> np.ndarray:
    """Lexicographic index of coordinates (..., nd), periodic."""
    idx = np.zeros(coords.shape[:-1], dtype=np.int64)
    stride = 1
    for mu, L in enumerate(dims):
        idx += (coords[..., mu] % L) * stride
        stride *= L
    return idx
