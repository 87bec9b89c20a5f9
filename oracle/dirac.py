"""Wilson-Dirac operator (oracle; test infrastructure only).

The operator is the one defined right after Eq. (1) of the paper:

  (D psi)(x) = (d + m) psi(x)
               - 1/2 sum_mu [ (1 - gamma_mu) U_mu(x) psi(x + mu)
                              + (1 + gamma_mu) U_mu(x - mu)^dagger psi(x - mu) ].

Reading of the diagonal term: the paper prints (2d + m) next to the 1/2
normalised hopping term.  With that normalisation the free operator has its
critical mass at m = -d, whereas the conventional Wilson operator with the
same hopping term has diagonal (d + m) and critical mass 0.  We use d + m;
every comparison in the paper is made in terms of the mass gap
m_hat = m - m_crit, which is unchanged (m_paper = m - d).

D^dagger is written out on its own (hopping projectors swapped), not as
gamma_5 D gamma_5, so that gamma_5-hermiticity is a real check.

Field layouts: psi[x_d, ..., x_1, spin, colour]; U[mu, x_d, ..., x_1, a, b].
For U(1) (two dimensions) n_c = 1 and U has trailing shape (1, 1).
"""
from __future__ import annotations

import numpy as np

from .lattice import gammas, shift, site_coords, site_index


def apply_D(U: np.ndarray, psi: np.ndarray, m: float, dagger: bool = False) -> np.ndarray:
    """D psi (or D^dagger psi) by the formula, FP64 complex."""
    nd = U.shape[0]
    ns = psi.shape[-2]
    g = gammas(nd)
    eye = np.eye(ns, dtype=np.complex128)
    out = (nd + m) * psi.astype(np.complex128)
    for mu in range(nd):
        fwd = np.einsum("...ab,...sb->...sa", U[mu], shift(psi, mu, +1, nd))
        U_xm = shift(U[mu], mu, -1, nd)                       # U_mu(x - mu)
        bwd = np.einsum("...ba,...sb->...sa", np.conj(U_xm), shift(psi, mu, -1, nd))
        p_fwd = eye + g[mu] if dagger else eye - g[mu]
        p_bwd = eye - g[mu] if dagger else eye + g[mu]
        out -= 0.5 * (np.einsum("st,...tc->...sc", p_fwd, fwd)
                      + np.einsum("st,...tc->...sc", p_bwd, bwd))
    return out


def dense_D(U: np.ndarray, m: float) -> np.ndarray:
    """The N x N matrix D_{x,y}, entry by entry from the definition.

    Row/column index i = site * (ns*nc) + spin * nc + colour with the site in
    lexicographic order (x_1 fastest).  Meant for lattices up to ~16^2.
    """
    nd = U.shape[0]
    dims = tuple(reversed(U.shape[1:1 + nd]))
    nc = U.shape[-1]
    ns = 2 if nd == 2 else 4
    g = gammas(nd)
    V = int(np.prod(dims))
    dof = ns * nc
    N = V * dof
    M = np.zeros((N, N), dtype=np.complex128)
    coords = site_coords(dims)
    Uflat = U.reshape(nd, V, nc, nc)
    for x in range(V):
        for s in range(ns):
            for a in range(nc):
                i = x * dof + s * nc + a
                M[i, i] += nd + m
        for mu in range(nd):
            e = np.zeros(nd, dtype=np.int64)
            e[mu] = 1
            y_f = int(site_index(coords[x] + e, dims))
            y_b = int(site_index(coords[x] - e, dims))
            for s in range(ns):
                for t in range(ns):
                    pm = (1.0 if s == t else 0.0) - g[mu][s, t]
                    pp = (1.0 if s == t else 0.0) + g[mu][s, t]
                    for a in range(nc):
                        for b in range(nc):
                            i = x * dof + s * nc + a
                            M[i, y_f * dof + t * nc + b] += -0.5 * pm * Uflat[mu, x, a, b]
                            M[i, y_b * dof + t * nc + b] += -0.5 * pp * np.conj(Uflat[mu, y_b, b, a])
    return M


def u1_field(theta: np.ndarray) -> np.ndarray:
    """Complex U(1) links with the colour axes attached: (2, L2, L1, 1, 1)."""
    return np.exp(1j * theta)[..., None, None]


def gauge_transform(U: np.ndarray, gx: np.ndarray) -> np.ndarray:
    """U_mu(x) -> g(x) U_mu(x) g(x + mu)^dagger for a site field g(x) of (nc, nc)."""
    nd = U.shape[0]
    out = np.empty_like(U)
    for mu in range(nd):
        g_xp = shift(gx, mu, +1, nd)
        out[mu] = gx @ U[mu] @ np.conj(np.swapaxes(g_xp, -1, -2))
    return out


def free_field_eigenvalues(dims, m: float, nc: int = 1) -> np.ndarray:
    """Closed-form spectrum of D at U = 1 (periodic): for each momentum
    p_mu = 2 pi n_mu / L_mu, lambda = m + sum_mu (1 - cos p_mu) +- i sqrt(sum_mu sin^2 p_mu),
    each with multiplicity nc (and twice that in four dimensions)."""
    nd = len(dims)
    ps = np.meshgrid(*[2 * np.pi * np.arange(L) / L for L in dims], indexing="ij")
    re = m + sum(1 - np.cos(p) for p in ps)
    im = np.sqrt(sum(np.sin(p) ** 2 for p in ps))
    mult = nc * (1 if nd == 2 else 2)
    ev = np.concatenate([(re + 1j * im).ravel(), (re - 1j * im).ravel()])
    return np.repeat(ev, mult)
