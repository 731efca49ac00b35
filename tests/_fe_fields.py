"""Evaluation of a stored state at points of every element (numpy only): the compatible B_h
from its grid coefficients (B_x: GLL_{m+1} x Gauss_m, B_y: Gauss_m x GLL_{m+1}, B_z: GLL_m x
GLL_m per element), used by the paper-scalar tests."""
import numpy as np

from paper_2609_10849_amd.workloads import gauss_nodes, gll_nodes
from tests._vortex_norms import lagrange_matrix


def element_origins(L):
    EX, EY = np.meshgrid(np.arange(L.nx), np.arange(L.ny), indexing="xy")
    return EX.ravel(), EY.ravel()


def B_at(L, Bx, By, Bz, z):
    """B_h at the tensor points z (reference coordinates, both directions) of every element:
    array [3][K][len(z)][len(z)], index [.., y point, x point]."""
    m = L.m; M1 = m + 1
    Iw = lagrange_matrix(gll_nodes(m + 1), z); Ig = lagrange_matrix(gauss_nodes(m), z)
    Iv = lagrange_matrix(gll_nodes(m), z)
    EX, EY = element_origins(L)

    def patch(G, ni, nj):
        ny_t, nx_t = G.shape
        rows = (EY[:, None] * M1 + np.arange(nj)[None, :]) % ny_t
        cols = (EX[:, None] * M1 + np.arange(ni)[None, :]) % nx_t
        return G[rows[:, :, None], cols[:, None, :]]

    bx = np.einsum("ki,eji,lj->elk", Iw, patch(Bx, m + 2, m + 1), Ig)
    by = np.einsum("ki,eji,lj->elk", Ig, patch(By, m + 1, m + 2), Iw)
    bz = np.einsum("ki,eji,lj->elk", Iv, patch(Bz, m + 1, m + 1), Iv)
    return np.stack([bx, by, bz])


def points(L, z):
    """Physical coordinates X, Y [K][len(z)][len(z)] of the tensor points z of every element."""
    EX, EY = element_origins(L)
    X = (L.x0 + EX * L.hx)[:, None, None] + 0.5 * (z[None, None, :] + 1.0) * L.hx
    Y = (L.y0 + EY * L.hy)[:, None, None] + 0.5 * (z[None, :, None] + 1.0) * L.hy
    return np.broadcast_to(X, (len(EX), len(z), len(z))), np.broadcast_to(Y, (len(EX), len(z), len(z)))


def primitives(L, U):
    """rho, u (3), p at the velocity nodes from the conservative nodal state."""
    rho = U[0]
    u = U[1:4] / rho
    p = (L.gamma - 1.0) * (U[4] - 0.5 * rho * (u ** 2).sum(0))
    return rho, u, p
