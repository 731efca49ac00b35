"""L2(Omega) errors of u, B, E, J against the exact reduced Alfven wave of the section "Reduced
Alfven-wave magnetic-stage convergence" (numpy only, vectorised over the elements): every field is
interpolated from its stored nodal values to a tensor Gauss rule of p+3 points per direction on
every element, as in the per-element evaluation of tests/test_oracle_magnetic.py, which a CPU test
checks it against."""
import math

import numpy as np

from paper_2609_10849_amd.workloads import gauss_nodes, gll_nodes
from tests._vortex_norms import lagrange_matrix


def exact_fields(x, y, t, eps=0.1):
    """B, u, E = -u x B and J = curl B of the wave travelling along (1, 1)/sqrt 2 with rho0 = B0 = 1:
    B = n + eps (t_vec cos th, sin th), u = -(B - n), th = x + y - sqrt 2 t."""
    th = x + y - math.sqrt(2.0) * t
    c, s = np.cos(th), np.sin(th)
    r = 1.0 / math.sqrt(2.0)
    B = np.stack([r - eps * r * c, r + eps * r * c, eps * s])
    u = np.stack([eps * r * c, -eps * r * c, -eps * s])
    E = -np.cross(u, B, axis=0)
    J = np.stack([eps * c, -eps * c, -eps * math.sqrt(2.0) * s])
    return B, u, E, J


def alfven_errors(L, u, Bx, By, Bz, JE, t, eps=0.1):
    """(e_u, e_B, e_E, e_J) for the state u [3][K][(p+1)^2], B grids and JE = (J_x, J_y, J_z, E_x, E_y,
    E_z) grids."""
    p, m = L.p, L.m
    NP, A, Bn = p + 1, m + 2, m + 1
    zq, wq = np.polynomial.legendre.leggauss(p + 3)
    Ip = lagrange_matrix(gll_nodes(p), zq)
    Iw = lagrange_matrix(gll_nodes(m + 1), zq)
    Ig = lagrange_matrix(gauss_nodes(m), zq)
    Iv = lagrange_matrix(gll_nodes(m), zq)
    W2 = np.outer(wq, wq) * L.hx * L.hy / 4.0
    EX, EY = np.meshgrid(np.arange(L.nx), np.arange(L.ny), indexing="xy")
    EX = EX.ravel(); EY = EY.ravel()
    K = len(EX)
    X = L.x0 + EX[:, None, None] * L.hx + 0.5 * (zq[None, None, :] + 1.0) * L.hx
    Y = L.y0 + EY[:, None, None] * L.hy + 0.5 * (zq[None, :, None] + 1.0) * L.hy
    X = np.broadcast_to(X, (K, len(zq), len(zq))); Y = np.broadcast_to(Y, X.shape)
    Be, ue, Ee, Je = exact_fields(X, Y, t, eps)
    M1 = m + 1

    def patch(G, ni, nj):
        ny_t, nx_t = G.shape
        rows = (EY[:, None] * M1 + np.arange(nj)[None, :]) % ny_t
        cols = (EX[:, None] * M1 + np.arange(ni)[None, :]) % nx_t
        return G[rows[:, :, None], cols[:, None, :]]  # [e][j][i]

    at_q = lambda Ix, v, Iy: np.einsum("ki,eji,lj->elk", Ix, v, Iy)  # [e][qy][qx]
    sq = lambda a, b: float((W2 * (a - b) ** 2).sum())
    un = np.asarray(u).reshape(3, K, NP, NP)
    e_u = sum(sq(at_q(Ip, un[d], Ip), ue[d]) for d in range(3))
    bh = (at_q(Iw, patch(Bx, A, Bn), Ig), at_q(Ig, patch(By, Bn, A), Iw), at_q(Iv, patch(Bz, Bn, Bn), Iv))
    e_B = sum(sq(bh[d], Be[d]) for d in range(3))
    # J and E: x component Gauss_m in x and GLL_{m+1} in y, y component the transpose, z on GLL_{m+1}^2
    rule = ((Ig, Bn, Iw, A), (Iw, A, Ig, Bn), (Iw, A, Iw, A))
    e_J = e_E = 0.0
    for c, (Ix, ni, Iy, nj) in enumerate(rule):
        e_J += sq(at_q(Ix, patch(JE[c], ni, nj), Iy), Je[c])
        e_E += sq(at_q(Ix, patch(JE[3 + c], ni, nj), Iy), Ee[c])
    return math.sqrt(e_u), math.sqrt(e_B), math.sqrt(e_E), math.sqrt(e_J)
