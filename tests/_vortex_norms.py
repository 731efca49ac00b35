"""L2(Omega_e) errors of a DG/compatible-FE state against the advected isodensity vortex of the
section "Advected MHD vortex" (numpy only: Lagrange interpolation of the stored nodal values to a
tensor Gauss rule of p+3 points per direction on every element inside Omega_e = [-5, 5]^2)."""
import math

import numpy as np

from paper_2609_10849_amd.workloads import gauss_nodes, gll_nodes


def lagrange_matrix(nodes, x):
    """M[k][i] = l_i(x_k) for the Lagrange basis on `nodes`."""
    M = np.ones((len(x), len(nodes)))
    for i, xi in enumerate(nodes):
        for j, xj in enumerate(nodes):
            if j != i:
                M[:, i] *= (x - xj) / (xi - xj)
    return M


def exact(x, y, t, gamma=5.0 / 3.0):
    """rho, u (3), p, B (3) of the vortex advected by (1, 1) on the periodic box [-10, 10]^2."""
    dx = (x - t) - 20.0 * np.round((x - t) / 20.0)
    dy = (y - t) - 20.0 * np.round((y - t) / 20.0)
    r2 = dx * dx + dy * dy
    g = np.exp(0.5 * (1.0 - r2))
    rho = np.ones_like(x)
    u = np.stack([1.0 - g * dy / (2 * math.pi), 1.0 + g * dx / (2 * math.pi), np.zeros_like(x)])
    p = 1.0 - r2 * g * g / (8.0 * math.pi ** 2)
    B = np.stack([-g * dy / (2 * math.pi), g * dx / (2 * math.pi), np.zeros_like(x)])
    return rho, u, p, B


def vortex_errors(L, U, Bx, By, Bz, t, box=5.0):
    p, m, gm = L.p, L.m, L.gamma
    zq, wq = np.polynomial.legendre.leggauss(p + 3)
    Ip = lagrange_matrix(gll_nodes(p), zq)
    Iw = lagrange_matrix(gll_nodes(m + 1), zq)
    Ig = lagrange_matrix(gauss_nodes(m), zq)
    Iv = lagrange_matrix(gll_nodes(m), zq)
    W2 = np.outer(wq, wq) * L.hx * L.hy / 4.0
    ex = np.arange(L.nx); ey = np.arange(L.ny)
    EX, EY = np.meshgrid(ex, ey, indexing="xy")
    EX = EX.ravel(); EY = EY.ravel()
    x0 = L.x0 + EX * L.hx; y0 = L.y0 + EY * L.hy
    inside = (x0 >= -box - 1e-12) & (x0 + L.hx <= box + 1e-12) & (y0 >= -box - 1e-12) & (y0 + L.hy <= box + 1e-12)
    idx = np.nonzero(inside)[0]
    X = x0[idx, None, None] + 0.5 * (zq[None, None, :] + 1.0) * L.hx
    Y = y0[idx, None, None] + 0.5 * (zq[None, :, None] + 1.0) * L.hy
    X = np.broadcast_to(X, (len(idx), len(zq), len(zq))); Y = np.broadcast_to(Y, X.shape)
    rho_e, u_e, p_e, B_e = exact(X, Y, t, gm)
    Ue = U[:, idx]  # [5][K'][j][i]
    rho_n = Ue[0]; u_n = Ue[1:4] / rho_n
    p_n = (gm - 1.0) * (Ue[4] - 0.5 * rho_n * (u_n ** 2).sum(0))
    at_q = lambda v: np.einsum("ki,eji,lj->elk", Ip, v, Ip)  # [e][qy][qx]
    err = {}
    err["rho"] = math.sqrt((W2 * (at_q(rho_n) - rho_e) ** 2).sum())
    err["u"] = math.sqrt(sum((W2 * (at_q(u_n[d]) - u_e[d]) ** 2).sum() for d in range(3)))
    err["p"] = math.sqrt((W2 * (at_q(p_n) - p_e) ** 2).sum())
    M1 = m + 1

    def patch(G, ni, nj):
        ny_t, nx_t = G.shape
        rows = (EY[idx, None] * M1 + np.arange(nj)[None, :]) % ny_t
        cols = (EX[idx, None] * M1 + np.arange(ni)[None, :]) % nx_t
        return G[rows[:, :, None], cols[:, None, :]]  # [e][j][i]

    bx = np.einsum("ki,eji,lj->elk", Iw, patch(Bx, m + 2, m + 1), Ig)
    by = np.einsum("ki,eji,lj->elk", Ig, patch(By, m + 1, m + 2), Iw)
    bz = np.einsum("ki,eji,lj->elk", Iv, patch(Bz, m + 1, m + 1), Iv)
    err["B"] = math.sqrt(sum((W2 * (b - B_e[d]) ** 2).sum() for d, b in enumerate((bx, by, bz))))
    return err


def exact_EJ(x, y, t):
    """E_z and J_z of the advected vortex: u = (1, 1, 0) + B, so E_z = -(u x B)_z = B_x - B_y =
    -g (dx + dy) / (2 pi), and J_z = d_x B_y - d_y B_x = g (2 - r^2) / (2 pi)."""
    dx = (x - t) - 20.0 * np.round((x - t) / 20.0)
    dy = (y - t) - 20.0 * np.round((y - t) / 20.0)
    r2 = dx * dx + dy * dy
    g = np.exp(0.5 * (1.0 - r2))
    return -g * (dx + dy) / (2 * math.pi), g * (2.0 - r2) / (2 * math.pi)


def EJ_errors(L, JE, t, box=5.0):
    """L2(Omega_e) errors of the reconstructed E_z and J_z (continuous GLL_{m+1} x GLL_{m+1} fields,
    grids 5 and 2 of JE = (J_x, J_y, J_z, E_x, E_y, E_z)) against the exact vortex fields, with the
    same per-element Gauss rule as vortex_errors."""
    p, m = L.p, L.m
    zq, wq = np.polynomial.legendre.leggauss(p + 3)
    Iw = lagrange_matrix(gll_nodes(m + 1), zq)
    W2 = np.outer(wq, wq) * L.hx * L.hy / 4.0
    EX, EY = np.meshgrid(np.arange(L.nx), np.arange(L.ny), indexing="xy")
    EX = EX.ravel(); EY = EY.ravel()
    x0 = L.x0 + EX * L.hx; y0 = L.y0 + EY * L.hy
    inside = (x0 >= -box - 1e-12) & (x0 + L.hx <= box + 1e-12) & (y0 >= -box - 1e-12) & (y0 + L.hy <= box + 1e-12)
    idx = np.nonzero(inside)[0]
    X = x0[idx, None, None] + 0.5 * (zq[None, None, :] + 1.0) * L.hx
    Y = y0[idx, None, None] + 0.5 * (zq[None, :, None] + 1.0) * L.hy
    X = np.broadcast_to(X, (len(idx), len(zq), len(zq))); Y = np.broadcast_to(Y, X.shape)
    Ez_e, Jz_e = exact_EJ(X, Y, t)
    M1 = m + 1

    def patch(G):
        ny_t, nx_t = G.shape
        rows = (EY[idx, None] * M1 + np.arange(m + 2)[None, :]) % ny_t
        cols = (EX[idx, None] * M1 + np.arange(m + 2)[None, :]) % nx_t
        return G[rows[:, :, None], cols[:, None, :]]

    at_q = lambda G: np.einsum("ki,eji,lj->elk", Iw, patch(G), Iw)
    return {"Ez": math.sqrt((W2 * (at_q(JE[5]) - Ez_e) ** 2).sum()),
            "Jz": math.sqrt((W2 * (at_q(JE[2]) - Jz_e) ** 2).sum())}
