"""Pins of the oracle's hydrodynamic operator L_E (eq. euler-nodal-index) and stage
machinery against what the paper and the mathematics fix: free-stream preservation,
global conservation and (EC interfaces) entropy conservation (theorem "Euler DGSEM
conservation and entropy stability"), consistency with -div F at the design order,
and third-order SSP-RK(3,3) (eq. euler-ssprk33)."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2609_10849_amd import workloads as W

G = 5.0 / 3.0


def mass_weights(M):
    x, w = O.gll(M.p)
    return M.hx * M.hy / 4.0 * np.outer(w, w)  # [j][i]


def entropy_vars(U):
    rho = U[0]; p = (G - 1) * (U[4] - (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / (2 * rho))
    s = np.log(p) - G * np.log(rho)
    b = rho / p
    u2 = (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / rho ** 2
    return np.stack([(G - s) / (G - 1) - 0.5 * b * u2, b * U[1] / rho, b * U[2] / rho, b * U[3] / rho, -b])


def mesh_of(L):
    return O.Mesh(L.nx, L.ny, L.p, L.m, L.x0, L.x1, L.y0, L.y1, L.gamma)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_free_stream(p):
    M = O.Mesh(5, 3, p, p - 1, 0.0, 1.0, -2.0, 0.5)
    sh = (M.K, p + 1, p + 1)
    U = W.conservative(np.full(sh, 1.7), np.full(sh, 0.3), np.full(sh, -0.8), np.full(sh, 0.45), np.full(sh, 2.2), G)
    dU = O.rhs_hydro(M, U)
    scale = np.abs(np.stack([O.phys_flux(U[:, 0, 0, 0], d, G) for d in (0, 1)])).max() * 2 / min(M.hx, M.hy) * p * p
    assert np.abs(dU).max() <= 1e-14 * scale


@pytest.mark.parametrize("flux", [0, 1])
@pytest.mark.parametrize("p", [2, 3, 4])
def test_conservation(p, flux):
    L, U, *_ = W.random_state(6, 5, p, p - 1, seed=p, domain=(0, 2, 0, 1), amp=0.2)
    M = mesh_of(L)
    dU = O.rhs_hydro(M, U, iface_flux=flux)
    Mw = mass_weights(M)
    for c in range(5):
        tot = (Mw * dU[c]).sum()
        scale = (Mw * np.abs(dU[c])).sum()
        assert abs(tot) <= 1e-13 * scale


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_entropy_conservation_with_ec_interfaces(p):
    L, U, *_ = W.random_state(5, 4, p, p - 1, seed=10 + p, domain=(0, 1, 0, 1), amp=0.3)
    M = mesh_of(L)
    dU = O.rhs_hydro(M, U, iface_flux=1)
    V = entropy_vars(U)
    Mw = mass_weights(M)
    prod = (Mw * (V * dU).sum(0)).sum()
    scale = (Mw * np.abs(V * dU).sum(0)).sum()
    assert abs(prod) <= 1e-12 * scale


@pytest.mark.parametrize("p", [2, 3, 4])
def test_entropy_dissipation_with_llf(p):
    L, U, *_ = W.random_state(5, 4, p, p - 1, seed=20 + p, domain=(0, 1, 0, 1), amp=0.3)
    M = mesh_of(L)
    V = entropy_vars(U)
    Mw = mass_weights(M)
    prod = (Mw * (V * O.rhs_hydro(M, U, iface_flux=0)).sum(0)).sum()
    prod_ec = (Mw * (V * O.rhs_hydro(M, U, iface_flux=1)).sum(0)).sum()
    assert prod < 0 and abs(prod_ec) < 1e-6 * abs(prod)


def smooth_state(X, Y):
    rho = 1.0 + 0.2 * np.sin(X) * np.cos(Y)
    ux = 0.5 + 0.1 * np.cos(X + Y); uy = -0.3 + 0.1 * np.sin(2 * Y - X); uz = 0.2 * np.cos(X)
    p = 1.0 + 0.1 * np.cos(X) * np.sin(Y)
    return rho, ux, uy, uz, p


def exact_div(X, Y):
    """-(d_x F_x + d_y F_y) of the smooth state by complex-step differentiation."""
    h = 1e-30

    def flux(Xc, Yc, d):
        rho, ux, uy, uz, p = smooth_state(Xc, Yc)
        E = p / (G - 1) + 0.5 * rho * (ux ** 2 + uy ** 2 + uz ** 2)
        ud = ux if d == 0 else uy
        return np.stack([rho * ud, rho * ux * ud + (p if d == 0 else 0), rho * uy * ud + (p if d == 1 else 0),
                         rho * uz * ud, (E + p) * ud])

    return -(flux(X + 1j * h, Y.astype(complex), 0).imag + flux(X.astype(complex), Y + 1j * h, 1).imag) / h


@pytest.mark.parametrize("p", [2, 3, 4])
def test_consistency_order(p):
    errs = []
    for n in (8, 16, 32):
        L = W.Layout(n, n, p, p - 1, 0, 2 * math.pi, 0, 2 * math.pi)
        X, Y = L.u_nodes()
        U = W.conservative(*smooth_state(X, Y), G)
        dU = O.rhs_hydro(mesh_of(L), U)
        errs.append(np.abs(dU - exact_div(X, Y)).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > p - 0.6, (errs, rates)


def test_ssprk3_order_no_stabilization():
    L = W.Layout(8, 8, 3, 2, 0, 2 * math.pi, 0, 2 * math.pi)
    X, Y = L.u_nodes()
    U0 = W.conservative(*smooth_state(X, Y), G)
    M = mesh_of(L); opts = O.Options()
    T = 0.2
    sols = []
    for n in (4, 8, 16):
        U = U0.copy()
        for _ in range(n):
            U, rep, *_ = O.hydro_substep(M, opts, U, T / n)
            assert rep["accepted"] == 1 and rep["attempted"] == 1
        sols.append(U)
    d1 = np.abs(sols[0] - sols[1]).max(); d2 = np.abs(sols[1] - sols[2]).max()
    assert 2.7 < math.log2(d1 / d2) < 3.3, (d1, d2)


def _dense_skew_rhs(nx, ny, p, hx, hy, U, iface_flux):
    """L_E assembled as dense global operators in the skew form M dU/dt = -[(S_x o F_x) 1 +
    (S_y o F_y) 1 + B-weighted interface fluxes], with S = Q - Q^T = 2Q - B from the SBP property of
    eq. euler-nodal-index's Q (Q + Q^T = B): the boundary corrections of eq. euler-nodal-index then
    leave only the numerical flux at the face nodes.  Tables from numpy's Legendre polynomials,
    matrices over all K (p+1)^2 nodes, fluxes from the oracle's (separately pinned) two-point and
    interface flux routines."""
    np1 = p + 1
    xi = W.gll_nodes(p)
    Pp = np.polynomial.legendre.Legendre.basis(p)(xi)
    w = 2.0 / (p * (p + 1) * Pp ** 2)
    bw = np.array([np.prod([xi[j] - xi[k] for k in range(np1) if k != j]) for j in range(np1)])
    D = np.zeros((np1, np1))
    for i in range(np1):
        for j in range(np1):
            if i != j:
                D[i, j] = (1.0 / bw[j]) / (1.0 / bw[i]) / (xi[i] - xi[j])
        D[i, i] = -D[i].sum()
    Q = np.diag(w) @ D
    S = Q - Q.T
    K = nx * ny
    N = K * np1 * np1
    node = lambda e, i, j: e * np1 * np1 + j * np1 + i
    Sx = np.zeros((N, N)); Sy = np.zeros((N, N)); Mg = np.zeros(N)
    for e in range(K):
        for j in range(np1):
            for i in range(np1):
                n = node(e, i, j)
                Mg[n] = hx * hy / 4 * w[i] * w[j]
                for r in range(np1):
                    Sx[n, node(e, r, j)] = S[i, r] * w[j] * hy / 2
                    Sy[n, node(e, i, r)] = w[i] * S[j, r] * hx / 2
    V = U.reshape(5, N).T
    R = np.zeros((N, 5))
    for n in range(N):
        for n2 in np.nonzero(Sx[n])[0]:
            R[n] += Sx[n, n2] * O.ec_flux(V[n], V[n2], 0, G)
        for n2 in np.nonzero(Sy[n])[0]:
            R[n] += Sy[n, n2] * O.ec_flux(V[n], V[n2], 1, G)
    fstar = (lambda a, b, d: O.ec_flux(a, b, d, G)) if iface_flux else (lambda a, b, d: O.llf_flux(a, b, d, G))
    for e in range(K):
        ex, ey = e % nx, e // nx
        right, top = ey * nx + (ex + 1) % nx, ((ey + 1) % ny) * nx + ex
        for k in range(np1):
            # x-face between e (node i = p) and its right neighbour (node i = 0): minus side is e
            a, b = node(e, p, k), node(right, 0, k)
            F = fstar(V[a], V[b], 0) * w[k] * hy / 2
            R[a] += F; R[b] -= F
            a, b = node(e, k, p), node(top, k, 0)
            F = fstar(V[a], V[b], 1) * w[k] * hx / 2
            R[a] += F; R[b] -= F
    return (-R / Mg[:, None]).T.reshape(U.shape)


@pytest.mark.parametrize("nx,ny,p,flux", [(2, 2, 2, 0), (3, 2, 3, 0), (3, 2, 2, 1), (2, 2, 3, 1)])
def test_dense_skew_form_equals_literal_sum(nx, ny, p, flux):
    """Brute force on tiny meshes: the oracle's literal double sum with the boundary corrections of
    eq. euler-nodal-index equals the dense skew-form assembly to rounding (hx != hy)."""
    L, U, *_ = W.random_state(nx, ny, p, p - 1, seed=40 + 3 * p + nx, domain=(0, 1.2, 0, 0.5), amp=0.3)
    M = mesh_of(L)
    ref = _dense_skew_rhs(nx, ny, p, M.hx, M.hy, U, flux)
    got = O.rhs_hydro(M, U, iface_flux=flux)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
