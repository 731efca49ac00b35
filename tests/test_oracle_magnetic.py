"""Pins of the oracle's magnetic-velocity operator L_M (eq. magnetic-dae) and its
stabilisation: the semidiscrete power identity (theorem "Semidiscrete magnetic-step
energy balance") with the exact magnetic product evaluated independently, divergence
of the curl increment (theorem "Preservation of the in-plane divergence-free
constraint"), closed-form special cases, velocity-OE identities (proposition
"Magnetic velocity-OE map"), a hand-computed artificial-resistivity coefficient
(eq. magnetic-ar-coefficient), and Alfven-wave magnetic-stage accuracy against the
paper's table of the reduced Alfven wave."""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2609_10849_amd import workloads as W
from tests._poly import B_product, Fields, div_max, ev2d, fit2d

G = 5.0 / 3.0
HERE = os.path.dirname(os.path.abspath(__file__))


def mesh_of(L):
    return O.Mesh(L.nx, L.ny, L.p, L.m, L.x0, L.x1, L.y0, L.y1, L.gamma)


def state(nx, ny, p, m, seed, amp=0.3):
    L, U, Bx, By, Bz = W.random_state(nx, ny, p, m, seed=seed, domain=(0, 1.5, 0, 1.0), amp=amp)
    M = mesh_of(L)
    rho, e, u = O.to_primitive(M, U)
    return L, M, rho, e, u, Bx, By, Bz


@pytest.mark.parametrize("pm", [(1, 0), (2, 1), (2, 2), (3, 2), (4, 3)])
@pytest.mark.parametrize("with_eta", [False, True])
def test_power_identity(pm, with_eta):
    p, m = pm
    L, M, rho, e, u, Bx, By, Bz = state(4, 3, p, m, seed=p * 10 + m)
    rng = np.random.default_rng(4)
    eta = rng.uniform(0.0, 0.05, M.K) if with_eta else None
    de, du, dBx, dBy, dBz = O.rhs_magnetic(M, rho, u, Bx, By, Bz, eta)
    x, w = O.gll(p)
    Mw = M.hx * M.hy / 4 * np.outer(w, w)
    kin = (Mw * rho * (u * du).sum(0)).sum()
    F = Fields(M.nx, M.ny, p, m, M.hx, M.hy)
    mag = B_product(F, (Bx, By, Bz), (dBx, dBy, dBz))
    heat = (Mw * rho * de).sum()
    scale = abs(kin) + abs(mag) + abs(heat)
    assert abs(kin + mag + heat) <= 1e-13 * scale, (kin, mag, heat)
    if not with_eta:
        assert (de == 0).all()
    else:
        assert heat > 0


@pytest.mark.parametrize("pm", [(1, 0), (2, 1), (2, 2), (3, 2), (4, 3), (4, 4)])
def test_curl_increment_divergence_free(pm):
    p, m = pm
    L, M, rho, e, u, Bx, By, Bz = state(4, 4, p, m, seed=7)
    de, du, dBx, dBy, dBz = O.rhs_magnetic(M, rho, u, Bx, By, Bz)
    F = Fields(M.nx, M.ny, p, m, M.hx, M.hy)
    scale = max(np.abs(dBx).max(), np.abs(dBy).max()) / min(M.hx, M.hy)
    assert div_max(F, dBx, dBy) <= 1e-12 * scale
    # the oracle's own divergence norm agrees
    assert O.divB_L2(M, dBx, dBy) <= 1e-12 * scale


def test_uniform_fields_closed_form():
    p, m = 3, 2
    M = O.Mesh(3, 4, p, m, 0, 1, 0, 1)
    sh = (M.K, p + 1, p + 1)
    rho = np.full(sh, 1.3)
    u = np.stack([np.full(sh, 0.2), np.full(sh, -0.7), np.full(sh, 0.4)])
    B = np.array([0.5, -0.3, 0.8])
    Bx, By, Bz = [np.full(M.gshape(), b) for b in B]
    JE = O.reconstruct_JE(M, u, Bx, By, Bz)
    E = -np.cross(u[:, 0, 0, 0], B)
    assert np.abs(JE[:3]).max() < 1e-13  # J = curl of a uniform field
    for c in range(3):
        np.testing.assert_allclose(JE[3 + c], E[c], rtol=1e-13)
    de, du, dBx, dBy, dBz = O.rhs_magnetic(M, rho, u, Bx, By, Bz, np.full(M.K, 0.1))
    for a in (de, du, dBx, dBy, dBz):
        assert np.abs(a).max() < 1e-12


@pytest.mark.parametrize("m", [0, 1, 2, 3])
def test_potential_field_divergence_free_and_current(m):
    # B = grad^perp A_h for A = sin x sin y on [0, 2pi]^2: div B = 0 exactly, J_z -> -2 sin x sin y
    errs = []
    for n in (8, 16, 32):
        L = W.Layout(n, n, m + 1, m, 0, 2 * math.pi, 0, 2 * math.pi)
        wX, wY = L.w_nodes()
        A = np.sin(wX) * np.sin(wY)
        M = mesh_of(L)
        Bx, By = O.B_from_potential(M, A)
        Bx2, By2 = L.curl_of_potential(A)
        np.testing.assert_allclose(Bx, Bx2, atol=1e-12); np.testing.assert_allclose(By, By2, atol=1e-12)
        if n == 8:
            assert div_max(Fields(n, n, m + 1, m, M.hx, M.hy), Bx, By) < 1e-11
        u = np.zeros((3, M.K, m + 2, m + 2))
        JE = O.reconstruct_JE(M, u, Bx, By, np.zeros_like(Bx))
        errs.append(np.abs(JE[2] + 2 * A).max())
    rate = math.log2(errs[1] / errs[2])
    assert rate > (m if m % 2 == 0 else m - 1) - 0.3 or errs[2] < 1e-9, (errs, rate)


def test_velocity_oe_identities():
    p, m = 3, 2
    L, M, rho, e, u, Bx, By, Bz = state(5, 4, p, m, seed=11, amp=0.6)
    e = np.abs(e) + 0.5
    o = O.Options(oe_mag=1)
    u2, e2, D = O.velocity_oe(M, o, 0.05, rho, u, e, Bx, By, Bz)
    x, w = O.gll(p)
    Mw = M.hx * M.hy / 4 * np.outer(w, w)
    mom0 = (Mw * rho * u).sum(axis=(2, 3)); mom1 = (Mw * rho * u2).sum(axis=(2, 3))
    np.testing.assert_allclose(mom1, mom0, atol=1e-14 * np.abs(mom0).max())
    kin0 = 0.5 * (Mw * rho * (u * u).sum(0)).sum(axis=(1, 2))
    kin1 = 0.5 * (Mw * rho * (u2 * u2).sum(0)).sum(axis=(1, 2))
    heat = (Mw * rho * (e2 - e)).sum(axis=(1, 2))
    np.testing.assert_allclose(kin0 - kin1, heat, atol=1e-14 * kin0.max())
    assert (e2 >= e).all() and (D[:, 1:] < 1).all()
    assert (kin0 - kin1 >= -1e-15).all()


def test_ar_hand_computed():
    # B_y = +b on the left half of the x-elements, -b on the right half; B_x = B_z = 0.
    # Elements touching a switch face have J_0 = 2b, Delta^B_x = b, sigma = 1, R = 1.
    p, m, nx, ny, b = 2, 1, 8, 3, 0.4
    M = O.Mesh(nx, ny, p, m, 0, 2.0, 0, 1.0)
    M1 = m + 1
    By = np.zeros(M.gshape())
    for ex in range(nx):
        By[:, ex * M1:(ex + 1) * M1] = b if ex < nx // 2 else -b
    Bx = np.zeros_like(By); Bz = np.zeros_like(By)
    sh = (M.K, p + 1, p + 1)
    rho = np.full(sh, 4.0)
    u = np.stack([np.full(sh, 0.3), np.full(sh, 0.1), np.zeros(sh)])
    o = O.Options(ar=1, C_s=5.0, C_eta=0.2)
    eta = O.ar_eta(M, o, rho, u, Bx, By, Bz).reshape(ny, nx)
    a_x = 0.3 + b / 2.0
    expect = 0.2 * M.hx / (2 * p + 1) * a_x
    for ex in range(nx):
        touching = ex in (0, nx // 2 - 1, nx // 2, nx - 1)
        np.testing.assert_allclose(eta[:, ex], expect if touching else 0.0, rtol=1e-13, atol=1e-13 * expect)
    # uniform field: no resistivity
    eta0 = O.ar_eta(M, o, rho, u, np.full_like(By, .3), np.full_like(By, .2), np.full_like(By, .1))
    assert (eta0 == 0).all()


def l2_errors(L, M, u, Bx, By, Bz, JE, fields):
    """L2(Omega) errors of u, B, E, J against the exact Alfven wave (Gauss rule of p+3 points)."""
    zq, wq = np.polynomial.legendre.leggauss(L.p + 3)
    X, Y = np.meshgrid(zq, zq, indexing="xy")
    Wt = np.outer(wq, wq) * L.hx * L.hy / 4
    F = Fields(L.nx, L.ny, L.p, L.m, L.hx, L.hy)
    eu = eB = eE = eJ = 0.0
    for ey in range(L.ny):
        for ex in range(L.nx):
            e = ey * L.nx + ex
            px = L.x0 + (ex + 0.5 * (X + 1)) * L.hx; py = L.y0 + (ey + 0.5 * (Y + 1)) * L.hy
            Bex, uex = fields(px, py)
            th = px + py - math.sqrt(2) * fields.t
            xi = W.gll_nodes(L.p)
            for d in range(3):
                uh = ev2d(fit2d(xi, xi, u[d][e]), X, Y)
                eu += (Wt * (uh - uex[d]) ** 2).sum()
            for k, fn in enumerate((F.bx, F.by, F.bz)):
                eB += (Wt * (ev2d(fn((Bx, By, Bz)[k], ex, ey), X, Y) - Bex[k]) ** 2).sum()
            # exact E = -u x B, J = curl B
            Ue = np.stack(uex); Be = np.stack(Bex)
            Eex = -np.cross(Ue, Be, axis=0)
            eps = 0.1
            # J = curl B for B = n + eps (t cos th + e_z sin th), th = x + y - w t
            Jex = np.stack([eps * np.cos(th), -eps * np.cos(th), -eps * math.sqrt(2) * np.sin(th)])
            xw = W.gll_nodes(L.m + 1); zg = W.gauss_nodes(L.m)
            comps = [(zg, xw), (xw, zg), (xw, xw)]
            for c in range(3):
                nxs, nys = comps[c]
                loc = F._loc(JE[c], ex, ey, len(nxs), len(nys))
                eJ += (Wt * (ev2d(fit2d(nxs, nys, loc), X, Y) - Jex[c]) ** 2).sum()
                loc = F._loc(JE[3 + c], ex, ey, len(nxs), len(nys))
                eE += (Wt * (ev2d(fit2d(nxs, nys, loc), X, Y) - Eex[c]) ** 2).sum()
    return math.sqrt(eu), math.sqrt(eB), math.sqrt(eE), math.sqrt(eJ)


def run_alfven(p, m, n, dt, tf=1.0):
    L, U, Bx, By, Bz, fields = W.alfven_wave(n, n, p, m)
    M = mesh_of(L)
    rho, e, u = O.to_primitive(M, U)
    o = O.Options()
    nsteps = int(round(tf / dt))
    for _ in range(nsteps):
        e, u, Bx, By, Bz, _ = O.step_magnetic(M, o, rho, e, u, Bx, By, Bz, dt)
    _, _, _, _, _, f_end = W.alfven_wave(n, n, p, m, t=tf)
    f_end.t = tf
    JE = O.reconstruct_JE(M, u, Bx, By, Bz)
    return l2_errors(L, M, u, Bx, By, Bz, JE, f_end)


def test_alfven_wave_against_table():
    """(p, m) = (2, 2), N = 16: errors of u, B, E, J within 25% of the paper's table of the
    reduced Alfven wave.  The time error is negligible at dt = 4e-3 (a run at dt = 2e-3
    agrees to three digits)."""
    gold = json.load(open(os.path.join(HERE, "golden", "alfven_table1.json")))
    row = gold["rows"]["2,2,16"]
    errs = run_alfven(2, 2, 16, dt=4e-3)
    for got, ref in zip(errs, (row["e_u"], row["e_B"], row["e_E"], row["e_J"])):
        assert 0.75 * ref < got < 1.25 * ref, (errs, row)


@pytest.mark.slow
def test_alfven_wave_rates_slow():
    """(2,2) at N = 32 within 25% of the table; (3,2) primary-field rates 3.0 +- 0.3 between
    N = 16 and 32 (its magnitudes are not pinned: the initial projection and the L2
    quadrature are unstated, and nodal interpolation alone already exceeds the printed
    (3,2) B and J errors)."""
    gold = json.load(open(os.path.join(HERE, "golden", "alfven_table1.json")))
    errs = run_alfven(2, 2, 32, dt=2e-3)
    row = gold["rows"]["2,2,32"]
    for got, ref in zip(errs, (row["e_u"], row["e_B"], row["e_E"], row["e_J"])):
        assert 0.75 * ref < got < 1.25 * ref, (errs, row)
    e16 = run_alfven(3, 2, 16, dt=4e-3)
    e32 = run_alfven(3, 2, 32, dt=2e-3)
    for a, b in zip(e16[:3], e32[:3]):
        assert 2.7 < math.log2(a / b) < 3.3, (e16, e32)


def test_velocity_oe_factor_hand_computed():
    """Eqs. magnetic-oe-sensor, magnetic-oe-rate and magnetic-oe-factor by hand on a p = m = 2
    state whose x-profile is the same in every element of a row: in row ey, u_x = a_ey (xhat +
    xhat^2), u_z = c a_ey xhat, u_y = 0.3 (constant: contributes zero), with non-uniform nodal rho
    and |B| (uniform in-plane B, nodal B_z).  With GLL_2 weights (1/3, 4/3, 1/3):
      x (row): u_x jumps 2 a in value and 8 a / hx in slope at every x-face, u_z 2 c a in value;
        row amplitudes 5 a / 3 (u_x) and c a (u_z), floored at 1e-6 Delta_Omega; the shared
        Delta^u_x is their maximum, sigma_x0 = max(2 a, 2 c a) / Delta^u_x, sigma_x1 =
        (3 hx / 2)(16 a / hx) / Delta^u_x, sigma_x2 = 0;
      y (column = the whole mesh here): the y-face jumps (a' - a)(xhat + xhat^2) and c (a' - a) xhat
        give (1/|F|) int [[.]]^2 = 2 (a' - a)^2 / 3 and c^2 (a' - a)^2 / 3; amplitudes are the global
        ones; no slope jumps;
      lam_I = 5 / h_I max_q (|u_I| + |B| / sqrt(rho)) over the element's nodes;
      D_l = exp(-s_M tau sum_I lam_I sum_{r <= l} sigma_{I,r}).
    A wrong rate (|B| / rho), a per-component amplitude, a dropped order r, or a missing floor in the
    nearly constant row 2 each move D far outside the tolerance."""
    p = m = 2
    nx, hx, hy, tau, sM, c = 3, 0.5, 0.4, 0.1, 0.02, 0.3
    a = np.array([0.4, 0.1, 4e-8, 0.25])
    ny = len(a)
    M = O.Mesh(nx, ny, p, m, 0, nx * hx, 0, ny * hy)
    xi, w = O.gll(p)
    X, Y = np.meshgrid(xi, xi)  # [j][i]: X = xhat_i, Y = yhat_j
    K = M.K
    ey = np.arange(K) // nx
    u = np.zeros((3, K, 3, 3))
    u[0] = a[ey][:, None, None] * (X + X * X)[None]
    u[1] = 0.3
    u[2] = c * a[ey][:, None, None] * X[None]
    rho = np.empty((K, 3, 3))
    rho[:] = 1.0 + 0.4 * X * Y + 0.2 * Y
    e = np.full((K, 3, 3), 2.0)
    G1 = (m + 1)
    Bx = np.full((ny * G1, nx * G1), 0.3)
    By = np.full_like(Bx, -0.2)
    Bz = np.zeros_like(Bx)
    Bzq = np.empty((K, 3, 3))
    for k in range(K):
        ex_, ey_ = k % nx, k // nx
        Bzq[k] = 0.2 + 0.3 * X + 0.1 * (ey_ + 1) * Y
        Bz[ey_ * G1:(ey_ + 1) * G1, ex_ * G1:(ex_ + 1) * G1] = Bzq[k]
    _, _, D = O.velocity_oe(M, O.Options(oe_mag=1, s_M=sM), tau, rho, u, e, Bx, By, Bz)

    # hand computation
    mean_x, mean_z = a.mean() / 3, 0.0
    dOm_x = max(max(abs(2 * aa - mean_x), abs(0 - mean_x)) for aa in a)
    dOm_z = c * a.max()
    rowx = np.maximum(5 * a / 3, 1e-6 * dOm_x)
    rowz = np.maximum(c * a, 1e-6 * dOm_z)
    Dsx = np.maximum(rowx, rowz)
    sx0 = np.maximum(2 * a, 2 * c * a) / Dsx
    sx1 = 1.5 * hx * (16 * a / hx) / Dsx
    Dsy = max(dOm_x, dOm_z)
    da_lo, da_hi = np.abs(a - np.roll(a, 1)), np.abs(np.roll(a, -1) - a)
    jyx = math.sqrt(2 / 3) * (da_lo + da_hi)
    jyz = c / math.sqrt(3) * (da_lo + da_hi)
    sy0 = 0.5 * np.maximum(jyx, jyz) / Dsy
    B2 = 0.3 ** 2 + 0.2 ** 2 + Bzq ** 2
    va = np.sqrt(B2) / np.sqrt(rho)
    lam_x = 5 / hx * (np.abs(u[0]) + va).reshape(K, -1).max(1)
    lam_y = 5 / hy * (np.abs(u[1]) + va).reshape(K, -1).max(1)
    th1 = lam_x * (sx0[ey] + sx1[ey]) + lam_y * sy0[ey]
    ref = np.exp(-sM * tau * th1)
    np.testing.assert_allclose(D[:, 1], ref, rtol=1e-10)
    np.testing.assert_allclose(D[:, 2], ref, rtol=1e-10)  # no second-derivative jumps
    assert (D[:, 1] < 0.99).all() and (D[:, 1] > 0.05).all()
    # the floor row's shared amplitude is the floor of u_x, not its own 5 a / 3
    assert rowx[2] == 1e-6 * dOm_x and Dsx[2] == rowx[2]


def test_ar_uniform_field_contributes_nothing_on_large_mesh():
    """A uniform field has only roundoff-level variation, so every direction contributes zero and
    eta = 0 exactly (eq. magnetic-ar-sensor), however many elements the mean is summed over: the
    test for roundoff-level variation is the exact nodal spread, not the deviation from a mean
    whose summation error grows with the mesh (1024 x 32 elements here, as the blast strip)."""
    L, U, Bx, By, Bz = W.blast(1024, 32, 4, 3)
    M = mesh_of(L)
    rho, e, u = O.to_primitive(M, U)
    u = u + 0.1  # nonzero speeds, so a spurious sensor response would show in eta
    eta = O.ar_eta(M, O.Options(ar=1), rho, u, Bx, By, Bz)
    assert (eta == 0.0).all(), eta.max()


@pytest.mark.parametrize("pmn", [(1, 0, 4), (2, 1, 5), (3, 3, 4)])
def test_vectorised_alfven_norms_equal_per_element_norms(pmn):
    """The vectorised Alfven-wave norms that the GPU table tests use (tests/_alfven_norms.py) equal
    the per-element evaluation above on an oracle state after three magnetic substeps."""
    from tests._alfven_norms import alfven_errors
    p, m, n = pmn
    L, U, Bx, By, Bz, _ = W.alfven_wave(n, n, p, m)
    M = mesh_of(L)
    rho, e, u = O.to_primitive(M, U)
    o = O.Options()
    for _ in range(3):
        e, u, Bx, By, Bz, _ = O.step_magnetic(M, o, rho, e, u, Bx, By, Bz, 0.01)
    _, _, _, _, _, f_end = W.alfven_wave(n, n, p, m, t=0.03)
    f_end.t = 0.03
    JE = O.reconstruct_JE(M, u, Bx, By, Bz)
    a = l2_errors(L, M, u, Bx, By, Bz, JE, f_end)
    b = alfven_errors(L, u, Bx, By, Bz, JE, 0.03)
    for x, y in zip(a, b):
        assert abs(x / y - 1.0) < 1e-12, (a, b)
