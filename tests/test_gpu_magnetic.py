"""GPU parity of the magnetic-velocity family through the C ABI: J/E reconstruction
(eq. mag-current-proj, eq. mag-electric-proj), L_M, the artificial-resistivity coefficient,
the velocity OE and the magnetic substep; plus the power identity and divergence-free curl
increments checked on the GPU outputs with independent polynomial helpers."""
import numpy as np
import pytest

import oracle as O
from paper_2609_10849_amd import workloads as W
from tests._gpu import announce, assert_parity, dev, host
from tests._poly import B_product, Fields, div_max

pytestmark = pytest.mark.gpu

PM = [(1, 0), (1, 1), (2, 1), (2, 2), (3, 2), (3, 3), (4, 3), (4, 4)]


def setup(nx, ny, p, m, seed, amp=0.3):
    import paper_2609_10849_amd as pk
    L, U, Bx, By, Bz = W.random_state(nx, ny, p, m, seed=seed, domain=(0, 1.5, 0, 1.0), amp=amp)
    M = O.Mesh(L.nx, L.ny, p, m, L.x0, L.x1, L.y0, L.y1)
    rho, e, u = O.to_primitive(M, U)
    return L, M, rho, e, u, Bx, By, Bz


def solver(L, o=None):
    import paper_2609_10849_amd as pk
    return pk.Solver.from_layout(L, o)


@pytest.mark.parametrize("pm", PM)
def test_reconstruct_and_rhs_parity(pm):
    p, m = pm
    announce("magnetic rhs p=%d m=%d" % pm)
    L, M, rho, e, u, Bx, By, Bz = setup(5, 4, p, m, seed=10 * p + m)
    eta = np.random.default_rng(1).uniform(0, 0.05, M.K)
    S = solver(L)
    for et in (None, eta):
        ref_je = O.reconstruct_JE(M, u, Bx, By, Bz, et)
        got_je = host(S.reconstruct_JE(dev(u), dev(Bx), dev(By), dev(Bz), None if et is None else dev(et)))
        for k in range(6):
            assert_parity(got_je[k], ref_je[k], 1e-12, "JE %d" % k)
        ref = O.rhs_magnetic(M, rho, u, Bx, By, Bz, et)
        got = [host(t) for t in S.rhs_magnetic(dev(rho), dev(u), dev(Bx), dev(By), dev(Bz),
                                                None if et is None else dev(et))]
        for name, g, r in zip(("de", "du", "dBx", "dBy", "dBz"), got, ref):
            if np.abs(r).max() == 0:
                assert np.abs(g).max() == 0, name
            else:
                assert_parity(g, r, 1e-12, name)


@pytest.mark.parametrize("pm", [(2, 2), (3, 2), (4, 3)])
def test_power_identity_and_divergence_on_gpu(pm):
    p, m = pm
    announce("power identity p=%d m=%d" % pm)
    L, M, rho, e, u, Bx, By, Bz = setup(4, 3, p, m, seed=5)
    eta = np.random.default_rng(2).uniform(0, 0.05, M.K)
    S = solver(L)
    de, du, dBx, dBy, dBz = [host(t) for t in S.rhs_magnetic(dev(rho), dev(u), dev(Bx), dev(By), dev(Bz), dev(eta))]
    x, w = W.gll_nodes(p), np.polynomial.legendre.leggauss(1)[1]
    wq = O.gll(p)[1]
    Mw = M.hx * M.hy / 4 * np.outer(wq, wq)
    F = Fields(M.nx, M.ny, p, m, M.hx, M.hy)
    kin = (Mw * rho * (u * du).sum(0)).sum()
    mag = B_product(F, (Bx, By, Bz), (dBx, dBy, dBz))
    heat = (Mw * rho * de).sum()
    assert abs(kin + mag + heat) <= 1e-13 * (abs(kin) + abs(mag) + abs(heat))
    assert div_max(F, dBx, dBy) <= 1e-12 * max(np.abs(dBx).max(), np.abs(dBy).max()) / min(M.hx, M.hy)


@pytest.mark.parametrize("pm", [(2, 1), (2, 2), (3, 2), (4, 3)])
def test_ar_eta_parity(pm):
    p, m = pm
    announce("ar_eta p=%d m=%d" % pm)
    L, M, rho, e, u, Bx, By, Bz = setup(8, 6, p, m, seed=3, amp=0.5)
    o = O.Options(ar=1)
    ref = O.ar_eta(M, o, rho, u, Bx, By, Bz)
    import paper_2609_10849_amd as pk
    got = host(solver(L, pk.Options.make(ar=1)).ar_eta(dev(rho), dev(u), dev(Bx), dev(By), dev(Bz)))
    assert ref.max() > 0
    assert_parity(got, ref, 1e-12, "eta")


@pytest.mark.parametrize("pm", [(1, 0), (2, 2), (3, 2), (4, 3)])
def test_velocity_oe_parity(pm):
    p, m = pm
    announce("velocity_oe p=%d m=%d" % pm)
    L, M, rho, e, u, Bx, By, Bz = setup(7, 5, p, m, seed=4, amp=0.6)
    e = np.abs(e) + 0.5
    o = O.Options(oe_mag=1)
    ur, er, D = O.velocity_oe(M, o, 0.05, rho, u, e, Bx, By, Bz)
    import paper_2609_10849_amd as pk
    S = solver(L, pk.Options.make(oe_mag=1))
    tu, te = dev(u), dev(e)
    S.velocity_oe(0.05, dev(rho), tu, te, dev(Bx), dev(By), dev(Bz))
    assert_parity(host(tu), ur, 1e-12, "u")
    assert_parity(host(te) - e, er - e, 1e-11, "heating")
    assert_parity(host(te), er, 1e-12, "e")


@pytest.mark.parametrize("pm", [(2, 2), (3, 2), (4, 3)])
def test_step_magnetic_parity(pm):
    p, m = pm
    announce("step_magnetic p=%d m=%d" % pm)
    L, M, rho, e, u, Bx, By, Bz = setup(6, 5, p, m, seed=8, amp=0.5)
    e = np.abs(e) + 0.5
    o = O.Options(oe_mag=1, ar=1)
    ref = O.step_magnetic(M, o, rho, e, u, Bx, By, Bz, 0.01)
    import paper_2609_10849_amd as pk
    S = solver(L, pk.Options.make(oe_mag=1, ar=1))
    t = [dev(a) for a in (e, u, Bx, By, Bz)]
    rep = S.step_magnetic(dev(rho), *t, 0.01)
    for name, g, r in zip(("e", "u", "Bx", "By", "Bz"), t, ref[:5]):
        assert_parity(host(g), r, 1e-12, name)
    assert abs(rep["eta_max"] - ref[5]["eta_max"]) <= 1e-12 * ref[5]["eta_max"]
