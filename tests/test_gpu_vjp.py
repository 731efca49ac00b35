"""GPU hand-written adjoints through the C ABI.

Hydro: Ubar = (dL_E/dU)^T cot.  Magnetic: (ubar, Bbar) = (dL_M/d(u,B))^T (de, du, dB cot) with
rho and eta frozen.  Checked (1) elementwise against the oracle's FP64 reference gradient,
assembled column by column from its complex-step JVP on a small mesh, (2) by the dot-product
test <VJP(cot), v> = <cot, JVP(v)> with the oracle JVP at the adjoint workload size
(128 x 128, N = 3, k = 2, noisy vortex, cotangent seed 7), and (3) by central finite
differences (step 1e-6) of the GPU forward operator over 64 random directions."""
import numpy as np
import pytest

import oracle as O
from paper_2609_10849_amd import workloads as W
from tests._gpu import announce, assert_parity, dev, host

pytestmark = pytest.mark.gpu


def omesh(L):
    return O.Mesh(L.nx, L.ny, L.p, L.m, L.x0, L.x1, L.y0, L.y1, L.gamma)


def solver(L, opts=None):
    import paper_2609_10849_amd as pk
    return pk.Solver.from_layout(L, opts)


@pytest.mark.parametrize("p,iface", [(2, 0), (3, 0), (4, 0), (3, 1)])
def test_hydro_vjp_elementwise_reference(p, iface):
    announce("hydro vjp elementwise p=%d iface=%d" % (p, iface))
    L, U, *_ = W.random_state(3, 3, p, p - 1, seed=20 + p, amp=0.3)
    M = omesh(L)
    n = U.size
    J = np.zeros((n, n))
    for k in range(n):
        v = np.zeros(n); v[k] = 1.0
        J[:, k] = O.rhs_hydro_jvp(M, U, v.reshape(U.shape), iface_flux=iface).ravel()
    cot = np.random.default_rng(7).standard_normal(U.shape)
    ref = (J.T @ cot.ravel()).reshape(U.shape)
    import paper_2609_10849_amd as pk
    S = solver(L, pk.Options.make(iface_flux=iface))
    got = host(S.rhs_hydro_vjp(dev(U), dev(cot)))
    assert_parity(got, ref, 1e-12, "Ubar")


def adjoint_state():
    return W.noisy_vortex(128, 128, 3, 2, seed=0)


def test_hydro_vjp_dot_product_full_size():
    announce("hydro vjp dot product 128^2 N=3")
    L, U, Bx, By, Bz = adjoint_state()
    M = omesh(L)
    cot = np.random.default_rng(7).standard_normal(U.shape)
    S = solver(L)
    Ub = host(S.rhs_hydro_vjp(dev(U), dev(cot)))
    for s in range(3):
        v = np.random.default_rng(1000 + s).standard_normal(U.shape)
        jv = O.rhs_hydro_jvp(M, U, v)
        lhs = (Ub * v).sum(); rhs = (cot * jv).sum()
        scale = np.abs(Ub * v).sum()
        assert abs(lhs - rhs) <= 1e-12 * scale, (lhs, rhs)


@pytest.mark.parametrize("iface", [1, 0])
def test_hydro_vjp_central_fd_64_directions(iface):
    """Central differences (per-entry step 1e-6 |U| v, v ~ N(0,1), 64 directions) of the GPU
    forward operator against <Ubar, v> on the adjoint workload (128 x 128, N = 3, noisy vortex).
    With EC interfaces L_E is smooth and v is unrestricted.  The LLF operator is only piecewise
    smooth (max/abs at faces; a 1e-6 step flips branches at faces where the two wave speeds are
    within the step), so for it v is restricted to element-interior nodes, which never enter an
    interface flux; the face-node part of its adjoint is pinned elementwise against the oracle."""
    import paper_2609_10849_amd as pk
    announce("hydro vjp central FD 64 directions iface=%d" % iface)
    L, U, Bx, By, Bz = adjoint_state()
    h = 1e-6
    cot = np.random.default_rng(7).standard_normal(U.shape)
    S = solver(L, pk.Options.make(iface_flux=iface))
    Ub = host(S.rhs_hydro_vjp(dev(U), dev(cot)))
    mask = np.ones(U.shape)
    if iface == 0:
        mask[:, :, 0, :] = mask[:, :, -1, :] = 0.0
        mask[:, :, :, 0] = mask[:, :, :, -1] = 0.0
    worst = 0.0
    for s in range(64):
        v = np.random.default_rng(1000 + s).standard_normal(U.shape) * mask
        fp = host(S.rhs_hydro(dev(U + h * v * np.abs(U))))
        fm = host(S.rhs_hydro(dev(U - h * v * np.abs(U))))
        fd = ((fp - fm) / (2 * h) * cot).sum()
        ad = (Ub * v * np.abs(U)).sum()
        worst = max(worst, abs(fd - ad) / max(abs(ad), 1e-300))
    assert worst < 1e-6, worst


MAG_PM = [(2, 2), (3, 2), (4, 3)]


def mag_state(nx, ny, p, m, seed):
    L, U, Bx, By, Bz = W.random_state(nx, ny, p, m, seed=seed, domain=(0, 1.5, 0, 1.0), amp=0.3)
    M = omesh(L)
    rho, e, u = O.to_primitive(M, U)
    return L, M, rho, e, u, Bx, By, Bz


@pytest.mark.parametrize("pm", MAG_PM)
@pytest.mark.parametrize("with_eta", [False, True])
def test_magnetic_vjp_elementwise_reference(pm, with_eta):
    p, m = pm
    announce("magnetic vjp elementwise p=%d m=%d eta=%d" % (p, m, with_eta))
    L, M, rho, e, u, Bx, By, Bz = mag_state(3, 2, p, m, seed=3)
    eta = np.random.default_rng(5).uniform(0, 0.05, M.K) if with_eta else None
    rng = np.random.default_rng(7)
    cots = [rng.standard_normal(a.shape) for a in (e, u, Bx, By, Bz)]
    ins = [u, Bx, By, Bz]
    sizes = [a.size for a in ins]
    grads = [np.zeros(s) for s in sizes]
    for blk, a in enumerate(ins):
        for k in range(a.size):
            V = [np.zeros_like(x) for x in ins]
            V[blk].reshape(-1)[k] = 1.0
            outs = O.rhs_magnetic_jvp(M, rho, u, Bx, By, Bz, eta, *V)
            grads[blk][k] = sum((c * o).sum() for c, o in zip(cots, outs))
    S = solver(L)
    got = S.rhs_magnetic_vjp(dev(rho), dev(u), dev(Bx), dev(By), dev(Bz), None if eta is None else dev(eta),
                             *[dev(c) for c in cots])
    for name, g, r, a in zip(("ubar", "Bxbar", "Bybar", "Bzbar"), got, grads, ins):
        assert_parity(host(g), r.reshape(a.shape), 1e-12, name)


def test_magnetic_vjp_dot_product_full_size():
    announce("magnetic vjp dot product 128^2 N=3 k=2")
    L, U, Bx, By, Bz = adjoint_state()
    M = omesh(L)
    rho, e, u = O.to_primitive(M, U)
    eta = np.random.default_rng(11).uniform(0, 1e-3, M.K)
    rng = np.random.default_rng(7)
    cots = [rng.standard_normal(a.shape) for a in (e, u, Bx, By, Bz)]
    S = solver(L)
    got = [host(t) for t in S.rhs_magnetic_vjp(dev(rho), dev(u), dev(Bx), dev(By), dev(Bz), dev(eta),
                                               *[dev(c) for c in cots])]
    for s in range(2):
        r2 = np.random.default_rng(1000 + s)
        V = [r2.standard_normal(a.shape) for a in (u, Bx, By, Bz)]
        outs = O.rhs_magnetic_jvp(M, rho, u, Bx, By, Bz, eta, *V)
        lhs = sum((g * v).sum() for g, v in zip(got, V))
        rhs = sum((c * o).sum() for c, o in zip(cots, outs))
        scale = sum(np.abs(g * v).sum() for g, v in zip(got, V))
        assert abs(lhs - rhs) <= 1e-12 * scale, (lhs, rhs)


def test_autograd_wrappers_use_the_vjp_entry_points():
    """torch.autograd through HydroRHS / MagneticRHS returns exactly the VJP entry points' output
    and satisfies the dot-product test against the oracle JVP."""
    import torch
    from paper_2609_10849_amd import autograd as AG
    announce("autograd wrappers 16^2 N=3 k=2")
    L, U, Bx, By, Bz = W.noisy_vortex(16, 16, 3, 2, seed=0)
    M = omesh(L)
    S = solver(L)
    Ud = dev(U).requires_grad_(True)
    out = AG.rhs_hydro(S, Ud)
    assert (host(out.detach()) == host(S.rhs_hydro(dev(U)))).all()
    cot = np.random.default_rng(7).standard_normal(U.shape)
    (g,) = torch.autograd.grad(out, Ud, dev(cot))
    assert (host(g) == host(S.rhs_hydro_vjp(dev(U), dev(cot)))).all()
    v = np.random.default_rng(1000).standard_normal(U.shape)
    lhs = (host(g) * v).sum(); rhs = (cot * O.rhs_hydro_jvp(M, U, v)).sum()
    assert abs(lhs - rhs) <= 1e-12 * np.abs(host(g) * v).sum()

    rho, e, u = O.to_primitive(M, U)
    eta = np.random.default_rng(11).uniform(0, 1e-3, M.K)
    ins = [dev(a).requires_grad_(True) for a in (u, Bx, By, Bz)]
    outs = AG.rhs_magnetic(S, dev(rho), *ins, eta=dev(eta))
    rng = np.random.default_rng(7)
    cots = [rng.standard_normal(a.shape) for a in (e, u, Bx, By, Bz)]
    grads = torch.autograd.grad(outs, ins, [dev(c) for c in cots])
    direct = S.rhs_magnetic_vjp(dev(rho), dev(u), dev(Bx), dev(By), dev(Bz), dev(eta), *[dev(c) for c in cots])
    for a, b in zip(grads, direct):
        assert (host(a) == host(b)).all()
    V = [np.random.default_rng(1001).standard_normal(a.shape) for a in (u, Bx, By, Bz)]
    jv = O.rhs_magnetic_jvp(M, rho, u, Bx, By, Bz, eta, *V)
    lhs = sum((host(g) * x).sum() for g, x in zip(grads, V))
    rhs = sum((c * o).sum() for c, o in zip(cots, jv))
    assert abs(lhs - rhs) <= 1e-12 * sum(np.abs(host(g) * x).sum() for g, x in zip(grads, V))
