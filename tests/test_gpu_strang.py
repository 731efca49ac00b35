"""GPU parity of the full Strang step (algorithm "Strang split MHD step") through the C ABI,
on the workloads' own states: the small vortex (20 steps at CFL 0.3), the scaled Orszag-Tang
state with full stabilisation (64^2 two steps and the full 256^2 mesh one step), and
invariants of the 1024^2 blast-like stress state in the benchmark's configuration."""
import numpy as np
import pytest

import oracle as O
from paper_2609_10849_amd import workloads as W
from tests._gpu import announce, assert_parity, dev, host

pytestmark = pytest.mark.gpu


def omesh(L):
    return O.Mesh(L.nx, L.ny, L.p, L.m, L.x0, L.x1, L.y0, L.y1, L.gamma)


def compare(state_g, state_o, tol, what):
    for name, g, r in zip(("U", "Bx", "By", "Bz"), state_g, state_o):
        if np.abs(r).max() == 0:
            assert np.abs(host(g)).max() == 0, (what, name)
        else:
            assert_parity(host(g), r, tol, "%s %s" % (what, name))


def test_strang_vortex_small_20_steps():
    import paper_2609_10849_amd as pk
    announce("strang C1 vortex 20 steps")
    L, U, Bx, By, Bz = W.isentropic_vortex(16, 16, 3, 2)
    S = pk.Solver.from_layout(L)
    g = [dev(a) for a in (U, Bx, By, Bz)]
    dt = S.cfl_dt(*g, 0.3)
    M = omesh(L); o = O.Options()
    st = (U, Bx, By, Bz)
    for k in range(20):
        r, rep = S.strang_step(*g, dt)
        assert r == 0
        st = O.strang_step(M, o, *st, dt)[:4]
    compare(g, st, 1e-12, "C1 after 20 steps")


@pytest.mark.parametrize("n,steps", [(64, 2), (256, 1)])
def test_strang_orszag_tang_full_stabilisation(n, steps):
    import paper_2609_10849_amd as pk
    announce("strang OT %d^2 N=4 steps=%d" % (n, steps))
    L, U, Bx, By, Bz = W.orszag_tang_scaled(n, n, 4, 3)
    S = pk.Solver.from_layout(L, pk.Options.full())
    g = [dev(a) for a in (U, Bx, By, Bz)]
    dt = S.cfl_dt(*g, 0.3)
    M = omesh(L); o = O.Options.full()
    st = (U, Bx, By, Bz)
    for k in range(steps):
        r, rep = S.strang_step(*g, dt)
        out = O.strang_step(M, o, *st, dt)
        st = out[:4]
        assert r == 0 == out[6]
        for key in ("n_rho_limited", "n_p_limited", "n_collapsed", "max_depth"):
            assert rep[key] == out[4][key], key
        assert (S.decisions() == out[5]).all()
        # eta is O(rounding) on this smooth state; its error is measured against its scale at
        # full sensor response R = 1: C_eta * h/(2p+1) * max(|u| + |B|/sqrt(rho))
        eta_scale = 0.2 * L.hx / 9.0 * eta_speed(st[0], st[1], st[2], st[3])
        assert abs(rep["eta_max"] - out[4]["eta_max"]) <= 1e-12 * eta_scale
    compare(g, st, 1e-12, "OT %d" % n)


def eta_speed(U, Bx, By, Bz):
    u = np.abs(U[1:3] / U[0]).max()
    b = np.sqrt(np.abs(Bx).max() ** 2 + np.abs(By).max() ** 2 + np.abs(Bz).max() ** 2)
    return u + b / np.sqrt(U[0].min())


def test_strang_blast_full_size_invariants():
    """1024^2, N = 4, k = 3, full stabilisation, the benchmark's step: mass conserved to
    rounding, nodal rho and p positive, div B at rounding level, accepted accounting."""
    import paper_2609_10849_amd as pk
    announce("strang blast 1024^2 invariants")
    L, U, Bx, By, Bz = W.blast(1024, 1024, 4, 3)
    S = pk.Solver.from_layout(L, pk.Options.full())
    g = [dev(a) for a in (U, Bx, By, Bz)]
    d0 = S.diagnostics(*g)
    dt = S.cfl_dt(*g, 0.3)
    for k in range(2):
        r, rep = S.strang_step(*g, dt)
        assert r == 0 and rep["substeps_accepted"] >= 2
    d1 = S.diagnostics(*g)
    assert abs(d1["mass"] - d0["mass"]) <= 1e-13 * d0["mass"]
    assert d1["rho_min"] > 0 and d1["p_min"] > 0
    assert d1["divB_L2"] < 1e-10


@pytest.mark.parametrize("case", ["orszag_tang", "blast"])
def test_reduced_2d2v_equals_general(case):
    """The 2D2V reduced system skips only identically zero variables (u_z, B_z, in-plane E and
    J), so on 2D2V states its Strang steps equal the general path's: three steps with full
    stabilisation agree to 1e-14 relative, u_z and B_z stay exactly zero; one step at 32^2 also
    equals the oracle's general step to 1e-12."""
    import paper_2609_10849_amd as pk
    announce("2d2v reduced vs general %s" % case)
    if case == "orszag_tang":
        L, U, Bx, By, Bz = W.orszag_tang_scaled(64, 64, 4, 3)
    else:
        L, U, Bx, By, Bz = W.blast(64, 64, 4, 3, p_in=100.0)
    runs = []
    for r2 in (0, 1):
        S = pk.Solver.from_layout(L, pk.Options.full(reduced_2d2v=r2))
        g = [dev(a) for a in (U, Bx, By, Bz)]
        dt = S.cfl_dt(*g, 0.3)
        for _ in range(3):
            r, rep = S.strang_step(*g, dt)
            assert r == 0
        runs.append([host(a) for a in g])
        S.close()
    for a, b in zip(*runs):
        assert np.abs(a - b).max() <= 1e-14 * max(np.abs(a).max(), 1e-300)
    assert np.abs(runs[1][0][3]).max() == 0.0 and np.abs(runs[1][3]).max() == 0.0
    announce("2d2v reduced vs oracle %s" % case)
    L, U, Bx, By, Bz = (W.orszag_tang_scaled(32, 32, 4, 3) if case == "orszag_tang"
                        else W.blast(32, 32, 4, 3, p_in=100.0))
    S = pk.Solver.from_layout(L, pk.Options.full(reduced_2d2v=1))
    g = [dev(a) for a in (U, Bx, By, Bz)]
    dt = S.cfl_dt(*g, 0.3)
    r, rep = S.strang_step(*g, dt)
    assert r == 0
    ref = O.strang_step(omesh(L), O.Options.full(), U, Bx, By, Bz, dt)[:4]
    compare(g, ref, 1e-12, "2d2v %s" % case)
    S.close()


def test_strang_magnetic_outer_parity():
    """strang_order = 1 (M(dt/2) H(dt) M(dt/2)) with full stabilisation on the scaled Orszag-Tang
    state, 32^2, N = 4, two steps: equal to the oracle's magnetic-outer composition to 1e-12, limiter
    flags bit for bit."""
    import paper_2609_10849_amd as pk
    announce("strang magnetic-outer OT 32^2 N=4")
    L, U, Bx, By, Bz = W.orszag_tang_scaled(32, 32, 4, 3)
    S = pk.Solver.from_layout(L, pk.Options.full(strang_order=1))
    g = [dev(a) for a in (U, Bx, By, Bz)]
    dt = S.cfl_dt(*g, 0.3)
    M = omesh(L); o = O.Options.full(strang_order=1)
    st = (U, Bx, By, Bz)
    for k in range(2):
        r, rep = S.strang_step(*g, dt)
        out = O.strang_step(M, o, *st, dt)
        st = out[:4]
        assert r == 0 == out[6] and rep["substeps_accepted"] == out[4]["accepted"] == 1
        assert (S.decisions() == out[5]).all()
    compare(g, st, 1e-12, "OT magnetic-outer")
    S.close()


def test_checkpoint_restart_bit_exact():
    """Checkpoint and restart through host memory: n Strang steps, the state copied to the host,
    the context closed, a new context and fresh device buffers filled from the host copy, then n
    more steps; the result equals 2n uninterrupted steps bit for bit (full stabilisation, dt from
    the CFL rule at every step, 64^2, N = 4)."""
    import paper_2609_10849_amd as pk
    announce("checkpoint/restart, OT 64^2 N=4, 3 + 3 steps")
    L, U, Bx, By, Bz = W.orszag_tang_scaled(64, 64, 4, 3)

    def advance(S, g, n):
        for _ in range(n):
            r, _ = S.strang_step(*g, S.cfl_dt(*g, 0.3))
            assert r == 0

    S = pk.Solver.from_layout(L, pk.Options.full())
    g = [dev(a) for a in (U, Bx, By, Bz)]
    advance(S, g, 6)
    straight = [host(a) for a in g]
    S.close()
    S = pk.Solver.from_layout(L, pk.Options.full())
    g = [dev(a) for a in (U, Bx, By, Bz)]
    advance(S, g, 3)
    ckpt = [host(a).copy() for a in g]
    S.close()
    del g
    S = pk.Solver.from_layout(L, pk.Options.full())
    g = [dev(a) for a in ckpt]
    advance(S, g, 3)
    restarted = [host(a) for a in g]
    S.close()
    for a, b in zip(restarted, straight):
        assert np.array_equal(a, b)
