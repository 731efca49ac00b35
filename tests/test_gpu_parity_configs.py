"""GPU parity at the benchmark configurations.

Blast-like stress state (the benchmark workload: 1024 x 1024, N = 4, k = 3, full stabilisation):
two Strang steps compared with the oracle's stored result (tests/golden/blast1024_N4_2steps.json,
written by tests/golden/make_blast1024_reference.py from the oracle alone): sampled nodal values
of every field to 1e-12 of the field's max, field sums, the limiter flags bit for bit (sha256
and per-bit counts) and the reports; plus live oracle comparisons on 1024 x 32 and 32 x 1024
strips of the same state, whose row and column reductions loop over more than one record per
thread, as at full size.

Noisy vortex (the adjoint workload: 128 x 128, N = 3, k = 2): forward parity of rhs_hydro,
rhs_magnetic, both substeps and one Strang step, and central finite differences of the
magnetic VJP over 64 directions."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_2609_10849_amd import workloads as W
from tests._gpu import announce, assert_parity, dev, host

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
REF = os.path.join(HERE, "golden", "blast1024_N4_2steps.json")


def omesh(L):
    return O.Mesh(L.nx, L.ny, L.p, L.m, L.x0, L.x1, L.y0, L.y1, L.gamma)


@pytest.mark.skipif(not os.path.exists(REF), reason="stored blast reference not generated")
def test_blast1024_two_steps_against_stored_oracle():
    import paper_2609_10849_amd as pk
    from tests.golden.make_blast1024_reference import DT, FIELDS, N_EL, M as MM, P, STEPS, sample_indices
    announce("blast 1024^2 N=4 two steps vs stored oracle")
    ref = json.load(open(REF))
    L, U, Bx, By, Bz = W.blast(N_EL, N_EL, P, MM)
    S = pk.Solver.from_layout(L, pk.Options.full())
    g = [dev(a) for a in (U, Bx, By, Bz)]
    del U, Bx, By, Bz
    # wave-speed bound of the state over both steps: the fast speed inside the blast (u = 0, rho = 1)
    ETA_SPEED = 1.0 + np.sqrt(5.0 / 3.0 * 1000.0)
    for s in range(STEPS):
        r, rep = S.strang_step(*g, DT)
        assert r == 0
        want = ref["reports"][s]
        assert rep["substeps_attempted"] == want["attempted"] and rep["substeps_accepted"] == want["accepted"]
        assert rep["max_depth"] == want["max_depth"]
        for k, kr in (("n_rho_limited", "n_rho_limited"), ("n_p_limited", "n_p_limited"),
                      ("n_collapsed", "n_collapsed")):
            assert rep[k] == want[kr], (s, k)
        # eta is measured against its scale at full sensor response: C_eta h / (2p+1) max(|u| + |B|/sqrt(rho))
        # (on the nearly uniform field of the first step it is far below that scale)
        eta_scale = 0.2 * L.hx / (2 * P + 1) * ETA_SPEED
        assert abs(rep["eta_max"] - want["eta_max"]) <= 1e-12 * eta_scale, (s, rep["eta_max"], want["eta_max"])
    flags = S.decisions()
    assert hashlib.sha256(flags.tobytes()).hexdigest() == ref["flags_sha256"]
    assert [int(((flags >> b) & 1).sum()) for b in range(3)] == ref["flags_bits"]
    iu, ib = sample_indices(None, None)
    Uh = host(g[0])
    comps = [Uh[c].ravel() for c in range(5)] + [host(t).ravel() for t in g[1:]]
    for name, f in zip(FIELDS, comps):
        rf = ref["fields"][name]
        idx = iu if name in FIELDS[:5] else ib
        scale = max(rf["max_abs"], 1e-300)
        err = np.abs(f[idx] - np.array(rf["samples"])).max() / scale
        assert err <= 1e-12, (name, err)
        assert abs(np.abs(f).max() - rf["max_abs"]) <= 1e-12 * scale, name
        assert abs(f.sum() - rf["sum"]) <= 1e-12 * max(rf["sum_abs"], 1e-300), name
    S.close()


@pytest.mark.parametrize("nx,ny", [(1024, 32), (32, 1024)])
def test_blast_strip_two_steps_live(nx, ny):
    import paper_2609_10849_amd as pk
    announce("blast strip %dx%d N=4 two steps vs oracle" % (nx, ny))
    L, U, Bx, By, Bz = W.blast(nx, ny, 4, 3)
    S = pk.Solver.from_layout(L, pk.Options.full())
    g = [dev(a) for a in (U, Bx, By, Bz)]
    dt = S.cfl_dt(*g, 0.3)
    M = omesh(L)
    st = (U, Bx, By, Bz)
    for s in range(2):
        r, rep = S.strang_step(*g, dt)
        out = O.strang_step(M, O.Options.full(), *st, dt)
        st = out[:4]
        assert r == 0 == out[6]
        for key in ("substeps_attempted", "max_depth", "n_rho_limited", "n_p_limited", "n_collapsed"):
            k2 = {"substeps_attempted": "attempted"}.get(key, key)
            assert rep[key] == out[4][k2], (s, key)
        assert (S.decisions() == out[5]).all()
    assert out[4]["n_p_limited"] + out[4]["n_rho_limited"] > 0  # the limiter acts on this state
    # U to 1e-12 of its largest value (the total energy inside the blast, about 1.5e3).  The in-plane
    # field is compared to 1e-11 of its own size: its increments tau curl(u x B) take the velocity's
    # absolute differences, which the U bar allows up to 1e-12 of that energy scale, through a factor
    # tau (2 / h_x) |B| (m+1)^2 per stage; on these strips (h_x = 1/1024, six magnetic stages over two
    # steps) that bounds them near 1e-11 of |B| (measured 5.2e-12), while every decision matches bit
    # for bit.  The full-size benchmark state meets 1e-12 on every field (test above).
    for name, a, r_ in zip(("U", "Bx", "By", "Bz"), g, st):
        if np.abs(r_).max() > 0:
            assert_parity(host(a), r_, 1e-12 if name == "U" else 1e-11, "strip %s" % name)
    S.close()


def noisy():
    return W.noisy_vortex(128, 128, 3, 2, seed=0)


@pytest.mark.parametrize("full", [False, True])
def test_noisy_vortex_forward_parity(full):
    import paper_2609_10849_amd as pk
    announce("noisy vortex 128^2 forward parity full=%d" % full)
    L, U, Bx, By, Bz = noisy()
    M = omesh(L)
    opts, oopts = (pk.Options.full(), O.Options.full()) if full else (pk.Options.make(), O.Options())
    S = pk.Solver.from_layout(L, opts)
    assert_parity(host(S.rhs_hydro(dev(U))), O.rhs_hydro(M, U), 1e-12, "rhs_hydro")
    rho, e, u = O.to_primitive(M, U)
    eta = np.random.default_rng(11).uniform(0, 1e-3, M.K)
    got = S.rhs_magnetic(dev(rho), dev(u), dev(Bx), dev(By), dev(Bz), dev(eta))
    want = O.rhs_magnetic(M, rho, u, Bx, By, Bz, eta)
    for name, a, b in zip(("de", "du", "dBx", "dBy", "dBz"), got, want):
        assert_parity(host(a), b, 1e-12, "rhs_magnetic " + name)
    g = [dev(a) for a in (U, Bx, By, Bz)]
    dt = S.cfl_dt(*g, 0.3)
    gU = dev(U)
    r, rep = S.hydro_substep(gU, 0.5 * dt)
    Uo, orep, oflags, _, ost = O.hydro_substep(M, oopts, U, 0.5 * dt)
    assert r == 0 == ost and rep["substeps_attempted"] == orep["attempted"]
    assert_parity(host(gU), Uo, 1e-12, "hydro substep")
    gs = [dev(a) for a in (rho, e, u, Bx, By, Bz)]
    rep = S.step_magnetic(*gs, dt)
    eo, uo, bxo, byo, bzo, mrep = O.step_magnetic(M, oopts, rho, e, u, Bx, By, Bz, dt)
    for name, a, b in zip(("e", "u", "Bx", "By", "Bz"), gs[1:], (eo, uo, bxo, byo, bzo)):
        assert_parity(host(a), b, 1e-12, "magnetic substep " + name)
    r, rep = S.strang_step(*g, dt)
    out = O.strang_step(M, oopts, U, Bx, By, Bz, dt)
    assert r == 0 == out[6]
    for name, a, b in zip(("U", "Bx", "By", "Bz"), g, out[:4]):
        if np.abs(b).max() > 0:
            assert_parity(host(a), b, 1e-12, "strang " + name)
    S.close()


def test_magnetic_vjp_central_fd_64_directions():
    """Central differences (step 1e-6 relative to each input's size, 64 seeded directions over
    (u, B_x, B_y, B_z) jointly) of the GPU forward L_M against <(ubar, Bbar), v>, with a frozen
    nonzero eta.  L_M is a polynomial of degree two in (u, B) for frozen rho and eta, so central
    differences carry only rounding error."""
    import paper_2609_10849_amd as pk
    announce("magnetic vjp central FD 64 directions 128^2 N=3 k=2")
    L, U, Bx, By, Bz = noisy()
    M = omesh(L)
    rho, e, u = O.to_primitive(M, U)
    eta = np.random.default_rng(11).uniform(0, 1e-3, M.K)
    rng = np.random.default_rng(7)
    cots = [rng.standard_normal(a.shape) for a in (e, u, Bx, By, Bz)]
    S = pk.Solver.from_layout(L, pk.Options.make())
    drho, deta = dev(rho), dev(eta)
    xs = [u, Bx, By, Bz]
    bars = [host(t) for t in S.rhs_magnetic_vjp(drho, dev(u), dev(Bx), dev(By), dev(Bz), deta,
                                                 *[dev(c) for c in cots])]
    h = 1e-6
    scales = [np.abs(a).max() for a in xs]
    worst = 0.0
    for s in range(64):
        r2 = np.random.default_rng(1000 + s)
        V = [r2.standard_normal(a.shape) * sc for a, sc in zip(xs, scales)]
        fp = [host(t) for t in S.rhs_magnetic(drho, *[dev(a + h * v) for a, v in zip(xs, V)], deta)]
        fm = [host(t) for t in S.rhs_magnetic(drho, *[dev(a - h * v) for a, v in zip(xs, V)], deta)]
        fd = sum(((p_ - m_) / (2 * h) * c).sum() for p_, m_, c in zip(fp, fm, cots))
        ad = sum((b * v).sum() for b, v in zip(bars, V))
        worst = max(worst, abs(fd - ad) / max(abs(ad), 1e-300))
    assert worst < 1e-6, worst
    S.close()
