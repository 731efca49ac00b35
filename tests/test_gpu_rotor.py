"""Mirror walls (section "MHD rotor"; reading in paper_2609_10849_amd.workloads.MIRROR_PARITY, mesh
flag walls = 3): a box with mirror walls is solved as its mirror-doubled periodic mesh, with the
stabilisers' amplitudes taken over the box.

Parity: mirror-symmetric states with every field nonzero on doubled meshes, two fully stabilised
Strang steps against the oracle (1e-12 per field, limiter decisions bit for bit, identical
reports), and the symmetry kept to rounding.

Paper numbers (tests/golden/nonsmooth_scalars.json, "rotor"): the rotor of that section, p = m = 2,
256^2 box, t = 0.295, OE and positivity on, without and with A.R."""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_2609_10849_amd import workloads as W
from tests._gpu import announce, assert_parity, dev, host
from tests._mirror import mirror_errors, mirror_state, wall_mass_flux

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def omesh(L):
    return O.Mesh(L.nx, L.ny, L.p, L.m, L.x0, L.x1, L.y0, L.y1, L.gamma, walls=L.walls)


@pytest.mark.parametrize("n,p,m,walls", [(8, 2, 2, 3), (6, 3, 2, 3), (8, 2, 2, 2)])
def test_mirror_state_parity(n, p, m, walls):
    """walls 3: mirror walls on all four sides; 2: only the y-normal ones (periodic in x)."""
    import paper_2609_10849_amd as pk
    announce("mirror state %d^2 box p=%d m=%d walls=%d" % (n, p, m, walls))
    L, U, Bx, By, Bz = mirror_state(n, p, m)
    L.walls = walls
    S = pk.Solver.from_layout(L, pk.Options.full())
    g = [dev(a) for a in (U, Bx, By, Bz)]
    dt = S.cfl_dt(*g, 0.3)
    M = omesh(L); o = O.Options.full()
    st = (U, Bx, By, Bz)
    for k in range(2):
        r, rep = S.strang_step(*g, dt)
        out = O.strang_step(M, o, *st, dt)
        st = out[:4]
        assert r == 0 == out[6]
        for key in ("n_rho_limited", "n_p_limited", "n_collapsed", "max_depth"):
            assert rep[key] == out[4][key], key
        assert (S.decisions() == out[5]).all()
        assert abs(rep["eta_max"] - out[4]["eta_max"]) <= 1e-12 * max(out[4]["eta_max"], 1e-300) + 1e-300
    for name, a, b in zip(("U", "Bx", "By", "Bz"), g, st):
        assert_parity(host(a), b, 1e-12, "mirror %s" % name)
    fin = [host(a) for a in g]
    assert max(mirror_errors(L, *fin, axes=("x", "y") if walls == 3 else ("y",)).values()) < 1e-12
    if walls == 3:
        assert wall_mass_flux(L, fin[0]) < 1e-13
    S.close()


def run_rotor(ar):
    """The rotor to t = 0.295 (readings R25, R6: CFL 0.3), returning the final state, the final
    diagnostics and the last step's A.R. maximum."""
    import paper_2609_10849_amd as pk
    L, U, Bx, By, Bz = W.rotor_mirror(256, 2, 2)
    S = pk.Solver.from_layout(L, pk.Options.make(1, 1, 1, ar, C_eta=0.2, C_s=5.0))
    g = [dev(a) for a in (U, Bx, By, Bz)]
    t, eta = 0.0, 0.0
    while t < 0.295 - 1e-14:
        dt = min(S.cfl_dt(*g, 0.3), 0.295 - t)
        r, rep = S.strang_step(*g, dt)
        assert r == 0
        eta, t = rep["eta_max"], t + dt
    d1 = S.diagnostics(*g)
    out = [host(a) for a in g]
    S.close()
    return L, out, d1, eta


def test_rotor_paper_scalars():
    """Rotor, p = m = 2, 256^2 box with mirror walls, t = 0.295, OE and positivity on, without and
    with A.R.: magnetic-pressure maxima (at the velocity nodes, R26) within 0.5 % of 0.7051 and
    0.7038; the box's divergence norm (half the doubled mesh's, by symmetry) within 5 % of 4.60e-12;
    the final-step A.R. maximum within 20 % of 8.63e-5; the doubled state mirror-symmetric to 1e-10
    after about 5 150 steps; the extremes of rho, p_m and the Mach number contain the caption's
    common contour ranges."""
    from tests._fe_fields import B_at, primitives
    from paper_2609_10849_amd.workloads import gll_nodes
    gold = json.load(open(os.path.join(HERE, "golden", "nonsmooth_scalars.json")))["rotor"]
    for ar in (0, 1):
        announce("rotor ar=%d" % ar)
        L, (Uf, Bxf, Byf, Bzf), d1, eta = run_rotor(ar)
        assert max(mirror_errors(L, Uf, Bxf, Byf, Bzf).values()) < 1e-10
        rho, u, p = primitives(L, Uf)
        Bn = B_at(L, Bxf, Byf, Bzf, np.array(gll_nodes(2))).reshape(3, *rho.shape)
        pm = 0.5 * (Bn ** 2).sum(0)
        mach = np.sqrt((u ** 2).sum(0)) / np.sqrt(L.gamma * p / rho)
        assert abs(pm.max() / gold["pm_max"][ar] - 1.0) < 5e-3, (ar, pm.max())
        assert abs(0.5 * d1["divB_L2"] / gold["divB"] - 1.0) < 0.05, d1
        if ar:
            assert abs(eta / gold["eta_max_final"] - 1.0) < 0.2, eta
        for name, f in (("rho", rho), ("pm", pm), ("mach", mach)):
            lo, hi = gold[name + "_levels"]
            assert f.min() <= lo and f.max() >= hi, (name, f.min(), f.max())
