"""Batched ensemble through the C ABI: one Strang step of uneven runs by run-table launches (each
launch covers every run of a degree group), plainly and replayed from a HIP graph captured on one
stream, must equal, bit for bit, each run stepped alone with the plain entry point (same kernel
bodies); one member is checked against the oracle; a member that needs a halving takes the
individual redo.  Every graph replay is checked against the eager result, with the eager steps and
host synchronisations in between."""

import numpy as np
import pytest

import oracle as O
from paper_2609_10849_amd import workloads as W
from tests._gpu import announce, assert_parity, dev, host

pytestmark = pytest.mark.gpu


def runs_small():
    specs = [(12, 10, 2, 1, 0.3, (0.1, 0.05)), (16, 16, 3, 2, 0.5, (0.0, 0.2)), (8, 14, 4, 3, 0.7, (0.25, 0.0)),
             (20, 12, 2, 2, 0.2, (0.1, 0.1)), (10, 10, 3, 3, 0.6, (0.0, 0.0))]
    out = []
    for nx, ny, p, m, kappa, B in specs:
        L, U, Bx, By, Bz = W.isentropic_vortex(nx, ny, p, m, kappa=kappa, B=B, background=(0.3, -0.2))
        out.append((L, U, Bx, By, Bz))
    return out


def to_dev(run):
    return [dev(a) for a in run[1:]]


@pytest.mark.parametrize("graph", [False, True])
def test_batch_equals_individual_and_oracle(graph):
    import paper_2609_10849_amd as pk
    announce("run-table batch vs individual graph=%d" % graph)
    runs = runs_small()
    opts = pk.Options.full()
    B = pk.Batch([r[0] for r in runs], opts)
    B.graph(graph)
    dts = []
    single = []
    for r in runs:
        S = pk.Solver.from_layout(r[0], opts)
        g = to_dev(r)
        dts.append(0.5 * S.cfl_dt(*g, 0.3))
        single.append((S, g))
    bat = [to_dev(r) for r in runs]
    for step in range(3):  # with graph=True: one capture, then every replay checked against the eager path
        st, reps = B.strang_step([b[0] for b in bat], [b[1] for b in bat], [b[2] for b in bat], [b[3] for b in bat],
                                 dts)
        assert st == 0
        for k, (S, g) in enumerate(single):
            r, rep = S.strang_step(*g, dts[k])
            assert r == 0
            for a, b in zip(bat[k], g):
                assert (host(a) == host(b)).all(), (step, k)
            assert reps[k]["n_p_limited"] == rep["n_p_limited"]
            assert reps[k]["eta_max"] == rep["eta_max"]
    # one member against the oracle (3 steps)
    L, U, Bx, By, Bz = runs[1]
    M = O.Mesh(L.nx, L.ny, L.p, L.m, L.x0, L.x1, L.y0, L.y1, L.gamma)
    st = (U, Bx, By, Bz)
    for _ in range(3):
        st = O.strang_step(M, O.Options.full(), *st, dts[1])[:4]
    for a, r in zip(bat[1], st):
        if np.abs(r).max() > 0:
            assert_parity(host(a), r, 1e-12, "batched member vs oracle")
    B.close()


@pytest.mark.parametrize("graph", [False, True])
def test_batch_rejection_fallback(graph):
    import paper_2609_10849_amd as pk
    announce("run-table batch rejection fallback graph=%d" % graph)
    runs = runs_small()[:2]
    Lb, Ub, Bxb, Byb, Bzb = W.blast(8, 8, 2, 1, p_in=1000.0)
    runs.append((Lb, Ub, Bxb, Byb, Bzb))
    opts = pk.Options.make(oe_hydro=1, pp=1)
    B = pk.Batch([r[0] for r in runs], opts)
    B.graph(graph)
    dts = [1e-3, 1e-3, 1e-2]  # the blast member needs halvings at this step
    bat = [to_dev(r) for r in runs]
    single = [to_dev(r) for r in runs]
    for step in range(2):
        st, reps = B.strang_step([b[0] for b in bat], [b[1] for b in bat], [b[2] for b in bat], [b[3] for b in bat],
                                 dts)
        assert st == 0
        assert reps[2]["substeps_attempted"] > reps[2]["substeps_accepted"]
        for k, r in enumerate(runs):
            S = pk.Solver.from_layout(r[0], opts)
            S.strang_step(*single[k], dts[k])
            S.close()
            for a, b in zip(bat[k], single[k]):
                assert (host(a) == host(b)).all(), (step, k)
    B.close()
