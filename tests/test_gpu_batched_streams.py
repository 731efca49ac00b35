"""Batched ensemble without a graph: one Strang step of uneven runs launched directly on the
batch's concurrent branch streams must equal, bit for bit, each run stepped alone with the plain
entry point (same kernels); one member is checked against the oracle; a member that needs a
halving takes the individual fallback.  The event-timed autotuner (plain launches, no graph)
writes and reuses its cache."""
import json

import numpy as np
import pytest

import oracle as O
from paper_2609_10849_amd import workloads as W
from tests._gpu import announce, assert_parity, dev, host
from tests.test_gpu_batched import runs_small, to_dev

pytestmark = pytest.mark.gpu


def test_streams_batch_equals_individual_and_oracle():
    import paper_2609_10849_amd as pk
    announce("streams batch vs individual")
    runs = runs_small()
    opts = pk.Options.full()
    B = pk.Batch([r[0] for r in runs], opts)
    dts, single = [], []
    for r in runs:
        S = pk.Solver.from_layout(r[0], opts)
        g = to_dev(r)
        dts.append(0.5 * S.cfl_dt(*g, 0.3))
        single.append((S, g))
    bat = [to_dev(r) for r in runs]
    for step in range(3):
        st, reps = B.strang_step([b[0] for b in bat], [b[1] for b in bat], [b[2] for b in bat], [b[3] for b in bat],
                                 dts, streams=True)
        assert st == 0
        for k, (S, g) in enumerate(single):
            r, rep = S.strang_step(*g, dts[k])
            assert r == 0
            for a, b in zip(bat[k], g):
                assert (host(a) == host(b)).all(), (step, k)
            assert reps[k]["n_p_limited"] == rep["n_p_limited"]
            assert reps[k]["eta_max"] == rep["eta_max"]
    L, U, Bx, By, Bz = runs[1]
    M = O.Mesh(L.nx, L.ny, L.p, L.m, L.x0, L.x1, L.y0, L.y1, L.gamma)
    st = (U, Bx, By, Bz)
    for _ in range(3):
        st = O.strang_step(M, O.Options.full(), *st, dts[1])[:4]
    for a, r in zip(bat[1], st):
        if np.abs(r).max() > 0:
            assert_parity(host(a), r, 1e-12, "batched member vs oracle")
    B.close()


def test_streams_batch_rejection_fallback():
    import paper_2609_10849_amd as pk
    announce("streams batch rejection fallback")
    runs = runs_small()[:2]
    Lb, Ub, Bxb, Byb, Bzb = W.blast(8, 8, 2, 1, p_in=1000.0)
    runs.append((Lb, Ub, Bxb, Byb, Bzb))
    opts = pk.Options.make(oe_hydro=1, pp=1)
    B = pk.Batch([r[0] for r in runs], opts)
    dts = [1e-3, 1e-3, 1e-2]  # the blast member needs halvings at this step
    bat = [to_dev(r) for r in runs]
    st, reps = B.strang_step([b[0] for b in bat], [b[1] for b in bat], [b[2] for b in bat], [b[3] for b in bat], dts,
                             streams=True)
    assert st == 0
    assert reps[2]["substeps_attempted"] > reps[2]["substeps_accepted"]
    for k, r in enumerate(runs):
        S = pk.Solver.from_layout(r[0], opts)
        g = to_dev(r)
        S.strang_step(*g, dts[k])
        for a, b in zip(bat[k], g):
            assert (host(a) == host(b)).all(), k
    B.close()


def test_batch_autotune_event_timed(tmp_path):
    """Tile choice timed with plain launches (no graph capture while tuning), cache written and
    reused, states untouched."""
    import paper_2609_10849_amd as pk
    announce("batch autotune (event-timed tiles)")
    runs = runs_small()
    B = pk.Batch([r[0] for r in runs], pk.Options.full())
    bat = [to_dev(r) for r in runs]
    before = [host(a).copy() for b in bat for a in b]
    cache = str(tmp_path / "tune.jsonl")
    dts = [1e-3] * len(runs)
    S1 = B.autotune([b[0] for b in bat], [b[1] for b in bat], [b[2] for b in bat], [b[3] for b in bat], dts, cache)
    assert 2 <= S1 <= 8
    after = [host(a) for b in bat for a in b]
    assert all((x == y).all() for x, y in zip(before, after))  # tuning works on scratch copies
    line = json.loads(open(cache).read().strip().splitlines()[-1])
    assert line["branches"] == S1
    S2 = B.autotune([b[0] for b in bat], [b[1] for b in bat], [b[2] for b in bat], [b[3] for b in bat], dts, cache)
    assert S2 == S1
