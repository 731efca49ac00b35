"""Boundary calls on the GPU: connectivity and node coordinates against the oracle (maps bit for
bit), and the admissibility refusal (status 2, input left unmodified) of the step entry points."""
import numpy as np
import pytest

import oracle as O
from paper_2609_10849_amd import workloads as W
from tests._gpu import announce, dev, host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nx,ny,p,m", [(1, 1, 1, 0), (7, 5, 3, 2), (256, 256, 4, 3), (33, 17, 6, 5)])
def test_maps_and_coords_match_oracle(nx, ny, p, m):
    import paper_2609_10849_amd as pk
    announce("maps %dx%d p=%d m=%d" % (nx, ny, p, m))
    S = pk.Solver(nx, ny, p, m, -0.5, 0.5, -0.5, 0.5)
    M = O.Mesh(nx, ny, p, m, -0.5, 0.5, -0.5, 0.5)
    nbr, dof = S.get_maps()
    onbr, odof = O.get_maps(M)
    assert np.array_equal(host(nbr), onbr)
    assert np.array_equal(host(dof), odof)
    for space in range(7):
        x, y = S.node_coords(space)
        ox, oy = O.node_coords(M, space)
        assert np.abs(host(x).ravel() - ox).max() <= 1e-15 and np.abs(host(y).ravel() - oy).max() <= 1e-15, space
    S.close()


def test_inadmissible_input_status_2():
    import paper_2609_10849_amd as pk
    from tests.test_oracle_maps import bad_states
    announce("status 2 on inadmissible input")
    L, U, cases = bad_states()
    S = pk.Solver.from_layout(L, pk.Options.full())
    for name, u, bx, by, bz in cases:
        g = [dev(a) for a in (u, bx, by, bz)]
        r, rep = S.strang_step(*g, 1e-3)
        assert r == 2 and rep["status"] == 2 and rep["substeps_attempted"] == 0, name
        for a, b in zip(g, (u, bx, by, bz)):
            assert np.array_equal(host(a), b, equal_nan=True), name
        if name != "nan Bx":
            gu = dev(u)
            r2, rep2 = S.hydro_substep(gu, 1e-3)
            assert r2 == 2 and rep2["status"] == 2, name
            assert np.array_equal(host(gu), u, equal_nan=True), name
    # admissible input afterwards: ordinary step, equal to the oracle
    Lv, Uv, Bx, By, Bz = W.isentropic_vortex(4, 3, 2, 1)
    g = [dev(a) for a in (Uv, Bx, By, Bz)]
    r, rep = S.strang_step(*g, 1e-3)
    assert r == 0
    M = O.Mesh(L.nx, L.ny, L.p, L.m, L.x0, L.x1, L.y0, L.y1, L.gamma)
    ref = O.strang_step(M, O.Options.full(), Uv, Bx, By, Bz, 1e-3)
    for a, b in zip(g, ref[:4]):
        if np.abs(b).max() > 0:
            assert np.abs(host(a) - b).max() <= 1e-12 * np.abs(b).max()
    rho, e, u = O.to_primitive(M, Uv)
    e[1, 0, 0] = -1.0
    ge, gu = dev(e), dev(u)
    rep = S.step_magnetic(dev(rho), ge, gu, dev(Bx), dev(By), dev(Bz), 1e-3)
    assert rep["status"] == 2
    assert np.array_equal(host(ge), e) and np.array_equal(host(gu), u)
    S.close()
