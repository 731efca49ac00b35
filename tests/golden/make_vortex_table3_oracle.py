"""Writes tests/golden/vortex_table3_oracle.json with the oracle only: the advected isodensity vortex
of the section "Advected MHD vortex" in the setting of its temporal self-convergence table
((p, m) = (2, 2), 64 x 64, t_f = 1, stabilisation off, dt = 1e-2 * 2^-l for l = 0..3).  Stored:
the Cauchy differences d_rho and d_u over [-5, 5]^2 (same norm as tests/test_oracle_strang.py)
and, for every dt, sampled final nodal values (64 seeded node indices of each conservative field
and of B_x) for element-wise GPU parity.  Run: python tests/golden/make_vortex_table3_oracle.py"""
import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_2609_10849_amd import workloads as W  # noqa: E402
from tests.test_oracle_strang import cauchy  # noqa: E402

N, P, M, TF = 64, 2, 2, 1.0
DTS = [1e-2 * 2.0 ** -l for l in range(4)]


def main():
    O.set_threads(0)
    sols = []
    for dt in DTS:
        L, U, Bx, By, Bz = W.balsara_vortex(N, N, P, M)
        Mh = O.Mesh(L.nx, L.ny, L.p, L.m, L.x0, L.x1, L.y0, L.y1, L.gamma)
        for _ in range(int(round(TF / dt))):
            U, Bx, By, Bz, rep, flags, st = O.strang_step(Mh, O.Options(), U, Bx, By, Bz, dt)
            assert st == 0
        sols.append((U, Bx, By, Bz))
        print("dt", dt, "done", flush=True)
    d = cauchy(L, Mh, sols)
    rng = np.random.default_rng(42)
    iu = rng.choice(sols[0][0][0].size, 64, replace=False)
    ib = rng.choice(sols[0][1].size, 64, replace=False)
    samples = []
    for U, Bx, By, Bz in sols:
        samples.append({"U": [U[c].ravel()[iu].tolist() for c in range(5)], "Bx": Bx.ravel()[ib].tolist()})
    out = {"source": "oracle, " + __doc__.split("\n")[0], "N": N, "p": P, "m": M, "t_f": TF, "dt": DTS,
           "d_rho": [x["rho"] for x in d], "d_u": [x["u"] for x in d], "node_index": iu.tolist(),
           "bx_index": ib.tolist(), "samples": samples}
    json.dump(out, open(os.path.join(HERE, "vortex_table3_oracle.json"), "w"), indent=0)


if __name__ == "__main__":
    main()
