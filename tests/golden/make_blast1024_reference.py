"""Writes tests/golden/blast1024_N4_2steps.json with the oracle only: two Strang steps of the
blast-like stress state (1024 x 1024 elements on [-0.5, 0.5]^2, N = 4, k = 3, rho = 1, u = 0,
p = 0.1 with p = 1000 at nodes inside r < 0.1, B = (1, 1, 0)/sqrt2) with every stabilisation on
(hydro OE, positivity scaling, velocity OE, artificial resistivity; paper constants) at the fixed
step DT (the CFL-0.3 step of this state, rounded).  Stored per field (the five conservative
components, B_x, B_y, B_z): the values at seeded sample nodes (sample_indices, half spread over
the whole mesh, half inside the blast region), max |f|, sum f and sum |f|; the per-element limiter
flags of the last stage map as a sha256 and per-bit counts; both steps' reports.
Run (about 10 minutes on 8 cores, 20 GB of memory): python tests/golden/make_blast1024_reference.py"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_2609_10849_amd import workloads as W  # noqa: E402

N_EL, P, M, DT, STEPS = 1024, 4, 3, 4.0e-7, 2
OUT = os.path.join(HERE, "blast1024_N4_2steps.json")
FIELDS = ("rho", "mx", "my", "mz", "E", "Bx", "By", "Bz")


def sample_indices(K_shape_u, g_shape, n_el=N_EL, p=P, m=M, n=512, seed=2024):
    """Seeded sample indices into a conservative component ([K][p+1][p+1] flattened) and into a
    magnetic grid (flattened): n uniform over the mesh and n in the elements with |x|, |y| < 0.15."""
    rng = np.random.default_rng(seed)
    nn = (p + 1) ** 2
    KN = n_el * n_el * nn
    lo, hi = int(0.35 * n_el), int(0.65 * n_el)
    ex = rng.integers(lo, hi, n); ey = rng.integers(lo, hi, n); q = rng.integers(0, nn, n)
    iu = np.concatenate([rng.choice(KN, n, replace=False), (ey * n_el + ex) * nn + q])
    G1 = n_el * (m + 1)
    gx = rng.integers(lo * (m + 1), hi * (m + 1), n); gy = rng.integers(lo * (m + 1), hi * (m + 1), n)
    ib = np.concatenate([rng.choice(G1 * G1, n, replace=False), gy * G1 + gx])
    return iu, ib


def summary(U, Bx, By, Bz):
    iu, ib = sample_indices(None, None)
    out = {}
    comps = [U[c].ravel() for c in range(5)] + [Bx.ravel(), By.ravel(), Bz.ravel()]
    for name, f in zip(FIELDS, comps):
        idx = iu if name in FIELDS[:5] else ib
        out[name] = {"samples": [float(v) for v in f[idx]], "max_abs": float(np.abs(f).max()),
                     "sum": float(f.sum()), "sum_abs": float(np.abs(f).sum())}
    return out


def main():
    nt = O.set_threads(0)
    L, U, Bx, By, Bz = W.blast(N_EL, N_EL, P, M)
    Mh = O.Mesh(L.nx, L.ny, L.p, L.m, L.x0, L.x1, L.y0, L.y1, L.gamma)
    reps = []
    t0 = time.time()
    for s in range(STEPS):
        U, Bx, By, Bz, rep, flags, st = O.strang_step(Mh, O.Options.full(), U, Bx, By, Bz, DT)
        assert st == 0, st
        reps.append(rep)
        print("step", s, rep, "%.0f s" % (time.time() - t0), flush=True)
    doc = {
        "what": "oracle: 2 Strang steps of the blast-like state, 1024x1024, N=4, k=3, full stabilisation",
        "dt": DT, "steps": STEPS, "threads": nt,
        "reports": [{k: (float(v) if isinstance(v, float) else int(v)) for k, v in r.items()} for r in reps],
        "flags_sha256": hashlib.sha256(flags.tobytes()).hexdigest(),
        "flags_bits": [int(((flags >> b) & 1).sum()) for b in range(3)],
        "fields": summary(U, Bx, By, Bz),
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=0)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
