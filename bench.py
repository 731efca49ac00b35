"""Benchmark: DOF-stage updates/s (FP64) per Strang step on one MI355X.

Workload: the blast-like stress state on [-0.5, 0.5]^2, 1024 x 1024 elements, DGSEM degree
N = 4, magnetic degree k = 3, FP64, rho = 1, u = 0, p = 0.1 outside and 1000 inside r < 0.1,
B = (1, 1, 0)/sqrt(2); full Strang step with hydro OE, positivity scaling, velocity OE and
artificial resistivity; dt from the positivity CFL rule at CFL 0.3 before every step.
One Strang step = 6 hydro + 3 magnetic stages; value = K (N+1)^2 * 9 / t_step.

Prints one JSON line.  The roofline object describes the hydro stage kernel (L_E + SSP combine
+ element statistics), roofline_oe_pp the hydro stage map (OE + PP), which takes about as long per
launch; both are timed with HIP events on the library's stream.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6
VALU_FILE = os.path.join(ROOT, "profiles", "hydro_valu_flops.json")
TRAFFIC_FILES = {"stage": os.path.join(ROOT, "profiles", "hydro_stage_traffic.json"),
                 "oe_pp": os.path.join(ROOT, "profiles", "hydro_oe_pp_traffic.json")}
KERNEL_SRC = os.path.join(ROOT, "paper_2609_10849_amd", "csrc", "hydro.hip")


def stage_bytes(K, nn):
    """Algorithmic HBM bytes of one hydro-stage launch, averaged over the three SSP-RK(3,3) stages:
    the first reads U^n once, the second and third read U_s and U^n; each writes the raw stage
    (one U is 5 fields x K x nn doubles) and 15 statistics per element."""
    u = 5 * K * nn * 8
    return (2 * u + 3 * u + 3 * u) / 3.0 + K * 15 * 8


def stage_flops(K, NP):
    """Algorithmic FP64 flops of one hydro-stage launch (+, -, *, / and log, exp, sqrt count 1,
    FMA 2), per element: node primitives 20 per node; EC flux differencing 74 per node pair
    (flux, six divisions, two-sided accumulation) over (N+1)^2 N pairs; the LLF flux, 50 per
    face point, over the element's 2(N+1) own face points; the lift, 15 per face point over
    4(N+1); inverse mass and SSP combine 25 per node; statistics 20 per node."""
    nn = NP * NP
    return K * (20 * nn + 74 * nn * (NP - 1) + 50 * 2 * NP + 15 * 4 * NP + 25 * nn + 20 * nn)


def oe_pp_flops(K, NP):
    """Algorithmic FP64 flops of one stage-map launch, per element: the derivative traces of
    both sides of one face per direction, line and component (2 (N+1) dot products of length
    N+1) with the weighted squared jumps (3 per order); the per-order sums and sigma terms; the
    forward and inverse two-dimensional Legendre transforms (two passes each, 2 (N+1)^3 flops
    per pass and component); the shell damping; the positivity scaling, 30 per node."""
    nn = NP * NP
    jumps = 10 * NP * (4 * NP * NP + 3 * NP)
    sigma = 10 * NP * (NP + 4)
    return K * (jumps + sigma + 40 * NP ** 3 + 5 * nn + 4 * NP + 30 * nn)


def valu_per_launch(kind, K=1048576, N=4):
    """Executed FP64 flops per launch of a hydro kernel from the committed SQ counter run
    (SQ_INSTS_VALU_FLOPS_FP64 counts 2 FMA + ADD + MUL + TRANS instructions per wave; times
    the active lanes), or None when missing or taken on a different kernel source or workload."""
    try:
        d = json.load(open(VALU_FILE))[kind]
    except (OSError, ValueError, KeyError):
        return None
    if d.get("kernel_src_sha") != kernel_sha(kind) or d.get("elements") != K or d.get("N") != N:
        return None
    return d.get("flops_per_launch")


def valu_object(flops_alg, flops_ctr, avg_ms):
    """FP64 VALU view of a kernel: algorithmic and counter-measured TFLOP/s against the FP64
    vector peak."""
    t = avg_ms * 1e-3
    out = {"peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
           "algorithmic": flops_alg / t / 1e12, "algorithmic_frac": flops_alg / t / 1e12 / FP64_PEAK_TFS,
           "counter": None, "counter_frac": None}
    if flops_ctr is not None:
        out["counter"] = flops_ctr / t / 1e12
        out["counter_frac"] = flops_ctr / t / 1e12 / FP64_PEAK_TFS
    return out


def traffic_rate(traffic, avg_ms):
    """Counter-measured HBM bytes per launch over the launch time: GB/s and the fraction of the
    HBM peak, or None when the counters are not valid for this kernel source."""
    if traffic is None:
        return None, None
    r = traffic / (avg_ms * 1e-3) / 1e9
    return r, r / HBM_PEAK_GBS


def oe_pp_bytes(K, nn):
    """Algorithmic HBM bytes of one stage-map launch, averaged over the six launches of a Strang
    step: the raw stage read and the limited stage written (one U each), the six element
    statistics it uses read and its decision flag written; the last launch of the first hydro
    half-step also writes the primitive copy (rho, e, u) for the magnetic substep."""
    u = 5 * K * nn * 8
    return 2 * u + u / 6.0 + K * (6 * 8 + 1)


def kernel_sha(kind="stage"):
    """Hash of the source a hydro kernel is built from.  "stage": hydro.hip up to the end of the
    stage kernel (its device helpers and element statistics), its launch helpers and launcher, and
    the headers it includes; edits elsewhere (the OE/PP map) leave its counters valid.
    "oe_pp": hydro.hip up to the end of the stage map (so the stage kernel's source as well), its
    launcher, and the same headers."""
    src = open(KERNEL_SRC, encoding="utf-8").read()
    if kind == "stage":
        end = src.index("template <int P>\n__global__ __launch_bounds__(256) void k_elem_stats(")
        a = src.index("static int eb_of(")  # launch helpers (block size choice) and the launcher
        b = src.index("int line_global_reduce(", a)
    elif kind == "oe_pp":
        end = src.index("}  // namespace\n", src.index("void k_hydro_oe_pp("))
        a = src.index("int hydro_stage_b(")
        b = src.index("int reset_attempt(", a)
    else:
        raise ValueError(kind)
    h = hashlib.sha256((src[:end] + src[a:b]).encode())
    for name in ("common.h", "xcd.h", "ec_log.h", "rsqrt.h"):
        h.update(open(os.path.join(os.path.dirname(KERNEL_SRC), name), "rb").read())
    return h.hexdigest()[:16]


def traffic_per_launch(kind="stage", K=1048576, N=4):
    """HBM bytes per launch of a hydro kernel from the committed rocprofv3 counter runs, or None
    when they are missing or were taken on a different kernel source or workload (K, N)."""
    try:
        d = json.load(open(TRAFFIC_FILES[kind]))
    except (OSError, ValueError):
        return None
    if d.get("kernel_src_sha") != kernel_sha(kind) or d.get("elements") != K or d.get("N") != N:
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(seconds_hint=20.0):
    """The plain FP64 oracle, timed on this host: two Strang steps of the same blast workload on
    a 128 x 128 sub-resolution mesh (same domain, N = 4, k = 3, same options)."""
    import numpy as np

    import oracle as O
    from paper_2609_10849_amd import workloads as W

    n = 128
    L, U, Bx, By, Bz = W.blast(n, n, 4, 3)
    M = O.Mesh(L.nx, L.ny, L.p, L.m, L.x0, L.x1, L.y0, L.y1, L.gamma)
    threads = O.set_threads(0)
    dt = 2.0e-5
    steps = 6
    t0 = time.perf_counter()
    st = (U, Bx, By, Bz)
    for _ in range(steps):
        st = O.strang_step(M, O.Options.full(), *st, dt)[:4]
    t = time.perf_counter() - t0
    rate = M.K * 25 * 9 * steps / t
    return {"value": rate, "unit": "DOF-stage updates/s", "cores": threads, "kind": "oracle",
            "sample": "blast workload at 128x128 elements (N=4, k=3, full stabilisation), %d Strang steps, "
                      "%.1f s on %d OpenMP threads" % (steps, t, threads)}


def _event_ms(fn, reps, warm=3):
    """Average time of fn() in ms from HIP events on torch's current stream (the library's)."""
    import torch
    for _ in range(warm):
        fn()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def adjoint_ratio():
    """Cost of the hand-written VJPs relative to their forward operators on the noisy isentropic
    vortex, 128 x 128 elements, N = 3, k = 2 (cotangents N(0,1), seed 7)."""
    import numpy as np
    import torch

    import paper_2609_10849_amd as pk
    from paper_2609_10849_amd import workloads as W

    L, U, Bx, By, Bz = W.noisy_vortex(128, 128, 3, 2, seed=0)
    S = pk.Solver.from_layout(L)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    Ud, Bxd, Byd, Bzd = dev(U), dev(Bx), dev(By), dev(Bz)
    rng = np.random.default_rng(7)
    cot = dev(rng.standard_normal(U.shape))
    out, gb = torch.empty_like(Ud), torch.empty_like(Ud)
    tf = _event_ms(lambda: S.rhs_hydro(Ud, out), 50)
    tb = _event_ms(lambda: S.rhs_hydro_vjp(Ud, cot, gb), 50)
    rho, e, u = S.to_primitive(Ud)
    eta = dev(rng.uniform(0, 1e-3, L.K))
    cots = [dev(rng.standard_normal(tuple(a.shape))) for a in (e, u, Bxd, Byd, Bzd)]
    mf = _event_ms(lambda: S.rhs_magnetic(rho, u, Bxd, Byd, Bzd, eta), 50)
    mb = _event_ms(lambda: S.rhs_magnetic_vjp(rho, u, Bxd, Byd, Bzd, eta, *cots), 50)
    S.close()
    return {"hydro": tb / tf, "magnetic": mb / mf, "hydro_fwd_ms": tf, "hydro_vjp_ms": tb,
            "magnetic_fwd_ms": mf, "magnetic_vjp_ms": mb,
            "workload": "noisy isentropic vortex, 128x128 elements, N=3, k=2"}


def batched_speedup(steps=50, streams=False):
    """Ensemble of 64 uneven runs (n in {32..192}, N in {2,3,4}, k = N-1, vortex amplitude and
    field drawn from PCG64 seed 0; full stabilisation; per-run dt from CFL 0.3 at the start):
    time per Strang step of all runs, sequential plain launches vs the batch step: the captured
    multi-branch graph, or with streams=True the same deferred steps launched directly on the
    concurrent branch streams."""
    import numpy as np
    import torch

    import paper_2609_10849_amd as pk
    from paper_2609_10849_amd import workloads as W

    draws = W.ensemble_draws(64, seed=0)
    states, layouts = [], []
    for d in draws:
        L, U, Bx, By, Bz = W.isentropic_vortex(d["n"], d["n"], d["p"], d["m"], kappa=d["kappa"], B=d["B"])
        layouts.append(L)
        states.append((U, Bx, By, Bz))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    dts = []
    for L, st in zip(layouts, states):
        S = pk.Solver.from_layout(L, pk.Options.full())
        dts.append(S.cfl_dt(*[dev(a) for a in st], 0.3))
        S.close()
    B = pk.Batch(layouts, pk.Options.full())
    if streams:  # tile and branch choice by the event-timed autotuner (on scratch copies; untimed)
        g0 = [[dev(a) for a in st] for st in states]
        B.autotune(*[[x[i] for x in g0] for i in range(4)], dts)
        del g0

    def run(sequential, nsteps):
        g = [[dev(a) for a in st] for st in states]
        args = [[x[i] for x in g] for i in range(4)]
        B.strang_step(*args, dts, sequential=sequential, streams=streams)  # warm-up (and capture)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nsteps):
            r, _ = B.strang_step(*args, dts, sequential=sequential, streams=streams)
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / nsteps

    ts = run(True, steps)
    tb = run(False, steps)
    B.close()
    nodes = sum(L.K * (L.p + 1) ** 2 for L in layouts)
    return {"value": ts / tb, "sequential_ms_per_step": ts, "batched_ms_per_step": tb, "runs": 64,
            "steps": steps, "nodes": nodes,
            "path": "branch streams, no graph, autotuned tiles" if streams else "captured graph"}


def reduced_2d2v(S, g, steps=10, warm=2):
    """The same workload and state through the 2D2V reduced system (u_z = B_z = 0; the paper
    solves that system for such states): steps timed like the main run.  The headline value
    above is the general path's."""
    import torch
    S.set_options(S_options(reduced_2d2v=1))
    try:
        for _ in range(warm):
            dt = S.cfl_dt(*g, 0.3)
            S.strang_step(*g, dt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            dt = S.cfl_dt(*g, 0.3)
            r, rep = S.strang_step(*g, dt)
            if r != 0:
                raise RuntimeError("strang step failed: %r" % (rep,))
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / steps
    finally:
        S.set_options(S_options(reduced_2d2v=0))
    K, nn = S.K, (S.p + 1) ** 2
    return {"value": K * nn * 9 / t, "ms_per_step": 1e3 * t, "steps": steps,
            "note": "same workload through the 2D2V reduced system (u_z, B_z and the in-plane E, J skipped)"}


def hydro_only(S, g, steps=10, warm=2):
    """The hydro part of a Strang step alone: two half-step substeps (six SSP stages with their
    OE/PP maps and reject checks) on a copy of the state, at the step's dt; rate K (N+1)^2 6 / t.
    Rejected attempts would show as attempted > accepted."""
    import torch
    U = g[0].clone()
    dt = S.cfl_dt(*g, 0.3)
    for _ in range(warm):
        S.hydro_substep(U, 0.5 * dt)
    torch.cuda.synchronize()
    attempted = accepted = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        for _ in range(2):
            r, rep = S.hydro_substep(U, 0.5 * dt)
            if r != 0:
                raise RuntimeError("hydro substep failed: %r" % (rep,))
            attempted += rep["substeps_attempted"]
            accepted += rep["substeps_accepted"]
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    K, nn = S.K, (S.p + 1) ** 2
    return {"value": K * nn * 6 / t, "unit": "DOF-stage updates/s", "ms_per_step": 1e3 * t, "steps": steps,
            "substeps_attempted": attempted, "substeps_accepted": accepted,
            "note": "the two hydro half-steps of a Strang step alone (6 stages), same state and dt"}


def S_options(reduced_2d2v):
    import paper_2609_10849_amd as pk
    return pk.Options.full(reduced_2d2v=reduced_2d2v)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1024, help="elements per direction")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the adjoint-ratio and ensemble measurements")
    ap.add_argument("--reduced-2d2v", action="store_true",
                    help="time the 2D2V reduced system instead of the general path (for profiling it)")
    ap.add_argument("--ensemble-only", action="store_true",
                    help="time only the 64-run ensemble (streams batch step against sequential launches), for "
                         "profiling it; prints its own JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (see DESIGN.md, "
              "'How the path would shard')", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2609_10849_amd as pk
    from paper_2609_10849_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.ensemble_only:
        print(json.dumps({"batched_streams_speedup": batched_speedup(steps=args.steps, streams=True)}), flush=True)
        return
    n, N, k = args.n, 4, 3
    L, U, Bx, By, Bz = W.blast(n, n, N, k)
    S = pk.Solver.from_layout(L, pk.Options.full(reduced_2d2v=int(args.reduced_2d2v)))
    g = [torch.from_numpy(a).to("cuda") for a in (U, Bx, By, Bz)]
    del U, Bx, By, Bz
    K = L.K
    nn = (N + 1) ** 2

    def step():
        dt = S.cfl_dt(*g, 0.3)
        r, rep = S.strang_step(*g, dt)
        if r != 0:
            raise RuntimeError("strang step failed: %r" % (rep,))
        return rep

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    S.timing_read()  # discard
    S.timing(True)
    attempted = accepted = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rep = step()
        attempted += rep["substeps_attempted"]
        accepted += rep["substeps_accepted"]
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    S.timing(False)
    launches, kms = S.timing_read(0)
    launches_b, kms_b = S.timing_read(1)
    ms_per_step = 1e3 * t / args.steps
    value = K * nn * 9 / (t / args.steps)
    avg_ms = kms / max(launches, 1)
    ach = stage_bytes(K, nn) / (avg_ms * 1e-3) / 1e9
    tr = traffic_per_launch("stage", K, N)
    avg_b = kms_b / max(launches_b, 1)
    tr_b = traffic_per_launch("oe_pp", K, N)
    ach_b = oe_pp_bytes(K, nn) / (avg_b * 1e-3) / 1e9
    out = {
        "metric": "DOF-stage updates/s (FP64) per Strang step",
        "value": value,
        "unit": "DOF-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "blast-like stress state, [-0.5,0.5]^2 periodic, %dx%d elements, N=%d, k=%d, "
                               "p_in/p_out=1e4, full stabilisation (OE, PP, velocity OE, A.R.), CFL 0.3" % (n, n, N, k),
                   "elements": K, "N": N, "k": k, "dofs": K * nn,
                   "system": "2D2V reduced" if args.reduced_2d2v else "general"},
        "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                     "traffic": tr, "kernel": "k_hydro_stage<4,1> (L_E + SSP combine + element statistics)",
                     "avg_ms": avg_ms, "launches": launches,
                     "traffic_achieved": traffic_rate(tr, avg_ms)[0], "traffic_frac": traffic_rate(tr, avg_ms)[1],
                     "valu": valu_object(stage_flops(K, N + 1), valu_per_launch("stage", K, N), avg_ms)},
        "roofline_oe_pp": {"bound": "hbm", "achieved": ach_b, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": ach_b / HBM_PEAK_GBS, "traffic": tr_b,
                           "kernel": "k_hydro_oe_pp<4,128> (hydro OE + PP map)", "avg_ms": avg_b,
                           "launches": launches_b,
                           "traffic_achieved": traffic_rate(tr_b, avg_b)[0],
                           "traffic_frac": traffic_rate(tr_b, avg_b)[1],
                           "valu": valu_object(oe_pp_flops(K, N + 1), valu_per_launch("oe_pp", K, N), avg_b)},
        "accepted_substep_rate": accepted / max(attempted, 1),
    }
    if not args.no_extras and not args.reduced_2d2v:
        out["hydro_only"] = hydro_only(S, g, steps=min(args.steps, 10))
        out["reduced_2d2v"] = reduced_2d2v(S, g, steps=min(args.steps, 10))
        out["adjoint_cost_ratio"] = adjoint_ratio()
        # the captured-graph ensemble path is held off the GPU until the cause of a host
        # segmentation fault seen in one build of it is shown (last measured speedup: 1.63)
        out["batched_speedup"] = None
        out["batched_streams_speedup"] = batched_speedup(steps=min(args.steps, 20), streams=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
