"""Benchmark: DOF-stage updates/s (FP64) per Strang step on one MI355X.

Workload: the blast-like stress state on [-0.5, 0.5]^2, 1024 x 1024 elements, DGSEM degree
N = 4, magnetic degree k = 3, FP64, rho = 1, u = 0, p = 0.1 outside and 1000 inside r < 0.1,
B = (1, 1, 0)/sqrt(2); full Strang step with hydro OE, positivity scaling, velocity OE and
artificial resistivity; dt from the positivity CFL rule at CFL 0.3 before every step.
One Strang step = 6 hydro + 3 magnetic stages; value = K (N+1)^2 * 9 / t_step.

Prints one JSON line.  Every large kernel of the step is timed with HIP events on the library's
stream (mhd25_timing_read); "roofline" describes the kernel with the largest share of the step
time, "roofline_kernels" all of them, each with its algorithmic HBM bytes (and FP64 flops where
the kernel is arithmetic) per launch against the MI355X peaks, and the counter-measured traffic
and FP64 flops of profiles/kernel_counters.json when those were taken on the same kernel sources
and workload (bench.py --ingest writes that record from rocprofv3 counter runs).
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
COUNTER_FILE = os.path.join(ROOT, "profiles", "kernel_counters.json")
CSRC = os.path.join(ROOT, "paper_2609_10849_amd", "csrc")
KERNEL_SRC = os.path.join(CSRC, "hydro.hip")


def kernel_table(N, k):
    """The timed kernels of a Strang step: (timing id, name, rocprofv3 name prefix, source file,
    algorithmic HBM bytes per element and launch, algorithmic FP64 flops per element and launch or
    None, fraction of a block's lanes that carry work).  Bytes count each array the kernel must
    touch once (neighbour data counted as cache hits); the stage kernel's and the map's are the
    averages over the launches of a step (see stage_bytes, oe_pp_bytes)."""
    NP, nn = N + 1, (N + 1) ** 2
    A, B = k + 2, k + 1
    psi = nn * (nn + (nn % 2)) * 8
    grid3 = 3 * B * B * 8
    loads = (2 * A * B + A * A) * 8
    y = 4 * nn * 8 + grid3  # (e, u, B) of one element
    blk = lambda bs, nt: (bs // nt) * nt / bs
    nt = max(nn, A * A)
    return [
        (0, "hydro stage (L_E + SSP combine + statistics)", "k_hydro_stage<", "hydro.hip",
         (8.0 / 3.0) * 5 * nn * 8 + 15 * 8, stage_flops(1, NP), blk(128, nn)),
        (1, "hydro stage map (OE + PP)", "k_hydro_oe_pp<", "hydro.hip",
         2 * 5 * nn * 8 + 5 * nn * 8 / 6.0 + 49, oe_pp_flops(1, NP), blk(128, nn)),
        (2, "magnetic update (curl, Lorentz, Ohm, SSP combine)", "k_mag_update<", "magnetic.hip",
         2 * grid3 + nn * 8 + 8 + y + (2.0 / 3.0) * y + y + 9 * 8, None, blk(256, nt)),
        (3, "velocity-OE projection", "k_vel_proj<", "magnetic.hip",
         psi + 3 * nn * 8 + 2 * nn * 8 + NP * 8 + 4 * nn * 8, None, blk(128, nn)),
        (4, "velocity-OE preparation (Gram, Cholesky, basis)", "k_vel_prep<", "magnetic.hip",
         nn * 8 + psi, None, blk(128, nn)),
        (5, "E loads", "k_E_loads<", "magnetic.hip", 3 * nn * 8 + 2 * grid3 + 8 + loads, None, blk(128, nt)),
        (6, "velocity-OE sensor", "k_vel_sensor<", "magnetic.hip", 4 * nn * 8 + grid3 + NP * 8, None, blk(256, nn)),
        (7, "J loads", "k_J_loads<", "magnetic.hip", grid3 + loads, None, blk(256, nt)),
        (8, "gathers of shared DOFs", "k_gather<", "magnetic.hip", loads + grid3, None, 1.0),
        (9, "A.R. traces", "k_ar_traces<", "magnetic.hip", 4 * nn * 8 + grid3 + (8 * A + 2) * 8, None, blk(256, nn)),
    ]


def source_sha(fname):
    """Hash of a kernel source file and the headers every kernel file includes."""
    h = hashlib.sha256(open(os.path.join(CSRC, fname), "rb").read())
    for name in ("common.h", "xcd.h", "ec_log.h", "rsqrt.h"):
        h.update(open(os.path.join(CSRC, name), "rb").read())
    return h.hexdigest()[:16]


def counter_record(prefix, fname, K, N):
    """Counter-measured bytes and FP64 flops per launch of a kernel from profiles/kernel_counters.json,
    or None when missing or taken on other kernel sources or another workload."""
    try:
        d = json.load(open(COUNTER_FILE))
    except (OSError, ValueError):
        return None
    r = d.get("kernels", {}).get(prefix)
    if not r or r.get("src_sha") != source_sha(fname) or d.get("elements") != K or d.get("N") != N:
        return None
    return r


def ingest_counters(dirs, K=1048576, N=4, k=3, steps=1):
    """Write profiles/kernel_counters.json (and a readable summary) from rocprofv3 --pmc runs of
    `bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-extras`: one directory with FETCH_SIZE, one
    with WRITE_SIZE and one with the FP64 instruction counters (SQ_INSTS_VALU_FLOPS_FP64, SQ_INSTS_VALU,
    SQ_WAVES).  FETCH_SIZE and WRITE_SIZE are scaled by what they read for the entry snapshot kernel,
    which copies the state (5 K (N+1)^2 doubles) once: known bytes over counter value.  FP64 flops per
    launch are SQ_INSTS_VALU_FLOPS_FP64 (2 FMA + ADD + MUL + TRANS FP64 instructions per wave) times 64
    lanes times the fraction of a block's lanes that carry work."""
    import csv
    import glob
    vals = {}  # counter -> kernel prefix -> [values per dispatch]
    cmd = []
    for d in dirs:
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for row in csv.DictReader(open(f)):
                name, ctr = row["Kernel_Name"], row["Counter_Name"]
                val = float(row["Counter_Value"])
                for pre in [t[2] for t in kernel_table(N, k)] + ["k_snap_check_U"]:
                    if pre in name:
                        vals.setdefault(ctr, {}).setdefault(pre, []).append(val)
    known = 5.0 * K * (N + 1) ** 2 * 8
    fetch_cal = known / vals["FETCH_SIZE"]["k_snap_check_U"][0]
    write_cal = known / vals["WRITE_SIZE"]["k_snap_check_U"][0]
    out = {"elements": K, "N": N, "k": k, "workload": "blast-like state %dx%d elements, N=%d, k=%d, one Strang step"
           % (int(K ** 0.5), int(K ** 0.5), N, k),
           "calibration": {"kernel": "k_snap_check_U (entry snapshot: copies the state)", "bytes": known,
                           "fetch_factor": fetch_cal, "write_factor": write_cal},
           "commands": ["rocprofv3 --pmc %s --output-format csv -d gpurun_out/%s -o %s -- python -u bench.py --steps 1 "
                        "--warmup 0 --no-cpu-baseline --no-extras" % (c, d, d[-1].lower())
                        for c, d in (("FETCH_SIZE", "pmcF"), ("WRITE_SIZE", "pmcW"),
                                     ("SQ_WAVES SQ_INSTS_VALU SQ_INSTS_VALU_FLOPS_FP64", "pmcV"))],
           "kernels": {}}
    for kid, name, prefix, fname, bytes_el, flops_el, lanes in kernel_table(N, k):
        f = vals.get("FETCH_SIZE", {}).get(prefix)
        w = vals.get("WRITE_SIZE", {}).get(prefix)
        if not f or not w:
            continue
        per = [a * fetch_cal + b * write_cal for a, b in zip(f, w)]
        r = {"kernel": name, "src_sha": source_sha(fname), "launches": len(per),
             "fetch_bytes_per_launch": sum(a * fetch_cal for a in f) / len(f),
             "write_bytes_per_launch": sum(b * write_cal for b in w) / len(w),
             "bytes_per_launch": sum(per) / len(per), "algorithmic_bytes_per_launch": K * bytes_el}
        fl = vals.get("SQ_INSTS_VALU_FLOPS_FP64", {}).get(prefix)
        if fl:
            r["flops_per_launch"] = sum(fl) / len(fl) * 64 * lanes
            r["valu_insts_per_launch"] = sum(vals["SQ_INSTS_VALU"][prefix]) / len(fl)
            r["waves_per_launch"] = sum(vals["SQ_WAVES"][prefix]) / len(fl)
            if flops_el is not None:
                r["algorithmic_flops_per_launch"] = K * flops_el
        out["kernels"][prefix] = r
    json.dump(out, open(COUNTER_FILE, "w"), indent=1)
    lines = ["# Per-kernel HBM traffic and FP64 work, blast-like state 1024x1024, N=4, k=3", "",
             "Counter runs (one Strang step each, on one MI355X):", ""]
    lines += ["    " + c for c in out["commands"]]
    lines += ["", "Calibration on the entry snapshot kernel, which copies the state (%d bytes): FETCH_SIZE x %.4f, "
              "WRITE_SIZE x %.4f." % (known, fetch_cal, write_cal), "",
              "| kernel | launches | measured GB/launch | algorithmic GB/launch | ratio | FP64 Gflop/launch (counter) |",
              "|---|---|---|---|---|---|"]
    for pre, r in out["kernels"].items():
        lines.append("| `%s` | %d | %.3f | %.3f | %.2f | %s |" % (
            pre.rstrip("<"), r["launches"], r["bytes_per_launch"] / 1e9, r["algorithmic_bytes_per_launch"] / 1e9,
            r["bytes_per_launch"] / r["algorithmic_bytes_per_launch"],
            "%.2f" % (r["flops_per_launch"] / 1e9) if "flops_per_launch" in r else "-"))
    lines += ["", "Source hashes (bench.source_sha): " + ", ".join(
        "%s %s" % (f, source_sha(f)) for f in ("hydro.hip", "magnetic.hip")) + "."]
    open(os.path.join(ROOT, "profiles", "kernel_counters_blast1024_N4.md"), "w").write("\n".join(lines) + "\n")
    return out


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


def valu_object(flops_alg, flops_ctr, avg_ms):
    """FP64 VALU view of a kernel: algorithmic and counter-measured TFLOP/s against the FP64
    vector peak (either may be None)."""
    t = avg_ms * 1e-3
    out = {"peak": FP64_PEAK_TFS, "unit": "TFLOP/s", "algorithmic": None, "algorithmic_frac": None,
           "counter": None, "counter_frac": None}
    if flops_alg is not None:
        out["algorithmic"] = flops_alg / t / 1e12
        out["algorithmic_frac"] = flops_alg / t / 1e12 / FP64_PEAK_TFS
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


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline():
    """The plain FP64 oracle, timed on this host: Strang steps of the same blast workload (same
    domain, N = 4, k = 3, full stabilisation) on a 128 x 128 sub-resolution mesh with all host
    threads, and one step on 32 x 32 with one thread."""
    import numpy as np

    import oracle as O
    from paper_2609_10849_amd import workloads as W

    def run(n, steps, threads):
        L, U, Bx, By, Bz = W.blast(n, n, 4, 3)
        M = O.Mesh(L.nx, L.ny, L.p, L.m, L.x0, L.x1, L.y0, L.y1, L.gamma)
        used = O.set_threads(threads)
        # the positivity-CFL step at CFL 0.3 of the initial state (fast speed sqrt(gamma p_in + |B|^2)
        # inside the blast, u = 0), as the GPU run takes it
        cf = (5.0 / 3.0 * 1000.0 + 1.0) ** 0.5
        dt = 0.3 / (9.0 * 2.0 * cf * n)
        t0 = time.perf_counter()
        st = (U, Bx, By, Bz)
        for _ in range(steps):
            st = O.strang_step(M, O.Options.full(), *st, dt)[:4]
        t = time.perf_counter() - t0
        return M.K * 25 * 9 * steps / t, t, used

    ncpu = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    rate, t, used = run(128, 6, ncpu)
    rate1, t1, _ = run(32, 1, 1)
    O.set_threads(ncpu)
    return {"value": rate, "unit": "DOF-stage updates/s", "cores": used, "kind": "oracle",
            "sample": "blast workload at 128x128 elements (N=4, k=3, full stabilisation), 6 Strang steps, "
                      "%.1f s on %d OpenMP threads" % (t, used),
            "cpu_model": cpu_model(), "host_cpus": ncpu,
            "one_thread": {"value": rate1, "sample": "blast workload at 32x32 elements, 1 Strang step, %.1f s" % t1}}


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


def adjoint_ratio_full(S, U, Bx, By, Bz, reps=10):
    """The same ratios on the timed workload itself (the blast-like state at 1024 x 1024, N = 4,
    k = 3, where neither operator is launch-bound); cotangents N(0,1) from torch's generator
    (seed 7), eta U[0, 1e-3]."""
    import torch

    gen = torch.Generator(device="cuda").manual_seed(7)
    cot = torch.randn(U.shape, dtype=U.dtype, device="cuda", generator=gen)
    out, gb = torch.empty_like(U), torch.empty_like(U)
    tf = _event_ms(lambda: S.rhs_hydro(U, out), reps)
    tb = _event_ms(lambda: S.rhs_hydro_vjp(U, cot, gb), reps)
    del cot, out, gb
    rho, e, u = S.to_primitive(U)
    eta = torch.rand(S.K, dtype=U.dtype, device="cuda", generator=gen) * 1e-3
    cots = [torch.randn(a.shape, dtype=U.dtype, device="cuda", generator=gen) for a in (e, u, Bx, By, Bz)]
    mf = _event_ms(lambda: S.rhs_magnetic(rho, u, Bx, By, Bz, eta), reps)
    mb = _event_ms(lambda: S.rhs_magnetic_vjp(rho, u, Bx, By, Bz, eta, *cots), reps)
    return {"hydro": tb / tf, "magnetic": mb / mf, "hydro_fwd_ms": tf, "hydro_vjp_ms": tb,
            "magnetic_fwd_ms": mf, "magnetic_vjp_ms": mb, "workload": "the timed blast-like state"}


def rejection_cost(S, U, Bx, By, Bz):
    """Cost of reject-and-halve on the timed workload: one hydro substep of the step's first half
    (tau = dt/2, dt from CFL 0.3) from the current state, at tau and then at 2^k tau (k = 4, 5, ...
    up to 12) until the positivity check refuses an attempt and the substep is bisected; each run
    starts from a copy of the state.  Reports the attempts, the bisection depth and the time per
    attempt of the plain and of the bisected substep."""
    import torch

    dt = S.cfl_dt(U, Bx, By, Bz, 0.3)
    W = torch.empty_like(U)

    def run(m):
        W.copy_(U)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        r, rep = S.hydro_substep(W, m * dt / 2)
        b.record()
        torch.cuda.synchronize()
        return {"multiple": m, "status": r, "ms": a.elapsed_time(b), "attempted": rep["substeps_attempted"],
                "accepted": rep["substeps_accepted"], "max_depth": rep["max_depth"]}

    plain = run(1)
    out = {"plain": plain, "ms_per_attempt_plain": plain["ms"] / max(plain["attempted"], 1), "bisected": None}
    for k in range(4, 13):
        o = run(2 ** k)
        if o["attempted"] > o["accepted"] or o["status"] != 0:
            out["bisected"] = o
            out["ms_per_attempt_bisected"] = o["ms"] / max(o["attempted"], 1)
            break
    return out


def batched_speedup(steps=50, only=None):
    """Ensemble of 64 uneven runs (n in {32..192}, N in {2,3,4}, k = N-1, vortex amplitude and
    field drawn from PCG64 seed 0; full stabilisation; per-run dt from CFL 0.3 at the start):
    time per Strang step of all runs for sequential plain launches, the run-table step (one launch
    per kernel and degree group over all runs) replayed from its HIP graph, the same launched
    plainly, and the per-run steps on concurrent branch streams.  value = sequential / graph."""
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
    g0 = [[dev(a) for a in st] for st in states]  # tiles and branch count by the event-timed autotuner (untimed)
    B.autotune(*[[x[i] for x in g0] for i in range(4)], dts)
    del g0

    def run(nsteps, sequential=False, streams=False, graph=False):
        B.graph(graph)
        g = [[dev(a) for a in st] for st in states]
        args = [[x[i] for x in g] for i in range(4)]
        B.strang_step(*args, dts, sequential=sequential, streams=streams)  # warm-up (plan, capture)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nsteps):
            r, _ = B.strang_step(*args, dts, sequential=sequential, streams=streams)
            if r != 0:
                raise RuntimeError("batch step failed: %d" % r)
        torch.cuda.synchronize()
        B.graph(False)
        return 1e3 * (time.perf_counter() - t0) / nsteps

    if only == "graph":
        tg = run(steps, graph=True)
        B.close()
        return {"graph_ms_per_step": tg}
    ts = run(steps, sequential=True)
    tg = run(steps, graph=True)
    te = run(steps)
    tb = run(steps, streams=True)
    B.close()
    nodes = sum(L.K * (L.p + 1) ** 2 for L in layouts)
    return {"value": ts / tg, "sequential_ms_per_step": ts, "graph_ms_per_step": tg, "run_table_ms_per_step": te,
            "run_table_speedup": ts / te, "streams_ms_per_step": tb, "streams_speedup": ts / tb,
            "runs": 64, "steps": steps, "nodes": nodes,
            "path": "run-table launches (one per kernel and degree group over all runs) replayed from a HIP graph; "
                    "autotuned stage tiles"}


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
                    help="time only the 64-run ensemble (batch steps against sequential launches); prints its own "
                         "JSON line")
    ap.add_argument("--ingest", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "VALU_DIR"),
                    help="write profiles/kernel_counters.json from three rocprofv3 --pmc output directories (no GPU)")
    ap.add_argument("--ensemble-graph-only", action="store_true",
                    help="time only the graph-replayed run-table batch step of the 64-run ensemble (for profiling)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="time only the forward operators and their VJPs on the timed workload (for profiling)")
    args = ap.parse_args()
    if args.ingest:
        out = ingest_counters(args.ingest)
        print(json.dumps({k: v["bytes_per_launch"] for k, v in out["kernels"].items()}))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2609_10849_amd as pk
    from paper_2609_10849_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.ensemble_only:
        print(json.dumps({"batched_speedup": batched_speedup(steps=args.steps)}), flush=True)
        return
    if args.ensemble_graph_only:
        print(json.dumps({"batched_graph": batched_speedup(steps=args.steps, only="graph")}), flush=True)
        return
    n, N, k = args.n, 4, 3
    L, U, Bx, By, Bz = W.blast(n, n, N, k)
    S = pk.Solver.from_layout(L, pk.Options.full(reduced_2d2v=int(args.reduced_2d2v)))
    g = [torch.from_numpy(a).to("cuda") for a in (U, Bx, By, Bz)]
    del U, Bx, By, Bz
    if args.adjoint_only:
        print(json.dumps({"adjoint_cost_ratio_full_size": adjoint_ratio_full(S, *g, reps=5)}), flush=True)
        return
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
    ms_per_step = 1e3 * t / args.steps
    value = K * nn * 9 / (t / args.steps)
    kernels = []
    for kid, name, prefix, fname, bytes_el, flops_el, lanes in kernel_table(N, k):
        launches, kms = S.timing_read(kid)
        if launches == 0:
            continue
        avg = kms / launches
        ach = K * bytes_el / (avg * 1e-3) / 1e9
        rec = counter_record(prefix, fname, K, N)
        tr = rec.get("bytes_per_launch") if rec else None
        o = {"kernel": name, "name": prefix.rstrip("<"), "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
             "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": tr, "avg_ms": avg,
             "launches_per_step": launches / args.steps, "ms_per_step": kms / args.steps,
             "share": kms / args.steps / ms_per_step,
             "algorithmic_bytes_per_launch": K * bytes_el,
             "traffic_achieved": traffic_rate(tr, avg)[0], "traffic_frac": traffic_rate(tr, avg)[1]}
        fl_ctr = rec.get("flops_per_launch") if rec else None
        if flops_el is not None or fl_ctr is not None:
            o["valu"] = valu_object(K * flops_el if flops_el is not None else None, fl_ctr, avg)
        kernels.append(o)
    kernels.sort(key=lambda o: -o["ms_per_step"])
    dominant = dict(kernels[0])
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
        "roofline": dominant,
        "roofline_kernels": kernels,
        "timed_kernels_ms_per_step": sum(o["ms_per_step"] for o in kernels),
        "accepted_substep_rate": accepted / max(attempted, 1),
    }
    if not args.no_extras and not args.reduced_2d2v:
        out["hydro_only"] = hydro_only(S, g, steps=min(args.steps, 10))
        out["reduced_2d2v"] = reduced_2d2v(S, g, steps=min(args.steps, 10))
        out["adjoint_cost_ratio"] = adjoint_ratio()
        out["adjoint_cost_ratio_full_size"] = adjoint_ratio_full(S, *g)
        out["rejection_cost"] = rejection_cost(S, *g)
        out["batched_speedup"] = batched_speedup(steps=min(args.steps, 20))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
