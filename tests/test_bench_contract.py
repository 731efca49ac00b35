"""bench.py's contract on the CPU: more than one GPU is refused with a message, and the roofline
bytes of the hydro stage kernel and of the stage map follow from the state sizes."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)


def test_multi_gpu_request_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_stage_bytes():
    import bench
    K, nn = 1024 * 1024, 25
    u = 5 * K * nn * 8  # one conservative state
    # stage 1 reads U^n and writes the raw stage; stages 2 and 3 read U_s and U^n and write
    assert bench.stage_bytes(K, nn) == (2 * u + 3 * u + 3 * u) / 3.0 + 15 * 8 * K
    assert abs(bench.stage_bytes(K, nn) - 2.922e9) < 1e6


def test_oe_pp_bytes():
    import bench
    K, nn = 1024 * 1024, 25
    u = 5 * K * nn * 8
    # U* read and U^(s) written on every launch, the primitive copy on one launch in six
    assert bench.oe_pp_bytes(K, nn) == 2 * u + u / 6.0 + K * 49
    assert abs(bench.oe_pp_bytes(K, nn) - 2.3233e9) < 1e6


def test_algorithmic_flop_counts():
    import bench
    K = 1024 * 1024
    # N = 4: 25 nodes, 100 EC pairs, 10 own and 20 lifted face points per element
    assert bench.stage_flops(K, 5) == K * (20 * 25 + 74 * 100 + 50 * 10 + 15 * 20 + 25 * 25 + 20 * 25)
    assert bench.stage_flops(K, 5) / K == 9825
    assert bench.oe_pp_flops(K, 5) / K == 12095
    v = bench.valu_object(bench.stage_flops(K, 5), None, 1.0)
    assert abs(v["algorithmic"] - 9825 * K / 1e-3 / 1e12) < 1e-9 and v["counter"] is None


def test_traffic_rate():
    import bench
    assert bench.traffic_rate(None, 1.0) == (None, None)
    r, f = bench.traffic_rate(4e9, 1.0)  # 4 GB in 1 ms
    assert abs(r - 4000.0) < 1e-9 and abs(f - 0.5) < 1e-12


def test_counter_records_apply_only_to_their_workload():
    import bench
    for prefix, fname in (("k_hydro_stage<", "hydro.hip"), ("k_hydro_oe_pp<", "hydro.hip"), ("k_vel_proj<", "magnetic.hip")):
        # a record is never attached to another mesh size or degree
        assert bench.counter_record(prefix, fname, 64 * 64, 4) is None
        assert bench.counter_record(prefix, fname, 1024 * 1024, 3) is None


def test_kernel_hashes():
    import bench
    h, g = bench.source_sha("hydro.hip"), bench.source_sha("magnetic.hip")
    assert len(h) == 16 and int(h, 16) >= 0 and len(g) == 16 and g != h
    assert bench.source_sha("hydro.hip") == h


def test_velocity_oe_bytes():
    import bench
    # N = 4: the basis table holds 25 rows of 25 values, each row padded to 26
    t = {r[2]: r for r in bench.kernel_table(4, 3)}
    assert t["k_vel_prep<"][4] == 25 * 8 + 25 * 26 * 8
    assert t["k_vel_proj<"][4] == 25 * 26 * 8 + 3 * 25 * 8 + 2 * 25 * 8 + 5 * 8 + 4 * 25 * 8
