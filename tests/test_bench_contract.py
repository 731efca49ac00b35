"""bench.py's contract on the CPU: more than one GPU is refused with a message, and the roofline
bytes of the hydro stage kernel follow from the state sizes."""
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


def test_kernel_hash_covers_only_the_stage_kernel():
    import bench
    h = bench.kernel_sha()
    assert len(h) == 16 and int(h, 16) >= 0
