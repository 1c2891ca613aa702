"""bench.py's command line (CPU): more than one GPU is refused with a message
before anything touches a device, and the default step counts are those the
measurement notes quote."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_default_step_counts():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert r.returncode == 0 and "--workload" in r.stdout
    sys.path.insert(0, ROOT)
    import bench
    args = bench.build_parser().parse_args([])
    assert args.steps == 20 and args.warmup == 5 and args.gpus == 1 and args.workload == "room"
