"""Host-side checks of bench.py (no GPU): it refuses more than one GPU before
touching a device, and its workload tables describe the benchmarked shapes."""
import pathlib
import subprocess
import sys

ROOT = pathlib.Path(__file__).resolve().parents[1]
sys.path.insert(0, str(ROOT))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""                     # no JSON line for a refused run


def test_workload_tables():
    import bench
    c2, c3 = bench.WORKLOADS["c2"], bench.WORKLOADS["c3"]
    assert (c2["m"], c2["n"], c2["r"], c2["precision"]) == (10000, 10000, 20, 0)
    assert (c3["m"], c3["n"], c3["r"], c3["precision"]) == (50000, 50000, 50, 1)
    assert bench.BATCH["c4"]["njobs"] == 256
    names = [c[0] for c in bench.SERVE["c5"]["classes"]]
    assert names == ["A", "B", "C"]
    # every filter form the library reports has a name, a kernel and a counter key
    assert set(bench.FORM_NAMES) == set(bench.FORM_KERNELS) == set(bench.FORM_KEYS)
