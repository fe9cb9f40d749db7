"""Host-side pieces of the benchmark contract (no GPU needed)."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    return b


def test_more_than_one_gpu_exits_with_a_message():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode != 0
    assert "one GPU" in res.stderr
    assert res.stdout.strip() == ""


def test_kernel_models_are_positive_and_bounded():
    b = load_bench()
    N, m, nnz = 256 ** 3, 60 * 384 * 256, 1318656524
    for name in ("project", "backproject", "tv", "trial", "extrapolate", "transpose"):
        for stored in (False, True):
            bound, amount, unit, peak = b.kernel_model(name, N, m, nnz, 4, stored)
            assert bound in ("hbm", "alu") and amount > 0 and peak > 0
            assert unit in ("GB/s", "TFLOP/s")
    # the stored product moves 8 bytes per non-zero plus r and the volume
    _, amount, _, _ = b.kernel_model("backproject", N, m, nnz, 4, True)
    assert amount == 8 * nnz + 4 * (m + N)


def test_measured_traffic_is_tied_to_the_kernel_text():
    b = load_bench()
    src = b.kernel_source(os.path.join(ROOT, b.MEASURED_TRAFFIC["source"]),
                          b.MEASURED_TRAFFIC["function"])
    assert src.startswith("constexpr int MB")
    assert "void spmv_voxels_block(" in src and src.rstrip().endswith("}")
    assert b.measured_traffic("project", True) is None
    assert b.measured_traffic("backproject", False) is None
