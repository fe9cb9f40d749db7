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
            assert unit in ("GB/s", "TFLOP/s", "T lane-instr/s")
    # the stored product, in the gather model: one value of r per non-zero,
    # the volume written and its compulsory second pass (8 B per voxel)
    _, amount, _, _ = b.kernel_model("backproject", N, m, nnz, 4, True)
    assert amount == 4 * nnz + 8 * N
    # the projector against the issue rate: its vector instructions per step
    bound, amount, unit, peak = b.kernel_model("project", N, m, nnz, 4, True)
    assert bound == "alu" and amount == b.PROJECT_VALU_PER_STEP * nnz
    assert peak == 256 * 64 * 2.4e9


def test_measured_traffic_is_tied_to_the_kernel_text():
    """Each measured figure is reported only for the form it was measured on
    (the backprojector from the stored A^T or on the fly, the projector at
    its ray tile) and only while its sources hash to the measured text."""
    b = load_bench()
    forms = [(e["kernel"], e["stored"], e["tile"]) for e in b.MEASURED_TRAFFIC]
    assert forms and len(set(forms)) == len(forms)
    assert b.measured_traffic("tv", True) is None
    for e in b.MEASURED_TRAFFIC:
        assert e["bytes"] > 0 and len(e["sha256_prefix"]) == 16
        for p in e["sources"]:
            assert os.path.isfile(os.path.join(ROOT, p))
        stored = True if e["stored"] is None else e["stored"]
        current = b.sources_sha(e["sources"]).startswith(e["sha256_prefix"])
        got = b.measured_traffic(e["kernel"], stored, e["tile"])
        assert got == (round(e["bytes"] / 1e9, 3) if current else None)
        if e["tile"] is not None:
            assert b.measured_traffic(e["kernel"], stored, (3, 3)) is None
        if e["stored"] is not None and (e["kernel"], not e["stored"], e["tile"]) not in forms:
            assert b.measured_traffic(e["kernel"], not e["stored"], e["tile"]) is None
        saved = e["sha256_prefix"]
        try:
            e["sha256_prefix"] = "0" * 16
            assert b.measured_traffic(e["kernel"], stored, e["tile"]) is None
        finally:
            e["sha256_prefix"] = saved
