"""Host logic (no GPU): bench.py's refusal of more than one GPU, the traffic
summary's counter scaling, the matching of a stored summary to the kernel
instance bench.py reports, and the package's refusal to run without a GPU or
without its library."""
import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _counter_csv(path, counter, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_traffic_summary_scaling(tmp_path):
    """Counters in KiB per dispatch, scaled by what the same counter reads for
    the probe's five 1 GiB copies; the largest block_sweep instance is the
    dominant one."""
    from paper_1605_02620_amd import profiling
    main = "void rsosk::block_sweep<8, 32, 8, 256, signed char, short, 0>(args)"
    fb = "void rsosk::block_sweep<8, 32, 8, 256, short, void, 0>(args)"
    copy = "__amd_rocclr_copyBuffer"
    gib_kib = float(1 << 20)
    # FETCH reads half the copy's bytes (scale 2), WRITE all of them (scale 1)
    _counter_csv(tmp_path / "f", "FETCH_SIZE",
                 [(copy, 10.0)] * 3 + [(copy, gib_kib / 2)] * 5 + [(main, 600000.0), (main, 700000.0), (fb, 4.0)])
    _counter_csv(tmp_path / "w", "WRITE_SIZE",
                 [(copy, gib_kib)] * 5 + [(main, 1000000.0), (fb, 2.0)])
    out = profiling.summarize_traffic(str(tmp_path / "f"), str(tmp_path / "w"))
    assert out["kernel"] == main
    assert abs(out["fetch_scale"] - 2.0) < 1e-12 and abs(out["write_scale"] - 1.0) < 1e-12
    assert out["fetch_bytes_per_launch"] == round(650000.0 * 1024 * 2)
    assert out["write_bytes_per_launch"] == round(1000000.0 * 1024)
    assert out["traffic_bytes_per_launch"] == out["fetch_bytes_per_launch"] + out["write_bytes_per_launch"]
    assert out["kernel_source_sha256_16"] == profiling.kernel_hash()


def test_traffic_lookup_matches_instance(monkeypatch):
    import bench
    from paper_1605_02620_amd import profiling
    stored = {}

    def fake(path):
        return stored.get(os.path.basename(path))

    monkeypatch.setattr(profiling, "current_traffic", fake)
    stored["block_sweep_traffic.json"] = {
        "kernel": "void rsosk::block_sweep<8, 32, 8, 256, signed char, short, 0>(rsosk::SurfDev*, int, int const*, int, int)",
        "traffic_bytes_per_launch": 11}
    stored["block_sweep16_traffic.json"] = {
        "kernel": "void rsosk::block_sweep16<8, 32, 8, 256, 0>(rsosk::SurfDev*, int, int const*, int, int)",
        "traffic_bytes_per_launch": 22}
    stored["block_sweep_dt_traffic.json"] = {
        "kernel": "void rsosk::block_sweep<8, 32, 8, 256, signed char, short, 1>(rsosk::SurfDev*, int, int const*, int, int)",
        "traffic_bytes_per_launch": 33}
    assert bench.kernel_instance(stored["block_sweep_traffic.json"]["kernel"]) == "block_sweep<8,32,8,256,int8,int16,0>"
    assert bench._traffic("block_sweep<8,32,8,256,int8,int16,0>", False) == 11
    assert bench._traffic("block_sweep16<8,32,8,256,0>", True) == 22
    assert bench._traffic("block_sweep<8,32,8,256,int8,int16,1>", False, "double") == 33
    # another shape, staging type or schedule is never reported
    assert bench._traffic("block_sweep<8,32,8,192,int8,int16,0>", False) is None
    assert bench._traffic("block_sweep<8,32,8,256,int16,void,0>", False) is None
    assert bench._traffic("block_sweep<8,32,8,256,int8,int16,0>", False, "double") is None
    stored["block_sweep_traffic.json"]["kernel"] = stored["block_sweep_dt_traffic.json"]["kernel"]
    assert bench._traffic("block_sweep<8,32,8,256,int8,int16,0>", False) is None


def test_committed_summaries_describe_current_source():
    """The committed traffic summaries were taken from the current kernel
    source (otherwise bench.py reports traffic as null)."""
    from paper_1605_02620_amd import profiling
    for name in ("block_sweep_traffic.json", "block_sweep16_traffic.json", "block_sweep_dt_traffic.json"):
        d = json.load(open(os.path.join(ROOT, "profiles", name)))
        assert d["kernel_source_sha256_16"] == profiling.kernel_hash(), name
        assert profiling.current_traffic(os.path.join(ROOT, "profiles", name)) is not None


def test_no_cpu_fallback():
    """Without a GPU every entry of the Python package refuses to run, and
    without the built library the binding raises instead of computing."""
    import pytest
    import torch
    import paper_1605_02620_amd as pkg
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1605_02620_amd import serve
    for make in (lambda: pkg.Surface(64, N=1, D=8), lambda: pkg.Batch([(64, 1, 1)], D=8),
                 lambda: pkg.MultiSurface(16, N=1, seed=1, groups=1), lambda: serve.Engine(1 << 20)):
        with pytest.raises(RuntimeError, match="no CPU fallback"):
            make()
    code = ("import os; os.environ['RSOS_LIBRARY'] = '/nonexistent/librsos.so'\n"
            "from paper_1605_02620_amd import _lib\n"
            "try:\n    _lib.lib()\nexcept ImportError as e:\n    print('refused:', e)\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 0 and r.stdout.startswith("refused:"), (r.stdout, r.stderr)
