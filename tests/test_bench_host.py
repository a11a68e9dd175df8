"""Host logic of bench.py (no GPU): the autotune-cache lookup per split format and the
traffic summary of rocprofv3 counter files."""
import json
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_tuned_batch_per_format(tmp_path):
    """A cache line matches only its own precision and slice counts; the last matching line wins;
    a line without n_slices_adjoint stands for the forward's count; FP64 lines carry no slices."""
    p = tmp_path / "cache.jsonl"
    lines = [
        {"o": 2, "v": 3, "n": 4, "precision": 1, "n_slices": 5, "flags": 0, "n_abatch": 3},
        {"o": 2, "v": 3, "n": 4, "precision": 1, "n_slices": 5, "n_slices_adjoint": 4, "flags": 0, "n_abatch": 2},
        {"o": 2, "v": 3, "n": 4, "precision": 2, "n_slices": 6, "n_slices_adjoint": 5, "flags": 0, "n_abatch": 1},
        {"o": 2, "v": 3, "n": 4, "precision": 0, "n_slices": 0, "flags": 0, "n_abatch": 3},
        {"o": 2, "v": 3, "n": 4, "precision": 2, "n_slices": 6, "n_slices_adjoint": 5, "flags": 0, "n_abatch": 2},
    ]
    p.write_text("\n".join(json.dumps(d) for d in lines) + "\nnot json\n")
    assert bench.tuned_batch(str(p), 2, 3, 4, 1, 5, 0) == 3           # 5 / 5 (no adjoint field)
    assert bench.tuned_batch(str(p), 2, 3, 4, 1, 5, 0, 4) == 2        # 5 / 4
    assert bench.tuned_batch(str(p), 2, 3, 4, 2, 6, 0, 5) == 2        # INT8 6 / 5, the last line wins
    assert bench.tuned_batch(str(p), 2, 3, 4, 2, 5, 0, 5) is None     # no INT8 5 / 5 line
    assert bench.tuned_batch(str(p), 2, 3, 4, 0, 0, 0) == 3           # FP64
    assert bench.tuned_batch(str(p), 2, 3, 4, 1, 5, 2, 4) is None     # other flags
    assert bench.tuned_batch(str(tmp_path / "missing.jsonl"), 2, 3, 4, 1, 5, 0) is None


def test_committed_cache_has_the_benchmark_configurations():
    """The committed cache holds the retinal batch sizes of both split formats at the benchmark's
    slice counts and of the FP64 path."""
    o, v, n, _ = bench.WORKLOADS["retinal"]
    for prec, (sf, sa) in (("int8", bench.DEFAULT_SLICES["int8"]), ("bf16", bench.DEFAULT_SLICES["bf16"])):
        assert bench.tuned_batch(bench.TUNED_CACHE, o, v, n, bench.PREC_CODE[prec], sf, 0, sa)
    assert bench.tuned_batch(bench.TUNED_CACHE, o, v, n, 0, 0, 0)


def _counter_csv(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w") as fh:
        fh.write('"Dispatch_Id","Kernel_Name","Counter_Name","Counter_Value"\n')
        for i, (name, counter, value) in enumerate(rows):
            fh.write('%d,"%s","%s",%r\n' % (i, name, counter, value))


def test_traffic_summary(tmp_path):
    """Counter files of two passes -> bytes per launch of each split GEMM stage, each counter
    scaled by what it reads for the 1 GiB copy; the record carries the source hash and batch size
    that bench.py checks before it reports the value."""
    fetch, write = tmp_path / "fetch", tmp_path / "write"
    gf = "void ladder::gemm_i8_kernel<5, ladder::EpiStrided, 4>(ladder::SplitShape, ladder::EpiStrided)"
    gb = "void ladder::gemm_i8_kernel<6, ladder::EpiSwapMid, 0>(ladder::SplitShape, ladder::EpiSwapMid)"
    copy = "__amd_rocclr_copyBuffer"
    _counter_csv(fetch, [(copy, "FETCH_SIZE", 524288.0), (copy, "FETCH_SIZE", 1.0), (gf, "FETCH_SIZE", 100.0),
                         (gf, "FETCH_SIZE", 300.0), (gb, "FETCH_SIZE", 50.0)])
    _counter_csv(write, [(copy, "WRITE_SIZE", 1048576.0), (gf, "WRITE_SIZE", 10.0), (gf, "WRITE_SIZE", 30.0),
                         (gb, "WRITE_SIZE", 5.0)])
    out = os.path.join(ROOT, "profiles", "traffic_tiny_int8_pm.json")
    try:
        res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "tiny", "--n-abatch", "3",
                              "--traffic-summary", str(fetch), str(write)], capture_output=True, text=True, cwd=ROOT)
        assert res.returncode == 0, res.stderr
        rec = json.load(open(out))
    finally:
        if os.path.exists(out):
            os.remove(out)
    assert rec["fetch_factor"] == 2.0 and rec["write_factor"] == 1.0
    assert rec["n_abatch"] == 3 and rec["precision"] == "int8" and rec["sources_sha256_16"] == bench.gemm_source_hash()
    assert rec["kernels"]["gemm_f"]["bytes"] == pytest.approx((200.0 * 2.0 + 20.0) * 1024)
    assert rec["kernels"]["gemm_b"]["bytes"] == pytest.approx((50.0 * 2.0 + 5.0) * 1024)
    assert rec["kernels"]["gemm_f"]["slices"] == 5 and rec["kernels"]["gemm_b"]["slices"] == 6
    assert "gemm_i8_kernel<5" in res.stdout
