"""Host-side pieces of bench.py that need no GPU: the profiler-traffic lookup and the refusal of
more than one GPU."""
import hashlib
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_is_read_only_for_the_profiled_kernel_source(tmp_path):
    b = _bench()
    src = tmp_path / "k.hip"
    src.write_bytes(b"__global__ void k() {}\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()[:16]
    prof = tmp_path / "traffic.txt"
    prof.write_text("# header: with a colon\n"
                    f"raster.hip sha256[:16]: {sha}\n"
                    "stage1_fast_kernel<64, 4, false, false, 0> hbm bytes per launch: 12012658469\n")
    k = "stage1_fast_kernel<64, 4, false, false, 0>"
    assert b.read_traffic(k, str(prof), str(src)) == 12012658469
    assert b.read_traffic("other_kernel", str(prof), str(src)) is None
    src.write_bytes(b"__global__ void k() { /* changed */ }\n")
    assert b.read_traffic(k, str(prof), str(src)) is None
    assert b.read_traffic(k, str(tmp_path / "missing.txt"), str(src)) is None


def test_traffic_recorded_with_a_runtime_sha_needs_that_runtime(tmp_path):
    b = _bench()
    src, rt = tmp_path / "k.hip", tmp_path / "runtime.hip"
    src.write_bytes(b"__global__ void k() {}\n")
    rt.write_bytes(b"void launch() {}\n")
    sha = lambda p: hashlib.sha256(p.read_bytes()).hexdigest()[:16]
    prof = tmp_path / "traffic.txt"
    prof.write_text(f"raster.hip sha256[:16]: {sha(src)}\nruntime.hip sha256[:16]: {sha(rt)}\n"
                    "kern hbm bytes per launch: 77\n")
    assert b.read_traffic("kern", str(prof), str(src), runtime_path=str(rt)) == 77
    rt.write_bytes(b"void launch() { /* other launch options */ }\n")
    assert b.read_traffic("kern", str(prof), str(src), runtime_path=str(rt)) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "no multi-GPU path" in r.stderr
