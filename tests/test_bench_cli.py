"""The benchmark script parses and keeps its command-line contract on the
CPU (no device work): it compiles, prints the kernel-source hash, and refuses
more than one GPU with a message."""
import os
import py_compile
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def test_bench_compiles():
    py_compile.compile(BENCH, doraise=True)


def test_bench_source_hash():
    import json
    out = subprocess.run([sys.executable, BENCH, "--source-hash"], capture_output=True, text=True, check=True)
    hashes = json.loads(out.stdout)
    assert set(hashes) == {"pair_phase_kernel", "pair_qp_batch_kernel"}
    assert all(len(v) == 16 for v in hashes.values())


def test_bench_refuses_several_gpus():
    out = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True)
    assert out.returncode == 2
    assert "one GPU" in out.stderr
