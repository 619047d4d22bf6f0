"""bench.py on the CPU (no GPU): the multi-GPU request is refused with a message, the traffic
ratio is read from the committed counter summaries only while they match the kernel source, and
the algorithmic-byte model is the one the roofline divides by."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_traffic_ratio_comes_from_the_matching_profile(storage):
    b = _bench()
    r = b.traffic_ratio(storage)
    # the committed summaries were taken on the current kernel source
    assert r is not None and 1.0 < r < 1.3, r
    assert b.traffic_ratio("bf16") is None


def test_roofline_byte_model():
    from paper_1603_09493_amd import roofline as RL
    N, nnz = 1000, 20000
    full = RL.eval_bytes(N, nnz, 1, 4)
    sym = RL.eval_bytes(N, nnz, 1, 4, symmetric=True)
    half = RL.eval_bytes(N, nnz, 1, 4, symmetric=True, ps=2)
    rest = nnz * (8 + 7 * 4) + N * (12 + 2 * 4) + N * 4 * 35.5
    assert full == pytest.approx(4 * N * N + rest)
    assert sym == pytest.approx(4 * N * (N + 1) / 2 + rest)
    assert half == pytest.approx(2 * N * (N + 1) / 2 + rest)
