"""Host-side checks of the benchmark's bookkeeping: algorithmic bytes per update and the
code hash that ties counter summaries to kernel code."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402
from paper_2605_01774_amd import inputs as I  # noqa: E402


def test_bytes_per_update():
    """Every stored population read and written once, plus one read of each per-node field."""
    decay = I.fourier_decay(n=8, steps=1)
    assert bench.bytes_per_lup("f64", decay) == 2 * 19 * 8
    assert bench.bytes_per_lup("f32", decay) == 2 * 19 * 4
    assert bench.bytes_per_lup("bf16", decay) == 2 * 19 * 2
    assert bench.bytes_per_lup("fp16r", decay) == 2 * (4 + 18 * 2)
    porous = I.porous_spheres(n=8, steps=1)
    assert bench.bytes_per_lup("f32", porous) == 152 + 6 * 4             # tensor field
    assert bench.bytes_per_lup("f32", porous, phases=True) == 152 + 1    # material index
    assert bench.bytes_per_lup("f64", porous, phases=True) == 304 + 1
    assert bench.bytes_per_lup("bf16r", porous, phases=True) == 80 + 1
    field = I.variable_tensor_source(n=8, steps=1)
    assert bench.bytes_per_lup("f32", field) == 152 + (6 + 3 + 1) * 4
    assert bench.bytes_per_lup("f64", field) == 304 + (6 + 3 + 1) * 8


def test_code_hash_ignores_comments_only():
    a = "int f(int x) {\n    // twice\n    return 2 * x;  // doubled\n}\n"
    b = "int f(int x) {   return 2 * x;\n}"
    c = "int f(int x) { return 3 * x; }"
    assert bench.code_without_comments(a) == bench.code_without_comments(b)
    assert bench.code_without_comments(a) != bench.code_without_comments(c)


def test_q27_bytes_per_update():
    decay = I.fourier_decay(n=8, steps=1)
    old = bench.Q
    try:
        bench.Q = 27
        assert bench.bytes_per_lup("f32", decay) == 2 * 27 * 4
        assert bench.bytes_per_lup("bf16r", decay) == 2 * (4 + 26 * 2)
    finally:
        bench.Q = old


def test_more_than_one_gpu_is_refused():
    """bench.py measures one GPU; --gpus N > 1 exits with a message (before any GPU work)."""
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
