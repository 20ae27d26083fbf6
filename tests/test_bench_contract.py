"""Host-side checks of bench.py's contract and the surrogate driver's
bookkeeping (no GPU)."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_multi_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_only_for_matching_kernel_hash(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    # the committed counter summary is either current (a number) or stale (None)
    t = bench._traffic(1)
    assert t is None or t > 1e9


def test_summarize_records():
    sys.path.insert(0, ROOT)
    from paper_1003_4570_amd import surrogate as S
    recs = []
    for i in range(3):
        recs.append(dict(zero=dict(iterations=200 + i, seconds=16.0 + i, converged=True),
                         mean=dict(iterations=150, seconds=12.0, converged=True, fell_back=False, err0=0.5),
                         learned=dict(iterations=90, seconds=8.0, converged=True, fell_back=i == 2,
                                      err0=0.05),
                         zero_err0=2.5))
    s = S.summarize(recs)
    assert s["n"] == 3 and s["zero_iters"] == 201 and s["learned_iters"] == 90
    assert abs(s["speedup_time"] - 17.0 / 8.0) < 1e-12
    assert s["fallbacks"] == 1


def test_surrogate_init_weights_shape():
    sys.path.insert(0, ROOT)
    import workloads as W
    w = W.init_surrogate_weights(0)
    assert w.dtype == np.float32
    assert w.size == 32 * 27 + 32 + 2 * (32 * 32 * 27 + 32) + 32 * 27 + 1
