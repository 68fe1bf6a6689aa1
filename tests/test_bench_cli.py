"""bench.py's command-line contract on the CPU: one GPU only (N > 1 exits with a message and status 2
before touching a GPU), and the pass accounting behind `value` (every pass over A counts m n 8 bytes:
the sketch, one residual pass per step, one per inner iteration and one per sketched-KW check)."""

import json
import os
import subprocess
import sys
import types

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_pass_accounting():
    sys.path.insert(0, ROOT)
    import bench

    info = types.SimpleNamespace(iters=[6, 1], kw_evals=1)
    # sketch + 2 step heads + 7 iterations + 1 KW check
    assert bench.passes_of(info) == 11
    info = types.SimpleNamespace(iters=[11, 16], kw_evals=4)
    assert bench.passes_of(info) == 1 + 2 + 27 + 4
