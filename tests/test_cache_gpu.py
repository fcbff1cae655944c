"""The on-disk code-object cache across processes on the GPU: a second
process builds the same pattern set from the cache (no compilation) and
evaluates it bit for bit like the first; the device footprint estimate
bounds what a model really allocates."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = """
import hashlib, json, sys, time
sys.path.insert(0, {root!r})
import numpy as np, torch
from exa_modeling.generators import kernel_sweep
from paper_2608_16265_amd import ExaModel
w = kernel_sweep(8, 5000, 1)
t0 = time.perf_counter()
em = ExaModel(w.model, cache_dir={d!r})
create_ms = (time.perf_counter() - t0) * 1e3
x = torch.as_tensor(w.x, device="cuda:0")
y = torch.as_tensor(w.y, device="cuda:0")
h = em.hess_coord(x, y, 1.0).cpu().numpy()
j = em.jac_coord(x).cpu().numpy()
print(json.dumps(dict(create_ms=create_ms, info=em.build_info(),
                      digest=hashlib.sha256(h.tobytes() + j.tobytes()).hexdigest())))
"""


def test_second_process_loads_from_cache(tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = str(tmp_path)
    outs = []
    for _ in range(2):
        print("child process", len(outs), flush=True)
        r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, d=d)], capture_output=True, text=True,
                           timeout=240)
        assert r.returncode == 0, r.stderr[-3000:]
        outs.append(json.loads(r.stdout.strip().splitlines()[-1]))
    first, second = outs
    print(json.dumps(outs))
    assert first["info"]["origin"] == "compiled" and second["info"]["origin"] == "cache"
    assert second["info"]["compile_ms"] < 0.2 * first["info"]["compile_ms"]
    assert second["create_ms"] < first["create_ms"]
    assert first["digest"] == second["digest"]


def test_device_bytes_estimate_bounds_allocation():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from exa_modeling.generators import acopf, pde
    from paper_2608_16265_amd import ExaModel
    for w in (acopf(2000, 3), pde(120, 1)):
        est = ExaModel(w.model, host_only=True).device_bytes()
        em = ExaModel(w.model, max_device_bytes=est)  # the budget admits what the estimate says
        assert 0 < em.device_bytes() <= est, (em.device_bytes(), est)
        em.close()
