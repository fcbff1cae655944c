"""Failure paths and run-time facilities that need no GPU: the on-disk
code-object cache (compile check of host-only models), a forced compile
error (EXA_ECOMPILE, the handle stays usable), the device-memory budget
(EXA_ENOMEM) and the EXA_LOG lines.  Each case runs in a fresh Python
process, since the library reads its environment switches there."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PRELUDE = f"""
import json, os, sys, time
sys.path.insert(0, {ROOT!r})
import numpy as np
from exa_modeling.generators import acopf, kernel_sweep
from paper_2608_16265_amd import ExaModel, ExaError
"""


def run(code, env=None, timeout=600):
    e = dict(os.environ)
    e.update(env or {})
    r = subprocess.run([sys.executable, "-c", PRELUDE + code], capture_output=True, text=True, env=e,
                       timeout=timeout)
    assert r.returncode == 0, r.stdout + r.stderr
    return r


def last_json(r):
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_code_object_cache_roundtrip(tmp_path):
    d = str(tmp_path / "cache")
    os.makedirs(d)
    code = f"""
w = kernel_sweep(2, 64, 0)
em = ExaModel(w.model, host_only=True, cache_dir={d!r})
t0 = time.perf_counter(); em.compile_check(); t1 = time.perf_counter()
print(json.dumps(dict(ms=(t1 - t0) * 1e3, files=sorted(os.listdir({d!r})))))
"""
    first = last_json(run(code))
    assert any(f.endswith(".hsaco") for f in first["files"]) and any(f.endswith(".hip") for f in first["files"])
    second = last_json(run(code))          # a new process: read from the cache
    assert second["files"] == first["files"]
    assert second["ms"] < 0.25 * first["ms"], (first, second)
    # a corrupted stored source is not trusted: the code is compiled again
    src = [f for f in first["files"] if f.endswith(".hip")][0]
    with open(os.path.join(d, src), "a") as fh:
        fh.write("// changed\n")
    third = last_json(run(code))
    assert third["ms"] > 0.25 * first["ms"]
    # the environment variable names the cache when the option does not
    d2 = str(tmp_path / "env_cache")
    os.makedirs(d2)
    run(f"""
em = ExaModel(kernel_sweep(2, 64, 0).model, host_only=True)
em.compile_check()
print(json.dumps(sorted(os.listdir({d2!r}))))
""", env={"EXA_CACHE_DIR": d2})
    assert any(f.endswith(".hsaco") for f in os.listdir(d2))


def test_unwritable_cache_only_costs_the_compilation(tmp_path):
    r = run("""
em = ExaModel(kernel_sweep(1, 16, 0).model, host_only=True, cache_dir="/proc/no-such-dir")
em.compile_check()
print("ok")
""", env={"EXA_LOG": "1"})
    assert "cannot write" in r.stderr


def test_forced_compile_error_keeps_the_handle():
    r = run("""
from paper_2608_16265_amd import _lib
em = ExaModel(acopf(30, 0).model, host_only=True)
os.environ["EXA_TEST_BAD_SOURCE"] = "1"
try:
    em.compile_check()
    raise SystemExit("expected EXA_ECOMPILE")
except ExaError as e:
    assert e.code == _lib.EXA_ECOMPILE, e
    assert "does not compile" in str(e) or "error" in str(e).lower(), e
del os.environ["EXA_TEST_BAD_SOURCE"]
em.compile_check()               # the same handle, now fine
print(em.nnzj, em.jac_structure()[0].size)
""")
    assert r.stdout.split()[-2:] == ["1160", "1160"]


def test_device_memory_budget():
    r = run("""
from paper_2608_16265_amd import _lib
w = acopf(300, 1)
em = ExaModel(w.model, host_only=True)
need = em.device_bytes()
assert need > 8 * (em.nnzj + em.nnzh), need
try:
    ExaModel(w.model, host_only=True, max_device_bytes=need // 2)
    raise SystemExit("expected EXA_ENOMEM")
except ExaError as e:
    assert e.code == _lib.EXA_ENOMEM and "budget" in str(e), e
ok = ExaModel(w.model, host_only=True, max_device_bytes=need)
try:
    ExaModel(w.model, host_only=True, max_device_bytes=-1)
    raise SystemExit("expected EXA_EINVAL")
except ExaError as e:
    assert e.code == _lib.EXA_EINVAL
print(json.dumps(dict(need=need, info=ok.build_info())))
""")
    out = last_json(r)
    assert out["info"]["origin"] == "host_only" and out["info"]["device_bytes"] == out["need"]


def test_log_lines():
    r = run("""
em = ExaModel(acopf(30, 0).model, host_only=True)
print("built")
""", env={"EXA_LOG": "1"})
    assert "[exa] create: 13 patterns" in r.stderr and "host only" in r.stderr
    quiet = run("""
em = ExaModel(acopf(30, 0).model, host_only=True)
""", env={"EXA_LOG": "0"})
    assert "[exa]" not in quiet.stderr
