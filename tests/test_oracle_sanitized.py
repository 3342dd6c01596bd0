"""The oracle built with the undefined-behaviour sanitizer, and built with
the address sanitizer (each aborting on the first report), runs the step,
the pair and cell queries, the profile, moving walls with specular
reflection, the attractive-repulsive force and the adjoint window on small
systems without a report."""
import os
import subprocess
import sys

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r'''
import numpy as np
import oracle, workloads
s = workloads.tiny_slab_system()
s.vel = (s.vel * 3).astype(np.float32)
o = oracle.Oracle(s)
o.step(15)
o.pairs(); o.cells(); o.profile(axis=2, nbins=7)
c = workloads.couette_system(U=1.0, specular=True, seed=52)
oc = oracle.Oracle(c)
oc.step(10)
p = workloads.tiny_slab_system(seed=14)
pp = dict(p.params); pp["sph"] = workloads.sph_force(); p.params = pp
op = oracle.Oracle(p)
op.step(10)
w = oracle.Oracle(workloads.tiny_slab_system(seed=15))
w.window(6)
print("ok")
'''


def test_oracle_under_undefined_behaviour_sanitizer(tmp_path):
    so = oracle.build_oracle(force=True, sanitize=True, path=str(tmp_path / "liboracle_ubsan.so"))
    env = dict(os.environ, DPD_ORACLE_LIB=so, OMP_NUM_THREADS="2",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", SCRIPT], env=env, cwd=ROOT, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr
    assert r.stdout.strip().endswith("ok")


def test_oracle_under_address_sanitizer(tmp_path):
    """Out-of-bounds and use-after-free accesses abort the run.  The Python
    process that loads the instrumented library preloads the gcc address
    sanitizer runtime; leak checking is off (the interpreter keeps its own
    allocations until exit)."""
    import shutil
    gcc = shutil.which("gcc")
    runtime = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True,
                             text=True).stdout.strip()
    if not runtime or not os.path.isabs(runtime) or not os.path.exists(runtime):
        import pytest
        pytest.skip("gcc's address sanitizer runtime is not installed")
    so = oracle.build_oracle(force=True, sanitize="address", path=str(tmp_path / "liboracle_asan.so"))
    env = dict(os.environ, DPD_ORACLE_LIB=so, OMP_NUM_THREADS="2", LD_PRELOAD=runtime,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-c", SCRIPT], env=env, cwd=ROOT, capture_output=True,
                       text=True, timeout=900)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "AddressSanitizer" not in r.stderr
    assert r.stdout.strip().endswith("ok")
