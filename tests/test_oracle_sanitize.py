"""The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): the small channel and the 480 x 60 workload run through it with
every out-of-bounds access, use after free, signed overflow or invalid shift
turned into a failure (-fno-sanitize-recover=all)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import numpy as np, oracle
from helpers import oracle_sim
from paper_2210_06043_amd import inputs
oracle.set_threads(2)
for cfg, steps in ((inputs.config_tiny(), 300), (inputs.config_c1(), 150),
                   (inputs.config_contact(), 50), (inputs.config_tiny(walls=0, kinds=(0, 2)), 50)):
    s = oracle_sim(cfg)
    s.step(steps)
    s.macro(); s.totals(); s.node_fields()
    for k in range(len(cfg.bodies)):
        s.body_diag(k); s.body_work(k); st = s.body_state(k)
        s.set_body_state(k, st["xy"], st["dxy_prev"], st["rigid"])
    for bd in cfg.bonds:
        s.set_bonds(bd.body, *s.bonds(bd.body))
    s.step(2)
oracle.membrane_forces(inputs.circle(16, 3.0, 5.0, 5.0), inputs.circle(16, 3.2, 5.0, 5.0), 1e-3, 1e-4, 1.0, 1 / 3)
oracle.relax_membrane(inputs.circle(16, 3.0, 5.0, 5.0), inputs.circle(16, 3.2, 5.0, 5.0), 1e-3, 1e-4, 1.0, 1 / 3, 1.0, 20)
print("SANITIZED_RUN_OK", flush=True)
"""


def test_oracle_under_address_and_ub_sanitizers():
    from oracle import build
    try:
        lib = build.build(sanitize=True)
    except (OSError, subprocess.CalledProcessError) as e:
        pytest.fail(f"sanitizer build failed: {e}")
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    assert os.path.isabs(asan) and os.path.exists(asan), "gcc has no AddressSanitizer runtime"
    env = dict(os.environ)
    env.update(ORACLE_LIB=lib, LD_PRELOAD=":".join(p for p in (asan, env.get("LD_PRELOAD", "")) if p),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
               PYTHONPATH=os.pathsep.join([ROOT, os.path.join(ROOT, "tests")]), OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    report = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0 and "SANITIZED_RUN_OK" in r.stdout, report
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, report
