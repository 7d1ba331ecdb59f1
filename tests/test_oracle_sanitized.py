"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer:
the same source built with both sanitizers (gcc, host code only) runs a jet
ensemble in both storage modes, the periodic and zero-gradient boundary modes,
the limiter off and on, and the per-node helpers, in a child process; any
out-of-bounds access, use of freed memory or undefined operation aborts it."""
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "vlbm_oracle.c")

SCENARIO = r"""
import numpy as np
import oracle as O
from paper_2605_25282_amd import inputs
coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, 2)
for storage in ("fp64", "mixed"):
    for alpha in (0.0, 1.0 / 3.0):
        p = O.Params(alpha=alpha, storage=storage)
        g = O.Grid(37, 21, 1.0 / 37, -0.25)
        st, t, n, a, rc = O.run(p, g, O.init(p, g, coefs[0]), 1e30, max_steps=25)
        assert rc == O.OK and n == 25, (storage, alpha, rc, n)
for bc in ("periodic", "neumann"):
    for theta in ("limiter", "zero", "one"):
        p = O.Params(bc=bc, theta_mode=theta)
        g = O.Grid(24, 17, 1.0 / 24, 0.0)
        u = np.zeros((4, 17, 24))
        u[0] = 1.0 + 0.2 * np.sin(np.arange(24) * 0.7)[None, :]
        u[1] = 0.3 * u[0]
        u[3] = 2.5 + 0.5 * u[1] ** 2 / u[0]
        st = O.from_macroscopic(p, g, u)
        st, t, n, a, rc = O.run(p, g, st, 1e30, max_steps=15)
        assert rc == O.OK, (bc, theta, rc)
print("sanitized oracle ok")
"""


def _asan_runtime():
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_under_address_and_undefined_behaviour_sanitizers():
    asan = _asan_runtime()
    if shutil.which("gcc") is None or asan is None:
        pytest.skip("gcc with the AddressSanitizer runtime is not available")
    with tempfile.TemporaryDirectory() as d:
        lib = os.path.join(d, "libvlbm_oracle_san.so")
        subprocess.run(["gcc", "-O1", "-g", "-std=gnu99", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                        "-shared", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        "-fno-omit-frame-pointer", SRC, "-o", lib, "-lquadmath", "-lm"], check=True)
        env = dict(os.environ, ORACLE_LIB=lib, LD_PRELOAD=asan,
                   ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
                   PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
        r = subprocess.run([sys.executable, "-c", SCENARIO], cwd=ROOT, env=env, capture_output=True,
                           text=True, timeout=600)
    msg = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, msg
    assert "sanitized oracle ok" in r.stdout
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, msg
