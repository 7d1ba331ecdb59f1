"""The C ABI on its own: `tests/abi_c_caller.c`, a plain C program (gcc, the
library's header and the HIP runtime for device memory, no Python on its
path), draws the KL coefficients with the library's generator, runs 8
realizations of the 128 x 64 jet for 50 steps and writes the state; it must
equal the oracle's, bit for bit, with the same times and step counts."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle as O
from paper_2605_25282_amd import build, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def test_plain_c_caller_matches_the_oracle():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if shutil.which("gcc") is None or not os.path.exists(os.path.join(ROCM, "include", "hip", "hip_runtime_api.h")):
        pytest.skip("gcc or the HIP runtime headers are not available")
    if not os.path.exists(build.OUT):
        pytest.fail("the HIP library is not built")
    nx, ny, R, steps = 128, 64, 8, 50
    with tempfile.TemporaryDirectory() as d:
        exe, out = os.path.join(d, "abi_c_caller"), os.path.join(d, "state.bin")
        libdir = os.path.dirname(build.OUT)
        subprocess.run(["gcc", "-std=c99", "-O2", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include",
                        f"-I{os.path.join(ROOT, 'include')}", os.path.join(ROOT, "tests", "abi_c_caller.c"),
                        "-o", exe, f"-L{libdir}", "-lvlbm_hip", f"-L{ROCM}/lib", "-lamdhip64",
                        f"-Wl,-rpath,{libdir}", f"-Wl,-rpath,{ROCM}/lib"], check=True)
        print(f"abi_c_caller {nx} {ny} {R} {steps}", flush=True)
        r = subprocess.run([exe, str(nx), str(ny), str(R), str(steps), out], capture_output=True, text=True,
                           timeout=120)
        assert r.returncode == 0, r.stderr
        raw = np.fromfile(out, dtype=np.uint8)
    n = 20 * R * ny * nx
    state = raw[: 8 * n].view(np.float64).reshape(4, 5, R, ny, nx)
    t = raw[8 * n: 8 * n + 8 * R].view(np.float64)
    s = raw[8 * n + 8 * R:].view(np.int64)
    assert np.all(s == steps)
    w = inputs.WORKLOADS["jet128"]
    assert (w.nx, w.ny, w.dx, w.y_min) == (nx, ny, 1.0 / nx, -0.25)
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, R)
    ref, t_ref, n_ref, status = O.run_ensemble(O.Params(), O.Grid(nx, ny, w.dx, w.y_min), coefs, 1e30,
                                               max_steps=steps)
    assert np.all(status == O.OK) and np.all(n_ref == steps)
    assert np.array_equal(t, t_ref)
    for m in range(R):
        mine = state[:, :, m].transpose(1, 0, 2, 3).reshape(20, ny, nx)
        assert np.array_equal(mine, ref[m]), m
