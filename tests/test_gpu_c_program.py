"""The C ABI from a plain C99 program on the GPU (tests/c/gpu_from_c.c): no
Python, no torch, device memory from hipMalloc and a stream of its own.  The
program runs kappa_sample in both precisions, a three-species plan (direct and
graph launches, compared bit for bit by the program itself) and
kappa_sample_backward, and dumps the outputs; here they are compared with the
oracle at the tolerances of the other parity tests.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from gpu_helpers import TOL_FP32, TOL_FP64, norm_rel_err
from paper_2602_05606_amd import _lib

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
N = 100003
SEGS = [(2.0, 1.0, (0.25, 0.0, 0.0), 40000, 0), (4.1, 0.7, (0.0, 0.0, 0.0), 1, 1),
        (10.0, 2.0, (0.0, -0.5, 0.125), 33333, 2)]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_c_program_on_the_gpu(orc, tmp_path):
    exe = tmp_path / "gpu_from_c"
    lib_dir = os.path.dirname(_lib.LIB_PATH)
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-isystem", os.path.join(ROCM, "include"), "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "c", "gpu_from_c.c"), "-L", lib_dir, "-lkappa", f"-Wl,-rpath,{lib_dir}",
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}", "-lm",
           "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    print("running the C program", flush=True)
    res = subprocess.run([str(exe), str(tmp_path)], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.startswith("ok")

    f32 = np.fromfile(tmp_path / "f32.bin", dtype=np.float32).astype(np.float64).reshape(3, N)
    ref = orc.sample(3.0, 1.0, N, 5, counter_offset=17, seg=3, mode=orc.MODE_FP32)
    assert norm_rel_err(tuple(f32), ref[:3]) <= TOL_FP32

    f64 = np.fromfile(tmp_path / "f64.bin", dtype=np.float64).reshape(3, N)
    ref = orc.sample(6.0, 0.5, N, 8, mode=orc.MODE_FP64)
    assert norm_rel_err(tuple(f64), ref[:3]) <= TOL_FP64

    total = sum(s[3] for s in SEGS)
    plan = np.fromfile(tmp_path / "plan.bin", dtype=np.float32).astype(np.float64).reshape(3, total)
    start = 0
    for kappa, theta, drift, count, seg in SEGS:
        r = orc.sample(kappa, theta, count, 4, seg=seg, mode=orc.MODE_FP32, drift=drift)
        got = plan[:, start:start + count]
        # drift can make a velocity small: errors relative to the drift-free speed plus |drift|
        d = np.sqrt(sum((got[c] - r[c]) ** 2 for c in range(3)))
        scale = np.sqrt(sum((r[c] - drift[c]) ** 2 for c in range(3))) + np.linalg.norm(drift)
        assert np.max(d / scale) <= TOL_FP32, seg
        start += count

    g = np.fromfile(tmp_path / "g.bin", dtype=np.float32).reshape(3, N)
    grad = np.fromfile(tmp_path / "grad.bin", dtype=np.float64)
    want = orc.backward(2.5, 1.3, N, 2, g[0], g[1], g[2], mode=orc.MODE_FP32)
    print(f"C program backward {grad} oracle {want}")
    for a, b in zip(grad, want):
        assert abs(a - b) <= 1e-4 * (abs(b) + np.sqrt(N) * 1e-3)
