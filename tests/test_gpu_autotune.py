"""Launch-shape tuning of the single-species path (kappa_sample_autotune), the
autotune cache policy (KAPPA_AUTOTUNE=off|use|refresh) and launch logging
(KAPPA_LOG).  Shapes never change the output, so every sample is compared bit
for bit with the default shape's.  Each case runs in a child process of its
own, because the policy and the tuned shapes are process-wide."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
N = (1 << 20) + 3  # size bucket 2^21

CHILD = r"""
import json, sys
import torch
sys.path.insert(0, sys.argv[1])
import paper_2602_05606_amd as kp
n = int(sys.argv[2])
tune = sys.argv[3] == "tune"
ref = [t.cpu() for t in kp.sample(2.5, 1.0, n, 7, precision=kp.FP32)]
shape = kp.sample_autotune(n, kp.FP32, reps=2) if tune else None
got = [t.cpu() for t in kp.sample(2.5, 1.0, n, 7, precision=kp.FP32)]
same = all(torch.equal(a.view(torch.int32), b.view(torch.int32)) for a, b in zip(ref, got))
print(json.dumps({"shape": shape, "same": same}), flush=True)
"""


def run_child(env_extra, tune):
    env = dict(os.environ)
    env.update(env_extra)
    print(f"child: {env_extra} tune={tune}", flush=True)
    res = subprocess.run([sys.executable, "-c", CHILD, ROOT, str(N), "tune" if tune else "plain"], env=env,
                         capture_output=True, text=True, timeout=240)
    assert res.returncode == 0, res.stderr[-2000:]
    out = json.loads(res.stdout.strip().splitlines()[-1])
    logs = [l for l in res.stderr.splitlines() if l.startswith("[kappa] forward_kernel")]
    return out, logs


def test_autotune_keeps_the_bits_and_records_the_shape(tmp_path):
    cache = tmp_path / "cache.json"
    out, logs = run_child({"KAPPA_AUTOTUNE_CACHE": str(cache), "KAPPA_LOG": "1"}, tune=True)
    b, u = out["shape"]
    assert b in (64, 128, 256) and u in (1, 2, 4, 8)
    assert out["same"]
    # the last launch (after tuning) used the tuned shape
    assert f"block={b} per_thread={u}" in logs[-1], logs[-3:]
    assert json.load(open(cache))["forward|mode1|n2^21"].startswith(f"{b},{u},")


@pytest.mark.parametrize("policy,expect", [("use", (64, 2)), ("off", (256, 4)), ("refresh", (256, 4))])
def test_cache_policy(tmp_path, policy, expect):
    cache = tmp_path / "cache.json"
    cache.write_text(json.dumps({"forward|mode1|n2^21": "64,2,0"}))
    out, logs = run_child({"KAPPA_AUTOTUNE_CACHE": str(cache), "KAPPA_LOG": "1", "KAPPA_AUTOTUNE": policy},
                          tune=False)
    assert out["same"]
    assert logs and all(f"block={expect[0]} per_thread={expect[1]}" in l for l in logs), logs[:2]
    # nothing was tuned, so the file is unchanged
    assert json.load(open(cache)) == {"forward|mode1|n2^21": "64,2,0"}
