"""bench.py's command-line contract that needs no GPU: more than one GPU is
refused with a message (there is no multi-GPU path), and so are forms or legs
that a restricted workload has no kernel for, before anything touches a
device."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


@pytest.mark.parametrize("config,args,message", [
    ("mid12", ["--forms", "fp64,bf16x2", "--no-phonon", "--no-adjoint"], "no 16-bit instance at 12 orbitals"),
    ("mid12", ["--forms", "fp64,fp32"], "--no-phonon --no-adjoint"),
    ("direct5", ["--no-phonon", "--no-adjoint"], "fp64 only"),
    ("direct5", ["--forms", "fp64"], "--no-phonon --no-adjoint"),
])
def test_restricted_workloads_refuse_what_they_have_no_kernel_for(config, args, message):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--config", config] + args,
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 1
    assert message in r.stderr and r.stdout.strip() == ""
