"""The core SVD's pair order, checked on the host: the schedule helpers that
the Jacobi kernel and the V replay share (`jac_slot`, `jac_level_steps`,
`jac_sweep_steps`, `jac_groups` in `csrc/small_body.hpp`) are compiled into a
small host program (`jacobi_order_check.hip`) that walks one sweep for every
width l <= 128: every pair met exactly once, the pairs of a step disjoint,
every pair in a slot below the rotation log's stride, the step count that of
jac_sweep_steps (at most 127). One-sided Jacobi converges for any cyclic
order that meets every pair once per sweep, so this is the property the
kernel relies on; the GPU tests check the SVD it produces.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1804_00462_amd", "csrc")


def _hipcc():
    for cand in ("/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    return None


def test_pair_order_meets_every_pair_once(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "jacobi_order_check")
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", CSRC, os.path.join(HERE, "jacobi_order_check.hip"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr
