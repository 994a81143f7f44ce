"""The library's host code under the address and undefined-behaviour sanitizers.

engine.hip is built for the host only and linked with an emulation of the HIP
runtime and of the kernel launchers (tests/host_asan/hip_emul.cpp) in which
device memory is heap memory and a launch reads every descriptor of its table.
The driver (tests/host_asan/engine_driver.cpp) makes the calls of the serving
loop (pool admission, batches whose composition changes and repeats, scans
closed and opened between steps), of prepared batches and of checkpoints, and
runs two streams of which one defers its kernels, so that a descriptor table
rewritten by a call on the other stream before the deferred launches read it
is reported.  No GPU is used.
"""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SCRIPT = os.path.join(HERE, "host_asan", "build_and_run.sh")


@pytest.mark.skipif(not (os.path.exists("/opt/rocm/bin/hipcc") and os.path.exists(SCRIPT)),
                    reason="needs hipcc and the host harness sources")
def test_engine_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    r = subprocess.run(["bash", SCRIPT, str(tmp_path)], capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "0 emulation findings, 0 failed expectations" in out, out[-4000:]
