"""Host-only check that every entry point's planning pass sizes the workspace
its executing pass uses (tests/plan_check.hip: all library sources in one
translation unit, every launch recorded or dropped, fake device addresses).
An executing pass that takes more than its plan writes past the end of the
caller's workspace, into whatever the allocator placed after it, or faults
the GPU.  No GPU is needed; hipcc builds the checker (about 30 s, cached by
the sources' digest)."""

import hashlib
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1804_07531_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "plan_check.hip")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _digest():
    h = hashlib.sha256()
    files = [SRC] + sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC))
    files.append(os.path.join(ROOT, "include", "rsvd.h"))
    for f in files:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


@pytest.fixture(scope="module")
def checker():
    if not (os.path.exists(HIPCC) or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    bdir = os.path.join(ROOT, "paper_1804_07531_amd", "_build")
    os.makedirs(bdir, exist_ok=True)
    exe = os.path.join(bdir, f"plan_check_{_digest()}")
    if not os.path.exists(exe):
        cmd = [HIPCC, "--offload-arch=gfx950", "-O0", "-std=c++20", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", SRC, "-o", exe + ".tmp"]
        res = subprocess.run(cmd, capture_output=True, text=True)
        assert res.returncode == 0, res.stderr[-4000:]
        os.replace(exe + ".tmp", exe)
    return exe


def test_planning_pass_covers_executing_pass(checker):
    res = subprocess.run([checker], capture_output=True, text=True, timeout=300)
    bad = [line for line in res.stdout.splitlines() if "OVERFLOW" in line or "ERROR" in line or "status:" in line]
    assert res.returncode == 0 and not bad, "\n".join(bad[:20]) + "\n" + res.stdout[-400:]
    assert "0 failed" in res.stdout.splitlines()[-1]
