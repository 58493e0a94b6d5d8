"""The workspace plan covers every launch (host only, no GPU): a C++ audit
(layout_audit.cpp) links the library's own sizing code and checks, over a sweep
of particle counts, boxes (down to three cells), mode counts and skins, that
each buffer the kernels index holds the largest index their launch shapes
reach on every cell grid a system can use -- including the finer grid that a
hot system's default skin drops to at its first step -- and that each fine
grid's 5 x 5 x 5 stencil covers its list radius.  Where no GPU is visible it
also checks that every launcher refuses, on the host and before any launch,
arguments a kernel cannot run on (a missing buffer, a grid of fewer than six
cells, a structure-factor group beyond the staging area, ...): without a device
an unrefused launch returns hipErrorNoDevice, not hipErrorInvalidValue, so a
missing check fails the audit."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2501_10946_amd")


@pytest.fixture(scope="module")
def audit_exe(tmp_path_factory):
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    if not hipcc:
        pytest.skip("hipcc not available")
    lib = os.path.join(PKG, "librbsog.so")
    if not os.path.exists(lib):
        pytest.skip("librbsog.so is not built")
    exe = str(tmp_path_factory.mktemp("audit") / "layout_audit")
    subprocess.run([hipcc, "-O1", "-std=c++17", "--offload-arch=gfx950", "-Wno-unused-result",
                    f"-I{os.path.join(ROOT, 'include')}", f"-I{os.path.join(PKG, 'csrc')}",
                    os.path.join(ROOT, "tests", "layout_audit.cpp"), "-o", exe, f"-L{PKG}", "-lrbsog",
                    f"-Wl,-rpath,{PKG}"], check=True, capture_output=True)
    return exe


def test_workspace_plan_covers_every_launch(audit_exe):
    r = subprocess.run([audit_exe], capture_output=True, text=True, timeout=300)
    print(r.stdout[-2000:])
    assert r.returncode == 0, r.stdout[-4000:]
    assert "0 failures" in r.stdout
    assert "launch guards checked" in r.stdout or "a GPU is visible" in r.stdout
