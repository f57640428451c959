"""The C ABI driven from plain host code, without Python or torch
(paper_2305_09910_amd/examples/abi_tgv.cpp): a 32^3 Taylor-Green vortex
whose workspace and fields come from hipMalloc.  The program checks mass to
1e-7 relative and the amplitude decay exp(-2 nu k^2 t) to 1% itself and
exits non-zero otherwise."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_2305_09910_amd", "examples", "abi_tgv")


def test_c_abi_from_host_code():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(EXE):
        from paper_2305_09910_amd import build
        build.build()
    print("[case] examples/abi_tgv (32^3 Taylor-Green through the C ABI)", flush=True)
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stdout + r.stderr
    fields = r.stdout.split()
    assert fields[0] == "mass" and abs(float(fields[1]) / 32 ** 3 - 1) < 1e-7
