"""The entry points in one fresh process, in the order a harness may use them.

The package's library loaded before anything imports torch (as build()
does) must still reach the GPU in smoke(): msgfem.load() imports torch
first so that the library binds to the HIP runtime torch loads.
"""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_load_library_first_then_smoke():
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2211_13893_amd import msgfem\n"
            "msgfem.load()\n"
            "import __graft_entry__ as g\n"
            "g.smoke()\n") % ROOT
    print("[entry] fresh process: msgfem.load(), then smoke()", flush=True)
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0
    assert "smoke ok" in r.stdout
