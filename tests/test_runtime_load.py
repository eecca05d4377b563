"""The library shares torch's HIP runtime: importing the binding must not
leave a second copy of the HIP runtime in the process (two runtimes each
start their own HSA runtime, and the second finds no device)."""
import os
import subprocess
import sys

import pytest


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_single_hip_runtime_after_import():
    pytest.importorskip("torch")
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import paper_2512_04389_amd\n"
        "import torch\n"
        "maps = open('/proc/self/maps').read().splitlines()\n"
        "libs = sorted({l.split()[-1] for l in maps if 'libamdhip64' in l})\n"
        "print('\\n'.join(libs))\n"
        "assert len(libs) == 1, libs\n" % (ROOT,))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
