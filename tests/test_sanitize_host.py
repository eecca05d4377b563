"""The host analysis (ordering, symbolic fill, Algorithms 2-3, the plan and
its threaded parts) built with the address and undefined-behaviour
sanitizers, and separately with the thread sanitizer, then run on grids,
random, bordered block-diagonal and stacked systems in every ordering with
one and eight host threads (tests/sanitize/analyze_harness.cpp).  Host code
only: g++ builds it, no GPU code is involved."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2512_04389_amd", "csrc")
SOURCES = [os.path.join(ROOT, "tests", "sanitize", "analyze_harness.cpp"), os.path.join(CSRC, "analyze.cpp"),
           os.path.join(CSRC, "nd_graph.cpp")]


def _slu_default_options_stub(tmp):
    # slu_default_options lives in the C ABI file (with the HIP runtime);
    # the harness gets the same defaults from this stub
    src = os.path.join(tmp, "defaults.cpp")
    with open(src, "w") as fh:
        fh.write('#include <cstring>\n#include "slu.h"\n'
                 'extern "C" void slu_default_options(slu_options *o) {\n'
                 '  std::memset(o, 0, sizeof(*o)); o->sample_points = 1000; o->step = 2; o->max_num = 3;\n'
                 '  o->advance = 1; o->blocking = SLU_BLOCK_IRREGULAR; o->ordering = SLU_ORDER_NATURAL; }\n')
    return src


@pytest.mark.parametrize("flags", [["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"],
                                   ["-fsanitize=thread"]], ids=["asan-ubsan", "tsan"])
def test_host_analysis_under_sanitizers(flags, tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = str(tmp_path / "harness")
    cmd = [gxx, "-O1", "-g", "-std=c++17", "-pthread", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC] + flags + \
        SOURCES + [_slu_default_options_stub(str(tmp_path)), "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", TSAN_OPTIONS="halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert run.returncode == 0 and run.stdout.strip().endswith("ok"), (run.stdout[-2000:], run.stderr[-4000:])
