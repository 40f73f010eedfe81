"""The host tree builder (csrc/tree.cpp) under the address and undefined-behaviour sanitizers:
tests/native/tree_driver.cpp drives its C ABI through valid trees of every kind (geometric, graph,
whole-face, custom, merged, forests; bonds and exports) and malformed inputs that must be refused,
built with g++ for the host only (no GPU code is involved)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_tree_builder_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    exe = tmp_path / "tree_driver"
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", os.path.join(HERE, "native", "tree_driver.cpp"),
           os.path.join(ROOT, "paper_1702_05167_amd", "csrc", "tree.cpp"), "-o", str(exe)]
    build = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert build.returncode == 0, build.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0 and run.stdout.strip().endswith("ok"), (run.stdout[-3000:], run.stderr[-3000:])
