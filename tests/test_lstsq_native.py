"""The host least-squares routine behind Anderson mixing (paper_1702_05167_amd/csrc/lstsq.h), built
with g++ and AddressSanitizer for the host only, against numpy.linalg.lstsq: full-rank cases of the
sizes the self-consistent loop uses, and the cases it must report as dependent (a repeated or zero
column, more columns than rows) so that the loop restarts its history there as the oracle does."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path_factory.mktemp("lstsq") / "lstsq_driver"
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(HERE, "native", "lstsq_driver.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True)
    return exe


def _run(exe, cases):
    text = []
    for A, b in cases:
        n, m = A.shape
        text.append(f"{n} {m}")
        text.append(" ".join(repr(float(v)) for v in A.T.ravel()))
        text.append(" ".join(repr(float(v)) for v in b))
    out = subprocess.run([str(exe)], input="\n".join(text) + "\n", capture_output=True, text=True, check=True)
    return out.stdout.strip().splitlines()


def test_full_rank_cases_match_numpy(driver):
    rng = np.random.default_rng(11)
    cases = []
    for n, m in ((3, 1), (5, 3), (40, 4), (36, 16), (2000, 8), (7, 7)):
        cases.append((rng.normal(size=(n, m)) * np.exp(rng.normal(size=m)), rng.normal(size=n)))
    lines = _run(driver, cases)
    assert len(lines) == len(cases)
    for (A, b), line in zip(cases, lines):
        words = line.split()
        assert words[0] == "ok", line
        g = np.array([float(w) for w in words[1:]])
        ref = np.linalg.lstsq(A, b, rcond=None)[0]
        assert np.abs(g - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max())


def test_dependent_cases_are_reported(driver):
    rng = np.random.default_rng(12)
    A = rng.normal(size=(10, 3))
    rep = np.column_stack([A, A[:, 1]])              # a repeated column
    zero = np.column_stack([A, np.zeros(10)])         # a zero column
    near = np.column_stack([A, A[:, 0] + 1e-15 * rng.normal(size=10)])   # dependent to rounding
    wide = rng.normal(size=(3, 4))                    # more columns than rows
    b = rng.normal(size=10)
    lines = _run(driver, [(rep, b), (zero, b), (near, b), (wide, b[:3])])
    assert lines == ["dependent"] * 4
