"""The ctypes structures of the Python binding against the C header: every field at the same offset,
every structure of the same size (a C program built with gcc from include/ prints offsetof / sizeof)."""
import ctypes as C
import os
import shutil
import subprocess

import pytest

import paper_1702_05167_amd.hsc as H
import paper_1702_05167_amd.mlp as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PAIRS = [(H.Contact, "hsc_contact"), (H.TreeOpts, "hsc_tree_opts"), (H.TreeStats, "hsc_tree_stats"),
         (H.SolveOpts, "hsc_solve_opts"), (H.Outputs, "hsc_outputs"), (H.Grid, "hsc_grid"),
         (H.ScfOpts, "hsc_scf_opts"), (M.TrainOpts, "hsc_train_opts")]


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("gcc not available")
    d = tmp_path_factory.mktemp("abi")
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "hsc.h"', '#include "hsc_mlp.h"',
             'int main(void) {']
    for cls, cname in PAIRS:
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for name, _ in cls._fields_:
            lines.append(f'  printf("{cname} {name} %zu\\n", offsetof({cname}, {name}));')
    lines += ['  return 0;', '}']
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    return {(a, b): int(c) for a, b, c in (line.split() for line in out.strip().splitlines())}


@pytest.mark.parametrize("cls,cname", PAIRS, ids=[p[1] for p in PAIRS])
def test_ctypes_layout_matches_the_header(c_layout, cls, cname):
    assert C.sizeof(cls) == c_layout[(cname, "sizeof")]
    for name, _ in cls._fields_:
        assert getattr(cls, name).offset == c_layout[(cname, name)], name
