"""The Python binding's ctypes structures have the C header's layout: a small C program compiled
with gcc against include/vstab.h prints every structure's size and field offsets (no GPU)."""
import ctypes as C
import os
import subprocess

import pytest

from paper_1701_03572_amd import vstab as V

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = [V.vs_pyramid, V.vs_detect_params, V.vs_lk_params, V.vs_fit_params, V.vs_fit_state, V.vs_fit_info,
           V.vs_rect, V.vs_smooth_params, V.vs_tuning, V.vs_stream]


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    d = tmp_path_factory.mktemp("layout")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "vstab.h"', "int main(void) {"]
    for st in STRUCTS:
        n = st.__name__
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (n, n))
        for f, _ in st._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (n, f, n, f))
    lines += ["return 0;", "}"]
    src, exe = d / "layout.c", d / "layout"
    src.write_text("\n".join(lines) + "\n")
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True)
    return {tuple(l.split()[:2]): int(l.split()[2]) for l in out.splitlines()}


@pytest.mark.parametrize("st", STRUCTS, ids=lambda s: s.__name__)
def test_struct_layout_matches_header(st, c_layout):
    assert C.sizeof(st) == c_layout[(st.__name__, "size")]
    for f, _ in st._fields_:
        assert getattr(st, f).offset == c_layout[(st.__name__, f)], f
