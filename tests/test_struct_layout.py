"""The ctypes mirrors in the binding match the C structs of include/dfa_spec.h:
a small C program built with the host compiler prints sizeof and every field's
offsetof, compared with ctypes.sizeof and the ctypes field offsets."""
import ctypes
import os
import shutil
import subprocess

import pytest

import paper_1210_5093_amd as dfa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = [dfa.dfa_info_t, dfa.dfa_match_opts_t, dfa.dfa_plan_info_t, dfa.dfa_result_t,
           dfa.dfa_server_done_t, dfa.dfa_server_opts_t, dfa.dfa_server_stats_t]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_ctypes_structs_match_the_header(tmp_path):
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "dfa_spec.h"', 'int main(void) {']
    for S in STRUCTS:
        name = S.__name__
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in S._fields_:
            lines.append(f'  printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src),
                           "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        name, key, val = line.split()
        got[(name, key)] = int(val)
    for S in STRUCTS:
        name = S.__name__
        assert got[(name, "size")] == ctypes.sizeof(S), name
        for f, _ in S._fields_:
            assert got[(name, f)] == getattr(S, f).offset, (name, f)
