"""CPU-side checks of the C ABI: the library loads, exports every entry point that
include/mdot.h declares, and the ctypes mirrors of the public structs match the C layout
(checked by compiling the header with gcc). No compute call is made here."""
from __future__ import annotations

import ctypes as ct
import os
import re
import subprocess

import pytest

from paper_2307_08507_amd import mdot as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mdot.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mdot_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert "mdot_solve" in names and "mdot_lse2" in names and "mdot_round_certify" in names
    lib = ct.CDLL(M.LIB_PATH)
    missing = [f for f in names if not hasattr(lib, f)]
    assert not missing, missing


def test_version_string():
    assert "gfx950" in M.version()


def test_struct_layouts_match_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "mdot.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu\\n\", sizeof(mdot_cost_desc), sizeof(mdot_params),"
        " sizeof(mdot_result), offsetof(mdot_params, max_sweeps), offsetof(mdot_result, pncg_iters),"
        " offsetof(mdot_cost_desc, data)); return 0;}\n"
    )
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = list(map(int, subprocess.check_output([str(exe)]).split()))
    want = [ct.sizeof(M.CostDesc), ct.sizeof(M.Params), ct.sizeof(M.Result), M.Params.max_sweeps.offset,
            M.Result.pncg_iters.offset, M.CostDesc.data.offset]
    assert got == want


def test_default_params_match_paper():
    p = M.default_params()
    assert p.p == 1.5 and p.gamma_i == 16.0
    assert p.q == pytest.approx(2 ** (1 / 3), rel=1e-15)
    assert p.gamma_f == 0.0 and p.precision == M.PREC_F32


def test_null_context_is_rejected():
    assert M.lib().mdot_solve(None, None, None, None, 1e-6, None, None, None, None) == -1
    assert M.lib().mdot_ctx_create(0, None, 0, None) == -1
