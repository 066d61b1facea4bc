"""CPU-side checks of the C ABI: the library loads, exports every declared
symbol, and the binding's struct layouts match the header (no compute calls)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2011_02107_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dacp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dacp_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = binding.load_library()
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    # the binding declares exactly the header's functions
    assert set(binding.SIGNATURES) == set(names)


def test_version_string():
    assert binding.load_library().dacp_version().decode().startswith("dacp-mi355x")


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "dacp.h"\n'
        "int main(void){\n"
        'printf("%zu %zu %zu %zu %zu\\n", sizeof(dacp_term), sizeof(dacp_filter_params), sizeof(dacp_basis_params),'
        " sizeof(dacp_opts), sizeof(dacp_report));\n"
        'printf("%zu %zu %zu\\n", offsetof(dacp_opts, seed), offsetof(dacp_report, evol_steps), offsetof(dacp_report, max_err_est));\n'
        "return 0;}\n"
    )
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    sizes = list(map(int, out))
    from paper_2011_02107_amd.inputs import TERM_DTYPE

    assert sizes[0] == TERM_DTYPE.itemsize == 16
    assert sizes[1] == ctypes.sizeof(binding.FilterParams)
    assert sizes[2] == ctypes.sizeof(binding.BasisParams)
    assert sizes[3] == ctypes.sizeof(binding.Opts)
    assert sizes[4] == ctypes.sizeof(binding.Report)
    assert sizes[5] == binding.Opts.seed.offset
    assert sizes[6] == binding.Report.evol_steps.offset
    assert sizes[7] == binding.Report.max_err_est.offset


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(binding, "_lib", None)
    monkeypatch.setattr(binding, "LIB_PATH", "/nonexistent/libdacp.so")
    with pytest.raises(RuntimeError, match="no fallback"):
        binding.load_library()


def test_default_opts_from_library():
    o = binding.default_opts()
    assert o.kfac == 18.0 and o.eps == 1e-12 and o.tol_rel == 1e-10
