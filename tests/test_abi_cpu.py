"""CPU checks of the C-ABI library: it loads and exports every declared symbol."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sipo.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sipo_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for required in ("sipo_project", "sipo_backproject", "sipo_blur", "sipo_pdhg_solve"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2604_08997_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libsipo.so not built")
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (sipo_[a-z0-9_]+)\b", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    # the binding describes exactly the declared calls
    assert set(binding.SIGNATURES) == set(declared_functions())
    lib = binding.lib()
    assert lib.sipo_version().decode().startswith("sipo")


def test_binding_has_no_cpu_fallback(monkeypatch):
    from paper_2604_08997_amd import binding
    monkeypatch.setattr(binding, "LIB_PATH", "/nonexistent/libsipo.so")
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(binding.SipoError):
        binding.lib()


def test_binding_structures_match_the_header(tmp_path):
    # the ctypes mirrors of the ABI structures have the C layout: size and every field's offset, as a
    # C compiler lays the header out (a field added on one side only would shift all that follow)
    import ctypes as C
    from paper_2604_08997_amd import binding
    pairs = {"sipo_geometry": binding.Geometry, "sipo_psf": binding.Psf, "sipo_problem": binding.Problem,
             "sipo_pdhg_options": binding.PdhgOptions, "sipo_pdhg_result": binding.PdhgResult,
             "sipo_tuning": binding.Tuning, "sipo_resin": binding.Resin, "sipo_metrics": binding.Metrics}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sipo.h"', 'int main(void) {']
    for cname, py in pairs.items():
        lines.append(f'    printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'    printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ['    return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for ln in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        name, field, val = ln.split()
        got[(name, field)] = int(val)
    for cname, py in pairs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for field, _ in py._fields_:
            assert got[(cname, field)] == getattr(py, field).offset, (cname, field)
