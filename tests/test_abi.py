"""Host-side checks of the C-ABI library: it loads, exports every declared
function, and rejects bad arguments before touching the device."""
import ctypes
import subprocess

import pytest

from paper_1107_0538_amd import capi


def test_exports_every_header_function():
    lib = capi.load()
    names = capi.header_functions()
    assert "cg_create" in names and "cg_solve" in names and "spmv" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) <= set(capi.SIGNATURES), set(names) - set(capi.SIGNATURES)


def test_exports_are_c_symbols():
    out = subprocess.run(["nm", "-D", "--defined-only", capi.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    syms = {line.split()[-1] for line in out.splitlines() if line.strip()}
    probe = capi.header_functions(capi.PROBE_HEADER)
    assert probe == ["jpcg_stream_triad"]
    for n in capi.header_functions() + probe:
        assert n in syms, n
        assert n in capi.SIGNATURES, n


def test_strerror_and_null_arguments():
    lib = capi.load()
    assert lib.cg_strerror(capi.CG_EDIAG).decode().startswith("diagonal")
    assert lib.cg_strerror(12345).decode() == "unknown status"
    out = ctypes.c_void_p()
    assert lib.cg_create(None, None, None, ctypes.byref(out)) == capi.CG_EINVAL and not out.value
    csr = capi.cg_csr(0, capi.CG_MEM_HOST, 0, None, None, None)
    assert lib.cg_create(ctypes.byref(csr), None, None, ctypes.byref(out)) == capi.CG_EINVAL
    assert lib.cg_solve(None, None, None, 1e-10, 0, None) == capi.CG_EINVAL
    assert lib.spmv(None, None, None) == capi.CG_EINVAL
    lib.cg_destroy(None)
    assert lib.cg_last_error(None) == b""


def test_opts_default():
    o = capi.cg_opts()
    capi.load().cg_opts_default(ctypes.byref(o))
    assert o.precond == capi.CG_PRECOND_JACOBI and o.autotune == 0 and o.fp32_copy == 0


def test_load_fails_loudly_without_the_library(monkeypatch, tmp_path):
    # No CPU fallback: a missing library is an error, not a silent substitute.
    from paper_1107_0538_amd import capi

    monkeypatch.setattr(capi, "_lib", None)
    monkeypatch.setattr(capi, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        capi.load()


def test_struct_layouts_match_the_header(tmp_path):
    # The ctypes mirrors of cg_csr, cg_opts, cg_info and cg_config have the
    # header's size and field offsets (a C program compiled against
    # include/jpcg.h prints them).
    import os
    import shutil

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"cg_csr": capi.cg_csr, "cg_opts": capi.cg_opts, "cg_info": capi.cg_info, "cg_config": capi.cg_config}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "jpcg.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} . %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    include = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([cc, "-std=c99", "-I", include, str(src), "-o", str(exe)], check=True)
    out = [ln for ln in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n") if ln]
    assert len(out) == sum(1 + len(cls._fields_) for cls in structs.values())
    for line in out:
        name, field, value = line.split()
        cls = structs[name]
        got = ctypes.sizeof(cls) if field == "." else getattr(cls, field).offset
        assert got == int(value), (name, field, got, value)
