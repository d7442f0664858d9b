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
    for n in capi.header_functions():
        assert n in syms, n


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
