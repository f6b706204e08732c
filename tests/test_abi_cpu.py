"""CPU-side checks of the C ABI boundary (no GPU calls).

* the shared library loads and exports every function include/signfn.h declares;
* the ctypes mirrors of the ABI structs have the header's sizes and offsets
  (checked against a C program compiled from the header with gcc).
"""
import ctypes as C
import os
import re
import subprocess

import pytest

import paper_2210_03356_amd as sf
from paper_2210_03356_amd import signfn as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "signfn.h")


def _declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"SIGNFN_API\s+[\w\s\*]+?\b(sign_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("sign_ns", "sign_newton", "sign_serve_submit", "sign_serve_poll"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = sf.load()
    out = subprocess.run(["nm", "-D", "--defined-only", sf.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (\w+)", out))
    for name in _declared_functions():
        assert name in exported, name
        assert hasattr(lib, name)
    # nothing but the ABI is exported as a function symbol
    assert {e for e in exported if e.startswith("sign_")} == set(_declared_functions())


STRUCTS = {
    "sign_csr": B.sign_csr,
    "sign_opts": B.sign_opts,
    "sign_stats": B.sign_stats,
    "sign_iter_stats": B.sign_iter_stats,
    "sign_server_opts": B.sign_server_opts,
    "sign_server_stats": B.sign_server_stats,
}


def test_struct_layouts_match_header(tmp_path):
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"',
             'int main(void) {']
    for name, cls in STRUCTS.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'printf("{name}.{field} %zu\\n", offsetof({name}, {field}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", str(src), "-o", str(exe)], check=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True,
                                                        text=True, check=True).stdout.split("\n")
               if l)
    for name, cls in STRUCTS.items():
        assert int(got[f"{name} size"]) == C.sizeof(cls), name
        for field, _ in cls._fields_:
            assert int(got[f"{name}.{field}"]) == getattr(cls, field).offset, (name, field)


def test_default_options_match_header_comments():
    o = sf.default_opts()
    assert o.tol == 1e-12 and o.stop_rule == 0 and o.c_fixed == 1e-4 and o.switch_res == 1e-6
    assert o.max_iter == 100 and o.precision == 0 and o.polish_steps == 2
    assert o.filter_y == 0 and o.scale == 0.0 and o.staging_bytes == 0


def test_invalid_options_rejected_without_gpu_work():
    """Option checks run before any device call, so they are testable here."""
    lib = sf.load()
    o = sf.default_opts(tol=-1.0)
    out = C.c_void_p()
    a = B.sign_csr(n=4, nnz=0, row_ptr=None, col=None, val=None, val_f32=0)
    st = lib.sign_ns(C.byref(a), C.byref(o), None, C.byref(out))
    assert st == -1 and out.value is None
    assert b"tol" in lib.sign_last_error()
    o = sf.default_opts(precision=3)
    assert lib.sign_ns(C.byref(a), C.byref(o), None, C.byref(out)) == -1
    assert b"precision" in lib.sign_last_error()


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(RuntimeError, match="missing"):
        B.load()


def test_noalloc_entry_point_allocates_nothing_and_checks_its_limit():
    """sign_filter_noalloc's object code references no device allocator, its row
    limit matches the header, and an oversized input is rejected on the host."""
    from paper_2210_03356_amd import build as bld
    obj = os.path.join(bld.BUILD, "noalloc.hip.o")
    if not os.path.exists(obj):
        bld.build()
    undef = subprocess.run(["nm", "-u", "-C", obj], capture_output=True, text=True,
                           check=True).stdout
    for name in ("hipMalloc", "hipFree", "hipMallocAsync", "hipExtMallocWithFlags",
                 "hipHostMalloc", "hipMallocManaged", "Pool", "Allocator", "DevBuf"):
        assert name not in undef, name
    assert "hipGetSymbolAddress" in undef
    m = re.search(r"#define SIGN_NOALLOC_MAX_ROWS (\d+)", open(HEADER).read())
    assert m and int(m.group(1)) == sf.NOALLOC_MAX_ROWS
    lib = sf.load()
    a = B.sign_csr(n=sf.NOALLOC_MAX_ROWS + 1, nnz=0, row_ptr=None, col=None, val=None, val_f32=0)
    o = B.sign_csr()
    st = lib.sign_filter_noalloc(C.byref(a), 1e-3, None, C.byref(o), 0, None, None)
    assert st == -1
    assert b"row limit" in lib.sign_last_error()
