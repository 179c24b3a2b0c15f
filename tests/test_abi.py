"""Host-side checks of the C ABI: the library builds, loads and exports every
symbol include/ddks.h declares; calls that need a device fail cleanly
without one.  CPU only (no compute calls)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ddks.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ddks_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2106_13706_amd import native
    if not os.path.exists(native.LIB_PATH):
        from paper_2106_13706_amd import build
        build.build(force=False)
    return native.load()


def test_exports_every_declared_symbol(lib):
    from paper_2106_13706_amd import native
    names = _declared()
    assert len(names) >= 12
    assert set(names) == set(native.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", native.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (ddks_[a-z0-9_]+)$", out, flags=re.M))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(lib, n)


def test_status_strings_and_version(lib):
    from paper_2106_13706_amd import native
    assert lib.ddks_status_string(0) == b"ok"
    assert lib.ddks_status_string(native.DDKS_E_NONFINITE) == b"non-finite input value"
    assert lib.ddks_status_string(12345) == b"unknown status"
    assert b"gfx950" in lib.ddks_version()


def test_null_arguments_rejected(lib):
    from paper_2106_13706_amd import native
    assert lib.ddks_create(None, None) == native.DDKS_E_INVALID_ARG
    assert lib.ddks_destroy(None) == 0
    r = native._Result()
    assert lib.ddks_distance(None, None, 1, None, 1, 2, 0, ctypes.byref(r), None) == \
        native.DDKS_E_INVALID_ARG
    assert lib.ddks_last_error(None) == b""


def test_create_without_device(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2106_13706_amd import native
    h = ctypes.c_void_p()
    assert lib.ddks_create(None, ctypes.byref(h)) == native.DDKS_E_NO_DEVICE
    with pytest.raises(native.DDKSError):
        native.Context()


def test_constants_match_header():
    """Every DDKS_ flag and status the binding defines has the header's value."""
    from paper_2106_13706_amd import native
    src = open(HEADER).read()
    defs = {m.group(1): int(m.group(2), 0)
            for m in re.finditer(r"#define (DDKS_[A-Z0-9_]+) (0x[0-9a-fA-F]+|-?[0-9]+)u?", src)}
    enum = {m.group(1): int(m.group(2))
            for m in re.finditer(r"\b(DDKS_E_[A-Z_]+|DDKS_OK)\s*=\s*(-?[0-9]+)", src)}
    defs.update(enum)
    names = [n for n in dir(native) if n.startswith("DDKS_")]
    assert len(names) >= 15
    for n in names:
        assert n in defs, n
        assert getattr(native, n) == defs[n], n


def test_struct_layouts_match_header(tmp_path):
    """Every ctypes mirror of a header struct has the C compiler's size and
    field offsets (a mismatch would silently corrupt results)."""
    import shutil
    from paper_2106_13706_amd import native
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    mirrors = {"ddks_options": native._Options, "ddks_result": native._Result,
               "ddks_request": native._Request, "ddks_serve_stats": native._ServeStats,
               "ddks_perm_summary": native._PermSummary, "ddks_profile": native._Profile}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ddks.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, py in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
