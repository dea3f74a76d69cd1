"""The C ABI without a GPU: the library loads, exports every function include/rebk.h declares,
and host-side argument validation answers before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "rebk.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rebk_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_interface():
    names = declared_functions()
    for required in ("rebk_create", "rebk_solve", "rebk_solve_ex", "rebk_destroy", "rebk_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2001_04179_amd import _native
    lib = _native.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(_native.SIGNATURES)


def test_version_and_error_strings():
    from paper_2001_04179_amd import _native
    lib = _native.load()
    assert lib.rebk_version().decode().startswith("rebk")
    assert isinstance(lib.rebk_last_error(), bytes)


def test_host_validation_without_device():
    from paper_2001_04179_amd import _native as N
    lib = N.load()
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    ro = (ctypes.c_int64 * 3)(0, 5, 10)
    co = (ctypes.c_int64 * 2)(0, 4)
    bad_ro = (ctypes.c_int64 * 3)(0, 7, 5)
    # NULL A
    assert lib.rebk_create(ctypes.byref(h), None, 0, 0, 10, 4, 4, ro, 2, co, 1, 1.0, 0, None) == N.ERR_INVALID
    # non-increasing offsets
    assert lib.rebk_create(ctypes.byref(h), fake, 0, 0, 10, 4, 4, bad_ro, 2, co, 1, 1.0, 0, None) == N.ERR_INVALID
    assert "increasing" in lib.rebk_last_error().decode() or "end at" in lib.rebk_last_error().decode()
    # alpha <= 0, unknown dtype, lda < n
    assert lib.rebk_create(ctypes.byref(h), fake, 0, 0, 10, 4, 4, ro, 2, co, 1, 0.0, 0, None) == N.ERR_INVALID
    assert lib.rebk_create(ctypes.byref(h), fake, 0, 9, 10, 4, 4, ro, 2, co, 1, 1.0, 0, None) == N.ERR_INVALID
    assert lib.rebk_create(ctypes.byref(h), fake, 0, 0, 10, 4, 3, ro, 2, co, 1, 1.0, 0, None) == N.ERR_INVALID
    assert lib.rebk_create(ctypes.byref(h), fake, 2, 0, 10, 4, 4, ro, 2, co, 1, 1.0, 0, None) == N.ERR_INVALID
    # NULL handle everywhere
    assert lib.rebk_solve_ex(None, None, None) == N.ERR_INVALID
    assert lib.rebk_solve_ex_static(None, None, None) == N.ERR_INVALID
    assert lib.rebk_get_weights(None, None, None) == N.ERR_INVALID
    ms = ctypes.c_double(-1.0)
    assert lib.rebk_pipe_prepare(None, ctypes.byref(ms)) == N.ERR_INVALID and ms.value == 0.0
    lib.rebk_pipe_release(None)
    lib.rebk_destroy(None)


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    from paper_2001_04179_amd import _native
    monkeypatch.setattr(_native, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(_native, "_lib", None)
    with pytest.raises(_native.NativeLibraryMissing):
        _native.load()


def test_ctypes_structs_match_the_header(tmp_path):
    """Sizes and field offsets of the option and result structs, as the C compiler lays them out
    from the header, equal those of the binding's ctypes mirrors."""
    import ctypes
    import shutil
    import subprocess

    from paper_2001_04179_amd import _native as N

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"rebk_solve_opts_t": N.SolveOpts, "rebk_result_t": N.Result, "rebk_refine_opts_t": N.RefineOpts,
               "rebk_batch_opts_t": N.BatchOpts, "rebk_batch_rhs_t": N.BatchRhs}
    lines = ["#include <stddef.h>", "#include <stdio.h>", "#include \"rebk.h\"", "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        cname, field, val = line.split()
        got[(cname, field)] = int(val)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
