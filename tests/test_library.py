"""The C-ABI library loads on the host and exports every function include/sai.h declares.

No compute call is made (there may be no GPU here).  The binding's ctypes structures
are checked against the C layout of the header.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sai.h")
LIB = os.path.join(ROOT, "paper_1211_6866_amd", "libsai.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(sai_[a-z0-9_]+)\s*\(", text))
    return sorted(n for n in names if not n.endswith("_fn"))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["sai_split", "sai_build", "sai_krylov", "sai_smw", "sai_solve", "sai_backward"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        from paper_1211_6866_amd import build
        build.build()
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    lib.sai_strerror.restype = ctypes.c_char_p
    assert lib.sai_strerror(0) == b"ok"


def test_tuning_knobs_host_only():
    # sai_tune_* touch no device: set, read back, environment override, clear,
    # rejected names
    if not os.path.exists(LIB):
        from paper_1211_6866_amd import build
        build.build()
    lib = ctypes.CDLL(LIB)
    lib.sai_tune_set.argtypes = [ctypes.c_char_p, ctypes.c_int32]
    lib.sai_tune_get.argtypes = [ctypes.c_char_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    v = ctypes.c_int32()
    assert lib.sai_tune_get(b"ZZ_TEST_KNOB", 7, ctypes.byref(v)) == 0 and v.value == 7
    assert lib.sai_tune_set(b"ZZ_TEST_KNOB", 3) == 0
    assert lib.sai_tune_get(b"ZZ_TEST_KNOB", 7, ctypes.byref(v)) == 0 and v.value == 3
    os.environ["SAI_TUNE_ZZ_TEST_KNOB"] = "5"
    try:
        assert lib.sai_tune_get(b"ZZ_TEST_KNOB", 7, ctypes.byref(v)) == 0 and v.value == 5
    finally:
        del os.environ["SAI_TUNE_ZZ_TEST_KNOB"]
    assert lib.sai_tune_clear() == 0
    assert lib.sai_tune_get(b"ZZ_TEST_KNOB", 7, ctypes.byref(v)) == 0 and v.value == 7
    for bad in [b"", b"lower", b"A" * 64, b"SP ACE"]:
        assert lib.sai_tune_set(bad, 1) == 1          # SAI_EINVAL
    assert lib.sai_tune_get(b"X", 0, None) == 1


def test_binding_structs_match_header(tmp_path):
    """The ctypes structures of the binding have the size and field offsets of
    the C structures in include/sai.h (compiled here with the host C compiler)."""
    import ctypes as C
    import shutil
    import subprocess
    import paper_1211_6866_amd as P
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    pairs = [("sai_allocator", P._Allocator), ("sai_split_opts", P.SplitOpts),
             ("sai_split_info", P.SplitInfo), ("sai_build_opts", P.BuildOpts),
             ("sai_build_stats", P.BuildStats), ("sai_precond_info", P.PrecondInfo),
             ("sai_solve_opts", P.SolveOpts), ("sai_solve_stats", P.SolveStats)]
    lines = ['#include <stdio.h>', '#include "sai.h"', "int main(void) {"]
    for cname, py in pairs:
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, *_ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    subprocess.run([cc, "-std=c99", "-I", os.path.join(root, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for ln in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        a, b, v = ln.split()
        got[(a, b)] = int(v)
    for cname, py in pairs:
        assert got[(cname, "size")] == C.sizeof(py), cname
        for fname, *_ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_binding_fails_loudly_without_library():
    """With no libsai.so the binding raises on first use: there is no CPU fallback."""
    import subprocess
    import sys
    code = ("import paper_1211_6866_amd as P\n"
            "P.LIB_PATH = '/nonexistent/libsai.so'\n"
            "try:\n"
            "    P.lib()\n"
            "except RuntimeError as e:\n"
            "    print('raised:', e)\n"
            "else:\n"
            "    raise SystemExit('the binding loaded without its library')\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "raised:" in r.stdout, (r.stdout, r.stderr)
