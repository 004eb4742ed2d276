"""Host-side checks of the C ABI: the library loads and exports every entry
point declared in include/symnmf.h, and the binding wraps each of them.
No compute call is made (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "symnmf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(symnmf_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("symnmf_create", "symnmf_lai", "symnmf_iterate", "symnmf_residual", "symnmf_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_2402_08134_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("libsymnmf.so not built")
    L = ctypes.CDLL(P.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    # the binding declares a signature for each and exposes a same-named wrapper
    for n in declared_functions():
        assert n in P._SIGS
        if n not in ("symnmf_last_error", "symnmf_mlp_last_error"):
            assert hasattr(P, n), n


def test_default_options_match_the_paper():
    import paper_2402_08134_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("libsymnmf.so not built")
    o = P.symnmf_default_options()
    assert o.struct_size == ctypes.sizeof(P.Options)
    assert o.stop_tol == 1e-4 and o.stop_patience == 4 and o.rule == P.RULE_HALS
    assert o.tau < 0  # tau = 1/s (Section 5.2)


def test_struct_layouts_match_header(tmp_path):
    """Every field offset and struct size of the binding equals what a C
    compiler makes of include/symnmf.h."""
    import shutil
    import subprocess
    import paper_2402_08134_amd as P
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"symnmf_matrix": P.Matrix, "symnmf_options": P.Options, "symnmf_stats": P.Stats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "symnmf.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_create_rejects_null_arguments_without_gpu():
    import paper_2402_08134_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("libsymnmf.so not built")
    L = P.lib()
    h = ctypes.c_void_p()
    assert L.symnmf_create(ctypes.byref(h), None, 4, 0.0, 0, 0, None, None) == P.E_INVALID
    assert b"null" in L.symnmf_last_error(None)
