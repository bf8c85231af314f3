"""The C ABI: libofks.so loads and exports every entry point include/ofks.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ofks.h")
LIB = os.path.join(ROOT, "paper_2007_14228_amd", "libofks.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ofks_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("ofks_create", "ofks_assemble", "ofks_csr_load", "ofks_set_params", "ofks_set_x0",
                 "ofks_step", "ofks_energy", "ofks_residual", "ofks_postprocess", "ofks_spmm", "ofks_gram",
                 "ofks_precondition", "ofks_build_hamiltonian"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libofks.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libofks.so not built")
def test_binding_signatures_cover_the_header():
    from paper_2007_14228_amd import _lib
    bound = {s[0] for s in _lib.SIGNATURES}
    assert set(declared()) <= bound


@pytest.mark.skipif(not os.path.exists(LIB), reason="libofks.so not built")
def test_default_params_without_a_device():
    from paper_2007_14228_amd import _lib
    lib = _lib.load()
    p = _lib.Params()
    lib.ofks_default_params(ctypes.byref(p))
    assert p.beta == 1.0 and p.tol == 1e-8 and p.max_iter == 1000 and p.occupation == 2.0
    assert p.precond == _lib.PRECOND["paper"] and p.step_rule == _lib.STEP["bb2"]



def test_struct_layouts_match_the_c_compiler(tmp_path):
    """ctypes mirrors of ofks_params / ofks_iter_stats have the C sizes and offsets."""
    import shutil
    import subprocess
    from paper_2007_14228_amd import _lib
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    fields_p = [f for f, _ in _lib.Params._fields_]
    fields_s = [f for f, _ in _lib.IterStats._fields_]
    src = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', 'int main(void){',
           'printf("%zu %zu\\n", sizeof(ofks_params), sizeof(ofks_iter_stats));']
    for f in fields_p:
        src.append(f'printf("%zu\\n", offsetof(ofks_params, {f}));')
    for f in fields_s:
        src.append(f'printf("%zu\\n", offsetof(ofks_iter_stats, {f}));')
    src.append("return 0;}")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", str(c), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split()
    vals = [int(x) for x in out]
    assert vals[0] == ctypes.sizeof(_lib.Params) and vals[1] == ctypes.sizeof(_lib.IterStats)
    want = [getattr(_lib.Params, f).offset for f in fields_p] + [getattr(_lib.IterStats, f).offset for f in fields_s]
    assert vals[2:] == want
