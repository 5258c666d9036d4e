"""The C-ABI library loads and exports every symbol include/svar.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "svar.h")
LIB = os.path.join(ROOT, "paper_2105_06975_amd", "libsvar.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(svar_[A-Za-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("svar_create", "svar_destroy", "svar_apply_A", "svar_apply_P", "svar_solve",
                 "svar_last_error", "svar_apply_op"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsvar.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsvar.so not built")
def test_binding_struct_sizes_match_header_layout():
    """The ctypes mirrors have the sizes the C compiler gives the structs (checked with a
    host-only compile of the header)."""
    import shutil
    import subprocess
    import tempfile

    from paper_2105_06975_amd import svar as sv
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = r'''
#include <stdio.h>
#include "svar.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(svar_model_desc),
         sizeof(svar_window_desc), sizeof(svar_prec_opts), sizeof(svar_solve_opts),
         sizeof(svar_solve_info), sizeof(svar_net_desc), sizeof(svar_adam_opts),
         sizeof(svar_train_opts));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.check_call([cc, "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        sizes = [int(x) for x in subprocess.check_output([exe]).split()]
    assert sizes == [ctypes.sizeof(sv.ModelDesc), ctypes.sizeof(sv.WindowDesc),
                     ctypes.sizeof(sv.PrecOpts), ctypes.sizeof(sv.SolveOpts),
                     ctypes.sizeof(sv.SolveInfo), ctypes.sizeof(sv.NetDesc),
                     ctypes.sizeof(sv.AdamOpts), ctypes.sizeof(sv.TrainOpts)]


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsvar.so not built")
def test_errors_without_device_calls():
    """Argument validation runs on the host and reports through svar_last_error."""
    from paper_2105_06975_amd import svar as sv
    lib = sv.lib()
    h = ctypes.c_void_p()
    rc = lib.svar_create(None, 0, None, ctypes.byref(h), None)
    assert rc == sv.E_INVAL
    assert b"window" in lib.svar_last_error()
    assert lib.svar_system_size(None, 0) == -1
    # network argument checks (no device call before validation)
    n = ctypes.c_void_p()
    d = sv.NetDesc(3, 40, 1, 0)  # 1 + 40 + 3 > 32 input channels
    assert lib.svar_net_create(ctypes.byref(d), ctypes.byref(n)) == sv.E_INVAL
    assert b"n_bound" in lib.svar_last_error()
    assert lib.svar_net_nparams(None) == -1
    assert lib.svar_set_net(None, None) == sv.E_INVAL
    assert lib.svar_destroy(None) == sv.OK
    assert lib.svar_train(None, 1, 1, 1, None, None, None, None, None, None) == sv.E_INVAL
    assert lib.svar_load_learned(None, b"x", None) == sv.E_INVAL
