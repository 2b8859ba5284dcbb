"""Host-side checks of the C ABI library (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "lbrx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbrx_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for n in ("lbrx_create", "lbrx_step", "lbrx_fields", "lbrx_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1410_3464_amd import lbrx

    if not os.path.exists(lbrx.LIB_PATH):
        pytest.skip("liblbrx.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(lbrx.LIB_PATH)
    for n in _declared_functions():
        assert hasattr(lib, n), n
    assert set(_declared_functions()) == set(lbrx.SYMBOLS)


def test_binding_struct_layout_matches_header():
    """The ctypes mirror of lbrx_params / lbrx_ledger has the C layout: checked by
    compiling a tiny host program against include/lbrx.h with gcc."""
    import subprocess
    import tempfile

    from paper_1410_3464_amd import lbrx

    prog = r'''
#include <stdio.h>
#include <stddef.h>
#include "lbrx.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(lbrx_params), offsetof(lbrx_params, hom),
         offsetof(lbrx_params, het), offsetof(lbrx_params, node_type), sizeof(lbrx_ledger),
         sizeof(lbrx_fields_out), sizeof(lbrx_het_rxn), sizeof(lbrx_hom_rxn),
         offsetof(lbrx_params, psi_prefactor), offsetof(lbrx_params, alloc_user));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(prog)
        exe = os.path.join(d, "t")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", exe, c])
        got = [int(v) for v in subprocess.check_output([exe]).split()]
    want = [ctypes.sizeof(lbrx.Params), lbrx.Params.hom.offset, lbrx.Params.het.offset,
            lbrx.Params.node_type.offset, lbrx.LEDGER_LEN * 8, ctypes.sizeof(lbrx.FieldsOut),
            ctypes.sizeof(lbrx.HetRxn), ctypes.sizeof(lbrx.HomRxn), lbrx.Params.psi_prefactor.offset,
            lbrx.Params.alloc_user.offset]
    assert got == want


def test_missing_library_fails_loudly(tmp_path):
    from paper_1410_3464_amd import lbrx

    saved = lbrx._lib
    try:
        lbrx._lib = None
        with pytest.raises(ImportError):
            lbrx.load_library(str(tmp_path / "nope.so"))
    finally:
        lbrx._lib = saved


def test_create_validates_before_touching_the_device():
    """lbrx_create checks the problem before any device call, so its refusals
    show without a GPU: a free outlet with 16-bit storage or with a periodic
    y axis, unknown boundary bits, tau <= 1/2; each with a message."""
    from paper_1410_3464_amd import lbrx
    from paper_1410_3464_amd import workloads as W

    if not os.path.exists(lbrx.LIB_PATH):
        pytest.skip("liblbrx.so not built (run __graft_entry__.build())")
    lib = lbrx.load_library()
    p = W.beaker(nx=20, ny=24, level=12, radius=3.0, centre=(10.0, 8.0))
    cases = [(p, "f16dev", "FP64 or FP32"), (p, "bf16dev", "FP64 or FP32"),
             (p.copy(periodic_y=True), "f64", "walls in y"), (p.copy(tau=(0.5, 1.0)), "f32", "tau")]
    for prob, prec, words in cases:
        with pytest.raises(lbrx.LbrxError) as ei:
            lbrx.Lbrx(prob, prec)
        assert ei.value.status == 1 and words in str(ei.value), (prec, str(ei.value))
    params, keep = lbrx.make_params(p, "f64", 0)
    params.periodic = 8
    h = ctypes.c_void_p()
    assert lib.lbrx_create(ctypes.byref(params), None, ctypes.byref(h)) == 1
    assert b"unknown bits" in lib.lbrx_create_error()
    del keep
