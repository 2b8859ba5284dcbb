"""The allocation-free read-out (lbrx_fields_noalloc) through the C ABI: the
same fields as lbrx_fields on two calls in a row, the second on a smaller
lattice, without any device allocation; a lattice whose read-out exceeds the
static array is refused with a message."""
import numpy as np
import pytest

from paper_1410_3464_amd import workloads as W

pytestmark = pytest.mark.gpu


def _same(a, b):
    for k in ("rho1", "rho2", "ux", "uy", "C", "V", "type", "liquid"):
        assert np.array_equal(a[k], b[k]), k
    for k in a["ledger"]:
        assert np.array_equal(np.asarray(a["ledger"][k]), np.asarray(b["ledger"][k])), k
    assert a["rho_max_prev"] == b["rho_max_prev"]


@pytest.mark.parametrize("precision", ["f64", "f32", "f16dev"])
def test_noalloc_fields_equal_fields(precision):
    import torch

    from paper_1410_3464_amd.lbrx import Lbrx

    big = W.config1(nx=400, ny=300, seed=5)
    small = W.config0()
    sims = [Lbrx(big, precision), Lbrx(small, precision)]
    for s in sims:
        s.step(37)
        s.sync()
    torch.cuda.synchronize()
    # nothing is allocated by the read-out without allocation (the first
    # lbrx_fields of a context allocates its staging, so it comes after)
    free0 = torch.cuda.mem_get_info()[0]
    first = [s.fields(noalloc=True) for s in sims]   # larger lattice, then smaller
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    for s, f in zip(sims, first):
        _same(f, s.fields())
    # again after more steps: the static array keeps the last call's contents
    for s in sims:
        s.step(5)
    again = [s.fields(noalloc=True) for s in sims]
    for s, f in zip(sims, again):
        _same(f, s.fields())
    for s in sims:
        s.close()


def test_noalloc_refuses_a_read_out_larger_than_the_array():
    from paper_1410_3464_amd.lbrx import Lbrx, LbrxError

    # (5 + 4) planes of 2048 x 1024 doubles exceed 128 MiB
    big = W.config1(nx=2048, ny=1024, seed=6)
    s = Lbrx(big, "f32")
    s.step(2)
    with pytest.raises(LbrxError) as ei:
        s.fields(noalloc=True)
    assert ei.value.status == 1 and "static" in str(ei.value)
    s.fields()   # the allocating read-out still works
    s.close()
