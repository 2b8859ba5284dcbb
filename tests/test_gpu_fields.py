"""lbrx_fields reads out only the fields whose host buffers are given."""
import numpy as np
import pytest

from paper_1410_3464_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_fields_selected_by_buffers(precision):
    """After 25 steps of a 130x70 porous medium: a read-out of V, type,
    ledger and rho_max alone (which runs no read-out kernel), and one of rho1
    and C alone, equal the same fields of a full read-out; the fields not
    asked for are not returned."""
    from paper_1410_3464_amd.lbrx import Lbrx

    g = Lbrx(W.config1(nx=130, ny=70, seed=11), precision)
    g.step(25)
    full = g.fields()
    a = g.fields(only={"V", "type", "ledger", "rho_max_prev"})
    b = g.fields(only={"rho1", "C"})
    assert set(a) == {"V", "type", "ledger", "rho_max_prev"} and set(b) == {"rho1", "C"}
    for k in ("V", "type"):
        assert np.array_equal(a[k], full[k]), k
    assert a["rho_max_prev"] == full["rho_max_prev"]
    for k, v in full["ledger"].items():
        assert np.array_equal(np.asarray(a["ledger"][k]), np.asarray(v)), k
    for k in ("rho1", "C"):
        assert np.array_equal(b[k], full[k]), k
    g.close()
