"""The work decomposition changes the speed of a step, not its result: every
item height gives the same fields bit for bit (each node's arithmetic is the
same; only the per-item balance records, and so the order in which the
balances are summed, change)."""
import numpy as np
import pytest

from paper_1410_3464_amd import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("rho1", "rho2", "ux", "uy", "C", "V", "type", "liquid")


@pytest.mark.parametrize("precision", ["f64", "f32", "f16dev"])
def test_item_height_changes_speed_not_fields(precision):
    """The ragged 130 x 70 porous medium after 150 steps with items of 1, 2,
    5 and 30 rows and the default against 16-row items: fields and masks
    equal bit for bit, balances within 1e-12 (relative to their size).  The
    default gives this lattice shorter items than 16 rows (it would fill a
    small part of the device): its state holds more balance records."""
    from paper_1410_3464_amd.lbrx import Lbrx

    p = W.config1(nx=130, ny=70, seed=11)
    ref = Lbrx(p, precision, seg_rows=16)
    ref.step(150)
    R = ref.fields()
    ref_bytes = ref.save_state().size
    ref.close()
    for h in (0, 1, 2, 5, 30):
        g = Lbrx(p, precision, seg_rows=h)
        g.step(150)
        G = g.fields()
        for k in KEYS:
            assert np.array_equal(G[k], R[k]), (h, k)
        for k, v in R["ledger"].items():
            a, b = np.asarray(G["ledger"][k], dtype=float), np.asarray(v, dtype=float)
            scale = max(float(np.abs(b).max()) if b.size else 0.0, 1e-300)
            assert float(np.abs(a - b).max() if b.size else 0.0) <= 1e-12 * scale, (h, k)
        if h == 0:
            assert g.save_state().size > ref_bytes
        g.close()
