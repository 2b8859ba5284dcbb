"""Parity at the workloads' full sizes, in the launch configuration the
benchmark uses (same lattice generator, same kernel, default item shape).

The 1024 x 512 porous medium is compared field by field against the FP64
oracle in FP64 and FP32; the 4096 x 4096 roofline workload is compared field
by field for a few FP32 steps (the oracle needs about 4 s per step there) and
then checked, after many more GPU steps, on properties that hold at any size:
the mass balance closes with the ledger and the masks stay consistent.
"""
import os
import sys

import numpy as np
import pytest

from oracle import OracleSim
from paper_1410_3464_amd import workloads as W

pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.dirname(__file__))
from parity import compare  # noqa: E402


def _lbrx():
    from paper_1410_3464_amd.lbrx import Lbrx

    return Lbrx


def _check(G, O, prob, tol, label):
    errs, masks, near = compare(G, O, prob, tol)
    print(f"[{label}] " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()) + f" masks={masks}", flush=True)
    assert masks, f"{label}: node masks differ"
    for k, v in errs.items():
        assert v <= tol, f"{label}: {k} error {v:.3e} > {tol:.1e}"


@pytest.mark.parametrize("precision,steps,tol", [("f64", 40, 1e-12), ("f32", 10, 1e-5)])
def test_porous_1024x512_full_field(precision, steps, tol):
    """The 1024 x 512 porous medium (seed 1): every field of every node."""
    prob = W.config1()
    o = OracleSim(prob)
    g = _lbrx()(prob, precision)
    o.step(steps)
    g.step(steps)
    _check(g.fields(), o.fields(), prob, tol, f"porous-1024x512 {precision} {steps}")
    g.close()
    o.close()


def test_porous_4096_full_field_and_balances():
    """The 4096 x 4096 roofline workload in FP32: every field after 2 steps
    against the oracle; then 200 more GPU steps close the mass ledger
    (initial mass + sources + injections - removals = current mass, per
    component, to FP32 summation accuracy) and keep every liquid node fluid."""
    prob = W.config2()
    g = _lbrx()(prob, "f32")
    o = OracleSim(prob)
    o.step(2)
    g.step(2)
    _check(g.fields(), o.fields(), prob, 1e-5, "porous-4096 f32 2")
    o.close()
    del o
    g.step(200)
    F = g.fields()
    L = F["ledger"]
    fl0 = prob.type0 == 0
    M0 = np.array([prob.rho1[fl0].sum(), prob.rho2[fl0].sum()])
    fl = F["type"] == 0
    # every node's density (a node that just turned solid still holds, for one
    # step, the populations it passes on)
    M = np.array([F["rho1"].sum(), F["rho2"].sum()])
    bal = M0 + L["mass_src"] + L["mass_inj"] - L["mass_rem"]
    print("[porous-4096 f32 202] mass", M, "balance", bal, flush=True)
    # FP32 collisions are not exactly mass-conserving: each step can move a
    # node's total by at most about 18 roundings (2^-24 relative each)
    rtol = 202 * 18 * 2.0 ** -24
    assert np.allclose(M, bal, rtol=rtol, atol=0)
    assert not np.any(F["liquid"].astype(bool) & ~fl)
    g.close()
