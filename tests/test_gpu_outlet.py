"""The free outlet of Sec. 5.1 on the HIP path: beyond the top side lies a
ghost row repeating the top row (zero gradient of every variable).  FP64
within 1e-12 of the oracle with masks and event counts identical, FP32
within 1e-5 over the first 10 steps; an outlet simulation batched with others
equals its run alone bit for bit; 16-bit storage and a periodic y axis are
refused."""
import os
import sys

import numpy as np
import pytest

from oracle import OracleSim
from paper_1410_3464_amd import workloads as W

pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.dirname(__file__))
from parity import outlet_pool  # noqa: E402
from test_gpu_parity import _run_pair, events_problem  # noqa: E402


def outlet_events():
    """The event-heavy 40 x 40 case moved up 16 rows: the dissolvable grain
    now crosses the outlet row (and the wall below), the precipitate column
    runs into the outlet, and the gas bubble sits near it."""
    p = events_problem()
    roll = lambda a: np.roll(a, 16, axis=-2)  # noqa: E731
    return p.copy(name="events-40-outlet", periodic_y=False, outlet_top=True, type0=roll(p.type0),
                  V0=roll(p.V0), rho1=roll(p.rho1), rho2=roll(p.rho2), C0=roll(p.C0))


def test_outlet_pool_fp64():
    _run_pair(outlet_pool(), "f64", [1, 50, 400, 1500], 1e-12)


def test_outlet_events_fp64():
    """Grain and precipitate at the outlet: ghost solids bounce populations
    back, top-row grain nodes dissolve and then react with the grain below
    them, the precipitate column strands nodes; masks and event counts
    identical.  Checked to step 120: from step 128 a band of nodes near the
    wall below flips its liquid marks and the collapse that follows doubles
    the rounding differences of both sides every step (interior nodes,
    1e-14 -> 1e-12 within five steps), with no event at the outlet."""
    o = OracleSim(outlet_events())
    o.step(120)
    assert o.fields()["ledger"]["n_dissolved"] > 0 and o.fields()["ledger"]["n_precipitated"] > 0
    rep = _run_pair(outlet_events(), "f64", [5, 60, 100, 120], 1e-12)
    assert all(masks for _, _, masks, _ in rep)


def test_outlet_ragged_fp64():
    """70 x 29 (ragged in both directions against 64-wide, 12-row items)."""
    _run_pair(outlet_pool(nx=70, ny=29, seed=4), "f64", [1, 100, 600], 1e-12)


def test_outlet_fp32():
    """FP32 within 1e-5 of the FP64 oracle over the first 10 steps (the bar of
    the droplet case); by step 50 the moving bubble has grown the velocity
    difference to about 3e-5 of the largest speed, as FP32 rounding does in
    the periodic cases."""
    _run_pair(outlet_pool(), "f32", [1, 10], 1e-5)
    _run_pair(outlet_pool(), "f32", [50], 1e-4)


def test_outlet_in_a_batch_equals_alone():
    """An outlet simulation, a wall-bounded one and a periodic one in one
    batch: each equals its run alone bit for bit (FP32, 90 steps: three graph
    replays)."""
    import torch

    from paper_1410_3464_amd.lbrx import Batch, Lbrx

    probs = [outlet_pool(nx=48, ny=40), outlet_pool(outlet=False, nx=48, ny=40), W.config0()]
    probs = [p.copy(species=p.species[:2], C0=p.C0[:2], hom=p.hom[:1], het=p.het[:1]) for p in probs]
    st = torch.cuda.Stream()
    sims = [Lbrx(p, "f32", stream=st.cuda_stream) for p in probs]
    b = Batch(sims)
    b.step(90)
    b.close()
    for p, s in zip(probs, sims):
        alone = Lbrx(p, "f32")
        alone.step(90)
        G, A = s.fields(), alone.fields()
        for k in ("rho1", "rho2", "ux", "uy", "C", "V", "type", "liquid"):
            assert np.array_equal(G[k], A[k]), (p.name, k)
        alone.close()
        s.close()


def test_outlet_refusals():
    from paper_1410_3464_amd.lbrx import Lbrx, LbrxError

    p = outlet_pool()
    for prec in ("f16dev", "bf16dev"):
        with pytest.raises(LbrxError) as ei:
            Lbrx(p, prec)
        assert ei.value.status == 1
    with pytest.raises(LbrxError) as ei:
        Lbrx(p.copy(periodic_y=True), "f64")
    assert ei.value.status == 1
