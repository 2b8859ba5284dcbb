"""Batched stepping (lbrx_batch_*): several simulations advanced by one launch
per step give, field by field and bit for bit, what each gives alone."""
import numpy as np
import pytest

from paper_1410_3464_amd import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("rho1", "rho2", "ux", "uy", "C", "V", "type", "liquid")


def _problems():
    return [W.config1(nx=96, ny=64, seed=3), W.config1(nx=200, ny=150, seed=4),
            W.config1(nx=130, ny=70, seed=5), W.config1(nx=64, ny=64, seed=6)]


@pytest.mark.parametrize("precision", ["f64", "f32", "f16dev"])
def test_batch_equals_alone(precision):
    """Four porous media of different sizes advanced by batched launches and,
    independently, each alone by single launches; every field equal bit for
    bit at every check.  The batch runs: 30 steps (the graph is captured and
    replayed once), 30 more (second replay of the same graph), then one member
    steps 5 times on its own (eager work between replays; the batch table and
    graph are rebuilt), 67 batched steps (a new graph replayed twice, then
    single launches), 30 more (third replay of the new graph)."""
    import torch

    from paper_1410_3464_amd.lbrx import Batch, Lbrx

    probs = _problems()
    st = torch.cuda.Stream()
    sims = [Lbrx(p, precision, stream=st.cuda_stream) for p in probs]
    alone = [Lbrx(p, precision) for p in probs]
    done = [0] * len(probs)

    def check(tag):
        for i, (p, g, a) in enumerate(zip(probs, sims, alone)):
            a.step(g.steps_done - done[i])
            done[i] = g.steps_done
            G, A = g.fields(), a.fields()
            for k in KEYS:
                assert np.array_equal(G[k], A[k]), (tag, p.name, precision, k)
            for k, v in A["ledger"].items():
                assert np.array_equal(np.asarray(G["ledger"][k]), np.asarray(v)), (tag, p.name, k)

    b = Batch(sims)
    b.step(30)
    check("first replay")
    b.step(30)
    check("second replay")
    sims[2].step(5)
    check("member alone")
    b.step(67)
    check("rebuilt graph")
    b.step(30)
    check("third replay")
    b.close()
    for s in sims + alone:
        s.close()


def test_batch_rejects_mixed_contexts():
    """Contexts of different precision (or stream) cannot share a batch."""
    from paper_1410_3464_amd.lbrx import Batch, Lbrx, LbrxError

    p = W.config1(nx=64, ny=64, seed=1)
    a, c = Lbrx(p, "f32"), Lbrx(p, "f64")
    with pytest.raises(LbrxError):
        Batch([a, c])
    with pytest.raises(LbrxError):
        Batch([a, a])
    a.close()
    c.close()


@pytest.mark.parametrize("precision", ["f64", "f32", "f16dev"])
def test_single_context_graph_replays(precision):
    """lbrx_step replays a captured 30-step graph for aligned runs of 30:
    stepped in chunks of 30, 30, 7, 60 and 13 (first capture, replays, a
    misaligned stretch of single launches, then replays again), the fields
    equal, at every check, those of the same problem stepped one launch at a
    time."""
    from paper_1410_3464_amd.lbrx import Lbrx

    p = W.config1(nx=130, ny=70, seed=8)
    g = Lbrx(p, precision)
    one = Lbrx(p, precision)
    for chunk in (30, 30, 7, 60, 13):
        g.step(chunk)
        for _ in range(chunk):
            one.step(1)
        G, O = g.fields(), one.fields()
        for k in KEYS:
            assert np.array_equal(G[k], O[k]), (chunk, k)
        for k, v in O["ledger"].items():
            assert np.array_equal(np.asarray(G["ledger"][k]), np.asarray(v)), (chunk, k)
    g.close()
    one.close()


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_batch_matches_oracle(precision, tol):
    """A batch of three porous media of different sizes (96x64, 200x150,
    130x70) against the oracle: after 40 batched steps (a captured graph of 30
    launches replayed once, then single batched launches) every field of every
    member within 1e-12 (FP64) or 1e-5 (FP32) of the oracle's (max-norm
    relative), node masks and event counts identical."""
    import os
    import sys

    import torch

    from oracle import OracleSim
    from paper_1410_3464_amd.lbrx import Batch, Lbrx

    sys.path.insert(0, os.path.dirname(__file__))
    from parity import compare, ledger_errors

    probs = _problems()[:3]
    st = torch.cuda.Stream()
    sims = [Lbrx(p, precision, stream=st.cuda_stream) for p in probs]
    b = Batch(sims)
    b.step(40)
    for p, g in zip(probs, sims):
        o = OracleSim(p)
        o.step(40)
        G, O = g.fields(), o.fields()
        errs, masks, near = compare(G, O, p, tol)
        print(f"[batch {precision} {p.name}] " + " ".join(f"{k}={v:.2e}" for k, v in errs.items())
              + f" masks={masks}", flush=True)
        assert masks, p.name
        for k, v in errs.items():
            assert v <= tol, (p.name, k, v)
        le = ledger_errors(G["ledger"], O["ledger"], p.n_species)
        for k in ("n_dissolved", "n_precipitated", "n_liq_to_gas", "n_gas_to_liq", "steps"):
            assert le[k] == 0, (p.name, k, le[k])
        o.close()
    b.close()
    for s in sims:
        s.close()
