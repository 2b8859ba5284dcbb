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
    """Four porous media of different sizes: 37 batched steps (one replay of
    the captured 30-step graph, then single launches), one member stepped on
    its own in between, 13 more batched steps: every field equal to running
    each simulation alone for the same steps."""
    import torch

    from paper_1410_3464_amd.lbrx import Batch, Lbrx

    probs = _problems()
    st = torch.cuda.Stream()
    sims = [Lbrx(p, precision, stream=st.cuda_stream) for p in probs]
    b = Batch(sims)
    b.step(37)
    sims[2].step(5)
    b.step(13)
    got = [s.fields() for s in sims]
    b.close()
    steps = [50, 50, 55, 50]
    for p, g, n in zip(probs, got, steps):
        a = Lbrx(p, precision)
        a.step(n)
        ref = a.fields()
        for k in KEYS:
            assert np.array_equal(g[k], ref[k]), (p.name, precision, k)
        for k, v in ref["ledger"].items():
            assert np.array_equal(np.asarray(g["ledger"][k]), np.asarray(v)), (p.name, k)
        a.close()
    for s in sims:
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
