"""Device memory through the caller's allocator (lbrx_params.dev_alloc /
dev_free): PyTorch's caching allocator supplies every buffer of a context and
of a batch built on it, and gets all of it back."""
import numpy as np
import pytest

from paper_1410_3464_amd import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("rho1", "rho2", "ux", "uy", "C", "V", "type", "liquid")


def test_torch_allocator_supplies_and_recovers_memory():
    import torch

    from paper_1410_3464_amd.lbrx import Batch, Lbrx

    p = W.config1(nx=160, ny=96, seed=4)
    q = W.config1(nx=96, ny=64, seed=5)
    refs = []
    for prob in (p, q):
        r = Lbrx(prob, "f32")
        r.step(40)
        refs.append(r.fields())
        r.close()

    torch.cuda.synchronize()
    m0 = torch.cuda.memory_allocated()
    g = Lbrx(p, "f32", allocator="torch")
    m1 = torch.cuda.memory_allocated()
    pitch = (p.nx + 63) // 64 * 64
    state = 2 * (18 + 20) * pitch * p.ny * 4  # both buffers of the FP32 populations
    assert m1 - m0 >= state, (m1 - m0, state)
    h = Lbrx(q, "f32", allocator="torch", stream=g.stream)
    b = Batch([g, h])  # its table and instance list come from g's allocator
    b.step(40)
    F = [g.fields(), h.fields()]  # read-out planes allocated on first use
    assert torch.cuda.memory_allocated() > m1
    for got, want in zip(F, refs):
        for k in KEYS:
            assert np.array_equal(got[k], want[k]), k
    b.close()
    g.close()
    h.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == m0
