"""The oracle's host threads change no result: every node loop that runs in
parallel touches only its own node's results, and every balance is summed
serially in node order.  Populations, solute states, fields and every balance
after the same steps are bit-identical for 1 and 4 threads, on the event-heavy
8 x 8 lattices and on a porous medium with walls."""
import numpy as np
import pytest

from oracle import OracleSim
from paper_1410_3464_amd import workloads as W
from test_oracle_brute_force import event_box


@pytest.mark.parametrize("case", ["events", "events-outlet", "porous"])
def test_threads_give_identical_results(case):
    if case == "porous":
        prob, steps = W.config1(nx=160, ny=96, seed=4), 150
    else:
        prob, steps = event_box(case == "events-outlet"), 20
    out = []
    for th in (1, 4):
        s = OracleSim(prob, threads=th)
        s.step(steps)
        out.append((s.fields(), s.state()))
        s.close()
    (A, sa), (B, sb) = out
    for k in ("rho1", "rho2", "ux", "uy", "C", "V", "type", "liquid"):
        assert np.array_equal(A[k], B[k]), k
    for k in A["ledger"]:
        assert np.array_equal(np.asarray(A["ledger"][k]), np.asarray(B["ledger"][k])), k
    for x, y in zip(sa, sb):
        assert np.array_equal(x, y)
