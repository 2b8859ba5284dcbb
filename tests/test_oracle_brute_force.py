"""The FP64 oracle against a second, literal transcription of the step
(tests/brute_force.py: plain Python loops, one block per equation) on 8 x 8
lattices built to run every branch within 20 steps: dissolution to removal,
precipitation to a new solid node, liquid-gas changes both ways, solute
shares in transit and kept content, stranded populations, the surface-enhanced
R1 rate, unequal relaxation times and pair strengths, adhesion, a body force,
walls and the free outlet.  Populations, node types, solute states, volumes
and every balance agree to 1e-13 (relative to each quantity's largest value)
after every step.  This pins, by transcription, the readings that no closed
form or invariant fixes: which density each phi of Eq. 15 takes, the liquid
mark and its threshold, and the status-change amendments.
"""
import numpy as np
import pytest

from brute_force import BruteForce
from oracle import OracleSim
from paper_1410_3464_amd import workloads as W

TOL = 1e-13


def event_box(outlet):
    """8 x 8: a dissolvable 2 x 2 grain of small volume, a precipitate node
    whose liquid neighbours already hold nearly a node's worth of precipitate,
    and an inert node; smooth liquid and vapour bands (periodic; with the
    outlet, liquid below a wavy interface) whose middle lies near the liquid
    threshold; four species with R1
    (surface-enhanced next to D), B + E -> F, fast dissolution consuming B
    into E and fast precipitation of F.  rho10 = 0.5 and rho20 = 0.05 keep
    both effective masses of Eq. 15 varying over the box (the workloads'
    values saturate them, so the pair force would hardly show)."""
    n = 8
    a, b, R = W.EOS_PAPER
    T = 0.75 * W.critical_temperature(a, b, R)
    yy, xx = np.mgrid[0:n, 0:n]
    t = np.zeros((n, n), np.uint8)
    t[2:4, 2:4] = W.SOLID_D
    t[1, 5] = W.SOLID_F
    t[5, 6] = W.SOLID_INERT
    rl, rv = W.RHO_L_075_PAPER, W.RHO_V_075_PAPER
    if outlet:   # liquid below a wavy interface, vapour towards the outlet
        s = 0.5 * (1 - np.tanh((yy - 4.5 + 1.2 * np.sin(2 * np.pi * xx / n)) / 1.5))
    else:
        s = 0.5 + 0.5 * np.sin(2 * np.pi * yy / n + 0.7 * np.sin(2 * np.pi * xx / n))
    rng = np.random.default_rng(5)
    rho1 = np.where(t == 0, (rv + (rl - rv) * s) * (1 + rng.uniform(-0.02, 0.02, (n, n))), 0.0)
    if not outlet:   # a lone liquid node in the vapour band: it turns gas with no liquid neighbour
        rho1[6, 0] = 0.52 * rho1.max()
    rho2 = np.where(t == 0, 0.1 + rng.uniform(-0.01, 0.01, (n, n)), 0.0)
    V0 = np.where(t == W.SOLID_D, 0.05, np.where(t == W.SOLID_F, 1.0, 0.0))
    for (y, x) in ((0, 5), (2, 5), (1, 4), (1, 6)):
        V0[y, x] = 0.97
    C0 = np.zeros((4, n, n))
    C0[0] = 1.0 + 0.1 * np.sin(xx)
    C0[1] = 0.6
    C0[2] = 0.3
    C0[3] = 0.8 + 0.05 * yy
    sp = [W.Species("A", 1.0, 0.9), W.Species("B", 0.8, 0.8), W.Species("E", 1.2, 0.85), W.Species("F", 0.9, 0.7)]
    hom = [W.HomRxn("r1_gas", re=(0, -1), pr=(1, -1), k=0.05, K_eq=1.0, M_gas=0.01,
                    surface=(W.SOLID_D,), surface_factor=10.0),
           W.HomRxn("bimolecular", re=(1, 2), pr=(3, -1), k=0.1)]
    het = [W.HetRxn(1, 2, (W.SOLID_D,), "consumes", True, 1.0, 0.0, 5.0),
           W.HetRxn(3, -1, (W.SOLID_D, W.SOLID_F), "grows", True, 0.5, 0.0, 2.0)]
    return W.Problem(
        name=f"events-8x8{'-outlet' if outlet else ''}", nx=n, ny=n, periodic_x=True, periodic_y=not outlet,
        outlet_top=outlet, tau=(1.0, 0.8), w_adh=(-0.05, 0.02), gbody=(1e-5, -2e-5), a=a, b=b, R=R, T=T,
        G11=-1.0, G12=0.5, G21=0.4, a0=0.005, rho10=0.5, rho20=0.05,
        species=sp, hom=hom, het=het, type0=t, V0=V0, rho1=rho1, rho2=rho2, C0=C0)


def _rel(a, b):
    scale = max(np.abs(b).max(), 1e-300)
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / scale)


@pytest.mark.parametrize("outlet", [False, True])
def test_oracle_matches_brute_force(outlet):
    prob = event_box(outlet)
    o = OracleSim(prob)
    bf = BruteForce(prob)
    seen = dict(share=0, hold=0, stranded=0)
    for n in range(1, 21):
        o.step(1)
        bf.step(1)
        f, g, flags = o.state()
        F = o.fields()
        t_bf = np.array(bf.type)
        assert np.array_equal(F["type"], t_bf), f"node types differ at step {n}"
        sflag = flags & 3
        stranded = (flags >> 2) & 1
        assert np.array_equal(sflag, np.array(bf.sflag)), f"solute states differ at step {n}"
        assert np.array_equal(stranded.astype(bool), np.array(bf.stranded)), f"stranded flags differ at step {n}"
        fb = np.array(bf.f)
        valid_f = (t_bf == W.FLUID) | np.array(bf.stranded)
        assert _rel(f[:, :, valid_f], fb[:, :, valid_f]) < TOL, f"flow populations differ at step {n}"
        gb = np.array(bf.g)
        valid_g = sflag != 0
        assert _rel(g[:, :, valid_g], gb[:, :, valid_g]) < TOL, f"solute populations differ at step {n}"
        assert _rel(F["V"], np.array(bf.V)) < TOL
        rho, liq, C = bf.densities_and_content()
        assert np.array_equal(F["liquid"].astype(bool), np.array(liq)), f"liquid marks differ at step {n}"
        assert _rel(F["rho1"], np.array(rho[0])) < TOL and _rel(F["rho2"], np.array(rho[1])) < TOL
        assert _rel(F["C"], np.array(C)) < TOL
        assert abs(F["rho_max_prev"] - bf.rho_max_prev) <= TOL * bf.rho_max_prev
        L = F["ledger"]
        for k, v in bf.ledger.items():
            ref = np.asarray(v, dtype=np.float64)
            got = np.asarray(L[k], dtype=np.float64).reshape(-1)[: ref.size]
            assert np.allclose(got, ref, rtol=TOL, atol=TOL * max(1.0, np.abs(ref).max())), (n, k, got, ref)
        seen["share"] += int((sflag == 3).sum())
        seen["hold"] += int((sflag == 2).sum())
        seen["stranded"] += int(stranded.sum())
    L = o.fields()["ledger"]
    print(outlet, seen, {k: L[k] for k in ("n_dissolved", "n_precipitated", "n_liq_to_gas", "n_gas_to_liq")})
    # every branch ran
    assert L["n_dissolved"] > 0 and L["n_precipitated"] > 0
    assert L["n_liq_to_gas"] > 0 and L["n_gas_to_liq"] > 0
    assert seen["share"] > 0 and seen["stranded"] > 0
    if not outlet:
        assert seen["hold"] > 0
