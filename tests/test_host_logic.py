"""Host-side logic without a GPU: the seeded workload generators keep the
recipes they state, the serving helpers, the autotuner's size classes and the
benchmark's algorithmic byte count on hand-counted cases."""
import math
import os
import sys

import numpy as np
import pytest

from paper_1410_3464_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_porous_generator_keeps_its_recipe():
    """config1 at 256 x 128: porosity at most 0.55 and within 0.5 % of it
    (disks are added until it is reached), at least 20 % of the solid dissolvable, at least 30 %
    of the pore space vapour, walls in y, four species with A = 1 at liquid
    density and the same problem for the same seed."""
    p = W.config1(nx=256, ny=128, seed=9)
    fl = p.type0 == W.FLUID
    solid = ~fl
    assert 0.545 <= fl.mean() <= 0.55
    assert (p.type0 == W.SOLID_D).sum() >= 0.2 * solid.sum()
    vap = fl & (p.rho1 < 0.5 * (W.RHO_L_075_PAPER + W.RHO_V_075_PAPER))
    assert vap.sum() >= 0.3 * fl.sum()
    assert p.periodic_x and not p.periodic_y
    assert p.n_species == 4 and np.all(p.C0[0] == 1.0) and np.all(p.C0[1:] == 0.0)
    assert np.all(p.rho1[solid] == 0.0) and np.all(p.rho2[solid] == 0.0)
    assert np.all(np.abs(p.rho2[fl] - 0.1) <= 1e-4)
    q = W.config1(nx=256, ny=128, seed=9)
    assert np.array_equal(p.type0, q.type0) and np.array_equal(p.rho1, q.rho1)
    r = W.config1(nx=256, ny=128, seed=10)
    assert not np.array_equal(p.type0, r.type0)


def test_batch_instances_span_the_stated_ranges():
    """Sides log-uniform in [64, 1024], porosity in [0.4, 0.8] (within a few
    percent above the drawn target where the last grain had to be shrunk:
    on 64^2 one grain covers up to 40 % of the lattice), rates in [1e-6,
    1e-1], over 64 seeds."""
    sides, rates = [], []
    for s in range(64):
        p = W.batch_instance(s, smin=64, smax=1024)
        assert p.nx == p.ny and 64 <= p.nx <= 1024
        sides.append(p.nx)
        rates += [r.k for r in p.hom] + [r.k for r in p.het]
        if p.nx <= 256:
            assert 0.4 - 0.005 <= (p.type0 == W.FLUID).mean() <= 0.8 + 0.05
    assert min(sides) < 128 and max(sides) > 512
    assert all(1e-6 <= k <= 1e-1 for k in rates)


def test_fracture_geometry():
    """App. A.3's box: the middle h0 rows open, the rest dissolvable mineral
    with volume 1; k = Da D / h0 with D from Eq. 24."""
    p = W.fracture(L=100, H=90, h0=30, Da=0.001)
    fl = p.type0 == W.FLUID
    assert fl.sum() == 100 * 30 and fl[30:60].all() and not fl[:30].any() and not fl[60:].any()
    assert np.all(p.V0[~fl] == 1.0)
    D = 0.5 * (1 - 0.9) * (1.0 - 0.5)
    assert math.isclose(p.het[0].k, 0.001 * D / 30, rel_tol=1e-15)


def test_poisson_requests_and_summary():
    """Arrivals start at 0 and increase, with the stated mean gap (within
    the sampling error of 400 draws); step counts and sizes in range; the
    summary's percentiles and throughput are those of the recorded times."""
    from paper_1410_3464_amd import serve

    reqs = serve.poisson_requests(400, 0.01, seed=2, steps=(200, 2000), sizes=(64, 96))
    t = np.array([r.arrival for r in reqs])
    assert t[0] == 0.0 and np.all(np.diff(t) >= 0)
    assert abs(np.diff(t).mean() / 0.01 - 1) < 0.15
    assert all(200 <= r.steps <= 2000 for r in reqs)
    assert all(64 <= r.prob.nx <= 96 for r in reqs)
    assert {r.precision for r in reqs} == {"f32", "f16dev"}
    few = reqs[:4]
    for i, r in enumerate(few):
        r.start, r.finish, r.status = r.arrival, r.arrival + 0.1 * (i + 1), "ok"
    s = serve.summarize(few, makespan=2.0)
    lat = [100.0, 200.0, 300.0, 400.0]
    assert s["completed"] == 4
    assert s["p50_ms"] == pytest.approx(np.percentile(lat, 50))
    assert s["p99_ms"] == pytest.approx(np.percentile(lat, 99))
    assert s["mlups"] == pytest.approx(round(sum(r.updates for r in few) / 2.0 / 1e6, 1))


def test_footprint_counts_every_buffer():
    """FP32, 4 species, 64 x 64: two buffers of 18 flow and 20 solute values
    and a status word per node, solid volumes, balance records of items of 62
    columns by 2 rows (or more: the shortest item a lattice is given) and the
    read-out planes; 16-bit storage halves the populations and adds the code
    words."""
    from paper_1410_3464_amd import serve

    p = W.config1(nx=64, ny=64, seed=1)
    plane = 64 * 64
    items = 2 * 32
    want = 2 * (38 * plane * 4 + plane * 4) + plane * 8 + items * 38 * 8 + 8 * plane * 8
    assert serve.footprint_bytes(p, "f32") == want
    want16 = 2 * (38 * plane * 2 + plane * 4 * 2) + plane * 8 + items * 38 * 8 + 8 * plane * 8
    assert serve.footprint_bytes(p, "f16dev") == want16


def test_autotune_size_classes():
    from paper_1410_3464_amd.autotune import size_class

    assert size_class(64, 64) == 64 and size_class(10, 10) == 64
    assert size_class(100, 90) == 128 and size_class(700, 300) == 512
    assert size_class(1024, 1024) == 1024 and size_class(4096, 4096) == 4096


def test_algorithmic_bytes_on_a_hand_counted_case():
    """A 4 x 3 periodic box: one dissolvable solid node at (1, 1), its D2Q5
    neighbours liquid, every other fluid node gas.  Fluid 11 nodes x 36 s,
    liquid 4 x 10 N_s s, 2 bytes per node, 16 per interface node (the solid
    and its 4 liquid neighbours)."""
    sys.path.insert(0, ROOT)
    import bench

    t = np.zeros((3, 4), np.uint8)
    t[1, 1] = W.SOLID_D
    liq = np.zeros((3, 4), np.uint8)
    for x, y in ((0, 1), (2, 1), (1, 0), (1, 2)):
        liq[y, x] = 1
    p = W.uniform_problem(4, 3, species=[W.Species("A"), W.Species("B")], C0=np.zeros((2, 3, 4)))
    b, counts = bench.algorithmic_bytes({"type": t, "liquid": liq}, p, 4)
    assert counts == dict(fluid=11, liquid=4, interface=5, nodes=12)
    assert b == 11 * 36 * 4 + 4 * 10 * 2 * 4 + 2 * 12 + 16 * 5
    b16, _ = bench.algorithmic_bytes({"type": t, "liquid": liq}, p, 2)
    assert b16 == 11 * 36 * 2 + 4 * 10 * 2 * 2 + 2 * 12 + 16 * 5 + 4 * 8


def test_beaker_geometry():
    """Sec. 5: 100 x 160 lattice units, walls left, right and below, a free
    outlet on top, a D(s) particle of radius 15 at (50, 50) with volume 1,
    liquid (8.31, 1e-4) below y = 100 and gas (0.05, 0.05) above, joined by
    a tanh of width 1.5; A = 1 in the liquid only; T = 0.65 T_c."""
    p = W.beaker()
    assert (p.nx, p.ny) == (100, 160)
    assert not p.periodic_x and not p.periodic_y and p.outlet_top
    yy, xx = np.mgrid[0:160, 0:100]
    part = (xx - 50) ** 2 + (yy - 50) ** 2 <= 225
    assert np.array_equal(p.type0 == W.SOLID_D, part) and np.all(p.V0[part] == 1.0)
    fl = ~part
    assert np.all(np.abs(p.rho1[10][fl[10]] - 8.31) < 1e-5) and np.all(np.abs(p.rho1[150] - 0.05) < 1e-5)
    assert np.allclose(p.rho2[10][fl[10]], 1e-4) and np.allclose(p.rho2[150], 0.05)
    assert np.all(p.rho1[~fl] == 0.0)
    assert np.all(p.C0[0][10][fl[10]] == 1.0) and np.all(p.C0[0][150] == 0.0)
    assert p.species[0].tau_g == 0.65 and p.species[0].J0 == 0.9
    assert math.isclose(p.T, 0.65 * W.critical_temperature(p.a, p.b, p.R))
