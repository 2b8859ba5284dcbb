"""Seeded synthetic problem descriptions for the coupled reactive-transport step.

This module only builds inputs: lattice geometry, node types, initial densities
and concentrations, and the parameter sets.  It contains none of the step's
arithmetic, so the GPU library and the CPU oracle can both consume what it
produces without sharing any of the method.

Problem layout (all arrays row-major, index ``y*nx + x``):

* ``type0`` uint8 ``[ny, nx]``: 0 fluid, 1 inert solid, 2 dissolvable solid D,
  3 precipitate solid F (the node types of Fig. 2 of the paper).
* ``V0`` float64 ``[ny, nx]``: solid volume at D/F nodes, precipitate fraction at fluid nodes.
* ``rho1``, ``rho2`` float64 ``[ny, nx]``: initial liquid- and gas-component densities.
* ``C0`` float64 ``[n_species, ny, nx]``: initial concentrations (used at liquid nodes only).
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

import numpy as np

FLUID, SOLID_INERT, SOLID_D, SOLID_F = 0, 1, 2, 3

def beaker(nx=100, ny=160, level=100, radius=15.0, centre=(50.0, 50.0), G12=0.5, seed=0,
           species=("A",), hom=(), het=()):
    """The beaker of Sec. 5 (100 x 160 lattice units of 1 mm): walls on the
    left, right and bottom with w = 0 (90-degree contact angle), a free outlet
    on top, a dissolvable D(s) particle of radius 15 at (50, 50) with volume 1.
    Sec. 5.1's start: rho1 = 8.31, rho2 = 1e-4 below y = level, rho1 = 0.05,
    rho2 = 0.05 above (joined by a tanh of width 1.5), at T = 0.65 T_c of the
    adopted EOS set; tau = 1; every
    species with J0 = 0.9, tau_g = 0.65 and, for the first one (A), C = 1 in
    the liquid.  The paper's G12, G21 are in its Table 1, which is not
    available; the default is that of the other workloads here.  Noise of
    +-1e-6 (seeded) breaks the mirror symmetry.  Input description only."""
    a, b, R = EOS_PAPER
    T = 0.65 * critical_temperature(a, b, R)
    yy, xx = np.mgrid[0:ny, 0:nx]
    t = np.zeros((ny, nx), np.uint8)
    part = (xx - centre[0]) ** 2 + (yy - centre[1]) ** 2 <= radius ** 2
    t[part] = SOLID_D
    below = yy < level
    # the step between the two phases as a tanh of width 1.5 (a sharp step
    # drives the density negative at the interface within two steps)
    s = 0.5 * (1.0 - np.tanh((yy + 0.5 - level) / 1.5))
    rng = _rng(seed)
    fl = t == FLUID
    rho1 = np.where(fl, 0.05 + (8.31 - 0.05) * s + rng.uniform(-1e-6, 1e-6, (ny, nx)), 0.0)
    rho2 = np.where(fl, 0.05 + (1e-4 - 0.05) * s, 0.0)
    ns = len(species)
    C0 = np.zeros((ns, ny, nx))
    if ns:
        C0[0] = np.where(fl & below, 1.0, 0.0)
    return Problem(
        name=f"beaker-{nx}x{ny}", nx=nx, ny=ny, periodic_x=False, periodic_y=False, outlet_top=True,
        tau=(1.0, 1.0), a=a, b=b, R=R, T=T, G11=-1.0, G12=G12, G21=G12,
        a0=0.005, rho10=paper_rho10(0.005), rho20=0.003,
        species=[Species(n, tau_g=0.65, J0=0.9) for n in species], hom=list(hom), het=list(het),
        type0=t, V0=np.where(part, 1.0, 0.0), rho1=rho1, rho2=rho2, C0=C0, steps=50000,
    )


# Carnahan-Starling parameter sets named in the text after Eq. 13: the original
# (a=1, b=4, R=1) and the one the paper adopts because the two-component system
# diverges at the small vapour density of the first (a=0.09926, b=0.18727, R=0.2).
EOS_ORIGINAL = (1.0, 4.0, 1.0)
EOS_PAPER = (0.09926, 0.18727, 0.2)

# Coexistence densities at T = 0.75 T_c from Maxwell's equal-area rule, stored as
# constants so that this module stays free of the EOS; a CPU test recomputes them.
RHO_L_075 = 0.3331630195715653     # EOS_ORIGINAL
RHO_V_075 = 0.01454506511014443
RHO_L_075_PAPER = 7.116206964736306  # EOS_PAPER
RHO_V_075_PAPER = 0.3106758180173559


@dataclass
class Species:
    name: str
    tau_g: float = 1.0
    J0: float = 0.9


@dataclass
class HomRxn:
    """Homogeneous reaction (Eq. 5a, 5c, or first order).

    kind: "first_order" (R = k C_re0), "r1_gas" (R = k (C_re0 - C_pr0 sqrt(rho2/M_gas)/K_eq),
    with half a mole of gas per mole moved from the liquid to the gas component),
    "bimolecular" (R = k C_re0 C_re1).  Indices refer to the species list; -1 = none.
    surface, surface_factor: at a liquid node with a D2Q5 neighbour of one of the
    solid types in `surface`, k is multiplied by surface_factor (the paper's R1 is
    1000 times faster at the D(s) surface).
    """

    kind: str
    re: tuple = (-1, -1)
    pr: tuple = (-1, -1)
    k: float = 0.0
    K_eq: float = 1.0
    M_gas: float = 1.0
    surface: tuple = ()
    surface_factor: float = 1.0


@dataclass
class HetRxn:
    """Heterogeneous surface reaction (Eq. 29-31, A2).

    mode: "consumes" (solid node volume decreases, R2-like), "grows" (precipitate
    accumulates at the liquid node, R4-like), "mineral" (solid node volume follows
    the sign of the flux, Appendix A.3).  surface: solid types it acts on.
    """

    reactant: int
    product: int = -1
    surface: tuple = (SOLID_D,)
    mode: str = "consumes"
    irreversible: bool = True
    k: float = 0.0
    C_eq: float = 0.0
    molar_volume: float = 1.0


@dataclass
class Problem:
    name: str
    nx: int
    ny: int
    periodic_x: bool
    periodic_y: bool
    outlet_top: bool = False  # the side beyond y = ny - 1 is a zero-gradient free outlet (Sec. 5.1)
    tau: tuple = (1.0, 1.0)
    w_adh: tuple = (0.0, 0.0)
    gbody: tuple = (0.0, 0.0)
    a: float = 1.0
    b: float = 4.0
    R: float = 1.0
    T: float = 0.0
    G11: float = -1.0
    G12: float = 0.0
    G21: float = 0.0
    a0: float = 0.005
    rho10: float = 0.0
    rho20: float = 0.003
    liquid_frac: float = 0.5
    psi_prefactor: float = 0.0  # 0: 2 (weights of Eq. 11 reproduce Eq. 12); 6: as printed in Eq. 13
    # Sec. 4.1: species whose concentration at a liquid node is the total liquid
    # concentration (subtract_total * rho_1) minus the others; -1: none
    subtract_species: int = -1
    subtract_total: float = 0.0
    species: list = field(default_factory=list)
    hom: list = field(default_factory=list)
    het: list = field(default_factory=list)
    type0: np.ndarray = None
    V0: np.ndarray = None
    rho1: np.ndarray = None
    rho2: np.ndarray = None
    C0: np.ndarray = None
    steps: int = 0

    @property
    def n_species(self):
        return len(self.species)

    def copy(self, **kw):
        return dataclasses.replace(self, **kw)


def critical_temperature(a, b, R):
    """T_c from the definitions of a and b in the text after Eq. 12."""
    return (0.1873 / 0.4963) * a / (b * R)


def paper_rho10(a0=0.005):
    """rho_10 = -0.008 / ln(a0) (text after Eq. 15, natural logarithm)."""
    return -0.008 / math.log(a0)


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _disk_mask(nx, ny, cx, cy, r, periodic_x=True, periodic_y=True):
    x = np.arange(nx)[None, :].astype(np.float64)
    y = np.arange(ny)[:, None].astype(np.float64)
    dx = x - cx
    dy = y - cy
    if periodic_x:
        dx = (dx + nx / 2) % nx - nx / 2
    if periodic_y:
        dy = (dy + ny / 2) % ny - ny / 2
    return dx * dx + dy * dy <= r * r


def _stamp_disk(mask, cx, cy, r, periodic_x, periodic_y):
    """Lattice nodes (ys, xs) of the disk of radius r centred at (cx, cy), found
    within its bounding box."""
    ny, nx = mask.shape
    ri = int(math.ceil(r))
    xs = np.arange(int(math.floor(cx)) - ri, int(math.floor(cx)) + ri + 2)
    ys = np.arange(int(math.floor(cy)) - ri, int(math.floor(cy)) + ri + 2)
    dx = xs[None, :] - cx
    dy = ys[:, None] - cy
    inside = dx * dx + dy * dy <= r * r
    if periodic_x:
        xs = xs % nx
    if periodic_y:
        ys = ys % ny
    okx = (xs >= 0) & (xs < nx)
    oky = (ys >= 0) & (ys < ny)
    inside = inside & okx[None, :] & oky[:, None]
    yy, xx = np.nonzero(inside)
    return None, ys[yy], xs[xx]


def config0(seed=0):
    """96x64 periodic box: a droplet of radius 16 in its vapour at T = 0.75 T_c, a
    non-condensable gas at 0.1, one dissolvable disk of radius 10 at (20, 32); species
    A, B with A -> B (k = 1e-3) in the liquid and surface dissolution consuming B
    (k_s = 1e-2).  The fluid uses the paper's adopted EOS set."""
    nx, ny = 96, 64
    a, b, R = EOS_PAPER
    T = 0.75 * critical_temperature(a, b, R)
    type0 = np.zeros((ny, nx), np.uint8)
    solid = _disk_mask(nx, ny, 20.0, 32.0, 10.0)
    type0[solid] = SOLID_D
    V0 = np.where(solid, 1.0, 0.0)
    drop = _disk_mask(nx, ny, 48.0, 32.0, 16.0)
    rho1 = np.where(drop, RHO_L_075_PAPER, RHO_V_075_PAPER)
    rho2 = np.full((ny, nx), 0.1)
    rng = _rng(seed)
    n1 = rng.uniform(-1e-4, 1e-4, size=(ny, nx))
    n2 = rng.uniform(-1e-4, 1e-4, size=(ny, nx))
    fl = type0 == FLUID
    rho1 = np.where(fl, rho1 + n1, 0.0)
    rho2 = np.where(fl, rho2 + n2, 0.0)
    C0 = np.zeros((2, ny, nx))
    C0[0] = 1.0
    return Problem(
        name="droplet-96x64", nx=nx, ny=ny, periodic_x=True, periodic_y=True,
        tau=(1.0, 1.0), a=a, b=b, R=R, T=T, G11=-1.0, G12=0.5, G21=0.5,
        a0=0.005, rho10=paper_rho10(0.005), rho20=0.003,
        species=[Species("A", 1.0, 0.9), Species("B", 1.0, 0.9)],
        hom=[HomRxn("first_order", re=(0, -1), pr=(1, -1), k=1e-3)],
        het=[HetRxn(reactant=1, product=-1, surface=(SOLID_D,), mode="consumes",
                    irreversible=True, k=1e-2, C_eq=0.0, molar_volume=1.0)],
        type0=type0, V0=V0, rho1=rho1, rho2=rho2, C0=C0, steps=2000,
    )


def porous_medium(nx, ny, seed, porosity=0.55, rmin=8.0, rmax=24.0, reactive_frac=0.2,
                  gas_frac=0.3, bmin=6.0, bmax=16.0):
    """Random overlapping disks (periodic in x) until the porosity target; a
    disk that would overshoot the target by more than 0.5 % of the lattice (on
    small lattices a single grain can) is shrunk to the largest radius that
    does not, and ends the loop; grains chosen in random order become
    dissolvable (D) until the reactive fraction of solid nodes is reached, the
    rest inert; vapour bubbles on pore nodes until gas_frac of the pore space.
    Returns (type0, gas, rng)."""
    rng = _rng(seed)
    grain_id = np.full((ny, nx), -1, np.int64)
    n_solid = 0
    target = (1.0 - porosity) * nx * ny
    gid = 0
    while n_solid < target:
        cx = rng.uniform(0, nx)
        cy = rng.uniform(0, ny)
        r = rng.uniform(rmin, rmax)
        _, ys, xs = _stamp_disk(grain_id, cx, cy, r, True, False)
        new = grain_id[ys, xs] < 0
        last = False
        if n_solid + int(new.sum()) - target > 0.005 * nx * ny:
            lo, hi = 0.0, r  # the largest radius whose new nodes stay within the target
            for _ in range(40):
                mid = 0.5 * (lo + hi)
                _, ys_, xs_ = _stamp_disk(grain_id, cx, cy, mid, True, False)
                if n_solid + int((grain_id[ys_, xs_] < 0).sum()) <= target:
                    lo = mid
                else:
                    hi = mid
            _, ys, xs = _stamp_disk(grain_id, cx, cy, lo, True, False)
            new = grain_id[ys, xs] < 0
            last = True
        grain_id[ys[new], xs[new]] = gid
        n_solid += int(new.sum())
        gid += 1
        if last:
            break
    type0 = np.where(grain_id >= 0, SOLID_INERT, FLUID).astype(np.uint8)
    counts = np.bincount(grain_id[grain_id >= 0].ravel(), minlength=gid)
    order = rng.permutation(gid)
    need = reactive_frac * n_solid
    got = 0
    reactive = np.zeros(gid, bool)
    for g_ in order:
        if got >= need:
            break
        if counts[g_] == 0:
            continue
        reactive[g_] = True
        got += counts[g_]
    sel = (grain_id >= 0) & reactive[np.maximum(grain_id, 0)]
    type0[sel] = SOLID_D
    pore = type0 == FLUID
    n_pore = int(pore.sum())
    gas = np.zeros((ny, nx), bool)
    n_gas = 0
    pys, pxs = np.nonzero(pore)
    while n_gas < gas_frac * n_pore:
        i = int(rng.integers(0, n_pore))
        cx, cy = float(pxs[i]), float(pys[i])
        r = rng.uniform(bmin, bmax)
        _, ys, xs = _stamp_disk(gas, cx, cy, r, True, False)
        ok = pore[ys, xs] & ~gas[ys, xs]
        gas[ys[ok], xs[ok]] = True
        n_gas += int(ok.sum())
    return type0, gas, rng


def config1(nx=1024, ny=512, seed=1, steps=20000, porosity=0.55, rates=(1e-1, 1e-5, 1e-3, 1e-4)):
    """Porous medium: porosity 0.55, 20% of solid dissolvable, 30% of the pore space
    vapour bubbles, body force 1e-6 along x, periodic in x with walls in y; species
    A, B, E, F with A <-> B + C(g) (k1 = 0.1, K_eq = 1, M_C = 1e-3), B + E -> F
    (k3 = 1e-5), surface dissolution of D by B -> E (1e-3) and precipitation of F on
    D or F (1e-4, C_sa = 0).  `rates` are (k1, k3, dissolution, precipitation)."""
    a, b, R = EOS_PAPER
    T = 0.75 * critical_temperature(a, b, R)
    k1, k3, kd, kp = rates
    type0, gas, rng = porous_medium(nx, ny, seed, porosity=porosity)
    fl = type0 == FLUID
    rho1 = np.where(gas, RHO_V_075_PAPER, RHO_L_075_PAPER)
    rho2 = np.full((ny, nx), 0.1)
    n1 = rng.uniform(-1e-4, 1e-4, size=(ny, nx))
    n2 = rng.uniform(-1e-4, 1e-4, size=(ny, nx))
    rho1 = np.where(fl, rho1 + n1, 0.0)
    rho2 = np.where(fl, rho2 + n2, 0.0)
    V0 = np.where(type0 == SOLID_D, 1.0, 0.0)
    C0 = np.zeros((4, ny, nx))
    C0[0] = 1.0
    return Problem(
        name=f"porous-{nx}x{ny}", nx=nx, ny=ny, periodic_x=True, periodic_y=False,
        tau=(1.0, 1.0), gbody=(1e-6, 0.0), a=a, b=b, R=R, T=T, G11=-1.0, G12=0.5, G21=0.5,
        a0=0.005, rho10=paper_rho10(0.005), rho20=0.003,
        species=[Species("A"), Species("B"), Species("E"), Species("F")],
        hom=[HomRxn("r1_gas", re=(0, -1), pr=(1, -1), k=k1, K_eq=1.0, M_gas=1e-3),
             HomRxn("bimolecular", re=(1, 2), pr=(3, -1), k=k3)],
        het=[HetRxn(reactant=1, product=2, surface=(SOLID_D,), mode="consumes",
                    irreversible=True, k=kd, C_eq=0.0, molar_volume=1.0),
             HetRxn(reactant=3, product=-1, surface=(SOLID_D, SOLID_F), mode="grows",
                    irreversible=True, k=kp, C_eq=0.0, molar_volume=1.0)],
        type0=type0, V0=V0, rho1=rho1, rho2=rho2, C0=C0, steps=steps,
    )


def config2(n=4096, seed=2, steps=10000):
    """The porous-medium generator at 4096 x 4096 (the throughput workload)."""
    p = config1(nx=n, ny=n, seed=seed, steps=steps)
    p.name = f"porous-{n}x{n}"
    return p


def batch_instance_side(seed, smin=64, smax=1024):
    """The lattice side batch_instance(seed, smin, smax) draws (without
    generating the instance)."""
    rng = _rng(10_000 + seed)
    return int(round(np.exp(rng.uniform(np.log(smin), np.log(smax)))))


def batch_instance(seed, smin=64, smax=1024):
    """One instance of the many-simulations workload: the porous-medium
    generator on a square lattice whose side is log-uniform in [smin, smax],
    porosity uniform in [0.4, 0.8], each of the four rate constants log-uniform
    in [1e-6, 1e-1]."""
    rng = _rng(10_000 + seed)
    side = int(round(np.exp(rng.uniform(np.log(smin), np.log(smax)))))
    porosity = float(rng.uniform(0.4, 0.8))
    rates = tuple(float(np.exp(rng.uniform(np.log(1e-6), np.log(1e-1)))) for _ in range(4))
    p = config1(nx=side, ny=side, seed=seed, porosity=porosity, rates=rates)
    p.name = f"batch-{seed}-{side}x{side}"
    return p


def fracture(L=100, H=90, h0=30, g=1e-5, Da=0.001, Cs=1.0, molar_volume=300.0, k_sink=1e-3,
             tau_g=1.0, J0=0.9):
    """The dissolving fracture of App. A.3: an L x H box whose middle h0 rows
    are an open channel between two walls of dissolvable mineral, periodic in
    x, with one single-phase fluid (an ideal gas, no cohesion) driven by a body
    acceleration g along x.  The dissolved species starts at zero; the walls
    dissolve by the first-order law of Eq. A2 towards the saturation Cs with
    rate constant k = Da D / h0 (D from Eq. 24 for tau_g, J0).  A first-order
    sink of the dissolved species (rate k_sink) stands for the fresh solvent
    that flows in through the paper's inlet, so that the walls stay far from
    saturation and dissolve evenly along the channel; molar_volume sets how
    many steps a wall row lasts.  Input description only."""
    t = np.full((H, L), SOLID_D, np.uint8)
    lo = (H - h0) // 2
    t[lo:lo + h0] = FLUID
    D = 0.5 * (1.0 - J0) * (tau_g - 0.5)
    k = Da * D / h0
    p = uniform_problem(L, H, periodic_x=True, periodic_y=False, rho1=1.0, rho2=0.0,
                        species=[Species("M", tau_g=tau_g, J0=J0)], C0=np.zeros((1, H, L)),
                        gbody=(g, 0.0),
                        hom=[HomRxn("first_order", re=(0, -1), pr=(-1, -1), k=k_sink)],
                        het=[HetRxn(reactant=0, product=-1, surface=(SOLID_D,), mode="mineral",
                                    irreversible=False, k=k, C_eq=Cs, molar_volume=molar_volume)])
    return p.copy(type0=t, V0=np.where(t > 0, 1.0, 0.0), rho1=np.where(t == FLUID, 1.0, 0.0),
                  rho2=np.zeros((H, L)), name=f"fracture-{L}x{H}-h{h0}")


def uniform_problem(nx, ny, periodic_x=True, periodic_y=True, rho1=1.0, rho2=0.0,
                    species=(), C0=None, ideal=True, **kw):
    """A uniform fluid box.  With ideal=True the liquid component is an ideal gas
    with R T = 1/3 and a = b = 0, so its effective mass vanishes (no cohesion)."""
    type0 = np.zeros((ny, nx), np.uint8)
    r1 = np.full((ny, nx), float(rho1))
    r2 = np.full((ny, nx), float(rho2))
    ns = len(species)
    C = np.zeros((ns, ny, nx)) if C0 is None else np.asarray(C0, np.float64).reshape(ns, ny, nx)
    base = dict(name=f"uniform-{nx}x{ny}", nx=nx, ny=ny, periodic_x=periodic_x,
                periodic_y=periodic_y, species=list(species), type0=type0,
                V0=np.zeros((ny, nx)), rho1=r1, rho2=r2, C0=C)
    if ideal:
        base.update(a=0.0, b=0.0, R=1.0, T=1.0 / 3.0, G11=-1.0, G12=0.0, G21=0.0)
    base.update(kw)
    return Problem(**base)
