"""Field-by-field comparison helpers for the HIP path against the FP64 oracle.

Rules:
* fields (rho1, rho2, ux, uy, every C_k, V): max |gpu - oracle| / max |oracle|
  per field, below the tolerance of the precision;
* node types and liquid marks: identical, unless the oracle's state sits
  within the tolerance of a threshold that decides them (then the first
  step where that happens is reported and the comparison of masks stops).
"""
import dataclasses

import numpy as np

from paper_1410_3464_amd import workloads as W

FIELDS = ("rho1", "rho2", "ux", "uy", "V")


def rel_err(a, b):
    scale = np.abs(b).max()
    if scale == 0:
        return float(np.abs(a).max())
    return float(np.abs(a - b).max() / scale)


def field_errors(G, O, ns):
    err = {k: rel_err(G[k], O[k]) for k in FIELDS}
    for k in range(ns):
        err[f"C{k}"] = rel_err(G["C"][k], O["C"][k])
    return err


def near_threshold(O, prob, tol):
    """True when some mask decision of the oracle's last step was within tol of
    its threshold (liquid mark, solid volume 0, precipitate volume 1)."""
    fl = O["type"] == 0
    thr = prob.liquid_frac * O["rho_max_prev"]
    if fl.any() and np.any(np.abs(O["rho1"][fl] - thr) <= tol * max(thr, 1e-300)):
        return True
    V = O["V"]
    if np.any((np.abs(V) < tol) & (O["type"] >= 2)):
        return True
    if np.any((np.abs(V - 1.0) < tol) & fl):
        return True
    return False


def compare(G, O, prob, tol, led_tol=None):
    """Returns (errors, masks_equal, near)."""
    errs = field_errors(G, O, prob.n_species)
    masks = bool(np.array_equal(G["type"], O["type"]) and np.array_equal(G["liquid"], O["liquid"]))
    near = near_threshold(O, prob, tol)
    return errs, masks, near


def ledger_errors(LG, LO, ns):
    out = {}
    for k in ("mass_src", "mass_inj", "mass_rem"):
        out[k] = float(np.abs(np.asarray(LG[k]) - np.asarray(LO[k])).max())
    for k in ("sol_src", "sol_het", "sol_rem"):
        out[k] = float(np.abs(np.asarray(LG[k])[:ns] - np.asarray(LO[k])[:ns]).max()) if ns else 0.0
    for k in ("vol_dv", "vol_clip"):
        out[k] = abs(LG[k] - LO[k])
    for k in ("n_psi_clamp", "n_dissolved", "n_precipitated", "n_liq_to_gas", "n_gas_to_liq", "steps"):
        out[k] = abs(LG[k] - LO[k])
    return out


def species_variant(prob, ns):
    """The porous problem with `ns` species: the first min(ns, 4) as given
    (reactions that name a dropped species are dropped), the others copies of
    species 0-3 shifted by 4 with their own initial concentration and
    reactions, so that every species slot carries distinct values."""
    sp, C0 = [], np.zeros((ns,) + prob.C0.shape[1:])
    for q in range(ns):
        sp.append(dataclasses.replace(prob.species[q % 4], name=f"S{q}", tau_g=0.8 + 0.05 * q))
        C0[q] = prob.C0[q % 4] * (1.0 + 0.1 * (q // 4)) + 0.05 * q
    def ok(idx):
        return all(i < ns for i in idx if i >= 0)
    hom, het = [], []
    for off in range(0, ns, 4):
        for r in prob.hom:
            re_ = tuple(i + off if i >= 0 else -1 for i in r.re)
            pr_ = tuple(i + off if i >= 0 else -1 for i in r.pr)
            if ok(re_ + pr_):
                hom.append(dataclasses.replace(r, re=re_, pr=pr_))
        for r in prob.het:
            rp = r.product + off if r.product >= 0 else -1
            if ok((r.reactant + off, rp)):
                het.append(dataclasses.replace(r, reactant=r.reactant + off, product=rp))
    return prob.copy(species=sp, C0=C0, hom=hom[:8], het=het[:8], name=f"{prob.name}-ns{ns}")


def outlet_pool(outlet=True, seed=3, nx=32, ny=24):
    """nx x ny (32 x 24 by default), periodic in x, wall below; liquid (config-0 fluid) everywhere
    but a vapour bubble of radius 5, a sideways and downward body force, two
    species with A -> B."""
    a, b, R = W.EOS_PAPER
    T = 0.75 * W.critical_temperature(a, b, R)
    yy, xx = np.mgrid[0:ny, 0:nx]
    bub = (xx - nx // 2) ** 2 + (yy - ny // 2) ** 2 <= 25
    rng = np.random.Generator(np.random.PCG64(seed))
    rho1 = np.where(bub, W.RHO_V_075_PAPER, W.RHO_L_075_PAPER) + rng.uniform(-1e-4, 1e-4, (ny, nx))
    C0 = np.zeros((2, ny, nx))
    C0[0] = 1.0 + 0.1 * np.sin(2 * np.pi * xx / nx)
    return W.uniform_problem(
        nx, ny, periodic_x=True, periodic_y=False, outlet_top=outlet, ideal=False, a=a, b=b, R=R, T=T,
        G11=-1.0, G12=0.5, G21=0.5, rho10=W.paper_rho10(), rho20=0.003, a0=0.005, rho1=1.0,
        gbody=(2e-5, -1e-5), species=[W.Species("A", 1.0, 0.9), W.Species("B", 1.0, 0.9)],
        hom=[W.HomRxn("first_order", re=(0, -1), pr=(1, -1), k=1e-3)],
    ).copy(rho1=rho1, rho2=np.full((ny, nx), 0.1), C0=C0)
