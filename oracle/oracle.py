"""ctypes wrapper of the plain FP64 C oracle (oracle/lbrx_oracle.c).

Test infrastructure only: it is called by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbrx_oracle.c")
_LIB = os.path.join(_HERE, "liblbrx_oracle.so")

MAXS = 8
MAXR = 8
_HOM_KIND = {"first_order": 0, "r1_gas": 1, "bimolecular": 2}
_HET_MODE = {"consumes": 0, "grows": 1, "mineral": 2}


class _Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("periodic_x", C.c_int32), ("periodic_y", C.c_int32),
        ("tau", C.c_double * 2), ("w_adh", C.c_double * 2), ("gbody", C.c_double * 2),
        ("a", C.c_double), ("b", C.c_double), ("R", C.c_double), ("T", C.c_double),
        ("G11", C.c_double), ("G12", C.c_double), ("G21", C.c_double),
        ("a0", C.c_double), ("rho10", C.c_double), ("rho20", C.c_double),
        ("liquid_frac", C.c_double), ("psi_pre", C.c_double),
        ("n_species", C.c_int32), ("tau_g", C.c_double * MAXS), ("J0", C.c_double * MAXS),
        ("n_hom", C.c_int32), ("hom_kind", C.c_int32 * MAXR),
        ("hom_re", (C.c_int32 * 2) * MAXR), ("hom_pr", (C.c_int32 * 2) * MAXR),
        ("hom_k", C.c_double * MAXR), ("hom_Keq", C.c_double * MAXR), ("hom_Mgas", C.c_double * MAXR),
        ("hom_surface", C.c_int32 * MAXR), ("hom_sfac", C.c_double * MAXR),
        ("n_het", C.c_int32), ("het_reactant", C.c_int32 * MAXR), ("het_product", C.c_int32 * MAXR),
        ("het_surface", C.c_int32 * MAXR), ("het_mode", C.c_int32 * MAXR), ("het_irrev", C.c_int32 * MAXR),
        ("het_k", C.c_double * MAXR), ("het_Ceq", C.c_double * MAXR), ("het_mvol", C.c_double * MAXR),
        ("outlet_top", C.c_int32),
        ("sub_species", C.c_int32),
        ("sub_total", C.c_double),
    ]


LEDGER_FIELDS = (
    [("mass_src", 2), ("mass_inj", 2), ("mass_rem", 2), ("sol_src", MAXS), ("sol_het", MAXS),
     ("sol_rem", MAXS), ("vol_dv", 1), ("vol_clip", 1), ("n_psi_clamp", 1), ("n_dissolved", 1),
     ("n_precipitated", 1), ("n_liq_to_gas", 1), ("n_gas_to_liq", 1), ("steps", 1)]
)
_LEDGER_LEN = sum(n for _, n in LEDGER_FIELDS)


def oracle_lib_path():
    return _LIB


def build_oracle(force=False):
    """Compile the oracle with gcc (plain -O2, no FP contraction, no fast-math;
    OpenMP for the optional host threads, which change no result)."""
    hdr = os.path.join(_HERE, "lbrx_oracle.h")
    stale = not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC), os.path.getmtime(hdr))
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build_oracle()
        lib = C.CDLL(_LIB)
        lib.orc_create.restype = C.c_void_p
        lib.orc_create.argtypes = [C.POINTER(_Params), C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_char_p, C.c_int]
        lib.orc_step.restype = C.c_int
        lib.orc_step.argtypes = [C.c_void_p, C.c_int]
        lib.orc_fields.restype = None
        lib.orc_fields.argtypes = [C.c_void_p] + [C.c_void_p] * 10
        lib.orc_state.restype = None
        lib.orc_state.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        lib.orc_error.restype = C.c_char_p
        lib.orc_error.argtypes = [C.c_void_p]
        lib.orc_step_count.restype = C.c_int64
        lib.orc_step_count.argtypes = [C.c_void_p]
        lib.orc_destroy.restype = None
        lib.orc_destroy.argtypes = [C.c_void_p]
        lib.orc_set_threads.restype = None
        lib.orc_set_threads.argtypes = [C.c_void_p, C.c_int]
        lib.orc_margins.restype = None
        lib.orc_margins.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _params(prob, psi_literal=False):
    p = _Params()
    p.nx, p.ny = prob.nx, prob.ny
    p.periodic_x, p.periodic_y = int(prob.periodic_x), int(prob.periodic_y)
    p.tau[:] = list(prob.tau)
    p.w_adh[:] = list(prob.w_adh)
    p.gbody[:] = list(prob.gbody)
    for k in ("a", "b", "R", "T", "G11", "G12", "G21", "a0", "rho10", "rho20", "liquid_frac"):
        setattr(p, k, float(getattr(prob, k)))
    # Eq. 13 as printed (6) when asked for, else the problem's prefactor (0: 2)
    p.psi_pre = 6.0 if psi_literal else (float(prob.psi_prefactor) or 2.0)
    if prob.n_species > MAXS or len(prob.hom) > MAXR or len(prob.het) > MAXR:
        raise ValueError("too many species or reactions")
    p.n_species = prob.n_species
    for i, sp in enumerate(prob.species):
        p.tau_g[i] = sp.tau_g
        p.J0[i] = sp.J0
    p.n_hom = len(prob.hom)
    for i, r in enumerate(prob.hom):
        p.hom_kind[i] = _HOM_KIND[r.kind]
        p.hom_re[i][0], p.hom_re[i][1] = r.re
        p.hom_pr[i][0], p.hom_pr[i][1] = r.pr
        p.hom_k[i], p.hom_Keq[i], p.hom_Mgas[i] = r.k, r.K_eq, r.M_gas
        p.hom_surface[i] = sum(1 << t for t in r.surface)
        p.hom_sfac[i] = r.surface_factor
    p.n_het = len(prob.het)
    for i, r in enumerate(prob.het):
        p.het_reactant[i], p.het_product[i] = r.reactant, r.product
        p.het_surface[i] = sum(1 << t for t in r.surface)
        p.het_mode[i] = _HET_MODE[r.mode]
        p.het_irrev[i] = int(r.irreversible)
        p.het_k[i], p.het_Ceq[i], p.het_mvol[i] = r.k, r.C_eq, r.molar_volume
    p.outlet_top = int(prob.outlet_top)
    p.sub_species = int(getattr(prob, "subtract_species", -1))
    p.sub_total = float(getattr(prob, "subtract_total", 0.0))
    return p


class OracleSim:
    """One oracle simulation of a workloads.Problem.  threads: host threads for
    the node loops (balances stay serial in node order; results are the same
    for any count)."""

    def __init__(self, prob, psi_literal=False, threads=1):
        lib = _load()
        self.prob = prob
        self.nx, self.ny, self.ns = prob.nx, prob.ny, prob.n_species
        self._p = _params(prob, psi_literal)
        N = prob.nx * prob.ny
        t0 = np.ascontiguousarray(prob.type0, np.uint8).reshape(N)
        V0 = None if prob.V0 is None else np.ascontiguousarray(prob.V0, np.float64).reshape(N)
        r1 = np.ascontiguousarray(prob.rho1, np.float64).reshape(N)
        r2 = np.ascontiguousarray(prob.rho2, np.float64).reshape(N)
        c0 = np.ascontiguousarray(prob.C0, np.float64).reshape(max(prob.n_species, 0) * N)
        if c0.size == 0:
            c0 = np.zeros(1)
        err = C.create_string_buffer(256)
        h = lib.orc_create(C.byref(self._p), _ptr(t0), _ptr(V0), _ptr(r1), _ptr(r2), _ptr(c0), err, 256)
        if not h:
            raise ValueError(err.value.decode())
        self._h = h
        self._lib = lib
        lib.orc_set_threads(h, int(threads))

    def step(self, n=1):
        if self._lib.orc_step(self._h, int(n)) != 0:
            raise FloatingPointError(self._lib.orc_error(self._h).decode())

    @property
    def steps_done(self):
        return int(self._lib.orc_step_count(self._h))

    def fields(self):
        N, ny, nx, ns = self.nx * self.ny, self.ny, self.nx, self.ns
        r1, r2, ux, uy, V = (np.zeros(N) for _ in range(5))
        Cc = np.zeros(max(ns, 1) * N)
        t = np.zeros(N, np.uint8)
        lq = np.zeros(N, np.uint8)
        led = np.zeros(_LEDGER_LEN)
        rmax = np.zeros(1)
        self._lib.orc_fields(self._h, _ptr(r1), _ptr(r2), _ptr(ux), _ptr(uy), _ptr(Cc), _ptr(t),
                             _ptr(lq), _ptr(V), _ptr(led), _ptr(rmax))
        out = dict(rho1=r1.reshape(ny, nx), rho2=r2.reshape(ny, nx), ux=ux.reshape(ny, nx),
                   uy=uy.reshape(ny, nx), C=Cc[: ns * N].reshape(ns, ny, nx), type=t.reshape(ny, nx),
                   liquid=lq.reshape(ny, nx), V=V.reshape(ny, nx), rho_max_prev=float(rmax[0]))
        out["ledger"] = unpack_ledger(led)
        return out

    def state(self):
        N, ns = self.nx * self.ny, self.ns
        f = np.zeros(18 * N)
        g = np.zeros(max(5 * ns * N, 1))
        fl = np.zeros(N, np.uint8)
        self._lib.orc_state(self._h, _ptr(f), _ptr(g), _ptr(fl))
        return f.reshape(2, 9, self.ny, self.nx), g[: 5 * ns * N].reshape(ns, 5, self.ny, self.nx), \
            fl.reshape(self.ny, self.nx)

    def margins(self):
        """(liquid, volume): the smallest decision margins of the steps since
        the previous call (relative for the liquid threshold, absolute for the
        volume thresholds 0 and 1); inf when no such decision was taken."""
        a, b = C.c_double(), C.c_double()
        self._lib.orc_margins(self._h, C.byref(a), C.byref(b))
        return a.value, b.value

    def close(self):
        if getattr(self, "_h", None):
            self._lib.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def unpack_ledger(arr):
    out = {}
    o = 0
    for name, n in LEDGER_FIELDS:
        v = np.array(arr[o:o + n], dtype=np.float64)
        out[name] = v if n > 1 else float(v[0])
        o += n
    return out
