"""ctypes binding of the lbrx C ABI (include/lbrx.h).

Argument marshalling only: every part of the step runs in the HIP kernels of
liblbrx.so.  There is no CPU fallback; if the library is missing the import of
this module's functions raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbrx.so")

ABI_VERSION = 6
MAXS = 8
MAXR = 8
F64, F32, F16DEV, BF16DEV = 0, 1, 2, 3
_PREC = {"f64": F64, "f32": F32, "f16dev": F16DEV, "bf16dev": BF16DEV}
_HOM = {"first_order": 0, "r1_gas": 1, "bimolecular": 2}
_HET = {"consumes": 0, "grows": 1, "mineral": 2}
STATUS = {0: "LBRX_OK", 1: "LBRX_E_INVAL", 2: "LBRX_E_NOMEM", 3: "LBRX_E_DEVICE",
          4: "LBRX_E_UNSTABLE", 5: "LBRX_E_STATE"}

# every symbol include/lbrx.h declares
SYMBOLS = ("lbrx_create", "lbrx_create_error", "lbrx_step", "lbrx_sync", "lbrx_fields", "lbrx_fields_noalloc",
           "lbrx_step_count", "lbrx_stream", "lbrx_destroy", "lbrx_last_error",
           "lbrx_status_string", "lbrx_batch_create", "lbrx_batch_step", "lbrx_batch_last_error",
           "lbrx_batch_destroy", "lbrx_state_bytes", "lbrx_save_state", "lbrx_load_state")


class HomRxn(C.Structure):
    _fields_ = [("kind", C.c_int32), ("re", C.c_int32 * 2), ("pr", C.c_int32 * 2),
                ("k", C.c_double), ("K_eq", C.c_double), ("M_gas", C.c_double),
                ("surface", C.c_uint32), ("surface_factor", C.c_double)]


class HetRxn(C.Structure):
    _fields_ = [("reactant", C.c_int32), ("product", C.c_int32), ("surface", C.c_uint32),
                ("mode", C.c_int32), ("irreversible", C.c_int32),
                ("k", C.c_double), ("C_eq", C.c_double), ("molar_volume", C.c_double)]


class Params(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32), ("nx", C.c_int32), ("ny", C.c_int32), ("periodic", C.c_uint32),
        ("precision", C.c_int32),
        ("tau", C.c_double * 2), ("w_adh", C.c_double * 2), ("gbody", C.c_double * 2),
        ("a", C.c_double), ("b", C.c_double), ("R", C.c_double), ("T", C.c_double),
        ("G11", C.c_double), ("G12", C.c_double), ("G21", C.c_double),
        ("a0", C.c_double), ("rho10", C.c_double), ("rho20", C.c_double),
        ("liquid_frac", C.c_double),
        ("n_species", C.c_int32), ("tau_g", C.c_double * MAXS), ("J0", C.c_double * MAXS),
        ("n_hom", C.c_int32), ("hom", HomRxn * MAXR),
        ("n_het", C.c_int32), ("het", HetRxn * MAXR),
        ("node_type", C.c_void_p), ("V0", C.c_void_p), ("rho1", C.c_void_p), ("rho2", C.c_void_p),
        ("C0", C.c_void_p), ("seg_rows", C.c_int32), ("psi_prefactor", C.c_double),
        ("dev_alloc", C.c_void_p), ("dev_free", C.c_void_p), ("alloc_user", C.c_void_p),
        ("subtract_species", C.c_int32), ("subtract_total", C.c_double),
    ]


# device allocator callbacks of lbrx_params
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_uint64, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


def torch_allocator(stream=None):
    """(dev_alloc, dev_free) callbacks drawing the context's device memory from
    PyTorch's caching allocator (associated with `stream`, a HIP stream handle,
    if given).  Keep the returned pair alive as long as the context."""
    import torch

    def alloc(n, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(n), stream=stream)
        except RuntimeError:  # out of memory: the library reports LBRX_E_NOMEM
            return None

    def free(ptr, user):
        torch.cuda.caching_allocator_delete(ptr)

    return ALLOC_FN(alloc), FREE_FN(free)


LEDGER_FIELDS = [("mass_src", 2), ("mass_inj", 2), ("mass_rem", 2), ("sol_src", MAXS),
                 ("sol_het", MAXS), ("sol_rem", MAXS), ("vol_dv", 1), ("vol_clip", 1),
                 ("n_psi_clamp", 1), ("n_dissolved", 1), ("n_precipitated", 1),
                 ("n_liq_to_gas", 1), ("n_gas_to_liq", 1), ("steps", 1)]
LEDGER_LEN = sum(n for _, n in LEDGER_FIELDS)


class FieldsOut(C.Structure):
    _fields_ = [("rho1", C.c_void_p), ("rho2", C.c_void_p), ("ux", C.c_void_p), ("uy", C.c_void_p),
                ("C", C.c_void_p), ("V", C.c_void_p), ("type", C.c_void_p), ("liquid", C.c_void_p),
                ("ledger", C.c_void_p), ("rho_max", C.c_void_p)]


class LbrxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def _init_torch_first():
    """PyTorch carries its own HIP runtime.  When the library's runtime
    initialises the device first, PyTorch's later finds no device, so PyTorch
    (whose streams and allocator the binding uses) is initialised before the
    library is loaded; without a device nothing is done."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.device_count() > 0:
        torch.cuda.init()


def load_library(path=LIB_PATH):
    """Load liblbrx.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with `python -m paper_1410_3464_amd.build`")
    _init_torch_first()
    lib = C.CDLL(path)
    lib.lbrx_create.restype = C.c_int
    lib.lbrx_create.argtypes = [C.POINTER(Params), C.c_void_p, C.POINTER(C.c_void_p)]
    lib.lbrx_create_error.restype = C.c_char_p
    lib.lbrx_create_error.argtypes = []
    lib.lbrx_step.restype = C.c_int
    lib.lbrx_step.argtypes = [C.c_void_p, C.c_int64]
    lib.lbrx_sync.restype = C.c_int
    lib.lbrx_sync.argtypes = [C.c_void_p]
    lib.lbrx_fields.restype = C.c_int
    lib.lbrx_fields.argtypes = [C.c_void_p, C.POINTER(FieldsOut)]
    lib.lbrx_fields_noalloc.restype = C.c_int
    lib.lbrx_fields_noalloc.argtypes = [C.c_void_p, C.POINTER(FieldsOut)]
    lib.lbrx_step_count.restype = C.c_int64
    lib.lbrx_step_count.argtypes = [C.c_void_p]
    lib.lbrx_stream.restype = C.c_void_p
    lib.lbrx_stream.argtypes = [C.c_void_p]
    lib.lbrx_destroy.restype = C.c_int
    lib.lbrx_destroy.argtypes = [C.c_void_p]
    lib.lbrx_last_error.restype = C.c_char_p
    lib.lbrx_last_error.argtypes = [C.c_void_p]
    lib.lbrx_status_string.restype = C.c_char_p
    lib.lbrx_status_string.argtypes = [C.c_int]
    lib.lbrx_state_bytes.restype = C.c_int
    lib.lbrx_state_bytes.argtypes = [C.c_void_p, C.POINTER(C.c_uint64)]
    lib.lbrx_save_state.restype = C.c_int
    lib.lbrx_save_state.argtypes = [C.c_void_p, C.c_void_p, C.c_uint64]
    lib.lbrx_load_state.restype = C.c_int
    lib.lbrx_load_state.argtypes = [C.c_void_p, C.c_void_p, C.c_uint64]
    lib.lbrx_batch_create.restype = C.c_int
    lib.lbrx_batch_create.argtypes = [C.POINTER(C.c_void_p), C.c_int, C.POINTER(C.c_void_p)]
    lib.lbrx_batch_step.restype = C.c_int
    lib.lbrx_batch_step.argtypes = [C.c_void_p, C.c_int64]
    lib.lbrx_batch_last_error.restype = C.c_char_p
    lib.lbrx_batch_last_error.argtypes = [C.c_void_p]
    lib.lbrx_batch_destroy.restype = C.c_int
    lib.lbrx_batch_destroy.argtypes = [C.c_void_p]
    _lib = lib
    return lib


def make_params(prob, precision="f64", seg_rows=0):
    """lbrx_params for a workloads.Problem; returns (params, keep-alive arrays)."""
    p = Params()
    p.abi_version = ABI_VERSION
    p.seg_rows = int(seg_rows)
    p.nx, p.ny = prob.nx, prob.ny
    p.periodic = (1 if prob.periodic_x else 0) | (2 if prob.periodic_y else 0) | (4 if prob.outlet_top else 0)
    p.precision = _PREC[precision]
    p.tau[:] = list(prob.tau)
    p.w_adh[:] = list(prob.w_adh)
    p.gbody[:] = list(prob.gbody)
    for k in ("a", "b", "R", "T", "G11", "G12", "G21", "a0", "rho10", "rho20", "liquid_frac"):
        setattr(p, k, float(getattr(prob, k)))
    if prob.n_species > MAXS or len(prob.hom) > MAXR or len(prob.het) > MAXR:
        raise ValueError("too many species or reactions")
    p.n_species = prob.n_species
    for i, sp in enumerate(prob.species):
        p.tau_g[i], p.J0[i] = sp.tau_g, sp.J0
    p.n_hom = len(prob.hom)
    for i, r in enumerate(prob.hom):
        h = p.hom[i]
        h.kind = _HOM[r.kind]
        h.re[0], h.re[1] = r.re
        h.pr[0], h.pr[1] = r.pr
        h.k, h.K_eq, h.M_gas = r.k, r.K_eq, r.M_gas
        h.surface = sum(1 << t for t in r.surface)
        h.surface_factor = r.surface_factor
    p.psi_prefactor = float(prob.psi_prefactor)
    p.subtract_species = int(getattr(prob, "subtract_species", -1))
    p.subtract_total = float(getattr(prob, "subtract_total", 0.0))
    p.n_het = len(prob.het)
    for i, r in enumerate(prob.het):
        h = p.het[i]
        h.reactant, h.product = r.reactant, r.product
        h.surface = sum(1 << t for t in r.surface)
        h.mode = _HET[r.mode]
        h.irreversible = int(r.irreversible)
        h.k, h.C_eq, h.molar_volume = r.k, r.C_eq, r.molar_volume
    N = prob.nx * prob.ny
    keep = dict(
        t=np.ascontiguousarray(prob.type0, np.uint8).reshape(N),
        V=None if prob.V0 is None else np.ascontiguousarray(prob.V0, np.float64).reshape(N),
        r1=np.ascontiguousarray(prob.rho1, np.float64).reshape(N),
        r2=np.ascontiguousarray(prob.rho2, np.float64).reshape(N),
        C=np.ascontiguousarray(prob.C0, np.float64).reshape(-1) if prob.n_species else None,
    )
    p.node_type = keep["t"].ctypes.data
    p.V0 = keep["V"].ctypes.data if keep["V"] is not None else None
    p.rho1 = keep["r1"].ctypes.data
    p.rho2 = keep["r2"].ctypes.data
    p.C0 = keep["C"].ctypes.data if keep["C"] is not None else None
    return p, keep


def _ptr(a):
    return a.ctypes.data if a is not None else None


class Lbrx:
    """One GPU simulation of a workloads.Problem (a context of the C ABI)."""

    def __init__(self, prob, precision="f64", stream=None, seg_rows=0, allocator=None):
        """allocator: None (the library's hipMalloc) or "torch" (PyTorch's
        caching allocator supplies the device memory)."""
        lib = load_library()
        self._lib = lib
        self.prob = prob
        self.nx, self.ny, self.ns = prob.nx, prob.ny, prob.n_species
        self.precision = precision
        params, keep = make_params(prob, precision, seg_rows)
        self._hooks = None
        if allocator == "torch":
            self._hooks = torch_allocator(stream)
            params.dev_alloc = C.cast(self._hooks[0], C.c_void_p)
            params.dev_free = C.cast(self._hooks[1], C.c_void_p)
        elif allocator is not None:
            raise ValueError(f"unknown allocator {allocator!r}")
        h = C.c_void_p()
        st = lib.lbrx_create(C.byref(params), stream, C.byref(h))
        if st != 0:
            raise LbrxError(st, lib.lbrx_create_error().decode())
        self._h = h
        del keep

    def _check(self, st):
        if st != 0:
            raise LbrxError(st, self._lib.lbrx_last_error(self._h).decode())

    def step(self, n=1):
        self._check(self._lib.lbrx_step(self._h, int(n)))

    def sync(self):
        self._check(self._lib.lbrx_sync(self._h))

    @property
    def steps_done(self):
        return int(self._lib.lbrx_step_count(self._h))

    @property
    def stream(self):
        return self._lib.lbrx_stream(self._h)

    def fields(self, noalloc=False, only=None):
        """The fields in FP64 (lbrx_fields; lbrx_fields_noalloc with noalloc=True).
        `only`: names of the fields wanted (rho1, rho2, ux, uy, C, V, type,
        liquid, ledger, rho_max_prev); the others are not read out."""
        N, ny, nx, ns = self.nx * self.ny, self.ny, self.nx, self.ns
        want = (lambda k: True) if only is None else (lambda k: k in only)
        r1, r2, ux, uy, V = (np.zeros(N) for _ in range(5))
        Cc = np.zeros(max(ns, 1) * N)
        t = np.zeros(N, np.uint8)
        lq = np.zeros(N, np.uint8)
        led = np.zeros(LEDGER_LEN)
        rmax = np.zeros(1)
        arrs = dict(rho1=r1, rho2=r2, ux=ux, uy=uy, C=Cc, V=V, type=t, liquid=lq, ledger=led, rho_max_prev=rmax)
        o = FieldsOut(*(_ptr(a) if want(k) else None for k, a in arrs.items()))
        fn = self._lib.lbrx_fields_noalloc if noalloc else self._lib.lbrx_fields
        self._check(fn(self._h, C.byref(o)))
        out = dict(rho1=r1.reshape(ny, nx), rho2=r2.reshape(ny, nx), ux=ux.reshape(ny, nx),
                   uy=uy.reshape(ny, nx), C=Cc[: ns * N].reshape(ns, ny, nx), type=t.reshape(ny, nx),
                   liquid=lq.reshape(ny, nx), V=V.reshape(ny, nx), rho_max_prev=float(rmax[0]))
        out["ledger"] = unpack_ledger(led)
        return {k: v for k, v in out.items() if want(k)}

    def save_state(self):
        """The whole simulation state (lbrx_save_state) as a uint8 array."""
        n = C.c_uint64()
        self._check(self._lib.lbrx_state_bytes(self._h, C.byref(n)))
        buf = np.empty(n.value, np.uint8)
        self._check(self._lib.lbrx_save_state(self._h, buf.ctypes.data, n.value))
        return buf

    def load_state(self, buf):
        """Replace the state by one returned by save_state (lbrx_load_state)."""
        buf = np.ascontiguousarray(buf, np.uint8)
        self._check(self._lib.lbrx_load_state(self._h, buf.ctypes.data, buf.size))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.lbrx_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def unpack_ledger(arr):
    out, o = {}, 0
    for name, n in LEDGER_FIELDS:
        v = np.array(arr[o:o + n], dtype=np.float64)
        out[name] = v if n > 1 else float(v[0])
        o += n
    return out


class Batch:
    """Several Lbrx contexts (same stream, precision and species count)
    advanced by one kernel launch per step (lbrx_batch_*)."""

    def __init__(self, sims):
        lib = load_library()
        self._lib = lib
        self.sims = list(sims)
        arr = (C.c_void_p * len(self.sims))(*[s._h.value for s in self.sims])
        h = C.c_void_p()
        st = lib.lbrx_batch_create(arr, len(self.sims), C.byref(h))
        if st != 0:
            raise LbrxError(st, "lbrx_batch_create rejected the contexts")
        self._h = h

    def step(self, n=1):
        st = self._lib.lbrx_batch_step(self._h, int(n))
        if st != 0:
            raise LbrxError(st, self._lib.lbrx_batch_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.lbrx_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
