"""ctypes binding of libes.so (the HIP/gfx950 C-ABI declared in include/es.h).

Argument marshalling only: every step of the scheme runs in the library's
kernels.  PyTorch supplies device memory and the current stream.  Importing
this module loads libes.so and raises if it is missing; creating a Context
raises if no HIP device is present.  There is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libes.so")

ES_OK, ES_EINVAL, ES_EUNSUPPORTED, ES_EHIP, ES_ENONPHYS, ES_ETANGLE = 0, -1, -2, -3, -4, -5
ES_ST_NONPHYS, ES_ST_TANGLE = 1, 2
ES_FP64, ES_MIXED = 0, 1
ES_WENO_MR, ES_WENO_JS = 0, 1
ES_MONITOR_GRAD2, ES_MONITOR_GRAD_LAP = 0, 1
ES_METRICS_VCL_ONLY = 1
ES_BC_PERIODIC, ES_BC_REFLECT, ES_BC_OUTFLOW, ES_BC_INFLOW = 0, 1, 2, 3


class EsError(RuntimeError):
    def __init__(self, name, code):
        super().__init__(f"{name} failed with code {code}")
        self.code = code


class EsGrid(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("nspec", C.c_int), ("n", C.c_int * 3), ("ng", C.c_int),
        ("dxi", C.c_double * 3), ("len", C.c_double * 3), ("w", C.c_int),
        ("gamma", C.c_double * 2), ("cv", C.c_double * 2), ("pinf", C.c_double * 2),
        ("chi", C.c_double * 3), ("weno_eps", C.c_double), ("dissipation", C.c_int),
        ("precision", C.c_int), ("reconstruction", C.c_int), ("bc", (C.c_int * 2) * 3),
        ("wall", (C.c_double * 2) * 3), ("inflow", ((C.c_double * 6) * 2) * 3),
        ("sign_tol", C.c_double), ("sign_tol32", C.c_double),
    ]


class EsMonitor(C.Structure):
    _fields_ = [
        ("nsig", C.c_int), ("sigma", C.c_int * 6), ("alpha", C.c_double * 6),
        ("n_smooth", C.c_int), ("n_sweeps", C.c_int), ("form", C.c_int), ("beta", C.c_double * 6),
        ("psi", C.c_double * 2),
    ]


_P = C.c_void_p
_SIGS = {
    "es_create": [C.POINTER(EsGrid), C.POINTER(C.c_void_p)],
    "es_destroy": [_P],
    "es_fill_ghosts": [_P, _P, C.c_int, _P],
    "es_fill_ghosts_x": [_P, _P, _P],
    "es_fill_ghosts_state": [_P, _P, _P, _P],
    "es_metrics": [_P, _P, _P, C.c_double, _P, _P, _P, C.c_int, _P],
    "es_rhs": [_P, _P, _P, _P, _P, _P, _P, _P],
    "es_rk_stage": [_P, C.c_int, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P],
    "max_wavespeed": [_P, _P, _P, _P, C.c_double, _P, _P, _P],
    "max_wavespeed_noalloc": [C.POINTER(EsGrid), _P, _P, _P, C.c_double, _P, _P, _P, _P],
    "mesh_redistribute": [_P, C.POINTER(EsMonitor), _P, _P, _P, _P, _P, _P, _P],
    "es_jacobian": [_P, _P, _P, _P, _P],
    "es_entropy": [_P, _P, _P, _P, _P],
    "es_entropy_rate": [_P, _P, _P, _P, _P, _P, _P],
    "es_step": [_P, C.POINTER(EsMonitor), C.c_double, C.c_double, C.c_int, _P, _P, _P, _P, _P, _P],
    "es_status": [_P, _P, C.POINTER(C.c_uint), C.c_int],
    "es_npoints": [_P],
    "es_batch_create": [C.c_void_p, C.c_int, _P],
    "es_batch_destroy": [_P],
    "es_rk_stage_batched": [_P, C.c_int, _P, _P, _P],
    "max_wavespeed_batched": [_P, _P, _P, _P, C.c_double, _P, _P, _P],
    "es_step_batched": [_P, C.c_double, _P, _P, _P, _P, _P, _P],
    "es_batch_autotune": [_P, _P, _P, _P, _P, _P, C.c_int, _P, _P],
    "es_batch_set_tiling": [_P, C.c_int, C.c_int, C.c_int],
    "es_batch_status": [_P, _P, C.POINTER(C.c_uint), C.c_int],
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2202_07989_amd/build.py "
                          "(there is no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    for name, args in _SIGS.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_long if name == "es_npoints" else C.c_int
    return lib


lib = _load()


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if t.device.type != "cuda" or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("libes takes contiguous float64 device tensors")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _check(name, rc):
    if rc != ES_OK:
        raise EsError(name, rc)


def make_grid(spec, precision=ES_FP64) -> EsGrid:
    g = EsGrid()
    g.dim, g.nspec = spec["dim"], spec["nspec"]
    n = list(spec["n"]) + [1] * (3 - len(spec["n"]))
    for k in range(3):
        g.n[k] = n[k]
        g.dxi[k] = spec["dxi"][k] if k < len(spec["dxi"]) else 1.0
        g.len[k] = spec["len"][k] if k < len(spec["len"]) else 1.0
    g.ng, g.w = spec.get("ng", 3), spec.get("w", 3)
    for l in range(2):
        g.gamma[l] = spec["gamma"][l] if l < len(spec["gamma"]) else 1.4
        g.cv[l] = spec["cv"][l] if l < len(spec["cv"]) else 1.0
        g.pinf[l] = spec["pinf"][l] if l < len(spec["pinf"]) else 0.0
    for m in range(3):
        g.chi[m] = spec["chi"][m]
    g.weno_eps = spec.get("weno_eps", 1e-10)
    g.dissipation = spec.get("dissipation", 1)
    g.reconstruction = spec.get("reconstruction", ES_WENO_MR)
    g.precision = precision
    for k, faces in enumerate(spec.get("bc", [])):
        for side in range(2):
            g.bc[k][side] = faces[side]
    for k, faces in enumerate(spec.get("wall", [])):
        for side in range(2):
            g.wall[k][side] = faces[side]
    for (k, side), U in spec.get("inflow", {}).items():
        for c, u in enumerate(U):
            g.inflow[k][side][c] = u
    # zero tolerances of the sign matrix (0: the paper's rule as printed)
    g.sign_tol = spec.get("sign_tol", 1e-12)
    g.sign_tol32 = spec.get("sign_tol32", 1e-6)
    return g


def make_monitor(mon) -> EsMonitor:
    m = EsMonitor()
    sig, al = mon.get("sigma", [0]), mon.get("alpha", [1200.0])
    m.nsig = len(sig)
    for t in range(len(sig)):
        m.sigma[t], m.alpha[t] = sig[t], al[t]
    m.n_smooth, m.n_sweeps = mon.get("n_smooth", 3), mon.get("n_sweeps", 10)
    m.form = mon.get("form", ES_MONITOR_GRAD2)
    for t, b in enumerate(mon.get("beta", [])):
        m.beta[t] = b
    for t, q in enumerate(mon.get("psi", [])):
        m.psi[t] = q
    return m


def max_wavespeed_noalloc(spec, JU, J, jxi_x, cfl, lambda_dev=None, dt_dev=None, status_dev=None,
                          precision=ES_FP64, stream=None):
    """max_wavespeed without a context and without any allocation (the
    library's static device scratch); status_dev is an int32 device tensor
    of one element or None."""
    g = make_grid(spec, precision)
    st = None
    if status_dev is not None:
        if status_dev.device.type != "cuda" or status_dev.dtype != torch.int32:
            raise ValueError("status_dev must be a one-element int32 device tensor")
        st = C.c_void_p(status_dev.data_ptr())
    _check("max_wavespeed_noalloc",
           lib.max_wavespeed_noalloc(C.byref(g), _ptr(JU), _ptr(J), _ptr(jxi_x), cfl, _ptr(lambda_dev),
                                     _ptr(dt_dev), st, _stream(stream)))


class Context:
    """One es_ctx: a grid on the current HIP device."""

    def __init__(self, spec, precision=ES_FP64):
        if not torch.cuda.is_available():
            raise RuntimeError("libes needs a HIP device; there is no CPU fallback")
        self.spec = spec
        self.grid = make_grid(spec, precision)
        h = C.c_void_p()
        _check("es_create", lib.es_create(C.byref(self.grid), C.byref(h)))
        self.h = h
        self.P = lib.es_npoints(self.h)
        self.nc = spec["nspec"] + spec["dim"] + 1
        self.dim = spec["dim"]

    def close(self):
        if self.h:
            lib.es_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the C-ABI, one method per entry point --------------------------------
    def es_fill_ghosts(self, a, ncomp, stream=None):
        _check("es_fill_ghosts", lib.es_fill_ghosts(self.h, _ptr(a), ncomp, _stream(stream)))

    def es_fill_ghosts_x(self, x, stream=None):
        _check("es_fill_ghosts_x", lib.es_fill_ghosts_x(self.h, _ptr(x), _stream(stream)))

    def es_fill_ghosts_state(self, JU, J, stream=None):
        _check("es_fill_ghosts_state", lib.es_fill_ghosts_state(self.h, _ptr(JU), _ptr(J), _stream(stream)))

    def es_metrics(self, x_n, disp, c_s, dt_dev, jxi_x, jxi_t, flags=0, stream=None):
        _check("es_metrics", lib.es_metrics(self.h, _ptr(x_n), _ptr(disp), float(c_s), _ptr(dt_dev),
                                            _ptr(jxi_x), _ptr(jxi_t), flags, _stream(stream)))

    def es_rhs(self, JU, J, jxi_x, jxi_t, dJU, dJ, stream=None):
        _check("es_rhs", lib.es_rhs(self.h, _ptr(JU), _ptr(J), _ptr(jxi_x), _ptr(jxi_t), _ptr(dJU),
                                    _ptr(dJ), _stream(stream)))

    def es_rk_stage(self, stage, dt_dev, JU_n, J_n, JU_s, J_s, jxi_x, jxi_t, JU_out, J_out,
                    stream=None):
        _check("es_rk_stage", lib.es_rk_stage(self.h, stage, _ptr(dt_dev), _ptr(JU_n), _ptr(J_n),
                                              _ptr(JU_s), _ptr(J_s), _ptr(jxi_x), _ptr(jxi_t),
                                              _ptr(JU_out), _ptr(J_out), _stream(stream)))

    def max_wavespeed(self, JU, J, jxi_x, cfl, lambda_dev=None, dt_dev=None, stream=None):
        _check("max_wavespeed", lib.max_wavespeed(self.h, _ptr(JU), _ptr(J), _ptr(jxi_x), float(cfl),
                                                  _ptr(lambda_dev), _ptr(dt_dev), _stream(stream)))

    def mesh_redistribute(self, mon, JU, J, x_n, disp, dtau_dev=None, resid_dev=None, stream=None):
        m = make_monitor(mon)
        _check("mesh_redistribute", lib.mesh_redistribute(self.h, C.byref(m), _ptr(JU), _ptr(J),
                                                          _ptr(x_n), _ptr(disp), _ptr(dtau_dev),
                                                          _ptr(resid_dev), _stream(stream)))

    def es_jacobian(self, x, jxi_x, J, stream=None):
        _check("es_jacobian", lib.es_jacobian(self.h, _ptr(x), _ptr(jxi_x), _ptr(J), _stream(stream)))

    def es_entropy(self, JU, J, total_dev, stream=None):
        _check("es_entropy", lib.es_entropy(self.h, _ptr(JU), _ptr(J), _ptr(total_dev), _stream(stream)))

    def es_entropy_rate(self, JU, J, dJU, dJ, rate_dev, stream=None):
        _check("es_entropy_rate", lib.es_entropy_rate(self.h, _ptr(JU), _ptr(J), _ptr(dJU), _ptr(dJ),
                                                      _ptr(rate_dev), _stream(stream)))

    def es_step(self, JU, J, x, mon=None, cfl=0.4, dt_fixed=0.0, move_mesh=False, dt_dev=None,
                dtau_dev=None, stream=None):
        m = make_monitor(mon) if mon is not None else None
        _check("es_step", lib.es_step(self.h, C.byref(m) if m is not None else None, float(cfl),
                                      float(dt_fixed), int(move_mesh), _ptr(JU), _ptr(J), _ptr(x),
                                      _ptr(dt_dev), _ptr(dtau_dev), _stream(stream)))

    def es_status(self, reset=False, stream=None):
        flags = C.c_uint(0)
        rc = lib.es_status(self.h, _stream(stream), C.byref(flags), int(reset))
        if rc not in (ES_OK, ES_ENONPHYS, ES_ETANGLE):
            raise EsError("es_status", rc)
        return rc, flags.value


class EsBatchStageArgs(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("JU_n", "J_n", "JU_s", "J_s", "jxi_x", "jxi_t", "JU_out",
                                          "J_out")]


class PtrTable:
    """Device array of the data pointers of a list of tensors (one per
    instance); keeps the tensors alive as long as the table."""

    def __init__(self, tensors):
        self.tensors = list(tensors)
        for t in self.tensors:
            _ptr(t)                          # type / device / layout check
        self.dev = torch.tensor([t.data_ptr() for t in self.tensors], dtype=torch.int64, device="cuda")

    @property
    def ptr(self):
        return C.c_void_p(self.dev.data_ptr())


def _table(x):
    if x is None:
        return None
    return x if isinstance(x, PtrTable) else PtrTable(x)


class Batch:
    """One es_batch: independent 2D instances (a list of specs that differ
    only in their grid) advanced together.  Array arguments are lists of
    tensors, one per instance, or PtrTable objects built from them."""

    def __init__(self, specs, precision=ES_FP64):
        if not torch.cuda.is_available():
            raise RuntimeError("libes needs a HIP device; there is no CPU fallback")
        self.specs = list(specs)
        self.count = len(self.specs)
        grids = (EsGrid * self.count)(*[make_grid(sp, precision) for sp in self.specs])
        self._grids = grids
        h = C.c_void_p()
        _check("es_batch_create", lib.es_batch_create(C.cast(grids, C.c_void_p), self.count, C.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            lib.es_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def es_rk_stage_batched(self, stage, dt_dev, JU_n, J_n, JU_s, J_s, jxi_x, jxi_t, JU_out, J_out,
                            stream=None):
        tabs = [_table(a) for a in (JU_n, J_n, JU_s, J_s, jxi_x, jxi_t, JU_out, J_out)]
        args = EsBatchStageArgs(*[t.ptr if t is not None else None for t in tabs])
        _check("es_rk_stage_batched", lib.es_rk_stage_batched(self.h, stage, _ptr(dt_dev), C.byref(args),
                                                              _stream(stream)))
        return tabs

    def max_wavespeed_batched(self, JU, J, jxi_x, cfl, lambda_dev=None, dt_dev=None, stream=None):
        tabs = [_table(a) for a in (JU, J, jxi_x)]
        _check("max_wavespeed_batched", lib.max_wavespeed_batched(
            self.h, tabs[0].ptr, tabs[1].ptr, tabs[2].ptr, float(cfl), _ptr(lambda_dev), _ptr(dt_dev),
            _stream(stream)))
        return tabs

    def es_step_batched(self, cfl, JU, J, jxi_x, jxi_t, dt_dev, stream=None):
        tabs = [_table(a) for a in (JU, J, jxi_x, jxi_t)]
        _check("es_step_batched", lib.es_step_batched(
            self.h, float(cfl), tabs[0].ptr, tabs[1].ptr, tabs[2].ptr,
            tabs[3].ptr if tabs[3] is not None else None, _ptr(dt_dev), _stream(stream)))
        return tabs

    def es_batch_autotune(self, JU, J, jxi_x, jxi_t, dt_dev, reps=3, stream=None):
        tabs = [_table(a) for a in (JU, J, jxi_x, jxi_t)]
        out = (C.c_int * 3)()
        _check("es_batch_autotune", lib.es_batch_autotune(
            self.h, tabs[0].ptr, tabs[1].ptr, tabs[2].ptr, tabs[3].ptr if tabs[3] is not None else None,
            _ptr(dt_dev), int(reps), _stream(stream), C.cast(out, C.c_void_p)))
        return (out[0], out[1]), out[2]

    def es_batch_set_tiling(self, region, persistent=True):
        """region: (TX, TY), one of the batch's region shapes."""
        tx, ty = region
        _check("es_batch_set_tiling", lib.es_batch_set_tiling(self.h, int(tx), int(ty), int(bool(persistent))))

    def es_batch_status(self, stream=None, reset=False):
        f = C.c_uint()
        rc = lib.es_batch_status(self.h, _stream(stream), C.byref(f), int(reset))
        if rc not in (ES_OK, ES_ENONPHYS, ES_ETANGLE):
            raise EsError("es_batch_status", rc)
        return rc, f.value
