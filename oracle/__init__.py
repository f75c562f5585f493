"""Plain CPU FP64 oracle of the entropy-stable moving-mesh scheme (arXiv 2202.07989).

TEST INFRASTRUCTURE ONLY.  This package wraps ``liboracle.so`` (built from
``es_oracle.c`` with gcc) through ctypes.  Only the tests, the smoke check and
the CPU-baseline leg of the benchmark import it; the GPU library never does,
and this package imports nothing from the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "es_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(openmp: bool = True, out: str | None = None, sanitize: bool = False) -> str:
    """Compile liboracle.so with gcc (plain -O2, no fast-math).  sanitize:
    an AddressSanitizer + UndefinedBehaviorSanitizer build (for the CPU
    sanitizer run of the pins; load it with ES_ORACLE_LIB and libasan
    preloaded)."""
    out = out or _LIB
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", out + ".tmp", _SRC, "-lm"]
    if openmp:
        cmd.insert(1, "-fopenmp")
    if sanitize:
        cmd[1:1] = ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined"]
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


class Grid(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("nspec", C.c_int), ("n", C.c_int * 3), ("ng", C.c_int),
        ("dxi", C.c_double * 3), ("len", C.c_double * 3), ("w", C.c_int),
        ("gamma", C.c_double * 2), ("cv", C.c_double * 2), ("pinf", C.c_double * 2),
        ("chi", C.c_double * 3), ("weno_eps", C.c_double), ("dissipation", C.c_int),
        ("reconstruction", C.c_int), ("bc", (C.c_int * 2) * 3), ("wall", (C.c_double * 2) * 3),
        ("inflow", ((C.c_double * 6) * 2) * 3), ("sign_tol", C.c_double),
    ]


class Monitor(C.Structure):
    _fields_ = [
        ("nsig", C.c_int), ("sigma", C.c_int * 6), ("alpha", C.c_double * 6),
        ("n_smooth", C.c_int), ("n_sweeps", C.c_int), ("form", C.c_int), ("beta", C.c_double * 6),
        ("psi", C.c_double * 2),
    ]


_D = C.POINTER(C.c_double)
_G = C.POINTER(Grid)


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("ES_ORACLE_LIB")   # another build of the same source (sanitizers)
        if not path:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
        L = C.CDLL(path)
        sig = {
            "orc_ncomp": (C.c_int, [_G]),
            "orc_alpha": (None, [C.c_int, _D]),
            "orc_logmean": (C.c_double, [C.c_double, C.c_double]),
            "orc_prim": (C.c_int, [_G, _D, _D, _D, _D, _D]),
            "orc_entropy_vars": (C.c_int, [_G, _D, _D]),
            "orc_entropy": (C.c_double, [_G, _D]),
            "orc_potential": (C.c_double, [_G, _D]),
            "orc_sound_speed": (C.c_double, [_G, _D]),
            "orc_phys_flux": (None, [_G, _D, C.c_int, _D]),
            "orc_ec_flux": (C.c_int, [_G, _D, _D, _D, _D, _D]),
            "orc_rotation": (None, [_G, _D, _D]),
            "orc_interface_frame": (C.c_int, [_G, _D, _D, _D, _D, _D]),
            "orc_mr5": (C.c_double, [_D, _D, C.c_double]),
            "orc_sign_bound": (C.c_int, [_G, _D, _D, _D, _D]),
            "orc_mixed_bound": (C.c_int, [_G, _D, _D, _D, _D, C.c_double, C.c_double, C.c_double,
                                           C.c_double, C.c_int, C.POINTER(C.c_long), _D]),
            "orc_sign_test": (C.c_int, [_G, _D, _D, _D, _D, C.c_int, C.c_int, C.POINTER(C.c_long),
                                         _D, _D, _D, C.POINTER(C.c_int), _D]),
            "orc_js5": (C.c_double, [_D, C.c_double]),
            "orc_jacobian": (C.c_int, [_G, _D, _D, _D]),
            "orc_npoints": (C.c_long, [_G]),
            "orc_fill_ghosts": (None, [_G, _D, C.c_int]),
            "orc_fill_ghosts_x": (None, [_G, _D]),
            "orc_fill_ghosts_kind": (None, [_G, _D, C.c_int, C.c_int]),
            "orc_fill_ghosts_state": (None, [_G, _D, _D]),
            "orc_metrics": (C.c_int, [_G, _D, _D, C.c_double, C.c_double, _D, _D]),
            "orc_rhs": (C.c_int, [_G, _D, _D, _D, _D, _D, _D]),
            "orc_rhs_points": (C.c_int, [_G, _D, _D, _D, _D, C.c_int, C.POINTER(C.c_long), _D, _D]),
            "orc_rk_coeffs": (None, [C.c_int, _D, _D, _D]),
            "orc_rk_stage": (C.c_int, [_G, C.c_int, C.c_double, _D, _D, _D, _D, _D, _D, _D, _D]),
            "orc_max_wavespeed": (C.c_int, [_G, _D, _D, _D, C.c_double, _D, _D]),
            "orc_monitor_fn": (C.c_int, [_G, C.POINTER(Monitor), _D, _D, _D]),
            "orc_schlieren": (C.c_int, [_G, C.POINTER(Monitor), _D, _D, _D]),
            "orc_mesh_redistribute": (C.c_int, [_G, C.POINTER(Monitor), _D, _D, _D, _D, _D, _D]),
            "orc_total_entropy": (C.c_double, [_G, _D, _D]),
            "orc_entropy_rate": (C.c_double, [_G, _D, _D, _D, _D]),
            "orc_es_production": (C.c_double, [_G, _D, _D, _D, _D]),
            "orc_step": (C.c_int, [_G, C.POINTER(Monitor), C.c_double, C.c_double, C.c_int,
                                    _D, _D, _D, _D, _D]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous, "oracle wants C-contiguous float64"
    return a.ctypes.data_as(_D)


def grid(spec) -> Grid:
    """Build the oracle's grid struct from a workload spec dict."""
    g = Grid()
    g.dim = spec["dim"]
    g.nspec = spec["nspec"]
    n = list(spec["n"]) + [1] * (3 - len(spec["n"]))
    for k in range(3):
        g.n[k] = n[k]
        g.dxi[k] = spec["dxi"][k] if k < len(spec["dxi"]) else 1.0
        g.len[k] = spec["len"][k] if k < len(spec["len"]) else 1.0
    g.ng = spec.get("ng", 3)
    g.w = spec.get("w", 3)
    for l in range(2):
        g.gamma[l] = spec["gamma"][l] if l < len(spec["gamma"]) else 1.4
        g.cv[l] = spec["cv"][l] if l < len(spec["cv"]) else 1.0
        g.pinf[l] = spec["pinf"][l] if l < len(spec["pinf"]) else 0.0
    for m in range(3):
        g.chi[m] = spec["chi"][m]
    g.weno_eps = spec.get("weno_eps", 1e-10)
    g.dissipation = spec.get("dissipation", 1)
    g.reconstruction = spec.get("reconstruction", 0)
    for k, faces in enumerate(spec.get("bc", [])):
        for side in range(2):
            g.bc[k][side] = faces[side]
    for k, faces in enumerate(spec.get("wall", [])):
        for side in range(2):
            g.wall[k][side] = faces[side]
    for (k, side), U in spec.get("inflow", {}).items():
        for c, u in enumerate(U):
            g.inflow[k][side][c] = u
    # zero tolerance of the sign matrix (0: the paper's rule as printed)
    g.sign_tol = spec.get("sign_tol", 1e-12)
    return g


def monitor(spec) -> Monitor:
    m = Monitor()
    sig = spec.get("sigma", [0])
    al = spec.get("alpha", [1200.0])
    m.nsig = len(sig)
    for t in range(len(sig)):
        m.sigma[t] = sig[t]
        m.alpha[t] = al[t]
    m.n_smooth = spec.get("n_smooth", 3)
    m.n_sweeps = spec.get("n_sweeps", 10)
    m.form = spec.get("form", 0)
    for t, b in enumerate(spec.get("beta", [])):
        m.beta[t] = b
    for t, q in enumerate(spec.get("psi", [])):
        m.psi[t] = q
    return m


class Oracle:
    """Thin numpy front-end over liboracle for one grid."""

    def __init__(self, spec):
        self.spec = spec
        self.g = grid(spec)
        self.gp = C.byref(self.g)
        self.L = lib()
        self.nc = self.L.orc_ncomp(self.gp)
        self.P = self.L.orc_npoints(self.gp)

    # pointwise --------------------------------------------------------
    def alpha(self, w):
        a = np.zeros(3)
        self.L.orc_alpha(w, _p(a))
        return a

    def logmean(self, a, b):
        return self.L.orc_logmean(a, b)

    def prim(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        rho = np.zeros(2); v = np.zeros(3); T = C.c_double(); p = C.c_double()
        rc = self.L.orc_prim(self.gp, _p(U), _p(rho), _p(v), C.byref(T), C.byref(p))
        return rc, rho[: self.g.nspec], v[: self.g.dim], T.value, p.value

    def entropy_vars(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        V = np.zeros(self.nc)
        self.L.orc_entropy_vars(self.gp, _p(U), _p(V))
        return V

    def entropy(self, U):
        return self.L.orc_entropy(self.gp, _p(np.ascontiguousarray(U, dtype=np.float64)))

    def potential(self, U):
        return self.L.orc_potential(self.gp, _p(np.ascontiguousarray(U, dtype=np.float64)))

    def sound_speed(self, U):
        return self.L.orc_sound_speed(self.gp, _p(np.ascontiguousarray(U, dtype=np.float64)))

    def phys_flux(self, U, j):
        F = np.zeros(self.nc)
        self.L.orc_phys_flux(self.gp, _p(np.ascontiguousarray(U, dtype=np.float64)), j, _p(F))
        return F

    def ec_flux(self, Ul, Ur, ml, mr):
        F = np.zeros(self.nc)
        args = [np.ascontiguousarray(a, dtype=np.float64) for a in (Ul, Ur, ml, mr)]
        self.L.orc_ec_flux(self.gp, *[_p(a) for a in args], _p(F))
        return F

    def rotation(self, n):
        T = np.zeros((self.nc, self.nc))
        self.L.orc_rotation(self.gp, _p(np.ascontiguousarray(n, dtype=np.float64)), _p(T))
        return T

    def interface_frame(self, Ul, Ur, m):
        R = np.zeros((self.nc, self.nc)); s = C.c_double()
        args = [np.ascontiguousarray(a, dtype=np.float64) for a in (Ul, Ur, m)]
        self.L.orc_interface_frame(self.gp, *[_p(a) for a in args], _p(R), C.byref(s))
        return R, s.value

    def sign_bound(self, Ul, Ur, m):
        B = np.zeros(self.nc)
        args = [np.ascontiguousarray(a, dtype=np.float64) for a in (Ul, Ur, m)]
        rc = self.L.orc_sign_bound(self.gp, *[_p(a) for a in args], _p(B))
        return rc, B

    def sign_test(self, JU, J, jx, jt, k, flat_idx):
        """Sign test at the interfaces right of the given nodes along k:
        (rc, jump, WENO jump, bound, Y, s), per node and field."""
        pts = np.ascontiguousarray(flat_idx, dtype=np.int64)
        n = len(pts)
        jump, jw, bound = np.zeros((n, self.nc)), np.zeros((n, self.nc)), np.zeros((n, self.nc))
        Y = np.zeros((n, self.nc), dtype=np.int32)
        s = np.zeros(n)
        rc = self.L.orc_sign_test(self.gp, _p(JU), _p(J), _p(jx), _p(jt), k, n,
                                  pts.ctypes.data_as(C.POINTER(C.c_long)), _p(jump), _p(jw),
                                  _p(bound), Y.ctypes.data_as(C.POINTER(C.c_int)), _p(s))
        return rc, jump, jw, bound, Y.astype(bool), s

    # constants of the a-priori bound of the mixed-precision path
    MIXED_KF, MIXED_KW, U32 = 16.0, 64.0, 2.0 ** -24

    def mixed_bound(self, JU, J, jx, jt, flat_idx, tol32=None):
        """Per-node a-priori bound (npts, nc) on |mixed GPU - FP64| of the
        right-hand side at the given nodes."""
        pts = np.ascontiguousarray(flat_idx, dtype=np.int64)
        n = len(pts)
        tol32 = self.spec.get("sign_tol32", 1e-6) if tol32 is None else tol32
        out = np.zeros((n, self.nc))
        rc = self.L.orc_mixed_bound(self.gp, _p(JU), _p(J), _p(jx), _p(jt), self.MIXED_KF, self.MIXED_KW,
                                    self.U32, tol32, n, pts.ctypes.data_as(C.POINTER(C.c_long)), _p(out))
        assert rc == 0, rc
        return out

    def js5(self, q, eps=None):
        eps = self.g.weno_eps if eps is None else eps
        return self.L.orc_js5(_p(np.ascontiguousarray(q, dtype=np.float64)), eps)

    def mr5(self, q, chi=None, eps=None):
        chi = np.array(self.spec["chi"] if chi is None else chi, dtype=np.float64)
        eps = self.g.weno_eps if eps is None else eps
        return self.L.orc_mr5(_p(np.ascontiguousarray(q, dtype=np.float64)), _p(chi), eps)

    # whole grid ---------------------------------------------------------
    def fill_ghosts(self, a, ncomp):
        self.L.orc_fill_ghosts(self.gp, _p(a), ncomp)

    def fill_ghosts_x(self, x):
        self.L.orc_fill_ghosts_x(self.gp, _p(x))

    def fill_ghosts_kind(self, a, ncomp, what):
        """what: 0 plain, 1 mesh, 2 displacement, 3 jxi_x, 4 jxi_t."""
        self.L.orc_fill_ghosts_kind(self.gp, _p(a), ncomp, what)

    def fill_ghosts_state(self, JU, J):
        self.L.orc_fill_ghosts_state(self.gp, _p(JU), _p(J))

    def metrics(self, x, disp=None, c_s=0.0, dt=0.0):
        d = self.g.dim
        jx = np.zeros((d * d,) + x.shape[1:])
        jt = np.zeros((d,) + x.shape[1:])
        rc = self.L.orc_metrics(self.gp, _p(x), _p(disp), c_s, dt, _p(jx), _p(jt))
        assert rc == 0, rc
        return jx, jt

    def jacobian(self, x, jx):
        J = np.zeros((1,) + x.shape[1:])
        rc = self.L.orc_jacobian(self.gp, _p(x), _p(jx), _p(J))
        assert rc == 0, rc
        return J

    def rhs(self, JU, J, jx, jt):
        dJU = np.zeros_like(JU)
        dJ = np.zeros_like(J)
        rc = self.L.orc_rhs(self.gp, _p(JU), _p(J), _p(jx), _p(jt), _p(dJU), _p(dJ))
        return rc, dJU, dJ

    def rhs_points(self, JU, J, jx, jt, flat_idx):
        pts = np.ascontiguousarray(flat_idx, dtype=np.int64)
        n = len(pts)
        dJU = np.zeros((n, self.nc)); dJ = np.zeros(n)
        rc = self.L.orc_rhs_points(self.gp, _p(JU), _p(J), _p(jx), _p(jt), n,
                                   pts.ctypes.data_as(C.POINTER(C.c_long)), _p(dJU), _p(dJ))
        return rc, dJU, dJ

    def rk_coeffs(self, stage):
        a, b, c = C.c_double(), C.c_double(), C.c_double()
        self.L.orc_rk_coeffs(stage, C.byref(a), C.byref(b), C.byref(c))
        return a.value, b.value, c.value

    def rk_stage(self, stage, dt, JUn, Jn, JUs, Js, jx, jt):
        JUo = np.zeros_like(JUn); Jo = np.zeros_like(Jn)
        rc = self.L.orc_rk_stage(self.gp, stage, dt, _p(JUn), _p(Jn), _p(JUs), _p(Js),
                                 _p(jx), _p(jt), _p(JUo), _p(Jo))
        return rc, JUo, Jo

    def max_wavespeed(self, JU, J, jx, cfl):
        lam, dt = C.c_double(), C.c_double()
        rc = self.L.orc_max_wavespeed(self.gp, _p(JU), _p(J), _p(jx), cfl, C.byref(lam), C.byref(dt))
        return rc, lam.value, dt.value

    def monitor_fn(self, mon, JU, J):
        m = monitor(mon)
        th = np.zeros_like(J)
        rc = self.L.orc_monitor_fn(self.gp, C.byref(m), _p(JU), _p(J), _p(th))
        return rc, th

    def schlieren(self, mon, JU, J):
        m = monitor(mon)
        phi = np.zeros_like(J)
        rc = self.L.orc_schlieren(self.gp, C.byref(m), _p(JU), _p(J), _p(phi))
        assert rc == 0, rc
        return phi

    def mesh_redistribute(self, mon, JU, J, x):
        m = monitor(mon)
        disp = np.zeros_like(x)
        dtau = C.c_double()
        resid = np.zeros(max(1, m.n_sweeps))
        rc = self.L.orc_mesh_redistribute(self.gp, C.byref(m), _p(JU), _p(J), _p(x), _p(disp),
                                          C.byref(dtau), _p(resid))
        return rc, disp, dtau.value, resid[: m.n_sweeps]

    def total_entropy(self, JU, J):
        return self.L.orc_total_entropy(self.gp, _p(JU), _p(J))

    def entropy_rate(self, JU, J, dJU, dJ):
        return self.L.orc_entropy_rate(self.gp, _p(JU), _p(J), _p(dJU), _p(dJ))

    def es_production(self, JU, J, jx, jt):
        return self.L.orc_es_production(self.gp, _p(JU), _p(J), _p(jx), _p(jt))

    def step(self, JU, J, x, mon=None, cfl=0.4, dt_fixed=0.0, move_mesh=False):
        m = monitor(mon) if mon is not None else None
        dt, dtau = C.c_double(), C.c_double()
        rc = self.L.orc_step(self.gp, C.byref(m) if m is not None else None, cfl, dt_fixed,
                             int(move_mesh), _p(JU), _p(J), _p(x), C.byref(dt), C.byref(dtau))
        return rc, dt.value, dtau.value
