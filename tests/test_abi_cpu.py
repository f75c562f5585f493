"""The C-ABI library loads and exports every entry point of include/es.h, and
rejects bad arguments synchronously (no GPU needed for these checks)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "es.h")
LIB = os.path.join(ROOT, "paper_2202_07989_amd", "libes.so")


def declared_functions():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|long)\s+(\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libes.so is not built (run __graft_entry__.build())")
    return C.CDLL(LIB)


def test_header_declares_the_path():
    names = declared_functions()
    for n in ("es_create", "es_destroy", "es_fill_ghosts", "es_fill_ghosts_x", "es_metrics", "es_rhs",
              "es_rk_stage", "max_wavespeed", "mesh_redistribute", "es_entropy", "es_entropy_rate",
              "es_step", "es_status", "es_npoints"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_invalid_arguments_rejected_before_any_launch(lib):
    from paper_2202_07989_amd import es
    from paper_2202_07989_amd import inputs as I
    sp = I.spec_c1(8)
    h = C.c_void_p()
    for bad, code in (("dim", es.ES_EUNSUPPORTED), ("nspec", es.ES_EUNSUPPORTED), ("w", es.ES_EUNSUPPORTED),
                      ("ng", es.ES_EUNSUPPORTED), ("dxi", es.ES_EINVAL), ("gamma", es.ES_EINVAL),
                      ("chi", es.ES_EINVAL), ("precision", es.ES_EUNSUPPORTED),
                      ("reconstruction", es.ES_EUNSUPPORTED), ("js-mixed", es.ES_EUNSUPPORTED),
                      ("sign_tol", es.ES_EINVAL), ("sign_tol32", es.ES_EINVAL), ("sign_tol-nan", es.ES_EINVAL)):
        g = es.make_grid(sp)
        if bad == "dim":
            g.dim = 4
        elif bad == "nspec":
            g.nspec = 3
        elif bad == "w":
            g.w = 4
        elif bad == "ng":
            g.ng = 2
        elif bad == "dxi":
            g.dxi[0] = 0.0
        elif bad == "gamma":
            g.gamma[0] = 1.0
        elif bad == "chi":
            g.chi[1] = -0.1
        elif bad == "precision":
            g.precision = 7
        elif bad == "reconstruction":
            g.reconstruction = 2
        elif bad == "js-mixed":
            g.reconstruction, g.precision = es.ES_WENO_JS, es.ES_MIXED
        elif bad == "sign_tol":
            g.sign_tol = -1e-12
        elif bad == "sign_tol32":
            g.sign_tol32 = 1.0
        elif bad == "sign_tol-nan":
            g.sign_tol = float("nan")
        assert es.lib.es_create(C.byref(g), C.byref(h)) == code, bad
    assert es.lib.es_create(None, C.byref(h)) == es.ES_EINVAL
    null = None
    assert es.lib.es_rhs(null, null, null, null, null, null, null, null) == es.ES_EINVAL
    assert es.lib.es_rk_stage(null, 0, null, null, null, null, null, null, null, null, null, null) == es.ES_EINVAL
    assert es.lib.max_wavespeed(null, null, null, null, 0.4, null, null, null) == es.ES_EINVAL
    assert es.lib.mesh_redistribute(null, null, null, null, null, null, null, null, null) == es.ES_EINVAL
    assert es.lib.es_metrics(null, null, null, 0.0, null, null, null, 0, null) == es.ES_EINVAL
    assert es.lib.es_step(null, null, 0.4, 0.0, 0, null, null, null, null, null, null) == es.ES_EINVAL
    assert es.lib.es_status(null, null, null, 0) == es.ES_EINVAL
    assert es.lib.es_destroy(null) == es.ES_EINVAL


def test_face_conditions_checked_before_any_launch(lib):
    """A direction is periodic on both faces or on neither; faces of a
    non-periodic direction need wall[k][1] > wall[k][0]; kinds stay in
    ES_BC_*; inflow states are finite; batches take periodic grids only."""
    from paper_2202_07989_amd import es
    from paper_2202_07989_amd import inputs as I
    h = C.c_void_p()
    sp = I.spec_shock_bubble_walled("he", (16, 8))
    for bad in ("half-periodic", "wall-order", "kind", "inflow-nan"):
        g = es.make_grid(sp)
        if bad == "half-periodic":
            g.bc[1][0] = es.ES_BC_PERIODIC
        elif bad == "wall-order":
            g.wall[1][0], g.wall[1][1] = 1.0, -1.0
        elif bad == "kind":
            g.bc[0][1] = 7
        elif bad == "inflow-nan":
            g.inflow[0][1][2] = float("nan")
        assert es.lib.es_create(C.byref(g), C.byref(h)) == es.ES_EINVAL, bad
    grids = (es.EsGrid * 1)(es.make_grid(sp))
    assert es.lib.es_batch_create(C.cast(grids, C.c_void_p), 1, C.byref(h)) == es.ES_EUNSUPPORTED
    assert es.lib.es_fill_ghosts_state(None, None, None, None) == es.ES_EINVAL


def test_invalid_grids_rejected_by_library_and_oracle(lib):
    """The same malformed grids (zero spacing, a half-periodic direction,
    faces out of order, an unknown face kind, a sign-test tolerance outside
    [0, 1)) are argument errors of both implementations: es_create returns
    ES_EINVAL and the oracle's calls return its EINVAL (-1), before any
    array is read."""
    import numpy as np

    import oracle
    from paper_2202_07989_amd import es
    from paper_2202_07989_amd import inputs as I
    h = C.c_void_p()
    base = I.spec_shock_bubble_walled("he", (16, 8))
    for bad in ("dxi", "half-periodic", "wall-order", "kind", "sign_tol", "sign_tol-big", "sign_tol-nan"):
        g = es.make_grid(base)
        o = oracle.Oracle(base)
        for gg in (g, o.g):
            if bad == "dxi":
                gg.dxi[0] = 0.0
            elif bad == "half-periodic":
                gg.bc[1][0] = es.ES_BC_PERIODIC
            elif bad == "wall-order":
                gg.wall[1][0], gg.wall[1][1] = 1.0, -1.0
            elif bad == "kind":
                gg.bc[0][1] = 7
            elif bad == "sign_tol":
                gg.sign_tol = -1e-12
            elif bad == "sign_tol-big":
                gg.sign_tol = 1.0
            elif bad == "sign_tol-nan":
                gg.sign_tol = float("nan")
        assert es.lib.es_create(C.byref(g), C.byref(h)) == es.ES_EINVAL, bad
        z = np.zeros(8)
        assert o.L.orc_rhs(o.gp, *(z.ctypes.data_as(C.POINTER(C.c_double)) for _ in range(6))) == -1, bad
