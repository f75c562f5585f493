"""max_wavespeed_noalloc, the CFL reduction for callers that cannot
allocate (its scratch is a static device array), against max_wavespeed of a
context on the same data: lambda and dt bitwise equal (same kernels, same
partial count), on two calls in a row, the second on a smaller grid; the
status bits of a non-physical node reach the caller's word."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_2202_07989_amd import es  # noqa: E402
from gpu_util import dev, host, say  # noqa: E402
from cases import prepared  # noqa: E402


def reference(sp, JU, J, jx, cfl):
    ctx = es.Context(sp)
    lam = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.max_wavespeed(JU, J, jx, cfl, lam, dt)
    return host(lam)[0], host(dt)[0]


def test_noalloc_wavespeed_equals_context_wavespeed_twice_shrinking():
    out = []
    for name in ("3d-n2-bubble", "2d-n1"):     # the second grid is smaller
        say(f"[noalloc wavespeed] {name}")
        sp, o, JU, J, x, disp, jx, jt = prepared(name)
        gU, gJ, gx = dev(JU), dev(J), dev(jx)
        lam = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
        dt = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        es.max_wavespeed_noalloc(sp, gU, gJ, gx, 0.3, lam, dt, st)
        l_ref, d_ref = reference(sp, gU, gJ, gx, 0.3)
        assert host(lam)[0] == l_ref and host(dt)[0] == d_ref, name
        assert host(st)[0] == 0
        _, l_orc, d_orc = o.max_wavespeed(JU, J, jx, 0.3)
        assert host(lam)[0] == pytest.approx(l_orc, rel=1e-13)
        out.append(host(lam)[0])
    assert out[0] != out[1]


def test_noalloc_reports_a_nonphysical_node_and_rejects_bad_grids():
    sp, o, JU, J, x, disp, jx, jt = prepared("2d-n1")
    bad = JU.copy()
    ng = sp["ng"]
    bad[0][0, ng + 2, ng + 3] = -abs(bad[0][0, ng + 2, ng + 3])   # a negative density at an interior node
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    lam = torch.zeros(1, dtype=torch.float64, device="cuda")
    es.max_wavespeed_noalloc(sp, dev(bad), dev(J), dev(jx), 0.3, lam, None, st)
    assert host(st)[0] & es.ES_ST_NONPHYS
    g = es.make_grid(sp)
    g.dim = 5
    null = None
    rc = es.lib.max_wavespeed_noalloc(C.byref(g), C.c_void_p(dev(JU).data_ptr()), null, null, 0.3, null,
                                      null, null, null)
    assert rc == es.ES_EINVAL
    g = es.make_grid(sp)
    g.dim = 5
    t = dev(JU)
    rc = es.lib.max_wavespeed_noalloc(C.byref(g), C.c_void_p(t.data_ptr()), C.c_void_p(t.data_ptr()),
                                      C.c_void_p(t.data_ptr()), 0.3, null, null, null, null)
    assert rc == es.ES_EUNSUPPORTED
