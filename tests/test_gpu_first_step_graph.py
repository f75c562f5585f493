"""The whole workspace of a context is allocated by es_create, so the very
first es_step of a fresh context can be captured in a HIP graph: nothing in
it allocates or synchronises.  Each replay must leave the state, the mesh
and dt bitwise equal to the same step run eagerly on another fresh context
(two replays: the second reuses the metrics the first kept)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_2202_07989_amd import es  # noqa: E402
from gpu_util import dev, host, say  # noqa: E402
from cases import prepared  # noqa: E402
from test_gpu_bc import bc_case  # noqa: E402


@pytest.mark.parametrize("name,precision", [("3d-n2-bubble", "fp64"), ("2d-shock-bubble", "fp64"),
                                            ("3d-n2-bubble", "mixed")])
def test_first_step_of_a_fresh_context_is_capturable(name, precision):
    say(f"[first step in a graph] {name} {precision}")
    if name == "2d-shock-bubble":
        sp, JU, J, x, mon = bc_case(name)
        cfl = 0.4
    else:
        sp, _, JU, J, x, *_ = prepared(name, moving=False)
        mon = dict(sigma=[0], alpha=[1200.0], n_smooth=3, n_sweeps=5)
        cfl = 0.3
    prec = es.ES_MIXED if precision == "mixed" else es.ES_FP64
    cg = es.Context(sp, prec)     # fresh: nothing has run on it before the capture
    ce = es.Context(sp, prec)
    gU, gJ, gx = dev(JU), dev(J), dev(x)
    eU, eJ, ex = dev(JU), dev(J), dev(x)
    dtg = torch.zeros(1, dtype=torch.float64, device="cuda")
    dte = torch.zeros(1, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        cg.es_step(gU, gJ, gx, mon=mon, cfl=cfl, move_mesh=True, dt_dev=dtg)
    for r in range(2):
        graph.replay()
        torch.cuda.synchronize()
        ce.es_step(eU, eJ, ex, mon=mon, cfl=cfl, move_mesh=True, dt_dev=dte)
        torch.cuda.synchronize()
        assert host(dtg)[0] == host(dte)[0], r
        np.testing.assert_array_equal(host(gU), host(eU))
        np.testing.assert_array_equal(host(gJ), host(eJ))
        np.testing.assert_array_equal(host(gx), host(ex))
    assert cg.es_status()[0] == es.ES_OK
    assert ce.es_status()[0] == es.ES_OK
