"""Metrics carried from one es_step to the next.

A step forms its c = 1 stage mesh x^n + disp once, with its ghost layers by
the face rules, and keeps the metrics of that mesh, which is the next step's
x^n; on a fixed mesh it keeps the metrics of x itself.  The next step
compares its mesh with the kept copy on the device and forms the metrics
afresh only where they differ.  So a context that reuses its metrics must
leave the state, the mesh and dt bitwise equal to a fresh context (which has
nothing to reuse) started from the same data, and a mesh that the caller
changed between steps must be noticed."""
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

CASES = [("2d-n2-bubble", True, "fp64"), ("3d-n2-bubble", True, "fp64"), ("2d-n1", False, "fp64"),
         ("2d-shock-bubble", True, "fp64"), ("3d-mixed", True, "fp64"), ("3d-mixed", False, "fp64"),
         ("2d-shock-bubble", True, "mixed"), ("3d-n2-bubble", True, "mixed")]


def setup(name, move):
    if name in ("2d-shock-bubble", "3d-mixed"):
        sp, JU, J, x, mon = bc_case(name)
    else:
        sp, _, JU, J, x, *_ = prepared(name, moving=move)
        mon = dict(sigma=[0], alpha=[1200.0], n_smooth=3, n_sweeps=5)
    return sp, JU, J, x, mon


def step(ctx, st, mon, move):
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.es_step(*st, mon=mon, cfl=0.3, move_mesh=move, dt_dev=dt)
    return dt


def assert_same(a, b, what):
    for k, (u, v) in enumerate(zip(a, b)):
        np.testing.assert_array_equal(host(u), host(v), err_msg=f"{what}: array {k}")


def versus_fresh(sp, prec, ctx, st, mon, move, what):
    """One step on ctx and one on a fresh context from a copy of st."""
    other = [t.clone() for t in st]
    da = step(ctx, st, mon, move)
    db = step(es.Context(sp, precision=prec), other, mon, move)
    assert_same(st + [da], other + [db], what)


@pytest.mark.parametrize("name,move,precision", CASES)
def test_kept_metrics_equal_fresh_ones(name, move, precision):
    say(f"[metric reuse] {name} move={move} {precision}")
    sp, JU, J, x, mon = setup(name, move)
    prec = es.ES_MIXED if precision == "mixed" else es.ES_FP64
    ctx = es.Context(sp, precision=prec)
    st = [dev(JU), dev(J), dev(x)]
    step(ctx, st, mon, move)
    versus_fresh(sp, prec, ctx, st, mon, move, "second step")
    # the caller moves one interior node by a thousandth of the spacing there
    ng, n = sp["ng"], sp["n"]
    z = ng + n[2] // 2 if sp["dim"] == 3 else 0
    y, i = ng + n[1] // 2, ng + n[0] // 2
    hx = host(st[2])
    st[2][0, z, y, i] += 1e-3 * (hx[0, z, y, i + 1] - hx[0, z, y, i])
    versus_fresh(sp, prec, ctx, st, mon, move, "after the caller moved a node")
    versus_fresh(sp, prec, ctx, st, mon, move, "the step after that")
    assert ctx.es_status()[0] == es.ES_OK
