"""The isentropic-vortex workloads of Section 5 (Examples 5.1 and 5.5) on
the GPU: moving mesh driven by the gradient + Laplacian monitor, time step
C_CFL (Delta xi / L)^(5/3) so that the spatial error dominates.

- whole steps against the CPU FP64 oracle (2D and 3D), to the FP64 bar;
- convergence in rho against the exact solution (the initial vortex carried
  by the mean flow).  On the fixed uniform mesh the fifth order shows as an
  observed l1 order above 4.5 between 80^2 and 160^2 at t = 4 (measured
  4.7; 5.0 between 160^2 and 320^2).  On the moving mesh the observed l1
  order stays near 4 up to 160^2 at t = 0.5 (measured 3.9 and 3.8; the
  oracle measures 3.1 and 3.9 on 20/40 and 40/80)."""
import numpy as np
import pytest

import oracle
from paper_2202_07989_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_2202_07989_amd import es  # noqa: E402
from gpu_util import TOL_FP64, dev, host, parity, state_scale, say  # noqa: E402


def accuracy_dt(dim, n, t_end):
    dt0 = (0.4 if dim == 2 else 0.3) * (1.0 / n) ** (5.0 / 3.0)
    ns = int(np.ceil(t_end / dt0))
    return t_end / ns, ns


@pytest.mark.parametrize("dim,n,nsteps", [(2, 32, 4), (3, 12, 2)])
def test_vortex_steps_parity(dim, n, nsteps):
    say(f"[vortex steps] {dim}D {n} steps={nsteps}")
    sp = I.spec_vortex(dim, n)
    o = oracle.Oracle(sp)
    JU, J, x = I.init_vortex(sp)
    o.fill_ghosts(JU, o.nc)
    o.fill_ghosts(J, 1)
    o.fill_ghosts_x(x)
    mon = I.vortex_monitor()
    dt, _ = accuracy_dt(dim, n, 1.0)
    ctx = es.Context(sp)
    gU, gJ, gx = dev(JU), dev(J), dev(x)
    tau_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(nsteps):
        rc, _, tau = o.step(JU, J, x, mon=mon, dt_fixed=dt, move_mesh=True)
        assert rc == 0
        ctx.es_step(gU, gJ, gx, mon=mon, dt_fixed=dt, move_mesh=True, dtau_dev=tau_dev)
        assert host(tau_dev)[0] == pytest.approx(tau, rel=1e-12)
    Iin = I.interior(sp)
    _, lam, _ = o.max_wavespeed(JU, J, o.metrics(x)[0], 1.0)
    sc = state_scale(JU, sp, lam)
    hU, hx = host(gU), host(gx)
    for c in range(o.nc):
        assert parity(hU[c][Iin[1:]], JU[c][Iin[1:]], sc[c]) <= TOL_FP64, c
    for c in range(dim):
        assert parity(hx[c], x[c], np.abs(x[c]).max()) <= TOL_FP64, c
    assert ctx.es_status()[0] == es.ES_OK


def vortex_error(dim, n, t_end, dissipation=1, move=True):
    sp = I.spec_vortex(dim, n)
    sp["dissipation"] = dissipation
    JU, J, x = I.init_vortex(sp)
    ctx = es.Context(sp)
    gU, gJ, gx = dev(JU), dev(J), dev(x)
    ctx.es_fill_ghosts(gU, 2 + dim)
    ctx.es_fill_ghosts(gJ, 1)
    ctx.es_fill_ghosts_x(gx)
    mon = I.vortex_monitor()
    dt, ns = accuracy_dt(dim, n, t_end)
    for _ in range(ns):
        ctx.es_step(gU, gJ, gx, mon=mon if move else None, dt_fixed=dt, move_mesh=move)
    assert ctx.es_status()[0] == es.ES_OK
    Iin = I.interior(sp)
    hU, hJ, hx = host(gU), host(gJ), host(gx)
    rho = hU[Iin][0] / hJ[Iin][0]
    ex, _, _ = I.vortex_prims(dim, [hx[Iin][k] for k in range(dim)], t_end)
    return np.abs(rho - ex).mean(), np.abs(rho - ex).max()


def test_vortex_convergence_2d_fixed_mesh():
    errs = []
    for n in (80, 160):
        say(f"[vortex convergence, fixed mesh] 2D {n}")
        errs.append(vortex_error(2, n, 4.0, move=False))
    e = np.array(errs)
    orders = np.log2(e[:-1] / e[1:])
    say(f"    l1 {e[:, 0]} linf {e[:, 1]} orders {orders.tolist()}")
    assert orders[-1, 0] > 4.5, orders


def test_vortex_convergence_2d_moving_mesh():
    errs = []
    for n in (40, 80, 160):
        say(f"[vortex convergence, moving mesh] 2D {n}")
        errs.append(vortex_error(2, n, 0.5))
    e = np.array(errs)
    orders = np.log2(e[:-1] / e[1:])
    say(f"    l1 {e[:, 0]} linf {e[:, 1]} orders {orders.tolist()}")
    assert (orders[:, 0] > 3.5).all(), orders
