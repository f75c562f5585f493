"""Parity at the full sizes of the workload configurations, in the launch
configurations the benchmark and the step driver use.

- 2D one-species 64^2 fixed curvilinear mesh, smooth advection, 10 SSP-RK3
  steps at CFL 0.5: whole steps against the oracle, every node.
- 2D two-species 512^2 shock-bubble on the adaptive moving mesh (10 Jacobi
  sweeps, 3 filter passes, alpha 1200), CFL 0.4: two whole steps against
  the oracle, every node.
- 3D two-species 384^3 shock-bubble, FP64 and mixed: the right-hand side on
  a moving mesh at sampled nodes (the oracle evaluates node by node).
- The 64-instance batched 2D form at its full sizes (128^2..965^2): one
  batched stage equals the per-instance stage bit for bit for every
  instance, and matches the oracle on the two largest instances."""
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



def _ghosts(o, JU, J, x):
    o.fill_ghosts(JU, o.nc)
    o.fill_ghosts(J, 1)
    o.fill_ghosts_x(x)


def _compare_states(sp, o, JU, J, x, gU, gJ, gx, tol, what):
    Iin = I.interior(sp)
    _, lam, _ = o.max_wavespeed(JU, J, o.metrics(x)[0], 1.0)
    sc = state_scale(JU, sp, lam)
    hU, hJ, hx = host(gU), host(gJ), host(gx)
    errs = [parity(hU[c][Iin[1:]], JU[c][Iin[1:]], sc[c]) for c in range(o.nc)]
    say(f"    {what}: state error / scale {' '.join(f'{e:.1e}' for e in errs)}")
    assert max(errs) <= tol, errs
    assert parity(hJ[Iin], J[Iin], np.abs(J).max()) <= tol
    for c in range(sp["dim"]):
        assert parity(hx[c], x[c], np.abs(x[c]).max()) <= tol


def test_c1_full_10_steps():
    say("[config] 2D 64^2 curvilinear, 10 steps CFL 0.5")
    sp = I.spec_c1(64)
    o = oracle.Oracle(sp)
    JU, J, x = I.init_c1(sp)
    _ghosts(o, JU, J, x)
    ctx = es.Context(sp)
    gU, gJ, gx = dev(JU), dev(J), dev(x)
    dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    for n in range(10):
        rc, dt, _ = o.step(JU, J, x, cfl=0.5, move_mesh=False)
        assert rc == 0
        ctx.es_step(gU, gJ, gx, cfl=0.5, move_mesh=False, dt_dev=dt_dev)
        assert host(dt_dev)[0] == pytest.approx(dt, rel=1e-12), n
    _compare_states(sp, o, JU, J, x, gU, gJ, gx, TOL_FP64, "64^2 after 10 steps")
    assert ctx.es_status()[0] == es.ES_OK


def test_c2_full_moving_steps():
    say("[config] 2D 512^2 shock-bubble, moving mesh, 2 steps CFL 0.4")
    sp = I.spec_c2(512)
    o = oracle.Oracle(sp)
    JU, J, x = I.init_shock_bubble(sp)
    _ghosts(o, JU, J, x)
    mon = I.monitor_spec(n_sweeps=10, n_smooth=3, sigma=(0,), alpha=(1200.0,))
    ctx = es.Context(sp)
    gU, gJ, gx = dev(JU), dev(J), dev(x)
    dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    tau_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    for n in range(2):
        rc, dt, tau = o.step(JU, J, x, mon=mon, cfl=0.4, move_mesh=True)
        assert rc == 0
        ctx.es_step(gU, gJ, gx, mon=mon, cfl=0.4, move_mesh=True, dt_dev=dt_dev, dtau_dev=tau_dev)
        assert host(dt_dev)[0] == pytest.approx(dt, rel=1e-11), n
        assert host(tau_dev)[0] == pytest.approx(tau, rel=1e-11), n
    _compare_states(sp, o, JU, J, x, gU, gJ, gx, TOL_FP64, "512^2 after 2 moving steps")
    assert ctx.es_status()[0] == es.ES_OK


@pytest.fixture(scope="module")
def c4():
    say("[config] building the 384^3 workload and the oracle metrics")
    sp = I.spec_c3(384)
    o = oracle.Oracle(sp)
    JU, J, x = I.init_shock_bubble(sp)
    Iin = I.interior(sp)
    x[Iin] += 0.003 * (np.stack(I.random_mesh(sp, seed=41, amp=1.0)) - np.stack(I.xi_nodes(sp)))
    disp = I.zeros(sp, 3)
    disp[Iin] = 0.002 * (np.stack(I.random_mesh(sp, seed=42, amp=1.0)) - np.stack(I.xi_nodes(sp)))
    _ghosts(o, JU, J, x)
    o.fill_ghosts(disp, 3)
    jx, jt = o.metrics(x, disp, c_s=0.5, dt=1e-6)
    _, lam, _ = o.max_wavespeed(JU, J, jx, 1.0)
    rng = np.random.default_rng(384)
    flat = np.arange(o.P).reshape(J.shape[1:])
    inner = flat[Iin[1:]]
    grad = np.abs(np.diff(JU[0], axis=2, append=JU[0][..., :1]))[Iin[1:]]
    front = inner[grad > 0.1 * grad.max()]
    pts = np.unique(np.concatenate([rng.choice(inner.reshape(-1), size=1500, replace=False),
                                    rng.choice(front, size=min(1500, front.size), replace=False)]))
    rc, oU, oJ = o.rhs_points(JU, J, jx, jt, pts)
    assert rc == 0
    bound = o.mixed_bound(JU, J, jx, jt, pts)       # a-priori bound of the mixed path
    say(f"[config] {pts.size} sampled nodes")
    return dict(sp=sp, JU=JU, J=J, jx=jx, jt=jt, lam=lam, pts=pts, oU=oU, oJ=oJ, nc=o.nc, bound=bound)


@pytest.mark.parametrize("precision", [es.ES_FP64, es.ES_MIXED])
def test_c4_rhs_sampled(c4, precision):
    say(f"[config] 3D 384^3 RHS, precision {precision}")
    sp = c4["sp"]
    ctx = es.Context(sp, precision=precision)
    gJU, gJ = dev(c4["JU"]), dev(c4["J"])
    gU, gdJ = torch.empty_like(gJU), torch.empty_like(gJ)
    ctx.es_rhs(gJU, gJ, dev(c4["jx"]), dev(c4["jt"]), gU, gdJ)
    torch.cuda.synchronize()
    idx = torch.from_numpy(c4["pts"]).cuda()
    hU = gU.reshape(c4["nc"], -1)[:, idx].cpu().numpy().T
    hJ = gdJ.reshape(-1)[idx].cpu().numpy()
    sc = state_scale(c4["JU"], sp, c4["lam"])
    errs = [np.abs(hU[:, c] - c4["oU"][:, c]).max() / (sc[c] * c4["lam"]) for c in range(c4["nc"])]
    say(f"    per-component error / S_c: {' '.join(f'{e:.1e}' for e in errs)}")
    if precision == es.ES_FP64:
        assert max(errs) <= TOL_FP64, errs
    else:
        r = (np.abs(hU - c4["oU"]) / c4["bound"]).max(axis=0)
        say(f"    per-component max error / bound: {' '.join(f'{v:.2f}' for v in r)}")
        assert r.max() <= 1.0, r
    assert np.abs(hJ - c4["oJ"]).max() / (np.abs(c4["J"]).max() * c4["lam"]) <= TOL_FP64
    assert ctx.es_status()[0] == es.ES_OK


def test_c5_full_batch_stage():
    say("[config] 64-instance batch at full size")
    insts = I.init_c5()
    specs = [sp for sp, _, _, _ in insts]
    gU, gJ, jx, dts = [], [], [], []
    big = sorted(range(len(insts)), key=lambda b: -specs[b]["n"][0])[:2]
    orc = {}
    for b, (sp, JU, J, x) in enumerate(insts):
        ctx = es.Context(sp)
        u, j, xm = dev(JU), dev(J), dev(x)
        ctx.es_fill_ghosts(u, sp["nspec"] + 3)
        ctx.es_fill_ghosts(j, 1)
        ctx.es_fill_ghosts_x(xm)
        m = torch.empty((4,) + tuple(J.shape[1:]), dtype=torch.float64, device="cuda")
        ctx.es_metrics(xm, None, 0.0, None, m, None)
        gU.append(u)
        gJ.append(j)
        jx.append(m)
        if b in big:
            o = oracle.Oracle(sp)
            o.fill_ghosts(JU, o.nc)
            o.fill_ghosts(J, 1)
            o.fill_ghosts_x(x)
            ojx, _ = o.metrics(x)
            orc[b] = (o, JU, J, ojx)
    batch = es.Batch(specs)
    dt = torch.zeros(len(insts), dtype=torch.float64, device="cuda")
    batch.max_wavespeed_batched(gU, gJ, jx, 0.4, None, dt)
    outU = [torch.empty_like(t) for t in gU]
    outJ = [torch.empty_like(t) for t in gJ]
    batch.es_rk_stage_batched(1, dt, gU, gJ, gU, gJ, jx, None, outU, outJ)
    torch.cuda.synchronize()
    for b, sp in enumerate(specs):
        ctx = es.Context(sp)
        rU, rJ = torch.empty_like(gU[b]), torch.empty_like(gJ[b])
        ctx.es_rk_stage(1, dt[b:b + 1].clone(), gU[b], gJ[b], gU[b], gJ[b], jx[b], None, rU, rJ)
        ctx.es_fill_ghosts(rU, sp["nspec"] + 3)
        ctx.es_fill_ghosts(rJ, 1)
        assert torch.equal(outU[b], rU), b
        assert torch.equal(outJ[b], rJ), b
    hdt = host(dt)
    for b, (o, JU, J, ojx) in orc.items():
        sp = specs[b]
        _, lam, odt = o.max_wavespeed(JU, J, ojx, 0.4)
        assert hdt[b] == pytest.approx(odt, rel=1e-13)
        rc, oU, oJ = o.rk_stage(1, odt, JU, J, JU, J, ojx, np.zeros((2,) + J.shape[1:]))
        assert rc == 0
        o.fill_ghosts(oU, o.nc)
        sc = state_scale(JU, sp, lam)
        hU = host(outU[b])
        errs = [parity(hU[c], oU[c], sc[c]) for c in range(o.nc)]
        say(f"    instance {b} ({sp['n'][0]}^2) vs oracle: {max(errs):.1e}")
        assert max(errs) <= TOL_FP64
    assert batch.es_batch_status()[0] == es.ES_OK
