"""Pins of the CPU oracle's whole-grid steps (no GPU): ghost layers, discrete
GCL metrics, free-stream preservation, entropy conservation / stability,
design order, mesh redistribution and the CFL step."""
import numpy as np
import pytest

import oracle
from paper_2202_07989_amd import inputs as I


def ghosts_all(o, JU, J, x):
    o.fill_ghosts(JU, o.nc)
    o.fill_ghosts(J, 1)
    o.fill_ghosts_x(x)


def padded_xi(sp):
    """Computational coordinates of every padded node."""
    ng, d = sp["ng"], sp["dim"]
    ax = [(np.arange(sp["n"][k] + 2 * ng) - ng + 0.5) * sp["dxi"][k] if k < d else np.zeros(1)
          for k in range(3)]
    g2, g1, g0 = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return [g0, g1, g2][:d]


def delta(a, k, w, alpha):
    """2w-th order undivided central difference along array axis of direction k."""
    ax = a.ndim - 1 - k
    s = np.zeros_like(a)
    for m in range(1, w + 1):
        s += alpha[m - 1] * (np.roll(a, -m, axis=ax) - np.roll(a, m, axis=ax))
    return 0.5 * s


# -- periodic ghost layers (Section 5 periodic runs) --------------------------
@pytest.mark.parametrize("dim", [2, 3])
def test_ghost_fill_periodic_and_mesh_offsets(dim):
    sp = I.make_spec(dim, 1, (6,) * dim, box=(2.0, 3.0, 5.0)[:dim])
    o = oracle.Oracle(sp)
    xi = padded_xi(sp)
    x = np.stack(xi)                          # x = xi on the padded grid (exact ghosts)
    xg = np.zeros_like(x)
    Iin = I.interior(sp)
    xg[Iin] = x[Iin]
    o.fill_ghosts_x(xg)
    np.testing.assert_allclose(xg, x, rtol=0, atol=1e-14)
    f = np.zeros((2,) + x.shape[1:])
    rng = np.random.default_rng(0)
    f[Iin] = rng.uniform(size=f[Iin].shape)
    o.fill_ghosts(f, 2)
    # every padded node equals its periodic image
    ng = sp["ng"]
    for ax in range(dim):
        axis = 3 - ax
        n = sp["n"][ax]
        g = np.take(f, range(0, ng), axis=axis)
        img = np.take(f, range(n, n + ng), axis=axis)
        np.testing.assert_array_equal(g, img)


# -- eq SCLCoeff: discrete SCL, affine exactness, order ------------------------
@pytest.mark.parametrize("dim,w", [(2, 3), (3, 3), (3, 2), (3, 1)])
def test_discrete_scl(dim, w):
    n = (12,) * dim if dim == 3 else (20, 16)
    sp = I.make_spec(dim, 1, n, box=(1.0, 2.0, 1.5)[:dim], w=w)
    o = oracle.Oracle(sp)
    x = I.zeros(sp, dim)
    x[I.interior(sp)] = np.stack(I.random_mesh(sp, seed=3, amp=0.05))
    o.fill_ghosts_x(x)
    jx, _ = o.metrics(x)
    al = o.alpha(w)
    Iin = I.interior(sp)
    for j in range(dim):
        div = sum(delta(jx[k * dim + j], k, w, al) / sp["dxi"][k] for k in range(dim))
        scale = max(np.abs(jx[k * dim + j][Iin[1:]]).max() / sp["dxi"][k] for k in range(dim))
        assert np.abs(div[Iin[1:]]).max() < 1e-13 * scale


def test_metrics_affine_exact_3d():
    """For x = A xi + b (ghosts evaluated exactly) the metrics are the
    cofactors J dxi_k/dx_j = det(A) (A^-1)_{kj}, exactly."""
    sp = I.make_spec(3, 1, (7, 8, 9), box=(1.0, 1.3, 0.7))
    o = oracle.Oracle(sp)
    A = np.array([[1.2, 0.3, -0.1], [0.2, 0.9, 0.25], [-0.15, 0.1, 1.1]])
    b = np.array([0.3, -0.2, 0.5])
    xi = padded_xi(sp)
    x = np.stack([sum(A[p, q] * xi[q] for q in range(3)) + b[p] for p in range(3)])
    jx, jt = o.metrics(np.ascontiguousarray(x))
    cof = np.linalg.det(A) * np.linalg.inv(A)
    Iin = I.interior(sp)
    for k in range(3):
        for j in range(3):
            np.testing.assert_allclose(jx[k * 3 + j][Iin[1:]], cof[k, j], rtol=1e-12, atol=1e-12)
    assert np.abs(jt).max() == 0.0


def test_metrics_affine_exact_2d():
    sp = I.make_spec(2, 2, (9, 7), box=(1.0, 1.3))
    o = oracle.Oracle(sp)
    A = np.array([[1.2, 0.3], [-0.2, 0.9]])
    xi = padded_xi(sp)
    x = np.stack([sum(A[p, q] * xi[q] for q in range(2)) for p in range(2)])
    jx, _ = o.metrics(np.ascontiguousarray(x))
    cof = np.linalg.det(A) * np.linalg.inv(A)
    Iin = I.interior(sp)
    for k in range(2):
        for j in range(2):
            np.testing.assert_allclose(jx[k * 2 + j][Iin[1:]], cof[k, j], rtol=1e-13)


def test_metrics_sixth_order_on_curvilinear_mesh():
    """Config-1 mesh: J dxi/dx -> analytic cofactors (y_eta, -x_eta, -y_xi,
    x_xi) at order 2w = 6."""
    errs = []
    for n in (16, 32):
        sp = I.spec_c1(n)
        o = oracle.Oracle(sp)
        _, _, x = I.init_c1(sp)
        o.fill_ghosts_x(x)
        jx, _ = o.metrics(x)
        xi, eta = I.xi_nodes(sp)
        a = 0.1 * 2 * np.pi
        x_xi = 1 + a * np.cos(2 * np.pi * xi) * np.sin(2 * np.pi * eta)
        x_eta = a * np.sin(2 * np.pi * xi) * np.cos(2 * np.pi * eta)
        y_xi, y_eta = x_xi - 1, x_eta + 1
        ref = [y_eta, -x_eta, -y_xi, x_xi]
        Iin = I.interior(sp)
        errs.append(max(np.abs(jx[c][Iin[1:]] - ref[c]).max() for c in range(4)))
    order = np.log2(errs[0] / errs[1])
    assert order > 5.7, (errs, order)


# -- Remark 3.1: free stream on a moving mesh ---------------------------------
@pytest.mark.parametrize("dim,nspec", [(2, 1), (2, 2), (3, 2)])
def test_free_stream_moving_mesh(dim, nspec):
    n = (16, 12) if dim == 2 else (8, 8, 8)
    sp = I.make_spec(dim, nspec, n, gamma=(4.4, 1.4)[:nspec] if nspec == 2 else (1.4,),
                     cv=(1.0, 1.0)[:nspec], pinf=(6e8, 0.0)[:nspec] if nspec == 2 else (0.0,),
                     chi=I.CHI_SHOCK)
    o = oracle.Oracle(sp)
    xi = I.xi_nodes(sp)
    rho = [np.full_like(xi[0], r) for r in (1000.0, 1.5)[:nspec]]
    v = [np.full_like(xi[0], a) for a in (0.7, -0.4, 0.2)[:dim]]
    p = np.full_like(xi[0], 1e5)
    U = I.conserved(sp, rho, v, p)
    mesh = I.random_mesh(sp, seed=5, amp=0.04)
    J = 1.0 + 0.3 * np.sin(2 * np.pi * xi[0]) * np.cos(2 * np.pi * xi[1])
    JU, Jp, x = I.assemble(sp, U, J, mesh)
    mon = I.monitor_spec(n_sweeps=4)
    for _ in range(3):
        rc, dt, dtau = o.step(JU, Jp, x, mon=mon, cfl=0.3, move_mesh=True)
        assert rc == 0 and dtau > 0
    Iin = I.interior(sp)
    Uc = JU[Iin] / Jp[Iin]
    for c in range(o.nc):
        ref = U[c]
        np.testing.assert_allclose(Uc[c], ref, rtol=1e-12, atol=1e-12 * max(1.0, np.abs(ref).max()))


# -- Prop. 3.1 / eq NumEntropyID: global entropy conservation of the EC scheme -
def entropy_scale(o, sp, JU, J, dJU, dJ):
    Iin = I.interior(sp)
    U = (JU[Iin] / J[Iin]).reshape(o.nc, -1)
    dU = dJU[Iin].reshape(o.nc, -1)
    dj = dJ[Iin].reshape(-1)
    tot = 0.0
    for i in range(U.shape[1]):
        V = o.entropy_vars(U[:, i].copy())
        tot += np.abs(V * dU[:, i]).sum() + abs(o.potential(U[:, i].copy()) * dj[i])
    return tot * np.prod(sp["dxi"][: sp["dim"]])


@pytest.mark.parametrize("dim,nspec,pinf", [(2, 1, (0.0,)), (2, 2, (6e8, 0.0)), (3, 2, (100.0, 0.0)),
                                            (3, 1, (2.0,))])
def test_ec_scheme_conserves_entropy(dim, nspec, pinf):
    n = (14, 12) if dim == 2 else (8, 9, 7)
    sp = I.make_spec(dim, nspec, n, gamma=(4.4, 1.4)[:nspec] if nspec == 2 else (1.4,),
                     cv=(1.0, 2.0)[:nspec], pinf=pinf, dissipation=0)
    o = oracle.Oracle(sp)
    kw = dict(p_range=(1e5, 3e5)) if sum(pinf) > 1e3 else {}
    JU, J, x = I.init_random(sp, seed=21, noise=0.3, **kw)
    disp = I.zeros(sp, dim)
    disp[I.interior(sp)] = 0.01 * np.stack(I.random_mesh(sp, seed=9, amp=1.0)) \
        - 0.01 * np.stack(I.xi_nodes(sp))
    ghosts_all(o, JU, J, x)
    o.fill_ghosts(disp, dim)
    jx, jt = o.metrics(x, disp, c_s=0.5, dt=0.01)
    assert np.abs(jt).max() > 0
    rc, dJU, dJ = o.rhs(JU, J, jx, jt)
    assert rc == 0
    rate = o.entropy_rate(JU, J, dJU, dJ)
    assert abs(rate) < 1e-12 * entropy_scale(o, sp, JU, J, dJU, dJ)


@pytest.mark.parametrize("sign_tol", [0.0, I.SIGN_TOL_FP64])
@pytest.mark.parametrize("recon", [0, 1])
@pytest.mark.parametrize("dim,nspec,pinf", [(2, 1, (0.0,)), (2, 2, (6e8, 0.0)), (3, 2, (100.0, 0.0))])
def test_es_scheme_entropy_production(dim, nspec, pinf, recon, sign_tol):
    """The ES flux adds -s/2 sum_m Y_mm [[W_m]][[W_m]]^WENO <= 0 per interface
    (eq HOstable with the sign matrix), nothing else; with either
    reconstruction (multi-resolution, or the classical WENO5 of MM-WENOJS)
    and with the sign test as printed (sign_tol = 0) or with its zero
    tolerance."""
    n = (14, 12) if dim == 2 else (8, 9, 7)
    kw = dict(gamma=(4.4, 1.4)[:nspec] if nspec == 2 else (1.4,), cv=(1.0, 2.0)[:nspec],
              pinf=pinf, chi=I.CHI_SHOCK, reconstruction=recon, weno_eps=1e-6 if recon else 1e-10,
              sign_tol=sign_tol)
    sp_es = I.make_spec(dim, nspec, n, dissipation=1, **kw)
    sp_ec = I.make_spec(dim, nspec, n, dissipation=0, **kw)
    o_es, o_ec = oracle.Oracle(sp_es), oracle.Oracle(sp_ec)
    pk = dict(p_range=(1e5, 3e5)) if sum(pinf) > 1e3 else {}
    JU, J, x = I.init_random(sp_es, seed=31, noise=0.5, **pk)
    ghosts_all(o_es, JU, J, x)
    disp = I.zeros(sp_es, dim)
    jx, jt = o_es.metrics(x, disp, c_s=0.0, dt=1.0)
    _, dJU_es, dJ_es = o_es.rhs(JU, J, jx, jt)
    _, dJU_ec, dJ_ec = o_ec.rhs(JU, J, jx, jt)
    r_es = o_es.entropy_rate(JU, J, dJU_es, dJ_es)
    r_ec = o_ec.entropy_rate(JU, J, dJU_ec, dJ_ec)
    prod = o_es.es_production(JU, J, jx, jt)
    assert prod < 0
    assert r_es < 0
    scale = entropy_scale(o_es, sp_es, JU, J, dJU_es, dJ_es)
    assert abs((r_es - r_ec) - prod) < 1e-12 * scale
    np.testing.assert_allclose(dJ_es, dJ_ec, rtol=0, atol=0)


def test_constant_state_rhs_vanishes_on_fixed_mesh():
    sp = I.spec_c1(12)
    o = oracle.Oracle(sp)
    _, J, x = I.init_c1(sp)
    xi = I.xi_nodes(sp)
    U = I.conserved(sp, [np.full_like(xi[0], 1.3)], [np.full_like(xi[0], 0.4), np.full_like(xi[0], -0.2)],
                    np.full_like(xi[0], 2.0))
    JU, J, x = I.assemble(sp, U, J[I.interior(sp)][0], [x[I.interior(sp)][c] for c in range(2)])
    ghosts_all(o, JU, J, x)
    jx, jt = o.metrics(x)
    rc, dJU, dJ = o.rhs(JU, J, jx, jt)
    assert rc == 0
    assert np.abs(dJU).max() < 1e-11 * np.abs(JU).max() * 12
    assert np.abs(dJ).max() == 0.0


def test_rhs_points_matches_rhs():
    sp = I.make_spec(3, 2, (8, 7, 6), gamma=(4.4, 1.4), cv=(1.0, 1.0), pinf=(6e8, 0.0),
                     chi=I.CHI_SHOCK)
    o = oracle.Oracle(sp)
    JU, J, x = I.init_shock_bubble(sp)
    ghosts_all(o, JU, J, x)
    jx, jt = o.metrics(x)
    _, dJU, dJ = o.rhs(JU, J, jx, jt)
    Iin = I.interior(sp)
    flat = np.arange(o.P).reshape(J.shape[1:])[Iin[1:]].reshape(-1)[::7]
    _, pU, pJ = o.rhs_points(JU, J, jx, jt, flat)
    np.testing.assert_array_equal(pU, dJU.reshape(o.nc, -1)[:, flat].T)
    np.testing.assert_array_equal(pJ, dJ.reshape(-1)[flat])


# -- Section 5: design order on smooth advection (config-1 mesh) ---------------
@pytest.mark.parametrize("dissipation,recon,min_order", [(1, 0, 4.5), (0, 0, 5.0), (1, 1, 4.5)])
def test_design_order_smooth_advection(dissipation, recon, min_order):
    T = 0.04
    errs = []
    for n in (16, 32, 64):
        sp = I.spec_c1(n)
        sp["dissipation"] = dissipation
        if recon:
            sp["reconstruction"], sp["weno_eps"] = recon, 1e-6
        o = oracle.Oracle(sp)
        JU, J, x = I.init_c1(sp)
        dt0 = 0.5 * (1.0 / n) ** (5.0 / 3.0)
        nsteps = int(np.ceil(T / dt0))
        dt = T / nsteps
        for _ in range(nsteps):
            rc, _, _ = o.step(JU, J, x, dt_fixed=dt)
            assert rc == 0
        Iin = I.interior(sp)
        rho = JU[Iin][0] / J[Iin][0]
        ex = I.c1_exact_rho(x[Iin][0], x[Iin][1], T)
        errs.append(np.abs(rho - ex).mean())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert orders[-1] > min_order, (errs, orders)


# -- Section 4: mesh redistribution --------------------------------------------
def test_jacobian_affine_exact_and_sixth_order():
    """The discrete Jacobian of a mesh: exact (to rounding) on an affine mesh
    of either dimension, where the central differences are exact, and order
    6 against the analytic Jacobian of the curvilinear C1 mesh."""
    rng = np.random.default_rng(51)
    for dim in (2, 3):
        n = (10, 9) if dim == 2 else (8, 7, 9)
        sp = I.make_spec(dim, 1, n)
        o = oracle.Oracle(sp)
        A = np.eye(dim) + 0.3 * rng.uniform(-1, 1, (dim, dim))
        xi = I.xi_nodes(sp)
        x = I.zeros(sp, dim)
        Iin = I.interior(sp)
        for k in range(dim):
            x[k][Iin[1:]] = sum(A[k, j] * xi[j] for j in range(dim))
        # periodic images of an affine map: x(xi + L e_j) = x(xi) + L A e_j, so
        # the ghost layers are filled by extrapolating the affine map
        pad = padded_xi(sp)
        for k in range(dim):
            x[k] = sum(A[k, j] * pad[j] for j in range(dim))
        jx, _ = o.metrics(x)
        Jd = o.jacobian(x, jx)
        np.testing.assert_allclose(Jd[Iin], np.linalg.det(A), rtol=1e-12)
    errs = []
    for n in (16, 32):
        sp = I.spec_c1(n)
        o = oracle.Oracle(sp)
        JU, J, x = I.init_c1(sp)
        o.fill_ghosts_x(x)
        jx, _ = o.metrics(x)
        Iin = I.interior(sp)
        errs.append(np.abs(o.jacobian(x, jx)[Iin] - J[Iin]).max())
    assert np.log2(errs[0] / errs[1]) > 5.5, errs


@pytest.mark.parametrize("dim", [2, 3])
def test_vortex_monitor_closed_form(dim):
    """The monitor of the isentropic-vortex examples (form 1), unfiltered, on
    rho = 1.5 + 0.5 sin(kappa xi_0): the second-order central differences of
    a sine are exact in closed form, |grad| = 0.5 |cos(kappa xi_0)| sin(kappa h)/h
    and |lap| = 0.5 |sin(kappa xi_0)| (2 - 2 cos(kappa h))/h^2, so Theta^2 =
    1 + 20 |grad|/max|grad| + 10 |lap|/max|lap| node by node; the maxima are
    over the grid nodes.  An exactly constant field drops both terms (Theta = 1)."""
    n = (24, 20) if dim == 2 else (16, 12, 10)
    sp = I.make_spec(dim, 1, n, box=(20.0,) * dim)
    o = oracle.Oracle(sp)
    JU, J, x = I.init_random(sp, seed=41, noise=0.0)
    ghosts_all(o, JU, J, x)
    Iin = I.interior(sp)
    xi0 = I.xi_nodes(sp)[0]
    h = sp["dxi"][0]
    kap = 2.0 * np.pi / (sp["n"][0] * h)
    rho = 1.5 + 0.5 * np.sin(kap * xi0)
    JU[0][Iin[1:]] = J[0][Iin[1:]] * rho
    o.fill_ghosts(JU, o.nc)
    mon = dict(sigma=[0], alpha=[20.0], beta=[10.0], form=1, n_smooth=0, n_sweeps=1)
    rc, th = o.monitor_fn(mon, JU, J)
    assert rc == 0
    gr = 0.5 * np.abs(np.cos(kap * xi0)) * np.sin(kap * h) / h
    lp = 0.5 * np.abs(np.sin(kap * xi0)) * (2.0 - 2.0 * np.cos(kap * h)) / h ** 2
    ref = np.sqrt(1.0 + 20.0 * gr / gr.max() + 10.0 * lp / lp.max())
    np.testing.assert_allclose(th[Iin][0], ref, rtol=1e-12)
    # (J = 1, so that rho = JU/J is exactly constant: the normalisation by
    # the maximum would lift rounding-level gradients to O(1))
    J[...] = 1.0
    JU[0][...] = 1.25
    rc, th = o.monitor_fn(mon, JU, J)
    np.testing.assert_array_equal(th[Iin][0], 1.0)
    # more than two variables is not a valid form-1 monitor
    rc, _ = o.monitor_fn(dict(mon, sigma=[0, 3, 0], alpha=[1.0] * 3, beta=[1.0] * 3), JU, J)
    assert rc != 0


@pytest.mark.parametrize("dim", [2, 3])
def test_mesh_uniform_fixed_point_and_filter(dim):
    n = (16, 12) if dim == 2 else (6, 7, 8)
    sp = I.make_spec(dim, 1, n)
    o = oracle.Oracle(sp)
    xi = I.xi_nodes(sp)
    U = I.conserved(sp, [np.full_like(xi[0], 1.0)], [np.zeros_like(xi[0])] * dim, np.ones_like(xi[0]))
    JU, J, x = I.assemble(sp, U, np.ones_like(xi[0]), xi)
    ghosts_all(o, JU, J, x)
    rc, th = o.monitor_fn(I.monitor_spec(), JU, J)
    assert rc == 0
    np.testing.assert_array_equal(th[I.interior(sp)], 1.0)
    rc, disp, dtau, resid = o.mesh_redistribute(I.monitor_spec(n_sweeps=10), JU, J, x)
    assert rc == 0
    assert np.abs(disp).max() < 1e-15
    assert resid.max() < 1e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_mesh_limiter_and_monotone_motion(dim):
    """Delta_tau keeps each node within half a neighbour spacing of x^n along
    its own coordinate, and the mesh follows the density gradient."""
    n = (24, 20) if dim == 2 else (10, 10, 10)
    sp = I.make_spec(dim, 2, n, gamma=(4.4, 1.4), cv=(1.0, 1.0), pinf=(6e8, 0.0), chi=I.CHI_SHOCK)
    o = oracle.Oracle(sp)
    JU, J, x = I.init_shock_bubble(sp)
    ghosts_all(o, JU, J, x)
    rc, disp, dtau, resid = o.mesh_redistribute(I.monitor_spec(n_sweeps=10), JU, J, x)
    assert rc == 0
    assert 0 < dtau <= 1
    assert np.abs(disp).max() > 0
    Iin = I.interior(sp)
    for k in range(dim):
        ax = 3 - k
        d = disp[k]
        xp = np.roll(x[k], -1, axis=ax - 1)
        xm = np.roll(x[k], 1, axis=ax - 1)
        right = (xp - x[k])[Iin[1:]]
        left = (x[k] - xm)[Iin[1:]]
        dk = d[Iin[1:]]
        assert np.all(dk <= 0.5 * right * (1 + 1e-12))
        assert np.all(-dk <= 0.5 * left * (1 + 1e-12))
    # Jacobi residuals decrease
    assert resid[-1] < resid[0]


@pytest.mark.parametrize("dim", [2, 3])
def test_filter_weights_preserve_constants(dim):
    n = (10, 9) if dim == 2 else (6, 5, 7)
    sp = I.make_spec(dim, 1, n)
    o = oracle.Oracle(sp)
    xi = I.xi_nodes(sp)
    U = I.conserved(sp, [np.full_like(xi[0], 2.0)], [np.zeros_like(xi[0])] * dim, np.ones_like(xi[0]))
    JU, J, x = I.assemble(sp, U, np.ones_like(xi[0]), xi)
    ghosts_all(o, JU, J, x)
    # a constant monitor through n_smooth passes stays exactly 1
    rc, disp, dtau, resid = o.mesh_redistribute(I.monitor_spec(n_smooth=7, n_sweeps=1), JU, J, x)
    assert rc == 0 and np.abs(disp).max() < 1e-15


# -- eq cfl: closed form on a Cartesian mesh -------------------------------------
@pytest.mark.parametrize("dim,nspec", [(2, 1), (3, 2)])
def test_cfl_closed_form(dim, nspec):
    """Stretched Cartesian mesh x_k = s_k xi_k (J = prod s_k): lambda =
    sum_k (|v_k| + c) / (s_k dxi_k), the physical-spacing CFL."""
    n = (12, 10) if dim == 2 else (6, 5, 4)
    kw = dict(gamma=(4.4, 1.4), cv=(1.0, 1.0), pinf=(6e8, 0.0)) if nspec == 2 else {}
    sp = I.make_spec(dim, nspec, n, box=(1.0, 2.0, 3.0)[:dim], **kw)
    s = (1.5, 0.5, 2.0)[:dim]
    sp["len"] = tuple(sp["len"][k] * (s[k] if k < dim else 1.0) for k in range(3))
    o = oracle.Oracle(sp)
    xi = I.xi_nodes(sp)
    vel = (0.3, -1.2, 0.5)[:dim]
    rho = [np.full_like(xi[0], r) for r in (1000.0, 1.0)[:nspec]]
    p = 1e5 if nspec == 2 else 1.0
    U = I.conserved(sp, rho, [np.full_like(xi[0], a) for a in vel], np.full_like(xi[0], p))
    Jv = np.prod(s)
    JU, J, x = I.assemble(sp, U, np.full_like(xi[0], Jv), [s[k] * xi[k] for k in range(dim)])
    ghosts_all(o, JU, J, x)
    jx, _ = o.metrics(x)
    rc, lam, dt = o.max_wavespeed(JU, J, jx, 0.4)
    c = o.sound_speed(U[:, 0, 0, 0].copy())
    ref = sum((abs(vel[k]) + c) / (s[k] * sp["dxi"][k]) for k in range(dim))
    assert lam == pytest.approx(ref, rel=1e-12)
    assert dt == pytest.approx(0.4 / ref, rel=1e-12)


# -- eq VCLCoeff + eq semi_J: J follows the mesh's own Jacobian ---------------
def _geometric_jacobian(sp, x_int):
    """det(dx/dxi) with spectral derivatives of the periodic part x - xi."""
    d = sp["dim"]
    xi = I.xi_nodes(sp)
    A = np.zeros((d, d) + x_int[0].shape)
    for p in range(d):
        f = x_int[p] - xi[p]
        F = np.fft.fftn(f)
        for q in range(d):
            ax = 2 - q                       # arrays are (n2, n1, n0)
            n = f.shape[ax]
            k = np.fft.fftfreq(n, d=sp["dxi"][q]) * 2j * np.pi
            shape = [1] * f.ndim
            shape[ax] = n
            A[p, q] = np.real(np.fft.ifftn(F * k.reshape(shape))) + (1.0 if p == q else 0.0)
    return np.linalg.det(np.moveaxis(A, (0, 1), (-2, -1)))


@pytest.mark.parametrize("dim", [2, 3])
def test_vcl_matches_geometric_jacobian_rate(dim):
    n = (32, 32) if dim == 2 else (24, 24, 24)
    sp = I.make_spec(dim, 1, n)
    o = oracle.Oracle(sp)
    Iin = I.interior(sp)
    xm = I.random_mesh(sp, seed=41, amp=0.03)
    vel = [0.05 * v for v in I.random_mesh(sp, seed=42, amp=1.0)]
    vel = [vel[k] - I.xi_nodes(sp)[k] * 0.05 for k in range(dim)]          # periodic field
    JU, J, x = I.assemble(sp, I.conserved(sp, [np.ones_like(xm[0])], [np.zeros_like(xm[0])] * dim,
                                          np.ones_like(xm[0])), np.ones_like(xm[0]), xm)
    disp = I.zeros(sp, dim)
    disp[Iin] = np.stack(vel)
    ghosts_all(o, JU, J, x)
    o.fill_ghosts(disp, dim)
    jx, jt = o.metrics(x, disp, c_s=0.0, dt=1.0)          # xdot = vel
    _, _, dJ = o.rhs(JU, J, jx, jt)
    eps = 1e-4
    Jp = _geometric_jacobian(sp, [xm[k] + eps * vel[k] for k in range(dim)])
    Jm = _geometric_jacobian(sp, [xm[k] - eps * vel[k] for k in range(dim)])
    rate = (Jp - Jm) / (2 * eps)
    got = dJ[Iin][0]
    assert np.abs(got - rate).max() < 2e-3 * np.abs(rate).max()


# -- Section 4: Jacobi iteration converges to the discrete equidistribution ----
def test_jacobi_fixed_point_is_equidistribution():
    """Theta varying along xi_1 only: the converged iterate satisfies
    Theta_{i+1/2} (x_{i+1} - x_i) = const, the discrete form of
    (Theta x_xi)_xi = 0."""
    sp = I.make_spec(2, 1, (24, 4))
    o = oracle.Oracle(sp)
    xi = I.xi_nodes(sp)
    rho = 1.0 + 0.5 * np.exp(-((xi[0] - 0.4) / 0.08) ** 2)
    U = I.conserved(sp, [rho], [np.zeros_like(rho)] * 2, np.ones_like(rho))
    JU, J, x = I.assemble(sp, U, np.ones_like(rho), xi)
    ghosts_all(o, JU, J, x)
    mon = I.monitor_spec(n_sweeps=3000, n_smooth=0, alpha=(50.0,))
    _, th = o.monitor_fn(mon, JU, J)
    rc, disp, dtau, resid = o.mesh_redistribute(mon, JU, J, x)
    assert rc == 0 and dtau > 0
    Iin = I.interior(sp)
    xmu = (x + disp / dtau)[Iin]
    x1 = xmu[0, 0, 0]                     # one row along xi_1
    t1 = th[Iin][0, 0, 0]
    # periodic neighbour across the seam carries +L
    x1e = np.concatenate([x1, [x1[0] + 1.0]])
    te = np.concatenate([t1, [t1[0]]])
    flux = 0.5 * (te[1:] + te[:-1]) * np.diff(x1e)
    assert flux.std() < 1e-9 * flux.mean()
    np.testing.assert_allclose(xmu[1], x[Iin][1], atol=1e-15)
    assert resid[-1] < 1e-14


def test_limiter_binds_at_half_spacing():
    sp = I.make_spec(2, 2, (32, 32), gamma=(4.4, 1.4), cv=(1.0, 1.0), pinf=(6e8, 0.0), chi=I.CHI_SHOCK)
    o = oracle.Oracle(sp)
    JU, J, x = I.init_shock_bubble(sp)
    ghosts_all(o, JU, J, x)
    rc, disp, dtau, _ = o.mesh_redistribute(I.monitor_spec(n_sweeps=200, alpha=(1e5,)), JU, J, x)
    assert rc == 0 and 0 < dtau < 1
    Iin = I.interior(sp)
    worst = 0.0
    for k in range(2):
        ax = 3 - k - 1
        xp = np.roll(x[k], -1, axis=ax)
        xm = np.roll(x[k], 1, axis=ax)
        dk = disp[k][Iin[1:]]
        sp_r = (xp - x[k])[Iin[1:]]
        sp_l = (x[k] - xm)[Iin[1:]]
        ratio = np.where(dk > 0, dk / (0.5 * sp_r), np.where(dk < 0, -dk / (0.5 * sp_l), 0.0))
        worst = max(worst, ratio.max())
    assert worst == pytest.approx(1.0, rel=1e-12)


def test_filter_is_separable_binomial():
    """The low-pass filter's weights (1/2)^(|j|_1 + d) factor into the 1D
    [1/4, 1/2, 1/4] filter along each direction."""
    for dim, n in ((2, (12, 10)), (3, (6, 7, 5))):
        sp = I.make_spec(dim, 2, n, gamma=(4.4, 1.4), cv=(1.0, 1.0), pinf=(6e8, 0.0), chi=I.CHI_SHOCK)
        o = oracle.Oracle(sp)
        JU, J, x = I.init_random(sp, seed=51, noise=0.5, p_range=(1e5, 2e5))
        ghosts_all(o, JU, J, x)
        _, th0 = o.monitor_fn(I.monitor_spec(n_smooth=0), JU, J)
        _, th2 = o.monitor_fn(I.monitor_spec(n_smooth=2), JU, J)
        Iin = I.interior(sp)
        f = th0[Iin][0].copy()
        for _ in range(2):
            for ax in range(f.ndim):
                if f.shape[ax] > 1:
                    f = 0.25 * np.roll(f, 1, ax) + 0.5 * f + 0.25 * np.roll(f, -1, ax)
        np.testing.assert_allclose(th2[Iin][0], f, rtol=1e-14)


# -- reflection equivariance of the whole semi-discrete operator -------------------
@pytest.mark.parametrize("dim", [2, 3])
def test_rhs_reflection_equivariance(dim):
    """Mirroring xi_1 and x_1 (and v_1) maps the RHS onto its mirror image:
    every stencil, the interface averages, the WENO pair and the sign test
    treat left and right alike."""
    n = (12, 10) if dim == 2 else (8, 7, 6)
    sp = I.make_spec(dim, 2, n, gamma=(4.4, 1.4), cv=(1.0, 2.0), pinf=(100.0, 0.0), chi=I.CHI_SHOCK)
    o = oracle.Oracle(sp)
    Iin = I.interior(sp)
    JU, J, x = I.init_random(sp, seed=61, noise=0.4, mesh_amp=0.04)
    disp = I.zeros(sp, dim)
    disp[Iin] = 0.02 * (np.stack(I.random_mesh(sp, seed=62, amp=1.0)) - np.stack(I.xi_nodes(sp)))

    def run(JU, J, x, disp):
        JU, J, x, disp = JU.copy(), J.copy(), x.copy(), disp.copy()
        ghosts_all(o, JU, J, x)
        o.fill_ghosts(disp, dim)
        jx, jt = o.metrics(x, disp, c_s=0.5, dt=0.1)
        rc, dJU, dJ = o.rhs(JU, J, jx, jt)
        assert rc == 0
        return dJU[Iin], dJ[Iin]

    def mirror(a, neg):
        b = a.copy()
        b[Iin] = a[Iin][..., ::-1]
        for c in neg:
            b[c][Iin[1:]] *= -1
        return b

    N = 2
    L1 = sp["len"][0]
    xr = mirror(x, [0])
    xr[0][Iin[1:]] += L1             # keep x_1 in [0, L_1) (periodic shift)
    dU, dJ = run(JU, J, x, disp)
    dUr, dJr = run(mirror(JU, [N]), mirror(J, []), xr, mirror(disp, [0]))
    ref = dU[..., ::-1].copy()
    ref[N] *= -1
    scale = np.abs(dU).max(axis=(1, 2, 3), keepdims=True)
    assert np.abs(dUr - ref).max() / 1.0 < 1e-11 * scale.max()
    for c in range(o.nc):
        assert np.abs(dUr[c] - ref[c]).max() < 1e-11 * scale[c].max(), c
    np.testing.assert_allclose(dJr, dJ[..., ::-1], atol=1e-11 * np.abs(dJ).max())


# -- Sections 3.2 + 5: design order on a moving mesh (prescribed smooth motion) -
def test_design_order_prescribed_moving_mesh():
    """The mesh moves as x(xi, t) = x0 + b(xi) sin(40 t) with one displacement
    per step applied linearly over the step (stage meshes x^n + c_s disp,
    xdot = disp/dt); J follows the VCL only.  The error against the exact
    advected density at the moving nodes falls at high order.  (Monitor-
    driven meshes at 16..64 points carry unresolved high-wavenumber content,
    so this pin prescribes the motion.)"""
    T = 0.04
    errs = []
    for n in (16, 32, 64):
        sp = I.spec_c1(n)
        o = oracle.Oracle(sp)
        JU, J, x = I.init_c1(sp)
        Iin = I.interior(sp)
        xi = I.xi_nodes(sp)
        base = [x[Iin][0].copy(), x[Iin][1].copy()]
        bump = 0.05 * np.sin(2 * np.pi * xi[0]) * np.cos(2 * np.pi * xi[1])

        def mesh(t):
            return np.stack([base[0] + bump * np.sin(40 * t), base[1] + 0.5 * bump * np.sin(40 * t)])

        dt0 = 0.5 * (1.0 / n) ** (5.0 / 3.0)
        nsteps = int(np.ceil(T / dt0))
        dt = T / nsteps
        t = 0.0
        for _ in range(nsteps):
            ghosts_all(o, JU, J, x)
            disp = I.zeros(sp, 2)
            disp[Iin] = mesh(t + dt) - x[Iin]
            o.fill_ghosts(disp, 2)
            JUn, Jn = JU.copy(), J.copy()
            for st in range(3):
                _, _, c = o.rk_coeffs(st)
                jx, jt = o.metrics(x, disp, c, dt)
                rc, JU, J = o.rk_stage(st, dt, JUn, Jn, JU, J, jx, jt)
                assert rc == 0
                o.fill_ghosts(JU, o.nc)
                o.fill_ghosts(J, 1)
            x = x + disp
            t += dt
        rho = JU[Iin][0] / J[Iin][0]
        ex = I.c1_exact_rho(x[Iin][0], x[Iin][1], T)
        errs.append(np.abs(rho - ex).mean())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert orders[-1] > 4.4, (errs, orders)


@pytest.mark.parametrize("dim", [2, 3])
def test_mesh_redistribution_reflection_equivariance(dim):
    """Mirroring xi_k and x_k mirrors the displacement and leaves Delta_tau
    unchanged, for every direction k: monitor, filter, Jacobi sweeps and both
    limiter branches treat left and right alike."""
    n = (24, 20) if dim == 2 else (10, 9, 8)
    sp = I.make_spec(dim, 2, n, gamma=(4.4, 1.4), cv=(1.0, 1.0), pinf=(6e8, 0.0), chi=I.CHI_SHOCK)
    o = oracle.Oracle(sp)
    Iin = I.interior(sp)
    JU, J, x = I.init_shock_bubble(sp, shock_x=0.3)
    x[Iin] += 0.01 * (np.stack(I.random_mesh(sp, seed=71, amp=1.0)) - np.stack(I.xi_nodes(sp)))
    mon = I.monitor_spec(n_sweeps=40, alpha=(3e4,))

    def mirror(a, k, neg):
        b = a.copy()
        ax = 3 - k
        b[Iin] = np.flip(a[Iin], axis=ax)
        for c in neg:
            b[c][Iin[1:]] *= -1
        return b

    def redistribute(JUa, Ja, xa):
        ghosts_all(o, JUa, Ja, xa)
        rc, disp, dtau, _ = o.mesh_redistribute(mon, JUa, Ja, xa)
        assert rc == 0
        return disp, dtau

    d0, t0 = redistribute(JU.copy(), J.copy(), x.copy())
    assert t0 < 1
    for k in range(dim):
        xr = mirror(x, k, [k])
        xr[k][Iin[1:]] += sp["len"][k]
        d1, t1 = redistribute(mirror(JU, k, [2 + k]), mirror(J, k, []), xr)
        assert t1 == pytest.approx(t0, rel=1e-12), k
        ref = np.flip(d0[Iin], axis=3 - k).copy()
        ref[k] *= -1
        np.testing.assert_allclose(d1[Iin], ref, atol=1e-13 * np.abs(d0).max())
