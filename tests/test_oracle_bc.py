"""Pins of the oracle's non-periodic boundary rules (no GPU).

The paper runs its shock-bubble examples with reflecting walls on two faces
and outflow / inflow on the other two (Example 5.8), without the discrete
rules.  The oracle's reading (cell-centred nodes, mirror images across each
face) is pinned here by what it must reproduce exactly:

- a reflecting wall is a mirror plane: the walled problem equals the periodic
  problem on twice the domain with mirror-symmetric data, node by node, for
  the ghost layers, the metrics, the right-hand side and whole moving-mesh
  steps (mesh redistribution included);
- outflow and inflow ghosts are the values a larger domain would hold there:
  with the outermost states continued (outflow) or the inflow state placed
  outside, the right-hand side equals that of the larger periodic domain;
- with walls on every face, mass of each species and total energy are
  conserved over moving-mesh steps, and the mesh stays inside the walls.
"""
import numpy as np
import pytest

import oracle
from paper_2202_07989_amd import inputs as I

REFLECT, OUTFLOW, INFLOW = 1, 2, 3


def walled(dim, nspec, n, bc, **kw):
    """Spec on the unit box [0, 1]^d with the given per-face conditions
    (walls at 0 and 1 of every non-periodic direction)."""
    sp = I.make_spec(dim, nspec, n, **kw)
    sp["bc"] = [list(bc[k]) for k in range(dim)]
    sp["wall"] = [[0.0, 1.0] for _ in range(dim)]
    return sp


def inside_mesh(sp, seed, amp=0.02):
    """Curvilinear mesh whose coordinate k stays inside [0, 1] along every
    non-periodic direction k (its perturbation vanishes at the walls)."""
    rng = np.random.default_rng(seed)
    xi = I.xi_nodes(sp)
    x = []
    for k in range(sp["dim"]):
        f = I._smooth_field(rng, xi)
        if sp["bc"][k][0]:
            f = f * np.sin(np.pi * xi[k])
        x.append(xi[k] + amp * f)
    return x


def state(sp, seed):
    rho, v, p = I.random_state(sp, seed, noise=0.2)
    U = I.conserved(sp, rho, v, p)
    rng = np.random.default_rng(seed + 5)
    J = 1.0 + 0.1 * I._smooth_field(rng, I.xi_nodes(sp))
    return U, J


def unfold(sp, U, J, x, k):
    """Interior data of the walled grid -> interior data of the periodic grid
    twice as long along k: nodes n..2n-1 mirror nodes n-1..0 across the wall
    at 1 (momentum k negated, x_k -> 2 - x_k)."""
    N = sp["nspec"]
    ax = 3 - k                      # array axis of direction k in (C, n2, n1, n0)
    Um = np.flip(U, axis=ax).copy()
    Um[N + k] *= -1.0
    Jm = np.flip(J, axis=ax - 1).copy()
    xm = [np.flip(c, axis=ax - 1).copy() for c in x]
    xm[k] = 2.0 - xm[k]
    U2 = np.concatenate([U, Um], axis=ax)
    J2 = np.concatenate([J, Jm], axis=ax - 1)
    x2 = [np.concatenate([a, b], axis=ax - 1) for a, b in zip(x, xm)]
    return U2, J2, x2


def doubled_spec(sp, dirs):
    n = list(sp["n"][: sp["dim"]])
    for k in dirs:
        n[k] *= 2
    box = [2.0 if k in dirs else 1.0 for k in range(sp["dim"])]
    d2 = I.make_spec(sp["dim"], sp["nspec"], n, box=box, gamma=sp["gamma"], cv=sp["cv"],
                     pinf=sp["pinf"], chi=sp["chi"])
    return d2


def first_block(sp, a):
    """The walled grid's padded extent, cut from a doubled grid's array."""
    ng = sp["ng"]
    np_ = [sp["n"][k] + 2 * ng if k < sp["dim"] else 1 for k in range(3)]
    return a[:, : np_[2], : np_[1], : np_[0]]


def interior_first(sp, d2, a):
    ng = sp["ng"]
    sl = [slice(ng, ng + sp["n"][k]) if k < sp["dim"] else slice(0, 1) for k in range(3)]
    return a[:, sl[2], sl[1], sl[0]]


CASES = [
    (2, 2, (13, 11), [(0, 0), (REFLECT, REFLECT)], [1]),
    (2, 1, (12, 10), [(REFLECT, REFLECT), (REFLECT, REFLECT)], [0, 1]),
    (3, 2, (8, 7, 6), [(0, 0), (REFLECT, REFLECT), (REFLECT, REFLECT)], [1, 2]),
]


def build_pair(dim, nspec, n, bc, dirs, seed=3):
    kw = dict(chi=I.CHI_SHOCK, gamma=(1.4, 1.67)[:nspec], cv=(1.0, 2.5)[:nspec], pinf=(0.0, 0.0)[:nspec])
    sp = walled(dim, nspec, n, bc, **kw)
    U, J, x = state(sp, seed) + (inside_mesh(sp, seed + 1),)
    U2, J2, x2 = U, J, x
    for k in dirs:
        U2, J2, x2 = unfold(sp, U2, J2, x2, k)
    d2 = doubled_spec(sp, dirs)
    a = I.assemble(sp, U, J, x)
    b = I.assemble(d2, U2, J2, x2)
    return sp, d2, a, b


@pytest.mark.parametrize("case", CASES, ids=["2d-wall-y", "2d-walls-xy", "3d-walls-yz"])
def test_reflecting_wall_is_a_mirror_plane(case):
    dim, nspec, n, bc, dirs = case
    sp, d2, (JU, J, x), (JU2, J2, x2) = build_pair(dim, nspec, n, bc, dirs)
    o, o2 = oracle.Oracle(sp), oracle.Oracle(d2)
    o.fill_ghosts_state(JU, J)
    o.fill_ghosts_x(x)
    o2.fill_ghosts(JU2, o2.nc)
    o2.fill_ghosts(J2, 1)
    o2.fill_ghosts_x(x2)
    # ghost layers: the walled grid's padded block is the doubled grid's
    np.testing.assert_array_equal(JU, first_block(sp, JU2))
    np.testing.assert_array_equal(J, first_block(sp, J2))
    np.testing.assert_allclose(x, first_block(sp, x2), rtol=0, atol=4e-16)
    # metrics (ghosts by the mirror rules) and the right-hand side
    disp = 0.01 * np.stack(inside_mesh(sp, 9)) - 0.01 * np.stack(I.xi_nodes(sp))
    dp = I.zeros(sp, dim)
    dp[I.interior(sp)] = disp
    dp2 = I.zeros(d2, dim)
    D2 = disp
    for k in dirs:
        ax = 3 - k
        m = np.flip(D2, axis=ax).copy()
        m[k] *= -1.0
        D2 = np.concatenate([D2, m], axis=ax)
    dp2[I.interior(d2)] = D2
    o.fill_ghosts_kind(dp, dim, 2)
    o2.fill_ghosts(dp2, dim)
    np.testing.assert_array_equal(dp, first_block(sp, dp2))
    jx, jt = o.metrics(x, dp, 0.5, 1e-3)
    jx2, jt2 = o2.metrics(x2, dp2, 0.5, 1e-3)
    np.testing.assert_allclose(jx, first_block(sp, jx2), rtol=0, atol=1e-13)
    np.testing.assert_allclose(jt, first_block(sp, jt2), rtol=0, atol=1e-11)
    rc, dJU, dJ = o.rhs(JU, J, jx, jt)
    rc2, dJU2, dJ2 = o2.rhs(JU2, J2, jx2, jt2)
    assert rc == 0 and rc2 == 0
    Iin = I.interior(sp)
    scale = np.abs(dJU2).max(axis=(1, 2, 3), keepdims=True)
    err = np.abs(dJU[Iin] - interior_first(sp, d2, dJU2)) / scale
    assert err.max() < 1e-12, err.max()
    assert np.abs(dJ[Iin] - interior_first(sp, d2, dJ2)).max() < 1e-12 * np.abs(dJ2).max()


@pytest.mark.parametrize("case", CASES, ids=["2d-wall-y", "2d-walls-xy", "3d-walls-yz"])
def test_reflecting_wall_moving_mesh_steps_match_the_mirrored_problem(case):
    dim, nspec, n, bc, dirs = case
    sp, d2, (JU, J, x), (JU2, J2, x2) = build_pair(dim, nspec, n, bc, dirs, seed=21)
    o, o2 = oracle.Oracle(sp), oracle.Oracle(d2)
    mon = I.monitor_spec(n_sweeps=5, n_smooth=3, sigma=(0,), alpha=(200.0,))
    for _ in range(2):
        rc, dt, dtau = o.step(JU, J, x, mon=mon, cfl=0.4, move_mesh=True)
        rc2, dt2, dtau2 = o2.step(JU2, J2, x2, mon=mon, cfl=0.4, move_mesh=True)
        assert rc == 0 and rc2 == 0
        assert abs(dt - dt2) <= 1e-13 * dt and abs(dtau - dtau2) <= 1e-12
    Iin = I.interior(sp)
    scale = np.abs(JU2).max(axis=(1, 2, 3), keepdims=True)
    assert (np.abs(JU[Iin] - interior_first(sp, d2, JU2)) / scale).max() < 1e-12
    assert np.abs(x[Iin] - interior_first(sp, d2, x2)).max() < 1e-13
    assert np.abs(J[Iin] - interior_first(sp, d2, J2)).max() < 1e-12


def test_outflow_and_inflow_ghosts_are_the_extended_domain():
    """Direction 0: outflow at 0, inflow at 1; direction 1 periodic.  On a
    mesh uniform along 0 the mirrored mesh ghosts are the mesh's own
    continuation, so the right-hand side must equal that of the periodic
    domain ng nodes longer on each side that holds the outermost state
    (outflow side) and the inflow state (inflow side) there."""
    nspec, n0, n1, ng = 2, 14, 9, 3
    kw = dict(chi=I.CHI_SHOCK, gamma=(1.4, 1.67), cv=(1.0, 2.5), pinf=(0.0, 0.0))
    sp = walled(2, nspec, (n0, n1), [(OUTFLOW, INFLOW), (0, 0)], **kw)
    rho, v, p = I.random_state(sp, 31, noise=0.2)
    U = I.conserved(sp, rho, v, p)
    rng = np.random.default_rng(4)
    xi = I.xi_nodes(sp)
    Jrow = 1.0 + 0.1 * np.sin(2 * np.pi * xi[1][:, :1])          # J varies with eta only
    J = np.broadcast_to(Jrow, xi[0].shape).copy()
    x = [xi[0].copy(), xi[1] + 0.02 * np.sin(2 * np.pi * xi[1])]  # uniform along direction 0
    Uin = I.conserved(sp, [np.array(1.3), np.array(0.2)], [np.array(-0.4), np.array(0.1)],
                      np.array(1.7))[:, ...].reshape(-1)
    sp["inflow"] = {(0, 1): list(Uin)}
    JU, Jp, xp = I.assemble(sp, U, J, x)
    o = oracle.Oracle(sp)
    o.fill_ghosts_state(JU, Jp)
    o.fill_ghosts_x(xp)
    # the extended periodic domain: ng outflow copies, the interior, ng inflow states
    h = sp["dxi"][0]
    ext = I.make_spec(2, nspec, (n0 + 2 * ng, n1), box=((n0 + 2 * ng) * h, 1.0), **kw)
    Ue = np.concatenate([np.repeat(U[..., :1], ng, axis=3), U,
                         np.broadcast_to(Uin[:, None, None, None], U.shape[:3] + (ng,))], axis=3)
    Je = np.concatenate([np.repeat(J[..., :1], ng, axis=2), J, np.repeat(J[..., :1], ng, axis=2)], axis=2)
    xie = I.xi_nodes(ext)
    xe = [xie[0] - ng * h, xie[1] + 0.02 * np.sin(2 * np.pi * xie[1])]
    JUe, Jpe, xpe = I.assemble(ext, Ue, Je, xe)
    oe = oracle.Oracle(ext)
    oe.fill_ghosts(JUe, oe.nc)
    oe.fill_ghosts(Jpe, 1)
    oe.fill_ghosts_x(xpe)
    # the walled ghosts are the extended domain's nodes there
    sl = (slice(None), slice(None), slice(ng, ng + n1))
    np.testing.assert_allclose(JU[sl + (slice(0, n0 + 2 * ng),)], JUe[sl + (slice(ng, n0 + 3 * ng),)],
                               rtol=1e-15, atol=0)
    jx, jt = o.metrics(xp)
    jxe, jte = oe.metrics(xpe)
    rc, dJU, dJ = o.rhs(JU, Jp, jx, None)
    rce, dJUe, dJe = oe.rhs(JUe, Jpe, jxe, None)
    assert rc == 0 and rce == 0
    a = dJU[:, 0, ng:ng + n1, ng:ng + n0]
    b = dJUe[:, 0, ng:ng + n1, 2 * ng:2 * ng + n0]
    scale = np.abs(b).max(axis=(1, 2), keepdims=True)
    assert (np.abs(a - b) / scale).max() < 1e-12


def test_walls_everywhere_conserve_mass_and_energy_and_keep_the_mesh_inside():
    """Reflecting walls on all faces: the wall fluxes of mass and energy
    vanish (the mirrored states cancel), so sum_i J_i rho_l,i and
    sum_i J_i E_i stay constant under moving-mesh steps.  Data: the
    tri-point problem on [0, 7] x [0, 3] with its material interfaces spread
    over about one cell."""
    sp = I.spec_tripoint((28, 12))
    JU, J, x = I.init_tripoint(sp)
    o = oracle.Oracle(sp)
    mon = I.monitor_spec(n_sweeps=5, n_smooth=3, sigma=(0,), alpha=(1200.0,))
    Iin = I.interior(sp)
    x0 = x[Iin].copy()
    m0 = JU[Iin].sum(axis=(1, 2, 3))
    for _ in range(4):
        rc, dt, dtau = o.step(JU, J, x, mon=mon, cfl=0.4, move_mesh=True)
        assert rc == 0
    m1 = JU[Iin].sum(axis=(1, 2, 3))
    N = 2
    for c in list(range(N)) + [N + 2]:
        assert abs(m1[c] - m0[c]) <= 1e-13 * abs(m0[c]), (c, m0[c], m1[c])
    assert abs(m1[N] - m0[N]) > 1e-3 * abs(m0[N + 2]) * dt   # the walls push: momentum changes
    xin = x[Iin]
    assert xin[0].min() > 0.0 and xin[0].max() < 7.0
    assert xin[1].min() > 0.0 and xin[1].max() < 3.0
    assert np.abs(xin - x0).max() > 1e-3                      # the mesh did move
