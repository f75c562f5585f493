"""Pins of the oracle's extra monitor variables (no GPU): the speed |v| and
the schlieren function Phi = exp(-Psi |grad rho| / max |grad rho|) of eq
schlieren, which the multi-variable monitor of Example 5.9 combines with
rho_1, rho_2 and p.  The pins check what the definitions fix without
retyping them: ranges, where Phi is 1 and where it is smallest, invariance
under scaling the density, which species weight applies where, and that a
channel proportional to another merges with it."""
import numpy as np
import pytest

import oracle
from paper_2202_07989_amd import inputs as I


def two_species(seed, n=(24, 20), const_rho=False):
    sp = I.make_spec(2, 2, n, gamma=(1.4, 1.67), cv=(1.0, 2.5), pinf=(0.0, 0.0), chi=I.CHI_SHOCK)
    rho, v, p = I.random_state(sp, seed)
    if const_rho:                       # composition varies, total density does not
        r1 = np.round(64.0 * (0.2 + 0.8 * (rho[0] - 0.5) / 1.5)) / 64.0   # multiples of 1/64: sums exact
        rho = [r1, 1.25 - r1]
    JU, J, x = I.assemble(sp, I.conserved(sp, rho, v, p), np.ones_like(p), I.xi_nodes(sp))
    o = oracle.Oracle(sp)
    o.fill_ghosts(JU, o.nc)
    o.fill_ghosts(J, 1)
    return sp, o, JU, J


def grad_rho(sp, JU):
    """|grad_xi rho| at the interior (periodic central differences)."""
    Iin = I.interior(sp)
    rho = (JU[0] + JU[1])[Iin[1:]]
    g2 = 0.0
    for k in range(2):
        ax = 2 - k
        d = (np.roll(rho, -1, axis=ax) - np.roll(rho, 1, axis=ax)) / (2 * sp["dxi"][k])
        g2 = g2 + d * d
    return np.sqrt(g2)


def test_phi_range_extremes_and_species_weights():
    sp, o, JU, J = two_species(5)
    psi = (30.0, 150.0)
    phi = o.schlieren(dict(psi=list(psi)), JU, J)[0][I.interior(sp)[1:]]
    Iin = I.interior(sp)
    r1, r2 = JU[0][Iin[1:]], JU[1][Iin[1:]]
    Psi = (psi[0] * r1 + psi[1] * r2) / (r1 + r2)
    assert np.all(phi <= 1.0) and np.all(phi >= np.exp(-Psi) * (1 - 1e-14))
    g = grad_rho(sp, JU)
    k = np.unravel_index(np.argmax(g), g.shape)
    assert phi[k] == pytest.approx(np.exp(-Psi[k]), rel=1e-13)     # the steepest node
    # Phi decreases with |grad rho| where Psi is the same: order is preserved
    psi_same = o.schlieren(dict(psi=[40.0, 40.0]), JU, J)[0][I.interior(sp)[1:]]
    order_g = np.argsort(g.ravel())
    assert np.all(np.diff(psi_same.ravel()[order_g]) <= 1e-15)


def test_phi_sees_total_density_and_is_scale_free():
    sp, o, JU, J = two_species(6, const_rho=True)
    phi = o.schlieren(dict(psi=[30.0, 150.0]), JU, J)
    np.testing.assert_array_equal(phi[I.interior(sp)], 1.0)           # grad rho = 0 everywhere
    sp, o, JU, J = two_species(7)
    a = o.schlieren(dict(psi=[30.0, 150.0]), JU, J)
    JU2 = JU.copy()
    JU2[:2] *= 3.0                                                     # rho_l -> 3 rho_l
    b = o.schlieren(dict(psi=[30.0, 150.0]), JU2, J)
    np.testing.assert_allclose(b, a, rtol=1e-12, atol=0)   # exp of an argument up to ~35


def test_pure_species_regions_take_their_own_weight():
    """Where rho_2 = 0 the weight is psi_1, where rho_1 = 0 it is psi_2."""
    sp = I.make_spec(2, 2, (30, 8), gamma=(1.4, 1.67), cv=(1.0, 2.5), pinf=(0.0, 0.0), chi=I.CHI_SHOCK)
    xi = I.xi_nodes(sp)
    left = xi[0] < 0.5
    rho_tot = 1.0 + 0.3 * np.sin(2 * np.pi * xi[0])                    # same gradient pattern in both halves
    r1 = np.where(left, rho_tot, 0.0)
    r2 = np.where(left, 0.0, rho_tot)
    z = np.zeros_like(r1)
    JU, J, x = I.assemble(sp, I.conserved(sp, [r1, r2], [z, z], 1.0 + z), np.ones_like(r1), xi)
    o = oracle.Oracle(sp)
    o.fill_ghosts(JU, o.nc)
    o.fill_ghosts(J, 1)
    phi = o.schlieren(dict(psi=[10.0, 50.0]), JU, J)[0][I.interior(sp)[1:]]
    g = grad_rho(sp, JU)
    G = g.max()
    i_l, i_r = 4, 19                     # interior of each half, away from the species switch
    for i, ps in ((i_l, 10.0), (i_r, 50.0)):
        col = phi[0, :, i]
        np.testing.assert_allclose(-np.log(col), ps * g[0, :, i] / G, rtol=1e-12)


def test_phi_channel_vanishes_without_weights_and_speed_merges_with_rho():
    sp, o, JU, J = two_species(8)
    base = dict(sigma=[0], alpha=[50.0], n_smooth=2, n_sweeps=1)
    rc, th0 = o.monitor_fn(base, JU, J)
    rc2, th1 = o.monitor_fn(dict(base, sigma=[0, 5], alpha=[50.0, 700.0], psi=[0.0, 0.0]), JU, J)
    assert rc == 0 and rc2 == 0
    np.testing.assert_array_equal(th1, th0)                            # Phi = 1: the term is dropped
    # |v| = c rho: the speed channel's normalised gradient equals rho's
    rng = np.random.default_rng(9)
    Iin = I.interior(sp)
    rho = (JU[0] + JU[1])[Iin[1:]] / J[Iin][0]
    theta = 2 * np.pi * I._smooth_field(rng, I.xi_nodes(sp))
    U = JU[Iin] / J[Iin][0]
    U[2] = rho * 0.3 * rho * np.cos(theta)
    U[3] = rho * 0.3 * rho * np.sin(theta)
    JU2 = JU.copy()
    JU2[Iin] = U * J[Iin][0]
    o.fill_ghosts(JU2, o.nc)
    _, a = o.monitor_fn(dict(base, sigma=[0, 4], alpha=[50.0, 30.0]), JU2, J)
    _, b = o.monitor_fn(dict(base, sigma=[0], alpha=[80.0]), JU2, J)
    np.testing.assert_allclose(a, b, rtol=1e-12)
