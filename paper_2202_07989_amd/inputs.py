"""Seeded synthetic inputs shaped like the paper's workloads.

This module is shared by the tests of the CPU oracle and by the GPU path.  It
holds no step of the scheme: it only lays out padded structure-of-arrays
buffers and writes initial data.  Initial data given in primitive variables
(rho_l, v, p) are turned into conserved variables with the stiffened-gas
equation of state of the problem statement (Section 1, eq StiffenedEOS):
T = (p + sum p_inf,l) / sum rho_l R_l and E = sum (c_vl rho_l T + p_inf,l)
+ rho |v|^2 / 2.

Layout: a field with C components is a float64 array of shape
(C, np2, np1, np0), np_k = n_k + 2 ng for the active directions (np2 = 1 in
2D), i.e. component c starts at c * P and i is fastest.  Ghost layers are left
at zero; filling them is a step of the scheme.
"""
from __future__ import annotations

import math

import numpy as np

CHI_DEFAULT = (1.0 / 111.0, 10.0 / 111.0, 100.0 / 111.0)   # Appendix A default
CHI_SHOCK = (0.95, 0.045, 0.005)                            # Ex. 5.3 / 5.10 weights
WATER_AIR = dict(gamma=(4.4, 1.4), cv=(1.0, 1.0), pinf=(6.0e8, 0.0))
# zero tolerances of the sign matrix, relative to the bound on the terms that
# form a jump of the scaled entropy variables: FP64 arithmetic, and the FP32
# arithmetic of the mixed-precision form (0 is the paper's rule as printed)
SIGN_TOL_FP64 = 1.0e-12
SIGN_TOL_FP32 = 1.0e-6


# --------------------------------------------------------------------------
# workload specs
# --------------------------------------------------------------------------
BC_PERIODIC, BC_REFLECT, BC_OUTFLOW, BC_INFLOW = 0, 1, 2, 3


def make_spec(dim, nspec, n, *, box=None, gamma=(1.4,), cv=(1.0,), pinf=(0.0,),
              chi=CHI_DEFAULT, w=3, ng=3, dissipation=1, weno_eps=1e-10, reconstruction=0,
              bc=None, wall=None, inflow=None, sign_tol=SIGN_TOL_FP64, sign_tol32=SIGN_TOL_FP32):
    """Workload spec.  Periodic in every direction unless bc gives per-face
    conditions [(low, high), ...] (BC_*); wall then holds the physical
    coordinates [(x_low, x_high), ...] of the faces (the computational box is
    [0, x_high - x_low]) and inflow maps (direction, side) to the conserved
    state U prescribed on an inflow face.  sign_tol / sign_tol32 are the
    zero tolerances of the sign matrix in FP64 and in the FP32 arithmetic of
    the mixed-precision form."""
    n = tuple(n) + (1,) * (3 - len(n))
    box = box or (1.0,) * dim
    box = tuple(box) + (1.0,) * (3 - len(box))
    dxi = tuple(box[k] / n[k] if k < dim else 1.0 for k in range(3))
    sp = dict(dim=dim, nspec=nspec, n=n, ng=ng, dxi=dxi, len=box, w=w,
              gamma=tuple(gamma), cv=tuple(cv), pinf=tuple(pinf), chi=tuple(chi),
              weno_eps=weno_eps, dissipation=dissipation, reconstruction=reconstruction,
              sign_tol=sign_tol, sign_tol32=sign_tol32)
    if bc is not None:
        sp["bc"] = [tuple(b) for b in bc]
        sp["wall"] = [tuple(wl) for wl in (wall or [(0.0, box[k]) for k in range(dim)])]
        sp["inflow"] = dict(inflow or {})
    return sp


def spec_c1(n=64):
    """2D single-species ideal gas (Gamma 1.4), periodic curvilinear mesh."""
    return make_spec(2, 1, (n, n), gamma=(1.4,), cv=(1.0,), pinf=(0.0,), chi=CHI_DEFAULT)


def spec_c2(n=512):
    """2D two-species stiffened gas (water Gamma 4.4, p_inf 6e8; air 1.4)."""
    return make_spec(2, 2, (n, n), chi=CHI_SHOCK, **WATER_AIR)


def spec_c3(n=256):
    """3D two-species stiffened gas, same materials as spec_c2."""
    return make_spec(3, 2, (n, n, n), chi=CHI_SHOCK, **WATER_AIR)


def monitor_spec(n_sweeps=10, n_smooth=3, sigma=(0,), alpha=(1200.0,)):
    return dict(sigma=list(sigma), alpha=list(alpha), n_smooth=n_smooth, n_sweeps=n_sweeps)


MON_RHO, MON_RHO1, MON_RHO2, MON_P, MON_SPEED, MON_SCHLIEREN = 0, 1, 2, 3, 4, 5


def monitor_m7(n_sweeps=10, n_smooth=3):
    """Example 5.9's monitor: (Phi, u, rho_1, rho_2, p) with alpha (600, 500,
    1200, 1200, 1200) and the schlieren weights Psi = (120 rho_1 + 20 rho_2)
    / rho."""
    return dict(sigma=[MON_SCHLIEREN, MON_SPEED, MON_RHO1, MON_RHO2, MON_P],
                alpha=[600.0, 500.0, 1200.0, 1200.0, 1200.0], psi=[120.0, 20.0],
                n_smooth=n_smooth, n_sweeps=n_sweeps)


# --------------------------------------------------------------------------
# layout helpers
# --------------------------------------------------------------------------
def padded_dims(spec):
    ng = spec["ng"]
    return tuple(spec["n"][k] + 2 * ng if k < spec["dim"] else 1 for k in range(3))


def npoints(spec):
    a, b, c = padded_dims(spec)
    return a * b * c


def ncomp(spec):
    return spec["nspec"] + spec["dim"] + 1


def zeros(spec, ncomp_):
    np0, np1, np2 = padded_dims(spec)
    return np.zeros((ncomp_, np2, np1, np0), dtype=np.float64)


def interior(spec):
    """Index tuple selecting the interior of a (C, np2, np1, np0) array."""
    ng, d = spec["ng"], spec["dim"]
    sl = [slice(ng, ng + spec["n"][k]) if k < d else slice(0, 1) for k in range(3)]
    return (slice(None), sl[2], sl[1], sl[0])


def xi_nodes(spec):
    """Cell-centred computational coordinates of the interior nodes,
    returned as a list of d arrays shaped (n2, n1, n0)."""
    d = spec["dim"]
    ax = [(np.arange(spec["n"][k]) + 0.5) * spec["dxi"][k] if k < d else np.zeros(1)
          for k in range(3)]
    g2, g1, g0 = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return [g0, g1, g2][:d]


def conserved(spec, rho, v, p):
    """Stiffened-gas EOS: (rho_l list, v list, p) -> U (C, n2, n1, n0)."""
    N, d = spec["nspec"], spec["dim"]
    cv, gam, pinf = spec["cv"], spec["gamma"], spec["pinf"]
    rR = sum(rho[l] * cv[l] * (gam[l] - 1.0) for l in range(N))
    pinf_t = sum(pinf[l] for l in range(N))
    T = (p + pinf_t) / rR
    rhot = sum(rho[l] for l in range(N))
    kin = 0.5 * rhot * sum(v[m] * v[m] for m in range(d))
    E = sum(cv[l] * rho[l] * T + pinf[l] for l in range(N)) + kin
    comps = [rho[l] for l in range(N)] + [rhot * v[m] for m in range(d)] + [E]
    return np.stack([np.broadcast_to(c, rho[0].shape) for c in comps])


def assemble(spec, U, J, x):
    """Place interior U (C,...), J (...) and x (d,...) into padded buffers
    and return (JU, J, x) with JU = J * U."""
    I = interior(spec)
    nc = ncomp(spec)
    JUp = zeros(spec, nc)
    Jp = zeros(spec, 1)
    xp = zeros(spec, spec["dim"])
    JUp[I] = J[None] * U
    Jp[I] = J[None]
    xp[I] = np.stack(x)
    return JUp, Jp, xp


# --------------------------------------------------------------------------
# C1: smooth advection on the periodic curvilinear mesh
#   x = xi + 0.1 sin(2 pi xi) sin(2 pi eta), y = eta + (same),
#   J = 1 + 0.2 pi sin(2 pi (xi + eta)); rho = 1 + 0.2 sin(2 pi (x + y)),
#   v = (1, 1), p = 1.  Exact: rho(x, y, t) = 1 + 0.2 sin(2 pi (x + y - 2 t)).
# --------------------------------------------------------------------------
def c1_mesh(spec, amp=0.1):
    xi, eta = xi_nodes(spec)
    pert = amp * np.sin(2 * np.pi * xi) * np.sin(2 * np.pi * eta)
    x, y = xi + pert, eta + pert
    J = (1 + 2 * np.pi * amp * np.cos(2 * np.pi * xi) * np.sin(2 * np.pi * eta)) * \
        (1 + 2 * np.pi * amp * np.sin(2 * np.pi * xi) * np.cos(2 * np.pi * eta)) - \
        (2 * np.pi * amp) ** 2 * np.sin(2 * np.pi * xi) * np.cos(2 * np.pi * eta) * \
        np.cos(2 * np.pi * xi) * np.sin(2 * np.pi * eta)
    return [x, y], J


def c1_exact_rho(x, y, t):
    return 1.0 + 0.2 * np.sin(2 * np.pi * (x + y - 2.0 * t))


def init_c1(spec, amp=0.1):
    (x, y), J = c1_mesh(spec, amp)
    rho = c1_exact_rho(x, y, 0.0)
    one = np.ones_like(rho)
    U = conserved(spec, [rho], [one, one], one)
    return assemble(spec, U, J, [x, y])


# --------------------------------------------------------------------------
# isentropic vortex (Section 5, Examples 5.1 and 5.5): a smooth isentropic
# vortex of strength eps = 5 carried by a uniform flow on the periodic box
# [-10, 10]^d, one ideal-gas species (Gamma 1.4, c_v 1, p_inf 0).  2D: centre
# (-2, -2) at t = 0, mean flow (1, 1).  3D: the cylindrical vortex turned
# onto the diagonal through the maps xhat = (-x1 + x2, x1 - x3) (wrapped to
# [-10, 10)^2) and xtilde = (xhat1 + 2 xhat2, sqrt(3) xhat1)/sqrt(6), with the
# velocity map of Example 5.5.  T = 1 - eps^2/(8 Gamma pi^2) e^(1 - r^2),
# rho = T^(1/(Gamma-1)), p = (Gamma - 1) rho T.  The exact solution is the
# initial field translated by the mean velocity.  The mesh starts uniform,
# x = xi - 10.
# --------------------------------------------------------------------------
VORTEX_EPS = 5.0


def spec_vortex(dim, n):
    return make_spec(dim, 1, (n,) * dim, box=(20.0,) * dim, gamma=(1.4,), cv=(1.0,), pinf=(0.0,))


def vortex_mean_velocity(dim):
    if dim == 2:
        return (1.0, 1.0)
    s2, s3, s6 = math.sqrt(2.0), math.sqrt(3.0), math.sqrt(6.0)
    return ((1.0 - s3 + s2) / s6, (1.0 + s3 + s2) / s6, (-2.0 + s2) / s6)


def _wrap20(a):
    return (a + 10.0) % 20.0 - 10.0


def vortex_prims(dim, x, t=0.0, eps=VORTEX_EPS, gamma=1.4):
    """rho, [v_1..v_d], p of the exact solution at physical points x (list
    of d arrays) and time t."""
    vm = vortex_mean_velocity(dim)
    y = [x[k] - vm[k] * t for k in range(dim)]
    if dim == 2:
        a, b = _wrap20(y[0] + 2.0), _wrap20(y[1] + 2.0)
        r2 = a * a + b * b
        f = eps / (2.0 * math.pi) * np.exp(0.5 * (1.0 - r2))
        v = [1.0 + f * b, 1.0 - f * a]
    else:
        s2, s3, s6 = math.sqrt(2.0), math.sqrt(3.0), math.sqrt(6.0)
        h1, h2 = _wrap20(-y[0] + y[1]), _wrap20(y[0] - y[2])
        t1, t2 = (h1 + 2.0 * h2) / s6, s3 * h1 / s6
        r2 = t1 * t1 + t2 * t2
        f = eps / (2.0 * math.pi) * np.exp(0.5 * (1.0 - r2))
        w1, w2 = 1.0 + f * t2, 1.0 - f * t1
        v = [(w1 - s3 * w2 + s2) / s6, (w1 + s3 * w2 + s2) / s6, (-2.0 * w1 + s2) / s6]
    T = 1.0 - eps ** 2 / (8.0 * gamma * math.pi ** 2) * np.exp(1.0 - r2)
    rho = T ** (1.0 / (gamma - 1.0))
    return rho, v, (gamma - 1.0) * rho * T


def init_vortex(spec):
    d = spec["dim"]
    x = [xi - 10.0 for xi in xi_nodes(spec)]
    rho, v, p = vortex_prims(d, x, 0.0)
    U = conserved(spec, [rho], v, p)
    return assemble(spec, U, np.ones_like(rho), x)


def vortex_monitor(n_sweeps=10, n_smooth=10):
    """The monitor of the vortex examples: Theta = (1 + 20 |grad rho_1| / max
    + 10 |lap rho_1| / max)^(1/2), filtered 10 times (the upper end of the
    3-10 passes of Remark 4.1: the Laplacian term lets grid-scale content of
    the solution into the mesh, and with 3 passes the moving-mesh error stops
    converging past 160^2)."""
    return dict(sigma=[1], alpha=[20.0], beta=[10.0], form=1, n_smooth=n_smooth, n_sweeps=n_sweeps)


# --------------------------------------------------------------------------
# shock-bubble data (C2, C3): water with a trace of air, an air bubble with a
# trace of water, and a planar Mach-M_s shock in the water.
# Post-shock state: stiffened-gas normal-shock relations for a shock moving
# into the pre-shock state at rest (ideal-gas relations with p -> p + p_inf):
#   rho1/rho0 = (G+1) M^2 / ((G-1) M^2 + 2),
#   p1 + pinf = (p0 + pinf)(2 G M^2 - G + 1)/(G + 1),
#   u1 = M c0 (1 - rho0/rho1), c0^2 = G (p0 + pinf)/rho0,
# with the mixture Gamma and p_inf of the pre-shock water; mass fractions kept.
# --------------------------------------------------------------------------
def _post_shock(spec, rho0, p0, mach):
    cv, gam, pinf = spec["cv"], spec["gamma"], spec["pinf"]
    N = spec["nspec"]
    G = sum(gam[l] * cv[l] * rho0[l] for l in range(N)) / sum(cv[l] * rho0[l] for l in range(N))
    pi = sum(pinf[:N])
    r0 = sum(rho0)
    ratio = (G + 1) * mach ** 2 / ((G - 1) * mach ** 2 + 2)
    p1 = (p0 + pi) * (2 * G * mach ** 2 - G + 1) / (G + 1) - pi
    c0 = math.sqrt(G * (p0 + pi) / r0)
    u1 = mach * c0 * (1 - 1 / ratio)
    return [r * ratio for r in rho0], p1, u1


def _bubble_radius_3d(n_hat, seed=2202079, modes=10, amp=0.02, r0=0.2):
    rng = np.random.default_rng(seed)
    e = rng.normal(size=(modes, 3))
    e /= np.linalg.norm(e, axis=1, keepdims=True)
    l = rng.integers(2, 9, size=modes)
    psi = rng.uniform(0, 2 * np.pi, size=modes)
    a = rng.uniform(-1, 1, size=modes)
    a /= np.abs(a).sum()
    r = np.ones(n_hat.shape[1:])
    for m in range(modes):
        cosang = np.clip(np.tensordot(e[m], n_hat, axes=(0, 0)), -1.0, 1.0)
        r += amp * a[m] * np.cos(l[m] * np.arccos(cosang) + psi[m])
    return r0 * r


def init_shock_bubble(spec, mach=1.5, shock_x=0.2, trace=1e-3, p0=1.0e5,
                      rho_water=1000.0, rho_air=1.0, seed=2202079, width=2.0):
    """Water/air shock-bubble data.  width > 0 spreads the bubble interface
    and the shock over a tanh profile of that many cells (a smoothed
    initial condition; the scheme has no positivity limiter)."""
    d = spec["dim"]
    xi = xi_nodes(spec)
    x = [c.copy() for c in xi]                                   # initial mesh x = xi
    J = np.ones_like(xi[0])
    water = [rho_water - trace, trace]
    air = [trace, rho_air - trace]
    centre = [0.5] * d
    rel = np.stack([x[k] - centre[k] for k in range(d)])
    rad = np.sqrt((rel ** 2).sum(axis=0))
    if d == 3:
        n_hat = rel / np.maximum(rad, 1e-300)
        rb = _bubble_radius_3d(n_hat, seed=seed)
    else:
        rb = 0.2
    h = min(spec["dxi"][:d])
    if width > 0:
        fb = 0.5 * (1.0 - np.tanh((rad - rb) / (width * h)))           # 1 inside the bubble
        fs = 0.5 * (1.0 - np.tanh((x[0] - shock_x) / (width * h)))     # 1 behind the shock
    else:
        fb = (rad < rb).astype(float)
        fs = (x[0] < shock_x).astype(float)
    rho_s, p1, u1 = _post_shock(spec, water, p0, mach)
    rho = [fb * air[l] + (1 - fb) * (fs * rho_s[l] + (1 - fs) * water[l]) for l in range(2)]
    p = fb * p0 + (1 - fb) * (fs * p1 + (1 - fs) * p0)
    v = [(1 - fb) * fs * u1] + [np.zeros_like(p) for _ in range(d - 1)]
    U = conserved(spec, rho, v, p)
    return assemble(spec, U, J, x)


# --------------------------------------------------------------------------
# the paper's two-species examples on walled domains (Examples 5.7 - 5.9).
# Initial mesh uniform, x = wall_low + xi, J = 1.  Region boundaries are
# spread over a tanh profile `width` cells wide: the scheme has no positivity
# limiter, and with the examples' sharp data (partial densities down to
# 1e-5 next to 1) a partial density turns negative in the first step.
# --------------------------------------------------------------------------
def _walled_mesh(spec):
    xi = xi_nodes(spec)
    return [xi[k] + spec["wall"][k][0] for k in range(spec["dim"])]


def _step(phi, h, width):
    """Smoothed indicator of phi > 0 (phi a signed distance)."""
    return 0.5 * (1.0 + np.tanh(phi / (width * h))) if width > 0 else (phi > 0).astype(float)


def _prims_at(spec, states, weights):
    """Blend primitive states (rho_1, rho_2, v_1 .. v_d, p) with weights."""
    N, d = spec["nspec"], spec["dim"]
    rho = [sum(w * st[l] for st, w in zip(states, weights)) for l in range(N)]
    v = [sum(w * st[N + j] for st, w in zip(states, weights)) for j in range(d)]
    p = sum(w * st[N + d] for st, w in zip(states, weights))
    return rho, v, p


def spec_tripoint(n=(350, 150)):
    """Example 5.7: [0, 7] x [0, 3], Gamma (1.5, 1.4), c_v 1, p_inf 0;
    reflecting walls on all four faces (the paper does not name them)."""
    return make_spec(2, 2, n, box=(7.0, 3.0), gamma=(1.5, 1.4), cv=(1.0, 1.0), pinf=(0.0, 0.0),
                     chi=CHI_SHOCK, bc=[(BC_REFLECT, BC_REFLECT)] * 2, wall=[(0.0, 7.0), (0.0, 3.0)])


def init_tripoint(spec, eps=1e-5, width=1.0):
    """Three states: Omega_1 = [0,1]x[0,3] (1-eps, eps, 0, 0, 1), Omega_2 =
    [1,7]x[1.5,3] (0.125-eps, eps, 0, 0, 0.1), Omega_3 = [1,7]x[0,1.5]
    (eps, 1-eps, 0, 0, 0.1)."""
    x = _walled_mesh(spec)
    h = min(spec["dxi"][:2])
    fl = _step(1.0 - x[0], h, width)
    ft = _step(x[1] - 1.5, h, width)
    z = np.zeros_like(x[0])
    s1 = (1.0 - eps, eps, z, z, 1.0)
    s2 = (0.125 - eps, eps, z, z, 0.1)
    s3 = (eps, 1.0 - eps, z, z, 0.1)
    rho, v, p = _prims_at(spec, [s1, s2, s3], [fl, (1 - fl) * ft, (1 - fl) * (1 - ft)])
    return assemble(spec, conserved(spec, rho, v, p), np.ones_like(x[0]), x)


# Examples 5.8 / 5.10 (air / helium, ideal gases) and 5.9 / 5.11 (stiffened
# gas around an ideal-gas bubble), 2D or 3D: domain [0, 445] x [-44.5, 44.5]
# (x [-44.5, 44.5] in 3D), reflecting walls on the lateral faces, outflow on
# the left, inflow of the post-shock state on the right; a bubble of radius
# 25 at (225, 0, 0); the shock at x_1 = 275 moving left.
SB_CASES = {
    "he": dict(gamma=(1.4, 1.647), Rg=(0.287, 1.578), pinf=(0.0, 0.0), eps=0.03,
               bubble=lambda e, R: (e, 1.225 * (R[0] / R[1]) - e, 101325.0),
               pre=lambda e: (1.225 - e, e, 101325.0),
               post=lambda e: (1.6861 - e, e, -113.5243, 159060.0)),
    "stiff": dict(gamma=(3.0, 1.4), cv=(1.0, 1.0), pinf=(100.0, 0.0), eps=0.05,
                  bubble=lambda e, R: (e, 5.0 - e, 100.0),
                  pre=lambda e: (1.0 - e, e, 100.0),
                  post=lambda e: (1.980198 - e, e, -121.2497, 29800.0)),
}


def spec_shock_bubble_walled(case="he", n=(800, 160)):
    """Examples 5.8 / 5.9 (n of length 2) or 5.10 / 5.11 (length 3)."""
    c = SB_CASES[case]
    d = len(n)
    if "Rg" in c:
        cv = tuple(R / (g - 1.0) for R, g in zip(c["Rg"], c["gamma"]))     # R_l = c_v,l (Gamma_l - 1)
    else:
        cv = c["cv"]
    sp = make_spec(d, 2, n, box=(445.0,) + (89.0,) * (d - 1), gamma=c["gamma"], cv=cv, pinf=c["pinf"],
                   chi=CHI_SHOCK, bc=[(BC_OUTFLOW, BC_INFLOW)] + [(BC_REFLECT, BC_REFLECT)] * (d - 1),
                   wall=[(0.0, 445.0)] + [(-44.5, 44.5)] * (d - 1))
    post = c["post"](c["eps"])
    v = [np.array(post[2])] + [np.array(0.0)] * (d - 1)
    Uin = conserved(sp, [np.array(post[0]), np.array(post[1])], v, np.array(post[3])).reshape(-1)
    sp["inflow"] = {(0, 1): [float(u) for u in Uin]}
    sp["example"] = case
    return sp


def init_shock_bubble_walled(spec, width=1.0):
    c = SB_CASES[spec["example"]]
    e = c["eps"]
    R = c.get("Rg", (1.0, 1.0))
    d = spec["dim"]
    x = _walled_mesh(spec)
    h = min(spec["dxi"][:d])
    r = np.sqrt((x[0] - 225.0) ** 2 + sum(x[k] ** 2 for k in range(1, d)))
    fb = _step(25.0 - r, h, width)
    fs = _step(x[0] - 275.0, h, width)
    z = np.zeros_like(x[0])
    b, a, q = c["bubble"](e, R), c["pre"](e), c["post"](e)
    states = [(b[0], b[1]) + (z,) * d + (b[2],), (a[0], a[1]) + (z,) * d + (a[2],),
              (q[0], q[1], q[2] + z) + (z,) * (d - 1) + (q[3],)]
    rho, v, p = _prims_at(spec, states, [fb * (1 - fs), (1 - fb) * (1 - fs), fs])
    return assemble(spec, conserved(spec, rho, v, p), np.ones_like(x[0]), x)


# --------------------------------------------------------------------------
# random smooth periodic data (tests): a few Fourier modes per field
# --------------------------------------------------------------------------
def _smooth_field(rng, xi, modes=3):
    f = np.zeros_like(xi[0])
    for _ in range(modes):
        kv = rng.integers(-2, 3, size=len(xi))
        ph = rng.uniform(0, 2 * np.pi)
        a = rng.uniform(-1, 1)
        f += a * np.sin(2 * np.pi * sum(int(kv[k]) * xi[k] for k in range(len(xi))) + ph)
    return f / modes


def random_mesh(spec, seed, amp=0.03):
    """x = xi + smooth periodic perturbation (a valid, untangled mesh)."""
    rng = np.random.default_rng(seed)
    xi = xi_nodes(spec)
    return [xi[k] + amp * spec["len"][k] * _smooth_field(rng, xi) for k in range(spec["dim"])]


def random_state(spec, seed, noise=0.0, rho_range=(0.5, 2.0), p_range=(0.5, 2.0), vmax=0.5):
    """Smooth random primitive fields, optionally with white noise (tests
    nonlinear WENO weights everywhere)."""
    rng = np.random.default_rng(seed)
    xi = xi_nodes(spec)
    N, d = spec["nspec"], spec["dim"]

    def fld(lo, hi):
        f = 0.5 + 0.5 * _smooth_field(rng, xi)
        if noise:
            f = np.clip(f + noise * rng.uniform(-1, 1, size=f.shape), 0.0, 1.0)
        return lo + (hi - lo) * f

    rho = [fld(*rho_range) for _ in range(N)]
    p = fld(*p_range)
    v = [fld(-vmax, vmax) for _ in range(d)]
    return rho, v, p


def init_random(spec, seed, noise=0.0, mesh_amp=0.03, **kw):
    from_mesh = random_mesh(spec, seed + 1, amp=mesh_amp)
    rho, v, p = random_state(spec, seed, noise=noise, **kw)
    U = conserved(spec, rho, v, p)
    rng = np.random.default_rng(seed + 2)
    J = 1.0 + 0.2 * _smooth_field(rng, xi_nodes(spec))
    return assemble(spec, U, J, from_mesh)


# --------------------------------------------------------------------------
# batched form: many 2D two-species instances of uneven size
# --------------------------------------------------------------------------
def c5_sizes(count=64, seed=2202):
    """Square instance sizes N_b = floor(128 * 8**u_b), u_b ~ U[0, 1) (so
    log-uniform between 128 and 1024), drawn in instance order."""
    rng = np.random.default_rng(seed)
    return [int(math.floor(128.0 * 8.0 ** u)) for u in rng.uniform(0.0, 1.0, size=count)]


def spec_c5(n):
    """One instance of the batch: n x n on the unit box, water/air."""
    return make_spec(2, 2, (n, n), chi=CHI_SHOCK, **WATER_AIR)


def c5_quadrants(rng):
    """Primitive states of the four quadrants of one instance: rho ~ U[0.5, 2],
    Y_1 ~ U[0.05, 0.95], p log-uniform in [1e5, 1e9], v in a uniformly drawn
    direction with |v| ~ U[0, 1]; quadrant order (x<1/2,y<1/2), (x>=1/2,
    y<1/2), (x<1/2, y>=1/2), (x>=1/2, y>=1/2)."""
    q = []
    for _ in range(4):
        rho = rng.uniform(0.5, 2.0)
        y1 = rng.uniform(0.05, 0.95)
        p = 10.0 ** rng.uniform(5.0, 9.0)
        th = rng.uniform(0.0, 2.0 * math.pi)
        s = rng.uniform(0.0, 1.0)
        q.append(dict(rho=(rho * y1, rho * (1.0 - y1)), v=(s * math.cos(th), s * math.sin(th)), p=p))
    return q


def init_riemann4(spec, rng, width=2.0):
    """Four-quadrant Riemann data split at (1/2, 1/2) of the unit box on a
    fixed uniform mesh (x = xi).  The quadrant states are blended across
    tanh layers `width` cells wide: the periodic box has the two splits at
    1/2 and the seam at 0/1, all smoothed the same way (the sharp data trips
    the positivity of the partial densities, as for the shock-bubble)."""
    q = c5_quadrants(rng)
    x, y = xi_nodes(spec)
    h = spec["dxi"][0]

    def step(s):                       # 0 left of 1/2, 1 right of it; periodic seam at 0/1
        return 0.5 * (np.tanh((s - 0.5) / (width * h)) - np.tanh((s - 1.0) / (width * h))
                      - np.tanh(s / (width * h)) + 1.0)

    sx, sy = np.clip(step(x), 0.0, 1.0), np.clip(step(y), 0.0, 1.0)
    w = [(1 - sx) * (1 - sy), sx * (1 - sy), (1 - sx) * sy, sx * sy]
    rho = [sum(w[k] * q[k]["rho"][l] for k in range(4)) for l in range(2)]
    v = [sum(w[k] * q[k]["v"][m] for k in range(4)) for m in range(2)]
    # log-blend the pressure (it spans four decades)
    p = np.exp(sum(w[k] * math.log(q[k]["p"]) for k in range(4)))
    U = conserved(spec, rho, v, p)
    J = np.ones_like(x)
    return assemble(spec, U, J, [x, y])


def init_c5(count=64, seed=2202, sizes=None):
    """Specs and initial (JU, J, x) of every instance of the batch; instance
    b draws its data from default_rng([seed, b])."""
    sizes = sizes if sizes is not None else c5_sizes(count, seed)
    out = []
    for b, n in enumerate(sizes):
        sp = spec_c5(n)
        out.append((sp,) + init_riemann4(sp, np.random.default_rng([seed, b])))
    return out
