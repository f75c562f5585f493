"""Seeded parity cases shared by the GPU tests (inputs + oracle metrics)."""
import numpy as np

import oracle
from paper_2202_07989_amd import inputs as I
from gpu_util import ghosts, moving_metrics

WATER = dict(gamma=(4.4, 1.4), cv=(1.0, 1.0), pinf=(6e8, 0.0))


def case_spec(name, dissipation=1):
    if name == "2d-n1":
        sp = I.make_spec(2, 1, (37, 29), gamma=(1.4,), cv=(1.0,), pinf=(0.0,))
        init = lambda s: I.init_random(s, seed=11, noise=0.3)
    elif name == "2d-n1-stiff":
        sp = I.make_spec(2, 1, (33, 18), gamma=(3.0,), cv=(1.0,), pinf=(100.0,), chi=I.CHI_SHOCK)
        init = lambda s: I.init_random(s, seed=12, noise=0.5, p_range=(50.0, 200.0))
    elif name == "2d-n2-bubble":
        sp = I.make_spec(2, 2, (35, 33), chi=I.CHI_SHOCK, **WATER)
        init = lambda s: I.init_shock_bubble(s)
    elif name == "3d-n1":
        sp = I.make_spec(3, 1, (19, 18, 17), gamma=(1.4,), cv=(1.0,), pinf=(0.0,))
        init = lambda s: I.init_random(s, seed=13, noise=0.3)
    elif name == "3d-n2-bubble":
        sp = I.make_spec(3, 2, (21, 18, 17), chi=I.CHI_SHOCK, **WATER)
        init = lambda s: I.init_shock_bubble(s)
    elif name == "2d-n2-random":
        sp = I.make_spec(2, 2, (31, 22), chi=I.CHI_SHOCK, **WATER)
        init = lambda s: I.init_random(s, seed=15, noise=0.4, p_range=(1e5, 1e9))
    elif name == "3d-n2-water":
        sp = I.make_spec(3, 2, (17, 16, 19), chi=I.CHI_SHOCK, **WATER)
        init = lambda s: I.init_random(s, seed=16, noise=0.4, p_range=(1e5, 1e9))
    elif name == "3d-n2-thin":
        # one ragged tile along x (5 < 16) and z (4), ragged last tiles along
        # y (33), for the x-y launch and the z-walking stencil kernels
        sp = I.make_spec(3, 2, (5, 33, 4), chi=I.CHI_SHOCK, **WATER)
        init = lambda s: I.init_random(s, seed=17, noise=0.4, p_range=(1e5, 1e9))
    elif name == "3d-n2-random":
        sp = I.make_spec(3, 2, (17, 19, 18), gamma=(4.4, 1.4), cv=(1.0, 2.0), pinf=(100.0, 0.0),
                         chi=I.CHI_SHOCK)
        init = lambda s: I.init_random(s, seed=14, noise=0.4, p_range=(100.0, 300.0))
    else:
        raise KeyError(name)
    sp["dissipation"] = dissipation
    return sp, init


CASES = ["2d-n1", "2d-n1-stiff", "2d-n2-bubble", "3d-n1", "3d-n2-bubble", "3d-n2-random", "3d-n2-thin"]
# noisy random states, one and two species, up to the water stiffness
RANDOM_CASES = ["2d-n1", "2d-n1-stiff", "2d-n2-random", "3d-n1", "3d-n2-random", "3d-n2-water"]


def prepared(name, dissipation=1, moving=True):
    sp, init = case_spec(name, dissipation)
    o = oracle.Oracle(sp)
    JU, J, x = init(sp)
    Iin = I.interior(sp)
    x[Iin] += 0.01 * (np.stack(I.random_mesh(sp, seed=99, amp=1.0)) - np.stack(I.xi_nodes(sp)))
    ghosts(o, JU, J, x)
    if moving:
        disp, jx, jt = moving_metrics(o, sp, x, seed=7)
    else:
        disp = None
        jx, jt = o.metrics(x)
    return sp, o, JU, J, x, disp, jx, jt


