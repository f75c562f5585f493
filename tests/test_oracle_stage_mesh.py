"""Ghost layers of the c = 1 stage mesh (no GPU).

The stage meshes of Sections 4-5 are x^n + c_s disp, and the c = 1 one is the
mesh x^{n+1} that the step ends with.  Its ghost layers can be formed two
ways: x^n's ghost values plus disp's (the oracle's form), or the mesh's face
rules applied to x^n + disp itself (the GPU step's form, which makes that
stage mesh exactly the next step's x^n).  The mesh's rules are affine in the
mesh (periodic: image + L; a non-periodic face: 2 wall - image along its own
direction), and the displacement's rules are their linear parts (periodic:
image; non-periodic: component k negated), so the two forms agree in exact
arithmetic: bit for bit at the interior nodes and to rounding at the ghost
nodes.  A displacement rule that is not the linear part of the mesh rule (a
missed sign, a shifted image) shows up as a difference of the size of disp.
"""
import numpy as np
import pytest

import oracle
from paper_2202_07989_amd import inputs as I
from test_oracle_bc import inside_mesh, walled

R, O = 1, 2
KW = dict(chi=I.CHI_SHOCK, gamma=(1.4,), cv=(1.0,), pinf=(0.0,))
CASES = {
    "2d-periodic": (2, (19, 13), [(0, 0), (0, 0)]),
    "2d-walls": (2, (17, 12), [(R, R), (R, R)]),
    "2d-walls-outflow": (2, (16, 11), [(O, O), (R, R)]),
    "3d-mixed": (3, (9, 8, 7), [(R, R), (O, O), (0, 0)]),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_stage_mesh_ghosts_agree_to_rounding(name):
    dim, n, bc = CASES[name]
    sp = walled(dim, 1, n, bc, **KW)
    o = oracle.Oracle(sp)
    Iin = I.interior(sp)
    xi = np.stack(I.xi_nodes(sp))
    x = I.zeros(sp, dim)
    x[Iin] = np.stack(inside_mesh(sp, 3))
    o.fill_ghosts_x(x)
    disp = I.zeros(sp, dim)
    disp[Iin] = 0.5 * (np.stack(inside_mesh(sp, 4, amp=0.01)) - xi)
    o.fill_ghosts_kind(disp, dim, 2)
    assert np.abs(disp[Iin]).max() > 1e-4          # a displacement that matters
    a = x + disp                                   # ghosts of x^n plus ghosts of disp
    b = x + disp
    o.fill_ghosts_x(b)                             # the mesh's face rules on x^n + disp
    np.testing.assert_array_equal(a[Iin], b[Iin])
    for c in range(dim):
        scale = np.abs(x[c]).max()
        err = np.abs(a[c] - b[c]).max()
        assert err <= 4 * np.finfo(float).eps * scale, (c, err)


def test_a_wrong_displacement_rule_is_seen():
    """The same comparison with the displacement's ghosts taken as plain
    copies (no sign change at the walls) differs by the size of disp."""
    sp = walled(2, 1, (17, 12), [(R, R), (R, R)], **KW)
    o = oracle.Oracle(sp)
    Iin = I.interior(sp)
    x = I.zeros(sp, 2)
    x[Iin] = np.stack(inside_mesh(sp, 3))
    o.fill_ghosts_x(x)
    disp = I.zeros(sp, 2)
    disp[Iin] = 0.5 * (np.stack(inside_mesh(sp, 4, amp=0.01)) - np.stack(I.xi_nodes(sp)))
    o.fill_ghosts_kind(disp, 2, 0)                 # plain fields: mirrored copies
    b = x + disp
    o.fill_ghosts_x(b)
    assert np.abs((x + disp) - b).max() > 1e-4
