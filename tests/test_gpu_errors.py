"""Data errors, the same injected states through the oracle and the GPU
path: a negative partial density, a non-positive temperature (energy below
the kinetic and p_inf parts) and a non-finite momentum give the
non-physical code, a non-positive Jacobian the tangled-mesh code, from the
oracle's return value and from the GPU status word (Section 1 defines the
admissible states; J > 0 is the mesh's orientation)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_2202_07989_amd import es  # noqa: E402
from cases import prepared  # noqa: E402
from gpu_util import dev, say  # noqa: E402

NODE = (6, 7, 5)   # an interior node of the 3D case (padded indices)


def injected(sp, JU, J, kind):
    N = sp["nspec"]
    U, Jv = JU.copy(), J.copy()
    if kind == "negative-density":
        U[0][NODE] = -abs(U[0][NODE])
    elif kind == "nonpositive-temperature":
        U[-1][NODE] = 0.0
    elif kind == "nan-momentum":
        U[N][NODE] = np.nan
    elif kind == "nonpositive-jacobian":
        Jv[0][NODE] = -0.5
    elif kind == "zero-jacobian":
        Jv[0][NODE] = 0.0
    return U, Jv


@pytest.mark.parametrize("kind,code", [("negative-density", es.ES_ENONPHYS),
                                       ("nonpositive-temperature", es.ES_ENONPHYS),
                                       ("nan-momentum", es.ES_ENONPHYS),
                                       ("nonpositive-jacobian", es.ES_ETANGLE),
                                       ("zero-jacobian", es.ES_ETANGLE)])
def test_same_code_from_oracle_and_gpu(kind, code):
    say(f"[errors] {kind}")
    sp, o, JU, J, x, disp, jx, jt = prepared("3d-n2-water")
    U, Jv = injected(sp, JU, J, kind)
    rc_o, _, _ = o.rhs(U, Jv, jx, jt)
    assert rc_o == code
    ctx = es.Context(sp)
    gU, gJ = torch.zeros_like(dev(JU)), torch.zeros_like(dev(J))
    ctx.es_rhs(dev(JU), dev(J), dev(jx), dev(jt), gU, gJ)
    assert ctx.es_status(reset=True)[0] == es.ES_OK          # the clean state first
    ctx.es_rhs(dev(U), dev(Jv), dev(jx), dev(jt), gU, gJ)
    rc_g, flags = ctx.es_status(reset=True)
    assert rc_g == code, (rc_g, flags)
    assert ctx.es_status()[0] == es.ES_OK                    # reset clears the word
