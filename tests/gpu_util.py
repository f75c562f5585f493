"""Shared helpers of the GPU parity tests (GPU path vs CPU oracle)."""
import sys

import numpy as np
import torch

import oracle
from paper_2202_07989_amd import inputs as I

TOL_FP64 = 1e-11          # parity gate of the FP64 path, per component


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def ghosts(o, JU, J, x):
    o.fill_ghosts(JU, o.nc)
    o.fill_ghosts(J, 1)
    o.fill_ghosts_x(x)


def parity(a, b, scale):
    """max |a - b| / scale over the arrays (scale > 0)."""
    return float(np.abs(a - b).max() / scale)


def state_scale(JU, sp, lam):
    """Per-component magnitude of the state: max|JU_c|; the momentum
    components share max(max|J rho v|, max|J rho| * lambda * min dxi), the
    second term being rho (|v| + c) (lambda * dxi ~ |v| + c on unit metrics),
    so a component that is zero in the input still has a physical scale."""
    N, d = sp["nspec"], sp["dim"]
    Iin = interior_slices(sp)
    mags = [np.abs(JU[c][Iin]).max() for c in range(JU.shape[0])]
    rho = sum(np.abs(JU[l][Iin]) for l in range(N)).max()
    mom = max(max(mags[N:N + d]), rho * lam * min(sp["dxi"][:d]))
    for j in range(d):
        mags[N + j] = mom
    return mags


def interior_slices(sp):
    return I.interior(sp)[1:]


def rhs_scale(JU, J, lam, Iin, sp=None):
    """Per-component scale of a right-hand side: state magnitude * lambda
    (a CFL-1 increment)."""
    if sp is None:
        s = [np.abs(JU[c][Iin[1:]]).max() * lam for c in range(JU.shape[0])]
    else:
        s = [m * lam for m in state_scale(JU, sp, lam)]
    return s, np.abs(J[Iin]).max() * lam


def moving_metrics(o, sp, x, seed, amp=0.01, c_s=0.5, dt=0.01):
    """Oracle metrics of a stage mesh with a smooth random displacement."""
    disp = I.zeros(sp, sp["dim"])
    Iin = I.interior(sp)
    disp[Iin] = amp * (np.stack(I.random_mesh(sp, seed=seed, amp=1.0)) - np.stack(I.xi_nodes(sp)))
    o.fill_ghosts(disp, sp["dim"])
    jx, jt = o.metrics(x, disp, c_s=c_s, dt=dt)
    return disp, jx, jt


# ---------------------------------------------------------------------------
# a-priori bound of the mixed-precision path (the oracle's orc_mixed_bound):
# per node and component, with K_F = 16, K_W = 64, u = 2^-24 fixed in advance
# ---------------------------------------------------------------------------
def interior_flat(sp, shape):
    """Flat padded indices of the interior nodes, in interior order."""
    return np.arange(int(np.prod(shape))).reshape(shape)[interior_slices(sp)].ravel()


def mixed_rhs_bound(o, sp, JU, J, jx, jt):
    """Bound (nc, *interior shape) on |mixed - FP64| of the right-hand side."""
    shape = J.shape[1:]
    idx = interior_flat(sp, shape)
    b = o.mixed_bound(JU, J, jx, jt, idx)
    ishape = J[I.interior(sp)].shape[1:]
    return b.T.reshape((o.nc,) + ishape)


def mixed_ratio(h, ref, bound):
    """max |h - ref| / bound over nodes (per component arrays of equal shape)."""
    return float((np.abs(h - ref) / bound).max())


def mixed_step_growth(cfl):
    """Assumed max-norm growth of a perturbation over one step (stated a priori)."""
    return 1.0 + 6.0 * cfl
