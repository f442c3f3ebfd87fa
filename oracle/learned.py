"""Oracle: the learned pressure correction inside CPR, in FP64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  No counterpart in the
paper.  After the multigrid cycle of the pressure stage,
    r' = r~_p - A_p dp_mg,
the network input per cell is (standardised ln k_x, standardised ln of the
total volumetric mobility, D^-1 r' / s) with D = diag A_p and
s = rms(D^-1 r') (standardisation: mean and population standard deviation
over the grid, a zero spread replaced by 1).  The network output d is a
direction; the correction dp_nn = alpha d takes the step that minimises
||r' - alpha A_p d||_2, alpha = <A_p d, r'> / <A_p d, A_p d> (0 when A_p d
vanishes), and is kept only if ||r' - A_p dp_nn||_2 < ||r'||_2.
"""
import numpy as np

from . import cpr, model, nn


def _pressure_stage_rt(pc, rt0):
    dp = cpr.vcycle(pc["mg"], rt0)
    Ap = pc["mg"]["levels"][0]
    return rt0 - cpr.scalar_spmv(Ap, dp), dp


def pressure_stage(pc, v):
    """(r', dp_mg, r~_p) for one vector v[b, grid]."""
    rt0 = cpr.decouple(pc, v)[0]
    rp, dp = _pressure_stage_rt(pc, rt0)
    return rp, dp, rt0


def _standardise(f):
    m = f.mean()
    sd = f.std()
    return (f - m) / (sd if sd * sd > 1e-24 else 1.0)


def total_mobility(fluid, poro, x):
    return model.cell_state(fluid, poro, x)["lam_t"][0]


def features(perm_md, lam_t, Ap, rprime):
    """Network input [nz, ny, nx, 3] and the scale s."""
    q = rprime / Ap[0]
    s = float(np.sqrt(np.mean(q * q)))
    f2 = q / s if s > 0 else np.zeros_like(q)
    return np.stack([_standardise(np.log(perm_md[0])), _standardise(np.log(lam_t)), f2], axis=-1), s


def learned_cpr_apply(pc, v, theta, perm_md, lam_t, composition="two-stage"):
    """CPR application with the judged network correction in the pressure
    stage; returns (z, accepted).  With composition "fpf" the pressure stage
    sees the residual left by the first block ILU(0) stage, as in
    cpr.cpr_apply."""
    At = pc["At"]
    Ap = pc["mg"]["levels"][0]
    rt = cpr.decouple(pc, v)
    z1 = None
    if composition == "fpf":
        z1 = cpr.ilu_apply(At, pc["Dinv"], rt)
        rt = rt - cpr.block_spmv(At, z1)
    rt0 = rt[0]
    rp, dp = _pressure_stage_rt(pc, rt0)
    feat, s = features(perm_md, lam_t, Ap, rp)
    y, _ = nn.forward(theta, feat[None])
    d = y[0]
    q = cpr.scalar_spmv(Ap, d)
    qq = float(np.sum(q * q))
    alpha = float(np.sum(q * rp)) / qq if qq > 0 else 0.0
    dpnn = alpha * d
    accepted = np.linalg.norm(rp - cpr.scalar_spmv(Ap, dpnn)) < np.linalg.norm(rp)
    if accepted:
        dp = dp + dpnn
    r2 = rt.copy()
    for d in range(7):
        sdp = cpr.shift(dp, d)
        for r in range(v.shape[0]):
            r2[r] -= At[d, r, 0] * sdp
    z = cpr.ilu_apply(At, pc["Dinv"], r2)
    z[0] += dp
    if z1 is not None:
        z = z1 + z
    return z, accepted
