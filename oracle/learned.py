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

The same judged step can act inside the multigrid cycle on a coarse level l
(learned_cpr_apply(level=l)): after that level's post-smoothing, r' is the
level's residual r_l - A_l x_l, the features are the means of ln k_x and
ln lambda_t over each coarse cell's block of fine cells with D = diag A_l,
and the accepted correction is added to x_l before the cycle returns to the
finer levels, whose post-smoothing then smooths it.
"""
import numpy as np
import scipy.linalg

from . import cpr, model, nn


def _pressure_stage_rt(pc, rt0, alpha=1.0):
    dp = cpr.vcycle(pc["mg"], rt0, 0, alpha)
    Ap = pc["mg"]["levels"][0]
    return rt0 - cpr.scalar_spmv(Ap, dp), dp


def pressure_stage(pc, v, alpha=1.0):
    """(r', dp_mg, r~_p) for one vector v[b, grid]; alpha scales the
    cycle's coarse corrections as in cpr.vcycle."""
    rt0 = cpr.decouple(pc, v)[0]
    rp, dp = _pressure_stage_rt(pc, rt0, alpha)
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


def level_fields(perm_md, lam_t, level):
    """ln k_x and ln lambda_t for multigrid level `level` of a grid whose
    dimensions are divisible by 2^level: the mean of the fine values over
    each coarse cell's 2^level x 2^level x 2^level block of fine cells (the
    composite aggregate of the 2x2x2 aggregation)."""
    lk, ll = np.log(perm_md[0]), np.log(lam_t)
    if level == 0:
        return lk, ll
    f = 2 ** level
    nz, ny, nx = lk.shape
    red = lambda a: a.reshape(nz // f, f, ny // f, f, nx // f, f).mean(axis=(1, 3, 5))
    return red(lk), red(ll)


def level_features(lnk, lnl, A, rprime):
    """Network input [nz, ny, nx, 3] on one level from its ln k / ln lambda
    fields, its operator A and the residual r' there; and the scale s."""
    q = rprime / A[0]
    s = float(np.sqrt(np.mean(q * q)))
    f2 = q / s if s > 0 else np.zeros_like(q)
    return np.stack([_standardise(lnk), _standardise(lnl), f2], axis=-1), s


def judged_step(A, theta, lnk, lnl, rp):
    """The network's judged correction of the residual rp on a level with
    operator A: (correction, accepted)."""
    feat, s = level_features(lnk, lnl, A, rp)
    y, _ = nn.forward(theta, feat[None])
    d = y[0]
    q = cpr.scalar_spmv(A, d)
    qq = float(np.sum(q * q))
    alpha = float(np.sum(q * rp)) / qq if qq > 0 else 0.0
    dnn = alpha * d
    accepted = bool(np.linalg.norm(rp - cpr.scalar_spmv(A, dnn)) < np.linalg.norm(rp))
    return (dnn if accepted else np.zeros_like(rp)), accepted


def vcycle_with_hook(mg, r, hook_level, hook, level=0, alpha=1.0):
    """cpr.vcycle with one addition: on level hook_level, after its
    post-smoothing, x += hook(r, x) (the learned correction inside the
    cycle, which the finer levels' post-smoothing then smooths)."""
    levels = mg["levels"]
    A = levels[level]
    shape = A.shape[1:]
    if level == len(levels) - 1:
        return scipy.linalg.lu_solve(mg["lu"], r.ravel()).reshape(shape)
    col = cpr.colour(shape)
    x = np.zeros_like(r)
    for _ in range(mg.get("pre", 1)):
        cpr.gs_half_sweep(A, r, x, col, 0)
        cpr.gs_half_sweep(A, r, x, col, 1)
    res = r - cpr.scalar_spmv(A, x)
    P = cpr.prolongator(shape)
    rc = (P.T @ res.ravel()).reshape(cpr.coarse_shape(shape))
    ec = vcycle_with_hook(mg, rc, hook_level, hook, level + 1, alpha)
    x += alpha * (P @ ec.ravel()).reshape(shape)
    for _ in range(mg.get("post", 1)):
        cpr.gs_half_sweep(A, r, x, col, 1)
        cpr.gs_half_sweep(A, r, x, col, 0)
    if level == hook_level:
        x = x + hook(r, x)
    return x


def level_residual(pc, v, level, alpha=1.0):
    """The residual r - A_l x that the pressure stage's cycle leaves on
    level `level` (after that level's post-smoothing) for the vector v."""
    rt0 = cpr.decouple(pc, v)[0]
    mg = pc["mg"]
    out = {}

    def capture(r, x):
        out["rp"] = r - cpr.scalar_spmv(mg["levels"][level], x)
        return np.zeros_like(x)
    vcycle_with_hook(mg, rt0, level, capture, 0, alpha)
    return out["rp"]


def learned_cpr_apply(pc, v, theta, perm_md, lam_t, composition="two-stage", level=0, alpha=1.0):
    """CPR application with the judged network correction in the pressure
    stage; returns (z, accepted).  level 0: on the fine pressure residual
    after the multigrid cycle; level l >= 1: inside the cycle on multigrid
    level l, after its post-smoothing (features from level_fields).  With
    composition "fpf" the pressure stage sees the residual left by the first
    block ILU(0) stage, as in cpr.cpr_apply.  alpha scales the cycle's
    coarse corrections as in cpr.cpr_apply (on level l >= 1 the finer
    levels scale the corrected level's result as well)."""
    At = pc["At"]
    Ap = pc["mg"]["levels"][0]
    rt = cpr.decouple(pc, v)
    z1 = None
    if composition == "fpf":
        z1 = cpr.ilu_solve(pc, rt)
        rt = rt - cpr.block_spmv(At, z1)
    rt0 = rt[0]
    if level == 0:
        rp, dp = _pressure_stage_rt(pc, rt0, alpha)
        lnk, lnl = level_fields(perm_md, lam_t, 0)
        dpnn, accepted = judged_step(Ap, theta, lnk, lnl, rp)
        dp = dp + dpnn
    else:
        mg = pc["mg"]
        A_l = mg["levels"][level]
        lnk, lnl = level_fields(perm_md, lam_t, level)
        acc = []

        def hook(r, x):
            d, a = judged_step(A_l, theta, lnk, lnl, r - cpr.scalar_spmv(A_l, x))
            acc.append(a)
            return d
        dp = vcycle_with_hook(mg, rt0, level, hook, 0, alpha)
        accepted = acc[0]
    r2 = rt.copy()
    for d in range(7):
        sdp = cpr.shift(dp, d)
        for r in range(v.shape[0]):
            r2[r] -= At[d, r, 0] * sdp
    z = cpr.ilu_solve(pc, r2)
    z[0] += dp
    if z1 is not None:
        z = z1 + z
    return z, accepted
