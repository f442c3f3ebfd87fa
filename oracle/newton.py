"""Oracle: one inexact Newton iteration (Algorithm 1) of the scaled system.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Algorithm 1 assembles A = J(x) and b = -F(x), finds dx with
||b - A dx|| <= theta ||b|| (eq. (13)) and sets x = x + dx.  The forcing term
is fixed (theta = rtol) here.  Reading for the update, which the paper does
not spell out: saturation changes are chopped to |dS| <= 0.2 per cell and the
updated saturations clamped to [0, 1]; pressure is updated unchopped.
"""
import numpy as np

from . import cpr, krylov, model

DS_MAX = 0.2


def newton_update(x, dx):
    xn = x.copy()
    xn[0] = x[0] + dx[0]
    for s in range(1, x.shape[0]):
        xn[s] = np.clip(x[s] + np.clip(dx[s], -DS_MAX, DS_MAX), 0.0, 1.0)
    return xn


def newton_step(grid, fluid, perm, poro, wells, x_old, x, dt_days, restart=30,
                rtol=1e-6, max_iter=300, coarsest=512):
    """Assemble, set up CPR, solve with FGMRES, update.  Returns
    (x_new, dx, stats, R) with R the residual at the input state."""
    R, J = model.assemble(grid, fluid, perm, poro, wells, x_old, x, dt_days)
    rhs = -R
    pc = cpr.cpr_setup(J, coarsest)
    dx, st = krylov.fgmres(lambda v: cpr.block_spmv(J, v), lambda v: cpr.cpr_apply(pc, v),
                           rhs, restart=restart, rtol=rtol, max_iter=max_iter)
    return newton_update(x, dx), dx, st, R
