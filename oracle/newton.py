"""Oracle: one inexact Newton iteration (Algorithm 1) of the scaled system.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Algorithm 1 assembles A = J(x) and b = -F(x), finds dx with
||b - A dx|| <= theta ||b|| (eq. (13)) and sets x = x + dx.  newton_step is
one such iteration with a fixed theta = rtol; time_step runs the whole
iteration of one backward-Euler step with the forcing terms of eq. (14).
Readings where the paper is silent:
  * the update chops saturation changes to |dS| <= 0.2 per cell and clamps
    the updated saturations to [0, 1]; pressure is updated unchopped;
  * the stopping test of Algorithm 1 is relative, ||b^l|| < newton_tol
    ||b^0|| with b^0 = -F(x_old) of the step (the paper's tolerances 1e-2 and
    1e-3 of Sec. 4 are read as relative reductions);
  * eq. (14) for l >= 1 with theta_0 = 0.1 for the first iteration, choice 2
    with the absolute value of the difference of norms, choice 3 with
    gamma = 0.9, beta = 2 (the paper gives no values), every theta_l clamped
    to [1e-6, 0.5];
  * a time-step cut (Sec. 4 reports one) halves dt and restarts from x_old
    when an attempt does not converge in max_newton iterations, meets a
    non-finite residual or a singular preconditioner block.
"""
import numpy as np

from . import cpr, krylov, model

DS_MAX = 0.2


def newton_update(x, dx, pb_min=None):
    """x + dx with the chops and clamps below; black oil (3 unknowns)
    switches its third unknown with the phase state:
      * saturated (x2 = S_g >= 0): S_g + clip(dS_g) below zero means the free
        gas has dissolved: the cell becomes undersaturated at its bubble
        point, x2 = -p (p_b = p after the update); otherwise S_g is clamped
        to [0, 1];
      * undersaturated (x2 = -p_b): p_b - dx2 (unchopped) above the updated
        pressure means free gas appears: the cell becomes saturated with
        S_g = 0; otherwise p_b is floored at pb_min (the first PVT node)."""
    xn = x.copy()
    xn[0] = x[0] + dx[0]
    if x.shape[0] > 1:
        xn[1] = np.clip(x[1] + np.clip(dx[1], -DS_MAX, DS_MAX), 0.0, 1.0)
    if x.shape[0] < 3:
        return xn
    sat = x[2] >= 0.0
    sg = x[2] + np.clip(dx[2], -DS_MAX, DS_MAX)
    pb = -(x[2] + dx[2])
    sat_new = np.where(sg >= 0.0, np.minimum(sg, 1.0), -xn[0])
    und_new = np.where(pb > xn[0], 0.0, -np.maximum(pb, pb_min))
    xn[2] = np.where(sat, sat_new, und_new)
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
    return newton_update(x, dx, _pb_min(fluid)), dx, st, R


def _pb_min(fluid):
    return float(np.asarray(fluid["pvt"])[0][0]) if fluid["model"] == 3 else None


# ------------------------------------------------------------ time step

FORCING = ("fixed", "ew1", "ew2", "ew3")


def forcing_term(choice, l, bn, bn_prev, rn_prev, diff_prev, theta0, theta_min, theta_max,
                 gamma, beta, rtol):
    """theta_l of Algorithm 1 step 4.  "fixed": the standard Newton method's
    constant rtol.  Otherwise eq. (14), choice 1, 2 or 3, for l >= 1, with
    bn = ||b^l||, bn_prev = ||b^(l-1)||, rn_prev = ||r^(l-1)|| and
    diff_prev = ||b^l - r^(l-1)||; theta0 for l = 0; clamped to
    [theta_min, theta_max].  Choice 2 takes the absolute value of the
    difference of norms."""
    if choice == "fixed":
        return rtol
    if l == 0:
        t = theta0
    elif choice == "ew1":
        t = diff_prev / bn_prev
    elif choice == "ew2":
        t = abs(bn - rn_prev) / bn_prev
    else:
        t = gamma * (bn / bn_prev) ** beta
    return min(max(t, theta_min), theta_max)


def border_operators(J, W, pc, composition, shape):
    """The Jacobian of eq. (16) with the rate wells' BHP unknowns appended
    to the cell unknowns (flat vectors [cells..., p_h...]) and its
    preconditioner: CPR on the cell block, then each well's BHP from its
    own equation given the cell correction (block lower-triangular):
    z_w = (r_w - C_w z_cells) / D_w."""
    nr = len(W["D"])
    n = int(np.prod(shape))

    def split(v):
        return v[:n].reshape(shape), v[n:]

    def A(v):
        c, w = split(v)
        y = cpr.block_spmv(J, c)
        for q in range(nr):
            y = y + W["B"][q] * w[q]
        yw = np.array([np.sum(W["C"][q] * c) + W["D"][q] * w[q] for q in range(nr)])
        return np.concatenate([y.ravel(), yw])

    def M(v):
        c, w = split(v)
        z = cpr.cpr_apply(pc, c, composition=composition)
        zw = np.array([(w[q] - np.sum(W["C"][q] * z)) / W["D"][q] for q in range(nr)])
        return np.concatenate([z.ravel(), zw])
    return A, M


def time_step(grid, fluid, perm, poro, wells, x_old, dt_days, forcing="ew1", theta0=0.1,
              theta_min=1e-6, theta_max=0.5, gamma=0.9, beta=2.0, newton_tol=1e-3, max_newton=20,
              max_cuts=6, krylov_method="fgmres", restart=30, max_iter=300, rtol=1e-6, coarsest=512,
              decoupling="qimpes", composition="two-stage", bhp_old=None):
    """One backward-Euler time step by the inexact Newton method
    (Algorithm 1) from x^0 = x_old, with time-step cuts.

    Newton iterations run while ||b^l|| >= newton_tol * ||b^0|| (b = -R at
    the current iterate, b^0 at x_old) and stop with failure after
    max_newton iterations, or when a residual is not finite or a
    preconditioner block is singular.  A failed attempt halves dt and starts
    again from x_old, at most max_cuts times.  A linear solve that does not
    reach theta within max_iter iterations still updates x (inexact Newton);
    one whose residual is not finite fails the attempt.  Rate-controlled
    wells add their bottom-hole pressures to the unknowns (starting from
    bhp_old, default the wells' "bhp" entries; updated unchopped) and their
    rate equations to the system.  Returns (x, stats): x the accepted state
    (x_old if every attempt failed), stats with dt_taken, cuts, converged,
    bhp (the rate wells' final BHPs), the per-iteration history of the
    accepted (or last) attempt (theta, linear iterations, ||b||) and totals
    over attempts."""
    assert forcing in FORCING
    solve = krylov.fgmres if krylov_method == "fgmres" else krylov.bicgstab
    nr = len(model.rate_wells(wells))
    if bhp_old is None:
        bhp_old = np.array([w["bhp"] for w in model.rate_wells(wells)], dtype=np.float64)
    shape = x_old.shape
    n = x_old.size
    dt = float(dt_days)
    total_newton = total_linear = 0

    def residual(x, xw):
        R, J, W = model.assemble(grid, fluid, perm, poro, wells, x_old, x, dt, bhp=xw, border=True)
        return -np.concatenate([R.ravel(), W["R"]]), J, W

    for cut in range(max_cuts + 1):
        x = x_old.copy()
        xw = np.array(bhp_old, dtype=np.float64)
        b, J, W = residual(x, xw)
        bn = float(np.linalg.norm(b))
        b0 = bn
        hist = {"theta": [], "linear_iterations": [], "bnorm": [bn]}
        bn_prev = rn_prev = diff_prev = None
        l = 0
        ok = False
        while np.isfinite(bn):
            if bn == 0.0 or bn < newton_tol * b0:
                ok = True
                break
            if l >= max_newton:
                break
            theta = forcing_term(forcing, l, bn, bn_prev, rn_prev, diff_prev, theta0, theta_min,
                                 theta_max, gamma, beta, rtol)
            try:
                pc = cpr.cpr_setup(J, coarsest, decoupling=decoupling)
            except (FloatingPointError, np.linalg.LinAlgError):
                break
            A, M = border_operators(J, W, pc, composition, shape)
            kw = {"restart": restart} if krylov_method == "fgmres" else {}
            with np.errstate(all="ignore"):
                try:
                    dx, st = solve(A, M, b, rtol=theta, max_iter=max_iter, **kw)
                except ValueError:          # a non-finite Hessenberg entry
                    break
                r = b - A(dx)
            if not (np.isfinite(st["true_rel"]) and np.all(np.isfinite(r))):
                break
            x = newton_update(x, dx[:n].reshape(shape), _pb_min(fluid))
            xw = xw + dx[n:]
            with np.errstate(all="ignore"):
                b_new, J, W = residual(x, xw)
            bn_prev, rn_prev = bn, float(np.linalg.norm(r))
            diff_prev = float(np.linalg.norm(b_new - r))
            b, bn = b_new, float(np.linalg.norm(b_new))
            l += 1
            hist["theta"].append(theta)
            hist["linear_iterations"].append(st["iterations"])
            hist["bnorm"].append(bn)
        total_newton += l
        total_linear += sum(hist["linear_iterations"])
        stats = {"dt_taken": dt, "cuts": cut, "converged": ok, "newton_iterations": l,
                 "total_newton": total_newton, "total_linear": total_linear, "history": hist,
                 "bhp": xw if ok else np.array(bhp_old, dtype=np.float64)}
        if ok:
            return x, stats
        dt *= 0.5
    return x_old.copy(), stats


def simulate(grid, fluid, perm, poro, wells, x0, t_end, dt0, dt_max, growth=2.0, **step_kw):
    """Backward-Euler time stepping from x0 over [0, t_end] days: each step is
    time_step (with its cuts); after a step that needed no cut the next dt
    grows by `growth` up to dt_max, after a cut it stays at the step taken;
    the last step is shortened to end at t_end.  Returns (x, stats) with the
    number of steps, the sums of cuts, Newton and linear iterations over
    every attempt, the step sizes taken, the same counts per accepted step
    (its cuts included), and whether t_end was reached."""
    x = x0.copy()
    t = 0.0
    dt = float(dt0)
    bhp = step_kw.pop("bhp_old", None)
    st = {"steps": 0, "cuts": 0, "total_newton": 0, "total_linear": 0, "dts": [], "completed": False,
          "step_newton": [], "step_linear": [], "step_cuts": []}
    while t < t_end:
        h = min(dt, t_end - t)
        x_new, s = time_step(grid, fluid, perm, poro, wells, x, h, bhp_old=bhp, **step_kw)
        st["cuts"] += s["cuts"]
        st["total_newton"] += s["total_newton"]
        st["total_linear"] += s["total_linear"]
        if not s["converged"]:
            return x, st
        x = x_new
        bhp = s["bhp"]
        st["bhp"] = bhp
        st["steps"] += 1
        st["dts"].append(s["dt_taken"])
        st["step_newton"].append(s["total_newton"])
        st["step_linear"].append(s["total_linear"])
        st["step_cuts"].append(s["cuts"])
        t = t + s["dt_taken"]
        dt = min(growth * s["dt_taken"], dt_max) if s["cuts"] == 0 else s["dt_taken"]
    st["completed"] = True
    return x, st
