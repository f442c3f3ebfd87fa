"""Oracle: restarted flexible GMRES with classical Gram-Schmidt twice.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper solves each Newton system A dx = b until ||b - A dx|| <= theta ||b||
(Algorithm 1, eq. (13)); the norm is read as the Euclidean 2-norm over every
unknown of the scaled system.  The Krylov method here is right-preconditioned
flexible GMRES(m) (Saad's FGMRES): the preconditioned directions z_j are kept,
so a preconditioner that changes between applications (mixed precision, the
learned stage) is allowed.

Algorithm (one restart cycle, x0 = 0 on entry):
    r = b - A x, beta = ||r||, v_0 = r / beta, g = beta e_0
    for j = 0 .. m-1:
        z_j = M^-1 v_j;  w = A z_j
        h = V^T w; w -= V h; h' = V^T w; w -= V h'; h += h'     (CGS2)
        h_{j+1,j} = ||w||
        apply the previous Givens rotations to column j, form a new one,
        rotate g; stop when |g_{j+1}| <= rtol ||b||, when
        h_{j+1,j} <= 1e-14 ||A z_j|| (happy breakdown; ||A z_j|| taken as the
        2-norm of the full column h_{0..j+1,j}), or when max_iter matvecs
        have been spent;  v_{j+1} = w / h_{j+1,j}
    solve the upper-triangular least-squares system for y; x += Z y;
    recompute the true residual; restart while it exceeds rtol ||b|| and
    iterations remain.
The iteration count is the number of Arnoldi matvecs (true-residual
products are not counted).
"""
import numpy as np
import scipy.linalg

BREAKDOWN = 1e-14


def _dot(a, b):
    return float(np.dot(a.ravel(), b.ravel()))


def fgmres(apply_A, apply_M, b, restart=30, rtol=1e-6, max_iter=300, x0=None,
           record=None):
    """Returns (x, stats).  stats: iterations, cycles, converged, est_rel,
    true_rel, history (estimated relative residual after each iteration).
    `record`, if given, is called with (j, v_j, z_j) for every preconditioner
    application (used to harvest pressure-stage inputs)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bnorm = np.sqrt(_dot(b, b))
    st = {"iterations": 0, "cycles": 0, "converged": False, "est_rel": 0.0,
          "true_rel": 0.0, "history": []}
    if bnorm == 0.0:
        x[...] = 0.0
        st["converged"] = True
        return x, st
    r = b - apply_A(x) if x0 is not None else b.copy()
    its = 0
    while True:
        beta = np.sqrt(_dot(r, r))
        st["true_rel"] = beta / bnorm
        if beta <= rtol * bnorm:
            st["converged"] = True
            break
        if its >= max_iter:
            break
        m = restart
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        k = 0
        for j in range(m):
            z = apply_M(V[j])
            if record is not None:
                record(its, V[j], z)
            Z.append(z)
            w = apply_A(z)
            its += 1
            h = np.array([_dot(V[i], w) for i in range(j + 1)])
            for i in range(j + 1):
                w = w - h[i] * V[i]
            h2 = np.array([_dot(V[i], w) for i in range(j + 1)])
            for i in range(j + 1):
                w = w - h2[i] * V[i]
            h = h + h2
            hn = np.sqrt(_dot(w, w))
            col = np.zeros(m + 1)
            col[:j + 1] = h
            col[j + 1] = hn
            az = np.sqrt(np.sum(col[:j + 2] ** 2))
            for i in range(j):
                t = cs[i] * col[i] + sn[i] * col[i + 1]
                col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1]
                col[i] = t
            den = np.hypot(col[j], col[j + 1])
            if den == 0.0:
                cs[j], sn[j] = 1.0, 0.0
            else:
                cs[j], sn[j] = col[j] / den, col[j + 1] / den
            col[j] = den
            col[j + 1] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            H[:, j] = col
            k = j + 1
            st["history"].append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= rtol * bnorm or hn <= BREAKDOWN * az or its >= max_iter:
                break
            V.append(w / hn)
        y = scipy.linalg.solve_triangular(H[:k, :k], g[:k], lower=False)
        for i in range(k):
            x = x + y[i] * Z[i]
        st["cycles"] += 1
        st["est_rel"] = abs(g[k]) / bnorm
        r = b - apply_A(x)
    st["iterations"] = its
    return x, st


def bicgstab(apply_A, apply_M, b, rtol=1e-6, max_iter=300):
    """Right-preconditioned BiCGSTAB (van der Vorst, 1992), the Krylov method
    of every example in the paper (Sec. 4), with the same CPR preconditioner.

    x0 = 0, r = b, shadow residual rh = r, rho_prev = alpha = omega = 1,
    p = v = 0; each iteration:
        rho = <rh, r>;  beta = (rho / rho_prev) (alpha / omega)
        p = r + beta (p - omega v);  ph = M^-1 p;  v = A ph
        alpha = rho / <rh, v>;  s = r - alpha v
        sh = M^-1 s;  t = A sh;  omega = <t, s> / <t, t> (0 when t = 0)
        x += alpha ph + omega sh;  r = s - omega t
    until ||r|| <= rtol ||b||; then the true residual b - A x is formed and,
    if it still exceeds rtol ||b|| and iterations remain, the method restarts
    from x with r and rh set to the true residual.  A vanishing rho, <rh, v>
    or omega stops the iteration (breakdown) with the current x.  The
    iteration count is the number of BiCGSTAB iterations (two products with
    A and two preconditioner applications each).
    Returns (x, stats) like fgmres."""
    x = np.zeros_like(b)
    bnorm = np.sqrt(_dot(b, b))
    stats = {"iterations": 0, "cycles": 0, "converged": False, "bnorm": bnorm, "breakdown": False}
    if bnorm == 0.0:
        stats.update(converged=True, true_rel=0.0)
        return x, stats
    its = 0
    r = b.copy()
    while True:
        stats["cycles"] += 1
        rh = r.copy()
        rho_prev = alpha = omega = 1.0
        p = np.zeros_like(b)
        v = np.zeros_like(b)
        stop = False
        while its < max_iter:
            rho = _dot(rh, r)
            if rho == 0.0 or not np.isfinite(rho):
                stats["breakdown"] = True
                stop = True
                break
            beta = (rho / rho_prev) * (alpha / omega)
            p = r + beta * (p - omega * v)
            ph = apply_M(p)
            v = apply_A(ph)
            rv = _dot(rh, v)
            if rv == 0.0 or not np.isfinite(rv):
                stats["breakdown"] = True
                stop = True
                break
            alpha = rho / rv
            s = r - alpha * v
            sh = apply_M(s)
            t = apply_A(sh)
            tt = _dot(t, t)
            omega = _dot(t, s) / tt if tt > 0.0 else 0.0
            x = x + alpha * ph + omega * sh
            r = s - omega * t
            its += 1
            rho_prev = rho
            if np.sqrt(_dot(r, r)) <= rtol * bnorm:
                break
            if omega == 0.0:
                stats["breakdown"] = True
                stop = True
                break
        r = b - apply_A(x)
        true_rel = np.sqrt(_dot(r, r)) / bnorm
        if true_rel <= rtol:
            stats["converged"] = True
            break
        if stop or its >= max_iter:
            break
    stats.update(iterations=its, true_rel=true_rel)
    return x, stats
