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

Orthogonalisation "dcgs2" (the default) computes the same basis with the
second Gram-Schmidt pass of each vector delayed to the next step
(delayed classical Gram-Schmidt twice, as in Swirydowicz, Langou,
Ananthan, Yang and Thomas, "Low synchronization Gram-Schmidt and GMRES
algorithms", 2020), so that each step projects the new vector and
reorthogonalises the previous one from the same two sets of inner products.
With u_j = the once-projected vector of step j-1, nu_j = ||u_j|| and
uh_j = u_j / nu_j (what the preconditioner receives at step j):
    w = A M^-1 uh_j
    a = V_{j-1}^T uh_j, c = V_{j-1}^T w, d = uh_j^T w, e = uh_j^T uh_j
    beta_j = sqrt(e - |a|^2),  v_j = (uh_j - V_{j-1} a) / beta_j
    column j-1 of H: += nu_j a (rows < j), row j = nu_j beta_j
    column j of H:   c (rows < j), g_j = (d - a.c) / beta_j (row j),
                     nu_{j+1} = ||w - V_{j-1} c - g_j v_j|| (row j+1)
Step 0 has no previous vector: v_0 = r / beta, g_0 = v_0^T w.  In exact
arithmetic a = 0 and e = 1, so every quantity equals its CGS2 value; the
Givens rotations are recomputed from H after each step (its previous column
changes), and the last column keeps its once-projected values.  A
vanishing beta_j (uh_j in the span of the basis) ends the cycle before step
j, like a happy breakdown.  "cgs2" keeps both passes in the step; restarts
longer than 32 use it as well.
"""
import numpy as np
import scipy.linalg

BREAKDOWN = 1e-14


def _dot(a, b):
    return float(np.dot(a.ravel(), b.ravel()))


def _givens_qr(H, beta, k):
    """Givens QR of the (k+1) x k Hessenberg block: returns (R, g) with
    g = Q^T beta e_0 (g[k] is the least-squares residual)."""
    R = H[:k + 1, :k].copy()
    g = np.zeros(k + 1)
    g[0] = beta
    for i in range(k):
        den = np.hypot(R[i, i], R[i + 1, i])
        if den == 0.0:
            c, s = 1.0, 0.0
        else:
            c, s = R[i, i] / den, R[i + 1, i] / den
        ri, ri1 = R[i, i:].copy(), R[i + 1, i:].copy()
        R[i, i:] = c * ri + s * ri1
        R[i + 1, i:] = -s * ri + c * ri1
        g[i + 1] = -s * g[i]
        g[i] = c * g[i]
    return R, g


def dcgs2_step(V, uh, w):
    """One step of delayed CGS2 against the orthonormal vectors V (j >= 1 of
    them): reorthogonalise uh and project w with the same inner products.
    Returns (v, a, beta, c, g, u): v = (uh - V a) / beta the new basis
    vector, a = V^T uh, beta = sqrt(uh.uh - |a|^2), c = V^T w,
    g = v^T w = (uh.w - a.c) / beta, u = w - V c - g v; or None when beta
    vanishes (uh in the span of V)."""
    j = len(V)
    a = np.array([_dot(V[i], uh) for i in range(j)])
    c = np.array([_dot(V[i], w) for i in range(j)])
    d = _dot(uh, w)
    e = _dot(uh, uh)
    b2 = e - float(np.dot(a, a))
    if not b2 > 0.0:
        return None
    bj = np.sqrt(b2)
    v = uh.copy()
    for i in range(j):
        v = v - a[i] * V[i]
    v = v / bj
    g = (d - float(np.dot(a, c))) / bj
    u = w.copy()
    for i in range(j):
        u = u - c[i] * V[i]
    u = u - g * v
    return v, a, bj, c, g, u


def _fgmres_cycle_dcgs2(apply_A, apply_M, r, beta, bnorm, m, rtol, max_iter, its, st, record):
    """One restart cycle with delayed reorthogonalisation (module docstring).
    Returns (Z, y, its, est)."""
    V = [r / beta]
    Z = []
    H = np.zeros((m + 1, m))
    uh, nu = None, None
    k, g = 0, np.array([beta])
    for j in range(m):
        q = V[0] if j == 0 else uh
        z = apply_M(q)
        if record is not None:
            record(its, q, z)
        w = apply_A(z)
        if j == 0:
            c = np.zeros(0)
            gj = _dot(V[0], w)
            u = w - gj * V[0]
        else:
            out = dcgs2_step(V, uh, w)
            if out is None:
                break                      # uh_j in the span of the basis: stop before step j
            v, a, bj, c, gj, u = out
            V.append(v)
            H[:j, j - 1] += nu * a
            H[j, j - 1] = nu * bj
        Z.append(z)
        its += 1
        nu = np.sqrt(_dot(u, u))
        H[:j, j] = c
        H[j, j] = gj
        H[j + 1, j] = nu
        k = j + 1
        R, g = _givens_qr(H, beta, k)
        st["history"].append(abs(g[k]) / bnorm)
        az = np.sqrt(np.sum(H[:j + 2, j] ** 2))
        if abs(g[k]) <= rtol * bnorm or nu <= BREAKDOWN * az or its >= max_iter:
            break
        uh = u / nu
    R, g = _givens_qr(H, beta, k)
    y = scipy.linalg.solve_triangular(R[:k, :k], g[:k], lower=False)
    return Z, y, its, abs(g[k])


def fgmres(apply_A, apply_M, b, restart=30, rtol=1e-6, max_iter=300, x0=None,
           record=None, orth="dcgs2"):
    """Returns (x, stats).  stats: iterations, cycles, converged, est_rel,
    true_rel, history (estimated relative residual after each iteration).
    `record`, if given, is called with (j, v_j, z_j) for every preconditioner
    application (used to harvest pressure-stage inputs).  orth: "dcgs2"
    (default) or "cgs2"."""
    if orth not in ("dcgs2", "cgs2"):
        raise ValueError(orth)
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
        if orth == "dcgs2" and m <= 32:
            Z, y, its, est = _fgmres_cycle_dcgs2(apply_A, apply_M, r, beta, bnorm, m, rtol, max_iter,
                                                 its, st, record)
            for i in range(len(y)):
                x = x + y[i] * Z[i]
            st["cycles"] += 1
            st["est_rel"] = est / bnorm
            r = b - apply_A(x)
            continue
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
