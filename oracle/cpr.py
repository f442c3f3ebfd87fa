"""Oracle: the two-stage CPR preconditioner on the 7-point block Jacobian.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain FP64 numpy/scipy.

The paper's linear-solver section (Sec. 2.5, the block matrix of eq. (16))
builds a constrained-pressure-residual preconditioner: decouple the pressure
equation (quasi-IMPES), solve the pressure sub-problem A_pp by algebraic
multigrid, then smooth the full system.  Readings for what the paper leaves
to its cited CPR paper:
  * Quasi-IMPES: w_i = D_i^-T e_0 / (D_i^-1)_00 for the diagonal block D_i of
    cell i; row 0 of every block in block-row i becomes w_i^T A_ij and the
    other rows are kept, giving A~ = W A.  A_p[i][j] = (A~_ij)_00.  If
    |(D_i^-1)_00| <= 1e-300 the cell keeps w_i = e_0.
  * Multigrid: 2x2x2 piecewise-constant aggregation (a grid dimension of 1
    stays 1, coarse size ceil(n/2)), Galerkin A_c = P^T A P, coarsen while a
    level has more than `coarsest` cells, LU solve on the last level;
    V(1,1) cycle (V(pre, post) as an option) with a zero initial guess,
    red-black Gauss-Seidel (each pre-sweep red then black; each post-sweep
    black then red), prolongation x += alpha P e.
    Red cells have (i+j+k) even.
  * Full-system stage: block ILU(0) of A~ in red-then-black order.  The
    7-point graph has no triangles, so ILU(0) keeps the off-diagonal blocks
    and only modifies the diagonal: D'_i = A~_ii - sum over lower-coloured
    neighbours k of A~_ik D'_k^-1 A~_ki (the test suite checks this against
    a textbook dense block ILU(0)).
  * Composition: r~ = v with r~_0 = w^T v; dp = Vcycle(r~_0);
    r2 = r~ - A~(:, p) dp; y = ILU^-1 r2; z = y + e_0 dp.
  * ABF decoupling (the alternative the paper names): W_i = D_i^-1 for the
    diagonal block D_i, A~ = W A (every diagonal block becomes I), r~ = W v,
    A_p[i][j] = (A~_ij)_00.  The paper's CPR-FPF is defined in its cited
    reference, which is not part of the paper; it is read here as the
    multiplicative F-P-F composition of the same two stages:
    z1 = ILU^-1 r~, then the P-then-F correction of r1 = r~ - A~ z1,
    z = z1 + that correction, so I - M^-1 A = (I - F A~)(I - C A~)(I - F A~)
    with F = ILU^-1 and C = e_0 Vcycle e_0^T.
"""
import numpy as np
import scipy.linalg
import scipy.sparse as sp

from .model import DIRS, OPP


def shift(x, d):
    """y[cell] = x[neighbour d of cell], zero where the neighbour is outside.
    x has trailing shape (nz, ny, nx)."""
    if d == 0:
        return x.copy()
    di, dj, dk = DIRS[d]
    y = np.zeros_like(x)
    ax, step = (-1, di) if di else ((-2, dj) if dj else (-3, dk))
    n = x.shape[ax]
    src = [slice(None)] * x.ndim
    dst = [slice(None)] * x.ndim
    if step > 0:
        dst[ax], src[ax] = slice(0, n - 1), slice(1, n)
    else:
        dst[ax], src[ax] = slice(1, n), slice(0, n - 1)
    y[tuple(dst)] = x[tuple(src)]
    return y


def colour(shape):
    """0 for red ((i+j+k) even), 1 for black."""
    nz, ny, nx = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return (i + j + k) & 1


def block_spmv(J, x):
    """y = A x for the 7-point block matrix J[7, b, b, grid] and x[b, grid]."""
    b = J.shape[1]
    y = np.zeros_like(x)
    for d in range(7):
        xs = shift(x, d)
        for r in range(b):
            for c in range(b):
                y[r] += J[d, r, c] * xs[c]
    return y


def scalar_spmv(A, x):
    """y = A x for a scalar 7-point stencil A[7, grid]."""
    y = np.zeros_like(x)
    for d in range(7):
        y += A[d] * shift(x, d)
    return y


def to_sparse(A):
    """scipy CSR matrix of a scalar 7-point stencil (natural order)."""
    shape = A.shape[1:]
    n = int(np.prod(shape))
    idx = np.arange(n).reshape(shape)
    rows, cols, vals = [], [], []
    for d in range(7):
        nb = shift(idx.astype(np.float64) + 1.0, d) - 1.0   # -1 where outside
        ok = nb >= 0
        rows.append(idx[ok]); cols.append(nb[ok].astype(np.int64)); vals.append(A[d][ok])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


def block_to_dense(J):
    """Dense matrix of a block 7-point operator, point-block ordered:
    unknown (cell, r) at row cell*b + r (natural cell order)."""
    b = J.shape[1]
    shape = J.shape[3:]
    n = int(np.prod(shape))
    idx = np.arange(n).reshape(shape)
    M = np.zeros((n * b, n * b))
    for d in range(7):
        nb = shift(idx.astype(np.float64) + 1.0, d) - 1.0
        for cell in range(n):
            kk = np.unravel_index(cell, shape)
            t = int(nb[kk])
            if t < 0:
                continue
            M[cell * b:(cell + 1) * b, t * b:(t + 1) * b] = J[(d, slice(None), slice(None)) + kk]
    return M


# ---------------------------------------------------------------- quasi-IMPES

def quasi_impes(J):
    """Decoupling weights w[b, grid] and row 0 of every decoupled block,
    R0[7, b, grid] = w_i^T J[d, :, :, i]."""
    b = J.shape[1]
    shape = J.shape[3:]
    D = np.moveaxis(J[0], (0, 1), (-2, -1))          # (grid, b, b)
    e0 = np.zeros(shape + (b,))
    e0[..., 0] = 1.0
    y = np.linalg.solve(np.swapaxes(D, -1, -2), e0[..., None])[..., 0]   # D^-T e0
    y0 = y[..., 0]
    bad = ~(np.abs(y0) > 1e-300)
    w = np.where(bad[..., None], e0, y / np.where(bad, 1.0, y0)[..., None])
    w = np.moveaxis(w, -1, 0)                         # (b, grid)
    R0 = np.zeros((7, b) + shape)
    for d in range(7):
        for c in range(b):
            for r in range(b):
                R0[d, c] += w[r] * J[d, r, c]
    return w, R0, int(bad.sum())


def decoupled_blocks(J, R0):
    """A~ = W A as a full block array: row 0 from R0, other rows from J."""
    At = J.copy()
    At[:, 0] = R0
    return At


# ---------------------------------------------------------------- multigrid

def coarse_shape(shape):
    return tuple((n + 1) // 2 for n in shape)


def prolongator(shape):
    """Piecewise-constant P (fine x coarse) for 2x2x2 aggregation."""
    nz, ny, nx = shape
    cz, cy, cx = coarse_shape(shape)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    agg = (i // 2) + cx * ((j // 2) + cy * (k // 2))
    n = nx * ny * nz
    return sp.csr_matrix((np.ones(n), (np.arange(n), agg.ravel())), shape=(n, cx * cy * cz))


def from_sparse(M, shape):
    """Scalar 7-point stencil array from a sparse matrix that has no entries
    outside the 7-point pattern (asserted)."""
    n = int(np.prod(shape))
    M = M.tocsr()
    A = np.zeros((7,) + shape)
    idx = np.arange(n).reshape(shape)
    taken = 0
    for d in range(7):
        nb = (shift(idx.astype(np.float64) + 1.0, d) - 1.0).astype(np.int64)
        ok = nb >= 0
        vals = np.asarray(M[idx[ok], nb[ok]]).ravel()
        A[d][ok] = vals
        taken += int(ok.sum())
    assert M.nnz <= taken, "Galerkin operator left the 7-point pattern"
    return A


def mg_setup(Ap, coarsest=512, pre=1, post=1):
    """Hierarchy [(A_l, shape_l)]; the last level is factorised by LU.
    pre / post: red-black Gauss-Seidel sweeps before and after the coarse
    correction (V(pre, post))."""
    levels = [Ap]
    while int(np.prod(levels[-1].shape[1:])) > coarsest:
        A = levels[-1]
        shape = A.shape[1:]
        P = prolongator(shape)
        Ac = (P.T @ to_sparse(A) @ P)
        levels.append(from_sparse(Ac, coarse_shape(shape)))
    last = levels[-1]
    lu = scipy.linalg.lu_factor(to_sparse(last).toarray())
    return {"levels": levels, "lu": lu, "pre": pre, "post": post}


def gs_half_sweep(A, r, x, col, which):
    """One red (which=0) or black (which=1) Gauss-Seidel half-sweep: for
    cells of that colour x_i = (r_i - sum_{j != i} a_ij x_j) / a_ii."""
    off = np.zeros_like(x)
    for d in range(1, 7):
        off += A[d] * shift(x, d)
    m = col == which
    x[m] = (r[m] - off[m]) / A[0][m]


def vcycle(mg, r, level=0, alpha=1.0):
    """V(pre, post) cycle (default V(1,1)) with a zero initial guess on
    level `level`: each pre-sweep is red then black, each post-sweep black
    then red."""
    levels = mg["levels"]
    A = levels[level]
    shape = A.shape[1:]
    if level == len(levels) - 1:
        return scipy.linalg.lu_solve(mg["lu"], r.ravel()).reshape(shape)
    col = colour(shape)
    x = np.zeros_like(r)
    for _ in range(mg.get("pre", 1)):
        gs_half_sweep(A, r, x, col, 0)
        gs_half_sweep(A, r, x, col, 1)
    res = r - scalar_spmv(A, x)
    P = prolongator(shape)
    rc = (P.T @ res.ravel()).reshape(coarse_shape(shape))
    ec = vcycle(mg, rc, level + 1, alpha)
    x += alpha * (P @ ec.ravel()).reshape(shape)
    for _ in range(mg.get("post", 1)):
        gs_half_sweep(A, r, x, col, 1)
        gs_half_sweep(A, r, x, col, 0)
    return x


# ---------------------------------------------------------------- block ILU(0)

def _inv_blocks(D):
    """Inverse of every b x b block, D shaped (b, b, grid); LAPACK LU with
    partial pivoting.  Raises FloatingPointError on a singular block."""
    Dm = np.moveaxis(D, (0, 1), (-2, -1))
    if not np.all(np.isfinite(Dm)):
        raise FloatingPointError("non-finite diagonal block")
    try:
        inv = np.linalg.inv(Dm)
    except np.linalg.LinAlgError as e:
        raise FloatingPointError("singular diagonal block") from e
    return np.moveaxis(inv, (-2, -1), (0, 1))


def _bmv(M, v):
    """Per-cell block matrix-vector product M[b,b,grid] v[b,grid]."""
    return np.einsum("rc...,c...->r...", M, v)


def _bmm(A, B):
    return np.einsum("rk...,kc...->rc...", A, B)


def ilu_setup(At):
    """Modified diagonals of the red-black block ILU(0); returns D'^-1."""
    shape = At.shape[3:]
    col = colour(shape)
    red, black = col == 0, col == 1
    Dinv = _inv_blocks(At[0])                       # red: D' = A~_ii
    Dp = At[0].copy()
    for d in range(1, 7):
        # A~_ik D'_k^-1 A~_ki with k = neighbour d of i; k is red for black i
        Aik = At[d]
        Dk_inv = np.stack([np.stack([shift(Dinv[r, c], d) for c in range(Dinv.shape[1])])
                           for r in range(Dinv.shape[0])])
        Aki = np.stack([np.stack([shift(At[OPP[d], r, c], d) for c in range(At.shape[2])])
                        for r in range(At.shape[1])])
        corr = _bmm(_bmm(Aik, Dk_inv), Aki)
        Dp[:, :, black] -= corr[:, :, black]
    Dinv_black = _inv_blocks(Dp)
    Dinv[:, :, black] = Dinv_black[:, :, black]
    return Dinv


def ilu_apply(At, Dinv, r):
    """Solve (D'+L) D'^-1 (D'+U) z = r: forward over red then black, backward
    over black then red."""
    shape = r.shape[1:]
    col = colour(shape)
    red, black = col == 0, col == 1

    def offdiag(v):
        s = np.zeros_like(v)
        for d in range(1, 7):
            s += _bmv(At[d], np.stack([shift(v[c], d) for c in range(v.shape[0])]))
        return s

    y = np.zeros_like(r)
    y[:, red] = _bmv(Dinv, r)[:, red]
    t = r - offdiag(y)                 # y is zero on black, so only red neighbours count
    y[:, black] = _bmv(Dinv, t)[:, black]
    z = y.copy()
    zb = np.where(black, z, 0.0)
    u = offdiag(zb)                    # upper neighbours of red cells are black
    z[:, red] = y[:, red] - _bmv(Dinv, u)[:, red]
    return z


# ------------------------------------------- block ILU(0) in a general order

def _neighbours(shape):
    """nbr[d, cell] = natural index of neighbour d of each cell, -1 outside."""
    nz, ny, nx = shape
    n = nx * ny * nz
    cells = np.arange(n)
    i, j, k = cells % nx, (cells // nx) % ny, cells // (nx * ny)
    nbr = np.full((7, n), -1)
    nbr[0] = cells
    for d in range(1, 7):
        di, dj, dk = DIRS[d]
        ok = (i + di >= 0) & (i + di < nx) & (j + dj >= 0) & (j + dj < ny) & (k + dk >= 0) & (k + dk < nz)
        nbr[d, ok] = (cells + di + nx * dj + nx * ny * dk)[ok]
    return nbr


def _wavefronts(nbr, r, earlier):
    """Wavefront number of every cell: 0 without a neighbour that comes
    before it (earlier=True: lower rank; False: higher rank), else one more
    than the latest such neighbour's.  Cells of one wavefront do not depend
    on each other, so taking them together gives the sequential result."""
    n = r.size
    dep = [(nbr[d] >= 0) & ((r[np.maximum(nbr[d], 0)] < r) if earlier else (r[np.maximum(nbr[d], 0)] > r))
           for d in range(1, 7)]
    lev = np.zeros(n, dtype=np.int64)
    while True:
        new = np.zeros(n, dtype=np.int64)
        for d in range(1, 7):
            m = dep[d - 1]
            new[m] = np.maximum(new[m], lev[nbr[d + 0][m]] + 1)
        if np.array_equal(new, lev):
            return lev, dep
        lev = new


def ordered_ilu_setup(At, rank):
    """Block ILU(0) of A~ with the cells eliminated in the order of `rank`
    (grid-shaped, distinct integers, lower first).  The paper's potential
    reordering (Sec. 4, Example 2) is one such order; the tiled red-black
    order of tile_rank is another.  On the 7-point graph (no triangles)
    ILU(0) in any order keeps the off-diagonal blocks and only changes the
    diagonal: D'_i = A~_ii - sum over neighbours k ranked before i, in
    direction order, of A~_ik D'_k^-1 A~_ki.  Cells are taken wavefront by
    wavefront (see _wavefronts), which is the sequential order's result.
    Returns the factor for ordered_ilu_apply."""
    b = At.shape[1]
    shape = At.shape[3:]
    n = int(np.prod(shape))
    Ab = np.moveaxis(At.reshape(7, b, b, n), 3, 1)           # [7][n][b][b]
    nbr = _neighbours(shape)
    r = np.asarray(rank).ravel()
    lev, low = _wavefronts(nbr, r, True)
    ulev, up = _wavefronts(nbr, r, False)
    Dinv = np.zeros((n, b, b))
    for L in range(lev.max() + 1):
        c = np.where(lev == L)[0]
        D = Ab[0, c].copy()
        for d in range(1, 7):
            m = low[d - 1][c]
            cc, q = c[m], nbr[d, c[m]]
            D[m] -= Ab[d, cc] @ Dinv[q] @ Ab[OPP[d], q]
        Dinv[c] = np.moveaxis(_inv_blocks(np.moveaxis(D, 0, -1)), -1, 0)
    return {"Ab": Ab, "nbr": nbr, "lev": lev, "low": low, "ulev": ulev, "up": up, "Dinv": Dinv,
            "shape": (b,) + tuple(shape)}


def ordered_ilu_apply(fac, rhs):
    """Solve (D'+L) D'^-1 (D'+U) z = r for the factor of ordered_ilu_setup:
    forward y_i = D'_i^-1 (r_i - sum over earlier neighbours A~_ik y_k),
    backward z_i = y_i - D'_i^-1 sum over later neighbours A~_ik z_k, each
    wavefront by wavefront (forward in rank order, backward in reverse)."""
    Ab, nbr, Dinv = fac["Ab"], fac["nbr"], fac["Dinv"]
    b = Ab.shape[2]
    rv = rhs.reshape(b, -1).T                                # [n][b]
    y = np.zeros_like(rv)
    for L in range(fac["lev"].max() + 1):
        c = np.where(fac["lev"] == L)[0]
        t = rv[c].copy()
        for d in range(1, 7):
            m = fac["low"][d - 1][c]
            t[m] -= np.einsum("nrc,nc->nr", Ab[d, c[m]], y[nbr[d, c[m]]])
        y[c] = np.einsum("nrc,nc->nr", Dinv[c], t)
    z = y.copy()
    for L in range(fac["ulev"].max() + 1):
        c = np.where(fac["ulev"] == L)[0]
        u = np.zeros((c.size, b))
        for d in range(1, 7):
            m = fac["up"][d - 1][c]
            u[m] += np.einsum("nrc,nc->nr", Ab[d, c[m]], z[nbr[d, c[m]]])
        z[c] = y[c] - np.einsum("nrc,nc->nr", Dinv[c], u)
    return z.T.reshape(fac["shape"])


def tile_rank(shape):
    """The tiled red-black order: tiles of 1 x 2 x 2 cells (one cell in x,
    two in y and z), coloured red or black by the parity of (i + j // 2 +
    k // 2) so that face-neighbouring tiles differ; every red tile comes
    before every black tile, and inside a tile the cells follow the natural
    order (y before z).  Red-black is the case of one-cell tiles."""
    nz, ny, nx = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    tj, tk = j // 2, k // 2
    colour = (i + tj + tk) & 1
    tile = i + nx * (tj + ((ny + 1) // 2) * tk)
    ntiles = nx * ((ny + 1) // 2) * ((nz + 1) // 2)
    return (colour * ntiles + tile) * 4 + (j % 2) + 2 * (k % 2)


def potential_rank(p, depth, rho, g=9.80665):
    """Ranks of the cells by decreasing potential p - rho g depth (bar, with
    rho in kg/m^3 and depth in m): upstream cells first."""
    phi = np.asarray(p, dtype=np.float64) - rho * g * np.asarray(depth) * 1e-5
    order = np.argsort(-phi.ravel(), kind="stable")
    rank = np.empty(order.size, dtype=np.int64)
    rank[order] = np.arange(order.size)
    return rank.reshape(np.shape(p))


# ---------------------------------------------------------------- CPR

def abf(J):
    """Alternate block factorisation decoupling (named beside quasi-IMPES in
    Sec. 2.5): W_i = D_i^-1, the inverse of the cell's diagonal block, and
    A~_ij = D_i^-1 A_ij for every block of the row, so A~_ii = I."""
    W = _inv_blocks(J[0])
    At = np.stack([_bmm(W, J[d]) for d in range(7)])
    return W, At


def _ilu(pc, ilu_order):
    """Adds the block ILU(0) of pc["At"] in the given order: "red-black"
    (ilu_setup) or "tiles" (tile_rank through ordered_ilu_setup; its D'^-1
    is also stored as pc["Dinv"] in the [b][b][grid] layout)."""
    At = pc["At"]
    if ilu_order == "red-black":
        pc["Dinv"] = ilu_setup(At)
    elif ilu_order == "tiles":
        fac = ordered_ilu_setup(At, tile_rank(At.shape[3:]))
        pc["ilu_fac"] = fac
        pc["Dinv"] = np.moveaxis(fac["Dinv"], 0, -1).reshape(At.shape[1:3] + At.shape[3:])
    else:
        raise ValueError(ilu_order)
    pc["ilu_order"] = ilu_order
    return pc


def ilu_solve(pc, r):
    """The second stage's ILU(0) solve in the order chosen at setup."""
    if pc.get("ilu_order", "red-black") == "tiles":
        return ordered_ilu_apply(pc["ilu_fac"], r)
    return ilu_apply(pc["At"], pc["Dinv"], r)


def cpr_setup(J, coarsest=512, decoupling="qimpes", pre=1, post=1, ilu_order="red-black"):
    """CPR preconditioner data: decoupling (quasi-IMPES weights w and rows R0,
    or ABF blocks W), the decoupled blocks A~, the pressure multigrid on
    A_p = A~[:, 0, 0] and the block ILU(0) of A~ (red-black order, or the
    tiled red-black order of tile_rank)."""
    if decoupling == "abf":
        W, At = abf(J)
        mg = mg_setup(At[:, 0, 0].copy(), coarsest, pre, post)
        return _ilu({"decoupling": "abf", "W": W, "At": At, "mg": mg, "nbad": 0}, ilu_order)
    w, R0, nbad = quasi_impes(J)
    At = decoupled_blocks(J, R0)
    mg = mg_setup(R0[:, 0].copy(), coarsest, pre, post)
    return _ilu({"decoupling": "qimpes", "w": w, "R0": R0, "At": At, "mg": mg, "nbad": nbad}, ilu_order)


def decouple(pc, v):
    """r~ = W v: quasi-IMPES combines the rows into row 0 and keeps the
    others; ABF multiplies every cell's rows by D_i^-1."""
    if pc["decoupling"] == "abf":
        return _bmv(pc["W"], v)
    rt = v.copy()
    rt[0] = np.sum(pc["w"] * v, axis=0)
    return rt


def _two_stage(pc, rt, alpha):
    """Pressure stage then full-system stage on a decoupled residual rt:
    dp = V-cycle(rt_p); y = ILU^-1 (rt - A~(:, p) dp); y + e0 dp."""
    At = pc["At"]
    dp = vcycle(pc["mg"], rt[0], 0, alpha)
    r2 = rt.copy()
    for d in range(7):
        sdp = shift(dp, d)
        for r in range(rt.shape[0]):
            r2[r] -= At[d, r, 0] * sdp
    y = ilu_solve(pc, r2)
    y[0] += dp
    return y


def cpr_apply(pc, v, alpha=1.0, composition="two-stage"):
    """z = M^-1 v.  Two-stage (P then F): the pressure correction of the
    decoupled residual, then block ILU(0) on what it leaves.  FPF (the
    paper's CPR-FPF, Sec. 2.5, read as the multiplicative three-stage
    composition): z1 = ILU^-1 r~; the two-stage correction of the remaining
    decoupled residual r1 = r~ - A~ z1 (pressure stage, then ILU of what
    that leaves); z = z1 + that correction."""
    rt = decouple(pc, v)
    if composition == "fpf":
        At = pc["At"]
        z1 = ilu_solve(pc, rt)
        r1 = rt - block_spmv(At, z1)
        return z1 + _two_stage(pc, r1, alpha)
    return _two_stage(pc, rt, alpha)
