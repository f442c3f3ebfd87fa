"""Pins of the oracle's preconditioner and Krylov solver against dense linear
algebra, closed forms and textbook special cases."""
import numpy as np
import pytest
import scipy.linalg

from oracle import cpr, krylov, model, newton
from paper_1606_00548_amd import synth
from tests.dense import dense_from_blocks, dense_from_stencil, from_pointblock, to_pointblock


def _system(maker, seed=5):
    case = maker()
    x = synth.random_state_perturbation(case, seed)
    R, J = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"],
                          case["wells"], case["x_old"], x, case["dt"])
    return case, J, -R


def test_block_spmv_matches_dense():
    _, J, b = _system(lambda: synth.black_oil_layered(5, 4, 3, seed=40))
    M = dense_from_blocks(J)
    y = cpr.block_spmv(J, b)
    assert np.allclose(to_pointblock(y), M @ to_pointblock(b), rtol=1e-13, atol=1e-12)


def test_quasi_impes_decouples_the_diagonal():
    _, J, _ = _system(lambda: synth.black_oil_layered(4, 4, 3, seed=41))
    w, R0, nbad = cpr.quasi_impes(J)
    assert nbad == 0
    assert np.all(w[0] == 1.0)
    D = J[0]
    scale = np.abs(D).max(axis=(0, 1))
    # row 0 of the decoupled diagonal block has no saturation coupling
    for s in range(1, J.shape[1]):
        assert np.all(np.abs(R0[0, s]) <= 1e-13 * scale)
    # and its pressure entry is the Schur complement d_pp - D_ps D_ss^-1 D_sp
    Dm = np.moveaxis(D, (0, 1), (-2, -1))
    schur = Dm[..., 0, 0] - np.einsum("...i,...i->...", Dm[..., 0, 1:],
                                      np.linalg.solve(Dm[..., 1:, 1:], Dm[..., 1:, 0][..., None])[..., 0])
    assert np.allclose(R0[0, 0], schur, rtol=1e-11)


def test_galerkin_closed_form_uniform_single_phase():
    # T + diag(acc) on a uniform grid: each coarse face collects the 4 fine
    # faces between two 2x2x2 aggregates, and (since T 1 = 0) a coarse row
    # sum is the sum of its 8 fine accumulation terms.
    case = synth.single_phase_uniform(8, 8, 8)
    case["fluid"] = dict(case["fluid"], c_w=0.0)
    x = synth.initial_state(case["grid"], case["fluid"])
    _, J = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], [],
                          x, x, 1.0)
    A = J[:, 0, 0]
    mg = cpr.mg_setup(A, coarsest=64)
    Ac = mg["levels"][1]
    assert Ac.shape == (7, 4, 4, 4)
    tx = A[2][0, 0, 0]
    assert np.allclose(Ac[2][:, :, :-1], 4 * tx, rtol=1e-13)
    acc = A.sum(axis=0)
    agg = acc.reshape(4, 2, 4, 2, 4, 2).sum(axis=(1, 3, 5))
    assert np.allclose(Ac.sum(axis=0), agg, rtol=1e-9, atol=1e-12 * np.abs(Ac).max())


def test_galerkin_matches_dense_triple_product():
    rng = np.random.default_rng(2)
    shape = (3, 5, 6)
    A = rng.uniform(-1, 0, (7,) + shape)
    A[0] = 7.0
    # zero the couplings that leave the grid
    A[1][:, :, 0] = A[2][:, :, -1] = A[3][:, 0, :] = A[4][:, -1, :] = A[5][0] = A[6][-1] = 0
    mg = cpr.mg_setup(A, coarsest=1)
    Ac = mg["levels"][1]
    nz, ny, nx = shape
    cz, cy, cx = 2, 3, 3
    P = np.zeros((nx * ny * nz, cx * cy * cz))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                P[i + nx * (j + ny * k), i // 2 + cx * (j // 2 + cy * (k // 2))] = 1.0
    ref = P.T @ dense_from_stencil(A) @ P
    assert np.allclose(dense_from_stencil(Ac), ref, rtol=1e-13, atol=1e-13)


def test_red_half_sweep_zeroes_red_residuals():
    _, J, b = _system(lambda: synth.oil_water_lognormal(6, 6, 4, seed=42))
    A = J[:, 0, 0]
    r = b[0]
    col = cpr.colour(r.shape)
    x = np.random.default_rng(1).standard_normal(r.shape)
    cpr.gs_half_sweep(A, r, x, col, 0)
    res = r - cpr.scalar_spmv(A, x)
    assert np.abs(res[col == 0]).max() <= 1e-13 * np.abs(r).max()
    assert np.abs(res[col == 1]).max() > 1e-6 * np.abs(r).max()


def test_one_level_hierarchy_is_exact():
    _, J, b = _system(lambda: synth.oil_water_lognormal(6, 6, 4, seed=43))
    w, R0, _ = cpr.quasi_impes(J)
    A = R0[:, 0]
    mg = cpr.mg_setup(A, coarsest=10 ** 6)
    assert len(mg["levels"]) == 1
    x = cpr.vcycle(mg, b[0])
    assert np.allclose(dense_from_stencil(A) @ x.ravel(), b[0].ravel(), rtol=1e-10,
                       atol=1e-12 * np.abs(b[0]).max())


def test_vcycle_contracts_on_poisson():
    for n in (16, 32):
        case = synth.single_phase_uniform(n, n, 8)
        x = synth.initial_state(case["grid"], case["fluid"])
        _, J = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], [],
                              x, x, 1.0)
        A = J[:, 0, 0]
        mg = cpr.mg_setup(A, coarsest=64)
        rng = np.random.default_rng(n)
        e = rng.standard_normal(A.shape[1:])
        for _ in range(3):
            e = e - cpr.vcycle(mg, cpr.scalar_spmv(A, e))
        e1 = e - cpr.vcycle(mg, cpr.scalar_spmv(A, e))
        assert np.linalg.norm(e1) < 0.9 * np.linalg.norm(e)


def test_vcycle_without_coarse_correction_is_red_black_gauss_seidel():
    # alpha = 0 leaves only the smoothing: from x = 0, pointwise Gauss-Seidel
    # over the red cells, the black cells (pre-sweep), then the black and the
    # red cells (post-sweep), done here one cell at a time on the dense matrix
    _, J, b = _system(lambda: synth.oil_water_lognormal(6, 4, 4, seed=44))
    A = J[:, 0, 0]
    mg = cpr.mg_setup(A, coarsest=8)
    assert len(mg["levels"]) >= 2
    r = b[0]
    x = cpr.vcycle(mg, r, alpha=0.0)
    M = dense_from_stencil(A)
    col = cpr.colour(r.shape).ravel()
    rr = r.ravel()
    y = np.zeros_like(rr)
    for which in (0, 1, 1, 0):
        for i in np.flatnonzero(col == which):
            y[i] = (rr[i] - (M[i] @ y - M[i, i] * y[i])) / M[i, i]
    assert np.allclose(x.ravel(), y, rtol=1e-12, atol=1e-14 * np.abs(y).max())
    assert not np.allclose(cpr.vcycle(mg, r), x, rtol=1e-3)


def test_coarse_correction_scaling_is_affine_on_two_levels():
    # two levels with an exact coarse solve: the cycle is affine in alpha,
    # x(alpha) = x(0) + alpha (x(1) - x(0)), alpha = 1 is the default cycle,
    # and x(1) - x(0) is the post-smoothing's linear part applied to the
    # prolongated exact coarse correction P A_c^-1 P^T (r - A x_pre)
    _, J, b = _system(lambda: synth.oil_water_lognormal(8, 6, 4, seed=45))
    A = J[:, 0, 0]
    mg = cpr.mg_setup(A, coarsest=100)
    assert len(mg["levels"]) == 2
    r = b[0]
    x0, x1, xa = (cpr.vcycle(mg, r, alpha=a) for a in (0.0, 1.0, 1.25))
    assert np.array_equal(cpr.vcycle(mg, r), x1)
    scale = np.abs(x1).max()
    assert np.allclose(xa, x0 + 1.25 * (x1 - x0), rtol=0, atol=1e-11 * scale)
    # the coarse correction from the dense matrices
    M = dense_from_stencil(A)
    col = cpr.colour(r.shape).ravel()
    P = cpr.prolongator(r.shape).toarray()
    xp = np.zeros(r.size)
    for which in (0, 1):
        for i in np.flatnonzero(col == which):
            xp[i] = (r.ravel()[i] - (M[i] @ xp - M[i, i] * xp[i])) / M[i, i]
    e = P @ np.linalg.solve(P.T @ M @ P, P.T @ (r.ravel() - M @ xp))
    # post-sweep (black then red) acting on a correction, right-hand side 0
    d = e.copy()
    for which in (1, 0):
        for i in np.flatnonzero(col == which):
            d[i] = -(M[i] @ d - M[i, i] * d[i]) / M[i, i]
    assert np.allclose((x1 - x0).ravel(), d, rtol=0, atol=1e-10 * scale)


@pytest.mark.parametrize("nu", [1, 2])
def test_symmetric_vcycle_is_a_symmetric_operator(nu):
    # With post-smoothing in the reverse colour order of pre-smoothing,
    # Galerkin coarse operators and an exact coarsest solve, V(nu, nu) on a
    # symmetric A is a symmetric linear operator (swapping the post-sweep
    # order, or dropping a sweep, breaks the symmetry); more sweeps contract
    # more.
    case = synth.single_phase_uniform(8, 6, 4)
    case["fluid"] = dict(case["fluid"], c_w=0.0)      # constant density: symmetric TPFA
    x = synth.initial_state(case["grid"], case["fluid"])
    rng = np.random.default_rng(5)
    k = np.exp(rng.standard_normal(case["poro"].shape))
    _, J = model.assemble(case["grid"], case["fluid"], np.stack([k, k, k]), case["poro"], [], x, x, 1.0)
    A = J[:, 0, 0]
    assert np.allclose(dense_from_stencil(A), dense_from_stencil(A).T, rtol=1e-12, atol=0)
    mg = cpr.mg_setup(A, coarsest=8, pre=nu, post=nu)
    assert len(mg["levels"]) >= 3
    n = A[0].size
    M = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        M[:, c] = cpr.vcycle(mg, e.reshape(A.shape[1:])).ravel()
    assert np.allclose(M, M.T, rtol=1e-10, atol=1e-12 * np.abs(M).max())
    Ad = dense_from_stencil(A)
    rho = np.abs(np.linalg.eigvals(np.eye(n) - M @ Ad)).max()
    mg1 = cpr.mg_setup(A, coarsest=8)
    M1 = np.stack([cpr.vcycle(mg1, np.eye(n)[c].reshape(A.shape[1:])).ravel() for c in range(n)], axis=1)
    rho1 = np.abs(np.linalg.eigvals(np.eye(n) - M1 @ Ad)).max()
    assert rho < 1.0 and (nu == 1 or rho < rho1)


def _textbook_block_ilu0(M, b, order):
    """Dense block ILU(0) (IKJ variant) of M in the given cell order, keeping
    only the blocks of M's sparsity pattern.  Returns L (unit lower, block)
    and U (upper incl. diagonal) in that order."""
    n = len(order)
    perm = np.concatenate([np.arange(c * b, (c + 1) * b) for c in order])
    A = M[np.ix_(perm, perm)].copy()
    pattern = np.zeros((n, n), dtype=bool)
    for I in range(n):
        for K in range(n):
            pattern[I, K] = np.any(A[I * b:(I + 1) * b, K * b:(K + 1) * b] != 0)
    blk = lambda I, K: (slice(I * b, (I + 1) * b), slice(K * b, (K + 1) * b))
    for I in range(1, n):
        for K in range(I):
            if not pattern[I, K]:
                continue
            A[blk(I, K)] = A[blk(I, K)] @ np.linalg.inv(A[blk(K, K)])
            for Jc in range(K + 1, n):
                if pattern[I, Jc]:
                    A[blk(I, Jc)] -= A[blk(I, K)] @ A[blk(K, Jc)]
    L = np.eye(n * b)
    U = np.zeros_like(A)
    for I in range(n):
        for K in range(n):
            if K < I:
                L[blk(I, K)] = A[blk(I, K)]
            else:
                U[blk(I, K)] = A[blk(I, K)]
    return L, U, perm


@pytest.mark.parametrize("maker", [lambda: synth.oil_water_lognormal(4, 4, 2, seed=44),
                                   lambda: synth.black_oil_layered(4, 4, 2, seed=45)])
def test_red_black_ilu0_matches_textbook(maker):
    _, J, b = _system(maker)
    w, R0, _ = cpr.quasi_impes(J)
    At = cpr.decoupled_blocks(J, R0)
    Dinv = cpr.ilu_setup(At)
    M = dense_from_blocks(At)
    bs = J.shape[1]
    shape = J.shape[3:]
    col = cpr.colour(shape).ravel()
    order = np.concatenate([np.where(col == 0)[0], np.where(col == 1)[0]])
    L, U, perm = _textbook_block_ilu0(M, bs, order)
    # solve with the textbook factors and compare with the oracle's sweeps
    rhs = to_pointblock(b)
    z_tb = np.zeros_like(rhs)
    # U is block upper triangular with full diagonal blocks: general solve
    z_tb[perm] = np.linalg.solve(U, scipy.linalg.solve_triangular(
        L, rhs[perm], lower=True, unit_diagonal=True))
    z = to_pointblock(cpr.ilu_apply(At, Dinv, b))
    assert np.allclose(z, z_tb, rtol=1e-10, atol=1e-12 * np.abs(z_tb).max())
    # LU - A~ is non-zero only between black cells two steps apart
    E = L @ U - M[np.ix_(perm, perm)]
    nz, ny, nx = shape
    coords = [np.unravel_index(c, shape) for c in order]
    for I in range(len(order)):
        for K in range(len(order)):
            e = np.abs(E[I * bs:(I + 1) * bs, K * bs:(K + 1) * bs]).max()
            if e > 1e-12 * np.abs(M).max():
                (k1, j1, i1), (k2, j2, i2) = coords[I], coords[K]
                dist = abs(k1 - k2) + abs(j1 - j2) + abs(i1 - i2)
                assert col[order[I]] == 1 and col[order[K]] == 1 and dist == 2


def test_cpr_single_phase_exact_pressure_solve_is_one_iteration():
    # b = 1: the pressure stage with an exact coarse solve inverts A, so the
    # second stage sees a zero residual and FGMRES converges in one step.
    case = synth.single_phase_uniform(6, 5, 4, wells=[synth.well(0, 0, 4, "inj", 300.0),
                                                       synth.well(5, 4, 4, "prod", 150.0)])
    x = synth.random_state_perturbation(case, 3)
    R, J = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"],
                          case["wells"], case["x_old"], x, case["dt"])
    pc = cpr.cpr_setup(J, coarsest=10 ** 6)
    dx, st = krylov.fgmres(lambda v: cpr.block_spmv(J, v), lambda v: cpr.cpr_apply(pc, v), -R,
                           rtol=1e-10)
    assert st["iterations"] == 1 and st["converged"]


def test_gmres_dense_small_converges_within_n():
    rng = np.random.default_rng(7)
    n = 24
    A = rng.standard_normal((n, n)) + n * np.eye(n) * 0.3
    b = rng.standard_normal(n)
    x, st = krylov.fgmres(lambda v: A @ v, lambda v: v, b, restart=30, rtol=1e-12)
    assert st["iterations"] <= n
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-10)


def test_gmres_k_distinct_eigenvalues_takes_k_steps():
    rng = np.random.default_rng(8)
    eig = np.repeat([1.0, 2.0, 5.0, 9.0, 13.0], 8)
    b = rng.standard_normal(eig.size)
    x, st = krylov.fgmres(lambda v: eig * v, lambda v: v, b, restart=30, rtol=1e-12)
    assert st["iterations"] == 5
    assert np.allclose(x, b / eig, rtol=1e-11)


def test_gmres_restart_and_zero_rhs():
    rng = np.random.default_rng(9)
    n = 60
    A = np.diag(np.linspace(1, 50, n)) + 0.1 * rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    x, st = krylov.fgmres(lambda v: A @ v, lambda v: v, b, restart=5, rtol=1e-8, max_iter=500)
    assert st["converged"] and st["cycles"] > 1
    assert np.linalg.norm(b - A @ x) <= 1e-8 * np.linalg.norm(b)
    x0, st0 = krylov.fgmres(lambda v: A @ v, lambda v: v, np.zeros(n))
    assert st0["iterations"] == 0 and np.all(x0 == 0)
    # max_iter stops early and reports non-convergence with a usable iterate
    x1, st1 = krylov.fgmres(lambda v: A @ v, lambda v: v, b, restart=30, rtol=1e-14, max_iter=3)
    assert st1["iterations"] == 3 and not st1["converged"]
    assert np.linalg.norm(b - A @ x1) < np.linalg.norm(b)


@pytest.mark.parametrize("maker", [lambda: synth.oil_water_lognormal(6, 6, 4, seed=50),
                                   lambda: synth.black_oil_layered(6, 6, 4, seed=51),
                                   lambda: synth.black_oil_channelised(6, 4, 4, seed=52)])
def test_cpr_fgmres_solves_tiny_systems(maker):
    case, J, b = _system(maker)
    pc = cpr.cpr_setup(J, coarsest=16)
    assert len(pc["mg"]["levels"]) >= 2
    x, st = krylov.fgmres(lambda v: cpr.block_spmv(J, v), lambda v: cpr.cpr_apply(pc, v), b)
    assert st["converged"]
    M = dense_from_blocks(J)
    xd = np.linalg.solve(M, to_pointblock(b))
    r = to_pointblock(b) - M @ to_pointblock(x)
    assert np.linalg.norm(r) <= 1e-6 * np.linalg.norm(b)
    cond = np.linalg.cond(M)
    err = np.linalg.norm(to_pointblock(x) - xd) / np.linalg.norm(xd)
    assert err <= cond * 1e-6
    # with a tight tolerance the iterate reaches the dense solution
    x2, _ = krylov.fgmres(lambda v: cpr.block_spmv(J, v), lambda v: cpr.cpr_apply(pc, v), b,
                          rtol=1e-13)
    assert np.allclose(to_pointblock(x2), xd, rtol=1e-8, atol=1e-9 * np.abs(xd).max())


def test_newton_update_chops_and_clamps():
    x = np.array([[200.0, 200.0, 200.0], [0.3, 0.95, 0.1], [0.05, 0.05, 0.05]])
    dx = np.array([[5.0, -3.0, 1.0], [0.5, 0.1, -0.3], [0.01, -0.1, 0.0]])
    xn = newton.newton_update(x[:2], dx[:2])
    assert np.allclose(xn[0], [205.0, 197.0, 201.0])
    assert np.allclose(xn[1], [0.5, 1.0, 0.0])
    xn = newton.newton_update(x, dx, pb_min=50.0)
    assert np.allclose(xn[1], [0.5, 1.0, 0.0])
    # the middle cell's gas would go negative: undersaturated at p_b = p
    assert np.allclose(xn[2], [0.06, -197.0, 0.05])


def test_newton_update_switches_the_black_oil_state():
    # columns: saturated stays, saturated -> undersaturated, undersaturated
    # stays (p_b moves, unchopped), undersaturated -> saturated (p_b > p),
    # p_b floored at the first PVT node, S_g clamped at 1
    x = np.array([[200.0, 200.0, 200.0, 200.0, 60.0, 200.0],
                  [0.3, 0.3, 0.3, 0.3, 0.3, 0.2],
                  [0.1, 0.02, -150.0, -190.0, -55.0, 0.9]])
    dx = np.array([[1.0, 2.0, 3.0, 1.0, -1.0, 0.0],
                   [0.0] * 6,
                   [-0.05, -0.1, -30.0, -12.0, 10.0, 0.5]])
    xn = newton.newton_update(x, dx, pb_min=50.0)
    assert np.allclose(xn[0], [201.0, 202.0, 203.0, 201.0, 59.0, 200.0])
    assert np.allclose(xn[2], [0.05, -202.0, -180.0, 0.0, -50.0, 1.0])


# ---- BiCGSTAB (the paper's Krylov method, Sec. 4)

def test_bicgstab_dense_matches_solve():
    rng = np.random.default_rng(70)
    n = 30
    A = rng.standard_normal((n, n)) + 8.0 * np.eye(n)        # nonsymmetric, well conditioned
    b = rng.standard_normal(n)
    x, st = krylov.bicgstab(lambda v: A @ v, lambda v: v, b, rtol=1e-13)
    xd = np.linalg.solve(A, b)
    assert st["converged"] and np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
    # a preconditioner changes the path, not the limit
    D = np.diag(A).copy()
    x2, st2 = krylov.bicgstab(lambda v: A @ v, lambda v: v / D, b, rtol=1e-13)
    assert st2["converged"] and np.linalg.norm(x2 - xd) <= 1e-10 * np.linalg.norm(xd)


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_bicgstab_k_distinct_eigenvalues_within_k(k):
    # BiCG's residual polynomial annihilates a k-dimensional Krylov space in
    # at most k steps, and BiCGSTAB's residual carries that factor
    rng = np.random.default_rng(71 + k)
    d = np.repeat(np.linspace(1.0, 7.0, k), 4)
    b = rng.standard_normal(d.size)
    x, st = krylov.bicgstab(lambda v: d * v, lambda v: v, b, rtol=1e-10)
    assert st["converged"] and st["iterations"] <= k
    assert np.allclose(x, b / d, rtol=1e-8)


def test_bicgstab_exact_preconditioner_and_zero_rhs():
    rng = np.random.default_rng(76)
    A = rng.standard_normal((12, 12)) + 6.0 * np.eye(12)
    Ai = np.linalg.inv(A)
    b = rng.standard_normal(12)
    x, st = krylov.bicgstab(lambda v: A @ v, lambda v: Ai @ v, b)
    assert st["iterations"] == 1 and st["converged"] and st["true_rel"] <= 1e-12
    x0, st0 = krylov.bicgstab(lambda v: A @ v, lambda v: v, np.zeros(12))
    assert st0["iterations"] == 0 and st0["converged"] and np.all(x0 == 0)
    # max_iter stops early with a usable iterate and no claim of convergence
    x1, st1 = krylov.bicgstab(lambda v: A @ v, lambda v: v, b, rtol=1e-14, max_iter=2)
    assert st1["iterations"] == 2 and not st1["converged"]
    assert np.linalg.norm(b - A @ x1) < np.linalg.norm(b)


@pytest.mark.parametrize("maker", [lambda: synth.oil_water_lognormal(6, 6, 4, seed=50),
                                   lambda: synth.black_oil_layered(6, 6, 4, seed=51)])
def test_cpr_bicgstab_solves_tiny_systems(maker):
    case, J, b = _system(maker)
    pc = cpr.cpr_setup(J, coarsest=16)
    x, st = krylov.bicgstab(lambda v: cpr.block_spmv(J, v), lambda v: cpr.cpr_apply(pc, v), b)
    assert st["converged"]
    M = dense_from_blocks(J)
    xd = np.linalg.solve(M, to_pointblock(b))
    r = to_pointblock(b) - M @ to_pointblock(x)
    assert np.linalg.norm(r) <= 1e-6 * np.linalg.norm(b)
    assert np.linalg.norm(to_pointblock(x) - xd) / np.linalg.norm(xd) <= np.linalg.cond(M) * 1e-6


# ---- ABF decoupling and the CPR-FPF composition (Sec. 2.5)

def _dense_op(f, n, shape):
    """Dense matrix of a linear map given on arrays of `shape`, columns in
    point-block order."""
    M = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        M[:, c] = to_pointblock(f(from_pointblock(e, shape)))
    return M


def test_abf_decoupling_against_dense():
    _, J, _ = _system(lambda: synth.black_oil_layered(4, 3, 3, seed=60))
    W, At = cpr.abf(J)
    b = J.shape[1]
    M = dense_from_blocks(J)
    n = M.shape[0]
    Dbd = np.zeros_like(M)
    for c in range(n // b):
        Dbd[c * b:(c + 1) * b, c * b:(c + 1) * b] = M[c * b:(c + 1) * b, c * b:(c + 1) * b]
    Mt = np.linalg.solve(Dbd, M)                       # (block diag of A)^-1 A
    assert np.allclose(dense_from_blocks(At), Mt, rtol=1e-12, atol=1e-12 * np.abs(Mt).max())
    eye = np.broadcast_to(np.eye(b)[..., None, None, None], At[0].shape)
    assert np.allclose(At[0], eye, atol=1e-12)
    pc = cpr.cpr_setup(J, coarsest=16, decoupling="abf")
    assert np.array_equal(pc["mg"]["levels"][0], At[:, 0, 0])
    # decouple() is W applied to a vector: W A = A~
    shape = (b,) + J.shape[3:]
    Wd = _dense_op(lambda v: cpr.decouple(pc, v), n, shape)
    assert np.allclose(Wd @ M, Mt, rtol=1e-11, atol=1e-11 * np.abs(Mt).max())


@pytest.mark.parametrize("decoupling", ["qimpes", "abf"])
def test_compositions_are_products_of_stage_error_propagators(decoupling):
    # With F = ILU(0)^-1 of A~ and C = e0 Vcycle e0^T, multiplicative stages
    # give I - M^-1 A = (I - F A~)(I - C A~) for P-then-F and
    # (I - F A~)(I - C A~)(I - F A~) for F-P-F, where M^-1 = B W.
    _, J, _ = _system(lambda: synth.black_oil_layered(4, 3, 2, seed=61))
    pc = cpr.cpr_setup(J, coarsest=4, decoupling=decoupling)
    assert len(pc["mg"]["levels"]) >= 2
    b = J.shape[1]
    shape = (b,) + J.shape[3:]
    M = dense_from_blocks(J)
    n = M.shape[0]
    Mt = dense_from_blocks(pc["At"])
    F = _dense_op(lambda v: cpr.ilu_apply(pc["At"], pc["Dinv"], v), n, shape)

    def coarse(v):
        z = np.zeros_like(v)
        z[0] = cpr.vcycle(pc["mg"], v[0])
        return z
    C = _dense_op(coarse, n, shape)
    I = np.eye(n)
    EF, EC = I - F @ Mt, I - C @ Mt
    for comp, expect in (("two-stage", EF @ EC), ("fpf", EF @ EC @ EF)):
        Minv = _dense_op(lambda v: cpr.cpr_apply(pc, v, composition=comp), n, shape)
        E = I - Minv @ M
        assert np.allclose(E, expect, atol=1e-9 * max(1.0, np.abs(expect).max())), comp
    # the extra smoothing stage contracts more on this system
    rho2 = np.abs(np.linalg.eigvals(EF @ EC)).max()
    rho3 = np.abs(np.linalg.eigvals(EF @ EC @ EF)).max()
    assert rho3 < rho2 < 1.0


@pytest.mark.parametrize("decoupling", ["qimpes", "abf"])
@pytest.mark.parametrize("composition", ["two-stage", "fpf"])
def test_block_diagonal_system_is_inverted_exactly(decoupling, composition):
    _, J, b = _system(lambda: synth.oil_water_lognormal(4, 4, 2, seed=62))
    Jd = J.copy()
    Jd[1:] = 0.0
    pc = cpr.cpr_setup(Jd, coarsest=4, decoupling=decoupling)
    z = cpr.cpr_apply(pc, b, composition=composition)
    assert np.allclose(cpr.block_spmv(Jd, z), b, rtol=1e-10, atol=1e-10 * np.abs(b).max())


@pytest.mark.parametrize("composition", ["two-stage", "fpf"])
def test_abf_single_phase_exact_pressure_solve_is_one_iteration(composition):
    # b = 1: ABF divides each row by its diagonal; with an exact coarse
    # solve the pressure stage inverts A~ and FGMRES needs one step.
    case = synth.single_phase_uniform(6, 5, 4, wells=[synth.well(0, 0, 4, "inj", 300.0),
                                                       synth.well(5, 4, 4, "prod", 150.0)])
    x = synth.random_state_perturbation(case, 3)
    R, J = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"],
                          case["wells"], case["x_old"], x, case["dt"])
    pc = cpr.cpr_setup(J, coarsest=10 ** 6, decoupling="abf")
    assert np.allclose(pc["At"][0], 1.0)
    dx, st = krylov.fgmres(lambda v: cpr.block_spmv(J, v),
                           lambda v: cpr.cpr_apply(pc, v, composition=composition), -R, rtol=1e-10)
    assert st["iterations"] == 1 and st["converged"]


@pytest.mark.parametrize("maker", [lambda: synth.oil_water_lognormal(6, 6, 4, seed=50),
                                   lambda: synth.black_oil_layered(6, 6, 4, seed=51),
                                   lambda: synth.black_oil_channelised(6, 4, 4, seed=52)])
@pytest.mark.parametrize("decoupling,composition", [("abf", "two-stage"), ("qimpes", "fpf"),
                                                    ("abf", "fpf")])
def test_cpr_variants_solve_tiny_systems(maker, decoupling, composition):
    case, J, b = _system(maker)
    pc = cpr.cpr_setup(J, coarsest=16, decoupling=decoupling)
    M = dense_from_blocks(J)
    xd = np.linalg.solve(M, to_pointblock(b))
    for solve in (krylov.fgmres, krylov.bicgstab):
        x, st = solve(lambda v: cpr.block_spmv(J, v),
                      lambda v: cpr.cpr_apply(pc, v, composition=composition), b)
        assert st["converged"]
        r = to_pointblock(b) - M @ to_pointblock(x)
        assert np.linalg.norm(r) <= 1e-6 * np.linalg.norm(b)
        assert np.linalg.norm(to_pointblock(x) - xd) / np.linalg.norm(xd) <= np.linalg.cond(M) * 1e-6


@pytest.mark.parametrize("maker", [lambda: synth.oil_water_lognormal(4, 4, 2, seed=46),
                                   lambda: synth.black_oil_layered(4, 3, 2, seed=47)])
@pytest.mark.parametrize("ordering", ["natural", "random", "potential", "tiles"])
def test_ordered_ilu0_matches_textbook(maker, ordering):
    # the block ILU(0) in a general elimination order (the paper's potential
    # reordering) against the dense textbook factorisation in that order
    case, J, b = _system(maker)
    w, R0, _ = cpr.quasi_impes(J)
    At = cpr.decoupled_blocks(J, R0)
    shape = J.shape[3:]
    n = int(np.prod(shape))
    if ordering == "natural":
        rank = np.arange(n).reshape(shape)
    elif ordering == "random":
        rank = np.random.default_rng(5).permutation(n).reshape(shape)
    elif ordering == "tiles":
        rank = cpr.tile_rank(shape)
    else:
        depth = case["grid"]["top"] + case["grid"]["dz"] * (np.arange(shape[0])[:, None, None] + 0.5)
        rank = cpr.potential_rank(case["x"][0], np.broadcast_to(depth, shape), 800.0)
    fac = cpr.ordered_ilu_setup(At, rank)
    order = np.argsort(rank.ravel(), kind="stable")
    L, U, perm = _textbook_block_ilu0(dense_from_blocks(At), J.shape[1], order)
    rhs = to_pointblock(b)
    z_tb = np.zeros_like(rhs)
    z_tb[perm] = np.linalg.solve(U, scipy.linalg.solve_triangular(L, rhs[perm], lower=True, unit_diagonal=True))
    z = to_pointblock(cpr.ordered_ilu_apply(fac, b))
    assert np.allclose(z, z_tb, rtol=1e-10, atol=1e-12 * np.abs(z_tb).max())


def test_ordered_ilu0_in_red_black_order_is_the_red_black_ilu0():
    case = synth.black_oil_layered(8, 6, 4, seed=48)
    R, J = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                          case["x_old"], case["x"], case["dt"])
    w, R0, _ = cpr.quasi_impes(J)
    At = cpr.decoupled_blocks(J, R0)
    col = cpr.colour(At.shape[3:])
    rank = col * col.size + np.arange(col.size).reshape(col.shape)
    fac = cpr.ordered_ilu_setup(At, rank)
    D = cpr.ilu_setup(At)
    assert np.allclose(np.moveaxis(D.reshape(3, 3, -1), 2, 0), fac["Dinv"], rtol=1e-13, atol=0)
    z1, z2 = cpr.ilu_apply(At, D, -R), cpr.ordered_ilu_apply(fac, -R)
    assert np.linalg.norm(z1 - z2) <= 1e-13 * np.linalg.norm(z1)


def test_potential_rank_puts_high_potential_first():
    # nz = 2, ny = 1, nx = 3; the lower layer is 0.5 bar higher in pressure
    # but 10 m deeper, which lowers its potential by rho g dz = 0.98 bar
    p = np.array([[[200.0, 210.0, 205.0]], [[200.5, 210.5, 205.5]]])
    depth = np.array([[[2000.0] * 3], [[2010.0] * 3]])
    rank = cpr.potential_rank(p, depth, 1000.0)
    assert rank.ravel().tolist() == [4, 0, 2, 5, 1, 3]
    rank_flat = cpr.potential_rank(p, np.zeros_like(depth), 1000.0)
    assert rank_flat.ravel().tolist() == [5, 1, 3, 4, 0, 2]


@pytest.mark.parametrize("shape", [(4, 6, 5), (3, 5, 2), (1, 1, 4), (5, 1, 3)])
def test_tile_rank_structure(shape):
    # 1 x 2 x 2 tiles: a tile's cells are consecutive in the order, every red
    # tile precedes every black one, and face neighbours in different tiles
    # have tiles of different colours (so tiles of one colour are independent)
    nz, ny, nx = shape
    rank = cpr.tile_rank(shape)
    assert sorted(rank.ravel().tolist()) == sorted(set(rank.ravel().tolist()))
    tile = lambda i, j, k: (i, j // 2, k // 2)
    colour = lambda i, j, k: (i + j // 2 + k // 2) & 1
    cells = [(i, j, k) for k in range(nz) for j in range(ny) for i in range(nx)]
    for a in cells:
        for b in cells:
            if tile(*a) == tile(*b):
                assert abs(int(rank[a[2], a[1], a[0]]) // 4 - int(rank[b[2], b[1], b[0]]) // 4) == 0
            elif colour(*a) < colour(*b):
                assert rank[a[2], a[1], a[0]] < rank[b[2], b[1], b[0]]
            if sum(abs(x - y) for x, y in zip(a, b)) == 1 and tile(*a) != tile(*b):
                assert colour(*a) != colour(*b)
    # inside a tile: natural order, y before z
    assert rank[0, 0, 0] % 4 == 0
    if ny > 1:
        assert rank[0, 1, 0] % 4 == 1
    if nz > 1:
        assert rank[1, 0, 0] % 4 == 2
