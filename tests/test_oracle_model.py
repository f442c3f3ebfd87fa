"""Pins of the oracle's residual and Jacobian against the paper's printed
closed forms and against physical invariants that hold for any state."""
import copy
import os

import numpy as np
import pytest

from oracle import model, newton
from paper_1606_00548_amd import synth
from tests.dense import dense_from_blocks

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _assemble(case, x=None, dt=None, wells=None):
    return model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"],
                          case["wells"] if wells is None else wells, case["x_old"],
                          case["x"] if x is None else x, case["dt"] if dt is None else dt)


def test_corey_matches_paper_values():
    # eqs. (17)-(18), values in tests/golden/corey_eq17_18.txt
    tab = np.loadtxt(os.path.join(GOLDEN, "corey_eq17_18.txt"))
    krw, _, kro, _ = model.corey(tab[:, 0], 0.2, 0.2)
    assert np.allclose(krw, tab[:, 1], rtol=0, atol=1e-15)
    assert np.allclose(kro, tab[:, 2], rtol=0, atol=1e-15)


def test_corey_derivative_and_clamp():
    s = np.linspace(0.25, 0.75, 11)
    h = 1e-7
    krw, dkrw, kro, dkro = model.corey(s, 0.2, 0.2)
    a, _, c, _ = model.corey(s + h, 0.2, 0.2)
    b, _, d, _ = model.corey(s - h, 0.2, 0.2)
    assert np.allclose(dkrw, (a - b) / (2 * h), rtol=1e-7)
    assert np.allclose(dkro, (c - d) / (2 * h), rtol=1e-7)
    krw, dkrw, kro, dkro = model.corey(np.array([0.0, 0.1, 0.9, 1.0]), 0.2, 0.2)
    assert np.all(krw[:2] == 0) and np.all(dkrw[:2] == 0)
    assert np.all(kro[2:] == 0) and np.all(dkro[2:] == 0)


def test_stone2_reductions():
    # Stone II reduces to the oil-water curve without gas and to the
    # oil-gas curve at connate water (textbook identities of the model).
    sw = np.linspace(0.2, 0.8, 13)
    _, _, _, _, kro, _, _ = model.stone2(sw, np.zeros_like(sw), 0.2, 0.2, 0.7)
    _, _, krow, _ = model.corey(sw, 0.2, 0.2)
    assert np.allclose(kro, krow, rtol=0, atol=1e-15)
    sg = np.linspace(0.0, 0.7, 15)
    _, _, _, _, kro, _, _ = model.stone2(np.full_like(sg, 0.2), sg, 0.2, 0.2, 0.7)
    assert np.allclose(kro, ((0.7 - sg) / 0.7) ** 2, rtol=0, atol=1e-15)
    # clamped at zero where the raw Stone II value is negative
    _, _, _, _, kro, dw, dg = model.stone2(np.array([0.7]), np.array([0.25]), 0.2, 0.2, 0.7)
    assert kro[0] == 0.0 and dw[0] == 0.0 and dg[0] == 0.0


def test_stone2_derivatives():
    rng = np.random.default_rng(1)
    sw = rng.uniform(0.25, 0.5, 20)
    sg = rng.uniform(0.05, 0.3, 20)
    h = 1e-7
    out = model.stone2(sw, sg, 0.2, 0.2, 0.7)
    kro, dw, dg = out[4], out[5], out[6]
    pos = kro > 1e-3
    fw = (model.stone2(sw + h, sg, 0.2, 0.2, 0.7)[4] - model.stone2(sw - h, sg, 0.2, 0.2, 0.7)[4]) / (2 * h)
    fg = (model.stone2(sw, sg + h, 0.2, 0.2, 0.7)[4] - model.stone2(sw, sg - h, 0.2, 0.2, 0.7)[4]) / (2 * h)
    assert np.allclose(dw[pos], fw[pos], rtol=1e-6, atol=1e-9)
    assert np.allclose(dg[pos], fg[pos], rtol=1e-6, atol=1e-9)


def test_pvt_interp_segments():
    tp = np.array([1.0, 2.0, 4.0])
    ty = np.array([10.0, 20.0, 0.0])
    y, dy = model.pvt_interp(tp, ty, np.array([0.0, 1.0, 1.5, 2.0, 3.0, 4.0, 5.0]))
    assert np.allclose(y, [0.0, 10.0, 15.0, 20.0, 10.0, 0.0, -10.0])
    # at a breakpoint the right-hand segment's slope is used
    assert np.allclose(dy, [10.0, 10.0, 10.0, -10.0, -10.0, -10.0, -10.0])


def test_transmissibility_harmonic_and_symmetric():
    grid = synth.grid_of(3, 2, 2)
    perm = np.full((3, 2, 2, 3), 50.0)
    Tx, Ty, Tz = model.transmissibilities(grid, perm)
    # equal permeabilities: the harmonic mean is k, T = k A / d
    k = 50.0 * model.MD
    assert np.allclose(Tx, k * 10.0 * 5.0 / 10.0)
    assert np.allclose(Tz, k * 10.0 * 10.0 / 5.0)
    perm[0, 0, 0, 0] = 10.0
    Tx, _, _ = model.transmissibilities(grid, perm)
    # series resistances: 2A/(d/k1 + d/k2)
    assert np.isclose(Tx[0, 0, 0], 2 * 50.0 / (10.0 / (10.0 * model.MD) + 10.0 / (50.0 * model.MD)))


def test_peaceman_isotropic_radius():
    # Peaceman's equivalent radius of a square isotropic block is ~0.198 dx.
    wi = model.peaceman_wi(100.0, 100.0, 10.0, 10.0, 5.0, 0.1, 0.0)
    ro = 0.1 * np.exp(2 * np.pi * 100.0 * model.MD * 5.0 / wi)
    assert abs(ro / 10.0 - 0.198) < 1e-3
    # anisotropic formula is symmetric under swapping x and y
    a = model.peaceman_wi(100.0, 10.0, 10.0, 20.0, 5.0, 0.1, 0.0)
    b = model.peaceman_wi(10.0, 100.0, 20.0, 10.0, 5.0, 0.1, 0.0)
    assert np.isclose(a, b, rtol=1e-14)


def _two_cell_single_phase():
    case = synth.single_phase_uniform(2, 1, 1)
    fl = dict(case["fluid"], c_w=0.0, c_r=0.0)
    case["fluid"] = fl
    return case


def test_two_cell_flux_closed_form():
    # Darcy, eqs. (1)-(2): mass flow T (rho / mu) (p1 - p2) from the
    # high-pressure cell; with incompressible fluid and rock the accumulation
    # vanishes and R_1 = -R_2 = that flow divided by the row scale.
    case = _two_cell_single_phase()
    x = case["x"].copy()
    x[0, 0, 0, 0] = 210.0
    x[0, 0, 0, 1] = 200.0
    R, J = _assemble(case, x=x)
    T = 100.0 * model.MD * 10.0 * 5.0 / 10.0
    flow = T * 1000.0 / (0.5 * model.CP) * 10.0 * model.BAR
    s = model.row_scales(case["grid"], case["fluid"], case["poro"], 1.0)[0]
    assert np.isclose(R[0, 0, 0, 0], flow / s, rtol=1e-13)
    assert np.isclose(R[0, 0, 0, 1], -flow / s, rtol=1e-13)


def test_single_phase_frozen_mobility_is_symmetric_zero_rowsum():
    # Incompressible single phase, one layer (no gravity): J is the TPFA
    # Laplacian -- symmetric, zero row sums, non-positive off-diagonals.
    case = synth.single_phase_uniform(5, 4, 1)
    case["perm"] = np.exp(np.random.default_rng(3).standard_normal(case["perm"].shape)) * 100
    case["perm"][1] = case["perm"][0]
    case["fluid"] = dict(case["fluid"], c_w=0.0, c_r=0.0)
    x = synth.random_state_perturbation(case, 4)
    _, J = _assemble(case, x=x)
    M = dense_from_blocks(J)
    assert np.allclose(M, M.T, rtol=0, atol=1e-12 * np.abs(M).max())
    assert np.allclose(M.sum(axis=1), 0.0, atol=1e-12 * np.abs(M).max())
    off = M - np.diag(np.diag(M))
    assert np.all(off <= 0.0) and np.all(np.diag(M) > 0)


def test_hydrostatic_column_has_no_flux():
    # Phi = p - rho g z (z depth): an incompressible column initialised
    # hydrostatically with the same density is in equilibrium, R = 0.
    case = synth.single_phase_uniform(2, 2, 6)
    case["fluid"] = dict(case["fluid"], c_w=0.0, c_r=0.0)
    x = synth.initial_state(case["grid"], case["fluid"])
    case["x_old"] = x.copy()
    R, _ = _assemble(case, x=x)
    assert np.abs(R).max() < 1e-9
    # a column that is too light in its lower half flows upward: bottom cells lose mass
    x2 = x.copy()
    x2[0, 3:] += 1.0
    R2, _ = _assemble(case, x=x2)
    assert np.all(R2[0, 3] > 0) and np.all(R2[0, 2] < 0)


@pytest.mark.parametrize("maker", [
    lambda: synth.oil_water_lognormal(5, 4, 3, seed=11),
    lambda: synth.black_oil_layered(4, 4, 3, seed=12),
    lambda: synth.black_oil_channelised(6, 4, 3, seed=13),
])
def test_flux_conservation_any_state(maker):
    # Every face flow leaves one cell and enters its neighbour, so with the
    # accumulation and wells removed the residuals of each component sum to
    # zero, and so do the Jacobian's column sums per component.
    case = maker()
    x = synth.random_state_perturbation(case, 7)
    case["x_old"] = x.copy()
    R, J = _assemble(case, x=x, dt=1e20, wells=[])
    b = R.shape[0]
    M = dense_from_blocks(J)
    acc_free = M.copy()
    # remove the (O(1)) accumulation part: the flux part is scaled by dt
    for c in range(b):
        tot = R[c].sum()
        assert abs(tot) <= 1e-12 * np.abs(R[c]).sum()
        rows = slice(c, None, b)
        colsum = acc_free[rows].sum(axis=0)
        assert np.all(np.abs(colsum) <= 1e-9 * np.abs(M).max())


@pytest.mark.parametrize("maker", [
    lambda: synth.oil_water_lognormal(4, 3, 3, seed=21),
    lambda: synth.black_oil_layered(3, 3, 3, seed=22),
])
def test_jacobian_matches_central_differences(maker):
    case = maker()
    x = synth.random_state_perturbation(case, 8)
    _, J = _assemble(case, x=x)
    M = dense_from_blocks(J)
    b = x.shape[0]
    n = x[0].size
    fd = np.zeros_like(M)
    for cell in range(n):
        k, j, i = np.unravel_index(cell, x[0].shape)
        for u in range(b):
            eps = 1e-7 * max(1.0, abs(x[u, k, j, i]))
            xp, xm = x.copy(), x.copy()
            xp[u, k, j, i] += eps
            xm[u, k, j, i] -= eps
            Rp, _ = _assemble(case, x=xp)
            Rm, _ = _assemble(case, x=xm)
            fd[:, cell * b + u] = (np.moveaxis((Rp - Rm).reshape(b, -1), 0, 1).ravel()) / (2 * eps)
    scale = np.abs(M).max()
    assert np.allclose(M, fd, rtol=1e-6, atol=1e-7 * scale)


def test_wells_zero_drawdown_and_sign():
    # eq. (6): no flow when p_h equals the wellbore hydrostatic pressure at
    # the perforation; a producer below reservoir pressure removes mass.
    case = _two_cell_single_phase()
    x = case["x"].copy()
    depth = model.cell_depth(case["grid"])[0, 0, 0]
    rho = 1000.0
    p_h = x[0, 0, 0, 0] - rho * model.G * (depth - case["grid"]["top"]) / model.BAR
    x[0, 0, 0, 1] = x[0, 0, 0, 0]
    w = [synth.well(0, 0, 1, "prod", p_h)]
    R, _ = _assemble(case, x=x, wells=w)
    assert abs(R[0, 0, 0, 0]) < 1e-12
    w = [synth.well(0, 0, 1, "prod", p_h - 10.0)]
    R, _ = _assemble(case, x=x, wells=w)
    assert R[0, 0, 0, 0] > 0          # residual = -(-q) > 0: mass leaves
    w = [synth.well(0, 0, 1, "inj", p_h + 10.0)]
    R, _ = _assemble(case, x=x, wells=w)
    assert R[0, 0, 0, 0] < 0


def test_black_oil_without_gas_reduces_to_oil_water():
    # With Rs = 0, constant Bo = 1 and mu_o, and no free gas, the black-oil
    # oil and water rows are the oil-water model's (c_o = 0) and the gas row
    # is identically zero.
    ow = synth.oil_water_lognormal(4, 3, 3, seed=31)
    ow["fluid"] = dict(ow["fluid"], c_o=0.0)
    x = synth.random_state_perturbation(ow, 9)
    pvt = synth.BLACK_OIL_PVT.copy()
    pvt[1] = 0.0
    pvt[2] = 1.0
    pvt[3] = ow["fluid"]["mu_o"]
    bo_fluid = dict(synth.BLACK_OIL, pvt=pvt, rho_o_sc=ow["fluid"]["rho_o_ref"])
    bo = copy.deepcopy(ow)
    bo["fluid"] = bo_fluid
    xb = np.concatenate([x, np.zeros_like(x[:1])])
    bo["x_old"] = np.concatenate([ow["x_old"], np.zeros_like(x[:1])])
    R1, J1 = _assemble(ow, x=x)
    R2, J2 = _assemble(bo, x=xb)
    assert np.allclose(R2[:2], R1, rtol=1e-13, atol=1e-13 * np.abs(R1).max())
    assert np.allclose(J2[:, :2, :2], J1, rtol=1e-13, atol=1e-13 * np.abs(J1).max())
    assert np.abs(R2[2]).max() == 0.0


def test_solution_gas_ratio():
    # the dissolved-gas mass over the oil-component mass in the oil phase is
    # Rs rho_g^sc / rho_o^sc (definition of the solution gas-oil ratio)
    fl = synth.BLACK_OIL
    p = np.array([120.0, 200.0, 333.0])
    x = np.stack([p, np.full(3, 0.3), np.zeros(3)])
    st = model.cell_state(fl, np.full(3, 0.2), x)
    rs, _ = model.pvt_interp(fl["pvt"][0], fl["pvt"][1], p)
    assert np.allclose(st["acc"][2] / st["acc"][0], rs * fl["rho_g_sc"] / fl["rho_o_sc"], rtol=1e-14)


# ---- variable switching: undersaturated black oil (third unknown -p_b)

def _mixed_state(case, seed):
    return synth.undersaturated_cells(case, synth.random_state_perturbation(case, seed), seed + 100)


def test_undersaturated_jacobian_matches_central_differences():
    case = synth.black_oil_layered(3, 3, 3, seed=23)
    x = _mixed_state(case, 8)
    assert 0 < int((x[2] < 0).sum()) < x[2].size
    _, J = _assemble(case, x=x)
    M = dense_from_blocks(J)
    b = x.shape[0]
    n = x[0].size
    fd = np.zeros_like(M)
    for cell in range(n):
        k, j, i = np.unravel_index(cell, x[0].shape)
        for u in range(b):
            eps = 1e-7 * max(1.0, abs(x[u, k, j, i]))
            xp, xm = x.copy(), x.copy()
            xp[u, k, j, i] += eps
            xm[u, k, j, i] -= eps
            Rp, _ = _assemble(case, x=xp)
            Rm, _ = _assemble(case, x=xm)
            fd[:, cell * b + u] = (np.moveaxis((Rp - Rm).reshape(b, -1), 0, 1).ravel()) / (2 * eps)
    scale = np.abs(M).max()
    assert np.allclose(M, fd, rtol=1e-6, atol=1e-7 * scale)


def test_undersaturated_flux_conservation():
    case = synth.black_oil_layered(4, 4, 3, seed=24)
    x = _mixed_state(case, 9)
    case["x_old"] = x.copy()
    R, J = _assemble(case, x=x, dt=1e20, wells=[])
    M = dense_from_blocks(J)
    for c in range(3):
        assert abs(R[c].sum()) <= 1e-12 * np.abs(R[c]).sum()
        assert np.all(np.abs(M[c::3].sum(axis=0)) <= 1e-9 * np.abs(M).max())


def test_residual_is_continuous_at_the_switch():
    # S_g = 0 (saturated) and p_b = p (undersaturated) are the same fluid
    case = synth.black_oil_layered(4, 4, 3, seed=25)
    x = synth.random_state_perturbation(case, 10)
    rng = np.random.default_rng(3)
    pick = rng.uniform(size=x[0].shape) < 0.5
    xs, xu = x.copy(), x.copy()
    xs[2] = np.where(pick, 0.0, x[2])
    xu[2] = np.where(pick, -x[0], x[2])
    Rs, _ = _assemble(case, x=xs)
    Ru, _ = _assemble(case, x=xu)
    assert np.array_equal(Rs, Ru)


def test_undersaturated_oil_compressibility():
    # at a fixed bubble point the oil phase obeys (1/rho) d rho / dp = c_o,
    # and Rs does not change with p
    case = synth.black_oil_layered(2, 2, 1, seed=26)
    x = synth.random_state_perturbation(case, 11)
    x[2] = -(x[0] - 20.0)
    h = 1e-3
    xp, xm = x.copy(), x.copy()
    xp[0] += h
    xm[0] -= h
    st = [model.cell_state(case["fluid"], case["poro"], y) for y in (xp, xm)]
    rho_o = [s["phases"][0][0] for s in st]
    c = (np.log(rho_o[0]) - np.log(rho_o[1])) / (2 * h)
    assert np.allclose(c, case["fluid"]["c_o"], rtol=1e-6)
    # no free gas; dissolved gas per unit oil component fixed by p_b
    a0 = [s["acc"][0] for s in st]
    a2 = [s["acc"][2] for s in st]
    assert np.allclose(a2[0] / a0[0], a2[1] / a0[1], rtol=1e-13)


# ---- rate-controlled wells: BHP unknowns and the border of eq. (16)

def _rate_case():
    case = synth.oil_water_lognormal(4, 3, 2, seed=31)
    inj, prod = case["wells"]
    case["wells"] = [dict(inj, control="rate", rate=40.0, bhp=260.0),
                     dict(prod, control="rate", rate=25.0, bhp=170.0)]
    return case


def test_rate_well_border_matches_central_differences():
    case = _rate_case()
    x = synth.random_state_perturbation(case, 12)
    bhp = np.array([255.0, 175.0])
    R, J, W = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                             case["x_old"], x, 1.0, bhp=bhp, border=True)
    b = x.shape[0]
    n = x[0].size

    def F(xx, ww):
        R, _, W = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                                 case["x_old"], xx, 1.0, bhp=ww, border=True)
        return np.concatenate([np.moveaxis(R.reshape(b, -1), 0, 1).ravel(), W["R"]])
    # full bordered Jacobian in point-block order + the two BHP unknowns
    M = np.zeros((b * n + 2, b * n + 2))
    M[:b * n, :b * n] = dense_from_blocks(J)
    for q in range(2):
        M[:b * n, b * n + q] = np.moveaxis(W["B"][q].reshape(b, -1), 0, 1).ravel()
        M[b * n + q, :b * n] = np.moveaxis(W["C"][q].reshape(b, -1), 0, 1).ravel()
        M[b * n + q, b * n + q] = W["D"][q]
    fd = np.zeros_like(M)
    for col in range(b * n + 2):
        xp, xm, wp, wm = x.copy(), x.copy(), bhp.copy(), bhp.copy()
        if col < b * n:
            cell, u = divmod(col, b)
            k, j, i = np.unravel_index(cell, x[0].shape)
            eps = 1e-7 * max(1.0, abs(x[u, k, j, i]))
            xp[u, k, j, i] += eps
            xm[u, k, j, i] -= eps
        else:
            eps = 1e-7 * bhp[col - b * n]
            wp[col - b * n] += eps
            wm[col - b * n] -= eps
        fd[:, col] = (F(xp, wp) - F(xm, wm)) / (2 * eps)
    assert np.allclose(M, fd, rtol=1e-6, atol=1e-7 * np.abs(M).max())
    # the rate wells couple only their own perforations
    assert np.count_nonzero(W["D"]) == 2 and np.count_nonzero(W["B"][0][0]) == 0


def _well_rate(case, x, w):
    """Surface rate of well w (BHP w["bhp"]) at state x, from the rate
    equation with a zero target."""
    w0 = dict(w, control="rate", rate=0.0)
    others = [v for v in case["wells"] if v is not w]
    R, J, W = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], [w0] + others,
                             case["x_old"], x, 1.0, bhp=np.array([w["bhp"]]), border=True)
    m = case["fluid"]["model"]
    c = 1 if w["kind"] == "inj" else 0
    sc = model.row_scales(case["grid"], case["fluid"], case["poro"], 1.0)[c]
    q = W["R"][0] * sc * model.DAY / model.surface_density(case["fluid"], c)
    return q if w["kind"] == "inj" else -q


def test_rate_control_at_the_bhp_wells_own_rate_recovers_its_bhp():
    # Solve a step with BHP wells, read each well's rate, then impose those
    # rates with wrong initial BHPs: the Newton iteration must return the
    # original BHPs and state.
    case = synth.oil_water_lognormal(6, 4, 2, seed=32)
    tight = dict(forcing="fixed", rtol=1e-12, newton_tol=1e-11)
    x1, s1 = newton.time_step(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                              case["x_old"], 1.0, **tight)
    assert s1["converged"]
    rates = [_well_rate(case, x1, w) for w in case["wells"]]
    assert rates[0] > 0 and rates[1] > 0
    rcase = dict(case, wells=[dict(w, control="rate", rate=q, bhp=w["bhp"] + (-30.0 if w["kind"] == "inj" else 20.0))
                              for w, q in zip(case["wells"], rates)])
    x2, s2 = newton.time_step(rcase["grid"], rcase["fluid"], rcase["perm"], rcase["poro"], rcase["wells"],
                              rcase["x_old"], 1.0, **tight)
    assert s2["converged"]
    assert np.allclose(s2["bhp"], [w["bhp"] for w in case["wells"]], rtol=1e-7)
    assert np.allclose(x2, x1, rtol=1e-7, atol=1e-9)
