"""Pins of the oracle's learned correction inside the multigrid cycle on a
coarse level: the cycle with a hook that adds nothing is the plain cycle bit
for bit; a hook that adds the level's exact remaining correction gives the
cycle whose level is solved exactly; the level fields are block means of
the fine ones; a network whose output is zero is rejected and leaves plain
CPR."""
import numpy as np
import pytest

from oracle import cpr, learned, model, nn
from paper_1606_00548_amd import synth


def _system():
    case = synth.oil_water_lognormal(32, 32, 16, seed=71)
    R, J = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                          case["x_old"], case["x"], case["dt"])
    return case, J, -R, cpr.cpr_setup(J)


def test_zero_hook_is_the_plain_cycle():
    case, J, b, pc = _system()
    r = cpr.decouple(pc, b / np.linalg.norm(b))[0]
    for level in (1, 2):
        x = learned.vcycle_with_hook(pc["mg"], r, level, lambda rr, xx: np.zeros_like(xx))
        assert np.array_equal(x, cpr.vcycle(pc["mg"], r))


def test_exact_hook_equals_the_cycle_with_that_level_solved_exactly():
    case, J, b, pc = _system()
    mg = pc["mg"]
    r = cpr.decouple(pc, b / np.linalg.norm(b))[0]
    level = 1
    A_l = mg["levels"][level]
    Ad = cpr.to_sparse(A_l).toarray()

    after = []

    def exact_hook(rr, xx):
        e = np.linalg.solve(Ad, (rr - cpr.scalar_spmv(A_l, xx)).ravel()).reshape(xx.shape)
        after.append(np.linalg.norm(rr - cpr.scalar_spmv(A_l, xx + e)) / np.linalg.norm(rr))
        return e

    def cycle_exact(rr, lev):
        # cpr.vcycle's recursion with level `level` solved by a dense solve
        A = mg["levels"][lev]
        shape = A.shape[1:]
        if lev == level:
            return np.linalg.solve(Ad, rr.ravel()).reshape(shape)
        col = cpr.colour(shape)
        x = np.zeros_like(rr)
        cpr.gs_half_sweep(A, rr, x, col, 0)
        cpr.gs_half_sweep(A, rr, x, col, 1)
        res = rr - cpr.scalar_spmv(A, x)
        P = cpr.prolongator(shape)
        ec = cycle_exact((P.T @ res.ravel()).reshape(cpr.coarse_shape(shape)), lev + 1)
        x += (P @ ec.ravel()).reshape(shape)
        cpr.gs_half_sweep(A, rr, x, col, 1)
        cpr.gs_half_sweep(A, rr, x, col, 0)
        return x

    x1 = learned.vcycle_with_hook(mg, r, level, exact_hook)
    x2 = cycle_exact(r, 0)
    assert np.linalg.norm(x1 - x2) <= 1e-10 * np.linalg.norm(x2)
    # the level's residual after the hook vanishes; before it, it is what
    # level_residual reports
    assert after[0] <= 1e-12
    rl = learned.level_residual(pc, b / np.linalg.norm(b), level)
    x_plain = learned.vcycle_with_hook(mg, r, level, lambda rr, xx: np.zeros_like(xx))
    assert np.linalg.norm(rl) > 1e-3 * np.linalg.norm(r) and np.array_equal(x_plain, cpr.vcycle(mg, r))


def test_level_fields_are_block_means():
    case = synth.oil_water_lognormal(16, 8, 8, seed=72)
    lam = learned.total_mobility(case["fluid"], case["poro"], case["x"])
    lk, ll = learned.level_fields(case["perm"], lam, 2)
    assert lk.shape == (2, 2, 4)
    for k in range(2):
        for j in range(2):
            for i in range(4):
                blk = (slice(4 * k, 4 * k + 4), slice(4 * j, 4 * j + 4), slice(4 * i, 4 * i + 4))
                assert np.isclose(lk[k, j, i], np.log(case["perm"][0][blk]).mean(), rtol=1e-14)
                assert np.isclose(ll[k, j, i], np.log(lam[blk]).mean(), rtol=1e-14)
    lk0, ll0 = learned.level_fields(case["perm"], lam, 0)
    assert np.array_equal(lk0, np.log(case["perm"][0]))


@pytest.mark.parametrize("level", [0, 1])
def test_zero_network_is_rejected_at_every_level(level):
    case, J, b, pc = _system()
    lam = learned.total_mobility(case["fluid"], case["poro"], case["x"])
    v = b / np.linalg.norm(b)
    z, acc = learned.learned_cpr_apply(pc, v, np.zeros(nn.num_params()), case["perm"], lam, level=level)
    assert not acc
    assert np.array_equal(z, cpr.cpr_apply(pc, v))


def test_accepted_level_correction_reduces_the_level_residual():
    # a network whose output is the level's exact correction (a delta kernel
    # cannot produce it, so the judged step is checked directly)
    case, J, b, pc = _system()
    lam = learned.total_mobility(case["fluid"], case["poro"], case["x"])
    level = 1
    A_l = pc["mg"]["levels"][level]
    lnk, lnl = learned.level_fields(case["perm"], lam, level)
    rl = learned.level_residual(pc, b / np.linalg.norm(b), level)
    theta = synth.nn_initial_weights(5).astype(np.float64)
    d, acc = learned.judged_step(A_l, theta, lnk, lnl, rl)
    if acc:
        assert np.linalg.norm(rl - cpr.scalar_spmv(A_l, d)) < np.linalg.norm(rl)
    else:
        assert not np.any(d)


def test_scaled_cycle_threads_alpha_through_the_learned_stage():
    # with the coarse corrections scaled (V(2,2), alpha = 1.25): a hook that
    # adds nothing gives cpr.vcycle with that alpha bit for bit, and a
    # rejected network leaves cpr.cpr_apply with that alpha bit for bit, on
    # the fine level and inside the cycle; alpha = 1 there differs
    case, J, b, _ = _system()
    pc = cpr.cpr_setup(J, pre=2, post=2)
    v = b / np.linalg.norm(b)
    r = cpr.decouple(pc, v)[0]
    for level in (1, 2):
        x = learned.vcycle_with_hook(pc["mg"], r, level, lambda rr, xx: np.zeros_like(xx), 0, 1.25)
        assert np.array_equal(x, cpr.vcycle(pc["mg"], r, 0, 1.25))
    lam = learned.total_mobility(case["fluid"], case["poro"], case["x"])
    ref = cpr.cpr_apply(pc, v, alpha=1.25)
    for level in (0, 1):
        z, acc = learned.learned_cpr_apply(pc, v, np.zeros(nn.num_params()), case["perm"], lam, level=level,
                                           alpha=1.25)
        assert not acc and np.array_equal(z, ref)
    rp, dp, _ = learned.pressure_stage(pc, v, alpha=1.25)
    assert np.array_equal(dp, cpr.vcycle(pc["mg"], r, 0, 1.25))
    assert not np.allclose(ref, cpr.cpr_apply(pc, v), rtol=1e-6, atol=0)
