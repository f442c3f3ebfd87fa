"""Pins of the oracle's inexact Newton time step (Algorithm 1, eq. (14))."""
import numpy as np
import pytest

from oracle import model, newton
from paper_1606_00548_amd import synth


def _run(case, dt, **kw):
    return newton.time_step(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                            case["x_old"], dt, **kw)


def _linear_case():
    # constant water density: accumulation, fluxes and wells are affine in p
    case = synth.single_phase_uniform(16, 16, 8, wells=[synth.well(0, 0, 8, "inj", 300.0),
                                                         synth.well(15, 15, 8, "prod", 150.0)])
    case["fluid"] = dict(case["fluid"], c_w=0.0)
    return case


@pytest.mark.parametrize("forcing", ["ew1", "ew2", "ew3"])
def test_affine_residual_gives_the_forcing_floor(forcing):
    # For affine F the next right-hand side is the linear residual itself,
    # b^(l+1) = b^l - A dx = r^l, so choices 1 and 2 of eq. (14) vanish and
    # are clamped to theta_min; choice 3 is at most gamma theta_0^beta.
    case = _linear_case()
    x, st = _run(case, 1.0, forcing=forcing, coarsest=16, theta0=0.1)
    h = st["history"]
    assert st["converged"] and st["cuts"] == 0 and st["newton_iterations"] == 2
    assert h["theta"][0] == 0.1
    if forcing in ("ew1", "ew2"):
        assert h["theta"][1] == 1e-6
    else:
        assert 1e-6 <= h["theta"][1] <= 0.9 * 0.1 ** 2
    # the first solve stopped at theta_0: ||b^1|| = ||r^0|| <= 0.1 ||b^0||
    assert h["bnorm"][1] <= 0.1 * h["bnorm"][0]


def test_fixed_forcing_repeats_the_newton_step():
    case = synth.oil_water_lognormal(8, 6, 3, seed=80)
    x, st = _run(case, 1.0, forcing="fixed", rtol=1e-6)
    xr = case["x_old"].copy()
    R0, _ = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                           case["x_old"], xr, 1.0)
    its = 0
    while True:
        R, _ = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                              case["x_old"], xr, 1.0)
        if np.linalg.norm(R) < 1e-3 * np.linalg.norm(R0):
            break
        xr, _, _, _ = newton.newton_step(case["grid"], case["fluid"], case["perm"], case["poro"],
                                         case["wells"], case["x_old"], xr, 1.0, rtol=1e-6)
        its += 1
        assert its <= 20
    assert st["converged"] and st["newton_iterations"] == its
    assert np.array_equal(x, xr)


def test_cuts_halve_the_step_and_the_accepted_state_meets_the_criterion():
    case = synth.oil_water_lognormal(8, 6, 3, seed=81)
    x, st = _run(case, 30.0, max_newton=6)
    assert st["converged"] and st["cuts"] >= 1
    assert st["dt_taken"] == 30.0 / 2 ** st["cuts"]
    R, _ = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                          case["x_old"], x, st["dt_taken"])
    R0, _ = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                           case["x_old"], case["x_old"], st["dt_taken"])
    assert np.linalg.norm(R) < 1e-3 * np.linalg.norm(R0)
    assert st["total_newton"] == st["newton_iterations"] + 6 * st["cuts"]
    # no cut allowed: the failed attempt returns x_old
    x1, st1 = _run(case, 30.0, max_newton=6, max_cuts=0)
    assert not st1["converged"] and np.array_equal(x1, case["x_old"])


@pytest.mark.parametrize("forcing", ["fixed", "ew1", "ew2", "ew3"])
def test_time_step_converges_and_inexact_forcing_saves_linear_work(forcing):
    case = synth.oil_water_lognormal(16, 12, 4, seed=6)
    x, st = _run(case, 1.0, forcing=forcing)
    R, _ = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                          case["x_old"], x, 1.0)
    assert st["converged"] and st["cuts"] == 0
    assert np.linalg.norm(R) < 1e-3 * st["history"]["bnorm"][0]
    assert np.isclose(np.linalg.norm(R), st["history"]["bnorm"][-1], rtol=1e-12)
    if forcing != "fixed":
        _, sf = _run(case, 1.0, forcing="fixed")
        assert st["total_linear"] < sf["total_linear"]


def test_simulate_steps_add_up_and_grow():
    case = synth.black_oil_layered(16, 12, 4, seed=5)
    x, st = newton.simulate(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                            case["x_old"], 1.0, 0.01, 0.25)
    assert st["completed"] and abs(sum(st["dts"]) - 1.0) <= 1e-12
    t = 0.0
    for a, b in zip(st["dts"][:-1], st["dts"][1:]):
        t += a
        assert b == min(2.0 * a, 0.25, 1.0 - t) or np.isclose(b, 1.0 - t, rtol=1e-12)
    assert max(st["dts"]) == 0.25
    # per-step counts add up to the totals (every step converged without cuts here or with them)
    assert sum(st["step_newton"]) == st["total_newton"] and sum(st["step_linear"]) == st["total_linear"]
    assert sum(st["step_cuts"]) == st["cuts"] and len(st["step_newton"]) == st["steps"]


def test_paper_table_columns_and_jsonl(tmp_path):
    # the binding's table helpers on a stats record of known counts: averages
    # per Newton iteration as in the paper's tables
    import json
    from paper_1606_00548_amd import cprmi
    st = {"steps": 2, "total_newton": 7, "total_linear": 63, "seconds": 3.5, "completed": 1, "t_reached": 3.0,
          "dts": [1.0, 2.0], "step_newton": [3, 4], "step_linear": [27, 36], "step_cuts": [0, 1],
          "step_seconds": [1.0, 2.0]}
    row = cprmi.paper_table(st)
    assert row == {"steps": 2, "newton": 7, "solver": 63, "avg_solver": 9.0, "time_s": 3.5, "avg_time_s": 0.5}
    cprmi.write_jsonl(tmp_path / "r.jsonl", st)
    lines = [json.loads(l) for l in (tmp_path / "r.jsonl").read_text().splitlines()]
    assert [l["t_days"] for l in lines[:2]] == [1.0, 3.0] and lines[1]["cuts"] == 1
    assert lines[2]["avg_solver"] == 9.0 and lines[2]["completed"] is True


def test_simulate_is_a_sequence_of_time_steps():
    case = synth.oil_water_lognormal(8, 6, 3, seed=82)
    x, st = newton.simulate(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                            case["x_old"], 3.0, 1.0, 1.0, growth=1.0)
    xr = case["x_old"]
    for _ in range(3):
        xr, s = _run(dict(case, x_old=xr), 1.0)
        assert s["converged"] and s["cuts"] == 0
    assert st["completed"] and st["steps"] == 3 and np.array_equal(x, xr)
