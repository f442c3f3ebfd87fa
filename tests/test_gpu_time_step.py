"""The inexact Newton time step (Algorithm 1, eq. (14), time-step cuts) on
the GPU against the oracle's.

Both sides run the same iteration in FP64; norms that choose theta_l and
stop the iteration agree to rounding, so the GPU must take the same
decisions: the same number of cuts, Newton iterations and linear
iterations per Newton iteration, theta_l and ||b^l|| within 1e-9 relative,
and the final state within 1e-8 relative (FGMRES parity bound).  BiCGSTAB
reacts chaotically to rounding (see its parity test), so with it only
convergence and the stopping criterion, recomputed by the oracle, are
checked.
"""
import json

import numpy as np
import pytest

from oracle import model, newton
from paper_1606_00548_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _gpu(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _solver(case):
    from paper_1606_00548_amd import cprmi
    return cprmi.Solver.from_case(case)


def _compare(case, dt, newton_kw, label):
    from paper_1606_00548_amd import cprmi
    s = _solver(case)
    xg, sg = s.time_step(_gpu(case["x_old"]), dt, newton=newton_kw)
    xo, so = newton.time_step(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                              case["x_old"], dt, **newton_kw)
    hg, ho = sg["history"], so["history"]
    print(f"[time-step] {label}: cuts {sg['cuts']} (oracle {so['cuts']}), Newton {sg['newton_iterations']} "
          f"(oracle {so['newton_iterations']}), linear {hg['linear_iterations']} "
          f"(oracle {ho['linear_iterations']})", flush=True)
    assert bool(sg["converged"]) == so["converged"]
    assert sg["status"] == (cprmi.CPR_OK if so["converged"] else cprmi.CPR_NOT_CONVERGED)
    assert sg["cuts"] == so["cuts"] and sg["dt_taken"] == so["dt_taken"]
    assert sg["newton_iterations"] == so["newton_iterations"]
    assert sg["total_newton"] == so["total_newton"]
    assert hg["linear_iterations"] == ho["linear_iterations"]
    assert np.allclose(hg["theta"], ho["theta"], rtol=1e-9, atol=0)
    assert np.allclose(hg["bnorm"], ho["bnorm"], rtol=1e-9, atol=0)
    x = xg.cpu().numpy()
    assert np.linalg.norm(x - xo) <= 1e-8 * np.linalg.norm(xo)
    s.close()
    return sg


@pytest.mark.parametrize("forcing", ["fixed", "ew1", "ew2", "ew3"])
def test_time_step_matches_oracle(forcing):
    case = synth.oil_water_lognormal(16, 12, 4, seed=6)
    _compare(case, 1.0, {"forcing": forcing}, f"oil-water 16x12x4 {forcing}")


def test_time_step_cuts_match_oracle():
    case = synth.oil_water_lognormal(8, 6, 3, seed=81)
    st = _compare(case, 30.0, {"max_newton": 6}, "oil-water 8x6x3, dt 30, max 6 Newton")
    assert st["cuts"] >= 1


def test_black_oil_time_step_matches_oracle():
    # cells near the injector become undersaturated; with variable switching
    # the step needs no cut (cuts with switching: the switching tests)
    case = synth.black_oil_layered(16, 12, 4, seed=5)
    st = _compare(case, 0.1, {}, "black oil 16x12x4, dt 0.1")
    assert st["converged"] and st["cuts"] == 0


def test_failed_step_returns_x_old():
    case = synth.oil_water_lognormal(8, 6, 3, seed=81)
    st = _compare(case, 30.0, {"max_newton": 6, "max_cuts": 0}, "oil-water 8x6x3, no cut allowed")
    assert not st["converged"]


@pytest.mark.parametrize("krylov", ["bicgstab"])
def test_time_step_with_bicgstab_converges(krylov):
    case = synth.oil_water_lognormal(16, 12, 4, seed=6)
    s = _solver(case)
    xg, sg = s.time_step(_gpu(case["x_old"]), 1.0, newton={"krylov": krylov})
    x = xg.cpu().numpy()
    R, _ = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                          case["x_old"], x, sg["dt_taken"])
    R0, _ = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                           case["x_old"], case["x_old"], sg["dt_taken"])
    print(f"[time-step] BiCGSTAB: Newton {sg['newton_iterations']}, linear {sg['history']['linear_iterations']}")
    assert sg["converged"] and np.linalg.norm(R) < 1e-3 * np.linalg.norm(R0)
    s.close()


def test_time_step_mixed_learned_meets_the_criterion():
    # the learned stage and the FP32 preconditioner inside the Newton loop
    from paper_1606_00548_amd import cprmi, train
    case = synth.oil_water_lognormal(16, 16, 8, seed=7)
    s = _solver(case)
    s.attach_network(np.load(train.weights_path("oil-water")))
    for lo in (cprmi.default_options(precision="mixed"), cprmi.default_options(precision="mixed", learned=1)):
        xg, sg = s.time_step(_gpu(case["x_old"]), 1.0, options=lo)
        x = xg.cpu().numpy()
        R, _ = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                              case["x_old"], x, sg["dt_taken"])
        R0, _ = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                               case["x_old"], case["x_old"], sg["dt_taken"])
        print(f"[time-step] mixed learned={lo.learned}: Newton {sg['newton_iterations']}, "
              f"linear {sg['history']['linear_iterations']}")
        assert sg["converged"] and np.linalg.norm(R) < 1e-3 * np.linalg.norm(R0)
    s.attach_network(None)
    s.close()


def test_time_step_rejects_bad_options():
    from paper_1606_00548_amd import cprmi
    case = synth.oil_water_lognormal(8, 6, 3, seed=81)
    s = _solver(case)
    for bad in ({"forcing": 7}, {"krylov": 3}, {"newton_tol": 0.0}, {"theta_max": 1e-9}):
        with pytest.raises(cprmi.CPRError) as e:
            s.time_step(_gpu(case["x_old"]), 1.0, newton=bad)
        assert e.value.code == -1
    with pytest.raises(cprmi.CPRError):
        s.time_step(_gpu(case["x_old"]), -1.0)
    s.close()


@pytest.mark.parametrize("name", ["black-oil", "oil-water"])
def test_simulate_matches_oracle(name, tmp_path):
    if name == "black-oil":
        case, t_end, dt0, dt_max = synth.black_oil_layered(16, 12, 4, seed=5), 1.0, 0.01, 1.0
    else:
        case, t_end, dt0, dt_max = synth.oil_water_lognormal(16, 12, 4, seed=6), 10.0, 0.1, 5.0
    s = _solver(case)
    log = tmp_path / "run.jsonl"
    xg, sg = s.simulate(_gpu(case["x_old"]), t_end, dt0, dt_max, log=str(log))
    xo, so = newton.simulate(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                             case["x_old"], t_end, dt0, dt_max)
    x = xg.cpu().numpy()
    print(f"[time-step] simulate {name}: steps {sg['steps']} (oracle {so['steps']}), Newton {sg['total_newton']} "
          f"(oracle {so['total_newton']}), linear {sg['total_linear']} (oracle {so['total_linear']})")
    assert sg["completed"] and so["completed"] and sg["status"] == 0
    assert sg["steps"] == so["steps"] and sg["cuts"] == so["cuts"]
    assert sg["total_newton"] == so["total_newton"] and sg["total_linear"] == so["total_linear"]
    assert sg["dts"] == so["dts"] and sg["t_reached"] == sum(so["dts"])
    assert np.linalg.norm(x - xo) <= 1e-8 * np.linalg.norm(xo)
    # the per-step columns of the paper's tables, and the JSON-lines record
    assert sg["step_newton"] == so["step_newton"] and sg["step_linear"] == so["step_linear"]
    assert sg["step_cuts"] == so["step_cuts"]
    assert 0 < sum(sg["step_seconds"]) <= sg["seconds"]
    lines = [json.loads(l) for l in log.read_text().splitlines()]
    assert len(lines) == sg["steps"] + 1
    assert [l["newton"] for l in lines[:-1]] == so["step_newton"]
    assert lines[-1]["newton"] == so["total_newton"] and lines[-1]["solver"] == so["total_linear"]
    assert lines[-1]["avg_solver"] == so["total_linear"] / so["total_newton"]
    s.close()
