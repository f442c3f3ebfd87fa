"""Stall check: when an FGMRES restart cycle with the FP32 preconditioner
or with the learned stage does not bring the true residual below
stall_ratio times the one it started from, the remaining cycles apply plain
FP64 CPR (FP64 preconditioner, no learned stage).  The condition is forced
from the host (a tiny stall_ratio makes every completed cycle count as
stalled); the run must then equal, to rounding, one cycle of the chosen
form followed by a plain FP64 solve from its iterate, and that second part
must match the oracle's FGMRES from the same iterate (same iterations,
1e-8)."""
import numpy as np
import pytest

from oracle import cpr, krylov, model
from paper_1606_00548_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

M = 5   # restart length: several cycles on these systems


def _gpu(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


# grid sides divisible by 8, as the learned stage's network needs
@pytest.mark.parametrize("name,make", [("bo-32x24x8", lambda: synth.black_oil_layered(32, 24, 8, seed=102)),
                                       ("ow-40x16x8", lambda: synth.oil_water_lognormal(40, 16, 8, seed=101))])
@pytest.mark.parametrize("precision,learned", [("mixed", 0), ("mixed", 1), ("fp64", 1)])
def test_forced_fallback_is_one_cycle_then_plain_fp64(name, make, precision, learned):
    from paper_1606_00548_amd import cprmi, train
    case = make()
    x = synth.random_state_perturbation(case, 17)
    R, J = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                          case["x_old"], x, case["dt"])
    b = -R
    s = cprmi.Solver.from_case(case)
    if learned:
        # the network's inputs come from the assembled state
        fam = "black-oil" if case["x"].shape[0] == 3 else "oil-water"
        s.attach_network(np.load(train.weights_path(fam)))
        bg = s.assemble(_gpu(case["x_old"]), _gpu(x), case["dt"])
    else:
        s.import_jacobian(J)
        bg = _gpu(b)
    # forced: every cycle that does not converge counts as stalled
    s.setup(precision=precision, restart=M, stall_ratio=1e-300, learned=learned)
    dxf, stf = s.solve(bg)
    # reference: one cycle of that form, then plain FP64 CPR from its iterate
    s.setup(precision=precision, restart=M, max_iter=M, learned=learned)
    x1, st1 = s.solve(bg)
    assert st1["status"] == 1 and st1["iterations"] == M and st1["fp64_fallback"] == 0
    x1h = _np(x1)
    s.setup(precision="fp64", restart=M, x0=1, learned=0)
    dx2, st2 = s.solve(bg, dx=x1.clone())
    print(f"[fallback] {name} {precision} learned={learned}: {stf['iterations']} iterations, FP64 after cycle "
          f"{stf['fp64_fallback']}; reference {M} + {st2['iterations']}", flush=True)
    assert stf["status"] == 0 and stf["fp64_fallback"] == 1
    assert stf["iterations"] == M + st2["iterations"]
    xf, x2 = _np(dxf), _np(dx2)
    assert np.linalg.norm(xf - x2) <= 1e-12 * np.linalg.norm(x2)
    assert np.linalg.norm(b - cpr.block_spmv(J, xf)) <= 1e-6 * np.linalg.norm(b)
    if not learned:
        # the FP64 part against the oracle's FGMRES from the same iterate
        # (with learned = 1 the GPU assembled its own Jacobian)
        pc = cpr.cpr_setup(J)
        xo, so = krylov.fgmres(lambda u: cpr.block_spmv(J, u), lambda u: cpr.cpr_apply(pc, u), b,
                               x0=x1h, restart=M)
        assert so["converged"] and so["iterations"] == st2["iterations"]
        assert np.linalg.norm(xf - xo) <= 1e-8 * np.linalg.norm(xo)
    s.close()


def test_default_stall_check_keeps_fp32_on_a_converging_solve():
    # default stall_ratio 0.5: cycles that more than halve the residual keep
    # FP32; stall_ratio <= 0 disables the check; both runs are then identical
    from paper_1606_00548_amd import cprmi
    case = synth.black_oil_layered(34, 20, 6, seed=102)
    R, J = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                          case["x_old"], synth.random_state_perturbation(case, 17), case["dt"])
    b = -R
    s = cprmi.Solver.from_case(case)
    s.import_jacobian(J)
    s.setup(precision="mixed", restart=M)
    dxa, sta = s.solve(_gpu(b))
    s.setup(precision="mixed", restart=M, stall_ratio=0.0)
    dxb, stb = s.solve(_gpu(b))
    assert sta["status"] == 0 and sta["cycles"] > 1 and sta["fp64_fallback"] == 0
    assert stb["fp64_fallback"] == 0 and sta["iterations"] == stb["iterations"]
    assert np.array_equal(_np(dxa), _np(dxb))
    with pytest.raises(cprmi.CPRError) as e:
        s.setup(precision="mixed", stall_ratio=float("nan"))
    assert e.value.code == -1
    s.close()


@pytest.mark.parametrize("orth", ["dcgs2", "cgs2"])
def test_early_stall_ends_the_cycle_after_ten_steps(orth):
    # restart 30 and a forced stall: the first cycle ends after ten steps
    # (FGMRES's estimate is above the bound), the check after the cycle
    # hands the rest to plain FP64 CPR; the run equals ten steps of the
    # mixed form followed by a plain FP64 solve from that iterate
    from paper_1606_00548_amd import cprmi
    case = synth.black_oil_channelised(32, 24, 8, seed=103)
    x = synth.random_state_perturbation(case, 17)
    R, J = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                          case["x_old"], x, case["dt"])
    b = -R
    s = cprmi.Solver.from_case(case)
    s.import_jacobian(J)
    bg = _gpu(b)
    s.setup(precision="mixed", restart=30, stall_ratio=1e-300, orth=orth)
    dxf, stf = s.solve(bg)
    s.setup(precision="mixed", restart=30, max_iter=10, orth=orth)
    x1, st1 = s.solve(bg)
    assert st1["status"] == 1 and st1["iterations"] == 10
    s.setup(precision="fp64", restart=30, x0=1, orth=orth)
    dx2, st2 = s.solve(bg, dx=x1.clone())
    print(f"[early-stall] {orth}: {stf['iterations']} iterations, FP64 after cycle {stf['fp64_fallback']}; "
          f"reference 10 + {st2['iterations']}", flush=True)
    assert stf["status"] == 0 and stf["fp64_fallback"] == 1
    assert stf["iterations"] == 10 + st2["iterations"]
    xf, x2 = _np(dxf), _np(dx2)
    assert np.linalg.norm(xf - x2) <= 1e-12 * np.linalg.norm(x2)
    assert np.linalg.norm(b - cpr.block_spmv(J, xf)) <= 1e-6 * np.linalg.norm(b)
    # an unforced solve of the same system never stops early
    s.setup(precision="mixed", restart=30, orth=orth)
    _, st3 = s.solve(bg)
    assert st3["fp64_fallback"] == 0
    s.close()
