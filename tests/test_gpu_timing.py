"""Phase timers (cpr_set_timing): with timing on, a solve's stats carry the
device time of the last assembly and setup, of the solve, and of its
preconditioner applications, SpMVs and orthogonalisation; the inner phases
do not overlap, so they add up to at most the solve; the solution is
bit-identical to an untimed one; with timing off every field is 0."""
import numpy as np
import pytest

from paper_1606_00548_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FIELDS = ("ms_assemble", "ms_setup", "ms_solve", "ms_precond", "ms_spmv", "ms_orth")


def _step(s, case, timing, orth="dcgs2", krylov="fgmres"):
    s.set_timing(timing)
    rhs = s.assemble(torch.as_tensor(case["x_old"]).cuda(), torch.as_tensor(case["x"]).cuda(), case["dt"])
    s.setup(orth=orth)
    dx, st = s.solve(rhs) if krylov == "fgmres" else s.bicgstab(rhs)
    torch.cuda.synchronize()
    return dx.cpu().numpy(), st


@pytest.mark.parametrize("orth,krylov", [("dcgs2", "fgmres"), ("cgs2", "fgmres"), ("dcgs2", "bicgstab")])
def test_phase_times_cover_the_solve_and_change_nothing(orth, krylov):
    from paper_1606_00548_amd import cprmi
    case = synth.black_oil_layered(64, 48, 16, seed=31)
    s = cprmi.Solver.from_case(case)
    x0, st0 = _step(s, case, False, orth, krylov)
    x1, st1 = _step(s, case, True, orth, krylov)
    x2, st2 = _step(s, case, False, orth, krylov)
    print(f"[timing] {orth} {krylov}: " + ", ".join(f"{f} {st1[f]:.3f}" for f in FIELDS), flush=True)
    assert st0["converged"] and st1["converged"]
    assert np.array_equal(x0, x1) and np.array_equal(x0, x2)
    assert st0["iterations"] == st1["iterations"]
    for f in FIELDS:
        assert st0[f] == 0.0 and st2[f] == 0.0
        assert st1[f] > 0.0, f
    inner = st1["ms_precond"] + st1["ms_spmv"] + st1["ms_orth"]
    assert inner <= st1["ms_solve"] * 1.01 + 0.01
    # the solve is mostly these three phases (the rest: norms, scalings,
    # the update, host waits)
    assert inner >= 0.5 * st1["ms_solve"]
    s.close()


def test_timing_survives_many_solves_without_overflow():
    # more timed pairs than the ring holds within one solve: a long
    # restart-free solve of a harder system with a tiny tolerance
    from paper_1606_00548_amd import cprmi
    case = synth.black_oil_layered(32, 32, 8, seed=32)
    s = cprmi.Solver.from_case(case)
    s.set_timing(True)
    rhs = s.assemble(torch.as_tensor(case["x_old"]).cuda(), torch.as_tensor(case["x"]).cuda(), case["dt"])
    s.setup(rtol=1e-14, max_iter=200, restart=60, mg_pre=1, mg_post=1)
    for _ in range(3):
        dx, st = s.solve(rhs)
        assert st["iterations"] > 0 and st["ms_solve"] > 0
        inner = st["ms_precond"] + st["ms_spmv"] + st["ms_orth"]
        assert 0 < inner <= st["ms_solve"] * 1.01 + 0.01
    s.close()
