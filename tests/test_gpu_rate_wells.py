"""Rate-controlled wells (eqs. (8)-(9)) on the GPU against the oracle: the
bordered system of eq. (16) with the wells' BHPs appended to the cell
unknowns.  Tolerances: assembly as for the cells (1e-11 relative + 1e-13 of
the row scale per entry), the bordered SpMV 1e-13 of the row scale, one
preconditioner application 1e-9 in norm, FGMRES the oracle's iteration
count and 1e-8, time steps the oracle's decisions (see the time-step
parity tests) with BHPs to 1e-8."""
import numpy as np
import pytest

from oracle import cpr, krylov, model, newton
from paper_1606_00548_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _ow_case(both=False):
    case = synth.oil_water_lognormal(16, 12, 4, seed=6)
    inj, prod = case["wells"]
    if both:
        inj = dict(inj, control="rate", rate=250.0, bhp=260.0)
    case["wells"] = [inj, dict(prod, control="rate", rate=120.0, bhp=180.0)]
    return case, 1.0


def _bo_case():
    case = synth.black_oil_layered(16, 12, 4, seed=7)
    inj, *prods = case["wells"]
    rates = [120.0, 128.0, 96.0, 113.0]
    case["wells"] = [dict(inj, control="rate", rate=700.0, bhp=250.0)] + \
        [dict(p, control="rate", rate=q, bhp=185.0) for p, q in zip(prods, rates)]
    return case, 0.1


CASES = {"ow-prod-rate": lambda: _ow_case(), "ow-both-rate": lambda: _ow_case(True), "bo-all-rate": _bo_case}


def _flat(x, bhp):
    return np.concatenate([x.ravel(), bhp])


def _gpu(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _system(case, dt, seed=17):
    x = synth.random_state_perturbation(case, seed)
    rws = model.rate_wells(case["wells"])
    bhp = np.array([w["bhp"] for w in rws]) + np.linspace(-3.0, 3.0, len(rws))
    R, J, W = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                             case["x_old"], x, dt, bhp=bhp, border=True)
    return x, bhp, R, J, W


@pytest.mark.parametrize("name", list(CASES))
def test_bordered_assembly_spmv_and_preconditioner_match_oracle(name):
    from paper_1606_00548_amd import cprmi
    case, dt = CASES[name]()
    x, bhp, R, J, W = _system(case, dt)
    s = cprmi.Solver.from_case(case)
    nr = len(bhp)
    n = x.size
    assert s.unknowns() == n + nr
    xold = _flat(case["x_old"], bhp)
    rhs = s.assemble(_gpu(xold), _gpu(_flat(x, bhp)), dt)
    torch.cuda.synchronize()
    rg = rhs.cpu().numpy()
    bo = -np.concatenate([R.ravel(), W["R"]])
    assert np.all(np.abs(rg - bo) <= 1e-10 * np.abs(bo) + 1e-12 * np.abs(bo).max())
    Jg = s.export_jacobian().cpu().numpy()
    rowscale = np.abs(J).max(axis=(0, 2), keepdims=True)
    assert np.all(np.abs(Jg - J) <= 1e-11 * np.abs(J) + 1e-13 * rowscale)
    # the bordered product and the preconditioner on random vectors
    pc = cpr.cpr_setup(J)
    A, M = newton.border_operators(J, W, pc, "two-stage", x.shape)
    v = np.random.default_rng(3).standard_normal(n + nr)
    y = s.spmv(_gpu(v)).cpu().numpy()
    yo = A(v)
    assert np.linalg.norm(y - yo) <= 1e-13 * np.linalg.norm(yo) * 100
    s.setup()
    z = s.precond(_gpu(v)).cpu().numpy()
    zo = M(v)
    print(f"[rate-wells] {name}: {nr} rate wells, |y - y_o| / |y_o| {np.linalg.norm(y - yo) / np.linalg.norm(yo):.1e}, "
          f"|z - z_o| / |z_o| {np.linalg.norm(z - zo) / np.linalg.norm(zo):.1e}", flush=True)
    assert np.linalg.norm(z - zo) <= 1e-9 * np.linalg.norm(zo)
    # FGMRES on the bordered system
    b = bo
    dx, st = s.solve(_gpu(b))
    xo, so = krylov.fgmres(A, M, b)
    assert st["status"] == 0 and so["converged"] and st["iterations"] == so["iterations"]
    assert np.linalg.norm(dx.cpu().numpy() - xo) <= 1e-8 * np.linalg.norm(xo)
    s.close()


@pytest.mark.parametrize("name", list(CASES))
def test_time_step_with_rate_wells_matches_oracle(name):
    from paper_1606_00548_amd import cprmi
    case, dt = CASES[name]()
    rws = model.rate_wells(case["wells"])
    bhp0 = np.array([w["bhp"] for w in rws])
    s = cprmi.Solver.from_case(case)
    xg, sg = s.time_step(_gpu(_flat(case["x_old"], bhp0)), dt)
    xo, so = newton.time_step(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                              case["x_old"], dt)
    x = xg.cpu().numpy()
    n = case["x_old"].size
    print(f"[rate-wells] {name} time step: Newton {sg['newton_iterations']} (oracle {so['newton_iterations']}), "
          f"linear {sg['history']['linear_iterations']}, BHP {np.round(x[n:], 2)} (oracle {np.round(so['bhp'], 2)})",
          flush=True)
    assert sg["converged"] and so["converged"]
    assert sg["cuts"] == so["cuts"] and sg["newton_iterations"] == so["newton_iterations"]
    assert sg["history"]["linear_iterations"] == so["history"]["linear_iterations"]
    assert np.allclose(sg["history"]["bnorm"], so["history"]["bnorm"], rtol=1e-6, atol=0)
    assert np.linalg.norm(x[:n] - xo.ravel()) <= 1e-8 * np.linalg.norm(xo)
    assert np.allclose(x[n:], so["bhp"], rtol=1e-8)
    s.close()


@pytest.mark.parametrize("opts,krylov", [(dict(precision="mixed"), "fgmres"),
                                         (dict(decoupling="abf", composition="fpf"), "fgmres"),
                                         (dict(precision="mixed", composition="fpf"), "bicgstab")])
def test_rate_wells_with_other_solver_forms_meet_their_targets(opts, krylov):
    # the well rows ride along with every form of the cell preconditioner
    # and both Krylov methods: the accepted state meets the Newton criterion
    # and every rate equation, recomputed by the oracle
    from paper_1606_00548_amd import cprmi
    case, dt = _bo_case()
    rws = model.rate_wells(case["wells"])
    bhp0 = np.array([w["bhp"] for w in rws])
    s = cprmi.Solver.from_case(case)
    xg, sg = s.time_step(_gpu(_flat(case["x_old"], bhp0)), dt, options=cprmi.default_options(**opts),
                         newton={"krylov": krylov})
    x = xg.cpu().numpy()
    n = case["x_old"].size
    xc, bhp = x[:n].reshape(case["x_old"].shape), x[n:]
    R, _, W = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                             case["x_old"], xc, sg["dt_taken"], bhp=bhp, border=True)
    R0, _, W0 = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                               case["x_old"], case["x_old"], sg["dt_taken"], bhp=bhp0, border=True)
    f = np.linalg.norm(np.concatenate([R.ravel(), W["R"]]))
    f0 = np.linalg.norm(np.concatenate([R0.ravel(), W0["R"]]))
    print(f"[rate-wells] {opts} {krylov}: Newton {sg['newton_iterations']}, cuts {sg['cuts']}, "
          f"|F|/|F0| {f / f0:.1e}, max |R_w| {np.abs(W['R']).max():.1e}")
    assert sg["converged"] and f < 1e-3 * f0
    assert np.abs(W["R"]).max() < 1e-3 * f0
    s.close()
