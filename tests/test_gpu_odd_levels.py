"""Multigrid hierarchies with a level of odd nx above the coarsest (stored
colour-split with a ghost column) against the oracle, whose levels have
ceil(n/2) cells per axis whatever the parity:
  * 6 x 32 x 32 oil water with mg_coarsest = 64: 3 x 16 x 16 (padded),
    2 x 8 x 8, 1 x 4 x 4 (natural coarsest);
  * 100 x 100 x 20 black oil: 50 x 50 x 10, 25 x 25 x 5 (padded),
    13 x 13 x 3 (natural coarsest);
  * the 60 x 220 x 85 shape of the paper's SPE10 oil-water model (Sec. 3.1):
    30 x 110 x 43, 15 x 55 x 22 (padded), 8 x 28 x 11, 4 x 14 x 6.
Tolerances as in the other parity tests: levels 1e-12 of the row scale, one
CPR application 1e-9, FGMRES the oracle's iteration count and 1e-8 (a fixed
path of ten iterations on the SPE10-shaped grid, whose full solve the oracle
would take minutes for), the same for the mixed-precision application at
1e-5 and its true residual at 1e-6."""
import numpy as np
import pytest

from oracle import cpr, krylov, model
from paper_1606_00548_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = {
    "ow-6x32x32-coarsest-64": (lambda: synth.oil_water_lognormal(6, 32, 32, seed=111), 64, None),
    "bo-100x100x20": (lambda: synth.black_oil_layered(100, 100, 20, seed=112), 512, None),
    "ow-spe10-shaped-60x220x85": (lambda: synth.spe10_shaped_oil_water(), 512, 10),
}


@pytest.fixture(scope="module", params=list(CASES))
def system(request):
    make, coarsest, fixed = CASES[request.param]
    case = make()
    print(f"[odd-levels] case {request.param}", flush=True)
    R, J = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                          case["x_old"], case["x"], case["dt"])
    pc = cpr.cpr_setup(J, coarsest)
    return request.param, case, J, -R, pc, coarsest, fixed


def _gpu(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _solver(case, J, **opts):
    from paper_1606_00548_amd import cprmi
    s = cprmi.Solver.from_case(case)
    s.import_jacobian(_gpu(J))
    s.setup(**opts)
    return s


def test_hierarchy_has_an_odd_level_and_matches_oracle(system):
    name, case, J, b, pc, coarsest, _ = system
    s = _solver(case, J, mg_coarsest=coarsest)
    levels = pc["mg"]["levels"]
    shapes = [A.shape[1:] for A in levels]
    print(f"[odd-levels] {name}: levels {shapes}")
    assert any(sh[2] % 2 == 1 for sh in shapes[1:-1])        # a smoothed level with odd nx
    for l, A in enumerate(levels):
        assert s.mg_level_shape(l) == A.shape[1:]
        Ag = s.export_mg_level(l).cpu().numpy()
        assert np.all(np.abs(Ag - A) <= 1e-12 * np.abs(A).max(axis=0)), l
    assert s.mg_level_shape(len(levels)) is None
    s.close()


def test_precond_and_fgmres_match_oracle(system):
    name, case, J, b, pc, coarsest, fixed = system
    kw = dict(mg_coarsest=coarsest)
    if fixed:
        kw.update(rtol=0.0, max_iter=fixed)
    s = _solver(case, J, **kw)
    v = b / np.linalg.norm(b)
    z = s.precond(_gpu(v)).cpu().numpy()
    ref = cpr.cpr_apply(pc, v)
    d_apply = np.linalg.norm(z - ref) / np.linalg.norm(ref)
    dx, st = s.solve(_gpu(b))
    A = lambda u: cpr.block_spmv(J, u)
    M = lambda u: cpr.cpr_apply(pc, u)
    if fixed:
        xo, so = krylov.fgmres(A, M, b, rtol=0.0, max_iter=fixed)
    else:
        xo, so = krylov.fgmres(A, M, b)
    d = np.linalg.norm(dx.cpu().numpy() - xo) / np.linalg.norm(xo)
    print(f"[odd-levels] {name}: apply rel. diff {d_apply:.1e}; FGMRES {st['iterations']} iterations "
          f"(oracle {so['iterations']}), rel. diff {d:.1e}")
    assert d_apply <= 1e-9
    assert st["iterations"] == so["iterations"]
    assert st["status"] == (1 if fixed else 0)
    assert d <= 1e-8
    # the FP32 preconditioner on the same hierarchy
    s.setup(precision="mixed", **dict(kw, rtol=1e-6, max_iter=300))
    zf = s.precond(_gpu(v)).cpu().numpy()
    assert np.linalg.norm(zf - ref) <= 1e-5 * np.linalg.norm(ref)
    dxf, stf = s.solve(_gpu(b))
    res = np.linalg.norm(b - A(dxf.cpu().numpy())) / np.linalg.norm(b)
    print(f"[odd-levels] {name}: mixed apply {np.linalg.norm(zf - ref) / np.linalg.norm(ref):.1e}, "
          f"{stf['iterations']} iterations, true rel. {res:.1e}")
    assert stf["status"] == 0 and res <= 1e-6
    s.close()


def test_spe10_shaped_newton_step_runs_from_assembly():
    # the library's own assembly on the SPE10-shaped grid (no import): a full
    # Newton step reaches 1e-6 with the padded hierarchy
    from paper_1606_00548_amd import cprmi
    case = synth.spe10_shaped_oil_water()
    print("[odd-levels] SPE10-shaped Newton step", flush=True)
    s = cprmi.Solver.from_case(case)
    x = _gpu(case["x"])
    dx, st = cprmi.newton_step(s, _gpu(case["x_old"]), x, case["dt"])
    print(f"[odd-levels] SPE10-shaped: {st['iterations']} FGMRES iterations, true rel. {st['true_rel']:.1e}, "
          f"{st['mg_levels']} levels")
    assert st["status"] == 0 and st["true_rel"] <= 1e-6 and st["mg_levels"] == 5
    s.close()


def test_benchmark_cycle_on_odd_levels_matches_oracle(system):
    # V(2,2) with the coarse correction scaled by 1.25 (the benchmark's
    # cycle) through the padded levels: one application at 1e-9 and a fixed
    # FGMRES path of five iterations at 1e-8
    name, case, J, b, _, coarsest, _ = system
    s = _solver(case, J, mg_coarsest=coarsest, mg_pre=2, mg_post=2, mg_alpha=1.25, rtol=0.0, max_iter=5)
    pc = cpr.cpr_setup(J, coarsest, pre=2, post=2)
    v = b / np.linalg.norm(b)
    z = s.precond(_gpu(v)).cpu().numpy()
    ref = cpr.cpr_apply(pc, v, alpha=1.25)
    d_apply = np.linalg.norm(z - ref) / np.linalg.norm(ref)
    dx, st = s.solve(_gpu(b))
    xo, so = krylov.fgmres(lambda u: cpr.block_spmv(J, u), lambda u: cpr.cpr_apply(pc, u, alpha=1.25), b,
                           rtol=0.0, max_iter=5)
    d = np.linalg.norm(dx.cpu().numpy() - xo) / np.linalg.norm(xo)
    print(f"[odd-levels] {name} V(2,2) alpha 1.25: apply rel. diff {d_apply:.1e}; 5 FGMRES iterations "
          f"rel. diff {d:.1e}")
    assert d_apply <= 1e-9
    assert st["iterations"] == so["iterations"] == 5
    assert d <= 1e-8
    s.close()
