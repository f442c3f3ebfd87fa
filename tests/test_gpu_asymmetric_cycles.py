"""V-cycles with different pre- and post-smoothing counts, V(1,2) and V(2,1)
with the coarse correction scaled by 1.25, in both ILU orders, against the
oracle: one FP64 CPR application to 1e-9, FGMRES with the same iteration
count and 1e-8, the FP32 preconditioner's application within 1e-5 of the
FP64 oracle's.  Grids with odd ny or nz and all three model families.
Tolerances as in the other parity tests."""
import numpy as np
import pytest

from oracle import cpr, krylov, model
from paper_1606_00548_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _gpu(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


CASES = {
    "ow-40x18x7": lambda: synth.oil_water_lognormal(40, 18, 7, seed=141),
    "bo-34x21x6": lambda: synth.black_oil_layered(34, 21, 6, seed=142),
    "bo-chan-48x24x8": lambda: synth.black_oil_channelised(48, 24, 8, seed=143),
}


@pytest.fixture(scope="module", params=list(CASES))
def system(request):
    case = CASES[request.param]()
    x = synth.random_state_perturbation(case, 29)
    R, J = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                          case["x_old"], x, case["dt"])
    print(f"[asymmetric-cycles] case {request.param}", flush=True)
    return request.param, case, J, -R


@pytest.mark.parametrize("order", ["red-black", "tiles"])
@pytest.mark.parametrize("pre,post", [(1, 2), (2, 1)])
def test_asymmetric_cycle_matches_oracle(system, pre, post, order):
    from paper_1606_00548_amd import cprmi
    name, case, J, b = system
    s = cprmi.Solver.from_case(case)
    s.import_jacobian(J)
    pc = cpr.cpr_setup(J, pre=pre, post=post, ilu_order=order)
    M = lambda u: cpr.cpr_apply(pc, u, alpha=1.25)
    v = b / np.linalg.norm(b)
    ref = M(v)
    s.setup(ilu_order=order, mg_pre=pre, mg_post=post, mg_alpha=1.25)
    e64 = np.linalg.norm(_np(s.precond(_gpu(v))) - ref) / np.linalg.norm(ref)
    xo, so = krylov.fgmres(lambda u: cpr.block_spmv(J, u), M, b)
    dx, st = s.solve(_gpu(b))
    ep = np.linalg.norm(_np(dx) - xo) / np.linalg.norm(xo)
    s.setup(precision="mixed", ilu_order=order, mg_pre=pre, mg_post=post, mg_alpha=1.25)
    e32 = np.linalg.norm(_np(s.precond(_gpu(v))) - ref) / np.linalg.norm(ref)
    print(f"[asymmetric-cycles] {name} V({pre},{post}) {order}: apply {e64:.1e}, FGMRES {st['iterations']} "
          f"iterations (oracle {so['iterations']}), rel. diff {ep:.1e}, FP32 apply {e32:.1e}", flush=True)
    assert e64 <= 1e-9
    assert so["converged"] and st["converged"]
    assert st["iterations"] == so["iterations"]
    assert ep <= 1e-8
    assert e32 <= 1e-5
    s.close()
