"""The single-workgroup kernel of the small multigrid levels in both of its
forms: with the levels staged in LDS (their arrays fit in 96 KB) and with
them in global memory (they do not).  On a 64x48x16 grid the first fused
level has 768 cells (FP64 and FP32 staged); on 96x96x16 it has 2,304 cells
(FP64 in global memory, FP32 staged).  Each form against the oracle: one
FP64 CPR application to 1e-9, and a fixed 5-step FGMRES path with the
V(2,2), alpha = 1.25 cycle (rtol = 0) to 1e-8; the FP32 preconditioner's
application within 1e-5 of the FP64 oracle's.  Tolerances as in the other
parity tests."""
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


CASES = {"bo-64x48x16": lambda: synth.black_oil_layered(64, 48, 16, seed=121),
         "bo-96x96x16": lambda: synth.black_oil_channelised(96, 96, 16, seed=122)}
FUSED_CELLS = {"bo-64x48x16": 768, "bo-96x96x16": 2304}


@pytest.fixture(scope="module", params=list(CASES))
def system(request):
    case = CASES[request.param]()
    x = synth.random_state_perturbation(case, 23)
    R, J = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                          case["x_old"], x, case["dt"])
    print(f"[coarse-levels] case {request.param}", flush=True)
    return request.param, case, J, -R


def _solver(case):
    from paper_1606_00548_amd import cprmi
    return cprmi.Solver.from_case(case)


def test_fused_level_sizes(system):
    name, case, J, b = system
    s = _solver(case)
    s.import_jacobian(J)
    s.setup()
    shapes = []
    lv = 0
    while (sh := s.mg_level_shape(lv)) is not None:
        shapes.append(int(np.prod(sh)))
        lv += 1
    # the first level of at most 4096 cells below the fine one
    first = next(n for n in shapes[1:] if n <= 4096)
    assert first == FUSED_CELLS[name], shapes
    s.close()


@pytest.mark.parametrize("pre,post,alpha", [(1, 1, 1.0), (2, 2, 1.25)])
def test_apply_and_fixed_path_match_oracle(system, pre, post, alpha):
    name, case, J, b = system
    s = _solver(case)
    s.import_jacobian(J)
    pc = cpr.cpr_setup(J, pre=pre, post=post)
    M = lambda u: cpr.cpr_apply(pc, u, alpha=alpha)
    v = b / np.linalg.norm(b)
    ref = M(v)
    s.setup(mg_pre=pre, mg_post=post, mg_alpha=alpha, rtol=0.0, max_iter=5)
    z = _np(s.precond(_gpu(v)))
    e64 = np.linalg.norm(z - ref) / np.linalg.norm(ref)
    dx, st = s.solve(_gpu(b))
    xo, so = krylov.fgmres(lambda u: cpr.block_spmv(J, u), M, b, rtol=0.0, max_iter=5)
    ep = np.linalg.norm(_np(dx) - xo) / np.linalg.norm(xo)
    s.setup(precision="mixed", mg_pre=pre, mg_post=post, mg_alpha=alpha)
    z32 = _np(s.precond(_gpu(v)))
    e32 = np.linalg.norm(z32 - ref) / np.linalg.norm(ref)
    print(f"[coarse-levels] {name} V({pre},{post}) alpha {alpha}: apply {e64:.1e}, 5-step path {ep:.1e}, "
          f"FP32 apply {e32:.1e}", flush=True)
    assert e64 <= 1e-9
    assert st["iterations"] == so["iterations"] == 5
    assert ep <= 1e-8
    assert e32 <= 1e-5
    s.close()
