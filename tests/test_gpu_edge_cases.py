"""Degenerate shapes and inputs on the GPU against the oracle: one-cell-thick
grids (1-D, 2-D), the smallest grid the layout allows (2 x 1 x 1), a grid with
no wells, and wells on the grid boundary of a one-layer grid."""
import numpy as np
import pytest

from oracle import cpr, krylov, model, newton
from paper_1606_00548_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _gpu(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


SHAPES = [(2, 1, 1), (4, 1, 1), (2, 3, 1), (6, 1, 5), (8, 8, 1), (10, 1, 1), (4, 7, 3)]


@pytest.mark.parametrize("model_name", ["oil-water", "black-oil"])
@pytest.mark.parametrize("shape", SHAPES)
def test_thin_and_tiny_grids_match_oracle(shape, model_name):
    from paper_1606_00548_amd import cprmi
    nx, ny, nz = shape
    if model_name == "oil-water":
        case = synth.oil_water_lognormal(nx, ny, nz, seed=90 + nx)
    else:
        case = synth.black_oil_layered(nx, ny, nz, seed=91 + nx)
        case["wells"] = [synth.well(0, 0, nz, "inj", 300.0), synth.well(nx - 1, ny - 1, nz, "prod", 150.0)]
    x = synth.random_state_perturbation(case, 3)
    R, J = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                          case["x_old"], x, case["dt"])
    s = cprmi.Solver.from_case(case)
    rhs = s.assemble(_gpu(case["x_old"]), _gpu(x), case["dt"])
    torch.cuda.synchronize()
    Jg = s.export_jacobian().cpu().numpy()
    rowscale = np.abs(J).max(axis=(0, 2), keepdims=True)
    assert np.all(np.abs(Jg - J) <= 1e-11 * np.abs(J) + 1e-13 * rowscale)
    b = -R
    assert np.all(np.abs(rhs.cpu().numpy() - b) <= 1e-10 * np.abs(b) + 1e-12 * np.abs(b).max())
    s.setup()
    dx, st = s.solve(rhs)
    pc = cpr.cpr_setup(J)
    xo, so = krylov.fgmres(lambda u: cpr.block_spmv(J, u), lambda u: cpr.cpr_apply(pc, u), b)
    assert st["status"] == 0 and so["converged"] and st["iterations"] == so["iterations"]
    assert np.linalg.norm(dx.cpu().numpy() - xo) <= 1e-8 * np.linalg.norm(xo)
    s.close()


def test_no_wells_time_step():
    # without wells only the small imbalance of the initial state (built with
    # one initialisation density, while phase densities vary with pressure)
    # drives flow: the step settles in a couple of Newton iterations
    from paper_1606_00548_amd import cprmi
    case = synth.oil_water_lognormal(8, 6, 4, seed=95)
    case["wells"] = []
    s = cprmi.Solver.from_case(case)
    xg, st = s.time_step(_gpu(case["x_old"]), 1.0)
    xo, so = newton.time_step(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                              case["x_old"], 1.0)
    print(f"[edge] no wells: |b0| gpu {st['history']['bnorm'][0]:.2e}, oracle {so['history']['bnorm'][0]:.2e}")
    assert st["converged"] and so["converged"]
    assert st["newton_iterations"] == so["newton_iterations"] <= 3
    assert np.allclose(xg.cpu().numpy(), xo, rtol=1e-10, atol=1e-12)
    s.close()


def test_boundary_wells_and_single_layer():
    # wells in the last row/column of a one-layer grid: the perforation's
    # missing neighbours are on the no-flow boundary
    from paper_1606_00548_amd import cprmi
    case = synth.oil_water_lognormal(12, 9, 1, seed=96)
    case["wells"] = [synth.well(11, 0, 1, "inj", 300.0), synth.well(0, 8, 1, "prod", 150.0)]
    s = cprmi.Solver.from_case(case)
    xg, sg = s.time_step(_gpu(case["x_old"]), 1.0)
    xo, so = newton.time_step(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                              case["x_old"], 1.0)
    assert sg["converged"] and so["converged"] and sg["newton_iterations"] == so["newton_iterations"]
    assert sg["history"]["linear_iterations"] == so["history"]["linear_iterations"]
    assert np.linalg.norm(xg.cpu().numpy() - xo) <= 1e-8 * np.linalg.norm(xo)
    s.close()
