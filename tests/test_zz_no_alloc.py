"""cpr_spmv_noalloc (the SpMV staged through the library's static device
buffer, for callers that cannot allocate) against cpr_spmv, through the C
ABI: identical kernels, so the products must agree bit for bit, on two calls
in a row with the second on a smaller system (the buffer keeps the first
call's contents), then on a system with rate-controlled wells; a system
larger than the buffer is refused with a clear error and leaves y alone."""
import numpy as np
import pytest

from paper_1606_00548_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _solver_and_x(case, seed, bhp=()):
    from paper_1606_00548_amd import cprmi
    s = cprmi.Solver.from_case(case)
    state = [np.concatenate([case[k].ravel(), bhp]) if len(bhp) else case[k] for k in ("x_old", "x")]
    x_old, x_new = (torch.as_tensor(np.ascontiguousarray(a)).cuda() for a in state)
    s.assemble(x_old, x_new, case["dt"])
    x = s.vector()
    x.copy_(torch.as_tensor(np.random.default_rng(seed).standard_normal(tuple(x.shape))))
    return s, x


def test_noalloc_spmv_matches_spmv_on_successive_calls():
    from paper_1606_00548_amd import cprmi
    assert cprmi.load().cpr_spmv_noalloc_max_unknowns() == 1 << 22
    big = synth.black_oil_layered(128, 64, 32, seed=901)        # 786,432 unknowns
    small = synth.oil_water_lognormal(34, 20, 6, seed=902)       # 8,160 unknowns
    for case, seed in ((big, 11), (small, 12)):
        print(f"[no-alloc] {case['name']}", flush=True)
        s, x = _solver_and_x(case, seed)
        ref = s.spmv(x)
        y = torch.full_like(ref, np.nan)
        s.spmv_noalloc(x, y)
        torch.cuda.synchronize()
        assert torch.equal(y, ref)
        s.close()


def test_noalloc_spmv_with_rate_wells():
    case = synth.oil_water_lognormal(16, 12, 4, seed=903)
    case["wells"] = [dict(case["wells"][0], control="rate", rate=40.0),
                     dict(case["wells"][1], control="rate", rate=30.0)]
    print(f"[no-alloc] {case['name']} with two rate wells", flush=True)
    s, x = _solver_and_x(case, 13, bhp=np.array([260.0, 180.0]))
    ref = s.spmv(x)
    y = torch.full_like(ref, np.nan)
    s.spmv_noalloc(x, y)
    torch.cuda.synchronize()
    assert x.numel() == 2 * 16 * 12 * 4 + 2 and torch.equal(y, ref)
    s.close()


def test_noalloc_spmv_refuses_systems_beyond_its_buffer():
    from paper_1606_00548_amd import cprmi
    case = synth.black_oil_layered(128, 128, 96, seed=904)       # 4,718,592 unknowns
    print(f"[no-alloc] {case['name']} (too large)", flush=True)
    s = cprmi.Solver.from_case(case)
    x = s.vector()
    y = torch.full_like(x, 7.0)
    with pytest.raises(cprmi.CPRError) as e:
        s.spmv_noalloc(x, y)
    assert e.value.code == -1 and "static buffer" in str(e.value)
    torch.cuda.synchronize()
    assert bool((y == 7.0).all())
    s.close()
