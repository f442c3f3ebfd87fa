"""A caller's device allocator (cpr_set_allocator): torch's caching
allocator supplies every block of a context and of its network, every block
goes back when the context is destroyed, and results are bit-identical to
those of a context on hipMalloc."""
import numpy as np
import pytest

from paper_1606_00548_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _run(case, theta):
    from paper_1606_00548_amd import cprmi
    s = cprmi.Solver.from_case(case)
    rhs = s.assemble(torch.as_tensor(case["x_old"]).cuda(), torch.as_tensor(case["x"]).cuda(), case["dt"])
    s.setup()
    dx, st = s.solve(rhs)
    s.attach_network(theta)
    s.setup(precision="mixed", learned=1)
    dx2, st2 = s.solve(rhs)
    torch.cuda.synchronize()
    out = (dx.cpu().numpy(), dx2.cpu().numpy(), st["iterations"], st2["iterations"])
    s.close()
    return out


def test_torch_caching_allocator_supplies_library_memory():
    from paper_1606_00548_amd import cprmi, train
    case = synth.oil_water_lognormal(16, 16, 8, seed=71)
    theta = np.load(train.weights_path("oil-water"))
    live, count = {}, [0]

    def alloc(n):
        p = torch.cuda.caching_allocator_alloc(n)
        live[p] = n
        count[0] += 1
        return p

    def free(p):
        torch.cuda.caching_allocator_delete(p)
        live.pop(p)

    cprmi.set_allocator(alloc, free)
    try:
        got = _run(case, theta)
    finally:
        cprmi.set_allocator()
    print(f"[allocator] {count[0]} blocks from the caching allocator, {len(live)} left after destroy")
    assert count[0] > 20 and not live
    ref = _run(case, theta)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]) and got[2:] == ref[2:]
    # exactly one callback is rejected and leaves the default in place
    one = cprmi._ALLOC_FN(lambda n, u: None)
    assert cprmi.load().cpr_set_allocator(one, cprmi._FREE_FN(), None) == -1
    assert np.array_equal(_run(case, theta)[0], ref[0])
