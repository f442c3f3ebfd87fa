"""Parity of the GPU pressure-correction network (BF16 matrix cores, FP32
accumulation) and of the learned CPR stage with the FP64 oracle.

Tolerances (parameters are BF16-exact, see _theta): BF16 operands carry 8
significant bits (relative rounding 2^-9 ~ 2e-3 per operand); sums over
27*64 products and seven stacked convolutions grow that to ~1e-2, so forward
outputs are compared in relative 2-norm at 3e-2 and gradients at 2e-2 (3e-2
per layer) in a regime where no ReLU can change state; where ReLU masks can
flip, only the gradient direction is required to agree (cosine >= 0.99).
FP32 features at 1e-5, FP64 residuals at 1e-9 relative.
"""
import numpy as np
import pytest

from oracle import cpr, learned, model, nn
from paper_1606_00548_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _bf16(a):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    a = np.asarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def _theta(seed):
    """Parameters that BF16 represents exactly: the network's convolutions run
    with BF16 weights, so the oracle then sees the very same weights and the
    comparison measures activation and gradient rounding only."""
    rng = np.random.default_rng(seed)
    th = synth.nn_initial_weights(seed).astype(np.float64)
    convs, head = nn.unpack(th)
    return _bf16(nn.pack([(W, rng.uniform(-0.05, 0.1, b.shape)) for W, b in convs], head))


def _rel(a, b):
    return np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b)


def _net(shape, batch):
    from paper_1606_00548_amd import cprmi
    nz, ny, nx = shape
    return cprmi.Network(nx, ny, nz, max_batch=batch)


# (batch, (nz, ny, nx)): the small grid runs every convolution with its
# K-steps split over a workgroup's waves; the larger one (>= 65,536 cells)
# runs the full-resolution convolutions with whole-tile waves and, for
# inference, the head fused into the last convolution.
SHAPES = [(2, (8, 16, 16)), (1, (16, 64, 64))]


@pytest.mark.parametrize("batch,shape", SHAPES)
def test_forward_matches_oracle(batch, shape):
    theta = _theta(1)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((batch,) + shape + (3,)).astype(np.float32)
    net = _net(shape, batch)
    net.set_params(theta.astype(np.float32))
    xg = torch.from_numpy(x).cuda()
    y = net.forward(xg).cpu().numpy()
    yo, _ = nn.forward(theta.astype(np.float32).astype(np.float64), x.astype(np.float64))
    print(f"[nn] forward {batch}x{shape}: rel. diff {_rel(y, yo):.2e}")
    assert _rel(y, yo) <= 3e-2
    # the inference form: same kernels, head possibly fused (FP32 order only)
    yi = np.stack([net.infer(xg[i:i + 1].contiguous()).cpu().numpy()[0] for i in range(batch)])
    print(f"[nn] inference vs forward rel. diff {_rel(yi, y):.2e}")
    assert _rel(yi, y) <= 1e-5


def _grads(theta, seed, batch=2, shape=(8, 16, 16)):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((batch,) + shape + (3,)).astype(np.float32)
    dy = rng.standard_normal((batch,) + shape).astype(np.float32)
    net = _net(shape, batch)
    net.set_params(theta.astype(np.float32))
    net.forward(torch.from_numpy(x).cuda())
    g = net.backward(torch.from_numpy(dy).cuda()).cpu().numpy().astype(np.float64)
    yo, cache = nn.forward(theta, x.astype(np.float64))
    return g, nn.backward(theta, cache, dy.astype(np.float64))


@pytest.mark.parametrize("batch,shape", SHAPES)
def test_backward_matches_oracle_without_relu_flips(batch, shape):
    # Large biases keep every ReLU open, so no unit can switch sides under
    # BF16 rounding: the gradient then differs only by rounding (~1e-2);
    # a wrong index, tap or dropped term would give an O(1) difference.
    convs, head = nn.unpack(synth.nn_initial_weights(3).astype(np.float64))
    theta = _bf16(nn.pack([(0.3 * W, np.full(b.shape, 3.0)) for W, b in convs], head))
    g, go = _grads(theta, 4, batch, shape)
    print(f"[nn] gradient {batch}x{shape}: rel. diff (open ReLUs) {_rel(g, go):.2e}")
    assert _rel(g, go) <= 2e-2
    o = 0
    for k, (ci, co) in enumerate(nn.CONVS):
        m = 27 * ci * co + co
        r = _rel(g[o:o + m], go[o:o + m])
        print(f"[nn]   conv {k}: {r:.2e}")
        assert r <= 3e-2
        o += m
    assert _rel(g[o:], go[o:]) <= 2e-2


def test_backward_direction_matches_oracle():
    # With half the units near their kink, BF16 rounding flips some ReLU
    # masks and moves gradients by several percent (the FP64 oracle itself
    # moves as much when only its weights are rounded to BF16); the
    # direction must still agree.
    g, go = _grads(_theta(3), 4)
    cos = float(np.dot(g, go) / (np.linalg.norm(g) * np.linalg.norm(go)))
    print(f"[nn] gradient rel. diff {_rel(g, go):.2e}, cosine {cos:.5f}")
    assert cos >= 0.99 and _rel(g, go) <= 0.15


def test_train_step_loss_matches_oracle_and_decreases():
    theta = _theta(5)
    rng = np.random.default_rng(6)
    x = rng.standard_normal((2, 8, 16, 16, 3)).astype(np.float32)
    t = rng.standard_normal((2, 8, 16, 16)).astype(np.float32)
    net = _net((8, 16, 16), 2)
    net.set_params(theta.astype(np.float32))
    xg, tg = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    L0 = net.train_step(xg, tg, lr=1e-3)
    yo, _ = nn.forward(theta.astype(np.float32).astype(np.float64), x.astype(np.float64))
    Lo, _ = nn.loss(yo, t.astype(np.float64))
    assert abs(L0 - Lo) <= 3e-2 * Lo
    for _ in range(40):
        L = net.train_step(xg, tg, lr=2e-3)
    print(f"[nn] loss {L0:.4f} -> {L:.4f} after 41 Adam steps")
    assert L < 0.7 * L0
    # parameters round-trip
    th = net.get_params()
    assert th.shape == (nn.num_params(),) and np.all(np.isfinite(th))


def test_resumed_training_reproduces_the_uninterrupted_run(tmp_path):
    # parameters, Adam moments and step, and the shuffling generator from the
    # checkpoint of epoch 1: the second epoch then repeats the uninterrupted
    # run bit for bit (the training kernels are deterministic)
    from paper_1606_00548_amd import train
    rng = np.random.default_rng(8)
    X = torch.from_numpy(rng.standard_normal((6, 8, 16, 16, 3)).astype(np.float32)).cuda()
    T = torch.from_numpy(rng.standard_normal((6, 8, 16, 16)).astype(np.float32)).cuda()
    th_a, hist_a = train.train(X, T, 2, batch=2, val_frac=0.34, log=None)
    ck = str(tmp_path / "ck.npz")
    th_1, _ = train.train(X, T, 1, batch=2, val_frac=0.34, log=None, checkpoint=ck)
    saved = train.load_checkpoint(ck)
    assert saved["epoch"] == 1 and saved["adam_step"] == 2 and np.array_equal(saved["theta"], th_1)
    th_b, hist_b = train.train(X, T, 2, batch=2, val_frac=0.34, log=None, resume=ck)
    print(f"[nn] resume: losses {[h['train_loss'] for h in hist_a]} / {[h['train_loss'] for h in hist_b]}")
    assert np.array_equal(th_a, th_b)
    assert [h["train_loss"] for h in hist_a] == [h["train_loss"] for h in hist_b]
    assert not np.array_equal(th_1, th_b)


def _ow_case():
    return synth.oil_water_lognormal(16, 16, 8, seed=70)


def test_pressure_stage_and_features_match_oracle():
    from paper_1606_00548_amd import cprmi
    case = _ow_case()
    s = cprmi.Solver.from_case(case)
    rhs = s.assemble(torch.as_tensor(case["x_old"]).cuda(), torch.as_tensor(case["x"]).cuda(), case["dt"])
    s.setup()
    R, J = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                          case["x_old"], case["x"], case["dt"])
    pc = cpr.cpr_setup(J)
    b = -R
    v = b / np.linalg.norm(b)
    rp_g, dp_g = s.pressure_stage(torch.as_tensor(v).cuda().contiguous())
    rp_o, dp_o, rt0 = learned.pressure_stage(pc, v)
    assert np.linalg.norm(dp_g.cpu().numpy() - dp_o) <= 1e-10 * np.linalg.norm(dp_o)
    assert np.linalg.norm(rp_g.cpu().numpy() - rp_o) <= 1e-9 * np.linalg.norm(rt0)
    f_g, sc_g = s.features(torch.as_tensor(rp_o).cuda().contiguous())
    lam = learned.total_mobility(case["fluid"], case["poro"], case["x"])
    f_o, sc_o = learned.features(case["perm"], lam, pc["mg"]["levels"][0], rp_o)
    assert abs(sc_g - sc_o) <= 1e-12 * sc_o
    assert np.allclose(f_g.cpu().numpy(), f_o, rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_learned_cpr_apply_matches_oracle(precision):
    # One CPR application with the learned stage against the oracle's: the
    # network runs in BF16 on the GPU and in FP64 in the oracle, so only the
    # network's correction (z_learned - z_plain) carries the network
    # tolerance; everything else is FP64 (or the FP32 preconditioner).
    from paper_1606_00548_amd import cprmi
    case = _ow_case()
    theta = _theta(9)
    s = cprmi.Solver.from_case(case)
    s.assemble(torch.as_tensor(case["x_old"]).cuda(), torch.as_tensor(case["x"]).cuda(), case["dt"])
    R, J = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                          case["x_old"], case["x"], case["dt"])
    pc = cpr.cpr_setup(J)
    b = -R
    v = b / np.linalg.norm(b)
    lam = learned.total_mobility(case["fluid"], case["poro"], case["x"])
    z_o, acc = learned.learned_cpr_apply(pc, v, theta, case["perm"], lam)
    z_p = cpr.cpr_apply(pc, v)
    s.attach_network(theta.astype(np.float32))
    s.setup(learned=1, precision=precision)
    z_g = s.precond(torch.as_tensor(v).cuda().contiguous()).cpu().numpy()
    corr = np.linalg.norm(z_o - z_p)
    err = np.linalg.norm(z_g - z_o)
    base = 1e-9 if precision == "fp64" else 1e-5
    print(f"[learned] {precision} apply: accepted {acc}, |correction| {corr:.3e}, |gpu - oracle| {err:.3e}")
    assert acc and corr > 1e-3 * np.linalg.norm(z_p)
    assert err <= 3e-2 * corr + base * np.linalg.norm(z_o)
    # a network that outputs zero is rejected: plain CPR is what remains
    s.attach_network(np.zeros(nn.num_params(), np.float32))
    s.setup(learned=1, precision=precision)
    z0 = s.precond(torch.as_tensor(v).cuda().contiguous()).cpu().numpy()
    assert np.linalg.norm(z0 - z_p) <= base * np.linalg.norm(z_p)


@pytest.mark.parametrize("decoupling,composition", [("abf", "two-stage"), ("qimpes", "fpf"),
                                                    ("abf", "fpf")])
def test_learned_stage_in_cpr_variants_matches_oracle(decoupling, composition):
    # the learned correction inside the ABF-decoupled and the F-P-F
    # preconditioner (FP64), tolerances as for the default one
    from paper_1606_00548_amd import cprmi
    case = _ow_case()
    theta = _theta(9)
    s = cprmi.Solver.from_case(case)
    s.assemble(torch.as_tensor(case["x_old"]).cuda(), torch.as_tensor(case["x"]).cuda(), case["dt"])
    R, J = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                          case["x_old"], case["x"], case["dt"])
    pc = cpr.cpr_setup(J, decoupling=decoupling)
    v = -R / np.linalg.norm(R)
    lam = learned.total_mobility(case["fluid"], case["poro"], case["x"])
    z_o, acc = learned.learned_cpr_apply(pc, v, theta, case["perm"], lam, composition=composition)
    z_p = cpr.cpr_apply(pc, v, composition=composition)
    s.attach_network(theta.astype(np.float32))
    s.setup(learned=1, decoupling=decoupling, composition=composition)
    z_g = s.precond(torch.as_tensor(v).cuda().contiguous()).cpu().numpy()
    corr = np.linalg.norm(z_o - z_p)
    err = np.linalg.norm(z_g - z_o)
    print(f"[learned] {decoupling}/{composition} apply: accepted {acc}, |correction| {corr:.3e}, "
          f"|gpu - oracle| {err:.3e}")
    if acc:
        assert err <= 3e-2 * corr + 1e-9 * np.linalg.norm(z_o)
    else:
        assert err <= 1e-9 * np.linalg.norm(z_o)
    s.close()


def test_learned_solve_keeps_accuracy_and_counts_decisions():
    from paper_1606_00548_amd import cprmi
    case = _ow_case()
    s = cprmi.Solver.from_case(case)
    rhs = s.assemble(torch.as_tensor(case["x_old"]).cuda(), torch.as_tensor(case["x"]).cuda(), case["dt"])
    s.attach_network(_theta(9).astype(np.float32))
    for prec in ("fp64", "mixed"):
        s.setup(learned=1, precision=prec)
        dx, st = s.solve(rhs)
        R, J = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                              case["x_old"], case["x"], case["dt"])
        b = -R
        res = np.linalg.norm(b - cpr.block_spmv(J, dx.cpu().numpy())) / np.linalg.norm(b)
        print(f"[learned] {prec}: iterations {st['iterations']}, accepted {st['nn_accepted']}, "
              f"rejected {st['nn_rejected']}, true rel. residual {res:.2e}")
        assert st["status"] == 0 and res <= 1e-6
        assert st["nn_accepted"] + st["nn_rejected"] == st["iterations"]
    # without a network the option is refused
    s.attach_network(None)
    with pytest.raises(cprmi.CPRError):
        s.setup(learned=1)


def test_nan_network_always_falls_back_to_plain_cpr():
    # a network whose output is NaN (NaN head weights: the ReLUs inside would
    # turn NaN activations into zeros) fails the judge on every application:
    # the solve is bit for bit the plain CPR solve, every decision a reject
    from paper_1606_00548_amd import cprmi
    case = _ow_case()
    s = cprmi.Solver.from_case(case)
    rhs = s.assemble(torch.as_tensor(case["x_old"]).cuda(), torch.as_tensor(case["x"]).cuda(), case["dt"])
    theta = _theta(9).astype(np.float32)
    theta[-17:] = np.nan          # the 1x1x1 head: 16 weights and its bias, last in the layout
    s.attach_network(theta)
    for prec in ("fp64", "mixed"):
        s.setup(precision=prec)
        dx0, st0 = s.solve(rhs)
        x0 = dx0.cpu().numpy()
        s.setup(precision=prec, learned=1)
        dx1, st1 = s.solve(rhs)
        print(f"[learned] NaN network, {prec}: {st1['iterations']} iterations, accepted {st1['nn_accepted']}, "
              f"rejected {st1['nn_rejected']}")
        assert st1["nn_accepted"] == 0 and st1["nn_rejected"] == st1["iterations"] == st0["iterations"]
        assert np.array_equal(dx1.cpu().numpy(), x0)
    s.close()


def test_train_step_gradient_and_adam_match_oracle():
    # One cpr_nn_train_step from zero Adam moments, read back through the
    # checkpoint entry points.  The first moment is (1 - beta1) g, so it
    # gives the gradient the library formed from its own direction-loss
    # gradient and backward pass.  Checked part by part:
    #  * loss and dL/dy: the oracle's nn.loss evaluated at the GPU's own
    #    forward output gives the loss to FP32 rounding, and backward() of
    #    its dL/dy gives the train step's gradient to 1e-3 (FP32 dL/dy);
    #  * end to end against nn.loss + nn.backward at the oracle's output:
    #    the loss's gradient is orthogonal to y (the loss ignores scale), so
    #    BF16 rounding of y is amplified and only the direction is held
    #    (cosine >= 0.99), as for the backward pass with ReLU flips;
    #  * Adam: the second moment, the parameters after the step and after a
    #    second step (bias correction at k = 2) follow nn.adam_step applied
    #    to the library's gradient, to FP32 rounding.
    convs, head = nn.unpack(synth.nn_initial_weights(9).astype(np.float64))
    theta = _bf16(nn.pack([(0.3 * W, np.full(b.shape, 3.0)) for W, b in convs], head))
    rng = np.random.default_rng(10)
    shape, B = (8, 16, 16), 2
    x = rng.standard_normal((B,) + shape + (3,)).astype(np.float32)
    yo, cache = nn.forward(theta, x.astype(np.float64))
    t = np.stack([yo[b] / np.linalg.norm(yo[b]) + rng.standard_normal(shape) / np.sqrt(yo[b].size)
                  for b in range(B)]).astype(np.float32)
    Lo, dyo = nn.loss(yo, t.astype(np.float64))
    go = nn.backward(theta, cache, dyo)
    xg, tg = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    # the GPU's forward output and backward() of the oracle's dL/dy at it
    net2 = _net(shape, B)
    net2.set_params(theta.astype(np.float32))
    yg = net2.forward(xg).cpu().numpy().astype(np.float64)
    Lg, dyg = nn.loss(yg, t.astype(np.float64))
    gb = net2.backward(torch.from_numpy(dyg.astype(np.float32)).cuda()).cpu().numpy().astype(np.float64)
    net = _net(shape, B)
    net.set_params(theta.astype(np.float32))
    lr = 1e-3
    L0 = net.train_step(xg, tg, lr=lr)
    m1, v1, k1 = net.get_adam()
    th1 = net.get_params().astype(np.float64)
    assert k1 == 1
    g1 = m1.astype(np.float64) / (1 - 0.9)
    cos = float(np.dot(g1, go) / (np.linalg.norm(g1) * np.linalg.norm(go)))
    print(f"[nn] train step: loss {L0:.6f} (oracle at the GPU output {Lg:.6f}, at its own {Lo:.6f}); "
          f"gradient vs backward(oracle dL/dy) {_rel(g1, gb):.2e}, vs oracle {_rel(g1, go):.2e}, cosine {cos:.5f}")
    assert abs(L0 - Lg) <= 1e-5 * Lg and abs(L0 - Lo) <= 1e-2 * Lo
    assert _rel(g1, gb) <= 1e-3
    assert cos >= 0.99 and _rel(g1, go) <= 0.15
    # Adam from zero moments (step 1) and the next step (step 2)
    _, m_ref, v_ref = nn.adam_step(theta, g1, 0.0, 0.0, 1, lr=lr)
    assert np.allclose(v1, v_ref, rtol=3e-5, atol=0)
    th_ref, _, _ = nn.adam_step(theta, g1, np.zeros_like(g1), np.zeros_like(g1), 1, lr=lr)
    tol = 2e-5 * lr + 4 * 2.0 ** -24 * np.abs(theta)
    assert np.all(np.abs(th1 - th_ref) <= tol), np.abs(th1 - th_ref).max()
    net.train_step(xg, tg, lr=lr)
    m2, v2, k2 = net.get_adam()
    th2 = net.get_params().astype(np.float64)
    assert k2 == 2
    g2 = (m2.astype(np.float64) - 0.9 * m1) / (1 - 0.9)
    th2_ref, _, v2_ref = nn.adam_step(th1, g2, m1.astype(np.float64), v1.astype(np.float64), 2, lr=lr)
    assert np.allclose(v2, v2_ref, rtol=3e-5, atol=1e-30)
    tol = 2e-5 * lr + 4 * 2.0 ** -24 * np.abs(th1)
    assert np.all(np.abs(th2 - th2_ref) <= tol), np.abs(th2 - th2_ref).max()
    net.close()
    net2.close()


def _level_case():
    # 64 x 64 x 16: level 1 (32 x 32 x 8, 8,192 cells) is smoothed by
    # multi-block kernels, the levels from 16 x 16 x 4 down run in one
    # workgroup
    return synth.oil_water_lognormal(64, 64, 16, seed=73)


def test_level_pressure_stage_and_features_match_oracle():
    from paper_1606_00548_amd import cprmi
    case = _level_case()
    s = cprmi.Solver.from_case(case)
    s.assemble(torch.as_tensor(case["x_old"]).cuda(), torch.as_tensor(case["x"]).cuda(), case["dt"])
    s.setup(nn_level=1)
    R, J = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                          case["x_old"], case["x"], case["dt"])
    pc = cpr.cpr_setup(J)
    b = -R
    v = b / np.linalg.norm(b)
    rp_g, _ = s.pressure_stage(torch.as_tensor(v).cuda().contiguous(), level=1)
    rp_o = learned.level_residual(pc, v, 1)
    d = np.linalg.norm(rp_g.cpu().numpy() - rp_o) / np.linalg.norm(rp_o)
    print(f"[learned-level] level-1 residual rel. diff {d:.1e}")
    assert rp_g.shape == rp_o.shape and d <= 1e-9
    f_g, sc_g = s.features(torch.as_tensor(rp_o).cuda().contiguous())
    lam = learned.total_mobility(case["fluid"], case["poro"], case["x"])
    lnk, lnl = learned.level_fields(case["perm"], lam, 1)
    f_o, sc_o = learned.level_features(lnk, lnl, pc["mg"]["levels"][1], rp_o)
    assert abs(sc_g - sc_o) <= 1e-12 * sc_o
    assert np.allclose(f_g.cpu().numpy(), f_o, rtol=1e-5, atol=1e-5)
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_level_learned_cpr_apply_matches_oracle(precision):
    # the learned correction inside the cycle on level 1 against the oracle,
    # with the tolerances of the fine-level stage: only the network's
    # correction carries the BF16 tolerance
    from paper_1606_00548_amd import cprmi
    case = _level_case()
    theta = _theta(9)
    s = cprmi.Solver.from_case(case)
    s.assemble(torch.as_tensor(case["x_old"]).cuda(), torch.as_tensor(case["x"]).cuda(), case["dt"])
    R, J = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                          case["x_old"], case["x"], case["dt"])
    pc = cpr.cpr_setup(J)
    b = -R
    v = b / np.linalg.norm(b)
    lam = learned.total_mobility(case["fluid"], case["poro"], case["x"])
    z_o, acc = learned.learned_cpr_apply(pc, v, theta, case["perm"], lam, level=1)
    z_p = cpr.cpr_apply(pc, v)
    s.attach_network(theta.astype(np.float32))
    s.setup(learned=1, nn_level=1, precision=precision)
    z_g = s.precond(torch.as_tensor(v).cuda().contiguous()).cpu().numpy()
    corr = np.linalg.norm(z_o - z_p)
    err = np.linalg.norm(z_g - z_o)
    base = 1e-9 if precision == "fp64" else 1e-5
    print(f"[learned-level] {precision} apply: accepted {acc}, |correction| {corr:.3e}, |gpu - oracle| {err:.3e}")
    assert acc and corr > 1e-4 * np.linalg.norm(z_p)
    assert err <= 3e-2 * corr + base * np.linalg.norm(z_o)
    # a network that outputs zero is rejected: plain CPR remains
    s.attach_network(np.zeros(nn.num_params(), np.float32))
    s.setup(learned=1, nn_level=1, precision=precision)
    z0 = s.precond(torch.as_tensor(v).cuda().contiguous()).cpu().numpy()
    assert np.linalg.norm(z0 - z_p) <= base * np.linalg.norm(z_p)
    # a level inside the single-workgroup cycle is refused
    with pytest.raises(cprmi.CPRError):
        s.setup(learned=1, nn_level=2)
    s.close()


@pytest.mark.parametrize("make,expected", [
    (lambda: synth.oil_water_lognormal(64, 64, 16, seed=73), 0),      # level 1: 8,192 cells
    (lambda: synth.black_oil_layered(128, 128, 32, seed=2000), 1),    # level 1: 65,536 cells
    (lambda: synth.oil_water_lognormal(48, 40, 16, seed=74), 0),      # level 1: 24 x 20 x 8, too small
    (lambda: synth.black_oil_lattice(256, 256, 64, seed=5000), 1),    # level 1: 2^19 cells
])
def test_automatic_level_choice(make, expected):
    # nn_level = CPR_NN_LEVEL_AUTO (the default) resolves at setup to the
    # coarsest level of at least 2^19 cells, else of at least 2^16 cells
    # (among the levels the stage can run on), else the fine level
    from paper_1606_00548_amd import cprmi
    case = make()
    s = cprmi.Solver.from_case(case)
    s.assemble(torch.as_tensor(case["x_old"]).cuda(), torch.as_tensor(case["x"]).cuda(), case["dt"])
    s.setup()
    assert s.nn_level() == expected
    s.setup(nn_level=0)
    assert s.nn_level() == 0
    s.close()


@pytest.mark.parametrize("order", ["red-black", "tiles"])
@pytest.mark.parametrize("level", [0, 1])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_learned_apply_with_the_tuned_cycle_matches_oracle(precision, level, order):
    # the learned correction with the V(2,2) cycle whose coarse corrections
    # are scaled by 1.25, on the fine level and inside the cycle on level 1,
    # in both ILU orders, against the oracle; tolerances of the V(1,1) tests
    from paper_1606_00548_amd import cprmi
    case = _level_case()
    theta = _theta(9)
    s = cprmi.Solver.from_case(case)
    s.assemble(torch.as_tensor(case["x_old"]).cuda(), torch.as_tensor(case["x"]).cuda(), case["dt"])
    R, J = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                          case["x_old"], case["x"], case["dt"])
    pc = cpr.cpr_setup(J, pre=2, post=2, ilu_order=order)
    b = -R
    v = b / np.linalg.norm(b)
    lam = learned.total_mobility(case["fluid"], case["poro"], case["x"])
    z_o, acc = learned.learned_cpr_apply(pc, v, theta, case["perm"], lam, level=level, alpha=1.25)
    z_p = cpr.cpr_apply(pc, v, alpha=1.25)
    s.attach_network(theta.astype(np.float32))
    s.setup(learned=1, nn_level=level, precision=precision, ilu_order=order, mg_pre=2, mg_post=2, mg_alpha=1.25)
    z_g = s.precond(torch.as_tensor(v).cuda().contiguous()).cpu().numpy()
    corr = np.linalg.norm(z_o - z_p)
    err = np.linalg.norm(z_g - z_o)
    base = 1e-9 if precision == "fp64" else 1e-5
    print(f"[learned-tuned] {precision} level {level} {order}: accepted {acc}, |correction| {corr:.3e}, "
          f"|gpu - oracle| {err:.3e} ({err / np.linalg.norm(z_o):.1e} relative)", flush=True)
    if acc:
        assert corr > 1e-4 * np.linalg.norm(z_p)
        assert err <= 3e-2 * corr + base * np.linalg.norm(z_o)
    else:
        assert err <= base * np.linalg.norm(z_o)
    s.attach_network(None)
    s.close()
