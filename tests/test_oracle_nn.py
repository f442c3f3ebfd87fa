"""Pins of the FP64 network oracle: central-difference gradients, a delta
kernel reproducing its input, linearity, and the adjoint identities of the
pooling and upsampling steps."""
import numpy as np
import pytest

from oracle import nn
from paper_1606_00548_amd import synth


def test_parameter_count_matches_layout():
    assert nn.num_params() == synth.nn_initial_weights(0).size
    convs, head = nn.unpack(synth.nn_initial_weights(0))
    assert [W.shape[1:] for W, _ in convs] == [tuple(s) for s in synth.NN_CONVS]


def test_delta_kernel_is_identity_and_conv_is_linear():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 4, 6, 8, 5))
    W = np.zeros((27, 5, 5))
    W[13] = np.eye(5)      # centre tap (0, 0, 0)
    assert np.allclose(nn.conv3(x, W, np.zeros(5)), x)
    # a shifted delta picks the neighbour (+1 in x) with zero padding
    W = np.zeros((27, 5, 5))
    W[nn.TAPS.index((0, 0, 1))] = np.eye(5)
    out = nn.conv3(x, W, np.zeros(5))
    assert np.allclose(out[..., :-1, :], x[..., 1:, :]) and np.all(out[..., -1, :] == 0)
    W = rng.standard_normal((27, 5, 3))
    x2 = rng.standard_normal(x.shape)
    lhs = nn.conv3(2.0 * x - 3.0 * x2, W, np.zeros(3))
    rhs = 2.0 * nn.conv3(x, W, np.zeros(3)) - 3.0 * nn.conv3(x2, W, np.zeros(3))
    assert np.allclose(lhs, rhs)


def test_conv_backward_is_the_adjoint():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((1, 4, 4, 4, 3))
    W = rng.standard_normal((27, 3, 2))
    g = rng.standard_normal((1, 4, 4, 4, 2))
    dx, dW, db = nn.conv3_backward(x, W, g)
    assert np.isclose(np.sum(nn.conv3(x, W, np.zeros(2)) * g), np.sum(x * dx))
    assert np.isclose(np.sum(nn.conv3(x, W, np.zeros(2)) * g), np.sum(W * dW))
    assert np.allclose(db, g.sum(axis=(0, 1, 2, 3)))


def test_pool_and_up_adjoints():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 4, 4, 8, 3))
    y = rng.standard_normal((2, 2, 2, 4, 3))
    assert np.isclose(np.sum(nn.pool(x) * y), np.sum(x * nn.pool_backward(y)))
    assert np.isclose(np.sum(nn.up(y) * x), np.sum(y * nn.up_backward(x)))
    # pooling a piecewise-constant field returns its values
    assert np.allclose(nn.pool(nn.up(y)), y)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    theta = synth.nn_initial_weights(11).astype(np.float64)
    # non-zero biases so that no unit sits exactly on a ReLU kink
    convs, head = nn.unpack(theta)
    theta = nn.pack([(W, rng.uniform(0.05, 0.2, b.shape)) for W, b in convs], head)
    x = rng.standard_normal((2, 8, 8, 8, 3))
    t = rng.standard_normal((2, 8, 8, 8))
    y, cache = nn.forward(theta, x)
    L, dy = nn.loss(y, t)
    g = nn.backward(theta, cache, dy)
    # parameters from every layer, weights and biases
    idx = []
    o = 0
    for ci, co in nn.CONVS:
        idx += list(rng.integers(o, o + 27 * ci * co, 4)) + [o + 27 * ci * co + int(rng.integers(co))]
        o += 27 * ci * co + co
    idx += [o + 3, o + 16]
    for i in idx:
        h = 1e-6 * max(1.0, abs(theta[i]))
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (nn.loss(nn.forward(tp, x)[0], t)[0] - nn.loss(nn.forward(tm, x)[0], t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(fd), 1e-3), (i, fd, g[i])


def _ow_system(nx=8, ny=8, nz=8, seed=60):
    from oracle import cpr, model
    case = synth.oil_water_lognormal(nx, ny, nz, seed=seed)
    R, J = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                          case["x_old"], case["x"], case["dt"])
    return case, J, -R, cpr.cpr_setup(J, coarsest=64)


def test_learned_stage_pieces():
    from oracle import cpr, learned
    case, J, b, pc = _ow_system()
    v = b / np.linalg.norm(b)
    rp, dp, rt0 = learned.pressure_stage(pc, v)
    lam = learned.total_mobility(case["fluid"], case["poro"], case["x"])
    feat, s = learned.features(case["perm"], lam, pc["mg"]["levels"][0], rp)
    assert feat.shape == (8, 8, 8, 3)
    assert np.allclose(feat[..., 0].mean(), 0, atol=1e-12) and np.isclose(feat[..., 0].std(), 1)
    assert np.isclose(np.sqrt(np.mean(feat[..., 2] ** 2)), 1.0)
    # a network that outputs zero is rejected by the judge and leaves plain CPR
    theta = np.zeros(nn.num_params())
    z, acc = learned.learned_cpr_apply(pc, v, theta, case["perm"], lam)
    assert not acc
    assert np.allclose(z, cpr.cpr_apply(pc, v), rtol=1e-13, atol=1e-15)
    # with an exact pressure solve nothing is left for the network
    pc1 = cpr.cpr_setup(J, coarsest=10 ** 6)
    rp1, _, _ = learned.pressure_stage(pc1, v)
    assert np.linalg.norm(rp1) <= 1e-10 * np.linalg.norm(rt0)


def test_direction_loss_values():
    rng = np.random.default_rng(12)
    t = rng.standard_normal((2, 2, 2, 4))
    assert nn.loss(-3.0 * t, t)[0] < 1e-15          # any multiple is exact
    u = rng.standard_normal(t.shape)
    y = u - (np.sum(u * t, axis=(1, 2, 3), keepdims=True) / np.sum(t * t, axis=(1, 2, 3), keepdims=True)) * t
    assert abs(nn.loss(y, t)[0] - 1.0) < 1e-12       # orthogonal: nothing explained
    assert np.isclose(nn.loss(5.0 * u, t)[0], nn.loss(u, t)[0])


def test_adam_first_step_moves_by_lr():
    theta = np.zeros(4)
    g = np.array([1.0, -2.0, 0.5, 0.0])
    t2, m, v = nn.adam_step(theta, g, np.zeros(4), np.zeros(4), 1, lr=1e-3)
    # bias-corrected first step: -lr * sign(g) (and 0 where g = 0)
    assert np.allclose(t2, -1e-3 * np.sign(g), atol=1e-10)


@pytest.mark.parametrize("decoupling,composition", [("abf", "two-stage"), ("qimpes", "fpf"), ("abf", "fpf")])
def test_rejected_network_leaves_each_cpr_variant(decoupling, composition):
    from oracle import cpr, learned
    case, J, b, _ = _ow_system()
    pc = cpr.cpr_setup(J, coarsest=64, decoupling=decoupling)
    v = b / np.linalg.norm(b)
    lam = learned.total_mobility(case["fluid"], case["poro"], case["x"])
    z, acc = learned.learned_cpr_apply(pc, v, np.zeros(nn.num_params()), case["perm"], lam,
                                       composition=composition)
    assert not acc
    assert np.allclose(z, cpr.cpr_apply(pc, v, composition=composition), rtol=1e-13, atol=1e-15)
