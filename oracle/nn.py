"""Oracle: the pressure-correction network, forward and backward, in FP64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  The paper has no
learned component; this is the project's own design, shared with the GPU
kernels:

  3-D U-Net on channels-last tensors x[b, z, y, x, c], four levels with 16,
  32, 64, 64 channels, one 3x3x3 convolution (zero padding, correlation)
  per level on each path, ReLU, 2x2x2 average pooling down, nearest
  upsampling up, additive skips, and a 1x1x1 output convolution:
      e0 = relu(c0(x))            e1 = relu(c1(pool e0))
      e2 = relu(c2(pool e1))      e3 = relu(c3(pool e2))
      d2 = relu(c4(up e3)) + e2   d1 = relu(c5(up d2)) + e1
      d0 = relu(c6(up d1)) + e0   y  = wo . d0 + bo
  Loss: the error of the best multiple of y_b, (1/B) sum_b min_a
  |a y_b - t_b|^2 / |t_b|^2 (the network supplies a direction only).

Parameters travel as one flat float vector: for c0..c6 the weights
W[27][Cin][Cout] (tap = (dz+1)*9 + (dy+1)*3 + (dx+1)) then the bias[Cout],
followed by wo[16] and bo[1].
"""
import numpy as np

CONVS = [(3, 16), (16, 32), (32, 64), (64, 64), (64, 64), (64, 32), (32, 16)]
TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def num_params():
    return sum(27 * ci * co + co for ci, co in CONVS) + 16 + 1


def unpack(theta):
    """Flat vector -> list of (W[27,Cin,Cout], b[Cout]) and (wo[16], bo[1])."""
    theta = np.asarray(theta, dtype=np.float64)
    out, o = [], 0
    for ci, co in CONVS:
        W = theta[o:o + 27 * ci * co].reshape(27, ci, co)
        o += 27 * ci * co
        b = theta[o:o + co]
        o += co
        out.append((W, b))
    wo = theta[o:o + 16]
    bo = theta[o + 16:o + 17]
    assert o + 17 == theta.size
    return out, (wo, bo)


def pack(convs, head):
    parts = []
    for W, b in convs:
        parts += [W.ravel(), b.ravel()]
    parts += [head[0].ravel(), head[1].ravel()]
    return np.concatenate(parts)


def conv3(x, W, b):
    """3x3x3 correlation with zero padding: out[v] = sum_t x[v + off_t] W[t] + b."""
    B, nz, ny, nx, ci = x.shape
    xp = np.zeros((B, nz + 2, ny + 2, nx + 2, ci))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    out = np.zeros((B, nz, ny, nx, W.shape[2])) + b
    for t, (dz, dy, dx) in enumerate(TAPS):
        sl = xp[:, 1 + dz:1 + dz + nz, 1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]
        out += sl @ W[t]
    return out


def conv3_backward(x, W, dout):
    """Gradients of conv3 with respect to its input, weights and bias."""
    B, nz, ny, nx, ci = x.shape
    xp = np.zeros((B, nz + 2, ny + 2, nx + 2, ci))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for t, (dz, dy, dx) in enumerate(TAPS):
        sl = (slice(None), slice(1 + dz, 1 + dz + nz), slice(1 + dy, 1 + dy + ny),
              slice(1 + dx, 1 + dx + nx))
        dW[t] = np.einsum("bzyxc,bzyxd->cd", xp[sl], dout)
        dxp[sl] += dout @ W[t].T
    db = dout.sum(axis=(0, 1, 2, 3))
    return dxp[:, 1:-1, 1:-1, 1:-1], dW, db


def pool(x):
    B, nz, ny, nx, c = x.shape
    return x.reshape(B, nz // 2, 2, ny // 2, 2, nx // 2, 2, c).mean(axis=(2, 4, 6))


def pool_backward(dp):
    return np.repeat(np.repeat(np.repeat(dp, 2, axis=1), 2, axis=2), 2, axis=3) / 8.0


def up(x):
    return np.repeat(np.repeat(np.repeat(x, 2, axis=1), 2, axis=2), 2, axis=3)


def up_backward(du):
    B, nz, ny, nx, c = du.shape
    return du.reshape(B, nz // 2, 2, ny // 2, 2, nx // 2, 2, c).sum(axis=(2, 4, 6))


def relu(z):
    return np.maximum(z, 0.0)


def forward(theta, x):
    """x[B, nz, ny, nx, 3] (each dimension divisible by 8) -> y[B, nz, ny, nx]."""
    convs, (wo, bo) = unpack(theta)
    c = {}
    c["x"] = x
    c["e0"] = relu(conv3(x, *convs[0]))
    c["p1"] = pool(c["e0"])
    c["e1"] = relu(conv3(c["p1"], *convs[1]))
    c["p2"] = pool(c["e1"])
    c["e2"] = relu(conv3(c["p2"], *convs[2]))
    c["p3"] = pool(c["e2"])
    c["e3"] = relu(conv3(c["p3"], *convs[3]))
    c["u2"] = up(c["e3"])
    c["a4"] = relu(conv3(c["u2"], *convs[4]))
    c["d2"] = c["a4"] + c["e2"]
    c["u1"] = up(c["d2"])
    c["a5"] = relu(conv3(c["u1"], *convs[5]))
    c["d1"] = c["a5"] + c["e1"]
    c["u0"] = up(c["d1"])
    c["a6"] = relu(conv3(c["u0"], *convs[6]))
    c["d0"] = c["a6"] + c["e0"]
    y = c["d0"] @ wo + bo[0]
    return y, c


def backward(theta, c, dy):
    """Gradient of sum(dy * y) with respect to the flat parameter vector."""
    convs, (wo, bo) = unpack(theta)
    g = [None] * 7
    dwo = np.einsum("bzyxc,bzyx->c", c["d0"], dy)
    dbo = np.array([dy.sum()])
    dd0 = dy[..., None] * wo
    de0 = dd0.copy()
    dz6 = dd0 * (c["a6"] > 0)
    du0, dW, db = conv3_backward(c["u0"], convs[6][0], dz6)
    g[6] = (dW, db)
    dd1 = up_backward(du0)
    de1 = dd1.copy()
    dz5 = dd1 * (c["a5"] > 0)
    du1, dW, db = conv3_backward(c["u1"], convs[5][0], dz5)
    g[5] = (dW, db)
    dd2 = up_backward(du1)
    de2 = dd2.copy()
    dz4 = dd2 * (c["a4"] > 0)
    du2, dW, db = conv3_backward(c["u2"], convs[4][0], dz4)
    g[4] = (dW, db)
    de3 = up_backward(du2)
    dz3 = de3 * (c["e3"] > 0)
    dp3, dW, db = conv3_backward(c["p3"], convs[3][0], dz3)
    g[3] = (dW, db)
    de2 = de2 + pool_backward(dp3)
    dz2 = de2 * (c["e2"] > 0)
    dp2, dW, db = conv3_backward(c["p2"], convs[2][0], dz2)
    g[2] = (dW, db)
    de1 = de1 + pool_backward(dp2)
    dz1 = de1 * (c["e1"] > 0)
    dp1, dW, db = conv3_backward(c["p1"], convs[1][0], dz1)
    g[1] = (dW, db)
    de0 = de0 + pool_backward(dp1)
    dz0 = de0 * (c["e0"] > 0)
    _, dW, db = conv3_backward(c["x"], convs[0][0], dz0)
    g[0] = (dW, db)
    return pack(g, (dwo, dbo))


def loss(y, t):
    """Scale-free error of the predicted direction, averaged over the batch:
        L_b = min_a |a y_b - t_b|^2 / |t_b|^2 = 1 - (y_b.t_b)^2 / (|y_b|^2 |t_b|^2)
    (the network supplies a direction; its length is chosen when it is
    used), and its gradient with respect to y."""
    B = y.shape[0]
    yf, tf = y.reshape(B, -1), t.reshape(B, -1)
    yt = np.sum(yf * tf, axis=1)
    yy = np.sum(yf * yf, axis=1)
    tt = np.sum(tf * tf, axis=1)
    L = float(np.mean(1.0 - yt * yt / (yy * tt)))
    c = (yt / (yy * tt))[:, None]
    dy = -(2.0 / B) * (c * tf - (c * yt[:, None] / yy[:, None]) * yf)
    return L, dy.reshape(y.shape)


def adam_step(theta, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """Adam with bias correction (step counts from 1)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
