"""Seeded synthetic reservoir inputs (grid, rock, fluid, wells, state).

This module is the one piece shared by the HIP path's tests and benchmark and
by the CPU checker: it draws inputs only and holds none of the solver's
arithmetic.  The paper's own inputs (the SPE10 and SPE1 decks) are not
available, so these fields stand in for them with the shapes, contrasts and
well patterns of the workloads listed below; every generator takes a seed and
uses numpy's PCG64.

Geometry shared by every case: cells of 10 m x 10 m x 5 m, top at 2000 m
depth, pressure 200 bar at the top and hydrostatic below, vertical wells
perforated through every layer and controlled by bottom-hole pressure
(injectors 300 bar, producers 150 bar, referenced to the top), well radius
0.1 m, no skin.  Fluid constants are this project's own synthetic values.
"""
import numpy as np
import scipy.ndimage

G_ACC = 9.80665

OIL_WATER = {
    "model": 2, "p_ref": 200.0,
    "rho_w_ref": 1000.0, "rho_o_ref": 800.0,
    "c_w": 4.5e-5, "c_o": 1.0e-4, "c_r": 5.0e-5,
    "mu_w": 0.5, "mu_o": 2.0,
    "s_wc": 0.2, "s_or": 0.2,
    "rho_init": 800.0,
}

# Saturated black-oil PVT: rows p [bar], Rs [sm3/sm3], Bo, mu_o [cP], Bg, mu_g [cP]
BLACK_OIL_PVT = np.array([
    [50.0, 100.0, 150.0, 200.0, 250.0, 300.0, 350.0],
    [18.0, 38.0, 59.0, 80.0, 101.0, 122.0, 143.0],
    [1.10, 1.15, 1.20, 1.25, 1.30, 1.35, 1.40],
    [1.60, 1.40, 1.25, 1.10, 1.00, 0.92, 0.85],
    [0.0240, 0.0120, 0.0081, 0.0061, 0.0049, 0.0041, 0.0036],
    [0.013, 0.015, 0.017, 0.019, 0.021, 0.023, 0.025],
])

BLACK_OIL = {
    "model": 3, "p_ref": 200.0,
    "rho_w_ref": 1000.0, "rho_o_sc": 850.0, "rho_g_sc": 0.9,
    "c_w": 4.5e-5, "c_o": 1.0e-4, "c_r": 5.0e-5, "mu_w": 0.5,
    "s_wc": 0.2, "s_or": 0.2, "sg_den": 0.7,
    "pvt": BLACK_OIL_PVT,
    "rho_init": 740.0,
}

SINGLE_PHASE = {
    "model": 1, "p_ref": 200.0, "rho_w_ref": 1000.0, "c_w": 4.5e-5, "c_r": 5.0e-5,
    "mu_w": 0.5, "rho_init": 1000.0,
}


def grid_of(nx, ny, nz, dx=10.0, dy=10.0, dz=5.0, top=2000.0):
    return {"nx": nx, "ny": ny, "nz": nz, "dx": dx, "dy": dy, "dz": dz, "top": top}


def gaussian_field(rng, shape, corr):
    """iid N(0,1) smoothed by a separable Gaussian of the given correlation
    lengths (cells, per axis z, y, x; 0 = uncorrelated), unit variance."""
    f = rng.standard_normal(shape)
    if any(c > 0 for c in corr):
        f = scipy.ndimage.gaussian_filter(f, sigma=corr, mode="wrap")
    f -= f.mean()
    sd = f.std()
    return f / sd if sd > 0 else f


def initial_state(grid, fluid, sw=0.3, sg=0.05, p_top=200.0):
    """Hydrostatic pressure (constant initialisation density) and uniform
    saturations; shape (b, nz, ny, nx)."""
    nz, ny, nx = grid["nz"], grid["ny"], grid["nx"]
    depth_below_top = (np.arange(nz) + 0.5) * grid["dz"]
    p = p_top + fluid["rho_init"] * G_ACC * depth_below_top / 1.0e5
    p3 = np.broadcast_to(p[:, None, None], (nz, ny, nx))
    m = fluid["model"]
    if m == 1:
        return p3[None].copy()
    if m == 2:
        return np.stack([p3, np.full((nz, ny, nx), sw)]).astype(np.float64)
    return np.stack([p3, np.full((nz, ny, nx), sw), np.full((nz, ny, nx), sg)]).astype(np.float64)


def well(i, j, nz, kind, bhp, rw=0.1, skin=0.0):
    return {"i": int(i), "j": int(j), "k0": 0, "k1": nz - 1, "kind": kind,
            "bhp": float(bhp), "rw": rw, "skin": skin}


def five_spot(nx, ny, nz, p_top=200.0):
    """Injector in the centre, producers in the four corners."""
    return [well(nx // 2, ny // 2, nz, "inj", p_top + 100.0)] + [
        well(i, j, nz, "prod", p_top - 50.0)
        for (i, j) in [(0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1)]]


def lattice_wells(nx, ny, nz, per_side=5, p_top=200.0):
    """per_side^2 wells at ((2a+1) nx/(2 per_side), (2b+1) ny/(2 per_side));
    injector iff a+b is even."""
    out = []
    for a in range(per_side):
        for b in range(per_side):
            i = (2 * a + 1) * nx // (2 * per_side)
            j = (2 * b + 1) * ny // (2 * per_side)
            inj = (a + b) % 2 == 0
            out.append(well(i, j, nz, "inj" if inj else "prod", p_top + (100.0 if inj else -50.0)))
    return out


def _case(grid, fluid, perm, poro, wells, dt, name):
    x0 = initial_state(grid, fluid)
    return {"name": name, "grid": grid, "fluid": fluid, "perm": perm, "poro": poro,
            "wells": wells, "x_old": x0.copy(), "x": x0, "dt": dt}


def oil_water_lognormal(nx=32, ny=32, nz=8, seed=1000):
    """Two-phase case: ln k ~ N(ln 100 mD, 1) iid isotropic, porosity
    U(0.1, 0.3) iid, injector and producer in opposite corners, dt 1 day."""
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    k = np.exp(np.log(100.0) + rng.standard_normal(shape))
    perm = np.stack([k, k, k])
    poro = rng.uniform(0.1, 0.3, shape)
    wells = [well(0, 0, nz, "inj", 300.0), well(nx - 1, ny - 1, nz, "prod", 150.0)]
    return _case(grid_of(nx, ny, nz), OIL_WATER, perm, poro, wells, 1.0,
                 f"oil-water lognormal {nx}x{ny}x{nz}")


def black_oil_layered(nx=128, ny=128, nz=32, seed=2000):
    """Saturated black oil, layered lognormal permeability
    ln kx = ln 100 + 0.8 L_k + 0.6 eps (L_k per layer, eps per cell),
    ky = kx, kz = 0.1 kx, porosity U(0.1, 0.3), inverted five-spot, dt 1 day."""
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    layer = rng.standard_normal(nz)[:, None, None]
    eps = rng.standard_normal(shape)
    kx = np.exp(np.log(100.0) + 0.8 * layer + 0.6 * eps)
    perm = np.stack([kx, kx, 0.1 * kx])
    poro = rng.uniform(0.1, 0.3, shape)
    return _case(grid_of(nx, ny, nz), BLACK_OIL, perm, poro, five_spot(nx, ny, nz), 1.0,
                 f"black-oil layered {nx}x{ny}x{nz}")


def black_oil_channelised(nx=256, ny=256, nz=64, seed=3000, shale_md=10.0):
    """Binary facies: a Gaussian field (correlation 16, 4, 2 cells in x, y, z)
    thresholded at its 70th percentile gives 1000 mD channels (30 %) in a
    background of `shale_md`; kz = kx; five-spot; dt 10 days."""
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    f = gaussian_field(rng, shape, (2.0, 4.0, 16.0))
    k = np.where(f > np.percentile(f, 70.0), 1000.0, shale_md)
    perm = np.stack([k, k, k])
    poro = rng.uniform(0.1, 0.3, shape)
    return _case(grid_of(nx, ny, nz), BLACK_OIL, perm, poro, five_spot(nx, ny, nz), 10.0,
                 f"black-oil channelised {nx}x{ny}x{nz}")


def black_oil_lattice(nx=512, ny=512, nz=128, seed=5000):
    """ln k ~ N(ln 100, 1.5^2) correlated (4, 4, 1 cells), kz = 0.1 kx,
    25 wells on a 5x5 lattice, dt 1 day."""
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    f = gaussian_field(rng, shape, (1.0, 4.0, 4.0))
    kx = np.exp(np.log(100.0) + 1.5 * f)
    perm = np.stack([kx, kx, 0.1 * kx])
    poro = rng.uniform(0.1, 0.3, shape)
    return _case(grid_of(nx, ny, nz), BLACK_OIL, perm, poro, lattice_wells(nx, ny, nz), 1.0,
                 f"black-oil lattice {nx}x{ny}x{nz}")


def spe10_shaped_oil_water(nx=60, ny=220, nz=85, seed=8000):
    """The shape of the paper's SPE10 oil-water model (Sec. 3.1: 60 x 220 x 85
    cells of 20 x 10 x 2 ft, permeability between 6.65e-7 and 20 Darcy,
    porosity up to 0.5, one injector and four producers), filled with
    synthetic fields: ln kx = ln 50 mD + 2.5 G with G a Gaussian field of
    correlation (1, 8, 4) cells in (z, y, x), clipped to the quoted range;
    ky = kx, kz = 0.1 kx (clipped likewise); porosity 0.2 + 0.1 G' clipped to
    [0.01, 0.5]; injector in the centre, producers in the corners; dt 1 day.
    None of the benchmark's own data is used."""
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    lo, hi = 6.65e-4, 2.0e4
    kx = np.clip(np.exp(np.log(50.0) + 2.5 * gaussian_field(rng, shape, (1.0, 8.0, 4.0))), lo, hi)
    perm = np.stack([kx, kx, np.clip(0.1 * kx, lo, hi)])
    poro = np.clip(0.2 + 0.1 * gaussian_field(rng, shape, (1.0, 8.0, 4.0)), 0.01, 0.5)
    ft = 0.3048
    grid = grid_of(nx, ny, nz, dx=20 * ft, dy=10 * ft, dz=2 * ft)
    return _case(grid, OIL_WATER, perm, poro, five_spot(nx, ny, nz), 1.0,
                 f"oil-water SPE10-shaped {nx}x{ny}x{nz}")


def oil_water_training(nx=64, ny=64, nz=32, seed=5000):
    """Pressure-stage training systems: ln k sigma ~ U(0.5, 1.5), horizontal
    correlation ~ U{2..8}, vertical 1; S_w a Gaussian field mapped to
    [0.2, 0.8]; 1-4 random injector/producer pairs; dt 1 day."""
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    sigma = rng.uniform(0.5, 1.5)
    lh = int(rng.integers(2, 9))
    f = gaussian_field(rng, shape, (1.0, float(lh), float(lh)))
    k = np.exp(np.log(100.0) + sigma * f)
    perm = np.stack([k, k, k])
    poro = rng.uniform(0.1, 0.3, shape)
    s = gaussian_field(rng, shape, (1.0, float(lh), float(lh)))
    sw = 0.2 + 0.6 * (s - s.min()) / max(s.max() - s.min(), 1e-30)
    npair = int(rng.integers(1, 5))
    cols = rng.choice(nx * ny, size=2 * npair, replace=False)   # distinct columns
    wells = []
    for q in range(npair):
        a, b = cols[2 * q], cols[2 * q + 1]
        wells.append(well(a % nx, a // nx, nz, "inj", 300.0))
        wells.append(well(b % nx, b // nx, nz, "prod", 150.0))
    c = _case(grid_of(nx, ny, nz), OIL_WATER, perm, poro, wells, 1.0,
              f"oil-water training {nx}x{ny}x{nz}")
    c["x"][1] = sw
    c["x_old"][1] = sw
    return c


def black_oil_training(nx=64, ny=64, nz=32, seed=7000):
    """Pressure-stage training systems for black oil: anisotropic
    permeability (kz/kx = 10^U(-1.5, -0.5)), half of the systems layered
    (ln kx = ln 100 + a L_k + c eps, a ~ U(0.5, 1.2), c ~ U(0.3, 0.9)), half
    a correlated field (sigma ~ U(0.5, 1.5), horizontal correlation U{2..8},
    vertical 1); wells a five-spot, a 2x2 or 3x3 lattice, or 1-4 random
    injector/producer pairs; porosity U(0.1, 0.3); dt 1 day."""
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    if rng.uniform() < 0.5:
        a, c = rng.uniform(0.5, 1.2), rng.uniform(0.3, 0.9)
        lnk = a * rng.standard_normal(nz)[:, None, None] + c * rng.standard_normal(shape)
    else:
        sigma, lh = rng.uniform(0.5, 1.5), float(rng.integers(2, 9))
        lnk = sigma * gaussian_field(rng, shape, (1.0, lh, lh))
    kx = np.exp(np.log(100.0) + lnk)
    perm = np.stack([kx, kx, 10.0 ** rng.uniform(-1.5, -0.5) * kx])
    poro = rng.uniform(0.1, 0.3, shape)
    pattern = int(rng.integers(0, 3))
    if pattern == 0:
        wells = five_spot(nx, ny, nz)
    elif pattern == 1:
        wells = lattice_wells(nx, ny, nz, per_side=int(rng.integers(2, 4)))
    else:
        npair = int(rng.integers(1, 5))
        cols = rng.choice(nx * ny, size=2 * npair, replace=False)   # distinct columns
        wells = []
        for q in range(npair):
            i, j = cols[2 * q], cols[2 * q + 1]
            wells.append(well(i % nx, i // nx, nz, "inj", 300.0))
            wells.append(well(j % nx, j // nx, nz, "prod", 150.0))
    return _case(grid_of(nx, ny, nz), BLACK_OIL, perm, poro, wells, 1.0,
                 f"black-oil training {nx}x{ny}x{nz}")


def black_oil_lattice_training(nx=256, ny=256, nz=64, seed=5100):
    """Training systems for a learned stage on a coarse multigrid level:
    lognormal fields around the lattice workload's (sigma ~ U(1, 2),
    horizontal correlation U{2..8} cells, vertical 1), kz/kx =
    10^U(-1.5, -0.5), a 3x3 to 5x5 lattice of wells, porosity U(0.1, 0.3),
    dt 1 day."""
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    sigma, lh = rng.uniform(1.0, 2.0), float(rng.integers(2, 9))
    kx = np.exp(np.log(100.0) + sigma * gaussian_field(rng, shape, (1.0, lh, lh)))
    perm = np.stack([kx, kx, 10.0 ** rng.uniform(-1.5, -0.5) * kx])
    poro = rng.uniform(0.1, 0.3, shape)
    wells = lattice_wells(nx, ny, nz, per_side=int(rng.integers(3, 6)))
    return _case(grid_of(nx, ny, nz), BLACK_OIL, perm, poro, wells, 1.0,
                 f"black-oil lattice training {nx}x{ny}x{nz}")


def oil_water_eval(nx=128, ny=128, nz=64, seed=6000):
    """Evaluation systems for the learned stage: sigma 1.0, correlation
    (4, 4, 1), five-spot, S_w field as in training."""
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    f = gaussian_field(rng, shape, (1.0, 4.0, 4.0))
    k = np.exp(np.log(100.0) + 1.0 * f)
    perm = np.stack([k, k, k])
    poro = rng.uniform(0.1, 0.3, shape)
    s = gaussian_field(rng, shape, (1.0, 4.0, 4.0))
    sw = 0.2 + 0.6 * (s - s.min()) / max(s.max() - s.min(), 1e-30)
    c = _case(grid_of(nx, ny, nz), OIL_WATER, perm, poro, five_spot(nx, ny, nz), 1.0,
              f"oil-water eval {nx}x{ny}x{nz}")
    c["x"][1] = sw
    c["x_old"][1] = sw
    return c


def single_phase_uniform(nx, ny, nz, k_md=100.0, poro=0.2, wells=()):
    """Homogeneous single-phase (water) test case."""
    shape = (nz, ny, nx)
    perm = np.full((3,) + shape, k_md)
    return _case(grid_of(nx, ny, nz), SINGLE_PHASE, perm, np.full(shape, poro), list(wells),
                 1.0, f"single-phase uniform {nx}x{ny}x{nz}")


# (input, output) channels of the seven 3x3x3 convolutions of the pressure
# network, in parameter order; the 1x1x1 head maps 16 channels to 1.
NN_CONVS = [(3, 16), (16, 32), (32, 64), (64, 64), (64, 64), (64, 32), (32, 16)]


def nn_initial_weights(seed):
    """Random initial parameters of the pressure network as one flat float32
    vector (per convolution: weights [27][Cin][Cout] ~ N(0, 2/(27 Cin)),
    zero bias; head weights ~ N(0, 1/16), zero bias)."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in NN_CONVS:
        parts.append(rng.standard_normal(27 * ci * co) * np.sqrt(2.0 / (27 * ci)))
        parts.append(np.zeros(co))
    parts.append(rng.standard_normal(16) * 0.25)
    parts.append(np.zeros(1))
    return np.concatenate(parts).astype(np.float32)


def undersaturated_cells(case, x, seed, frac=0.4, margin=(5.0, 40.0)):
    """A black-oil state with a random fraction of cells undersaturated: their
    third unknown becomes -p_b with p_b = p - U(margin) bar (no free gas)."""
    rng = np.random.default_rng(seed)
    x = x.copy()
    pick = rng.uniform(size=x[0].shape) < frac
    pb = x[0] - rng.uniform(margin[0], margin[1], x[0].shape)
    x[2] = np.where(pick, -pb, x[2])
    return x


def random_state_perturbation(case, seed, dp=5.0, ds=0.05):
    """A perturbed current state x (x_old unchanged) for Jacobian tests."""
    rng = np.random.default_rng(seed)
    x = case["x"].copy()
    x[0] += dp * rng.standard_normal(x[0].shape)
    for s in range(1, x.shape[0]):
        x[s] = np.clip(x[s] + ds * rng.standard_normal(x[s].shape), 0.02, 0.9)
    return x
