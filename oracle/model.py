"""Oracle: residual F(x) and analytic Jacobian of the fully implicit models.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain FP64 numpy, natural
cell order n = i + nx*(j + ny*k), arrays shaped (nz, ny, nx), k downward.

Paper passages followed
  * Darcy flux, eqs. (1)-(2); mass conservation of the black-oil model,
    eq. (3); constitutive relations, eq. (4) (capillary pressure zero, as in
    the paper's examples, Sec. 3.1); oil-water model, eq. (5).
  * Well sink/source with the Peaceman well index, eq. (6); bottom-hole
    pressure constraint, eq. (7) (the BHP is known, so it adds no unknown).
  * Backward Euler in time, eq. (10); cell-centred finite differences with
    transmissibility T = K Kr rho A / (mu dd), eq. (11).
  * Corey relative permeabilities with s_wc = s_or = 0.2, eqs. (17)-(18);
    Stone II for the three-phase oil relative permeability (Sec. 2.1).

Readings where the paper is silent (the GPU library takes the same ones)
  * Unknowns per cell: (p [bar], S_w) oil-water, (p_o [bar], S_w, x2) black
    oil, (p [bar]) for the single-phase test model.  Black oil switches its
    third unknown with the phase state (Sec. 2.4: gas saturation or bubble
    point pressure): x2 = S_g >= 0 where free gas may exist (saturated oil,
    Rs, B_o, mu_o at p) and x2 = -p_b < 0 where it does not (undersaturated
    oil: S_g = 0, Rs and mu_o at p_b, B_o = B_o(p_b) exp(-c_o (p - p_b))).
    The sign of x2 carries the state, so x alone describes it.  Rows in
    the order (oil, water[, gas]) components; single phase has one water row.
  * Phi_a = p - rho_a g z with z the depth (positive downward), so a
    hydrostatic column has no potential gradient; the symbol in eq. (6) is g.
  * Face quantities: harmonic transmissibility, upstream mass mobility
    rho k_r / mu, arithmetic mean of the two cells' phase densities for
    gravity.  Upstream cell: the one with the higher potential; when
    |dPhi| <= 1e-9 bar the lower-index cell of the face.
  * Water injectors use the cell's total volumetric mobility with the water
    density; producers use eq. (6) phase by phase.
  * Each component's rows are divided by rho_c * Vbar * phibar / dt (rho_c the
    component's reservoir density at p_ref, Vbar the cell volume, phibar the
    mean porosity) so saturation derivatives are O(1); the pressure column is
    in bar.
"""
import numpy as np

G = 9.80665           # m s^-2
BAR = 1.0e5           # Pa per bar
MD = 9.869233e-16     # m^2 per millidarcy
CP = 1.0e-3           # Pa s per centipoise
DAY = 86400.0         # s per day
TIE_BAR = 1.0e-9      # upstream tie tolerance on the potential difference

# direction index d of a 7-point block row: 0 self, then -x, +x, -y, +y, -z, +z
DIRS = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
OPP = [0, 2, 1, 4, 3, 6, 5]


def nblock(model):
    """Unknowns per cell: 1 single phase, 2 oil-water, 3 black oil."""
    return {1: 1, 2: 2, 3: 3}[model]


def cell_depth(grid):
    """Depth of each cell centre (m), k = 0 at the top face."""
    nz, dz, top = grid["nz"], grid["dz"], grid["top"]
    z = top + (np.arange(nz) + 0.5) * dz
    return np.broadcast_to(z[:, None, None], (nz, grid["ny"], grid["nx"])).copy()


def transmissibilities(grid, perm_md):
    """Harmonic-mean TPFA transmissibilities (m^3), the geometric part of
    eq. (11): T = 2 A / (dd/k_a + dd/k_b) for the face between a and b.
    Returns (Tx, Ty, Tz) of shapes (nz,ny,nx-1), (nz,ny-1,nx), (nz-1,ny,nx)."""
    dx, dy, dz = grid["dx"], grid["dy"], grid["dz"]
    k = perm_md * MD

    def harm(ka, kb, area, dd):
        s = ka + kb
        return np.where(s > 0, 2.0 * area * ka * kb / (dd * np.where(s > 0, s, 1.0)), 0.0)

    Tx = harm(k[0][:, :, :-1], k[0][:, :, 1:], dy * dz, dx)
    Ty = harm(k[1][:, :-1, :], k[1][:, 1:, :], dx * dz, dy)
    Tz = harm(k[2][:-1, :, :], k[2][1:, :, :], dx * dy, dz)
    return Tx, Ty, Tz


def peaceman_wi(kx_md, ky_md, dx, dy, dz, rw, skin):
    """Peaceman well index (m^3) for a vertical well in an anisotropic cell
    (the W_i of eq. (6)): 2 pi sqrt(kx ky) dz / (ln(r_o / r_w) + s), with the
    equivalent radius r_o of an anisotropic rectangular block."""
    kx, ky = kx_md * MD, ky_md * MD
    rxy, ryx = np.sqrt(ky / kx), np.sqrt(kx / ky)
    ro = 0.28 * np.sqrt(rxy * dx * dx + ryx * dy * dy) / (np.sqrt(rxy) + np.sqrt(ryx))
    return 2.0 * np.pi * np.sqrt(kx * ky) * dz / (np.log(ro / rw) + skin)


def _clip01(a):
    """Clamp to [0, 1]; derivative factor 1 strictly inside, 0 elsewhere."""
    inside = (a > 0.0) & (a < 1.0)
    return np.clip(a, 0.0, 1.0), inside.astype(np.float64)


def corey(sw, s_wc, s_or):
    """Two-phase Corey curves of eqs. (17)-(18) (exponent 2), with their
    derivatives in S_w.  Normalised saturations are clamped to [0, 1]."""
    den = 1.0 - s_wc - s_or
    a, ia = _clip01((sw - s_wc) / den)
    o, io = _clip01((1.0 - s_or - sw) / den)
    krw, dkrw = a * a, 2.0 * a * ia / den
    kro, dkro = o * o, -2.0 * o * io / den
    return krw, dkrw, kro, dkro


def stone2(sw, sg, s_wc, s_or, sg_den):
    """Three-phase relative permeabilities (Sec. 2.1: Kro by Stone II).
    k_rw and k_row are the two-phase Corey curves, k_rg = (S_g/sg_den)^2,
    k_rog = ((sg_den - S_g)/sg_den)^2, k_rocw = 1, and
        k_ro = (k_row + k_rw)(k_rog + k_rg) - k_rw - k_rg   (clamped at 0).
    Returns krw, dkrw/dSw, krg, dkrg/dSg, kro, dkro/dSw, dkro/dSg."""
    krw, dkrw, krow, dkrow = corey(sw, s_wc, s_or)
    g, ig = _clip01(sg / sg_den)
    h, ih = _clip01((sg_den - sg) / sg_den)
    krg, dkrg = g * g, 2.0 * g * ig / sg_den
    krog, dkrog = h * h, -2.0 * h * ih / sg_den
    raw = (krow + krw) * (krog + krg) - krw - krg
    pos = raw > 0.0
    kro = np.where(pos, raw, 0.0)
    dkro_w = np.where(pos, (dkrow + dkrw) * (krog + krg) - dkrw, 0.0)
    dkro_g = np.where(pos, (krow + krw) * (dkrog + dkrg) - dkrg, 0.0)
    return krw, dkrw, krg, dkrg, kro, dkro_w, dkro_g


def pvt_interp(tp, ty, p):
    """Piecewise-linear table y(p) and dy/dp.  p in [tp[k], tp[k+1]) uses
    segment k; the first and last segments extend beyond the table."""
    m = len(tp)
    seg = np.clip(np.searchsorted(tp, p, side="right") - 1, 0, m - 2)
    p0, p1 = tp[seg], tp[seg + 1]
    y0, y1 = ty[seg], ty[seg + 1]
    slope = (y1 - y0) / (p1 - p0)
    return y0 + slope * (p - p0), slope


def component_density_ref(fluid):
    """Reservoir density (kg/m^3) at p_ref of each component, in row order;
    used only for the row scaling."""
    m = fluid["model"]
    if m == 1:
        return [fluid["rho_w_ref"]]
    if m == 2:
        return [fluid["rho_o_ref"], fluid["rho_w_ref"]]
    pvt = np.asarray(fluid["pvt"], dtype=np.float64)
    bo, _ = pvt_interp(pvt[0], pvt[2], np.array([fluid["p_ref"]]))
    bg, _ = pvt_interp(pvt[0], pvt[4], np.array([fluid["p_ref"]]))
    return [fluid["rho_o_sc"] / bo[0], fluid["rho_w_ref"], fluid["rho_g_sc"] / bg[0]]


def cell_state(fluid, poro, x):
    """Per-cell accumulation, phase densities and component mobilities.

    x has shape (b, nz, ny, nx).  Returns a dict with
      acc   (b, ...)        component mass per unit bulk volume, phi*S*rho
      dacc  (b, b, ...)     d acc[c] / d x[u]
      phases: list of (rho, drho (b, ...)) per phase, drho[u] = d rho / d x[u]
      terms:  list of (row c, phase index, lam, dlam (b, ...)) -- the mass
              mobility rho_c k_r / mu of component c carried by that phase
      lam_t:  total volumetric mobility sum k_r/mu and its derivative (b, ...)
    """
    m = fluid["model"]
    b = nblock(m)
    p = x[0]
    pref = fluid["p_ref"]
    phi = poro * (1.0 + fluid["c_r"] * (p - pref))
    dphi = poro * fluid["c_r"]
    rho_w = fluid["rho_w_ref"] * np.exp(fluid["c_w"] * (p - pref))
    drho_w = fluid["c_w"] * rho_w
    mu_w = fluid["mu_w"] * CP
    zero = np.zeros_like(p)
    out = {"phases": [], "terms": []}
    acc = np.zeros((b,) + p.shape)
    dacc = np.zeros((b, b) + p.shape)
    def dvec(dp, d2=None):
        v = np.zeros((b,) + p.shape)
        v[0] = dp
        if d2 is not None:
            v[2] = d2
        return v

    if m == 1:
        acc[0] = phi * rho_w
        dacc[0, 0] = dphi * rho_w + phi * drho_w
        out["phases"] = [(rho_w, dvec(drho_w))]
        dl = np.zeros((1,) + p.shape)
        dl[0] = drho_w / mu_w
        out["terms"] = [(0, 0, rho_w / mu_w, dl)]
        lt = np.ones_like(p) / mu_w
        out["lam_t"] = (lt, np.zeros((1,) + p.shape))
    elif m == 2:
        sw = x[1]
        so = 1.0 - sw
        rho_o = fluid["rho_o_ref"] * np.exp(fluid["c_o"] * (p - pref))
        drho_o = fluid["c_o"] * rho_o
        mu_o = fluid["mu_o"] * CP
        krw, dkrw, kro, dkro = corey(sw, fluid["s_wc"], fluid["s_or"])
        acc[0] = phi * so * rho_o
        acc[1] = phi * sw * rho_w
        dacc[0, 0] = so * (dphi * rho_o + phi * drho_o)
        dacc[0, 1] = -phi * rho_o
        dacc[1, 0] = sw * (dphi * rho_w + phi * drho_w)
        dacc[1, 1] = phi * rho_w
        out["phases"] = [(rho_o, dvec(drho_o)), (rho_w, dvec(drho_w))]
        dlo = np.stack([drho_o * kro / mu_o, rho_o * dkro / mu_o])
        dlw = np.stack([drho_w * krw / mu_w, rho_w * dkrw / mu_w])
        out["terms"] = [(0, 0, rho_o * kro / mu_o, dlo), (1, 1, rho_w * krw / mu_w, dlw)]
        out["lam_t"] = (krw / mu_w + kro / mu_o, np.stack([zero, dkrw / mu_w + dkro / mu_o]))
    else:
        # third unknown: S_g >= 0 in saturated cells, -p_b (bar) < 0 in
        # undersaturated cells (no free gas, bubble point p_b < p)
        sw, x2 = x[1], x[2]
        sat = x2 >= 0.0
        sg = np.where(sat, x2, 0.0)
        dsg = sat.astype(np.float64)                  # d S_g / d x2
        pb = np.where(sat, p, -x2)
        so = 1.0 - sw - sg
        pvt = np.asarray(fluid["pvt"], dtype=np.float64)
        tp = pvt[0]
        rs, drs_b = pvt_interp(tp, pvt[1], pb)
        bo_b, dbo_b = pvt_interp(tp, pvt[2], pb)
        muo, dmuo_b = pvt_interp(tp, pvt[3], pb)
        bg, dbg = pvt_interp(tp, pvt[4], p)
        mug, dmug = pvt_interp(tp, pvt[5], p)
        # undersaturated oil: Rs and mu_o at the bubble point, and
        # B_o = B_o(p_b) exp(-c_o (p - p_b)); saturated: functions of p
        c_o = fluid.get("c_o", 0.0)
        e = np.where(sat, 1.0, np.exp(-c_o * (p - pb)))
        bo = bo_b * e
        rs_p, rs_2 = np.where(sat, drs_b, 0.0), np.where(sat, 0.0, -drs_b)
        bo_p = np.where(sat, dbo_b, -c_o * bo)
        bo_2 = np.where(sat, 0.0, -(dbo_b * e + c_o * bo))
        mu_p, mu_2 = np.where(sat, dmuo_b, 0.0), np.where(sat, 0.0, -dmuo_b)
        muo, mu_p, mu_2 = muo * CP, mu_p * CP, mu_2 * CP
        mug, dmug = mug * CP, dmug * CP
        rsc_o, rsc_g = fluid["rho_o_sc"], fluid["rho_g_sc"]
        rho_oo = rsc_o / bo                       # oil component in the oil phase
        rho_oo_p = -rsc_o * bo_p / (bo * bo)
        rho_oo_2 = -rsc_o * bo_2 / (bo * bo)
        rho_og = rsc_g * rs / bo                  # dissolved gas in the oil phase
        rho_og_p = rsc_g * (rs_p * bo - rs * bo_p) / (bo * bo)
        rho_og_2 = rsc_g * (rs_2 * bo - rs * bo_2) / (bo * bo)
        rho_g = rsc_g / bg                        # free gas
        drho_g = -rsc_g * dbg / (bg * bg)
        krw, dkrw, krg, dkrg, kro, dkro_w, dkro_g = stone2(
            sw, sg, fluid["s_wc"], fluid["s_or"], fluid["sg_den"])
        dkrg, dkro_g = dkrg * dsg, dkro_g * dsg    # per unit of x2
        acc[0] = phi * so * rho_oo
        acc[1] = phi * sw * rho_w
        acc[2] = phi * (so * rho_og + sg * rho_g)
        dacc[0, 0] = so * (dphi * rho_oo + phi * rho_oo_p)
        dacc[0, 1] = -phi * rho_oo
        dacc[0, 2] = -phi * rho_oo * dsg + phi * so * rho_oo_2
        dacc[1, 0] = sw * (dphi * rho_w + phi * drho_w)
        dacc[1, 1] = phi * rho_w
        dacc[2, 0] = dphi * (so * rho_og + sg * rho_g) + phi * (so * rho_og_p + sg * drho_g)
        dacc[2, 1] = -phi * rho_og
        dacc[2, 2] = phi * (-rho_og * dsg + so * rho_og_2 + rho_g * dsg)
        rho_O = rho_oo + rho_og
        out["phases"] = [(rho_O, dvec(rho_oo_p + rho_og_p, rho_oo_2 + rho_og_2)),
                         (rho_w, dvec(drho_w)), (rho_g, dvec(drho_g))]

        # mobility rho k_r / mu and its derivatives in (p, Sw, x2)
        def mob(rho, rho_p, rho_2, kr, dkr_w, dkr_2, mu, dmu_p, dmu_2):
            lam = rho * kr / mu
            return lam, np.stack([(rho_p * kr - rho * kr * dmu_p / mu) / mu,
                                  rho * dkr_w / mu,
                                  (rho_2 * kr + rho * dkr_2 - rho * kr * dmu_2 / mu) / mu])
        lam_oo, dl_oo = mob(rho_oo, rho_oo_p, rho_oo_2, kro, dkro_w, dkro_g, muo, mu_p, mu_2)
        lam_og, dl_og = mob(rho_og, rho_og_p, rho_og_2, kro, dkro_w, dkro_g, muo, mu_p, mu_2)
        lam_w, dl_w = mob(rho_w, drho_w, zero, krw, dkrw, zero, mu_w, zero, zero)
        lam_g, dl_g = mob(rho_g, drho_g, zero, krg, zero, dkrg, mug, dmug, zero)
        out["terms"] = [(0, 0, lam_oo, dl_oo), (1, 1, lam_w, dl_w),
                        (2, 0, lam_og, dl_og), (2, 2, lam_g, dl_g)]
        lt = krw / mu_w + kro / muo + krg / mug
        dlt = np.stack([-kro * mu_p / (muo * muo) - krg * dmug / (mug * mug),
                        dkrw / mu_w + dkro_w / muo,
                        dkro_g / muo - kro * mu_2 / (muo * muo) + dkrg / mug])
        out["lam_t"] = (lt, dlt)
    out["acc"], out["dacc"] = acc, dacc
    return out


def _face_slices(axis):
    """(lower-cell slice, upper-cell slice, direction index lower->upper)."""
    lo = [slice(None)] * 3
    hi = [slice(None)] * 3
    lo[2 - axis] = slice(None, -1)
    hi[2 - axis] = slice(1, None)
    return tuple(lo), tuple(hi), 2 * axis + 2


def row_scales(grid, fluid, poro, dt_days):
    """Global per-component row divisors rho_c * Vbar * phibar / dt."""
    vol = grid["dx"] * grid["dy"] * grid["dz"]
    phibar = float(np.mean(poro))
    dt = dt_days * DAY
    return np.array([r * vol * phibar / dt for r in component_density_ref(fluid)])


def rate_wells(wells):
    """Wells under a rate constraint (eqs. (8)-(9)), whose bottom-hole
    pressure is an unknown; the others are under eq. (7)."""
    return [w for w in wells if w.get("control", "bhp") == "rate"]


def surface_density(fluid, comp):
    """Density converting the controlled component's mass rate to the rate
    of eqs. (8)-(9): water rho_w_ref; oil rho_o_sc (black oil) or rho_o_ref."""
    m = fluid["model"]
    if m == 1 or comp == 1:
        return fluid["rho_w_ref"]
    return fluid["rho_o_sc"] if m == 3 else fluid["rho_o_ref"]


def assemble(grid, fluid, perm_md, poro, wells, x_old, x, dt_days, bhp=None, border=False):
    """Residual R(x) and Jacobian J = dR/dx of the scaled system.

    Residual of component c in cell i (backward Euler, eq. (10); TPFA
    fluxes, eq. (11); wells, eq. (6)):
        R_c,i = [ V (acc_c(x) - acc_c(x_old)) / dt + sum_faces F_c,ij - q_c,i ] / s_c
    with F_c,ij = T_ij lam_c,up (Phi_i - Phi_j) the mass flow out of i.

    Returns R of shape (b, nz, ny, nx) and J of shape (7, b, b, nz, ny, nx),
    J[d, r, c, cell] = dR_r(cell) / dx_c(neighbour d of cell); blocks that
    would reach outside the grid (no-flow boundary) are zero.  The Newton
    right-hand side is b = -R.

    Rate-controlled wells (eqs. (8)-(9)): their bottom-hole pressures are
    unknowns, bhp[w] (bar) in the order of rate_wells(wells) (default: each
    well's "bhp" entry).  An injector's water rate or a producer's oil rate
    sums its perforations' mass rates; with Q the target (surface m^3/day)
    and rho_s the surface density of the component c,
        R_w = (sum_m q_c,m - Q rho_s / 86400) / s_c    (injector)
        R_w = (sum_m q_c,m + Q rho_s / 86400) / s_c    (producer, q_c,m < 0)
    With border=True a third value W holds the border of the Jacobian of
    eq. (16): W["R"] (nr,), W["B"] (nr, b, grid) = dR_cells / dp_h,
    W["C"] (nr, b, grid) = dR_w / dx_cells, W["D"] (nr,) = dR_w / dp_h.
    """
    m = fluid["model"]
    b = nblock(m)
    vol = grid["dx"] * grid["dy"] * grid["dz"]
    dt = dt_days * DAY
    depth = cell_depth(grid)
    shape = x.shape[1:]
    st = cell_state(fluid, poro, x)
    st0 = cell_state(fluid, poro, x_old)
    R = np.zeros((b,) + shape)
    J = np.zeros((7, b, b) + shape)
    # accumulation, eq. (10)
    R += vol * (st["acc"] - st0["acc"]) / dt
    J[0] += vol * st["dacc"] / dt
    # fluxes, eqs. (1)-(3), (11)
    Ts = transmissibilities(grid, perm_md)
    for axis in range(3):
        lo, hi, dplus = _face_slices(axis)
        dminus = OPP[dplus]
        T = Ts[axis]
        dz = depth[lo] - depth[hi]
        p_lo, p_hi = x[0][lo], x[0][hi]
        dphis = []
        for rho, drho in st["phases"]:
            dphi = (p_lo - p_hi) * BAR - 0.5 * (rho[lo] + rho[hi]) * G * dz
            ddphi_lo = np.stack([-0.5 * G * dz * drho[u][lo] for u in range(b)])
            ddphi_hi = np.stack([-0.5 * G * dz * drho[u][hi] for u in range(b)])
            ddphi_lo[0] += BAR
            ddphi_hi[0] -= BAR
            up_lo = dphi >= -TIE_BAR * BAR  # ties go to the lower-index cell
            dphis.append((dphi, ddphi_lo, ddphi_hi, up_lo))
        for (c, ph, lam, dlam) in st["terms"]:
            dphi, ddphi_lo, ddphi_hi, up_lo = dphis[ph]
            lam_up = np.where(up_lo, lam[lo], lam[hi])
            F = T * lam_up * dphi
            dF_lo = np.zeros((b,) + F.shape)
            dF_hi = np.zeros((b,) + F.shape)
            for u in range(b):
                dF_lo[u] = T * np.where(up_lo, dlam[u][lo], 0.0) * dphi
                dF_hi[u] = T * np.where(up_lo, 0.0, dlam[u][hi]) * dphi
            for u in range(b):
                dF_lo[u] += T * lam_up * ddphi_lo[u]
                dF_hi[u] += T * lam_up * ddphi_hi[u]
            R[c][lo] += F
            R[c][hi] -= F
            for u in range(b):
                J[0, c, u][lo] += dF_lo[u]
                J[dplus, c, u][lo] += dF_hi[u]
                J[dminus, c, u][hi] -= dF_lo[u]
                J[0, c, u][hi] -= dF_hi[u]
    # wells, eq. (6); BHP constraint eq. (7) or rate constraint eqs. (8)-(9)
    rws = rate_wells(wells)
    nr = len(rws)
    if bhp is None:
        bhp = np.array([w["bhp"] for w in rws], dtype=np.float64)
    W = {"R": np.zeros(nr), "B": np.zeros((nr, b) + shape), "C": np.zeros((nr, b) + shape),
         "D": np.zeros(nr)}
    for w in wells:
        i, j = w["i"], w["j"]
        iw = next((q for q, rw in enumerate(rws) if rw is w), None)
        ph_w = w["bhp"] if iw is None else bhp[iw]
        if iw is not None:
            wc = (0 if m == 1 else 1) if w["kind"] == "inj" else 0    # controlled component
            sgn = -1.0 if w["kind"] == "inj" else 1.0
            W["R"][iw] += sgn * w["rate"] * surface_density(fluid, wc) / DAY
        for k in range(w["k0"], w["k1"] + 1):
            cell = (k, j, i)
            wi = peaceman_wi(perm_md[0][cell], perm_md[1][cell], grid["dx"], grid["dy"],
                             grid["dz"], w["rw"], w["skin"])
            dh = ph_w - x[0][cell]                # bar
            dzh = grid["top"] - depth[cell]       # z_h - z
            if w["kind"] == "inj":
                rho, drho = st["phases"][-1 if m == 1 else 1]
                wc = 0 if m == 1 else 1
                lt, dlt = st["lam_t"]
                drive = dh * BAR - rho[cell] * G * dzh
                q = wi * rho[cell] * lt[cell] * drive
                R[wc][cell] -= q
                for u in range(b):
                    dq = wi * rho[cell] * dlt[u][cell] * drive
                    if u == 0:
                        dq += wi * drho[0][cell] * lt[cell] * drive
                        dq += wi * rho[cell] * lt[cell] * (-BAR - drho[0][cell] * G * dzh)
                    J[0, wc, u][cell] -= dq
                    if iw is not None:
                        W["C"][iw][(u,) + cell] += dq
                if iw is not None:
                    dqh = wi * rho[cell] * lt[cell] * BAR
                    W["B"][iw][(wc,) + cell] -= dqh
                    W["R"][iw] += q
                    W["D"][iw] += dqh
            else:
                for (c, ph, lam, dlam) in st["terms"]:
                    rho, drho = st["phases"][ph]
                    drive = dh * BAR - rho[cell] * G * dzh
                    q = wi * lam[cell] * drive
                    R[c][cell] -= q
                    for u in range(b):
                        dq = wi * dlam[u][cell] * drive
                        if u == 0:
                            dq += wi * lam[cell] * (-BAR - drho[0][cell] * G * dzh)
                        else:
                            dq += wi * lam[cell] * (-drho[u][cell] * G * dzh)
                        J[0, c, u][cell] -= dq
                        if iw is not None and c == 0:
                            W["C"][iw][(u,) + cell] += dq
                    if iw is not None:
                        dqh = wi * lam[cell] * BAR
                        W["B"][iw][(c,) + cell] -= dqh
                        if c == 0:
                            W["R"][iw] += q
                            W["D"][iw] += dqh
    s = row_scales(grid, fluid, poro, dt_days)
    for c in range(b):
        R[c] /= s[c]
        J[:, c] /= s[c]
        W["B"][:, c] /= s[c]
    for iw, w in enumerate(rws):
        sc = s[(0 if m == 1 else 1) if w["kind"] == "inj" else 0]
        W["R"][iw] /= sc
        W["C"][iw] /= sc
        W["D"][iw] /= sc
    if border:
        return R, J, W
    return R, J
