// Jacobian and residual assembly on the GPU.
//
// Residual of component c in cell i (eqs. (3)/(5) with backward Euler,
// eq. (10), and TPFA fluxes, eq. (11)):
//   R_c,i = [ V (acc_c(x) - acc_c(x_old)) / dt + sum_faces F_c,ij - q_c,i ] / s_c
// with F_c,ij = T_ij lam_c,up (Phi_i - Phi_j) the mass flow from i to j,
// Phi = p - rho g z (z depth), upstream = higher potential (ties, within
// 1e-9 bar, go to the lower-index cell of the face), face density the mean
// of the two cells, and q from eq. (6) (Peaceman index, BHP constraint).
// s_c = rho_c V mean(phi) / dt.  The output right-hand side is -R.
//
// Three kernels: per-cell fluid state (phase densities and mobilities with
// their derivatives) into SoA planes; a cell-centric flux kernel in which
// every cell evaluates its own six faces and writes its whole block row
// (no atomics: the face flow is computed identically from both sides); and
// a per-perforation well kernel.  Built without FP contraction so that both
// sides of a face round identically.
#include <cmath>

#include "internal.h"

namespace {

constexpr double G_ACC = 9.80665;
constexpr double BAR = 1.0e5;
constexpr double CP = 1.0e-3;
constexpr double DAY = 86400.0;
constexpr double TIE_BAR = 1.0e-9;

template <int MODEL>
struct Traits;
template <>
struct Traits<1> {   // single-phase (water) test model
  static constexpr int B = 1, NP = 1, NT = 1;
  __host__ __device__ static constexpr int row(int) { return 0; }
  __host__ __device__ static constexpr int phase(int) { return 0; }
};
template <>
struct Traits<2> {
  static constexpr int B = 2, NP = 2, NT = 2;
  __host__ __device__ static constexpr int row(int t) { return t; }
  __host__ __device__ static constexpr int phase(int t) { return t; }
};
template <>
struct Traits<3> {
  static constexpr int B = 3, NP = 3, NT = 4;
  // terms: oil comp. in oil phase, water, dissolved gas in oil phase, free gas
  __host__ __device__ static constexpr int row(int t) { return t == 3 ? 2 : t; }
  __host__ __device__ static constexpr int phase(int t) { return t == 2 ? 0 : (t == 3 ? 2 : t); }
};
static_assert(Traits<3>::phase(0) == 0 && Traits<3>::phase(1) == 1 && Traits<3>::phase(2) == 0 &&
                  Traits<3>::phase(3) == 2 && Traits<3>::row(2) == 2 && Traits<3>::row(3) == 2,
              "black-oil term table");

template <int MODEL>
struct CellState {
  static constexpr int B = Traits<MODEL>::B, NP = Traits<MODEL>::NP, NT = Traits<MODEL>::NT;
  double acc[B], dacc[B][B];
  double rho[NP], drho[NP];
  double drho_o2 = 0.0;   // black oil: d rho_oil-phase / d x2 (undersaturated cells)
  double lam[NT], dlam[NT][B];
  double lt, dlt[B];
};

__host__ __device__ inline double pvt_eval(const FluidDev& f, int row, double p, double& slope) {
  int m = f.npvt;
  int cnt = 0;
  for (int q = 0; q < m; ++q) cnt += (f.pvt[0][q] <= p) ? 1 : 0;
  int seg = cnt - 1;
  seg = seg < 0 ? 0 : (seg > m - 2 ? m - 2 : seg);
  double p0 = f.pvt[0][seg], p1 = f.pvt[0][seg + 1];
  double y0 = f.pvt[row][seg], y1 = f.pvt[row][seg + 1];
  slope = (y1 - y0) / (p1 - p0);
  return y0 + slope * (p - p0);
}

__device__ inline void clip01(double a, double& v, double& inside) {
  inside = (a > 0.0 && a < 1.0) ? 1.0 : 0.0;
  v = a < 0.0 ? 0.0 : (a > 1.0 ? 1.0 : a);
}

__device__ inline void corey(double sw, double swc, double sor, double& krw, double& dkrw,
                             double& kro, double& dkro) {
  double den = 1.0 - swc - sor;
  double a, ia, o, io;
  clip01((sw - swc) / den, a, ia);
  clip01((1.0 - sor - sw) / den, o, io);
  krw = a * a;
  dkrw = 2.0 * a * ia / den;
  kro = o * o;
  dkro = -2.0 * o * io / den;
}

template <int MODEL>
__device__ void cell_state(const FluidDev& f, double poro, const double* xv, CellState<MODEL>& s) {
  double p = xv[0];
  double pref = f.p_ref;
  double phi = poro * (1.0 + f.c_r * (p - pref));
  double dphi = poro * f.c_r;
  double rho_w = f.rho_w_ref * exp(f.c_w * (p - pref));
  double drho_w = f.c_w * rho_w;
  double mu_w = f.mu_w * CP;
  if constexpr (MODEL == 1) {
    s.acc[0] = phi * rho_w;
    s.dacc[0][0] = dphi * rho_w + phi * drho_w;
    s.rho[0] = rho_w; s.drho[0] = drho_w;
    s.lam[0] = rho_w / mu_w;
    s.dlam[0][0] = drho_w / mu_w;
    s.lt = 1.0 / mu_w;
    s.dlt[0] = 0.0;
  } else if constexpr (MODEL == 2) {
    double sw = xv[1];
    double so = 1.0 - sw;
    double rho_o = f.rho_o_ref * exp(f.c_o * (p - pref));
    double drho_o = f.c_o * rho_o;
    double mu_o = f.mu_o * CP;
    double krw, dkrw, kro, dkro;
    corey(sw, f.s_wc, f.s_or, krw, dkrw, kro, dkro);
    s.acc[0] = phi * so * rho_o;
    s.acc[1] = phi * sw * rho_w;
    s.dacc[0][0] = so * (dphi * rho_o + phi * drho_o);
    s.dacc[0][1] = -phi * rho_o;
    s.dacc[1][0] = sw * (dphi * rho_w + phi * drho_w);
    s.dacc[1][1] = phi * rho_w;
    s.rho[0] = rho_o; s.drho[0] = drho_o;
    s.rho[1] = rho_w; s.drho[1] = drho_w;
    s.lam[0] = rho_o * kro / mu_o;
    s.dlam[0][0] = drho_o * kro / mu_o;
    s.dlam[0][1] = rho_o * dkro / mu_o;
    s.lam[1] = rho_w * krw / mu_w;
    s.dlam[1][0] = drho_w * krw / mu_w;
    s.dlam[1][1] = rho_w * dkrw / mu_w;
    s.lt = krw / mu_w + kro / mu_o;
    s.dlt[0] = 0.0;
    s.dlt[1] = dkrw / mu_w + dkro / mu_o;
  } else {
    // third unknown: S_g >= 0 (saturated), -p_b < 0 (undersaturated: no free
    // gas, Rs and mu_o at p_b, B_o = B_o(p_b) exp(-c_o (p - p_b)))
    double sw = xv[1], x2 = xv[2];
    const bool sat = x2 >= 0.0;
    double sg = sat ? x2 : 0.0;
    double dsg = sat ? 1.0 : 0.0;
    double pb = sat ? p : -x2;
    double so = 1.0 - sw - sg;
    double drs_b, dbo_b, dmuo_b, dbg, dmug;
    double rs = pvt_eval(f, 1, pb, drs_b);
    double bo_b = pvt_eval(f, 2, pb, dbo_b);
    double muo = pvt_eval(f, 3, pb, dmuo_b);
    double bg = pvt_eval(f, 4, p, dbg);
    double mug = pvt_eval(f, 5, p, dmug);
    double e = sat ? 1.0 : exp(-f.c_o * (p - pb));
    double bo = bo_b * e;
    double rs_p = sat ? drs_b : 0.0, rs_2 = sat ? 0.0 : -drs_b;
    double bo_p = sat ? dbo_b : -f.c_o * bo;
    double bo_2 = sat ? 0.0 : -(dbo_b * e + f.c_o * bo);
    double mu_p = sat ? dmuo_b : 0.0, mu_2 = sat ? 0.0 : -dmuo_b;
    muo *= CP; mu_p *= CP; mu_2 *= CP; mug *= CP; dmug *= CP;
    double rsc_o = f.rho_o_sc, rsc_g = f.rho_g_sc;
    double rho_oo = rsc_o / bo;
    double rho_oo_p = -rsc_o * bo_p / (bo * bo);
    double rho_oo_2 = -rsc_o * bo_2 / (bo * bo);
    double rho_og = rsc_g * rs / bo;
    double rho_og_p = rsc_g * (rs_p * bo - rs * bo_p) / (bo * bo);
    double rho_og_2 = rsc_g * (rs_2 * bo - rs * bo_2) / (bo * bo);
    double rho_g = rsc_g / bg;
    double drho_g = -rsc_g * dbg / (bg * bg);
    // relative permeabilities: Corey water / oil-water, quadratic gas, Stone II oil
    double krw, dkrw, krow, dkrow;
    corey(sw, f.s_wc, f.s_or, krw, dkrw, krow, dkrow);
    double g, ig, h, ih;
    clip01(sg / f.sg_den, g, ig);
    clip01((f.sg_den - sg) / f.sg_den, h, ih);
    double krg = g * g, dkrg = 2.0 * g * ig / f.sg_den;
    double krog = h * h, dkrog = -2.0 * h * ih / f.sg_den;
    double raw = (krow + krw) * (krog + krg) - krw - krg;
    bool pos = raw > 0.0;
    double kro = pos ? raw : 0.0;
    double dkro_w = pos ? (dkrow + dkrw) * (krog + krg) - dkrw : 0.0;
    double dkro_g = pos ? (krow + krw) * (dkrog + dkrg) - dkrg : 0.0;
    dkrg *= dsg;      // per unit of x2
    dkro_g *= dsg;
    s.acc[0] = phi * so * rho_oo;
    s.acc[1] = phi * sw * rho_w;
    s.acc[2] = phi * (so * rho_og + sg * rho_g);
    s.dacc[0][0] = so * (dphi * rho_oo + phi * rho_oo_p);
    s.dacc[0][1] = -phi * rho_oo;
    s.dacc[0][2] = -phi * rho_oo * dsg + phi * so * rho_oo_2;
    s.dacc[1][0] = sw * (dphi * rho_w + phi * drho_w);
    s.dacc[1][1] = phi * rho_w;
    s.dacc[1][2] = 0.0;
    s.dacc[2][0] = dphi * (so * rho_og + sg * rho_g) + phi * (so * rho_og_p + sg * drho_g);
    s.dacc[2][1] = -phi * rho_og;
    s.dacc[2][2] = phi * (-rho_og * dsg + so * rho_og_2 + rho_g * dsg);
    s.rho[0] = rho_oo + rho_og; s.drho[0] = rho_oo_p + rho_og_p;
    s.drho_o2 = rho_oo_2 + rho_og_2;
    s.rho[1] = rho_w; s.drho[1] = drho_w;
    s.rho[2] = rho_g; s.drho[2] = drho_g;
    // mass mobilities rho k_r / mu of each (component, phase) term
    auto mob = [](int t, CellState<MODEL>& st, double rho, double rho_p, double rho_2, double kr, double dkr_w,
                  double dkr_2, double mu, double dmu_p, double dmu_2) {
      st.lam[t] = rho * kr / mu;
      st.dlam[t][0] = (rho_p * kr - rho * kr * dmu_p / mu) / mu;
      st.dlam[t][1] = rho * dkr_w / mu;
      st.dlam[t][2] = (rho_2 * kr + rho * dkr_2 - rho * kr * dmu_2 / mu) / mu;
    };
    mob(0, s, rho_oo, rho_oo_p, rho_oo_2, kro, dkro_w, dkro_g, muo, mu_p, mu_2);
    mob(1, s, rho_w, drho_w, 0.0, krw, dkrw, 0.0, mu_w, 0.0, 0.0);
    mob(2, s, rho_og, rho_og_p, rho_og_2, kro, dkro_w, dkro_g, muo, mu_p, mu_2);
    mob(3, s, rho_g, drho_g, 0.0, krg, 0.0, dkrg, mug, dmug, 0.0);
    s.lt = krw / mu_w + kro / muo + krg / mug;
    s.dlt[0] = -kro * mu_p / (muo * muo) - krg * dmug / (mug * mug);
    s.dlt[1] = dkrw / mu_w + dkro_w / muo;
    s.dlt[2] = dkro_g / muo - kro * mu_2 / (muo * muo) + dkrg / mug;
  }
}

// planes of the per-cell state stored for the flux kernel
template <int MODEL>
struct PropPlanes {
  static constexpr int B = Traits<MODEL>::B, NP = Traits<MODEL>::NP, NT = Traits<MODEL>::NT;
  static constexpr int RHO = 0, DRHO = NP, LAM = 2 * NP, DLAM = 2 * NP + NT;
  static constexpr int LT = 2 * NP + NT + NT * B;   // total volumetric mobility (network feature)
  static constexpr int DRHO_O2 = LT + 1;            // black oil: d rho_oil-phase / d x2
  static constexpr int ACC = MODEL == 3 ? DRHO_O2 + 1 : LT + 1;   // acc(x) - acc(x_old) [B]
  static constexpr int DACC = ACC + B;                            // d acc / d x [B][B]
  static constexpr int COUNT = DACC + B * B;
};

// Per-cell state for the flux kernel: phase densities and mobilities with
// their derivatives, and the accumulation change acc(x) - acc(x_old) with
// its derivative (so the flux kernel, which needs every neighbour's state,
// does not evaluate the fluid model itself).
template <int MODEL>
__global__ __launch_bounds__(256) void props_kernel(FluidDev f, Lay L, const double* __restrict__ poro,
                                                    const double* __restrict__ xold, const double* __restrict__ x,
                                                    double* __restrict__ props) {
  using PP = PropPlanes<MODEL>;
  constexpr int B = Traits<MODEL>::B;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= L.n) return;
  double xv[B];
  for (int u = 0; u < B; ++u) xv[u] = x[(size_t)u * L.n + t];
  CellState<MODEL> s;
  cell_state<MODEL>(f, poro[t], xv, s);
  size_t n = L.n;
  {
    double xo[B];
    for (int u = 0; u < B; ++u) xo[u] = xold[(size_t)u * L.n + t];
    CellState<MODEL> so;
    cell_state<MODEL>(f, poro[t], xo, so);
    for (int r = 0; r < B; ++r) {
      props[(PP::ACC + r) * n + t] = s.acc[r] - so.acc[r];
      for (int u = 0; u < B; ++u) props[(PP::DACC + r * B + u) * n + t] = s.dacc[r][u];
    }
  }
  for (int q = 0; q < PP::NP; ++q) {
    props[(PP::RHO + q) * n + t] = s.rho[q];
    props[(PP::DRHO + q) * n + t] = s.drho[q];
  }
  for (int q = 0; q < PP::NT; ++q) {
    props[(PP::LAM + q) * n + t] = s.lam[q];
    for (int u = 0; u < B; ++u) props[(PP::DLAM + q * B + u) * n + t] = s.dlam[q][u];
  }
  props[PP::LT * n + t] = s.lt;
  if constexpr (MODEL == 3) props[PP::DRHO_O2 * n + t] = s.drho_o2;
}

template <int MODEL>
__global__ __launch_bounds__(256) void flux_kernel(Lay L, double dz, double top, double vol, double dt, double s0,
                                                   double s1, double s2, const double* __restrict__ tp,
                                                   const double* __restrict__ x, const double* __restrict__ props,
                                                   double* __restrict__ J, double* __restrict__ rhs) {
  using PP = PropPlanes<MODEL>;
  constexpr int B = Traits<MODEL>::B, NP = Traits<MODEL>::NP, NT = Traits<MODEL>::NT;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= L.n) return;
  const size_t n = L.n;
  int i, j, k;
  lay_coords(L, t, i, j, k);
  double xv[B];
  for (int u = 0; u < B; ++u) xv[u] = x[u * n + t];
  double R[B], Jd[B][B];
  for (int r = 0; r < B; ++r) {
    R[r] = vol * props[(PP::ACC + r) * n + t] / dt;
    for (int u = 0; u < B; ++u) Jd[r][u] = vol * props[(PP::DACC + r * B + u) * n + t] / dt;
  }
  const double scale[3] = {s0, s1, s2};
  // own state as stored (both sides of a face see identical values)
  double rho_s[NP], drho_s[NP], lam_s[NT], dlam_s[NT][B];
  for (int q = 0; q < NP; ++q) {
    rho_s[q] = props[(PP::RHO + q) * n + t];
    drho_s[q] = props[(PP::DRHO + q) * n + t];
  }
  double dro2_s = 0.0;
  if constexpr (MODEL == 3) dro2_s = props[PP::DRHO_O2 * n + t];
  for (int q = 0; q < NT; ++q) {
    lam_s[q] = props[(PP::LAM + q) * n + t];
    for (int u = 0; u < B; ++u) dlam_s[q][u] = props[(PP::DLAM + q * B + u) * n + t];
  }
  const double z_self = top + (k + 0.5) * dz;
  for (int d = 1; d < 7; ++d) {
    double Jo[B][B];
    for (int r = 0; r < B; ++r)
      for (int u = 0; u < B; ++u) Jo[r][u] = 0.0;
    int nb = lay_nbr(L, i, j, k, d);
    if (nb >= 0) {
      int axis = (d - 1) >> 1;
      bool plus = (d & 1) == 0;
      double T = plus ? tp[axis * n + t] : tp[axis * n + nb];
      int kn = k + (d == 5 ? -1 : (d == 6 ? 1 : 0));
      double z_nb = top + (kn + 0.5) * dz;
      double rho_n[NP], drho_n[NP], lam_n[NT], dlam_n[NT][B];
      for (int q = 0; q < NP; ++q) {
        rho_n[q] = props[(PP::RHO + q) * n + nb];
        drho_n[q] = props[(PP::DRHO + q) * n + nb];
      }
      for (int q = 0; q < NT; ++q) {
        lam_n[q] = props[(PP::LAM + q) * n + nb];
        for (int u = 0; u < B; ++u) dlam_n[q][u] = props[(PP::DLAM + q * B + u) * n + nb];
      }
      double dro2_n = 0.0;
      if constexpr (MODEL == 3) dro2_n = props[PP::DRHO_O2 * n + nb];
      // x2 derivative of the oil-phase potential difference (undersaturated cells)
      const double dd2lo = -0.5 * G_ACC * (plus ? (z_self - z_nb) : (z_nb - z_self)) * (plus ? dro2_s : dro2_n);
      const double dd2hi = -0.5 * G_ACC * (plus ? (z_self - z_nb) : (z_nb - z_self)) * (plus ? dro2_n : dro2_s);
      // orient the face lower-index cell -> upper-index cell
      const double* rho_lo = plus ? rho_s : rho_n;
      const double* rho_hi = plus ? rho_n : rho_s;
      const double* drho_lo = plus ? drho_s : drho_n;
      const double* drho_hi = plus ? drho_n : drho_s;
      double p_lo = plus ? xv[0] : x[nb];
      double p_hi = plus ? x[nb] : xv[0];
      double dzf = plus ? (z_self - z_nb) : (z_nb - z_self);
      double dphi[NP], ddlo[NP], ddhi[NP];
      bool uplo[NP];
      for (int q = 0; q < NP; ++q) {
        dphi[q] = (p_lo - p_hi) * BAR - 0.5 * (rho_lo[q] + rho_hi[q]) * G_ACC * dzf;
        ddlo[q] = BAR - 0.5 * G_ACC * dzf * drho_lo[q];
        ddhi[q] = -BAR - 0.5 * G_ACC * dzf * drho_hi[q];
        uplo[q] = dphi[q] >= -TIE_BAR * BAR;
      }
      for (int q = 0; q < NT; ++q) {
        int c = Traits<MODEL>::row(q), ph = Traits<MODEL>::phase(q);
        double lam_lo = plus ? lam_s[q] : lam_n[q];
        double lam_hi = plus ? lam_n[q] : lam_s[q];
        double lam_up = uplo[ph] ? lam_lo : lam_hi;
        double F = T * lam_up * dphi[ph];
        double dFlo[B], dFhi[B];
        for (int u = 0; u < B; ++u) {
          double dl_lo = plus ? dlam_s[q][u] : dlam_n[q][u];
          double dl_hi = plus ? dlam_n[q][u] : dlam_s[q][u];
          dFlo[u] = T * (uplo[ph] ? dl_lo : 0.0) * dphi[ph];
          dFhi[u] = T * (uplo[ph] ? 0.0 : dl_hi) * dphi[ph];
        }
        dFlo[0] += T * lam_up * ddlo[ph];
        dFhi[0] += T * lam_up * ddhi[ph];
        if (MODEL == 3 && ph == 0) {
          dFlo[B - 1] += T * lam_up * dd2lo;
          dFhi[B - 1] += T * lam_up * dd2hi;
        }
        if (plus) {
          R[c] += F;
          for (int u = 0; u < B; ++u) {
            Jd[c][u] += dFlo[u];
            Jo[c][u] += dFhi[u];
          }
        } else {
          R[c] -= F;
          for (int u = 0; u < B; ++u) {
            Jo[c][u] -= dFlo[u];
            Jd[c][u] -= dFhi[u];
          }
        }
      }
    }
    for (int r = 0; r < B; ++r)
      for (int u = 0; u < B; ++u) J[tix(7 * B * B, (d * B + r) * B + u, t)] = Jo[r][u] / scale[r];
  }
  for (int r = 0; r < B; ++r) {
    rhs[r * n + t] = -(R[r] / scale[r]);
    for (int u = 0; u < B; ++u) J[tix(7 * B * B, r * B + u, t)] = Jd[r][u] / scale[r];
  }
}

// One thread per perforated cell (cells are distinct; checked at creation).
// A perforation of a rate-controlled well takes the BHP from the unknowns
// (x[b n + well]) and also records its border entries: B = dR_cell/dp_h,
// C = dR_w/dx_cell (scaled like the controlled component's rows), and the
// controlled component's mass rate and its derivative in p_h (unscaled) for
// the well equation.
template <int MODEL>
__global__ void well_kernel(FluidDev f, Lay L, int nperf, const Perf* __restrict__ perfs,
                            const RateWell* __restrict__ rwells, double s0, double s1, double s2,
                            const double* __restrict__ poro, const double* __restrict__ x,
                            double* __restrict__ J, double* __restrict__ rhs, double* __restrict__ bord,
                            double* __restrict__ pq) {
  constexpr int B = Traits<MODEL>::B, NT = Traits<MODEL>::NT;
  int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nperf) return;
  const size_t n = L.n;
  Perf pf = perfs[w];
  int t = pf.cell;
  double xv[B];
  for (int u = 0; u < B; ++u) xv[u] = x[u * n + t];
  CellState<MODEL> s;
  cell_state<MODEL>(f, poro[t], xv, s);
  const double scale[3] = {s0, s1, s2};
  const double ph = pf.rw >= 0 ? x[(size_t)B * n + pf.rw] : pf.bhp;
  double dh = ph - xv[0];
  double q[B], dq[B][B], dqh[B];
  for (int r = 0; r < B; ++r) {
    q[r] = 0.0;
    dqh[r] = 0.0;
    for (int u = 0; u < B; ++u) dq[r][u] = 0.0;
  }
  if (pf.kind == CPR_WELL_INJECTOR) {
    // water injector: total mobility of the cell, water density
    constexpr int WR = MODEL == 1 ? 0 : 1;   // water row and phase
    double rho = s.rho[WR], drho = s.drho[WR];
    double drive = dh * BAR - rho * G_ACC * pf.dzh;
    q[WR] = pf.wi * rho * s.lt * drive;
    dqh[WR] = pf.wi * rho * s.lt * BAR;
    for (int u = 0; u < B; ++u) {
      double v = pf.wi * rho * s.dlt[u] * drive;
      if (u == 0) {
        v += pf.wi * drho * s.lt * drive;
        v += pf.wi * rho * s.lt * (-BAR - drho * G_ACC * pf.dzh);
      }
      dq[WR][u] = v;
    }
  } else {
    for (int tt = 0; tt < NT; ++tt) {
      int c = Traits<MODEL>::row(tt), ph_ = Traits<MODEL>::phase(tt);
      double rho = s.rho[ph_], drho = s.drho[ph_];
      double drive = dh * BAR - rho * G_ACC * pf.dzh;
      q[c] += pf.wi * s.lam[tt] * drive;
      dqh[c] += pf.wi * s.lam[tt] * BAR;
      for (int u = 0; u < B; ++u) {
        double v = pf.wi * s.dlam[tt][u] * drive;
        if (u == 0) v += pf.wi * s.lam[tt] * (-BAR - drho * G_ACC * pf.dzh);
        if (MODEL == 3 && u == 2 && ph_ == 0) v += pf.wi * s.lam[tt] * (-s.drho_o2 * G_ACC * pf.dzh);
        dq[c][u] += v;
      }
    }
  }
  for (int r = 0; r < B; ++r) {
    rhs[r * n + t] += q[r] / scale[r];
    for (int u = 0; u < B; ++u) J[tix(7 * B * B, r * B + u, t)] -= dq[r][u] / scale[r];
  }
  if (pf.rw >= 0) {
    const int c = rwells[pf.rw].comp;
    double* bq = bord + (size_t)w * 6;
    for (int r = 0; r < 3; ++r) {
      bq[r] = r < B ? -dqh[r] / scale[r] : 0.0;
      bq[3 + r] = r < B ? dq[c][r] / scale[c] : 0.0;
    }
    pq[2 * w] = q[c];
    pq[2 * w + 1] = dqh[c];
  }
}

// Well equation of each rate-controlled well, summed over its perforations
// in order: R_w = (sum q_c - target) / s_c, D = sum dq_c/dp_h / s_c; the
// right-hand side tail receives -R_w.
__global__ void rate_well_kernel(int b, int n, int nrate, const RateWell* __restrict__ rwells,
                                 const double* __restrict__ pq, double s0, double s1, double s2,
                                 double* __restrict__ bordD, double* __restrict__ rhs) {
  int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nrate) return;
  const double scale[3] = {s0, s1, s2};
  const RateWell R = rwells[w];
  const double sc = scale[R.comp];
  double acc = -R.target, d = 0.0;
  for (int q = R.p0; q < R.p1; ++q) {
    acc += pq[2 * q];
    d += pq[2 * q + 1];
  }
  rhs[(size_t)b * n + w] = -(acc / sc);
  bordD[w] = d / sc;
}

__global__ void trans_kernel(Lay L, double dx, double dy, double dz, const double* __restrict__ perm,
                             double* __restrict__ tp) {
  const double MD = 9.869233e-16;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= L.n) return;
  const size_t n = L.n;
  int i = t % L.nx, jk = t / L.nx;
  int j = jk % L.ny, k = jk / L.ny;
  int c = lay_index(L, i, j, k);
  const int nbr[3] = {i + 1 < L.nx ? t + 1 : -1, j + 1 < L.ny ? t + L.nx : -1,
                      k + 1 < L.nz ? t + L.nx * L.ny : -1};
  const double area[3] = {dy * dz, dx * dz, dx * dy};
  const double dd[3] = {dx, dy, dz};
  for (int a = 0; a < 3; ++a) {
    double T = 0.0;
    if (nbr[a] >= 0) {
      double ka = perm[a * n + t] * MD, kb = perm[a * n + nbr[a]] * MD;
      double s = ka + kb;
      T = s > 0.0 ? 2.0 * area[a] * ka * kb / (dd[a] * s) : 0.0;
    }
    tp[a * n + c] = T;
  }
}

}  // namespace

void launch_transmissibility(const Lay& L, const cpr_grid_t& g, const double* perm_nat,
                             double* tp, hipStream_t s) {
  trans_kernel<<<div_up(L.n, 256), 256, 0, s>>>(L, g.dx, g.dy, g.dz, perm_nat, tp);
}

void launch_assemble(cpr_ctx* ctx, const double* xold_cs, const double* x_cs, double dt_days,
                     double* rhs_cs) {
  const Lay& L = ctx->lay;
  double dt = dt_days * DAY;
  double sc[3] = {0, 0, 0};
  for (int c = 0; c < ctx->b; ++c) sc[c] = ctx->rho_scale[c] * ctx->cell_vol * ctx->phibar / dt;
  // per-cell kernels in one-wave workgroups
  int nb = div_up(L.n, 64);
  int np = (int)ctx->perfs.size();
  hipStream_t s = ctx->stream;
  if (ctx->fl.model == 1) {
    props_kernel<1><<<nb, 64, 0, s>>>(ctx->fl, L, ctx->poro, xold_cs, x_cs, ctx->props);
    prof_begin(ctx, CPR_KCLASS_ASSEMBLE);
    flux_kernel<1><<<nb, 64, 0, s>>>(L, ctx->grid.dz, ctx->grid.top, ctx->cell_vol, dt, sc[0], sc[1],
                                      sc[2], ctx->tp, x_cs, ctx->props, ctx->J, rhs_cs);
    prof_end(ctx, CPR_KCLASS_ASSEMBLE);
    if (np) well_kernel<1><<<div_up(np, 64), 64, 0, s>>>(ctx->fl, L, np, ctx->perfs_d, ctx->rwells_d, sc[0],
                                                        sc[1], sc[2], ctx->poro, x_cs, ctx->J, rhs_cs,
                                                        ctx->bord, ctx->pq);
  } else if (ctx->fl.model == 2) {
    props_kernel<2><<<nb, 64, 0, s>>>(ctx->fl, L, ctx->poro, xold_cs, x_cs, ctx->props);
    prof_begin(ctx, CPR_KCLASS_ASSEMBLE);
    flux_kernel<2><<<nb, 64, 0, s>>>(L, ctx->grid.dz, ctx->grid.top, ctx->cell_vol, dt, sc[0], sc[1],
                                      sc[2], ctx->tp, x_cs, ctx->props, ctx->J, rhs_cs);
    prof_end(ctx, CPR_KCLASS_ASSEMBLE);
    if (np) well_kernel<2><<<div_up(np, 64), 64, 0, s>>>(ctx->fl, L, np, ctx->perfs_d, ctx->rwells_d, sc[0],
                                                        sc[1], sc[2], ctx->poro, x_cs, ctx->J, rhs_cs,
                                                        ctx->bord, ctx->pq);
  } else {
    props_kernel<3><<<nb, 64, 0, s>>>(ctx->fl, L, ctx->poro, xold_cs, x_cs, ctx->props);
    prof_begin(ctx, CPR_KCLASS_ASSEMBLE);
    flux_kernel<3><<<nb, 64, 0, s>>>(L, ctx->grid.dz, ctx->grid.top, ctx->cell_vol, dt, sc[0], sc[1],
                                      sc[2], ctx->tp, x_cs, ctx->props, ctx->J, rhs_cs);
    prof_end(ctx, CPR_KCLASS_ASSEMBLE);
    if (np) well_kernel<3><<<div_up(np, 64), 64, 0, s>>>(ctx->fl, L, np, ctx->perfs_d, ctx->rwells_d, sc[0],
                                                        sc[1], sc[2], ctx->poro, x_cs, ctx->J, rhs_cs,
                                                        ctx->bord, ctx->pq);
  }
  if (ctx->nrate)
    rate_well_kernel<<<div_up(ctx->nrate, 64), 64, 0, s>>>(ctx->b, L.n, ctx->nrate, ctx->rwells_d, ctx->pq, sc[0],
                                                          sc[1], sc[2], ctx->bord_d, rhs_cs);
}

// Number of SoA planes the per-cell state needs (allocation size).
int props_planes(int model) {
  return model == 1 ? PropPlanes<1>::COUNT : model == 2 ? PropPlanes<2>::COUNT : PropPlanes<3>::COUNT;
}

// Plane of the per-cell state that holds the total volumetric mobility.
int props_lt_plane(int model) {
  return model == 1 ? PropPlanes<1>::LT : model == 2 ? PropPlanes<2>::LT : PropPlanes<3>::LT;
}

double host_pvt(const FluidDev& f, int row, double p) {
  double s;
  return pvt_eval(f, row, p, s);
}
