// One backward-Euler time step by the inexact Newton method (Algorithm 1)
// with the forcing terms of eq. (14) and time-step cuts.
//
// Everything stays on the device in the colour-split layout: x_old and the
// iterate x, the right-hand side b = -F(x) (ctx->rs), the Newton correction
// (ctx->xs) and the linear residual r = b - A dx that the Krylov solver
// leaves behind (FGMRES: ctx->tmp; BiCGSTAB: the first workspace vector).
// The host reads the norms it needs to choose theta_l and to stop.
#include <cmath>

#include "internal.h"

namespace {

// d = a - b (for ||b^l - r^(l-1)||)
__global__ void diff_kernel(long len, const double* __restrict__ a, const double* __restrict__ b,
                            double* __restrict__ d) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < len) d[t] = a[t] - b[t];
}

double forcing(const cpr_newton_options_t& no, double rtol, int l, double bn, double bn_prev,
               double rn_prev, double diff_prev) {
  if (no.forcing == CPR_FORCING_FIXED) return rtol;
  double t;
  if (l == 0)
    t = no.theta0;
  else if (no.forcing == CPR_FORCING_EW1)
    t = diff_prev / bn_prev;
  else if (no.forcing == CPR_FORCING_EW2)
    t = std::fabs(bn - rn_prev) / bn_prev;
  else
    t = no.gamma * std::pow(bn / bn_prev, no.beta);
  return std::fmin(std::fmax(t, no.theta_min), no.theta_max);
}

// Conditions that fail a Newton attempt (and cut the step) rather than
// the call.
bool attempt_failure(int rc) { return rc == CPR_ESINGULAR || rc == CPR_ENONFINITE || rc == CPR_EBREAKDOWN; }

}  // namespace

int time_step(cpr_ctx* ctx, const double* xold_cs, double* x_cs, double dt_days, const cpr_options_t& lin,
              const cpr_newton_options_t& no, cpr_newton_stats_t* st) {
  hipStream_t s = ctx->stream;
  const int b = ctx->b;
  const long len = vec_len(ctx);
  const bool bicg = no.krylov == CPR_KRYLOV_BICGSTAB;
  cpr_newton_stats_t S = {};
  double dt = dt_days;
  int rc;
  if (bicg && (rc = ensure_krylov_capacity(ctx, lin.restart > 8 ? lin.restart : 8)) != CPR_OK) return rc;
  for (int cut = 0; cut <= no.max_cuts; ++cut) {
    CPR_TRY(hipMemcpyAsync(x_cs, xold_cs, len * sizeof(double), hipMemcpyDeviceToDevice, s));
    launch_assemble(ctx, xold_cs, x_cs, dt, ctx->rs);
    ctx->assembled = 1;
    ctx->setup_done = 0;
    double bb;
    if ((rc = reduce_dot(ctx, ctx->rs, ctx->rs, len, &bb)) != CPR_OK) return rc;
    double bn = std::sqrt(bb);
    const double b0 = bn;
    double bn_prev = 0.0, rn_prev = 0.0, diff_prev = 0.0;
    int l = 0, lin_total = 0;
    bool ok = false;
    S.bnorm[0] = bn;
    while (std::isfinite(bn)) {
      if (bn == 0.0 || bn < no.newton_tol * b0) { ok = true; break; }
      if (l >= no.max_newton) break;
      cpr_options_t o = lin;
      o.rtol = forcing(no, lin.rtol, l, bn, bn_prev, rn_prev, diff_prev);
      o.x0 = 0;   // every Newton correction starts from zero
      rc = setup_with_options(ctx, o);
      if (attempt_failure(rc)) break;
      if (rc != CPR_OK) return rc;
      if (ctx->opt.learned) CPR_TRY(hipMemsetAsync(ctx->nncount, 0, 2 * sizeof(int), s));
      cpr_stats_t ls = {};
      rc = bicg ? bicgstab_solve(ctx, &ls) : fgmres_solve(ctx, &ls);
      if (attempt_failure(rc)) break;
      if (rc < 0) return rc;
      const double* r = bicg ? ctx->V : ctx->tmp;   // b - A dx
      double rr;
      if ((rc = reduce_dot(ctx, r, r, len, &rr)) != CPR_OK) return rc;
      launch_newton_update(b, ctx->lay.n, ctx->nrate, pb_floor(ctx->fl), x_cs, ctx->xs, s);
      launch_assemble(ctx, xold_cs, x_cs, dt, ctx->rs);
      ctx->setup_done = 0;
      diff_kernel<<<div_up(len, 256), 256, 0, s>>>(len, ctx->rs, r, ctx->vout);
      double dd;
      if ((rc = reduce_dot(ctx, ctx->vout, ctx->vout, len, &dd)) != CPR_OK) return rc;
      if ((rc = reduce_dot(ctx, ctx->rs, ctx->rs, len, &bb)) != CPR_OK) return rc;
      bn_prev = bn;
      rn_prev = std::sqrt(rr);
      diff_prev = std::sqrt(dd);
      bn = std::sqrt(bb);
      if (l < CPR_NEWTON_HIST) {
        S.theta[l] = o.rtol;
        S.lin_its[l] = ls.iterations;
        S.bnorm[l + 1] = bn;
      }
      lin_total += ls.iterations;
      l += 1;
    }
    S.total_newton += l;
    S.total_linear += lin_total;
    S.newton_iterations = l;
    S.linear_iterations = lin_total;
    S.cuts = cut;
    S.dt_taken = dt;
    S.converged = ok ? 1 : 0;
    if (ok) {
      ctx->err.clear();
      if (st) *st = S;
      return launch_check(ctx, "cpr_time_step");
    }
    dt *= 0.5;
  }
  CPR_TRY(hipMemcpyAsync(x_cs, xold_cs, len * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (st) *st = S;
  int rc2 = launch_check(ctx, "cpr_time_step");
  if (rc2 != CPR_OK) return rc2;
  set_err(ctx, CPR_NOT_CONVERGED, "the Newton iteration did not converge after the last time-step cut");
  return CPR_NOT_CONVERGED;
}
