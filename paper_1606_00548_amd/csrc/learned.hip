// Learned pressure correction inside the CPR preconditioner (an addition to
// the paper's method).
//
// After the multigrid cycle has produced dp_mg for the decoupled pressure
// residual r~_p, the network sees what the cycle left behind,
//   r' = r~_p - A_p dp_mg,
// through three per-cell features (standardised ln k_x, standardised ln of
// the total mobility, and D^-1 r' / s with s = rms(D^-1 r'), D = diag A_p)
// and proposes a direction d = N(features); the step minimising the
// pressure residual, alpha = <A_p d, r'> / <A_p d, A_p d>, gives
// dp_nn = alpha d.  Plain CPR judges it in FP64: the correction is kept only
// if ||r' - A_p dp_nn||_2 < ||r'||_2, otherwise the multigrid result stands.
// For this alpha, ||r' - alpha A_p d||^2 = ||r'||^2 - <A_p d, r'>^2 / ||A_p d||^2,
// so the judge is evaluated from the two sums that give alpha: it rejects a
// correction whose sums are not finite or whose A_p d or <A_p d, r'>
// vanishes.  Everything stays on the device (the decision is a flag read by
// the kernel that applies the correction), so the learned stage adds no
// host synchronisation to an FGMRES iteration.
//
// Per application: r' and its sums (writing the unscaled third feature
// D^-1 r' straight into the network input; the first two features depend
// only on the state and are written at setup), the sums' totals (s and
// 1/s, which the first convolution applies as it loads the input), the
// network, A_p d with its sums read from the network output in natural
// order, alpha and the decision, and the correction.
//
// With options.nn_level = l >= 1 the same kernels run inside the multigrid
// cycle on level l (called after that level's post-smoothing): r' =
// r_l - A_l x_l, D = diag A_l, and the state features are the means of
// ln k_x and ln lambda_t over each coarse cell's 2^l x 2^l x 2^l block of
// fine cells, formed at setup; a second network object on that level's
// grid holds the same parameters.
#include <cmath>

#include "internal.h"

int nn_infer(cpr_nn* nn, const float* x3, float* y, const double* xscale);
float* nn_output(cpr_nn* nn);
int props_lt_plane(int model);

namespace {

constexpr int LB = 256;
// device scalars (ctx->nnscal)
enum { S_MK = 0, S_SK, S_ML, S_SL, S_RMS, S_R2, S_RR2, S_ACC, S_ALPHA, S_INV, S_COUNT };

__device__ inline double block_sum(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < LB / 64; ++w) s += sh[w];
  return s;
}

// Sum of nblk block partials by one block of LB threads, in a fixed order
// (strided per-thread sums, then the wavefront and block tree); the total
// is returned to thread 0.
__device__ inline double partial_total(const double* __restrict__ part, int nblk, double* sh) {
  double v = 0.0;
  for (int k = threadIdx.x; k < nblk; k += LB) v += part[k];
  return block_sum(v, sh);
}

// per-block partials of ln kx, ln kx^2, ln lt, ln lt^2
__global__ __launch_bounds__(LB) void stats_partial_kernel(int n, const double* __restrict__ lnk,
                                                           const double* __restrict__ lt, double* __restrict__ part,
                                                           int nblk) {
  __shared__ double sh[LB / 64];
  double a = 0, b = 0, c = 0, d = 0;
  for (int t = blockIdx.x * LB + threadIdx.x; t < n; t += nblk * LB) {
    double k = lnk[t], l = log(lt[t]);
    a += k; b += k * k; c += l; d += l * l;
  }
  double r[4] = {a, b, c, d};
  for (int q = 0; q < 4; ++q) {
    double s = block_sum(r[q], sh);
    if (threadIdx.x == 0) part[(size_t)q * nblk + blockIdx.x] = s;
  }
}

__global__ __launch_bounds__(LB) void stats_final_kernel(int n, const double* __restrict__ part, int nblk,
                                                         double* __restrict__ scal) {
  __shared__ double sh[LB / 64];
  double s[4];
  for (int q = 0; q < 4; ++q) s[q] = partial_total(part + (size_t)q * nblk, nblk, sh);
  if (threadIdx.x != 0) return;
  double mk = s[0] / n, ml = s[2] / n;
  double vk = s[1] / n - mk * mk, vl = s[3] / n - ml * ml;
  scal[S_MK] = mk;
  scal[S_SK] = vk > 1e-24 ? sqrt(vk) : 1.0;
  scal[S_ML] = ml;
  scal[S_SL] = vl > 1e-24 ? sqrt(vl) : 1.0;
}

// r' = rp - A_p dp on the fine colour-split level, with block partials of
// sum (r'/a_0)^2 and sum r'^2.  rp / dp null: r' already stored.  feat
// (optional): the network input [natural cell][3], whose third channel
// receives r'/a_0 (unscaled).
template <typename T>
__global__ __launch_bounds__(LB) void rprime_kernel(Lay L, const double* __restrict__ A, const T* __restrict__ rp,
                                                    const T* __restrict__ dp, double* __restrict__ rprime,
                                                    double* __restrict__ part, int nblk, float* __restrict__ feat) {
  __shared__ double sh[LB / 64];
  double a = 0, b = 0;
  for (int t = blockIdx.x * LB + threadIdx.x; t < L.n; t += nblk * LB) {
    double r;
    if (rp) {
      CsCell cc = cs_decode(L, t);
      double y = A[t] * (double)dp[t];
#pragma unroll
      for (int d = 1; d < 7; ++d) {
        int nb = cs_nb(L, cc, d);
        if (nb >= 0) y += A[(size_t)d * L.n + t] * (double)dp[nb];
      }
      r = (double)rp[t] - y;
      rprime[t] = r;
    } else {
      r = rprime[t];
    }
    double q = r / A[t];
    a += q * q;
    b += r * r;
    if (feat) {
      int i, j, k;
      lay_coords(L, t, i, j, k);
      feat[(i + (long)L.nx * (j + (long)L.ny * k)) * 3 + 2] = (float)q;
    }
  }
  double s = block_sum(a, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
  s = block_sum(b, sh);
  if (threadIdx.x == 0) part[(size_t)nblk + blockIdx.x] = s;
}

__global__ __launch_bounds__(LB) void rprime_final_kernel(int n, const double* __restrict__ part, int nblk,
                                                          double* __restrict__ scal) {
  __shared__ double sh[LB / 64];
  double a = partial_total(part, nblk, sh);
  double b = partial_total(part + nblk, nblk, sh);
  if (threadIdx.x != 0) return;
  const double rms = sqrt(a / n);
  scal[S_RMS] = rms;
  scal[S_INV] = rms > 0 ? 1.0 / rms : 0.0;
  scal[S_R2] = b;
}

// network input [natural cell][3]
__global__ __launch_bounds__(LB) void features_kernel(Lay L, const double* __restrict__ lnk,
                                                      const double* __restrict__ lt, const double* __restrict__ A,
                                                      const double* __restrict__ rprime,
                                                      const double* __restrict__ scal, float* __restrict__ feat) {
  int t = blockIdx.x * LB + threadIdx.x;
  if (t >= L.n) return;
  int i, j, k;
  lay_coords(L, t, i, j, k);
  long nat = i + (long)L.nx * (j + (long)L.ny * k);
  double s = scal[S_RMS];
  feat[nat * 3 + 0] = (float)((lnk[t] - scal[S_MK]) / scal[S_SK]);
  feat[nat * 3 + 1] = (float)((log(lt[t]) - scal[S_ML]) / scal[S_SL]);
  feat[nat * 3 + 2] = s > 0 ? (float)((rprime[t] / A[t]) / s) : 0.f;
}

// The two state features of the network input (channels 0 and 1).
__global__ __launch_bounds__(LB) void state_features_kernel(Lay L, const double* __restrict__ lnk,
                                                            const double* __restrict__ lt,
                                                            const double* __restrict__ scal, float* __restrict__ feat) {
  int t = blockIdx.x * LB + threadIdx.x;
  if (t >= L.n) return;
  int i, j, k;
  lay_coords(L, t, i, j, k);
  long nat = i + (long)L.nx * (j + (long)L.ny * k);
  feat[nat * 3 + 0] = (float)((lnk[t] - scal[S_MK]) / scal[S_SK]);
  feat[nat * 3 + 1] = (float)((log(lt[t]) - scal[S_ML]) / scal[S_SL]);
}

// q = A_p d for the network output d (FP32, natural order), with block
// partials of <q, r'> and <q, q>.
__global__ __launch_bounds__(LB) void apply_dir_kernel(Lay L, const double* __restrict__ A,
                                                       const double* __restrict__ rprime,
                                                       const float* __restrict__ y, double* __restrict__ q,
                                                       double* __restrict__ part, int nblk) {
  __shared__ double sh[LB / 64];
  const long sx = 1, sy = L.nx, sz = (long)L.nx * L.ny;
  double a = 0, b = 0;
  for (int t = blockIdx.x * LB + threadIdx.x; t < L.n; t += nblk * LB) {
    int i, j, k;
    lay_coords(L, t, i, j, k);
    const long nat = i + sy * j + sz * k;
    double v = ldnt(A + t) * (double)y[nat];
    // directions 1..6: -x, +x, -y, +y, -z, +z
    if (i > 0) v += ldnt(A + (size_t)1 * L.n + t) * (double)y[nat - sx];
    if (i < L.nx - 1) v += ldnt(A + (size_t)2 * L.n + t) * (double)y[nat + sx];
    if (j > 0) v += ldnt(A + (size_t)3 * L.n + t) * (double)y[nat - sy];
    if (j < L.ny - 1) v += ldnt(A + (size_t)4 * L.n + t) * (double)y[nat + sy];
    if (k > 0) v += ldnt(A + (size_t)5 * L.n + t) * (double)y[nat - sz];
    if (k < L.nz - 1) v += ldnt(A + (size_t)6 * L.n + t) * (double)y[nat + sz];
    q[t] = v;
    a += v * rprime[t];
    b += v * v;
  }
  double s = block_sum(a, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
  s = block_sum(b, sh);
  if (threadIdx.x == 0) part[(size_t)nblk + blockIdx.x] = s;
}

// alpha = <q, r'> / <q, q> and the judge: the correction is kept when
// ||r'||^2 - <q, r'>^2 / <q, q> < ||r'||^2 with finite sums, i.e. when q and
// <q, r'> do not vanish.
__global__ __launch_bounds__(LB) void alpha_kernel(const double* __restrict__ part, int nblk,
                                                   double* __restrict__ scal, int* __restrict__ count) {
  __shared__ double sh[LB / 64];
  double a = partial_total(part, nblk, sh);
  double b = partial_total(part + nblk, nblk, sh);
  if (threadIdx.x != 0) return;
  const bool finite = isfinite(a) && isfinite(b) && b > 0;
  const double al = finite ? a / b : 0.0;
  const double rr2 = finite ? scal[S_R2] - a * al : scal[S_R2];
  const bool accept = finite && isfinite(al) && a * al > 0;
  scal[S_ALPHA] = accept ? al : 0.0;
  scal[S_RR2] = rr2;
  scal[S_ACC] = accept ? 1.0 : 0.0;
  if (accept) count[0] += 1; else count[1] += 1;
}

// dp += alpha d when the judge accepted (d: network output, natural order)
template <typename T>
__global__ __launch_bounds__(LB) void correct_kernel(Lay L, const double* __restrict__ scal,
                                                     const float* __restrict__ y, T* __restrict__ dp) {
  int t = blockIdx.x * LB + threadIdx.x;
  if (t >= L.n || !(scal[S_ACC] > 0.0)) return;
  int i, j, k;
  lay_coords(L, t, i, j, k);
  dp[t] = (T)((double)dp[t] + scal[S_ALPHA] * (double)y[i + (long)L.nx * (j + (long)L.ny * k)]);
}

// Undo the count of the last application (one the solver ran ahead and
// then did not use).
__global__ void discard_kernel(const double* __restrict__ scal, int* __restrict__ count) {
  if (threadIdx.x == 0) count[scal[S_ACC] > 0.0 ? 0 : 1] -= 1;
}

// State fields of multigrid level C (grid = fine grid / f per axis): the
// mean of the fine ln kx over each coarse cell's f^3 block, and
// exp(mean ln lambda_t) so that the feature kernels' log gives the mean.
__global__ void level_fields_kernel(Lay F, Lay C, int f, const double* __restrict__ lnk,
                                    const double* __restrict__ lt, double* __restrict__ lnk_l,
                                    double* __restrict__ lt_l) {
  int tc = blockIdx.x * blockDim.x + threadIdx.x;
  if (tc >= C.n) return;
  int ci, cj, ck;
  lay_coords(C, tc, ci, cj, ck);
  double a = 0.0, b = 0.0;
  for (int dz = 0; dz < f; ++dz)
    for (int dy = 0; dy < f; ++dy)
      for (int dx = 0; dx < f; ++dx) {
        const int t = lay_index(F, ci * f + dx, cj * f + dy, ck * f + dz);
        a += lnk[t];
        b += log(lt[t]);
      }
  const double inv = 1.0 / ((double)f * f * f);
  lnk_l[tc] = a * inv;
  lt_l[tc] = exp(b * inv);
}

__global__ void lnk_kernel(Lay L, const double* __restrict__ perm, double* __restrict__ lnk) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= L.n) return;
  int i = t % L.nx, jk = t / L.nx, j = jk % L.ny, k = jk / L.ny;
  lnk[lay_index(L, i, j, k)] = log(perm[t]);
}

}  // namespace

void launch_lnk(const Lay& L, const double* perm_nat, double* lnk, hipStream_t s) {
  lnk_kernel<<<div_up(L.n, 256), 256, 0, s>>>(L, perm_nat, lnk);
}


// Feature statistics of the current state (after assembly), at setup, on
// the level the learned stage acts on (options.nn_level).
int learned_setup(cpr_ctx* ctx, bool need_nn) {
  if (need_nn && !ctx->nn) return set_err(ctx, CPR_EINVAL, "options.learned set but no network attached");
  if (!ctx->assembled) return set_err(ctx, CPR_EINVAL, "the learned stage needs an assembled state");
  const double* lt = ctx->props + (size_t)props_lt_plane(ctx->fl.model) * ctx->lay.n;
  const int lv = ctx->opt.nn_level;
  if (lv == 0) {
    stats_partial_kernel<<<ctx->nblk, LB, 0, ctx->stream>>>(ctx->lay.n, ctx->lnk, lt, ctx->part, ctx->nblk);
    stats_final_kernel<<<1, LB, 0, ctx->stream>>>(ctx->lay.n, ctx->part, ctx->nblk, ctx->nnscal);
    state_features_kernel<<<div_up(ctx->lay.n, LB), LB, 0, ctx->stream>>>(ctx->lay, ctx->lnk, lt, ctx->nnscal,
                                                                         ctx->feat);
    return launch_check(ctx, "learned_setup");
  }
  if (lv >= (int)ctx->levels.size() || lv >= vcycle_fused_level(ctx))
    return set_err(ctx, CPR_EINVAL, "nn_level must name a multigrid level above those of the single-workgroup cycle");
  const Lay& L = ctx->levels[lv].lay;
  const Lay& F = ctx->lay;
  if (!L.cs || L.nxr != L.nx || L.nx % 8 || L.ny % 8 || L.nz % 8 || F.nx != L.nx << lv || F.ny != L.ny << lv ||
      F.nz != L.nz << lv)
    return set_err(ctx, CPR_EINVAL, "nn_level: the level needs dimensions divisible by 8 and exactly 2^-l of the grid");
  if (need_nn) {
    if (ctx->theta.empty()) return set_err(ctx, CPR_EINVAL, "options.learned set but no network attached");
    if (!ctx->nn_lv || ctx->nn_lv_dims[0] != L.nx || ctx->nn_lv_dims[1] != L.ny || ctx->nn_lv_dims[2] != L.nz) {
      if (ctx->nn_lv) cpr_nn_destroy(ctx->nn_lv);
      ctx->nn_lv = nullptr;
      cpr_nn_t* nn = nullptr;
      int rc = cpr_nn_create(L.nx, L.ny, L.nz, 1, ctx->stream, &nn);
      if (rc != CPR_OK) {
        std::string m = nn ? cpr_nn_last_error(nn) : "network creation failed";
        if (nn) cpr_nn_destroy(nn);
        return set_err(ctx, rc, m);
      }
      ctx->nn_lv = nn;
      ctx->nn_lv_dims[0] = L.nx; ctx->nn_lv_dims[1] = L.ny; ctx->nn_lv_dims[2] = L.nz;
      rc = cpr_nn_set_params(nn, ctx->theta.data());
      if (rc != CPR_OK) return set_err(ctx, rc, cpr_nn_last_error(nn));
    }
  }
  if (ctx->lvl_cap < (size_t)L.n) {
    dev_free(ctx->mem, ctx->lnk_l);
    dev_free(ctx->mem, ctx->lt_l);
    ctx->lnk_l = ctx->lt_l = nullptr;
    ctx->lvl_cap = 0;
    CPR_TRY(dev_malloc(ctx->mem, (void**)&ctx->lnk_l, (size_t)L.n * sizeof(double)));
    CPR_TRY(dev_malloc(ctx->mem, (void**)&ctx->lt_l, (size_t)L.n * sizeof(double)));
    ctx->lvl_cap = L.n;
  }
  level_fields_kernel<<<div_up(L.n, LB), LB, 0, ctx->stream>>>(F, L, 1 << lv, ctx->lnk, lt, ctx->lnk_l, ctx->lt_l);
  stats_partial_kernel<<<ctx->nblk, LB, 0, ctx->stream>>>(L.n, ctx->lnk_l, ctx->lt_l, ctx->part, ctx->nblk);
  stats_final_kernel<<<1, LB, 0, ctx->stream>>>(L.n, ctx->part, ctx->nblk, ctx->nnscal);
  state_features_kernel<<<div_up(L.n, LB), LB, 0, ctx->stream>>>(L, ctx->lnk_l, ctx->lt_l, ctx->nnscal, ctx->feat);
  return launch_check(ctx, "learned_setup");
}

// Blocks of the per-application stage kernels on n cells: one cell per
// thread where the partial-sum buffer (66 nblk values, two per block here)
// allows.
static int stage_blocks(const cpr_ctx* ctx, int n) {
  const long nb = div_up((long)n, LB), cap = 32L * ctx->nblk;
  return (int)(nb < cap ? nb : cap);
}

// The level the learned stage acts on: its layout, operator and state fields.
struct StageLevel {
  Lay L;
  const double* A;
  const double* lnk;
  const double* lt;
};

static StageLevel stage_level(const cpr_ctx* ctx) {
  const int lv = ctx->opt.nn_level;
  if (lv == 0)
    return {ctx->lay, ctx->levels[0].A, ctx->lnk, ctx->props + (size_t)props_lt_plane(ctx->fl.model) * ctx->lay.n};
  return {ctx->levels[lv].lay, ctx->levels[lv].A, ctx->lnk_l, ctx->lt_l};
}

// r' and its norms for rp, dp of the stage's level (T = preconditioner
// type); with rp == nullptr, ctx->rprime already holds r'.
template <typename T>
static void rprime_launch(cpr_ctx* ctx, const StageLevel& S, const T* rp, const T* dp, float* feat = nullptr) {
  const int nb = stage_blocks(ctx, S.L.n);
  rprime_kernel<T><<<nb, LB, 0, ctx->stream>>>(S.L, S.A, rp, dp, ctx->rprime, ctx->part, nb, feat);
  rprime_final_kernel<<<1, LB, 0, ctx->stream>>>(S.L.n, ctx->part, nb, ctx->nnscal);
}

static void features_launch(cpr_ctx* ctx, const StageLevel& S) {
  features_kernel<<<div_up(S.L.n, LB), LB, 0, ctx->stream>>>(S.L, S.lnk, S.lt, S.A, ctx->rprime, ctx->nnscal,
                                                             ctx->feat);
}

// The learned stage on (rp, dp) of the stage's level in one CPR application.
template <typename T>
static int learned_stage_t(cpr_ctx* ctx, const StageLevel& S, cpr_nn* net, const T* rp, T* dp) {
  hipStream_t s = ctx->stream;
  rprime_launch<T>(ctx, S, rp, dp, ctx->feat);
  int rc = nn_infer(net, ctx->feat, nullptr, ctx->nnscal + S_INV);
  if (rc) return set_err(ctx, rc, "network inference failed");
  const float* y = nn_output(net);
  const int nb = stage_blocks(ctx, S.L.n);
  apply_dir_kernel<<<nb, LB, 0, s>>>(S.L, S.A, ctx->rprime, y, ctx->qbuf, ctx->part, nb);
  alpha_kernel<<<1, LB, 0, s>>>(ctx->part, nb, ctx->nnscal, ctx->nncount);
  correct_kernel<T><<<div_up(S.L.n, LB), LB, 0, s>>>(S.L, ctx->nnscal, y, dp);
  return CPR_OK;
}

void learned_discard_last(cpr_ctx* ctx) {
  discard_kernel<<<1, 64, 0, ctx->stream>>>(ctx->nnscal, ctx->nncount);
}

int learned_stage(cpr_ctx* ctx) {
  MGLevel& L0 = ctx->levels[0];
  const StageLevel S = stage_level(ctx);
  if (precond_fp32(ctx)) return learned_stage_t<float>(ctx, S, ctx->nn, L0.rf, L0.xf);
  return learned_stage_t<double>(ctx, S, ctx->nn, L0.r, L0.x);
}

int learned_stage_at(cpr_ctx* ctx, int level) {
  MGLevel& M = ctx->levels[level];
  const StageLevel S = stage_level(ctx);
  if (precond_fp32(ctx)) return learned_stage_t<float>(ctx, S, ctx->nn_lv, M.rf, M.xf);
  return learned_stage_t<double>(ctx, S, ctx->nn_lv, M.r, M.x);
}

// r' on the stage's level after a plain pressure stage (FP64 path).
void learned_rprime(cpr_ctx* ctx) {
  MGLevel& M = ctx->levels[ctx->opt.nn_level];
  rprime_launch<double>(ctx, stage_level(ctx), M.r, M.x);
}

// Features for a residual already stored in ctx->rprime.
void learned_features_from_rprime(cpr_ctx* ctx) {
  const StageLevel S = stage_level(ctx);
  rprime_launch<double>(ctx, S, nullptr, nullptr);
  features_launch(ctx, S);
}
