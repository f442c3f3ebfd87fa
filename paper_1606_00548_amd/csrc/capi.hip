// C ABI entry points: argument checks, layout conversion at the boundary,
// ownership of device buffers.  No exception leaves this file.
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <new>

#include "internal.h"

void release_hierarchy(cpr_ctx* ctx);
void launch_mixed_copies(cpr_ctx* ctx);

int set_err(cpr_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

int set_hip_err(cpr_ctx* ctx, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return set_err(ctx, e == hipErrorOutOfMemory ? CPR_ENOMEM : CPR_EHIP, m);
}

int launch_check(cpr_ctx* ctx, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_hip_err(ctx, e, what);
  return CPR_OK;
}

namespace {

template <typename T>
int dalloc(cpr_ctx* ctx, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = dev_malloc(ctx->mem, (void**)p, count * sizeof(T));
  if (e != hipSuccess) return set_hip_err(ctx, e, "device allocation");
  return CPR_OK;
}

void free_all(cpr_ctx* ctx) {
  release_hierarchy(ctx);
  void* bufs[] = {ctx->poro, ctx->tp, ctx->perfs_d, ctx->J, ctx->props, ctx->vin, ctx->vin2, ctx->vout,
                  ctx->w, ctx->R0, ctx->Dinv, ctx->Jf, ctx->Dinvf, ctx->flag, ctx->V, ctx->Z,
                  ctx->Y, ctx->rp, ctx->xs, ctx->rs, ctx->tmp, ctx->vf, ctx->zf, ctx->Yf, ctx->rpf,
                  ctx->part, ctx->hdev, ctx->lnk, ctx->rprime, ctx->qbuf, ctx->feat, ctx->nnscal,
                  ctx->nncount, ctx->Wabf, ctx->Jt, ctx->Rt, ctx->Rtf, ctx->Z1, ctx->Z1f, ctx->rwells_d,
                  ctx->bord, ctx->pq, ctx->bord_d, ctx->lnk_l, ctx->lt_l};
  for (void* b : bufs) dev_free(ctx->mem, b);
  if (ctx->hhost) (void)hipHostFree(ctx->hhost);
  ctx->hhost = nullptr;
  for (hipEvent_t e : ctx->ev) (void)hipEventDestroy(e);
  phase_timing_release(ctx);
  for (hipEvent_t e : {ctx->ev_q, ctx->ev_rap, ctx->ev_gj, ctx->ev_iter[0], ctx->ev_iter[1]})
    if (e) (void)hipEventDestroy(e);
  ctx->ev_q = ctx->ev_rap = ctx->ev_gj = ctx->ev_iter[0] = ctx->ev_iter[1] = nullptr;
  if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
  ctx->aux = nullptr;
  if (ctx->nn) cpr_nn_destroy(ctx->nn);
  ctx->nn = nullptr;
  if (ctx->nn_lv) cpr_nn_destroy(ctx->nn_lv);
  ctx->nn_lv = nullptr;
  ctx->ev.clear();
}

// Peaceman well index of a vertical well in an anisotropic block (m^3).
double peaceman(double kx_md, double ky_md, double dx, double dy, double dz, double rw, double skin) {
  const double MD = 9.869233e-16;
  double kx = kx_md * MD, ky = ky_md * MD;
  double rxy = std::sqrt(ky / kx), ryx = std::sqrt(kx / ky);
  double ro = 0.28 * std::sqrt(rxy * dx * dx + ryx * dy * dy) / (std::sqrt(rxy) + std::sqrt(ryx));
  return 2.0 * 3.141592653589793 * std::sqrt(kx * ky) * dz / (std::log(ro / rw) + skin);
}

int check_ctx(cpr_ctx* ctx) { return ctx ? CPR_OK : CPR_EINVAL; }

int create_impl(const cpr_grid_t* g, const cpr_fluid_t* f, const double* perm3, const double* poro,
                const cpr_well_t* wells, int nwells, void* stream, cpr_ctx* ctx) {
  if (!g || !f || !perm3 || !poro || (nwells > 0 && !wells) || nwells < 0)
    return set_err(ctx, CPR_EINVAL, "null argument");
  if (g->nx < 2 || g->ny < 1 || g->nz < 1 || (g->nx & 1))
    return set_err(ctx, CPR_EINVAL, "grid needs nx >= 2 even, ny >= 1, nz >= 1");
  long long n = (long long)g->nx * g->ny * g->nz;
  if (n > INT_MAX / 2) return set_err(ctx, CPR_EINVAL, "grid too large");
  if (!(g->dx > 0 && g->dy > 0 && g->dz > 0)) return set_err(ctx, CPR_EINVAL, "cell sizes must be > 0");
  if (f->model != CPR_MODEL_SINGLE_PHASE && f->model != CPR_MODEL_OIL_WATER && f->model != CPR_MODEL_BLACK_OIL)
    return set_err(ctx, CPR_EINVAL, "model must be 1 (single phase), 2 (oil-water) or 3 (black oil)");
  if (f->model == CPR_MODEL_BLACK_OIL && (!f->pvt || f->n_pvt < 2 || f->n_pvt > CPR_MAX_PVT))
    return set_err(ctx, CPR_EINVAL, "black oil needs a PVT table with 2..16 nodes");
  ctx->stream = (hipStream_t)stream;
  CPR_TRY(hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
  CPR_TRY(hipEventCreateWithFlags(&ctx->ev_q, hipEventDisableTiming));
  CPR_TRY(hipEventCreateWithFlags(&ctx->ev_rap, hipEventDisableTiming));
  CPR_TRY(hipEventCreateWithFlags(&ctx->ev_gj, hipEventDisableTiming));
  CPR_TRY(hipEventCreateWithFlags(&ctx->ev_iter[0], hipEventDisableTiming));
  CPR_TRY(hipEventCreateWithFlags(&ctx->ev_iter[1], hipEventDisableTiming));
  ctx->grid = *g;
  ctx->b = f->model;
  FluidDev& fl = ctx->fl;
  std::memset(&fl, 0, sizeof(fl));
  fl.model = f->model;
  fl.p_ref = f->p_ref; fl.rho_w_ref = f->rho_w_ref; fl.rho_o_ref = f->rho_o_ref;
  fl.rho_o_sc = f->rho_o_sc; fl.rho_g_sc = f->rho_g_sc;
  fl.c_w = f->c_w; fl.c_o = f->c_o; fl.c_r = f->c_r; fl.mu_w = f->mu_w; fl.mu_o = f->mu_o;
  fl.s_wc = f->s_wc; fl.s_or = f->s_or; fl.sg_den = f->sg_den;
  if (f->model == CPR_MODEL_BLACK_OIL) {
    fl.npvt = f->n_pvt;
    for (int r = 0; r < 6; ++r)
      for (int q = 0; q < f->n_pvt; ++q) fl.pvt[r][q] = f->pvt[(size_t)r * f->n_pvt + q];
    for (int q = 0; q + 1 < f->n_pvt; ++q)
      if (!(fl.pvt[0][q + 1] > fl.pvt[0][q])) return set_err(ctx, CPR_EINVAL, "PVT pressures must increase");
  }
  ctx->lay = make_lay(g->nx, g->ny, g->nz, true);
  const int b = ctx->b;
  const size_t N = (size_t)n;
  int rc;
  // rate-controlled wells append their BHPs to every vector
  for (int q = 0; q < nwells; ++q) {
    if (wells[q].control != CPR_CONTROL_BHP && wells[q].control != CPR_CONTROL_RATE)
      return set_err(ctx, CPR_EINVAL, "unknown well control");
    if (wells[q].control == CPR_CONTROL_RATE) {
      if (!(wells[q].rate >= 0) || !std::isfinite(wells[q].rate))
        return set_err(ctx, CPR_EINVAL, "well rate must be >= 0");
      ctx->nrate += 1;
    }
  }
  const size_t NV = b * N + ctx->nrate;
#define ALLOC(p, cnt) if ((rc = dalloc(ctx, &(p), (cnt))) != CPR_OK) return rc
  ALLOC(ctx->poro, N);
  ALLOC(ctx->tp, 3 * N);
  ALLOC(ctx->J, tiled_len(N, 7 * b * b));
  ALLOC(ctx->props, (size_t)props_planes(f->model) * N);
  ALLOC(ctx->vin, NV);
  ALLOC(ctx->vin2, NV);
  ALLOC(ctx->vout, NV);
  ALLOC(ctx->w, b * N);
  ALLOC(ctx->R0, tiled_len(N, 7 * b));
  ALLOC(ctx->Dinv, tiled_len(N, b * b));
  ALLOC(ctx->Y, b * N);
  ALLOC(ctx->xs, NV);
  ALLOC(ctx->rs, NV);
  ALLOC(ctx->tmp, NV);
  ALLOC(ctx->flag, 4);
  ALLOC(ctx->lnk, N);
  ALLOC(ctx->rprime, N);
  ALLOC(ctx->qbuf, N);
  ALLOC(ctx->feat, 3 * N);
  ALLOC(ctx->nnscal, 16);
  ALLOC(ctx->nncount, 2);
  ctx->nblk = div_up((long)b * n, 1024);
  if (ctx->nblk > 1024) ctx->nblk = 1024;
  ALLOC(ctx->part, 66 * (size_t)ctx->nblk);
  ALLOC(ctx->hdev, 1024);
#undef ALLOC
  {
    hipError_t e = hipHostMalloc((void**)&ctx->hhost, 1024 * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) return set_hip_err(ctx, e, "hipHostMalloc");
    CPR_TRY(hipHostGetDevicePointer((void**)&ctx->hhost_dev, ctx->hhost, 0));
  }
  hipStream_t s = ctx->stream;
  launch_nat_to_cs(ctx->lay, 1, poro, ctx->poro, s);
  launch_transmissibility(ctx->lay, *g, perm3, ctx->tp, s);
  launch_lnk(ctx->lay, perm3, ctx->lnk, s);
  if ((rc = launch_check(ctx, "cpr_create kernels")) != CPR_OK) return rc;
  // mean porosity (compensated sum) for the row scaling
  {
    std::vector<double> h(N);
    CPR_TRY(hipMemcpyAsync(h.data(), poro, N * sizeof(double), hipMemcpyDeviceToHost, s));
    CPR_TRY(hipStreamSynchronize(s));
    double sum = 0.0, comp = 0.0;
    for (size_t q = 0; q < N; ++q) {
      double yv = h[q] - comp;
      double t = sum + yv;
      comp = (t - sum) - yv;
      sum = t;
    }
    ctx->phibar = sum / (double)N;
    if (!(ctx->phibar > 0.0)) return set_err(ctx, CPR_EINVAL, "mean porosity must be > 0");
  }
  ctx->cell_vol = g->dx * g->dy * g->dz;
  if (f->model == CPR_MODEL_SINGLE_PHASE) {
    ctx->rho_scale[0] = f->rho_w_ref;
  } else if (f->model == CPR_MODEL_OIL_WATER) {
    ctx->rho_scale[0] = f->rho_o_ref;
    ctx->rho_scale[1] = f->rho_w_ref;
  } else {
    ctx->rho_scale[0] = f->rho_o_sc / host_pvt(fl, 2, f->p_ref);
    ctx->rho_scale[1] = f->rho_w_ref;
    ctx->rho_scale[2] = f->rho_g_sc / host_pvt(fl, 4, f->p_ref);
  }
  // perforations (each well's contiguous, in the order given)
  for (int q = 0; q < nwells; ++q) {
    const cpr_well_t& w = wells[q];
    const bool rate = w.control == CPR_CONTROL_RATE;
    if (rate) {
      RateWell r;
      r.p0 = (int)ctx->perfs.size();
      r.p1 = r.p0 + (w.k1 - w.k0 + 1);
      // single phase: the water row of either kind; otherwise water (injector) or oil (producer)
      const bool water = w.kind == CPR_WELL_INJECTOR || f->model == CPR_MODEL_SINGLE_PHASE;
      r.comp = f->model == CPR_MODEL_SINGLE_PHASE ? 0 : (water ? 1 : 0);
      const double rho_s = water ? f->rho_w_ref
                                 : (f->model == CPR_MODEL_BLACK_OIL ? f->rho_o_sc : f->rho_o_ref);
      const double mass = w.rate * rho_s / 86400.0;
      r.target = w.kind == CPR_WELL_INJECTOR ? mass : -mass;
      ctx->rwells.push_back(r);
    }
    if (w.i < 0 || w.i >= g->nx || w.j < 0 || w.j >= g->ny || w.k0 < 0 || w.k1 >= g->nz || w.k0 > w.k1)
      return set_err(ctx, CPR_EINVAL, "well perforation outside the grid");
    if (w.kind != CPR_WELL_INJECTOR && w.kind != CPR_WELL_PRODUCER)
      return set_err(ctx, CPR_EINVAL, "unknown well kind");
    if (!(w.rw > 0)) return set_err(ctx, CPR_EINVAL, "well radius must be > 0");
    for (int k = w.k0; k <= w.k1; ++k) {
      size_t nat = (size_t)w.i + (size_t)g->nx * ((size_t)w.j + (size_t)g->ny * k);
      double kxy[2];
      CPR_TRY(hipMemcpy(&kxy[0], perm3 + nat, sizeof(double), hipMemcpyDeviceToHost));
      CPR_TRY(hipMemcpy(&kxy[1], perm3 + N + nat, sizeof(double), hipMemcpyDeviceToHost));
      Perf p;
      p.cell = lay_index(ctx->lay, w.i, w.j, k);
      p.kind = w.kind;
      p.rw = rate ? (int)ctx->rwells.size() - 1 : -1;
      p.wi = peaceman(kxy[0], kxy[1], g->dx, g->dy, g->dz, w.rw, w.skin);
      p.bhp = w.bhp;
      double depth = g->top + (k + 0.5) * g->dz;
      p.dzh = g->top - depth;
      for (const Perf& o : ctx->perfs)
        if (o.cell == p.cell) return set_err(ctx, CPR_EINVAL, "two perforations in one cell");
      ctx->perfs.push_back(p);
    }
  }
  if (!ctx->perfs.empty()) {
    if ((rc = dalloc(ctx, &ctx->perfs_d, ctx->perfs.size())) != CPR_OK) return rc;
    CPR_TRY(hipMemcpyAsync(ctx->perfs_d, ctx->perfs.data(), ctx->perfs.size() * sizeof(Perf),
                           hipMemcpyHostToDevice, s));
  }
  if (ctx->nrate) {
    if ((rc = dalloc(ctx, &ctx->rwells_d, ctx->rwells.size())) != CPR_OK) return rc;
    if ((rc = dalloc(ctx, &ctx->bord, 6 * ctx->perfs.size())) != CPR_OK) return rc;
    if ((rc = dalloc(ctx, &ctx->pq, 2 * ctx->perfs.size())) != CPR_OK) return rc;
    if ((rc = dalloc(ctx, &ctx->bord_d, (size_t)ctx->nrate)) != CPR_OK) return rc;
    CPR_TRY(hipMemcpyAsync(ctx->rwells_d, ctx->rwells.data(), ctx->rwells.size() * sizeof(RateWell),
                           hipMemcpyHostToDevice, s));
    CPR_TRY(hipMemsetAsync(ctx->bord, 0, 6 * ctx->perfs.size() * sizeof(double), s));
  }
  CPR_TRY(hipStreamSynchronize(s));
  cpr_default_options(&ctx->opt);
  return CPR_OK;
}

int ensure_krylov(cpr_ctx* ctx, int m) {
  if (m <= ctx->mcap) return CPR_OK;
  dev_free(ctx->mem, ctx->V);
  dev_free(ctx->mem, ctx->Z);
  ctx->V = ctx->Z = nullptr;
  ctx->mcap = 0;
  size_t len = (size_t)vec_len(ctx);
  int rc;
  if ((rc = dalloc(ctx, &ctx->V, (size_t)(m + 1) * len)) != CPR_OK) return rc;
  if ((rc = dalloc(ctx, &ctx->Z, (size_t)m * len)) != CPR_OK) return rc;
  ctx->mcap = m;
  return CPR_OK;
}

// Buffers of the ABF decoupling and of the F-P-F composition, allocated on
// first use.
int ensure_variants(cpr_ctx* ctx, const cpr_options_t& o) {
  size_t N = ctx->lay.n;
  int b = ctx->b, rc;
  if (o.decoupling == CPR_DECOUPLE_ABF && !ctx->Jt) {
    if ((rc = dalloc(ctx, &ctx->Wabf, (size_t)b * b * N)) != CPR_OK) return rc;
    if ((rc = dalloc(ctx, &ctx->Jt, tiled_len(N, 7 * b * b))) != CPR_OK) return rc;
  }
  if (o.decoupling == CPR_DECOUPLE_ABF || o.composition == CPR_COMPOSE_FPF) {
    if (!ctx->Rt && (rc = dalloc(ctx, &ctx->Rt, (size_t)b * N)) != CPR_OK) return rc;
    if (!ctx->Z1 && (rc = dalloc(ctx, &ctx->Z1, (size_t)b * N)) != CPR_OK) return rc;
    if (o.precision == CPR_PREC_MIXED) {
      if (!ctx->Rtf && (rc = dalloc(ctx, &ctx->Rtf, (size_t)b * N)) != CPR_OK) return rc;
      if (!ctx->Z1f && (rc = dalloc(ctx, &ctx->Z1f, (size_t)b * N)) != CPR_OK) return rc;
    }
  }
  return CPR_OK;
}

int ensure_mixed(cpr_ctx* ctx) {
  if (ctx->Jf) return CPR_OK;
  size_t N = ctx->lay.n;
  int b = ctx->b, rc;
  if ((rc = dalloc(ctx, &ctx->Jf, tiled_len(N, 7 * b * b))) != CPR_OK) return rc;
  if ((rc = dalloc(ctx, &ctx->Dinvf, tiled_len(N, b * b))) != CPR_OK) return rc;
  if ((rc = dalloc(ctx, &ctx->Yf, (size_t)b * N)) != CPR_OK) return rc;
  return CPR_OK;
}

// The level the learned stage acts on with nn_level = CPR_NN_LEVEL_AUTO,
// among the coarse levels it can run on (dimensions divisible by 8, exactly
// 2^-l of the grid, colour-split, above the single-workgroup levels): the
// coarsest one of at least 2^19 cells, else the coarsest one of at least
// 2^16 cells, else the fine level.
int auto_nn_level(const cpr_ctx* ctx) {
  const Lay& F = ctx->lay;
  const int fuse = vcycle_fused_level(ctx);
  int big = 0, mid = 0;
  for (int l = 1; l < (int)ctx->levels.size() && l < fuse; ++l) {
    const Lay& L = ctx->levels[l].lay;
    if ((long)L.n < (1L << 16)) break;
    if (L.cs && L.nxr == L.nx && L.nx % 8 == 0 && L.ny % 8 == 0 && L.nz % 8 == 0 && F.nx == L.nx << l &&
        F.ny == L.ny << l && F.nz == L.nz << l) {
      if ((long)L.n >= (1L << 19)) big = l;
      mid = l;
    }
  }
  return big ? big : mid;
}

}  // namespace

int ensure_krylov_capacity(cpr_ctx* ctx, int m) { return ensure_krylov(ctx, m); }

// Validate the options, allocate what they need and build the preconditioner.
int setup_with_options(cpr_ctx* ctx, const cpr_options_t& opt) {
  if (opt.restart < 1 || opt.restart > 64) return set_err(ctx, CPR_EINVAL, "restart must be 1..64");
  if (opt.max_iter < 0) return set_err(ctx, CPR_EINVAL, "max_iter must be >= 0");
  if (!(opt.rtol >= 0) || !std::isfinite(opt.rtol)) return set_err(ctx, CPR_EINVAL, "rtol must be >= 0");
  if (opt.mg_coarsest < 1 || opt.mg_coarsest > 4096)
    return set_err(ctx, CPR_EINVAL, "mg_coarsest must be 1..4096");
  if (opt.mg_pre < 1 || opt.mg_pre > 8 || opt.mg_post < 1 || opt.mg_post > 8)
    return set_err(ctx, CPR_EINVAL, "mg_pre and mg_post must be 1..8");
  if (!std::isfinite(opt.mg_alpha)) return set_err(ctx, CPR_EINVAL, "mg_alpha must be finite");
  if (std::isnan(opt.stall_ratio)) return set_err(ctx, CPR_EINVAL, "stall_ratio must not be NaN");
  if (opt.precision != CPR_PREC_FP64 && opt.precision != CPR_PREC_MIXED)
    return set_err(ctx, CPR_EINVAL, "unknown precision");
  if (opt.decoupling != CPR_DECOUPLE_QIMPES && opt.decoupling != CPR_DECOUPLE_ABF)
    return set_err(ctx, CPR_EINVAL, "unknown decoupling");
  if (opt.composition != CPR_COMPOSE_PF && opt.composition != CPR_COMPOSE_FPF)
    return set_err(ctx, CPR_EINVAL, "unknown composition");
  if (opt.orth != CPR_ORTH_DCGS2 && opt.orth != CPR_ORTH_CGS2)
    return set_err(ctx, CPR_EINVAL, "unknown orthogonalisation");
  if (opt.nn_level < CPR_NN_LEVEL_AUTO) return set_err(ctx, CPR_EINVAL, "nn_level must be >= -1");
  if (opt.ilu_order != CPR_ILU_RED_BLACK && opt.ilu_order != CPR_ILU_TILES)
    return set_err(ctx, CPR_EINVAL, "unknown ILU order");
  if (opt.ilu_order == CPR_ILU_TILES && opt.composition != CPR_COMPOSE_PF)
    return set_err(ctx, CPR_EINVAL, "the tiled ILU order supports the P-then-F composition only");
  if (opt.learned && !ctx->nn) return set_err(ctx, CPR_EINVAL, "no pressure-correction network attached");
  ctx->opt = opt;
  ctx->setup_done = 0;
  int rc;
  if ((rc = ensure_krylov(ctx, opt.restart)) != CPR_OK) return rc;
  if (opt.precision == CPR_PREC_MIXED && (rc = ensure_mixed(ctx)) != CPR_OK) return rc;
  if ((rc = ensure_variants(ctx, opt)) != CPR_OK) return rc;
  if ((rc = setup_cpr(ctx)) != CPR_OK) return rc;
  if (ctx->opt.nn_level == CPR_NN_LEVEL_AUTO) ctx->opt.nn_level = auto_nn_level(ctx);
  if (opt.learned) {
    if ((rc = learned_setup(ctx, true)) != CPR_OK) {
      ctx->setup_done = 0;
      return rc;
    }
  }
  return CPR_OK;
}

#define GUARD_BEGIN try {
#define GUARD_END                                                        \
  }                                                                      \
  catch (const std::bad_alloc&) {                                        \
    return set_err(ctx, CPR_ENOMEM, "host allocation failed");           \
  }                                                                      \
  catch (...) {                                                          \
    return set_err(ctx, CPR_EINVAL, "internal error");                   \
  }

extern "C" {

void cpr_default_options(cpr_options_t* o) {
  if (!o) return;
  o->precision = CPR_PREC_FP64;
  o->learned = 0;
  o->restart = 30;
  o->max_iter = 300;
  o->rtol = 1e-6;
  o->mg_coarsest = 512;
  o->mg_alpha = 1.0;
  o->stall_ratio = 0.5;
  o->decoupling = CPR_DECOUPLE_QIMPES;
  o->composition = CPR_COMPOSE_PF;
  o->x0 = 0;
  o->mg_pre = 1;
  o->mg_post = 1;
  o->orth = CPR_ORTH_DCGS2;
  o->nn_level = CPR_NN_LEVEL_AUTO;
  o->ilu_order = CPR_ILU_RED_BLACK;
}

int cpr_create(const cpr_grid_t* g, const cpr_fluid_t* f, const double* perm3, const double* poro,
               const cpr_well_t* wells, int nwells, void* stream, cpr_ctx_t** out) {
  if (!out) return CPR_EINVAL;
  *out = nullptr;
  cpr_ctx* ctx = nullptr;
  try {
    ctx = new cpr_ctx();
  } catch (...) {
    return CPR_ENOMEM;
  }
  ctx->mem = current_allocator();
  int rc;
  try {
    rc = create_impl(g, f, perm3, poro, wells, nwells, stream, ctx);
  } catch (...) {
    rc = CPR_ENOMEM;
  }
  *out = ctx;   // returned even on failure so cpr_last_error can explain; caller destroys
  return rc;
}

void cpr_destroy(cpr_ctx_t* ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  free_all(ctx);
  delete ctx;
}

const char* cpr_last_error(const cpr_ctx_t* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int cpr_block_size(const cpr_ctx_t* ctx) { return ctx ? ctx->b : 0; }

long long cpr_num_cells(const cpr_ctx_t* ctx) { return ctx ? (long long)ctx->lay.n : 0; }

long long cpr_num_unknowns(const cpr_ctx_t* ctx) { return ctx ? (long long)vec_len(ctx) : 0; }

int assemble_jacobian(cpr_ctx_t* ctx, const double* x_old, const double* x, double dt_days,
                      double* rhs_out) {
  if (check_ctx(ctx)) return CPR_EINVAL;
  GUARD_BEGIN
  if (!x_old || !x || !rhs_out) return set_err(ctx, CPR_EINVAL, "null argument");
  if (!(dt_days > 0) || !std::isfinite(dt_days)) return set_err(ctx, CPR_EINVAL, "dt must be > 0");
  TraceRange tr("assemble_jacobian");
  ph_outer_begin(ctx, PH_ASSEMBLE);
  CPR_TRY(vec_nat_to_cs(ctx, x_old, ctx->vin2));
  CPR_TRY(vec_nat_to_cs(ctx, x, ctx->vin));
  launch_assemble(ctx, ctx->vin2, ctx->vin, dt_days, ctx->vout);
  CPR_TRY(vec_cs_to_nat(ctx, ctx->vout, rhs_out));
  ph_outer_end(ctx, PH_ASSEMBLE);
  ctx->assembled = 1;
  ctx->setup_done = 0;
  return launch_check(ctx, "assemble_jacobian");
  GUARD_END
}

int cpr_import_jacobian(cpr_ctx_t* ctx, const double* blocks) {
  if (check_ctx(ctx)) return CPR_EINVAL;
  if (!blocks) return set_err(ctx, CPR_EINVAL, "null argument");
  launch_nat_to_tiled(ctx->lay, 7 * ctx->b * ctx->b, blocks, ctx->J, ctx->stream);
  ctx->setup_done = 0;
  return launch_check(ctx, "cpr_import_jacobian");
}

int cpr_export_jacobian(cpr_ctx_t* ctx, double* blocks) {
  if (check_ctx(ctx)) return CPR_EINVAL;
  if (!blocks) return set_err(ctx, CPR_EINVAL, "null argument");
  launch_tiled_to_nat(ctx->lay, 7 * ctx->b * ctx->b, ctx->J, blocks, ctx->stream);
  return launch_check(ctx, "cpr_export_jacobian");
}

int cpr_setup(cpr_ctx_t* ctx, const cpr_options_t* o) {
  if (check_ctx(ctx)) return CPR_EINVAL;
  GUARD_BEGIN
  cpr_options_t opt;
  if (o) opt = *o; else cpr_default_options(&opt);
  TraceRange tr("cpr_setup");
  ph_outer_begin(ctx, PH_SETUP);
  int rc = setup_with_options(ctx, opt);
  ph_outer_end(ctx, PH_SETUP);
  return rc;
  GUARD_END
}

int cpr_gmres_solve(cpr_ctx_t* ctx, const double* rhs, double* dx, cpr_stats_t* st) {
  if (check_ctx(ctx)) return CPR_EINVAL;
  GUARD_BEGIN
  if (!rhs || !dx) return set_err(ctx, CPR_EINVAL, "null argument");
  if (!ctx->setup_done) return set_err(ctx, CPR_EINVAL, "cpr_setup has not been called for this Jacobian");
  TraceRange tr("cpr_gmres_solve");
  hipStream_t s = ctx->stream;
  CPR_TRY(vec_nat_to_cs(ctx, rhs, ctx->rs));
  if (ctx->opt.x0) CPR_TRY(vec_nat_to_cs(ctx, dx, ctx->xs));
  if (ctx->opt.learned) CPR_TRY(hipMemsetAsync(ctx->nncount, 0, 2 * sizeof(int), s));
  int rc = fgmres_solve(ctx, st);
  if (rc < 0) return rc;
  CPR_TRY(vec_cs_to_nat(ctx, ctx->xs, dx));
  int rc2 = launch_check(ctx, "cpr_gmres_solve");
  if (rc2 != CPR_OK) return rc2;
  if (ctx->opt.learned && st) {
    int cnt[2] = {0, 0};
    CPR_TRY(hipMemcpyAsync(cnt, ctx->nncount, sizeof(cnt), hipMemcpyDeviceToHost, s));
    CPR_TRY(hipStreamSynchronize(s));
    st->nn_accepted = cnt[0];
    st->nn_rejected = cnt[1];
  }
  return rc;
  GUARD_END
}

void cpr_default_newton_options(cpr_newton_options_t* o) {
  if (!o) return;
  o->forcing = CPR_FORCING_EW1;
  o->krylov = CPR_KRYLOV_FGMRES;
  o->max_newton = 20;
  o->max_cuts = 6;
  o->newton_tol = 1e-3;
  o->theta0 = 0.1;
  o->theta_min = 1e-6;
  o->theta_max = 0.5;
  o->gamma = 0.9;
  o->beta = 2.0;
}

int cpr_time_step(cpr_ctx_t* ctx, const double* x_old, double* x, double dt_days, const cpr_options_t* lin,
                  const cpr_newton_options_t* nopt, cpr_newton_stats_t* st) {
  if (check_ctx(ctx)) return CPR_EINVAL;
  GUARD_BEGIN
  if (!x_old || !x) return set_err(ctx, CPR_EINVAL, "null argument");
  if (!(dt_days > 0) || !std::isfinite(dt_days)) return set_err(ctx, CPR_EINVAL, "dt must be > 0");
  cpr_options_t lo;
  if (lin) lo = *lin; else cpr_default_options(&lo);
  cpr_newton_options_t no;
  if (nopt) no = *nopt; else cpr_default_newton_options(&no);
  if (no.forcing < CPR_FORCING_FIXED || no.forcing > CPR_FORCING_EW3)
    return set_err(ctx, CPR_EINVAL, "unknown forcing");
  if (no.krylov != CPR_KRYLOV_FGMRES && no.krylov != CPR_KRYLOV_BICGSTAB)
    return set_err(ctx, CPR_EINVAL, "unknown Krylov method");
  if (no.max_newton < 0 || no.max_cuts < 0) return set_err(ctx, CPR_EINVAL, "negative iteration limit");
  if (!(no.newton_tol > 0) || !(no.theta_min > 0) || !(no.theta_max >= no.theta_min) || !(no.theta0 > 0) ||
      !std::isfinite(no.theta_max) || !std::isfinite(no.gamma) || !std::isfinite(no.beta))
    return set_err(ctx, CPR_EINVAL, "bad Newton tolerances");
  TraceRange tr("cpr_time_step");
  CPR_TRY(vec_nat_to_cs(ctx, x_old, ctx->vin2));
  int rc = time_step(ctx, ctx->vin2, ctx->vin, dt_days, lo, no, st);
  if (rc < 0) return rc;
  CPR_TRY(vec_cs_to_nat(ctx, ctx->vin, x));
  int rc2 = launch_check(ctx, "cpr_time_step");
  return rc2 != CPR_OK ? rc2 : rc;
  GUARD_END
}

int cpr_simulate(cpr_ctx_t* ctx, const double* x0, double* x, double t_end_days, double dt0_days,
                 double dt_max_days, double growth, const cpr_options_t* lin, const cpr_newton_options_t* nopt,
                 cpr_sim_stats_t* st) {
  if (check_ctx(ctx)) return CPR_EINVAL;
  GUARD_BEGIN
  if (!x0 || !x) return set_err(ctx, CPR_EINVAL, "null argument");
  if (!(t_end_days > 0) || !(dt0_days > 0) || !(dt_max_days > 0) || !(growth >= 1.0) ||
      !std::isfinite(t_end_days) || !std::isfinite(dt_max_days) || !std::isfinite(growth))
    return set_err(ctx, CPR_EINVAL, "bad time-stepping parameters");
  cpr_options_t lo;
  if (lin) lo = *lin; else cpr_default_options(&lo);
  TraceRange tr("cpr_simulate");
  cpr_newton_options_t no;
  if (nopt) no = *nopt; else cpr_default_newton_options(&no);
  hipStream_t s = ctx->stream;
  const long len = vec_len(ctx);
  double* xa = ctx->vin2;   // state at the start of the step (colour-split)
  CPR_TRY(vec_nat_to_cs(ctx, x0, xa));
  cpr_sim_stats_t S = {};
  double t = 0.0, dt = dt0_days;
  int rc = CPR_OK;
  using clock = std::chrono::steady_clock;
  const auto t_call = clock::now();
  while (t < t_end_days) {
    double h = std::fmin(dt, t_end_days - t);
    cpr_newton_stats_t ns = {};
    const auto t_step = clock::now();
    rc = time_step(ctx, xa, ctx->vin, h, lo, no, &ns);
    if (rc < 0) break;
    S.cuts += ns.cuts;
    S.total_newton += ns.total_newton;
    S.total_linear += ns.total_linear;
    if (rc != CPR_OK) break;
    CPR_TRY(hipMemcpyAsync(xa, ctx->vin, len * sizeof(double), hipMemcpyDeviceToDevice, s));
    CPR_TRY(hipStreamSynchronize(s));
    if (S.steps < CPR_SIM_HIST) {
      S.dts[S.steps] = ns.dt_taken;
      S.step_newton[S.steps] = ns.total_newton;
      S.step_linear[S.steps] = ns.total_linear;
      S.step_cuts[S.steps] = ns.cuts;
      S.step_seconds[S.steps] = std::chrono::duration<double>(clock::now() - t_step).count();
    }
    S.steps += 1;
    t += ns.dt_taken;
    dt = ns.cuts == 0 ? std::fmin(growth * ns.dt_taken, dt_max_days) : ns.dt_taken;
  }
  S.t_reached = t;
  S.completed = (rc == CPR_OK && t >= t_end_days) ? 1 : 0;
  if (rc >= 0) CPR_TRY(vec_cs_to_nat(ctx, xa, x));
  if (rc >= 0) CPR_TRY(hipStreamSynchronize(s));
  S.seconds = std::chrono::duration<double>(clock::now() - t_call).count();
  if (st) *st = S;
  if (rc < 0) return rc;
  int rc2 = launch_check(ctx, "cpr_simulate");
  return rc2 != CPR_OK ? rc2 : rc;
  GUARD_END
}

int cpr_bicgstab_solve(cpr_ctx_t* ctx, const double* rhs, double* dx, cpr_stats_t* st) {
  if (check_ctx(ctx)) return CPR_EINVAL;
  GUARD_BEGIN
  if (!rhs || !dx) return set_err(ctx, CPR_EINVAL, "null argument");
  if (!ctx->setup_done) return set_err(ctx, CPR_EINVAL, "cpr_setup has not been called for this Jacobian");
  int rc;
  if ((rc = ensure_krylov(ctx, ctx->opt.restart > 8 ? ctx->opt.restart : 8)) != CPR_OK) return rc;
  TraceRange tr("cpr_bicgstab_solve");
  hipStream_t s = ctx->stream;
  CPR_TRY(vec_nat_to_cs(ctx, rhs, ctx->rs));
  if (ctx->opt.learned) CPR_TRY(hipMemsetAsync(ctx->nncount, 0, 2 * sizeof(int), s));
  rc = bicgstab_solve(ctx, st);
  if (rc < 0) return rc;
  CPR_TRY(vec_cs_to_nat(ctx, ctx->xs, dx));
  int rc2 = launch_check(ctx, "cpr_bicgstab_solve");
  if (rc2 != CPR_OK) return rc2;
  if (ctx->opt.learned && st) {
    int cnt[2] = {0, 0};
    CPR_TRY(hipMemcpyAsync(cnt, ctx->nncount, sizeof(cnt), hipMemcpyDeviceToHost, s));
    CPR_TRY(hipStreamSynchronize(s));
    st->nn_accepted = cnt[0];
    st->nn_rejected = cnt[1];
  }
  return rc;
  GUARD_END
}

int cpr_nn_attach(cpr_ctx_t* ctx, const float* theta) {
  if (check_ctx(ctx)) return CPR_EINVAL;
  GUARD_BEGIN
  if (!theta) {
    if (ctx->nn) cpr_nn_destroy(ctx->nn);
    ctx->nn = nullptr;
    if (ctx->nn_lv) cpr_nn_destroy(ctx->nn_lv);
    ctx->nn_lv = nullptr;
    ctx->theta.clear();
    if (ctx->opt.learned) ctx->setup_done = 0;
    return CPR_OK;
  }
  const cpr_grid_t& g = ctx->grid;
  if (g.nx % 8 || g.ny % 8 || g.nz % 8)
    return set_err(ctx, CPR_EINVAL, "the learned stage needs grid dimensions divisible by 8");
  if (!ctx->nn) {
    cpr_nn_t* nn = nullptr;
    int rc = cpr_nn_create(g.nx, g.ny, g.nz, 1, ctx->stream, &nn);
    if (rc != CPR_OK) {
      std::string m = nn ? cpr_nn_last_error(nn) : "network allocation failed";
      cpr_nn_destroy(nn);
      return set_err(ctx, rc, m);
    }
    ctx->nn = nn;
  }
  int rc = cpr_nn_set_params(ctx->nn, theta);
  if (rc != CPR_OK) return set_err(ctx, rc, cpr_nn_last_error(ctx->nn));
  ctx->theta.assign(theta, theta + cpr_nn_num_params());
  if (ctx->nn_lv && (rc = cpr_nn_set_params(ctx->nn_lv, theta)) != CPR_OK)
    return set_err(ctx, rc, cpr_nn_last_error(ctx->nn_lv));
  return CPR_OK;
  GUARD_END
}

int cpr_pressure_stage(cpr_ctx_t* ctx, const double* v, double* rprime, double* dp_mg) {
  if (check_ctx(ctx)) return CPR_EINVAL;
  if (!v || !rprime) return set_err(ctx, CPR_EINVAL, "null argument");
  if (!ctx->setup_done) return set_err(ctx, CPR_EINVAL, "cpr_setup has not been called for this Jacobian");
  if (ctx->opt.decoupling != CPR_DECOUPLE_QIMPES)
    return set_err(ctx, CPR_EINVAL, "the pressure stage export needs quasi-IMPES decoupling");
  hipStream_t s = ctx->stream;
  const int lv = ctx->opt.nn_level;
  if (lv >= (int)ctx->levels.size()) return set_err(ctx, CPR_EINVAL, "nn_level beyond the hierarchy");
  const Lay& L = ctx->levels[lv].lay;
  if (lv > 0 && (!L.cs || L.nxr != L.nx))
    return set_err(ctx, CPR_EINVAL, "nn_level: the level must be stored colour-split without a ghost column");
  launch_nat_to_cs(ctx->lay, ctx->b, v, ctx->vin, s);
  precond_pressure_stage(ctx, ctx->vin);
  learned_rprime(ctx);
  launch_cs_to_nat(L, 1, ctx->rprime, rprime, s);
  if (dp_mg) launch_cs_to_nat(L, 1, ctx->levels[lv].x, dp_mg, s);
  return launch_check(ctx, "cpr_pressure_stage");
}

int cpr_nn_features(cpr_ctx_t* ctx, const double* rprime, float* feat, double* scale) {
  if (check_ctx(ctx)) return CPR_EINVAL;
  GUARD_BEGIN
  if (!rprime || !feat) return set_err(ctx, CPR_EINVAL, "null argument");
  if (!ctx->setup_done) return set_err(ctx, CPR_EINVAL, "cpr_setup has not been called for this Jacobian");
  int rc = learned_setup(ctx, false);
  if (rc != CPR_OK) return rc;
  hipStream_t s = ctx->stream;
  const Lay& L = ctx->levels[ctx->opt.nn_level].lay;
  launch_nat_to_cs(L, 1, rprime, ctx->rprime, s);
  learned_features_from_rprime(ctx);
  CPR_TRY(hipMemcpyAsync(feat, ctx->feat, 3 * (size_t)L.n * sizeof(float), hipMemcpyDeviceToDevice, s));
  double sc[8];
  CPR_TRY(hipMemcpyAsync(sc, ctx->nnscal, sizeof(sc), hipMemcpyDeviceToHost, s));
  CPR_TRY(hipStreamSynchronize(s));
  if (scale) *scale = sc[4];
  return launch_check(ctx, "cpr_nn_features");
  GUARD_END
}

int cpr_export_krylov(cpr_ctx_t* ctx, int j, double* v) {
  if (check_ctx(ctx)) return CPR_EINVAL;
  if (!v || j < 0 || j > ctx->mcap || !ctx->V) return set_err(ctx, CPR_EINVAL, "bad basis index");
  CPR_TRY(vec_cs_to_nat(ctx, ctx->V + (size_t)j * vec_len(ctx), v));
  return launch_check(ctx, "cpr_export_krylov");
}

int cpr_newton_update(cpr_ctx_t* ctx, double* x, const double* dx) {
  if (check_ctx(ctx)) return CPR_EINVAL;
  if (!x || !dx) return set_err(ctx, CPR_EINVAL, "null argument");
  launch_newton_update(ctx->b, ctx->lay.n, ctx->nrate, pb_floor(ctx->fl), x, dx, ctx->stream);
  return launch_check(ctx, "cpr_newton_update");
}

int cpr_spmv(cpr_ctx_t* ctx, const double* x, double* y) {
  if (check_ctx(ctx)) return CPR_EINVAL;
  if (!x || !y) return set_err(ctx, CPR_EINVAL, "null argument");
  CPR_TRY(vec_nat_to_cs(ctx, x, ctx->vin));
  system_spmv(ctx, ctx->vin, ctx->vout, nullptr);
  CPR_TRY(vec_cs_to_nat(ctx, ctx->vout, y));
  return launch_check(ctx, "cpr_spmv");
}

int cpr_precond_apply(cpr_ctx_t* ctx, const double* v, double* z) {
  if (check_ctx(ctx)) return CPR_EINVAL;
  if (!v || !z) return set_err(ctx, CPR_EINVAL, "null argument");
  if (!ctx->setup_done) return set_err(ctx, CPR_EINVAL, "cpr_setup has not been called for this Jacobian");
  CPR_TRY(vec_nat_to_cs(ctx, v, ctx->vin));
  precond_apply(ctx, ctx->vin, ctx->vin, nullptr, ctx->vout);
  CPR_TRY(vec_cs_to_nat(ctx, ctx->vout, z));
  return launch_check(ctx, "cpr_precond_apply");
}

int cpr_export_qimpes(cpr_ctx_t* ctx, double* w) {
  if (check_ctx(ctx)) return CPR_EINVAL;
  if (!w || !ctx->setup_done) return set_err(ctx, CPR_EINVAL, "null argument or no setup");
  if (ctx->opt.decoupling != CPR_DECOUPLE_QIMPES) return set_err(ctx, CPR_EINVAL, "not quasi-IMPES decoupling");
  launch_cs_to_nat(ctx->lay, ctx->b, ctx->w, w, ctx->stream);
  return launch_check(ctx, "cpr_export_qimpes");
}

int cpr_mg_level_shape(const cpr_ctx_t* ctx, int level, int* nx, int* ny, int* nz) {
  if (!ctx || level < 0 || level >= (int)ctx->levels.size() || !nx || !ny || !nz) return CPR_EINVAL;
  const Lay& L = ctx->levels[level].lay;
  *nx = L.nxr; *ny = L.ny; *nz = L.nz;
  return CPR_OK;
}

int cpr_nn_level(const cpr_ctx_t* ctx, int* level) {
  if (!ctx || !level || !ctx->setup_done) return CPR_EINVAL;
  *level = ctx->opt.nn_level;
  return CPR_OK;
}

int cpr_export_mg_level(cpr_ctx_t* ctx, int level, double* a7) {
  if (check_ctx(ctx)) return CPR_EINVAL;
  if (!a7 || !ctx->setup_done || level < 0 || level >= (int)ctx->levels.size())
    return set_err(ctx, CPR_EINVAL, "bad level or no setup");
  const MGLevel& L = ctx->levels[level];
  launch_cs_to_nat(L.lay, 7, L.A, a7, ctx->stream);
  return launch_check(ctx, "cpr_export_mg_level");
}

int cpr_export_ilu(cpr_ctx_t* ctx, double* dinv) {
  if (check_ctx(ctx)) return CPR_EINVAL;
  if (!dinv || !ctx->setup_done) return set_err(ctx, CPR_EINVAL, "null argument or no setup");
  launch_tiled_to_nat(ctx->lay, ctx->b * ctx->b, ctx->Dinv, dinv, ctx->stream);
  return launch_check(ctx, "cpr_export_ilu");
}

int cpr_set_timing(cpr_ctx_t* ctx, int on) {
  if (check_ctx(ctx)) return CPR_EINVAL;
  GUARD_BEGIN
  return phase_timing_enable(ctx, on != 0);
  GUARD_END
}

int cpr_profile_kernel(cpr_ctx_t* ctx, int kclass) {
  if (check_ctx(ctx)) return CPR_EINVAL;
  if (kclass < -1 || kclass > CPR_KCLASS_ASSEMBLE) return set_err(ctx, CPR_EINVAL, "unknown kernel class");
  GUARD_BEGIN
  if (kclass >= 0 && ctx->ev.empty()) {
    ctx->ev.resize(2 * 8192);
    for (auto& e : ctx->ev) CPR_TRY(hipEventCreate(&e));
  }
  ctx->prof_class = kclass;
  ctx->ev_used = 0;
  return CPR_OK;
  GUARD_END
}

int cpr_profile_read(cpr_ctx_t* ctx, int* launches, double* total_ms) {
  if (check_ctx(ctx)) return CPR_EINVAL;
  if (!launches || !total_ms) return set_err(ctx, CPR_EINVAL, "null argument");
  CPR_TRY(hipStreamSynchronize(ctx->stream));
  double tot = 0.0;
  for (int q = 0; q < ctx->ev_used; ++q) {
    float ms = 0.f;
    CPR_TRY(hipEventElapsedTime(&ms, ctx->ev[2 * q], ctx->ev[2 * q + 1]));
    tot += ms;
  }
  *launches = ctx->ev_used;
  *total_ms = tot;
  ctx->ev_used = 0;
  return CPR_OK;
}

}  // extern "C"
