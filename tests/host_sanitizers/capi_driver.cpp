// Exercises every entry point of the C ABI, its error paths included, on
// small oil-water and black-oil grids.  Built with the host code of the
// library and of this driver under AddressSanitizer and
// UndefinedBehaviorSanitizer (the GPU code is built as usual), it checks
// the host side -- option validation, hierarchy construction, the Krylov
// bookkeeping, phase timers, the network's host logic, the caller
// allocator -- for memory errors and undefined behaviour.  Exit status 0
// when every call returned what it should.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "cprmi.h"

#define CHECK(cond, what)                                                          \
  do {                                                                             \
    if (!(cond)) {                                                                 \
      std::fprintf(stderr, "FAIL line %d: %s (%s)\n", __LINE__, what, #cond);     \
      return 1;                                                                    \
    }                                                                              \
  } while (0)
#define HIPOK(expr) CHECK((expr) == hipSuccess, #expr)

namespace {

struct DevBuf {
  void* p = nullptr;
  explicit DevBuf(size_t bytes) { (void)hipMalloc(&p, bytes); }
  ~DevBuf() { (void)hipFree(p); }
  double* d() const { return static_cast<double*>(p); }
  float* f() const { return static_cast<float*>(p); }
};

int put(DevBuf& b, const std::vector<double>& h) {
  return hipMemcpy(b.p, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess ? 0 : 1;
}

std::vector<double> get(const DevBuf& b, size_t n) {
  std::vector<double> h(n);
  (void)hipMemcpy(h.data(), b.p, n * sizeof(double), hipMemcpyDeviceToHost);
  return h;
}

const double kPvt[6][7] = {{50, 100, 150, 200, 250, 300, 350},
                           {18, 38, 59, 80, 101, 122, 143},
                           {1.10, 1.15, 1.20, 1.25, 1.30, 1.35, 1.40},
                           {1.60, 1.40, 1.25, 1.10, 1.00, 0.92, 0.85},
                           {0.0240, 0.0120, 0.0081, 0.0061, 0.0049, 0.0041, 0.0036},
                           {0.013, 0.015, 0.017, 0.019, 0.021, 0.023, 0.025}};

long g_live = 0;   // blocks handed out by the counting allocator
void* count_alloc(size_t bytes, void*) {
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  ++g_live;
  return p;
}
void count_free(void* p, void*) {
  if (p) {
    --g_live;
    (void)hipFree(p);
  }
}

// One model on an nx x ny x nz grid: create, assemble, every solver form,
// the verification and measurement entry points, a time step, the learned
// stage, then error paths and destroy.
int run_model(int model, int nx, int ny, int nz, bool rate_well) {
  const int n = nx * ny * nz, b = model == CPR_MODEL_BLACK_OIL ? 3 : 2;
  cpr_grid_t g{nx, ny, nz, 10.0, 10.0, 5.0, 2000.0};
  cpr_fluid_t f{};
  f.model = model;
  f.p_ref = 200.0;
  f.rho_w_ref = 1000.0;
  f.c_w = 4.5e-5;
  f.c_o = 1.0e-4;
  f.c_r = 5.0e-5;
  f.mu_w = 0.5;
  f.s_wc = 0.2;
  f.s_or = 0.2;
  std::vector<double> pvt;
  if (model == CPR_MODEL_BLACK_OIL) {
    f.rho_o_sc = 850.0;
    f.rho_g_sc = 0.9;
    f.sg_den = 0.7;
    f.n_pvt = 7;
    for (int r = 0; r < 6; ++r)
      for (int c = 0; c < 7; ++c) pvt.push_back(kPvt[r][c]);
    f.pvt = pvt.data();
  } else {
    f.rho_o_ref = 800.0;
    f.mu_o = 2.0;
  }
  std::vector<double> perm(3 * (size_t)n), poro(n), x0((size_t)b * n);
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const int c = i + nx * (j + ny * k);
        const double kx = 100.0 * std::exp(0.8 * std::sin(0.7 * i + 1.3 * j) + 0.5 * std::cos(0.9 * k + 0.4 * i));
        perm[c] = perm[n + c] = kx;
        perm[2 * (size_t)n + c] = 0.1 * kx;
        poro[c] = 0.15 + 0.1 * (0.5 + 0.5 * std::sin(0.37 * c));
        x0[c] = 200.0 + 740.0 * 9.80665 * (k + 0.5) * 5.0 / 1e5;
        x0[n + c] = 0.3;
        if (b == 3) x0[2 * (size_t)n + c] = 0.05;
      }
  std::vector<cpr_well_t> wells = {
      {nx / 2, ny / 2, 0, nz - 1, CPR_WELL_INJECTOR, 300.0, 0.1, 0.0, CPR_CONTROL_BHP, 0.0},
      {0, 0, 0, nz - 1, CPR_WELL_PRODUCER, 150.0, 0.1, 0.0, CPR_CONTROL_BHP, 0.0},
      {nx - 1, ny - 1, 0, nz - 1, CPR_WELL_PRODUCER, 150.0, 0.1, 0.0,
       rate_well ? CPR_CONTROL_RATE : CPR_CONTROL_BHP, 50.0}};

  DevBuf dperm(perm.size() * 8), dporo(poro.size() * 8);
  CHECK(put(dperm, perm) == 0 && put(dporo, poro) == 0, "upload");
  cpr_ctx_t* ctx = nullptr;
  // invalid creations first
  // (a failed create still returns a context, for cpr_last_error)
  cpr_grid_t bad = g;
  bad.nx = 0;
  CHECK(cpr_create(&bad, &f, dperm.d(), dporo.d(), wells.data(), 3, nullptr, &ctx) == CPR_EINVAL, "nx = 0");
  CHECK(std::strlen(cpr_last_error(ctx)) > 0, "create error text");
  cpr_destroy(ctx);
  CHECK(cpr_create(&g, &f, nullptr, dporo.d(), wells.data(), 3, nullptr, &ctx) == CPR_EINVAL, "null perm");
  cpr_destroy(ctx);
  CHECK(cpr_create(&g, &f, dperm.d(), dporo.d(), wells.data(), 3, nullptr, &ctx) == CPR_OK, "create");
  CHECK(cpr_block_size(ctx) == b && cpr_num_cells(ctx) == n, "shape");
  const long long nu = cpr_num_unknowns(ctx);
  CHECK(nu == (long long)b * n + (rate_well ? 1 : 0), "unknowns");

  std::vector<double> xs(nu, 0.0);
  std::copy(x0.begin(), x0.end(), xs.begin());
  if (rate_well) xs[(size_t)b * n] = 150.0;
  DevBuf dx_old(nu * 8), dx(nu * 8), rhs(nu * 8), dxs(nu * 8), y(nu * 8), z(nu * 8);
  CHECK(put(dx_old, xs) == 0 && put(dx, xs) == 0, "state");
  CHECK(cpr_gmres_solve(ctx, rhs.d(), dxs.d(), nullptr) == CPR_EINVAL, "solve before setup");
  CHECK(assemble_jacobian(ctx, dx_old.d(), dx.d(), -1.0, rhs.d()) == CPR_EINVAL, "dt < 0");
  CHECK(cpr_set_timing(ctx, 1) == CPR_OK, "timing on");
  CHECK(assemble_jacobian(ctx, dx_old.d(), dx.d(), 1.0, rhs.d()) == CPR_OK, "assemble");

  cpr_options_t o;
  cpr_default_options(&o);
  cpr_options_t wrong = o;
  wrong.restart = 0;
  CHECK(cpr_setup(ctx, &wrong) == CPR_EINVAL, "restart 0");
  wrong = o;
  wrong.nn_level = -2;
  CHECK(cpr_setup(ctx, &wrong) == CPR_EINVAL, "nn_level -2");
  wrong = o;
  wrong.learned = 1;
  CHECK(cpr_setup(ctx, &wrong) == CPR_EINVAL, "learned without a network");
  CHECK(std::strlen(cpr_last_error(ctx)) > 0, "error text");
  wrong = o;
  wrong.ilu_order = 5;
  CHECK(cpr_setup(ctx, &wrong) == CPR_EINVAL, "unknown ILU order");
  wrong.ilu_order = CPR_ILU_TILES;
  wrong.composition = CPR_COMPOSE_FPF;
  CHECK(cpr_setup(ctx, &wrong) == CPR_EINVAL, "tiled ILU with F-P-F");

  struct Form {
    int precision, decoupling, composition, orth, pre, post;
    double alpha;
    int ilu_order;
  } forms[] = {{CPR_PREC_FP64, CPR_DECOUPLE_QIMPES, CPR_COMPOSE_PF, CPR_ORTH_DCGS2, 1, 1, 1.0, CPR_ILU_RED_BLACK},
               {CPR_PREC_MIXED, CPR_DECOUPLE_QIMPES, CPR_COMPOSE_PF, CPR_ORTH_DCGS2, 2, 2, 1.25, CPR_ILU_RED_BLACK},
               {CPR_PREC_FP64, CPR_DECOUPLE_ABF, CPR_COMPOSE_FPF, CPR_ORTH_CGS2, 1, 2, 1.0, CPR_ILU_RED_BLACK},
               {CPR_PREC_MIXED, CPR_DECOUPLE_QIMPES, CPR_COMPOSE_FPF, CPR_ORTH_DCGS2, 2, 1, 1.5, CPR_ILU_RED_BLACK},
               {CPR_PREC_FP64, CPR_DECOUPLE_QIMPES, CPR_COMPOSE_PF, CPR_ORTH_DCGS2, 2, 2, 1.25, CPR_ILU_TILES},
               {CPR_PREC_MIXED, CPR_DECOUPLE_ABF, CPR_COMPOSE_PF, CPR_ORTH_DCGS2, 1, 1, 1.0, CPR_ILU_TILES}};
  for (const Form& fm : forms) {
    cpr_options_t q = o;
    q.ilu_order = fm.ilu_order;
    q.precision = fm.precision;
    q.decoupling = fm.decoupling;
    q.composition = fm.composition;
    q.orth = fm.orth;
    q.mg_pre = fm.pre;
    q.mg_post = fm.post;
    q.mg_alpha = fm.alpha;
    CHECK(cpr_setup(ctx, &q) == CPR_OK, "setup form");
    cpr_stats_t st{};
    CHECK(cpr_gmres_solve(ctx, rhs.d(), dxs.d(), &st) == CPR_OK, "fgmres");
    CHECK(st.converged && st.true_rel <= 1e-6, "fgmres converged");
    CHECK(st.ms_solve > 0.0 && st.ms_spmv > 0.0 && st.ms_precond > 0.0 && st.ms_orth > 0.0, "phase times");
    CHECK(cpr_bicgstab_solve(ctx, rhs.d(), dxs.d(), &st) == CPR_OK, "bicgstab");
  }
  // restart longer than the delayed form supports (CGS2 path) and a tiny
  // restart with a capped iteration count
  o.restart = 40;
  CHECK(cpr_setup(ctx, &o) == CPR_OK, "setup m = 40");
  CHECK(cpr_gmres_solve(ctx, rhs.d(), dxs.d(), nullptr) == CPR_OK, "fgmres m = 40");
  o.restart = 3;
  o.max_iter = 4;
  o.rtol = 0.0;
  CHECK(cpr_setup(ctx, &o) == CPR_OK, "setup m = 3");
  CHECK(cpr_gmres_solve(ctx, rhs.d(), dxs.d(), nullptr) == CPR_NOT_CONVERGED, "capped solve");
  cpr_default_options(&o);
  CHECK(cpr_set_timing(ctx, 0) == CPR_OK, "timing off");
  CHECK(cpr_setup(ctx, &o) == CPR_OK, "setup default");

  // verification entry points
  CHECK(cpr_spmv(ctx, dxs.d(), y.d()) == CPR_OK, "spmv");
  CHECK(cpr_precond_apply(ctx, rhs.d(), z.d()) == CPR_OK, "precond");
  if (nu <= cpr_spmv_noalloc_max_unknowns()) CHECK(cpr_spmv_noalloc(ctx, dxs.d(), z.d()) == CPR_OK, "noalloc");
  DevBuf blocks((size_t)7 * b * b * n * 8);
  CHECK(cpr_export_jacobian(ctx, blocks.d()) == CPR_OK, "export J");
  CHECK(cpr_import_jacobian(ctx, blocks.d()) == CPR_OK, "import J");
  CHECK(cpr_setup(ctx, &o) == CPR_OK, "setup after import");
  DevBuf w((size_t)b * n * 8), dinv((size_t)b * b * n * 8), a7((size_t)7 * n * 8);
  CHECK(cpr_export_qimpes(ctx, w.d()) == CPR_OK, "qimpes");
  CHECK(cpr_export_ilu(ctx, dinv.d()) == CPR_OK, "ilu");
  int lx, ly, lz, levels = 0;
  while (cpr_mg_level_shape(ctx, levels, &lx, &ly, &lz) == CPR_OK) {
    CHECK(cpr_export_mg_level(ctx, levels, a7.d()) == CPR_OK, "level export");
    ++levels;
  }
  CHECK(levels >= 2, "hierarchy");
  CHECK(cpr_export_mg_level(ctx, levels, a7.d()) == CPR_EINVAL, "level past the hierarchy");
  CHECK(cpr_profile_kernel(ctx, CPR_KCLASS_SPMV) == CPR_OK, "profile on");
  CHECK(cpr_gmres_solve(ctx, rhs.d(), dxs.d(), nullptr) == CPR_OK, "profiled solve");
  int launches = 0;
  double ms = 0.0;
  CHECK(cpr_profile_read(ctx, &launches, &ms) == CPR_OK && launches > 0, "profile read");
  CHECK(cpr_profile_kernel(ctx, -1) == CPR_OK, "profile off");
  CHECK(cpr_profile_kernel(ctx, 99) == CPR_EINVAL, "profile class");
  CHECK(cpr_export_krylov(ctx, 0, z.d()) == CPR_OK, "krylov export");
  CHECK(cpr_newton_update(ctx, dx.d(), dxs.d()) == CPR_OK, "newton update");

  // the learned stage with an untrained network (judged, so any output is safe)
  if (nx % 8 == 0 && ny % 8 == 0 && nz % 8 == 0) {
    const long long np = cpr_nn_num_params();
    std::vector<float> theta(np);
    for (long long i = 0; i < np; ++i) theta[i] = 0.01f * std::sin(0.1f * (float)i);
    CHECK(cpr_nn_attach(ctx, theta.data()) == CPR_OK, "attach");
    o.learned = 1;
    o.precision = CPR_PREC_MIXED;
    CHECK(cpr_setup(ctx, &o) == CPR_OK, "setup learned");
    int lv = -5;
    CHECK(cpr_nn_level(ctx, &lv) == CPR_OK && lv >= 0, "nn level");
    cpr_stats_t st{};
    CHECK(cpr_gmres_solve(ctx, rhs.d(), dxs.d(), &st) == CPR_OK, "learned solve");
    // (after a stalled cycle the rest runs as plain FP64 CPR, without the stage)
    CHECK(st.nn_accepted + st.nn_rejected <= st.iterations, "judge counts");
    DevBuf rp(n * 8), dp(n * 8), feat((size_t)3 * n * 4);
    CHECK(cpr_pressure_stage(ctx, rhs.d(), rp.d(), dp.d()) == CPR_OK, "pressure stage");
    double scale = 0.0;
    CHECK(cpr_nn_features(ctx, rp.d(), feat.f(), &scale) == CPR_OK, "features");
    o.nn_level = 99;
    CHECK(cpr_setup(ctx, &o) == CPR_EINVAL, "nn level beyond the hierarchy");
    CHECK(cpr_nn_attach(ctx, nullptr) == CPR_OK, "detach");
    cpr_default_options(&o);
    CHECK(cpr_setup(ctx, &o) == CPR_OK, "setup plain again");
  }

  // one backward-Euler step and a short simulation
  cpr_newton_options_t no;
  cpr_default_newton_options(&no);
  cpr_newton_stats_t ns{};
  CHECK(put(dx_old, xs) == 0, "state");
  const int rc = cpr_time_step(ctx, dx_old.d(), dx.d(), 0.5, &o, &no, &ns);
  CHECK(rc == CPR_OK || rc == CPR_NOT_CONVERGED, "time step");
  no.forcing = 7;
  CHECK(cpr_time_step(ctx, dx_old.d(), dx.d(), 0.5, &o, &no, &ns) == CPR_EINVAL, "bad forcing");
  cpr_default_newton_options(&no);
  cpr_sim_stats_t ss{};
  const int rs = cpr_simulate(ctx, dx_old.d(), dx.d(), 1.0, 0.25, 1.0, 2.0, &o, &no, &ss);
  CHECK(rs == CPR_OK || rs == CPR_NOT_CONVERGED, "simulate");
  CHECK(cpr_simulate(ctx, dx_old.d(), dx.d(), -1.0, 0.25, 1.0, 2.0, &o, &no, &ss) == CPR_EINVAL, "bad t_end");
  std::vector<double> xh = get(dx, nu);
  for (double v : xh) CHECK(std::isfinite(v), "finite state");
  cpr_destroy(ctx);
  return 0;
}

// The network's own entry points: forward, backward, a training step,
// Adam state round trip, loss evaluation, targets; and their error paths.
int run_network() {
  const int nx = 16, ny = 16, nz = 8, B = 2, n = nx * ny * nz;
  cpr_nn_t* nn = nullptr;
  CHECK(cpr_nn_create(3, 16, 8, 1, nullptr, &nn) == CPR_EINVAL, "grid not divisible by 8");
  cpr_nn_destroy(nn);
  CHECK(cpr_nn_create(nx, ny, nz, B, nullptr, &nn) == CPR_OK, "nn create");
  const long long np = cpr_nn_num_params();
  std::vector<float> theta(np), m(np), v(np);
  for (long long i = 0; i < np; ++i) theta[i] = 0.05f * std::cos(0.37f * (float)i);
  CHECK(cpr_nn_set_params(nn, theta.data()) == CPR_OK, "set params");
  std::vector<float> xh((size_t)B * n * 3), th((size_t)B * n);
  for (size_t i = 0; i < xh.size(); ++i) xh[i] = std::sin(0.01f * (float)i);
  for (size_t i = 0; i < th.size(); ++i) th[i] = std::cos(0.02f * (float)i);
  DevBuf x(xh.size() * 4), t(th.size() * 4), yv(th.size() * 4), dy(th.size() * 4), grad(np * 4);
  HIPOK(hipMemcpy(x.p, xh.data(), xh.size() * 4, hipMemcpyHostToDevice));
  HIPOK(hipMemcpy(t.p, th.data(), th.size() * 4, hipMemcpyHostToDevice));
  CHECK(cpr_nn_forward(nn, x.f(), B, yv.f()) == CPR_OK, "forward");
  CHECK(cpr_nn_forward(nn, x.f(), B + 1, yv.f()) == CPR_EINVAL, "batch beyond the maximum");
  HIPOK(hipMemcpy(dy.p, t.p, th.size() * 4, hipMemcpyDeviceToDevice));
  CHECK(cpr_nn_backward(nn, dy.f(), grad.f()) == CPR_OK, "backward");
  CHECK(cpr_nn_infer(nn, x.f(), yv.f()) == CPR_OK, "infer");
  float loss = 0.f, loss2 = 0.f;
  CHECK(cpr_nn_train_step(nn, x.f(), t.f(), B, 1e-3f, &loss) == CPR_OK, "train step");
  CHECK(cpr_nn_eval_loss(nn, x.f(), t.f(), B, &loss2) == CPR_OK, "eval loss");
  CHECK(std::isfinite(loss) && std::isfinite(loss2), "finite losses");
  long long step = 0;
  CHECK(cpr_nn_get_adam(nn, m.data(), v.data(), &step) == CPR_OK && step == 1, "adam get");
  CHECK(cpr_nn_set_adam(nn, m.data(), v.data(), step) == CPR_OK, "adam set");
  CHECK(cpr_nn_get_params(nn, theta.data()) == CPR_OK, "get params");
  DevBuf e(n * 8), tt(n * 4);
  std::vector<double> eh(n, 1.5);
  CHECK(put(e, eh) == 0, "upload e");
  CHECK(cpr_nn_make_target(e.d(), n, 2.0, tt.f(), nullptr) == CPR_OK, "target");
  CHECK(cpr_nn_make_target(e.d(), n, 0.0, tt.f(), nullptr) == CPR_EINVAL, "zero scale");
  CHECK(cpr_nn_last_error(nn) != nullptr, "nn error text");
  cpr_nn_destroy(nn);
  return 0;
}

int run_all() {
  // the caller's allocator: every block the library takes goes back
  CHECK(cpr_set_allocator(count_alloc, count_free, nullptr) == CPR_OK, "allocator on");
  std::printf("oil-water 24x16x8, caller allocator\n");
  if (run_model(CPR_MODEL_OIL_WATER, 24, 16, 8, false)) return 1;
  CHECK(g_live == 0, "allocator blocks returned");
  CHECK(cpr_set_allocator(nullptr, nullptr, nullptr) == CPR_OK, "allocator off");
  std::printf("black oil 32x16x8 with a rate well\n");
  if (run_model(CPR_MODEL_BLACK_OIL, 32, 16, 8, true)) return 1;
  std::printf("black oil 34x20x6\n");
  if (run_model(CPR_MODEL_BLACK_OIL, 34, 20, 6, false)) return 1;
  std::printf("network\n");
  if (run_network()) return 1;
  HIPOK(hipDeviceSynchronize());
  std::printf("capi driver: all checks passed\n");
  return 0;
}

}  // namespace

int main() {
  std::setvbuf(stdout, nullptr, _IOLBF, 0);
  const int rc = run_all();
  std::fflush(stdout);
  std::fflush(stderr);
  // Every context and network has been destroyed above.  The HIP runtime's
  // own static destructors are skipped: under the AddressSanitizer runtime
  // the HSA runtime frees memory at unload that the sanitizer's device
  // allocator no longer accepts, which aborts the process after the checks.
  std::_Exit(rc);
}
