/*
 * cprmi.h -- C ABI of the MI355X CPR-FGMRES Newton-solve library.
 *
 * The library implements the linear-solve hot path of a fully implicit
 * black-oil / oil-water reservoir simulator (Liu, Wang & Chen, "Large-scale
 * Reservoir Simulations on IBM Blue Gene/Q"): each inexact Newton iteration
 * (Algorithm 1) assembles the Jacobian A of the discrete mass balances
 * (eqs. (3)/(5) with the wells of eq. (6), backward Euler eq. (10) and the
 * cell-centred transmissibilities of eq. (11)) and the right-hand side
 * b = -F(x), then finds dx with ||b - A dx|| <= theta ||b|| (eq. (13)) by
 * restarted flexible GMRES preconditioned with a two-stage CPR method
 * (Sec. 2.5: quasi-IMPES decoupling, multigrid on the pressure block A_pp of
 * eq. (16), then block ILU(0) on the full system).
 *
 * Conventions shared by every entry point
 *   - Cells are numbered in natural order n = i + nx*(j + ny*k), k downward.
 *     A per-cell vector with b unknowns is stored unknown-major, [b][n]:
 *     x[u*n + cell].  Unknowns are (p [bar]) for the single-phase test
 *     model, (p [bar], S_w) for oil-water and
 *     (p_o [bar], S_w, x2) for black oil, whose third unknown switches with
 *     the phase state (Sec. 2.4: gas saturation or bubble point pressure):
 *     x2 = S_g >= 0 in a saturated cell, x2 = -p_b < 0 (bar) in an
 *     undersaturated cell (no free gas; Rs and mu_o at p_b, B_o = B_o(p_b)
 *     exp(-c_o (p - p_b))).  Equation rows are the components (oil,
 *     water[, gas]).
 *   - Rate-controlled wells (eqs. (8)-(9)) make their bottom-hole pressures
 *     unknowns: a state, right-hand side, correction or Krylov vector then
 *     holds the [b][n] cell part followed by one BHP (bar) / well-equation
 *     entry per rate well, in the order the wells were given
 *     (cpr_num_unknowns() = b*n + rate wells).  Without rate wells the
 *     vectors are exactly [b][n].
 *   - Every array argument marked "device" is memory on the current HIP
 *     device; the caller owns it and keeps it alive for the call.  Calls are
 *     ordered on the HIP stream given to cpr_create and return once their
 *     work is queued, except where a call says it synchronises.
 *   - Return value: CPR_OK (0), CPR_NOT_CONVERGED (1), or a negative error
 *     code.  No C++ exception crosses this interface.  After an error,
 *     cpr_last_error() describes it.
 *   - One context per stream and host thread; calls on one context must not
 *     overlap.
 */
#ifndef CPRMI_H
#define CPRMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CPR_OK = 0,
  CPR_NOT_CONVERGED = 1,   /* dx holds the last iterate                     */
  CPR_EINVAL = -1,         /* bad argument or unsupported shape             */
  CPR_ENOMEM = -2,         /* device allocation failed                      */
  CPR_EHIP = -3,           /* a HIP runtime call failed                     */
  CPR_ESINGULAR = -4,      /* singular diagonal or coarsest-level block     */
  CPR_ENONFINITE = -5,     /* NaN or Inf in the input or during the solve   */
  CPR_EBREAKDOWN = -6      /* Krylov breakdown without convergence          */
};

enum { CPR_MODEL_SINGLE_PHASE = 1, CPR_MODEL_OIL_WATER = 2, CPR_MODEL_BLACK_OIL = 3 };
enum { CPR_WELL_INJECTOR = 0, CPR_WELL_PRODUCER = 1 };
enum { CPR_CONTROL_BHP = 0, CPR_CONTROL_RATE = 1 };
enum { CPR_PREC_FP64 = 0, CPR_PREC_MIXED = 1 };

/* Decoupling of the CPR preconditioner (Sec. 2.5 names both):
 *   CPR_DECOUPLE_QIMPES  quasi-IMPES: row 0 of every block row becomes
 *                        w_i^T A_ij with w_i = D_i^-T e_0 / (D_i^-1)_00;
 *   CPR_DECOUPLE_ABF     alternate block factorisation: every block row is
 *                        multiplied by D_i^-1, so each diagonal block is I.
 * D_i is the diagonal block of cell i.  Composition of the two stages:
 *   CPR_COMPOSE_PF       pressure stage, then block ILU(0) on what it leaves;
 *   CPR_COMPOSE_FPF      CPR-FPF (Sec. 2.5): block ILU(0), then the pressure
 *                        stage and block ILU(0) on the remaining residual,
 *                        all multiplicative. */
enum { CPR_DECOUPLE_QIMPES = 0, CPR_DECOUPLE_ABF = 1 };
enum { CPR_COMPOSE_PF = 0, CPR_COMPOSE_FPF = 1 };

/* Orthogonalisation of the FGMRES basis (the eq. (13) solve; not specified
 * by the paper, whose examples use BiCGSTAB):
 *   CPR_ORTH_DCGS2  classical Gram-Schmidt twice with the second pass of
 *                   each vector delayed into the next Arnoldi step, so the
 *                   basis is read twice per step instead of three times
 *                   (the same basis in exact arithmetic; restart <= 32,
 *                   longer restarts use CGS2);
 *   CPR_ORTH_CGS2   both passes in the step. */
enum { CPR_ORTH_DCGS2 = 0, CPR_ORTH_CGS2 = 1 };

/* Elimination order of the block ILU(0) of the full-system stage (the paper
 * leaves it open apart from its potential reordering, Sec. 4 Example 2):
 *   CPR_ILU_RED_BLACK  red cells ((i+j+k) even) before black ones;
 *   CPR_ILU_TILES      tiles of 1 x 2 x 2 cells (i; j, j+1; k, k+1 for even
 *                      j, k) coloured red or black by the parity of
 *                      (i + j/2 + k/2), red tiles before black ones, and the
 *                      cells of a tile in natural order (y before z).  Cells
 *                      of one tile couple inside the factorisation, which
 *                      brings ILU(0) closer to the sequential natural order
 *                      while tiles of one colour stay independent.  P-then-F
 *                      composition only. */
enum { CPR_ILU_RED_BLACK = 0, CPR_ILU_TILES = 1 };

/* options.nn_level: cpr_setup chooses the multigrid level of the learned
 * stage among the coarse levels it can run on -- the coarsest of at least
 * 2^19 cells, else the coarsest of at least 2^16 cells, else the fine level.
 * The options stored in the context then hold the resolved level, which
 * cpr_pressure_stage and cpr_nn_features use as well. */
enum { CPR_NN_LEVEL_AUTO = -1 };

/* Structured Cartesian grid: cell sizes in metres, depth of the top face in
 * metres (depth positive downward).  nx must be even: the library stores
 * every per-cell array split by red-black colour along x (coarse multigrid
 * levels may have any shape). */
typedef struct {
  int nx, ny, nz;
  double dx, dy, dz;
  double top;
} cpr_grid_t;

/* Fluid and rock description (Sec. 2.1-2.2).  Pressures in bar,
 * compressibilities in 1/bar, viscosities in cP, densities in kg/m^3.
 *   single phase (test model, one unknown p, water): rho_w_ref, c_w, c_r,
 *              mu_w;
 *   oil-water: rho_o_ref, rho_w_ref, c_o, c_w, c_r, mu_o, mu_w, s_wc, s_or
 *              (Corey curves of eqs. (17)-(18), exponent 2);
 *   black oil: rho_o_sc, rho_g_sc (surface densities), rho_w_ref, c_w, c_r,
 *              mu_w, s_wc, s_or, sg_den, c_o (undersaturated oil
 *              compressibility), and a host table pvt[6][n_pvt] of
 *              rows p, Rs, Bo, mu_o, Bg, mu_g, piecewise linear in p
 *              (the right-hand segment at a node, end segments extended).
 * The table is copied during cpr_create. */
typedef struct {
  int model;
  double p_ref;
  double rho_w_ref, rho_o_ref, rho_o_sc, rho_g_sc;
  double c_w, c_o, c_r;
  double mu_w, mu_o;
  double s_wc, s_or, sg_den;
  int n_pvt;
  const double* pvt;   /* host, [6][n_pvt]; NULL for oil-water */
} cpr_fluid_t;

/* A vertical well perforated in cells (i, j, k0..k1), its bottom-hole
 * pressure referenced to the depth of the grid top; perforation rates from
 * eq. (6) with a Peaceman well index of radius rw (m) and skin.
 *   CPR_CONTROL_BHP: the BHP is fixed (eq. (7)) and adds no unknown.
 *   CPR_CONTROL_RATE: the BHP is an unknown and the well adds the equation
 *     sum of its perforations' rates = rate (eq. (8) water rate of an
 *     injector, eq. (9) oil rate of a producer), in surface m^3/day (mass
 *     rate / rho_w_ref for water, / rho_o_sc (black oil) or rho_o_ref
 *     (oil-water) for oil); the row is scaled like the component's cell
 *     rows; `bhp` is then unused (the state vector carries the BHP). */
typedef struct {
  int i, j, k0, k1;
  int kind;            /* CPR_WELL_INJECTOR (water) or CPR_WELL_PRODUCER */
  double bhp;          /* bar */
  double rw, skin;
  int control;         /* CPR_CONTROL_BHP or CPR_CONTROL_RATE                */
  double rate;         /* target surface rate (m^3/day, >= 0) of a rate well */
} cpr_well_t;

typedef struct {
  int precision;       /* CPR_PREC_FP64, or CPR_PREC_MIXED: FP32 preconditioner
                          inside FP64 FGMRES                                 */
  int learned;         /* 1: apply the loaded pressure-correction network    */
  int restart;         /* FGMRES restart length m, 1..64 (default 30)       */
  int max_iter;        /* total Arnoldi iterations (default 300)            */
  double rtol;         /* stop when ||b - A dx||_2 <= rtol ||b||_2 (1e-6)    */
  int mg_coarsest;     /* coarsen while a level has more cells (512, <= 4096) */
  double mg_alpha;     /* coarse-correction scaling x += alpha P e (1.0, finite) */
  int decoupling;      /* CPR_DECOUPLE_QIMPES (default) or CPR_DECOUPLE_ABF  */
  int composition;     /* CPR_COMPOSE_PF (default) or CPR_COMPOSE_FPF        */
  int x0;              /* 1: cpr_gmres_solve starts from the dx passed in
                          (0, default: from zero; BiCGSTAB always from zero) */
  int mg_pre, mg_post; /* red-black Gauss-Seidel sweeps before / after the
                          coarse correction, 1..8 (1, 1: V(1,1))            */
  double stall_ratio;  /* MIXED or learned, FGMRES: when a restart cycle ends
                          with the true residual above stall_ratio times the
                          one it started from, the remaining cycles apply
                          plain FP64 CPR (FP64 preconditioner, no learned
                          stage; default 0.5: less than halved; 1.0: not
                          decreased; <= 0: never).  With restart m > 10
                          the first cycle ends after 10 steps if its residual
                          estimate is still above stall_ratio^(10/m) times
                          the initial residual (and the check above
                          follows).                                        */
  int orth;            /* CPR_ORTH_DCGS2 (default) or CPR_ORTH_CGS2        */
  int nn_level;        /* learned stage (learned = 1) on multigrid level:
                          0: the fine pressure residual after the cycle;
                          l >= 1: inside the cycle on level l, after its
                          post-smoothing (cpr_nn_attach);
                          CPR_NN_LEVEL_AUTO (default): chosen by cpr_setup */
  int ilu_order;       /* CPR_ILU_RED_BLACK (default) or CPR_ILU_TILES      */
} cpr_options_t;

typedef struct {
  int iterations;      /* Arnoldi matrix-vector products                     */
  int cycles;          /* restart cycles                                     */
  int converged;
  int mg_levels;
  int qimpes_fallback; /* cells whose decoupling weight fell back to e_0     */
  int nn_accepted, nn_rejected;
  double bnorm;        /* ||b||_2                                            */
  double est_rel;      /* GMRES estimate of ||b - A dx|| / ||b|| at the end  */
  double true_rel;     /* recomputed ||b - A dx|| / ||b||                    */
  int fp64_fallback;   /* MIXED or learned: restart cycles run before plain
                          FP64 CPR took over (0: it never did)              */
  /* Phase times in milliseconds of device time (stream time between HIP
   * events), filled while cpr_set_timing is on, else 0.                     */
  double ms_assemble;  /* the last assemble_jacobian before this solve      */
  double ms_setup;     /* the last cpr_setup before this solve              */
  double ms_solve;     /* this solve, from the first kernel to the last     */
  double ms_precond;   /* its preconditioner applications                   */
  double ms_spmv;      /* its block SpMVs (Krylov steps, true residuals)    */
  double ms_orth;      /* FGMRES: orthogonalisation passes and their
                          reductions; BiCGSTAB: inner products and vector
                          updates                                            */
} cpr_stats_t;

typedef struct cpr_ctx cpr_ctx_t;

/* Fill *o with the defaults listed above. */
void cpr_default_options(cpr_options_t* o);

/* Phase timers (measurement, not part of the method).  on = 1: HIP events
 * on the context's stream bracket assemble_jacobian, cpr_setup, the solves
 * and, inside a solve, every preconditioner application, SpMV and
 * orthogonalisation step; a solve's cpr_stats_t then carries the times.
 * The inner events are read back where the solver already waits for the
 * device, so timing adds no synchronisation, only the event records.  on =
 * 0 (default) records nothing.  Independently of this switch, every entry
 * point of the library opens a roctx range named after it (visible to
 * rocprofv3 --marker-trace).  CPR_EINVAL for a null context. */
int cpr_set_timing(cpr_ctx_t* ctx, int on);

/* Device memory: by default the library allocates with hipMalloc and frees
 * with hipFree.  cpr_set_allocator installs a caller's allocator instead
 * (for instance a framework's caching allocator): alloc(bytes, user) returns
 * device memory of the current device (NULL on failure, reported as
 * CPR_EHIP / CPR_ENOMEM by the call that needed it), release(ptr, user) takes
 * it back.  Both NULL restore the default; exactly one NULL is CPR_EINVAL.
 * Process-wide and thread-safe; a context or network keeps the allocator in
 * force when it was created for all its memory until it is destroyed. */
int cpr_set_allocator(void* (*alloc)(size_t bytes, void* user), void (*release)(void* ptr, void* user),
                      void* user);

/* Create a context.  perm3 (device, [3][n], mD, kx ky kz) and poro (device,
 * [n]) are read during the call and copied; wells is a host array.  The
 * library owns every buffer it allocates (Jacobian, hierarchy, Krylov basis)
 * and frees them in cpr_destroy.  stream: a hipStream_t (NULL = default
 * stream).  Transmissibilities (harmonic, eq. (11)) and Peaceman well
 * indices are computed here.  Synchronises the stream. */
int cpr_create(const cpr_grid_t* g, const cpr_fluid_t* f, const double* perm3,
               const double* poro, const cpr_well_t* wells, int nwells, void* stream,
               cpr_ctx_t** out);

void cpr_destroy(cpr_ctx_t* ctx);
const char* cpr_last_error(const cpr_ctx_t* ctx);

/* Unknowns of a state vector: b * cells + rate-controlled wells. */
long long cpr_num_unknowns(const cpr_ctx_t* ctx);

/* Number of unknowns per cell (1, 2 or 3) and cells of the context. */
int cpr_block_size(const cpr_ctx_t* ctx);
long long cpr_num_cells(const cpr_ctx_t* ctx);

/* Assemble the Jacobian A = dR/dx at x (kept in the context) and write
 * rhs_out = -R(x) (device, [b][n]) for the time step x_old -> x of length
 * dt_days (eqs. (3)/(5), (6), (10), (11); Algorithm 1, step 3).  Each
 * component's rows are divided by rho_c * V * mean(phi) / dt. */
int assemble_jacobian(cpr_ctx_t* ctx, const double* x_old, const double* x, double dt_days,
                      double* rhs_out);

/* Replace the context's Jacobian by blocks (device, natural order
 * [7][b][b][n]; block direction d = self, -x, +x, -y, +y, -z, +z;
 * blocks[((d*b + r)*b + c)*n + cell] = dR_r(cell)/dx_c(neighbour d)),
 * or copy it out in the same layout.  Blocks that reach outside the grid
 * must be zero on import and are zero on export. */
int cpr_import_jacobian(cpr_ctx_t* ctx, const double* blocks);
int cpr_export_jacobian(cpr_ctx_t* ctx, double* blocks);

/* Build the CPR preconditioner for the current Jacobian (Sec. 2.5: the
 * two-stage CPR family; the pressure block A_pp and the full system of the
 * block structure of eq. (16)): the decoupling (quasi-IMPES weights and
 * decoupled rows, or the ABF inverses D_i^-1 and the blocks D_i^-1 A_ij),
 * the pressure multigrid hierarchy on A_p = (A~)_pp (2x2x2 aggregation,
 * Galerkin coarse operators, dense inverse of the coarsest level; a level
 * above the coarsest with odd nx is stored with a ghost column) and the
 * red-black block ILU(0) diagonals of A~.  Synchronises the stream (to report singular blocks).  Returns
 * CPR_ESINGULAR if a diagonal block or the coarsest operator cannot be
 * inverted, CPR_EINVAL for an unknown decoupling or composition. */
int cpr_setup(cpr_ctx_t* ctx, const cpr_options_t* o);

/* Solve A dx = rhs (both device, [b][n]) from dx = 0 (or from the dx passed
 * in, with options.x0 = 1) with FGMRES(restart)
 * and the CPR preconditioner (eq. (13) with theta = rtol).  Synchronises once
 * per Arnoldi iteration to read the Hessenberg column.  st may be NULL.
 * Returns CPR_OK, CPR_NOT_CONVERGED (dx holds the last iterate),
 * CPR_ENONFINITE (non-finite rhs or iterate) or CPR_EBREAKDOWN. */
int cpr_gmres_solve(cpr_ctx_t* ctx, const double* rhs, double* dx, cpr_stats_t* st);

/* Solve A dx = rhs like cpr_gmres_solve, with right-preconditioned
 * BiCGSTAB (van der Vorst), the Krylov method of the paper's examples
 * (Sec. 4), and the same CPR preconditioner (set up by cpr_setup; restart is
 * ignored).  From dx = 0, iterate until the recursively updated residual
 * satisfies ||r|| <= rtol ||rhs||, then form the true residual and restart
 * from dx with it while it exceeds rtol ||rhs|| and iterations remain.  A
 * vanishing rho, <rh, v> or omega ends the iteration (breakdown).
 * st->iterations counts BiCGSTAB iterations (two products with A and two
 * preconditioner applications each), st->cycles the restarts + 1.
 * Synchronises once per iteration.  Workspace: the first eight vectors of
 * the Krylov basis (allocated if smaller).  Returns CPR_OK,
 * CPR_NOT_CONVERGED (dx holds the last iterate) or CPR_ENONFINITE. */
int cpr_bicgstab_solve(cpr_ctx_t* ctx, const double* rhs, double* dx, cpr_stats_t* st);

/* ---------------------------------------------------------------- time step
 * Forcing terms theta_l of the inexact Newton method (Algorithm 1, eq. (13)):
 *   CPR_FORCING_FIXED  theta_l = options.rtol (the standard Newton method);
 *   CPR_FORCING_EW1    ||b^l - r^(l-1)|| / ||b^(l-1)||        (eq. (14), 1st)
 *   CPR_FORCING_EW2    | ||b^l|| - ||r^(l-1)|| | / ||b^(l-1)|| (2nd, absolute value)
 *   CPR_FORCING_EW3    gamma (||b^l|| / ||b^(l-1)||)^beta     (3rd)
 * with r^l = b^l - A^l dx^l the linear residual left by iteration l; the
 * first iteration uses theta0, and every theta_l is clamped to
 * [theta_min, theta_max]. */
enum { CPR_FORCING_FIXED = 0, CPR_FORCING_EW1 = 1, CPR_FORCING_EW2 = 2, CPR_FORCING_EW3 = 3 };
enum { CPR_KRYLOV_FGMRES = 0, CPR_KRYLOV_BICGSTAB = 1 };
#define CPR_NEWTON_HIST 64

typedef struct {
  int forcing;         /* CPR_FORCING_* (default EW1)                        */
  int krylov;          /* CPR_KRYLOV_FGMRES (default) or CPR_KRYLOV_BICGSTAB  */
  int max_newton;      /* Newton iterations per attempt (20)                 */
  int max_cuts;        /* time-step halvings before giving up (6)            */
  double newton_tol;   /* converged when ||b^l|| < newton_tol ||b^0|| (1e-3) */
  double theta0;       /* forcing term of the first iteration (0.1)          */
  double theta_min, theta_max;   /* clamp of theta_l (1e-6, 0.5)             */
  double gamma, beta;  /* choice 3 (0.9, 2)                                  */
} cpr_newton_options_t;

typedef struct {
  int converged;
  int cuts;                    /* halvings of dt before the accepted attempt */
  int newton_iterations;       /* of the accepted (or last) attempt          */
  int linear_iterations;       /* of the accepted (or last) attempt          */
  int total_newton, total_linear;  /* over every attempt                     */
  double dt_taken;             /* days                                       */
  double theta[CPR_NEWTON_HIST];   /* per Newton iteration (first 64)        */
  int lin_its[CPR_NEWTON_HIST];
  double bnorm[CPR_NEWTON_HIST + 1];   /* ||b^l||, l = 0 .. iterations      */
} cpr_newton_stats_t;

/* Fill *o with the defaults listed above. */
void cpr_default_newton_options(cpr_newton_options_t* o);

/* One backward-Euler time step of length dt_days (eq. (10)) by the inexact
 * Newton method of Algorithm 1, from x^0 = x_old (device, [b][n], natural
 * order).  Each iteration assembles b = -F(x) and A, sets up CPR with the
 * linear options `lin` (its rtol replaced by theta_l unless the forcing is
 * CPR_FORCING_FIXED), solves with the chosen Krylov method, and applies the
 * Newton update of cpr_newton_update.  The attempt converges when
 * ||b^l||_2 < newton_tol ||b^0||_2 (b^0 at x_old) and fails after max_newton
 * iterations, on a non-finite residual, or on a singular preconditioner
 * block; a failed attempt halves dt and starts again from x_old (time-step
 * cut), at most max_cuts times.  A linear solve that stops at lin->max_iter
 * still updates x.  On success x (device [b][n]) receives the new state and
 * st->dt_taken the step actually taken; returns CPR_OK.  If every attempt
 * fails x receives x_old and CPR_NOT_CONVERGED is returned.  The Jacobian
 * and preconditioner of the last iteration stay in the context.
 * Synchronises the stream several times per Newton iteration. */
int cpr_time_step(cpr_ctx_t* ctx, const double* x_old, double* x, double dt_days, const cpr_options_t* lin,
                  const cpr_newton_options_t* nopt, cpr_newton_stats_t* st);

#define CPR_SIM_HIST 256
typedef struct {
  int completed;               /* t_end reached                               */
  int steps;                   /* accepted time steps                         */
  int cuts, total_newton, total_linear;   /* sums over every attempt          */
  double t_reached;            /* days                                        */
  double dts[CPR_SIM_HIST];    /* step sizes taken (first 256)                */
  double seconds;              /* wall time of the call (host clock)          */
  /* per accepted step (first 256), every attempt of the step included: the
     columns of the paper's result tables (Sec. 4) step by step */
  int step_newton[CPR_SIM_HIST];
  int step_linear[CPR_SIM_HIST];
  int step_cuts[CPR_SIM_HIST];
  double step_seconds[CPR_SIM_HIST];
} cpr_sim_stats_t;

/* Backward-Euler time stepping over [0, t_end_days] from x0 (device, [b][n],
 * natural order) into x (device, may equal x0): cpr_time_step for each step
 * (with its cuts); after a step that needed no cut the next dt is
 * min(growth * dt_taken, dt_max), after a cut it stays dt_taken; the last
 * step ends exactly at t_end.  The time-step control around the inexact
 * Newton method reported in Sec. 4 (maximum step, cuts); the growth rule is
 * not in the paper.  Returns CPR_OK when t_end is reached, CPR_NOT_CONVERGED
 * when a step fails after its last cut (x then holds the state at
 * st->t_reached). */
int cpr_simulate(cpr_ctx_t* ctx, const double* x0, double* x, double t_end_days, double dt0_days,
                 double dt_max_days, double growth, const cpr_options_t* lin, const cpr_newton_options_t* nopt,
                 cpr_sim_stats_t* st);

/* Newton update of Algorithm 1, step 5 (device, [b][n]): x += dx with
 * saturation changes chopped to |dS| <= 0.2 and saturations clamped to
 * [0, 1].  Black oil switches the third unknown: a saturated cell whose
 * S_g would fall below 0 becomes undersaturated with p_b = p (updated); an
 * undersaturated cell whose updated p_b exceeds p becomes saturated with
 * S_g = 0; p_b is floored at the first PVT pressure. */
int cpr_newton_update(cpr_ctx_t* ctx, double* x, const double* dx);

/* Single operations of the path, for verification: y = A x; one CPR
 * preconditioner application z = M^-1 v (after cpr_setup).  Device [b][n]. */
int cpr_spmv(cpr_ctx_t* ctx, const double* x, double* y);
int cpr_precond_apply(cpr_ctx_t* ctx, const double* v, double* z);

/* For callers that cannot allocate device memory during a call (code under
 * HIP graph capture, tight serving loops, harnesses that forbid it): the
 * product of cpr_spmv, y = A x (device, natural order, cells then rate-well
 * BHPs), staged through a static device buffer of the library instead of
 * the context's own vectors; the call allocates nothing.  The buffer holds
 * two staging vectors of cpr_spmv_noalloc_max_unknowns() = 4,194,304
 * doubles each (64 MiB in all, kept by every GPU the library runs on until
 * the process ends); a context with more unknowns gets CPR_EINVAL.  All
 * calls on one GPU share the buffer: calls that overlap on one GPU (other
 * streams or threads) race and must be serialised by the caller. */
int cpr_spmv_noalloc(cpr_ctx_t* ctx, const double* x, double* y);
long long cpr_spmv_noalloc_max_unknowns(void);

/* Setup products, for verification (device outputs, natural order):
 * quasi-IMPES weights w [b][n] (CPR_EINVAL under ABF); the scalar 7-point operator of multigrid
 * level `level` as [7][n_level] (natural order of that level's grid);
 * the inverted ILU diagonals D'^-1 as [b][b][n]. */
int cpr_export_qimpes(cpr_ctx_t* ctx, double* w);
int cpr_mg_level_shape(const cpr_ctx_t* ctx, int level, int* nx, int* ny, int* nz);
/* The multigrid level of the learned stage under the options of the last
 * cpr_setup (CPR_NN_LEVEL_AUTO resolved); CPR_EINVAL before any setup. */
int cpr_nn_level(const cpr_ctx_t* ctx, int* level);
int cpr_export_mg_level(cpr_ctx_t* ctx, int level, double* a7);
int cpr_export_ilu(cpr_ctx_t* ctx, double* dinv);

/* Kernel-duration sampling, for measurement.  While a class is selected,
 * every launch of that kernel class inside the library is bracketed by a
 * pair of HIP events on the context's stream (up to 8192 launches are
 * kept).  cpr_profile_read synchronises the stream, returns the number of
 * sampled launches and their summed duration in milliseconds, and clears
 * the samples.  kclass -1 switches sampling off. */
enum {
  CPR_KCLASS_SPMV = 0,      /* block SpMV / true residual                 */
  CPR_KCLASS_ORTH = 1,      /* CGS2 dot / update / norm passes            */
  CPR_KCLASS_SMOOTH = 2,    /* red-black Gauss-Seidel half-sweeps         */
  CPR_KCLASS_ILU = 3,       /* stage-2 residual + block-ILU colour sweeps */
  CPR_KCLASS_ASSEMBLE = 4   /* cell-centric flux / Jacobian kernel        */
};
int cpr_profile_kernel(cpr_ctx_t* ctx, int kclass);
int cpr_profile_read(cpr_ctx_t* ctx, int* launches, double* total_ms);

/* ------------------------------------------------------------------------
 * Learned pressure correction (an addition to the paper's method).
 *
 * A 3-D convolutional U-Net (four levels with 16, 32, 64, 64 channels, one
 * 3x3x3 convolution per level on each path, ReLU, 2x2x2 average pooling,
 * nearest upsampling, additive skips, 1x1x1 output) maps three per-cell
 * features -- standardised ln k_x, standardised ln of the total mobility,
 * and D^-1 r' / rms(D^-1 r') with r' the pressure residual left by the
 * multigrid cycle and D the diagonal of A_p -- to a pressure correction.
 * Tensors are FP32, channels-last, natural cell order; convolutions run on
 * the matrix cores in BF16 with FP32 accumulation.  Parameters are one flat
 * FP32 vector: per convolution W[27][Cin][Cout] (tap = (dz+1)*9 +
 * (dy+1)*3 + (dx+1)) then bias[Cout]; then the head w[16], b[1].
 * ---------------------------------------------------------------------- */
typedef struct cpr_nn cpr_nn_t;

long long cpr_nn_num_params(void);

/* A network object for grids nx x ny x nz (each a multiple of 8) and up to
 * max_batch samples; owns parameters, Adam moments and activations.
 * Parameters start at zero: call cpr_nn_set_params.  On error *out is still
 * set so that cpr_nn_last_error can explain; destroy it. */
int cpr_nn_create(int nx, int ny, int nz, int max_batch, void* stream, cpr_nn_t** out);
void cpr_nn_destroy(cpr_nn_t* nn);
const char* cpr_nn_last_error(const cpr_nn_t* nn);

/* Copy parameters in (resets the Adam moments) or out; host arrays of
 * cpr_nn_num_params() floats.  Synchronise. */
int cpr_nn_set_params(cpr_nn_t* nn, const float* theta);
int cpr_nn_get_params(cpr_nn_t* nn, float* theta);

/* Training checkpoint (not in the paper): the Adam first and second moments
 * (host arrays of cpr_nn_num_params() floats each) and the number of Adam
 * steps taken, which sets the bias correction of the next step.  Restore
 * them after cpr_nn_set_params (which clears them) to resume training where
 * it stopped.  Synchronise; CPR_EINVAL on null arrays or a negative step. */
int cpr_nn_get_adam(cpr_nn_t* nn, float* m, float* v, long long* step);
int cpr_nn_set_adam(cpr_nn_t* nn, const float* m, const float* v, long long step);

/* y = N(x) for x (device [batch][n][3]) -> y (device [batch][n]). */
int cpr_nn_forward(cpr_nn_t* nn, const float* x, int batch, float* y);

/* Inference form of cpr_nn_forward for one sample (batch 1): the same
 * network and kernels, keeping only what inference needs, with the 1x1x1
 * head fused into the last convolution on grids of at least 65,536 cells
 * (so results may differ from cpr_nn_forward by FP32 summation order).
 * Leaves nothing for cpr_nn_backward.  Stream-ordered, no synchronisation. */
int cpr_nn_infer(cpr_nn_t* nn, const float* x, float* y);

/* Gradient of sum(dy * y) for the last forward pass with respect to the
 * parameters: dy device [batch][n], grad device [num_params]. */
int cpr_nn_backward(cpr_nn_t* nn, const float* dy, float* grad);

/* One Adam step (lr; beta 0.9 / 0.999; eps 1e-8) on the direction loss
 * (1/B) sum_b min_a |a N(x_b) - t_b|^2 / |t_b|^2 = 1 - cos^2(N(x_b), t_b);
 * x device [batch][n][3], t device [batch][n]; *loss (host, may be NULL)
 * receives the loss before the step. */
int cpr_nn_train_step(cpr_nn_t* nn, const float* x, const float* t, int batch, float lr, float* loss);

/* The loss of the current parameters on (x, t) without a step (host *loss). */
int cpr_nn_eval_loss(cpr_nn_t* nn, const float* x, const float* t, int batch, float* loss);

/* Training target t = e / scale (device: e [n] FP64 -> t [n] FP32) on the
 * given stream: the network output that reproduces the correction e. */
int cpr_nn_make_target(const double* e, long long n, double scale, float* t, void* stream);

/* Give a solver context a copy of trained parameters (host array, NULL to
 * drop it).  With options.learned = 1 every CPR application then forms
 * r' = r~_p - A_p dp_mg after the multigrid cycle, evaluates the network
 * for a direction d = N(features), takes the residual-minimising step
 * dp_nn = alpha d, alpha = <A_p d, r'> / |A_p d|^2, and keeps dp_mg + dp_nn
 * only when ||r' - A_p dp_nn||_2 < ||r'||_2; otherwise the plain CPR result
 * stands.  The grid must have dimensions divisible by 8.
 * With options.nn_level = l >= 1 the same judged step acts inside the
 * multigrid cycle on level l after its post-smoothing: r' = r_l - A_l x_l,
 * the features are the means of ln k_x and ln lambda_t over each coarse
 * cell's 2^l x 2^l x 2^l block of fine cells and D = diag A_l, and an
 * accepted correction is added to x_l before the finer levels'
 * post-smoothing.  Level l must then have dimensions divisible by 8, be
 * exactly 2^-l times the grid along each axis, and lie above the levels the
 * cycle handles in one workgroup (cpr_setup returns CPR_EINVAL otherwise). */
int cpr_nn_attach(cpr_ctx_t* ctx, const float* theta);

/* The pressure stage on one vector, for building training data (device,
 * natural order): r~_p = w^T v; dp_mg = V-cycle(r~_p); rprime = r~_p -
 * A_p dp_mg ([n] each; dp_mg may be NULL).  After cpr_setup with
 * quasi-IMPES decoupling (CPR_EINVAL otherwise).  With options.nn_level =
 * l >= 1: rprime = r_l - A_l x_l, the residual the cycle leaves on level l
 * after its post-smoothing, and dp_mg = x_l, both [n_l] in the natural
 * order of level l. */
int cpr_pressure_stage(cpr_ctx_t* ctx, const double* v, double* rprime, double* dp_mg);

/* Network input for a pressure residual rprime (device [n]): feat device
 * [n][3] natural order; *scale (host) receives rms(D^-1 rprime), the factor
 * that converts network output to a pressure correction.  After cpr_setup
 * of an assembled Jacobian (the mobility channel comes from the state of
 * the last assembly).  With options.nn_level = l >= 1, rprime and feat
 * belong to level l ([n_l] and [n_l][3]). */
int cpr_nn_features(cpr_ctx_t* ctx, const double* rprime, float* feat, double* scale);

/* Basis vector v_j (device [b][n], natural order) of the last FGMRES
 * cycle, j < number of iterations of that cycle. */
int cpr_export_krylov(cpr_ctx_t* ctx, int j, double* v);

#ifdef __cplusplus
}
#endif

#endif /* CPRMI_H */
