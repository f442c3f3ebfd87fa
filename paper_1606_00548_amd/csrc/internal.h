// Internal declarations of the CPR-FGMRES library (not part of the C ABI).
//
// Storage order on the device.  Every per-cell array is colour-split
// ("CS"): cell (i, j, k) with colour c = (i + j + k) & 1 (0 red, 1 black)
// lives at  c * n/2 + (i >> 1) + (nx/2) * (j + ny * k).  Each colour is a
// contiguous half, so a red-black half-sweep streams whole cache lines and
// the +-y / +-z neighbours of a cell sit at a fixed offset in the other half.
// A block array holds one plane of n values per (direction, row, column):
// A[((d * b + r) * b + c) * n + cell], directions d = self, -x, +x, -y, +y,
// -z, +z.  A multigrid level above the coarsest whose nx is odd is stored
// colour-split on a grid one column wider: the extra column (i = nxr) holds
// ghost cells whose stencil row is the identity and to which no real cell
// couples, so they keep x = 0 and r = 0 through every sweep and add nothing
// to a restriction.  The coarsest level with an odd nx uses the natural
// order i + nx * (j + ny * k).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "cprmi.h"

#define CPR_MAX_PVT 16

// Device allocator of a context or network (alloc.hip): the caller's
// callbacks, or hipMalloc / hipFree when they are null.
struct DevAlloc {
  void* (*alloc)(size_t, void*) = nullptr;
  void (*free)(void*, void*) = nullptr;
  void* user = nullptr;
};
DevAlloc current_allocator();
hipError_t dev_malloc(const DevAlloc& a, void** p, size_t bytes);
void dev_free(const DevAlloc& a, void* p);
#define CPR_MAX_WELLS_PERF 65536

struct Lay {
  int nx, ny, nz;  // stored grid (nx includes a ghost column on padded levels)
  int n;     // stored cells
  int half;  // nx / 2 (colour-split only)
  int nh;    // n / 2 (colour-split only)
  int cs;    // 1 colour-split, 0 natural
  int nxr;   // real cells along x: nx, or nx - 1 on a padded level
};

__host__ __device__ inline int lay_index(const Lay& L, int i, int j, int k) {
  if (L.cs) return ((i + j + k) & 1) * L.nh + (i >> 1) + L.half * (j + L.ny * k);
  return i + L.nx * (j + L.ny * k);
}

__host__ __device__ inline void lay_coords(const Lay& L, int t, int& i, int& j, int& k) {
  if (L.cs) {
    int c = t >= L.nh ? 1 : 0;
    int r = t - c * L.nh;
    int m = r % L.half;
    int jk = r / L.half;
    j = jk % L.ny;
    k = jk / L.ny;
    i = 2 * m + ((j + k + c) & 1);
  } else {
    i = t % L.nx;
    int jk = t / L.nx;
    j = jk % L.ny;
    k = jk / L.ny;
  }
}

// Neighbour offsets of the 7 block directions.
__host__ __device__ inline void dir_offset(int d, int& di, int& dj, int& dk) {
  di = (d == 1) ? -1 : (d == 2) ? 1 : 0;
  dj = (d == 3) ? -1 : (d == 4) ? 1 : 0;
  dk = (d == 5) ? -1 : (d == 6) ? 1 : 0;
}

// Index of neighbour d of cell (i, j, k) in layout L, or -1 outside.
__host__ __device__ inline int lay_nbr(const Lay& L, int i, int j, int k, int d) {
  int di, dj, dk;
  dir_offset(d, di, dj, dk);
  int a = i + di, b = j + dj, c = k + dk;
  if (a < 0 || a >= L.nx || b < 0 || b >= L.ny || c < 0 || c >= L.nz) return -1;
  return lay_index(L, a, b, c);
}

// Tiled red-black order of the block ILU(0) (CPR_ILU_TILES): tile (i, tj,
// tk) holds the cells (i, 2tj + b, 2tk + c), b, c in {0, 1}, as q = b + 2c
// (natural order inside, y before z); its colour is (i + tj + tk) & 1.  A
// launch over the tiles of one colour takes thread t to u = t % (nx/2)
// fastest, i = 2u + parity, so consecutive threads read consecutive cells
// of each colour-split row.
__host__ __device__ inline long tile_threads(const Lay& L) {
  return (long)(L.nx >> 1) * ((L.ny + 1) >> 1) * ((L.nz + 1) >> 1);
}
__device__ inline bool tile_of_thread(const Lay& L, int colour, long t, int& i, int& tj, int& tk) {
  const int nu = L.nx >> 1, nty = (L.ny + 1) >> 1;
  if (t >= tile_threads(L)) return false;
  const int u = (int)(t % nu);
  const long tjk = t / nu;
  tj = (int)(tjk % nty);
  tk = (int)(tjk / nty);
  i = 2 * u + ((colour + tj + tk) & 1);
  return true;
}
// The tile-mate of cell q in direction d (-y, +y, -z, +z), or -1 when the
// neighbour in that direction lies in another tile.
__host__ __device__ inline int tile_mate(int q, int d) {
  if (d == 3) return (q & 1) ? q - 1 : -1;
  if (d == 4) return (q & 1) ? -1 : q + 1;
  if (d == 5) return (q & 2) ? q - 2 : -1;
  if (d == 6) return (q & 2) ? -1 : q + 2;
  return -1;
}

// A colour-split cell decoded once; its neighbours are then a few adds away.
// All neighbours of a cell of colour c live in colour 1-c: +-y / +-z at a
// fixed offset from `base` (same m), -x / +x at m or m -+ 1 by the parity
// of i.
struct CsCell {
  int c, m, j, k, i, base;
};

__host__ __device__ inline CsCell cs_decode(const Lay& L, int t) {
  CsCell q;
  q.c = t >= L.nh ? 1 : 0;
  int r = t - q.c * L.nh;
  int row = r / L.half;
  q.m = r - row * L.half;
  q.j = row % L.ny;
  q.k = row / L.ny;
  q.i = 2 * q.m + ((q.j + q.k + q.c) & 1);
  q.base = (1 - q.c) * L.nh + q.m + L.half * row;
  return q;
}

__host__ __device__ inline int cs_nb(const Lay& L, const CsCell& q, int d) {
  const int p = q.i & 1;
  switch (d) {
    case 1: return q.i > 0 ? q.base - (p ? 0 : 1) : -1;
    case 2: return q.i < L.nx - 1 ? q.base + p : -1;
    case 3: return q.j > 0 ? q.base - L.half : -1;
    case 4: return q.j < L.ny - 1 ? q.base + L.half : -1;
    case 5: return q.k > 0 ? q.base - L.half * L.ny : -1;
    case 6: return q.k < L.nz - 1 ? q.base + L.half * L.ny : -1;
    default: return -1;
  }
}

// The six neighbours of a colour-split cell for branch-free stencil code:
// nbr[d] is the neighbour's index, or the cell itself (ok[d] = false) where
// the neighbour lies outside the grid, so every load stays in bounds and
// the caller masks the value.
__host__ __device__ inline void cs_nbrs(const Lay& L, int t, const CsCell& cc, int (&nbr)[7], bool (&ok)[7]) {
  nbr[0] = t;
  ok[0] = true;
#pragma unroll
  for (int d = 1; d < 7; ++d) {
    int q = cs_nb(L, cc, d);
    ok[d] = q >= 0;
    nbr[d] = ok[d] ? q : t;
  }
}

// Block arrays of the fine level (the Jacobian J and its decoupled form,
// the decoupled pressure rows R0, the ILU inverse diagonals, their FP32
// copies) are tiled: 64 consecutive colour-split cells form a tile, and a
// tile holds each of the array's P planes as one run of 64 values, so a
// wave reading a cell's planes streams one contiguous P x 64-value block
// instead of P separate streams.  Element (plane p, cell t) lives at
// tix(P, p, t); an array of n cells holds tiled_len(n, P) values.
constexpr int TILE = 64;
__host__ __device__ inline size_t tix(int P, int p, size_t t) {
  return ((t / TILE) * (size_t)P + p) * TILE + (t % TILE);
}
inline size_t tiled_len(size_t n, int P) { return (n + TILE - 1) / TILE * TILE * (size_t)P; }

// XCD-aware workgroup order.  The device hands consecutive workgroups to
// its eight XCDs in turn, each with its own L2; renumbering them so that an
// XCD works through one contiguous eighth of the grid keeps the
// neighbouring rows a stencil reads in the L2 that already holds them.
__device__ inline int xcd_block(int b, int nblocks) {
  const int per = nblocks >> 3;
  if (b >= (per << 3)) return b;
  return (b & 7) * per + (b >> 3);
}

// Non-temporal load of a streamed operand (read once per kernel).
template <typename T>
__device__ inline T ldnt(const T* p) {
  return __builtin_nontemporal_load(p);
}

inline Lay make_lay(int nx, int ny, int nz, bool want_cs) {
  Lay L;
  L.nx = nx; L.ny = ny; L.nz = nz;
  L.n = nx * ny * nz;
  L.cs = (want_cs && (nx % 2 == 0)) ? 1 : 0;
  L.half = L.cs ? nx / 2 : 0;
  L.nh = L.cs ? L.n / 2 : 0;
  L.nxr = nx;
  return L;
}

// Colour-split layout of a grid with nxr real columns: an odd nxr gets one
// ghost column (see the storage notes at the top of this file).
inline Lay make_padded_lay(int nxr, int ny, int nz) {
  Lay L = make_lay(nxr + (nxr & 1), ny, nz, true);
  L.nxr = nxr;
  return L;
}

// Cells of the real grid of a layout.
inline long lay_real_cells(const Lay& L) { return (long)L.nxr * L.ny * L.nz; }

// Fluid description passed to kernels by value.
struct FluidDev {
  int model;  // 2 oil-water, 3 black oil
  int npvt;
  double p_ref, rho_w_ref, rho_o_ref, rho_o_sc, rho_g_sc;
  double c_w, c_o, c_r, mu_w, mu_o;
  double s_wc, s_or, sg_den;
  double pvt[6][CPR_MAX_PVT];
};

struct Perf {     // one perforated cell of a well
  int cell;       // colour-split index
  int kind;       // CPR_WELL_INJECTOR / CPR_WELL_PRODUCER
  int rw;         // index of its rate-controlled well, -1 for a BHP well
  double wi;      // Peaceman index (m^3)
  double bhp;     // bar (BHP wells)
  double dzh;     // z_h - z (m): reference depth minus cell depth
};

struct RateWell {     // a rate-controlled well: its perforations are perfs[p0, p1)
  int p0, p1;
  int comp;           // controlled component row (water for injectors, oil for producers)
  double target;      // signed target mass rate (kg/s): +injection, -production
};

struct MGLevel {
  Lay lay;
  double* A = nullptr;   // [7][n]
  float* Af = nullptr;   // FP32 copy for the mixed-precision preconditioner
  double* x = nullptr;   // correction
  double* r = nullptr;   // right-hand side
  float* xf = nullptr;
  float* rf = nullptr;
  double* res = nullptr; // black-cell residuals after the black pre-smoothing sweep [n/2]
  float* resf = nullptr;
};

// Phase timers (timing.hip): one event pair per outer phase and a ring of
// pairs for the inner phases of a solve (which do not nest), harvested in
// order wherever the host already waits for the device.
enum { PH_ASSEMBLE = 0, PH_SETUP = 1, PH_SOLVE = 2, PH_OUTER = 3 };
enum { PH_PRECOND = 0, PH_SPMV = 1, PH_ORTH = 2, PH_INNER = 3 };
struct PhaseTimer {
  bool on = false;
  hipEvent_t outer[PH_OUTER][2] = {};
  bool outer_pending[PH_OUTER] = {};
  double outer_ms[PH_OUTER] = {};
  std::vector<hipEvent_t> ring;   // 2 * RING events
  std::vector<int> kind;          // RING phase ids
  int head = 0, count = 0;        // oldest recorded pair, pairs outstanding
  bool open = false;              // an inner pair has begun and not ended
  double inner_ms[PH_INNER] = {};
};

struct cpr_ctx {
  std::string err;
  DevAlloc mem;                // device allocator taken at creation
  hipStream_t stream = nullptr;
  // setup runs the Galerkin chain and the coarsest inverse on a second
  // stream (default priority) while the ILU factorisation runs on `stream`
  hipStream_t aux = nullptr;
  hipEvent_t ev_q = nullptr, ev_rap = nullptr, ev_gj = nullptr;
  hipEvent_t ev_iter[2] = {nullptr, nullptr};   // completion of Arnoldi steps (even, odd)
  // set by FGMRES when a restart cycle with the FP32 preconditioner or the
  // learned stage stalls: the rest of that solve applies plain FP64 CPR
  bool fp64_now = false;
  cpr_grid_t grid;
  FluidDev fl;
  int b = 0;
  Lay lay;
  double phibar = 0.0;
  double cell_vol = 0.0;
  double rho_scale[3] = {0, 0, 0};  // component densities for the row scaling

  // rock (colour-split)
  double* poro = nullptr;      // [n]
  double* tp = nullptr;        // [3][n] transmissibility to the +x/+y/+z neighbour
  std::vector<Perf> perfs;
  Perf* perfs_d = nullptr;
  // rate-controlled wells: BHP unknowns appended to every vector
  int nrate = 0;
  std::vector<RateWell> rwells;
  RateWell* rwells_d = nullptr;
  double* bord = nullptr;      // [nperf][2][3]: dR_cell/dp_h (B) and dR_w/dx_cell (C) per perforation
  double* pq = nullptr;        // [nperf][2]: controlled-component mass rate and d/dp_h (unscaled)
  double* bord_d = nullptr;    // [nrate] dR_w/dp_h (D)

  // Jacobian and assembly scratch (colour-split)
  double* J = nullptr;         // [7][b][b] planes of n cells, tiled
  double* props = nullptr;     // per-cell phase/mobility state for the flux kernel
  double* vin = nullptr;       // [b][n] input permutation scratch
  double* vin2 = nullptr;      // [b][n]
  double* vout = nullptr;      // [b][n]

  // CPR setup (colour-split)
  cpr_options_t opt;
  int setup_done = 0;
  double* w = nullptr;         // [b][n]   quasi-IMPES weights
  double* R0 = nullptr;        // [7][b] planes, tiled: row 0 of the decoupled blocks
  double* Wabf = nullptr;      // [b][b][n] ABF decoupling D_i^-1
  double* Jt = nullptr;        // [7][b][b] planes, tiled: ABF decoupled blocks (rows >= 1; row 0 in R0)
  double* Rt = nullptr;        // [b][n] decoupled residual (ABF / FPF)
  float* Rtf = nullptr;
  double* Z1 = nullptr;        // [b][n] first ILU stage of CPR-FPF
  float* Z1f = nullptr;
  double* Dinv = nullptr;      // [b][b] planes, tiled: inverted ILU diagonals
  float* Jf = nullptr;         // FP32 copy of the decoupled blocks, [7][b][b] planes, tiled
  float* Dinvf = nullptr;
  std::vector<MGLevel> levels;
  double* cinv = nullptr;      // dense inverse of the coarsest level (column major)
  float* cinvf = nullptr;
  double* gj_work = nullptr;   // Gauss-Jordan workspace
  int* flag = nullptr;         // device status flag (singular / non-finite)
  int qimpes_bad = 0;

  // Krylov workspace (colour-split)
  int mcap = 0;                // restart capacity of V / Z
  double* V = nullptr;         // [m+1][b*n]
  double* Z = nullptr;         // [m][b*n]
  double* Y = nullptr;         // [b][n] ILU forward result
  double* rp = nullptr;        // [n] decoupled pressure residual
  double* xs = nullptr;        // [b][n] solution (colour-split)
  double* rs = nullptr;        // [b][n] right-hand side (colour-split)
  double* tmp = nullptr;       // [b][n]
  float* vf = nullptr;         // [b][n] FP32 preconditioner input
  float* zf = nullptr;         // [b][n] FP32 preconditioner output
  float* Yf = nullptr;
  float* rpf = nullptr;
  double* part = nullptr;      // reduction partials [64][nblk]
  double* hdev = nullptr;      // [4*64] device Hessenberg scratch
  double* hhost = nullptr;     // pinned host mirror
  double* hhost_dev = nullptr; // its device address (kernels write the Hessenberg column there)
  int nblk = 0;

  // kernel-duration sampling (one kernel class at a time)
  // learned pressure correction
  struct cpr_nn* nn = nullptr;  // inference network on this grid (batch 1)
  double* lnk = nullptr;       // [n] ln kx (colour-split)
  double* rprime = nullptr;    // [n] pressure residual after the V-cycle
  double* qbuf = nullptr;      // [n] A_p d
  float* feat = nullptr;       // [n][3] network input, natural order
  double* nnscal = nullptr;    // device scalars: feature statistics, norms
  int* nncount = nullptr;      // [2] accepted / rejected corrections
  int assembled = 0;           // a Jacobian was assembled (mobility plane valid)
  // learned stage on a coarse multigrid level (options.nn_level >= 1)
  std::vector<float> theta;    // the attached parameters (host copy)
  struct cpr_nn* nn_lv = nullptr;  // network on that level's grid
  int nn_lv_dims[3] = {0, 0, 0};
  double* lnk_l = nullptr;     // [n_l] mean ln kx over each coarse cell's fine block (level layout)
  double* lt_l = nullptr;      // [n_l] exp(mean ln lambda_t) over the same block
  size_t lvl_cap = 0;          // cells allocated in lnk_l / lt_l

  int prof_class = -1;
  std::vector<hipEvent_t> ev;  // start/stop pairs
  int ev_used = 0;

  PhaseTimer pt;
};

// Bracket one launch of kernel class `k` with HIP events when it is sampled.
inline void prof_begin(cpr_ctx* ctx, int k) {
  if (ctx->prof_class == k && 2 * ctx->ev_used + 1 < (int)ctx->ev.size())
    (void)hipEventRecord(ctx->ev[2 * ctx->ev_used], ctx->stream);
}
inline void prof_end(cpr_ctx* ctx, int k) {
  if (ctx->prof_class == k && 2 * ctx->ev_used + 1 < (int)ctx->ev.size()) {
    (void)hipEventRecord(ctx->ev[2 * ctx->ev_used + 1], ctx->stream);
    ctx->ev_used += 1;
  }
}

// Phase timers and roctx ranges (timing.hip).
int phase_timing_enable(cpr_ctx* ctx, bool on);
void phase_timing_release(cpr_ctx* ctx);
void ph_outer_begin(cpr_ctx* ctx, int k);
void ph_outer_end(cpr_ctx* ctx, int k);
bool ph_begin(cpr_ctx* ctx, int k);
void ph_end(cpr_ctx* ctx);
void ph_harvest(cpr_ctx* ctx, bool wait);
void ph_solve_start(cpr_ctx* ctx);
void ph_fill_stats(cpr_ctx* ctx, cpr_stats_t* st);
void trace_push(const char* name);
void trace_pop();
// A roctx range over one scope.
struct TraceRange {
  explicit TraceRange(const char* name) { trace_push(name); }
  ~TraceRange() { trace_pop(); }
};
// One inner phase over one scope.
struct PhaseScope {
  cpr_ctx* c;
  bool opened;
  PhaseScope(cpr_ctx* ctx, int k) : c(ctx), opened(ph_begin(ctx, k)) {}
  ~PhaseScope() {
    if (opened) ph_end(c);
  }
};

// ---------------------------------------------------------------- helpers
#define CPR_TRY(expr)                                                         \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess) return set_hip_err(ctx, e_, #expr);                 \
  } while (0)

int set_err(cpr_ctx* ctx, int code, const std::string& msg);
int set_hip_err(cpr_ctx* ctx, hipError_t e, const char* what);
int launch_check(cpr_ctx* ctx, const char* what);

inline int div_up(long a, long b) { return (int)((a + b - 1) / b); }

// Length of a state / Krylov vector: the cell unknowns and the BHPs of the
// rate-controlled wells.
inline long vec_len(const cpr_ctx* c) { return (long)c->b * c->lay.n + c->nrate; }

// ---------------------------------------------------------------- launchers
// layout.hip
void launch_nat_to_cs(const Lay& L, int planes, const double* src, double* dst, hipStream_t s);
void launch_cs_to_nat(const Lay& L, int planes, const double* src, double* dst, hipStream_t s);
// The same permutations between natural-order planes and a tiled block array.
void launch_nat_to_tiled(const Lay& L, int planes, const double* src, double* dst, hipStream_t s);
void launch_tiled_to_nat(const Lay& L, int planes, const double* src, double* dst, hipStream_t s);

// assemble.hip
void launch_transmissibility(const Lay& L, const cpr_grid_t& g, const double* perm_nat,
                             double* tp, hipStream_t s);
void launch_assemble(cpr_ctx* ctx, const double* xold_cs, const double* x_cs, double dt_days,
                     double* rhs_cs);
double host_pvt(const FluidDev& f, int row, double p);
int props_planes(int model);

// spmv.hip
void launch_spmv(int b, const Lay& L, const double* A, const double* x, double* y,
                 const double* rhs, hipStream_t s);
// y = A x (or rhs - A x) for the whole system: the block stencil and, with
// rate-controlled wells, their border (eq. (16)).
void system_spmv(cpr_ctx* ctx, const double* x, double* y, const double* rhs);
// Well part of a preconditioner application: z_w = (v_w - C z_cells) / D,
// normalising v_w = vin_w / sqrt(*nrm2) first when nrm2 is given.
void border_precond(cpr_ctx* ctx, const double* vin, double* v, const double* nrm2, double* z);
// Natural <-> colour-split order of a whole vector (cells, then the BHP tail).
hipError_t vec_nat_to_cs(cpr_ctx* ctx, const double* src, double* dst);
hipError_t vec_cs_to_nat(cpr_ctx* ctx, const double* src, double* dst);

// setup.hip
int setup_cpr(cpr_ctx* ctx);

// apply.hip
// z = M^-1 v.  If nrm2 (device) is given, vin holds an unnormalised Krylov
// vector: v = vin / sqrt(*nrm2) is formed and stored on the way (vin may
// equal v).  Otherwise v must equal vin.
void precond_apply(cpr_ctx* ctx, const double* vin, double* v, const double* nrm2, double* z);

void precond_pressure_stage(cpr_ctx* ctx, const double* v);

// learned.hip
int learned_setup(cpr_ctx* ctx, bool need_nn);
int learned_stage(cpr_ctx* ctx);
// The learned stage inside the V-cycle on multigrid level `level` (>= 1).
int learned_stage_at(cpr_ctx* ctx, int level);
// First multigrid level that the V-cycle smooths inside its single-workgroup
// kernel (levels.size() when there is none).
int vcycle_fused_level(const cpr_ctx* ctx);
void learned_discard_last(cpr_ctx* ctx);
void learned_rprime(cpr_ctx* ctx);
void learned_features_from_rprime(cpr_ctx* ctx);
void launch_lnk(const Lay& L, const double* perm_nat, double* lnk, hipStream_t s);

// capi.hip
int setup_with_options(cpr_ctx* ctx, const cpr_options_t& opt);
int ensure_krylov_capacity(cpr_ctx* ctx, int m);

// newton.hip
int time_step(cpr_ctx* ctx, const double* xold_cs, double* x_cs, double dt_days, const cpr_options_t& lin,
              const cpr_newton_options_t& no, cpr_newton_stats_t* st);

// krylov.hip
// The preconditioner runs in FP32: MIXED precision and no FP64 fallback.
inline bool precond_fp32(const cpr_ctx* c) { return c->opt.precision == CPR_PREC_MIXED && !c->fp64_now; }
// The learned stage runs: requested, and no stalled cycle has handed the
// solve to plain FP64 CPR.
inline bool learned_on(const cpr_ctx* c) { return c->opt.learned && !c->fp64_now; }

int fgmres_solve(cpr_ctx* ctx, cpr_stats_t* st);
int bicgstab_solve(cpr_ctx* ctx, cpr_stats_t* st);
void launch_newton_update(int b, int n, int nrate, double pb_min, double* x, const double* dx, hipStream_t s);
// Bubble-point floor of the black-oil update: the first PVT pressure node.
inline double pb_floor(const FluidDev& f) { return f.model == 3 ? f.pvt[0][0] : 0.0; }
int reduce_dot(cpr_ctx* ctx, const double* a, const double* b, long len, double* out);
