// Phase timers and roctx ranges (measurement; not part of the method).
//
// Outer phases (assembly, setup, a solve) get one event pair each; the inner
// phases of a solve (preconditioner, SpMV, orthogonalisation) alternate
// without nesting, so their pairs go into a ring in launch order and are read
// back oldest first, without blocking, wherever the solver already waits for
// the device (and with blocking once the solve is done).  Event records are
// the only cost on the solve's path.
#include <rocprofiler-sdk-roctx/roctx.h>

#include "internal.h"

namespace {
constexpr int RING = 256;   // inner pairs outstanding at most (a few Krylov steps' worth)
}

void trace_push(const char* name) { (void)roctxRangePushA(name); }
void trace_pop() { (void)roctxRangePop(); }

void phase_timing_release(cpr_ctx* ctx) {
  PhaseTimer& T = ctx->pt;
  for (auto& pr : T.outer)
    for (hipEvent_t& e : pr)
      if (e) { (void)hipEventDestroy(e); e = nullptr; }
  for (hipEvent_t e : T.ring) (void)hipEventDestroy(e);
  T.ring.clear();
  T.kind.clear();
  T.on = false;
  T.head = T.count = 0;
  T.open = false;
}

int phase_timing_enable(cpr_ctx* ctx, bool on) {
  PhaseTimer& T = ctx->pt;
  if (on && T.ring.empty()) {
    for (auto& pr : T.outer)
      for (hipEvent_t& e : pr) CPR_TRY(hipEventCreate(&e));
    T.ring.resize(2 * RING);
    for (hipEvent_t& e : T.ring) CPR_TRY(hipEventCreate(&e));
    T.kind.assign(RING, 0);
  }
  if (!on) ph_harvest(ctx, true);
  T.on = on;
  for (int k = 0; k < PH_OUTER; ++k) { T.outer_pending[k] = false; T.outer_ms[k] = 0.0; }
  for (double& v : T.inner_ms) v = 0.0;
  T.head = T.count = 0;
  T.open = false;
  return CPR_OK;
}

void ph_outer_begin(cpr_ctx* ctx, int k) {
  PhaseTimer& T = ctx->pt;
  if (!T.on) return;
  (void)hipEventRecord(T.outer[k][0], ctx->stream);
  T.outer_pending[k] = false;
}

void ph_outer_end(cpr_ctx* ctx, int k) {
  PhaseTimer& T = ctx->pt;
  if (!T.on) return;
  (void)hipEventRecord(T.outer[k][1], ctx->stream);
  T.outer_pending[k] = true;
}

// Fold the pending outer time of phase k into outer_ms (waits for its end).
static void outer_read(cpr_ctx* ctx, int k) {
  PhaseTimer& T = ctx->pt;
  if (!T.on || !T.outer_pending[k]) return;
  float ms = 0.f;
  if (hipEventSynchronize(T.outer[k][1]) == hipSuccess &&
      hipEventElapsedTime(&ms, T.outer[k][0], T.outer[k][1]) == hipSuccess)
    T.outer_ms[k] = ms;
  T.outer_pending[k] = false;
}

void ph_harvest(cpr_ctx* ctx, bool wait) {
  PhaseTimer& T = ctx->pt;
  while (T.count > 0) {
    const int q = T.head;
    hipEvent_t e1 = T.ring[2 * q + 1];
    if (wait) {
      if (hipEventSynchronize(e1) != hipSuccess) break;
    } else if (hipEventQuery(e1) != hipSuccess) {
      break;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, T.ring[2 * q], e1) == hipSuccess) T.inner_ms[T.kind[q]] += ms;
    T.head = (T.head + 1) % RING;
    T.count -= 1;
  }
}

// Opens an inner pair unless timing is off or one is already open (a phase
// inside another is counted in the outer one); true when it opened one.
bool ph_begin(cpr_ctx* ctx, int k) {
  PhaseTimer& T = ctx->pt;
  if (!T.on || T.open) return false;
  if (T.count == RING) ph_harvest(ctx, true);
  if (T.count == RING) return false;   // an event failed: leave this launch untimed
  const int q = (T.head + T.count) % RING;
  T.kind[q] = k;
  (void)hipEventRecord(T.ring[2 * q], ctx->stream);
  T.open = true;
  return true;
}

void ph_end(cpr_ctx* ctx) {
  PhaseTimer& T = ctx->pt;
  if (!T.on || !T.open) return;
  const int q = (T.head + T.count) % RING;
  (void)hipEventRecord(T.ring[2 * q + 1], ctx->stream);
  T.count += 1;
  T.open = false;
}

void ph_solve_start(cpr_ctx* ctx) {
  PhaseTimer& T = ctx->pt;
  if (!T.on) return;
  ph_harvest(ctx, true);
  for (double& v : T.inner_ms) v = 0.0;
  ph_outer_begin(ctx, PH_SOLVE);
}

void ph_fill_stats(cpr_ctx* ctx, cpr_stats_t* st) {
  PhaseTimer& T = ctx->pt;
  if (!T.on) return;
  ph_outer_end(ctx, PH_SOLVE);
  for (int k = 0; k < PH_OUTER; ++k) outer_read(ctx, k);
  ph_harvest(ctx, true);
  if (!st) return;
  st->ms_assemble = T.outer_ms[PH_ASSEMBLE];
  st->ms_setup = T.outer_ms[PH_SETUP];
  st->ms_solve = T.outer_ms[PH_SOLVE];
  st->ms_precond = T.inner_ms[PH_PRECOND];
  st->ms_spmv = T.inner_ms[PH_SPMV];
  st->ms_orth = T.inner_ms[PH_ORTH];
}
