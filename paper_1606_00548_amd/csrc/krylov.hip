// Restarted flexible GMRES with classical Gram-Schmidt twice (CGS2),
// right-preconditioned by CPR; stops when ||b - A dx|| <= rtol ||b||
// (eq. (13) with a fixed forcing term).
//
// Device side: the Krylov basis V[m+1][b*n] and the preconditioned
// directions Z[m][b*n] stay in HBM; every reduction is a deterministic two-
// stage sum (fixed per-block partials, then a fixed-order tree), so two runs
// give identical bits.  Host side: the Givens rotations and the small
// least-squares problem; the reductions of the Hessenberg column also write
// it to pinned host memory, and one stream synchronisation per iteration is
// the only one in the loop.
//
// Per Arnoldi step j, CGS2 (options.orth = CPR_ORTH_CGS2; nv = j+1):
//   z_j = M^-1 v_j ; w = A z_j            -> written into V[j+1]
//   h  = V^T w  (partials, reduce)
//   w -= V h, h' = V^T w (fused: each block updates its slice, then dots it)
//   w -= V h', ||w||^2 (fused)
//   h_{j+1,j} = ||w||; v_{j+1} = w / h_{j+1,j}
// Delayed CGS2 (the default): the second pass of each vector is done in the
// next step, from the same inner products as that step's projection, so V
// is read twice per step instead of three times.  Slot j holds uh_j, the
// once-projected vector of step j-1 scaled to unit norm (the
// preconditioner's first kernel scales it), w lands in slot j+1:
//   dots:   a = V_j^T uh_j, c = V_j^T w, d = uh_j . w, e = uh_j . uh_j
//   coef:   beta = sqrt(e - |a|^2), g = (d - a.c) / beta (one block)
//   update: v_j = (uh_j - V_j a) / beta over slot j; u = w - V_j c - g v_j
//           over slot j+1, with ||u||^2
// (V_j: the j final vectors before slot j).  The host adds nu_j a to column
// j-1 of the Hessenberg matrix, sets its entry (j, j-1) to nu_j beta,
// writes column j (c, g, nu_{j+1} = ||u||) and recomputes the Givens QR.
#include <cmath>
#include <vector>

#include "internal.h"

namespace {

constexpr int KB = 256;        // threads per block of the vector kernels
constexpr int CHUNK = 8;       // basis vectors handled per pass
constexpr double BREAKDOWN = 1e-14;
constexpr double SPECULATE = 10.0;   // run ahead while the residual estimate exceeds 10 x the tolerance

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Block-reduce CHUNK values; thread 0 of the block gets the totals in out.
__device__ inline void block_sum_chunk(double (&acc)[CHUNK], int cnt, double* sh, double* out) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < CHUNK; ++q) {
    if (q < cnt) {
      double v = wave_sum(acc[q]);
      if (lane == 0) sh[q * (KB / 64) + wid] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x < cnt) {
    double s = 0.0;
    for (int w = 0; w < KB / 64; ++w) s += sh[threadIdx.x * (KB / 64) + w];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// part[k][block] = sum over this block's slice of V_k . w, k < nv.
// If h != nullptr, first w -= sum_k hprev[k] V_k on the slice (and store w).
// If nrm != nullptr, also part[nv][block] = slice of ||w||^2 (after update).
__global__ __launch_bounds__(KB) void orth_kernel(long len, int nv, const double* __restrict__ V,
                                                  size_t stride, double* __restrict__ w,
                                                  const double* __restrict__ hprev, int do_dots,
                                                  int do_norm, double* __restrict__ part, int nblk) {
  __shared__ double sh[CHUNK * (KB / 64)];
  __shared__ double tot[CHUNK];
  __shared__ double hs[64];
  if (hprev && threadIdx.x < nv) hs[threadIdx.x] = hprev[threadIdx.x];
  __syncthreads();
  // this block's contiguous slice
  long per = (len + nblk - 1) / nblk;
  long beg = (long)blockIdx.x * per;
  long end = beg + per < len ? beg + per : len;
  if (hprev) {
    for (long e = beg + threadIdx.x; e < end; e += KB) {
      double x = w[e];
      for (int k = 0; k < nv; ++k) x -= hs[k] * V[k * stride + e];
      w[e] = x;
    }
    // the same thread re-reads only the elements it wrote: no block barrier needed
  }
  if (do_dots) {
    for (int k0 = 0; k0 < nv; k0 += CHUNK) {
      int cnt = nv - k0 < CHUNK ? nv - k0 : CHUNK;
      double acc[CHUNK];
#pragma unroll
      for (int q = 0; q < CHUNK; ++q) acc[q] = 0.0;
      for (long e = beg + threadIdx.x; e < end; e += KB) {
        double x = w[e];
#pragma unroll
        for (int q = 0; q < CHUNK; ++q)
          if (q < cnt) acc[q] += V[(k0 + q) * stride + e] * x;
      }
      block_sum_chunk(acc, cnt, sh, tot);
      if (threadIdx.x < cnt) part[(size_t)(k0 + threadIdx.x) * nblk + blockIdx.x] = tot[threadIdx.x];
    }
  }
  if (do_norm) {
    double acc[CHUNK];
#pragma unroll
    for (int q = 0; q < CHUNK; ++q) acc[q] = 0.0;
    for (long e = beg + threadIdx.x; e < end; e += KB) {
      double x = w[e];
      acc[0] += x * x;
    }
    block_sum_chunk(acc, 1, sh, tot);
    if (threadIdx.x == 0) part[(size_t)nv * nblk + blockIdx.x] = tot[0];
  }
}

// out[k] (+)= sum_b part[k][b], one block per k, fixed order; host (pinned
// host memory, optional) receives the same value and bare (optional) the
// sum without the added term.
__global__ __launch_bounds__(KB) void reduce_kernel(const double* __restrict__ part, int nblk,
                                                    double* __restrict__ out, const double* __restrict__ add,
                                                    double* __restrict__ host = nullptr,
                                                    double* __restrict__ bare = nullptr) {
  __shared__ double sh[CHUNK * (KB / 64)];
  __shared__ double tot[CHUNK];
  int k = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += KB) s += part[(size_t)k * nblk + b];
  double acc[CHUNK];
#pragma unroll
  for (int q = 0; q < CHUNK; ++q) acc[q] = 0.0;
  acc[0] = s;
  block_sum_chunk(acc, 1, sh, tot);
  if (threadIdx.x == 0) {
    const double v = tot[0] + (add ? add[k] : 0.0);
    out[k] = v;
    if (host) host[k] = v;
    if (bare) bare[k] = tot[0];
  }
}

// One CGS2 pass over the first nv basis vectors, register-blocked so that
// every element of V is read once: optionally w -= sum_k hprev[k] V_k, then
// either the partial dots V_k . w (mode 0) or the partial ||w||^2 (mode 1)
// of this block's slice.
template <int NV>
__global__ __launch_bounds__(KB) void orth_fused_kernel(long len, int nv, const double* __restrict__ V,
                                                        size_t stride, double* __restrict__ w,
                                                        const double* __restrict__ hprev, int mode,
                                                        double* __restrict__ part, int nblk) {
  __shared__ double sh[NV * (KB / 64)];
  __shared__ double hs[NV];
  if (hprev && threadIdx.x < nv) hs[threadIdx.x] = hprev[threadIdx.x];
  __syncthreads();
  long per = (len + nblk - 1) / nblk;
  long beg = (long)blockIdx.x * per;
  long end = beg + per < len ? beg + per : len;
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  for (long e = beg + threadIdx.x; e < end; e += KB) {
    double vv[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) vv[k] = k < nv && (hprev || mode == 0) ? V[k * stride + e] : 0.0;
    double x = w[e];
    if (hprev) {
#pragma unroll
      for (int k = 0; k < NV; ++k)
        if (k < nv) x -= hs[k] * vv[k];
      w[e] = x;
    }
    if (mode == 0) {
#pragma unroll
      for (int k = 0; k < NV; ++k)
        if (k < nv) acc[k] += vv[k] * x;
    } else {
      acc[0] += x * x;
    }
  }
  const int cnt = mode == 0 ? nv : 1;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    if (k < cnt) {
      double v = wave_sum(acc[k]);
      if (lane == 0) sh[k * (KB / 64) + wid] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x < cnt) {
    double s = 0.0;
    for (int q = 0; q < KB / 64; ++q) s += sh[threadIdx.x * (KB / 64) + q];
    int row = mode == 0 ? threadIdx.x : nv;
    part[(size_t)row * nblk + blockIdx.x] = s;
  }
}

// Delayed CGS2, dot pass of step j (j <= NV final vectors before slot j):
// part rows 0..j-1 = V_k . uh, rows j..2j-1 = V_k . w, row 2j = uh . w,
// row 2j+1 = uh . uh, each the sum over this block's slice.
template <int NV>
__global__ __launch_bounds__(KB) void dcgs_dots_kernel(long len, int j, const double* __restrict__ V, size_t stride,
                                                       const double* __restrict__ uh, const double* __restrict__ w,
                                                       double* __restrict__ part, int nblk) {
  __shared__ double sh[(2 * NV + 2) * (KB / 64)];
  long per = (len + nblk - 1) / nblk;
  long beg = (long)blockIdx.x * per;
  long end = beg + per < len ? beg + per : len;
  double aa[NV], cc[NV], dd = 0.0, ee = 0.0;
#pragma unroll
  for (int k = 0; k < NV; ++k) aa[k] = cc[k] = 0.0;
  for (long e = beg + threadIdx.x; e < end; e += KB) {
    // every basis load issued before the arithmetic (vectors past j read as 0)
    double vv[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) vv[k] = k < j ? ldnt(V + k * stride + e) : 0.0;
    const double u = uh[e], x = w[e];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      aa[k] += vv[k] * u;
      cc[k] += vv[k] * x;
    }
    dd += u * x;
    ee += u * u;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int rows = 2 * j + 2;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    if (k < j) {
      double v = wave_sum(aa[k]);
      if (lane == 0) sh[k * (KB / 64) + wid] = v;
      v = wave_sum(cc[k]);
      if (lane == 0) sh[(j + k) * (KB / 64) + wid] = v;
    }
  }
  {
    double v = wave_sum(dd);
    if (lane == 0) sh[(2 * j) * (KB / 64) + wid] = v;
    v = wave_sum(ee);
    if (lane == 0) sh[(2 * j + 1) * (KB / 64) + wid] = v;
  }
  __syncthreads();
  if (threadIdx.x < rows) {
    double t = 0.0;
    for (int q = 0; q < KB / 64; ++q) t += sh[threadIdx.x * (KB / 64) + q];
    part[(size_t)threadIdx.x * nblk + blockIdx.x] = t;
  }
}

// Offsets of the delayed CGS2 scalars: in the device scratch hdev (dots,
// update coefficients, ||u||^2) and in each of the two pinned host slots.
enum { D_DOTS = 384, D_COEF = 512, D_NRM = 640, D_HOST = 512, D_SLOT = 256 };
enum { C_A = 0, C_C = 32, C_INVB = 64, C_G = 65 };                       // in D_COEF
enum { S_A = 0, S_C = 32, S_BETA = 64, S_G = 65, S_NRM = 66, S_FLAG = 67 };   // in a host slot

// The scalars of step j from its reduced dots (one thread, fixed order):
// beta = sqrt(e - |a|^2) (1 at step 0, which has no vector to
// reorthogonalise) and g = (d - a.c) / beta; flag = 1 when beta^2 <= 0.
__global__ void dcgs_coef_kernel(int j, const double* __restrict__ dots, double* __restrict__ coef,
                                 double* __restrict__ host) {
  for (int i = threadIdx.x; i < j; i += blockDim.x) {
    coef[C_A + i] = dots[i];
    coef[C_C + i] = dots[j + i];
    host[S_A + i] = dots[i];
    host[S_C + i] = dots[j + i];
  }
  if (threadIdx.x != 0) return;
  double aa = 0.0, ac = 0.0;
  for (int i = 0; i < j; ++i) {
    aa += dots[i] * dots[i];
    ac += dots[i] * dots[j + i];
  }
  const double d = dots[2 * j], e = dots[2 * j + 1];
  const double b2 = j == 0 ? 1.0 : e - aa;
  const bool bad = !(b2 > 0.0);
  const double beta = bad ? 0.0 : sqrt(b2);
  const double g = j == 0 ? d : (bad ? 0.0 : (d - ac) / beta);
  coef[C_INVB] = bad ? 0.0 : 1.0 / beta;
  coef[C_G] = g;
  host[S_BETA] = beta;
  host[S_G] = g;
  host[S_FLAG] = bad ? 1.0 : 0.0;
}

// Delayed CGS2, update pass of step j: v_j = (uh - V a) / beta over uh,
// u = w - V c - g v_j over w, and part row 0 = this slice of ||u||^2.
template <int NV>
__global__ __launch_bounds__(KB) void dcgs_update_kernel(long len, int j, const double* __restrict__ V, size_t stride,
                                                         double* __restrict__ uh, double* __restrict__ w,
                                                         const double* __restrict__ coef, double* __restrict__ part,
                                                         int nblk) {
  __shared__ double cs[2 * NV + 2];
  __shared__ double sh[KB / 64];
  for (int i = threadIdx.x; i < NV; i += KB) {
    cs[i] = i < j ? coef[C_A + i] : 0.0;
    cs[NV + i] = i < j ? coef[C_C + i] : 0.0;
  }
  if (threadIdx.x == 0) {
    cs[2 * NV] = coef[C_INVB];
    cs[2 * NV + 1] = coef[C_G];
  }
  __syncthreads();
  const double invb = cs[2 * NV], g = cs[2 * NV + 1];
  long per = (len + nblk - 1) / nblk;
  long beg = (long)blockIdx.x * per;
  long end = beg + per < len ? beg + per : len;
  double acc = 0.0;
  for (long e = beg + threadIdx.x; e < end; e += KB) {
    double vv[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) vv[k] = k < j ? ldnt(V + k * stride + e) : 0.0;
    double va = uh[e], wa = w[e];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      va -= cs[k] * vv[k];
      wa -= cs[NV + k] * vv[k];
    }
    va *= invb;
    wa -= g * va;
    uh[e] = va;
    w[e] = wa;
    acc += wa * wa;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double v = wave_sum(acc);
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < KB / 64; ++q) t += sh[q];
    part[blockIdx.x] = t;
  }
}

__global__ void scale_kernel(long len, double a, const double* __restrict__ x, double* __restrict__ y) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < len) y[e] = x[e] / a;
}

// x += sum_k y[k] Z_k
__global__ void maxpy_kernel(long len, int nk, const double* __restrict__ Z, size_t stride,
                             const double* __restrict__ y, double* __restrict__ x) {
  __shared__ double ys[64];
  if (threadIdx.x < nk) ys[threadIdx.x] = y[threadIdx.x];
  __syncthreads();
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  double s = x[e];
  for (int k = 0; k < nk; ++k) s += ys[k] * Z[k * stride + e];
  x[e] = s;
}

__global__ void zero_kernel(long len, double* __restrict__ x) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < len) x[e] = 0.0;
}

// Newton update: x += dx, saturation changes chopped to |dS| <= 0.2,
// saturations clamped to [0, 1].  Black oil (b = 3) switches its third
// unknown with the phase state: a saturated cell (x2 = S_g >= 0) whose gas
// would go negative becomes undersaturated at its bubble point, x2 = -p
// (updated p); an undersaturated cell (x2 = -p_b) whose bubble point rises
// above the updated pressure becomes saturated with S_g = 0; otherwise p_b
// (unchopped) is floored at pb_min.
__global__ void newton_update_kernel(int b, int n, int nrate, double pb_min, double* __restrict__ x,
                                     const double* __restrict__ dx) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nrate) x[(size_t)b * n + t] += dx[(size_t)b * n + t];   // rate wells' BHPs, unchopped
  if (t >= n) return;
  const double p = x[t] + dx[t];
  x[t] = p;
  for (int s = 1; s < b; ++s) {
    size_t o = (size_t)s * n + t;
    double d = dx[o];
    double dc = d < -0.2 ? -0.2 : (d > 0.2 ? 0.2 : d);
    double v = x[o] + dc;
    if (s == 2) {
      if (x[o] >= 0.0) {
        x[o] = v >= 0.0 ? (v > 1.0 ? 1.0 : v) : -p;
      } else {
        double pb = -(x[o] + d);
        x[o] = pb > p ? 0.0 : -(pb > pb_min ? pb : pb_min);
      }
    } else {
      x[o] = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
    }
  }
}

// One orthogonalisation pass (see orth_fused_kernel); more than 32 basis
// vectors fall back to the chunked kernel, which reads V twice.
void orth_pass(cpr_ctx* ctx, long len, int nv, double* w, const double* hprev, int mode) {
  hipStream_t s = ctx->stream;
  const int nblk = ctx->nblk;
  const size_t stride = (size_t)len;
  prof_begin(ctx, CPR_KCLASS_ORTH);
  if (nv <= 8)
    orth_fused_kernel<8><<<nblk, KB, 0, s>>>(len, nv, ctx->V, stride, w, hprev, mode, ctx->part, nblk);
  else if (nv <= 16)
    orth_fused_kernel<16><<<nblk, KB, 0, s>>>(len, nv, ctx->V, stride, w, hprev, mode, ctx->part, nblk);
  else if (nv <= 32)
    orth_fused_kernel<32><<<nblk, KB, 0, s>>>(len, nv, ctx->V, stride, w, hprev, mode, ctx->part, nblk);
  else
    orth_kernel<<<nblk, KB, 0, s>>>(len, nv, ctx->V, stride, w, hprev, mode == 0, mode == 1, ctx->part, nblk);
  prof_end(ctx, CPR_KCLASS_ORTH);
}

// ------------------------------------------------------------ BiCGSTAB
// Device scalars of one BiCGSTAB iteration (ctx->hdev + 320 ...).
enum { B_RHO = 0, B_ALPHA, B_OMEGA, B_BETA, B_RV, B_TS, B_TT, B_RR, B_BRK, B_NSC };

// part rows 0 (and 1): block partials of <a0, b0> (and <a1, b1>)
__global__ __launch_bounds__(KB) void dot2_kernel(long len, const double* __restrict__ a0,
                                                  const double* __restrict__ b0, const double* __restrict__ a1,
                                                  const double* __restrict__ b1, double* __restrict__ part,
                                                  int nblk) {
  __shared__ double sh[CHUNK * (KB / 64)];
  __shared__ double tot[CHUNK];
  long per = (len + nblk - 1) / nblk;
  long beg = (long)blockIdx.x * per;
  long end = beg + per < len ? beg + per : len;
  double acc[CHUNK];
#pragma unroll
  for (int q = 0; q < CHUNK; ++q) acc[q] = 0.0;
  for (long e = beg + threadIdx.x; e < end; e += KB) {
    acc[0] += a0[e] * b0[e];
    if (a1) acc[1] += a1[e] * b1[e];
  }
  const int cnt = a1 ? 2 : 1;
  block_sum_chunk(acc, cnt, sh, tot);
  if (threadIdx.x < cnt) part[(size_t)threadIdx.x * nblk + blockIdx.x] = tot[threadIdx.x];
}

// One block sums nrows partial rows in a fixed order, then derives the
// iteration's scalars: mode 0 (after <rh, v>): alpha = rho / <rh, v>, or the
// breakdown flag; mode 1 (after <t, s>, <t, t>): omega (0 when t = 0);
// mode 2 (after <rh, r>, <r, r>): beta for the next p, rho updated, and
// ||r||^2, rho, omega, breakdown copied to pinned host memory.
__global__ __launch_bounds__(KB) void bicg_reduce_kernel(const double* __restrict__ part, int nblk, int nrows,
                                                         int mode, double* __restrict__ sc,
                                                         double* __restrict__ host) {
  __shared__ double sh[CHUNK * (KB / 64)];
  __shared__ double tot[CHUNK];
  double acc[CHUNK];
#pragma unroll
  for (int q = 0; q < CHUNK; ++q) acc[q] = 0.0;
  for (int b = threadIdx.x; b < nblk; b += KB) {
    acc[0] += part[b];
    if (nrows > 1) acc[1] += part[(size_t)nblk + b];
  }
  block_sum_chunk(acc, nrows, sh, tot);
  if (threadIdx.x != 0) return;
  if (mode == 0) {
    const double rv = tot[0];
    sc[B_RV] = rv;
    const bool bad = !(rv != 0.0) || !isfinite(rv);
    sc[B_ALPHA] = bad ? 0.0 : sc[B_RHO] / rv;
    if (bad) sc[B_BRK] = 1.0;
  } else if (mode == 1) {
    sc[B_TS] = tot[0];
    sc[B_TT] = tot[1];
    sc[B_OMEGA] = tot[1] > 0.0 ? tot[0] / tot[1] : 0.0;
  } else {
    const double rho = tot[0];
    sc[B_BETA] = (rho / sc[B_RHO]) * (sc[B_ALPHA] / sc[B_OMEGA]);
    sc[B_RHO] = rho;
    sc[B_RR] = tot[1];
    host[0] = tot[1];
    host[1] = rho;
    host[2] = sc[B_OMEGA];
    host[3] = sc[B_BRK];
  }
}

// start of a cycle: rho_prev = alpha = omega = 1 (so that p = r), no breakdown
__global__ void bicg_init_kernel(double* __restrict__ sc) {
  if (threadIdx.x == 0) {
    sc[B_RHO] = 1.0; sc[B_ALPHA] = 1.0; sc[B_OMEGA] = 1.0; sc[B_BRK] = 0.0;
  }
}

// p = r + beta (p - omega v)
__global__ void bicg_p_kernel(long len, const double* __restrict__ sc, const double* __restrict__ r,
                              const double* __restrict__ v, double* __restrict__ p) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  p[e] = r[e] + sc[B_BETA] * (p[e] - sc[B_OMEGA] * v[e]);
}

// s = r - alpha v (skipped after a breakdown)
__global__ void bicg_s_kernel(long len, const double* __restrict__ sc, const double* __restrict__ r,
                              const double* __restrict__ v, double* __restrict__ s) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len || sc[B_BRK] != 0.0) return;
  s[e] = r[e] - sc[B_ALPHA] * v[e];
}

// x += alpha ph + omega sh; r = s - omega t; block partials of <rh, r> and
// <r, r> (nothing changes after a breakdown: the partials of the old r)
__global__ __launch_bounds__(KB) void bicg_xr_kernel(long len, const double* __restrict__ sc,
                                                     const double* __restrict__ ph, const double* __restrict__ sh_,
                                                     const double* __restrict__ s, const double* __restrict__ t,
                                                     double* __restrict__ x, double* __restrict__ r,
                                                     const double* __restrict__ rh, double* __restrict__ part,
                                                     int nblk) {
  __shared__ double sh[CHUNK * (KB / 64)];
  __shared__ double tot[CHUNK];
  const bool brk = sc[B_BRK] != 0.0;
  const double al = sc[B_ALPHA], om = sc[B_OMEGA];
  long per = (len + nblk - 1) / nblk;
  long beg = (long)blockIdx.x * per;
  long end = beg + per < len ? beg + per : len;
  double acc[CHUNK];
#pragma unroll
  for (int q = 0; q < CHUNK; ++q) acc[q] = 0.0;
  for (long e = beg + threadIdx.x; e < end; e += KB) {
    double re;
    if (!brk) {
      x[e] = x[e] + al * ph[e] + om * sh_[e];
      re = s[e] - om * t[e];
      r[e] = re;
    } else {
      re = r[e];
    }
    acc[0] += rh[e] * re;
    acc[1] += re * re;
  }
  block_sum_chunk(acc, 2, sh, tot);
  if (threadIdx.x < 2) part[(size_t)threadIdx.x * nblk + blockIdx.x] = tot[threadIdx.x];
}

}  // namespace

void launch_newton_update(int b, int n, int nrate, double pb_min, double* x, const double* dx, hipStream_t s) {
  newton_update_kernel<<<div_up(n > nrate ? n : nrate, 256), 256, 0, s>>>(b, n, nrate, pb_min, x, dx);
}

// Dot product of two device vectors of length len into *out (host).  Syncs.
int reduce_dot(cpr_ctx* ctx, const double* a, const double* b, long len, double* out) {
  hipStream_t s = ctx->stream;
  // reuse the orthogonalisation kernel with V = a (one vector), w = b
  orth_kernel<<<ctx->nblk, KB, 0, s>>>(len, 1, a, 0, const_cast<double*>(b), nullptr, 1, 0, ctx->part,
                                       ctx->nblk);
  reduce_kernel<<<1, KB, 0, s>>>(ctx->part, ctx->nblk, ctx->hdev, nullptr);
  CPR_TRY(hipGetLastError());
  CPR_TRY(hipMemcpyAsync(ctx->hhost, ctx->hdev, sizeof(double), hipMemcpyDeviceToHost, s));
  CPR_TRY(hipStreamSynchronize(s));
  *out = ctx->hhost[0];
  return CPR_OK;
}

namespace {

void dcgs_dots(cpr_ctx* ctx, long len, int j, const double* uh, const double* w) {
  hipStream_t s = ctx->stream;
  const int nblk = ctx->nblk;
  const size_t stride = (size_t)len;
  prof_begin(ctx, CPR_KCLASS_ORTH);
  if (j <= 8)
    dcgs_dots_kernel<8><<<nblk, KB, 0, s>>>(len, j, ctx->V, stride, uh, w, ctx->part, nblk);
  else if (j <= 16)
    dcgs_dots_kernel<16><<<nblk, KB, 0, s>>>(len, j, ctx->V, stride, uh, w, ctx->part, nblk);
  else
    dcgs_dots_kernel<32><<<nblk, KB, 0, s>>>(len, j, ctx->V, stride, uh, w, ctx->part, nblk);
  prof_end(ctx, CPR_KCLASS_ORTH);
}

void dcgs_update(cpr_ctx* ctx, long len, int j, double* uh, double* w, const double* coef) {
  hipStream_t s = ctx->stream;
  const int nblk = ctx->nblk;
  const size_t stride = (size_t)len;
  prof_begin(ctx, CPR_KCLASS_ORTH);
  if (j <= 8)
    dcgs_update_kernel<8><<<nblk, KB, 0, s>>>(len, j, ctx->V, stride, uh, w, coef, ctx->part, nblk);
  else if (j <= 16)
    dcgs_update_kernel<16><<<nblk, KB, 0, s>>>(len, j, ctx->V, stride, uh, w, coef, ctx->part, nblk);
  else
    dcgs_update_kernel<32><<<nblk, KB, 0, s>>>(len, j, ctx->V, stride, uh, w, coef, ctx->part, nblk);
  prof_end(ctx, CPR_KCLASS_ORTH);
}

// Givens QR of the (k+1) x k Hessenberg block Hh (row stride m) into R (the
// same layout, upper triangle) and g = Q^T beta e_0.
void givens_qr(const std::vector<double>& Hh, int m, int k, double beta, std::vector<double>& R,
               std::vector<double>& g) {
  std::fill(R.begin(), R.end(), 0.0);
  for (int i = 0; i <= k; ++i)
    for (int c = 0; c < k; ++c) R[(size_t)i * m + c] = Hh[(size_t)i * m + c];
  std::fill(g.begin(), g.end(), 0.0);
  g[0] = beta;
  for (int i = 0; i < k; ++i) {
    const double a = R[(size_t)i * m + i], b = R[(size_t)(i + 1) * m + i];
    const double den = std::hypot(a, b);
    double c = 1.0, sn = 0.0;
    if (den != 0.0) { c = a / den; sn = b / den; }
    for (int col = i; col < k; ++col) {
      const double ri = R[(size_t)i * m + col], ri1 = R[(size_t)(i + 1) * m + col];
      R[(size_t)i * m + col] = c * ri + sn * ri1;
      R[(size_t)(i + 1) * m + col] = -sn * ri + c * ri1;
    }
    g[i + 1] = -sn * g[i];
    g[i] = c * g[i];
  }
}

}  // namespace

// One restart cycle of FGMRES with delayed CGS2 (slot 0 of V holds r / beta
// on entry).  On return R (row stride m) holds the triangular factor of the
// cycle's k x k least-squares problem and g its right-hand side, both from
// the corrected Hessenberg matrix; its counts the Arnoldi steps.
// Early stall check: ten steps into the first restart cycle (of m > ten),
// with the FP32 preconditioner or the learned stage in use, FGMRES's own
// residual estimate above stall_ratio^(10/m) times the initial residual
// (the cycle's bound shared out over its steps at a constant rate: 0.79 for
// the defaults) ends the cycle there, and the check after the cycle then
// hands the rest of the solve to plain FP64 CPR.  (Measured after ten
// first-cycle steps: 0.90-0.96 where the FP32 preconditioner stalls, at
// most 0.04 on the healthy forms of the bench's workloads; later cycles,
// which start from a restarted basis, are left to the check after the
// cycle.)
constexpr int STALL_EARLY = 10;
static bool early_stall(const cpr_ctx* ctx, int steps, int its, double est, double beta) {
  const int m = ctx->opt.restart;
  return steps == STALL_EARLY && its == steps && m > STALL_EARLY &&
         (ctx->opt.precision == CPR_PREC_MIXED || ctx->opt.learned) && !ctx->fp64_now &&
         ctx->opt.stall_ratio > 0 && est > std::pow(ctx->opt.stall_ratio, (double)STALL_EARLY / m) * beta;
}

int dcgs2_cycle(cpr_ctx* ctx, double beta, double bnorm, int& its, int& k, std::vector<double>& R,
                std::vector<double>& g) {
  hipStream_t s = ctx->stream;
  const long len = vec_len(ctx);
  const size_t stride = (size_t)len;
  const int m = ctx->opt.restart;
  const double rtol = ctx->opt.rtol;
  const int max_iter = ctx->opt.max_iter;
  const int nblk = ctx->nblk;
  double* hd = ctx->hdev;
  std::vector<double> Hh((size_t)(m + 1) * m, 0.0);
  auto launch_step = [&](int j) -> int {
    double* uj = ctx->V + (size_t)j * stride;
    double* zj = ctx->Z + (size_t)j * stride;
    double* w = ctx->V + (size_t)(j + 1) * stride;
    double* slot = ctx->hhost_dev + D_HOST + (j & 1) * D_SLOT;
    // slot j becomes uh_j = u_j / nu_j inside the preconditioner's first kernel
    {
      PhaseScope ps(ctx, PH_PRECOND);
      precond_apply(ctx, uj, uj, j == 0 ? nullptr : hd + D_NRM, zj);
    }
    {
      PhaseScope ps(ctx, PH_SPMV);
      prof_begin(ctx, CPR_KCLASS_SPMV);
      system_spmv(ctx, zj, w, nullptr);
      prof_end(ctx, CPR_KCLASS_SPMV);
    }
    {
      PhaseScope ps(ctx, PH_ORTH);
      dcgs_dots(ctx, len, j, uj, w);
      reduce_kernel<<<2 * j + 2, KB, 0, s>>>(ctx->part, nblk, hd + D_DOTS, nullptr);
      dcgs_coef_kernel<<<1, 64, 0, s>>>(j, hd + D_DOTS, hd + D_COEF, slot);
      dcgs_update(ctx, len, j, uj, w, hd + D_COEF);
      reduce_kernel<<<1, KB, 0, s>>>(ctx->part, nblk, hd + D_NRM, nullptr, slot + S_NRM);
    }
    CPR_TRY(hipGetLastError());
    CPR_TRY(hipEventRecord(ctx->ev_iter[j & 1], s));
    return CPR_OK;
  };
  double nu_prev = 0.0, est = beta;
  int launched = -1, rc;
  k = 0;
  for (int j = 0; j < m; ++j) {
    if (launched < j) {
      if ((rc = launch_step(j)) != CPR_OK) return rc;
      launched = j;
    }
    // run step j + 1 on the device while the host waits for step j (as in
    // the CGS2 path: only while the residual is far above the tolerance)
    if (j + 1 < m && its + 1 < max_iter && est > SPECULATE * rtol * bnorm) {
      if ((rc = launch_step(j + 1)) != CPR_OK) return rc;
      launched = j + 1;
    }
    CPR_TRY(hipEventSynchronize(ctx->ev_iter[j & 1]));
    ph_harvest(ctx, false);
    const double* sl = ctx->hhost + D_HOST + (j & 1) * D_SLOT;
    if (j > 0 && sl[S_FLAG] != 0.0) break;     // uh_j in the span of the basis: stop before step j
    its += 1;
    if (j > 0) {
      for (int i = 0; i < j; ++i) Hh[(size_t)i * m + j - 1] += nu_prev * sl[S_A + i];
      Hh[(size_t)j * m + j - 1] = nu_prev * sl[S_BETA];
    }
    for (int i = 0; i < j; ++i) Hh[(size_t)i * m + j] = sl[S_C + i];
    Hh[(size_t)j * m + j] = sl[S_G];
    const double nu = std::sqrt(sl[S_NRM]);
    Hh[(size_t)(j + 1) * m + j] = nu;
    k = j + 1;
    double az = 0.0;
    for (int i = 0; i <= j + 1; ++i) az += Hh[(size_t)i * m + j] * Hh[(size_t)i * m + j];
    az = std::sqrt(az);
    if (!std::isfinite(az)) return set_err(ctx, CPR_ENONFINITE, "non-finite Hessenberg column");
    givens_qr(Hh, m, k, beta, R, g);
    est = std::fabs(g[k]);
    if (est <= rtol * bnorm || nu <= BREAKDOWN * az || its >= max_iter) break;
    if (early_stall(ctx, k, its, est, beta)) break;
    nu_prev = nu;
  }
  if (launched >= k) {
    // a step ran ahead but the cycle ended: undo its learned-stage count
    if (learned_on(ctx)) learned_discard_last(ctx);
  }
  givens_qr(Hh, m, k, beta, R, g);
  return CPR_OK;
}

// ctx->rs holds the right-hand side, ctx->xs receives the solution
// (colour-split); with options.x0 it also holds the initial guess.
// Mirrors the oracle's FGMRES step for step.
int fgmres_solve(cpr_ctx* ctx, cpr_stats_t* st) {
  hipStream_t s = ctx->stream;
  const int b = ctx->b;
  const long len = vec_len(ctx);
  const size_t stride = (size_t)len;
  const int m = ctx->opt.restart;
  const double rtol = ctx->opt.rtol;
  const int max_iter = ctx->opt.max_iter;
  const int nblk = ctx->nblk;
  const int eb = div_up(len, 256);
  // delayed CGS2 keeps up to 32 vectors' coefficients in registers; longer
  // restarts use CGS2 (as the oracle does)
  const bool dcgs = ctx->opt.orth == CPR_ORTH_DCGS2 && m <= 32;
  double* x = ctx->xs;
  double* r = ctx->tmp;
  cpr_stats_t S = {};
  S.mg_levels = (int)ctx->levels.size();
  S.qimpes_fallback = ctx->qimpes_bad;
  // the FP64 fallback lasts for this solve only, whichever way it ends
  struct FallbackReset {
    cpr_ctx* c;
    ~FallbackReset() { c->fp64_now = false; }
  } fallback_reset{ctx};
  ctx->fp64_now = false;
  ph_solve_start(ctx);

  const bool from_x0 = ctx->opt.x0 != 0;
  if (!from_x0) zero_kernel<<<eb, 256, 0, s>>>(len, x);
  double bb;
  int rc = reduce_dot(ctx, ctx->rs, ctx->rs, len, &bb);
  if (rc) return rc;
  double bnorm = std::sqrt(bb);
  S.bnorm = bnorm;
  if (!std::isfinite(bnorm)) {
    if (st) *st = S;
    return set_err(ctx, CPR_ENONFINITE, "non-finite right-hand side");
  }
  if (bnorm == 0.0) {
    if (from_x0) zero_kernel<<<eb, 256, 0, s>>>(len, x);
    S.converged = 1;
    ph_fill_stats(ctx, &S);
    if (st) *st = S;
    return CPR_OK;
  }
  if (from_x0) {
    PhaseScope ps(ctx, PH_SPMV);
    system_spmv(ctx, x, r, ctx->rs);      // r = b - A x0
  } else {
    CPR_TRY(hipMemcpyAsync(r, ctx->rs, len * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), col(m + 1);
  int its = 0;
  int result = CPR_NOT_CONVERGED;
  double beta_start = 0.0;   // true residual at the start of the last cycle
  double* hd = ctx->hdev;  // h1 [0,64), h1+h2 [64,128), ||w||^2 [128], h2 [192,256), y [256,320)
  while (true) {
    double rr;
    rc = reduce_dot(ctx, r, r, len, &rr);
    if (rc) return rc;
    double beta = std::sqrt(rr);
    S.true_rel = beta / bnorm;
    if (!std::isfinite(beta)) {
      if (st) *st = S;
      return set_err(ctx, CPR_ENONFINITE, "non-finite residual");
    }
    if (beta <= rtol * bnorm) { result = CPR_OK; break; }
    if (its >= max_iter) break;
    // mixed precision or the learned stage: a restart cycle that left the
    // true residual above stall_ratio times the one it started from (by
    // default: less than halved, where a healthy cycle gains one to two
    // orders) hands the remaining cycles to plain FP64 CPR (FGMRES is
    // flexible, so the change of preconditioner between cycles needs nothing
    // else)
    if (S.cycles > 0 && (ctx->opt.precision == CPR_PREC_MIXED || ctx->opt.learned) && !ctx->fp64_now &&
        ctx->opt.stall_ratio > 0 && beta > ctx->opt.stall_ratio * beta_start) {
      ctx->fp64_now = true;
      S.fp64_fallback = S.cycles;
    }
    beta_start = beta;
    scale_kernel<<<eb, 256, 0, s>>>(len, beta, r, ctx->V);
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    if (dcgs) {
      if ((rc = dcgs2_cycle(ctx, beta, bnorm, its, k, H, g)) != CPR_OK) {
        if (st) *st = S;
        return rc;
      }
    } else {
      bool breakdown_stop = false;
      // Arnoldi step j on the device; its Hessenberg column lands in host slot
      // j % 2 and event ev_iter[j % 2] marks its completion.
      auto launch_step = [&](int j) -> int {
        double* vj = ctx->V + (size_t)j * stride;
        double* zj = ctx->Z + (size_t)j * stride;
        double* w = ctx->V + (size_t)(j + 1) * stride;
        const int nv = j + 1;
        double* slot = ctx->hhost_dev + (j & 1) * 128;
        // v_j = w_j / h_{j,j-1} is formed inside the preconditioner's first kernel
        {
          PhaseScope ps(ctx, PH_PRECOND);
          precond_apply(ctx, vj, vj, j == 0 ? nullptr : hd + 128, zj);
        }
        {
          PhaseScope ps(ctx, PH_SPMV);
          prof_begin(ctx, CPR_KCLASS_SPMV);
          system_spmv(ctx, zj, w, nullptr);
          prof_end(ctx, CPR_KCLASS_SPMV);
        }
        {
          PhaseScope ps(ctx, PH_ORTH);
          // CGS pass 1: h1 = V^T w
          orth_pass(ctx, len, nv, w, nullptr, 0);
          reduce_kernel<<<nv, KB, 0, s>>>(ctx->part, nblk, hd, nullptr);
          // w -= V h1 ; h2 = V^T w
          orth_pass(ctx, len, nv, w, hd, 0);
          // h = h1 + h2 (device and host) and h2 alone
          reduce_kernel<<<nv, KB, 0, s>>>(ctx->part, nblk, hd + 64, hd, slot, hd + 192);
          // w -= V h2 ; ||w||^2
          orth_pass(ctx, len, nv, w, hd + 192, 1);
          reduce_kernel<<<1, KB, 0, s>>>(ctx->part + (size_t)nv * nblk, nblk, hd + 128, nullptr, slot + 64);
        }
        CPR_TRY(hipGetLastError());
        CPR_TRY(hipEventRecord(ctx->ev_iter[j & 1], s));
        return CPR_OK;
      };
      int launched = -1;
      for (int j = 0; j < m; ++j) {
        if (launched < j) {
          if ((rc = launch_step(j)) != CPR_OK) return rc;
          launched = j;
        }
        its += 1;
        // While the host waits for step j, the device may already run step
        // j + 1: it needs nothing from the host.  Done only while the residual
        // estimate is far above the tolerance, so that a step launched but not
        // needed (the cycle ends at j) is rare; its results are then ignored.
        if (j + 1 < m && its < max_iter && std::fabs(g[j]) > SPECULATE * rtol * bnorm) {
          if ((rc = launch_step(j + 1)) != CPR_OK) return rc;
          launched = j + 1;
        }
        CPR_TRY(hipEventSynchronize(ctx->ev_iter[j & 1]));
        ph_harvest(ctx, false);
        const double* slot = ctx->hhost + (j & 1) * 128;
        const int nv = j + 1;
        double hn = std::sqrt(slot[64]);
        for (int i = 0; i <= m; ++i) col[i] = 0.0;
        for (int i = 0; i < nv; ++i) col[i] = slot[i];
        col[j + 1] = hn;
        double az = 0.0;
        for (int i = 0; i <= j + 1; ++i) az += col[i] * col[i];
        az = std::sqrt(az);
        if (!std::isfinite(az)) {
          if (st) *st = S;
          return set_err(ctx, CPR_ENONFINITE, "non-finite Hessenberg column");
        }
        for (int i = 0; i < j; ++i) {
          double t = cs[i] * col[i] + sn[i] * col[i + 1];
          col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
          col[i] = t;
        }
        double den = std::hypot(col[j], col[j + 1]);
        if (den == 0.0) { cs[j] = 1.0; sn[j] = 0.0; }
        else { cs[j] = col[j] / den; sn[j] = col[j + 1] / den; }
        col[j] = den;
        col[j + 1] = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        for (int i = 0; i <= m; ++i) H[(size_t)i * m + j] = col[i];
        k = j + 1;
        if (std::fabs(g[j + 1]) <= rtol * bnorm || its >= max_iter) break;
        if (hn <= BREAKDOWN * az) { breakdown_stop = true; break; }
        if (early_stall(ctx, k, its, std::fabs(g[j + 1]), beta)) break;
      }
      if (launched >= k) {
        // a step ran ahead but the cycle ended: undo its learned-stage count
        if (learned_on(ctx)) learned_discard_last(ctx);
      }
      (void)breakdown_stop;
    }
    // back substitution H[:k,:k] y = g[:k]
    for (int i = k - 1; i >= 0; --i) {
      double t = g[i];
      for (int c = i + 1; c < k; ++c) t -= H[(size_t)i * m + c] * y[c];
      y[i] = t / H[(size_t)i * m + i];
    }
    for (int i = 0; i < k; ++i) ctx->hhost[256 + i] = y[i];
    CPR_TRY(hipMemcpyAsync(hd + 256, ctx->hhost + 256, k * sizeof(double), hipMemcpyHostToDevice, s));
    maxpy_kernel<<<eb, 256, 0, s>>>(len, k, ctx->Z, stride, hd + 256, x);
    S.cycles += 1;
    S.est_rel = std::fabs(g[k]) / bnorm;
    PhaseScope ps(ctx, PH_SPMV);
    prof_begin(ctx, CPR_KCLASS_SPMV);
    system_spmv(ctx, x, r, ctx->rs);
    prof_end(ctx, CPR_KCLASS_SPMV);
  }
  S.iterations = its;
  S.converged = result == CPR_OK;
  ph_fill_stats(ctx, &S);
  if (st) *st = S;
  return result;
}

// Right-preconditioned BiCGSTAB on ctx->rs into ctx->xs (colour-split),
// step for step as the oracle's; workspace: the first eight Krylov vectors.
// The iteration's scalars stay on the device; one stream synchronisation
// per iteration reads ||r||^2, rho, omega and the breakdown flag.
int bicgstab_solve(cpr_ctx* ctx, cpr_stats_t* st) {
  hipStream_t s = ctx->stream;
  const int b = ctx->b;
  const long len = vec_len(ctx);
  const int nblk = ctx->nblk;
  const int eb = div_up(len, 256);
  const double rtol = ctx->opt.rtol;
  const int max_iter = ctx->opt.max_iter;
  double* x = ctx->xs;
  double* W = ctx->V;
  double *r = W, *rh = W + len, *p = W + 2 * len, *v = W + 3 * len, *ph = W + 4 * len, *sv = W + 5 * len,
         *sh = W + 6 * len, *t = W + 7 * len;
  double* sc = ctx->hdev + 320;
  double* host = ctx->hhost_dev + 320;
  const double* hh = ctx->hhost + 320;
  cpr_stats_t S = {};
  S.mg_levels = (int)ctx->levels.size();
  S.qimpes_fallback = ctx->qimpes_bad;
  ph_solve_start(ctx);

  zero_kernel<<<eb, 256, 0, s>>>(len, x);
  double bb;
  int rc = reduce_dot(ctx, ctx->rs, ctx->rs, len, &bb);
  if (rc) return rc;
  const double bnorm = std::sqrt(bb);
  S.bnorm = bnorm;
  if (!std::isfinite(bnorm)) {
    if (st) *st = S;
    return set_err(ctx, CPR_ENONFINITE, "non-finite right-hand side");
  }
  if (bnorm == 0.0) {
    S.converged = 1;
    ph_fill_stats(ctx, &S);
    if (st) *st = S;
    return CPR_OK;
  }
  CPR_TRY(hipMemcpyAsync(r, ctx->rs, len * sizeof(double), hipMemcpyDeviceToDevice, s));
  int its = 0;
  int result = CPR_NOT_CONVERGED;
  while (true) {
    S.cycles += 1;
    CPR_TRY(hipMemcpyAsync(rh, r, len * sizeof(double), hipMemcpyDeviceToDevice, s));
    zero_kernel<<<eb, 256, 0, s>>>(len, p);
    zero_kernel<<<eb, 256, 0, s>>>(len, v);
    bicg_init_kernel<<<1, 64, 0, s>>>(sc);
    // rho = <rh, r> and beta for the first p (= r)
    dot2_kernel<<<nblk, KB, 0, s>>>(len, rh, r, r, r, ctx->part, nblk);
    bicg_reduce_kernel<<<1, KB, 0, s>>>(ctx->part, nblk, 2, 2, sc, host);
    CPR_TRY(hipGetLastError());
    CPR_TRY(hipStreamSynchronize(s));
    bool stop = false;
    while (its < max_iter) {
      const double rho = hh[1];
      if (!(rho != 0.0) || !std::isfinite(rho)) { stop = true; break; }
      {
        PhaseScope ps(ctx, PH_ORTH);
        bicg_p_kernel<<<eb, 256, 0, s>>>(len, sc, r, v, p);
      }
      {
        PhaseScope ps(ctx, PH_PRECOND);
        precond_apply(ctx, p, p, nullptr, ph);
      }
      {
        PhaseScope ps(ctx, PH_SPMV);
        prof_begin(ctx, CPR_KCLASS_SPMV);
        system_spmv(ctx, ph, v, nullptr);
        prof_end(ctx, CPR_KCLASS_SPMV);
      }
      {
        PhaseScope ps(ctx, PH_ORTH);
        dot2_kernel<<<nblk, KB, 0, s>>>(len, rh, v, nullptr, nullptr, ctx->part, nblk);
        bicg_reduce_kernel<<<1, KB, 0, s>>>(ctx->part, nblk, 1, 0, sc, host);
        bicg_s_kernel<<<eb, 256, 0, s>>>(len, sc, r, v, sv);
      }
      {
        PhaseScope ps(ctx, PH_PRECOND);
        precond_apply(ctx, sv, sv, nullptr, sh);
      }
      {
        PhaseScope ps(ctx, PH_SPMV);
        prof_begin(ctx, CPR_KCLASS_SPMV);
        system_spmv(ctx, sh, t, nullptr);
        prof_end(ctx, CPR_KCLASS_SPMV);
      }
      {
        PhaseScope ps(ctx, PH_ORTH);
        dot2_kernel<<<nblk, KB, 0, s>>>(len, t, sv, t, t, ctx->part, nblk);
        bicg_reduce_kernel<<<1, KB, 0, s>>>(ctx->part, nblk, 2, 1, sc, host);
        bicg_xr_kernel<<<nblk, KB, 0, s>>>(len, sc, ph, sh, sv, t, x, r, rh, ctx->part, nblk);
        bicg_reduce_kernel<<<1, KB, 0, s>>>(ctx->part, nblk, 2, 2, sc, host);
      }
      CPR_TRY(hipGetLastError());
      CPR_TRY(hipStreamSynchronize(s));
      ph_harvest(ctx, false);
      if (hh[3] != 0.0) { stop = true; break; }       // <rh, v> vanished: x unchanged
      its += 1;
      const double rr = hh[0];
      S.est_rel = std::sqrt(rr) / bnorm;
      if (!std::isfinite(rr)) {
        S.iterations = its;
        if (st) *st = S;
        return set_err(ctx, CPR_ENONFINITE, "non-finite BiCGSTAB residual");
      }
      if (std::sqrt(rr) <= rtol * bnorm) break;
      if (hh[2] == 0.0) { stop = true; break; }       // omega vanished
    }
    // true residual r = b - A x
    {
      PhaseScope ps(ctx, PH_SPMV);
      prof_begin(ctx, CPR_KCLASS_SPMV);
      system_spmv(ctx, x, r, ctx->rs);
      prof_end(ctx, CPR_KCLASS_SPMV);
    }
    double rr;
    rc = reduce_dot(ctx, r, r, len, &rr);
    if (rc) return rc;
    S.true_rel = std::sqrt(rr) / bnorm;
    if (!std::isfinite(S.true_rel)) {
      S.iterations = its;
      if (st) *st = S;
      return set_err(ctx, CPR_ENONFINITE, "non-finite residual");
    }
    if (S.true_rel <= rtol) { result = CPR_OK; break; }
    if (stop || its >= max_iter) break;
  }
  S.iterations = its;
  S.converged = result == CPR_OK;
  ph_fill_stats(ctx, &S);
  if (st) *st = S;
  return result;
}
