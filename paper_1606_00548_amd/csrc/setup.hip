// CPR preconditioner setup (Sec. 2.5: decoupling, AMG on A_pp, full-system
// smoother).
//
//  * Quasi-IMPES weights w_i = D_i^-T e_0 / (D_i^-1)_00 per cell, and row 0
//    of every decoupled block, w_i^T A_ij (the pressure equation with the
//    saturation coupling of the diagonal block removed).  A cell whose
//    (D_i^-1)_00 is zero, tiny or non-finite keeps w_i = e_0 and is counted.
//  * Pressure multigrid: A_p = (W A)_{pp}; 2x2x2 aggregation with Galerkin
//    coarse operators P^T A P, which stay 7-point; the coarsest level is
//    inverted densely (Gauss-Jordan with partial pivoting).
//  * Block ILU(0) of W A in red-then-black order: on the 7-point graph it
//    keeps every off-diagonal block and changes only the black diagonals,
//    D'_i = A~_ii - sum_k A~_ik D'_k^-1 A~_ki over the red neighbours k.
#include <cmath>

#include "internal.h"

namespace {

constexpr double TINY = 1e-300;

// In-place inverse of a small dense matrix by Gauss-Jordan with partial
// pivoting.  Returns false for a zero, tiny or non-finite pivot.
template <int B>
__device__ bool small_inverse(double (&a)[B][B], double (&inv)[B][B]) {
  for (int r = 0; r < B; ++r)
    for (int c = 0; c < B; ++c) inv[r][c] = (r == c) ? 1.0 : 0.0;
  bool ok = true;
#pragma unroll
  for (int p = 0; p < B; ++p) {
    int piv = p;
    double best = fabs(a[p][p]);
#pragma unroll
    for (int r = p + 1; r < B; ++r)
      if (fabs(a[r][p]) > best) { best = fabs(a[r][p]); piv = r; }
    if (!(best > TINY) || !isfinite(best)) ok = false;
    if (piv != p) {
#pragma unroll
      for (int c = 0; c < B; ++c) {
        double t = a[p][c]; a[p][c] = a[piv][c]; a[piv][c] = t;
        t = inv[p][c]; inv[p][c] = inv[piv][c]; inv[piv][c] = t;
      }
    }
    double s = 1.0 / a[p][p];
#pragma unroll
    for (int c = 0; c < B; ++c) { a[p][c] *= s; inv[p][c] *= s; }
#pragma unroll
    for (int r = 0; r < B; ++r) {
      if (r == p) continue;
      double f = a[r][p];
#pragma unroll
      for (int c = 0; c < B; ++c) { a[r][c] -= f * a[p][c]; inv[r][c] -= f * inv[p][c]; }
    }
  }
  return ok;
}

// Solve D^T y = e_0 for y (small Gaussian elimination, partial pivoting).
template <int B>
__device__ bool solve_transposed_e0(const double (&D)[B][B], double (&y)[B]) {
  double a[B][B], rhs[B];
  for (int r = 0; r < B; ++r) {
    for (int c = 0; c < B; ++c) a[r][c] = D[c][r];
    rhs[r] = r == 0 ? 1.0 : 0.0;
  }
  bool ok = true;
#pragma unroll
  for (int p = 0; p < B; ++p) {
    int piv = p;
    double best = fabs(a[p][p]);
    for (int r = p + 1; r < B; ++r)
      if (fabs(a[r][p]) > best) { best = fabs(a[r][p]); piv = r; }
    if (!(best > 0.0)) ok = false;
    if (piv != p) {
      for (int c = 0; c < B; ++c) { double t = a[p][c]; a[p][c] = a[piv][c]; a[piv][c] = t; }
      double t = rhs[p]; rhs[p] = rhs[piv]; rhs[piv] = t;
    }
    for (int r = p + 1; r < B; ++r) {
      double f = a[r][p] / a[p][p];
      for (int c = p; c < B; ++c) a[r][c] -= f * a[p][c];
      rhs[r] -= f * rhs[p];
    }
  }
  for (int r = B - 1; r >= 0; --r) {
    double s = rhs[r];
    for (int c = r + 1; c < B; ++c) s -= a[r][c] * y[c];
    y[r] = s / a[r][r];
  }
  return ok;
}

template <int B>
__global__ void qimpes_kernel(int n, const double* __restrict__ J, double* __restrict__ w,
                              double* __restrict__ R0, double* __restrict__ Ap, int* __restrict__ nbad) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const size_t N = n;
  double D[B][B], y[B], wv[B];
  for (int r = 0; r < B; ++r)
    for (int c = 0; c < B; ++c) D[r][c] = J[((size_t)r * B + c) * N + t];
  bool ok = solve_transposed_e0<B>(D, y);
  double y0 = y[0];
  if (ok && fabs(y0) > TINY && isfinite(y0)) {
    for (int r = 0; r < B; ++r) wv[r] = y[r] / y0;
    wv[0] = 1.0;
  } else {
    for (int r = 0; r < B; ++r) wv[r] = r == 0 ? 1.0 : 0.0;
    atomicAdd(nbad, 1);
  }
  for (int r = 0; r < B; ++r) w[r * N + t] = wv[r];
  for (int d = 0; d < 7; ++d) {
    for (int c = 0; c < B; ++c) {
      double s = 0.0;
      for (int r = 0; r < B; ++r) s += wv[r] * J[((size_t)(d * B + r) * B + c) * N + t];
      R0[((size_t)d * B + c) * N + t] = s;
      if (c == 0) Ap[(size_t)d * N + t] = s;
    }
  }
}

// Galerkin coarse operator for piecewise-constant 2x2x2 aggregation: one
// thread per coarse cell sums the couplings of its (up to) 8 fine cells.
__global__ void rap_kernel(Lay F, Lay C, const double* __restrict__ Af, double* __restrict__ Ac) {
  int tc = blockIdx.x * blockDim.x + threadIdx.x;
  if (tc >= C.n) return;
  int ci, cj, ck;
  lay_coords(C, tc, ci, cj, ck);
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int fk = 2 * ck; fk <= 2 * ck + 1 && fk < F.nz; ++fk)
    for (int fj = 2 * cj; fj <= 2 * cj + 1 && fj < F.ny; ++fj)
      for (int fi = 2 * ci; fi <= 2 * ci + 1 && fi < F.nx; ++fi) {
        int f = lay_index(F, fi, fj, fk);
        acc[0] += Af[f];
        for (int d = 1; d < 7; ++d) {
          int di, dj, dk;
          dir_offset(d, di, dj, dk);
          int gi = fi + di, gj = fj + dj, gk = fk + dk;
          if (gi < 0 || gi >= F.nx || gj < 0 || gj >= F.ny || gk < 0 || gk >= F.nz) continue;
          double a = Af[(size_t)d * F.n + f];
          if ((gi >> 1) == ci && (gj >> 1) == cj && (gk >> 1) == ck)
            acc[0] += a;
          else
            acc[d] += a;
        }
      }
  for (int d = 0; d < 7; ++d) Ac[(size_t)d * C.n + tc] = acc[d];
}

// Dense [M | I] (row-major, 2*nc columns) of the coarsest 7-point operator,
// indexed by that level's storage order.
__global__ void dense_build_kernel(Lay L, const double* __restrict__ A, double* __restrict__ M) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  int nc = L.n;
  if (t >= nc) return;
  double* row = M + (size_t)t * 2 * nc;
  for (int c = 0; c < 2 * nc; ++c) row[c] = 0.0;
  row[nc + t] = 1.0;
  int i, j, k;
  lay_coords(L, t, i, j, k);
  row[t] += A[t];
  for (int d = 1; d < 7; ++d) {
    int nb = lay_nbr(L, i, j, k, d);
    if (nb >= 0) row[nb] += A[(size_t)d * nc + t];
  }
}

// One Gauss-Jordan column step p, double-buffered (src -> dst): every block
// finds the pivot row redundantly, then updates its share of the entries.
__global__ void gj_step_kernel(int nc, int p, const double* __restrict__ src, double* __restrict__ dst,
                               int* __restrict__ flag) {
  __shared__ double sval[256];
  __shared__ int sidx[256];
  const int w = 2 * nc;
  // pivot search over rows p..nc-1 (ties: lowest row)
  double best = -1.0;
  int bi = p;
  for (int r = p + threadIdx.x; r < nc; r += blockDim.x) {
    double v = fabs(src[(size_t)r * w + p]);
    if (v > best) { best = v; bi = r; }
  }
  sval[threadIdx.x] = best;
  sidx[threadIdx.x] = bi;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      double o = sval[threadIdx.x + s];
      int oi = sidx[threadIdx.x + s];
      if (o > sval[threadIdx.x] || (o == sval[threadIdx.x] && oi < sidx[threadIdx.x])) {
        sval[threadIdx.x] = o;
        sidx[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  int piv = sidx[0];
  double pv = src[(size_t)piv * w + p];
  if (blockIdx.x == 0 && threadIdx.x == 0 && (!(fabs(pv) > TINY) || !isfinite(pv))) atomicExch(flag, 1);
  double inv = 1.0 / pv;
  size_t total = (size_t)nc * w;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    int r = (int)(e / w), c = (int)(e % w);
    double prow = src[(size_t)piv * w + c] * inv;   // scaled pivot row
    double out;
    if (r == p) {
      out = prow;
    } else {
      int rr = (r == piv) ? p : r;                  // row piv receives old row p
      double f = src[(size_t)rr * w + p];
      out = src[(size_t)rr * w + c] - f * prow;
    }
    dst[e] = out;
  }
}

// Whole Gauss-Jordan inversion (partial pivoting, in place) of a small
// coarsest operator in one workgroup with the matrix held in LDS (nc <= 128).
// Thread layout: row r = tid / 8, columns lane + 8 q; rows are padded to an
// odd stride so the 8 rows a wavefront touches fall in different banks.  The
// dense matrix is built from the level's 7-point stencil; the inverse is
// written column major (and as FP32).
constexpr int GJ_LDS_MAX = 128;

__global__ __launch_bounds__(1024) void gj_lds_kernel(Lay L, const double* __restrict__ A,
                                                      double* __restrict__ inv, float* __restrict__ invf,
                                                      int* __restrict__ flag) {
  extern __shared__ double sm[];
  const int nc = L.n;
  const int ld = nc + 8;          // 8 consecutive rows then start in different LDS banks
  double* M = sm;                 // nc rows of stride ld
  double* fcol = sm + nc * ld;    // multipliers of the current column
  __shared__ int piv[GJ_LDS_MAX];
  __shared__ double pvs;
  __shared__ int prs;
  const int tid = threadIdx.x;
  const int r = tid >> 3, lane = tid & 7;
  const bool own = r < nc;
  if (own)
    for (int c = lane; c < nc; c += 8) M[r * ld + c] = 0.0;
  __syncthreads();
  if (own && lane == 0) {
    int i, j, k;
    lay_coords(L, r, i, j, k);
    M[r * ld + r] += A[r];
    for (int d = 1; d < 7; ++d) {
      int nb = lay_nbr(L, i, j, k, d);
      if (nb >= 0) M[r * ld + nb] += A[(size_t)d * nc + r];
    }
  }
  __syncthreads();
  for (int p = 0; p < nc; ++p) {
    if (tid < 64) {   // pivot: largest |M[q][p]|, q >= p, lowest row on ties
      double best = -1.0;
      int bi = p;
      for (int q = p + tid; q < nc; q += 64) {
        double v = fabs(M[q * ld + p]);
        if (v > best) { best = v; bi = q; }
      }
      for (int o = 32; o > 0; o >>= 1) {
        double ov = __shfl_down(best, o, 64);
        int oi = __shfl_down(bi, o, 64);
        if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
      }
      if (tid == 0) {
        prs = bi;
        pvs = M[bi * ld + p];
        piv[p] = bi;
        if (!(best > TINY) || !isfinite(best)) atomicExch(flag, 1);
      }
    }
    __syncthreads();
    const int pr = prs;
    const double pinv = 1.0 / pvs;
    // one thread per column interchanges rows p and pr and scales the new
    // pivot row (diagonal set to 1 first); other threads collect the
    // multipliers of column p for the rows the interchange does not touch
    if (tid < nc) {
      const int c = tid;
      double top = M[pr * ld + c], old = M[p * ld + c];
      if (pr != p) M[pr * ld + c] = old;
      M[p * ld + c] = (c == p ? 1.0 : top) * pinv;
      if (c == p) { fcol[p] = 0.0; fcol[pr] = pr == p ? 0.0 : old; }
    } else if (tid >= 512 && tid - 512 < nc) {
      const int q = tid - 512;
      if (q != p && q != pr) fcol[q] = M[q * ld + p];
    }
    __syncthreads();
    if (own && r != p) {
      const double f = fcol[r];
      for (int c = lane; c < nc; c += 8) M[r * ld + c] = (c == p ? 0.0 : M[r * ld + c]) - f * M[p * ld + c];
    }
    __syncthreads();
  }
  // undo the row interchanges as column interchanges, last first
  for (int p = nc - 1; p >= 0; --p) {
    int q = piv[p];
    if (q != p && own && lane == 0) {
      double t = M[r * ld + p]; M[r * ld + p] = M[r * ld + q]; M[r * ld + q] = t;
    }
    __syncthreads();
  }
  if (own)
    for (int c = lane; c < nc; c += 8) {
      double v = M[r * ld + c];
      inv[(size_t)c * nc + r] = v;
      if (invf) invf[(size_t)c * nc + r] = (float)v;
    }
}

// Copy the right half of [I | M^-1] into column-major storage.
__global__ void gj_extract_kernel(int nc, const double* __restrict__ M, double* __restrict__ inv,
                                  float* __restrict__ invf) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nc * nc) return;
  int col = e / nc, row = e % nc;
  double v = M[(size_t)row * 2 * nc + nc + col];
  inv[e] = v;
  if (invf) invf[e] = (float)v;
}

// Decoupled block (d, r, c) of cell t: row 0 from R0, other rows from J.
template <int B>
__device__ inline double at_blk(const double* __restrict__ J, const double* __restrict__ R0, size_t N,
                                int d, int r, int c, int t) {
  return r == 0 ? R0[((size_t)d * B + c) * N + t] : J[((size_t)(d * B + r) * B + c) * N + t];
}

template <int B>
__global__ void ilu_kernel(Lay L, int colour, const double* __restrict__ J, const double* __restrict__ R0,
                           double* __restrict__ Dinv, int* __restrict__ flag) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= L.nh) return;
  int t = colour * L.nh + q;
  const size_t N = L.n;
  double D[B][B];
  for (int r = 0; r < B; ++r)
    for (int c = 0; c < B; ++c) D[r][c] = at_blk<B>(J, R0, N, 0, r, c, t);
  if (colour == 1) {
    int i, j, k;
    lay_coords(L, t, i, j, k);
    for (int d = 1; d < 7; ++d) {
      int nb = lay_nbr(L, i, j, k, d);
      if (nb < 0) continue;
      int od = (d & 1) ? d + 1 : d - 1;   // direction from the neighbour back to t
      double Aik[B][B], Dk[B][B], Aki[B][B], T1[B][B];
      for (int r = 0; r < B; ++r)
        for (int c = 0; c < B; ++c) {
          Aik[r][c] = at_blk<B>(J, R0, N, d, r, c, t);
          Dk[r][c] = Dinv[((size_t)r * B + c) * N + nb];
          Aki[r][c] = at_blk<B>(J, R0, N, od, r, c, nb);
        }
      for (int r = 0; r < B; ++r)
        for (int c = 0; c < B; ++c) {
          double s = 0.0;
          for (int m = 0; m < B; ++m) s += Aik[r][m] * Dk[m][c];
          T1[r][c] = s;
        }
      for (int r = 0; r < B; ++r)
        for (int c = 0; c < B; ++c) {
          double s = 0.0;
          for (int m = 0; m < B; ++m) s += T1[r][m] * Aki[m][c];
          D[r][c] -= s;
        }
    }
  }
  double inv[B][B];
  if (!small_inverse<B>(D, inv)) atomicExch(flag, 1);
  for (int r = 0; r < B; ++r)
    for (int c = 0; c < B; ++c) Dinv[((size_t)r * B + c) * N + t] = inv[r][c];
}

__global__ void zero_int_kernel(int* p, int n) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = 0;
}

}  // namespace

static void free_levels(cpr_ctx* ctx) {
  for (size_t l = 0; l < ctx->levels.size(); ++l) {
    MGLevel& L = ctx->levels[l];
    hipFree(L.A); hipFree(L.Af); hipFree(L.x); hipFree(L.r); hipFree(L.xf); hipFree(L.rf);
    hipFree(L.res); hipFree(L.resf);
  }
  ctx->levels.clear();
  hipFree(ctx->cinv); ctx->cinv = nullptr;
  hipFree(ctx->cinvf); ctx->cinvf = nullptr;
  hipFree(ctx->gj_work); ctx->gj_work = nullptr;
}

void release_hierarchy(cpr_ctx* ctx) { free_levels(ctx); }

static int build_hierarchy(cpr_ctx* ctx) {
  int coarsest = ctx->opt.mg_coarsest;
  std::vector<Lay> shapes;
  shapes.push_back(ctx->lay);
  while (shapes.back().n > coarsest) {
    const Lay& f = shapes.back();
    if (!f.cs)
      return set_err(ctx, CPR_EINVAL, "multigrid level with odd nx has more than mg_coarsest cells");
    shapes.push_back(make_lay((f.nx + 1) / 2, (f.ny + 1) / 2, (f.nz + 1) / 2, true));
  }
  if (shapes.back().n > 4096) return set_err(ctx, CPR_EINVAL, "coarsest level too large");
  bool same = shapes.size() == ctx->levels.size();
  for (size_t l = 0; same && l < shapes.size(); ++l)
    same = shapes[l].nx == ctx->levels[l].lay.nx && shapes[l].ny == ctx->levels[l].lay.ny &&
           shapes[l].nz == ctx->levels[l].lay.nz && shapes[l].cs == ctx->levels[l].lay.cs;
  if (same) return CPR_OK;
  free_levels(ctx);
  ctx->levels.resize(shapes.size());
  for (size_t l = 0; l < shapes.size(); ++l) {
    MGLevel& L = ctx->levels[l];
    L.lay = shapes[l];
    size_t n = L.lay.n;
    CPR_TRY(hipMalloc(&L.A, 7 * n * sizeof(double)));
    CPR_TRY(hipMalloc(&L.Af, 7 * n * sizeof(float)));
    CPR_TRY(hipMalloc(&L.x, n * sizeof(double)));
    CPR_TRY(hipMalloc(&L.r, n * sizeof(double)));
    CPR_TRY(hipMalloc(&L.xf, n * sizeof(float)));
    CPR_TRY(hipMalloc(&L.rf, n * sizeof(float)));
    CPR_TRY(hipMalloc(&L.res, (n / 2 + 1) * sizeof(double)));
    CPR_TRY(hipMalloc(&L.resf, (n / 2 + 1) * sizeof(float)));
  }
  size_t nc = shapes.back().n;
  CPR_TRY(hipMalloc(&ctx->cinv, nc * nc * sizeof(double)));
  CPR_TRY(hipMalloc(&ctx->cinvf, nc * nc * sizeof(float)));
  CPR_TRY(hipMalloc(&ctx->gj_work, 2 * nc * 2 * nc * sizeof(double)));
  return CPR_OK;
}

// FP32 copies used by the mixed-precision preconditioner.
void launch_mixed_copies(cpr_ctx* ctx);

int setup_cpr(cpr_ctx* ctx) {
  int rc = build_hierarchy(ctx);
  if (rc != CPR_OK) return rc;
  hipStream_t s = ctx->stream;
  const Lay& L = ctx->lay;
  const int n = L.n;
  zero_int_kernel<<<1, 64, 0, s>>>(ctx->flag, 2);
  int nb = div_up(n, 256);
  if (ctx->b == 2)
    qimpes_kernel<2><<<nb, 256, 0, s>>>(n, ctx->J, ctx->w, ctx->R0, ctx->levels[0].A, ctx->flag + 1);
  else
    qimpes_kernel<3><<<nb, 256, 0, s>>>(n, ctx->J, ctx->w, ctx->R0, ctx->levels[0].A, ctx->flag + 1);
  // Galerkin chain and coarsest inverse on the auxiliary stream, the ILU
  // factorisation meanwhile on the caller's stream
  hipStream_t a = ctx->aux;
  CPR_TRY(hipEventRecord(ctx->ev_q, s));
  CPR_TRY(hipStreamWaitEvent(a, ctx->ev_q, 0));
  for (size_t l = 0; l + 1 < ctx->levels.size(); ++l) {
    const MGLevel& F = ctx->levels[l];
    MGLevel& C = ctx->levels[l + 1];
    rap_kernel<<<div_up(C.lay.n, 256), 256, 0, a>>>(F.lay, C.lay, F.A, C.A);
  }
  CPR_TRY(hipEventRecord(ctx->ev_rap, a));
  // dense inverse of the coarsest level
  const MGLevel& last = ctx->levels.back();
  int nc = last.lay.n;
  if (nc <= GJ_LDS_MAX) {
    size_t smem = ((size_t)nc * (nc + 8) + nc) * sizeof(double);
    static bool attr_set = false;
    if (!attr_set) {
      CPR_TRY(hipFuncSetAttribute((const void*)gj_lds_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(((size_t)GJ_LDS_MAX * (GJ_LDS_MAX + 8) + GJ_LDS_MAX) * sizeof(double))));
      attr_set = true;
    }
    gj_lds_kernel<<<1, 1024, smem, a>>>(last.lay, last.A, ctx->cinv, ctx->cinvf, ctx->flag);
  } else {
    double* bufA = ctx->gj_work;
    double* bufB = ctx->gj_work + (size_t)nc * 2 * nc;
    dense_build_kernel<<<div_up(nc, 256), 256, 0, a>>>(last.lay, last.A, bufA);
    int gblocks = div_up((long)nc * 2 * nc, 256);
    if (gblocks > 512) gblocks = 512;
    for (int p = 0; p < nc; ++p) {
      gj_step_kernel<<<gblocks, 256, 0, a>>>(nc, p, bufA, bufB, ctx->flag);
      double* t = bufA; bufA = bufB; bufB = t;
    }
    gj_extract_kernel<<<div_up((long)nc * nc, 256), 256, 0, a>>>(nc, bufA, ctx->cinv, ctx->cinvf);
  }
  CPR_TRY(hipEventRecord(ctx->ev_gj, a));
  // red-black block ILU(0): red diagonals first, black ones use them
  int nh = div_up(L.nh, 256);
  for (int colour = 0; colour < 2; ++colour) {
    if (ctx->b == 2)
      ilu_kernel<2><<<nh, 256, 0, s>>>(L, colour, ctx->J, ctx->R0, ctx->Dinv, ctx->flag);
    else
      ilu_kernel<3><<<nh, 256, 0, s>>>(L, colour, ctx->J, ctx->R0, ctx->Dinv, ctx->flag);
  }
  if (ctx->opt.precision == CPR_PREC_MIXED) {
    CPR_TRY(hipStreamWaitEvent(s, ctx->ev_rap, 0));   // FP32 copies of the levels
    launch_mixed_copies(ctx);
  }
  CPR_TRY(hipStreamWaitEvent(s, ctx->ev_gj, 0));
  rc = launch_check(ctx, "cpr_setup kernels");
  if (rc != CPR_OK) return rc;
  int hflag[2] = {0, 0};
  CPR_TRY(hipMemcpyAsync(hflag, ctx->flag, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  CPR_TRY(hipStreamSynchronize(s));
  ctx->qimpes_bad = hflag[1];
  if (hflag[0]) return set_err(ctx, CPR_ESINGULAR, "singular ILU diagonal block or coarsest operator");
  ctx->setup_done = 1;
  return CPR_OK;
}
