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
//  * or ABF: W_i = D_i^-1 for the diagonal block D_i, A~ = W A in full (each
//    diagonal block becomes I); a singular D_i is an error.
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
    for (int c = 0; c < B; ++c) D[r][c] = J[tix(7 * B * B, r * B + c, t)];
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
      for (int r = 0; r < B; ++r) s += wv[r] * J[tix(7 * B * B, (d * B + r) * B + c, t)];
      R0[tix(7 * B, d * B + c, t)] = s;
      if (c == 0) Ap[(size_t)d * N + t] = s;
    }
  }
}

// ABF decoupling: W_i = D_i^-1 and A~_ij = W_i A_ij for the seven blocks of
// block row i; row 0 of every decoupled block goes to R0 (and its (0, 0)
// entry to the pressure operator), rows >= 1 to Jt.  A singular diagonal
// block raises the flag.
template <int B>
__global__ void abf_kernel(int n, const double* __restrict__ J, double* __restrict__ W,
                           double* __restrict__ R0, double* __restrict__ Jt, double* __restrict__ Ap,
                           int* __restrict__ flag) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const size_t N = n;
  double D[B][B], inv[B][B];
  for (int r = 0; r < B; ++r)
    for (int c = 0; c < B; ++c) D[r][c] = J[tix(7 * B * B, r * B + c, t)];
  if (!small_inverse<B>(D, inv)) atomicExch(flag, 1);
  for (int r = 0; r < B; ++r)
    for (int c = 0; c < B; ++c) W[((size_t)r * B + c) * N + t] = inv[r][c];
  for (int d = 0; d < 7; ++d) {
    double a[B][B];
    for (int r = 0; r < B; ++r)
      for (int c = 0; c < B; ++c) a[r][c] = J[tix(7 * B * B, (d * B + r) * B + c, t)];
    for (int r = 0; r < B; ++r)
      for (int c = 0; c < B; ++c) {
        double s = 0.0;
        for (int m = 0; m < B; ++m) s += inv[r][m] * a[m][c];
        if (r == 0) {
          R0[tix(7 * B, d * B + c, t)] = s;
          if (c == 0) Ap[(size_t)d * N + t] = s;
        } else {
          Jt[tix(7 * B * B, (d * B + r) * B + c, t)] = s;
        }
      }
  }
}

// Galerkin coarse operator for piecewise-constant 2x2x2 aggregation: eight
// lanes per coarse cell, one per fine cell of its aggregate, each sorting
// its stencil row into the coarse couplings (inside the aggregate: the
// diagonal); the eight partial rows are summed by a fixed butterfly.  Ghost
// cells of a padded fine level take no part; a ghost coarse cell gets the
// identity row.
__global__ __launch_bounds__(256) void rap_kernel(Lay F, Lay C, const double* __restrict__ Af,
                                                  double* __restrict__ Ac) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int tc = g >> 3, sub = g & 7;
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  int ci = 0, cj = 0, ck = 0;
  if (tc < C.n) {
    lay_coords(C, tc, ci, cj, ck);
    const int fi = 2 * ci + (sub & 1), fj = 2 * cj + ((sub >> 1) & 1), fk = 2 * ck + (sub >> 2);
    if (fi < F.nxr && fj < F.ny && fk < F.nz) {
      const int f = lay_index(F, fi, fj, fk);
      acc[0] += Af[f];
#pragma unroll
      for (int d = 1; d < 7; ++d) {
        int di, dj, dk;
        dir_offset(d, di, dj, dk);
        const int gi = fi + di, gj = fj + dj, gk = fk + dk;
        if (gi < 0 || gi >= F.nxr || gj < 0 || gj >= F.ny || gk < 0 || gk >= F.nz) continue;
        const double a = Af[(size_t)d * F.n + f];
        if ((gi >> 1) == ci && (gj >> 1) == cj && (gk >> 1) == ck)
          acc[0] += a;
        else
          acc[d] += a;
      }
    }
  }
#pragma unroll
  for (int d = 0; d < 7; ++d) {
    acc[d] += __shfl_xor(acc[d], 1, 8);
    acc[d] += __shfl_xor(acc[d], 2, 8);
    acc[d] += __shfl_xor(acc[d], 4, 8);
  }
  if (tc < C.n && sub == 0) {
    if (ci >= C.nxr) {
      acc[0] = 1.0;
      for (int d = 1; d < 7; ++d) acc[d] = 0.0;
    }
    for (int d = 0; d < 7; ++d) Ac[(size_t)d * C.n + tc] = acc[d];
  }
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

constexpr int GJ_LDS_MAX = 128;   // coarsest levels up to this size are inverted in one workgroup

// Coarsest inverse through the red-black Schur complement (nc <= 128).  A
// 7-point operator couples red cells only to black ones, so with the cells
// ordered red then black A = [Dr B; C Db] with diagonal Dr, Db, and
//   S = Db - C Dr^-1 B,
//   A^-1 = [Dr^-1 - X C Dr^-1, X; -S^-1 C Dr^-1, S^-1],  X = -Dr^-1 B S^-1.
// Only S (at most 64 x 64) goes through Gauss-Jordan with partial pivoting
// (in LDS, 16 threads per row); B and C have at most six entries per row
// and column, so the other blocks are short sums.  Inverse written column
// major (and as FP32).  A zero or non-finite red diagonal or S pivot sets
// the singular flag.
constexpr int SCH_MAX = 64;
constexpr int SCH_LD = SCH_MAX + 1;

__global__ __launch_bounds__(1024) void gj_schur_kernel(Lay L, const double* __restrict__ A,
                                                        double* __restrict__ inv, float* __restrict__ invf,
                                                        int* __restrict__ flag) {
  extern __shared__ double sm[];
  double* S = sm;                        // [SCH_MAX][SCH_LD]
  double* X = sm + SCH_MAX * SCH_LD;     // [SCH_MAX][SCH_MAX]
  __shared__ int colr[GJ_LDS_MAX], pos[GJ_LDS_MAX];
  __shared__ int red[SCH_MAX], blk[SCH_MAX];
  __shared__ double Dinvr[SCH_MAX], Db[SCH_MAX], fcol[SCH_MAX];
  __shared__ int Bk[SCH_MAX][6], Ck[SCH_MAX][6];
  __shared__ double Bv[SCH_MAX][6], Cv[SCH_MAX][6], Tv[SCH_MAX][6];
  __shared__ int piv[SCH_MAX], idx[SCH_MAX];
  __shared__ double pvs;
  __shared__ int prs, nr_s;
  const int nc = L.n, tid = threadIdx.x;
  // colours and positions within a colour
  if (tid < nc) {
    int i, j, k;
    lay_coords(L, tid, i, j, k);
    colr[tid] = (i + j + k) & 1;
  }
  __syncthreads();
  if (tid < nc) {
    int q = 0;
    for (int u = 0; u < tid; ++u) q += colr[u] == colr[tid];
    pos[tid] = q;
    if (colr[tid] == 0) red[q] = tid; else blk[q] = tid;
  }
  if (tid == 0) {
    int q = 0;
    for (int u = 0; u < nc; ++u) q += colr[u] == 0;
    nr_s = q;
  }
  __syncthreads();
  const int nr = nr_s, nb = nc - nr;
  // red rows: 1/Dr, B (black neighbours), C^T (the black rows' coupling back)
  if (tid < nr) {
    const int c = red[tid];
    const double d = A[c];
    if (!(fabs(d) > TINY) || !isfinite(d)) atomicExch(flag, 1);
    Dinvr[tid] = 1.0 / d;
    int i, j, k;
    lay_coords(L, c, i, j, k);
    for (int e = 0; e < 6; ++e) {
      const int nbc = lay_nbr(L, i, j, k, e + 1);
      const int opp = (e ^ 1) + 1;
      Bk[tid][e] = nbc >= 0 ? pos[nbc] : -1;
      Bv[tid][e] = nbc >= 0 ? A[(size_t)(e + 1) * nc + c] : 0.0;
      Tv[tid][e] = nbc >= 0 ? A[(size_t)opp * nc + nbc] : 0.0;
    }
  } else if (tid >= 512 && tid - 512 < nb) {
    const int kb = tid - 512, c = blk[kb];
    Db[kb] = A[c];
    int i, j, k;
    lay_coords(L, c, i, j, k);
    for (int e = 0; e < 6; ++e) {
      const int nbc = lay_nbr(L, i, j, k, e + 1);
      Ck[kb][e] = nbc >= 0 ? pos[nbc] : -1;
      Cv[kb][e] = nbc >= 0 ? A[(size_t)(e + 1) * nc + c] : 0.0;
    }
  }
  __syncthreads();
  // S = Db - C Dr^-1 B
  for (int q = tid; q < nb * nb; q += 1024) {
    const int k1 = q / nb, k2 = q % nb;
    double v = k1 == k2 ? Db[k1] : 0.0;
    for (int e = 0; e < 6; ++e) {
      const int r = Ck[k1][e];
      if (r < 0) continue;
      double brk = 0.0;
      for (int e2 = 0; e2 < 6; ++e2) brk += Bk[r][e2] == k2 ? Bv[r][e2] : 0.0;
      v -= Cv[k1][e] * Dinvr[r] * brk;
    }
    S[k1 * SCH_LD + k2] = v;
  }
  __syncthreads();
  // Gauss-Jordan on S in place: thread (row tid / 16, columns tid % 16 + 16 q)
  const int row = tid >> 4, l16 = tid & 15;
  const bool own = row < nb;
  for (int p = 0; p < nb; ++p) {
    if (tid < 64) {
      double best = -1.0;
      int bi = p;
      if (p + tid < nb) { best = fabs(S[(p + tid) * SCH_LD + p]); bi = p + tid; }
      for (int o = 32; o > 0; o >>= 1) {
        double ov = __shfl_down(best, o, 64);
        int oi = __shfl_down(bi, o, 64);
        if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
      }
      if (tid == 0) {
        prs = bi;
        pvs = S[bi * SCH_LD + p];
        piv[p] = bi;
        if (!(best > TINY) || !isfinite(best)) atomicExch(flag, 1);
      }
    }
    __syncthreads();
    const int pr = prs;
    const double pinv = 1.0 / pvs;
    if (tid < nb) {
      const int c = tid;
      double top = S[pr * SCH_LD + c], old = S[p * SCH_LD + c];
      if (pr != p) S[pr * SCH_LD + c] = old;
      S[p * SCH_LD + c] = (c == p ? 1.0 : top) * pinv;
      if (c == p) { fcol[p] = 0.0; fcol[pr] = pr == p ? 0.0 : old; }
    } else if (tid >= 512 && tid - 512 < nb) {
      const int q = tid - 512;
      if (q != p && q != pr) fcol[q] = S[q * SCH_LD + p];
    }
    __syncthreads();
    if (own && row != p) {
      const double f = fcol[row];
      for (int c = l16; c < nb; c += 16) S[row * SCH_LD + c] = (c == p ? 0.0 : S[row * SCH_LD + c]) - f * S[p * SCH_LD + c];
    }
    __syncthreads();
  }
  // row interchanges undone as column interchanges, last first: column j of
  // S^-1 is column idx[j] of the eliminated matrix
  if (tid == 0) {
    for (int c = 0; c < nb; ++c) idx[c] = c;
    for (int p = nb - 1; p >= 0; --p) {
      const int q = piv[p];
      const int t = idx[p]; idx[p] = idx[q]; idx[q] = t;
    }
  }
  __syncthreads();
  auto Si = [&](int i, int j) { return S[i * SCH_LD + idx[j]]; };
  // X = -Dr^-1 B S^-1
  for (int q = tid; q < nr * nb; q += 1024) {
    const int r = q / nb, j = q % nb;
    double v = 0.0;
    for (int e = 0; e < 6; ++e)
      if (Bk[r][e] >= 0) v += Bv[r][e] * Si(Bk[r][e], j);
    X[r * SCH_MAX + j] = -Dinvr[r] * v;
  }
  __syncthreads();
  // the four blocks of A^-1, column major
  for (int q = tid; q < nc * nc; q += 1024) {
    const int ci = q / nc, ri = q % nc;       // column cell, row cell
    const int pc = pos[ci], pri = pos[ri];
    double v;
    if (colr[ri] == 1 && colr[ci] == 1) {
      v = Si(pri, pc);
    } else if (colr[ri] == 0 && colr[ci] == 1) {
      v = X[pri * SCH_MAX + pc];
    } else if (colr[ri] == 1) {               // black row, red column
      v = 0.0;
      for (int e = 0; e < 6; ++e)
        if (Bk[pc][e] >= 0) v += Si(pri, Bk[pc][e]) * Tv[pc][e];
      v = -v * Dinvr[pc];
    } else {                                  // red row, red column
      v = 0.0;
      for (int e = 0; e < 6; ++e)
        if (Bk[pc][e] >= 0) v += X[pri * SCH_MAX + Bk[pc][e]] * Tv[pc][e];
      v = (pri == pc ? Dinvr[pri] : 0.0) - v * Dinvr[pc];
    }
    inv[q] = v;
    if (invf) invf[q] = (float)v;
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
  return r == 0 ? R0[tix(7 * B, d * B + c, t)] : J[tix(7 * B * B, (d * B + r) * B + c, t)];
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
          Dk[r][c] = Dinv[tix(B * B, r * B + c, nb)];
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
    for (int c = 0; c < B; ++c) Dinv[tix(B * B, r * B + c, t)] = inv[r][c];
}

// Block ILU(0) diagonals in the tiled red-black order, one thread per tile
// of one colour (red tiles first): the tile's cells in order q = 0..3, each
// D'_q = A~_qq - sum over earlier neighbours k, in direction order, of
// A~_qk D'_k^-1 A~_kq.  Earlier: the tile-mates before q, and for a black
// tile every neighbour in another tile (all of them red).
template <int B>
__global__ void ilu_tiles_kernel(Lay L, int colour, const double* __restrict__ J, const double* __restrict__ R0,
                                 double* Dinv, int* __restrict__ flag) {
  int i, tj, tk;
  if (!tile_of_thread(L, colour, (long)blockIdx.x * blockDim.x + threadIdx.x, i, tj, tk)) return;
  const size_t N = L.n;
  for (int q = 0; q < 4; ++q) {
    const int j = 2 * tj + (q & 1), k = 2 * tk + (q >> 1);
    if (j >= L.ny || k >= L.nz) continue;
    const int t = lay_index(L, i, j, k);
    double D[B][B];
    for (int r = 0; r < B; ++r)
      for (int c = 0; c < B; ++c) D[r][c] = at_blk<B>(J, R0, N, 0, r, c, t);
    for (int d = 1; d < 7; ++d) {
      const int nb = lay_nbr(L, i, j, k, d);
      if (nb < 0) continue;
      const int mate = tile_mate(q, d);
      if (mate >= 0 ? mate > q : colour == 0) continue;   // a later neighbour
      const int od = (d & 1) ? d + 1 : d - 1;   // direction from the neighbour back to t
      double Aik[B][B], Dk[B][B], Aki[B][B], T1[B][B];
      for (int r = 0; r < B; ++r)
        for (int c = 0; c < B; ++c) {
          Aik[r][c] = at_blk<B>(J, R0, N, d, r, c, t);
          Dk[r][c] = Dinv[tix(B * B, r * B + c, nb)];
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
    double inv[B][B];
    if (!small_inverse<B>(D, inv)) atomicExch(flag, 1);
    for (int r = 0; r < B; ++r)
      for (int c = 0; c < B; ++c) Dinv[tix(B * B, r * B + c, t)] = inv[r][c];
  }
}

__global__ void zero_int_kernel(int* p, int n) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = 0;
}

}  // namespace

static void free_levels(cpr_ctx* ctx) {
  for (size_t l = 0; l < ctx->levels.size(); ++l) {
    MGLevel& L = ctx->levels[l];
    for (void* b : {(void*)L.A, (void*)L.Af, (void*)L.x, (void*)L.r, (void*)L.xf, (void*)L.rf, (void*)L.res,
                    (void*)L.resf})
      dev_free(ctx->mem, b);
  }
  ctx->levels.clear();
  dev_free(ctx->mem, ctx->cinv); ctx->cinv = nullptr;
  dev_free(ctx->mem, ctx->cinvf); ctx->cinvf = nullptr;
  dev_free(ctx->mem, ctx->gj_work); ctx->gj_work = nullptr;
}

void release_hierarchy(cpr_ctx* ctx) { free_levels(ctx); }

// Level shapes: each coarse grid has ceil(n/2) cells per axis of the real
// grid above it; coarsening continues while a level has more than
// mg_coarsest real cells.  Smoothed levels are colour-split (padded with a
// ghost column when nx is odd); the coarsest is colour-split for even nx and
// natural otherwise.
static int build_hierarchy(cpr_ctx* ctx) {
  int coarsest = ctx->opt.mg_coarsest;
  std::vector<Lay> shapes;
  shapes.push_back(ctx->lay);
  while (lay_real_cells(shapes.back()) > coarsest) {
    const Lay& f = shapes.back();
    const int nx = (f.nxr + 1) / 2, ny = (f.ny + 1) / 2, nz = (f.nz + 1) / 2;
    if ((long)nx * ny * nz > coarsest)
      shapes.push_back(make_padded_lay(nx, ny, nz));
    else
      shapes.push_back(make_lay(nx, ny, nz, true));
  }
  if (shapes.back().n > 4096) return set_err(ctx, CPR_EINVAL, "coarsest level too large");
  bool same = shapes.size() == ctx->levels.size();
  for (size_t l = 0; same && l < shapes.size(); ++l)
    same = shapes[l].nx == ctx->levels[l].lay.nx && shapes[l].ny == ctx->levels[l].lay.ny &&
           shapes[l].nz == ctx->levels[l].lay.nz && shapes[l].cs == ctx->levels[l].lay.cs &&
           shapes[l].nxr == ctx->levels[l].lay.nxr;
  if (same) return CPR_OK;
  free_levels(ctx);
  ctx->levels.resize(shapes.size());
  for (size_t l = 0; l < shapes.size(); ++l) {
    MGLevel& L = ctx->levels[l];
    L.lay = shapes[l];
    size_t n = L.lay.n;
    CPR_TRY(dev_malloc(ctx->mem, (void**)&L.A, 7 * n * sizeof(double)));
    CPR_TRY(dev_malloc(ctx->mem, (void**)&L.Af, 7 * n * sizeof(float)));
    CPR_TRY(dev_malloc(ctx->mem, (void**)&L.x, n * sizeof(double)));
    CPR_TRY(dev_malloc(ctx->mem, (void**)&L.r, n * sizeof(double)));
    CPR_TRY(dev_malloc(ctx->mem, (void**)&L.xf, n * sizeof(float)));
    CPR_TRY(dev_malloc(ctx->mem, (void**)&L.rf, n * sizeof(float)));
    CPR_TRY(dev_malloc(ctx->mem, (void**)&L.res, (n / 2 + 1) * sizeof(double)));
    CPR_TRY(dev_malloc(ctx->mem, (void**)&L.resf, (n / 2 + 1) * sizeof(float)));
  }
  size_t nc = shapes.back().n;
  CPR_TRY(dev_malloc(ctx->mem, (void**)&ctx->cinv, nc * nc * sizeof(double)));
  CPR_TRY(dev_malloc(ctx->mem, (void**)&ctx->cinvf, nc * nc * sizeof(float)));
  CPR_TRY(dev_malloc(ctx->mem, (void**)&ctx->gj_work, 2 * nc * 2 * nc * sizeof(double)));
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
  // per-cell kernels stream the Jacobian's planes in one-wave workgroups
  int nb = div_up(n, 64);
  const bool abf = ctx->opt.decoupling == CPR_DECOUPLE_ABF;
  if (abf) {
    if (ctx->b == 1)
      abf_kernel<1><<<nb, 64, 0, s>>>(n, ctx->J, ctx->Wabf, ctx->R0, ctx->Jt, ctx->levels[0].A, ctx->flag);
    else if (ctx->b == 2)
      abf_kernel<2><<<nb, 64, 0, s>>>(n, ctx->J, ctx->Wabf, ctx->R0, ctx->Jt, ctx->levels[0].A, ctx->flag);
    else
      abf_kernel<3><<<nb, 64, 0, s>>>(n, ctx->J, ctx->Wabf, ctx->R0, ctx->Jt, ctx->levels[0].A, ctx->flag);
  } else if (ctx->b == 1) {
    qimpes_kernel<1><<<nb, 64, 0, s>>>(n, ctx->J, ctx->w, ctx->R0, ctx->levels[0].A, ctx->flag + 1);
  } else if (ctx->b == 2) {
    qimpes_kernel<2><<<nb, 64, 0, s>>>(n, ctx->J, ctx->w, ctx->R0, ctx->levels[0].A, ctx->flag + 1);
  } else {
    qimpes_kernel<3><<<nb, 64, 0, s>>>(n, ctx->J, ctx->w, ctx->R0, ctx->levels[0].A, ctx->flag + 1);
  }
  // rows >= 1 of the decoupled blocks: the Jacobian's own (quasi-IMPES) or D^-1 A (ABF)
  const double* Jdec = abf ? ctx->Jt : ctx->J;
  // Galerkin chain and coarsest inverse on the auxiliary stream, the ILU
  // factorisation meanwhile on the caller's stream
  hipStream_t a = ctx->aux;
  CPR_TRY(hipEventRecord(ctx->ev_q, s));
  CPR_TRY(hipStreamWaitEvent(a, ctx->ev_q, 0));
  for (size_t l = 0; l + 1 < ctx->levels.size(); ++l) {
    const MGLevel& F = ctx->levels[l];
    MGLevel& C = ctx->levels[l + 1];
    rap_kernel<<<div_up(8L * C.lay.n, 256), 256, 0, a>>>(F.lay, C.lay, F.A, C.A);
  }
  CPR_TRY(hipEventRecord(ctx->ev_rap, a));
  // dense inverse of the coarsest level
  const MGLevel& last = ctx->levels.back();
  int nc = last.lay.n;
  if (nc <= GJ_LDS_MAX) {
    const size_t smem = ((size_t)SCH_MAX * SCH_LD + (size_t)SCH_MAX * SCH_MAX) * sizeof(double);
    static bool attr_set = false;
    if (!attr_set) {
      CPR_TRY(hipFuncSetAttribute((const void*)gj_schur_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)smem));
      attr_set = true;
    }
    gj_schur_kernel<<<1, 1024, smem, a>>>(last.lay, last.A, ctx->cinv, ctx->cinvf, ctx->flag);
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
  // block ILU(0): red diagonals (cells or tiles) first, black ones use them
  const bool tiles = ctx->opt.ilu_order == CPR_ILU_TILES;
  const int nh = tiles ? (int)div_up(tile_threads(L), 64) : div_up(L.nh, 64);
  for (int colour = 0; colour < 2; ++colour) {
    if (tiles) {
      if (ctx->b == 1)
        ilu_tiles_kernel<1><<<nh, 64, 0, s>>>(L, colour, Jdec, ctx->R0, ctx->Dinv, ctx->flag);
      else if (ctx->b == 2)
        ilu_tiles_kernel<2><<<nh, 64, 0, s>>>(L, colour, Jdec, ctx->R0, ctx->Dinv, ctx->flag);
      else
        ilu_tiles_kernel<3><<<nh, 64, 0, s>>>(L, colour, Jdec, ctx->R0, ctx->Dinv, ctx->flag);
    } else if (ctx->b == 1) {
      ilu_kernel<1><<<nh, 64, 0, s>>>(L, colour, Jdec, ctx->R0, ctx->Dinv, ctx->flag);
    } else if (ctx->b == 2) {
      ilu_kernel<2><<<nh, 64, 0, s>>>(L, colour, Jdec, ctx->R0, ctx->Dinv, ctx->flag);
    } else {
      ilu_kernel<3><<<nh, 64, 0, s>>>(L, colour, Jdec, ctx->R0, ctx->Dinv, ctx->flag);
    }
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
