// Block 7-point sparse matrix-vector product y = A x (or y = rhs - A x).
//
// One thread per cell, colour-split order.  The 7 b x b blocks of a block
// row sit in 7*b*b planes stored in 64-cell tiles, so a wave reads its
// cells' whole matrix rows as one contiguous block of 7*b*b runs of 64
// doubles; the neighbours' x values come from the other colour's half at a
// fixed offset (+-y, +-z) or at m / m +- 1 (+-x), and the XCD-aware
// workgroup order keeps the rows of x that neighbouring workgroups share in
// one L2.  HBM traffic per cell: 7 b^2 matrix values + b values of x + b of
// y (+ b of rhs).
#include "internal.h"

namespace {

// 3x3 systems up to this many cells take the one-wave kernel below: on
// MI355X it streams the 128x128x32 black-oil matrix about 15 % faster,
// while the kernel above is faster on the 4.2 M-cell grids.
constexpr int SPMV_SMALL_N = 1 << 20;

// Branch-free: blocks towards missing neighbours are stored as zeros,
// missing neighbours read the cell itself and are masked to zero.  The
// matrix is streamed once per call, so its loads are non-temporal and leave
// the caches to x.  y = rhs - A x and y = A x are separate instantiations:
// with the choice made per store the compiler kept all 63 matrix values
// live at once (130 VGPRs); without it it interleaves loads and FMAs in 64,
// and at 512x512x128 the product runs about 3 % faster.
template <int B, bool RHS>
__global__ __launch_bounds__(256) void spmv_kernel(Lay L, const double* __restrict__ A,
                                                   const double* __restrict__ x,
                                                   double* __restrict__ y,
                                                   const double* __restrict__ rhs) {
  int t = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (t >= L.n) return;
  const size_t n = L.n;
  CsCell cc = cs_decode(L, t);
  int nbr[7];
  bool ok[7];
  cs_nbrs(L, t, cc, nbr, ok);
  double a[7][B][B];
#pragma unroll
  for (int d = 0; d < 7; ++d)
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
      for (int c = 0; c < B; ++c) a[d][r][c] = __builtin_nontemporal_load(A + tix(7 * B * B, (d * B + r) * B + c, t));
  double acc[B];
#pragma unroll
  for (int r = 0; r < B; ++r) acc[r] = 0.0;
#pragma unroll
  for (int d = 0; d < 7; ++d) {
    double xv[B];
#pragma unroll
    for (int c = 0; c < B; ++c) {
      double v = x[c * n + nbr[d]];
      xv[c] = ok[d] ? v : 0.0;
    }
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
      for (int c = 0; c < B; ++c) acc[r] += a[d][r][c] * xv[c];
  }
#pragma unroll
  for (int r = 0; r < B; ++r) y[r * n + t] = RHS ? rhs[r * n + t] - acc[r] : acc[r];
}

// The same product for systems up to SPMV_SMALL_N cells, one wave per
// workgroup (a finer tail at these sizes).  Sums are formed in the same
// order as above.
template <int B>
__device__ inline void spmv_cell(const Lay& L, int t, const double* __restrict__ A, const double* __restrict__ x,
                                 double* __restrict__ y, const double* __restrict__ rhs) {
  const size_t n = L.n;
  CsCell cc = cs_decode(L, t);
  int nbr[7];
  bool ok[7];
  cs_nbrs(L, t, cc, nbr, ok);
  double acc[B];
#pragma unroll
  for (int r = 0; r < B; ++r) acc[r] = 0.0;
  double a[7][B][B];
#pragma unroll
  for (int d = 0; d < 7; ++d)
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
      for (int c = 0; c < B; ++c) a[d][r][c] = __builtin_nontemporal_load(A + tix(7 * B * B, (d * B + r) * B + c, t));
#pragma unroll
  for (int d = 0; d < 7; ++d) {
    double xv[B];
#pragma unroll
    for (int c = 0; c < B; ++c) {
      double v = x[c * n + nbr[d]];
      xv[c] = ok[d] ? v : 0.0;
    }
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
      for (int c = 0; c < B; ++c) acc[r] += a[d][r][c] * xv[c];
  }
#pragma unroll
  for (int r = 0; r < B; ++r) y[r * n + t] = rhs ? rhs[r * n + t] - acc[r] : acc[r];
}

template <int B>
__global__ __launch_bounds__(64) void spmv_small_kernel(Lay L, const double* __restrict__ A,
                                                        const double* __restrict__ x, double* __restrict__ y,
                                                        const double* __restrict__ rhs) {
  int t = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (t < L.n) spmv_cell<B>(L, t, A, x, y, rhs);
}

template <int B>
void launch_big(const Lay& L, const double* A, const double* x, double* y, const double* rhs, hipStream_t s) {
  const int nb = div_up(L.n, 256);
  if (rhs)
    spmv_kernel<B, true><<<nb, 256, 0, s>>>(L, A, x, y, rhs);
  else
    spmv_kernel<B, false><<<nb, 256, 0, s>>>(L, A, x, y, rhs);
}

}  // namespace

void launch_spmv(int b, const Lay& L, const double* A, const double* x, double* y,
                 const double* rhs, hipStream_t s) {
  if (b == 3 && L.n <= SPMV_SMALL_N)
    spmv_small_kernel<3><<<div_up(L.n, 64), 64, 0, s>>>(L, A, x, y, rhs);
  else if (b == 1)
    launch_big<1>(L, A, x, y, rhs, s);
  else if (b == 2)
    launch_big<2>(L, A, x, y, rhs, s);
  else
    launch_big<3>(L, A, x, y, rhs, s);
}
