// Block 7-point sparse matrix-vector product y = A x (or y = rhs - A x).
//
// One thread per cell, colour-split order.  The 7 b x b blocks of a block
// row sit in 7*b*b planes, so consecutive threads read consecutive doubles
// of every plane; the neighbours' x values come from the other colour's
// half at a fixed offset (+-y, +-z) or at m / m +- 1 (+-x).  HBM traffic per
// cell: 7 b^2 matrix values + b values of x + b of y (+ b of rhs).
#include "internal.h"

namespace {

template <int B>
__global__ __launch_bounds__(256) void spmv_kernel(Lay L, const double* __restrict__ A,
                                                   const double* __restrict__ x,
                                                   double* __restrict__ y,
                                                   const double* __restrict__ rhs) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= L.n) return;
  const size_t n = L.n;
  int i, j, k;
  lay_coords(L, t, i, j, k);
  double acc[B];
  for (int r = 0; r < B; ++r) acc[r] = 0.0;
#pragma unroll
  for (int d = 0; d < 7; ++d) {
    int nb = d == 0 ? t : lay_nbr(L, i, j, k, d);
    if (nb < 0) continue;
    double xv[B];
#pragma unroll
    for (int c = 0; c < B; ++c) xv[c] = x[c * n + nb];
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
      for (int c = 0; c < B; ++c) acc[r] += A[((size_t)(d * B + r) * B + c) * n + t] * xv[c];
  }
#pragma unroll
  for (int r = 0; r < B; ++r) y[r * n + t] = rhs ? rhs[r * n + t] - acc[r] : acc[r];
}

}  // namespace

void launch_spmv(int b, const Lay& L, const double* A, const double* x, double* y,
                 const double* rhs, hipStream_t s) {
  int nb = div_up(L.n, 256);
  if (b == 2)
    spmv_kernel<2><<<nb, 256, 0, s>>>(L, A, x, y, rhs);
  else
    spmv_kernel<3><<<nb, 256, 0, s>>>(L, A, x, y, rhs);
}
