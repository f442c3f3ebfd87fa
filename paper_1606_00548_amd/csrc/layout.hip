// Natural <-> colour-split permutation of per-cell planes.
#include "internal.h"

namespace {

// One thread per natural cell index of the real grid (nxr columns); the
// natural read is coalesced, the colour-split write lands in two contiguous
// halves.  Natural planes hold the real cells only; ghost cells of a padded
// layout are neither read nor written.
__global__ void nat_to_cs_kernel(Lay L, int planes, const double* __restrict__ src,
                                 double* __restrict__ dst) {
  const int nr = L.nxr * L.ny * L.nz;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nr) return;
  int i = t % L.nxr, jk = t / L.nxr;
  int j = jk % L.ny, k = jk / L.ny;
  int c = lay_index(L, i, j, k);
  for (int p = 0; p < planes; ++p) dst[(size_t)p * L.n + c] = src[(size_t)p * nr + t];
}

__global__ void cs_to_nat_kernel(Lay L, int planes, const double* __restrict__ src,
                                 double* __restrict__ dst) {
  const int nr = L.nxr * L.ny * L.nz;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nr) return;
  int i = t % L.nxr, jk = t / L.nxr;
  int j = jk % L.ny, k = jk / L.ny;
  int c = lay_index(L, i, j, k);
  for (int p = 0; p < planes; ++p) dst[(size_t)p * nr + t] = src[(size_t)p * L.n + c];
}

// Natural planes <-> tiled block array (cell t of plane p at tix(P, p, t)).
__global__ void nat_to_tiled_kernel(Lay L, int planes, const double* __restrict__ src,
                                    double* __restrict__ dst) {
  const int nr = L.nxr * L.ny * L.nz;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nr) return;
  int i = t % L.nxr, jk = t / L.nxr;
  int j = jk % L.ny, k = jk / L.ny;
  int c = lay_index(L, i, j, k);
  for (int p = 0; p < planes; ++p) dst[tix(planes, p, c)] = src[(size_t)p * nr + t];
}

__global__ void tiled_to_nat_kernel(Lay L, int planes, const double* __restrict__ src,
                                    double* __restrict__ dst) {
  const int nr = L.nxr * L.ny * L.nz;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nr) return;
  int i = t % L.nxr, jk = t / L.nxr;
  int j = jk % L.ny, k = jk / L.ny;
  int c = lay_index(L, i, j, k);
  for (int p = 0; p < planes; ++p) dst[(size_t)p * nr + t] = src[tix(planes, p, c)];
}

}  // namespace

void launch_nat_to_tiled(const Lay& L, int planes, const double* src, double* dst, hipStream_t s) {
  if (L.n == 0) return;
  nat_to_tiled_kernel<<<div_up(lay_real_cells(L), 256), 256, 0, s>>>(L, planes, src, dst);
}

void launch_tiled_to_nat(const Lay& L, int planes, const double* src, double* dst, hipStream_t s) {
  if (L.n == 0) return;
  tiled_to_nat_kernel<<<div_up(lay_real_cells(L), 256), 256, 0, s>>>(L, planes, src, dst);
}

void launch_nat_to_cs(const Lay& L, int planes, const double* src, double* dst, hipStream_t s) {
  if (L.n == 0) return;
  nat_to_cs_kernel<<<div_up(lay_real_cells(L), 256), 256, 0, s>>>(L, planes, src, dst);
}

void launch_cs_to_nat(const Lay& L, int planes, const double* src, double* dst, hipStream_t s) {
  if (L.n == 0) return;
  cs_to_nat_kernel<<<div_up(lay_real_cells(L), 256), 256, 0, s>>>(L, planes, src, dst);
}
