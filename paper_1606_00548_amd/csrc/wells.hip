// Rate-controlled wells (eqs. (8)-(9)): their bottom-hole pressures are
// unknowns appended to every vector, and the Jacobian gains the border of
// eq. (16):
//     [ A  B ] [dx  ]   [b_cells]
//     [ C  D ] [dp_h] = [b_wells]
// B = dR_cells/dp_h and C = dR_w/dx_cells are non-zero only at a well's own
// perforations (one column / row of b entries per perforation), D =
// dR_w/dp_h is diagonal.  One thread per rate well walks its perforations
// (distinct cells, so no two threads touch the same entry) in perforation
// order.  The preconditioner keeps CPR on A and solves each well equation
// for its BHP given the cell correction: z_w = (r_w - C z_cells) / D
// (block lower-triangular).
#include "internal.h"

namespace {

constexpr int BW = 64;   // threads per block of the per-well kernels

// Per perforation q: bord[q*6 + r] = B entries (rows r), bord[q*6 + 3 + u]
// = C entries (columns u).
__global__ void border_spmv_kernel(int b, int n, int nrate, const RateWell* __restrict__ rw,
                                   const Perf* __restrict__ perfs, const double* __restrict__ bord,
                                   const double* __restrict__ bordD, const double* __restrict__ x,
                                   double* __restrict__ y, const double* __restrict__ rhs) {
  int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nrate) return;
  const long bn = (long)b * n;
  const RateWell R = rw[w];
  const double xw = x[bn + w];
  double acc = 0.0;
  for (int q = R.p0; q < R.p1; ++q) {
    const int c = perfs[q].cell;
    const double* Bq = bord + (size_t)q * 6;
    for (int r = 0; r < b; ++r) {
      acc += Bq[3 + r] * x[(size_t)r * n + c];
      const double t = Bq[r] * xw;
      y[(size_t)r * n + c] += rhs ? -t : t;
    }
  }
  acc += bordD[w] * xw;
  y[bn + w] = rhs ? rhs[bn + w] - acc : acc;
}

__global__ void border_precond_kernel(int b, int n, int nrate, const RateWell* __restrict__ rw,
                                      const Perf* __restrict__ perfs, const double* __restrict__ bord,
                                      const double* __restrict__ bordD, const double* vin, double* v,
                                      const double* __restrict__ nrm2, double* __restrict__ z) {
  int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nrate) return;
  const long bn = (long)b * n;
  const RateWell R = rw[w];
  double vw = vin[bn + w];
  if (nrm2) {
    vw = vw / sqrt(*nrm2);
    v[bn + w] = vw;
  }
  double acc = 0.0;
  for (int q = R.p0; q < R.p1; ++q) {
    const int c = perfs[q].cell;
    const double* Cq = bord + (size_t)q * 6 + 3;
    for (int u = 0; u < b; ++u) acc += Cq[u] * z[(size_t)u * n + c];
  }
  z[bn + w] = (vw - acc) / bordD[w];
}

}  // namespace

void system_spmv(cpr_ctx* ctx, const double* x, double* y, const double* rhs) {
  launch_spmv(ctx->b, ctx->lay, ctx->J, x, y, rhs, ctx->stream);
  if (ctx->nrate)
    border_spmv_kernel<<<div_up(ctx->nrate, BW), BW, 0, ctx->stream>>>(
        ctx->b, ctx->lay.n, ctx->nrate, ctx->rwells_d, ctx->perfs_d, ctx->bord, ctx->bord_d, x, y, rhs);
}

void border_precond(cpr_ctx* ctx, const double* vin, double* v, const double* nrm2, double* z) {
  if (!ctx->nrate) return;
  border_precond_kernel<<<div_up(ctx->nrate, BW), BW, 0, ctx->stream>>>(
      ctx->b, ctx->lay.n, ctx->nrate, ctx->rwells_d, ctx->perfs_d, ctx->bord, ctx->bord_d, vin, v, nrm2, z);
}

hipError_t vec_nat_to_cs(cpr_ctx* ctx, const double* src, double* dst) {
  launch_nat_to_cs(ctx->lay, ctx->b, src, dst, ctx->stream);
  const long bn = (long)ctx->b * ctx->lay.n;
  if (!ctx->nrate) return hipSuccess;
  return hipMemcpyAsync(dst + bn, src + bn, ctx->nrate * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream);
}

hipError_t vec_cs_to_nat(cpr_ctx* ctx, const double* src, double* dst) {
  launch_cs_to_nat(ctx->lay, ctx->b, src, dst, ctx->stream);
  const long bn = (long)ctx->b * ctx->lay.n;
  if (!ctx->nrate) return hipSuccess;
  return hipMemcpyAsync(dst + bn, src + bn, ctx->nrate * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream);
}
