// CPR preconditioner application z = M^-1 v.
//
//   r~   = v with r~_0 = w^T v                    (quasi-IMPES decoupling)
//   dp   = V(1,1)-cycle on A_p r~_0               (pressure stage, Sec. 2.5)
//   r2   = r~ - A~(:, p) dp
//   y    = (D' + L)^-1 r2 ;  z = y - D'^-1 U z     (red-black block ILU(0))
//   z_0 += dp
//
// Kernels are templated on the preconditioner's scalar type T: double for
// the FP64 path, float for the mixed-precision path (v and z stay FP64 at
// the boundary; the coarsest pressure solve is always FP64).  Every colour
// kernel runs one thread per cell of that colour; in the colour-split
// layout all its neighbours live in the other half.
#include "internal.h"

namespace {

template <typename T>
struct Pre;
template <>
struct Pre<double> {
  static const double* R0(const cpr_ctx* c) { return c->R0; }
  static const double* J(const cpr_ctx* c) { return c->J; }
  static const double* Dinv(const cpr_ctx* c) { return c->Dinv; }
  static const double* A(const MGLevel& l) { return l.A; }
  static double* x(MGLevel& l) { return l.x; }
  static double* r(MGLevel& l) { return l.r; }
  static double* Y(cpr_ctx* c) { return c->Y; }
  static double* rp(cpr_ctx* c) { return c->rp; }
};
template <>
struct Pre<float> {
  static const float* R0(const cpr_ctx* c) { return c->Jf + 0; }   // row-0 planes of the FP32 copy
  static const float* J(const cpr_ctx* c) { return c->Jf; }
  static const float* Dinv(const cpr_ctx* c) { return c->Dinvf; }
  static const float* A(const MGLevel& l) { return l.Af; }
  static float* x(MGLevel& l) { return l.xf; }
  static float* r(MGLevel& l) { return l.rf; }
  static float* Y(cpr_ctx* c) { return c->Yf; }
  static float* rp(cpr_ctx* c) { return c->rpf; }
};

// Decoupled block entry (d, r, c) of cell t.  FP64: row 0 lives in R0
// [7][b][n]; FP32: the copy holds full decoupled blocks [7][b][b][n].
template <int B, typename T>
__device__ inline T at_blk(const T* __restrict__ J, const T* __restrict__ R0, size_t N, int d, int r,
                           int c, int t) {
  if constexpr (sizeof(T) == 8) {
    return r == 0 ? R0[((size_t)d * B + c) * N + t] : J[((size_t)(d * B + r) * B + c) * N + t];
  } else {
    return J[((size_t)(d * B + r) * B + c) * N + t];
  }
}

template <int B, typename T>
__global__ __launch_bounds__(256) void decouple_kernel(int n, const double* __restrict__ w,
                                                       const double* __restrict__ v, T* __restrict__ rp) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < B; ++r) s += w[(size_t)r * n + t] * v[(size_t)r * n + t];
  rp[t] = (T)s;
}

// Red-black Gauss-Seidel half-sweep on a scalar 7-point level:
// x_i = (r_i - sum_{d>0} a_id x_nb) / a_i0 for cells of one colour.
// zero_guess: the other colour is taken as zero (first pre-smoothing sweep).
template <typename T>
__global__ __launch_bounds__(256) void gs_kernel(Lay L, int colour, int zero_guess,
                                                 const T* __restrict__ A, const T* __restrict__ r,
                                                 T* __restrict__ x) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= L.nh) return;
  int t = colour * L.nh + q;
  T off = 0;
  if (!zero_guess) {
    int i, j, k;
    lay_coords(L, t, i, j, k);
#pragma unroll
    for (int d = 1; d < 7; ++d) {
      int nb = lay_nbr(L, i, j, k, d);
      if (nb >= 0) off += A[(size_t)d * L.n + t] * x[nb];
    }
  }
  x[t] = (r[t] - off) / A[t];
}

// Residual r - A x of the (up to) 8 fine cells of each coarse cell, summed
// into the coarse right-hand side (P^T applied to the residual).
template <typename T>
__global__ __launch_bounds__(256) void resid_restrict_kernel(Lay F, Lay C, const T* __restrict__ A,
                                                             const T* __restrict__ r,
                                                             const T* __restrict__ x,
                                                             T* __restrict__ rc) {
  int tc = blockIdx.x * blockDim.x + threadIdx.x;
  if (tc >= C.n) return;
  int ci, cj, ck;
  lay_coords(C, tc, ci, cj, ck);
  T acc = 0;
  for (int fk = 2 * ck; fk <= 2 * ck + 1 && fk < F.nz; ++fk)
    for (int fj = 2 * cj; fj <= 2 * cj + 1 && fj < F.ny; ++fj)
      for (int fi = 2 * ci; fi <= 2 * ci + 1 && fi < F.nx; ++fi) {
        int f = lay_index(F, fi, fj, fk);
        T y = A[f] * x[f];
#pragma unroll
        for (int d = 1; d < 7; ++d) {
          int nb = lay_nbr(F, fi, fj, fk, d);
          if (nb >= 0) y += A[(size_t)d * F.n + f] * x[nb];
        }
        acc += r[f] - y;
      }
  rc[tc] = acc;
}

// x_f += alpha * e_c[agg(f)] on the red cells (the black post-smoothing
// sweep overwrites the black values, so only red cells need it).
template <typename T>
__global__ __launch_bounds__(256) void prolong_red_kernel(Lay F, Lay C, T alpha, const T* __restrict__ ec,
                                                          T* __restrict__ x) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= F.nh) return;
  int i, j, k;
  lay_coords(F, q, i, j, k);
  x[q] += alpha * ec[lay_index(C, i >> 1, j >> 1, k >> 1)];
}

// Coarsest level: x = A^-1 r with the dense FP64 inverse (column major).
template <typename T>
__global__ void coarse_gemv_kernel(int nc, const double* __restrict__ inv, const T* __restrict__ r,
                                   T* __restrict__ x) {
  int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= nc) return;
  double s = 0.0;
  for (int c = 0; c < nc; ++c) s += inv[(size_t)c * nc + row] * (double)r[c];
  x[row] = (T)s;
}

// Stage-2 residual r2 = r~ - A~(:, p) dp at cell t.
template <int B, typename T>
__device__ inline void stage2_resid(const Lay& L, int t, int i, int j, int k, const T* J, const T* R0,
                                    const double* __restrict__ v, const T* __restrict__ rp,
                                    const T* __restrict__ dp, T (&r2)[B]) {
  const size_t N = L.n;
  r2[0] = rp[t];
#pragma unroll
  for (int r = 1; r < B; ++r) r2[r] = (T)v[r * N + t];
#pragma unroll
  for (int d = 0; d < 7; ++d) {
    int nb = d == 0 ? t : lay_nbr(L, i, j, k, d);
    if (nb < 0) continue;
    T p = dp[nb];
#pragma unroll
    for (int r = 0; r < B; ++r) r2[r] -= at_blk<B, T>(J, R0, N, d, r, 0, t) * p;
  }
}

template <int B, typename T>
__device__ inline void offdiag_apply(const Lay& L, int t, int i, int j, int k, const T* J, const T* R0,
                                     const T* __restrict__ Y, T (&s)[B]) {
  const size_t N = L.n;
#pragma unroll
  for (int r = 0; r < B; ++r) s[r] = 0;
#pragma unroll
  for (int d = 1; d < 7; ++d) {
    int nb = lay_nbr(L, i, j, k, d);
    if (nb < 0) continue;
    T y[B];
#pragma unroll
    for (int c = 0; c < B; ++c) y[c] = Y[c * N + nb];
#pragma unroll
    for (int r = 0; r < B; ++r) {
      T a = 0;
#pragma unroll
      for (int c = 0; c < B; ++c) a += at_blk<B, T>(J, R0, N, d, r, c, t) * y[c];
      s[r] += a;
    }
  }
}

template <int B, typename T>
__device__ inline void dinv_apply(const T* __restrict__ Dinv, size_t N, int t, const T (&in)[B], T (&out)[B]) {
#pragma unroll
  for (int r = 0; r < B; ++r) {
    T a = 0;
#pragma unroll
    for (int c = 0; c < B; ++c) a += Dinv[((size_t)r * B + c) * N + t] * in[c];
    out[r] = a;
  }
}

// red cells: forward ILU step y_r = D'^-1 r2_r (no lower neighbours)
template <int B, typename T>
__global__ __launch_bounds__(256) void stage2_red_fwd_kernel(Lay L, const T* __restrict__ J,
                                                             const T* __restrict__ R0,
                                                             const T* __restrict__ Dinv,
                                                             const double* __restrict__ v,
                                                             const T* __restrict__ rp,
                                                             const T* __restrict__ dp, T* __restrict__ Y) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= L.nh) return;
  int i, j, k;
  lay_coords(L, t, i, j, k);
  T r2[B], y[B];
  stage2_resid<B, T>(L, t, i, j, k, J, R0, v, rp, dp, r2);
  dinv_apply<B, T>(Dinv, L.n, t, r2, y);
#pragma unroll
  for (int r = 0; r < B; ++r) Y[(size_t)r * L.n + t] = y[r];
}

// black cells: y_b = D'^-1 (r2_b - sum_red A~_bk y_k); no upper neighbours,
// so z_b = y_b (+ dp on the pressure unknown)
template <int B, typename T>
__global__ __launch_bounds__(256) void stage2_black_kernel(Lay L, const T* __restrict__ J,
                                                           const T* __restrict__ R0,
                                                           const T* __restrict__ Dinv,
                                                           const double* __restrict__ v,
                                                           const T* __restrict__ rp,
                                                           const T* __restrict__ dp, T* __restrict__ Y,
                                                           double* __restrict__ z) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= L.nh) return;
  int t = L.nh + q;
  int i, j, k;
  lay_coords(L, t, i, j, k);
  T r2[B], s[B], y[B];
  stage2_resid<B, T>(L, t, i, j, k, J, R0, v, rp, dp, r2);
  offdiag_apply<B, T>(L, t, i, j, k, J, R0, Y, s);
#pragma unroll
  for (int r = 0; r < B; ++r) r2[r] -= s[r];
  dinv_apply<B, T>(Dinv, L.n, t, r2, y);
  const size_t N = L.n;
#pragma unroll
  for (int r = 0; r < B; ++r) Y[r * N + t] = y[r];
  z[t] = (double)y[0] + (double)dp[t];
#pragma unroll
  for (int r = 1; r < B; ++r) z[r * N + t] = (double)y[r];
}

// red cells, backward step: z_r = y_r - D'^-1 sum_black A~_rk y_k
template <int B, typename T>
__global__ __launch_bounds__(256) void stage2_red_bwd_kernel(Lay L, const T* __restrict__ J,
                                                             const T* __restrict__ R0,
                                                             const T* __restrict__ Dinv,
                                                             const T* __restrict__ dp,
                                                             const T* __restrict__ Y,
                                                             double* __restrict__ z) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= L.nh) return;
  int i, j, k;
  lay_coords(L, t, i, j, k);
  T s[B], u[B];
  offdiag_apply<B, T>(L, t, i, j, k, J, R0, Y, s);
  dinv_apply<B, T>(Dinv, L.n, t, s, u);
  const size_t N = L.n;
  z[t] = (double)(Y[t] - u[0]) + (double)dp[t];
#pragma unroll
  for (int r = 1; r < B; ++r) z[r * N + t] = (double)(Y[r * N + t] - u[r]);
}

template <typename T>
void vcycle(cpr_ctx* ctx, size_t l) {
  hipStream_t s = ctx->stream;
  MGLevel& L = ctx->levels[l];
  if (l + 1 == ctx->levels.size()) {
    int nc = L.lay.n;
    coarse_gemv_kernel<T><<<div_up(nc, 128), 128, 0, s>>>(nc, ctx->cinv, Pre<T>::r(L), Pre<T>::x(L));
    return;
  }
  MGLevel& C = ctx->levels[l + 1];
  const T* A = Pre<T>::A(L);
  T* x = Pre<T>::x(L);
  const T* r = Pre<T>::r(L);
  int nh = div_up(L.lay.nh, 256);
  prof_begin(ctx, CPR_KCLASS_SMOOTH);
  gs_kernel<T><<<nh, 256, 0, s>>>(L.lay, 0, 1, A, r, x);
  prof_end(ctx, CPR_KCLASS_SMOOTH);
  prof_begin(ctx, CPR_KCLASS_SMOOTH);
  gs_kernel<T><<<nh, 256, 0, s>>>(L.lay, 1, 0, A, r, x);
  prof_end(ctx, CPR_KCLASS_SMOOTH);
  resid_restrict_kernel<T><<<div_up(C.lay.n, 256), 256, 0, s>>>(L.lay, C.lay, A, r, x, Pre<T>::r(C));
  vcycle<T>(ctx, l + 1);
  prolong_red_kernel<T><<<nh, 256, 0, s>>>(L.lay, C.lay, (T)ctx->opt.mg_alpha, Pre<T>::x(C), x);
  prof_begin(ctx, CPR_KCLASS_SMOOTH);
  gs_kernel<T><<<nh, 256, 0, s>>>(L.lay, 1, 0, A, r, x);
  prof_end(ctx, CPR_KCLASS_SMOOTH);
  prof_begin(ctx, CPR_KCLASS_SMOOTH);
  gs_kernel<T><<<nh, 256, 0, s>>>(L.lay, 0, 0, A, r, x);
  prof_end(ctx, CPR_KCLASS_SMOOTH);
}

template <int B, typename T>
void apply_impl(cpr_ctx* ctx, const double* v, double* z) {
  hipStream_t s = ctx->stream;
  const Lay& L = ctx->lay;
  MGLevel& L0 = ctx->levels[0];
  T* rp = Pre<T>::r(L0);
  decouple_kernel<B, T><<<div_up(L.n, 256), 256, 0, s>>>(L.n, ctx->w, v, rp);
  vcycle<T>(ctx, 0);
  const T* dp = Pre<T>::x(L0);
  const T* J = Pre<T>::J(ctx);
  const T* R0 = Pre<T>::R0(ctx);
  const T* Dinv = Pre<T>::Dinv(ctx);
  T* Y = Pre<T>::Y(ctx);
  int nh = div_up(L.nh, 256);
  prof_begin(ctx, CPR_KCLASS_ILU);
  stage2_red_fwd_kernel<B, T><<<nh, 256, 0, s>>>(L, J, R0, Dinv, v, rp, dp, Y);
  prof_end(ctx, CPR_KCLASS_ILU);
  prof_begin(ctx, CPR_KCLASS_ILU);
  stage2_black_kernel<B, T><<<nh, 256, 0, s>>>(L, J, R0, Dinv, v, rp, dp, Y, z);
  prof_end(ctx, CPR_KCLASS_ILU);
  prof_begin(ctx, CPR_KCLASS_ILU);
  stage2_red_bwd_kernel<B, T><<<nh, 256, 0, s>>>(L, J, R0, Dinv, dp, Y, z);
  prof_end(ctx, CPR_KCLASS_ILU);
}

// FP32 copies: decoupled blocks (row 0 from R0), ILU diagonals, MG levels.
template <int B>
__global__ void mixed_copy_kernel(int n, const double* __restrict__ J, const double* __restrict__ R0,
                                  const double* __restrict__ Dinv, float* __restrict__ Jf,
                                  float* __restrict__ Dinvf) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const size_t N = n;
  for (int d = 0; d < 7; ++d)
    for (int r = 0; r < B; ++r)
      for (int c = 0; c < B; ++c) {
        size_t o = ((size_t)(d * B + r) * B + c) * N + t;
        Jf[o] = (float)(r == 0 ? R0[((size_t)d * B + c) * N + t] : J[o]);
      }
  for (int e = 0; e < B * B; ++e) Dinvf[e * N + t] = (float)Dinv[e * N + t];
}

__global__ void to_float_kernel(size_t n, const double* __restrict__ a, float* __restrict__ b) {
  size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) b[t] = (float)a[t];
}

}  // namespace

void launch_mixed_copies(cpr_ctx* ctx) {
  hipStream_t s = ctx->stream;
  int n = ctx->lay.n;
  if (ctx->b == 2)
    mixed_copy_kernel<2><<<div_up(n, 256), 256, 0, s>>>(n, ctx->J, ctx->R0, ctx->Dinv, ctx->Jf, ctx->Dinvf);
  else
    mixed_copy_kernel<3><<<div_up(n, 256), 256, 0, s>>>(n, ctx->J, ctx->R0, ctx->Dinv, ctx->Jf, ctx->Dinvf);
  for (auto& L : ctx->levels) {
    size_t m = (size_t)7 * L.lay.n;
    to_float_kernel<<<div_up((long)m, 256), 256, 0, s>>>(m, L.A, L.Af);
  }
}

void precond_apply(cpr_ctx* ctx, const double* v, double* z) {
  bool mixed = ctx->opt.precision == CPR_PREC_MIXED;
  if (ctx->b == 2) {
    if (mixed) apply_impl<2, float>(ctx, v, z); else apply_impl<2, double>(ctx, v, z);
  } else {
    if (mixed) apply_impl<3, float>(ctx, v, z); else apply_impl<3, double>(ctx, v, z);
  }
}
