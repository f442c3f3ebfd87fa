// CPR preconditioner application z = M^-1 v.
//
//   r~   = v with r~_0 = w^T v                    (quasi-IMPES decoupling)
//   dp   = V(1,1)-cycle on A_p r~_0               (pressure stage, Sec. 2.5)
//   r2   = r~ - A~(:, p) dp
//   y    = (D' + L)^-1 r2 ;  z = y - D'^-1 U z     (red-black block ILU(0))
//   z_0 += dp
//
// Variants (Sec. 2.5 names both): ABF decoupling r~ = D^-1 v per cell with
// A~ = D^-1 A, and the F-P-F composition, which first applies the block
// ILU(0) to r~ (z1), runs the two stages above on r1 = r~ - A~ z1 and adds
// z1 to the result.
//
// Kernels are templated on the preconditioner's scalar type T: double for
// the FP64 path, float for the mixed-precision path (v and z stay FP64 at
// the boundary; the coarsest pressure solve is always FP64).  Every colour
// kernel runs one thread per cell of that colour; in the colour-split
// layout all of a cell's neighbours live in the other half.
//
// V(1,1) cycle per level: red sweep from a zero guess (fused with the
// decoupling on the fine level), black sweep (which also records the black
// residuals), restriction of r - A x by 2x2x2 aggregation, coarse solve,
// black post-sweep reading the prolongated red values x + alpha e_c on the
// fly (the prolongated red values themselves are overwritten by the red
// post-sweep, so they are never stored), red post-sweep.  All levels from
// the first one with at most FUSE_MAX cells down to the dense coarsest solve
// run in one single-workgroup kernel, which removes a dozen latency-bound
// launches per cycle.
#include "internal.h"

namespace {

constexpr int FUSE_MAX = 4096;   // cells of the first level handled by the fused kernel
constexpr int DENSE_FUSED_MAX = 1024;
constexpr int DENSE_PF = 16;
constexpr int STAGE_UNROLL = 8;  // loads per thread in flight while the fused kernel stages its levels     // coarsest-inverse entries per thread loaded at the fused kernel's start
constexpr int MAXLV = 16;
// Threads per workgroup of the per-cell kernels (sweeps, restriction,
// decoupling): one wave per workgroup streams their planes faster than four.
constexpr int SB = 64;

template <typename T>
struct Pre;
template <>
struct Pre<double> {
  static const double* R0(const cpr_ctx* c) { return c->R0; }
  static const double* J(const cpr_ctx* c) { return c->opt.decoupling == CPR_DECOUPLE_ABF ? c->Jt : c->J; }
  static double* Rt(cpr_ctx* c) { return c->Rt; }
  static double* Z1(cpr_ctx* c) { return c->Z1; }
  static const double* Dinv(const cpr_ctx* c) { return c->Dinv; }
  static const double* A(const MGLevel& l) { return l.A; }
  static double* x(MGLevel& l) { return l.x; }
  static double* r(MGLevel& l) { return l.r; }
  static double* res(MGLevel& l) { return l.res; }
  static double* Y(cpr_ctx* c) { return c->Y; }
};
template <>
struct Pre<float> {
  static const float* R0(const cpr_ctx* c) { return c->Jf; }   // unused: full FP32 blocks
  static const float* J(const cpr_ctx* c) { return c->Jf; }
  static float* Rt(cpr_ctx* c) { return c->Rtf; }
  static float* Z1(cpr_ctx* c) { return c->Z1f; }
  static const float* Dinv(const cpr_ctx* c) { return c->Dinvf; }
  static const float* A(const MGLevel& l) { return l.Af; }
  static float* x(MGLevel& l) { return l.xf; }
  static float* r(MGLevel& l) { return l.rf; }
  static float* res(MGLevel& l) { return l.resf; }
  static float* Y(cpr_ctx* c) { return c->Yf; }
};

// Decoupled block entry (d, r, c) of cell t (tiled arrays).  FP64: row 0
// lives in R0 (7 b planes), rows >= 1 in J (7 b^2 planes); FP32: the copy
// holds the full decoupled blocks (7 b^2 planes).
template <int B, typename T>
__device__ inline T at_blk(const T* __restrict__ J, const T* __restrict__ R0, size_t N, int d, int r,
                           int c, int t) {
  if constexpr (sizeof(T) == 8) {
    return r == 0 ? ldnt(R0 + tix(7 * B, d * B + c, t)) : ldnt(J + tix(7 * B * B, (d * B + r) * B + c, t));
  } else {
    return ldnt(J + tix(7 * B * B, (d * B + r) * B + c, t));
  }
}

// ------------------------------------------------------------ per-cell steps

// red cell q: x = r / a_0 (zero initial guess: every neighbour is black = 0)
template <typename T>
__device__ inline void red_zero_cell(const T* __restrict__ A, const T* __restrict__ r, T* __restrict__ x,
                                     int q) {
  x[q] = r[q] / A[q];
}

// Stencil coefficients are read non-temporally by the multi-block sweeps,
// which stream them once, and through the caches by the single-workgroup
// kernel, which reads its small levels several times.
template <bool NT, typename T>
__device__ inline T ldc(const T* p) {
  if constexpr (NT) return ldnt(p); else return *p;
}

// sum_{d>0} a_d x_nb for a colour-split cell (branch-free, missing
// neighbours masked)
template <typename T, bool NT = true>
__device__ inline T offdiag_sum(const Lay& L, const T* __restrict__ A, const T* __restrict__ x, int t) {
  CsCell cc = cs_decode(L, t);
  int nbr[7];
  bool ok[7];
  cs_nbrs(L, t, cc, nbr, ok);
  T a[7];
#pragma unroll
  for (int d = 1; d < 7; ++d) a[d] = ldc<NT>(A + (size_t)d * L.n + t);
  T s = 0;
#pragma unroll
  for (int d = 1; d < 7; ++d) {
    T v = x[nbr[d]];
    s += a[d] * (ok[d] ? v : (T)0);
  }
  return s;
}

// black cell q: Gauss-Seidel update and its residual r - A x afterwards
template <typename T, bool NT = true>
__device__ inline void black_pre_cell(const Lay& L, const T* __restrict__ A, const T* __restrict__ r,
                                      T* __restrict__ x, T* __restrict__ res, int q) {
  int t = L.nh + q;
  T s = offdiag_sum<T, NT>(L, A, x, t);
  T xb = (r[t] - s) / A[t];
  x[t] = xb;
  res[q] = r[t] - (A[t] * xb + s);
}

// coarse cell tc: sum of the fine residuals of its aggregate (P^T r), fine
// cells in natural order; black residuals were recorded by the black sweep
template <typename T, bool NT = true>
__device__ inline void restrict_cell(const Lay& F, const Lay& C, const T* __restrict__ A,
                                     const T* __restrict__ r, const T* __restrict__ x,
                                     const T* __restrict__ res, T* __restrict__ rc, int tc) {
  int ci, cj, ck;
  lay_coords(C, tc, ci, cj, ck);
  T acc = 0;
  for (int fk = 2 * ck; fk <= 2 * ck + 1 && fk < F.nz; ++fk)
    for (int fj = 2 * cj; fj <= 2 * cj + 1 && fj < F.ny; ++fj)
      for (int fi = 2 * ci; fi <= 2 * ci + 1 && fi < F.nx; ++fi) {
        int f = lay_index(F, fi, fj, fk);
        if (f < F.nh) {
          T y = A[f] * x[f] + offdiag_sum<T, NT>(F, A, x, f);
          acc += r[f] - y;
        } else {
          acc += res[f - F.nh];
        }
      }
  rc[tc] = acc;
}

// black cell q after the coarse correction: neighbours are red cells whose
// corrected value is x + alpha e_c[aggregate]
template <typename T, bool NT = true>
__device__ inline void black_post_cell(const Lay& F, const Lay& C, T alpha, const T* __restrict__ A,
                                       const T* __restrict__ r, const T* __restrict__ ec,
                                       T* __restrict__ x, int q) {
  int t = F.nh + q;
  CsCell cc = cs_decode(F, t);
  int nbr[7];
  bool ok[7];
  cs_nbrs(F, t, cc, nbr, ok);
  T a[7];
#pragma unroll
  for (int d = 1; d < 7; ++d) a[d] = ldc<NT>(A + (size_t)d * F.n + t);
  T s = 0;
#pragma unroll
  for (int d = 1; d < 7; ++d) {
    int di, dj, dk;
    dir_offset(d, di, dj, dk);
    // a missing neighbour looks up the cell's own aggregate (in bounds) and is masked
    int gi = ok[d] ? cc.i + di : cc.i, gj = ok[d] ? cc.j + dj : cc.j, gk = ok[d] ? cc.k + dk : cc.k;
    T e = ec[lay_index(C, gi >> 1, gj >> 1, gk >> 1)];
    T v = x[nbr[d]] + alpha * e;
    s += a[d] * (ok[d] ? v : (T)0);
  }
  x[t] = (r[t] - s) / A[t];
}

// red cell q, general Gauss-Seidel update
template <typename T, bool NT = true>
__device__ inline void red_cell(const Lay& L, const T* __restrict__ A, const T* __restrict__ r,
                                T* __restrict__ x, int q) {
  T s = offdiag_sum<T, NT>(L, A, x, q);
  x[q] = (r[q] - s) / A[q];
}

// ------------------------------------------------------------ multi-block kernels

// Fine level entry: r~_0 = w^T v for every cell, and the zero-guess red
// sweep x_r = r~_0 / a_0.  If nrm2 is given, the input is an unnormalised
// Krylov vector: it is divided by sqrt(*nrm2) and written back first.
template <int B, typename T>
__global__ __launch_bounds__(256) void decouple_red_kernel(int n, int nh, const double* __restrict__ w,
                                                           const double* vin, double* vout,
                                                           const double* __restrict__ nrm2,
                                                           const T* __restrict__ A, T* __restrict__ rp,
                                                           T* __restrict__ x) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double hn = nrm2 ? sqrt(*nrm2) : 1.0;
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < B; ++r) {
    double v = vin[(size_t)r * n + t];
    if (nrm2) {
      v = v / hn;
      vout[(size_t)r * n + t] = v;
    }
    s += w[(size_t)r * n + t] * v;
  }
  T rs = (T)s;
  rp[t] = rs;
  if (t < nh) x[t] = rs / A[t];
}

// Decoupling for ABF or for the F-P-F composition: r~ = W v per cell (ABF:
// the b x b block D_i^-1; quasi-IMPES: row 0 becomes w^T v).  Two-stage
// (P then F): r~_0 and the zero-guess red sweep as above, rows >= 1 into Rt.
// F-P-F: all of r~ into Rt, and on red cells the forward ILU step
// Z1 = D'^-1 r~ (red cells have no lower neighbours).
template <int B, typename T, bool ABF, bool FPF>
__global__ __launch_bounds__(256) void decouple_full_kernel(int n, int nh, const double* __restrict__ w,
                                                            const double* vin, double* vout,
                                                            const double* __restrict__ nrm2,
                                                            const T* __restrict__ A, const T* __restrict__ Dinv,
                                                            T* __restrict__ rp, T* __restrict__ x,
                                                            T* __restrict__ Rt, T* __restrict__ Z1) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const size_t N = n;
  double hn = nrm2 ? sqrt(*nrm2) : 1.0;
  double v[B], rt[B];
#pragma unroll
  for (int r = 0; r < B; ++r) {
    v[r] = vin[(size_t)r * N + t];
    if (nrm2) {
      v[r] = v[r] / hn;
      vout[(size_t)r * N + t] = v[r];
    }
  }
  if constexpr (ABF) {
#pragma unroll
    for (int r = 0; r < B; ++r) {
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < B; ++c) s += w[((size_t)r * B + c) * N + t] * v[c];
      rt[r] = s;
    }
  } else {
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < B; ++r) s += w[(size_t)r * N + t] * v[r];
    rt[0] = s;
#pragma unroll
    for (int r = 1; r < B; ++r) rt[r] = v[r];
  }
  if constexpr (FPF) {
    T rr[B];
#pragma unroll
    for (int r = 0; r < B; ++r) {
      rr[r] = (T)rt[r];
      Rt[(size_t)r * N + t] = rr[r];
    }
    if (t < nh) {
#pragma unroll
      for (int r = 0; r < B; ++r) {
        T a = 0;
#pragma unroll
        for (int c = 0; c < B; ++c) a += Dinv[tix(B * B, r * B + c, t)] * rr[c];
        Z1[(size_t)r * N + t] = a;
      }
    }
  } else {
    T r0 = (T)rt[0];
    rp[t] = r0;
    if (t < nh) x[t] = r0 / A[t];
#pragma unroll
    for (int r = 1; r < B; ++r) Rt[(size_t)r * N + t] = (T)rt[r];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void black_pre_kernel(Lay L, const T* __restrict__ A, const T* __restrict__ r,
                                                        T* __restrict__ x, T* __restrict__ res) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < L.nh) black_pre_cell(L, A, r, x, res, q);
}

// Restriction with four threads per coarse cell: thread (cell, q, s) sums
// the two fine cells (2ci, 2ci+1) of fine row (2cj+q, 2ck+s); the four
// partials of a coarse cell sit in adjacent lanes and are combined in a
// fixed order.  Coarse cells are taken in natural order (ci fastest), so
// the lanes reading one fine row read consecutive cells of each colour half
// (in colour-split order consecutive coarse cells are two apart in x, and
// the fine reads would use every other value of each line).  Every lane
// takes its row's red cell (residual r - A x formed here) and its black
// cell (residual recorded by the black sweep) in the same order, so the
// lanes do not diverge on the colour; the two terms are added as a sum of
// two, whose value does not depend on their order.
// If xc is given, the coarse level's zero-guess red sweep is done here too:
// a red coarse cell stores x = r / a_0 as soon as its r is known.
template <typename T>
__global__ __launch_bounds__(256) void restrict4_kernel(Lay F, Lay C, const T* __restrict__ A,
                                                        const T* __restrict__ r, const T* __restrict__ x,
                                                        const T* __restrict__ res, T* __restrict__ rc,
                                                        const T* __restrict__ Ac, T* __restrict__ xc) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  int cn = g >> 2, sub = g & 3;
  T acc = 0;
  int tc = -1;
  if (cn < C.n) {
    const int ci = cn % C.nx, cjk = cn / C.nx;
    const int cj = cjk % C.ny, ck = cjk / C.ny;
    tc = lay_index(C, ci, cj, ck);
    int fj = 2 * cj + (sub & 1), fk = 2 * ck + (sub >> 1);
    if (fj < F.ny && fk < F.nz) {
      const int odd = (fj + fk) & 1;
      const int fr = 2 * ci + odd, fb = 2 * ci + 1 - odd;   // red and black cell of the pair
      T vr = 0, vb = 0;
      if (fr < F.nx) {
        const int f = lay_index(F, fr, fj, fk);
        T y = A[f] * x[f] + offdiag_sum(F, A, x, f);
        vr = r[f] - y;
      }
      if (fb < F.nx) vb = res[lay_index(F, fb, fj, fk) - F.nh];
      acc = vr + vb;
    }
  }
  acc += __shfl_down(acc, 2, 4);
  acc += __shfl_down(acc, 1, 4);
  if (tc >= 0 && sub == 0) {
    rc[tc] = acc;
    if (xc && tc < C.nh) red_zero_cell(Ac, rc, xc, tc);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void black_post_kernel(Lay F, Lay C, T alpha, const T* __restrict__ A,
                                                         const T* __restrict__ r, const T* __restrict__ ec,
                                                         T* __restrict__ x) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < F.nh) black_post_cell(F, C, alpha, A, r, ec, x, q);
}

template <typename T>
__global__ __launch_bounds__(256) void red_kernel(Lay L, const T* __restrict__ A, const T* __restrict__ r,
                                                  T* __restrict__ x) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < L.nh) red_cell(L, A, r, x, q);
}

// Coarsest level alone when it is too large for the fused kernel:
// x = A^-1 r with the dense FP64 inverse (column major).
template <typename T>
__global__ void coarse_gemv_kernel(int nc, const double* __restrict__ inv, const T* __restrict__ r,
                                   T* __restrict__ x) {
  int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= nc) return;
  double s = 0.0;
  for (int c = 0; c < nc; ++c) s += inv[(size_t)c * nc + row] * (double)r[c];
  x[row] = (T)s;
}

// ------------------------------------------------------------ fused small levels

template <typename T>
struct CoarseArgs {
  int count;                 // levels handled; the last one is solved densely
  Lay lay[MAXLV];
  const T* A[MAXLV];
  T* x[MAXLV];
  T* r[MAXLV];
  T* res[MAXLV];
  // element offsets of each level's arrays in the LDS copy (staged form)
  int sA[MAXLV], sx[MAXLV], sr[MAXLV], sres[MAXLV];
  const double* inv;
  T alpha;
  int pre, post;             // Gauss-Seidel sweeps before / after the coarse correction
};

// Bytes of LDS the staged form may take for its copy of the levels (the
// kernel adds 8 KB of its own): on gfx950 a workgroup may use up to 160 KB.
constexpr int COARSE_LDS_MAX = 96 * 1024;

// Staged form (LDS = true): the levels' stencils and the first level's
// right-hand side are copied into LDS once, every sweep, restriction and
// prolongation then reads and writes LDS, and the levels' x (and the
// restricted r) are copied back at the end; the coarsest inverse is read
// from global memory.  Every sweep depends on the one before, so with the
// arrays in global memory each costs an L2 round trip.  The arithmetic and
// its order are the same in both forms.
template <typename T, bool LDS>
__global__ __launch_bounds__(1024) void coarse_cycle_kernel(CoarseArgs<T> a) {
  extern __shared__ __align__(16) unsigned char stage_raw[];
  __shared__ double part[1024];
  T* sb = reinterpret_cast<T*>(stage_raw);
  const int tid = threadIdx.x, nt = blockDim.x;
  auto Ap = [&](int l) -> const T* { return LDS ? sb + a.sA[l] : a.A[l]; };
  auto xp = [&](int l) -> T* { return LDS ? sb + a.sx[l] : a.x[l]; };
  auto rp = [&](int l) -> T* { return LDS ? sb + a.sr[l] : a.r[l]; };
  auto resp = [&](int l) -> T* { return LDS ? sb + a.sres[l] : a.res[l]; };
  // The dense coarsest solve x = A^-1 r: thread (row, p) sums columns p,
  // p + parts, ... of its row.  When every thread has at most DENSE_PF of
  // them, they are loaded here, so that the loads overlap the sweeps of the
  // finer levels instead of forming a chain of dependent loads at the end.
  const int nc = a.lay[a.count - 1].n;
  const int parts = nt / nc;            // nc <= DENSE_FUSED_MAX <= nt
  const int drow = tid % nc, dp = tid / nc;
  const bool dactive = tid < nc * parts;
  const bool prefetch = nc * nc <= nt * DENSE_PF;
  double pre[DENSE_PF];
#pragma unroll
  for (int u = 0; u < DENSE_PF; ++u) {
    const int c = dp + u * parts;
    pre[u] = prefetch && dactive && c < nc ? a.inv[(size_t)c * nc + drow] : 0.0;
  }
  if constexpr (LDS) {
    // STAGE_UNROLL independent loads per thread in flight at a time
    auto stage = [&](const T* g, T* d, int len) {
      for (int base = 0; base < len; base += STAGE_UNROLL * nt) {
        T v[STAGE_UNROLL];
#pragma unroll
        for (int u = 0; u < STAGE_UNROLL; ++u) {
          const int i = base + u * nt + tid;
          v[u] = i < len ? g[i] : (T)0;
        }
#pragma unroll
        for (int u = 0; u < STAGE_UNROLL; ++u) {
          const int i = base + u * nt + tid;
          if (i < len) d[i] = v[u];
        }
      }
    };
    for (int l = 0; l + 1 < a.count; ++l) stage(a.A[l], sb + a.sA[l], 7 * a.lay[l].n);
    stage(a.r[0], sb + a.sr[0], a.lay[0].n);
    __syncthreads();
  }
  for (int l = 0; l + 1 < a.count; ++l) {
    const Lay F = a.lay[l], C = a.lay[l + 1];
    const T* A = Ap(l);
    T *x = xp(l), *r = rp(l), *res = resp(l);
    for (int q = tid; q < F.nh; q += nt) red_zero_cell(A, r, x, q);
    __syncthreads();
    for (int q = tid; q < F.nh; q += nt) black_pre_cell<T, false>(F, A, r, x, res, q);
    __syncthreads();
    for (int k = 1; k < a.pre; ++k) {
      for (int q = tid; q < F.nh; q += nt) red_cell<T, false>(F, A, r, x, q);
      __syncthreads();
      for (int q = tid; q < F.nh; q += nt) black_pre_cell<T, false>(F, A, r, x, res, q);
      __syncthreads();
    }
    T* rc = rp(l + 1);
    for (int tc = tid; tc < C.n; tc += nt) restrict_cell<T, false>(F, C, A, r, x, res, rc, tc);
    __syncthreads();
  }
  {
    const int L = a.count - 1;
    const T* rr = rp(L);
    if (dactive) {
      double s = 0.0;
      if (prefetch) {
#pragma unroll
        for (int u = 0; u < DENSE_PF; ++u) {
          const int c = dp + u * parts;
          if (c < nc) s += pre[u] * (double)rr[c];
        }
      } else {
        for (int c = dp; c < nc; c += parts) s += a.inv[(size_t)c * nc + drow] * (double)rr[c];
      }
      part[tid] = s;
    }
    __syncthreads();
    T* xc = xp(L);
    for (int row = tid; row < nc; row += nt) {
      double s = 0.0;
      for (int p = 0; p < parts; ++p) s += part[p * nc + row];
      xc[row] = (T)s;
    }
    __syncthreads();
  }
  for (int l = a.count - 2; l >= 0; --l) {
    const Lay F = a.lay[l], C = a.lay[l + 1];
    const T* A = Ap(l);
    T *x = xp(l), *r = rp(l), *res = resp(l);
    const T* ec = xp(l + 1);
    for (int q = tid; q < F.nh; q += nt) black_post_cell<T, false>(F, C, a.alpha, A, r, ec, x, q);
    __syncthreads();
    for (int q = tid; q < F.nh; q += nt) red_cell<T, false>(F, A, r, x, q);
    __syncthreads();
    for (int k = 1; k < a.post; ++k) {
      for (int q = tid; q < F.nh; q += nt) black_pre_cell<T, false>(F, A, r, x, res, q);
      __syncthreads();
      for (int q = tid; q < F.nh; q += nt) red_cell<T, false>(F, A, r, x, q);
      __syncthreads();
    }
  }
  if constexpr (LDS) {
    for (int l = 0; l < a.count; ++l) {
      const int n = a.lay[l].n;
      for (int i = tid; i < n; i += nt) a.x[l][i] = sb[a.sx[l] + i];
      if (l > 0)
        for (int i = tid; i < n; i += nt) a.r[l][i] = sb[a.sr[l] + i];
    }
  }
}

// Lays out the levels' arrays in the LDS copy; returns its size in bytes.
template <typename T>
size_t coarse_stage_layout(CoarseArgs<T>& a) {
  size_t off = 0;
  for (int q = 0; q < a.count; ++q) {
    const size_t n = (size_t)a.lay[q].n;
    a.sA[q] = a.sres[q] = 0;
    if (q + 1 < a.count) {
      a.sA[q] = (int)off;
      off += 7 * n;
      a.sres[q] = (int)off;
      off += n / 2 + 1;
    }
    a.sr[q] = (int)off;
    off += n;
    a.sx[q] = (int)off;
    off += n;
    off = (off + 1) & ~(size_t)1;   // 16-byte aligned arrays
  }
  return off * sizeof(T);
}

template <typename T>
void launch_coarse_cycle(CoarseArgs<T>& a, hipStream_t s) {
  // the staged form needs more than the default 64 KB of dynamic LDS
  static const bool big_lds = [] {
    const bool ok = hipFuncSetAttribute((const void*)coarse_cycle_kernel<T, true>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, COARSE_LDS_MAX) == hipSuccess;
    if (!ok) (void)hipGetLastError();   // leave no error for the launch checks
    return ok;
  }();
  const size_t bytes = coarse_stage_layout(a);
  if (big_lds && bytes <= (size_t)COARSE_LDS_MAX)
    coarse_cycle_kernel<T, true><<<1, 1024, bytes, s>>>(a);
  else
    coarse_cycle_kernel<T, false><<<1, 1024, 0, s>>>(a);
}

// ------------------------------------------------------------ stage 2 + block ILU(0)

// Stage-2 residual r2 = r~ - A~(:, p) dp at cell t.
template <int B, typename T, typename VT>
__device__ inline void stage2_resid(const Lay& L, int t, const CsCell& cc, const T* J, const T* R0,
                                    const VT* __restrict__ v, const T* __restrict__ rp,
                                    const T* __restrict__ dp, T (&r2)[B]) {
  const size_t N = L.n;
  int nbr[7];
  bool ok[7];
  cs_nbrs(L, t, cc, nbr, ok);
  T a[7][B];
#pragma unroll
  for (int d = 0; d < 7; ++d)
#pragma unroll
    for (int r = 0; r < B; ++r) a[d][r] = at_blk<B, T>(J, R0, N, d, r, 0, t);
  r2[0] = rp[t];
#pragma unroll
  for (int r = 1; r < B; ++r) r2[r] = (T)v[r * N + t];
#pragma unroll
  for (int d = 0; d < 7; ++d) {
    T p = dp[nbr[d]];
    p = ok[d] ? p : (T)0;
#pragma unroll
    for (int r = 0; r < B; ++r) r2[r] -= a[d][r] * p;
  }
}

template <int B, typename T>
__device__ inline void offdiag_apply(const Lay& L, int t, const CsCell& cc, const T* J, const T* R0,
                                     const T* __restrict__ Y, T (&s)[B]) {
  const size_t N = L.n;
  int nbr[7];
  bool ok[7];
  cs_nbrs(L, t, cc, nbr, ok);
  T a[7][B][B];
#pragma unroll
  for (int d = 1; d < 7; ++d)
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
      for (int c = 0; c < B; ++c) a[d][r][c] = at_blk<B, T>(J, R0, N, d, r, c, t);
#pragma unroll
  for (int r = 0; r < B; ++r) s[r] = 0;
#pragma unroll
  for (int d = 1; d < 7; ++d) {
    T y[B];
#pragma unroll
    for (int c = 0; c < B; ++c) {
      T v = Y[c * N + nbr[d]];
      y[c] = ok[d] ? v : (T)0;
    }
#pragma unroll
    for (int r = 0; r < B; ++r) {
      T acc = 0;
#pragma unroll
      for (int c = 0; c < B; ++c) acc += a[d][r][c] * y[c];
      s[r] += acc;
    }
  }
}

template <int B, typename T>
__device__ inline void dinv_apply(const T* __restrict__ Dinv, size_t N, int t, const T (&in)[B], T (&out)[B]) {
#pragma unroll
  for (int r = 0; r < B; ++r) {
    T a = 0;
#pragma unroll
    for (int c = 0; c < B; ++c) a += Dinv[tix(B * B, r * B + c, t)] * in[c];
    out[r] = a;
  }
}

// Stage 2 reads rows >= 1 of the decoupled residual from v: the Krylov
// vector itself for quasi-IMPES P-then-F (VT = double), the decoupled
// residual Rt otherwise (VT = T).  With z1 given (F-P-F) the first stage's
// result is added to z.

// red cells: forward ILU step y_r = D'^-1 r2_r (no lower neighbours)
template <int B, typename T, typename VT>
__global__ __launch_bounds__(256) void stage2_red_fwd_kernel(Lay L, const T* __restrict__ J,
                                                             const T* __restrict__ R0,
                                                             const T* __restrict__ Dinv,
                                                             const VT* __restrict__ v,
                                                             const T* __restrict__ rp,
                                                             const T* __restrict__ dp, T* __restrict__ Y) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= L.nh) return;
  CsCell cc = cs_decode(L, t);
  T r2[B], y[B];
  stage2_resid<B, T, VT>(L, t, cc, J, R0, v, rp, dp, r2);
  dinv_apply<B, T>(Dinv, L.n, t, r2, y);
#pragma unroll
  for (int r = 0; r < B; ++r) Y[(size_t)r * L.n + t] = y[r];
}

// black cells: y_b = D'^-1 (r2_b - sum_red A~_bk y_k); no upper neighbours,
// so z_b = y_b (+ dp on the pressure unknown)
template <int B, typename T, typename VT>
__global__ __launch_bounds__(256) void stage2_black_kernel(Lay L, const T* __restrict__ J,
                                                           const T* __restrict__ R0,
                                                           const T* __restrict__ Dinv,
                                                           const VT* __restrict__ v,
                                                           const T* __restrict__ rp,
                                                           const T* __restrict__ dp, T* __restrict__ Y,
                                                           const T* __restrict__ z1,
                                                           double* __restrict__ z) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= L.nh) return;
  int t = L.nh + q;
  CsCell cc = cs_decode(L, t);
  const size_t N = L.n;
  // r2 = r~ - A~(:,p) dp and s = sum_red A~_bk y_k, each off-diagonal block
  // read once (branch-free, non-temporal; missing neighbours masked)
  int nbr[7];
  bool ok[7];
  cs_nbrs(L, t, cc, nbr, ok);
  T a[7][B][B];
#pragma unroll
  for (int d = 0; d < 7; ++d)
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
      for (int c = 0; c < B; ++c)
        a[d][r][c] = (d == 0 && c > 0) ? (T)0 : at_blk<B, T>(J, R0, N, d, r, c, t);
  T r2[B], s[B], y[B];
  r2[0] = rp[t];
#pragma unroll
  for (int r = 1; r < B; ++r) r2[r] = (T)v[r * N + t];
  {
    T p = dp[t];
#pragma unroll
    for (int r = 0; r < B; ++r) r2[r] -= a[0][r][0] * p;
  }
#pragma unroll
  for (int r = 0; r < B; ++r) s[r] = 0;
#pragma unroll
  for (int d = 1; d < 7; ++d) {
    T p = dp[nbr[d]];
    p = ok[d] ? p : (T)0;
    T yk[B];
#pragma unroll
    for (int c = 0; c < B; ++c) {
      T vv = Y[c * N + nbr[d]];
      yk[c] = ok[d] ? vv : (T)0;
    }
#pragma unroll
    for (int r = 0; r < B; ++r) {
      r2[r] -= a[d][r][0] * p;
      T acc = a[d][r][0] * yk[0];
#pragma unroll
      for (int c = 1; c < B; ++c) acc += a[d][r][c] * yk[c];
      s[r] += acc;
    }
  }
#pragma unroll
  for (int r = 0; r < B; ++r) r2[r] -= s[r];
  dinv_apply<B, T>(Dinv, L.n, t, r2, y);
#pragma unroll
  for (int r = 0; r < B; ++r) Y[r * N + t] = y[r];
  z[t] = (double)y[0] + (double)dp[t];
#pragma unroll
  for (int r = 1; r < B; ++r) z[r * N + t] = (double)y[r];
  if (z1) {
#pragma unroll
    for (int r = 0; r < B; ++r) z[r * N + t] += (double)z1[r * N + t];
  }
}

// red cells, backward step: z_r = y_r - D'^-1 sum_black A~_rk y_k
template <int B, typename T>
__global__ __launch_bounds__(256) void stage2_red_bwd_kernel(Lay L, const T* __restrict__ J,
                                                             const T* __restrict__ R0,
                                                             const T* __restrict__ Dinv,
                                                             const T* __restrict__ dp,
                                                             const T* __restrict__ Y,
                                                             const T* __restrict__ z1,
                                                             double* __restrict__ z) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= L.nh) return;
  CsCell cc = cs_decode(L, t);
  T s[B], u[B];
  offdiag_apply<B, T>(L, t, cc, J, R0, Y, s);
  dinv_apply<B, T>(Dinv, L.n, t, s, u);
  const size_t N = L.n;
  z[t] = (double)(Y[t] - u[0]) + (double)dp[t];
#pragma unroll
  for (int r = 1; r < B; ++r) z[r * N + t] = (double)(Y[r * N + t] - u[r]);
  if (z1) {
#pragma unroll
    for (int r = 0; r < B; ++r) z[r * N + t] += (double)z1[r * N + t];
  }
}

// ------------------------------------------------------------ stage 2, tiled ILU order
// The same stage with the block ILU(0) in the tiled red-black order (one
// thread per tile of 1 x 2 x 2 cells, see tile_of_thread): forward over the
// red tiles, forward and backward over the black tiles (whose neighbours in
// other tiles are all red, so their backward step only involves
// tile-mates), backward over the red tiles.  Inside a thread the tile's
// cells are taken in order q = 0..3 forward and 3..0 backward, and each
// sum over neighbours runs in direction order.

template <int B, typename T>
__device__ inline void blk_add(const T* J, const T* R0, size_t N, int d, int t, const T (&v)[B], T (&acc)[B]) {
#pragma unroll
  for (int r = 0; r < B; ++r) {
    T a = 0;
#pragma unroll
    for (int c = 0; c < B; ++c) a += at_blk<B, T>(J, R0, N, d, r, c, t) * v[c];
    acc[r] += a;
  }
}

// Forward step's right-hand side of cell t: the stage-2 residual r2 = r~ -
// A~(:, p) dp minus the sum over the earlier neighbours (early[d]) of
// A~_tk y_k (yn[d]), each block read once: the full block where the
// neighbour is earlier, its pressure column otherwise.  The residual terms
// run in direction order, and the neighbour sum is subtracted at the end.
template <int B, typename T, typename VT>
__device__ inline void stage2_fwd_rhs(const Lay& L, int t, const T* J, const T* R0, const VT* __restrict__ v,
                                      const T* __restrict__ rp, const T* __restrict__ dp, const bool (&early)[7],
                                      const T (&yn)[7][B], T (&out)[B]) {
  const size_t N = L.n;
  CsCell cc = cs_decode(L, t);
  int nbr[7];
  bool ok[7];
  cs_nbrs(L, t, cc, nbr, ok);
  T r2[B], s[B];
  r2[0] = rp[t];
#pragma unroll
  for (int r = 1; r < B; ++r) r2[r] = (T)v[r * N + t];
  {
    const T p0 = dp[t];
#pragma unroll
    for (int r = 0; r < B; ++r) r2[r] -= at_blk<B, T>(J, R0, N, 0, r, 0, t) * p0;
  }
#pragma unroll
  for (int r = 0; r < B; ++r) s[r] = 0;
#pragma unroll
  for (int d = 1; d < 7; ++d) {
    T p = dp[nbr[d]];
    p = ok[d] ? p : (T)0;
    if (early[d]) {
      T a[B][B];
#pragma unroll
      for (int r = 0; r < B; ++r)
#pragma unroll
        for (int c = 0; c < B; ++c) a[r][c] = at_blk<B, T>(J, R0, N, d, r, c, t);
#pragma unroll
      for (int r = 0; r < B; ++r) {
        r2[r] -= a[r][0] * p;
        T acc = a[r][0] * yn[d][0];
#pragma unroll
        for (int c = 1; c < B; ++c) acc += a[r][c] * yn[d][c];
        s[r] += acc;
      }
    } else {
#pragma unroll
      for (int r = 0; r < B; ++r) r2[r] -= at_blk<B, T>(J, R0, N, d, r, 0, t) * p;
    }
  }
#pragma unroll
  for (int r = 0; r < B; ++r) out[r] = r2[r] - s[r];
}

template <int B, typename T, typename VT>
__global__ __launch_bounds__(256) void stage2_tiles_red_fwd_kernel(Lay L, const T* __restrict__ J,
                                                                   const T* __restrict__ R0,
                                                                   const T* __restrict__ Dinv,
                                                                   const VT* __restrict__ v,
                                                                   const T* __restrict__ rp,
                                                                   const T* __restrict__ dp, T* __restrict__ Y) {
  int i, tj, tk;
  if (!tile_of_thread(L, 0, (long)blockIdx.x * blockDim.x + threadIdx.x, i, tj, tk)) return;
  const size_t N = L.n;
  T y[4][B];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int j = 2 * tj + (q & 1), k = 2 * tk + (q >> 1);
    if (j >= L.ny || k >= L.nz) continue;
    const int t = lay_index(L, i, j, k);
    // earlier neighbours of a red tile's cell: its tile-mates below q (-y, -z)
    bool early[7] = {false, false, false, (q & 1) != 0, false, (q & 2) != 0, false};
    T yn[7][B];
#pragma unroll
    for (int c = 0; c < B; ++c) {
      yn[3][c] = (q & 1) ? y[(q & 1) ? q - 1 : 0][c] : (T)0;
      yn[5][c] = (q & 2) ? y[(q & 2) ? q - 2 : 0][c] : (T)0;
    }
    T r2[B];
    stage2_fwd_rhs<B, T, VT>(L, t, J, R0, v, rp, dp, early, yn, r2);
    dinv_apply<B, T>(Dinv, N, t, r2, y[q]);
#pragma unroll
    for (int r = 0; r < B; ++r) Y[(size_t)r * N + t] = y[q][r];
  }
}

template <int B, typename T, typename VT>
__global__ __launch_bounds__(256) void stage2_tiles_black_kernel(Lay L, const T* __restrict__ J,
                                                                 const T* __restrict__ R0,
                                                                 const T* __restrict__ Dinv,
                                                                 const VT* __restrict__ v,
                                                                 const T* __restrict__ rp,
                                                                 const T* __restrict__ dp, T* __restrict__ Y,
                                                                 double* __restrict__ z) {
  int i, tj, tk;
  if (!tile_of_thread(L, 1, (long)blockIdx.x * blockDim.x + threadIdx.x, i, tj, tk)) return;
  const size_t N = L.n;
  T y[4][B];
  int tq[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int j = 2 * tj + (q & 1), k = 2 * tk + (q >> 1);
    tq[q] = (j < L.ny && k < L.nz) ? lay_index(L, i, j, k) : -1;
    if (tq[q] < 0) continue;
    const int t = tq[q];
    CsCell cc = cs_decode(L, t);
    int nbr[7];
    bool ok[7];
    cs_nbrs(L, t, cc, nbr, ok);
    // earlier neighbours: tile-mates below q, and every neighbour in another
    // tile (red); the latter's y come from the red forward kernel
    bool early[7];
    T yn[7][B];
    early[0] = false;
#pragma unroll
    for (int d = 1; d < 7; ++d) {
      const int mate = tile_mate(q, d);
      early[d] = ok[d] && mate < q;
#pragma unroll
      for (int c = 0; c < B; ++c)
        yn[d][c] = !early[d] ? (T)0 : mate >= 0 ? y[mate < 0 ? 0 : mate][c] : Y[(size_t)c * N + nbr[d]];
    }
    T r2[B];
    stage2_fwd_rhs<B, T, VT>(L, t, J, R0, v, rp, dp, early, yn, r2);
    dinv_apply<B, T>(Dinv, N, t, r2, y[q]);
  }
  // backward: only tile-mates above q are later
  T zt[4][B];
#pragma unroll
  for (int q = 3; q >= 0; --q) {
    if (tq[q] < 0) continue;
    const int t = tq[q];
    T u[B], w[B];
#pragma unroll
    for (int r = 0; r < B; ++r) u[r] = 0;
    if (!(q & 1) && tq[q + 1 > 3 ? 3 : q + 1] >= 0) blk_add<B, T>(J, R0, N, 4, t, zt[q + 1 > 3 ? 3 : q + 1], u);
    if (!(q & 2) && tq[q + 2 > 3 ? 3 : q + 2] >= 0) blk_add<B, T>(J, R0, N, 6, t, zt[q + 2 > 3 ? 3 : q + 2], u);
    dinv_apply<B, T>(Dinv, N, t, u, w);
#pragma unroll
    for (int r = 0; r < B; ++r) zt[q][r] = y[q][r] - w[r];
#pragma unroll
    for (int r = 0; r < B; ++r) Y[(size_t)r * N + t] = zt[q][r];
    z[t] = (double)zt[q][0] + (double)dp[t];
#pragma unroll
    for (int r = 1; r < B; ++r) z[(size_t)r * N + t] = (double)zt[q][r];
  }
}

template <int B, typename T>
__global__ __launch_bounds__(256) void stage2_tiles_red_bwd_kernel(Lay L, const T* __restrict__ J,
                                                                   const T* __restrict__ R0,
                                                                   const T* __restrict__ Dinv,
                                                                   const T* __restrict__ dp,
                                                                   const T* __restrict__ Y,
                                                                   double* __restrict__ z) {
  int i, tj, tk;
  if (!tile_of_thread(L, 0, (long)blockIdx.x * blockDim.x + threadIdx.x, i, tj, tk)) return;
  const size_t N = L.n;
  int tq[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int j = 2 * tj + (q & 1), k = 2 * tk + (q >> 1);
    tq[q] = (j < L.ny && k < L.nz) ? lay_index(L, i, j, k) : -1;
  }
  // later neighbours of a red tile's cell: tile-mates above q, and every
  // neighbour in another tile (black, whose z the black kernel left in Y)
  T zt[4][B];
#pragma unroll
  for (int q = 3; q >= 0; --q) {
    if (tq[q] < 0) continue;
    const int t = tq[q];
    CsCell cc = cs_decode(L, t);
    int nbr[7];
    bool ok[7];
    cs_nbrs(L, t, cc, nbr, ok);
    T u[B], w[B];
#pragma unroll
    for (int r = 0; r < B; ++r) u[r] = 0;
#pragma unroll
    for (int d = 1; d < 7; ++d) {
      if (!ok[d]) continue;
      const int mate = tile_mate(q, d);
      if (mate >= 0 && mate < q) continue;
      T zk[B];
#pragma unroll
      for (int c = 0; c < B; ++c) zk[c] = mate >= 0 ? zt[mate < 0 ? 0 : mate][c] : Y[(size_t)c * N + nbr[d]];
      blk_add<B, T>(J, R0, N, d, t, zk, u);
    }
    dinv_apply<B, T>(Dinv, N, t, u, w);
#pragma unroll
    for (int r = 0; r < B; ++r) zt[q][r] = Y[(size_t)r * N + t] - w[r];
    z[t] = (double)zt[q][0] + (double)dp[t];
#pragma unroll
    for (int r = 1; r < B; ++r) z[(size_t)r * N + t] = (double)zt[q][r];
  }
}

// ------------------------------------------------------------ F-P-F first stage
// z1 = ILU(0)^-1 r~ and the residual r1 = r~ - A~ z1 that the P-then-F
// stages then see.  ILU(0) on the 7-point graph differs from A~ only between
// black cells two steps apart (through a red cell), so r1 vanishes on red
// cells: the red backward kernel stores those zeros (and the matching zero
// initial red sweep of the V-cycle), the residual kernel runs on black cells.

// black cells: z1_b = y_b = D'^-1 (r~_b - sum_red A~_bk y_k)
template <int B, typename T>
__global__ __launch_bounds__(256) void fpf_black_kernel(Lay L, const T* __restrict__ J, const T* __restrict__ R0,
                                                        const T* __restrict__ Dinv, const T* __restrict__ Rt,
                                                        T* __restrict__ Z1) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= L.nh) return;
  int t = L.nh + q;
  CsCell cc = cs_decode(L, t);
  const size_t N = L.n;
  T s[B], r[B], y[B];
  offdiag_apply<B, T>(L, t, cc, J, R0, Z1, s);
#pragma unroll
  for (int e = 0; e < B; ++e) r[e] = Rt[e * N + t] - s[e];
  dinv_apply<B, T>(Dinv, L.n, t, r, y);
#pragma unroll
  for (int e = 0; e < B; ++e) Z1[e * N + t] = y[e];
}

// red cells: z1_r = y_r - D'^-1 sum_black A~_rk z1_k; r1_r = 0 (rows of Rt,
// the pressure right-hand side and the zero-guess red sweep of level 0)
template <int B, typename T>
__global__ __launch_bounds__(256) void fpf_red_bwd_kernel(Lay L, const T* __restrict__ J, const T* __restrict__ R0,
                                                          const T* __restrict__ Dinv, T* __restrict__ Z1,
                                                          T* __restrict__ Rt, T* __restrict__ rp,
                                                          T* __restrict__ x) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= L.nh) return;
  CsCell cc = cs_decode(L, t);
  const size_t N = L.n;
  T s[B], u[B];
  offdiag_apply<B, T>(L, t, cc, J, R0, Z1, s);
  dinv_apply<B, T>(Dinv, L.n, t, s, u);
#pragma unroll
  for (int e = 0; e < B; ++e) {
    Z1[e * N + t] = Z1[e * N + t] - u[e];
    Rt[e * N + t] = (T)0;
  }
  rp[t] = (T)0;
  x[t] = (T)0;
}

// black cells: r1_b = r~_b - A~_bb z1_b - sum_red A~_bk z1_k; row 0 is the
// pressure right-hand side, rows >= 1 overwrite Rt
template <int B, typename T>
__global__ __launch_bounds__(256) void fpf_resid_kernel(Lay L, const T* __restrict__ J, const T* __restrict__ R0,
                                                        const T* __restrict__ Z1, T* __restrict__ Rt,
                                                        T* __restrict__ rp) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= L.nh) return;
  int t = L.nh + q;
  CsCell cc = cs_decode(L, t);
  const size_t N = L.n;
  T s[B], r[B];
  offdiag_apply<B, T>(L, t, cc, J, R0, Z1, s);
#pragma unroll
  for (int e = 0; e < B; ++e) {
    T a = s[e];
#pragma unroll
    for (int c = 0; c < B; ++c) a += at_blk<B, T>(J, R0, N, 0, e, c, t) * Z1[c * N + t];
    r[e] = Rt[e * N + t] - a;
  }
  rp[t] = r[0];
#pragma unroll
  for (int e = 1; e < B; ++e) Rt[e * N + t] = r[e];
}

// ------------------------------------------------------------ host side

#define TIMED(cls, launch) \
  do {                     \
    prof_begin(ctx, cls);  \
    launch;                \
    prof_end(ctx, cls);    \
  } while (0)

// First level handled by the single-workgroup kernel (nl: none).
int fused_level(const cpr_ctx* ctx) {
  const int nl = (int)ctx->levels.size();
  const int nc = ctx->levels.back().lay.n;
  int fuse = nl;
  if (nc <= DENSE_FUSED_MAX && nl <= MAXLV) {
    fuse = nl - 1;
    for (int l = 1; l < nl; ++l)
      if (ctx->levels[l].lay.n <= FUSE_MAX) { fuse = l; break; }
    if (nl == 1) fuse = 0;
  }
  return fuse;
}

template <typename T>
void vcycle(cpr_ctx* ctx) {
  hipStream_t s = ctx->stream;
  const int nl = (int)ctx->levels.size();
  const int nc = ctx->levels.back().lay.n;
  const int fuse = fused_level(ctx);
  const T alpha = (T)ctx->opt.mg_alpha;
  const int down = fuse < nl ? fuse : nl - 1;   // levels smoothed by multi-block kernels
  for (int l = 0; l < down; ++l) {
    MGLevel& L = ctx->levels[l];
    MGLevel& C = ctx->levels[l + 1];
    int nh = div_up(L.lay.nh, SB);
    // level 0's zero-guess red sweep is fused into the decoupling kernel and
    // that of the coarser multi-block levels into the restriction above them
    TIMED(CPR_KCLASS_SMOOTH, (black_pre_kernel<T><<<nh, SB, 0, s>>>(L.lay, Pre<T>::A(L), Pre<T>::r(L),
                                                                     Pre<T>::x(L), Pre<T>::res(L))));
    for (int k = 1; k < ctx->opt.mg_pre; ++k) {
      TIMED(CPR_KCLASS_SMOOTH, (red_kernel<T><<<nh, SB, 0, s>>>(L.lay, Pre<T>::A(L), Pre<T>::r(L), Pre<T>::x(L))));
      TIMED(CPR_KCLASS_SMOOTH, (black_pre_kernel<T><<<nh, SB, 0, s>>>(L.lay, Pre<T>::A(L), Pre<T>::r(L),
                                                                       Pre<T>::x(L), Pre<T>::res(L))));
    }
    const bool next_multi = l + 1 < down;
    restrict4_kernel<T><<<div_up(4L * C.lay.n, SB), SB, 0, s>>>(
        L.lay, C.lay, Pre<T>::A(L), Pre<T>::r(L), Pre<T>::x(L), Pre<T>::res(L), Pre<T>::r(C),
        next_multi ? Pre<T>::A(C) : nullptr, next_multi ? Pre<T>::x(C) : nullptr);
  }
  if (fuse < nl) {
    CoarseArgs<T> a;
    a.count = nl - fuse;
    for (int q = 0; q < a.count; ++q) {
      MGLevel& L = ctx->levels[fuse + q];
      a.lay[q] = L.lay;
      a.A[q] = Pre<T>::A(L);
      a.x[q] = Pre<T>::x(L);
      a.r[q] = Pre<T>::r(L);
      a.res[q] = Pre<T>::res(L);
    }
    a.inv = ctx->cinv;
    a.alpha = alpha;
    a.pre = ctx->opt.mg_pre;
    a.post = ctx->opt.mg_post;
    launch_coarse_cycle<T>(a, s);
  } else {
    MGLevel& L = ctx->levels.back();
    coarse_gemv_kernel<T><<<div_up(nc, 128), 128, 0, s>>>(nc, ctx->cinv, Pre<T>::r(L), Pre<T>::x(L));
  }
  for (int l = down - 1; l >= 0; --l) {
    MGLevel& L = ctx->levels[l];
    MGLevel& C = ctx->levels[l + 1];
    int nh = div_up(L.lay.nh, SB);
    TIMED(CPR_KCLASS_SMOOTH, (black_post_kernel<T><<<nh, SB, 0, s>>>(L.lay, C.lay, alpha, Pre<T>::A(L),
                                                                      Pre<T>::r(L), Pre<T>::x(C), Pre<T>::x(L))));
    TIMED(CPR_KCLASS_SMOOTH, (red_kernel<T><<<nh, SB, 0, s>>>(L.lay, Pre<T>::A(L), Pre<T>::r(L), Pre<T>::x(L))));
    for (int k = 1; k < ctx->opt.mg_post; ++k) {
      TIMED(CPR_KCLASS_SMOOTH, (black_pre_kernel<T><<<nh, SB, 0, s>>>(L.lay, Pre<T>::A(L), Pre<T>::r(L),
                                                                       Pre<T>::x(L), Pre<T>::res(L))));
      TIMED(CPR_KCLASS_SMOOTH, (red_kernel<T><<<nh, SB, 0, s>>>(L.lay, Pre<T>::A(L), Pre<T>::r(L), Pre<T>::x(L))));
    }
    // the learned correction on this level, before the finer levels'
    // post-smoothing (cpr_setup checked that it is a multi-block level)
    if (learned_on(ctx) && ctx->opt.nn_level == l && l > 0) learned_stage_at(ctx, l);
  }
}

template <int B, typename T, typename VT>
void stage2(cpr_ctx* ctx, const VT* vr, const T* z1, double* z) {
  hipStream_t s = ctx->stream;
  const Lay& L = ctx->lay;
  MGLevel& L0 = ctx->levels[0];
  const T* rp = Pre<T>::r(L0);
  const T* dp = Pre<T>::x(L0);
  const T* J = Pre<T>::J(ctx);
  const T* R0 = Pre<T>::R0(ctx);
  const T* Dinv = Pre<T>::Dinv(ctx);
  T* Y = Pre<T>::Y(ctx);
  if (ctx->opt.ilu_order == CPR_ILU_TILES) {   // P-then-F only: z1 is null
    const int nt = div_up(tile_threads(L), SB);
    TIMED(CPR_KCLASS_ILU,
          (stage2_tiles_red_fwd_kernel<B, T, VT><<<nt, SB, 0, s>>>(L, J, R0, Dinv, vr, rp, dp, Y)));
    TIMED(CPR_KCLASS_ILU,
          (stage2_tiles_black_kernel<B, T, VT><<<nt, SB, 0, s>>>(L, J, R0, Dinv, vr, rp, dp, Y, z)));
    TIMED(CPR_KCLASS_ILU, (stage2_tiles_red_bwd_kernel<B, T><<<nt, SB, 0, s>>>(L, J, R0, Dinv, dp, Y, z)));
    return;
  }
  int nh = div_up(L.nh, SB);
  TIMED(CPR_KCLASS_ILU, (stage2_red_fwd_kernel<B, T, VT><<<nh, SB, 0, s>>>(L, J, R0, Dinv, vr, rp, dp, Y)));
  TIMED(CPR_KCLASS_ILU, (stage2_black_kernel<B, T, VT><<<nh, SB, 0, s>>>(L, J, R0, Dinv, vr, rp, dp, Y, z1, z)));
  TIMED(CPR_KCLASS_ILU, (stage2_red_bwd_kernel<B, T><<<nh, SB, 0, s>>>(L, J, R0, Dinv, dp, Y, z1, z)));
}

template <int B, typename T, bool ABF, bool FPF>
void apply_variant(cpr_ctx* ctx, const double* vin, double* v, const double* nrm2, double* z) {
  hipStream_t s = ctx->stream;
  const Lay& L = ctx->lay;
  MGLevel& L0 = ctx->levels[0];
  T* rp = Pre<T>::r(L0);
  T* x0 = Pre<T>::x(L0);
  T* Rt = Pre<T>::Rt(ctx);
  T* Z1 = Pre<T>::Z1(ctx);
  const T* J = Pre<T>::J(ctx);
  const T* R0 = Pre<T>::R0(ctx);
  const T* Dinv = Pre<T>::Dinv(ctx);
  const double* w = ABF ? ctx->Wabf : ctx->w;
  decouple_full_kernel<B, T, ABF, FPF><<<div_up(L.n, SB), SB, 0, s>>>(L.n, L.nh, w, vin, v, nrm2, Pre<T>::A(L0),
                                                                        Dinv, rp, x0, Rt, Z1);
  if (FPF) {
    int nh = div_up(L.nh, SB);
    TIMED(CPR_KCLASS_ILU, (fpf_black_kernel<B, T><<<nh, SB, 0, s>>>(L, J, R0, Dinv, Rt, Z1)));
    TIMED(CPR_KCLASS_ILU, (fpf_red_bwd_kernel<B, T><<<nh, SB, 0, s>>>(L, J, R0, Dinv, Z1, Rt, rp, x0)));
    TIMED(CPR_KCLASS_ILU, (fpf_resid_kernel<B, T><<<nh, SB, 0, s>>>(L, J, R0, Z1, Rt, rp)));
  }
  vcycle<T>(ctx);
  if (learned_on(ctx) && ctx->opt.nn_level == 0) learned_stage(ctx);
  stage2<B, T, T>(ctx, Rt, FPF ? Z1 : nullptr, z);
}

template <int B, typename T>
void apply_impl(cpr_ctx* ctx, const double* vin, double* v, const double* nrm2, double* z) {
  const bool abf = ctx->opt.decoupling == CPR_DECOUPLE_ABF;
  const bool fpf = ctx->opt.composition == CPR_COMPOSE_FPF;
  if (abf && fpf) return apply_variant<B, T, true, true>(ctx, vin, v, nrm2, z);
  if (abf) return apply_variant<B, T, true, false>(ctx, vin, v, nrm2, z);
  if (fpf) return apply_variant<B, T, false, true>(ctx, vin, v, nrm2, z);
  hipStream_t s = ctx->stream;
  const Lay& L = ctx->lay;
  MGLevel& L0 = ctx->levels[0];
  decouple_red_kernel<B, T><<<div_up(L.n, SB), SB, 0, s>>>(L.n, L.nh, ctx->w, vin, v, nrm2, Pre<T>::A(L0),
                                                            Pre<T>::r(L0), Pre<T>::x(L0));
  vcycle<T>(ctx);
  if (learned_on(ctx) && ctx->opt.nn_level == 0) learned_stage(ctx);
  // rows >= 1 of the quasi-IMPES decoupled residual are those of v
  stage2<B, T, double>(ctx, v, nullptr, z);
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
        size_t o = tix(7 * B * B, (d * B + r) * B + c, t);
        Jf[o] = (float)(r == 0 ? R0[tix(7 * B, d * B + c, t)] : J[o]);
      }
  for (int e = 0; e < B * B; ++e) Dinvf[tix(B * B, e, t)] = (float)Dinv[tix(B * B, e, t)];
}

__global__ void to_float_kernel(size_t n, const double* __restrict__ a, float* __restrict__ b) {
  size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) b[t] = (float)a[t];
}

}  // namespace

int vcycle_fused_level(const cpr_ctx* ctx) { return fused_level(ctx); }

void launch_mixed_copies(cpr_ctx* ctx) {
  hipStream_t s = ctx->stream;
  int n = ctx->lay.n;
  const double* J = Pre<double>::J(ctx);
  if (ctx->b == 1)
    mixed_copy_kernel<1><<<div_up(n, 256), 256, 0, s>>>(n, J, ctx->R0, ctx->Dinv, ctx->Jf, ctx->Dinvf);
  else if (ctx->b == 2)
    mixed_copy_kernel<2><<<div_up(n, 256), 256, 0, s>>>(n, J, ctx->R0, ctx->Dinv, ctx->Jf, ctx->Dinvf);
  else
    mixed_copy_kernel<3><<<div_up(n, 256), 256, 0, s>>>(n, J, ctx->R0, ctx->Dinv, ctx->Jf, ctx->Dinvf);
  for (auto& L : ctx->levels) {
    size_t m = (size_t)7 * L.lay.n;
    to_float_kernel<<<div_up((long)m, 256), 256, 0, s>>>(m, L.A, L.Af);
  }
}

// Pressure stage alone (FP64, the plain cycle even when a learned stage is
// set up): r~_p = w^T v into level 0's r, dp_mg into its x.
void precond_pressure_stage(cpr_ctx* ctx, const double* v) {
  struct PlainCycle {
    cpr_ctx* c;
    int learned;
    ~PlainCycle() { c->opt.learned = learned; }
  } plain{ctx, ctx->opt.learned};
  ctx->opt.learned = 0;
  const Lay& L = ctx->lay;
  MGLevel& L0 = ctx->levels[0];
  if (ctx->b == 1)
    decouple_red_kernel<1, double><<<div_up(L.n, SB), SB, 0, ctx->stream>>>(L.n, L.nh, ctx->w, v, nullptr, nullptr,
                                                                               L0.A, L0.r, L0.x);
  else if (ctx->b == 2)
    decouple_red_kernel<2, double><<<div_up(L.n, SB), SB, 0, ctx->stream>>>(L.n, L.nh, ctx->w, v, nullptr, nullptr,
                                                                               L0.A, L0.r, L0.x);
  else
    decouple_red_kernel<3, double><<<div_up(L.n, SB), SB, 0, ctx->stream>>>(L.n, L.nh, ctx->w, v, nullptr, nullptr,
                                                                               L0.A, L0.r, L0.x);
  vcycle<double>(ctx);
}

void precond_apply(cpr_ctx* ctx, const double* vin, double* v, const double* nrm2, double* z) {
  const bool mixed = precond_fp32(ctx);
  if (ctx->b == 1) {
    if (mixed) apply_impl<1, float>(ctx, vin, v, nrm2, z); else apply_impl<1, double>(ctx, vin, v, nrm2, z);
  } else if (ctx->b == 2) {
    if (mixed) apply_impl<2, float>(ctx, vin, v, nrm2, z); else apply_impl<2, double>(ctx, vin, v, nrm2, z);
  } else {
    if (mixed) apply_impl<3, float>(ctx, vin, v, nrm2, z); else apply_impl<3, double>(ctx, vin, v, nrm2, z);
  }
  border_precond(ctx, vin, v, nrm2, z);   // rate wells' BHP rows, after the cell correction
}
