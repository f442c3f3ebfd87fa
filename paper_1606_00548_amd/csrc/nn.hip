// Pressure-correction network: training and inference kernels.
//
// The network (no counterpart in the paper; it supplies a correction to
// the pressure stage of the CPR preconditioner) is a 3-D U-Net on
// channels-last FP32 tensors T[b][voxel][c] (voxel = x + nx*(y + ny*z)):
//   e0 = relu(c0(x))            e1 = relu(c1(pool e0))
//   e2 = relu(c2(pool e1))      e3 = relu(c3(pool e2))
//   d2 = relu(c4(up e3)) + e2   d1 = relu(c5(up d2)) + e1
//   d0 = relu(c6(up d1)) + e0   y  = wo . d0 + bo
// with 3x3x3 zero-padded correlations, 2x2x2 average pooling, nearest
// upsampling (read on the fly by the convolution that consumes it), and a
// normalised mean-squared-error loss.  Parameters: FP32 master copy, Adam
// moments, BF16 copies laid out as MFMA B-fragments.
//
// Convolutions are implicit GEMMs on the CDNA matrix cores
// (v_mfma_f32_16x16x16_bf16, FP32 accumulation): one wavefront computes 16
// output voxels x all output channels, looping over 27 taps x input
// channels in K-steps of 16; activations are converted to BF16 as they are
// loaded.  The data gradient is the same kernel with mirrored taps and
// transposed channel blocks; the weight gradient is a GEMM over voxels
// (M = input channels, N = output channels) whose per-chunk partial sums
// are reduced in a fixed order, so training is deterministic.
#include <cmath>
#include <cstring>

#include "internal.h"

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int NCONV = 7;
constexpr int CIN[NCONV] = {3, 16, 32, 64, 64, 64, 32};
constexpr int COUT[NCONV] = {16, 32, 64, 64, 64, 32, 16};
constexpr int CIN_PAD[NCONV] = {16, 16, 32, 64, 64, 64, 32};
constexpr int WG_CHUNK = 2048;   // voxels per weight-gradient block

__device__ inline short f2bf(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even
  return (short)(u >> 16);
}

struct Geo {
  int nx, ny, nz, V;   // grid of the tensor being produced
  int batch;
};

// ------------------------------------------------------------ convolution
// out[b][v][co] = sum_t sum_ci X~[b][v + off_t][ci] W[t][ci][co]; X~ is X on
// the same grid, or X on the half-resolution grid read at (x/2, y/2, z/2)
// when UP.  EPI 1: a = relu(acc + bias) stored in outA, and a + skip in outD
// when skip is given; EPI 0: raw acc stored in outA (data gradient).
template <int CI, int CO, bool UP, int EPI>
__global__ __launch_bounds__(256) void conv_kernel(Geo g, const float* __restrict__ X,
                                                   const bf16x4* __restrict__ Wf,
                                                   const float* __restrict__ bias,
                                                   const float* __restrict__ skip,
                                                   float* __restrict__ outA, float* __restrict__ outD) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long total = (long)g.batch * g.V;
  const long vbase = ((long)blockIdx.x * 4 + wave) * 16;
  if (vbase >= total) return;
  const long gv = vbase + (lane & 15);
  const bool valid = gv < total;
  const int b = valid ? (int)(gv / g.V) : 0;
  const int v = valid ? (int)(gv - (long)b * g.V) : 0;
  const int x = v % g.nx, yz = v / g.nx, y = yz % g.ny, z = yz / g.ny;
  const int kq = lane >> 4;
  const int cnx = g.nx >> 1, cny = g.ny >> 1, cV = (g.nx >> 1) * (g.ny >> 1) * (g.nz >> 1);
  f32x4 acc[CO / 16];
#pragma unroll
  for (int n = 0; n < CO / 16; ++n) acc[n] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int t = 0; t < 27; ++t) {
    const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
    const int xx = x + dx, yy = y + dy, zz = z + dz;
    const bool inb = valid && xx >= 0 && xx < g.nx && yy >= 0 && yy < g.ny && zz >= 0 && zz < g.nz;
    long src;
    if (UP)
      src = (long)b * cV + (xx >> 1) + (long)cnx * ((yy >> 1) + (long)cny * (zz >> 1));
    else
      src = (long)b * g.V + xx + (long)g.nx * (yy + (long)g.ny * zz);
    const float* row = X + src * CI;
#pragma unroll
    for (int kc = 0; kc < CI / 16; ++kc) {
      f32x4 av = inb ? *(const f32x4*)(row + kc * 16 + kq * 4) : f32x4{0.f, 0.f, 0.f, 0.f};
      bf16x4 a;
      a[0] = f2bf(av[0]); a[1] = f2bf(av[1]); a[2] = f2bf(av[2]); a[3] = f2bf(av[3]);
      const bf16x4* wrow = Wf + ((size_t)(t * (CI / 16) + kc) * (CO / 16)) * 64 + lane;
#pragma unroll
      for (int n = 0; n < CO / 16; ++n)
        acc[n] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, wrow[n * 64], acc[n], 0, 0, 0);
    }
  }
#pragma unroll
  for (int n = 0; n < CO / 16; ++n) {
    const int co = n * 16 + (lane & 15);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const long o = vbase + 4 * kq + e;
      if (o >= total) continue;
      float val = acc[n][e];
      if (EPI == 1) {
        float a = fmaxf(val + bias[co], 0.f);
        outA[o * CO + co] = a;
        if (skip) outD[o * CO + co] = a + skip[o * CO + co];
      } else {
        outA[o * CO + co] = val;
      }
    }
  }
}

// Weight gradient partials: part[chunk][t][ci][co] = sum over the chunk's
// voxels v of X~[v + off_t][ci] dZ[v][co]; one block per (chunk, tap).
template <int CI, int CO, bool UP>
__global__ __launch_bounds__(256) void wgrad_kernel(Geo g, const float* __restrict__ X,
                                                    const float* __restrict__ dZ, float* __restrict__ part) {
  __shared__ float red[4][CI * CO];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int t = blockIdx.y;
  const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
  const long total = (long)g.batch * g.V;
  const long c0 = (long)blockIdx.x * WG_CHUNK;
  const int cnx = g.nx >> 1, cny = g.ny >> 1, cV = (g.nx >> 1) * (g.ny >> 1) * (g.nz >> 1);
  f32x4 acc[CI / 16][CO / 16];
#pragma unroll
  for (int m = 0; m < CI / 16; ++m)
#pragma unroll
    for (int n = 0; n < CO / 16; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int kq = lane >> 4, i16 = lane & 15;
  for (long vs = c0 + wave * 16; vs < c0 + WG_CHUNK && vs < total; vs += 64) {
    bf16x4 a[CI / 16], bb[CO / 16];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const long gv = vs + 4 * kq + e;
      const bool valid = gv < total;
      const int b = valid ? (int)(gv / g.V) : 0;
      const int v = valid ? (int)(gv - (long)b * g.V) : 0;
      const int x = v % g.nx, yz = v / g.nx, y = yz % g.ny, z = yz / g.ny;
      const int xx = x + dx, yy = y + dy, zz = z + dz;
      const bool inb = valid && xx >= 0 && xx < g.nx && yy >= 0 && yy < g.ny && zz >= 0 && zz < g.nz;
      long src;
      if (UP)
        src = (long)b * cV + (xx >> 1) + (long)cnx * ((yy >> 1) + (long)cny * (zz >> 1));
      else
        src = (long)b * g.V + xx + (long)g.nx * (yy + (long)g.ny * zz);
#pragma unroll
      for (int m = 0; m < CI / 16; ++m) a[m][e] = f2bf(inb ? X[src * CI + m * 16 + i16] : 0.f);
#pragma unroll
      for (int n = 0; n < CO / 16; ++n) bb[n][e] = f2bf(valid ? dZ[gv * CO + n * 16 + i16] : 0.f);
    }
#pragma unroll
    for (int m = 0; m < CI / 16; ++m)
#pragma unroll
      for (int n = 0; n < CO / 16; ++n)
        acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[m], bb[n], acc[m][n], 0, 0, 0);
  }
  // C tile element (ci = m*16 + 4*kq + e, co = n*16 + i16)
#pragma unroll
  for (int m = 0; m < CI / 16; ++m)
#pragma unroll
    for (int n = 0; n < CO / 16; ++n)
#pragma unroll
      for (int e = 0; e < 4; ++e) red[wave][(m * 16 + 4 * kq + e) * CO + n * 16 + i16] = acc[m][n][e];
  __syncthreads();
  float* out = part + ((size_t)blockIdx.x * 27 + t) * CI * CO;
  for (int q = threadIdx.x; q < CI * CO; q += 256) out[q] = ((red[0][q] + red[1][q]) + red[2][q]) + red[3][q];
}

// dW[t][ci][co] (only the real input channels) = sum over chunks, in order.
__global__ void wgrad_reduce_kernel(int nchunk, int ci_pad, int ci_real, int co, const float* __restrict__ part,
                                    float* __restrict__ dW) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  int per = 27 * ci_real * co;
  if (q >= per) return;
  int t = q / (ci_real * co), r = q % (ci_real * co);
  int ci = r / co, c = r % co;
  size_t src = ((size_t)t * ci_pad + ci) * co + c;
  float s = 0.f;
  for (int k = 0; k < nchunk; ++k) s += part[(size_t)k * 27 * ci_pad * co + src];
  dW[q] = s;
}

// Column sums sum_v T[v][c] for the bias gradient: per-block partials.
__global__ void colsum_partial_kernel(long nvox, int C, const float* __restrict__ T, float* __restrict__ part) {
  __shared__ float sh[256];
  const int c = threadIdx.x % C, grp = threadIdx.x / C, ngrp = 256 / C;
  const long per = (nvox + gridDim.x - 1) / gridDim.x;
  const long beg = (long)blockIdx.x * per, end = beg + per < nvox ? beg + per : nvox;
  float s = 0.f;
  if (grp < ngrp)
    for (long v = beg + grp; v < end; v += ngrp) s += T[v * C + c];
  sh[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < C) {
    float tot = 0.f;
    for (int q = 0; q < ngrp; ++q) tot += sh[q * C + threadIdx.x];
    part[(size_t)blockIdx.x * C + threadIdx.x] = tot;
  }
}

__global__ void colsum_final_kernel(int nblk, int C, const float* __restrict__ part, float* __restrict__ out) {
  int c = threadIdx.x;
  if (c >= C) return;
  float s = 0.f;
  for (int k = 0; k < nblk; ++k) s += part[(size_t)k * C + c];
  out[c] = s;
}

// ------------------------------------------------------------ elementwise
// 2x2x2 average pooling of X on grid g2 = 2 * (output grid g).
__global__ void pool_kernel(Geo g, int C, const float* __restrict__ X, float* __restrict__ out) {
  long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)g.batch * g.V * C;
  if (q >= total) return;
  int c = (int)(q % C);
  long bv = q / C;
  int b = (int)(bv / g.V), v = (int)(bv % g.V);
  int x = v % g.nx, yz = v / g.nx, y = yz % g.ny, z = yz / g.ny;
  int fx = 2 * g.nx, fy = 2 * g.ny, fV = 8 * g.V;
  float s = 0.f;
  for (int k = 0; k < 2; ++k)
    for (int j = 0; j < 2; ++j)
      for (int i = 0; i < 2; ++i)
        s += X[((long)b * fV + (2 * x + i) + (long)fx * ((2 * y + j) + (long)fy * (2 * z + k))) * C + c];
  out[q] = s * 0.125f;
}

// Fine-grid gradient += (coarse gradient of the pooled tensor) / 8.
__global__ void pool_bwd_kernel(Geo fine, int C, const float* __restrict__ dP, float* __restrict__ dX) {
  long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)fine.batch * fine.V * C;
  if (q >= total) return;
  int c = (int)(q % C);
  long bv = q / C;
  int b = (int)(bv / fine.V), v = (int)(bv % fine.V);
  int x = v % fine.nx, yz = v / fine.nx, y = yz % fine.ny, z = yz / fine.ny;
  int cnx = fine.nx / 2, cny = fine.ny / 2, cV = fine.V / 8;
  dX[q] += dP[((long)b * cV + (x >> 1) + (long)cnx * ((y >> 1) + (long)cny * (z >> 1))) * C + c] * 0.125f;
}

// Coarse gradient of an upsampled tensor: sum of its 8 children (g coarse).
// accumulate: out += sum, else out = sum.
__global__ void up_bwd_kernel(Geo g, int C, const float* __restrict__ dU, float* __restrict__ out, int accumulate) {
  long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)g.batch * g.V * C;
  if (q >= total) return;
  int c = (int)(q % C);
  long bv = q / C;
  int b = (int)(bv / g.V), v = (int)(bv % g.V);
  int x = v % g.nx, yz = v / g.nx, y = yz % g.ny, z = yz / g.ny;
  int fx = 2 * g.nx, fy = 2 * g.ny, fV = 8 * g.V;
  float s = 0.f;
  for (int k = 0; k < 2; ++k)
    for (int j = 0; j < 2; ++j)
      for (int i = 0; i < 2; ++i)
        s += dU[((long)b * fV + (2 * x + i) + (long)fx * ((2 * y + j) + (long)fy * (2 * z + k))) * C + c];
  out[q] = accumulate ? out[q] + s : s;
}

// out = g * (a > 0)
__global__ void relu_mask_kernel(long n, const float* __restrict__ gr, const float* __restrict__ a,
                                 float* __restrict__ out) {
  long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) out[q] = a[q] > 0.f ? gr[q] : 0.f;
}

// Input features [b][v][3] -> padded [b][v][16].
__global__ void pad_input_kernel(long nvox, const float* __restrict__ x3, float* __restrict__ x16) {
  long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nvox * 16) return;
  long v = q / 16;
  int c = (int)(q % 16);
  x16[q] = c < 3 ? x3[v * 3 + c] : 0.f;
}

// Head: y[v] = sum_c d0[v][c] wo[c] + bo.
__global__ void head_fwd_kernel(long nvox, const float* __restrict__ d0, const float* __restrict__ wb,
                                float* __restrict__ y) {
  long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvox) return;
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < 16; ++c) s += d0[v * 16 + c] * wb[c];
  y[v] = s + wb[16];
}

// dd0[v][c] = dy[v] wo[c]; the head-weight products d0*dy for their sums.
__global__ void head_bwd_kernel(long nvox, const float* __restrict__ d0, const float* __restrict__ dy,
                                const float* __restrict__ wb, float* __restrict__ dd0, float* __restrict__ prod) {
  long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nvox * 17) return;
  long v = q / 17;
  int c = (int)(q % 17);
  if (c < 16) {
    dd0[v * 16 + c] = dy[v] * wb[c];
    prod[v * 17 + c] = d0[v * 16 + c] * dy[v];
  } else {
    prod[v * 17 + 16] = dy[v];
  }
}

// Loss partials per sample over a block's voxels: y.t, y.y, t.t.
__global__ void loss_partial_kernel(int V, int nblk_per, const float* __restrict__ y, const float* __restrict__ t,
                                    float* __restrict__ part) {
  __shared__ float s1[256], s2[256], s3[256];
  int b = blockIdx.x / nblk_per, k = blockIdx.x % nblk_per;
  long per = (V + nblk_per - 1) / nblk_per;
  long beg = (long)k * per, end = beg + per < V ? beg + per : V;
  float a = 0.f, c = 0.f, e = 0.f;
  for (long v = beg + threadIdx.x; v < end; v += 256) {
    float yv = y[(long)b * V + v], tv = t[(long)b * V + v];
    a += yv * tv;
    c += yv * yv;
    e += tv * tv;
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = c;
  s3[threadIdx.x] = e;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      s1[threadIdx.x] += s1[threadIdx.x + o];
      s2[threadIdx.x] += s2[threadIdx.x + o];
      s3[threadIdx.x] += s3[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = s1[0];
    part[3 * blockIdx.x + 1] = s2[0];
    part[3 * blockIdx.x + 2] = s3[0];
  }
}

// Per-sample totals (fixed order); the direction loss
// L = mean_b (1 - (y.t)^2 / (|y|^2 |t|^2)) and
// dy = -(2/B) [c t - c (y.t)/|y|^2 y], c = (y.t) / (|y|^2 |t|^2).
__global__ void loss_grad_kernel(int B, int V, int nblk_per, const float* __restrict__ part,
                                 const float* __restrict__ y, const float* __restrict__ t, float* __restrict__ dy,
                                 float* __restrict__ loss) {
  __shared__ float yt[64], yy[64], tt[64];
  if (threadIdx.x < B) {
    float a = 0.f, c = 0.f, e = 0.f;
    for (int k = 0; k < nblk_per; ++k) {
      a += part[3 * (threadIdx.x * nblk_per + k)];
      c += part[3 * (threadIdx.x * nblk_per + k) + 1];
      e += part[3 * (threadIdx.x * nblk_per + k) + 2];
    }
    yt[threadIdx.x] = a;
    yy[threadIdx.x] = c;
    tt[threadIdx.x] = e;
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    float L = 0.f;
    for (int b = 0; b < B; ++b) L += 1.f - yt[b] * yt[b] / (yy[b] * tt[b]);
    *loss = L / B;
  }
  for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < (long)B * V; q += (long)gridDim.x * blockDim.x) {
    int b = (int)(q / V);
    float c = yt[b] / (yy[b] * tt[b]);
    dy[q] = -(2.f / B) * (c * t[q] - (c * yt[b] / yy[b]) * y[q]);
  }
}

// Training target: t = e / s in FP32.
__global__ void target_kernel(long n, const double* __restrict__ e, double inv, float* __restrict__ t) {
  long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) t[q] = (float)(e[q] * inv);
}

// Adam with bias correction; c1 = 1/(1 - b1^k), c2 = 1/(1 - b2^k).
__global__ void adam_kernel(long n, float lr, float b1, float b2, float eps, float c1, float c2,
                            const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                            float* __restrict__ w) {
  long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  float gq = g[q];
  float mq = b1 * m[q] + (1.f - b1) * gq;
  float vq = b2 * v[q] + (1.f - b2) * gq * gq;
  m[q] = mq;
  v[q] = vq;
  w[q] -= lr * (mq * c1) / (sqrtf(vq * c2) + eps);
}

// BF16 B-fragments of conv weights W[27][ci_real][co] (FP32 master):
// forward:  frag[t][kc][nc][lane][e] = W[t][kc*16 + 4*(lane/16) + e][nc*16 + lane%16]
// backward: taps mirrored (26 - t) and channels transposed (K = co, N = ci).
__global__ void frag_kernel(int ci_real, int ci_pad, int co, const float* __restrict__ W, bf16x4* __restrict__ fw,
                            bf16x4* __restrict__ bw) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  int nf = 27 * (ci_pad / 16) * (co / 16) * 64;
  if (q < nf) {
    int lane = q % 64, r = q / 64;
    int nc = r % (co / 16); r /= (co / 16);
    int kc = r % (ci_pad / 16);
    int t = r / (ci_pad / 16);
    bf16x4 f;
    for (int e = 0; e < 4; ++e) {
      int ci = kc * 16 + 4 * (lane / 16) + e, c = nc * 16 + lane % 16;
      f[e] = f2bf(ci < ci_real ? W[((size_t)t * ci_real + ci) * co + c] : 0.f);
    }
    fw[q] = f;
  }
  if (bw && q < 27 * (co / 16) * (ci_pad / 16) * 64) {
    int lane = q % 64, r = q / 64;
    int nc = r % (ci_pad / 16); r /= (ci_pad / 16);
    int kc = r % (co / 16);
    int t = r / (co / 16);
    bf16x4 f;
    for (int e = 0; e < 4; ++e) {
      int c = kc * 16 + 4 * (lane / 16) + e, ci = nc * 16 + lane % 16;
      f[e] = f2bf(ci < ci_real ? W[((size_t)(26 - t) * ci_real + ci) * co + c] : 0.f);
    }
    bw[q] = f;
  }
}

}  // namespace

// ------------------------------------------------------------ host object

struct cpr_nn {
  std::string err;
  hipStream_t stream = nullptr;
  Geo lv[4];           // grid per level (batch = max_batch)
  int max_batch = 0;
  long P = 0;
  long off[NCONV + 1]; // parameter offsets: conv k weights at off[k], bias after
  float* theta = nullptr;
  float* m = nullptr;
  float* vv = nullptr;
  float* grad = nullptr;
  bf16x4* wf[NCONV] = {};
  bf16x4* wb[NCONV] = {};
  // activations
  float *x16 = nullptr, *e0 = nullptr, *p1 = nullptr, *e1 = nullptr, *p2 = nullptr, *e2 = nullptr;
  float *p3 = nullptr, *e3 = nullptr, *a4 = nullptr, *d2 = nullptr, *a5 = nullptr, *d1 = nullptr;
  float *a6 = nullptr, *d0 = nullptr, *y = nullptr;
  // gradients
  float *dy = nullptr, *g0 = nullptr, *g0b = nullptr, *gu0 = nullptr, *g1 = nullptr, *g1b = nullptr;
  float *gu1 = nullptr, *g2 = nullptr, *g2b = nullptr, *gu2 = nullptr, *g3 = nullptr, *g3b = nullptr;
  float *gp = nullptr, *prod = nullptr, *part = nullptr, *lpart = nullptr, *loss = nullptr;
  size_t part_cap = 0;
  int cur_batch = 0;
  long adam_step = 0;
  bool frags_valid = false;
};

static int nn_err(cpr_nn* nn, int code, const std::string& msg) {
  if (nn) nn->err = msg;
  return code;
}

#define NN_TRY(expr)                                                            \
  do {                                                                          \
    hipError_t e_ = (expr);                                                     \
    if (e_ != hipSuccess) return nn_err(nn, CPR_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

static long nn_param_count() {
  long p = 0;
  for (int k = 0; k < NCONV; ++k) p += 27L * CIN[k] * COUT[k] + COUT[k];
  return p + 17;
}

static Geo with_batch(Geo g, int b) { g.batch = b; return g; }

static int nn_refresh_frags(cpr_nn* nn) {
  for (int k = 0; k < NCONV; ++k) {
    int nf = 27 * (CIN_PAD[k] / 16) * (COUT[k] / 16) * 64;
    frag_kernel<<<div_up(nf, 256), 256, 0, nn->stream>>>(CIN[k], CIN_PAD[k], COUT[k], nn->theta + nn->off[k],
                                                         nn->wf[k], k == 0 ? nullptr : nn->wb[k]);
  }
  nn->frags_valid = true;
  NN_TRY(hipGetLastError());
  return CPR_OK;
}

template <int CI, int CO, bool UP, int EPI>
static void conv(cpr_nn* nn, Geo g, const float* X, const bf16x4* W, const float* bias, const float* skip,
                 float* outA, float* outD) {
  long total = (long)g.batch * g.V;
  conv_kernel<CI, CO, UP, EPI><<<div_up(total, 64), 256, 0, nn->stream>>>(g, X, W, bias, skip, outA, outD);
}

template <int CI, int CO, bool UP>
static void wgrad(cpr_nn* nn, Geo g, const float* X, const float* dZ, int k) {
  long total = (long)g.batch * g.V;
  int nchunk = div_up(total, WG_CHUNK);
  dim3 grid(nchunk, 27);
  wgrad_kernel<CI, CO, UP><<<grid, 256, 0, nn->stream>>>(g, X, dZ, nn->part);
  int per = 27 * CIN[k] * CO;
  wgrad_reduce_kernel<<<div_up(per, 256), 256, 0, nn->stream>>>(nchunk, CI, CIN[k], CO, nn->part,
                                                               nn->grad + nn->off[k]);
  // bias gradient
  int nb = (int)std::min<long>(256, div_up(total, 256));
  colsum_partial_kernel<<<nb, 256, 0, nn->stream>>>(total, CO, dZ, nn->gp);
  colsum_final_kernel<<<1, 64, 0, nn->stream>>>(nb, CO, nn->gp, nn->grad + nn->off[k] + 27L * CIN[k] * CO);
}

static int nn_forward_impl(cpr_nn* nn, int B) {
  Geo L0 = with_batch(nn->lv[0], B), L1 = with_batch(nn->lv[1], B), L2 = with_batch(nn->lv[2], B),
      L3 = with_batch(nn->lv[3], B);
  hipStream_t s = nn->stream;
  auto bias = [&](int k) { return nn->theta + nn->off[k] + 27L * CIN[k] * COUT[k]; };
  conv<16, 16, false, 1>(nn, L0, nn->x16, nn->wf[0], bias(0), nullptr, nn->e0, nullptr);
  pool_kernel<<<div_up((long)B * L1.V * 16, 256), 256, 0, s>>>(L1, 16, nn->e0, nn->p1);
  conv<16, 32, false, 1>(nn, L1, nn->p1, nn->wf[1], bias(1), nullptr, nn->e1, nullptr);
  pool_kernel<<<div_up((long)B * L2.V * 32, 256), 256, 0, s>>>(L2, 32, nn->e1, nn->p2);
  conv<32, 64, false, 1>(nn, L2, nn->p2, nn->wf[2], bias(2), nullptr, nn->e2, nullptr);
  pool_kernel<<<div_up((long)B * L3.V * 64, 256), 256, 0, s>>>(L3, 64, nn->e2, nn->p3);
  conv<64, 64, false, 1>(nn, L3, nn->p3, nn->wf[3], bias(3), nullptr, nn->e3, nullptr);
  conv<64, 64, true, 1>(nn, L2, nn->e3, nn->wf[4], bias(4), nn->e2, nn->a4, nn->d2);
  conv<64, 32, true, 1>(nn, L1, nn->d2, nn->wf[5], bias(5), nn->e1, nn->a5, nn->d1);
  conv<32, 16, true, 1>(nn, L0, nn->d1, nn->wf[6], bias(6), nn->e0, nn->a6, nn->d0);
  long n0 = (long)B * L0.V;
  head_fwd_kernel<<<div_up(n0, 256), 256, 0, s>>>(n0, nn->d0, nn->theta + nn->off[NCONV], nn->y);
  nn->cur_batch = B;
  NN_TRY(hipGetLastError());
  return CPR_OK;
}

// Gradient of sum(dy * y) for the last forward pass into nn->grad.
static int nn_backward_impl(cpr_nn* nn) {
  const int B = nn->cur_batch;
  Geo L0 = with_batch(nn->lv[0], B), L1 = with_batch(nn->lv[1], B), L2 = with_batch(nn->lv[2], B),
      L3 = with_batch(nn->lv[3], B);
  hipStream_t s = nn->stream;
  long n0 = (long)B * L0.V, n1 = (long)B * L1.V, n2 = (long)B * L2.V, n3 = (long)B * L3.V;
  // head
  head_bwd_kernel<<<div_up(n0 * 17, 256), 256, 0, s>>>(n0, nn->d0, nn->dy, nn->theta + nn->off[NCONV], nn->g0,
                                                       nn->prod);
  {
    int nb = (int)std::min<long>(256, div_up(n0, 256));
    colsum_partial_kernel<<<nb, 255, 0, s>>>(n0, 17, nn->prod, nn->gp);
    colsum_final_kernel<<<1, 64, 0, s>>>(nb, 17, nn->gp, nn->grad + nn->off[NCONV]);
  }
  // level 0 decoder: d0 = a6 + e0; dz6 = dd0 * (a6 > 0); g0 keeps de0 = dd0
  relu_mask_kernel<<<div_up(n0 * 16, 256), 256, 0, s>>>(n0 * 16, nn->g0, nn->a6, nn->g0b);
  wgrad<32, 16, true>(nn, L0, nn->d1, nn->g0b, 6);
  conv<16, 32, false, 0>(nn, L0, nn->g0b, nn->wb[6], nullptr, nullptr, nn->gu0, nullptr);
  up_bwd_kernel<<<div_up(n1 * 32, 256), 256, 0, s>>>(L1, 32, nn->gu0, nn->g1, 0);      // dd1 = de1
  relu_mask_kernel<<<div_up(n1 * 32, 256), 256, 0, s>>>(n1 * 32, nn->g1, nn->a5, nn->g1b);
  wgrad<64, 32, true>(nn, L1, nn->d2, nn->g1b, 5);
  conv<32, 64, false, 0>(nn, L1, nn->g1b, nn->wb[5], nullptr, nullptr, nn->gu1, nullptr);
  up_bwd_kernel<<<div_up(n2 * 64, 256), 256, 0, s>>>(L2, 64, nn->gu1, nn->g2, 0);      // dd2 = de2
  relu_mask_kernel<<<div_up(n2 * 64, 256), 256, 0, s>>>(n2 * 64, nn->g2, nn->a4, nn->g2b);
  wgrad<64, 64, true>(nn, L2, nn->e3, nn->g2b, 4);
  conv<64, 64, false, 0>(nn, L2, nn->g2b, nn->wb[4], nullptr, nullptr, nn->gu2, nullptr);
  up_bwd_kernel<<<div_up(n3 * 64, 256), 256, 0, s>>>(L3, 64, nn->gu2, nn->g3, 0);      // de3
  // encoder
  relu_mask_kernel<<<div_up(n3 * 64, 256), 256, 0, s>>>(n3 * 64, nn->g3, nn->e3, nn->g3b);
  wgrad<64, 64, false>(nn, L3, nn->p3, nn->g3b, 3);
  conv<64, 64, false, 0>(nn, L3, nn->g3b, nn->wb[3], nullptr, nullptr, nn->gu2, nullptr);  // dp3 (L3)
  pool_bwd_kernel<<<div_up(n2 * 64, 256), 256, 0, s>>>(L2, 64, nn->gu2, nn->g2);          // de2 += pool'(dp3)
  relu_mask_kernel<<<div_up(n2 * 64, 256), 256, 0, s>>>(n2 * 64, nn->g2, nn->e2, nn->g2b);
  wgrad<32, 64, false>(nn, L2, nn->p2, nn->g2b, 2);
  conv<64, 32, false, 0>(nn, L2, nn->g2b, nn->wb[2], nullptr, nullptr, nn->gu1, nullptr);  // dp2 (L2, 32)
  pool_bwd_kernel<<<div_up(n1 * 32, 256), 256, 0, s>>>(L1, 32, nn->gu1, nn->g1);          // de1 += pool'(dp2)
  relu_mask_kernel<<<div_up(n1 * 32, 256), 256, 0, s>>>(n1 * 32, nn->g1, nn->e1, nn->g1b);
  wgrad<16, 32, false>(nn, L1, nn->p1, nn->g1b, 1);
  conv<32, 16, false, 0>(nn, L1, nn->g1b, nn->wb[1], nullptr, nullptr, nn->gu0, nullptr);  // dp1 (L1, 16)
  pool_bwd_kernel<<<div_up(n0 * 16, 256), 256, 0, s>>>(L0, 16, nn->gu0, nn->g0);          // de0 += pool'(dp1)
  relu_mask_kernel<<<div_up(n0 * 16, 256), 256, 0, s>>>(n0 * 16, nn->g0, nn->e0, nn->g0b);
  wgrad<16, 16, false>(nn, L0, nn->x16, nn->g0b, 0);
  NN_TRY(hipGetLastError());
  return CPR_OK;
}

static int nn_alloc(cpr_nn* nn) {
  const int B = nn->max_batch;
  long n[4];
  for (int l = 0; l < 4; ++l) n[l] = (long)B * nn->lv[l].V;
  auto A = [&](float** p, long cnt) -> hipError_t { return hipMalloc((void**)p, (cnt > 0 ? cnt : 1) * sizeof(float)); };
  NN_TRY(A(&nn->theta, nn->P)); NN_TRY(A(&nn->m, nn->P)); NN_TRY(A(&nn->vv, nn->P)); NN_TRY(A(&nn->grad, nn->P));
  for (int k = 0; k < NCONV; ++k) {
    size_t nf = 27 * (CIN_PAD[k] / 16) * (COUT[k] / 16) * 64;
    NN_TRY(hipMalloc((void**)&nn->wf[k], nf * sizeof(bf16x4)));
    NN_TRY(hipMalloc((void**)&nn->wb[k], nf * sizeof(bf16x4)));
  }
  NN_TRY(A(&nn->x16, n[0] * 16)); NN_TRY(A(&nn->e0, n[0] * 16)); NN_TRY(A(&nn->p1, n[1] * 16));
  NN_TRY(A(&nn->e1, n[1] * 32)); NN_TRY(A(&nn->p2, n[2] * 32)); NN_TRY(A(&nn->e2, n[2] * 64));
  NN_TRY(A(&nn->p3, n[3] * 64)); NN_TRY(A(&nn->e3, n[3] * 64)); NN_TRY(A(&nn->a4, n[2] * 64));
  NN_TRY(A(&nn->d2, n[2] * 64)); NN_TRY(A(&nn->a5, n[1] * 32)); NN_TRY(A(&nn->d1, n[1] * 32));
  NN_TRY(A(&nn->a6, n[0] * 16)); NN_TRY(A(&nn->d0, n[0] * 16)); NN_TRY(A(&nn->y, n[0]));
  NN_TRY(A(&nn->dy, n[0])); NN_TRY(A(&nn->g0, n[0] * 16)); NN_TRY(A(&nn->g0b, n[0] * 16));
  NN_TRY(A(&nn->gu0, n[0] * 32)); NN_TRY(A(&nn->g1, n[1] * 32)); NN_TRY(A(&nn->g1b, n[1] * 32));
  NN_TRY(A(&nn->gu1, n[1] * 64)); NN_TRY(A(&nn->g2, n[2] * 64)); NN_TRY(A(&nn->g2b, n[2] * 64));
  NN_TRY(A(&nn->gu2, n[2] * 64)); NN_TRY(A(&nn->g3, n[3] * 64)); NN_TRY(A(&nn->g3b, n[3] * 64));
  NN_TRY(A(&nn->gp, 256L * 64)); NN_TRY(A(&nn->prod, n[0] * 17));
  size_t pc = 0;
  for (int k = 0; k < NCONV; ++k) {
    int l = (k <= 3) ? k : 6 - k;   // resolution level of conv k's output
    size_t c = (size_t)div_up(n[l], WG_CHUNK) * 27 * CIN_PAD[k] * COUT[k];
    pc = std::max(pc, c);
  }
  nn->part_cap = pc;
  NN_TRY(A(&nn->part, (long)pc));
  NN_TRY(A(&nn->lpart, 3L * B * 64));
  NN_TRY(A(&nn->loss, 1));
  NN_TRY(hipMemsetAsync(nn->x16, 0, n[0] * 16 * sizeof(float), nn->stream));
  return CPR_OK;
}

static void nn_free(cpr_nn* nn) {
  float* fs[] = {nn->theta, nn->m, nn->vv, nn->grad, nn->x16, nn->e0, nn->p1, nn->e1, nn->p2, nn->e2, nn->p3,
                 nn->e3, nn->a4, nn->d2, nn->a5, nn->d1, nn->a6, nn->d0, nn->y, nn->dy, nn->g0, nn->g0b,
                 nn->gu0, nn->g1, nn->g1b, nn->gu1, nn->g2, nn->g2b, nn->gu2, nn->g3, nn->g3b, nn->gp,
                 nn->prod, nn->part, nn->lpart, nn->loss};
  for (float* p : fs)
    if (p) hipFree(p);
  for (int k = 0; k < NCONV; ++k) {
    if (nn->wf[k]) hipFree(nn->wf[k]);
    if (nn->wb[k]) hipFree(nn->wb[k]);
  }
}

// Internal use by the solver's learned stage (apply.hip).
int nn_infer(cpr_nn* nn, const float* x3, float* y);
float* nn_output(cpr_nn* nn) { return nn->y; }

int nn_infer(cpr_nn* nn, const float* x3, float* y) {
  long n0 = nn->lv[0].V;
  pad_input_kernel<<<div_up(n0 * 16, 256), 256, 0, nn->stream>>>(n0, x3, nn->x16);
  int rc = nn_forward_impl(nn, 1);
  if (rc) return rc;
  if (y && y != nn->y) NN_TRY(hipMemcpyAsync(y, nn->y, n0 * sizeof(float), hipMemcpyDeviceToDevice, nn->stream));
  return CPR_OK;
}

void nn_set_stream(cpr_nn* nn, hipStream_t s) { nn->stream = s; }

extern "C" {

long long cpr_nn_num_params(void) { return nn_param_count(); }

int cpr_nn_create(int nx, int ny, int nz, int max_batch, void* stream, cpr_nn_t** out) {
  if (!out) return CPR_EINVAL;
  *out = nullptr;
  cpr_nn* nn = nullptr;
  try {
    nn = new cpr_nn();
  } catch (...) {
    return CPR_ENOMEM;
  }
  *out = nn;
  if (nx < 8 || ny < 8 || nz < 8 || nx % 8 || ny % 8 || nz % 8 || max_batch < 1 || max_batch > 64)
    return nn_err(nn, CPR_EINVAL, "grid dimensions must be multiples of 8 (>= 8), batch 1..64");
  if ((long)nx * ny * nz * max_batch > (1L << 28)) return nn_err(nn, CPR_EINVAL, "network input too large");
  nn->stream = (hipStream_t)stream;
  nn->max_batch = max_batch;
  for (int l = 0; l < 4; ++l) {
    nn->lv[l].nx = nx >> l; nn->lv[l].ny = ny >> l; nn->lv[l].nz = nz >> l;
    nn->lv[l].V = nn->lv[l].nx * nn->lv[l].ny * nn->lv[l].nz;
    nn->lv[l].batch = max_batch;
  }
  nn->P = nn_param_count();
  long o = 0;
  for (int k = 0; k < NCONV; ++k) {
    nn->off[k] = o;
    o += 27L * CIN[k] * COUT[k] + COUT[k];
  }
  nn->off[NCONV] = o;
  int rc = nn_alloc(nn);
  if (rc) return rc;
  NN_TRY(hipMemsetAsync(nn->theta, 0, nn->P * sizeof(float), nn->stream));
  NN_TRY(hipMemsetAsync(nn->m, 0, nn->P * sizeof(float), nn->stream));
  NN_TRY(hipMemsetAsync(nn->vv, 0, nn->P * sizeof(float), nn->stream));
  NN_TRY(hipStreamSynchronize(nn->stream));
  return CPR_OK;
}

void cpr_nn_destroy(cpr_nn_t* nn) {
  if (!nn) return;
  hipStreamSynchronize(nn->stream);
  nn_free(nn);
  delete nn;
}

const char* cpr_nn_last_error(const cpr_nn_t* nn) { return nn ? nn->err.c_str() : "null network"; }

int cpr_nn_set_params(cpr_nn_t* nn, const float* theta) {
  if (!nn || !theta) return CPR_EINVAL;
  NN_TRY(hipMemcpyAsync(nn->theta, theta, nn->P * sizeof(float), hipMemcpyHostToDevice, nn->stream));
  NN_TRY(hipMemsetAsync(nn->m, 0, nn->P * sizeof(float), nn->stream));
  NN_TRY(hipMemsetAsync(nn->vv, 0, nn->P * sizeof(float), nn->stream));
  nn->adam_step = 0;
  int rc = nn_refresh_frags(nn);
  if (rc) return rc;
  NN_TRY(hipStreamSynchronize(nn->stream));
  return CPR_OK;
}

int cpr_nn_get_params(cpr_nn_t* nn, float* theta) {
  if (!nn || !theta) return CPR_EINVAL;
  NN_TRY(hipMemcpyAsync(theta, nn->theta, nn->P * sizeof(float), hipMemcpyDeviceToHost, nn->stream));
  NN_TRY(hipStreamSynchronize(nn->stream));
  return CPR_OK;
}

int cpr_nn_forward(cpr_nn_t* nn, const float* x, int batch, float* y) {
  if (!nn || !x || !y) return CPR_EINVAL;
  if (batch < 1 || batch > nn->max_batch) return nn_err(nn, CPR_EINVAL, "batch out of range");
  if (!nn->frags_valid) return nn_err(nn, CPR_EINVAL, "parameters not set");
  long n0 = (long)batch * nn->lv[0].V;
  pad_input_kernel<<<div_up(n0 * 16, 256), 256, 0, nn->stream>>>(n0, x, nn->x16);
  int rc = nn_forward_impl(nn, batch);
  if (rc) return rc;
  NN_TRY(hipMemcpyAsync(y, nn->y, n0 * sizeof(float), hipMemcpyDeviceToDevice, nn->stream));
  return CPR_OK;
}

int cpr_nn_backward(cpr_nn_t* nn, const float* dy, float* grad) {
  if (!nn || !dy || !grad) return CPR_EINVAL;
  if (nn->cur_batch < 1) return nn_err(nn, CPR_EINVAL, "no forward pass to differentiate");
  long n0 = (long)nn->cur_batch * nn->lv[0].V;
  NN_TRY(hipMemcpyAsync(nn->dy, dy, n0 * sizeof(float), hipMemcpyDeviceToDevice, nn->stream));
  int rc = nn_backward_impl(nn);
  if (rc) return rc;
  NN_TRY(hipMemcpyAsync(grad, nn->grad, nn->P * sizeof(float), hipMemcpyDeviceToDevice, nn->stream));
  return CPR_OK;
}

int cpr_nn_eval_loss(cpr_nn_t* nn, const float* x, const float* t, int batch, float* loss_out) {
  if (!nn || !x || !t || !loss_out) return CPR_EINVAL;
  if (batch < 1 || batch > nn->max_batch) return nn_err(nn, CPR_EINVAL, "batch out of range");
  if (!nn->frags_valid) return nn_err(nn, CPR_EINVAL, "parameters not set");
  hipStream_t s = nn->stream;
  const int V = nn->lv[0].V;
  long n0 = (long)batch * V;
  pad_input_kernel<<<div_up(n0 * 16, 256), 256, 0, s>>>(n0, x, nn->x16);
  int rc = nn_forward_impl(nn, batch);
  if (rc) return rc;
  const int per = 64;
  loss_partial_kernel<<<batch * per, 256, 0, s>>>(V, per, nn->y, t, nn->lpart);
  loss_grad_kernel<<<div_up(n0, 256) < 1024 ? div_up(n0, 256) : 1024, 256, 0, s>>>(batch, V, per, nn->lpart, nn->y,
                                                                                  t, nn->dy, nn->loss);
  NN_TRY(hipMemcpyAsync(loss_out, nn->loss, sizeof(float), hipMemcpyDeviceToHost, s));
  NN_TRY(hipStreamSynchronize(s));
  return CPR_OK;
}

int cpr_nn_make_target(const double* e, long long n, double scale, float* t, void* stream) {
  if (!e || !t || n < 0 || !(scale > 0)) return CPR_EINVAL;
  if (n == 0) return CPR_OK;
  target_kernel<<<div_up(n, 256), 256, 0, (hipStream_t)stream>>>(n, e, 1.0 / scale, t);
  return hipGetLastError() == hipSuccess ? CPR_OK : CPR_EHIP;
}

int cpr_nn_train_step(cpr_nn_t* nn, const float* x, const float* t, int batch, float lr, float* loss_out) {
  if (!nn || !x || !t) return CPR_EINVAL;
  if (batch < 1 || batch > nn->max_batch || batch > 64) return nn_err(nn, CPR_EINVAL, "batch out of range");
  if (!nn->frags_valid) return nn_err(nn, CPR_EINVAL, "parameters not set");
  hipStream_t s = nn->stream;
  const int V = nn->lv[0].V;
  long n0 = (long)batch * V;
  pad_input_kernel<<<div_up(n0 * 16, 256), 256, 0, s>>>(n0, x, nn->x16);
  int rc = nn_forward_impl(nn, batch);
  if (rc) return rc;
  const int per = 64;
  loss_partial_kernel<<<batch * per, 256, 0, s>>>(V, per, nn->y, t, nn->lpart);
  loss_grad_kernel<<<div_up(n0, 256) < 1024 ? div_up(n0, 256) : 1024, 256, 0, s>>>(batch, V, per, nn->lpart, nn->y,
                                                                                  t, nn->dy, nn->loss);
  rc = nn_backward_impl(nn);
  if (rc) return rc;
  nn->adam_step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  float c1 = 1.f / (1.f - powf(b1, (float)nn->adam_step));
  float c2 = 1.f / (1.f - powf(b2, (float)nn->adam_step));
  adam_kernel<<<div_up(nn->P, 256), 256, 0, s>>>(nn->P, lr, b1, b2, 1e-8f, c1, c2, nn->grad, nn->m, nn->vv,
                                                 nn->theta);
  rc = nn_refresh_frags(nn);
  if (rc) return rc;
  if (loss_out) {
    NN_TRY(hipMemcpyAsync(loss_out, nn->loss, sizeof(float), hipMemcpyDeviceToHost, s));
    NN_TRY(hipStreamSynchronize(s));
  }
  NN_TRY(hipGetLastError());
  return CPR_OK;
}

}  // extern "C"
