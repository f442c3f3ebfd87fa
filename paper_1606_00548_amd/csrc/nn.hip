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
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int NCONV = 7;
constexpr int CIN[NCONV] = {3, 16, 32, 64, 64, 64, 32};
constexpr int COUT[NCONV] = {16, 32, 64, 64, 64, 32, 16};
constexpr int CIN_PAD[NCONV] = {16, 16, 32, 64, 64, 64, 32};
constexpr int WG_CHUNK = 2048;   // voxels per weight-gradient block

// FP32 -> BF16, round to nearest even (one value; the staging of the
// convolutions converts pairs with pack_bf16x2)
__device__ inline short f2bf(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

typedef __bf16 bf16x2_v __attribute__((ext_vector_type(2)));
typedef float f32x2_v __attribute__((ext_vector_type(2)));

struct Geo {
  int nx, ny, nz, V;   // grid of the tensor being produced
  int batch;
};

// ------------------------------------------------------------ convolution
// out[b][v][co] = sum_t sum_ci X~[b][v + off_t][ci] W[t][ci][co]; X~ is X on
// the same grid, or X on the half-resolution grid read at (x/2, y/2, z/2)
// when UP.  EPI 1: a = relu(acc + bias), stored in outA when given, and
// a + skip stored in outD when skip is given; with head (inference only) the
// 1x1x1 head is applied to a + skip and only y is stored.  EPI 0: raw acc in
// outA (data gradient).
//
// Implicit GEMM on v_mfma_f32_16x16x32_bf16: M = voxels, N = output
// channels, K = (tap, input channel) in steps of 32.  A workgroup (4 waves)
// owns a tile of 16 x 4 x TZ output voxels and CO/NS of the output
// channels.  At the start it stages, with all loads in flight together,
// the input it needs (tile plus a one-voxel halo, or the half-resolution
// cells under it when UP) in LDS as BF16, and the B-fragments of its
// channels for every K-step; each input value is then read from memory
// about 2-3 times instead of 27, and the K loop touches LDS only.  With
// KS = 1 each wave owns one z-plane of the tile (4 M-blocks of 16 voxels
// along x) and every K-step; with KS = 4 (small grids, to keep enough waves
// in flight) the tile is one plane and the waves split the K-steps
// round-robin, their partial tiles summed in LDS in wave order, so results
// are deterministic either way.  POOL (KS = 1 only): the workgroup also
// writes the 2x2x2 average of its activations, which its tile holds whole.
//
// K ordering (must match frag_kernel): CI >= 32: step = t * (CI/32) + chunk,
// 32 channels per step; CI = 16: step s covers taps 2s, 2s+1; CI = 4 (the
// 3-channel input, padded): step s covers taps 8s..8s+7, 4 channels each.
// Taps past 26 have zero weights.
constexpr int TX = 16, TY = 4;

__host__ __device__ constexpr int ksteps(int ci) { return ci >= 32 ? 27 * (ci / 32) : (ci == 16 ? 14 : 4); }

// a in the low half, b in the high half, both rounded to nearest even by
// one v_cvt_pk_bf16_f32
__device__ inline unsigned pack_bf16x2(float a, float b) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2_v{a, b}, bf16x2_v));
}

struct ConvArgs {
  Geo g;
  const float* X;        // input [batch][voxel][CSRC] (half-resolution grid when UP)
  const bf16x8* W;       // all B-fragments [NK][CO/16][64]
  const float* bias;     // [CO] (EPI 1)
  const float* skip;     // [batch][voxel][CO] or null
  float* outA;           // EPI 1: relu(acc + bias) (null: not stored); EPI 0: acc
  float* outD;           // EPI 1 with skip: relu(acc + bias) + skip
  const float* head;     // fused 1x1x1 head [CO + 1] (CO = 16, KS = 1) or null
  float* y;              // head output [batch][voxel]
  float* pool;           // POOL: [batch][coarse voxel][CO]
  const double* xscale;  // CSRC = 3: device scalar multiplying input channel 2 as it is loaded, or null
};

template <int CI, int CSRC, int CO, bool UP, int EPI, int KS, int NS, bool POOL>
__global__ __launch_bounds__(256) void conv_kernel(ConvArgs p) {
  static_assert(KS == 1 || KS == 4, "K split is 1 or 4");
  static_assert(CI == 4 || CI == 16 || CI % 32 == 0, "channel layout");
  static_assert(CO % (16 * NS) == 0, "channel split");
  static_assert(!POOL || KS == 1, "pooling needs whole 2x2x2 cells in the tile");
  constexpr int TZ = 4 / KS;
  constexpr int HX = UP ? TX / 2 + 2 : TX + 2;
  constexpr int HY = UP ? TY / 2 + 2 : TY + 2;
  constexpr int HZ = UP ? TZ / 2 + 2 : TZ + 2;
  constexpr int HV = HX * HY * HZ;
  constexpr int NK = ksteps(CI);
  constexpr int NT = CO / 16;          // N-blocks of the whole convolution
  constexpr int COB = CO / NS;         // output channels of this workgroup
  constexpr int NTB = COB / 16;
  // halo voxel stride in BF16 values: padded by 16 bytes for CI >= 16 so
  // that 16 lanes reading 16 bytes of 16 neighbouring voxels hit distinct banks
  constexpr int CST = CI >= 16 ? CI + 8 : CI;
  constexpr int VB = CST * 2;
  constexpr int HALO_BYTES = HV * VB;
  constexpr int W_BYTES = NK * NTB * 64 * 16;
  constexpr int RED_BYTES = KS > 1 ? KS * 64 * COB * 4 : 0;
  constexpr int POOL_BYTES = POOL ? 64 * COB * 4 : 0;
  constexpr int MAIN_BYTES = HALO_BYTES + W_BYTES;
  constexpr int SMEM = MAIN_BYTES > RED_BYTES ? (MAIN_BYTES > POOL_BYTES ? MAIN_BYTES : POOL_BYTES)
                                              : (RED_BYTES > POOL_BYTES ? RED_BYTES : POOL_BYTES);
  __shared__ __align__(16) unsigned char smem[SMEM];
  const bf16x8* wl = (const bf16x8*)(smem + HALO_BYTES);
  const Geo& g = p.g;

  // (tile, channel block) of this workgroup; consecutive blocks go to the
  // same XCD, and the channel blocks of a tile are neighbours
  const int ntx = (g.nx + TX - 1) / TX, nty = (g.ny + TY - 1) / TY, ntz = (g.nz + TZ - 1) / TZ;
  const int nblocks = ntx * nty * ntz * g.batch * NS;
  int blk = blockIdx.x;
  if ((nblocks & 7) == 0) blk = (blockIdx.x & 7) * (nblocks >> 3) + (blockIdx.x >> 3);
  const int nb = blk % NS, tile = blk / NS;
  const int tx = tile % ntx, ty = (tile / ntx) % nty, tz = (tile / (ntx * nty)) % ntz, b = tile / (ntx * nty * ntz);
  const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;

  // stage the input window as BF16 (zero outside the grid) and this
  // block's weight fragments, eight loads per thread in flight
  const int sx = UP ? g.nx >> 1 : g.nx, sy = UP ? g.ny >> 1 : g.ny, sz = UP ? g.nz >> 1 : g.nz;
  const int ox = UP ? (x0 - 1) >> 1 : x0 - 1, oy = UP ? (y0 - 1) >> 1 : y0 - 1, oz = UP ? (z0 - 1) >> 1 : z0 - 1;
  const float* Xb = p.X + (long)b * sx * sy * sz * CSRC;
  const float xs2 = (CSRC != CI && p.xscale) ? (float)*p.xscale : 1.f;
  constexpr int NQ = HV * (CI / 4);
  constexpr int NWF = NK * NTB * 64;
  for (int q0 = 0; q0 < NQ; q0 += 8 * 256) {
    float4 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int q = q0 + u * 256 + threadIdx.x;
      v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (q < NQ) {
        const int hv = q / (CI / 4), c4 = (q % (CI / 4)) * 4;
        const int hx = hv % HX, hy = (hv / HX) % HY, hz = hv / (HX * HY);
        const int px = ox + hx, py = oy + hy, pz = oz + hz;
        if (px >= 0 && px < sx && py >= 0 && py < sy && pz >= 0 && pz < sz) {
          const float* src = Xb + ((long)px + (long)sx * (py + (long)sy * pz)) * CSRC + c4;
          if (CSRC == CI) {
            v[u] = *(const float4*)src;
          } else {
            v[u].x = src[0]; v[u].y = src[1]; v[u].z = src[2] * xs2;
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int q = q0 + u * 256 + threadIdx.x;
      if (q < NQ)
        *(uint2*)(smem + (size_t)(q / (CI / 4)) * VB + (q % (CI / 4)) * 8) =
            make_uint2(pack_bf16x2(v[u].x, v[u].y), pack_bf16x2(v[u].z, v[u].w));
    }
  }
  for (int q0 = 0; q0 < NWF; q0 += 8 * 256) {
    bf16x8 w[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int q = q0 + u * 256 + threadIdx.x;
      if (q < NWF) {
        const int ks = q / (NTB * 64), j = (q / 64) % NTB, lane = q % 64;
        w[u] = p.W[((size_t)ks * NT + nb * NTB + j) * 64 + lane];
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int q = q0 + u * 256 + threadIdx.x;
      if (q < NWF) ((bf16x8*)(smem + HALO_BYTES))[q] = w[u];
    }
  }
  __syncthreads();

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, i16 = lane & 15, kq = lane >> 4;
  const int lz = KS == 1 ? wave : 0;
  // Byte address in the halo of the input under output voxel (i16, m, lz)
  // at tap (dx, dy, dz) = per-lane part + a part known at compile time once
  // the K loop is unrolled (folded into the LDS instructions' offsets).
  // Same grid: (i16 + 1 + dx) + HX (m + 1 + dy) + HX HY (lz + 1 + dz).
  // UP (x0, y0 multiples of 16 and 4): ((i16 + dx) >> 1) + 1 along x,
  // ((m + dy) >> 1) + 1 along y, and ((z0 + lz + dz) >> 1) - ((z0 - 1) >> 1)
  // along z, which depends on z0 and is uniform over the wave.
  const int lane_chunk = CI >= 32 ? 16 * kq : (CI == 16 ? 16 * (kq & 1) : 0);
  int base = 0;            // same grid
  int upb[3][3] = {};      // UP: [dx + 1][dz + 1]
  if constexpr (UP) {
#pragma unroll
    for (int ddx = 0; ddx < 3; ++ddx)
#pragma unroll
      for (int ddz = 0; ddz < 3; ++ddz) {
        const int zc = ((z0 + lz + ddz - 1) >> 1) - oz;
        upb[ddx][ddz] = ((((i16 + ddx - 1) >> 1) + 1) + HX * HY * zc) * VB + lane_chunk;
      }
  } else {
    base = ((i16 + 1) + HX + HX * HY * (lz + 1)) * VB + lane_chunk;
  }
  // KS = 1 with a skip input: its values for this wave's outputs are loaded
  // before the K loop so that their latency hides behind the MFMAs
  const long V = g.V;
  const int c0 = nb * COB;
  float skv[KS == 1 && EPI == 1 ? 4 : 1][4][NTB];
  if constexpr (KS == 1 && EPI == 1) {
    const bool has_skip = p.skip != nullptr;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int x = x0 + 4 * kq + e, y = y0 + m, z = z0 + lz;
        const bool ok = has_skip && x < g.nx && y < g.ny && z < g.nz;
        const long o = (long)b * V + x + (long)g.nx * (y + (long)g.ny * z);
#pragma unroll
        for (int n = 0; n < NTB; ++n) skv[m][e][n] = ok ? p.skip[o * CO + c0 + n * 16 + i16] : 0.f;
      }
  }
  f32x4 acc[4][NTB];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < NTB; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
  // same-grid tap offset (bytes) relative to base, m = 0
  auto toff = [](int t) { return ((t % 3 - 1) + HX * ((t / 3) % 3 - 1) + HX * HY * (t / 9 - 1)) * VB; };
  if constexpr (CI >= 32) {
    // K-steps grouped by (dz, dx, channel chunk): the three dy taps of a
    // group read the same input rows, so the wave loads each row's A
    // fragment once (6 rows of the tile plus halo, or 4 half-resolution
    // rows when UP) and the three B-fragments, then issues 12 MFMA per
    // N-block.  Groups are split over the waves when KS = 4.
    constexpr int NCH = CI / 32;
    constexpr int NR = UP ? 4 : 6;
#pragma unroll
    for (int grp = 0; grp < 9 * NCH; ++grp) {
      if (KS > 1 && (grp % KS) != wave) continue;
      const int kc = grp % NCH, dx = (grp / NCH) % 3 - 1, dz = grp / (3 * NCH) - 1;
      bf16x8 bw[3][NTB];
#pragma unroll
      for (int ddy = 0; ddy < 3; ++ddy)
#pragma unroll
        for (int n = 0; n < NTB; ++n)
          bw[ddy][n] = wl[((size_t)(((dz + 1) * 9 + ddy * 3 + (dx + 1)) * NCH + kc) * NTB + n) * 64 + lane];
      bf16x8 ar[NR];
#pragma unroll
      for (int yy = 0; yy < NR; ++yy) {
        int addr;
        if constexpr (UP)
          addr = upb[dx + 1][dz + 1] + HX * yy * VB + kc * 64;
        else
          addr = base + (dx + HX * HY * dz) * VB + HX * (yy - 1) * VB + kc * 64;
        ar[yy] = __builtin_bit_cast(bf16x8, *(const uint4*)(smem + addr));
      }
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int ddy = 0; ddy < 3; ++ddy) {
          const int yy = UP ? ((m + ddy - 1) >> 1) + 1 : m + ddy;
#pragma unroll
          for (int n = 0; n < NTB; ++n)
            acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar[yy], bw[ddy][n], acc[m][n], 0, 0, 0);
        }
    }
  } else {
#pragma unroll
  for (int ks = 0; ks < NK; ++ks) {
    if (KS > 1 && (ks % KS) != wave) continue;
    bf16x8 bw[NTB];
#pragma unroll
    for (int n = 0; n < NTB; ++n) bw[n] = wl[((size_t)ks * NTB + n) * 64 + lane];
    int sel0 = 0, sel1 = 0;     // per-lane tap offsets of this step
    if constexpr (CI == 16) {
      sel0 = (kq >> 1) ? toff(min(2 * ks + 1, 26)) : toff(2 * ks);
    } else {
      const int ta[4] = {min(8 * ks, 26), min(8 * ks + 2, 26), min(8 * ks + 4, 26), min(8 * ks + 6, 26)};
      const int tb[4] = {min(8 * ks + 1, 26), min(8 * ks + 3, 26), min(8 * ks + 5, 26), min(8 * ks + 7, 26)};
      sel0 = kq == 0 ? toff(ta[0]) : kq == 1 ? toff(ta[1]) : kq == 2 ? toff(ta[2]) : toff(ta[3]);
      sel1 = kq == 0 ? toff(tb[0]) : kq == 1 ? toff(tb[1]) : kq == 2 ? toff(tb[2]) : toff(tb[3]);
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      uint4 raw;
      if constexpr (CI == 16) {
        raw = *(const uint4*)(smem + base + sel0 + HX * m * VB);
      } else {
        const uint2 lo = *(const uint2*)(smem + base + sel0 + HX * m * VB);
        const uint2 hi = *(const uint2*)(smem + base + sel1 + HX * m * VB);
        raw = make_uint4(lo.x, lo.y, hi.x, hi.y);
      }
      const bf16x8 a = __builtin_bit_cast(bf16x8, raw);
#pragma unroll
      for (int n = 0; n < NTB; ++n) acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[n], acc[m][n], 0, 0, 0);
    }
  }
  }

  if constexpr (KS == 1) {
    // C element (row 4*kq + e, column i16) of M-block m, N-block n is
    // voxel (x0 + 4*kq + e, y0 + m, z0 + lz), channel c0 + n*16 + i16
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int y = y0 + m, z = z0 + lz;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int x = x0 + 4 * kq + e;
        const bool ok = x < g.nx && y < g.ny && z < g.nz;
        const long o = (long)b * V + x + (long)g.nx * (y + (long)g.ny * z);
        if constexpr (EPI == 1 && CO == 16) {
          if (p.head) {
            // y = sum_c head[c] (relu(acc + bias) + skip)[c] + head[CO]
            const float a = fmaxf(acc[m][0][e] + p.bias[i16], 0.f) + skv[m][e][0];
            float h = a * p.head[i16];
            h += __shfl_xor(h, 8, 16);
            h += __shfl_xor(h, 4, 16);
            h += __shfl_xor(h, 2, 16);
            h += __shfl_xor(h, 1, 16);
            if (ok && i16 == 0) p.y[o] = h + p.head[CO];
            continue;
          }
        }
#pragma unroll
        for (int n = 0; n < NTB; ++n) {
          const int co = c0 + n * 16 + i16;
          float val = acc[m][n][e];
          if constexpr (EPI == 1) {
            val = fmaxf(val + p.bias[co], 0.f);
            acc[m][n][e] = val;
            if (!ok) continue;
            if (p.outA) p.outA[o * CO + co] = val;
            if (p.skip) p.outD[o * CO + co] = val + skv[m][e][n];
          } else if (ok) {
            p.outA[o * CO + co] = val;
          }
        }
      }
    }
    if constexpr (POOL) {
      // 2x2 (x, y) sums in registers, the z pairs (waves 2k, 2k+1) via LDS
      __syncthreads();
      float* ps = (float*)smem;   // [lz][py][px][COB]
#pragma unroll
      for (int py = 0; py < 2; ++py)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
          for (int n = 0; n < NTB; ++n) {
            const float sum = (acc[2 * py][n][2 * q] + acc[2 * py][n][2 * q + 1]) +
                              (acc[2 * py + 1][n][2 * q] + acc[2 * py + 1][n][2 * q + 1]);
            ps[((lz * 2 + py) * 8 + 2 * kq + q) * COB + n * 16 + i16] = sum;
          }
      __syncthreads();
      const int cnx = g.nx >> 1, cny = g.ny >> 1, cnz = g.nz >> 1;
      for (int q = threadIdx.x; q < 32 * COB; q += 256) {
        const int co = q % COB, cell = q / COB;
        const int px = cell & 7, py = (cell >> 3) & 1, pz = cell >> 4;
        const int cx = (x0 >> 1) + px, cy = (y0 >> 1) + py, cz = (z0 >> 1) + pz;
        if (cx >= cnx || cy >= cny || cz >= cnz) continue;
        const float v = ps[((2 * pz * 2 + py) * 8 + px) * COB + co] + ps[(((2 * pz + 1) * 2 + py) * 8 + px) * COB + co];
        p.pool[((long)b * cnx * cny * cnz + cx + (long)cnx * (cy + (long)cny * cz)) * CO + c0 + co] = 0.125f * v;
      }
    }
  } else {
    // partial tiles to LDS, summed in wave order by all threads
    __syncthreads();
    float* red = (float*)smem;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int n = 0; n < NTB; ++n)
#pragma unroll
        for (int e = 0; e < 4; ++e) red[((size_t)wave * 64 + m * 16 + 4 * kq + e) * COB + n * 16 + i16] = acc[m][n][e];
    __syncthreads();
    for (int q = threadIdx.x; q < 64 * COB; q += 256) {
      const int vox = q / COB, co = c0 + q % COB;
      const int x = x0 + (vox & 15), y = y0 + (vox >> 4), z = z0;
      if (x >= g.nx || y >= g.ny || z >= g.nz) continue;
      const long o = (long)b * V + x + (long)g.nx * (y + (long)g.ny * z);
      float val = red[q];
#pragma unroll
      for (int w = 1; w < KS; ++w) val += red[(size_t)w * 64 * COB + q];
      if (EPI == 1) {
        const float a = fmaxf(val + p.bias[co], 0.f);
        if (p.outA) p.outA[o * CO + co] = a;
        if (p.skip) p.outD[o * CO + co] = a + p.skip[o * CO + co];
      } else {
        p.outA[o * CO + co] = val;
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

// (tap, channel) of K-index kk (0..31) of K-step ks for a convolution whose
// K side has ck channels (the ordering the convolution kernel reads).
__device__ inline void k_index(int ck, int ks, int kk, int& t, int& c) {
  if (ck >= 32) {
    t = ks / (ck / 32);
    c = (ks % (ck / 32)) * 32 + kk;
  } else if (ck == 16) {
    t = 2 * ks + (kk >> 4);
    c = kk & 15;
  } else {
    const int k = ks * 32 + kk;
    t = k >> 2;
    c = k & 3;
  }
}

// BF16 B-fragments of conv weights W[27][ci][co] (FP32 master) for
// v_mfma_f32_16x16x32_bf16: frag[ks][nt][lane][e] is the weight at K-index
// kk = 8*(lane/16) + e of step ks and output column nt*16 + lane%16.
// Forward: K = (tap, ci) with ck = 4 for the 3-channel input, N = co.
// Backward (data gradient): taps mirrored (26 - t), K = (tap, co), N = ci.
__global__ void frag_kernel(int ci, int ck, int co, int backward, const float* __restrict__ W,
                            bf16x8* __restrict__ frag) {
  const int nt_n = backward ? ci / 16 : co / 16;
  const int kside = backward ? co : ck;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ksteps(kside) * nt_n * 64) return;
  const int lane = q % 64, nt = (q / 64) % nt_n, ks = q / (64 * nt_n);
  const int n = nt * 16 + lane % 16;
  bf16x8 f;
  for (int e = 0; e < 8; ++e) {
    int t, c;
    k_index(kside, ks, 8 * (lane / 16) + e, t, c);
    float w = 0.f;
    if (t < 27) {
      if (!backward && c < ci) w = W[((size_t)t * ci + c) * co + n];
      if (backward) w = W[((size_t)(26 - t) * ci + n) * co + c];
    }
    f[e] = __builtin_bit_cast(__bf16, (unsigned short)f2bf(w));
  }
  frag[q] = f;
}

}  // namespace

// ------------------------------------------------------------ host object

struct cpr_nn {
  std::string err;
  DevAlloc mem;        // device allocator taken at creation
  hipStream_t stream = nullptr;
  Geo lv[4];           // grid per level (batch = max_batch)
  int max_batch = 0;
  long P = 0;
  long off[NCONV + 1]; // parameter offsets: conv k weights at off[k], bias after
  float* theta = nullptr;
  float* m = nullptr;
  float* vv = nullptr;
  float* grad = nullptr;
  bf16x8* wf[NCONV] = {};
  bf16x8* wb[NCONV] = {};
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

static int fwd_frags(int k) { return ksteps(k == 0 ? 4 : CIN[k]) * (COUT[k] / 16) * 64; }
static int bwd_frags(int k) { return ksteps(COUT[k]) * (CIN[k] / 16) * 64; }

static int nn_refresh_frags(cpr_nn* nn) {
  for (int k = 0; k < NCONV; ++k) {
    const float* W = nn->theta + nn->off[k];
    frag_kernel<<<div_up(fwd_frags(k), 256), 256, 0, nn->stream>>>(CIN[k], k == 0 ? 4 : CIN[k], COUT[k], 0, W,
                                                                   nn->wf[k]);
    if (k > 0)
      frag_kernel<<<div_up(bwd_frags(k), 256), 256, 0, nn->stream>>>(CIN[k], CIN[k], COUT[k], 1, W, nn->wb[k]);
  }
  nn->frags_valid = true;
  NN_TRY(hipGetLastError());
  return CPR_OK;
}

// Grids of at least 64K voxels use whole-tile waves (K split 1); smaller
// ones, and 64-channel inputs at full resolution (whose LDS window would
// not fit beside the weights), split the K-steps over the 4 waves of a
// workgroup.  The output channels are split over NS workgroups so that a
// workgroup's weight fragments fit in 56 KB of LDS and, where the channels
// allow, the launch has at least 512 workgroups.
constexpr int WMAX = 56 * 1024;
constexpr int wbytes(int ci, int co, int ns) { return ksteps(ci) * (co / (16 * ns)) * 1024; }

static ConvArgs cargs(Geo g, const float* X, const bf16x8* W, const float* bias, const float* skip, float* outA,
                      float* outD) {
  ConvArgs a{};
  a.g = g; a.X = X; a.W = W; a.bias = bias; a.skip = skip; a.outA = outA; a.outD = outD;
  return a;
}

template <int CI, int CSRC, int CO, bool UP, int EPI, int KS, bool POOL>
static void conv_ns(cpr_nn* nn, const ConvArgs& a, long tiles, int ns) {
  if constexpr (wbytes(CI, CO, 1) <= WMAX)
    if (ns == 1) {
      conv_kernel<CI, CSRC, CO, UP, EPI, KS, 1, POOL><<<tiles, 256, 0, nn->stream>>>(a);
      return;
    }
  if constexpr (CO >= 32 && wbytes(CI, CO, 2) <= WMAX)
    if (ns == 2) {
      conv_kernel<CI, CSRC, CO, UP, EPI, KS, 2, POOL><<<tiles * 2, 256, 0, nn->stream>>>(a);
      return;
    }
  if constexpr (CO >= 64)
    if (ns == 4) conv_kernel<CI, CSRC, CO, UP, EPI, KS, 4, POOL><<<tiles * 4, 256, 0, nn->stream>>>(a);
}

// a.pool (POOL only): also write the 2x2x2 average of the activations,
// fused when the tiles hold whole cells, else by a separate pass.
template <int CI, int CSRC, int CO, bool UP, int EPI, bool POOL = false>
static void conv(cpr_nn* nn, ConvArgs a) {
  const Geo& g = a.g;
  const long vox = (long)g.batch * g.V;
  const long txy = (long)div_up(g.nx, TX) * div_up(g.ny, TY);
  const bool whole = vox >= 65536 && (UP || CI <= 32);
  const long tiles = whole ? txy * div_up(g.nz, 4) * g.batch : txy * g.nz * g.batch;
  int ns = 1;
  while (wbytes(CI, CO, ns) > WMAX) ns *= 2;
  while (CO / (16 * ns) >= 2 && ns < 4 && tiles * ns < 512) ns *= 2;
  if (whole) {
    conv_ns<CI, CSRC, CO, UP, EPI, 1, POOL>(nn, a, tiles, ns);
    return;
  }
  ConvArgs b = a;
  b.head = nullptr;
  b.y = nullptr;
  b.pool = nullptr;
  conv_ns<CI, CSRC, CO, UP, EPI, 4, false>(nn, b, tiles, ns);
  if (POOL) {
    Geo c = g;
    c.nx >>= 1; c.ny >>= 1; c.nz >>= 1;
    c.V = c.nx * c.ny * c.nz;
    pool_kernel<<<div_up((long)g.batch * c.V * CO, 256), 256, 0, nn->stream>>>(c, CO, a.outA, a.pool);
  }
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

// x3: input features [B][voxel][3].  train: keep what the backward pass
// needs (pre-skip activations, d0) and run the head separately; otherwise
// only what inference needs, with the head fused into the last convolution.
static int nn_forward_impl(cpr_nn* nn, const float* x3, int B, bool train, const double* xscale = nullptr) {
  Geo L0 = with_batch(nn->lv[0], B), L1 = with_batch(nn->lv[1], B), L2 = with_batch(nn->lv[2], B),
      L3 = with_batch(nn->lv[3], B);
  hipStream_t s = nn->stream;
  auto bias = [&](int k) { return nn->theta + nn->off[k] + 27L * CIN[k] * COUT[k]; };
  const float* head = nn->theta + nn->off[NCONV];
  ConvArgs a = cargs(L0, x3, nn->wf[0], bias(0), nullptr, nn->e0, nullptr);
  a.pool = nn->p1;
  a.xscale = xscale;
  conv<4, 3, 16, false, 1, true>(nn, a);
  a = cargs(L1, nn->p1, nn->wf[1], bias(1), nullptr, nn->e1, nullptr);
  a.pool = nn->p2;
  conv<16, 16, 32, false, 1, true>(nn, a);
  a = cargs(L2, nn->p2, nn->wf[2], bias(2), nullptr, nn->e2, nullptr);
  a.pool = nn->p3;
  conv<32, 32, 64, false, 1, true>(nn, a);
  conv<64, 64, 64, false, 1>(nn, cargs(L3, nn->p3, nn->wf[3], bias(3), nullptr, nn->e3, nullptr));
  conv<64, 64, 64, true, 1>(nn, cargs(L2, nn->e3, nn->wf[4], bias(4), nn->e2, train ? nn->a4 : nullptr, nn->d2));
  conv<64, 64, 32, true, 1>(nn, cargs(L1, nn->d2, nn->wf[5], bias(5), nn->e1, train ? nn->a5 : nullptr, nn->d1));
  const long n0 = (long)B * L0.V;
  if (train || n0 < 65536) {
    conv<32, 32, 16, true, 1>(nn, cargs(L0, nn->d1, nn->wf[6], bias(6), nn->e0, nn->a6, nn->d0));
    head_fwd_kernel<<<div_up(n0, 256), 256, 0, s>>>(n0, nn->d0, head, nn->y);
  } else {
    a = cargs(L0, nn->d1, nn->wf[6], bias(6), nn->e0, nullptr, nullptr);
    a.head = head;
    a.y = nn->y;
    conv<32, 32, 16, true, 1>(nn, a);
  }
  nn->cur_batch = train ? B : 0;
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
  conv<16, 16, 32, false, 0>(nn, cargs(L0, nn->g0b, nn->wb[6], nullptr, nullptr, nn->gu0, nullptr));
  up_bwd_kernel<<<div_up(n1 * 32, 256), 256, 0, s>>>(L1, 32, nn->gu0, nn->g1, 0);      // dd1 = de1
  relu_mask_kernel<<<div_up(n1 * 32, 256), 256, 0, s>>>(n1 * 32, nn->g1, nn->a5, nn->g1b);
  wgrad<64, 32, true>(nn, L1, nn->d2, nn->g1b, 5);
  conv<32, 32, 64, false, 0>(nn, cargs(L1, nn->g1b, nn->wb[5], nullptr, nullptr, nn->gu1, nullptr));
  up_bwd_kernel<<<div_up(n2 * 64, 256), 256, 0, s>>>(L2, 64, nn->gu1, nn->g2, 0);      // dd2 = de2
  relu_mask_kernel<<<div_up(n2 * 64, 256), 256, 0, s>>>(n2 * 64, nn->g2, nn->a4, nn->g2b);
  wgrad<64, 64, true>(nn, L2, nn->e3, nn->g2b, 4);
  conv<64, 64, 64, false, 0>(nn, cargs(L2, nn->g2b, nn->wb[4], nullptr, nullptr, nn->gu2, nullptr));
  up_bwd_kernel<<<div_up(n3 * 64, 256), 256, 0, s>>>(L3, 64, nn->gu2, nn->g3, 0);      // de3
  // encoder
  relu_mask_kernel<<<div_up(n3 * 64, 256), 256, 0, s>>>(n3 * 64, nn->g3, nn->e3, nn->g3b);
  wgrad<64, 64, false>(nn, L3, nn->p3, nn->g3b, 3);
  conv<64, 64, 64, false, 0>(nn, cargs(L3, nn->g3b, nn->wb[3], nullptr, nullptr, nn->gu2, nullptr));  // dp3 (L3)
  pool_bwd_kernel<<<div_up(n2 * 64, 256), 256, 0, s>>>(L2, 64, nn->gu2, nn->g2);          // de2 += pool'(dp3)
  relu_mask_kernel<<<div_up(n2 * 64, 256), 256, 0, s>>>(n2 * 64, nn->g2, nn->e2, nn->g2b);
  wgrad<32, 64, false>(nn, L2, nn->p2, nn->g2b, 2);
  conv<64, 64, 32, false, 0>(nn, cargs(L2, nn->g2b, nn->wb[2], nullptr, nullptr, nn->gu1, nullptr));  // dp2 (L2, 32)
  pool_bwd_kernel<<<div_up(n1 * 32, 256), 256, 0, s>>>(L1, 32, nn->gu1, nn->g1);          // de1 += pool'(dp2)
  relu_mask_kernel<<<div_up(n1 * 32, 256), 256, 0, s>>>(n1 * 32, nn->g1, nn->e1, nn->g1b);
  wgrad<16, 32, false>(nn, L1, nn->p1, nn->g1b, 1);
  conv<32, 32, 16, false, 0>(nn, cargs(L1, nn->g1b, nn->wb[1], nullptr, nullptr, nn->gu0, nullptr));  // dp1 (L1, 16)
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
  auto A = [&](float** p, long cnt) -> hipError_t {
    return dev_malloc(nn->mem, (void**)p, (cnt > 0 ? cnt : 1) * sizeof(float));
  };
  NN_TRY(A(&nn->theta, nn->P)); NN_TRY(A(&nn->m, nn->P)); NN_TRY(A(&nn->vv, nn->P)); NN_TRY(A(&nn->grad, nn->P));
  for (int k = 0; k < NCONV; ++k) {
    NN_TRY(dev_malloc(nn->mem, (void**)&nn->wf[k], fwd_frags(k) * sizeof(bf16x8)));
    NN_TRY(dev_malloc(nn->mem, (void**)&nn->wb[k], bwd_frags(k) * sizeof(bf16x8)));
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
  for (float* p : fs) dev_free(nn->mem, p);
  for (int k = 0; k < NCONV; ++k) {
    dev_free(nn->mem, nn->wf[k]);
    dev_free(nn->mem, nn->wb[k]);
  }
}

// Internal use by the solver's learned stage: x3's third channel is
// multiplied by *xscale (device scalar) as the network loads it.
int nn_infer(cpr_nn* nn, const float* x3, float* y, const double* xscale);
float* nn_output(cpr_nn* nn) { return nn->y; }

int nn_infer(cpr_nn* nn, const float* x3, float* y, const double* xscale) {
  long n0 = nn->lv[0].V;
  int rc = nn_forward_impl(nn, x3, 1, false, xscale);
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
  nn->mem = current_allocator();
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

int cpr_nn_get_adam(cpr_nn_t* nn, float* m, float* v, long long* step) {
  if (!nn || !m || !v || !step) return CPR_EINVAL;
  NN_TRY(hipMemcpyAsync(m, nn->m, nn->P * sizeof(float), hipMemcpyDeviceToHost, nn->stream));
  NN_TRY(hipMemcpyAsync(v, nn->vv, nn->P * sizeof(float), hipMemcpyDeviceToHost, nn->stream));
  NN_TRY(hipStreamSynchronize(nn->stream));
  *step = nn->adam_step;
  return CPR_OK;
}

int cpr_nn_set_adam(cpr_nn_t* nn, const float* m, const float* v, long long step) {
  if (!nn || !m || !v) return CPR_EINVAL;
  if (step < 0) return nn_err(nn, CPR_EINVAL, "negative Adam step count");
  NN_TRY(hipMemcpyAsync(nn->m, m, nn->P * sizeof(float), hipMemcpyHostToDevice, nn->stream));
  NN_TRY(hipMemcpyAsync(nn->vv, v, nn->P * sizeof(float), hipMemcpyHostToDevice, nn->stream));
  NN_TRY(hipStreamSynchronize(nn->stream));
  nn->adam_step = (long)step;
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
  pad_input_kernel<<<div_up(n0 * 16, 256), 256, 0, nn->stream>>>(n0, x, nn->x16);   // for the weight gradient
  int rc = nn_forward_impl(nn, x, batch, true);
  if (rc) return rc;
  NN_TRY(hipMemcpyAsync(y, nn->y, n0 * sizeof(float), hipMemcpyDeviceToDevice, nn->stream));
  return CPR_OK;
}

int cpr_nn_infer(cpr_nn_t* nn, const float* x, float* y) {
  if (!nn || !x || !y) return CPR_EINVAL;
  if (!nn->frags_valid) return nn_err(nn, CPR_EINVAL, "parameters not set");
  return nn_infer(nn, x, y, nullptr);
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
  int rc = nn_forward_impl(nn, x, batch, false);
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
  pad_input_kernel<<<div_up(n0 * 16, 256), 256, 0, s>>>(n0, x, nn->x16);   // for the weight gradient
  int rc = nn_forward_impl(nn, x, batch, true);
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
