// Learned grid preconditioner: a 3-level 3-D U-Net on the AIM grid with
// hand-written inference and training kernels for gfx950.
//
// The network (channels-last tensors [z][y][x][c], base width C):
//   a0 = relu(conv3(in, 2->C))           s0 = relu(conv3(a0, C->C))
//   a1 = relu(conv3(pool(s0), C->2C))    s1 = relu(conv3(a1, 2C->2C))
//   a2 = relu(conv3(pool(s1), 2C->4C))   a3 = relu(conv3(a2, 4C->4C))
//   a4 = relu(conv3([up(a3), s1], 6C->2C))  a5 = relu(conv3(a4, 2C->2C))
//   a6 = relu(conv3([up(a5), s0], 3C->C))   a7 = relu(conv3(a6, C->C))
//   out = a7 W^T + b (1x1x1, C->2)
// with 3x3x3 "same" convolutions, 2x2x2 average pooling and nearest
// upsampling.  A batch of samples is stacked along z (each sample Ds planes
// deep, Ds a multiple of 4, so pooling never mixes samples); the 3x3x3
// kernels treat the planes of other samples as the zero padding.  Weights
// and activations are bfloat16; the convolutions are LDS-tiled implicit GEMMs
// on the 16x16x32 bf16 MFMA with fp32 accumulation (the data gradient is the
// same GEMM with flipped, transposed weights); the weight gradients of the
// 3x3x3 layers (the 2-channel input layer on its input padded to 16
// channels) are GEMMs over bricks of positions, all 27 taps per workgroup, on
// the same MFMA, the 1x1 output layer's a one-pass fp32 reduction, all summed
// in two deterministic stages; master weights and Adam moments are fp32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <random>
#include <string>
#include <type_traits>
#include <vector>

#include "aim_internal.h"

namespace aim {
namespace unetk {

typedef float f32x4 __attribute__((__vector_size__(4 * sizeof(float))));

__device__ __forceinline__ uint16_t f2bf(float f) {  // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

__device__ __forceinline__ void pos_xyz(int64_t p, int W, int H, int& x, int& y, int& z) {
  x = int(p % W);
  y = int((p / W) % H);
  z = int(p / (int64_t(W) * H));
}

// ---------------------------------------------------------------------------
// 3x3x3 convolution, LDS-tiled: a workgroup computes a 16 x BY x 4 brick of
// output positions for all output channels.  It stages the 18 x (BY+2) x 6
// input tile (brick plus one-point halo, all CIN channels, bf16) in LDS once,
// so every input element feeds 27 taps from LDS.  Wave w takes the brick's z
// slice w: BY groups of 16 positions (its y rows) against TILES tiles of 16
// output channels, so each weight load feeds BY MFMAs (BY = 4 for layers
// with one output tile on grids that still give 1,024 workgroups: 6-7% less
// forward time at 64^3 and 128x128x64; else 2, as taller bricks with more
// tiles, or on small grids, cost occupancy or parallelism).  K is the
// flattened (tap, channel) index, 27 * CIN,
// walked in chunks of 32 on the 16x16x32 bf16 MFMA: lane l supplies
// A[co = l % 16][k = 8 (l / 16) + i] (weights, 16 bytes from global memory)
// and B[k][position l % 16] (16 bytes from LDS) and receives
// C[co = 4 (l / 16) + i][position l % 16].  The tail chunk is zero-padded.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int kBX = 16, kBZ = 4;                             // output brick (x, z)
constexpr int kTX = kBX + 2, kTZ = kBZ + 2;                  // input tile (x, z)
// output brick height (y): 2 rows, or 4 (each weight fragment then feeds
// four MFMAs) for layers with one 16-channel output tile on large grids
constexpr int conv_by(int) { return 2; }

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) {
  bf16x8 r;
  __builtin_memcpy(&r, &v, 16);
  return r;
}

template <int CIN, int TILES, bool OUT_BF16, int kBY = conv_by(CIN)>
__global__ __launch_bounds__(256) void conv3_lds_kernel(const uint16_t* __restrict__ X, int ldx,
                                                        int ox, int D, int Ds, int H, int W,
                                                        const uint16_t* __restrict__ Wt,
                                                        const float* __restrict__ bias, void* Y,
                                                        int ldy, int oy, int relu) {
  // the input channels are staged in CS parts of CH channels (two for 64 and
  // more, so the tile takes 28-41 KB of LDS instead of 55-83 KB and more
  // workgroups fit on a CU); the K walk covers one part after the other
  constexpr int CS = CIN >= 64 ? 2 : 1, CH = CIN / CS, C8 = CH / 8;
  constexpr int kTY = kBY + 2, kTilePos = kTX * kTY * kTZ;
  static_assert(CH % 8 == 0, "channels in groups of 8");
  __shared__ uint4 tile[kTilePos * C8];  // [position][channel / 8], 8 bf16 per entry
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nbx = (W + kBX - 1) / kBX, nby = (H + kBY - 1) / kBY;
  int b = int(blockIdx.x);
  const int bx = b % nbx;
  b /= nbx;
  const int by = b % nby, bz = b / nby;
  const int x0 = bx * kBX, y0 = by * kBY, z0 = bz * kBZ;
  const int col = lane & 15, kg = lane >> 4;
  constexpr int K = 27 * CIN, KH = 27 * CH, NCH = (KH + 31) / 32;
  // the wave's output plane and whether its z - 1 / z + 1 neighbours lie in
  // the same sample (a brick may straddle two samples)
  const int zo = z0 + wave, zs = (zo / Ds) * Ds;
  const bool lo_ok = zo - 1 >= zs, hi_ok = zo + 1 < zs + Ds;
  f32x4 acc[kBY][TILES];
#pragma unroll
  for (int g = 0; g < kBY; ++g)
#pragma unroll
    for (int t = 0; t < TILES; ++t) acc[g][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bf16x8 zero = as_bf16x8(make_uint4(0u, 0u, 0u, 0u));
  // weights stream through a ring of PF K steps held in registers: the
  // loads for step ch + PF are issued while step ch computes (on small grids
  // the few workgroups would otherwise wait out a load latency per step)
  // (depth 4, or 2 where the extra registers would cost occupancy that the
  // LDS tile leaves)
  constexpr int PF = CS > 1 ? 2 : TILES <= 2 ? 4 : 2;
#pragma unroll 1
  for (int part = 0; part < CS; ++part) {
    if (part > 0) __syncthreads();  // the previous part's tile has been read
    // stage the tile in batches of 8 loads per thread, all in flight together
    constexpr int kTileWords = kTilePos * C8, kBatch = 8 * 256;
    for (int u0 = 0; u0 < kTileWords; u0 += kBatch) {
      uint4 v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int u = u0 + j * 256 + tid;
        v[j] = make_uint4(0u, 0u, 0u, 0u);
        if (u < kTileWords) {
          const int c8 = u % C8, pos = u / C8;
          const int gx = x0 + pos % kTX - 1, gy = y0 + (pos / kTX) % kTY - 1,
                    gz = z0 + pos / (kTX * kTY) - 1;
          if (gx >= 0 && gy >= 0 && gz >= 0 && gx < W && gy < H && gz < D)
            v[j] = *reinterpret_cast<const uint4*>(X + ((int64_t(gz) * H + gy) * W + gx) * ldx +
                                                   ox + part * CH + 8 * c8);
        }
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int u = u0 + j * 256 + tid;
        if (u < kTileWords) tile[u] = v[j];
      }
    }
    __syncthreads();
    // K step index kp within the part: tap kp / CH, channel part * CH + kp % CH
    auto wload = [&](int kp, bf16x8* w) {
      const int tp = kp / CH, k = tp * CIN + part * CH + (kp - tp * CH);
#pragma unroll
      for (int t = 0; t < TILES; ++t)
        w[t] = kp < KH
                   ? as_bf16x8(*reinterpret_cast<const uint4*>(Wt + int64_t(t * 16 + col) * K + k))
                   : zero;
    };
    bf16x8 wq[PF][TILES];
#pragma unroll
    for (int j = 0; j < PF; ++j) wload(32 * j + 8 * kg, wq[j]);
    for (int c0 = 0; c0 < NCH; c0 += PF) {
#pragma unroll
      for (int j = 0; j < PF; ++j) {
        const int ch = c0 + j;
        if (ch < NCH) {
          const int kp = ch * 32 + 8 * kg;
          const bool kv = kp < KH;
          bf16x8 wc[TILES];
#pragma unroll
          for (int t = 0; t < TILES; ++t) wc[t] = wq[j][t];
          if (ch + PF < NCH) wload(kp + 32 * PF, wq[j]);
          const int tap = kv ? kp / CH : 0, ci = kv ? kp % CH : 0;
          const int dx = tap % 3, dy = (tap / 3) % 3, dz = tap / 9;
          const bool bok = kv && (dz == 1 || (dz == 0 ? lo_ok : hi_ok));
          bf16x8 bv[kBY];
#pragma unroll
          for (int g = 0; g < kBY; ++g) {
            const int pos = ((wave + dz) * kTY + g + dy) * kTX + col + dx;
            bv[g] = bok ? as_bf16x8(tile[pos * C8 + ci / 8]) : zero;
          }
#pragma unroll
          for (int t = 0; t < TILES; ++t)
#pragma unroll
            for (int g = 0; g < kBY; ++g)
              acc[g][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wc[t], bv[g], acc[g][t], 0, 0, 0);
        }
      }
    }
  }
  const int x = x0 + col, z = z0 + wave;
#pragma unroll
  for (int g = 0; g < kBY; ++g) {
    const int y = y0 + g;
    if (x >= W || y >= H || z >= D) continue;
    const int64_t p = (int64_t(z) * H + y) * W + x;
#pragma unroll
    for (int t = 0; t < TILES; ++t) {
      const int co = t * 16 + 4 * kg;
      float v[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        v[i] = acc[g][t][i] + (bias ? bias[co + i] : 0.f);
        if (relu) v[i] = fmaxf(v[i], 0.f);
      }
      if constexpr (OUT_BF16) {
        ushort4 o;
        o.x = f2bf(v[0]);
        o.y = f2bf(v[1]);
        o.z = f2bf(v[2]);
        o.w = f2bf(v[3]);
        *reinterpret_cast<ushort4*>(static_cast<uint16_t*>(Y) + p * ldy + oy + co) = o;
      } else {
        *reinterpret_cast<float4*>(static_cast<float*>(Y) + p * ldy + oy + co) =
            make_float4(v[0], v[1], v[2], v[3]);
      }
    }
  }
}

// first layer: 2 fp32 input channels (the complex64 grid), C outputs, relu
template <int C>
__global__ __launch_bounds__(256) void conv_first_kernel(const float* __restrict__ in, int D, int Ds,
                                                         int H, int W, const float* __restrict__ Wm,
                                                         const float* __restrict__ bias,
                                                         uint16_t* __restrict__ Y, int ldy, int oy) {
  __shared__ float w[C * 27 * 2];
  for (int i = threadIdx.x; i < C * 54; i += blockDim.x) w[i] = bf2f(f2bf(Wm[i]));  // bf16 weights
  __syncthreads();
  const int64_t P = int64_t(D) * H * W;
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= P) return;
  int x, y, z;
  pos_xyz(p, W, H, x, y, z);
  const int zs = (z / Ds) * Ds;  // the sample's first plane
  float acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = bias[c];
  // the 27 neighbours are loaded together (outside the sample: zero)
  float2 nb[27];
#pragma unroll
  for (int tap = 0; tap < 27; ++tap) {
    const int nx = x + tap % 3 - 1, ny = y + (tap / 3) % 3 - 1, nz = z + tap / 9 - 1;
    nb[tap] = make_float2(0.f, 0.f);
    if (nx >= 0 && ny >= 0 && nz >= zs && nx < W && ny < H && nz < zs + Ds)
      nb[tap] = *reinterpret_cast<const float2*>(in + 2 * ((int64_t(nz) * H + ny) * W + nx));
  }
#pragma unroll
  for (int tap = 0; tap < 27; ++tap) {
    // the first layer reads bf16-rounded inputs, like every other layer
    const float v0 = bf2f(f2bf(nb[tap].x)), v1 = bf2f(f2bf(nb[tap].y));
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] += w[(c * 27 + tap) * 2] * v0 + w[(c * 27 + tap) * 2 + 1] * v1;
  }
  // the C bf16 outputs as 16-byte words (the row stride and offset are
  // multiples of 8 channels)
  static_assert(C % 8 == 0, "outputs in groups of 8");
  uint32_t wv[C / 2];
#pragma unroll
  for (int c = 0; c < C; c += 2)
    wv[c / 2] = uint32_t(f2bf(fmaxf(acc[c], 0.f))) | (uint32_t(f2bf(fmaxf(acc[c + 1], 0.f))) << 16);
  uint4* dst = reinterpret_cast<uint4*>(Y + p * ldy + oy);
#pragma unroll
  for (int q = 0; q < C / 8; ++q)
    dst[q] = make_uint4(wv[4 * q], wv[4 * q + 1], wv[4 * q + 2], wv[4 * q + 3]);
}

// 1x1 output layer: out[p][2] = a[p][:] W^T + b (fp32)
template <int C>
__global__ void conv_out_kernel(const uint16_t* __restrict__ a, int64_t P,
                                const float* __restrict__ Wm, const float* __restrict__ b,
                                float* __restrict__ out) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= P) return;
  float o0 = b[0], o1 = b[1];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const float v = bf2f(a[p * C + c]);
    o0 += bf2f(f2bf(Wm[c])) * v;
    o1 += bf2f(f2bf(Wm[C + c])) * v;
  }
  out[2 * p] = o0;
  out[2 * p + 1] = o1;
}

// ---------------------------------------------------------------------------
// weight gradients: dW[co][t][ci] (+)= sum_p dY[p][co] X[p + d(t)][ci],
// computed per chunk of positions (two-stage, deterministic)
// ---------------------------------------------------------------------------
// Weight gradients of a 3x3x3 layer on MFMA for bf16 X and dY:
//   dW[co][t][ci] = sum_p dY[p][co] X[p + d(t)][ci]
// (p and p + d(t) in the same sample), a GEMM over positions per tap.  A
// workgroup takes one 16-channel tile of the input (blockIdx.y) and a strided
// set of bricks of 16 x 2 x 4 output positions, and does all 27 taps of every
// brick, so each dY and X element is staged once per brick rather than once
// per tap.  Per brick it stages dY transposed ([co][position], 128 positions)
// and the input brick with its one-point halo as three x-shifted copies
// ([shift][ci][halo row][x], copy s holding X at x + s - 1), so the operand
// of every tap is one aligned 16-byte LDS read; channel strides carry 16
// bytes of padding so the 16 lanes of a read hit distinct banks.  The K
// steps are the brick's 4 z-planes (32 positions: x 0..15 of two rows); lane
// l supplies A[co = l % 16][k = 8 (l / 16) + i] (dY) and B[k][ci = l % 16]
// (X) and holds C[co = 4 (l / 16) + i][ci = l % 16].  Wave w does the taps
// w, w + 4, ...  Partial sums per workgroup (part[chunk][co][t][ci], input
// channels ci < CST only: the first layer runs on its two channels padded to
// 16); the workgroups of the first tile also sum the bias gradient
// partb[chunk][co] = sum_p dY[p][co] (when partb is set).
template <int CIN, int COUT, int CST = CIN>
__global__ __launch_bounds__(256) void wgrad_mfma_kernel(
    const uint16_t* __restrict__ X, int ldx, int ox, const uint16_t* __restrict__ dY, int ldy,
    int oy, int D, int Ds, int H, int W, int nbrick, float* __restrict__ part,
    float* __restrict__ partb) {
  constexpr int BX = 16, BY = 2, BZ = 4, BP = BX * BY * BZ;   // output brick
  constexpr int RY = BY + 2, RZ = BZ + 2, ROWS = RY * RZ;     // halo rows (y, z)
  constexpr int NTC = COUT / 16, TW = 7;                      // co tiles, taps per wave
  constexpr int XS_CI = ROWS * BX + 8;                        // per channel, + 16 B pad
  constexpr int XS_COPY = 16 * XS_CI;                         // one shifted copy
  constexpr int DY_CO = BP + 8;                               // per output channel, + pad
  constexpr int BR = 256 / COUT;                              // bias: threads per channel
  static_assert(CIN % 16 == 0 && COUT % 16 == 0 && CST <= CIN && COUT <= 256, "layout");
  __shared__ __attribute__((aligned(16))) uint16_t xs[3 * XS_COPY];
  __shared__ __attribute__((aligned(16))) uint16_t dyT[COUT * DY_CO];
  __shared__ float red[256];
  const int ti = blockIdx.y;
  const bool bias = partb != nullptr && ti == 0;  // uniform over the block
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, kg = lane >> 4;
  const int yk = kg >> 1, xk = 8 * (kg & 1);  // this lane's K positions in a step
  const int nbx = (W + BX - 1) / BX, nby = (H + BY - 1) / BY;
  const bf16x8 zero = as_bf16x8(make_uint4(0u, 0u, 0u, 0u));
  f32x4 acc[TW][NTC];
#pragma unroll
  for (int j = 0; j < TW; ++j)
#pragma unroll
    for (int t = 0; t < NTC; ++t) acc[j][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;
  for (int br = blockIdx.x; br < nbrick; br += gridDim.x) {
    int b = br;
    const int x0 = (b % nbx) * BX;
    b /= nbx;
    const int y0 = (b % nby) * BY, z0 = (b / nby) * BZ;
    __syncthreads();  // the previous brick's operands have been read
    // dY, 8 channels (16 bytes) per load, transposed; zero outside the grid
    for (int u = tid; u < BP * (COUT / 8); u += 256) {
      const int c8 = u % (COUT / 8), pp = u / (COUT / 8);
      const int x = x0 + pp % BX, y = y0 + (pp / BX) % BY, z = z0 + pp / (BX * BY);
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (x < W && y < H && z < D)
        v = *reinterpret_cast<const uint4*>(dY + ((int64_t(z) * H + y) * W + x) * ldy + oy +
                                            8 * c8);
      const uint16_t* e = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
      for (int j = 0; j < 8; ++j) dyT[(8 * c8 + j) * DY_CO + pp] = e[j];
    }
    // X, this tile's 16 channels (two 16-byte loads per position), brick plus
    // halo, into the three shifted copies; zero outside the grid
    for (int u = tid; u < ROWS * (BX + 2) * 2; u += 256) {
      const int h = u & 1, q = u >> 1, xq = q % (BX + 2), row = q / (BX + 2);
      const int gx = x0 + xq - 1, gy = y0 + row % RY - 1, gz = z0 + row / RY - 1;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (gx >= 0 && gy >= 0 && gz >= 0 && gx < W && gy < H && gz < D)
        v = *reinterpret_cast<const uint4*>(X + ((int64_t(gz) * H + gy) * W + gx) * ldx + ox +
                                            16 * ti + 8 * h);
      const uint16_t* e = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
      for (int sft = 0; sft < 3; ++sft) {
        const int x = xq - sft;
        if (x >= 0 && x < BX) {
#pragma unroll
          for (int j = 0; j < 8; ++j)
            xs[sft * XS_COPY + (8 * h + j) * XS_CI + row * BX + x] = e[j];
        }
      }
    }
    __syncthreads();
    if (bias)  // positions outside the grid were staged as zero
      for (int pp = tid / COUT; pp < BP; pp += BR) bsum += bf2f(dyT[(tid % COUT) * DY_CO + pp]);
#pragma unroll
    for (int kc = 0; kc < BZ; ++kc) {
      // the step's plane and whether its z - 1 / z + 1 neighbours lie in the
      // same sample
      const int z = z0 + kc, zs = (z / Ds) * Ds;
      const bool lo_ok = z - 1 >= zs, hi_ok = z + 1 < zs + Ds;
      bf16x8 av[NTC];
#pragma unroll
      for (int t = 0; t < NTC; ++t)
        av[t] = as_bf16x8(*reinterpret_cast<const uint4*>(&dyT[(t * 16 + col) * DY_CO + kc * 32 +
                                                              8 * kg]));
#pragma unroll
      for (int j = 0; j < TW; ++j) {
        const int tap = wave + 4 * j;
        if (tap < 27) {
          const int dx = tap % 3, dy = (tap / 3) % 3, dz = tap / 9;
          const bool zok = dz == 1 || (dz == 0 ? lo_ok : hi_ok);
          const int row = (kc + dz) * RY + yk + dy;
          const bf16x8 bv =
              zok ? as_bf16x8(*reinterpret_cast<const uint4*>(
                        &xs[dx * XS_COPY + col * XS_CI + row * BX + xk]))
                  : zero;
#pragma unroll
          for (int t = 0; t < NTC; ++t)
            acc[j][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[t], bv, acc[j][t], 0, 0, 0);
        }
      }
    }
  }
  const int ci = 16 * ti + col;
#pragma unroll
  for (int j = 0; j < TW; ++j) {
    const int tap = wave + 4 * j;
    if (tap < 27 && ci < CST) {
#pragma unroll
      for (int t = 0; t < NTC; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int co = t * 16 + 4 * kg + i;
          part[((int64_t(blockIdx.x) * COUT + co) * 27 + tap) * CST + ci] = acc[j][t][i];
        }
    }
  }
  if (bias) {
    red[tid] = bsum;
    __syncthreads();
    if (tid < COUT) {
      float a = 0.f;
      for (int q = 0; q < BR; ++q) a += red[q * COUT + tid];
      partb[int64_t(blockIdx.x) * COUT + tid] = a;
    }
  }
}

// grad[i] (+)= sum_c part[c][i] for the weights and gradb[i] (+)= sum_c
// partb[c][i] for the biases of one layer, in one launch: a block takes 64
// consecutive entries (the first nwb blocks the weights, the rest the
// biases), its four waves a quarter of the chunks each, eight loads in
// flight per thread
__global__ __launch_bounds__(256) void reduce_chunks_kernel(const float* __restrict__ partw,
                                                            int nchunk, int64_t nw,
                                                            float* __restrict__ gradw, int nwb,
                                                            const float* __restrict__ partb,
                                                            int64_t nbias,
                                                            float* __restrict__ gradb) {
  __shared__ float red[4][64];
  const bool wt = int(blockIdx.x) < nwb;
  const float* part = wt ? partw : partb;
  float* grad = wt ? gradw : gradb;
  const int64_t n = wt ? nw : nbias;
  const int e = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int64_t i = int64_t(wt ? blockIdx.x : blockIdx.x - nwb) * 64 + e;
  float s = 0.f;
  if (i < n)
    for (int c0 = q; c0 < nchunk; c0 += 32) {
      float v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int c = c0 + 4 * j;
        v[j] = c < nchunk ? part[int64_t(c) * n + i] : 0.f;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) s += v[j];
    }
  red[q][e] = s;
  __syncthreads();
  if (q == 0 && i < n) grad[i] += (red[0][e] + red[1][e]) + (red[2][e] + red[3][e]);
}

// the first layer's input for its weight gradient: the complex64 grid
// [P][2] rounded to bf16 (as the forward pass reads it), zero-padded to 16
// channels
__global__ void pack_in16_kernel(const float* __restrict__ in, int64_t P,
                                 uint16_t* __restrict__ o) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const float2 v = *reinterpret_cast<const float2*>(in + 2 * p);
  uint4 a = make_uint4(uint32_t(f2bf(v.x)) | (uint32_t(f2bf(v.y)) << 16), 0u, 0u, 0u);
  uint4* d = reinterpret_cast<uint4*>(o + 16 * p);
  d[0] = a;
  d[1] = make_uint4(0u, 0u, 0u, 0u);
}


// ---------------------------------------------------------------------------
// pooling, upsampling, masks
// ---------------------------------------------------------------------------
// The elementwise kernels below take 8 consecutive channels (one 16-byte
// bf16 word, two fp32 float4) per thread; every channel count, row stride and
// channel offset they see is a multiple of 8, and every grid has fewer than
// 2^31 positions.
__device__ __forceinline__ void unpack8(uint4 v, float* f) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    f[2 * j] = __uint_as_float(w[j] << 16);
    f[2 * j + 1] = __uint_as_float(w[j] & 0xFFFF0000u);
  }
}
__device__ __forceinline__ uint4 pack8(const float* f) {
  uint32_t w[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) w[j] = uint32_t(f2bf(f[2 * j])) | (uint32_t(f2bf(f[2 * j + 1])) << 16);
  return make_uint4(w[0], w[1], w[2], w[3]);
}
__device__ __forceinline__ void load8(const float* p, float* f) {
  const float4 a = *reinterpret_cast<const float4*>(p), b = *reinterpret_cast<const float4*>(p + 4);
  f[0] = a.x; f[1] = a.y; f[2] = a.z; f[3] = a.w;
  f[4] = b.x; f[5] = b.y; f[6] = b.z; f[7] = b.w;
}
// fine position of child k (0..7) of coarse position (x, y, z)
__device__ __forceinline__ int64_t child(int x, int y, int z, int k, int H, int W) {
  return (int64_t(2 * z + (k >> 2)) * H + 2 * y + ((k >> 1) & 1)) * W + 2 * x + (k & 1);
}

// gradient of the 1x1 output layer, first stage: per chunk of positions
// part[chunk][co][ci] = sum_p dout[p][co] a[p][ci] and partb[chunk][co] =
// sum_p dout[p][co] (2 outputs, C bf16 inputs), each position read once
template <int C>
__global__ __launch_bounds__(256) void outgrad_partial_kernel(const uint16_t* __restrict__ a,
                                                              const float* __restrict__ dout,
                                                              int64_t P, int64_t chunk,
                                                              float* __restrict__ part,
                                                              float* __restrict__ partb) {
  constexpr int NE = 2 * C + 2;
  __shared__ float red[NE][257];
  float acc[NE];
#pragma unroll
  for (int j = 0; j < NE; ++j) acc[j] = 0.f;
  const int64_t pb = int64_t(blockIdx.x) * chunk, pe = min(P, pb + chunk);
  for (int64_t p = pb + threadIdx.x; p < pe; p += 256) {
    const float2 d = *reinterpret_cast<const float2*>(dout + 2 * p);
    float v[C];
#pragma unroll
    for (int c8 = 0; c8 < C / 8; ++c8)
      unpack8(*reinterpret_cast<const uint4*>(a + p * C + 8 * c8), v + 8 * c8);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      acc[c] += d.x * v[c];
      acc[C + c] += d.y * v[c];
    }
    acc[2 * C] += d.x;
    acc[2 * C + 1] += d.y;
  }
#pragma unroll
  for (int j = 0; j < NE; ++j) red[j][threadIdx.x] = acc[j];
  __syncthreads();
  if (threadIdx.x < NE) {
    float t = 0.f;
    for (int q = 0; q < 256; ++q) t += red[threadIdx.x][q];
    if (threadIdx.x < 2 * C)
      part[int64_t(blockIdx.x) * 2 * C + threadIdx.x] = t;
    else
      partb[int64_t(blockIdx.x) * 2 + threadIdx.x - 2 * C] = t;
  }
}

// Y[q][c] = bf16(mean of X over the 8 children of coarse position q)
__global__ void pool_kernel(const uint16_t* __restrict__ X, int ldx, int ox, int C, int D, int H,
                            int W, uint16_t* __restrict__ Y) {  // Y [P/8][C]
  const int Hc = H / 2, Wc = W / 2, C8 = C / 8;
  const int n = (D / 2) * Hc * Wc * C8;
  const int i = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = 8 * (i % C8), q = i / C8;
  const int x = q % Wc, y = (q / Wc) % Hc, z = q / (Wc * Hc);
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int k = 0; k < 8; ++k) {
    float f[8];
    unpack8(*reinterpret_cast<const uint4*>(X + child(x, y, z, k, H, W) * ldx + ox + c), f);
#pragma unroll
    for (int j = 0; j < 8; ++j) s[j] += f[j];
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) s[j] *= 0.125f;
  *reinterpret_cast<uint4*>(Y + int64_t(q) * C + c) = pack8(s);
}

// nearest upsampling: Y[p][oy + c] = X[parent(p)][c]
__global__ void up_kernel(const uint16_t* __restrict__ X, int C, int Dc, int Hc, int Wc,
                          uint16_t* __restrict__ Y, int ldy, int oy) {  // fine [8 Pc][ldy]
  const int H = 2 * Hc, W = 2 * Wc, C8 = C / 8;
  const int n = 2 * Dc * H * W * C8;
  const int i = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = 8 * (i % C8), p = i / C8;
  const int x = p % W, y = (p / W) % H, z = p / (W * H);
  const int64_t q = (int64_t(z / 2) * Hc + y / 2) * Wc + x / 2;
  *reinterpret_cast<uint4*>(Y + int64_t(p) * ldy + oy + c) =
      *reinterpret_cast<const uint4*>(X + q * C + c);
}

// gb[p][c] = bf16(g[p][og + c]) where act[p][oa + c] > 0, else 0
__global__ void mask_kernel(const float* __restrict__ g, int ldg, int og,
                            const uint16_t* __restrict__ act, int lda, int oa, int C, int64_t P,
                            uint16_t* __restrict__ gb) {
  const int C8 = C / 8;
  const int64_t n = P * C8;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = 8 * int(i % C8);
  const int64_t p = i / C8;
  float v[8], a[8];
  load8(g + p * ldg + og + c, v);
  unpack8(*reinterpret_cast<const uint4*>(act + p * lda + oa + c), a);
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = a[j] > 0.f ? v[j] : 0.f;
  *reinterpret_cast<uint4*>(gb + p * C + c) = pack8(v);
}

// coarse gb[q][c] = bf16(sum of the 8 children g[child][og + c]) masked by act[q][c] > 0
__global__ void up_backward_kernel(const float* __restrict__ g, int ldg, int og, int C, int Dc,
                                   int Hc, int Wc, const uint16_t* __restrict__ act,
                                   uint16_t* __restrict__ gb) {
  const int H = 2 * Hc, W = 2 * Wc, C8 = C / 8;
  const int n = Dc * Hc * Wc * C8;
  const int i = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = 8 * (i % C8), q = i / C8;
  const int x = q % Wc, y = (q / Wc) % Hc, z = q / (Wc * Hc);
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int k = 0; k < 8; ++k) {
    float f[8];
    load8(g + child(x, y, z, k, H, W) * ldg + og + c, f);
#pragma unroll
    for (int j = 0; j < 8; ++j) s[j] += f[j];
  }
  float a[8];
  unpack8(*reinterpret_cast<const uint4*>(act + int64_t(q) * C + c), a);
#pragma unroll
  for (int j = 0; j < 8; ++j) s[j] = a[j] > 0.f ? s[j] : 0.f;
  *reinterpret_cast<uint4*>(gb + int64_t(q) * C + c) = pack8(s);
}

// fine gb[p][c] = bf16((gc[parent][c] / 8 + skip[p][os + c]) * (act[p][oa + c] > 0))
__global__ void pool_backward_kernel(const float* __restrict__ gc, int C, int D, int H, int W,
                                     const float* __restrict__ skip, int lds, int os,
                                     const uint16_t* __restrict__ act, int lda, int oa,
                                     uint16_t* __restrict__ gb) {
  const int Hc = H / 2, Wc = W / 2, C8 = C / 8;
  const int n = D * H * W * C8;
  const int i = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = 8 * (i % C8), p = i / C8;
  const int x = p % W, y = (p / W) % H, z = p / (W * H);
  const int64_t q = (int64_t(z / 2) * Hc + y / 2) * Wc + x / 2;
  float v[8], sk[8], a[8];
  load8(gc + q * C + c, v);
  load8(skip + int64_t(p) * lds + os + c, sk);
  unpack8(*reinterpret_cast<const uint4*>(act + int64_t(p) * lda + oa + c), a);
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = a[j] > 0.f ? v[j] * 0.125f + sk[j] : 0.f;
  *reinterpret_cast<uint4*>(gb + int64_t(p) * C + c) = pack8(v);
}

// gradient through the 1x1 output layer: ga[p][c] = bf16((dout[p] W)[c]) masked by a7 > 0
template <int C>
__global__ void out_backward_kernel(const float* __restrict__ dout, const float* __restrict__ Wm,
                                    const uint16_t* __restrict__ act, int64_t P,
                                    uint16_t* __restrict__ ga) {
  static_assert(C % 8 == 0, "channels in 16-byte words");
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const float2 d = *reinterpret_cast<const float2*>(dout + 2 * p);
#pragma unroll
  for (int c8 = 0; c8 < C / 8; ++c8) {
    float a[8], v[8];
    unpack8(*reinterpret_cast<const uint4*>(act + p * C + 8 * c8), a);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int c = 8 * c8 + j;
      const float g = d.x * bf2f(f2bf(Wm[c])) + d.y * bf2f(f2bf(Wm[C + c]));
      v[j] = a[j] > 0.f ? g : 0.f;
    }
    *reinterpret_cast<uint4*>(ga + p * C + 8 * c8) = pack8(v);
  }
}

// ---------------------------------------------------------------------------
// parameters: fp32 master -> bf16 (same layout) and flipped [ci][26 - t][co]
// ---------------------------------------------------------------------------
__global__ void to_bf16_kernel(const float* __restrict__ w, int64_t n, uint16_t* __restrict__ o) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    o[i] = f2bf(w[i]);
}

// all flipped copies in one launch: blockIdx.y picks the layer
struct FlipSet {
  int n;                                  // layers
  int cout[12], cin[12];
  int64_t w_off[12], f_off[12];
};
__global__ void flip_kernel(const float* __restrict__ wall, FlipSet fs,
                            uint16_t* __restrict__ oall) {
  const int L = blockIdx.y;
  const int Cout = fs.cout[L], Cin = fs.cin[L];
  const float* w = wall + fs.w_off[L];
  uint16_t* o = oall + fs.f_off[L];
  const int64_t n = int64_t(Cout) * 27 * Cin;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int ci = int(i % Cin), t = int((i / Cin) % 27), co = int(i / (int64_t(Cin) * 27));
    o[(int64_t(ci) * 27 + (26 - t)) * Cout + co] = f2bf(w[i]);
  }
}

__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, int64_t n, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// mean-squared error: dout = scale (out - tgt); per-block partial sums of
// (out - tgt)^2 * lscale into part[blockIdx.x]
__global__ __launch_bounds__(256) void mse_kernel(const float* __restrict__ out,
                                                  const float* __restrict__ tgt, int64_t n,
                                                  float scale, float lscale,
                                                  float* __restrict__ dout,
                                                  float* __restrict__ part) {
  __shared__ float red[256];
  float s = 0.f;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const float d = out[i] - tgt[i];
    dout[i] = scale * d;
    s += d * d * lscale;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void fill_kernel(float* __restrict__ p, int64_t n, float v) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

// blocks of 256 threads for n elements taken 8 per thread (no grid-stride loop)
inline unsigned gsz8(int64_t n) { return unsigned((n / 8 + 255) / 256); }

inline unsigned gsz(int64_t n, int per = 256) {
  int64_t g = (n + per - 1) / per;
  return unsigned(g < 1 ? 1 : (g > 16384 ? 16384 : g));
}

}  // namespace unetk
}  // namespace aim

// ===========================================================================
// the network object
// ===========================================================================
using namespace aim::unetk;

namespace {

struct Layer {
  int cout, cin, taps;
  int64_t w_off, b_off;  // into the flat fp32 parameter vector
  int64_t flip_off;      // into the flipped bf16 vector (3x3x3 layers)
};

struct Acts {  // per-level activation / gradient buffers, reused while they fit
  int D = 0, Ds = 0, H = 0, W = 0;  // the current batch: D = samples x Ds planes
  int64_t cap = 0;                  // level-0 positions the buffers hold
  std::vector<void*> bufs;
  uint16_t *a0, *cat0, *p0, *a1, *cat1, *p1, *a2, *a3, *a4, *a5, *a6, *a7;
  float *out, *gcat0, *g0, *gcat1, *g1, *g2, *part, *partb;
  uint16_t *gb0, *gb1, *gb2, *in16;
  int64_t part_n = 0, partb_n = 0;
};

thread_local std::string g_unet_err;

}  // namespace

struct aim_unet_s {
  int C = 16;
  std::vector<Layer> layers;
  int64_t nparam = 0, nflip = 0;
  float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  uint16_t *wb = nullptr, *wf = nullptr;
  int64_t step = 0;
  Acts acts;

  void build_layers() {
    const int c0 = C, c1 = 2 * C, c2 = 4 * C;
    const int spec[11][3] = {{c0, 2, 27},       {c0, c0, 27}, {c1, c0, 27}, {c1, c1, 27},
                             {c2, c1, 27},      {c2, c2, 27}, {c1, c2 + c1, 27},
                             {c1, c1, 27},      {c0, c1 + c0, 27}, {c0, c0, 27}, {2, c0, 1}};
    int64_t off = 0, foff = 0;
    for (auto& s : spec) {
      Layer L{s[0], s[1], s[2], off, 0, foff};
      off += int64_t(s[0]) * s[1] * s[2];
      L.b_off = off;
      off += s[0];
      if (s[2] == 27) foff += int64_t(s[0]) * s[1] * 27;
      layers.push_back(L);
    }
    nparam = off;
    nflip = foff;
  }

  void alloc_params() {
    AIM_HIP(hipMalloc(&w, nparam * 4));
    AIM_HIP(hipMalloc(&g, nparam * 4));
    AIM_HIP(hipMalloc(&m, nparam * 4));
    AIM_HIP(hipMalloc(&v, nparam * 4));
    AIM_HIP(hipMalloc(&wb, nparam * 2));
    AIM_HIP(hipMalloc(&wf, nflip * 2));
    AIM_HIP(hipMemset(g, 0, nparam * 4));
    AIM_HIP(hipMemset(m, 0, nparam * 4));
    AIM_HIP(hipMemset(v, 0, nparam * 4));
  }

  void free_acts() {
    for (void* p : acts.bufs) (void)hipFree(p);
    acts = Acts();
  }

  ~aim_unet_s() {
    (void)hipDeviceSynchronize();
    free_acts();
    for (void* p : {(void*)w, (void*)g, (void*)m, (void*)v, (void*)wb, (void*)wf})
      if (p) (void)hipFree(p);
  }

  // derived bf16 copies of the master weights
  void refresh(hipStream_t s) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3(gsz(nparam)), dim3(256), 0, s, w, nparam, wb);
    AIM_HIP(hipGetLastError());
    FlipSet fs{};
    int64_t mx = 0;
    for (const auto& L : layers) {
      if (L.taps != 27 || L.cin == 2) continue;
      AIM_REQUIRE(fs.n < 12, AIM_ERR_STATE, "too many layers");
      fs.cout[fs.n] = L.cout;
      fs.cin[fs.n] = L.cin;
      fs.w_off[fs.n] = L.w_off;
      fs.f_off[fs.n] = L.flip_off;
      ++fs.n;
      mx = std::max<int64_t>(mx, int64_t(L.cout) * 27 * L.cin);
    }
    hipLaunchKernelGGL(flip_kernel, dim3(gsz(mx), unsigned(fs.n)), dim3(256), 0, s, w, fs, wf);
    AIM_HIP(hipGetLastError());
  }

  // buffers for nb samples of Ds x H x W stacked along z
  void ensure_acts(int nb, int Ds, int H, int W) {
    AIM_REQUIRE(Ds % 4 == 0 && H % 4 == 0 && W % 4 == 0 && Ds >= 4 && H >= 4 && W >= 4,
                AIM_ERR_GRID, "U-Net grid dimensions must be multiples of 4");
    AIM_REQUIRE(nb >= 1 && int64_t(nb) * Ds * H * W < (int64_t(1) << 31) / 96, AIM_ERR_GRID,
                "U-Net batch too large");
    const int D = nb * Ds;
    if (int64_t(D) * H * W > acts.cap) {
      free_acts();
      acts.cap = int64_t(D) * H * W;
      alloc_acts(acts.cap);
    }
    acts.D = D;
    acts.Ds = Ds;
    acts.H = H;
    acts.W = W;
  }

  void alloc_acts(int64_t P0) {
    const int64_t P1 = P0 / 8, P2 = P1 / 8;
    const int c0 = C, c1 = 2 * C, c2 = 4 * C;
    auto al = [&](int64_t bytes) {
      void* p = nullptr;
      AIM_HIP(hipMalloc(&p, bytes < 256 ? 256 : bytes));
      acts.bufs.push_back(p);
      return p;
    };
    auto b16 = [&](int64_t n) { return static_cast<uint16_t*>(al(n * 2)); };
    auto f32 = [&](int64_t n) { return static_cast<float*>(al(n * 4)); };
    acts.a0 = b16(P0 * c0);
    acts.cat0 = b16(P0 * (c1 + c0));
    acts.p0 = b16(P1 * c0);
    acts.a1 = b16(P1 * c1);
    acts.cat1 = b16(P1 * (c2 + c1));
    acts.p1 = b16(P2 * c1);
    acts.a2 = b16(P2 * c2);
    acts.a3 = b16(P2 * c2);
    acts.a4 = b16(P1 * c1);
    acts.a5 = b16(P1 * c1);
    acts.a6 = b16(P0 * c0);
    acts.a7 = b16(P0 * c0);
    acts.out = f32(P0 * 2);
    acts.gcat0 = f32(P0 * (c1 + c0));
    acts.g0 = f32(P0 * c0);
    acts.gcat1 = f32(P1 * (c2 + c1));
    acts.g1 = f32(P1 * c1);
    acts.g2 = f32(P2 * c2);
    acts.gb0 = b16(P0 * c0);
    acts.gb1 = b16(P1 * c1);
    acts.gb2 = b16(P2 * c2);
    acts.in16 = b16(P0 * 16);
    // two-stage gradient sums: weight partials (chunks x entries, at most
    // 2^22) and bias partials (chunks x output channels)
    acts.part_n = std::max<int64_t>(int64_t(1) << 22, int64_t(kMaxChunks) * 64);
    acts.part = f32(acts.part_n);
    acts.partb_n = int64_t(kMaxChunks) * 64;
    acts.partb = f32(acts.partb_n);
  }

  // at most this many chunks of positions per gradient reduction
  static constexpr int64_t kMaxChunks = 1024;

  // weight and bias partials of one layer (nchunk chunks each) into g
  void reduce(int64_t nchunk, int64_t nw, float* gw, int64_t nb, float* gb, hipStream_t s) {
    const int nwb = int((nw + 63) / 64), nbb = int((nb + 63) / 64);
    hipLaunchKernelGGL(reduce_chunks_kernel, dim3(unsigned(nwb + nbb)), dim3(256), 0, s,
                       acts.part, int(nchunk), nw, gw, nwb, acts.partb, nb, gb);
    AIM_HIP(hipGetLastError());
  }

  // -- launch helpers --------------------------------------------------------
  void conv(const uint16_t* X, int ldx, int ox, int cin, int D, int Ds, int H, int W, const uint16_t* Wt,
            const float* bias, void* Y, int ldy, int oy, int cout, bool out_bf16, bool relu,
            hipStream_t s) {
    AIM_REQUIRE(ox % 8 == 0 && ldx % 8 == 0 && oy % 4 == 0 && cout % 16 == 0, AIM_ERR_STATE,
                "channel blocks must be aligned");
    const int tiles = cout / 16;
    const int rl = relu ? 1 : 0;
    auto blocks = [&](int by) {
      return unsigned(((W + kBX - 1) / kBX) * ((H + by - 1) / by) * ((D + kBZ - 1) / kBZ));
    };
    const bool tall = tiles == 1 && blocks(4) >= 1024;
#define AIM_CONV_BY(CI, T, BY)                                                                  \
  {                                                                                             \
    const unsigned nb = blocks(BY);                                                             \
    if (out_bf16)                                                                               \
      hipLaunchKernelGGL((conv3_lds_kernel<CI, T, true, BY>), dim3(nb), dim3(256), 0, s, X, ldx, \
                         ox, D, Ds, H, W, Wt, bias, Y, ldy, oy, rl);                             \
    else                                                                                        \
      hipLaunchKernelGGL((conv3_lds_kernel<CI, T, false, BY>), dim3(nb), dim3(256), 0, s, X,    \
                         ldx, ox, D, Ds, H, W, Wt, bias, Y, ldy, oy, rl);                        \
    AIM_HIP(hipGetLastError());                                                                 \
    return;                                                                                     \
  }
#define AIM_CONV(CI, T)                                                                          \
  if (cin == CI && tiles == T) {                                                                \
    if (T == 1 && tall) AIM_CONV_BY(CI, T, (T == 1 ? 4 : 2))                                    \
    AIM_CONV_BY(CI, T, 2)                                                                       \
  }
    // the (input channels, output tiles) pairs of the network's forward and
    // data-gradient convolutions
    AIM_CONV(16, 1)
    AIM_CONV(16, 2)
    AIM_CONV(16, 3)
    AIM_CONV(32, 1)
    AIM_CONV(32, 2)
    AIM_CONV(32, 4)
    AIM_CONV(32, 6)
    AIM_CONV(48, 1)
    AIM_CONV(64, 2)
    AIM_CONV(64, 4)
    AIM_CONV(96, 2)
#undef AIM_CONV
#undef AIM_CONV_BY
    throw aim::Error(AIM_ERR_STATE, "unsupported channel count");
  }

  template <typename TX, typename TY>
  void wgrad(const TX* X, int ldx, int ox, int cin, const TY* dY, int ldy, int oy, int cout, int D,
             int Ds, int H, int W, const Layer& L, hipStream_t s) {
    const int64_t P = int64_t(D) * H * W;
    AIM_REQUIRE(int64_t(cout) * cin <= 256 * 24 && cout <= 64, AIM_ERR_STATE,
                "layer too wide for wgrad");
    const int64_t entries = int64_t(cout) * L.taps * cin;
    int64_t nchunk = 0;
    bool done = false;
    if constexpr (std::is_same_v<TY, uint16_t>) {
      if (L.taps == 27) {
        const uint16_t* Xb;
        int kcin = cin;
        if constexpr (std::is_same_v<TX, float>) {
          // the 2-channel first layer, on its bf16-rounded input padded to 16
          AIM_REQUIRE(cin == 2 && ldx == 2 && ox == 0, AIM_ERR_STATE, "first-layer input layout");
          hipLaunchKernelGGL(pack_in16_kernel, dim3(unsigned((P + 255) / 256)), dim3(256), 0, s, X,
                             P, acts.in16);
          AIM_HIP(hipGetLastError());
          Xb = acts.in16;
          ldx = 16;
          kcin = 16;
        } else {
          Xb = X;
        }
        // bricks of 16 x 2 x 4 positions, dealt to nchunk workgroups per input
        // tile: about 1,024 workgroups, at most 2^22 partial sums (or 16 chunks)
        const int64_t nbrick = int64_t((W + 15) / 16) * ((H + 1) / 2) * ((D + 3) / 4);
        const int nti = kcin / 16;
        nchunk = std::min<int64_t>(nbrick, (1024 + nti - 1) / nti);
        nchunk = std::max<int64_t>(1, std::min<int64_t>(
                                          nchunk, std::max<int64_t>(16, acts.part_n / entries)));
        AIM_REQUIRE(nchunk * entries <= acts.part_n && nchunk * cout <= acts.partb_n &&
                        nbrick < (int64_t(1) << 31),
                    AIM_ERR_STATE, "gradient partial buffer too small");
#define AIM_WG(CI, CO, CS)                                                                      \
  if (!done && kcin == CI && cin == CS && cout == CO) {                                       \
    hipLaunchKernelGGL((wgrad_mfma_kernel<CI, CO, CS>), dim3(unsigned(nchunk), CI / 16),       \
                       dim3(256), 0, s, Xb, ldx, ox, dY, ldy, oy, D, Ds, H, W, int(nbrick),    \
                       acts.part, acts.partb);                                                \
    done = true;                                                                              \
  }
        // the (input, output, stored input) channel triples of the 3x3x3 layers
        AIM_WG(16, 16, 2)
        AIM_WG(16, 16, 16)
        AIM_WG(16, 32, 16)
        AIM_WG(32, 32, 32)
        AIM_WG(32, 64, 32)
        AIM_WG(64, 64, 64)
        AIM_WG(96, 32, 96)
        AIM_WG(48, 16, 48)
#undef AIM_WG
      }
    }
    if constexpr (std::is_same_v<TX, uint16_t> && std::is_same_v<TY, float>) {
      if (!done && L.taps == 1 && cin == 16 && cout == 2 && ldx == 16 && ox == 0 && ldy == 2 &&
          oy == 0) {
        // the 1x1 output layer: one pass over the positions
        nchunk = std::min<int64_t>(1024, (P + 1023) / 1024);
        const int64_t chunk = (P + nchunk - 1) / nchunk;
        nchunk = (P + chunk - 1) / chunk;
        AIM_REQUIRE(nchunk * entries <= acts.part_n && nchunk * cout <= acts.partb_n,
                    AIM_ERR_STATE, "gradient partial buffer too small");
        hipLaunchKernelGGL((outgrad_partial_kernel<16>), dim3(unsigned(nchunk)), dim3(256), 0, s,
                           X, dY, P, chunk, acts.part, acts.partb);
        done = true;
      }
    }
    AIM_REQUIRE(done, AIM_ERR_STATE, "unsupported weight-gradient layer");
    AIM_HIP(hipGetLastError());
    reduce(nchunk, entries, g + L.w_off, cout, g + L.b_off, s);
  }

  // forward pass on nb samples stacked along z: in = complex64 grids
  // [nb][Ds][H][W] (2 fp32 each), out fp32 [nb Ds H W][2]
  void forward(const float* in, int nb, int Ds, int H, int W, float* out, hipStream_t s) {
    ensure_acts(nb, Ds, H, W);
    Acts& a = acts;
    const int D = a.D;
    const int c0 = C, c1 = 2 * C, c2 = 4 * C;
    const int D1 = D / 2, H1 = H / 2, W1 = W / 2, D2 = D / 4, H2 = H / 4, W2 = W / 4;
    const int Ds1 = Ds / 2, Ds2 = Ds / 4;
    const int64_t P0 = int64_t(D) * H * W, P1 = P0 / 8;
    const Layer* Ls = layers.data();
    AIM_REQUIRE(C == 16, AIM_ERR_STATE, "only base width 16 is built");
    AIM_REQUIRE(c0 % 8 == 0, AIM_ERR_STATE, "first-layer outputs go out as 16-byte words");
    hipLaunchKernelGGL((conv_first_kernel<16>), dim3(gsz(P0)), dim3(256), 0, s, in, D, Ds, H, W,
                       w + Ls[0].w_off, w + Ls[0].b_off, a.a0, c0, 0);
    AIM_HIP(hipGetLastError());
    conv(a.a0, c0, 0, c0, D, Ds, H, W, wb + Ls[1].w_off, w + Ls[1].b_off, a.cat0, c1 + c0, c1, c0, true, true, s);
    hipLaunchKernelGGL(pool_kernel, dim3(gsz8(P1 * c0)), dim3(256), 0, s, a.cat0, c1 + c0, c1, c0, D, H, W, a.p0);
    conv(a.p0, c0, 0, c0, D1, Ds1, H1, W1, wb + Ls[2].w_off, w + Ls[2].b_off, a.a1, c1, 0, c1, true, true, s);
    conv(a.a1, c1, 0, c1, D1, Ds1, H1, W1, wb + Ls[3].w_off, w + Ls[3].b_off, a.cat1, c2 + c1, c2, c1, true, true, s);
    hipLaunchKernelGGL(pool_kernel, dim3(gsz8(P1 / 8 * c1)), dim3(256), 0, s, a.cat1, c2 + c1, c2, c1, D1, H1, W1, a.p1);
    conv(a.p1, c1, 0, c1, D2, Ds2, H2, W2, wb + Ls[4].w_off, w + Ls[4].b_off, a.a2, c2, 0, c2, true, true, s);
    conv(a.a2, c2, 0, c2, D2, Ds2, H2, W2, wb + Ls[5].w_off, w + Ls[5].b_off, a.a3, c2, 0, c2, true, true, s);
    hipLaunchKernelGGL(up_kernel, dim3(gsz8(P1 * c2)), dim3(256), 0, s, a.a3, c2, D2, H2, W2, a.cat1, c2 + c1, 0);
    conv(a.cat1, c2 + c1, 0, c2 + c1, D1, Ds1, H1, W1, wb + Ls[6].w_off, w + Ls[6].b_off, a.a4, c1, 0, c1, true, true, s);
    conv(a.a4, c1, 0, c1, D1, Ds1, H1, W1, wb + Ls[7].w_off, w + Ls[7].b_off, a.a5, c1, 0, c1, true, true, s);
    hipLaunchKernelGGL(up_kernel, dim3(gsz8(P0 * c1)), dim3(256), 0, s, a.a5, c1, D1, H1, W1, a.cat0, c1 + c0, 0);
    conv(a.cat0, c1 + c0, 0, c1 + c0, D, Ds, H, W, wb + Ls[8].w_off, w + Ls[8].b_off, a.a6, c0, 0, c0, true, true, s);
    conv(a.a6, c0, 0, c0, D, Ds, H, W, wb + Ls[9].w_off, w + Ls[9].b_off, a.a7, c0, 0, c0, true, true, s);
    hipLaunchKernelGGL((conv_out_kernel<16>), dim3(gsz(P0)), dim3(256), 0, s, a.a7, P0,
                       w + Ls[10].w_off, w + Ls[10].b_off, out ? out : a.out);
    AIM_HIP(hipGetLastError());
  }

  // backward pass after forward(in) on the same batch; dout fp32 [P][2];
  // gradients (summed over the batch) are added to g
  void backward(const float* in, const float* dout, hipStream_t s) {
    Acts& a = acts;
    const int D = a.D, H = a.H, W = a.W, Ds = a.Ds, Ds1 = Ds / 2, Ds2 = Ds / 4;
    const int c0 = C, c1 = 2 * C, c2 = 4 * C;
    const int D1 = D / 2, H1 = H / 2, W1 = W / 2, D2 = D / 4, H2 = H / 4, W2 = W / 4;
    const int64_t P0 = int64_t(D) * H * W, P1 = P0 / 8, P2 = P1 / 8;
    const Layer* Ls = layers.data();
    // output layer
    wgrad<uint16_t, float>(a.a7, c0, 0, c0, dout, 2, 0, 2, D, Ds, H, W, Ls[10], s);
    hipLaunchKernelGGL((out_backward_kernel<16>), dim3(gsz(P0)), dim3(256), 0, s, dout,
                       w + Ls[10].w_off, a.a7, P0, a.gb0);
    // conv9
    wgrad<uint16_t, uint16_t>(a.a6, c0, 0, c0, a.gb0, c0, 0, c0, D, Ds, H, W, Ls[9], s);
    conv(a.gb0, c0, 0, c0, D, Ds, H, W, wf + Ls[9].flip_off, nullptr, a.g0, c0, 0, c0, false, false, s);
    hipLaunchKernelGGL(mask_kernel, dim3(gsz8(P0 * c0)), dim3(256), 0, s, a.g0, c0, 0, a.a6, c0, 0, c0, P0, a.gb0);
    // conv8 (input cat0 = [up(a5) | s0])
    wgrad<uint16_t, uint16_t>(a.cat0, c1 + c0, 0, c1 + c0, a.gb0, c0, 0, c0, D, Ds, H, W, Ls[8], s);
    conv(a.gb0, c0, 0, c0, D, Ds, H, W, wf + Ls[8].flip_off, nullptr, a.gcat0, c1 + c0, 0, c1 + c0, false, false, s);
    hipLaunchKernelGGL(up_backward_kernel, dim3(gsz8(P1 * c1)), dim3(256), 0, s, a.gcat0, c1 + c0, 0, c1, D1, H1, W1, a.a5, a.gb1);
    // conv7
    wgrad<uint16_t, uint16_t>(a.a4, c1, 0, c1, a.gb1, c1, 0, c1, D1, Ds1, H1, W1, Ls[7], s);
    conv(a.gb1, c1, 0, c1, D1, Ds1, H1, W1, wf + Ls[7].flip_off, nullptr, a.g1, c1, 0, c1, false, false, s);
    hipLaunchKernelGGL(mask_kernel, dim3(gsz8(P1 * c1)), dim3(256), 0, s, a.g1, c1, 0, a.a4, c1, 0, c1, P1, a.gb1);
    // conv6 (input cat1 = [up(a3) | s1])
    wgrad<uint16_t, uint16_t>(a.cat1, c2 + c1, 0, c2 + c1, a.gb1, c1, 0, c1, D1, Ds1, H1, W1, Ls[6], s);
    conv(a.gb1, c1, 0, c1, D1, Ds1, H1, W1, wf + Ls[6].flip_off, nullptr, a.gcat1, c2 + c1, 0, c2 + c1, false, false, s);
    hipLaunchKernelGGL(up_backward_kernel, dim3(gsz8(P2 * c2)), dim3(256), 0, s, a.gcat1, c2 + c1, 0, c2, D2, H2, W2, a.a3, a.gb2);
    // conv5
    wgrad<uint16_t, uint16_t>(a.a2, c2, 0, c2, a.gb2, c2, 0, c2, D2, Ds2, H2, W2, Ls[5], s);
    conv(a.gb2, c2, 0, c2, D2, Ds2, H2, W2, wf + Ls[5].flip_off, nullptr, a.g2, c2, 0, c2, false, false, s);
    hipLaunchKernelGGL(mask_kernel, dim3(gsz8(P2 * c2)), dim3(256), 0, s, a.g2, c2, 0, a.a2, c2, 0, c2, P2, a.gb2);
    // conv4 (input p1)
    wgrad<uint16_t, uint16_t>(a.p1, c1, 0, c1, a.gb2, c2, 0, c2, D2, Ds2, H2, W2, Ls[4], s);
    conv(a.gb2, c2, 0, c2, D2, Ds2, H2, W2, wf + Ls[4].flip_off, nullptr, a.g2, c1, 0, c1, false, false, s);
    hipLaunchKernelGGL(pool_backward_kernel, dim3(gsz8(P1 * c1)), dim3(256), 0, s, a.g2, c1, D1, H1, W1,
                       a.gcat1, c2 + c1, c2, a.cat1, c2 + c1, c2, a.gb1);
    // conv3
    wgrad<uint16_t, uint16_t>(a.a1, c1, 0, c1, a.gb1, c1, 0, c1, D1, Ds1, H1, W1, Ls[3], s);
    conv(a.gb1, c1, 0, c1, D1, Ds1, H1, W1, wf + Ls[3].flip_off, nullptr, a.g1, c1, 0, c1, false, false, s);
    hipLaunchKernelGGL(mask_kernel, dim3(gsz8(P1 * c1)), dim3(256), 0, s, a.g1, c1, 0, a.a1, c1, 0, c1, P1, a.gb1);
    // conv2 (input p0)
    wgrad<uint16_t, uint16_t>(a.p0, c0, 0, c0, a.gb1, c1, 0, c1, D1, Ds1, H1, W1, Ls[2], s);
    conv(a.gb1, c1, 0, c1, D1, Ds1, H1, W1, wf + Ls[2].flip_off, nullptr, a.g1, c0, 0, c0, false, false, s);
    hipLaunchKernelGGL(pool_backward_kernel, dim3(gsz8(P0 * c0)), dim3(256), 0, s, a.g1, c0, D, H, W,
                       a.gcat0, c1 + c0, c1, a.cat0, c1 + c0, c1, a.gb0);
    // conv1
    wgrad<uint16_t, uint16_t>(a.a0, c0, 0, c0, a.gb0, c0, 0, c0, D, Ds, H, W, Ls[1], s);
    conv(a.gb0, c0, 0, c0, D, Ds, H, W, wf + Ls[1].flip_off, nullptr, a.g0, c0, 0, c0, false, false, s);
    hipLaunchKernelGGL(mask_kernel, dim3(gsz8(P0 * c0)), dim3(256), 0, s, a.g0, c0, 0, a.a0, c0, 0, c0, P0, a.gb0);
    // conv0 (fp32 input, 2 channels)
    wgrad<float, uint16_t>(in, 2, 0, 2, a.gb0, c0, 0, c0, D, Ds, H, W, Ls[0], s);
    AIM_HIP(hipGetLastError());
  }

  void zero_grad(hipStream_t s) {
    hipLaunchKernelGGL(fill_kernel, dim3(gsz(nparam)), dim3(256), 0, s, g, nparam, 0.f);
    AIM_HIP(hipGetLastError());
  }

  void adam(double lr, hipStream_t s) {
    ++step;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, float(step)), c2 = 1.f - std::pow(b2, float(step));
    hipLaunchKernelGGL(adam_kernel, dim3(gsz(nparam)), dim3(256), 0, s, w, g, m, v, nparam,
                       float(lr), b1, b2, 1e-8f, c1, c2);
    AIM_HIP(hipGetLastError());
    refresh(s);
  }
};

namespace aim {
// used by the solver integration in abi.cpp
void unet_forward(aim_unet u, const void* in, int nb, int D, int H, int W, void* out,
                  hipStream_t s) {
  u->forward(static_cast<const float*>(in), nb, D, H, W, static_cast<float*>(out), s);
}
void unet_backward(aim_unet u, const void* in, const void* dout, hipStream_t s) {
  u->backward(static_cast<const float*>(in), static_cast<const float*>(dout), s);
}
void unet_zero_grad(aim_unet u, hipStream_t s) { u->zero_grad(s); }
void unet_adam(aim_unet u, double lr, hipStream_t s) { u->adam(lr, s); }
}  // namespace aim

// ===========================================================================
// C ABI
// ===========================================================================
namespace {
aim_status ufail(aim_status s, const std::string& m);
template <typename F>
aim_status uguard(F&& f) {
  try {
    f();
    return AIM_OK;
  } catch (const aim::Error& e) {
    return ufail(e.status, e.what());
  } catch (const std::bad_alloc&) {
    return ufail(AIM_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return ufail(AIM_ERR_DEVICE, e.what());
  }
}
}  // namespace

// error text shared with the rest of the library
namespace aim {
void set_last_error(const std::string& m);
}
namespace {
aim_status ufail(aim_status s, const std::string& m) {
  aim::set_last_error(m);
  return s;
}
}  // namespace

extern "C" {

aim_status aim_unet_create(int32_t base_channels, uint64_t seed, aim_unet* out) {
  if (!out) return ufail(AIM_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (base_channels != 16) return ufail(AIM_ERR_INVALID_ARG, "base_channels must be 16");
  std::unique_ptr<aim_unet_s> u(new aim_unet_s());
  const aim_status st = uguard([&] {
    u->C = base_channels;
    u->build_layers();
    u->alloc_params();
    // He-normal weights (the 1x1 output layer: variance 1/fan_in), zero biases
    std::vector<float> h(u->nparam, 0.f);
    std::mt19937_64 rng(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    for (size_t li = 0; li < u->layers.size(); ++li) {
      const auto& L = u->layers[li];
      const int64_t n = int64_t(L.cout) * L.taps * L.cin;
      const double fan = double(L.cin) * L.taps;
      const double std = li + 1 == u->layers.size() ? std::sqrt(1.0 / fan) : std::sqrt(2.0 / fan);
      for (int64_t i = 0; i < n; ++i) h[L.w_off + i] = float(nd(rng) * std);
    }
    AIM_HIP(hipMemcpy(u->w, h.data(), u->nparam * 4, hipMemcpyHostToDevice));
    u->refresh(nullptr);
    AIM_HIP(hipDeviceSynchronize());
  });
  if (st != AIM_OK) return st;
  *out = u.release();
  return AIM_OK;
}

aim_status aim_unet_destroy(aim_unet u) {
  return uguard([&] { delete u; });
}

aim_status aim_unet_num_params(aim_unet u, int64_t* n) {
  if (!u || !n) return ufail(AIM_ERR_INVALID_ARG, "null argument");
  *n = u->nparam;
  return AIM_OK;
}

aim_status aim_unet_get_params(aim_unet u, float* host, float* grad_host) {
  if (!u) return ufail(AIM_ERR_INVALID_ARG, "null argument");
  return uguard([&] {
    AIM_HIP(hipDeviceSynchronize());
    if (host) AIM_HIP(hipMemcpy(host, u->w, u->nparam * 4, hipMemcpyDeviceToHost));
    if (grad_host) AIM_HIP(hipMemcpy(grad_host, u->g, u->nparam * 4, hipMemcpyDeviceToHost));
  });
}

aim_status aim_unet_set_params(aim_unet u, const float* host) {
  if (!u || !host) return ufail(AIM_ERR_INVALID_ARG, "null argument");
  return uguard([&] {
    for (int64_t i = 0; i < u->nparam; ++i)
      AIM_REQUIRE(std::isfinite(host[i]), AIM_ERR_INVALID_ARG, "non-finite parameter");
    AIM_HIP(hipMemcpy(u->w, host, u->nparam * 4, hipMemcpyHostToDevice));
    u->refresh(nullptr);
    AIM_HIP(hipDeviceSynchronize());
  });
}

aim_status aim_unet_forward(aim_unet u, const void* in_dev, void* out_dev, int32_t nbatch,
                            const int32_t dims[3], void* hip_stream) {
  if (!u || !in_dev || !out_dev || !dims) return ufail(AIM_ERR_INVALID_ARG, "null argument");
  return uguard([&] {
    AIM_REQUIRE(nbatch >= 1, AIM_ERR_INVALID_ARG, "nbatch must be >= 1");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    u->forward(static_cast<const float*>(in_dev), nbatch, dims[2], dims[1], dims[0],
               static_cast<float*>(out_dev), s);
  });
}

aim_status aim_unet_train_grid(aim_unet u, const void* in_dev, const void* target_dev,
                               int32_t nbatch, const int32_t dims[3], double lr, int32_t apply,
                               double* loss_host, void* hip_stream) {
  if (!u || !in_dev || !target_dev || !dims) return ufail(AIM_ERR_INVALID_ARG, "null argument");
  return uguard([&] {
    AIM_REQUIRE(nbatch >= 1, AIM_ERR_INVALID_ARG, "nbatch must be >= 1");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int64_t P = int64_t(dims[0]) * dims[1] * dims[2];
    u->zero_grad(s);
    constexpr int kParts = 256;
    float* dout = nullptr;
    float* part = nullptr;
    AIM_HIP(hipMalloc(&dout, 2 * P * nbatch * 4));
    hipError_t e = hipMalloc(&part, size_t(kParts) * 4);
    if (e != hipSuccess) {
      (void)hipFree(dout);
      AIM_HIP(e);
    }
    std::vector<float> hp(kParts);
    try {
      // the whole batch in one pass, samples stacked along z
      const float* in = static_cast<const float*>(in_dev);
      const float* tg = static_cast<const float*>(target_dev);
      u->forward(in, nbatch, dims[2], dims[1], dims[0], nullptr, s);
      // mean squared error over all entries of the batch
      const float inv = 1.f / (float(2 * P) * float(nbatch));
      hipLaunchKernelGGL(mse_kernel, dim3(kParts), dim3(256), 0, s, u->acts.out, tg,
                         2 * P * nbatch, 2.f * inv, inv, dout, part);
      AIM_HIP(hipGetLastError());
      u->backward(in, dout, s);
      if (apply) u->adam(lr, s);
      AIM_HIP(hipMemcpyAsync(hp.data(), part, hp.size() * 4, hipMemcpyDeviceToHost, s));
      AIM_HIP(hipStreamSynchronize(s));
    } catch (...) {
      (void)hipFree(dout);
      (void)hipFree(part);
      throw;
    }
    (void)hipFree(dout);
    (void)hipFree(part);
    double loss = 0.0;
    for (float v : hp) loss += v;
    if (loss_host) *loss_host = loss;
  });
}

aim_status aim_unet_save(aim_unet u, const char* path) {
  if (!u || !path) return ufail(AIM_ERR_INVALID_ARG, "null argument");
  return uguard([&] {
    std::vector<float> h(u->nparam);
    AIM_HIP(hipDeviceSynchronize());
    AIM_HIP(hipMemcpy(h.data(), u->w, u->nparam * 4, hipMemcpyDeviceToHost));
    FILE* f = std::fopen(path, "wb");
    AIM_REQUIRE(f != nullptr, AIM_ERR_INVALID_ARG, std::string("cannot open ") + path);
    const char magic[8] = {'A', 'I', 'M', 'U', 'N', 'E', 'T', '1'};
    const int64_t hdr[2] = {u->C, u->nparam};
    bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(hdr, 8, 2, f) == 2 &&
              std::fwrite(h.data(), 4, h.size(), f) == h.size();
    ok = (std::fclose(f) == 0) && ok;
    AIM_REQUIRE(ok, AIM_ERR_INVALID_ARG, "write failed");
  });
}

aim_status aim_unet_load(const char* path, aim_unet* out) {
  if (!path || !out) return ufail(AIM_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  FILE* f = std::fopen(path, "rb");
  if (!f) return ufail(AIM_ERR_INVALID_ARG, std::string("cannot open ") + path);
  char magic[8];
  int64_t hdr[2];
  const bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "AIMUNET1", 8) == 0 &&
                  std::fread(hdr, 8, 2, f) == 2;
  if (!ok || hdr[0] != 16) {
    std::fclose(f);
    return ufail(AIM_ERR_INVALID_ARG, "not a U-Net weight file");
  }
  aim_unet u = nullptr;
  aim_status st = aim_unet_create(int32_t(hdr[0]), 0, &u);
  if (st != AIM_OK) {
    std::fclose(f);
    return st;
  }
  std::vector<float> h(u->nparam);
  const bool ok2 = hdr[1] == u->nparam && std::fread(h.data(), 4, h.size(), f) == h.size();
  std::fclose(f);
  if (!ok2) {
    aim_unet_destroy(u);
    return ufail(AIM_ERR_INVALID_ARG, "weight file size mismatch");
  }
  st = aim_unet_set_params(u, h.data());
  if (st != AIM_OK) {
    aim_unet_destroy(u);
    return st;
  }
  *out = u;
  return AIM_OK;
}

}  // extern "C"
