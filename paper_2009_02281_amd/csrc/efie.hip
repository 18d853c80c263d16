// Device kernels of the RWG EFIE under AIMx (Sec. II-A, eq. EFIEdis; Sec.
// II-B, eq. LAIMx), complex128.  One product y = Z x runs
//
//   efie_sources -> projection of 4 nrhs point-source vectors (the current
//   channels x, y, z and the charge channel) -> convolution of the 4 nrhs
//   grids with the spectrum H(k) of each vector's wavenumber -> interpolation
//   back to the points -> efie_test,
//
// with the projection, convolution and interpolation kernels of the scalar
// operator (the point stencils in place of the merged triangle stencils).
// Both kernels here are gathers over small fixed fan-ins: a point reads the
// three functions of its triangle, a function the six points of its two
// triangles and its near-list row; every output is written once, with a
// fixed summation order.
#include <hip/hip_runtime.h>

#include "aim_internal.h"

namespace aim {
namespace {

unsigned blocks(int64_t cnt, int per = 256) {
  int64_t g = (cnt + per - 1) / per;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return unsigned(g);
}

// src[c][r][p] for the point p = 3t + q: sum over the triangle's three edges
// of the function's channel value at the point times its coefficient
__global__ __launch_bounds__(256) void efie_sources_kernel(
    const double2* __restrict__ x, const double* __restrict__ vals,
    const int32_t* __restrict__ tri_rwg, double2* __restrict__ src, int64_t N, int64_t nrwg,
    int nrhs) {
  const int r = blockIdx.y;
  const int64_t P = 3 * N;
  for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < P;
       p += int64_t(gridDim.x) * blockDim.x) {
    const int64_t t = p / 3;
    const double* v = vals + 36 * t + 12 * (p - 3 * t);
    double2 acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = make_double2(0.0, 0.0);
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const int32_t n = tri_rwg[3 * t + e];
      if (n < 0) continue;
      const double2 xv = x[int64_t(r) * nrwg + n];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double w = v[4 * e + c];
        acc[c].x += w * xv.x;
        acc[c].y += w * xv.y;
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) src[(int64_t(c) * nrhs + r) * P + p] = acc[c];
  }
}

// y[r][n]: the function's channel values at the six points of its triangles
// against the interpolated potentials (current channels minus k^-2 times the
// charge channel), plus its near-list row of C_A - k^-2 C_phi.  LPR lanes
// per function: lanes 0..5 take one point each (T+ then T-, three points
// each), every lane strides over the near row; a fixed butterfly across the
// LPR lanes sums them.  RB right-hand sides per workgroup, so each near entry
// and channel value is loaded once for all of them.
template <int LPR, int RB>
__global__ __launch_bounds__(256) void efie_test_kernel(
    const double2* __restrict__ psi, const double* __restrict__ vals,
    const int32_t* __restrict__ rwg_te, const int32_t* __restrict__ rowptr,
    const int32_t* __restrict__ col, const double2* __restrict__ cc,
    const double* __restrict__ kv, const int32_t* __restrict__ rhs_freq,
    const double2* __restrict__ x, double2* __restrict__ y, int64_t N, int64_t nrwg, int nrhs) {
  const int sub = threadIdx.x % LPR;
  const int64_t n = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / LPR;
  const int r0 = int(blockIdx.y) * RB;
  const int nr = min(RB, nrhs - r0);
  const int64_t P = 3 * N;
  const int64_t cs = int64_t(nrhs) * P;  // channel stride of psi
  double ar[RB], ai[RB], qr[RB], qi[RB];
#pragma unroll
  for (int j = 0; j < RB; ++j) ar[j] = ai[j] = qr[j] = qi[j] = 0.0;
  if (n < nrwg) {
    if (sub < 6) {
      const int side = sub >= 3 ? 1 : 0, q = sub - 3 * side;
      const int64_t t = rwg_te[4 * n + 2 * side];
      const int e = rwg_te[4 * n + 2 * side + 1];
      const double* v = vals + 36 * t + 12 * q + 4 * e;
      const double v0 = v[0], v1 = v[1], v2 = v[2], v3 = v[3];
      const double2* base = psi + int64_t(r0) * P + 3 * t + q;
#pragma unroll
      for (int j = 0; j < RB; ++j)
        if (j < nr) {
          const double2* b = base + int64_t(j) * P;
          const double2 p0 = b[0], p1 = b[cs], p2 = b[2 * cs], p3 = b[3 * cs];
          ar[j] = v0 * p0.x + v1 * p1.x + v2 * p2.x;
          ai[j] = v0 * p0.y + v1 * p1.y + v2 * p2.y;
          qr[j] = v3 * p3.x;
          qi[j] = v3 * p3.y;
        }
    }
    const double2* xr = x + int64_t(r0) * nrwg;
    for (int32_t k = rowptr[n] + sub; k < rowptr[n + 1]; k += LPR) {
      const double2 c = cc[k];
      const int64_t m = col[k];
#pragma unroll
      for (int j = 0; j < RB; ++j)
        if (j < nr) {
          const double2 xv = xr[int64_t(j) * nrwg + m];
          ar[j] += c.x * xv.x;
          ai[j] += c.x * xv.y;
          qr[j] += c.y * xv.x;
          qi[j] += c.y * xv.y;
        }
    }
  }
#pragma unroll
  for (int j = 0; j < RB; ++j)
#pragma unroll
    for (int o = LPR / 2; o > 0; o >>= 1) {
      ar[j] += __shfl_xor(ar[j], o, LPR);
      ai[j] += __shfl_xor(ai[j], o, LPR);
      qr[j] += __shfl_xor(qr[j], o, LPR);
      qi[j] += __shfl_xor(qi[j], o, LPR);
    }
  if (sub == 0 && n < nrwg) {
#pragma unroll
    for (int j = 0; j < RB; ++j)
      if (j < nr) {
        const double k = kv[rhs_freq[r0 + j]];
        const double ik2 = 1.0 / (k * k);
        y[int64_t(r0 + j) * nrwg + n] = make_double2(ar[j] - ik2 * qr[j], ai[j] - ik2 * qi[j]);
      }
  }
}

}  // namespace

void launch_efie_sources(const void* x, const double* vals, const int32_t* tri_rwg, void* src,
                         int64_t N, int64_t nrwg, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(efie_sources_kernel, dim3(blocks(3 * N), nrhs), dim3(256), 0, s,
                     static_cast<const double2*>(x), vals, tri_rwg, static_cast<double2*>(src),
                     N, nrwg, nrhs);
  AIM_HIP(hipGetLastError());
}

void launch_efie_test(const void* psi, const double* vals, const int32_t* rwg_te,
                      const int32_t* rowptr, const int32_t* col, const double* cc,
                      const double* kv, const int32_t* rhs_freq, const void* x, void* y,
                      int64_t N, int64_t nrwg, int nrhs, hipStream_t s) {
  if (nrwg == 0) return;
  constexpr int LPR = 16;
  const int64_t gx = (nrwg * LPR + 255) / 256;
  // several right-hand sides per workgroup while 1024 workgroups remain
  int rb = 1;
  while (rb < 8 && 2 * rb <= nrhs && gx * ((nrhs + 2 * rb - 1) / (2 * rb)) >= 1024) rb *= 2;
  const dim3 grid(unsigned(gx), unsigned((nrhs + rb - 1) / rb));
  const double2* ps = static_cast<const double2*>(psi);
  const double2* c2 = reinterpret_cast<const double2*>(cc);
  const double2* xi = static_cast<const double2*>(x);
  double2* yo = static_cast<double2*>(y);
#define AIM_EFIE_TEST(R)                                                                       \
  hipLaunchKernelGGL((efie_test_kernel<LPR, R>), grid, dim3(256), 0, s, ps, vals, rwg_te,     \
                     rowptr, col, c2, kv, rhs_freq, xi, yo, N, nrwg, nrhs)
  switch (rb) {
    case 1: AIM_EFIE_TEST(1); break;
    case 2: AIM_EFIE_TEST(2); break;
    case 4: AIM_EFIE_TEST(4); break;
    default: AIM_EFIE_TEST(8); break;
  }
#undef AIM_EFIE_TEST
  AIM_HIP(hipGetLastError());
}

}  // namespace aim
