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
// triangles and its near-list row; every output is written once, so the
// result does not depend on the launch shape.
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
// charge channel), plus its near-list row of C_A - k^-2 C_phi
__global__ __launch_bounds__(256) void efie_test_kernel(
    const double2* __restrict__ psi, const double* __restrict__ vals,
    const int32_t* __restrict__ rwg_te, const int32_t* __restrict__ rowptr,
    const int32_t* __restrict__ col, const double* __restrict__ ca,
    const double* __restrict__ cphi, const double* __restrict__ kv,
    const int32_t* __restrict__ rhs_freq, const double2* __restrict__ x, double2* __restrict__ y,
    int64_t N, int64_t nrwg, int nrhs) {
  const int r = blockIdx.y;
  const int64_t P = 3 * N;
  const double k = kv[rhs_freq[r]];
  const double ik2 = 1.0 / (k * k);
  const double2* pa = psi + int64_t(r) * P;  // channel c at pa + c nrhs P
  const int64_t cs = int64_t(nrhs) * P;
  const double2* xr = x + int64_t(r) * nrwg;
  for (int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; n < nrwg;
       n += int64_t(gridDim.x) * blockDim.x) {
    double ar = 0.0, ai = 0.0, qr = 0.0, qi = 0.0;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int64_t t = rwg_te[4 * n + 2 * side];
      const int e = rwg_te[4 * n + 2 * side + 1];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const double* v = vals + 36 * t + 12 * q + 4 * e;
        const int64_t p = 3 * t + q;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double2 ph = pa[c * cs + p];
          ar += v[c] * ph.x;
          ai += v[c] * ph.y;
        }
        const double2 ph = pa[3 * cs + p];
        qr += v[3] * ph.x;
        qi += v[3] * ph.y;
      }
    }
    for (int32_t j = rowptr[n]; j < rowptr[n + 1]; ++j) {
      const double2 xv = xr[col[j]];
      ar += ca[j] * xv.x;
      ai += ca[j] * xv.y;
      qr += cphi[j] * xv.x;
      qi += cphi[j] * xv.y;
    }
    y[int64_t(r) * nrwg + n] = make_double2(ar - ik2 * qr, ai - ik2 * qi);
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
                      const int32_t* rowptr, const int32_t* col, const double* ca,
                      const double* cphi, const double* kv, const int32_t* rhs_freq,
                      const void* x, void* y, int64_t N, int64_t nrwg, int nrhs, hipStream_t s) {
  if (nrwg == 0) return;
  hipLaunchKernelGGL(efie_test_kernel, dim3(blocks(nrwg), nrhs), dim3(256), 0, s,
                     static_cast<const double2*>(psi), vals, rwg_te, rowptr, col, ca, cphi, kv,
                     rhs_freq, static_cast<const double2*>(x), static_cast<double2*>(y), N, nrwg,
                     nrhs);
  AIM_HIP(hipGetLastError());
}

}  // namespace aim
