// Device kernels of the RWG operators under AIMx, complex128 or complex64: the EFIE (Sec.
// II-A, eq. EFIEdis; Sec. II-B, eq. LAIMx) and the double layer (Sec. III-B,
// eq. KAIMx).  One EFIE product y = Z x runs
//
//   efie_sources -> projection of 4 nrhs point-source vectors (the current
//   channels x, y, z and the charge channel) -> convolution of the 4 nrhs
//   grids with the spectrum H(k) of each vector's wavenumber -> interpolation
//   back to the points -> efie_test,
//
// with the projection, convolution and interpolation kernels of the scalar
// operator (the point stencils in place of the merged triangle stencils).
// The double layer's product runs three current channels through the same
// projection and forward transforms, one z pass that forms the spectral
// cross product with the three components of grad G, the inverse transforms,
// interpolation of the field's three components and the test kernel; the
// combined field shares the EFIE's projection and forward transforms.
// Both kernels here are gathers over small fixed fan-ins: a point reads the
// three functions of its triangle, a function the six points of its two
// triangles and its near-list row; every output is written once, with a
// fixed summation order.
#include <hip/hip_runtime.h>

#include "aim_internal.h"

namespace aim {
namespace {

template <typename T>
struct C2T;
template <>
struct C2T<double> {
  using t = double2;
};
template <>
struct C2T<float> {
  using t = float2;
};
template <typename T>
using c2 = typename C2T<T>::t;
template <typename T>
__device__ __forceinline__ c2<T> mk2(T a, T b) {
  c2<T> r;
  r.x = a;
  r.y = b;
  return r;
}

unsigned blocks(int64_t cnt, int per = 256) {
  int64_t g = (cnt + per - 1) / per;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return unsigned(g);
}

// src[c][r][p] for the point p = 3t + q: sum over the triangle's three edges
// of the function's channel value at the point times its coefficient
template <int C, typename T>
__global__ __launch_bounds__(256) void efie_sources_kernel(
    const c2<T>* __restrict__ x, const T* __restrict__ vals,
    const int32_t* __restrict__ tri_rwg, c2<T>* __restrict__ src, int64_t N, int64_t nrwg,
    int nrhs) {
  const int r = blockIdx.y;
  const int64_t P = 3 * N;
  for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < P;
       p += int64_t(gridDim.x) * blockDim.x) {
    const int64_t t = p / 3;
    const T* v = vals + 36 * t + 12 * (p - 3 * t);
    c2<T> acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = mk2<T>(T(0), T(0));
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const int32_t n = tri_rwg[3 * t + e];
      if (n < 0) continue;
      const c2<T> xv = x[int64_t(r) * nrwg + n];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const T w = v[4 * e + c];
        acc[c].x += w * xv.x;
        acc[c].y += w * xv.y;
      }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) src[(int64_t(c) * nrhs + r) * P + p] = acc[c];
  }
}

// y[r][n] for the EFIE (E), the double layer (M) or their combination of
// eq. CFIEAIMx (both): over the six points of the function (T+ then T-,
// three points each) its channel values against the interpolated fields --
// EFIE: sum_c (w f_c) psi_c - k^-2 (w div f) psi_q; double layer:
// (w f x n) . V -- plus its near row: (C_A - k^-2 C_phi) x and
// (C_K + beta G) x.  Combined: y = y_E + (j/k) y_M.  LPR lanes per function:
// lanes 0..5 take one point each, every lane strides over the near row, a
// fixed butterfly sums them (fixed order: deterministic).  RB right-hand
// sides per workgroup, so each near entry and channel value is loaded once.
template <int LPR, int RB, bool E, bool M, typename T>
__global__ __launch_bounds__(256) void rwg_test_kernel(
    const c2<T>* __restrict__ psi_e, const c2<T>* __restrict__ psi_m,
    const T* __restrict__ vals, const T* __restrict__ nrm,
    const int32_t* __restrict__ rwg_te, const int32_t* __restrict__ rowptr,
    const int32_t* __restrict__ col, const c2<T>* __restrict__ cc,
    const c2<T>* __restrict__ ck, T beta, const double* __restrict__ kv,
    const int32_t* __restrict__ rhs_freq, const c2<T>* __restrict__ x, c2<T>* __restrict__ y,
    int64_t N, int64_t nrwg, int nrhs) {
  const int sub = threadIdx.x % LPR;
  const int64_t n = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / LPR;
  const int r0 = int(blockIdx.y) * RB;
  const int nr = min(RB, nrhs - r0);
  const int64_t P = 3 * N;
  const int64_t cs = int64_t(nrhs) * P;  // channel stride of psi_e and psi_m
  T ar[RB], ai[RB], qr[RB], qi[RB], mr[RB], mi[RB];
#pragma unroll
  for (int j = 0; j < RB; ++j) ar[j] = ai[j] = qr[j] = qi[j] = mr[j] = mi[j] = T(0);
  if (n < nrwg) {
    if (sub < 6) {
      const int side = sub >= 3 ? 1 : 0, q = sub - 3 * side;
      const int64_t t = rwg_te[4 * n + 2 * side];
      const int e = rwg_te[4 * n + 2 * side + 1];
      const T* v = vals + 36 * t + 12 * q + 4 * e;
      const T v0 = v[0], v1 = v[1], v2 = v[2], v3 = v[3];
      const int64_t off = int64_t(r0) * P + 3 * t + q;
      if constexpr (E) {
#pragma unroll
        for (int j = 0; j < RB; ++j)
          if (j < nr) {
            const c2<T>* b = psi_e + off + int64_t(j) * P;
            const c2<T> p0 = b[0], p1 = b[cs], p2 = b[2 * cs], p3 = b[3 * cs];
            ar[j] = v0 * p0.x + v1 * p1.x + v2 * p2.x;
            ai[j] = v0 * p0.y + v1 * p1.y + v2 * p2.y;
            qr[j] = v3 * p3.x;
            qi[j] = v3 * p3.y;
          }
      }
      if constexpr (M) {
        const T* nn = nrm + 3 * t;
        const T t0 = v1 * nn[2] - v2 * nn[1], t1 = v2 * nn[0] - v0 * nn[2],
                t2 = v0 * nn[1] - v1 * nn[0];
#pragma unroll
        for (int j = 0; j < RB; ++j)
          if (j < nr) {
            const c2<T>* b = psi_m + off + int64_t(j) * P;
            const c2<T> p0 = b[0], p1 = b[cs], p2 = b[2 * cs];
            mr[j] = t0 * p0.x + t1 * p1.x + t2 * p2.x;
            mi[j] = t0 * p0.y + t1 * p1.y + t2 * p2.y;
          }
      }
    }
    const c2<T>* xr = x + int64_t(r0) * nrwg;
    for (int32_t k = rowptr[n] + sub; k < rowptr[n + 1]; k += LPR) {
      const int64_t m = col[k];
      c2<T> c = mk2<T>(T(0), T(0));
      T w = T(0);
      if constexpr (E) c = cc[k];
      if constexpr (M) {
        const c2<T> d = ck[k];
        w = d.x + beta * d.y;
      }
#pragma unroll
      for (int j = 0; j < RB; ++j)
        if (j < nr) {
          const c2<T> xv = xr[int64_t(j) * nrwg + m];
          if constexpr (E) {
            ar[j] += c.x * xv.x;
            ai[j] += c.x * xv.y;
            qr[j] += c.y * xv.x;
            qi[j] += c.y * xv.y;
          }
          if constexpr (M) {
            mr[j] += w * xv.x;
            mi[j] += w * xv.y;
          }
        }
    }
  }
#pragma unroll
  for (int j = 0; j < RB; ++j)
#pragma unroll
    for (int o = LPR / 2; o > 0; o >>= 1) {
      if constexpr (E) {
        ar[j] += __shfl_xor(ar[j], o, LPR);
        ai[j] += __shfl_xor(ai[j], o, LPR);
        qr[j] += __shfl_xor(qr[j], o, LPR);
        qi[j] += __shfl_xor(qi[j], o, LPR);
      }
      if constexpr (M) {
        mr[j] += __shfl_xor(mr[j], o, LPR);
        mi[j] += __shfl_xor(mi[j], o, LPR);
      }
    }
  if (sub == 0 && n < nrwg) {
#pragma unroll
    for (int j = 0; j < RB; ++j)
      if (j < nr) {
        T yr = T(0), yi = T(0);
        if constexpr (E) {
          const double kd = kv[rhs_freq[r0 + j]];
          const T ik2 = T(1.0 / (kd * kd));
          yr = ar[j] - ik2 * qr[j];
          yi = ai[j] - ik2 * qi[j];
          if constexpr (M) {  // + (j/k)(mr + j mi) = (-mi + j mr)/k
            const T ik = T(1.0 / kd);
            yr -= ik * mi[j];
            yi += ik * mr[j];
          }
        } else {
          yr = mr[j];
          yi = mi[j];
        }
        y[int64_t(r0 + j) * nrwg + n] = mk2<T>(yr, yi);
      }
  }
}

// b[r][m]: the plane wave pol_r e^{-j k_r d_r . r} tested with function m by
// the 3-point rule over its two triangles: field 0 <f_m, E>, field 1
// <f_m, n x (d x E)>; prm [nrhs][6] = (d unit, pol)
__global__ __launch_bounds__(256) void rwg_plane_wave_kernel(
    const double* __restrict__ qp, const double* __restrict__ vals,
    const double* __restrict__ nrm, const int32_t* __restrict__ rwg_te,
    const double* __restrict__ prm, const double* __restrict__ kv,
    const int32_t* __restrict__ rhs_freq, int field, double2* __restrict__ b, int64_t nrwg) {
  const int r = blockIdx.y;
  const double* pr = prm + 6 * r;
  const double k = kv[rhs_freq[r]];
  for (int64_t m = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; m < nrwg;
       m += int64_t(gridDim.x) * blockDim.x) {
    double br = 0.0, bi = 0.0;
    for (int side = 0; side < 2; ++side) {
      const int64_t t = rwg_te[4 * m + 2 * side];
      const int e = rwg_te[4 * m + 2 * side + 1];
      double vx = pr[3], vy = pr[4], vz = pr[5];
      if (field == 1) {  // n x (d x pol)
        const double cx = pr[1] * pr[5] - pr[2] * pr[4], cy = pr[2] * pr[3] - pr[0] * pr[5],
                     cz = pr[0] * pr[4] - pr[1] * pr[3];
        const double* n = nrm + 3 * t;
        vx = n[1] * cz - n[2] * cy;
        vy = n[2] * cx - n[0] * cz;
        vz = n[0] * cy - n[1] * cx;
      }
      for (int q = 0; q < 3; ++q) {
        const double* x = qp + 3 * (3 * t + q);
        const double* v = vals + 36 * t + 12 * q + 4 * e;
        const double a = v[0] * vx + v[1] * vy + v[2] * vz;
        double sn, cs;
        sincos(k * (pr[0] * x[0] + pr[1] * x[1] + pr[2] * x[2]), &sn, &cs);
        br += a * cs;
        bi -= a * sn;
      }
    }
    b[int64_t(r) * nrwg + m] = make_double2(br, bi);
  }
}

}  // namespace

void launch_rwg_plane_wave(const double* qp, const double* vals, const double* nrm,
                           const int32_t* rwg_te, const double* prm, const double* kv,
                           const int32_t* rhs_freq, int field, void* b, int64_t nrwg, int nrhs,
                           hipStream_t s) {
  if (nrwg == 0) return;
  hipLaunchKernelGGL(rwg_plane_wave_kernel, dim3(blocks(nrwg), nrhs), dim3(256), 0, s, qp, vals,
                     nrm, rwg_te, prm, kv, rhs_freq, field, static_cast<double2*>(b), nrwg);
  AIM_HIP(hipGetLastError());
}

template <typename T>
void launch_mfie_sources(const void* x, const void* vals, const int32_t* tri_rwg, void* src,
                         int64_t N, int64_t nrwg, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL((efie_sources_kernel<3, T>), dim3(blocks(3 * N), nrhs), dim3(256), 0, s,
                     static_cast<const c2<T>*>(x), static_cast<const T*>(vals), tri_rwg,
                     static_cast<c2<T>*>(src), N, nrwg, nrhs);
  AIM_HIP(hipGetLastError());
}

template <typename T>
void launch_efie_sources(const void* x, const void* vals, const int32_t* tri_rwg, void* src,
                         int64_t N, int64_t nrwg, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL((efie_sources_kernel<4, T>), dim3(blocks(3 * N), nrhs), dim3(256), 0, s,
                     static_cast<const c2<T>*>(x), static_cast<const T*>(vals), tri_rwg,
                     static_cast<c2<T>*>(src), N, nrwg, nrhs);
  AIM_HIP(hipGetLastError());
}

template <typename T>
void launch_rwg_test(bool efie, bool mfie, const void* psi_e, const void* psi_m,
                     const void* vals, const void* nrm, const int32_t* rwg_te,
                     const int32_t* rowptr, const int32_t* col, const void* cc, const void* ck,
                     double beta, const double* kv, const int32_t* rhs_freq, const void* x,
                     void* y, int64_t N, int64_t nrwg, int nrhs, hipStream_t s) {
  if (nrwg == 0) return;
  AIM_REQUIRE(efie || mfie, AIM_ERR_INVALID_ARG, "no operator selected");
  constexpr int LPR = 16;
  const int64_t gx = (nrwg * LPR + 255) / 256;
  // several right-hand sides per workgroup while 1024 workgroups remain
  int rb = 1;
  while (rb < 8 && 2 * rb <= nrhs && gx * ((nrhs + 2 * rb - 1) / (2 * rb)) >= 1024) rb *= 2;
  const dim3 grid(unsigned(gx), unsigned((nrhs + rb - 1) / rb));
  const c2<T>* pe = static_cast<const c2<T>*>(psi_e);
  const c2<T>* pm = static_cast<const c2<T>*>(psi_m);
  const T* vl = static_cast<const T*>(vals);
  const T* nr = static_cast<const T*>(nrm);
  const c2<T>* cp = static_cast<const c2<T>*>(cc);
  const c2<T>* kp = static_cast<const c2<T>*>(ck);
  const c2<T>* xi = static_cast<const c2<T>*>(x);
  c2<T>* yo = static_cast<c2<T>*>(y);
  const T bt = T(beta);
#define AIM_RWG_TEST(R, E, M)                                                                  \
  hipLaunchKernelGGL((rwg_test_kernel<LPR, R, E, M, T>), grid, dim3(256), 0, s, pe, pm, vl,   \
                     nr, rwg_te, rowptr, col, cp, kp, bt, kv, rhs_freq, xi, yo, N, nrwg, nrhs)
#define AIM_RWG_RB(E, M)                      \
  switch (rb) {                               \
    case 1: AIM_RWG_TEST(1, E, M); break;     \
    case 2: AIM_RWG_TEST(2, E, M); break;     \
    case 4: AIM_RWG_TEST(4, E, M); break;     \
    default: AIM_RWG_TEST(8, E, M); break;    \
  }
  if (efie && mfie) AIM_RWG_RB(true, true)
  else if (efie) AIM_RWG_RB(true, false)
  else AIM_RWG_RB(false, true)
#undef AIM_RWG_RB
#undef AIM_RWG_TEST
  AIM_HIP(hipGetLastError());
}

#define AIM_RWG_INSTANTIATE(T)                                                                 \
  template void launch_mfie_sources<T>(const void*, const void*, const int32_t*, void*,       \
                                       int64_t, int64_t, int, hipStream_t);                   \
  template void launch_efie_sources<T>(const void*, const void*, const int32_t*, void*,       \
                                       int64_t, int64_t, int, hipStream_t);                   \
  template void launch_rwg_test<T>(bool, bool, const void*, const void*, const void*,         \
                                   const void*, const int32_t*, const int32_t*,               \
                                   const int32_t*, const void*, const void*, double,          \
                                   const double*, const int32_t*, const void*, void*,         \
                                   int64_t, int64_t, int, hipStream_t);
AIM_RWG_INSTANTIATE(double)
AIM_RWG_INSTANTIATE(float)
#undef AIM_RWG_INSTANTIATE

}  // namespace aim
