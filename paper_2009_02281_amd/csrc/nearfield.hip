// Near-field set-up on the device.
//
// AIMx (Sec. III-A): for every pair (i, j) of the near list, the static
// Galerkin entry A_s,NR[i, j] of the kernel 1/(4 pi R) (eq. hgfs) and the
// correction C = A_s,NR - A_s,P with the precorrection A_s,P = W H_s,NR P of
// eq. aimLPs (grid kernel 1/(4 pi R), self term 0 per eq. Hsmm).  These are
// the one-time static fill of the cost model of Sec. VI; they do not depend
// on the frequency.
//
// Conventional AIM (Sec. II-B, eqs. aimL, aimLFR, aimLP), for comparison:
// per wavenumber k the complex near correction A_NR(k) - A_P(k), where the
// near entries of the full kernel e^{-jkR}/(4 pi R) are the static entries
// above plus the smooth remainder G_d = (e^{-jkR} - 1)/(4 pi R) integrated by
// the 3 x 3 point rule, and A_P(k) = W H_NR(k) P uses the grid kernel
// G(k, R) with the same self term -jk/(4 pi) as the far-field H (eq. Hmm), so
// the self terms cancel.
//
// One thread per near pair.  The Galerkin entry uses the 3-point rule on the
// testing triangle and the closed-form integral of 1/R over the source
// triangle, written here as edge integrals plus the solid angle the triangle
// subtends (van Oosterom and Strackee, IEEE Trans. Biomed. Eng. 30(2), 1983):
//
//   int_T dS'/R = sum_i P0_i int_{edge i} dl/R  -  |h| Omega,
//
// which follows from div_s[(rho' - rho)/R] = 1/R + h^2/R^3 in the plane of T
// (h the height of r above it, P0_i the in-plane distance from the foot of
// r to edge i, positive on the inner side) and int_T |h|/R^3 dS' = Omega.
// The entry is symmetrised, (M_ij + M_ji)/2, so the matrix is exactly
// symmetric.  The precorrection is evaluated per quadrature-point pair as
// the separable correlation of the two stencils' 1-D Lagrange weights
// against the grid kernel.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "aim_internal.h"

namespace aim {
namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double kInvFourPi = 1.0 / (4.0 * kPi);

struct P3 {
  double x, y, z;
};
__device__ __forceinline__ P3 sub(P3 a, P3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ double dot(P3 a, P3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ P3 cross(P3 a, P3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ P3 scale(P3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ double len(P3 a) { return sqrt(dot(a, a)); }

// integral of dl / sqrt(l^2 + R0^2) from lm to lp (lm <= lp), with R = the
// distances of the endpoints, free of cancellation: the integrand is even in
// l, so a segment behind the foot is mirrored, and a segment across it uses
// (R + l)(R - l) = R0^2
__device__ double edge_integral(double lm, double lp, double Rm, double Rp, double R0sq) {
  if (lm >= 0.0) return log((Rp + lp) / (Rm + lm));
  if (lp <= 0.0) return log((Rm - lm) / (Rp - lp));
  return log((Rp + lp) * (Rm - lm) / R0sq);
}

// solid angle of triangle (A, B, C) seen from the origin, in [0, 2 pi)
__device__ double solid_angle(P3 A, P3 B, P3 C) {
  const double a = len(A), b = len(B), c = len(C);
  const double num = fabs(dot(A, cross(B, C)));
  const double den = a * b * c + dot(A, B) * c + dot(A, C) * b + dot(B, C) * a;
  return 2.0 * atan2(num, den);
}

// integral over triangle v[0..2] of 1 / |r - r'| dS'
__device__ double inv_r_integral(P3 r, const P3* v) {
  const P3 nn = cross(sub(v[1], v[0]), sub(v[2], v[0]));
  const double twice_area = len(nn);
  const P3 n = scale(nn, 1.0 / twice_area);
  const double h = dot(sub(r, v[0]), n);
  double acc = 0.0;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const P3 p = v[e], q = v[(e + 1) % 3];
    const P3 d = sub(q, p);
    const double L = len(d);
    const P3 u = scale(d, 1.0 / L);       // edge direction, counter-clockwise about n
    const P3 m = cross(u, n);             // outward in-plane normal of the edge
    const P3 pr = sub(p, r), qr = sub(q, r);
    const double P0 = dot(pr, m);
    if (fabs(P0) <= 1e-15 * L) continue;  // foot on the edge line: the term vanishes
    const double lm = dot(pr, u), lp = dot(qr, u);
    acc += P0 * edge_integral(lm, lp, len(pr), len(qr), P0 * P0 + h * h);
  }
  // finite for every r (0 at a vertex), so no guard: the term is 0 in the plane
  acc -= fabs(h) * solid_angle(sub(v[0], r), sub(v[1], r), sub(v[2], r));
  return acc;
}

// integral over triangle v[0..2] of |r - r'| dS': in the plane of T,
// div_s[(rho' - rho) R] = 3R - h^2/R gives (1/3)[sum_i P0_i int_{edge i} R dl
// + h^2 int_T dS'/R], with int R dl = [l R + R0^2 ln(l + R)]/2
__device__ double r_integral(P3 r, const P3* v) {
  const P3 nn = cross(sub(v[1], v[0]), sub(v[2], v[0]));
  const P3 n = scale(nn, 1.0 / len(nn));
  const double h = dot(sub(r, v[0]), n);
  double acc = 0.0;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const P3 p = v[e], q = v[(e + 1) % 3];
    const P3 d = sub(q, p);
    const double L = len(d);
    const P3 u = scale(d, 1.0 / L);
    const P3 m = cross(u, n);
    const P3 pr = sub(p, r), qr = sub(q, r);
    const double P0 = dot(pr, m);
    if (fabs(P0) <= 1e-15 * L) continue;
    const double lm = dot(pr, u), lp = dot(qr, u), Rm = len(pr), Rp = len(qr);
    const double R0sq = P0 * P0 + h * h;
    acc += P0 * 0.5 * (lp * Rp - lm * Rm + R0sq * edge_integral(lm, lp, Rm, Rp, R0sq));
  }
  if (h != 0.0) acc += h * h * inv_r_integral(r, v);
  return acc / 3.0;
}

// integral over triangle v[0..2] of r' / |r - r'| dS' (a vector), given
// s1 = the integral of 1/|r - r'|: with rho the foot of r in the plane,
// grad_s' R = (rho' - rho)/R, so the gradient theorem over T gives
// rho s1 + sum_i m_i int_{edge i} R dl (m_i the outward in-plane edge normal)
__device__ P3 rvec_r_integral(P3 r, const P3* v, double s1) {
  const P3 nn = cross(sub(v[1], v[0]), sub(v[2], v[0]));
  const P3 n = scale(nn, 1.0 / len(nn));
  const double h = dot(sub(r, v[0]), n);
  const P3 rho = sub(r, scale(n, h));
  P3 acc = scale(rho, s1);
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const P3 p = v[e], q = v[(e + 1) % 3];
    const P3 d = sub(q, p);
    const double L = len(d);
    const P3 u = scale(d, 1.0 / L);
    const P3 m = cross(u, n);
    const P3 pr = sub(p, r), qr = sub(q, r);
    const double P0 = dot(pr, m);
    const double lm = dot(pr, u), lp = dot(qr, u), Rm = len(pr), Rp = len(qr);
    const double R0sq = P0 * P0 + h * h;
    // on the edge's line R0^2 ln(...) vanishes
    const double lg = R0sq <= (1e-14 * L) * (1e-14 * L) ? 0.0 : edge_integral(lm, lp, Rm, Rp, R0sq);
    const double t = 0.5 * (lp * Rp - lm * Rm + R0sq * lg);
    acc = {acc.x + t * m.x, acc.y + t * m.y, acc.z + t * m.z};
  }
  return acc;
}

// integral over triangle v[0..2] of (r - r') / |r - r'|^3 dS' (a vector):
// the in-plane part is the gradient theorem for grad_s' (1/R) over T, the
// sum over the edges of the outward in-plane normal m_i times int dl/R; the
// normal part is n sign(h) times the solid angle T subtends at r, 0 for
// heights below hmin (in the plane: the principal value)
__device__ P3 grad_inv_r_integral(P3 r, const P3* v) {
  const P3 nn = cross(sub(v[1], v[0]), sub(v[2], v[0]));
  const double tw = len(nn);
  const P3 n = scale(nn, 1.0 / tw);
  const double h = dot(sub(r, v[0]), n);
  P3 acc = {0.0, 0.0, 0.0};
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const P3 p = v[e], q = v[(e + 1) % 3];
    const P3 d = sub(q, p);
    const P3 u = scale(d, 1.0 / len(d));
    const P3 m = cross(u, n);
    const P3 pr = sub(p, r), qr = sub(q, r);
    const double P0 = dot(pr, m);
    const double f = edge_integral(dot(pr, u), dot(qr, u), len(pr), len(qr), P0 * P0 + h * h);
    acc = {acc.x + f * m.x, acc.y + f * m.y, acc.z + f * m.z};
  }
  if (fabs(h) > 1e-14 * sqrt(tw)) {
    const double om = solid_angle(sub(v[0], r), sub(v[1], r), sub(v[2], r));
    const double sn = h > 0.0 ? om : -om;
    acc = {acc.x + sn * n.x, acc.y + sn * n.y, acc.z + sn * n.z};
  }
  return acc;
}

struct NearArgs {
  const double* tri;       // [N][3][3] corners
  const double* qp;        // [3N][3] quadrature points
  const double* qw;        // [3N] weights (area / 3)
  const int32_t* qstart;   // [3N][3] stencil start per axis
  const double* qlocal;    // [3N][3] local coordinate t - s per axis
  const int64_t* rowptr;   // [N+1] near list
  const int32_t* col;      // [nnz]
  int64_t N, nnz;
  double h;                // grid spacing
  double k;                // wavenumber (conventional AIM only)
};

__device__ int64_t row_of(const int64_t* rowptr, int64_t N, int64_t p) {
  int64_t lo = 0, hi = N;  // rowptr[lo] <= p < rowptr[hi]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) / 2;
    if (rowptr[mid] <= p) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <int ORDER>
__device__ __forceinline__ void lagrange(double u, double* w) {
#pragma unroll
  for (int a = 0; a <= ORDER; ++a) {
    double v = 1.0;
#pragma unroll
    for (int b = 0; b <= ORDER; ++b)
      if (b != a) v *= (u - double(b)) / double(a - b);
    w[a] = v;
  }
}

__device__ double galerkin_static(const NearArgs& a, int64_t i, int64_t j) {
  P3 v[3];
  for (int c = 0; c < 3; ++c)
    v[c] = {a.tri[9 * j + 3 * c], a.tri[9 * j + 3 * c + 1], a.tri[9 * j + 3 * c + 2]};
  double s = 0.0;
  for (int p = 0; p < 3; ++p) {
    const int64_t q = 3 * i + p;
    const P3 r = {a.qp[3 * q], a.qp[3 * q + 1], a.qp[3 * q + 2]};
    s += a.qw[q] * inv_r_integral(r, v);
  }
  return s * kInvFourPi;
}

// grid kernel at the integer offset (x, y, z): static 1/(4 pi R) with 0 at
// the origin (kind 0), e^{-jkR}/(4 pi R) with -jk/(4 pi) at the origin (kind
// 1), or the linear term G_lin = -R/(8 pi), 0 at the origin (kind 2)
template <int KIND>
struct GridKernel;
template <>
struct GridKernel<2> {
  using V = double;
  static __device__ V zero() { return 0.0; }
  static __device__ V at(int x, int y, int z, double h, double) {
    const int q = x * x + y * y + z * z;
    return -0.5 * kInvFourPi * h * sqrt(double(q));
  }
  static __device__ V fma(double w, V v, V acc) { return acc + w * v; }
};
template <>
struct GridKernel<0> {
  using V = double;
  static __device__ V zero() { return 0.0; }
  static __device__ V at(int x, int y, int z, double h, double) {
    const int q = x * x + y * y + z * z;
    return q == 0 ? 0.0 : kInvFourPi / (h * sqrt(double(q)));
  }
  static __device__ V fma(double w, V v, V acc) { return acc + w * v; }
};
template <>
struct GridKernel<1> {
  using V = double2;
  static __device__ V zero() { return make_double2(0.0, 0.0); }
  static __device__ V at(int x, int y, int z, double h, double k) {
    const int q = x * x + y * y + z * z;
    if (q == 0) return make_double2(0.0, -k * kInvFourPi);
    const double R = h * sqrt(double(q));
    double sn, cs;
    sincos(k * R, &sn, &cs);
    const double s = kInvFourPi / R;
    return make_double2(cs * s, -sn * s);
  }
  static __device__ V fma(double w, V v, V acc) {
    return make_double2(acc.x + w * v.x, acc.y + w * v.y);
  }
};

// the double layer's static gradient channels (Sec. III-B): component a is
// h d_a / (4 pi R^3), R = h |d|, 0 at the origin (kind 3)
struct Vec3d {
  double x, y, z;
};
template <>
struct GridKernel<3> {
  using V = Vec3d;
  static __device__ V zero() { return {0.0, 0.0, 0.0}; }
  static __device__ V at(int x, int y, int z, double h, double) {
    const int q = x * x + y * y + z * z;
    if (q == 0) return {0.0, 0.0, 0.0};
    const double R = h * sqrt(double(q));
    const double f = kInvFourPi * h / (R * R * R);
    return {f * x, f * y, f * z};
  }
  static __device__ V fma(double w, V v, V acc) {
    return {acc.x + w * v.x, acc.y + w * v.y, acc.z + w * v.z};
  }
};

// sum_{u, v} L_u(r_qa) H(u - v) L_v(r_qb) for the quadrature points qa, qb
template <int KIND, int ORDER>
__device__ typename GridKernel<KIND>::V point_pair(const NearArgs& a, int64_t qa, int64_t qb) {
  using GK = GridKernel<KIND>;
  constexpr int n = ORDER, S = n + 1, W = 2 * n + 1;
  // per axis: offset of the stencil starts and the correlation of the two
  // weight vectors, K[d + n] = sum_{alpha - beta = d} l_a l_b
  int d0[3];
  double K[3][W];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    double li[S], lj[S];
    lagrange<ORDER>(a.qlocal[3 * qa + ax], li);
    lagrange<ORDER>(a.qlocal[3 * qb + ax], lj);
    d0[ax] = a.qstart[3 * qa + ax] - a.qstart[3 * qb + ax];
#pragma unroll
    for (int d = 0; d < W; ++d) K[ax][d] = 0.0;
#pragma unroll
    for (int al = 0; al < S; ++al)
#pragma unroll
      for (int be = 0; be < S; ++be) K[ax][al - be + n] += li[al] * lj[be];
  }
  typename GK::V acc = GK::zero();
  for (int dz = 0; dz < W; ++dz)
    for (int dy = 0; dy < W; ++dy) {
      const double kyz = K[2][dz] * K[1][dy];
      typename GK::V row = GK::zero();
#pragma unroll
      for (int dx = 0; dx < W; ++dx)
        row = GK::fma(K[0][dx],
                      GK::at(d0[0] + dx - n, d0[1] + dy - n, d0[2] + dz - n, a.h, a.k), row);
      acc = GK::fma(kyz, row, acc);
    }
  return acc;
}

// sum over quadrature-point pairs of w_a w_b sum_{u, v} L_u(r_a) H(u - v) L_v(r_b)
template <int KIND, int ORDER>
__device__ typename GridKernel<KIND>::V precorrection(const NearArgs& a, int64_t i, int64_t j) {
  using GK = GridKernel<KIND>;
  typename GK::V pc = GK::zero();
  for (int p = 0; p < 3; ++p) {
    const int64_t qa = 3 * i + p;
    for (int q = 0; q < 3; ++q) {
      const int64_t qb = 3 * j + q;
      pc = GK::fma(a.qw[qa] * a.qw[qb], point_pair<KIND, ORDER>(a, qa, qb), pc);
    }
  }
  return pc;
}

// diagonal of the linear-term modification (Sec. III-A): per triangle,
// A_lin[i, i] - (W H_lin P)[i, i] with G_lin = -R/(8 pi) integrated directly
// (3-point outer rule, closed-form inner integral)
template <int ORDER>
__global__ __launch_bounds__(128) void lin_diag_kernel(NearArgs a, double* out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.N) return;
  P3 v[3];
  for (int c = 0; c < 3; ++c)
    v[c] = {a.tri[9 * i + 3 * c], a.tri[9 * i + 3 * c + 1], a.tri[9 * i + 3 * c + 2]};
  double s = 0.0;
  for (int p = 0; p < 3; ++p) {
    const int64_t q = 3 * i + p;
    const P3 r = {a.qp[3 * q], a.qp[3 * q + 1], a.qp[3 * q + 2]};
    s += a.qw[q] * r_integral(r, v);
  }
  out[i] = -0.5 * kInvFourPi * s - precorrection<2, ORDER>(a, i, i);
}

template <int ORDER>
__global__ __launch_bounds__(128) void near_static_kernel(NearArgs a, double* near_static,
                                                          double* corr) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= a.nnz) return;
  const int64_t i = row_of(a.rowptr, a.N, p), j = a.col[p];
  // (i, j) and (j, i) evaluate the same expression (pair in ascending order,
  // since the compiler may fuse a product into either sum), so the matrix
  // is symmetric to the bit
  const int64_t lo = i < j ? i : j, hi = i < j ? j : i;
  const double m = 0.5 * (galerkin_static(a, lo, hi) + galerkin_static(a, hi, lo));
  near_static[p] = m;
  corr[p] = m - precorrection<0, ORDER>(a, i, j);
}

// double-layer operator (Sec. III-B): K_s,NR[i, j] = sum_p w_ip (1/4 pi)
// int_{T_j} n_j.(r_ip - r') / R^3 dS' and C_K = K_s,NR - K_s,P.  The inner
// integral is h / |h| times the solid angle T_j subtends at r_ip (h its
// height above the plane of T_j along n_j; 0 in the plane, to rounding: the
// principal value of the self pairs); the precorrection dots the static gradient
// channels' grid product with n_j.
template <int ORDER>
__global__ __launch_bounds__(128) void dlp_near_kernel(NearArgs a, const double* nrm,
                                                       double* near_out, double* corr) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= a.nnz) return;
  const int64_t i = row_of(a.rowptr, a.N, p), j = a.col[p];
  P3 v[3];
  for (int c = 0; c < 3; ++c)
    v[c] = {a.tri[9 * j + 3 * c], a.tri[9 * j + 3 * c + 1], a.tri[9 * j + 3 * c + 2]};
  const P3 n = {nrm[3 * j], nrm[3 * j + 1], nrm[3 * j + 2]};
  // heights below 1e-14 of the triangle's size are rounding: the point is in
  // the plane (where the solid angle jumps by 4 pi)
  const double hmin = 1e-14 * sqrt(len(cross(sub(v[1], v[0]), sub(v[2], v[0]))));
  double s = 0.0;
  for (int q = 0; q < 3; ++q) {
    const int64_t qi = 3 * i + q;
    const P3 r = {a.qp[3 * qi], a.qp[3 * qi + 1], a.qp[3 * qi + 2]};
    const double h = dot(sub(r, v[0]), n);
    if (fabs(h) <= hmin) continue;
    const double om = solid_angle(sub(v[0], r), sub(v[1], r), sub(v[2], r));
    s += a.qw[qi] * (h > 0.0 ? om : -om);
  }
  s *= kInvFourPi;
  near_out[p] = s;
  const Vec3d pc = precorrection<3, ORDER>(a, i, j);
  corr[p] = s - (pc.x * n.x + pc.y * n.y + pc.z * n.z);
}

// RWG EFIE (Sec. II-A, II-B): for the pair (i, j) of the triangle pair
// list, the static inner integrals over T_j at the three points r_iq of
// T_i, int 1/R and int r'/R, and the nine point-pair precorrections
// sum_{u, v} L_u(r_iq) H_s(u - v) L_v(r_jq') (no quadrature weights); the
// host combines them into the functions' C_A and C_phi
template <int ORDER>
__global__ __launch_bounds__(128) void efie_pair_kernel(NearArgs a, double* out) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= a.nnz) return;
  const int64_t i = row_of(a.rowptr, a.N, p), j = a.col[p];
  P3 v[3];
  for (int c = 0; c < 3; ++c)
    v[c] = {a.tri[9 * j + 3 * c], a.tri[9 * j + 3 * c + 1], a.tri[9 * j + 3 * c + 2]};
  double* o = out + int64_t(kEfiePairVals) * p;
  for (int q = 0; q < 3; ++q) {
    const int64_t qi = 3 * i + q;
    const P3 r = {a.qp[3 * qi], a.qp[3 * qi + 1], a.qp[3 * qi + 2]};
    const double s1 = inv_r_integral(r, v);
    const P3 sv = rvec_r_integral(r, v, s1);
    o[q] = s1;
    o[3 + 3 * q] = sv.x;
    o[4 + 3 * q] = sv.y;
    o[5 + 3 * q] = sv.z;
  }
  for (int q = 0; q < 3; ++q)
    for (int q2 = 0; q2 < 3; ++q2)
      o[12 + 3 * q + q2] = point_pair<0, ORDER>(a, 3 * i + q, 3 * j + q2);
}

// RWG double layer (Sec. III-B): for the pair (i, j) of the triangle pair
// list, int_{T_j} (r - r')/R^3 dS' at the three points of T_i, then the
// point-pair sums sum_{u, v} L_u(r_iq) h (u - v) / (4 pi R^3) L_v(r_jq')
// (the static samples of -grad G, three components each)
template <int ORDER>
__global__ __launch_bounds__(128) void mfie_pair_kernel(NearArgs a, double* out) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= a.nnz) return;
  const int64_t i = row_of(a.rowptr, a.N, p), j = a.col[p];
  P3 v[3];
  for (int c = 0; c < 3; ++c)
    v[c] = {a.tri[9 * j + 3 * c], a.tri[9 * j + 3 * c + 1], a.tri[9 * j + 3 * c + 2]};
  double* o = out + int64_t(kMfiePairVals) * p;
  for (int q = 0; q < 3; ++q) {
    const int64_t qi = 3 * i + q;
    const P3 g = grad_inv_r_integral({a.qp[3 * qi], a.qp[3 * qi + 1], a.qp[3 * qi + 2]}, v);
    o[3 * q] = g.x;
    o[3 * q + 1] = g.y;
    o[3 * q + 2] = g.z;
  }
  for (int q = 0; q < 3; ++q)
    for (int q2 = 0; q2 < 3; ++q2) {
      const Vec3d w = point_pair<3, ORDER>(a, 3 * i + q, 3 * j + q2);
      double* d = o + 9 + 3 * (3 * q + q2);
      d[0] = w.x;
      d[1] = w.y;
      d[2] = w.z;
    }
}

// conventional AIM: A_NR(k) - A_P(k) from the static entries
template <int ORDER>
__global__ __launch_bounds__(128) void near_dynamic_kernel(NearArgs a, const double* near_static,
                                                           double2* out) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= a.nnz) return;
  const int64_t i = row_of(a.rowptr, a.N, p), j = a.col[p];
  // smooth remainder by the 3 x 3 point rule, G_d = (e^{-jkR} - 1)/(4 pi R)
  // written as (-2 sin^2(kR/2) - j sin(kR))/(4 pi R), -jk/(4 pi) at R = 0
  double dr = 0.0, di = 0.0;
  for (int s = 0; s < 3; ++s)
    for (int t = 0; t < 3; ++t) {
      const int64_t qa = 3 * i + s, qb = 3 * j + t;
      const P3 ra = {a.qp[3 * qa], a.qp[3 * qa + 1], a.qp[3 * qa + 2]};
      const P3 rb = {a.qp[3 * qb], a.qp[3 * qb + 1], a.qp[3 * qb + 2]};
      const double R = len(sub(ra, rb));
      const double w = a.qw[qa] * a.qw[qb];
      if (R == 0.0) {
        di -= w * a.k * kInvFourPi;
      } else {
        double sn, cs;
        sincos(0.5 * a.k * R, &sn, &cs);
        const double s2 = 2.0 * sn * cs;  // sin(kR)
        dr -= w * 2.0 * sn * sn * kInvFourPi / R;
        di -= w * s2 * kInvFourPi / R;
      }
    }
  const double2 pc = precorrection<1, ORDER>(a, i, j);
  out[p] = make_double2(near_static[p] + dr - pc.x, di - pc.y);
}

unsigned blocks_for(int64_t n) { return unsigned((n + 127) / 128); }

// Galerkin entry of the full kernel by the 3 x 3 point rule, split as the
// dense reference does: the smooth remainder G_d = G - G_s for every pair
// and, for pairs outside the near list, the static kernel too (pairs in the
// near list take their directly integrated static entry instead)
__device__ double2 pair_rule(const NearArgs& a, int64_t i, int64_t j, bool with_static) {
  double re = 0.0, im = 0.0;
  for (int s = 0; s < 3; ++s)
    for (int t = 0; t < 3; ++t) {
      const int64_t qa = 3 * i + s, qb = 3 * j + t;
      const P3 ra = {a.qp[3 * qa], a.qp[3 * qa + 1], a.qp[3 * qa + 2]};
      const P3 rb = {a.qp[3 * qb], a.qp[3 * qb + 1], a.qp[3 * qb + 2]};
      const double R = len(sub(ra, rb));
      const double w = a.qw[qa] * a.qw[qb];
      if (R == 0.0) {
        im -= w * a.k * kInvFourPi;
      } else {
        double sn, cs;
        sincos(0.5 * a.k * R, &sn, &cs);
        re -= w * 2.0 * sn * sn * kInvFourPi / R;
        im -= w * 2.0 * sn * cs * kInvFourPi / R;
        if (with_static) re += w * kInvFourPi / R;
      }
    }
  return make_double2(re, im);
}

// position of j in the sorted near-list row i, or -1
__device__ int64_t near_index(const NearArgs& a, int64_t i, int64_t j) {
  int64_t lo = a.rowptr[i], hi = a.rowptr[i + 1];
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    const int64_t c = a.col[mid];
    if (c == j) return mid;
    if (c < j) lo = mid + 1;
    else hi = mid;
  }
  return -1;
}

__device__ __forceinline__ double2 cmul2(double2 x, double2 y) {
  return make_double2(x.x * y.x - x.y * y.y, x.x * y.y + x.y * y.x);
}

// One workgroup per cluster: the block of the full-kernel Galerkin matrix
// over the cluster's triangles, then its inverse by Gauss-Jordan elimination
// with partial pivoting in LDS.  A zero pivot sets *singular.
constexpr int kMaxBlock = 64;
__global__ __launch_bounds__(256) void cluster_block_kernel(NearArgs a, const double* near_static,
                                                            const int32_t* cl_ptr,
                                                            const int32_t* perm,
                                                            const int64_t* cl_blk, double2* inv,
                                                            int* singular) {
  __shared__ double2 A[kMaxBlock * kMaxBlock];
  __shared__ double2 B[kMaxBlock * kMaxBlock];
  __shared__ double2 f[kMaxBlock];
  __shared__ double mag[kMaxBlock];
  __shared__ int arg[kMaxBlock];
  const int c = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  const int o = cl_ptr[c], m = cl_ptr[c + 1] - o;
  for (int e = tid; e < m * m; e += nt) {
    const int r = e / m, q = e - r * m;
    const int64_t i = perm[o + r], j = perm[o + q];
    const int64_t pn = near_index(a, i, j);
    double2 v = pair_rule(a, i, j, pn < 0);
    if (pn >= 0) v.x += near_static[pn];
    A[e] = v;
    B[e] = make_double2(r == q ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int kk = 0; kk < m; ++kk) {
    // pivot: the row at or below kk with the largest |A[r][kk]|
    if (tid < kMaxBlock) {
      const int r = kk + tid;
      mag[tid] = r < m ? A[r * m + kk].x * A[r * m + kk].x + A[r * m + kk].y * A[r * m + kk].y : -1.0;
      arg[tid] = r;
    }
    __syncthreads();
    for (int w = kMaxBlock / 2; w > 0; w >>= 1) {
      if (tid < w && (mag[tid + w] > mag[tid] ||
                      (mag[tid + w] == mag[tid] && arg[tid + w] < arg[tid]))) {
        mag[tid] = mag[tid + w];
        arg[tid] = arg[tid + w];
      }
      __syncthreads();
    }
    const int pr = arg[0];
    if (mag[0] <= 0.0) {
      if (tid == 0) *singular = 1;
      return;  // uniform: every thread reads the same mag[0]
    }
    if (pr != kk)
      for (int q = tid; q < m; q += nt) {
        const double2 t1 = A[kk * m + q], t2 = B[kk * m + q];
        A[kk * m + q] = A[pr * m + q];
        B[kk * m + q] = B[pr * m + q];
        A[pr * m + q] = t1;
        B[pr * m + q] = t2;
      }
    __syncthreads();
    // scale the pivot row by 1 / pivot (every thread reads the pivot before
    // any thread rewrites the row)
    const double2 pv = A[kk * m + kk];
    const double den = pv.x * pv.x + pv.y * pv.y;
    const double2 ip = make_double2(pv.x / den, -pv.y / den);
    __syncthreads();
    for (int q = tid; q < m; q += nt) {
      A[kk * m + q] = cmul2(A[kk * m + q], ip);
      B[kk * m + q] = cmul2(B[kk * m + q], ip);
    }
    __syncthreads();
    // eliminate column kk from every other row
    for (int r = tid; r < m; r += nt) f[r] = A[r * m + kk];
    __syncthreads();
    for (int e = tid; e < m * m; e += nt) {
      const int r = e / m, q = e - r * m;
      if (r == kk) continue;
      const double2 fr = f[r];
      const double2 ak = A[kk * m + q], bk = B[kk * m + q];
      A[e] = make_double2(A[e].x - (fr.x * ak.x - fr.y * ak.y), A[e].y - (fr.x * ak.y + fr.y * ak.x));
      B[e] = make_double2(B[e].x - (fr.x * bk.x - fr.y * bk.y), B[e].y - (fr.x * bk.y + fr.y * bk.x));
    }
    __syncthreads();
  }
  double2* out = inv + cl_blk[c];
  for (int e = tid; e < m * m; e += nt) out[e] = B[e];
}

}  // namespace

void* NearDevice::get(size_t bytes) {
  if (bytes == 0) bytes = 8;
  void* p = nullptr;
  if (alloc_) {
    p = alloc_(bytes, stream_, ctx_);
    AIM_REQUIRE(p != nullptr, AIM_ERR_OOM, "device allocator returned NULL");
  } else {
    const hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error(AIM_ERR_OOM, "near-field tables: device allocation failed");
    }
  }
  bufs_.push_back(p);
  return p;
}

template <typename T>
static void* put(void* dst, const std::vector<T>& v, hipStream_t s) {
  if (!v.empty())
    AIM_HIP(hipMemcpyAsync(dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return dst;
}

NearDevice::NearDevice(const HostTables& t, const double* V, const int32_t* T,
                       aim_alloc_fn alloc, aim_free_fn free_fn, void* ctx, hipStream_t s)
    : N_(t.N), nnz_(t.rowptr.empty() ? 0 : t.rowptr[t.N]), order_(t.order), h_(t.h),
      alloc_(alloc), free_(free_fn), ctx_(ctx), stream_(s) {
  try {
    if (V && T) {  // corners: only the static and double-layer fills need them
      std::vector<double> tri(9 * size_t(N_));
      for (int64_t j = 0; j < N_; ++j)
        for (int c = 0; c < 3; ++c)
          for (int ax = 0; ax < 3; ++ax)
            tri[9 * j + 3 * c + ax] = V[3 * int64_t(T[3 * j + c]) + ax];
      tri_ = put(get(tri.size() * 8), tri, s);
    } else if (t.corners.size() == 9 * size_t(N_)) {
      tri_ = put(get(t.corners.size() * 8), t.corners, s);
    }
    qp_ = put(get(t.qp_xyz.size() * 8), t.qp_xyz, s);
    qw_ = put(get(t.qp_w.size() * 8), t.qp_w, s);
    qstart_ = put(get(t.qp_start.size() * 4), t.qp_start, s);
    qlocal_ = put(get(t.qp_local.size() * 8), t.qp_local, s);
    rowptr_ = put(get(t.rowptr.size() * 8), t.rowptr, s);
    col_ = put(get(t.col.size() * 4), t.col, s);
    static_ = get(size_t(nnz_) * 8);
    AIM_HIP(hipStreamSynchronize(s));  // the host vectors above are temporaries
  } catch (...) {
    release();
    throw;
  }
}

void NearDevice::release() {
  (void)hipStreamSynchronize(stream_);
  for (void* p : bufs_) {
    if (alloc_)
      free_(p, stream_, ctx_);
    else
      (void)hipFree(p);
  }
  bufs_.clear();
}

NearDevice::~NearDevice() { release(); }

static NearArgs make_args(const void* tri, const void* qp, const void* qw, const void* qstart,
                          const void* qlocal, const void* rowptr, const void* col, int64_t N,
                          int64_t nnz, double h, double k) {
  NearArgs a{};
  a.tri = static_cast<const double*>(tri);
  a.qp = static_cast<const double*>(qp);
  a.qw = static_cast<const double*>(qw);
  a.qstart = static_cast<const int32_t*>(qstart);
  a.qlocal = static_cast<const double*>(qlocal);
  a.rowptr = static_cast<const int64_t*>(rowptr);
  a.col = static_cast<const int32_t*>(col);
  a.N = N;
  a.nnz = nnz;
  a.h = h;
  a.k = k;
  return a;
}

void NearDevice::fill_dlp(const std::vector<double>& nrm, std::vector<double>& near_out,
                          std::vector<double>& corr_out, hipStream_t s) {
  AIM_REQUIRE(tri_ != nullptr, AIM_ERR_STATE, "near-field tables built without the mesh");
  AIM_REQUIRE(nrm.size() == 3 * size_t(N_), AIM_ERR_INVALID_ARG, "one normal per triangle");
  const NearArgs a = make_args(tri_, qp_, qw_, qstart_, qlocal_, rowptr_, col_, N_, nnz_, h_,
                               0.0);
  near_out.assign(nnz_, 0.0);
  corr_out.assign(nnz_, 0.0);
  if (nnz_ == 0) return;
  void* buf = get(size_t(2 * nnz_ + 3 * N_) * 8);
  double* nd = static_cast<double*>(buf);
  double* cd = nd + nnz_;
  double* nr = cd + nnz_;
  AIM_HIP(hipMemcpyAsync(nr, nrm.data(), size_t(3 * N_) * 8, hipMemcpyHostToDevice, s));
  if (order_ == 2)
    hipLaunchKernelGGL(dlp_near_kernel<2>, dim3(blocks_for(nnz_)), dim3(128), 0, s, a, nr, nd,
                       cd);
  else
    hipLaunchKernelGGL(dlp_near_kernel<3>, dim3(blocks_for(nnz_)), dim3(128), 0, s, a, nr, nd,
                       cd);
  AIM_HIP(hipGetLastError());
  AIM_HIP(hipMemcpyAsync(near_out.data(), nd, size_t(nnz_) * 8, hipMemcpyDeviceToHost, s));
  AIM_HIP(hipMemcpyAsync(corr_out.data(), cd, size_t(nnz_) * 8, hipMemcpyDeviceToHost, s));
  AIM_HIP(hipStreamSynchronize(s));
}

void NearDevice::fill_rwg_pairs(int kind, const std::vector<int64_t>& rowptr,
                                const std::vector<int32_t>& col, std::vector<double>& out,
                                hipStream_t s) {
  AIM_REQUIRE(tri_ != nullptr, AIM_ERR_STATE, "near-field tables built without the mesh");
  AIM_REQUIRE(rowptr.size() == size_t(N_) + 1 && int64_t(col.size()) == rowptr[N_],
              AIM_ERR_INVALID_ARG, "pair list does not match the mesh");
  AIM_REQUIRE(kind == 0 || kind == 1, AIM_ERR_INVALID_ARG, "pair kind");
  const int per = kind == 0 ? kEfiePairVals : kMfiePairVals;
  const int64_t np = int64_t(col.size());
  out.assign(size_t(per) * np, 0.0);
  if (np == 0) return;
  void* rp = put(get(rowptr.size() * 8), rowptr, s);
  void* cp = put(get(col.size() * 4), col, s);
  double* od = static_cast<double*>(get(out.size() * 8));
  const NearArgs a = make_args(tri_, qp_, qw_, qstart_, qlocal_, rp, cp, N_, np, h_, 0.0);
  if (kind == 0) {
    if (order_ == 2)
      hipLaunchKernelGGL(efie_pair_kernel<2>, dim3(blocks_for(np)), dim3(128), 0, s, a, od);
    else
      hipLaunchKernelGGL(efie_pair_kernel<3>, dim3(blocks_for(np)), dim3(128), 0, s, a, od);
  } else {
    if (order_ == 2)
      hipLaunchKernelGGL(mfie_pair_kernel<2>, dim3(blocks_for(np)), dim3(128), 0, s, a, od);
    else
      hipLaunchKernelGGL(mfie_pair_kernel<3>, dim3(blocks_for(np)), dim3(128), 0, s, a, od);
  }
  AIM_HIP(hipGetLastError());
  AIM_HIP(hipMemcpyAsync(out.data(), od, out.size() * 8, hipMemcpyDeviceToHost, s));
  AIM_HIP(hipStreamSynchronize(s));
}

void NearDevice::fill_static(std::vector<double>& near_static, std::vector<double>& corr,
                             std::vector<double>& lin_diag, hipStream_t s) {
  AIM_REQUIRE(tri_ != nullptr, AIM_ERR_STATE, "near-field tables built without the mesh");
  const NearArgs a = make_args(tri_, qp_, qw_, qstart_, qlocal_, rowptr_, col_, N_, nnz_, h_,
                               0.0);
  void* cr = nullptr;
  {
    const hipError_t e = hipMalloc(&cr, size_t(nnz_ + N_) * 8);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error(AIM_ERR_OOM, "near-field set-up: device allocation failed");
    }
  }
  try {
    near_static.resize(nnz_);
    corr.resize(nnz_);
    lin_diag.resize(N_);
    double* ld = static_cast<double*>(cr) + nnz_;
    if (N_ > 0) {
      if (order_ == 2)
        hipLaunchKernelGGL(lin_diag_kernel<2>, dim3(blocks_for(N_)), dim3(128), 0, s, a, ld);
      else
        hipLaunchKernelGGL(lin_diag_kernel<3>, dim3(blocks_for(N_)), dim3(128), 0, s, a, ld);
      AIM_HIP(hipGetLastError());
      AIM_HIP(hipMemcpyAsync(lin_diag.data(), ld, size_t(N_) * 8, hipMemcpyDeviceToHost, s));
    }
    if (nnz_ > 0) {
      if (order_ == 2)
        hipLaunchKernelGGL(near_static_kernel<2>, dim3(blocks_for(nnz_)), dim3(128), 0, s, a,
                           static_cast<double*>(static_), static_cast<double*>(cr));
      else
        hipLaunchKernelGGL(near_static_kernel<3>, dim3(blocks_for(nnz_)), dim3(128), 0, s, a,
                           static_cast<double*>(static_), static_cast<double*>(cr));
      AIM_HIP(hipGetLastError());
      AIM_HIP(hipMemcpyAsync(near_static.data(), static_, size_t(nnz_) * 8,
                             hipMemcpyDeviceToHost, s));
      AIM_HIP(hipMemcpyAsync(corr.data(), cr, size_t(nnz_) * 8, hipMemcpyDeviceToHost, s));
    }
    AIM_HIP(hipStreamSynchronize(s));
  } catch (...) {
    (void)hipStreamSynchronize(s);
    if (cr) (void)hipFree(cr);
    throw;
  }
  if (cr) (void)hipFree(cr);
  have_static_ = true;
}

void NearDevice::set_static(const std::vector<double>& near_static, hipStream_t s) {
  AIM_REQUIRE(int64_t(near_static.size()) == nnz_, AIM_ERR_INVALID_ARG,
              "static near entries do not match the near list");
  put(static_, near_static, s);
  AIM_HIP(hipStreamSynchronize(s));
  have_static_ = true;
}

void NearDevice::fill_cluster_inverses(double k, const int32_t* cl_ptr, const int32_t* cl_perm,
                                       const int64_t* cl_blk, int ncl, int max_cluster,
                                       void* out_dev, hipStream_t s) {
  AIM_REQUIRE(have_static_, AIM_ERR_STATE, "static near field not on the device");
  AIM_REQUIRE(max_cluster <= kMaxBlock, AIM_ERR_INVALID_ARG, "cluster larger than 64 triangles");
  const NearArgs a = make_args(tri_, qp_, qw_, qstart_, qlocal_, rowptr_, col_, N_, nnz_, h_, k);
  int* flag = nullptr;
  AIM_HIP(hipMalloc(&flag, sizeof(int)));
  int h_flag = 0;
  try {
    AIM_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
    if (ncl > 0) {
      hipLaunchKernelGGL(cluster_block_kernel, dim3(unsigned(ncl)), dim3(256), 0, s, a,
                         static_cast<const double*>(static_), cl_ptr, cl_perm, cl_blk,
                         static_cast<double2*>(out_dev), flag);
      AIM_HIP(hipGetLastError());
    }
    AIM_HIP(hipMemcpyAsync(&h_flag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    AIM_HIP(hipStreamSynchronize(s));
  } catch (...) {
    (void)hipStreamSynchronize(s);
    (void)hipFree(flag);
    throw;
  }
  (void)hipFree(flag);
  AIM_REQUIRE(h_flag == 0, AIM_ERR_GEOMETRY, "singular near-field preconditioner block");
}

void NearDevice::fill_conventional(double k, void* out_dev, hipStream_t s) {
  AIM_REQUIRE(have_static_, AIM_ERR_STATE, "static near field not on the device");
  const NearArgs a = make_args(tri_, qp_, qw_, qstart_, qlocal_, rowptr_, col_, N_, nnz_, h_, k);
  if (nnz_ > 0) {
    if (order_ == 2)
      hipLaunchKernelGGL(near_dynamic_kernel<2>, dim3(blocks_for(nnz_)), dim3(128), 0, s, a,
                         static_cast<const double*>(static_), static_cast<double2*>(out_dev));
    else
      hipLaunchKernelGGL(near_dynamic_kernel<3>, dim3(blocks_for(nnz_)), dim3(128), 0, s, a,
                         static_cast<const double*>(static_), static_cast<double2*>(out_dev));
    AIM_HIP(hipGetLastError());
  }
}

}  // namespace aim
