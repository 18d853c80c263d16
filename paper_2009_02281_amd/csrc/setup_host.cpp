// Host-side set-up of the AIMx operator: everything that is independent of
// frequency and is computed once per geometry (the paper's one-time static
// fill, Sec. III-A and the cost model of Sec. VI).
//
//  * geometry: triangle areas, the 3-point quadrature rule (interior points
//    at barycentric (2/3,1/6,1/6) and permutations, weight area/3);
//  * grid: isotropic spacing, grid centred on the vertex bounding box;
//  * stencils: (n+1) points per direction starting at floor(t - (n-1)/2);
//  * near list: centroid distance below the threshold, by uniform cells;
//  * A_s,NR: Galerkin entries of the static kernel 1/(4 pi R) with the
//    closed-form inner integral over the source triangle and the 3-point outer
//    rule, symmetrised;
//  * A_s,P = W H_s,NR P on the near list (eq. aimLPs, H_s self term 0 per
//    eq. Hsmm), evaluated per quadrature-point pair through the separable
//    correlation of the two stencils' 1-D weights;
//  * the projection matrix P (merged over each triangle's three points) in
//    two sparse layouts, and near-block preconditioner clusters.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>

#include "aim_internal.h"

#pragma clang fp contract(off)

namespace aim {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kFourPi = 4.0 * kPi;

template <typename F>
void parallel_for(int64_t n, int nthreads, F&& fn) {
  if (nthreads <= 1 || n < 256) {
    fn(int64_t(0), n);
    return;
  }
  std::atomic<int64_t> next{0};
  const int64_t chunk = std::max<int64_t>(64, n / (int64_t(nthreads) * 16));
  std::vector<std::thread> pool;
  std::vector<std::exception_ptr> errs(nthreads);
  for (int t = 0; t < nthreads; ++t) {
    pool.emplace_back([&, t] {
      try {
        for (;;) {
          int64_t b = next.fetch_add(chunk);
          if (b >= n) break;
          fn(b, std::min(n, b + chunk));
        }
      } catch (...) {
        errs[t] = std::current_exception();
      }
    });
  }
  for (auto& th : pool) th.join();
  for (auto& e : errs)
    if (e) std::rethrow_exception(e);
}

inline void sub3(const double* a, const double* b, double* o) {
  o[0] = a[0] - b[0];
  o[1] = a[1] - b[1];
  o[2] = a[2] - b[2];
}
inline double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
inline void cross3(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
inline double norm3(const double* a) { return std::sqrt(dot3(a, a)); }

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Lagrange weights l_a(u) = prod_{b != a} (u - b)/(a - b), a = 0..order
inline void lagrange(double u, int order, double* out) {
  for (int a = 0; a <= order; ++a) {
    double w = 1.0;
    for (int b = 0; b <= order; ++b)
      if (b != a) w = w * (u - b) / double(a - b);
    out[a] = w;
  }
}

}  // namespace

void parallel_ranges(int64_t n, int nthreads, const std::function<void(int64_t, int64_t)>& fn) {
  parallel_for(n, nthreads, fn);
}

void lagrange_host(double u, int order, double* out) { lagrange(u, order, out); }

// Integral over the triangle (a, b, c) of 1/|r - r'| dS': the in-plane
// divergence identity div_s[(rho' - rho)/R] = 1/R + h^2/R^3 turns it into
// edge integrals, sum_i P0_i int_{edge i} dl/R, minus |h| times the solid
// angle the triangle subtends at r (van Oosterom and Strackee, 1983) -- the
// form the device fill uses.  The edge logarithm is written without
// cancellation on either side of the foot point.
double triangle_inv_r(const double r[3], const double a[3], const double b[3], const double c[3]) {
  const double* v[3] = {a, b, c};
  double e1[3], e2[3], nn[3];
  sub3(b, a, e1);
  sub3(c, a, e2);
  cross3(e1, e2, nn);
  const double tw = norm3(nn);
  const double n[3] = {nn[0] / tw, nn[1] / tw, nn[2] / tw};
  double ra[3];
  sub3(r, a, ra);
  const double h = dot3(ra, n);
  double acc = 0.0;
  for (int e = 0; e < 3; ++e) {
    const double* p = v[e];
    const double* q = v[(e + 1) % 3];
    double d[3];
    sub3(q, p, d);
    const double L = norm3(d);
    const double u[3] = {d[0] / L, d[1] / L, d[2] / L};  // counter-clockwise about n
    double m[3];
    cross3(u, n, m);  // outward in-plane normal of the edge
    double pr[3], qr[3];
    sub3(p, r, pr);
    sub3(q, r, qr);
    const double P0 = dot3(pr, m);
    if (std::fabs(P0) <= 1e-15 * L) continue;  // foot on the edge line: no term
    const double lm = dot3(pr, u), lp = dot3(qr, u);
    const double Rm = norm3(pr), Rp = norm3(qr), R0sq = P0 * P0 + h * h;
    double lg;
    if (lm >= 0.0)
      lg = std::log((Rp + lp) / (Rm + lm));
    else if (lp <= 0.0)
      lg = std::log((Rm - lm) / (Rp - lp));  // the segment mirrored through the foot
    else
      lg = std::log((Rp + lp) * (Rm - lm) / R0sq);  // (R + l)(R - l) = R0^2
    acc += P0 * lg;
  }
  double A[3], B[3], Cv[3], bc[3];
  sub3(a, r, A);
  sub3(b, r, B);
  sub3(c, r, Cv);
  cross3(B, Cv, bc);
  const double la = norm3(A), lb = norm3(B), lc = norm3(Cv);
  const double num = std::fabs(dot3(A, bc));
  const double den = la * lb * lc + dot3(A, B) * lc + dot3(A, Cv) * lb + dot3(B, Cv) * la;
  acc -= std::fabs(h) * 2.0 * std::atan2(num, den);
  return acc;
}

// Row blocks of a CSR matrix for the projection kernel: consecutive rows
// with at most kProjNnz non-zeros and kProjRows rows; a longer row forms a
// block of its own, and a run of at least kProjRows empty rows (nodes no
// stencil reaches) forms a zero block of up to kProjZeroRows rows.
std::vector<int32_t> row_blocks(const std::vector<int32_t>& rowptr) {
  const int64_t Ng = int64_t(rowptr.size()) - 1;
  std::vector<int32_t> blk(1, 0);
  int64_t r = 0;
  while (r < Ng) {
    int64_t e = r, nz = 0;
    while (e < Ng && e - r < kProjZeroRows && rowptr[e + 1] == rowptr[e]) ++e;
    if (e - r >= kProjRows || e == Ng) {
      blk.push_back(int32_t(e));
      r = e;
      continue;
    }
    e = r;
    while (e < Ng && e - r < kProjRows) {
      const int64_t len = rowptr[e + 1] - rowptr[e];
      if (e > r && nz + len > kProjNnz) break;
      nz += len;
      ++e;
      if (nz > kProjNnz) break;  // a single long row
    }
    blk.push_back(int32_t(e));
    r = e;
  }
  return blk;
}

// A_s,NR and C = A_s,NR - A_s,P on the near list (host).
void fill_near_host(HostTables& t, const double* V, const int32_t* T, int nthreads) {
  const auto t0 = std::chrono::steady_clock::now();
  const int64_t N = t.N;
  const int64_t nnz = t.rowptr[N];
  const double h = t.h;
  const int n = t.order, S = n + 1, W = 2 * n + 1;
  std::vector<double> lw(3 * N * 3 * S);  // [qp][axis][a]
  for (int64_t p = 0; p < 3 * N; ++p)
    for (int ax = 0; ax < 3; ++ax) lagrange(t.qp_local[3 * p + ax], n, &lw[(3 * p + ax) * S]);
  // -- static near field A_s,NR ----------------------------------------------
  auto Mij = [&](int64_t i, int64_t j) {  // sum_p (A_i/3) Phi_j(r_ip)
    const double* a = V + 3 * T[3 * j];
    const double* b = V + 3 * T[3 * j + 1];
    const double* c = V + 3 * T[3 * j + 2];
    double s = 0.0;
    for (int p = 0; p < 3; ++p)
      s += t.qp_w[3 * i + p] * (triangle_inv_r(&t.qp_xyz[3 * (3 * i + p)], a, b, c) / kFourPi);
    return s;
  };
  t.near_static.resize(nnz);
  parallel_for(N, nthreads, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i)
      for (int64_t p = t.rowptr[i]; p < t.rowptr[i + 1]; ++p) {
        const int64_t j = t.col[p];
        t.near_static[p] = 0.5 * (Mij(i, j) + Mij(j, i));
      }
  });

  // -- precorrection A_s,P and the correction C ------------------------------
  // 1/|d| table over squared integer distances
  int dmax = 0;
  for (int64_t i = 0; i < N; ++i)
    for (int64_t p = t.rowptr[i]; p < t.rowptr[i + 1]; ++p) {
      const int64_t j = t.col[p];
      for (int q1 = 0; q1 < 3; ++q1)
        for (int q2 = 0; q2 < 3; ++q2)
          for (int ax = 0; ax < 3; ++ax)
            dmax = std::max(dmax, std::abs(t.qp_start[3 * (3 * i + q1) + ax] -
                                           t.qp_start[3 * (3 * j + q2) + ax]) + n);
    }
  const int64_t d2max = 3 * int64_t(dmax) * dmax;
  std::vector<double> hs(d2max + 1);
  hs[0] = 0.0;  // H_s self term (eq. Hsmm)
  for (int64_t q = 1; q <= d2max; ++q) hs[q] = 1.0 / (kFourPi * h * std::sqrt(double(q)));
  t.corr.resize(nnz);
  parallel_for(N, nthreads, [&](int64_t b, int64_t e) {
    std::vector<double> K(3 * W);
    for (int64_t i = b; i < e; ++i)
      for (int64_t p = t.rowptr[i]; p < t.rowptr[i + 1]; ++p) {
        const int64_t j = t.col[p];
        double pc = 0.0;
        for (int q1 = 0; q1 < 3; ++q1)
          for (int q2 = 0; q2 < 3; ++q2) {
            const int64_t a1 = 3 * i + q1, a2 = 3 * j + q2;
            int d0[3];
            for (int ax = 0; ax < 3; ++ax) {
              d0[ax] = t.qp_start[3 * a1 + ax] - t.qp_start[3 * a2 + ax];
              const double* la = &lw[(3 * a1 + ax) * S];
              const double* lb = &lw[(3 * a2 + ax) * S];
              double* k = &K[ax * W];
              for (int dd = 0; dd < W; ++dd) k[dd] = 0.0;
              for (int al = 0; al < S; ++al)
                for (int be = 0; be < S; ++be) k[al - be + n] += la[al] * lb[be];
            }
            double acc = 0.0;
            for (int dz = 0; dz < W; ++dz) {
              const int64_t z = d0[2] + dz - n;
              for (int dy = 0; dy < W; ++dy) {
                const int64_t y = d0[1] + dy - n;
                const double kyz = K[2 * W + dz] * K[W + dy];
                const int64_t yz2 = y * y + z * z;
                double accx = 0.0;
                for (int dx = 0; dx < W; ++dx) {
                  const int64_t x = d0[0] + dx - n;
                  accx += K[dx] * hs[x * x + yz2];
                }
                acc += kyz * accx;
              }
            }
            pc += t.qp_w[a1] * t.qp_w[a2] * acc;
          }
        t.corr[p] = t.near_static[p] - pc;
      }
  });

  t.near_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// Dense inverses of A_s,NR over the preconditioner clusters (needs the
// static near entries).
void build_cluster_inverses(HostTables& t, int nthreads) {
  const int64_t ncl = int64_t(t.cl_ptr.size()) - 1;
  t.cl_inv.assign(t.cl_blk[ncl], 0.0);
  parallel_for(ncl, nthreads, [&](int64_t b, int64_t e) {
    std::vector<double> A, I;
    for (int64_t c = b; c < e; ++c) {
      const int64_t o = t.cl_ptr[c], m = t.cl_ptr[c + 1] - o;
      A.assign(m * m, 0.0);
      I.assign(m * m, 0.0);
      for (int64_t r = 0; r < m; ++r) {
        const int32_t i = t.cl_perm[o + r];
        I[r * m + r] = 1.0;
        for (int64_t cc = 0; cc < m; ++cc) {
          const int32_t j = t.cl_perm[o + cc];
          const auto beg = t.col.begin() + t.rowptr[i], end = t.col.begin() + t.rowptr[i + 1];
          const auto it = std::lower_bound(beg, end, j);
          if (it != end && *it == j) A[r * m + cc] = t.near_static[it - t.col.begin()];
        }
      }
      // Gauss-Jordan with partial pivoting
      for (int64_t k = 0; k < m; ++k) {
        int64_t piv = k;
        for (int64_t r = k + 1; r < m; ++r)
          if (std::fabs(A[r * m + k]) > std::fabs(A[piv * m + k])) piv = r;
        AIM_REQUIRE(A[piv * m + k] != 0.0, AIM_ERR_GEOMETRY, "singular near-field block");
        if (piv != k)
          for (int64_t cc = 0; cc < m; ++cc) {
            std::swap(A[k * m + cc], A[piv * m + cc]);
            std::swap(I[k * m + cc], I[piv * m + cc]);
          }
        const double inv = 1.0 / A[k * m + k];
        for (int64_t cc = 0; cc < m; ++cc) {
          A[k * m + cc] *= inv;
          I[k * m + cc] *= inv;
        }
        for (int64_t r = 0; r < m; ++r) {
          if (r == k) continue;
          const double f = A[r * m + k];
          if (f == 0.0) continue;
          for (int64_t cc = 0; cc < m; ++cc) {
            A[r * m + cc] -= f * A[k * m + cc];
            I[r * m + cc] -= f * I[k * m + cc];
          }
        }
      }
      std::copy(I.begin(), I.end(), t.cl_inv.begin() + t.cl_blk[c]);
    }
  });

}

int setup_threads(const aim_setup_desc& d) {
  return d.n_threads > 0 ? d.n_threads : int(std::max(1u, std::thread::hardware_concurrency()));
}

// ---------------------------------------------------------------------------
void build_host_tables(const aim_setup_desc& d, HostTables& t, bool near_on_host) {
  const auto t0 = std::chrono::steady_clock::now();
  AIM_REQUIRE(d.n_vertices >= 3 && d.n_triangles >= 1, AIM_ERR_INVALID_ARG,
              "need at least 3 vertices and 1 triangle");
  AIM_REQUIRE(d.vertices && d.triangles, AIM_ERR_INVALID_ARG, "null mesh array");
  AIM_REQUIRE(d.stencil_order == 2 || d.stencil_order == 3, AIM_ERR_INVALID_ARG,
              "stencil_order must be 2 or 3");
  for (int a = 0; a < 3; ++a)
    AIM_REQUIRE(is_pow2(d.grid_dims[a]) && d.grid_dims[a] >= 8 && d.grid_dims[a] <= 256,
                AIM_ERR_GRID, "grid_dims must be powers of two in [8, 256]");
  AIM_REQUIRE(std::isfinite(d.near_threshold) && d.near_threshold > 0.0, AIM_ERR_INVALID_ARG,
              "near_threshold must be positive");
  AIM_REQUIRE(std::isfinite(d.h), AIM_ERR_INVALID_ARG, "h must be finite");

  const int64_t N = d.n_triangles, NV = d.n_vertices;
  const double* V = d.vertices;
  const int32_t* T = d.triangles;
  for (int64_t i = 0; i < 3 * NV; ++i)
    AIM_REQUIRE(std::isfinite(V[i]), AIM_ERR_GEOMETRY, "non-finite vertex coordinate");
  for (int64_t i = 0; i < 3 * N; ++i)
    AIM_REQUIRE(T[i] >= 0 && T[i] < NV, AIM_ERR_GEOMETRY, "triangle vertex index out of range");

  const int nthreads = setup_threads(d);
  t.N = N;
  t.order = d.stencil_order;
  for (int a = 0; a < 3; ++a) t.dims[a] = d.grid_dims[a];

  // -- bounding box, spacing, origin -----------------------------------------
  double lo[3] = {V[0], V[1], V[2]}, hi[3] = {V[0], V[1], V[2]};
  for (int64_t i = 0; i < NV; ++i)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], V[3 * i + a]);
      hi[a] = std::max(hi[a], V[3 * i + a]);
    }
  double h = d.h;
  if (!(h > 0.0)) {
    h = 0.0;
    for (int a = 0; a < 3; ++a) h = std::max(h, (hi[a] - lo[a]) / double(t.dims[a] - 5));
  }
  AIM_REQUIRE(h > 0.0, AIM_ERR_GRID, "grid spacing is zero (degenerate bounding box)");
  t.h = h;
  for (int a = 0; a < 3; ++a) t.origin[a] = 0.5 * (lo[a] + hi[a]) - h * (t.dims[a] - 1.0) / 2.0;
  double diag = 0.0;
  for (int a = 0; a < 3; ++a) diag += (hi[a] - lo[a]) * (hi[a] - lo[a]);
  diag = std::sqrt(diag);

  // -- areas and quadrature points -------------------------------------------
  static const double bary[3][3] = {{2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0},
                                    {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0},
                                    {1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0}};
  t.area.resize(N);
  t.corners.resize(9 * N);
  t.tri_idx.assign(T, T + 3 * N);
  t.qp_xyz.resize(9 * N);
  t.qp_w.resize(3 * N);
  t.qp_start.resize(9 * N);
  t.qp_local.resize(9 * N);
  std::vector<double> cent(3 * N);
  for (int64_t j = 0; j < N; ++j) {
    const double* a = V + 3 * T[3 * j];
    const double* b = V + 3 * T[3 * j + 1];
    const double* c = V + 3 * T[3 * j + 2];
    double e1[3], e2[3], n[3];
    sub3(b, a, e1);
    sub3(c, a, e2);
    cross3(e1, e2, n);
    const double A = 0.5 * norm3(n);
    AIM_REQUIRE(std::isfinite(A) && A > 1e-14 * diag * diag, AIM_ERR_GEOMETRY,
                "zero-area triangle " + std::to_string(j));
    t.area[j] = A;
    for (int a2 = 0; a2 < 3; ++a2) {
      cent[3 * j + a2] = (a[a2] + b[a2] + c[a2]) / 3.0;
      t.corners[9 * j + a2] = a[a2];
      t.corners[9 * j + 3 + a2] = b[a2];
      t.corners[9 * j + 6 + a2] = c[a2];
    }
    for (int q = 0; q < 3; ++q) {
      const int64_t p = 3 * j + q;
      t.qp_w[p] = A / 3.0;
      for (int ax = 0; ax < 3; ++ax) {
        const double x = a[ax] * bary[q][0] + b[ax] * bary[q][1] + c[ax] * bary[q][2];
        t.qp_xyz[3 * p + ax] = x;
        const double tt = (x - t.origin[ax]) / h;
        const double s = std::floor(tt - (t.order - 1) / 2.0);
        AIM_REQUIRE(s >= 0.0 && s + t.order <= t.dims[ax] - 1, AIM_ERR_GRID,
                    "a projection stencil leaves the grid (triangle " + std::to_string(j) + ")");
        t.qp_start[3 * p + ax] = int32_t(s);
        t.qp_local[3 * p + ax] = tt - s;
      }
    }
  }

  // -- near list by uniform cells of edge tau ---------------------------------
  const double tau = d.near_threshold;
  int nc[3];
  double clo[3];
  for (int a = 0; a < 3; ++a) {
    clo[a] = lo[a];
    nc[a] = std::max(1, std::min(1 << 20, int(std::floor((hi[a] - lo[a]) / tau)) + 1));
  }
  auto cell_of = [&](const double* p, int* ci) {
    for (int a = 0; a < 3; ++a)
      ci[a] = std::min(nc[a] - 1, std::max(0, int(std::floor((p[a] - clo[a]) / tau))));
  };
  const int64_t ncells = int64_t(nc[0]) * nc[1] * nc[2];
  AIM_REQUIRE(ncells < (int64_t(1) << 31), AIM_ERR_INVALID_ARG, "near threshold too small");
  std::vector<int64_t> cell_ptr(ncells + 1, 0);
  std::vector<int32_t> cell_item(N);
  std::vector<int64_t> cell_id(N);
  for (int64_t j = 0; j < N; ++j) {
    int ci[3];
    cell_of(&cent[3 * j], ci);
    cell_id[j] = (int64_t(ci[2]) * nc[1] + ci[1]) * nc[0] + ci[0];
    cell_ptr[cell_id[j] + 1]++;
  }
  for (int64_t c = 0; c < ncells; ++c) cell_ptr[c + 1] += cell_ptr[c];
  {
    std::vector<int64_t> fill(cell_ptr.begin(), cell_ptr.end() - 1);
    for (int64_t j = 0; j < N; ++j) cell_item[fill[cell_id[j]]++] = int32_t(j);
  }
  std::vector<std::vector<int32_t>> nbrs(N);
  parallel_for(N, nthreads, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) {
      int ci[3];
      cell_of(&cent[3 * i], ci);
      auto& L = nbrs[i];
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            const int x = ci[0] + dx, y = ci[1] + dy, z = ci[2] + dz;
            if (x < 0 || y < 0 || z < 0 || x >= nc[0] || y >= nc[1] || z >= nc[2]) continue;
            const int64_t c = (int64_t(z) * nc[1] + y) * nc[0] + x;
            for (int64_t p = cell_ptr[c]; p < cell_ptr[c + 1]; ++p) {
              const int32_t j = cell_item[p];
              const double ddx = cent[3 * i] - cent[3 * j];
              const double ddy = cent[3 * i + 1] - cent[3 * j + 1];
              const double ddz = cent[3 * i + 2] - cent[3 * j + 2];
              if (j == i || std::sqrt(ddx * ddx + ddy * ddy + ddz * ddz) < tau) L.push_back(j);
            }
          }
      std::sort(L.begin(), L.end());
    }
  });
  t.rowptr.assign(N + 1, 0);
  for (int64_t i = 0; i < N; ++i) t.rowptr[i + 1] = t.rowptr[i] + int64_t(nbrs[i].size());
  const int64_t nnz = t.rowptr[N];
  AIM_REQUIRE(nnz < (int64_t(1) << 31), AIM_ERR_INVALID_ARG, "near list too large");
  t.col.resize(nnz);
  for (int64_t i = 0; i < N; ++i)
    std::copy(nbrs[i].begin(), nbrs[i].end(), t.col.begin() + t.rowptr[i]);
  nbrs.clear();
  nbrs.shrink_to_fit();

  const int n = t.order, S = n + 1;
  std::vector<double> lw(3 * N * 3 * S);  // [qp][axis][a]
  for (int64_t p = 0; p < 3 * N; ++p)
    for (int ax = 0; ax < 3; ++ax) lagrange(t.qp_local[3 * p + ax], n, &lw[(3 * p + ax) * S]);
  if (near_on_host) fill_near_host(t, V, T, nthreads);

  // -- projection matrix P (merged per triangle) -------------------------------
  {
    const int64_t Ng = int64_t(t.dims[0]) * t.dims[1] * t.dims[2];
    const int S3 = S * S * S;
    t.pt_rowptr.assign(N + 1, 0);
    std::vector<std::vector<std::pair<int32_t, double>>> rows(N);
    parallel_for(N, nthreads, [&](int64_t b, int64_t e) {
      std::vector<std::pair<int32_t, double>> tmp;
      for (int64_t j = b; j < e; ++j) {
        tmp.clear();
        for (int qd = 0; qd < 3; ++qd) {
          const int64_t p = 3 * j + qd;
          const int* s0 = &t.qp_start[3 * p];
          const double* lx = &lw[(3 * p + 0) * S];
          const double* ly = &lw[(3 * p + 1) * S];
          const double* lz = &lw[(3 * p + 2) * S];
          for (int c = 0; c < S; ++c)
            for (int bb = 0; bb < S; ++bb)
              for (int a = 0; a < S; ++a) {
                const int32_t u = int32_t((int64_t(s0[2] + c) * t.dims[1] + (s0[1] + bb)) *
                                              t.dims[0] + s0[0] + a);
                tmp.push_back({u, t.qp_w[p] * (lx[a] * ly[bb] * lz[c])});
              }
        }
        std::stable_sort(tmp.begin(), tmp.end(),
                         [](const auto& x, const auto& y) { return x.first < y.first; });
        auto& r = rows[j];
        r.reserve(std::min<size_t>(tmp.size(), size_t(3 * S3)));
        for (const auto& pr : tmp) {
          if (!r.empty() && r.back().first == pr.first)
            r.back().second += pr.second;
          else
            r.push_back(pr);
        }
      }
    });
    for (int64_t j = 0; j < N; ++j) t.pt_rowptr[j + 1] = t.pt_rowptr[j] + int32_t(rows[j].size());
    const int64_t nnzp = t.pt_rowptr[N];
    AIM_REQUIRE(nnzp < (int64_t(1) << 31), AIM_ERR_INVALID_ARG, "projection matrix too large");
    t.pt_col.resize(nnzp);
    t.pt_val.resize(nnzp);
    t.p_rowptr.assign(Ng + 1, 0);
    for (int64_t j = 0; j < N; ++j)
      for (int64_t k = 0; k < int64_t(rows[j].size()); ++k) {
        t.pt_col[t.pt_rowptr[j] + k] = rows[j][k].first;
        t.pt_val[t.pt_rowptr[j] + k] = rows[j][k].second;
        t.p_rowptr[rows[j][k].first + 1]++;
      }
    rows.clear();
    rows.shrink_to_fit();
    for (int64_t u = 0; u < Ng; ++u) t.p_rowptr[u + 1] += t.p_rowptr[u];
    t.p_col.resize(nnzp);
    t.p_val.resize(nnzp);
    std::vector<int32_t> fill(t.p_rowptr.begin(), t.p_rowptr.end() - 1);
    for (int64_t j = 0; j < N; ++j)  // ascending j keeps each node row sorted
      for (int64_t k = t.pt_rowptr[j]; k < t.pt_rowptr[j + 1]; ++k) {
        const int32_t u = t.pt_col[k];
        t.p_col[fill[u]] = int32_t(j);
        t.p_val[fill[u]++] = t.pt_val[k];
      }
    t.p_blk = row_blocks(t.p_rowptr);
  }

  // -- near-block preconditioner clusters (recursive coordinate bisection) ----
  const int kMaxCluster = 64;
  std::vector<int32_t> perm(N);
  std::iota(perm.begin(), perm.end(), 0);
  std::vector<std::pair<int64_t, int64_t>> stack{{0, N}}, leaves;
  while (!stack.empty()) {
    auto [b, e] = stack.back();
    stack.pop_back();
    if (e - b <= kMaxCluster) {
      leaves.push_back({b, e});
      continue;
    }
    double l3[3] = {1e300, 1e300, 1e300}, h3[3] = {-1e300, -1e300, -1e300};
    for (int64_t q = b; q < e; ++q)
      for (int a = 0; a < 3; ++a) {
        l3[a] = std::min(l3[a], cent[3 * perm[q] + a]);
        h3[a] = std::max(h3[a], cent[3 * perm[q] + a]);
      }
    int ax = 0;
    for (int a = 1; a < 3; ++a)
      if (h3[a] - l3[a] > h3[ax] - l3[ax]) ax = a;
    const int64_t mid = b + (e - b) / 2;
    std::nth_element(perm.begin() + b, perm.begin() + mid, perm.begin() + e,
                     [&](int32_t x, int32_t y) {
                       const double cx = cent[3 * x + ax], cy = cent[3 * y + ax];
                       return cx < cy || (cx == cy && x < y);
                     });
    stack.push_back({mid, e});
    stack.push_back({b, mid});
  }
  std::sort(leaves.begin(), leaves.end());
  const int64_t ncl = int64_t(leaves.size());
  t.cl_ptr.resize(ncl + 1);
  t.cl_perm = perm;
  t.cl_blk.resize(ncl + 1);
  t.cl_ptr[0] = 0;
  t.cl_blk[0] = 0;
  for (int64_t c = 0; c < ncl; ++c) {
    t.cl_ptr[c + 1] = int32_t(leaves[c].second);
    const int64_t m = leaves[c].second - leaves[c].first;
    t.cl_blk[c + 1] = t.cl_blk[c] + m * m;
  }
  if (near_on_host) build_cluster_inverses(t, nthreads);

  t.setup_seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace aim
