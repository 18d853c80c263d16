// Host-side tables of the RWG EFIE under AIMx (Sec. II-A, eq. EFIEdis, and
// Sec. II-B, eqs. aimLFR and LAIMx, with the static split of Sec. III-A).
//
// The operator on RWG functions f_n (Rao, Wilton and Glisson, 1982), with
// the gradient moved onto the testing function and the factor -j omega mu
// left out:
//
//   Z_mn = <f_m, G f_n> - k^-2 <div f_m, G div f_n>
//        ~= C_A - k^-2 C_phi + sum_{c=x,y,z} P_c^T H(k) P_c - k^-2 P_q^T H(k) P_q.
//
// Function n lives on an interior edge (length l) shared by T+ and T- (T+
// the triangle of lower index); with p+- the vertices opposite the edge,
// f_n = l/(2A+) (r - p+) on T+ and l/(2A-) (p- - r) on T-, so
// div f_n = +l/A+ on T+ and -l/A- on T-.  Functions are numbered by their
// edges' (smaller, larger) vertex index pairs in ascending order.
//
// The far part works on the quadrature points: the four channel values
// w_q f_c(r_q) and w_q div f(r_q) of every function at every point are
// gathered into point sources, projected with the point stencils
// Lambda_u(r_p) and interpolated back with the same stencils.
//
// C_A = A_s,NR - A_s,P and C_phi likewise use the static kernel 1/(4 pi R)
// (eq. hgfs) on the RWG near list: the inner integrals over a source
// triangle in closed form (int 1/R and int r'/R), the outer integral by the
// 3-point rule, the static part symmetrised, (M + M^T)/2; the precorrection
// is the grid product of the channel stencils through H_s (self term 0, eq.
// Hsmm), summed from its point-pair values.  Two functions are near when a
// triangle of one is near a triangle of the other (the triangle near list of
// the scalar operator).
#include <algorithm>
#include <cmath>
#include <tuple>

#include "aim_internal.h"

#pragma clang fp contract(off)

namespace aim {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kFourPi = 4.0 * kPi;

// index of column j in the sorted row i of a CSR list, or -1
int64_t find_in_row(const std::vector<int64_t>& rowptr, const std::vector<int32_t>& col,
                    int64_t i, int32_t j) {
  const auto beg = col.begin() + rowptr[i], end = col.begin() + rowptr[i + 1];
  const auto it = std::lower_bound(beg, end, j);
  return (it != end && *it == j) ? int64_t(it - col.begin()) : -1;
}

}  // namespace

void build_efie_tables(const HostTables& t, EfieTables& e, int nthreads) {
  const int64_t N = t.N;
  AIM_REQUIRE(t.tri_idx.size() == 3 * size_t(N) && t.corners.size() == 9 * size_t(N),
              AIM_ERR_STATE, "the RWG operator needs the mesh (not kept by loaded plans)");
  // -- RWG functions -----------------------------------------------------------
  std::vector<std::tuple<int32_t, int32_t, int32_t, int32_t>> edges;  // (a, b, t, e)
  edges.reserve(3 * size_t(N));
  for (int64_t j = 0; j < N; ++j)
    for (int ed = 0; ed < 3; ++ed) {
      const int32_t a = t.tri_idx[3 * j + (ed + 1) % 3], b = t.tri_idx[3 * j + (ed + 2) % 3];
      edges.emplace_back(std::min(a, b), std::max(a, b), int32_t(j), ed);
    }
  std::sort(edges.begin(), edges.end());
  e.tri_rwg.assign(3 * size_t(N), -1);
  e.sgn_len.assign(3 * size_t(N), 0.0);
  e.rwg_te.clear();
  size_t g = 0;
  while (g < edges.size()) {
    size_t h = g + 1;
    while (h < edges.size() && std::get<0>(edges[h]) == std::get<0>(edges[g]) &&
           std::get<1>(edges[h]) == std::get<1>(edges[g]))
      ++h;
    AIM_REQUIRE(h - g <= 2, AIM_ERR_GEOMETRY, "an edge is shared by more than two triangles");
    if (h - g == 2) {
      const int32_t n = int32_t(e.rwg_te.size() / 4);
      const auto [a, b, t1, e1] = edges[g];
      const auto t2 = std::get<2>(edges[g + 1]);
      const auto e2 = std::get<3>(edges[g + 1]);
      AIM_REQUIRE(t1 != t2, AIM_ERR_GEOMETRY, "a triangle repeats an edge");
      // the edge's endpoints are the corners of t1 after its vertex e1
      const double* p = &t.corners[9 * size_t(t1) + 3 * ((e1 + 1) % 3)];
      const double* q = &t.corners[9 * size_t(t1) + 3 * ((e1 + 2) % 3)];
      const double d[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]};
      const double L = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      e.tri_rwg[3 * size_t(t1) + e1] = n;
      e.tri_rwg[3 * size_t(t2) + e2] = n;
      e.sgn_len[3 * size_t(t1) + e1] = L;
      e.sgn_len[3 * size_t(t2) + e2] = -L;
      e.rwg_te.insert(e.rwg_te.end(), {t1, e1, t2, e2});
      (void)a;
      (void)b;
    }
    g = h;
  }
  const int64_t n = int64_t(e.rwg_te.size() / 4);
  e.n = n;
  edges.clear();
  edges.shrink_to_fit();

  // -- channel values at the points: w_q f(r_q) and w_q div f -----------------
  e.vals.assign(36 * size_t(N), 0.0);
  parallel_ranges(N, nthreads, [&](int64_t b0, int64_t b1) {
    for (int64_t j = b0; j < b1; ++j)
      for (int ed = 0; ed < 3; ++ed) {
        const double sl = e.sgn_len[3 * j + ed];
        if (sl == 0.0) continue;
        const double A = t.area[j];
        const double* fr = &t.corners[9 * j + 3 * ed];  // the free vertex
        for (int q = 0; q < 3; ++q) {
          const double w = t.qp_w[3 * j + q];
          const double* r = &t.qp_xyz[3 * (3 * j + q)];
          double* v = &e.vals[36 * j + 12 * q + 4 * ed];
          const double coef = sl / (2.0 * A);
          for (int c = 0; c < 3; ++c) v[c] = coef * (r[c] - fr[c]) * w;
          v[3] = sl / A * w;
        }
      }
  });

  // -- RWG near list ----------------------------------------------------------
  std::vector<std::vector<int32_t>> rows(n);
  parallel_ranges(n, nthreads, [&](int64_t b0, int64_t b1) {
    for (int64_t m = b0; m < b1; ++m) {
      auto& L = rows[m];
      for (int side = 0; side < 2; ++side) {
        const int64_t tm = e.rwg_te[4 * m + 2 * side];
        for (int64_t p = t.rowptr[tm]; p < t.rowptr[tm + 1]; ++p) {
          const int64_t j = t.col[p];
          for (int ed = 0; ed < 3; ++ed)
            if (e.tri_rwg[3 * j + ed] >= 0) L.push_back(e.tri_rwg[3 * j + ed]);
        }
      }
      std::sort(L.begin(), L.end());
      L.erase(std::unique(L.begin(), L.end()), L.end());
    }
  });
  e.rowptr.assign(n + 1, 0);
  for (int64_t m = 0; m < n; ++m) {
    const int64_t next = int64_t(e.rowptr[m]) + int64_t(rows[m].size());
    AIM_REQUIRE(next < (int64_t(1) << 31), AIM_ERR_INVALID_ARG, "RWG near list too large");
    e.rowptr[m + 1] = int32_t(next);
  }
  e.col.resize(e.rowptr[n]);
  for (int64_t m = 0; m < n; ++m)
    std::copy(rows[m].begin(), rows[m].end(), e.col.begin() + e.rowptr[m]);
  rows.clear();
  rows.shrink_to_fit();

  // -- triangle pairs behind the near list: (T of m, T of n) for every near
  // (m, n) -------------------------------------------------------------------
  std::vector<std::vector<int32_t>> prow(N);
  parallel_ranges(N, nthreads, [&](int64_t b0, int64_t b1) {
    for (int64_t i = b0; i < b1; ++i) {
      auto& L = prow[i];
      for (int ed = 0; ed < 3; ++ed) {
        const int32_t m = e.tri_rwg[3 * i + ed];
        if (m < 0) continue;
        for (int32_t p = e.rowptr[m]; p < e.rowptr[m + 1]; ++p) {
          const int32_t nn = e.col[p];
          L.push_back(e.rwg_te[4 * size_t(nn)]);
          L.push_back(e.rwg_te[4 * size_t(nn) + 2]);
        }
      }
      std::sort(L.begin(), L.end());
      L.erase(std::unique(L.begin(), L.end()), L.end());
    }
  });
  e.pair_rowptr.assign(N + 1, 0);
  for (int64_t i = 0; i < N; ++i) e.pair_rowptr[i + 1] = e.pair_rowptr[i] + int64_t(prow[i].size());
  e.pair_col.resize(e.pair_rowptr[N]);
  for (int64_t i = 0; i < N; ++i)
    std::copy(prow[i].begin(), prow[i].end(), e.pair_col.begin() + e.pair_rowptr[i]);
  prow.clear();
  prow.shrink_to_fit();

  // -- point projection -------------------------------------------------------
  const int o = t.order, S = o + 1, S3 = S * S * S;
  const int64_t P = 3 * N;
  const int64_t Ng = int64_t(t.dims[0]) * t.dims[1] * t.dims[2];
  AIM_REQUIRE(P * S3 < (int64_t(1) << 31), AIM_ERR_INVALID_ARG, "point projection too large");
  e.pt_rowptr.resize(P + 1);
  for (int64_t p = 0; p <= P; ++p) e.pt_rowptr[p] = int32_t(p * S3);
  e.pt_col.resize(P * S3);
  e.pt_val.resize(P * S3);
  parallel_ranges(P, nthreads, [&](int64_t b0, int64_t b1) {
    double lw[3][4];
    for (int64_t p = b0; p < b1; ++p) {
      for (int ax = 0; ax < 3; ++ax) lagrange_host(t.qp_local[3 * p + ax], o, lw[ax]);
      const int32_t* s0 = &t.qp_start[3 * p];
      int64_t k = p * S3;
      for (int c = 0; c < S; ++c)
        for (int b = 0; b < S; ++b)
          for (int a = 0; a < S; ++a, ++k) {
            e.pt_col[k] = int32_t((int64_t(s0[2] + c) * t.dims[1] + (s0[1] + b)) * t.dims[0] +
                                  s0[0] + a);
            e.pt_val[k] = lw[0][a] * lw[1][b] * lw[2][c];
          }
    }
  });
  e.p_rowptr.assign(Ng + 1, 0);
  for (int64_t k = 0; k < P * S3; ++k) e.p_rowptr[e.pt_col[k] + 1]++;
  for (int64_t u = 0; u < Ng; ++u) e.p_rowptr[u + 1] += e.p_rowptr[u];
  e.p_col.resize(P * S3);
  e.p_val.resize(P * S3);
  {
    std::vector<int32_t> fill(e.p_rowptr.begin(), e.p_rowptr.end() - 1);
    for (int64_t p = 0; p < P; ++p)  // ascending p keeps each node row sorted
      for (int64_t k = p * S3; k < (p + 1) * S3; ++k) {
        const int32_t u = e.pt_col[k];
        e.p_col[fill[u]] = int32_t(p);
        e.p_val[fill[u]++] = e.pt_val[k];
      }
  }
  e.p_blk = row_blocks(e.p_rowptr);
}

void assemble_efie_near(const HostTables& t, EfieTables& e, const std::vector<double>& pv,
                        int nthreads) {
  const int64_t n = e.n;
  AIM_REQUIRE(pv.size() == size_t(kEfiePairVals) * e.pair_col.size(), AIM_ERR_STATE,
              "pair values do not match the pair list");
  // static part of row m, column nn: sum over the testing triangles' points
  // of (w f_m) . int_{T_n} f_n / (4 pi R) and (w div f_m) int_{T_n} div f_n / (4 pi R)
  auto static_entry = [&](int32_t m, int32_t nn, double& sa, double& sq) {
    sa = sq = 0.0;
    for (int sm = 0; sm < 2; ++sm) {
      const int32_t tm = e.rwg_te[4 * size_t(m) + 2 * sm], em = e.rwg_te[4 * size_t(m) + 2 * sm + 1];
      for (int sn = 0; sn < 2; ++sn) {
        const int32_t tn = e.rwg_te[4 * size_t(nn) + 2 * sn];
        const int32_t en = e.rwg_te[4 * size_t(nn) + 2 * sn + 1];
        const int64_t idx = find_in_row(e.pair_rowptr, e.pair_col, tm, tn);
        AIM_REQUIRE(idx >= 0, AIM_ERR_STATE, "triangle pair missing from the pair list");
        const double* v = &pv[size_t(kEfiePairVals) * idx];
        const double sl = e.sgn_len[3 * size_t(tn) + en], A = t.area[tn];
        const double coef = sl / (2.0 * A), dn = sl / A;
        const double* fr = &t.corners[9 * size_t(tn) + 3 * en];
        for (int q = 0; q < 3; ++q) {
          const double* fm = &e.vals[36 * size_t(tm) + 12 * q + 4 * em];
          const double s1 = v[q];
          const double* sv = v + 3 + 3 * q;
          double dotv = 0.0;
          for (int c = 0; c < 3; ++c) dotv += fm[c] * (coef * (sv[c] - fr[c] * s1));
          sa += dotv;
          sq += fm[3] * s1 * dn;
        }
      }
    }
    sa /= kFourPi;
    sq /= kFourPi;
  };
  e.ca.assign(e.col.size(), 0.0);
  e.cphi.assign(e.col.size(), 0.0);
  parallel_ranges(n, nthreads, [&](int64_t b0, int64_t b1) {
    for (int64_t m = b0; m < b1; ++m)
      for (int32_t p = e.rowptr[m]; p < e.rowptr[m + 1]; ++p) {
        const int32_t nn = e.col[p];
        double a1, q1, a2, q2;
        static_entry(int32_t(m), nn, a1, q1);
        static_entry(nn, int32_t(m), a2, q2);
        // precorrection: point pairs of the two functions through H_s
        double pa = 0.0, pq = 0.0;
        for (int sm = 0; sm < 2; ++sm) {
          const int32_t tm = e.rwg_te[4 * m + 2 * sm], em = e.rwg_te[4 * m + 2 * sm + 1];
          for (int sn = 0; sn < 2; ++sn) {
            const int32_t tn = e.rwg_te[4 * size_t(nn) + 2 * sn];
            const int32_t en = e.rwg_te[4 * size_t(nn) + 2 * sn + 1];
            const int64_t idx = find_in_row(e.pair_rowptr, e.pair_col, tm, tn);
            AIM_REQUIRE(idx >= 0, AIM_ERR_STATE, "triangle pair missing from the pair list");
            const double* pp = &pv[size_t(kEfiePairVals) * idx + 12];
            for (int q = 0; q < 3; ++q) {
              const double* fm = &e.vals[36 * size_t(tm) + 12 * q + 4 * em];
              for (int q2 = 0; q2 < 3; ++q2) {
                const double* fn = &e.vals[36 * size_t(tn) + 12 * q2 + 4 * en];
                const double h = pp[3 * q + q2];
                pa += h * (fm[0] * fn[0] + fm[1] * fn[1] + fm[2] * fn[2]);
                pq += h * (fm[3] * fn[3]);
              }
            }
          }
        }
        e.ca[p] = 0.5 * (a1 + a2) - pa;
        e.cphi[p] = 0.5 * (q1 + q2) - pq;
      }
  });
}

// The double layer's near values.  With t_q = w_q f_m(r_q) x n_m (n_m the
// testing triangle's unit normal), f_m . (n_m x V) = t_q . V, and for
// f_n = s l/(2A) (r' - p) on its triangle,
//   int grad G_s x f_n dS' = -(s l/(2A)) (1/4 pi) g(r) x (r - p),
// g(r) = int (r - r')/R^3 dS' (the pair values); the precorrection is
// sum over point pairs of t_q . (H_s x J_q') with H_s = -(the pair's grid
// sums) the static samples of grad G and J_q' = w f_n(r_q'); the Gram
// entries come from triangles the two functions share.
void assemble_mfie_near(const HostTables& t, const EfieTables& e, const std::vector<double>& pv,
                        std::vector<double>& ck, int nthreads) {
  const int64_t n = e.n, N = t.N;
  AIM_REQUIRE(pv.size() == size_t(kMfiePairVals) * e.pair_col.size(), AIM_ERR_STATE,
              "pair values do not match the pair list");
  AIM_REQUIRE(e.vals.size() == 36 * size_t(N), AIM_ERR_STATE, "channel values not kept");
  std::vector<double> nrm(3 * size_t(N));
  for (int64_t j = 0; j < N; ++j) {
    const double* c = &t.corners[9 * j];
    const double e1[3] = {c[3] - c[0], c[4] - c[1], c[5] - c[2]};
    const double e2[3] = {c[6] - c[0], c[7] - c[1], c[8] - c[2]};
    const double v[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                         e1[0] * e2[1] - e1[1] * e2[0]};
    const double l = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int a = 0; a < 3; ++a) nrm[3 * j + a] = v[a] / l;
  }
  auto cross = [](const double* a, const double* b, double* o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
  };
  ck.assign(2 * std::max<size_t>(e.col.size(), 1), 0.0);
  parallel_ranges(n, nthreads, [&](int64_t b0, int64_t b1) {
    for (int64_t m = b0; m < b1; ++m)
      for (int32_t p = e.rowptr[m]; p < e.rowptr[m + 1]; ++p) {
        const int32_t nn = e.col[p];
        double sk = 0.0, pk = 0.0, gr = 0.0;
        for (int sm = 0; sm < 2; ++sm) {
          const int32_t tm = e.rwg_te[4 * m + 2 * sm], em = e.rwg_te[4 * m + 2 * sm + 1];
          double tv[3][3];  // t_q of the testing function on tm
          for (int q = 0; q < 3; ++q) cross(&e.vals[36 * size_t(tm) + 12 * q + 4 * em],
                                            &nrm[3 * size_t(tm)], tv[q]);
          for (int sn = 0; sn < 2; ++sn) {
            const int32_t tn = e.rwg_te[4 * size_t(nn) + 2 * sn];
            const int32_t en = e.rwg_te[4 * size_t(nn) + 2 * sn + 1];
            const int64_t idx = find_in_row(e.pair_rowptr, e.pair_col, tm, tn);
            AIM_REQUIRE(idx >= 0, AIM_ERR_STATE, "triangle pair missing from the pair list");
            const double* v = &pv[size_t(kMfiePairVals) * idx];
            const double sl = e.sgn_len[3 * size_t(tn) + en];
            const double coef = -sl / (2.0 * t.area[tn]) / kFourPi;
            const double* fr = &t.corners[9 * size_t(tn) + 3 * en];
            for (int q = 0; q < 3; ++q) {
              const double* r = &t.qp_xyz[3 * (3 * size_t(tm) + q)];
              const double rp[3] = {r[0] - fr[0], r[1] - fr[1], r[2] - fr[2]};
              double gx[3];
              cross(v + 3 * q, rp, gx);
              sk += coef * (tv[q][0] * gx[0] + tv[q][1] * gx[1] + tv[q][2] * gx[2]);
              for (int q2 = 0; q2 < 3; ++q2) {
                const double* hs = v + 9 + 3 * (3 * q + q2);
                const double* jn = &e.vals[36 * size_t(tn) + 12 * q2 + 4 * en];
                double hj[3];
                cross(hs, jn, hj);  // (-H_s) x J
                pk -= tv[q][0] * hj[0] + tv[q][1] * hj[1] + tv[q][2] * hj[2];
              }
            }
            if (tm == tn)
              for (int q = 0; q < 3; ++q) {
                const double* fm = &e.vals[36 * size_t(tm) + 12 * q + 4 * em];
                const double* fn = &e.vals[36 * size_t(tm) + 12 * q + 4 * en];
                gr += (fm[0] * fn[0] + fm[1] * fn[1] + fm[2] * fn[2]) / t.qp_w[3 * size_t(tm) + q];
              }
          }
        }
        ck[2 * size_t(p)] = sk - pk;
        ck[2 * size_t(p) + 1] = gr;
      }
  });
}

}  // namespace aim
