// Internal declarations shared by the host set-up, the device kernels and the
// C ABI of the AIMx library.  Not part of the public interface (include/aim.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/aim.h"

namespace aim {

// ---------------------------------------------------------------------------
// errors: every internal failure is an aim::Error carrying the ABI status
// ---------------------------------------------------------------------------
struct Error : std::runtime_error {
  aim_status status;
  Error(aim_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define AIM_HIP(call)                                                             \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      throw ::aim::Error(AIM_ERR_DEVICE, std::string(#call) + ": " +              \
                                             hipGetErrorString(e_));              \
  } while (0)

#define AIM_REQUIRE(cond, status, msg)                                            \
  do {                                                                            \
    if (!(cond)) throw ::aim::Error((status), (msg));                             \
  } while (0)

// ---------------------------------------------------------------------------
// host-side set-up results (setup_host.cpp)
// ---------------------------------------------------------------------------
struct HostTables {
  int64_t N = 0;                    // triangles
  int order = 2;                    // stencil order n
  int dims[3] = {0, 0, 0};          // unpadded grid
  double h = 0.0;
  double origin[3] = {0, 0, 0};
  std::vector<double> area;         // [N]
  std::vector<double> corners;      // [N][3][3] triangle corners (empty on loaded plans)
  std::vector<int32_t> tri_idx;     // [N][3] vertex indices (empty on loaded plans)
  std::vector<double> qp_xyz;       // [3N][3] quadrature points
  std::vector<double> qp_w;         // [3N] weights area/3
  std::vector<int32_t> qp_start;    // [3N][3] stencil start per axis
  std::vector<double> qp_local;     // [3N][3] t - s per axis
  // near field (CSR, rows sorted by column)
  std::vector<int64_t> rowptr;      // [N+1]
  std::vector<int32_t> col;         // [nnz]
  std::vector<double> near_static;  // [nnz] A_s,NR
  std::vector<double> corr;         // [nnz] C = A_s,NR - A_s,P
  // projection P[u, j] = sum_q (A_j/3) Lambda_u(r_jq), merged per triangle,
  // stored twice: by grid node (rows = nodes, for q = P x) and by triangle
  // (rows = triangles, for y = P^T phi); rows sorted by column
  std::vector<int32_t> p_rowptr;    // [Ng+1]
  std::vector<int32_t> p_col;       // triangle ids
  std::vector<double> p_val;
  std::vector<int32_t> p_blk;       // row blocks of P for the projection kernel
  std::vector<int32_t> pt_rowptr;   // [N+1]
  std::vector<int32_t> pt_col;      // grid node ids
  std::vector<double> pt_val;
  // near-block preconditioner: clusters of triangles
  std::vector<int32_t> cl_ptr;      // [ncl+1] offsets into cl_perm
  std::vector<int32_t> cl_perm;     // [N] triangle ids grouped by cluster
  std::vector<int64_t> cl_blk;      // [ncl+1] offsets into cl_inv
  std::vector<double> cl_inv;       // dense inverse blocks, row-major
  double setup_seconds = 0.0;
  double near_seconds = 0.0;        // the static near fill (host or device)
  // diagonal D of the linear-term modification (k^2 D added to C); empty
  // when not computed (host-only and loaded plans)
  std::vector<double> lin_diag;
};

// Builds every host table; throws aim::Error on invalid input.  With
// near_on_host false the static near entries, C and the cluster inverses
// are left out (every validation still happens here): the caller fills
// near_static and corr (on the device) and then calls
// build_cluster_inverses.
void build_host_tables(const aim_setup_desc& d, HostTables& t, bool near_on_host = true);
// A_s,NR and C on the near list, on the host
void fill_near_host(HostTables& t, const double* V, const int32_t* T, int nthreads);
// dense inverses of A_s,NR over the preconditioner clusters
void build_cluster_inverses(HostTables& t, int nthreads);
// host threads for set-up (the descriptor's n_threads, else all cores)
int setup_threads(const aim_setup_desc& d);
// fn(begin, end) over chunks of [0, n) on nthreads host threads
void parallel_ranges(int64_t n, int nthreads, const std::function<void(int64_t, int64_t)>& fn);
// Lagrange weights of the points 0..order at the local coordinate u
void lagrange_host(double u, int order, double* out);
// Row blocks of a CSR matrix for launch_project (see kProjNnz)
std::vector<int32_t> row_blocks(const std::vector<int32_t>& rowptr);

// ---------------------------------------------------------------------------
// RWG EFIE (Sec. II-A, eq. EFIEdis; Sec. II-B, eq. LAIMx): the operator
// L^A - k^-2 L^phi on RWG functions, with three Cartesian current channels
// and one charge channel projected from the quadrature points and convolved
// with the same spectrum H(k); C_A and C_phi are the static near corrections
// of the two parts (real, frequency independent)
// ---------------------------------------------------------------------------
// doubles per triangle pair (i, j) from the device fill: the integrals over
// T_j of 1/R [3] and r'/R [3][3] at the three points of T_i, then the
// point-pair precorrections sum_{u,v} L_u(r_iq) H_s(u - v) L_v(r_jq') [3][3]
constexpr int kEfiePairVals = 21;
// doubles per triangle pair for the double layer: int_{T_j} (r - r')/R^3
// [3 points][3] at the points of T_i, then the point-pair sums of the static
// grid samples h (u - v)/(4 pi R^3) [3][3][3]
constexpr int kMfiePairVals = 36;
struct EfieTables {
  int64_t n = 0;                      // RWG functions (interior edges)
  std::vector<int32_t> tri_rwg;       // [N][3] function on the edge opposite vertex e, or -1
  std::vector<double> sgn_len;        // [N][3] +-length (+ on the function's T+), 0 if none
  std::vector<int32_t> rwg_te;        // [n][4] (T+, its edge, T-, its edge)
  std::vector<double> vals;           // [N][3 points][3 edges][4]: w_q f(r_q), w_q div f
  std::vector<int64_t> pair_rowptr;   // [N+1] triangle pairs needed by the near corrections
  std::vector<int32_t> pair_col;
  std::vector<int32_t> rowptr;        // [n+1] RWG near list, columns ascending
  std::vector<int32_t> col;
  std::vector<double> ca, cphi;       // C_A, C_phi on the RWG near list
  // point projection Lambda_u(r_p) (no weights), p = 3t + q: by grid node
  // (columns = points) and by point (columns = nodes)
  std::vector<int32_t> p_rowptr, p_col, p_blk;
  std::vector<double> p_val;
  std::vector<int32_t> pt_rowptr, pt_col;
  std::vector<double> pt_val;
};
// RWG functions (numbered by their edges' sorted vertex pairs, T+ the
// triangle of lower index), the RWG near list (some triangle of one near
// some triangle of the other), the triangle pairs it needs and the point
// projection; throws AIM_ERR_GEOMETRY for an edge of more than two triangles
void build_efie_tables(const HostTables& t, EfieTables& e, int nthreads);
// C_A and C_phi from the pair values (kEfiePairVals per entry of the pair list)
void assemble_efie_near(const HostTables& t, EfieTables& e, const std::vector<double>& pv,
                        int nthreads);
// RWG double layer (Sec. III-B, eq. KAIMx): on the RWG near list, C_K =
// K_s,NR - K_s,P of K_mn = f_m . (n x K f_n) and the Gram matrix
// G_mn = int f_m . f_n, interleaved as ck [nnz][2], from the pair values
// (kMfiePairVals per entry of the pair list)
void assemble_mfie_near(const HostTables& t, const EfieTables& e, const std::vector<double>& pv,
                        std::vector<double>& ck, int nthreads);

// Closed-form integral of 1/|r - r'| over the triangle (a, b, c).
double triangle_inv_r(const double r[3], const double a[3], const double b[3],
                      const double c[3]);

// ---------------------------------------------------------------------------
// device launch wrappers (kernels.hip).  Complex data is interleaved.
// ---------------------------------------------------------------------------
struct GridShape {
  int N[3];      // unpadded dims
  int M[3];      // padded dims (2N)
  int64_t Ng;    // N0 N1 N2
  int64_t Nfold; // (N0+1)(N1+1)(N2+1)
};

struct CsrDevice {
  const int32_t* rowptr;  // [N+1]
  const int32_t* col;     // [nnz]
  const void* val;        // [nnz] T
  int64_t n;
};

// q = P x over row blocks of P (each block holds at most kProjNnz non-zeros
// and kProjRows rows, or is one longer row on its own, or is a run of empty
// rows)
constexpr int kProjNnz = 1024;
constexpr int kProjRows = 512;
constexpr int kProjZeroRows = 16384;  // rows of a block that only writes zeros
template <typename T>
void launch_project(const GridShape& g, const CsrDevice& P, const int32_t* blk, int nblk,
                    const void* x, int64_t n, void* q, int nrhs, hipStream_t s);

// Forward pruned 3-D FFT (unpadded q -> half-spectrum working grid), spectral
// multiply, inverse pruned FFT (-> unpadded phi).  work must hold 4 Ng complex
// per right-hand side; q and phi may alias.
// sched[5] selects the launch shape of the x-forward, y-forward, z, y-inverse
// and x-inverse passes (NULL: shape 0 everywhere).
constexpr int kFftVariants = AIM_FFT_SHAPES;
// shapes below this serve every pass (one set of lines per workgroup); the
// rest are persistent shapes of the fused z pass
constexpr int kFftShapesPerLine = 8;
// schedule = launch shape of each of the five FFT passes, the work layout,
// and the stage modes: bit 0 the interpolation (0: assembled P^T, 1:
// recomputed weights), bit 1 the projection fused into the x forward pass
constexpr int kSchedLen = 7;
constexpr int kModeImplicitInterp = 1, kModeFusedProject = 2;
constexpr int kLayouts = AIM_FFT_LAYOUTS;
// bytes added to every z plane of the convolution work grid, per layout
constexpr int64_t kLayoutPadBytes[kLayouts] = {0, 1024, 4096, 12288};
// complex elements of convolution workspace per right-hand side
int64_t work_elems(const GridShape& g, int layout, size_t elem_bytes);
template <typename T>
void launch_convolve(const GridShape& g, const void* q, void* work, void* phi, const void* spec,
                     const int32_t* rhs_freq, int nrhs, const void* const* tw, hipStream_t s,
                     hipEvent_t* between = nullptr,  // 4 events recorded between passes
                     const int* sched = nullptr,
                     int repeat = 1,  // each pass launched this many times (timing only)
                     // with P: q is not read; the x forward pass computes its
                     // lines as q = P x (x [nrhs][n]) itself
                     const CsrDevice* P = nullptr, const void* x = nullptr, int64_t n = 0,
                     // bit 0: the forward x and y passes (q -> work), bit 1:
                     // the fused z pass, bit 2: the inverse y and x passes
                     // (work -> phi)
                     int stages = 7);
// The double layers' z pass (Sec. III-B): for nvec vectors, three channels'
// forward-transformed grids in work_in (channel c of vector r is workspace
// grid c nvec + r), their spectral products with the gradient spectra spec3
// ([freq][3][Nfold], from launch_spectrum kinds 2-4) -- dot false: the cross
// product K x J (three grids), dot true: the sum -(K . q) (one grid, channel
// 0) -- transformed back into work_out (may equal work_in); the
// launch_convolve stages 1 before and 4 after it complete the product.
template <typename T>
void launch_zcross(const GridShape& g, const void* work_in, void* work_out, const void* spec3,
                   const int32_t* vec_freq, int nvec, const void* const* tw, hipStream_t s,
                   const int* sched, bool dot = false);
// whether launch shape v exists for FFT pass `pass` (0 x forward, 1 y
// forward, 2 fused z, 3 y inverse, 4 x inverse) of the grid g
bool fft_variant_ok(bool dbl, const GridShape& g, int pass, int v);

// y += Cc x with a complex CSR matrix (values complex128 or complex64 like
// the vectors): the near correction of the conventional AIM
template <typename T>
void launch_near_complex(const int32_t* rowptr, const int32_t* col, const void* val,
                         const void* x, void* y, int64_t n, int nrhs, hipStream_t s);
// y = P^T phi + C x: rows of P^T (by triangle) and of C, one group of lanes
// per triangle
// quadrature-point stencil records (implicit interpolation)
struct QpDevice {
  const int32_t* origin;  // [3N] grid index of the stencil's first node
  const void* local;      // [3N][3] t - s per axis (T)
  const void* w;          // [3N] quadrature weights (T)
  int order;
};

// y = P^T phi (+ C x) with the weights of P^T recomputed from the points
template <typename T>
void launch_interp_implicit(const GridShape& g, const QpDevice& qp, const CsrDevice& csr,
                            const void* phi, const void* x, void* y, int nrhs, bool do_near,
                            hipStream_t s);

template <typename T>
void launch_interp_near(const GridShape& g, const CsrDevice& Pt, const CsrDevice& csr,
                        const void* phi, const void* x, void* y, int nrhs, bool do_interp,
                        bool do_near, hipStream_t s);

// Kernel spectrum for one wavenumber: fills the folded, scaled spectrum
// (complex128) and optionally its complex64 rounding.  kind 0: the grid
// kernel G(k, R) with self term -jk/(4 pi); kind 1: the radial factor
// F(R) = h (1 + jkR) e^{-jkR} / (4 pi R^3) of the double layer's gradient
// channels (dG/dr'_a = (u_a - v_a) F), 0 at the origin; kinds 2, 3, 4: the
// component x, y, z of the gradient with respect to the observation point,
// -(u_a - v_a) F (odd along axis a; its folded spectrum is zero at the
// frequencies 0 and N of that axis).
void launch_spectrum(const GridShape& g, double k, double h, void* full_work, void* spec64,
                     void* spec32, const void* const* tw64, hipStream_t s, int kind = 0);
// double-layer operator, complex128: xs[a][r] = n_a x[r] (three channels,
// projected to grids a nrhs + r, then convolved and summed by launch_zcross
// with dot true)
void launch_dlp_sources(const void* x, const double* nrm, void* xs, int64_t n, int nrhs,
                        hipStream_t s);

// RWG EFIE, complex128 (T = double) or complex64 (T = float): src[c][r][3t + q] = sum_e vals[t][q][e][c] x[r][tri_rwg[t][e]]
// (c = x, y, z, charge; x is [nrhs][nrwg]); then, from the interpolated
// channel potentials psi (same layout), y[r][n] = sum over the function's
// two triangles and their points of the current channels' dot product minus
// k_r^-2 times the charge channel, plus (C_A - k_r^-2 C_phi) x[r], with
// k_r = kv[rhs_freq[r]] and cc [nnz][2] = (C_A, C_phi) interleaved
template <typename T>
void launch_efie_sources(const void* x, const void* vals, const int32_t* tri_rwg, void* src,
                         int64_t N, int64_t nrwg, int nrhs, hipStream_t s);
// RWG double layer: the three current channels of x at the points
// (src[a][r][p], as launch_efie_sources without the charge); their grids'
// field V = grad G x J is one spectral cross product (launch_zcross)
template <typename T>
void launch_mfie_sources(const void* x, const void* vals, const int32_t* tri_rwg, void* src,
                         int64_t N, int64_t nrwg, int nrhs, hipStream_t s);
// y for the EFIE (efie), the double layer (mfie) or the combined field of
// eq. CFIEAIMx (both: y = y_E + (j/k_r) y_M), from psi_e [4][nrhs][3N] and
// psi_m [3][nrhs][3N]; cc = (C_A, C_phi), ck = (C_K, G) interleaved; T the
// real type of every array but kv (wavenumbers, double)
template <typename T>
void launch_rwg_test(bool efie, bool mfie, const void* psi_e, const void* psi_m,
                     const void* vals, const void* nrm, const int32_t* rwg_te,
                     const int32_t* rowptr, const int32_t* col, const void* cc, const void* ck,
                     double beta, const double* kv, const int32_t* rhs_freq, const void* x,
                     void* y, int64_t N, int64_t nrwg, int nrhs, hipStream_t s);

// plane waves tested with the RWG functions (3-point rule): b[r][m] =
// <f_m, pol_r e^{-j k d_r . r}> (field 0) or <f_m, n x (d_r x pol_r)
// e^{-j k d_r . r}> (field 1), prm [nrhs][6] = (unit d, pol) on the device
void launch_rwg_plane_wave(const double* qp, const double* vals, const double* nrm,
                           const int32_t* rwg_te, const double* prm, const double* kv,
                           const int32_t* rhs_freq, int field, void* b, int64_t nrwg, int nrhs,
                           hipStream_t s);

void launch_excitation(int kind, const double* qp_xyz, const double* qp_w, int64_t n,
                       const double* params, int n_params, const double* kvals,
                       const int32_t* rhs_freq, int nrhs, void* b, hipStream_t s);

// GMRES state of one system in a restart cycle (device, givens_step)
struct GivensState {
  int len;        // columns of H in use this cycle
  int frozen;     // 1: takes no more steps this cycle
  int iters;      // Krylov steps over the whole solve
  int nonfinite;  // 1: a non-finite basis norm was met
};
// Krylov helpers on complex128 [nrhs][n] vectors; vector i of system r in a
// basis block starts at base + (i * si + r * sr) * n.  With gst (device, may
// be null) the helpers skip the systems whose state is frozen: the dots and
// norms of those are 0, their vectors are left as they are.
void launch_cast_c128_to_c64(const void* in, void* out, int64_t count, hipStream_t s);
void launch_cast_c64_to_c128(const void* in, void* out, int64_t count, hipStream_t s);
void launch_norms(const void* w, int64_t n, int nrhs, void* partial, double* out, hipStream_t s,
                  const GivensState* gst = nullptr);
// One Arnoldi step without reduction launches: the partials of
// conj(V_i,r) . w[r] over chunks of positions (launch_block_dot_partials)
// feed the Gram-Schmidt update w[r] -= sum_i h[r][i] V_i,r directly
// (launch_gs_update, which also stores h in h_out[r][i]), and the norm
// partials (launch_norm_partials) feed the scaling w[r] / ||w[r]|| directly
// (launch_scale_norm, which also stores the norms in nrm_out); partials are
// summed in chunk order (deterministic).  rows (device, may be null): system
// r uses only its first rows[r] <= n entries (the systems of a batch of
// uneven geometries, padded to n); the rest of its vectors is neither read
// nor written.
void launch_block_dot_partials(const void* V, int64_t si, int64_t sr, const void* w, int64_t n,
                               int nv, int nrhs, void* partial, hipStream_t s,
                               const GivensState* gst = nullptr, const int32_t* rows = nullptr);
void launch_gs_update(const void* V, int64_t si, int64_t sr, void* w, int64_t n, int nv, int nrhs,
                      const void* partial, void* h_out, hipStream_t s,
                      const GivensState* gst = nullptr, const int32_t* rows = nullptr);
void launch_norm_partials(const void* w, int64_t n, int nrhs, void* partial, hipStream_t s,
                          const GivensState* gst = nullptr, const int32_t* rows = nullptr);
void launch_scale_norm(const void* w, const void* partial, double* nrm_out, void* out, int64_t n,
                       int nrhs, int64_t out_stride, hipStream_t s,
                       const GivensState* gst = nullptr, const int32_t* rows = nullptr);
// out[r] = w[r] * (1 / nrm[r]) (0 if nrm == 0)
void launch_scale_inv(const void* w, const double* nrm, void* out, int64_t n, int nrhs,
                      int64_t out_stride, hipStream_t s, const GivensState* gst = nullptr,
                      const int32_t* rows = nullptr);
// One Arnoldi step's Hessenberg column, Givens rotation and residual estimate
// for every system (see givens_step_kernel)
void launch_givens_step(const void* h, const void* h2, const double* nrm, int nrhs, int j,
                        int mcap, void* H, void* cs, void* sn, void* g, GivensState* st,
                        const double* scale, double tol, int max_iter, hipStream_t s);
// x[r] += sum_{i < len_r} y[r][i] Z_i,r with len_r the system's basis length
// in st (at most nv), over the first rows[r] entries (all n if rows is null)
void launch_combine(const void* Z, int64_t si, int64_t sr, const void* y, int64_t ldy, int nv,
                    void* x, int64_t n, int nrhs, const GivensState* st, hipStream_t s,
                    const int32_t* rows = nullptr);
// r = b - r   (in place on r)
void launch_residual(const void* b, void* r, int64_t count, hipStream_t s);
void launch_axpy_inplace(void* x, const void* d, int64_t count, hipStream_t s);
void launch_diag_pc(const void* v, const double* dinv, void* z, int64_t n, int nrhs,
                    hipStream_t s);
void launch_block_pc(const void* v, void* z, const int32_t* cl_ptr, const int32_t* cl_perm,
                     const int64_t* cl_blk, const double* cl_inv, int ncl, int max_cl,
                     int64_t n, int nrhs, hipStream_t s);
// the same with complex128 block inverses, one set per wavenumber
// (freq_stride values apart), vector r taking the set rhs_freq[r] (device)
void launch_block_pc_complex(const void* v, void* z, const int32_t* cl_ptr,
                             const int32_t* cl_perm, const int64_t* cl_blk, const void* cl_inv,
                             int64_t freq_stride, const int32_t* rhs_freq, int ncl, int max_cl,
                             int64_t n, int nrhs, hipStream_t s);
// gather/scatter of whole right-hand-side rows: dst[r] = src[idx[r]] (or reverse)
void launch_gather_rows(const void* src, void* dst, const int32_t* idx, int64_t n, int nrhs,
                        bool scatter, hipStream_t s);

// learned-preconditioner glue
void launch_inv_norms_c64(const void* x, int64_t n, int nrhs, double mul, void* partial, double* s,
                          hipStream_t st);
void launch_inv_norms_c128(const void* v, int64_t n, int nrhs, double mul, void* partial,
                           double* s, hipStream_t st);
void launch_scale_cast_c64(const void* v, const double* s, void* out, int64_t n, int nrhs,
                           hipStream_t st);
void launch_scale_c64(void* x, const double* s, int64_t n, int nrhs, hipStream_t st);
// z += tau c / (area sv)   (z = base preconditioner applied to v on entry)
void launch_unet_combine(const void* c, const double* area, double tau, const double* sv, void* z,
                         int64_t n, int nrhs, hipStream_t st);
// w = (e - w) ir           (w = base preconditioner applied to r on entry)
void launch_unet_resid_target(const void* e, const double* ir, void* w, int64_t n, int nrhs,
                              hipStream_t st);
void launch_mesh_mse(const void* c, const void* w, const double* area, double inv_tau, int64_t n,
                     double inv_cnt, void* d, double* part, int nparts, hipStream_t st);
// out = tau c / area (complex64, one vector)
void launch_area_scale_c64(const void* c, const double* area, double tau, void* out, int64_t n,
                           hipStream_t st);
// rho = s - az; part[b] = partial sums of wgt |rho|^2; out = conj(rho)
void launch_resid_loss(const void* az, const void* sv, double wgt, int64_t n, void* out,
                       double* part, int nparts, hipStream_t st);
// d = coef conj(y) / area
void launch_resid_grad(const void* y, const double* area, double coef, void* d, int64_t n,
                       hipStream_t st);
// zero n 8-byte words
void launch_zero_words(void* p, int64_t n, hipStream_t st);
// y[r] += k_{f_r}^2 D x[r] (the linear-term modification), f_r = rhs_freq[r]
template <typename T>
void launch_lin_term(const double* D, const double* k, const int32_t* rhs_freq, const void* x,
                     void* y, int64_t n, int nrhs, hipStream_t s);
// bytes of the fixed device array behind the no-allocation matvec
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
// device address of that array on the current device (looked up once per
// device with it current); throws on failure
void* static_scratch();
// n complex values (complex128 if dbl, else complex64) of a fixed pseudo-random
// pattern, modulus <= 1 (timing input)
void launch_pattern(void* p, int64_t n, bool dbl, hipStream_t st);
// e = xs - e (one vector)
void launch_pair_error(const void* xs, void* e, int64_t n, hipStream_t st);
// nb samples of D x H x W, stored one after another (stacked along z)
void unet_forward(aim_unet u, const void* in, int nb, int D, int H, int W, void* out,
                  hipStream_t s);
void unet_backward(aim_unet u, const void* in, const void* dout, hipStream_t s);
void unet_zero_grad(aim_unet u, hipStream_t s);
void unet_adam(aim_unet u, double lr, hipStream_t s);

// Near-field tables on the device (nearfield.hip).  Uploads the geometry and
// the near list once; fills the static near entries A_s,NR and the AIMx
// correction C = A_s,NR - A_s,P (copied back to the host), and, per
// wavenumber, the complex correction A_NR(k) - A_P(k) of the conventional
// AIM into a caller's device buffer of nnz complex128 values.  V and T may be
// null when only the conventional fill is wanted (after set_static).
class NearDevice {
 public:
  NearDevice(const HostTables& t, const double* V, const int32_t* T, aim_alloc_fn alloc,
             aim_free_fn free_fn, void* ctx, hipStream_t s);
  ~NearDevice();
  NearDevice(const NearDevice&) = delete;
  NearDevice& operator=(const NearDevice&) = delete;
  // also the diagonal of the linear-term modification (lin_diag, N values)
  void fill_static(std::vector<double>& near_static, std::vector<double>& corr,
                   std::vector<double>& lin_diag, hipStream_t s);
  void set_static(const std::vector<double>& near_static, hipStream_t s);
  void fill_conventional(double k, void* out_dev, hipStream_t s);
  // double-layer operator (Sec. III-B): K_s,NR and C_K = K_s,NR - K_s,P on
  // the near list, for the unit normals nrm [N][3]
  void fill_dlp(const std::vector<double>& nrm, std::vector<double>& near_out,
                std::vector<double>& corr_out, hipStream_t s);
  // RWG operators: per triangle pair of the CSR list (rowptr [N+1], col),
  // kEfiePairVals values (kind 0, the EFIE) or kMfiePairVals (kind 1, the
  // double layer), see EfieTables and assemble_mfie_near
  void fill_rwg_pairs(int kind, const std::vector<int64_t>& rowptr,
                      const std::vector<int32_t>& col, std::vector<double>& out, hipStream_t s);
  // inverses of the clusters' blocks of the full-kernel Galerkin matrix at
  // wavenumber k (complex128, row-major, at cl_blk offsets; device arrays);
  // throws AIM_ERR_GEOMETRY for a singular block
  void fill_cluster_inverses(double k, const int32_t* cl_ptr, const int32_t* cl_perm,
                             const int64_t* cl_blk, int ncl, int max_cluster, void* out_dev,
                             hipStream_t s);
  int64_t nnz() const { return nnz_; }

 private:
  void* get(size_t bytes);
  void release();
  int64_t N_, nnz_;
  int order_;
  double h_;
  aim_alloc_fn alloc_;
  aim_free_fn free_;
  void* ctx_;
  hipStream_t stream_;
  std::vector<void*> bufs_;
  void *tri_ = nullptr, *qp_ = nullptr, *qw_ = nullptr, *qstart_ = nullptr, *qlocal_ = nullptr,
       *rowptr_ = nullptr, *col_ = nullptr, *static_ = nullptr;
  bool have_static_ = false;
};

// Twiddle table exp(-2 pi i m / L), m < L, in complex128 (and complex64).
std::vector<double> twiddles64(int L);

}  // namespace aim
