// C ABI of the AIMx library: plan life cycle, the matvec schedule and the
// batched (flexible) GMRES / iterative-refinement driver.
//
// One plan owns the frequency-independent tables of a geometry (quadrature
// points and stencils, projection bricks, the real CSR correction C, the
// preconditioner data) and one kernel spectrum per wavenumber of the sweep.
// Only the spectrum changes with frequency, which is the point of AIMx
// (Sec. III-A: the static near field is integrated once and reused at every
// frequency).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <functional>
#include <random>
#include <cstring>
#include <fstream>
#include <iterator>
#include <memory>
#include <string>
#include <vector>

#include "aim_internal.h"

using aim::Error;

struct aim_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~aim_graph_s() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

namespace {
thread_local std::string g_last_error;
}  // namespace

namespace aim {
void set_last_error(const std::string& m) { g_last_error = m; }
}  // namespace aim

namespace {

aim_status fail(aim_status s, const std::string& m) {
  g_last_error = m;
  return s;
}

template <typename F>
aim_status guarded(F&& f) {
  try {
    f();
    g_last_error.clear();
    return AIM_OK;
  } catch (const Error& e) {
    return fail(e.status, e.what());
  } catch (const std::bad_alloc&) {
    return fail(AIM_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(AIM_ERR_DEVICE, e.what());
  } catch (...) {
    return fail(AIM_ERR_DEVICE, "unknown error");
  }
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
}  // namespace

struct aim_plan_s {
  aim::HostTables t;
  aim::GridShape g{};
  int nfreq = 0;
  std::vector<double> k;
  uint32_t prec = 0;
  int max_rhs = 1;
  aim_alloc_fn alloc = nullptr;
  aim_free_fn free_fn = nullptr;
  void* actx = nullptr;
  hipStream_t setup_stream = nullptr;
  std::vector<std::pair<void*, size_t>> owned;
  int64_t device_bytes = 0;
  double spectra_seconds = 0.0;
  bool host_only = false;

  // device tables
  double* d_w64 = nullptr;     // quadrature weights (excitation, implicit interpolation)
  double* d_qpxyz = nullptr;   // quadrature points (excitation)
  float* d_w32 = nullptr;
  int32_t* d_qporigin = nullptr;  // grid index of each point's first stencil node
  double* d_qplocal64 = nullptr;  // [3N][3] local stencil coordinates
  float* d_qplocal32 = nullptr;
  int32_t* d_pblk = nullptr;   // row blocks of P
  int nblk = 0;
  int32_t* d_prow = nullptr;   // P by grid node
  int32_t* d_pcol = nullptr;
  double* d_pval64 = nullptr;
  float* d_pval32 = nullptr;
  int32_t* d_ptrow = nullptr;  // P^T by triangle
  int32_t* d_ptcol = nullptr;
  double* d_ptval64 = nullptr;
  float* d_ptval32 = nullptr;
  bool near_on_device = false;  // A_s,NR and C computed by the device fill
  int32_t* d_rowptr = nullptr;
  int32_t* d_col = nullptr;
  double* d_val64 = nullptr;
  float* d_val32 = nullptr;
  double* d_dinv = nullptr;
  int32_t* d_clptr = nullptr;
  int32_t* d_clperm = nullptr;
  int64_t* d_clblk = nullptr;
  double* d_clinv = nullptr;
  int ncl = 0, maxcl = 0;
  void* d_spec64 = nullptr;
  void* d_spec32 = nullptr;
  void* d_tw64[3] = {nullptr, nullptr, nullptr};
  void* d_tw32[3] = {nullptr, nullptr, nullptr};
  double* d_k = nullptr;
  double* d_lin = nullptr;               // linear-term diagonal D (may be absent)
  bool lin_on = false;                   // matvecs add k^2 D x
  double* d_area = nullptr;              // triangle areas (learned preconditioner)
  // learned preconditioner (not owned) and its buffers
  // batch of geometries (aim_setup_batch): instance i owns system i, whose
  // vectors are the first N_i entries of a row of length t.N = max N_i
  bool batch = false;
  std::vector<std::unique_ptr<aim_plan_s>> inst;
  int32_t* d_inst_rows = nullptr;  // [instances] N_i: the Krylov kernels skip the padding
  // worker streams of a batch plan: the instances' matvecs and
  // preconditioner applications run on them concurrently (default priority)
  std::vector<hipStream_t> workers;
  hipEvent_t fork_ev = nullptr;
  std::vector<hipEvent_t> join_ev;
  aim_unet unet = nullptr;
  aim_pc_kind unet_base = AIM_PC_DIAG;
  double unet_tau = 1.0;
  void *ug_in = nullptr, *ug_out = nullptr, *um1 = nullptr, *um2 = nullptr, *upart = nullptr;
  void* ug_x = nullptr;  // training: the selected input grids, stacked
  double* u_s = nullptr;
  double* u_s2 = nullptr;
  void* d_work[2] = {nullptr, nullptr};  // [prec] 6 Ng per rhs
  void* d_grid[2] = {nullptr, nullptr};  // [prec] Ng per rhs
  // FFT launch shapes, workspace layout and interpolation mode per precision
  int sched[2][aim::kSchedLen] = {{0, 0, 0, 0, 0, 0, 0}, {0, 0, 0, 0, 0, 0, 0}};
  int32_t* d_rhs_freq = nullptr;          // [max_rhs]
  int32_t* h_rhs_freq = nullptr;          // pinned staging
  std::vector<int32_t> cur_freq;          // what d_rhs_freq holds
  // conventional AIM (aim_conventional_fill): complex near correction of
  // wavenumber conv_freq, complex128 and complex64 copies
  std::unique_ptr<aim::NearDevice> conv_nd;
  // near-block preconditioner: complex128 inverses of the clusters'
  // full-kernel blocks, one set per wavenumber (built on first use)
  void* d_clinv_k = nullptr;
  std::vector<char> clinv_built;
  void* d_conv64 = nullptr;
  void* d_conv32 = nullptr;
  int conv_freq = -1;
  // double-layer operator (aim_matvec_dlp), built on first use
  bool dlp_ready = false;
  double* d_dlp_nrm = nullptr;     // [N][3] unit normals
  double* d_dlp_corr = nullptr;    // [nnz] C_K = K_s,NR - K_s,P on the near list
  void* d_dlp_src = nullptr;       // [3 max_rhs][N] channel sources n_a x
  void* d_dlp_grid = nullptr;      // [3 max_rhs][Ng] channel grids
  void* d_dlp_work = nullptr;      // convolution workspace of 3 max_rhs grids
  void* d_dlp_phi = nullptr;       // [max_rhs][Ng] combined potential
  int32_t* d_dlp_freq = nullptr;   // [4 max_rhs] spectrum index per grid
  int32_t* h_dlp_freq = nullptr;   // pinned staging
  std::vector<int32_t> dlp_cur_freq;
  std::vector<double> dlp_near, dlp_corr;  // host copies (aim_dlp_export)
  double dlp_seconds = 0.0;
  // RWG EFIE (aim_efie_setup, aim_matvec_efie), built on first use
  int host_threads = 1;            // set-up threads of the descriptor
  bool efie_ready = false;
  aim::EfieTables efie;            // host tables (aim_efie_export)
  double* d_efie_vals = nullptr;   // [N][3][3][4] channel values at the points
  int32_t* d_efie_trirwg = nullptr;
  int32_t* d_efie_te = nullptr;    // [n][4]
  int32_t* d_efie_rowptr = nullptr;
  int32_t* d_efie_col = nullptr;
  double* d_efie_cc = nullptr;     // [nnz][2] (C_A, C_phi)
  aim::CsrDevice efie_p{}, efie_pt{};  // point projection by node / by point
  int32_t* d_efie_pblk = nullptr;
  int efie_nblk = 0;
  void* d_efie_src = nullptr;      // [4 max_rhs][3N] point sources, then potentials
  void* d_efie_grid = nullptr;     // [4 max_rhs][Ng]
  void* d_efie_work = nullptr;     // convolution workspace of 4 max_rhs grids
  int32_t* d_efie_freq = nullptr;  // [4 max_rhs] spectrum index per grid
  int32_t* h_efie_freq = nullptr;  // pinned staging
  std::vector<int32_t> efie_cur_freq;
  double efie_seconds = 0.0;
  // RWG double layer (aim_matvec_mfie), built on first use on the EFIE's tables
  bool mfie_ready = false;
  std::vector<double> mfie_ck;      // [nnz][2] (C_K, Gram) on the RWG near list
  double* d_mfie_ck = nullptr;
  double* d_mfie_nrm = nullptr;     // [N][3] unit normals
  void* d_mfie_grid = nullptr;      // [3 max_rhs][Ng] currents, then the field
  void* d_mfie_work = nullptr;      // convolution workspace of 3 max_rhs grids
  void* d_curl_spec = nullptr;      // [nfreq][3] folded spectra of the components of grad G
  void* d_curl_spec32 = nullptr;    // their complex64 rounding
  int32_t* d_mfie_freq = nullptr;   // [6 max_rhs]
  int32_t* h_mfie_freq = nullptr;   // pinned staging
  void* d_cfie_psi = nullptr;       // [3 max_rhs][3N] the double layer's field (combined call)
  // complex64 copies of the RWG tables (plans with complex64 tables)
  float* d_efie_vals32 = nullptr;
  float* d_efie_cc32 = nullptr;
  float* d_mfie_ck32 = nullptr;
  float* d_mfie_nrm32 = nullptr;
  aim::CsrDevice efie_p32{}, efie_pt32{};
  // the operator the Krylov solver applies: 0 the plan's scalar operator,
  // else an RWG operator (aim_solve_rwg sets it for the duration of a solve)
  int rwg_op = 0;
  double rwg_gram = 0.0;
  std::vector<int32_t> rwg_fr;      // per-vector wavenumber index of that solve
  std::vector<int32_t> mfie_cur_freq;
  double mfie_seconds = 0.0;

  // captured matvec graphs used by the solver, keyed by (prec, nrhs, in, out, freq)
  struct GraphKey {
    int prec, nrhs;
    const void* in;
    void* out;
    std::vector<int32_t> freq;
  };
  std::vector<std::pair<GraphKey, std::unique_ptr<aim_graph_s>>> graphs;

  // solver workspace (grown on demand)
  struct Solver {
    int nrhs = 0, m = 0;
    int64_t n = 0;
    void *V = nullptr, *Z = nullptr, *w = nullptr, *r = nullptr, *d = nullptr, *bp = nullptr,
         *xp = nullptr, *h = nullptr, *h2 = nullptr, *y = nullptr, *partial = nullptr,
         *c64a = nullptr, *c64b = nullptr, *ain = nullptr;
    double* nrm = nullptr;
    int32_t* idx = nullptr;
    int32_t* freq = nullptr;
    double* nrm_host = nullptr;  // pinned
    // device-side Givens state of a restart cycle (givens_step) and its
    // pinned host mirrors
    void *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr;
    aim::GivensState* gst = nullptr;
    double* scale = nullptr;
    double2* H_host = nullptr;
    double2* g_host = nullptr;
    aim::GivensState* gst_host = nullptr;
    double* scale_host = nullptr;
  } sv;

  void* dalloc(size_t bytes, hipStream_t s) {
    if (bytes == 0) bytes = 256;
    void* p = nullptr;
    if (alloc) {
      p = alloc(bytes, s, actx);
      AIM_REQUIRE(p != nullptr, AIM_ERR_OOM, "device allocator returned NULL");
    } else {
      const hipError_t e = hipMalloc(&p, bytes);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error(AIM_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
      }
    }
    owned.push_back({p, bytes});
    device_bytes += int64_t(bytes);
    return p;
  }
  template <typename T>
  T* upload(const std::vector<T>& v, hipStream_t s) {
    T* p = static_cast<T*>(dalloc(v.size() * sizeof(T), s));
    if (!v.empty()) AIM_HIP(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return p;
  }
  ~aim_plan_s() {
    if (host_only) return;
    graphs.clear();
    conv_nd.reset();
    if (setup_stream) (void)hipStreamSynchronize(setup_stream);
    (void)hipDeviceSynchronize();
    for (auto& o : owned) {
      if (alloc)
        free_fn(o.first, nullptr, actx);
      else
        (void)hipFree(o.first);
    }
    for (hipStream_t w : workers) (void)hipStreamSynchronize(w);
    for (hipEvent_t e : join_ev) (void)hipEventDestroy(e);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    for (hipStream_t w : workers) (void)hipStreamDestroy(w);
    if (h_rhs_freq) (void)hipHostFree(h_rhs_freq);
    if (h_dlp_freq) (void)hipHostFree(h_dlp_freq);
    if (h_efie_freq) (void)hipHostFree(h_efie_freq);
    if (h_mfie_freq) (void)hipHostFree(h_mfie_freq);
    if (sv.nrm_host) (void)hipHostFree(sv.nrm_host);
    if (sv.H_host) (void)hipHostFree(sv.H_host);
    if (sv.g_host) (void)hipHostFree(sv.g_host);
    if (sv.gst_host) (void)hipHostFree(sv.gst_host);
    if (sv.scale_host) (void)hipHostFree(sv.scale_host);
  }
};

namespace {

aim::CsrDevice p_dev(aim_plan p, aim_precision prec) {
  aim::CsrDevice c;
  c.rowptr = p->d_prow;
  c.col = p->d_pcol;
  c.val = prec == AIM_C128 ? static_cast<const void*>(p->d_pval64) : p->d_pval32;
  c.n = p->g.Ng;
  return c;
}

aim::CsrDevice pt_dev(aim_plan p, aim_precision prec) {
  aim::CsrDevice c;
  c.rowptr = p->d_ptrow;
  c.col = p->d_ptcol;
  c.val = prec == AIM_C128 ? static_cast<const void*>(p->d_ptval64) : p->d_ptval32;
  c.n = p->t.N;
  return c;
}

aim::CsrDevice csr_dev(aim_plan p, aim_precision prec) {
  aim::CsrDevice c;
  c.rowptr = p->d_rowptr;
  c.col = p->d_col;
  c.val = prec == AIM_C128 ? static_cast<const void*>(p->d_val64) : p->d_val32;
  c.n = p->t.N;
  return c;
}

aim::QpDevice qp_dev(aim_plan p, aim_precision prec) {
  aim::QpDevice q;
  q.origin = p->d_qporigin;
  q.local = prec == AIM_C128 ? static_cast<const void*>(p->d_qplocal64) : p->d_qplocal32;
  q.w = prec == AIM_C128 ? static_cast<const void*>(p->d_w64) : p->d_w32;
  q.order = p->t.order;
  return q;
}

// y = P^T phi (+ C x) with the plan's interpolation mode for this precision,
// or y = C x alone (do_interp false)
template <typename T>
void interp_near(aim_plan p, aim_precision prec, const void* phi, const void* x, void* y,
                 int nrhs, bool do_interp, bool do_near, hipStream_t s, int mode = -1) {
  if (mode < 0) mode = p->sched[int(prec)][6] & aim::kModeImplicitInterp;
  if (do_interp && mode == 1)
    aim::launch_interp_implicit<T>(p->g, qp_dev(p, prec), csr_dev(p, prec), phi, x, y, nrhs,
                                   do_near, s);
  else
    aim::launch_interp_near<T>(p->g, pt_dev(p, prec), csr_dev(p, prec), phi, x, y, nrhs,
                               do_interp, do_near, s);
}

void no_batch(aim_plan p) {
  AIM_REQUIRE(!p->batch, AIM_ERR_STATE,
              "not available on a batch plan (use the instance plans' own set-up)");
}

void check_prec(aim_plan p, aim_precision prec) {
  AIM_REQUIRE(!p->host_only, AIM_ERR_STATE, "host-only plan has no device data");
  AIM_REQUIRE(prec == AIM_C128 || prec == AIM_C64, AIM_ERR_INVALID_ARG, "bad precision");
  AIM_REQUIRE(p->prec & (1u << prec), AIM_ERR_STATE, "precision not built in this plan");
}

// Makes d_rhs_freq hold freq (uploads only when it changed).
const int32_t* set_freq(aim_plan p, const int32_t* freq_host, int nrhs, hipStream_t s) {
  AIM_REQUIRE(nrhs >= 1 && nrhs <= p->max_rhs, AIM_ERR_INVALID_ARG,
              "nrhs must be in 1..max_rhs (" + std::to_string(p->max_rhs) + ")");
  std::vector<int32_t> want(nrhs, 0);
  if (freq_host)
    for (int r = 0; r < nrhs; ++r) {
      AIM_REQUIRE(freq_host[r] >= 0 && freq_host[r] < p->nfreq, AIM_ERR_INVALID_ARG,
                  "frequency index out of range");
      want[r] = freq_host[r];
    }
  bool same = int(p->cur_freq.size()) >= nrhs;
  for (int r = 0; same && r < nrhs; ++r) same = p->cur_freq[r] == want[r];
  if (!same) {
    AIM_HIP(hipStreamSynchronize(s));  // staging buffer may still feed a copy
    std::memcpy(p->h_rhs_freq, want.data(), nrhs * sizeof(int32_t));
    AIM_HIP(hipMemcpyAsync(p->d_rhs_freq, p->h_rhs_freq, nrhs * sizeof(int32_t),
                           hipMemcpyHostToDevice, s));
    p->cur_freq = want;
  }
  return p->d_rhs_freq;
}

// The matvec schedule: projection, the pruned FFT convolution (five passes),
// then interpolation fused with the near-field correction.  With ev != NULL,
// ev[0..7] are recorded before, between and after the seven kernels.
// With repeat > 1 (timing only) every kernel is launched `repeat` times in a
// row, which leaves garbage in the workspace and y.
// grid and work (both null: the plan's own) hold the projection grid and
// the convolution workspace of nrhs vectors.
// With near false the near correction C x is left out (y = W H P x).
template <typename T>
void matvec_impl(aim_plan p, aim_precision prec, const void* x, void* y, int nrhs,
                 const int32_t* dfreq, hipStream_t s, hipEvent_t* ev, int repeat = 1,
                 void* grid = nullptr, void* work = nullptr, bool near = true) {
  const int pi = int(prec);
  if (!grid) grid = p->d_grid[pi];
  if (!work) work = p->d_work[pi];
  const void* spec = prec == AIM_C128 ? p->d_spec64 : p->d_spec32;
  void* const* tw = prec == AIM_C128 ? p->d_tw64 : p->d_tw32;
  // the projection runs on its own, or inside the x forward pass (stage mode
  // bit 1; its time then counts in that pass)
  const bool fused = (p->sched[pi][6] & aim::kModeFusedProject) != 0;
  const aim::CsrDevice P = p_dev(p, prec);
  if (ev) AIM_HIP(hipEventRecord(ev[0], s));
  for (int r = 0; r < repeat && !fused; ++r)
    aim::launch_project<T>(p->g, P, p->d_pblk, p->nblk, x, p->t.N, grid, nrhs, s);
  if (ev) AIM_HIP(hipEventRecord(ev[1], s));
  aim::launch_convolve<T>(p->g, grid, work, grid, spec, dfreq, nrhs, tw, s,
                          ev ? ev + 2 : nullptr, p->sched[pi], repeat, fused ? &P : nullptr, x,
                          p->t.N);
  if (ev) AIM_HIP(hipEventRecord(ev[6], s));
  for (int r = 0; r < repeat; ++r) interp_near<T>(p, prec, grid, x, y, nrhs, true, near, s);
  if (near && p->lin_on) aim::launch_lin_term<T>(p->d_lin, p->d_k, dfreq, x, y, p->t.N, nrhs, s);
  if (ev) AIM_HIP(hipEventRecord(ev[7], s));
}

// skip (batch plans only, may be null): systems whose product is not
// needed (GMRES systems that have stopped); their rows of y are left as they
// are, and the caller must not read them
// Runs fn(i, stream) for the instances i of a batch plan that are not
// skipped, dealt round robin to the plan's worker streams after the work
// already queued on s and before the work queued on s afterwards (on s
// itself, one after another, while s is being captured into a graph or when
// at most one instance runs).
template <typename F>
void batch_fork(aim_plan p, int n, const char* skip, hipStream_t s, F&& fn) {
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  AIM_HIP(hipStreamIsCapturing(s, &cap));
  int running = 0;
  for (int i = 0; i < n; ++i) running += (skip && skip[i]) ? 0 : 1;
  // one running instance: no fork and join
  if (p->workers.empty() || cap != hipStreamCaptureStatusNone || running <= 1) {
    for (int i = 0; i < n; ++i)
      if (!(skip && skip[i])) fn(i, s);
    return;
  }
  const int W = int(p->workers.size());
  AIM_HIP(hipEventRecord(p->fork_ev, s));
  for (int w = 0; w < W; ++w) AIM_HIP(hipStreamWaitEvent(p->workers[w], p->fork_ev, 0));
  int next = 0;
  for (int i = 0; i < n; ++i) {
    if (skip && skip[i]) continue;
    fn(i, p->workers[next % W]);
    ++next;
  }
  for (int w = 0; w < W; ++w) {
    AIM_HIP(hipEventRecord(p->join_ev[w], p->workers[w]));
    AIM_HIP(hipStreamWaitEvent(s, p->join_ev[w], 0));
  }
}

// pad (batch plans): zero the padding rows of y (the GMRES loop, whose
// Krylov kernels never read them, leaves them as they are)
void matvec_any(aim_plan p, aim_precision prec, const void* x, void* y, int nrhs,
                const int32_t* dfreq, hipStream_t s, hipEvent_t* ev = nullptr,
                const char* skip = nullptr, bool pad = true) {
  if (p->batch) {
    // system i through instance i; the padding of y_i zeroed
    AIM_REQUIRE(nrhs == int(p->inst.size()) && !ev, AIM_ERR_INVALID_ARG,
                "a batch plan applies one system per instance");
    const size_t cb = prec == AIM_C128 ? 16 : 8;
    const int64_t nmax = p->t.N;
    batch_fork(p, nrhs, skip, s, [&](int i, hipStream_t si) {
      aim_plan_s* q = p->inst[i].get();
      const char* xi = static_cast<const char*>(x) + size_t(i) * nmax * cb;
      char* yi = static_cast<char*>(y) + size_t(i) * nmax * cb;
      matvec_any(q, prec, xi, yi, 1, dfreq + i, si);
      if (pad) aim::launch_zero_words(yi + size_t(q->t.N) * cb, (nmax - q->t.N) * int64_t(cb / 8), si);
    });
    return;
  }
  if (prec == AIM_C128)
    matvec_impl<double>(p, prec, x, y, nrhs, dfreq, s, ev);
  else
    matvec_impl<float>(p, prec, x, y, nrhs, dfreq, s, ev);
}

// Captures matvec_any on the given operands into an instantiated graph.
std::unique_ptr<aim_graph_s> capture_matvec(aim_plan p, aim_precision prec, const void* x, void* y,
                                            int nrhs, const int32_t* dfreq, hipStream_t s) {
  // the default (legacy) stream cannot be captured: capture on a private one
  hipStream_t cs = nullptr;
  AIM_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  AIM_HIP(hipStreamSynchronize(s));  // frequency indices uploaded on s are in place
  std::unique_ptr<aim_graph_s> g(new aim_graph_s());
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    try {
      matvec_any(p, prec, x, y, nrhs, dfreq, cs);
    } catch (...) {
      hipGraph_t junk = nullptr;
      (void)hipStreamEndCapture(cs, &junk);
      if (junk) (void)hipGraphDestroy(junk);
      (void)hipStreamDestroy(cs);
      throw;
    }
    e = hipStreamEndCapture(cs, &g->graph);
  }
  (void)hipStreamDestroy(cs);
  AIM_HIP(e);
  AIM_HIP(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
  return g;
}

}  // namespace

// ===========================================================================
extern "C" {

aim_status aim_matvec_capture(aim_plan p, aim_precision prec, const void* x, void* y,
                              int32_t nrhs, const int32_t* freq_idx_host, void* hip_stream,
                              aim_graph* out) {
  if (!p || !x || !y || !out) return fail(AIM_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  return guarded([&] {
    check_prec(p, prec);
    AIM_REQUIRE(x != y, AIM_ERR_INVALID_ARG, "x and y must not overlap");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int32_t* df = set_freq(p, freq_idx_host, nrhs, s);
    *out = capture_matvec(p, prec, x, y, nrhs, df, s).release();
  });
}

aim_status aim_graph_launch(aim_graph g, void* hip_stream) {
  if (!g || !g->exec) return fail(AIM_ERR_INVALID_ARG, "null graph");
  return guarded([&] { AIM_HIP(hipGraphLaunch(g->exec, static_cast<hipStream_t>(hip_stream))); });
}

aim_status aim_graph_destroy(aim_graph g) {
  return guarded([&] { delete g; });
}

const char* aim_last_error(void) { return g_last_error.c_str(); }
const char* aim_version(void) { return "aimx-gfx950 0.1"; }

static void validate_desc(const aim_setup_desc& d) {
    AIM_REQUIRE(d.n_freq >= 1 && d.k != nullptr, AIM_ERR_INVALID_ARG, "need n_freq >= 1 wavenumbers");
    for (int f = 0; f < d.n_freq; ++f)
      AIM_REQUIRE(std::isfinite(d.k[f]) && d.k[f] > 0.0, AIM_ERR_INVALID_ARG,
                  "wavenumbers must be positive and finite");
    AIM_REQUIRE(d.precisions != 0 && (d.precisions & ~3u) == 0, AIM_ERR_INVALID_ARG,
                "precisions must be a non-empty subset of {C128, C64}");
    AIM_REQUIRE(d.max_rhs >= 1 && d.max_rhs <= 65535, AIM_ERR_INVALID_ARG, "max_rhs out of range");
    AIM_REQUIRE((d.alloc == nullptr) == (d.free == nullptr), AIM_ERR_INVALID_ARG,
                "alloc and free must be given together");
}

aim_status aim_setup_host(const aim_setup_desc* desc, aim_plan* out) {
  if (!desc || !out) return fail(AIM_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  std::unique_ptr<aim_plan_s> p(new aim_plan_s());
  p->host_only = true;
  const aim_status st = guarded([&] {
    validate_desc(*desc);
    aim::build_host_tables(*desc, p->t);
    p->nfreq = desc->n_freq;
    p->k.assign(desc->k, desc->k + desc->n_freq);
    p->prec = desc->precisions;
    p->max_rhs = desc->max_rhs;
    for (int a = 0; a < 3; ++a) {
      p->g.N[a] = p->t.dims[a];
      p->g.M[a] = 2 * p->t.dims[a];
    }
    p->g.Ng = int64_t(p->g.N[0]) * p->g.N[1] * p->g.N[2];
    p->g.Nfold = int64_t(p->g.N[0] + 1) * (p->g.N[1] + 1) * (p->g.N[2] + 1);
    p->ncl = int(p->t.cl_ptr.size()) - 1;
    for (int c = 0; c < p->ncl; ++c)
      p->maxcl = std::max(p->maxcl, p->t.cl_ptr[c + 1] - p->t.cl_ptr[c]);
  });
  if (st != AIM_OK) return st;
  *out = p.release();
  return AIM_OK;
}

namespace {
// The static near entries and C on the device (copied back into the host
// tables), then the preconditioner's cluster inverses from them.
void fill_near_device(aim_plan_s* p, const aim_setup_desc& d, hipStream_t s) {
  const double t0 = now_s();
  {
    aim::NearDevice nd(p->t, d.vertices, d.triangles, d.alloc, d.free, d.alloc_ctx, s);
    nd.fill_static(p->t.near_static, p->t.corr, p->t.lin_diag, s);
  }
  p->t.near_seconds = now_s() - t0;
  p->near_on_device = true;
  aim::build_cluster_inverses(p->t, aim::setup_threads(d));
}

// Everything after the host tables: grid shape, uploads, workspace, spectra.
// Shared by aim_setup and aim_plan_load.
void init_device(aim_plan_s* p, hipStream_t hip_stream) {
    auto& g = p->g;
    for (int a = 0; a < 3; ++a) {
      g.N[a] = p->t.dims[a];
      g.M[a] = 2 * p->t.dims[a];
    }
    g.Ng = int64_t(g.N[0]) * g.N[1] * g.N[2];
    g.Nfold = int64_t(g.N[0] + 1) * (g.N[1] + 1) * (g.N[2] + 1);

    hipStream_t s = hip_stream;
    p->setup_stream = s;
    const auto& t = p->t;
    const int64_t N = t.N, Nq = 3 * N;
    // quadrature points (excitation) and the projection matrix in two layouts
    p->d_qpxyz = p->upload(t.qp_xyz, s);
    p->d_w64 = p->upload(t.qp_w, s);
    {
      const int64_t nq = 3 * t.N;
      std::vector<int32_t> org(nq);
      for (int64_t q = 0; q < nq; ++q)
        org[q] = int32_t((int64_t(t.qp_start[3 * q + 2]) * t.dims[1] + t.qp_start[3 * q + 1]) *
                             t.dims[0] + t.qp_start[3 * q]);
      p->d_qporigin = p->upload(org, s);
      p->d_qplocal64 = p->upload(t.qp_local, s);
      if (p->prec & (1u << AIM_C64)) {
        p->d_qplocal32 = p->upload(std::vector<float>(t.qp_local.begin(), t.qp_local.end()), s);
        p->d_w32 = p->upload(std::vector<float>(t.qp_w.begin(), t.qp_w.end()), s);
      }
    }
    p->d_prow = p->upload(t.p_rowptr, s);
    p->d_pblk = p->upload(t.p_blk, s);
    p->nblk = int(t.p_blk.size()) - 1;
    p->d_pcol = p->upload(t.p_col, s);
    p->d_ptrow = p->upload(t.pt_rowptr, s);
    p->d_ptcol = p->upload(t.pt_col, s);
    if (p->prec & (1u << AIM_C128)) {
      p->d_pval64 = p->upload(t.p_val, s);
      p->d_ptval64 = p->upload(t.pt_val, s);
    }
    if (p->prec & (1u << AIM_C64)) {
      std::vector<float> a(t.p_val.begin(), t.p_val.end()), b(t.pt_val.begin(), t.pt_val.end());
      p->d_pval32 = p->upload(a, s);
      p->d_ptval32 = p->upload(b, s);
    }
    std::vector<int32_t> rp32(t.rowptr.begin(), t.rowptr.end());
    p->d_rowptr = p->upload(rp32, s);
    p->d_col = p->upload(t.col, s);
    if (p->prec & (1u << AIM_C128)) p->d_val64 = p->upload(t.corr, s);
    if (p->prec & (1u << AIM_C64)) {
      std::vector<float> v32(t.corr.begin(), t.corr.end());
      p->d_val32 = p->upload(v32, s);
    }
    // preconditioners (complex128 solver side)
    {
      std::vector<double> dinv(N);
      for (int64_t i = 0; i < N; ++i) {
        double dv = 0.0;
        for (int64_t q = t.rowptr[i]; q < t.rowptr[i + 1]; ++q)
          if (t.col[q] == i) dv = t.near_static[q];
        AIM_REQUIRE(dv != 0.0, AIM_ERR_GEOMETRY, "zero static self term");
        dinv[i] = 1.0 / dv;
      }
      p->d_dinv = p->upload(dinv, s);
      p->ncl = int(t.cl_ptr.size()) - 1;
      for (int c = 0; c < p->ncl; ++c) p->maxcl = std::max(p->maxcl, t.cl_ptr[c + 1] - t.cl_ptr[c]);
      p->d_clptr = p->upload(t.cl_ptr, s);
      p->d_clperm = p->upload(t.cl_perm, s);
      p->d_clblk = p->upload(t.cl_blk, s);
      p->d_clinv = p->upload(t.cl_inv, s);
    }
    p->d_k = p->upload(p->k, s);
    if (!t.lin_diag.empty()) p->d_lin = p->upload(t.lin_diag, s);
    p->d_area = p->upload(t.area, s);
    // twiddles per axis
    for (int a = 0; a < 3; ++a) {
      const std::vector<double> tw = aim::twiddles64(g.M[a]);
      p->d_tw64[a] = p->upload(tw, s);
      std::vector<float> tw32(tw.begin(), tw.end());
      p->d_tw32[a] = p->upload(tw32, s);
    }
    // work buffers
    for (int pi = 0; pi < 2; ++pi) {
      if (!(p->prec & (1u << pi))) continue;
      const size_t cb = pi == 0 ? 16 : 8;
      // room for the layout with the largest plane padding
      p->d_work[pi] = p->dalloc(size_t(aim::work_elems(g, aim::kLayouts - 1, cb)) * cb * p->max_rhs,
                                s);
      p->d_grid[pi] = p->dalloc(size_t(g.Ng) * cb * p->max_rhs, s);
    }
    p->d_rhs_freq = static_cast<int32_t*>(p->dalloc(sizeof(int32_t) * p->max_rhs, s));
    AIM_HIP(hipHostMalloc(reinterpret_cast<void**>(&p->h_rhs_freq), sizeof(int32_t) * p->max_rhs, 0));
    // kernel spectra: one per wavenumber, folded (complex128 + complex64)
    const double ts = now_s();
    p->d_spec64 = p->dalloc(size_t(g.Nfold) * 16 * p->nfreq, s);
    if (p->prec & (1u << AIM_C64)) p->d_spec32 = p->dalloc(size_t(g.Nfold) * 8 * p->nfreq, s);
    {
      void* full = nullptr;
      const size_t fb = size_t(8) * g.Ng * 16;
      AIM_HIP(hipMalloc(&full, fb));
      try {
        for (int f = 0; f < p->nfreq; ++f)
          aim::launch_spectrum(g, p->k[f], t.h, full,
                               static_cast<char*>(p->d_spec64) + size_t(f) * g.Nfold * 16,
                               p->d_spec32 ? static_cast<char*>(p->d_spec32) + size_t(f) * g.Nfold * 8
                                           : nullptr,
                               p->d_tw64, s);
        AIM_HIP(hipStreamSynchronize(s));
      } catch (...) {
        (void)hipFree(full);
        throw;
      }
      AIM_HIP(hipFree(full));
    }
    p->spectra_seconds = now_s() - ts;
    AIM_HIP(hipStreamSynchronize(s));
}
}  // namespace

aim_status aim_setup(const aim_setup_desc* desc, void* hip_stream, aim_plan* out) {
  if (!desc || !out) return fail(AIM_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  std::unique_ptr<aim_plan_s> p(new aim_plan_s());
  const aim_status st = guarded([&] {
    const aim_setup_desc& d = *desc;
    validate_desc(d);
    const double t0 = now_s();
    // host work first: every validation happens before any device call
    aim::build_host_tables(d, p->t, false);
    p->nfreq = d.n_freq;
    p->host_threads = aim::setup_threads(d);
    p->k.assign(d.k, d.k + d.n_freq);
    p->prec = d.precisions;
    p->max_rhs = d.max_rhs;
    p->alloc = d.alloc;
    p->free_fn = d.free;
    p->actx = d.alloc_ctx;
    fill_near_device(p.get(), d, static_cast<hipStream_t>(hip_stream));
    init_device(p.get(), static_cast<hipStream_t>(hip_stream));
    p->t.setup_seconds = now_s() - t0;
  });
  if (st != AIM_OK) return st;
  *out = p.release();
  return AIM_OK;
}

aim_status aim_setup_batch(const aim_setup_desc* descs, int32_t n, void* hip_stream,
                           aim_plan* out) {
  if (!descs || !out) return fail(AIM_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (n < 1 || n > 65535) return fail(AIM_ERR_INVALID_ARG, "n must be in 1..65535");
  std::unique_ptr<aim_plan_s> b(new aim_plan_s());
  const aim_status st = guarded([&] {
    const double t0 = now_s();
    // every description is validated and every host table built before any
    // device call
    for (int i = 0; i < n; ++i) {
      validate_desc(descs[i]);
      AIM_REQUIRE((descs[i].alloc == descs[0].alloc) && (descs[i].free == descs[0].free) &&
                      (descs[i].alloc_ctx == descs[0].alloc_ctx),
                  AIM_ERR_INVALID_ARG, "the instances of a batch share one allocator");
    }
    for (int i = 0; i < n; ++i) {
      std::unique_ptr<aim_plan_s> q(new aim_plan_s());
      const aim_setup_desc& d = descs[i];
      aim::build_host_tables(d, q->t, false);
      q->nfreq = d.n_freq;
      q->k.assign(d.k, d.k + d.n_freq);
      q->prec = d.precisions;
      q->max_rhs = 1;
      q->alloc = d.alloc;
      q->free_fn = d.free;
      q->actx = d.alloc_ctx;
      b->inst.push_back(std::move(q));
    }
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    b->batch = true;
    b->alloc = descs[0].alloc;
    b->free_fn = descs[0].free;
    b->actx = descs[0].alloc_ctx;
    b->setup_stream = s;
    b->max_rhs = n;
    b->prec = 3u;
    b->nfreq = 1 << 30;
    b->t.N = 0;
    b->t.order = descs[0].stencil_order;
    for (int i = 0; i < n; ++i) {
      auto& q = b->inst[size_t(i)];
      fill_near_device(q.get(), descs[i], s);
      init_device(q.get(), s);
      b->t.N = std::max(b->t.N, q->t.N);
      b->prec &= q->prec;
      b->nfreq = std::min(b->nfreq, q->nfreq);
      b->device_bytes += q->device_bytes;
    }
    AIM_REQUIRE(b->prec != 0, AIM_ERR_INVALID_ARG, "the instances share no precision");
    b->d_rhs_freq = static_cast<int32_t*>(b->dalloc(sizeof(int32_t) * n, s));
    {
      std::vector<int32_t> rows(n);
      for (int i = 0; i < n; ++i) rows[i] = int32_t(b->inst[size_t(i)]->t.N);
      b->d_inst_rows = b->upload(rows, s);
    }
    // worker streams for the instances' concurrent matvecs (as many as the
    // device has hardware queues by default)
    constexpr int kWorkers = 4;
    for (int w = 0; w < kWorkers && w < n; ++w) {
      hipStream_t ws = nullptr;
      AIM_HIP(hipStreamCreateWithFlags(&ws, hipStreamNonBlocking));
      b->workers.push_back(ws);
      hipEvent_t e = nullptr;
      AIM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      b->join_ev.push_back(e);
    }
    AIM_HIP(hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming));
    AIM_HIP(hipHostMalloc(reinterpret_cast<void**>(&b->h_rhs_freq), sizeof(int32_t) * n, 0));
    AIM_HIP(hipStreamSynchronize(s));
    b->t.setup_seconds = now_s() - t0;
  });
  if (st != AIM_OK) return st;
  *out = b.release();
  return AIM_OK;
}

aim_status aim_batch_sizes(aim_plan p, int32_t* count, int64_t* n_host) {
  if (!p || !count) return fail(AIM_ERR_INVALID_ARG, "null argument");
  return guarded([&] {
    *count = p->batch ? int32_t(p->inst.size()) : 1;
    if (n_host) {
      if (p->batch)
        for (size_t i = 0; i < p->inst.size(); ++i) n_host[i] = p->inst[i]->t.N;
      else
        n_host[0] = p->t.N;
    }
  });
}

aim_status aim_destroy(aim_plan plan) {
  return guarded([&] { delete plan; });
}

aim_status aim_plan_query(aim_plan p, aim_plan_info* info) {
  if (!p || !info) return fail(AIM_ERR_INVALID_ARG, "null argument");
  return guarded([&] {
    aim_plan_info& o = *info;
    o.n = p->t.N;
    o.n_grid = p->g.Ng;
    o.nnz = int64_t(p->t.col.size());
    for (int a = 0; a < 3; ++a) {
      o.dims[a] = p->g.N[a];
      o.origin[a] = p->t.origin[a];
    }
    o.order = p->t.order;
    o.n_freq = p->nfreq;
    o.max_rhs = p->max_rhs;
    o.precisions = p->prec;
    o.h = p->t.h;
    o.setup_seconds = p->t.setup_seconds;
    o.spectra_seconds = p->spectra_seconds;
    o.device_bytes = p->device_bytes;
    o.n_clusters = p->ncl;
    o.max_cluster = p->maxcl;
    o.near_seconds = p->t.near_seconds;
    o.near_on_device = p->near_on_device ? 1 : 0;
    o.reserved = 0;
  });
}

aim_status aim_matvec(aim_plan p, aim_precision prec, const void* x, void* y, int32_t nrhs,
                      const int32_t* freq_idx_host, void* hip_stream) {
  if (!p || !x || !y) return fail(AIM_ERR_INVALID_ARG, "null argument");
  return guarded([&] {
    check_prec(p, prec);
    AIM_REQUIRE(x != y, AIM_ERR_INVALID_ARG, "x and y must not overlap");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int32_t* df = set_freq(p, freq_idx_host, nrhs, s);
    matvec_any(p, prec, x, y, nrhs, df, s);
  });
}

aim_status aim_matvec_static(aim_plan p, aim_precision prec, const void* x, void* y,
                             int32_t nrhs, const int32_t* freq_idx_host, void* hip_stream) {
  if (!p || !x || !y) return fail(AIM_ERR_INVALID_ARG, "null argument");
  return guarded([&] {
    no_batch(p);
    check_prec(p, prec);
    AIM_REQUIRE(x != y, AIM_ERR_INVALID_ARG, "x and y must not overlap");
    AIM_REQUIRE(nrhs >= 1 && nrhs <= p->max_rhs, AIM_ERR_INVALID_ARG,
                "nrhs must be in 1..max_rhs (" + std::to_string(p->max_rhs) + ")");
    // the projection grid, then the convolution workspace in the plan's
    // layout, each starting on a 256-byte boundary
    const int pi = int(prec);
    const size_t cb = prec == AIM_C128 ? 16 : 8;
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t grid_b = up(size_t(p->g.Ng) * cb * nrhs);
    const size_t work_b = up(size_t(aim::work_elems(p->g, p->sched[pi][5], cb)) * cb * nrhs);
    AIM_REQUIRE(grid_b + work_b <= aim::kStaticScratchBytes, AIM_ERR_INVALID_ARG,
                "aim_matvec_static: " + std::to_string(nrhs) + " vectors on this grid need " +
                    std::to_string(grid_b + work_b) + " bytes of scratch; the limit is " +
                    std::to_string(aim::kStaticScratchBytes) + " (use aim_matvec)");
    char* base = static_cast<char*>(aim::static_scratch());
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int32_t* df = set_freq(p, freq_idx_host, nrhs, s);
    // every scratch element is written before it is read (the projection
    // writes all grid nodes, each FFT pass every element the next one
    // reads), so nothing is cleared
    if (prec == AIM_C128)
      matvec_impl<double>(p, prec, x, y, nrhs, df, s, nullptr, 1, base, base + grid_b);
    else
      matvec_impl<float>(p, prec, x, y, nrhs, df, s, nullptr, 1, base, base + grid_b);
  });
}

namespace {
aim::NearDevice& near_device(aim_plan p, hipStream_t s);
}  // namespace

aim_status aim_set_lin_term(aim_plan p, int32_t on) {
  if (!p) return fail(AIM_ERR_INVALID_ARG, "null plan");
  return guarded([&] {
    auto set = [&](aim_plan q) {
      AIM_REQUIRE(!on || q->d_lin != nullptr, AIM_ERR_STATE,
                  "no linear-term diagonal in this plan (computed by the device set-up only)");
      q->lin_on = on != 0;
    };
    if (p->batch)
      for (auto& q : p->inst) set(q.get());
    else
      set(p);
    p->lin_on = on != 0;
  });
}

aim_status aim_export_lin_diag(aim_plan p, double* d_host) {
  if (!p || !d_host) return fail(AIM_ERR_INVALID_ARG, "null argument");
  return guarded([&] {
    no_batch(p);
    AIM_REQUIRE(!p->t.lin_diag.empty(), AIM_ERR_STATE, "no linear-term diagonal in this plan");
    std::copy(p->t.lin_diag.begin(), p->t.lin_diag.end(), d_host);
  });
}

aim_status aim_export_clusters(aim_plan p, int32_t* cl_ptr, int32_t* cl_perm) {
  if (!p || !cl_ptr || !cl_perm) return fail(AIM_ERR_INVALID_ARG, "null argument");
  return guarded([&] {
    no_batch(p);
    std::copy(p->t.cl_ptr.begin(), p->t.cl_ptr.end(), cl_ptr);
    std::copy(p->t.cl_perm.begin(), p->t.cl_perm.end(), cl_perm);
  });
}

aim_status aim_conventional_fill(aim_plan p, int32_t freq_idx, void* hip_stream) {
  if (!p) return fail(AIM_ERR_INVALID_ARG, "null plan");
  return guarded([&] {
    no_batch(p);
    AIM_REQUIRE(!p->host_only, AIM_ERR_STATE, "host-only plan has no device data");
    AIM_REQUIRE(freq_idx >= 0 && freq_idx < p->nfreq, AIM_ERR_INVALID_ARG,
                "frequency index out of range");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int64_t nnz = int64_t(p->t.col.size());
    aim::NearDevice& nd = near_device(p, s);
    if (!p->d_conv64) p->d_conv64 = p->dalloc(size_t(nnz) * 16, s);
    if ((p->prec & (1u << AIM_C64)) && !p->d_conv32) p->d_conv32 = p->dalloc(size_t(nnz) * 8, s);
    p->conv_freq = -1;
    nd.fill_conventional(p->k[freq_idx], p->d_conv64, s);
    if (p->d_conv32) aim::launch_cast_c128_to_c64(p->d_conv64, p->d_conv32, nnz, s);
    p->conv_freq = freq_idx;
  });
}

aim_status aim_matvec_conventional(aim_plan p, aim_precision prec, const void* x, void* y,
                                   int32_t nrhs, void* hip_stream) {
  if (!p || !x || !y) return fail(AIM_ERR_INVALID_ARG, "null argument");
  return guarded([&] {
    no_batch(p);
    check_prec(p, prec);
    AIM_REQUIRE(x != y, AIM_ERR_INVALID_ARG, "x and y must not overlap");
    AIM_REQUIRE(p->conv_freq >= 0, AIM_ERR_STATE,
                "no conventional near correction: call aim_conventional_fill first");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    AIM_REQUIRE(nrhs >= 1 && nrhs <= p->max_rhs, AIM_ERR_INVALID_ARG,
                "nrhs must be in 1..max_rhs (" + std::to_string(p->max_rhs) + ")");
    const std::vector<int32_t> fr(size_t(nrhs), p->conv_freq);
    const int32_t* df = set_freq(p, fr.data(), nrhs, s);
    // W H(k) P x, then the complex near correction of the same wavenumber
    if (prec == AIM_C128) {
      matvec_impl<double>(p, prec, x, y, nrhs, df, s, nullptr, 1, nullptr, nullptr, false);
      aim::launch_near_complex<double>(p->d_rowptr, p->d_col, p->d_conv64, x, y, p->t.N, nrhs, s);
    } else {
      matvec_impl<float>(p, prec, x, y, nrhs, df, s, nullptr, 1, nullptr, nullptr, false);
      aim::launch_near_complex<float>(p->d_rowptr, p->d_col, p->d_conv32, x, y, p->t.N, nrhs, s);
    }
  });
}

namespace {
// The folded spectra of the three components of grad G (Sec. III-B, the
// kernel of eq. KAIMx) for every wavenumber of the plan, [freq][3][Nfold]:
// the RWG double layer's grid operator as one cross product per frequency.
void ensure_curl_spectra(aim_plan p, hipStream_t s) {
  if (p->d_curl_spec) return;
  const auto& g = p->g;
  const size_t n3 = size_t(3) * g.Nfold;
  void* spec = p->dalloc(n3 * 16 * p->nfreq, s);
  void* spec32 = (p->prec & (1u << AIM_C64)) ? p->dalloc(n3 * 8 * p->nfreq, s) : nullptr;
  void* full = nullptr;
  AIM_HIP(hipMalloc(&full, size_t(8) * g.Ng * 16));
  try {
    for (int f = 0; f < p->nfreq; ++f)
      for (int a = 0; a < 3; ++a) {
        const size_t off = size_t(f) * n3 + size_t(a) * g.Nfold;
        aim::launch_spectrum(g, p->k[f], p->t.h, full, static_cast<char*>(spec) + off * 16,
                             spec32 ? static_cast<char*>(spec32) + off * 8 : nullptr, p->d_tw64,
                             s, 2 + a);
      }
    AIM_HIP(hipStreamSynchronize(s));
  } catch (...) {
    (void)hipStreamSynchronize(s);
    (void)hipFree(full);
    throw;
  }
  AIM_HIP(hipFree(full));
  p->d_curl_spec = spec;
  p->d_curl_spec32 = spec32;
}

// The double-layer operator's tables (Sec. III-B): unit normals, C_K on the
// near list (device fill), the folded spectra of grad G for every wavenumber
// of the plan, and the buffers of max_rhs products.
void ensure_dlp(aim_plan p, hipStream_t s) {
  if (p->dlp_ready) return;
  AIM_REQUIRE(p->t.corners.size() == 9 * size_t(p->t.N), AIM_ERR_STATE,
              "the double-layer operator needs the mesh (not kept by loaded plans)");
  const double t0 = now_s();
  const auto& t = p->t;
  const int64_t N = t.N;
  std::vector<double> nrm(3 * size_t(N));
  for (int64_t j = 0; j < N; ++j) {
    const double* c = &t.corners[9 * j];
    const double e1[3] = {c[3] - c[0], c[4] - c[1], c[5] - c[2]};
    const double e2[3] = {c[6] - c[0], c[7] - c[1], c[8] - c[2]};
    const double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                         e1[0] * e2[1] - e1[1] * e2[0]};
    const double l = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    for (int a = 0; a < 3; ++a) nrm[3 * j + a] = n[a] / l;
  }
  {
    aim::NearDevice nd(t, nullptr, nullptr, p->alloc, p->free_fn, p->actx, s);
    nd.fill_dlp(nrm, p->dlp_near, p->dlp_corr, s);
  }
  const auto& g = p->g;
  const int R = p->max_rhs;
  p->d_dlp_nrm = p->upload(nrm, s);
  p->d_dlp_corr = p->upload(p->dlp_corr.empty() ? std::vector<double>(1, 0.0) : p->dlp_corr, s);
  ensure_curl_spectra(p, s);
  p->d_dlp_src = p->dalloc(size_t(3) * R * N * 16, s);
  p->d_dlp_grid = p->dalloc(size_t(3) * R * g.Ng * 16, s);
  p->d_dlp_work = p->dalloc(size_t(aim::work_elems(g, aim::kLayouts - 1, 16)) * 16 * 3 * R, s);
  p->d_dlp_phi = p->dalloc(size_t(R) * g.Ng * 16, s);
  p->d_dlp_freq = static_cast<int32_t*>(p->dalloc(sizeof(int32_t) * R, s));
  AIM_HIP(hipHostMalloc(reinterpret_cast<void**>(&p->h_dlp_freq), sizeof(int32_t) * R, 0));
  p->dlp_cur_freq.clear();
  p->dlp_ready = true;
  p->dlp_seconds = now_s() - t0;
}
}  // namespace

aim_status aim_matvec_dlp(aim_plan p, const void* x, void* y, int32_t nrhs,
                          const int32_t* freq_idx_host, void* hip_stream) {
  if (!p || !x || !y) return fail(AIM_ERR_INVALID_ARG, "null argument");
  return guarded([&] {
    no_batch(p);
    check_prec(p, AIM_C128);
    AIM_REQUIRE(x != y, AIM_ERR_INVALID_ARG, "x and y must not overlap");
    AIM_REQUIRE(nrhs >= 1 && nrhs <= p->max_rhs, AIM_ERR_INVALID_ARG,
                "nrhs must be in 1..max_rhs (" + std::to_string(p->max_rhs) + ")");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    std::vector<int32_t> fr(size_t(nrhs), 0);
    for (int r = 0; r < nrhs; ++r) {
      if (freq_idx_host) {
        AIM_REQUIRE(freq_idx_host[r] >= 0 && freq_idx_host[r] < p->nfreq, AIM_ERR_INVALID_ARG,
                    "frequency index out of range");
        fr[r] = freq_idx_host[r];
      }
    }
    ensure_dlp(p, s);
    // one spectrum index per vector
    if (fr != p->dlp_cur_freq) {
      AIM_HIP(hipStreamSynchronize(s));  // the staging buffer may still feed a copy
      std::memcpy(p->h_dlp_freq, fr.data(), fr.size() * sizeof(int32_t));
      AIM_HIP(hipMemcpyAsync(p->d_dlp_freq, p->h_dlp_freq, fr.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice, s));
      p->dlp_cur_freq = fr;
    }
    // three channels: projection, forward x and y passes, the z pass that
    // sums their products with the gradient spectra into grid r of the
    // workspace, inverse y and x passes of that one grid per vector
    const int64_t N = p->t.N;
    aim::launch_dlp_sources(x, p->d_dlp_nrm, p->d_dlp_src, N, nrhs, s);
    aim::launch_project<double>(p->g, p_dev(p, AIM_C128), p->d_pblk, p->nblk, p->d_dlp_src, N,
                                p->d_dlp_grid, 3 * nrhs, s);
    aim::launch_convolve<double>(p->g, p->d_dlp_grid, p->d_dlp_work, nullptr, nullptr, nullptr,
                                 3 * nrhs, p->d_tw64, s, nullptr, p->sched[0], 1, nullptr,
                                 nullptr, 0, 1);
    aim::launch_zcross<double>(p->g, p->d_dlp_work, p->d_dlp_work, p->d_curl_spec,
                               p->d_dlp_freq, nrhs, p->d_tw64, s, p->sched[0], true);
    aim::launch_convolve<double>(p->g, nullptr, p->d_dlp_work, p->d_dlp_phi, nullptr, nullptr,
                                 nrhs, p->d_tw64, s, nullptr, p->sched[0], 1, nullptr, nullptr,
                                 0, 4);
    aim::CsrDevice kc = csr_dev(p, AIM_C128);
    kc.val = p->d_dlp_corr;
    aim::launch_interp_near<double>(p->g, pt_dev(p, AIM_C128), kc, p->d_dlp_phi, x, y, nrhs,
                                    true, true, s);
  });
}

aim_status aim_dlp_export(aim_plan p, double* near_host, double* corr_host, void* hip_stream) {
  if (!p) return fail(AIM_ERR_INVALID_ARG, "null plan");
  return guarded([&] {
    no_batch(p);
    check_prec(p, AIM_C128);
    ensure_dlp(p, static_cast<hipStream_t>(hip_stream));
    const size_t nnz = p->t.col.size();
    if (near_host && nnz) std::memcpy(near_host, p->dlp_near.data(), nnz * 8);
    if (corr_host && nnz) std::memcpy(corr_host, p->dlp_corr.data(), nnz * 8);
  });
}

namespace {
// The RWG EFIE's tables: functions, near list and point projection on the
// host, the triangle pairs' inner integrals and point precorrections on the
// device, C_A and C_phi assembled on the host, then the uploads and the
// buffers of max_rhs products.
void ensure_efie(aim_plan p, hipStream_t s) {
  if (p->efie_ready) return;
  const double t0 = now_s();
  const auto& t = p->t;
  aim::EfieTables& e = p->efie;
  aim::build_efie_tables(t, e, p->host_threads);
  {
    std::vector<double> pv;
    {
      aim::NearDevice nd(t, nullptr, nullptr, p->alloc, p->free_fn, p->actx, s);
      nd.fill_rwg_pairs(0, e.pair_rowptr, e.pair_col, pv, s);
    }
    aim::assemble_efie_near(t, e, pv, p->host_threads);
  }
  const auto& g = p->g;
  const int R = p->max_rhs;
  const int64_t P = 3 * t.N;
  std::vector<double> nrm(3 * size_t(t.N));
  for (int64_t j = 0; j < t.N; ++j) {
    const double* c = &t.corners[9 * j];
    const double e1[3] = {c[3] - c[0], c[4] - c[1], c[5] - c[2]};
    const double e2[3] = {c[6] - c[0], c[7] - c[1], c[8] - c[2]};
    const double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                         e1[0] * e2[1] - e1[1] * e2[0]};
    const double l = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    for (int a = 0; a < 3; ++a) nrm[3 * j + a] = n[a] / l;
  }
  p->d_mfie_nrm = p->upload(nrm, s);  // unit normals (double layer, excitation)
  p->d_efie_vals = p->upload(e.vals, s);
  p->d_efie_trirwg = p->upload(e.tri_rwg, s);
  p->d_efie_te = p->upload(e.rwg_te.empty() ? std::vector<int32_t>(4, 0) : e.rwg_te, s);
  p->d_efie_rowptr = p->upload(e.rowptr, s);
  p->d_efie_col = p->upload(e.col.empty() ? std::vector<int32_t>(1, 0) : e.col, s);
  {
    std::vector<double> cc(2 * std::max<size_t>(e.ca.size(), 1), 0.0);
    for (size_t j = 0; j < e.ca.size(); ++j) {
      cc[2 * j] = e.ca[j];
      cc[2 * j + 1] = e.cphi[j];
    }
    p->d_efie_cc = p->upload(cc, s);
    AIM_HIP(hipStreamSynchronize(s));  // cc is a temporary
  }
  p->efie_p.rowptr = p->upload(e.p_rowptr, s);
  p->efie_p.col = p->upload(e.p_col, s);
  p->efie_p.val = p->upload(e.p_val, s);
  p->efie_p.n = g.Ng;
  p->d_efie_pblk = p->upload(e.p_blk, s);
  p->efie_nblk = int(e.p_blk.size()) - 1;
  p->efie_pt.rowptr = p->upload(e.pt_rowptr, s);
  p->efie_pt.col = p->upload(e.pt_col, s);
  p->efie_pt.val = p->upload(e.pt_val, s);
  p->efie_pt.n = P;
  if (p->prec & (1u << AIM_C64)) {
    auto f32 = [](const std::vector<double>& v) { return std::vector<float>(v.begin(), v.end()); };
    p->d_efie_vals32 = p->upload(f32(e.vals), s);
    std::vector<float> cc32(2 * std::max<size_t>(e.ca.size(), 1), 0.0f);
    for (size_t j = 0; j < e.ca.size(); ++j) {
      cc32[2 * j] = float(e.ca[j]);
      cc32[2 * j + 1] = float(e.cphi[j]);
    }
    p->d_efie_cc32 = p->upload(cc32, s);
    p->d_mfie_nrm32 = p->upload(f32(nrm), s);
    p->efie_p32 = p->efie_p;
    p->efie_p32.val = p->upload(f32(e.p_val), s);
    p->efie_pt32 = p->efie_pt;
    p->efie_pt32.val = p->upload(f32(e.pt_val), s);
    AIM_HIP(hipStreamSynchronize(s));  // the float vectors are temporaries
  }
  p->d_efie_src = p->dalloc(size_t(4) * R * P * 16, s);
  p->d_efie_grid = p->dalloc(size_t(4) * R * g.Ng * 16, s);
  p->d_efie_work = p->dalloc(size_t(aim::work_elems(g, aim::kLayouts - 1, 16)) * 16 * 4 * R, s);
  p->d_efie_freq = static_cast<int32_t*>(p->dalloc(sizeof(int32_t) * 4 * R, s));
  AIM_HIP(hipHostMalloc(reinterpret_cast<void**>(&p->h_efie_freq), sizeof(int32_t) * 4 * R, 0));
  AIM_HIP(hipStreamSynchronize(s));  // the host vectors feed the uploads
  // the device copies serve the products; the host keeps what the export and
  // the double layer's assembly need (channel values, pair list)
  for (auto* v : {&e.p_val, &e.pt_val}) std::vector<double>().swap(*v);
  for (auto* v : {&e.p_rowptr, &e.p_col, &e.p_blk, &e.pt_rowptr, &e.pt_col})
    std::vector<int32_t>().swap(*v);
  p->efie_cur_freq.clear();
  p->efie_ready = true;
  p->efie_seconds = now_s() - t0;
}

void efie_checks(aim_plan p) {
  no_batch(p);
  check_prec(p, AIM_C128);
  AIM_REQUIRE(!p->host_only, AIM_ERR_STATE, "host-only plan");
}
}  // namespace

aim_status aim_efie_setup(aim_plan p, int64_t* n_rwg, int64_t* nnz, double* seconds,
                          void* hip_stream) {
  if (!p) return fail(AIM_ERR_INVALID_ARG, "null plan");
  return guarded([&] {
    efie_checks(p);
    ensure_efie(p, static_cast<hipStream_t>(hip_stream));
    if (n_rwg) *n_rwg = p->efie.n;
    if (nnz) *nnz = int64_t(p->efie.col.size());
    if (seconds) *seconds = p->efie_seconds;
  });
}

namespace {
// per-vector spectrum indices, validated (NULL: all 0)
std::vector<int32_t> freq_list(aim_plan p, int nrhs, const int32_t* freq_idx_host) {
  std::vector<int32_t> fr(size_t(nrhs), 0);
  for (int r = 0; r < nrhs && freq_idx_host; ++r) {
    AIM_REQUIRE(freq_idx_host[r] >= 0 && freq_idx_host[r] < p->nfreq, AIM_ERR_INVALID_ARG,
                "frequency index out of range");
    fr[r] = freq_idx_host[r];
  }
  return fr;
}

// one spectrum index per grid, `channels` blocks of nrhs grids that all take
// their vector's wavenumber (the first block doubles as the per-vector
// index); copied to the device only when it changes
void stage_freq(const std::vector<int32_t>& fr, int channels, std::vector<int32_t>& cur,
                int32_t* h, int32_t* d, hipStream_t s) {
  const size_t nrhs = fr.size();
  std::vector<int32_t> f(size_t(channels) * nrhs);
  for (int c = 0; c < channels; ++c)
    for (size_t r = 0; r < nrhs; ++r) f[size_t(c) * nrhs + r] = fr[r];
  if (f == cur) return;
  AIM_HIP(hipStreamSynchronize(s));  // the staging buffer may still feed a copy
  std::memcpy(h, f.data(), f.size() * sizeof(int32_t));
  AIM_HIP(hipMemcpyAsync(d, h, f.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  cur = f;
}

void check_rwg_call(aim_plan p, const void* x, const void* y, int nrhs) {
  efie_checks(p);
  AIM_REQUIRE(x != y, AIM_ERR_INVALID_ARG, "x and y must not overlap");
  AIM_REQUIRE(nrhs >= 1 && nrhs <= p->max_rhs, AIM_ERR_INVALID_ARG,
              "nrhs must be in 1..max_rhs (" + std::to_string(p->max_rhs) + ")");
}
}  // namespace

namespace {
// The RWG double layer's tables on top of the EFIE's: the triangle pairs'
// static gradient integrals and grid sums on the device, C_K and the Gram
// entries assembled on the host, the normals and max_rhs buffers.
void ensure_mfie(aim_plan p, hipStream_t s) {
  if (p->mfie_ready) return;
  ensure_efie(p, s);
  const double t0 = now_s();
  const auto& t = p->t;
  const auto& e = p->efie;
  {
    std::vector<double> pv;
    {
      aim::NearDevice nd(t, nullptr, nullptr, p->alloc, p->free_fn, p->actx, s);
      nd.fill_rwg_pairs(1, e.pair_rowptr, e.pair_col, pv, s);
    }
    aim::assemble_mfie_near(t, e, pv, p->mfie_ck, p->host_threads);
  }
  const auto& g = p->g;
  const int R = p->max_rhs;
  p->d_mfie_ck = p->upload(p->mfie_ck, s);
  if (p->prec & (1u << AIM_C64)) {
    p->d_mfie_ck32 = p->upload(std::vector<float>(p->mfie_ck.begin(), p->mfie_ck.end()), s);
    AIM_HIP(hipStreamSynchronize(s));
  }
  ensure_curl_spectra(p, s);
  p->d_mfie_grid = p->dalloc(size_t(3) * R * g.Ng * 16, s);
  p->d_mfie_work = p->dalloc(size_t(aim::work_elems(g, aim::kLayouts - 1, 16)) * 16 * 3 * R, s);
  p->d_mfie_freq = static_cast<int32_t*>(p->dalloc(sizeof(int32_t) * 6 * R, s));
  AIM_HIP(hipHostMalloc(reinterpret_cast<void**>(&p->h_mfie_freq), sizeof(int32_t) * 6 * R, 0));
  AIM_HIP(hipStreamSynchronize(s));
  p->mfie_cur_freq.clear();
  p->mfie_ready = true;
  p->mfie_seconds = now_s() - t0;
}

// One product of an RWG operator (op 1: the EFIE, 2: the double layer
// K + gram G, 3: the combined field Z + (j/k)(K + gram G)) on nrhs vectors,
// vector r at wavenumber index fr[r], in complex128 (T = double) or
// complex64 (T = float); the tables are built already.
extern "C++" {
template <typename T>
void rwg_matvec_t(aim_plan p, int op, const void* x, void* y, int nrhs,
                  const std::vector<int32_t>& fr, double gram, hipStream_t s) {
  constexpr bool dbl = sizeof(T) == 8;
  const bool efie = op == 1 || op == 3, dl = op == 2 || op == 3;
  const int64_t N = p->t.N, P = 3 * N, n = p->efie.n;
  const int pi = dbl ? int(AIM_C128) : int(AIM_C64);
  const void* vals = dbl ? static_cast<const void*>(p->d_efie_vals) : p->d_efie_vals32;
  const void* nrm = dbl ? static_cast<const void*>(p->d_mfie_nrm) : p->d_mfie_nrm32;
  const void* cc = dbl ? static_cast<const void*>(p->d_efie_cc) : p->d_efie_cc32;
  const void* ck = dbl ? static_cast<const void*>(p->d_mfie_ck) : p->d_mfie_ck32;
  const aim::CsrDevice& Pp = dbl ? p->efie_p : p->efie_p32;
  const aim::CsrDevice& Pt = dbl ? p->efie_pt : p->efie_pt32;
  const void* spec = dbl ? p->d_spec64 : p->d_spec32;
  const void* cspec = dbl ? p->d_curl_spec : p->d_curl_spec32;
  void* const* tw = dbl ? p->d_tw64 : p->d_tw32;
  const int* sched = p->sched[pi];
  aim::CsrDevice none{};
  none.n = P;  // interpolation only: the near rows are the test kernel's
  if (efie) stage_freq(fr, 4, p->efie_cur_freq, p->h_efie_freq, p->d_efie_freq, s);
  if (op == 2) stage_freq(fr, 1, p->mfie_cur_freq, p->h_mfie_freq, p->d_mfie_freq, s);
  if (dl && !p->d_cfie_psi) p->d_cfie_psi = p->dalloc(size_t(3) * p->max_rhs * P * 16, s);
  if (efie) {
    // the four channels; the double layer's cross-product z pass reads the
    // three current channels' forward transforms before the EFIE's own z
    // pass overwrites them, and writes its field into the double layer's
    // workspace
    aim::launch_efie_sources<T>(x, vals, p->d_efie_trirwg, p->d_efie_src, N, n, nrhs, s);
    aim::launch_project<T>(p->g, Pp, p->d_efie_pblk, p->efie_nblk, p->d_efie_src, P,
                           p->d_efie_grid, 4 * nrhs, s);
    aim::launch_convolve<T>(p->g, p->d_efie_grid, p->d_efie_work, p->d_efie_grid, spec,
                            p->d_efie_freq, 4 * nrhs, tw, s, nullptr, sched, 1, nullptr,
                            nullptr, 0, 1);
    if (dl) {
      aim::launch_zcross<T>(p->g, p->d_efie_work, p->d_mfie_work, cspec, p->d_efie_freq, nrhs,
                            tw, s, sched);
      aim::launch_convolve<T>(p->g, nullptr, p->d_mfie_work, p->d_mfie_grid, nullptr, nullptr,
                              3 * nrhs, tw, s, nullptr, sched, 1, nullptr, nullptr, 0, 4);
    }
    aim::launch_convolve<T>(p->g, p->d_efie_grid, p->d_efie_work, p->d_efie_grid, spec,
                            p->d_efie_freq, 4 * nrhs, tw, s, nullptr, sched, 1, nullptr,
                            nullptr, 0, 6);
    aim::launch_interp_near<T>(p->g, Pt, none, p->d_efie_grid, nullptr, p->d_efie_src, 4 * nrhs,
                               true, false, s);
    if (dl)
      aim::launch_interp_near<T>(p->g, Pt, none, p->d_mfie_grid, nullptr, p->d_cfie_psi,
                                 3 * nrhs, true, false, s);
    aim::launch_rwg_test<T>(true, dl, p->d_efie_src, p->d_cfie_psi, vals, nrm, p->d_efie_te,
                            p->d_efie_rowptr, p->d_efie_col, cc, ck, gram, p->d_k,
                            p->d_efie_freq, x, y, N, n, nrhs, s);
    return;
  }
  // the three current channels: forward x and y passes, the cross-product
  // z pass in place, inverse y and x passes
  aim::launch_mfie_sources<T>(x, vals, p->d_efie_trirwg, p->d_efie_src, N, n, nrhs, s);
  aim::launch_project<T>(p->g, Pp, p->d_efie_pblk, p->efie_nblk, p->d_efie_src, P,
                         p->d_mfie_grid, 3 * nrhs, s);
  aim::launch_convolve<T>(p->g, p->d_mfie_grid, p->d_mfie_work, p->d_mfie_grid, nullptr,
                          nullptr, 3 * nrhs, tw, s, nullptr, sched, 1, nullptr, nullptr, 0, 1);
  aim::launch_zcross<T>(p->g, p->d_mfie_work, p->d_mfie_work, cspec, p->d_mfie_freq, nrhs, tw,
                        s, sched);
  aim::launch_convolve<T>(p->g, nullptr, p->d_mfie_work, p->d_mfie_grid, nullptr, nullptr,
                          3 * nrhs, tw, s, nullptr, sched, 1, nullptr, nullptr, 0, 4);
  aim::launch_interp_near<T>(p->g, Pt, none, p->d_mfie_grid, nullptr, p->d_efie_src, 3 * nrhs,
                             true, false, s);
  aim::launch_rwg_test<T>(false, true, nullptr, p->d_efie_src, vals, nrm, p->d_efie_te,
                          p->d_efie_rowptr, p->d_efie_col, nullptr, ck, gram, p->d_k,
                          p->d_mfie_freq, x, y, N, n, nrhs, s);
}

}  // extern "C++"

void rwg_matvec(aim_plan p, aim_precision prec, int op, const void* x, void* y, int nrhs,
                const std::vector<int32_t>& fr, double gram, hipStream_t s) {
  if (prec == AIM_C128)
    rwg_matvec_t<double>(p, op, x, y, nrhs, fr, gram, s);
  else
    rwg_matvec_t<float>(p, op, x, y, nrhs, fr, gram, s);
}
}  // namespace

aim_status aim_matvec_efie(aim_plan p, aim_precision prec, const void* x, void* y, int32_t nrhs,
                           const int32_t* freq_idx_host, void* hip_stream) {
  if (!p || !x || !y) return fail(AIM_ERR_INVALID_ARG, "null argument");
  return guarded([&] {
    check_rwg_call(p, x, y, nrhs);
    check_prec(p, prec);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const std::vector<int32_t> fr = freq_list(p, nrhs, freq_idx_host);
    ensure_efie(p, s);
    rwg_matvec(p, prec, 1, x, y, nrhs, fr, 0.0, s);
  });
}

aim_status aim_matvec_mfie(aim_plan p, aim_precision prec, const void* x, void* y, int32_t nrhs,
                           const int32_t* freq_idx_host, double gram_coef, void* hip_stream) {
  if (!p || !x || !y) return fail(AIM_ERR_INVALID_ARG, "null argument");
  return guarded([&] {
    check_rwg_call(p, x, y, nrhs);
    check_prec(p, prec);
    AIM_REQUIRE(std::isfinite(gram_coef), AIM_ERR_INVALID_ARG, "gram_coef must be finite");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const std::vector<int32_t> fr = freq_list(p, nrhs, freq_idx_host);
    ensure_mfie(p, s);
    rwg_matvec(p, prec, 2, x, y, nrhs, fr, gram_coef, s);
  });
}

aim_status aim_matvec_cfie(aim_plan p, aim_precision prec, const void* x, void* y, int32_t nrhs,
                           const int32_t* freq_idx_host, double gram_coef, void* hip_stream) {
  if (!p || !x || !y) return fail(AIM_ERR_INVALID_ARG, "null argument");
  return guarded([&] {
    check_rwg_call(p, x, y, nrhs);
    check_prec(p, prec);
    AIM_REQUIRE(std::isfinite(gram_coef), AIM_ERR_INVALID_ARG, "gram_coef must be finite");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const std::vector<int32_t> fr = freq_list(p, nrhs, freq_idx_host);
    ensure_mfie(p, s);
    rwg_matvec(p, prec, 3, x, y, nrhs, fr, gram_coef, s);
  });
}

aim_status aim_rwg_excitation(aim_plan p, int32_t field, const double* params, int32_t nrhs,
                              const int32_t* freq_idx_host, void* b, void* hip_stream) {
  if (!p || !params || !b) return fail(AIM_ERR_INVALID_ARG, "null argument");
  return guarded([&] {
    efie_checks(p);
    AIM_REQUIRE(field == 0 || field == 1, AIM_ERR_INVALID_ARG, "field must be 0 (E) or 1 (H)");
    AIM_REQUIRE(nrhs >= 1 && nrhs <= p->max_rhs, AIM_ERR_INVALID_ARG,
                "nrhs must be in 1..max_rhs (" + std::to_string(p->max_rhs) + ")");
    std::vector<double> pr(params, params + size_t(6) * nrhs);
    for (int r = 0; r < nrhs; ++r) {
      double* d = &pr[6 * r];
      for (int a = 0; a < 6; ++a)
        AIM_REQUIRE(std::isfinite(d[a]), AIM_ERR_INVALID_ARG, "non-finite excitation parameter");
      const double nn = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      AIM_REQUIRE(nn > 0.0, AIM_ERR_INVALID_ARG, "zero plane-wave direction");
      for (int a = 0; a < 3; ++a) d[a] /= nn;
    }
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    ensure_efie(p, s);
    const int32_t* df = set_freq(p, freq_idx_host, nrhs, s);
    double* dpr = nullptr;
    AIM_HIP(hipMalloc(&dpr, pr.size() * sizeof(double)));
    hipError_t e = hipMemcpyAsync(dpr, pr.data(), pr.size() * sizeof(double),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
      try {
        aim::launch_rwg_plane_wave(p->d_qpxyz, p->d_efie_vals, p->d_mfie_nrm, p->d_efie_te, dpr,
                                   p->d_k, df, field, b, p->efie.n, nrhs, s);
      } catch (...) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(dpr);
        throw;
      }
      e = hipStreamSynchronize(s);
    }
    (void)hipFree(dpr);
    AIM_HIP(e);
  });
}

aim_status aim_mfie_export(aim_plan p, double* ck_host, double* gram_host, double* seconds,
                           void* hip_stream) {
  if (!p) return fail(AIM_ERR_INVALID_ARG, "null plan");
  return guarded([&] {
    efie_checks(p);
    ensure_mfie(p, static_cast<hipStream_t>(hip_stream));
    const size_t nnz = p->efie.col.size();
    for (size_t j = 0; j < nnz; ++j) {
      if (ck_host) ck_host[j] = p->mfie_ck[2 * j];
      if (gram_host) gram_host[j] = p->mfie_ck[2 * j + 1];
    }
    if (seconds) *seconds = p->mfie_seconds;
  });
}

aim_status aim_efie_export(aim_plan p, int32_t* tri_rwg, int32_t* rowptr, int32_t* col,
                           double* ca, double* cphi, void* hip_stream) {
  if (!p) return fail(AIM_ERR_INVALID_ARG, "null plan");
  return guarded([&] {
    efie_checks(p);
    ensure_efie(p, static_cast<hipStream_t>(hip_stream));
    const auto& e = p->efie;
    const size_t nnz = e.col.size();
    if (tri_rwg) std::memcpy(tri_rwg, e.tri_rwg.data(), e.tri_rwg.size() * 4);
    if (rowptr) std::memcpy(rowptr, e.rowptr.data(), e.rowptr.size() * 4);
    if (col && nnz) std::memcpy(col, e.col.data(), nnz * 4);
    if (ca && nnz) std::memcpy(ca, e.ca.data(), nnz * 8);
    if (cphi && nnz) std::memcpy(cphi, e.cphi.data(), nnz * 8);
  });
}

aim_status aim_conventional_export(aim_plan p, double* vals_host, void* hip_stream) {
  if (!p || !vals_host) return fail(AIM_ERR_INVALID_ARG, "null argument");
  return guarded([&] {
    AIM_REQUIRE(p->conv_freq >= 0, AIM_ERR_STATE, "no conventional near correction filled");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const size_t nnz = p->t.col.size();
    if (nnz) AIM_HIP(hipMemcpyAsync(vals_host, p->d_conv64, nnz * 16, hipMemcpyDeviceToHost, s));
    AIM_HIP(hipStreamSynchronize(s));
  });
}

aim_status aim_profile_matvec(aim_plan p, aim_precision prec, const void* x, void* y,
                              int32_t nrhs, const int32_t* freq_idx_host, int32_t reps,
                              double* kernel_ms, void* hip_stream) {
  if (!p || !x || !y || !kernel_ms) return fail(AIM_ERR_INVALID_ARG, "null argument");
  return guarded([&] {
    no_batch(p);
    check_prec(p, prec);
    AIM_REQUIRE(x != y, AIM_ERR_INVALID_ARG, "x and y must not overlap");
    AIM_REQUIRE(reps >= 1 && reps <= 1000, AIM_ERR_INVALID_ARG, "reps must be in 1..1000");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int32_t* df = set_freq(p, freq_idx_host, nrhs, s);
    // reps ordinary matvecs after one warm-up, events before, between and
    // after the seven kernels of each (the queue stays full, so an interval
    // is its kernel's duration)
    std::vector<hipEvent_t> ev(8 * size_t(reps), nullptr);
    auto destroy = [&] {
      for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    };
    try {
      for (auto& e : ev) AIM_HIP(hipEventCreate(&e));
      matvec_any(p, prec, x, y, nrhs, df, s);
      for (int r = 0; r < reps; ++r) {
        if (prec == AIM_C128)
          matvec_impl<double>(p, prec, x, y, nrhs, df, s, ev.data() + 8 * size_t(r));
        else
          matvec_impl<float>(p, prec, x, y, nrhs, df, s, ev.data() + 8 * size_t(r));
      }
      AIM_HIP(hipStreamSynchronize(s));
      for (int k = 0; k < AIM_N_KERNELS; ++k) {
        double tot = 0.0;
        for (int r = 0; r < reps; ++r) {
          float ms = 0.f;
          AIM_HIP(hipEventElapsedTime(&ms, ev[8 * size_t(r) + k], ev[8 * size_t(r) + k + 1]));
          tot += double(ms);
        }
        kernel_ms[k] = tot / reps;
      }
    } catch (...) {
      destroy();
      throw;
    }
    destroy();
  });
}

aim_status aim_set_schedule(aim_plan p, aim_precision prec, const int32_t* sched) {
  if (!p || !sched) return fail(AIM_ERR_INVALID_ARG, "null argument");
  return guarded([&] {
    no_batch(p);
    check_prec(p, prec);
    for (int k = 0; k < 5; ++k)
      AIM_REQUIRE(sched[k] >= 0 && sched[k] < aim::kFftVariants &&
                      aim::fft_variant_ok(prec == AIM_C128, p->g, k, sched[k]),
                  AIM_ERR_INVALID_ARG, "launch shape not available for this pass");
    AIM_REQUIRE(sched[5] >= 0 && sched[5] < aim::kLayouts, AIM_ERR_INVALID_ARG,
                "workspace layout out of range");
    AIM_REQUIRE(sched[6] >= 0 && sched[6] <= 3, AIM_ERR_INVALID_ARG,
                "stage modes must be in 0..3");
    for (int k = 0; k < aim::kSchedLen; ++k) p->sched[int(prec)][k] = sched[k];
    p->graphs.clear();
  });
}

aim_status aim_autotune(aim_plan p, aim_precision prec, int32_t nrhs, int32_t reps,
                        int32_t* sched_out, double* pass_ms_out, void* hip_stream) {
  if (!p) return fail(AIM_ERR_INVALID_ARG, "null plan");
  return guarded([&] {
    no_batch(p);
    check_prec(p, prec);
    AIM_REQUIRE(reps >= 1 && reps <= 1000, AIM_ERR_INVALID_ARG, "reps must be in 1..1000");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int32_t* df = set_freq(p, nullptr, nrhs, s);
    const int pi = int(prec);
    const bool dbl = prec == AIM_C128;
    const size_t cb = dbl ? 16 : 8;
    void* grid = p->d_grid[pi];
    // a pseudo-random input grid (timings on zeros run at a higher clock),
    // convolved into a buffer of its own so that every timed pass sees the
    // same values
    aim::launch_pattern(grid, p->g.Ng * nrhs, dbl, s);
    void* phi = nullptr;
    {
      const hipError_t e = hipMalloc(&phi, size_t(p->g.Ng) * cb * nrhs);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        throw aim::Error(AIM_ERR_OOM, "autotune: no memory for the output grid");
      }
    }
    std::vector<hipEvent_t> ev(6 * size_t(reps), nullptr);
    auto destroy = [&] {
      for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
      (void)hipStreamSynchronize(s);
      (void)hipFree(phi);
    };
    double best[5], lbest[5];
    int pick[aim::kSchedLen], lpick[5];
    double best_total = 1e300;
    for (int k = 0; k < aim::kSchedLen; ++k) pick[k] = 0;
    for (int k = 0; k < 5; ++k) best[k] = 0.0;
    try {
      for (auto& e : ev) AIM_HIP(hipEventCreate(&e));
      for (int layout = 0; layout < aim::kLayouts; ++layout) {
        for (int k = 0; k < 5; ++k) {
          lbest[k] = 1e300;
          lpick[k] = 0;
        }
        for (int v = 0; v < aim::kFftVariants; ++v) {
          int sch[aim::kSchedLen];
          bool any = false;
          for (int k = 0; k < 5; ++k) {
            const bool ok = aim::fft_variant_ok(dbl, p->g, k, v);
            sch[k] = ok ? v : 0;
            any = any || ok;
          }
          sch[5] = layout;
          sch[6] = 0;
          if (!any) continue;
          for (int r = -1; r < reps; ++r) {  // r = -1: warm-up
            hipEvent_t* e = &ev[6 * size_t(std::max(r, 0))];
            if (r >= 0) AIM_HIP(hipEventRecord(e[0], s));
            if (dbl)
              aim::launch_convolve<double>(p->g, grid, p->d_work[pi], phi, p->d_spec64, df, nrhs,
                                           p->d_tw64, s, r >= 0 ? e + 1 : nullptr, sch);
            else
              aim::launch_convolve<float>(p->g, grid, p->d_work[pi], phi, p->d_spec32, df, nrhs,
                                          p->d_tw32, s, r >= 0 ? e + 1 : nullptr, sch);
            if (r >= 0) AIM_HIP(hipEventRecord(e[5], s));
          }
          AIM_HIP(hipStreamSynchronize(s));
          for (int k = 0; k < 5; ++k) {
            if (sch[k] != v) continue;
            double tot = 0.0;
            for (int r = 0; r < reps; ++r) {
              float ms = 0.f;
              AIM_HIP(hipEventElapsedTime(&ms, ev[6 * size_t(r) + k], ev[6 * size_t(r) + k + 1]));
              tot += ms;
            }
            if (tot / reps < lbest[k]) {
              lbest[k] = tot / reps;
              lpick[k] = v;
            }
          }
        }
        double total = 0.0;
        for (int k = 0; k < 5; ++k) total += lbest[k];
        // a later layout has to be 2% faster to win: layouts within timing
        // noise of each other keep the earlier one, so repeated tunings agree
        if (total < (layout == 0 ? 1.0 : 0.98) * best_total) {
          best_total = total;
          for (int k = 0; k < 5; ++k) {
            best[k] = lbest[k];
            pick[k] = lpick[k];
          }
          pick[5] = layout;
        }
      }
    } catch (...) {
      destroy();
      throw;
    }
    destroy();
    // interpolation: assembled P^T against recomputed weights, timed as whole
    // matvecs (the mode also changes what the projection finds in cache)
    for (int k = 0; k < 6; ++k) p->sched[pi][k] = pick[k];
    {
      const size_t vb = size_t(p->t.N) * cb * nrhs;
      void* xy = nullptr;
      AIM_HIP(hipMalloc(&xy, 2 * vb));
      hipEvent_t e0 = nullptr, e1 = nullptr;
      double tm[4] = {0.0, 0.0, 0.0, 0.0};
      try {
        aim::launch_pattern(xy, p->t.N * nrhs, dbl, s);
        AIM_HIP(hipEventCreate(&e0));
        AIM_HIP(hipEventCreate(&e1));
        // three rounds alternating the four stage modes (interpolation from
        // the assembled P^T or recomputed weights, projection on its own or
        // fused into the x forward pass), best time of each: one round alone
        // flips between modes within a few percent of each other
        tm[0] = tm[1] = tm[2] = tm[3] = 1e300;
        for (int round = 0; round < 3; ++round)
          for (int mode = 0; mode < 4; ++mode) {
            p->sched[pi][6] = mode;
            auto run = [&] { matvec_any(p, prec, xy, static_cast<char*>(xy) + vb, nrhs, df, s); };
            run();  // warm-up
            AIM_HIP(hipEventRecord(e0, s));
            for (int r = 0; r < reps; ++r) run();
            AIM_HIP(hipEventRecord(e1, s));
            AIM_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            AIM_HIP(hipEventElapsedTime(&ms, e0, e1));
            tm[mode] = std::min(tm[mode], double(ms) / reps);
          }
      } catch (...) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipStreamSynchronize(s);
        (void)hipFree(xy);
        throw;
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      AIM_HIP(hipStreamSynchronize(s));
      AIM_HIP(hipFree(xy));
      pick[6] = 0;
      for (int mode = 1; mode < 4; ++mode)
        if (tm[mode] < tm[pick[6]]) pick[6] = mode;
    }
    for (int k = 0; k < aim::kSchedLen; ++k) {
      p->sched[pi][k] = pick[k];
      if (sched_out) sched_out[k] = pick[k];
    }
    for (int k = 0; k < 5; ++k)
      if (pass_ms_out) pass_ms_out[k] = best[k];
    p->graphs.clear();
  });
}

namespace {
void apply_unet_pc(aim_plan p, const void* v, void* z, int nrhs, const int32_t* dfreq,
                   hipStream_t s, const char* skip = nullptr);
void apply_base(aim_plan p, aim_pc_kind pc, const void* v, void* z, int nrhs,
                const int32_t* dfreq, hipStream_t s, const char* skip = nullptr);
void ensure_nearblock(aim_plan p, int f, hipStream_t s);
void ensure_nearblock_for(aim_plan p, const int32_t* freq_host, int nrhs, hipStream_t s);
void check_unet_plan(aim_plan p);
}  // namespace

aim_status aim_apply_stage(aim_plan p, aim_precision prec, aim_stage stage, const void* in,
                           void* out, int32_t nrhs, const int32_t* freq_idx_host,
                           void* hip_stream) {
  if (!p || !in || !out) return fail(AIM_ERR_INVALID_ARG, "null argument");
  return guarded([&] {
    no_batch(p);
    check_prec(p, prec);
    AIM_REQUIRE(in != out, AIM_ERR_INVALID_ARG, "in and out must not overlap");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int32_t* df = set_freq(p, freq_idx_host, nrhs, s);
    const int pi = int(prec);
    const bool d = prec == AIM_C128;
    switch (stage) {
      case AIM_STAGE_PROJECT:
        if (d)
          aim::launch_project<double>(p->g, p_dev(p, prec), p->d_pblk, p->nblk, in, p->t.N, out,
                                      nrhs, s);
        else
          aim::launch_project<float>(p->g, p_dev(p, prec), p->d_pblk, p->nblk, in, p->t.N, out,
                                     nrhs, s);
        break;
      case AIM_STAGE_CONVOLVE:
        if (d)
          aim::launch_convolve<double>(p->g, in, p->d_work[pi], out, p->d_spec64, df, nrhs,
                                       p->d_tw64, s, nullptr, p->sched[pi]);
        else
          aim::launch_convolve<float>(p->g, in, p->d_work[pi], out, p->d_spec32, df, nrhs,
                                      p->d_tw32, s, nullptr, p->sched[pi]);
        break;
      case AIM_STAGE_INTERPOLATE:
      case AIM_STAGE_NEAR: {
        const bool interp = stage == AIM_STAGE_INTERPOLATE;
        if (d)
          interp_near<double>(p, prec, interp ? in : nullptr, interp ? nullptr : in, out, nrhs,
                              interp, !interp, s);
        else
          interp_near<float>(p, prec, interp ? in : nullptr, interp ? nullptr : in, out, nrhs,
                             interp, !interp, s);
        break;
      }
      case AIM_STAGE_LEARNED_PC:
        AIM_REQUIRE(d, AIM_ERR_INVALID_ARG,
                    "the learned preconditioner maps complex128 vectors (prec = AIM_C128)");
        AIM_REQUIRE(nrhs >= 1 && nrhs <= p->max_rhs, AIM_ERR_INVALID_ARG,
                    "nrhs must be in 1..max_rhs");
        check_unet_plan(p);
        if (p->unet_base == AIM_PC_NEARBLOCK) ensure_nearblock_for(p, freq_idx_host, nrhs, s);
        apply_unet_pc(p, in, out, nrhs, df, s);
        break;
      case AIM_STAGE_NEARBLOCK_PC:
        AIM_REQUIRE(d, AIM_ERR_INVALID_ARG,
                    "the near-block preconditioner maps complex128 vectors (prec = AIM_C128)");
        ensure_nearblock_for(p, freq_idx_host, nrhs, s);
        apply_base(p, AIM_PC_NEARBLOCK, in, out, nrhs, df, s);
        break;
      default:
        throw Error(AIM_ERR_INVALID_ARG, "unknown stage");
    }
  });
}

aim_status aim_excitation(aim_plan p, aim_rhs_kind kind, const double* params, int32_t n_params,
                          int32_t nrhs, const int32_t* freq_idx_host, void* b, void* hip_stream) {
  if (!p || !params || !b) return fail(AIM_ERR_INVALID_ARG, "null argument");
  return guarded([&] {
    no_batch(p);
    AIM_REQUIRE(!p->host_only, AIM_ERR_STATE, "host-only plan has no device data");
    AIM_REQUIRE(kind == AIM_RHS_PLANE_WAVE || kind == AIM_RHS_GAUSSIAN_PATCH, AIM_ERR_INVALID_ARG,
                "unknown excitation kind");
    const int need = kind == AIM_RHS_PLANE_WAVE ? 3 : 4;
    AIM_REQUIRE(n_params == need, AIM_ERR_INVALID_ARG, "wrong number of excitation parameters");
    for (int r = 0; r < nrhs * n_params && r >= 0; ++r)
      AIM_REQUIRE(std::isfinite(params[r]), AIM_ERR_INVALID_ARG, "non-finite excitation parameter");
    if (kind == AIM_RHS_GAUSSIAN_PATCH)
      for (int r = 0; r < nrhs; ++r)
        AIM_REQUIRE(params[r * 4 + 3] > 0.0, AIM_ERR_INVALID_ARG, "patch width must be positive");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int32_t* df = set_freq(p, freq_idx_host, nrhs, s);
    std::vector<double> pr(params, params + size_t(nrhs) * n_params);
    if (kind == AIM_RHS_PLANE_WAVE)
      for (int r = 0; r < nrhs; ++r) {
        double* d3 = &pr[3 * r];
        const double nn = std::sqrt(d3[0] * d3[0] + d3[1] * d3[1] + d3[2] * d3[2]);
        AIM_REQUIRE(nn > 0.0, AIM_ERR_INVALID_ARG, "zero plane-wave direction");
        for (int a = 0; a < 3; ++a) d3[a] /= nn;
      }
    double* dpr = nullptr;
    AIM_HIP(hipMalloc(&dpr, pr.size() * sizeof(double)));
    hipError_t e = hipMemcpyAsync(dpr, pr.data(), pr.size() * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
      aim::launch_excitation(int(kind), p->d_qpxyz, p->d_w64, p->t.N, dpr, n_params, p->d_k, df,
                             nrhs, b, s);
      e = hipStreamSynchronize(s);
    }
    (void)hipFree(dpr);
    AIM_HIP(e);
  });
}

aim_status aim_export_tables(aim_plan p, int32_t* stencil_start, double* stencil_local,
                             int64_t* rowptr, int32_t* col, double* val, double* near_static) {
  if (!p) return fail(AIM_ERR_INVALID_ARG, "null plan");
  return guarded([&] {
    no_batch(p);
    const auto& t = p->t;
    if (stencil_start) std::copy(t.qp_start.begin(), t.qp_start.end(), stencil_start);
    if (stencil_local) std::copy(t.qp_local.begin(), t.qp_local.end(), stencil_local);
    if (rowptr) std::copy(t.rowptr.begin(), t.rowptr.end(), rowptr);
    if (col) std::copy(t.col.begin(), t.col.end(), col);
    if (val) std::copy(t.corr.begin(), t.corr.end(), val);
    if (near_static) std::copy(t.near_static.begin(), t.near_static.end(), near_static);
  });
}

}  // extern "C"

// ===========================================================================
// batched GMRES / FGMRES with right preconditioning (complex128 Arnoldi, CGS2)
// ===========================================================================
namespace {

using cplx = std::complex<double>;

// unknowns of the operator the solver applies
int64_t op_n(aim_plan p) { return p->rwg_op ? p->efie.n : p->t.N; }

void ensure_solver(aim_plan p, int nrhs, int m, hipStream_t s) {
  auto& w = p->sv;
  // vectors sized for the largest operator solved so far, so that solves
  // of the scalar and the RWG operators share one workspace
  const int64_t n = std::max(op_n(p), w.n);
  if (w.nrhs >= nrhs && w.m >= m && w.n >= op_n(p)) return;
  p->graphs.clear();  // captured graphs point at the old staging buffers
  // buffers are never freed individually: the plan owns them until destroy
  const int R = std::max(nrhs, w.nrhs), M = std::max(m, w.m);
  const size_t vec = size_t(n) * 16;
  w.V = p->dalloc(vec * R * (M + 1), s);
  w.Z = p->dalloc(vec * R * M, s);
  w.w = p->dalloc(vec * R, s);
  w.r = p->dalloc(vec * R, s);
  w.d = p->dalloc(vec * R, s);
  w.bp = p->dalloc(vec * R, s);
  w.xp = p->dalloc(vec * R, s);
  w.ain = p->dalloc(vec * R, s);
  // the two Gram-Schmidt coefficient sets and the basis norms of a step
  const size_t hb = size_t(16) * R * (M + 1);
  w.h = p->dalloc(2 * hb + sizeof(double) * R, s);
  w.h2 = static_cast<char*>(w.h) + hb;
  w.y = p->dalloc(size_t(16) * R * (M + 1), s);
  const int64_t nchunk = (n + 4095) / 4096;
  w.partial = p->dalloc(size_t(16) * R * (M + 1) * nchunk, s);
  w.nrm = reinterpret_cast<double*>(static_cast<char*>(w.h) + 2 * hb);
  w.idx = static_cast<int32_t*>(p->dalloc(sizeof(int32_t) * R, s));
  w.freq = static_cast<int32_t*>(p->dalloc(sizeof(int32_t) * R, s));
  if (p->prec & (1u << AIM_C64)) {
    w.c64a = p->dalloc(size_t(n) * 8 * R, s);
    w.c64b = p->dalloc(size_t(n) * 8 * R, s);
  }
  w.H = p->dalloc(size_t(16) * R * M * (M + 1), s);
  w.cs = p->dalloc(size_t(16) * R * M, s);
  w.sn = p->dalloc(size_t(16) * R * M, s);
  w.g = p->dalloc(size_t(16) * R * (M + 1), s);
  w.gst = static_cast<aim::GivensState*>(p->dalloc(sizeof(aim::GivensState) * R, s));
  w.scale = static_cast<double*>(p->dalloc(sizeof(double) * R, s));
  if (w.nrm_host) (void)hipHostFree(w.nrm_host);
  if (w.H_host) (void)hipHostFree(w.H_host);
  if (w.g_host) (void)hipHostFree(w.g_host);
  if (w.gst_host) (void)hipHostFree(w.gst_host);
  if (w.scale_host) (void)hipHostFree(w.scale_host);
  w.nrm_host = nullptr;
  w.H_host = w.g_host = nullptr;
  w.gst_host = nullptr;
  w.scale_host = nullptr;
  AIM_HIP(hipHostMalloc(reinterpret_cast<void**>(&w.H_host), size_t(16) * R * M * (M + 1), 0));
  AIM_HIP(hipHostMalloc(reinterpret_cast<void**>(&w.g_host), size_t(16) * R * (M + 1), 0));
  AIM_HIP(hipHostMalloc(reinterpret_cast<void**>(&w.gst_host), sizeof(aim::GivensState) * R, 0));
  AIM_HIP(hipHostMalloc(reinterpret_cast<void**>(&w.scale_host), sizeof(double) * R, 0));
  AIM_HIP(hipHostMalloc(reinterpret_cast<void**>(&w.nrm_host), sizeof(double) * R * 2, 0));
  w.nrhs = R;
  w.m = M;
  w.n = n;
}

// Operator application used by the Krylov loop: y = A(k_f) x in the requested
// precision on complex128 vectors (complex64 matvec through casts).  The
// Krylov loop leaves the host only every few steps, so the host enqueues well
// ahead of the GPU and the seven kernels are launched directly; with
// AIM_SOLVER_GRAPHS=1 they replay instead from a captured graph (one per
// precision, batch width and frequency set) fed through fixed staging
// buffers, which costs a copy per step.
bool solver_graphs_enabled() {
  const char* e = std::getenv("AIM_SOLVER_GRAPHS");
  return e && e[0] == '1';
}

void graph_matvec(aim_plan p, aim_precision prec, const void* in, void* out, int nrhs,
                  const int32_t* dfreq, hipStream_t s) {
  if (!solver_graphs_enabled()) {
    matvec_any(p, prec, in, out, nrhs, dfreq, s);
    return;
  }
  for (auto& kv : p->graphs) {
    const auto& k = kv.first;
    if (k.prec == int(prec) && k.nrhs == nrhs && k.in == in && k.out == out &&
        int(k.freq.size()) >= nrhs &&
        std::equal(p->cur_freq.begin(), p->cur_freq.begin() + nrhs, k.freq.begin())) {
      AIM_HIP(hipGraphLaunch(kv.second->exec, s));
      return;
    }
  }
  if (p->graphs.size() >= 16) p->graphs.erase(p->graphs.begin());
  aim_plan_s::GraphKey key{int(prec), nrhs, in, out,
                           std::vector<int32_t>(p->cur_freq.begin(), p->cur_freq.begin() + nrhs)};
  p->graphs.emplace_back(std::move(key), capture_matvec(p, prec, in, out, nrhs, dfreq, s));
  AIM_HIP(hipGraphLaunch(p->graphs.back().second->exec, s));
}

void apply_A(aim_plan p, aim_precision prec, const void* x, void* y, int nrhs, const int32_t* dfreq,
             hipStream_t s, const char* skip = nullptr) {
  if (p->rwg_op) {  // an RWG operator (complex128; wavenumbers from the solve's list)
    rwg_matvec(p, AIM_C128, p->rwg_op, x, y, nrhs, p->rwg_fr, p->rwg_gram, s);
    return;
  }
  const int64_t cnt = p->t.N * int64_t(nrhs);
  if (skip && p->batch) {  // direct launches, stopped instances skipped, padding left
    if (prec == AIM_C128) {
      matvec_any(p, AIM_C128, x, y, nrhs, dfreq, s, nullptr, skip, false);
      return;
    }
    // complex64 matvecs: each running instance casts its own rows, so the
    // stopped ones cost nothing
    const int64_t nmax = p->t.N;
    batch_fork(p, nrhs, skip, s, [&](int i, hipStream_t si) {
      aim_plan_s* q = p->inst[i].get();
      const int64_t ni = q->t.N, off = int64_t(i) * nmax;
      void* a = static_cast<char*>(p->sv.c64a) + size_t(off) * 8;
      void* b2 = static_cast<char*>(p->sv.c64b) + size_t(off) * 8;
      char* yi = static_cast<char*>(y) + size_t(off) * 16;
      aim::launch_cast_c128_to_c64(static_cast<const char*>(x) + size_t(off) * 16, a, ni, si);
      matvec_any(q, AIM_C64, a, b2, 1, dfreq + i, si);
      aim::launch_cast_c64_to_c128(b2, yi, ni, si);
    });
    return;
  }
  if (prec == AIM_C128) {
    if (!solver_graphs_enabled()) {
      matvec_any(p, AIM_C128, x, y, nrhs, dfreq, s);
      return;
    }
    AIM_HIP(hipMemcpyAsync(p->sv.ain, x, size_t(cnt) * 16, hipMemcpyDeviceToDevice, s));
    graph_matvec(p, AIM_C128, p->sv.ain, y, nrhs, dfreq, s);
  } else {
    aim::launch_cast_c128_to_c64(x, p->sv.c64a, cnt, s);
    graph_matvec(p, AIM_C64, p->sv.c64a, p->sv.c64b, nrhs, dfreq, s);
    aim::launch_cast_c64_to_c128(p->sv.c64b, y, cnt, s);
  }
}

void ensure_unet_buffers(aim_plan p, hipStream_t s) {
  if (p->ug_in) return;
  const int R = p->max_rhs;
  const int64_t n = p->t.N, Ng = p->g.Ng;
  p->ug_in = p->dalloc(size_t(Ng) * 8 * R, s);
  p->ug_out = p->dalloc(size_t(Ng) * 8 * R, s);
  p->ug_x = p->dalloc(size_t(Ng) * 8 * R, s);
  p->um1 = p->dalloc(size_t(n) * 8 * R, s);
  p->um2 = p->dalloc(size_t(n) * 8 * R, s);
  const int64_t nchunk = (std::max(n, Ng) + 4095) / 4096;
  p->upart = p->dalloc(size_t(16) * R * nchunk + 16 * 4096, s);
  p->u_s = static_cast<double*>(p->dalloc(sizeof(double) * R, s));
  p->u_s2 = static_cast<double*>(p->dalloc(sizeof(double) * R, s));
}

// Near-field tables on the device without the mesh (the static entries
// uploaded), for the conventional fill and the near-block blocks.
aim::NearDevice& near_device(aim_plan p, hipStream_t s) {
  if (!p->conv_nd) {
    p->conv_nd.reset(
        new aim::NearDevice(p->t, nullptr, nullptr, p->alloc, p->free_fn, p->actx, s));
    p->conv_nd->set_static(p->t.near_static, s);
  }
  return *p->conv_nd;
}

// Builds the near-block inverses of wavenumber index f if they are missing.
void ensure_nearblock(aim_plan p, int f, hipStream_t s) {
  AIM_REQUIRE(f >= 0 && f < p->nfreq, AIM_ERR_INVALID_ARG, "frequency index out of range");
  const int64_t per = p->t.cl_blk.back();  // complex values per wavenumber
  if (!p->d_clinv_k) {
    p->d_clinv_k = p->dalloc(size_t(per) * 16 * p->nfreq, s);
    p->clinv_built.assign(p->nfreq, 0);
  }
  if (p->clinv_built[f]) return;
  near_device(p, s).fill_cluster_inverses(
      p->k[f], p->d_clptr, p->d_clperm, p->d_clblk, p->ncl, p->maxcl,
      static_cast<char*>(p->d_clinv_k) + size_t(f) * per * 16, s);
  p->clinv_built[f] = 1;
}

// ... for the wavenumbers of nrhs systems (freq_host null: all index 0); a
// batch plan's system i is its instance i
void ensure_nearblock_for(aim_plan p, const int32_t* freq_host, int nrhs, hipStream_t s) {
  for (int r = 0; r < nrhs; ++r) {
    const int f = freq_host ? freq_host[r] : 0;
    ensure_nearblock(p->batch ? p->inst[size_t(r)].get() : p, f, s);
  }
}

// Classical (linear) preconditioners: z = v, D^{-1} v or a near-block
// inverse; dfreq (device) holds each system's wavenumber index.
// skip (batch plans only, may be null): systems whose result is not needed
// (GMRES systems that have stopped); their rows of z are left as they are,
// and so is the padding of every row (only the GMRES loop passes skip)
void apply_base(aim_plan p, aim_pc_kind pc, const void* v, void* z, int nrhs,
                const int32_t* dfreq, hipStream_t s, const char* skip) {
  const int64_t n = p->t.N;
  if (p->batch) {
    batch_fork(p, nrhs, skip, s, [&](int i, hipStream_t si) {
      aim_plan_s* q = p->inst[i].get();
      const char* vi = static_cast<const char*>(v) + size_t(i) * n * 16;
      char* zi = static_cast<char*>(z) + size_t(i) * n * 16;
      apply_base(q, pc, vi, zi, 1, dfreq + i, si);
      if (!skip) aim::launch_zero_words(zi + size_t(q->t.N) * 16, (n - q->t.N) * 2, si);
    });
    return;
  }
  switch (pc) {
    case AIM_PC_NONE:
      AIM_HIP(hipMemcpyAsync(z, v, size_t(n) * 16 * nrhs, hipMemcpyDeviceToDevice, s));
      break;
    case AIM_PC_DIAG:
      aim::launch_diag_pc(v, p->d_dinv, z, n, nrhs, s);
      break;
    case AIM_PC_NEARBLOCK:
      AIM_REQUIRE(p->d_clinv_k != nullptr, AIM_ERR_STATE, "near-block inverses not built");
      aim::launch_block_pc_complex(v, z, p->d_clptr, p->d_clperm, p->d_clblk, p->d_clinv_k,
                                   p->t.cl_blk.back(), dfreq, p->ncl, p->maxcl, n, nrhs, s);
      break;
    case AIM_PC_NEARBLOCK_STATIC:
      aim::launch_block_pc(v, z, p->d_clptr, p->d_clperm, p->d_clblk, p->d_clinv, p->ncl, p->maxcl,
                           n, nrhs, s);
      break;
    default:
      throw Error(AIM_ERR_STATE, "preconditioner not available");
  }
}

// Network input for nrhs complex128 mesh vectors v: the complex64 grid
// P (v / ||v||) scaled to unit RMS over the grid, written to grid[r] (Ng
// complex64 each).  Leaves 1/||v|| in p->u_s.
void unet_input(aim_plan p, const void* v, int nrhs, void* grid, hipStream_t s) {
  ensure_unet_buffers(p, s);
  AIM_REQUIRE(grid != nullptr, AIM_ERR_STATE, "network input buffer missing");
  const int64_t n = p->t.N, Ng = p->g.Ng;
  aim::launch_inv_norms_c128(v, n, nrhs, 1.0, p->upart, p->u_s, s);
  aim::launch_scale_cast_c64(v, p->u_s, p->um1, n, nrhs, s);
  aim::launch_project<float>(p->g, p_dev(p, AIM_C64), p->d_pblk, p->nblk, p->um1, n, grid, nrhs, s);
  aim::launch_inv_norms_c64(grid, Ng, nrhs, std::sqrt(double(Ng)), p->upart, p->u_s2, s);
  aim::launch_scale_c64(grid, p->u_s2, Ng, nrhs, s);
}

void check_unet_plan(aim_plan p) {
  AIM_REQUIRE(!p->host_only, AIM_ERR_STATE, "host-only plan");
  AIM_REQUIRE(p->prec & (1u << AIM_C64), AIM_ERR_STATE,
              "the learned preconditioner needs the complex64 tables (precisions bit 1)");
  for (int d = 0; d < 3; ++d)
    AIM_REQUIRE(p->g.N[d] % 4 == 0, AIM_ERR_GRID, "grid dimensions must be multiples of 4");
}

// Learned preconditioner (a nonlinear map, so the solve is flexible GMRES):
//   z = B v + tau ||v|| (P^T U(g)) / area,   g = unet_input(v),
// B the base preconditioner, U the network; the grid work is complex64.
// On a batch plan each instance applies the network on its own grid, one
// instance after another on s (the network's activation buffers are shared);
// skip as in apply_base.
void apply_unet_pc(aim_plan p, const void* v, void* z, int nrhs, const int32_t* dfreq,
                   hipStream_t s, const char* skip) {
  AIM_REQUIRE(p->unet != nullptr, AIM_ERR_STATE, "no learned preconditioner attached");
  if (p->batch) {
    const int64_t n = p->t.N;
    for (int i = 0; i < nrhs; ++i) {
      if (skip && skip[i]) continue;
      aim_plan_s* q = p->inst[size_t(i)].get();
      const char* vi = static_cast<const char*>(v) + size_t(i) * n * 16;
      char* zi = static_cast<char*>(z) + size_t(i) * n * 16;
      apply_unet_pc(q, vi, zi, 1, dfreq + i, s);
      if (!skip) aim::launch_zero_words(zi + size_t(q->t.N) * 16, (n - q->t.N) * 2, s);
    }
    return;
  }
  ensure_unet_buffers(p, s);  // before any of the buffers is read below
  const int64_t n = p->t.N, Ng = p->g.Ng;
  unet_input(p, v, nrhs, p->ug_in, s);
  // the nrhs grids lie one after another: one batched pass of the network
  aim::unet_forward(p->unet, p->ug_in, nrhs, p->g.N[2], p->g.N[1], p->g.N[0], p->ug_out, s);
  interp_near<float>(p, AIM_C64, p->ug_out, nullptr, p->um2, nrhs, true, false, s);
  apply_base(p, p->unet_base, v, z, nrhs, dfreq, s);
  aim::launch_unet_combine(p->um2, p->d_area, p->unet_tau, p->u_s, z, n, nrhs, s);
}

void apply_M(aim_plan p, aim_pc_kind pc, const void* v, void* z, int nrhs, const int32_t* dfreq,
             hipStream_t s, const char* skip = nullptr) {
  if (pc == AIM_PC_UNET)
    apply_unet_pc(p, v, z, nrhs, dfreq, s, skip);
  else
    apply_base(p, pc, v, z, nrhs, dfreq, s, skip);
}

void norms_host(aim_plan p, const void* v, int nrhs, hipStream_t s, std::vector<double>& out) {
  aim::launch_norms(v, op_n(p), nrhs, p->sv.partial, p->sv.nrm, s);
  AIM_HIP(hipMemcpyAsync(p->sv.nrm_host, p->sv.nrm, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
  AIM_HIP(hipStreamSynchronize(s));
  out.assign(p->sv.nrm_host, p->sv.nrm_host + nrhs);
}

struct CycleStats {
  std::vector<int> iters;  // Krylov steps per system
  int matvecs = 0;
};

// raised when a restart cycle with the learned preconditioner makes too
// little progress (the gate of the fallback logic)
struct GateFail {};

// called at every restart with (x, r, relative residuals) of all systems
using CycleHook = std::function<void(const void*, const void*, const std::vector<double>&)>;

// Restarted right-preconditioned GMRES on a packed batch: solves A x = b for
// nrhs systems in lock step (x holds the initial guess).  Each system stops
// extending its Krylov basis once its residual estimate is below tol * scale;
// the true residual decides convergence at every restart.  Returns per-system
// true relative residual (w.r.t. scale) in rel.
// Arnoldi steps between two looks of the host at the device-side GMRES state
// (a cycle whose systems have all converged runs at most this many steps
// too many)
constexpr int kSyncEvery = 4;

void gmres_batch(aim_plan p, aim_precision prec, aim_pc_kind pc, const void* b, void* x, int nrhs,
                 const int32_t* dfreq, const std::vector<double>& scale, double tol, int m,
                 int max_iter, bool x_is_zero, hipStream_t s, CycleStats& st,
                 std::vector<double>& rel, const CycleHook* hook = nullptr, double gate = 0.0,
                 const std::vector<double>* tols = nullptr) {
  // per-system tolerances (tols, relative to scale) or one for all; on the
  // device they are folded into the scales (estimate / (scale tol_r / tol)
  // against tol)
  auto tol_of = [&](int r) { return tols ? (*tols)[r] : tol; };
  std::vector<double> prev_rel;
  auto& w = p->sv;
  const int64_t n = op_n(p);
  const size_t vec = size_t(n) * 16;
  // basis layout [i][r][n]: the i-th vectors of all systems are contiguous
  const int64_t si = nrhs, sr = 1;
  // a batch of uneven geometries: each system's Krylov vectors use only its
  // own N_i rows (the padding stays as it is and is never read)
  const int32_t* rows = p->batch ? p->d_inst_rows : nullptr;
  std::vector<int>& active_iters = st.iters;
  active_iters.assign(nrhs, 0);
  rel.assign(nrhs, 1.0);
  std::vector<double> beta(nrhs);
  bool first = true;
  // complex64 inner solves stop each system at complex64's accuracy floor,
  // which shows in two ways: the system stopped its last cycle on its
  // residual estimate but its true residual is still above tol (the estimate
  // has run past what complex64 matvecs resolve, and further cycles are a
  // few steps long), or its true relative residual is below kC64Floor and
  // fell by less than a tenth over the last cycle (slow but genuine
  // convergence, e.g. 1.3x per cycle on the 327,680-triangle sphere, is left
  // alone).  A system that shows either at two restarts in a row is parked
  // (frozen for the rest of this solve); the solve returns when every system
  // has converged, reached max_iter or been parked, and the refinement loop
  // recomputes the residuals in complex128.
  constexpr double kC64Floor = 1e-4;
  std::vector<int> gaps(nrhs, 0);
  std::vector<char> parked(nrhs, 0), est_stop(nrhs, 0), frozen0(nrhs, 0);
  for (;;) {
    // r = b - A x (skipped when x is known to be zero)
    if (first && x_is_zero) {
      AIM_HIP(hipMemcpyAsync(w.r, b, vec * nrhs, hipMemcpyDeviceToDevice, s));
    } else {
      apply_A(p, prec, x, w.r, nrhs, dfreq, s);
      st.matvecs++;
      aim::launch_residual(b, w.r, n * int64_t(nrhs), s);
    }
    first = false;
    norms_host(p, w.r, nrhs, s, beta);
    int maxit_left = 0;
    for (int r = 0; r < nrhs; ++r) {
      rel[r] = beta[r] / scale[r];
      if (!std::isfinite(rel[r])) throw Error(AIM_ERR_BREAKDOWN, "non-finite residual");
      maxit_left = std::max(maxit_left, max_iter - active_iters[r]);
    }
    if (gate > 0.0 && !prev_rel.empty())
      for (int r = 0; r < nrhs; ++r)
        if (rel[r] > tol_of(r) && rel[r] > gate * prev_rel[r]) throw GateFail{};
    if (prec == AIM_C64 && !prev_rel.empty())
      for (int r = 0; r < nrhs; ++r)
        if (rel[r] > tol_of(r) && active_iters[r] < max_iter && !parked[r]) {
          const bool stalled = rel[r] < kC64Floor && rel[r] > 0.9 * prev_rel[r];
          gaps[r] = (stalled || est_stop[r]) ? gaps[r] + 1 : 0;
          if (gaps[r] >= 2) parked[r] = 1;
        }
    bool all_done = true;
    for (int r = 0; r < nrhs; ++r)
      if (rel[r] > tol_of(r) && active_iters[r] < max_iter && !parked[r]) all_done = false;
    prev_rel = rel;
    if (hook) (*hook)(x, w.r, rel);
    if (all_done) return;
    const int mm = std::min(m, maxit_left);
    // V_0 = r / beta
    aim::launch_scale_inv(w.r, w.nrm, w.V, n, nrhs, n, s, nullptr, rows);
    // cycle state on the device: g = (beta, 0, ...), the frozen flags and the
    // step counts; the Hessenberg columns and rotations stay there too, and
    // the host looks at the state only every kSyncEvery steps
    const int mc = w.m;  // column capacity of H, cs, sn, g
    for (int r = 0; r < nrhs; ++r) {
      for (int i = 0; i <= mc; ++i) w.g_host[size_t(r) * (mc + 1) + i] = make_double2(0.0, 0.0);
      w.g_host[size_t(r) * (mc + 1)] = make_double2(beta[r], 0.0);
      w.gst_host[r].len = 0;
      w.gst_host[r].frozen =
          (rel[r] <= tol_of(r) || active_iters[r] >= max_iter || parked[r]) ? 1 : 0;
      frozen0[r] = w.gst_host[r].frozen;
      w.gst_host[r].iters = active_iters[r];
      w.gst_host[r].nonfinite = 0;
      w.scale_host[r] = scale[r] * tol_of(r) / tol;
    }
    // systems stopped at the cycle's start (and, from each look of the host
    // on, those stopped since) need no matvec: on a batch plan their
    // instances are skipped, and the Krylov kernels and the Givens step never
    // read their rows of the product (they exit on the frozen flag)
    std::vector<char> skip(nrhs);
    for (int r = 0; r < nrhs; ++r) skip[r] = w.gst_host[r].frozen ? 1 : 0;
    AIM_HIP(hipMemcpyAsync(w.g, w.g_host, sizeof(double2) * nrhs * (mc + 1),
                           hipMemcpyHostToDevice, s));
    AIM_HIP(hipMemcpyAsync(w.gst, w.gst_host, sizeof(aim::GivensState) * nrhs,
                           hipMemcpyHostToDevice, s));
    AIM_HIP(hipMemcpyAsync(w.scale, w.scale_host, sizeof(double) * nrhs, hipMemcpyHostToDevice,
                           s));
    int j = 0;
    for (; j < mm; ++j) {
      void* Vj = static_cast<char*>(w.V) + size_t(j) * nrhs * vec;
      // z_j = M(v_j); without a preconditioner the basis Z is V itself
      void* Zj = pc == AIM_PC_NONE ? Vj : static_cast<char*>(w.Z) + size_t(j) * nrhs * vec;
      if (pc != AIM_PC_NONE) apply_M(p, pc, Vj, Zj, nrhs, dfreq, s, p->batch ? skip.data() : nullptr);
      apply_A(p, prec, Zj, w.d, nrhs, dfreq, s, p->batch ? skip.data() : nullptr);  // w.d = A z_j
      st.matvecs++;
      // classical Gram-Schmidt, twice
      // (systems frozen by the Givens step are skipped on the device; their
      // columns past len are never used)
      // (the updates sum the dot partials themselves and the scaling the
      // norm partials, so no reduction launches; the coefficients h, h2 and
      // the norm land in w.h, w.h2 and w.nrm for the Givens step)
      aim::launch_block_dot_partials(w.V, si, sr, w.d, n, j + 1, nrhs, w.partial, s, w.gst, rows);
      aim::launch_gs_update(w.V, si, sr, w.d, n, j + 1, nrhs, w.partial, w.h, s, w.gst, rows);
      aim::launch_block_dot_partials(w.V, si, sr, w.d, n, j + 1, nrhs, w.partial, s, w.gst, rows);
      aim::launch_gs_update(w.V, si, sr, w.d, n, j + 1, nrhs, w.partial, w.h2, s, w.gst, rows);
      aim::launch_norm_partials(w.d, n, nrhs, w.partial, s, w.gst, rows);
      aim::launch_scale_norm(w.d, w.partial, w.nrm,
                             static_cast<char*>(w.V) + size_t(j + 1) * nrhs * vec, n, nrhs, n, s,
                             w.gst, rows);
      aim::launch_givens_step(w.h, w.h2, w.nrm, nrhs, j, mc, w.H, w.cs, w.sn, w.g, w.gst, w.scale,
                              tol, max_iter, s);
      if ((j + 1) % kSyncEvery == 0 || j + 1 == mm) {
        AIM_HIP(hipMemcpyAsync(w.gst_host, w.gst, sizeof(aim::GivensState) * nrhs,
                               hipMemcpyDeviceToHost, s));
        AIM_HIP(hipStreamSynchronize(s));
        bool all_frozen = true;
        for (int r = 0; r < nrhs; ++r) {
          if (w.gst_host[r].nonfinite) throw Error(AIM_ERR_BREAKDOWN, "non-finite Arnoldi norm");
          if (!w.gst_host[r].frozen) all_frozen = false;
          skip[r] = w.gst_host[r].frozen ? 1 : 0;
        }
        if (all_frozen) {
          ++j;
          break;
        }
      }
    }
    // the cycle's columns of H and g back to the host
    AIM_HIP(hipMemcpyAsync(w.H_host, w.H, sizeof(double2) * ((nrhs - 1) * size_t(mc) + j) * (mc + 1),
                           hipMemcpyDeviceToHost, s));
    AIM_HIP(hipMemcpyAsync(w.g_host, w.g, sizeof(double2) * nrhs * (mc + 1),
                           hipMemcpyDeviceToHost, s));
    AIM_HIP(hipMemcpyAsync(w.gst_host, w.gst, sizeof(aim::GivensState) * nrhs,
                           hipMemcpyDeviceToHost, s));
    AIM_HIP(hipStreamSynchronize(s));
    std::vector<int> len(nrhs, 0);
    for (int r = 0; r < nrhs; ++r) {
      if (w.gst_host[r].nonfinite) throw Error(AIM_ERR_BREAKDOWN, "non-finite Arnoldi norm");
      len[r] = w.gst_host[r].len;
      active_iters[r] = w.gst_host[r].iters;
      // stopped during this cycle on its residual estimate
      est_stop[r] = (w.gst_host[r].frozen && !frozen0[r] && active_iters[r] < max_iter) ? 1 : 0;
    }
    // y = H^{-1} g per system (H upper triangular after the rotations), then
    // x += Z y
    const int nv = *std::max_element(len.begin(), len.end());
    if (nv > 0) {
      std::vector<double2> yh(size_t(nrhs) * m);
      for (auto& v : yh) v.x = v.y = 0.0;
      for (int r = 0; r < nrhs; ++r) {
        const int L = len[r];
        auto Hat = [&](int i, int c) {
          const double2 e = w.H_host[(size_t(r) * mc + c) * (mc + 1) + i];
          return cplx(e.x, e.y);
        };
        std::vector<cplx> yv(L);
        for (int i = L - 1; i >= 0; --i) {
          const double2 gi = w.g_host[size_t(r) * (mc + 1) + i];
          cplx acc(gi.x, gi.y);
          for (int c = i + 1; c < L; ++c) acc -= Hat(i, c) * yv[c];
          yv[i] = acc / Hat(i, i);
        }
        for (int i = 0; i < L; ++i) {
          yh[size_t(r) * m + i].x = yv[i].real();
          yh[size_t(r) * m + i].y = yv[i].imag();
        }
      }
      AIM_HIP(hipMemcpyAsync(w.y, yh.data(), sizeof(double2) * yh.size(), hipMemcpyHostToDevice, s));
      aim::launch_combine(pc == AIM_PC_NONE ? w.V : w.Z, si, sr, w.y, m, nv, x, n, nrhs, w.gst, s,
                          rows);
      AIM_HIP(hipStreamSynchronize(s));  // yh is pageable host memory
    }
  }
}

}  // namespace

extern "C" aim_status aim_solve(aim_plan p, const void* b, void* x, int32_t nrhs,
                                const int32_t* freq_idx_host, const aim_solve_opts* opts,
                                aim_solve_info* info, void* hip_stream) {
  if (!p || !b || !x || !opts || !info) return fail(AIM_ERR_INVALID_ARG, "null argument");
  aim_status result = AIM_OK;
  const aim_status st = guarded([&] {
    const aim_solve_opts& o = *opts;
    AIM_REQUIRE(o.rtol > 0.0 && std::isfinite(o.rtol), AIM_ERR_INVALID_ARG, "rtol must be positive");
    AIM_REQUIRE(o.restart >= 1 && o.restart <= 200, AIM_ERR_INVALID_ARG, "restart must be in 1..200");
    AIM_REQUIRE(o.max_iter >= 1, AIM_ERR_INVALID_ARG, "max_iter must be >= 1");
    AIM_REQUIRE(o.pc >= AIM_PC_NONE && o.pc <= AIM_PC_NEARBLOCK_STATIC, AIM_ERR_INVALID_ARG,
                "unknown preconditioner");
    AIM_REQUIRE(o.fallback_pc >= AIM_PC_NONE && o.fallback_pc <= AIM_PC_NEARBLOCK_STATIC &&
                    o.fallback_pc != AIM_PC_UNET,
                AIM_ERR_INVALID_ARG, "fallback preconditioner must be a classical one");
    AIM_REQUIRE(o.pc != AIM_PC_UNET || p->unet != nullptr, AIM_ERR_STATE,
                "no learned preconditioner attached (aim_plan_set_unet)");
    check_prec(p, AIM_C128);
    check_prec(p, o.inner);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const double t0 = now_s();
    const int32_t* df = set_freq(p, freq_idx_host, nrhs, s);
    ensure_solver(p, nrhs, o.restart, s);
    // full-kernel near-block inverses at the systems' wavenumbers, if used
    if (o.pc == AIM_PC_NEARBLOCK || o.fallback_pc == AIM_PC_NEARBLOCK ||
        (o.pc == AIM_PC_UNET && p->unet_base == AIM_PC_NEARBLOCK))
      ensure_nearblock_for(p, freq_idx_host, nrhs, s);
    auto& w = p->sv;
    const int64_t n = p->t.N;
    const size_t vec = size_t(n) * 16;
    std::vector<double> bn;
    norms_host(p, b, nrhs, s, bn);
    for (int r = 0; r < nrhs; ++r)
      AIM_REQUIRE(std::isfinite(bn[r]), AIM_ERR_BREAKDOWN, "non-finite right-hand side");
    std::vector<double> scale(nrhs);
    for (int r = 0; r < nrhs; ++r) scale[r] = bn[r] > 0.0 ? bn[r] : 1.0;
    std::vector<aim_solve_info> inf(nrhs);
    for (auto& v : inf) std::memset(&v, 0, sizeof(v));
    CycleStats cst;
    std::vector<double> rel;
    // The learned preconditioner is gated: if a restart cycle fails to cut a
    // residual by at least the gate factor, or a value is not finite, the
    // solve continues from the current iterate with the fallback
    // preconditioner (unpreconditioned or near-block GMRES).
    aim_pc_kind pc = o.pc;
    const double gate = pc == AIM_PC_UNET ? (o.gate > 0.0 ? o.gate : 0.7) : 0.0;
    int fallback = 0;
    auto run = [&](aim_pc_kind use_pc, double use_gate) {
      if (o.inner == AIM_C128) {
        AIM_HIP(hipMemcpyAsync(w.xp, x, vec * nrhs, hipMemcpyDeviceToDevice, s));
        CycleStats cs;
        gmres_batch(p, AIM_C128, use_pc, b, w.xp, nrhs, df, scale, o.rtol, o.restart, o.max_iter,
                    false, s, cs, rel, nullptr, use_gate);
        AIM_HIP(hipMemcpyAsync(x, w.xp, vec * nrhs, hipMemcpyDeviceToDevice, s));
        cst.matvecs += cs.matvecs;
        for (int r = 0; r < nrhs; ++r) {
          inf[r].matvecs = cst.matvecs;
          inf[r].iters += cs.iters[r];
        }
      } else {
        // complex128 iterative refinement around a complex64-matvec GMRES
        const double inner_tol = o.inner_rtol > 0.0 ? o.inner_rtol : 1e-4;
        int refine = 0;
        std::vector<double> rn;
        for (;;) {
          apply_A(p, AIM_C128, x, w.bp, nrhs, df, s);  // bp = A x (complex128)
          cst.matvecs++;
          aim::launch_residual(b, w.bp, n * int64_t(nrhs), s);  // bp = b - A x
          norms_host(p, w.bp, nrhs, s, rn);
          bool done = true;
          rel.assign(nrhs, 0.0);
          for (int r = 0; r < nrhs; ++r) {
            rel[r] = rn[r] / scale[r];
            if (!std::isfinite(rel[r])) throw Error(AIM_ERR_BREAKDOWN, "non-finite residual");
            if (rel[r] > o.rtol) done = false;
          }
          if (done || refine >= std::max(0, o.max_refine)) break;
          // systems already at rtol get a zero inner right-hand side, so the
          // inner solve stops them at once (and a batch plan skips them)
          for (int r = 0; r < nrhs; ++r)
            if (rel[r] <= o.rtol)
              aim::launch_zero_words(static_cast<char*>(w.bp) + size_t(r) * vec, int64_t(n) * 2, s);
          std::vector<double> iscale(nrhs);
          for (int r = 0; r < nrhs; ++r) iscale[r] = rn[r] > 0.0 ? rn[r] : 1.0;
          AIM_HIP(hipMemsetAsync(w.xp, 0, vec * nrhs, s));
          // inner tolerance per system: enough to reach rtol from its residual,
          // but not below what complex64 matvecs can resolve (unless the
          // caller fixed it)
          std::vector<double> itols(nrhs, inner_tol);
          if (o.inner_rtol <= 0.0)
            for (int r = 0; r < nrhs; ++r)
              itols[r] = std::max(3e-6, std::min(0.1, 0.3 * o.rtol / std::max(rel[r], 1e-300)));
          const double itol = *std::min_element(itols.begin(), itols.end());
          std::vector<double> irel;
          CycleStats ist;
          gmres_batch(p, AIM_C64, use_pc, w.bp, w.xp, nrhs, df, iscale, itol, o.restart,
                      o.max_iter, true, s, ist, irel, nullptr, use_gate, &itols);
          cst.matvecs += ist.matvecs;
          for (int r = 0; r < nrhs; ++r) inf[r].iters += ist.iters[r];
          aim::launch_axpy_inplace(x, w.xp, n * int64_t(nrhs), s);
          ++refine;
          for (int r = 0; r < nrhs; ++r) inf[r].refinements = refine;
        }
        for (int r = 0; r < nrhs; ++r) inf[r].matvecs = cst.matvecs;
      }
    };
    if (pc == AIM_PC_UNET) {
      try {
        run(pc, gate);
        bool ok = true;
        for (int r = 0; r < nrhs; ++r) ok = ok && rel[r] <= o.rtol;
        if (!ok) fallback = 1;
      } catch (const GateFail&) {
        // the gate fires at a restart, where the iterate is finite and its
        // residual was just measured: keep the progress made so far
        fallback = 1;
        if (o.inner == AIM_C128)
          AIM_HIP(hipMemcpyAsync(x, w.xp, vec * nrhs, hipMemcpyDeviceToDevice, s));
        else
          aim::launch_axpy_inplace(x, w.xp, n * int64_t(nrhs), s);
      } catch (const Error& e) {
        if (e.status != AIM_ERR_BREAKDOWN) throw;
        // a non-finite value: x holds the last finite iterate unless the
        // breakdown came from the outer residual, in which case start over
        fallback = 1;
        std::vector<double> xn;
        norms_host(p, x, nrhs, s, xn);
        bool finite = true;
        for (double v : xn) finite = finite && std::isfinite(v);
        if (!finite) AIM_HIP(hipMemsetAsync(x, 0, vec * nrhs, s));
      }
      if (fallback) run(o.fallback_pc, 0.0);
    } else {
      run(pc, 0.0);
    }
    for (int r = 0; r < nrhs; ++r) inf[r].fallback_used = fallback;
    AIM_HIP(hipStreamSynchronize(s));
    const double secs = now_s() - t0;
    bool all = true;
    for (int r = 0; r < nrhs; ++r) {
      inf[r].rel_resid = rel[r];
      inf[r].converged = rel[r] <= o.rtol ? 1 : 0;
      inf[r].seconds = secs;
      all = all && inf[r].converged;
    }
    std::memcpy(info, inf.data(), sizeof(aim_solve_info) * nrhs);
    if (!all) result = AIM_ERR_NOT_CONVERGED;
  });
  if (st != AIM_OK) return st;
  if (result != AIM_OK) return fail(result, "not every right-hand side reached rtol");
  return AIM_OK;
}

// Krylov solves of the RWG operators (the same batched GMRES as aim_solve)
extern "C" aim_status aim_solve_rwg(aim_plan p, int32_t op, double gram_coef, const void* b,
                                    void* x, int32_t nrhs, const int32_t* freq_idx_host,
                                    const aim_solve_opts* opts, aim_solve_info* info,
                                    void* hip_stream) {
  if (!p || !b || !x || !opts || !info) return fail(AIM_ERR_INVALID_ARG, "null argument");
  aim_status result = AIM_OK;
  const aim_status st = guarded([&] {
    const aim_solve_opts& o = *opts;
    AIM_REQUIRE(op >= 1 && op <= 3, AIM_ERR_INVALID_ARG, "op must be 1 (EFIE), 2 or 3");
    AIM_REQUIRE(std::isfinite(gram_coef), AIM_ERR_INVALID_ARG, "gram_coef must be finite");
    AIM_REQUIRE(o.rtol > 0.0 && std::isfinite(o.rtol), AIM_ERR_INVALID_ARG, "rtol must be positive");
    AIM_REQUIRE(o.restart >= 1 && o.restart <= 200, AIM_ERR_INVALID_ARG, "restart must be in 1..200");
    AIM_REQUIRE(o.max_iter >= 1, AIM_ERR_INVALID_ARG, "max_iter must be >= 1");
    AIM_REQUIRE(o.pc == AIM_PC_NONE && o.inner == AIM_C128, AIM_ERR_INVALID_ARG,
                "the RWG operators are solved unpreconditioned in complex128");
    check_rwg_call(p, b, x, nrhs);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const std::vector<int32_t> fr = freq_list(p, nrhs, freq_idx_host);
    if (op == 1) ensure_efie(p, s);
    else ensure_mfie(p, s);
    // the Krylov loop applies this operator for the duration of the call
    struct Restore {
      aim_plan q;
      ~Restore() { q->rwg_op = 0; }
    } restore{p};
    p->rwg_op = op;
    p->rwg_gram = gram_coef;
    p->rwg_fr = fr;
    const double t0 = now_s();
    ensure_solver(p, nrhs, o.restart, s);
    auto& w = p->sv;
    const size_t vec = size_t(p->efie.n) * 16;
    std::vector<double> bn;
    norms_host(p, b, nrhs, s, bn);
    for (int r = 0; r < nrhs; ++r)
      AIM_REQUIRE(std::isfinite(bn[r]), AIM_ERR_BREAKDOWN, "non-finite right-hand side");
    std::vector<double> scale(nrhs);
    for (int r = 0; r < nrhs; ++r) scale[r] = bn[r] > 0.0 ? bn[r] : 1.0;
    AIM_HIP(hipMemcpyAsync(w.xp, x, vec * nrhs, hipMemcpyDeviceToDevice, s));
    CycleStats cs;
    std::vector<double> rel;
    gmres_batch(p, AIM_C128, AIM_PC_NONE, b, w.xp, nrhs, set_freq(p, freq_idx_host, nrhs, s),
                scale, o.rtol, o.restart, o.max_iter, false, s, cs, rel);
    AIM_HIP(hipMemcpyAsync(x, w.xp, vec * nrhs, hipMemcpyDeviceToDevice, s));
    AIM_HIP(hipStreamSynchronize(s));
    const double secs = now_s() - t0;
    std::vector<aim_solve_info> inf(nrhs);
    bool all = true;
    for (int r = 0; r < nrhs; ++r) {
      std::memset(&inf[r], 0, sizeof(aim_solve_info));
      inf[r].iters = cs.iters[r];
      inf[r].matvecs = cs.matvecs;
      inf[r].rel_resid = rel[r];
      inf[r].converged = rel[r] <= o.rtol ? 1 : 0;
      inf[r].seconds = secs;
      all = all && inf[r].converged;
    }
    std::memcpy(info, inf.data(), sizeof(aim_solve_info) * nrhs);
    if (!all) result = AIM_ERR_NOT_CONVERGED;
  });
  if (st != AIM_OK) return st;
  if (result != AIM_OK) return fail(result, "not every right-hand side reached rtol");
  return AIM_OK;
}

// ---------------------------------------------------------------------------
// learned preconditioner: attach, training pairs, targets, training steps
// ---------------------------------------------------------------------------
extern "C" aim_status aim_plan_set_unet(aim_plan p, aim_unet net, aim_pc_kind base_pc,
                                        double tau) {
  if (!p) return fail(AIM_ERR_INVALID_ARG, "null plan");
  return guarded([&] {
    AIM_REQUIRE(base_pc >= AIM_PC_NONE && base_pc <= AIM_PC_NEARBLOCK_STATIC &&
                    base_pc != AIM_PC_UNET,
                AIM_ERR_INVALID_ARG, "base preconditioner must be a classical one");
    AIM_REQUIRE(std::isfinite(tau) && tau > 0.0, AIM_ERR_INVALID_ARG, "tau must be positive");
    // a batch plan: every instance applies the same network on its own grid
    std::vector<aim_plan_s*> targets;
    if (p->batch)
      for (auto& q : p->inst) targets.push_back(q.get());
    for (aim_plan_s* q : targets)
      if (net) check_unet_plan(q);
    if (!p->batch && net) check_unet_plan(p);
    for (aim_plan_s* q : targets) {
      q->unet = net;
      q->unet_base = base_pc;
      q->unet_tau = tau;
    }
    p->unet = net;
    p->unet_base = base_pc;
    p->unet_tau = tau;
  });
}

extern "C" aim_status aim_log_pairs(aim_plan p, const void* b, int32_t nrhs,
                                    const int32_t* freq_idx_host, double rtol, int32_t restart,
                                    int32_t max_iter, void* r_out, void* e_out,
                                    int32_t* rhs_out_host, int32_t max_pairs, int32_t* npairs,
                                    void* hip_stream) {
  if (!p || !b || !r_out || !e_out || !npairs) return fail(AIM_ERR_INVALID_ARG, "null argument");
  aim_status result = AIM_OK;
  const aim_status st = guarded([&] {
    AIM_REQUIRE(rtol > 0.0 && std::isfinite(rtol), AIM_ERR_INVALID_ARG, "rtol must be positive");
    AIM_REQUIRE(restart >= 1 && restart <= 200, AIM_ERR_INVALID_ARG, "restart must be in 1..200");
    AIM_REQUIRE(max_iter >= 1, AIM_ERR_INVALID_ARG, "max_iter must be >= 1");
    AIM_REQUIRE(max_pairs >= 0, AIM_ERR_INVALID_ARG, "max_pairs must be >= 0");
    check_prec(p, AIM_C128);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int32_t* df = set_freq(p, freq_idx_host, nrhs, s);
    ensure_solver(p, nrhs, restart, s);
    auto& w = p->sv;
    const int64_t n = p->t.N;
    const size_t vec = size_t(n) * 16;
    std::vector<double> bn;
    norms_host(p, b, nrhs, s, bn);
    std::vector<double> scale(nrhs);
    for (int r = 0; r < nrhs; ++r) {
      AIM_REQUIRE(std::isfinite(bn[r]), AIM_ERR_BREAKDOWN, "non-finite right-hand side");
      scale[r] = bn[r] > 0.0 ? bn[r] : 1.0;
    }
    AIM_HIP(hipMemsetAsync(w.xp, 0, vec * nrhs, s));
    int count = 0;
    std::vector<int32_t> owner;
    // at every restart, (r_t, x_t) of each unconverged system is stored
    CycleHook hook = [&](const void* x, const void* rr, const std::vector<double>& rel) {
      for (int r = 0; r < nrhs && count < max_pairs; ++r) {
        if (!(rel[r] > rtol)) continue;
        AIM_HIP(hipMemcpyAsync(static_cast<char*>(r_out) + size_t(count) * vec,
                               static_cast<const char*>(rr) + size_t(r) * vec, vec,
                               hipMemcpyDeviceToDevice, s));
        AIM_HIP(hipMemcpyAsync(static_cast<char*>(e_out) + size_t(count) * vec,
                               static_cast<const char*>(x) + size_t(r) * vec, vec,
                               hipMemcpyDeviceToDevice, s));
        owner.push_back(r);
        ++count;
      }
    };
    CycleStats cs;
    std::vector<double> rel;
    gmres_batch(p, AIM_C128, AIM_PC_NONE, b, w.xp, nrhs, df, scale, rtol, restart, max_iter, true,
                s, cs, rel, &hook);
    // e_t = x* - x_t against the converged solution
    for (int k = 0; k < count; ++k)
      aim::launch_pair_error(static_cast<const char*>(w.xp) + size_t(owner[k]) * vec,
                             static_cast<char*>(e_out) + size_t(k) * vec, n, s);
    AIM_HIP(hipStreamSynchronize(s));
    *npairs = count;
    if (rhs_out_host) std::copy(owner.begin(), owner.end(), rhs_out_host);
    for (int r = 0; r < nrhs; ++r)
      if (!(rel[r] <= rtol)) result = AIM_ERR_NOT_CONVERGED;
  });
  if (st != AIM_OK) return st;
  if (result != AIM_OK) return fail(result, "a logging solve did not reach rtol");
  return AIM_OK;
}

extern "C" aim_status aim_pc_targets(aim_plan p, aim_pc_kind base_pc, aim_pc_loss kind,
                                     const void* r_pairs, const void* e_pairs, int32_t npairs,
                                     void* grid_out, void* target_out, double* sums_host,
                                     void* hip_stream) {
  if (!p || (npairs > 0 && (!r_pairs || !e_pairs || !grid_out || !target_out)))
    return fail(AIM_ERR_INVALID_ARG, "null argument");
  return guarded([&] {
    no_batch(p);
    AIM_REQUIRE(npairs >= 0, AIM_ERR_INVALID_ARG, "npairs must be >= 0");
    AIM_REQUIRE(base_pc >= AIM_PC_NONE && base_pc <= AIM_PC_NEARBLOCK_STATIC &&
                    base_pc != AIM_PC_UNET,
                AIM_ERR_INVALID_ARG, "base preconditioner must be a classical one");
    AIM_REQUIRE(kind == AIM_LOSS_ERROR || kind == AIM_LOSS_RESIDUAL, AIM_ERR_INVALID_ARG,
                "unknown loss kind");
    check_unet_plan(p);
    if (kind == AIM_LOSS_RESIDUAL) check_prec(p, AIM_C128);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    ensure_solver(p, p->max_rhs, 1, s);  // norms of up to max_rhs targets at once
    const int64_t n = p->t.N, Ng = p->g.Ng;
    const size_t vec = size_t(n) * 16;
    double err2 = 0.0, res2 = 0.0;
    std::vector<double> tn;
    for (int k0 = 0; k0 < npairs; k0 += p->max_rhs) {
      const int nb = std::min(p->max_rhs, npairs - k0);
      const char* rr = static_cast<const char*>(r_pairs) + size_t(k0) * vec;
      const char* ee = static_cast<const char*>(e_pairs) + size_t(k0) * vec;
      char* tg = static_cast<char*>(target_out) + size_t(k0) * vec;
      unet_input(p, rr, nb, static_cast<char*>(grid_out) + size_t(k0) * Ng * 8, s);
      void* br = p->sv.w;
      // the pairs are logged at wavenumber index 0
      const int32_t* df0 = set_freq(p, nullptr, nb, s);
      if (base_pc == AIM_PC_NEARBLOCK) ensure_nearblock(p, 0, s);
      apply_base(p, base_pc, rr, br, nb, df0, s);  // B r
      if (kind == AIM_LOSS_RESIDUAL) {
        // s = (r - A B r) / ||r||: what is left of the normalised residual
        // after the base preconditioner's step
        const int32_t* df = set_freq(p, nullptr, nb, s);
        matvec_any(p, AIM_C128, br, tg, nb, df, s);
        aim::launch_unet_resid_target(rr, p->u_s, tg, n, nb, s);
        norms_host(p, tg, nb, s, tn);
        for (double v : tn) res2 += v * v;
      }
      // (e - B r) / ||r||: the error the network has to supply
      aim::launch_unet_resid_target(ee, p->u_s, br, n, nb, s);
      if (kind == AIM_LOSS_ERROR)
        AIM_HIP(hipMemcpyAsync(tg, br, vec * nb, hipMemcpyDeviceToDevice, s));
      norms_host(p, br, nb, s, tn);
      for (double v : tn) err2 += v * v;
    }
    AIM_HIP(hipStreamSynchronize(s));
    AIM_REQUIRE(std::isfinite(err2) && std::isfinite(res2), AIM_ERR_BREAKDOWN,
                "non-finite training target");
    if (sums_host) {
      sums_host[0] = err2;
      sums_host[1] = res2;
    }
  });
}

extern "C" aim_status aim_pc_train_step(aim_plan p, aim_unet net, aim_pc_loss kind,
                                        const void* grids, const void* targets, int32_t npairs,
                                        const int32_t* sample_idx_host, int32_t nsamples,
                                        double tau, double weight, double lr, int32_t apply,
                                        double* loss_host, void* hip_stream) {
  if (!p || !net || !grids || !targets || !sample_idx_host)
    return fail(AIM_ERR_INVALID_ARG, "null argument");
  return guarded([&] {
    no_batch(p);
    AIM_REQUIRE(nsamples >= 1, AIM_ERR_INVALID_ARG, "nsamples must be >= 1");
    AIM_REQUIRE(std::isfinite(tau) && tau > 0.0, AIM_ERR_INVALID_ARG, "tau must be positive");
    AIM_REQUIRE(std::isfinite(lr) && lr >= 0.0, AIM_ERR_INVALID_ARG, "lr must be >= 0");
    AIM_REQUIRE(kind == AIM_LOSS_ERROR || kind == AIM_LOSS_RESIDUAL, AIM_ERR_INVALID_ARG,
                "unknown loss kind");
    AIM_REQUIRE(std::isfinite(weight) && weight > 0.0, AIM_ERR_INVALID_ARG,
                "weight must be positive");
    for (int i = 0; i < nsamples; ++i)
      AIM_REQUIRE(sample_idx_host[i] >= 0 && sample_idx_host[i] < npairs, AIM_ERR_INVALID_ARG,
                  "sample index out of range");
    check_unet_plan(p);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    ensure_unet_buffers(p, s);
    const int64_t n = p->t.N, Ng = p->g.Ng;
    constexpr int kParts = 64;
    AIM_REQUIRE(int64_t(kParts) * nsamples * 8 <= int64_t(16) * 4096 +
                    int64_t(16) * p->max_rhs * ((std::max(n, Ng) + 4095) / 4096),
                AIM_ERR_INVALID_ARG, "too many samples in one step");
    double* part = static_cast<double*>(p->upart);
    aim::unet_zero_grad(net, s);
    const double inv_cnt = 1.0 / (double(n) * nsamples);
    // groups of up to max_rhs samples, each one batched pass: the selected
    // grids are gathered one after another (stacked along z for the network)
    for (int i0 = 0; i0 < nsamples; i0 += p->max_rhs) {
      const int nb = std::min(p->max_rhs, nsamples - i0);
      for (int j = 0; j < nb; ++j)
        AIM_HIP(hipMemcpyAsync(static_cast<char*>(p->ug_x) + size_t(j) * Ng * 8,
                               static_cast<const char*>(grids) +
                                   size_t(sample_idx_host[i0 + j]) * Ng * 8,
                               size_t(Ng) * 8, hipMemcpyDeviceToDevice, s));
      aim::unet_forward(net, p->ug_x, nb, p->g.N[2], p->g.N[1], p->g.N[0], p->ug_out, s);
      interp_near<float>(p, AIM_C64, p->ug_out, nullptr, p->um2, nb, true, false, s);
      auto mesh = [&](void* base, int j) { return static_cast<char*>(base) + size_t(j) * n * 8; };
      auto target = [&](int j) {
        return static_cast<const char*>(targets) + size_t(sample_idx_host[i0 + j]) * n * 16;
      };
      if (kind == AIM_LOSS_ERROR) {
        for (int j = 0; j < nb; ++j)
          aim::launch_mesh_mse(mesh(p->um2, j), target(j), p->d_area, 1.0 / tau, n,
                               inv_cnt * weight, mesh(p->um1, j),
                               part + size_t(i0 + j) * kParts, kParts, s);
      } else {
        // loss = weight mean |s - A z|^2, z = tau c / area; its gradient with
        // respect to c is -2 weight tau A^H (s - A z) / (area cnt)
        const int32_t* df = set_freq(p, nullptr, nb, s);
        for (int j = 0; j < nb; ++j)
          aim::launch_area_scale_c64(mesh(p->um2, j), p->d_area, tau, mesh(p->um1, j), n, s);
        matvec_any(p, AIM_C64, p->um1, p->um2, nb, df, s);
        for (int j = 0; j < nb; ++j)
          aim::launch_resid_loss(mesh(p->um2, j), target(j), weight * inv_cnt, n,
                                 mesh(p->um1, j), part + size_t(i0 + j) * kParts, kParts, s);
        matvec_any(p, AIM_C64, p->um1, p->um2, nb, df, s);
        for (int j = 0; j < nb; ++j)
          aim::launch_resid_grad(mesh(p->um2, j), p->d_area, -2.0 * weight * tau * inv_cnt,
                                 mesh(p->um1, j), n, s);
      }
      // d loss / d grid output = P (d loss / d mesh output), as the mesh
      // output is P^T of the grid output
      aim::launch_project<float>(p->g, p_dev(p, AIM_C64), p->d_pblk, p->nblk, p->um1, n,
                                 p->ug_in, nb, s);
      aim::unet_backward(net, p->ug_x, p->ug_in, s);
    }
    if (apply) aim::unet_adam(net, lr, s);
    std::vector<double> hp(size_t(kParts) * nsamples);
    AIM_HIP(hipMemcpyAsync(hp.data(), part, hp.size() * 8, hipMemcpyDeviceToHost, s));
    AIM_HIP(hipStreamSynchronize(s));
    double loss = 0.0;
    for (double v : hp) loss += v;
    if (loss_host) *loss_host = loss;
  });
}

// ---------------------------------------------------------------------------
// plan checkpoint: the frequency-independent host tables (the static near
// field, the precorrected C, P in both layouts, the preconditioner blocks),
// the wavenumbers and the tuned schedules, so that a later run skips the
// host set-up.  Little-endian binary: magic, version, header, length-prefixed
// arrays, FNV-1a 64 checksum of everything before it.  A loaded file is
// validated completely (sizes, index ranges, block structure, finiteness)
// before any of it reaches a device.
// ---------------------------------------------------------------------------
namespace {

constexpr char kPlanMagic[8] = {'A', 'I', 'M', 'X', 'P', 'L', 'A', 'N'};
constexpr uint32_t kPlanVersion = 1;

uint64_t fnv1a(const char* d, size_t n) {
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= uint8_t(d[i]);
    h *= 1099511628211ull;
  }
  return h;
}

struct Writer {
  std::string b;
  template <typename T>
  void pod(const T& v) {
    b.append(reinterpret_cast<const char*>(&v), sizeof(T));
  }
  template <typename T>
  void vec(const std::vector<T>& v) {
    pod(int64_t(v.size()));
    if (!v.empty()) b.append(reinterpret_cast<const char*>(v.data()), v.size() * sizeof(T));
  }
};

struct Reader {
  const std::string& b;
  size_t pos = 0;
  size_t end;
  template <typename T>
  void pod(T& v) {
    AIM_REQUIRE(end - pos >= sizeof(T), AIM_ERR_INVALID_ARG, "plan file truncated");
    std::memcpy(&v, b.data() + pos, sizeof(T));
    pos += sizeof(T);
  }
  template <typename T>
  void vec(std::vector<T>& v) {
    int64_t n = 0;
    pod(n);
    AIM_REQUIRE(n >= 0 && uint64_t(n) <= (end - pos) / sizeof(T), AIM_ERR_INVALID_ARG,
                "plan file truncated or corrupt");
    v.resize(size_t(n));
    if (n) std::memcpy(v.data(), b.data() + pos, size_t(n) * sizeof(T));
    pos += size_t(n) * sizeof(T);
  }
};

template <typename V>
void table_vectors(aim::HostTables& t, V&& f) {
  f(t.area);
  f(t.qp_xyz);
  f(t.qp_w);
  f(t.qp_start);
  f(t.qp_local);
  f(t.rowptr);
  f(t.col);
  f(t.near_static);
  f(t.corr);
  f(t.p_rowptr);
  f(t.p_col);
  f(t.p_val);
  f(t.p_blk);
  f(t.pt_rowptr);
  f(t.pt_col);
  f(t.pt_val);
  f(t.cl_ptr);
  f(t.cl_perm);
  f(t.cl_blk);
  f(t.cl_inv);
}

template <typename I>
void check_offsets(const std::vector<I>& off, int64_t rows, const char* what) {
  AIM_REQUIRE(int64_t(off.size()) == rows + 1 && off[0] == 0, AIM_ERR_INVALID_ARG,
              std::string("plan file: bad offsets of ") + what);
  for (int64_t i = 0; i < rows; ++i)
    AIM_REQUIRE(off[i + 1] >= off[i], AIM_ERR_INVALID_ARG,
                std::string("plan file: offsets of ") + what + " decrease");
}

template <typename I>
void check_range(const std::vector<I>& v, int64_t hi, const char* what) {
  for (const I x : v)
    AIM_REQUIRE(x >= 0 && int64_t(x) < hi, AIM_ERR_INVALID_ARG,
                std::string("plan file: index out of range in ") + what);
}

void check_finite(const std::vector<double>& v, const char* what) {
  for (const double x : v)
    AIM_REQUIRE(std::isfinite(x), AIM_ERR_INVALID_ARG,
                std::string("plan file: non-finite value in ") + what);
}

// every invariant the kernels rely on
void validate_tables(const aim::HostTables& t) {
  const int64_t N = t.N;
  AIM_REQUIRE(N >= 1 && N < (int64_t(1) << 31), AIM_ERR_INVALID_ARG, "plan file: bad size");
  AIM_REQUIRE(t.order == 2 || t.order == 3, AIM_ERR_INVALID_ARG, "plan file: bad stencil order");
  int64_t Ng = 1;
  for (int a = 0; a < 3; ++a) {
    const int d = t.dims[a];
    AIM_REQUIRE(d >= 8 && d <= 256 && (d & (d - 1)) == 0, AIM_ERR_INVALID_ARG,
                "plan file: bad grid dimension");
    Ng *= d;
  }
  AIM_REQUIRE(std::isfinite(t.h) && t.h > 0.0, AIM_ERR_INVALID_ARG, "plan file: bad spacing");
  AIM_REQUIRE(int64_t(t.area.size()) == N && int64_t(t.qp_w.size()) == 3 * N &&
                  int64_t(t.qp_xyz.size()) == 9 * N && int64_t(t.qp_start.size()) == 9 * N &&
                  int64_t(t.qp_local.size()) == 9 * N,
              AIM_ERR_INVALID_ARG, "plan file: bad quadrature tables");
  for (int64_t q = 0; q < 3 * N; ++q)
    for (int a = 0; a < 3; ++a) {
      const int32_t s0 = t.qp_start[3 * q + a];
      AIM_REQUIRE(s0 >= 0 && s0 + t.order <= t.dims[a] - 1, AIM_ERR_INVALID_ARG,
                  "plan file: stencil outside the grid");
    }
  check_finite(t.area, "areas");
  check_finite(t.qp_xyz, "quadrature points");
  check_finite(t.qp_w, "quadrature weights");
  check_finite(t.qp_local, "stencil coordinates");
  // near field
  check_offsets(t.rowptr, N, "C");
  const int64_t nnz = t.rowptr[N];
  AIM_REQUIRE(nnz < (int64_t(1) << 31) && int64_t(t.col.size()) == nnz &&
                  int64_t(t.near_static.size()) == nnz && int64_t(t.corr.size()) == nnz,
              AIM_ERR_INVALID_ARG, "plan file: bad near-field sizes");
  check_range(t.col, N, "C columns");
  check_finite(t.near_static, "A_s,NR");
  check_finite(t.corr, "C");
  // P by node, in row blocks
  check_offsets(t.p_rowptr, Ng, "P");
  const int64_t pn = t.p_rowptr[Ng];
  AIM_REQUIRE(int64_t(t.p_col.size()) == pn && int64_t(t.p_val.size()) == pn,
              AIM_ERR_INVALID_ARG, "plan file: bad P sizes");
  check_range(t.p_col, N, "P columns");
  check_finite(t.p_val, "P");
  AIM_REQUIRE(t.p_blk.size() >= 2 && t.p_blk.front() == 0 && t.p_blk.back() == Ng,
              AIM_ERR_INVALID_ARG, "plan file: bad P row blocks");
  for (size_t b = 0; b + 1 < t.p_blk.size(); ++b) {
    const int32_t r0 = t.p_blk[b], r1 = t.p_blk[b + 1];
    AIM_REQUIRE(r1 > r0, AIM_ERR_INVALID_ARG, "plan file: empty P row block");
    const int64_t nz = t.p_rowptr[r1] - t.p_rowptr[r0];
    AIM_REQUIRE(r1 - r0 == 1 || nz == 0 || (nz <= aim::kProjNnz && r1 - r0 <= aim::kProjRows),
                AIM_ERR_INVALID_ARG, "plan file: P row block too long");
  }
  // P^T by triangle
  check_offsets(t.pt_rowptr, N, "P^T");
  const int64_t tn = t.pt_rowptr[N];
  AIM_REQUIRE(int64_t(t.pt_col.size()) == tn && int64_t(t.pt_val.size()) == tn,
              AIM_ERR_INVALID_ARG, "plan file: bad P^T sizes");
  check_range(t.pt_col, Ng, "P^T columns");
  check_finite(t.pt_val, "P^T");
  // near-block preconditioner
  AIM_REQUIRE(t.cl_ptr.size() >= 2, AIM_ERR_INVALID_ARG, "plan file: no clusters");
  const int64_t ncl = int64_t(t.cl_ptr.size()) - 1;
  check_offsets(t.cl_ptr, ncl, "clusters");
  AIM_REQUIRE(t.cl_ptr[ncl] == N && int64_t(t.cl_perm.size()) == N, AIM_ERR_INVALID_ARG,
              "plan file: clusters do not cover the mesh");
  check_range(t.cl_perm, N, "cluster members");
  check_offsets(t.cl_blk, ncl, "cluster blocks");
  for (int64_t c = 0; c < ncl; ++c) {
    const int64_t m = t.cl_ptr[c + 1] - t.cl_ptr[c];
    AIM_REQUIRE(m >= 1 && m <= 64 && t.cl_blk[c + 1] - t.cl_blk[c] == m * m, AIM_ERR_INVALID_ARG,
                "plan file: bad cluster block");
  }
  AIM_REQUIRE(int64_t(t.cl_inv.size()) == t.cl_blk[ncl], AIM_ERR_INVALID_ARG,
              "plan file: bad cluster inverses");
  check_finite(t.cl_inv, "cluster inverses");
  // static self terms (the diagonal preconditioner divides by them)
  for (int64_t i = 0; i < N; ++i) {
    double dv = 0.0;
    for (int64_t q = t.rowptr[i]; q < t.rowptr[i + 1]; ++q)
      if (t.col[q] == i) dv = t.near_static[q];
    AIM_REQUIRE(dv != 0.0, AIM_ERR_INVALID_ARG, "plan file: zero static self term");
  }
}

// reads and validates a plan file into a fresh host-side plan
std::unique_ptr<aim_plan_s> read_plan(const char* path) {
  std::ifstream f(path, std::ios::binary);
  AIM_REQUIRE(bool(f), AIM_ERR_INVALID_ARG, std::string("cannot open ") + path);
  std::string buf((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
  AIM_REQUIRE(buf.size() >= sizeof(kPlanMagic) + 4 + 8, AIM_ERR_INVALID_ARG,
              "plan file truncated");
  uint64_t stored = 0;
  std::memcpy(&stored, buf.data() + buf.size() - 8, 8);
  AIM_REQUIRE(stored == fnv1a(buf.data(), buf.size() - 8), AIM_ERR_INVALID_ARG,
              "plan file checksum mismatch");
  AIM_REQUIRE(std::memcmp(buf.data(), kPlanMagic, sizeof(kPlanMagic)) == 0, AIM_ERR_INVALID_ARG,
              "not a plan file");
  Reader r{buf, sizeof(kPlanMagic), buf.size() - 8};
  uint32_t version = 0;
  r.pod(version);
  AIM_REQUIRE(version == kPlanVersion, AIM_ERR_INVALID_ARG, "unsupported plan file version");
  std::unique_ptr<aim_plan_s> p(new aim_plan_s());
  aim::HostTables& t = p->t;
  r.pod(t.N);
  r.pod(t.order);
  for (int a = 0; a < 3; ++a) r.pod(t.dims[a]);
  r.pod(t.h);
  for (int a = 0; a < 3; ++a) r.pod(t.origin[a]);
  r.pod(t.setup_seconds);
  int32_t nfreq = 0, max_rhs = 0;
  uint32_t prec = 0;
  r.pod(nfreq);
  r.pod(prec);
  r.pod(max_rhs);
  for (int pi = 0; pi < 2; ++pi)
    for (int k = 0; k < aim::kSchedLen; ++k) r.pod(p->sched[pi][k]);
  r.vec(p->k);
  table_vectors(t, [&](auto& v) { r.vec(v); });
  AIM_REQUIRE(r.pos == r.end, AIM_ERR_INVALID_ARG, "plan file has trailing data");
  AIM_REQUIRE(nfreq >= 1 && int64_t(p->k.size()) == nfreq, AIM_ERR_INVALID_ARG,
              "plan file: bad wavenumbers");
  for (const double k : p->k)
    AIM_REQUIRE(std::isfinite(k) && k > 0.0, AIM_ERR_INVALID_ARG, "plan file: bad wavenumber");
  AIM_REQUIRE(prec != 0 && (prec & ~3u) == 0, AIM_ERR_INVALID_ARG, "plan file: bad precisions");
  AIM_REQUIRE(max_rhs >= 1 && max_rhs <= 65535, AIM_ERR_INVALID_ARG, "plan file: bad max_rhs");
  validate_tables(t);
  p->nfreq = nfreq;
  p->prec = prec;
  p->max_rhs = max_rhs;
  for (int a = 0; a < 3; ++a) {
    p->g.N[a] = t.dims[a];
    p->g.M[a] = 2 * t.dims[a];
  }
  p->g.Ng = int64_t(t.dims[0]) * t.dims[1] * t.dims[2];
  p->g.Nfold = int64_t(t.dims[0] + 1) * (t.dims[1] + 1) * (t.dims[2] + 1);
  for (int pi = 0; pi < 2; ++pi) {
    for (int k = 0; k < 5; ++k)
      AIM_REQUIRE(p->sched[pi][k] >= 0 && p->sched[pi][k] < aim::kFftVariants &&
                      aim::fft_variant_ok(pi == 0, p->g, k, p->sched[pi][k]),
                  AIM_ERR_INVALID_ARG, "plan file: bad schedule");
    AIM_REQUIRE(p->sched[pi][5] >= 0 && p->sched[pi][5] < aim::kLayouts &&
                    p->sched[pi][6] >= 0 && p->sched[pi][6] <= 3,
                AIM_ERR_INVALID_ARG, "plan file: bad schedule");
  }
  p->ncl = int(t.cl_ptr.size()) - 1;
  for (int c = 0; c < p->ncl; ++c) p->maxcl = std::max(p->maxcl, t.cl_ptr[c + 1] - t.cl_ptr[c]);
  return p;
}

}  // namespace

extern "C" aim_status aim_plan_save(aim_plan p, const char* path) {
  if (!p || !path) return fail(AIM_ERR_INVALID_ARG, "null argument");
  return guarded([&] {
    no_batch(p);
    Writer w;
    w.b.append(kPlanMagic, sizeof(kPlanMagic));
    w.pod(kPlanVersion);
    aim::HostTables& t = p->t;
    w.pod(t.N);
    w.pod(t.order);
    for (int a = 0; a < 3; ++a) w.pod(t.dims[a]);
    w.pod(t.h);
    for (int a = 0; a < 3; ++a) w.pod(t.origin[a]);
    w.pod(t.setup_seconds);
    w.pod(int32_t(p->nfreq));
    w.pod(uint32_t(p->prec));
    w.pod(int32_t(p->max_rhs));
    for (int pi = 0; pi < 2; ++pi)
      for (int k = 0; k < aim::kSchedLen; ++k) w.pod(int32_t(p->sched[pi][k]));
    w.vec(p->k);
    table_vectors(t, [&](auto& v) { w.vec(v); });
    w.pod(fnv1a(w.b.data(), w.b.size()));
    std::ofstream f(path, std::ios::binary | std::ios::trunc);
    AIM_REQUIRE(bool(f), AIM_ERR_INVALID_ARG, std::string("cannot write ") + path);
    f.write(w.b.data(), std::streamsize(w.b.size()));
    AIM_REQUIRE(bool(f), AIM_ERR_INVALID_ARG, std::string("write failed: ") + path);
  });
}

extern "C" aim_status aim_plan_load_host(const char* path, aim_plan* out) {
  if (!path || !out) return fail(AIM_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  std::unique_ptr<aim_plan_s> p;
  const aim_status st = guarded([&] {
    p = read_plan(path);
    p->host_only = true;
  });
  if (st != AIM_OK) return st;
  *out = p.release();
  return AIM_OK;
}

extern "C" aim_status aim_plan_load(const char* path, aim_alloc_fn alloc, aim_free_fn free_fn,
                                    void* alloc_ctx, void* hip_stream, aim_plan* out) {
  if (!path || !out) return fail(AIM_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if ((alloc == nullptr) != (free_fn == nullptr))
    return fail(AIM_ERR_INVALID_ARG, "alloc and free must be given together");
  std::unique_ptr<aim_plan_s> p;
  const aim_status st = guarded([&] {
    p = read_plan(path);  // everything validated before any device call
    p->alloc = alloc;
    p->free_fn = free_fn;
    p->actx = alloc_ctx;
    init_device(p.get(), static_cast<hipStream_t>(hip_stream));
  });
  if (st != AIM_OK) return st;
  *out = p.release();
  return AIM_OK;
}
