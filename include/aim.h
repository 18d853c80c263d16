/*
 * aim.h -- C ABI of the MI355X AIMx library.
 *
 * The library applies and solves the extended adaptive-integral-method
 * (AIMx) operator of Sharma & Triverio, "AIMx: An Extended Adaptive Integral
 * Method for the Fast Electromagnetic Modeling of Complex Structures"
 * (arXiv 2009.02281), for the scalar single-layer Helmholtz operator with one
 * piecewise-constant basis function per flat triangle and Galerkin testing:
 *
 *     A(k) x ~= (A_s,NR - A_s,P) x + W H(k) P x            (eq. LAIMx)
 *
 * with P the projection of quadrature-point sources onto (n+1)^3 grid
 * stencils, H(k) the Toeplitz matrix of G = e^{-jkr}/(4 pi r) over grid
 * points with self term -jk/(4 pi) (eqs. Hmn, Hmm), W = P^T, A_s,NR the
 * static (1/(4 pi r)) near-region matrix by direct integration and A_s,P its
 * precorrection (eq. aimLPs, with H_s self term 0 per eq. Hsmm).
 *
 * Conventions common to every call:
 *  - Every function returns aim_status; no C++ exception crosses the ABI.
 *    On failure aim_last_error() returns a message (thread-local) and output
 *    buffers are unspecified.
 *  - "_dev" pointers are device (HBM) addresses owned by the caller; "_host"
 *    pointers are host memory owned by the caller.  The library never frees
 *    caller memory.
 *  - Complex vectors are interleaved (re, im): complex128 = two doubles for
 *    AIM_C128, complex64 = two floats for AIM_C64, laid out [nrhs][N] with N
 *    the number of triangles (basis functions).
 *  - Grids are x-fastest: node (ix, iy, iz) has flat index ix + Nx (iy + Ny iz).
 *  - A plan is not thread-safe; calls on one plan must be serialised.
 *  - hip_stream is a hipStream_t (NULL = the default stream).
 *  - Lengths and wavenumbers share one unit (k = 2 pi / lambda).
 */
#ifndef AIM_H
#define AIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AIM_OK = 0,
  AIM_ERR_INVALID_ARG = 1,   /* null pointer, size or enum out of range          */
  AIM_ERR_GEOMETRY = 2,      /* non-finite vertex, bad index, zero-area triangle */
  AIM_ERR_GRID = 3,          /* unsupported grid size, stencil leaves the grid   */
  AIM_ERR_OOM = 4,           /* device or host allocation failed                 */
  AIM_ERR_DEVICE = 5,        /* a HIP runtime call failed                        */
  AIM_ERR_NOT_CONVERGED = 6, /* solver hit its iteration cap; best iterate kept  */
  AIM_ERR_BREAKDOWN = 7,     /* solver met a non-finite value or a breakdown      */
  AIM_ERR_STATE = 8          /* call not valid for this plan (e.g. precision
                                not built, no preconditioner data)              */
} aim_status;

typedef enum { AIM_C128 = 0, AIM_C64 = 1 } aim_precision;

typedef enum {
  AIM_PC_NONE = 0,       /* unpreconditioned                                      */
  AIM_PC_DIAG = 1,       /* 1 / diag(A_s,NR): the frequency-independent diagonal
                            preconditioner of Sec. III-A ("Preconditioning")     */
  AIM_PC_NEARBLOCK = 2,  /* block-Jacobi on spatial clusters (recursive
                            coordinate bisection to at most 64 triangles) of the
                            full-kernel Galerkin matrix at each right-hand
                            side's wavenumber: the static near entries A_s,NR
                            with the dynamic part added (3 x 3 point rule), as
                            the same section suggests for near-region/block
                            preconditioners (built and inverted on the device
                            once per wavenumber used)                            */
  AIM_PC_UNET = 3,       /* learned grid preconditioner attached with
                            aim_plan_set_unet, applied inside flexible GMRES
                            (right preconditioning with stored Z), gated, with
                            aim_solve_opts.fallback_pc as its fallback             */
  AIM_PC_NEARBLOCK_STATIC = 4 /* the same clusters with the static entries
                            A_s,NR only (frequency independent; the form that
                            section expects to be less effective: over clusters
                            a sizeable fraction of a wavelength wide it can
                            stall GMRES)                                         */
} aim_pc_kind;

typedef enum {
  AIM_STAGE_PROJECT = 0,     /* x[nrhs][N]            -> q[nrhs][Ng]  (q = P x)        */
  AIM_STAGE_CONVOLVE = 1,    /* q[nrhs][Ng]           -> phi[nrhs][Ng] (phi = H(k) q)  */
  AIM_STAGE_INTERPOLATE = 2, /* phi[nrhs][Ng]         -> y[nrhs][N]   (y = P^T phi)    */
  AIM_STAGE_NEAR = 3,        /* x[nrhs][N]            -> y[nrhs][N]   (y = C x)        */
  AIM_STAGE_LEARNED_PC = 4,  /* x[nrhs][N] complex128 -> y[nrhs][N] complex128,
                                y = M(x) of the attached network (aim_plan_set_unet);
                                prec must be AIM_C128                             */
  AIM_STAGE_NEARBLOCK_PC = 5 /* x[nrhs][N] complex128 -> y[nrhs][N] complex128,
                                y = B_k^{-1} x of AIM_PC_NEARBLOCK at each vector's
                                wavenumber; prec must be AIM_C128                 */
} aim_stage;

typedef enum { AIM_RHS_PLANE_WAVE = 0, AIM_RHS_GAUSSIAN_PATCH = 1 } aim_rhs_kind;

typedef struct aim_plan_s* aim_plan;
typedef struct aim_graph_s* aim_graph;
typedef struct aim_unet_s* aim_unet;

/* Optional device allocator (e.g. a framework's caching allocator).  When
 * alloc is NULL the library uses hipMalloc / hipFree. */
typedef void* (*aim_alloc_fn)(size_t bytes, void* hip_stream, void* ctx);
typedef void (*aim_free_fn)(void* ptr, void* hip_stream, void* ctx);

/* Problem description (Sec. II: a triangulated surface, a regular grid over
 * its bounding box, stencils of n+1 points per direction, a near-region
 * threshold and the frequencies of the sweep).  All arrays are host memory
 * and are copied during aim_setup; the caller may free them afterwards. */
typedef struct {
  int64_t n_vertices;
  int64_t n_triangles;
  const double* vertices;    /* [n_vertices][3]                                  */
  const int32_t* triangles;  /* [n_triangles][3], 0-based vertex indices         */
  int32_t stencil_order;     /* n = 2 (27 nodes/point) or 3 (64 nodes/point)     */
  int32_t grid_dims[3];      /* unpadded Nx, Ny, Nz: powers of two in [8, 256];
                                padded internally to 2N per axis                  */
  double h;                  /* grid spacing; <= 0: max_a extent_a/(N_a - 5)     */
  double near_threshold;     /* pairs with centroid distance < this are near     */
  int32_t n_freq;            /* number of wavenumbers (>= 1)                      */
  const double* k;           /* [n_freq] wavenumbers (> 0)                        */
  uint32_t precisions;       /* bitmask of (1u << AIM_C128) | (1u << AIM_C64)     */
  int32_t max_rhs;           /* largest nrhs later passed to matvec/solve (>= 1)  */
  int32_t n_threads;         /* host threads for setup; <= 0: all cores           */
  aim_alloc_fn alloc;        /* optional; NULL = hipMalloc                        */
  aim_free_fn free;
  void* alloc_ctx;
} aim_setup_desc;

/* Facts about a built plan (host struct filled by aim_plan_query). */
typedef struct {
  int64_t n;                 /* basis functions (triangles)                      */
  int64_t n_grid;            /* Nx Ny Nz                                          */
  int64_t nnz;               /* non-zeros of C = A_s,NR - A_s,P                  */
  int32_t dims[3];
  int32_t order;
  int32_t n_freq;
  int32_t max_rhs;
  uint32_t precisions;
  double h;
  double origin[3];          /* position of node (0, 0, 0)                       */
  double setup_seconds;      /* host + device time of aim_setup                  */
  double spectra_seconds;    /* part of it spent building kernel spectra          */
  int64_t device_bytes;      /* device memory held by the plan                    */
  int32_t n_clusters;        /* near-block preconditioner clusters                */
  int32_t max_cluster;       /* largest cluster                                    */
  double near_seconds;       /* part of set-up spent on A_s,NR and C               */
  int32_t near_on_device;    /* 1: A_s,NR and C were computed on the device        */
  int32_t reserved;
} aim_plan_info;

/* Solver options (aim_solve).  rtol is the relative residual
 * ||b - A x|| / ||b|| at which a right-hand side counts as converged (the
 * paper's runs use GMRES to 1e-4, Sec. V).  inner = AIM_C64 runs the Krylov
 * matvecs in complex64 inside an iterative-refinement loop whose residual
 * and update are complex128; inner = AIM_C128 runs restarted GMRES directly.
 * Arnoldi orthogonalisation is always complex128 on the device. */
typedef struct {
  double rtol;               /* target relative residual (> 0)                    */
  /* (the solver launches the matvec kernels directly and reads its GMRES
     state back every 4 steps; AIM_SOLVER_GRAPHS=1 in the environment makes
     it replay captured matvec graphs instead) */
  int32_t restart;           /* Krylov subspace size m (1..200)                   */
  int32_t max_iter;          /* cap on inner iterations per right-hand side       */
  int32_t max_refine;        /* cap on refinement steps (inner = AIM_C64)          */
  aim_precision inner;       /* precision of the Krylov matvecs                    */
  aim_pc_kind pc;            /* right preconditioner                               */
  double inner_rtol;         /* inner tolerance per refinement step (0: adaptive,
                                0.3 rtol / current residual, kept within
                                [3e-6, 0.1]).  An inner solve also ends early
                                at complex64's accuracy floor: after two
                                restarts in a row at which either every system
                                had stopped its cycle on its residual estimate
                                yet its true residual is above the inner
                                tolerance, or every unconverged true relative
                                residual is below 1e-4 and fell by less than a
                                tenth over the cycle                              */
  aim_pc_kind fallback_pc;   /* pc = AIM_PC_UNET only: preconditioner the solve
                                continues with when the learned one is gated out
                                (AIM_PC_NONE or AIM_PC_NEARBLOCK; 0 = none)        */
  double gate;               /* pc = AIM_PC_UNET only: a restart cycle must cut
                                every unconverged residual to below gate times
                                its previous value (0: 0.7)                        */
} aim_solve_opts;

/* Per-right-hand-side outcome (host array of nrhs entries). */
typedef struct {
  int32_t iters;             /* inner Krylov iterations                           */
  int32_t refinements;       /* outer refinement steps                             */
  int32_t matvecs;           /* operator applications                              */
  int32_t fallback_used;     /* 1 if the learned preconditioner was switched off  */
  int32_t converged;
  double rel_resid;          /* final true relative residual (complex128)         */
  double seconds;            /* wall time of the whole batched solve               */
} aim_solve_info;

/* Build a plan: validates the mesh and grid on the host (before any device
 * call), computes quadrature points (3-point rule), stencils and the near
 * list on the host, then the static near-field matrix by closed-form
 * integration of 1/R (Sec. III-A, change (a) of the AIMx recipe) and its
 * precorrection on the device (one thread per near pair; the one-time
 * static fill of Sec. VI), uploads the tables and computes one kernel
 * spectrum per wavenumber on the device.
 * Errors: AIM_ERR_INVALID_ARG, AIM_ERR_GEOMETRY, AIM_ERR_GRID, AIM_ERR_OOM,
 * AIM_ERR_DEVICE.  A singular near-field preconditioner block (degenerate
 * geometry) is reported as AIM_ERR_GEOMETRY after the device fill.
 * Blocking. */
aim_status aim_setup(const aim_setup_desc* desc, void* hip_stream, aim_plan* out);

/* Host-only variant of aim_setup: builds and validates every
 * frequency-independent host table (quadrature points, stencils, near list,
 * A_s,NR and C = A_s,NR - A_s,P, preconditioner blocks) without touching
 * the device.  The plan answers aim_plan_query and aim_export_tables; every
 * device call on it returns AIM_ERR_STATE.  Blocking; runs without a GPU. */
aim_status aim_setup_host(const aim_setup_desc* desc, aim_plan* out);

/* A batch of geometries of uneven size (one batched solve over many
 * instances): n descriptions, each set up as by aim_setup (own grid,
 * frequencies, tables, spectra; max_rhs of each is ignored), behind one
 * handle.  System i belongs to instance i; its vectors are rows of length
 * N_max = max N_i, of which the first N_i entries are used and the rest must
 * be zero on input (b, x0) and are zero on output.  On a batch plan,
 * aim_matvec and aim_solve take nrhs = n (freq_idx_host[i] indexes
 * instance i's wavenumbers; all instances have at least the batch's n_freq),
 * with the diagonal and near-block preconditioners applied per instance;
 * stages, excitations, schedules, profiles, checkpoints and the learned
 * preconditioner are per instance and return AIM_ERR_STATE.  The instances
 * run one after another on the stream (one launch sequence each), not in one
 * fused launch.  All descriptions must share one allocator.  Blocking. */
aim_status aim_setup_batch(const aim_setup_desc* descs, int32_t n, void* hip_stream,
                           aim_plan* out);

/* Number of instances (1 for an ordinary plan) and, if n_host != NULL, each
 * instance's number of triangles N_i (n_host has room for the count). */
aim_status aim_batch_sizes(aim_plan plan, int32_t* count, int64_t* n_host);

/* Release every device and host resource of the plan (NULL is a no-op). */
aim_status aim_destroy(aim_plan plan);

/* Checkpoint of a plan: the frequency-independent host tables (the static
 * near-field matrix A_s,NR and C = A_s,NR - A_s,P of Sec. III-A, which the
 * paper suggests computing once and storing; P in both layouts; the
 * near-block preconditioner), the wavenumbers, precisions, max_rhs and the
 * tuned schedules, in one binary file with a checksum.  Works on host-only
 * plans too.  Blocking. */
aim_status aim_plan_save(aim_plan plan, const char* path);

/* Rebuild a plan from aim_plan_save output without the host set-up: the file
 * is read and validated completely (checksum, sizes, every index range, the
 * row-block and cluster structure, finiteness) before any device call, then
 * the tables are uploaded and the spectra computed as in aim_setup.  The
 * allocator arguments have aim_setup_desc's meaning.  AIM_ERR_INVALID_ARG for
 * an unreadable, corrupt or inconsistent file.  Blocking. */
aim_status aim_plan_load(const char* path, aim_alloc_fn alloc, aim_free_fn free_fn,
                         void* alloc_ctx, void* hip_stream, aim_plan* out);

/* Host-only counterpart of aim_plan_load (like aim_setup_host): answers
 * aim_plan_query and aim_export_tables; every device call on it returns
 * AIM_ERR_STATE.  Runs without a GPU. */
aim_status aim_plan_load_host(const char* path, aim_plan* out);

aim_status aim_plan_query(aim_plan plan, aim_plan_info* info_host);

/* y = A(k_f) x for nrhs right-hand sides (eq. LAIMx): projection, zero-padded
 * 3D FFT, multiplication by the kernel spectrum of wavenumber k_f, inverse
 * FFT, interpolation, plus the sparse correction C x.  x_dev and y_dev are
 * [nrhs][N] complex of the given precision and must not overlap.
 * freq_idx_host[r] selects the wavenumber of right-hand side r (NULL: all 0).
 * Asynchronous on hip_stream.  Errors: AIM_ERR_INVALID_ARG (nrhs outside
 * 1..max_rhs, bad frequency index), AIM_ERR_STATE (precision not built). */
aim_status aim_matvec(aim_plan plan, aim_precision prec, const void* x_dev, void* y_dev,
                      int32_t nrhs, const int32_t* freq_idx_host, void* hip_stream);

/* aim_matvec for callers that cannot allocate device memory during the call
 * or at all after set-up (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same operator, arguments, kernels and
 * results as aim_matvec; the projection grid and the convolution workspace
 * live in a fixed device array of the library (AIM_STATIC_SCRATCH_BYTES =
 * 64 MiB, held on each device that uses it until the process ends) instead
 * of the plan's workspace.  The call allocates nothing; the first call on a
 * device looks up that device's copy of the array.  Nothing in the array
 * needs clearing (every element is written before it is read).  All calls on
 * one device share the array: calls that overlap in time on one device (two
 * streams, two threads, two plans) race and give undefined results.  Not for
 * batch plans (AIM_ERR_STATE).  Errors as aim_matvec, plus
 * AIM_ERR_INVALID_ARG when nrhs vectors need more than the array holds:
 * 16 (complex128) or 8 (complex64) bytes per vector times (Ng + the
 * workspace, about 6 Ng), e.g. at most 2 complex128 vectors on a 64^3 grid. */
#define AIM_STATIC_SCRATCH_BYTES (64u << 20)
aim_status aim_matvec_static(aim_plan plan, aim_precision prec, const void* x_dev, void* y_dev,
                             int32_t nrhs, const int32_t* freq_idx_host, void* hip_stream);

/* The linear-term modification of Sec. III-A ("Modification for Increased
 * Accuracy", eqs. linterm and Lmatdecomplin): with on != 0, every matvec and
 * solve of the plan adds k^2 D x, where D is the real diagonal
 * A_lin[i, i] - (W H_lin P)[i, i] of G_lin = -R/(8 pi): the linear Taylor term
 * of the dynamic kernel integrated directly where a basis function overlaps
 * itself (3-point outer rule, closed-form inner integral), minus what the
 * grid already gives for it.  D is computed by aim_setup's device near fill
 * (AIM_ERR_STATE on plans without it: host-only or loaded from a file).
 * Off by default.  aim_export_lin_diag copies D ([N] doubles) to the host. */
aim_status aim_set_lin_term(aim_plan plan, int32_t on);
aim_status aim_export_lin_diag(aim_plan plan, double* d_host);

/* The near-block preconditioner's clusters: cl_ptr_host[n_clusters + 1]
 * offsets into cl_perm_host[N], the triangles of cluster c being
 * cl_perm_host[cl_ptr_host[c] .. cl_ptr_host[c+1]) (n_clusters from
 * aim_plan_query).  Host-only plans too. */
aim_status aim_export_clusters(aim_plan plan, int32_t* cl_ptr_host, int32_t* cl_perm_host);

/* Conventional AIM on the same plan (Sec. II-B, eqs. aimL, aimLFR, aimLP),
 * the method AIMx is measured against: per wavenumber the complex near
 * correction C(k) = A_NR(k) - A_P(k) is rebuilt, where A_NR(k) holds the
 * near-region Galerkin entries of e^{-jkR}/(4 pi R) (the plan's static
 * entries plus the smooth remainder (e^{-jkR} - 1)/(4 pi R) by the 3 x 3
 * point rule) and A_P(k) = W H_NR(k) P uses the grid kernel of H(k) with its
 * self term -jk/(4 pi), so that it cancels.  The far operator W H(k) P is
 * the AIMx one.
 * aim_conventional_fill computes C(k_f) on the device for wavenumber
 * freq_idx (one thread per near pair; asynchronous on hip_stream; the plan
 * keeps one wavenumber at a time, in complex128 and, if built, complex64).
 * aim_matvec_conventional: y = W H(k_f) P x + C(k_f) x for nrhs vectors, all
 * at that wavenumber (same layouts and rules as aim_matvec; AIM_ERR_STATE
 * before any fill).  aim_conventional_export copies C(k_f) to the host as
 * [nnz][2] doubles in the order of the near list (aim_export_tables);
 * blocking.  Not for batch plans. */
aim_status aim_conventional_fill(aim_plan plan, int32_t freq_idx, void* hip_stream);
aim_status aim_matvec_conventional(aim_plan plan, aim_precision prec, const void* x_dev,
                                   void* y_dev, int32_t nrhs, void* hip_stream);
aim_status aim_conventional_export(aim_plan plan, double* vals_host, void* hip_stream);

/* The double-layer potential operator under AIMx (Sec. III-B, eqs. opK,
 * ghgf, KAIMx, gH00), in the scalar setting of the plan: one
 * piecewise-constant density per flat triangle, Galerkin testing, kernel
 * dG/dn' = n_j.(r - r') (1 + jkR) e^{-jkR} / (4 pi R^3) (n_j the unit normal
 * (b - a) x (c - a) of the source triangle), so
 *   y_i = sum_j x_j int_{T_i} int_{T_j} dG/dn'(r, r') dS' dS
 * with the self pairs in the principal-value sense (0 for flat triangles;
 * the jump term +-x/2 of a closed surface is the caller's).  Evaluated as
 * K_s,NR - K_s,P + W H_grad(k) P^(K): the static near entries (inner
 * integral in closed form through the solid angle, 3-point outer rule) and
 * their precorrection on the plan's near list, and three gradient channels
 * n_a x through the plan's projection, the grid samples of dG/dr'_a (self
 * term 0 per component: eq. gH00 gives a scalar for this vector kernel, and
 * 0 is the symmetric value) and interpolation.  x_dev, y_dev: [nrhs][N]
 * complex128 device buffers (caller-owned, not overlapping), freq_idx_host
 * [nrhs] indices into the plan's wavenumbers (NULL: all 0).  The first call
 * builds the operator's tables on the device (normals, the near values, one
 * spectrum per wavenumber, buffers for max_rhs products: about 4 max_rhs
 * times the matvec's workspace); needs the complex128 tables and the mesh
 * (AIM_ERR_STATE on loaded or host-only plans).  Asynchronous after that
 * first call.  Not on batch plans. */
aim_status aim_matvec_dlp(aim_plan plan, const void* x_dev, void* y_dev, int32_t nrhs,
                          const int32_t* freq_idx_host, void* hip_stream);
/* The double-layer near values on the near list (aim_export_tables order):
 * K_s,NR into near_host[nnz] and C_K = K_s,NR - K_s,P into corr_host[nnz]
 * (either may be NULL).  Builds the tables if needed.  Blocking. */
aim_status aim_dlp_export(aim_plan plan, double* near_host, double* corr_host,
                          void* hip_stream);

/* The electric-field integral operator on RWG functions under AIMx (Sec.
 * II-A, eq. EFIEdis; Sec. II-B, eqs. aimLFR and LAIMx; the static split of
 * Sec. III-A), the factor -j omega mu left out:
 *   Z_mn = int int f_m(r).f_n(r') G dS' dS
 *          - k^-2 int int (div f_m)(r) (div' f_n)(r') G dS' dS,
 * evaluated as C_A - k^-2 C_phi + sum_{c=x,y,z} P_c^T H(k) P_c
 * - k^-2 P_q^T H(k) P_q: three Cartesian current channels and one charge
 * channel through the plan's grid, stencils and spectrum H(k) (self term
 * -jk/(4 pi)), and the real static corrections C_A = A_s,NR - A_s,P and
 * C_phi likewise (kernel 1/(4 pi R), inner integrals int 1/R and int r'/R in
 * closed form, 3-point outer rule, symmetrised; precorrection through H_s
 * with self term 0).  One function per edge shared by two triangles T+, T-
 * (T+ the lower triangle index), numbered in ascending order of the edge's
 * (smaller, larger) vertex index pair: f = l/(2A+) (r - p+) on T+ and
 * l/(2A-) (p- - r) on T-, p+- the vertices opposite the edge; edges of one
 * triangle carry none (open surfaces), an edge of three or more triangles is
 * AIM_ERR_GEOMETRY.  Two functions are near when a triangle of one is in the
 * near list of a triangle of the other.
 * aim_efie_setup builds the tables (functions, near list and point
 * projection on the host threads of the plan's descriptor, the near pairs'
 * integrals on the device; blocking) and returns the number of functions,
 * the near-list length and the build time (each pointer may be NULL); the
 * other two calls build them on first use.  Needs the complex128 tables and
 * the mesh (AIM_ERR_STATE on loaded, host-only or batch plans); the device
 * buffers hold 4 max_rhs point-source vectors, grids and convolution
 * workspaces.
 * aim_matvec_efie: y = Z(k_f) x, x_dev and y_dev [nrhs][n_rwg] device
 * buffers of the precision prec (caller-owned, not overlapping), freq_idx_host
 * [nrhs] indices into the plan's wavenumbers (NULL: all 0); asynchronous on
 * hip_stream.  AIM_C64 (the plan needs complex64 tables) runs the sources,
 * projection, FFTs, interpolation and near rows in complex64 with the
 * tables rounded from the complex128 ones.
 * aim_efie_export copies to the host, each pointer optional: tri_rwg [N][3]
 * (function on the edge opposite vertex e of triangle t, -1 none), the near
 * list rowptr [n_rwg + 1] and col [nnz], and C_A, C_phi [nnz]; blocking. */
aim_status aim_efie_setup(aim_plan plan, int64_t* n_rwg, int64_t* nnz, double* seconds,
                          void* hip_stream);
aim_status aim_matvec_efie(aim_plan plan, aim_precision prec, const void* x_dev, void* y_dev,
                           int32_t nrhs, const int32_t* freq_idx_host, void* hip_stream);
aim_status aim_efie_export(aim_plan plan, int32_t* tri_rwg, int32_t* rowptr, int32_t* col,
                           double* ca, double* cphi, void* hip_stream);

/* The double-layer operator on RWG functions under AIMx (Sec. III-B, eqs.
 * opK, ghgf, KAIMx, gH00; the K block of the discrete CFIE, eq. CFIEdis),
 * with Galerkin RWG testing:
 *   K_mn = int f_m(r) . [ n(r) x int grad G(r, r') x f_n(r') dS' ] dS,
 *   grad G = -(r - r') (1 + jkR) e^{-jkR} / (4 pi R^3),
 * n the unit normal (b - a) x (c - a) of the testing triangle, in the
 * principal-value sense (a flat triangle's own contribution at its points
 * is normal to it and drops out); the residue of the surface limit is a
 * multiple of the Gram matrix G_mn = int f_m . f_n, so the call applies
 *   y = (K(k_f) + gram_coef G) x
 * (the MFIE J/2 - n x K_PV J = n x H_inc of a closed surface, tested with
 * f_m, is (G/2 - K) J = <f_m, n x H_inc>: gram_coef = -1/2 with the sign of
 * y flipped).  Evaluated as
 * K_s,NR - K_s,P + W H_grad(k) P on the RWG functions, near list, point
 * projection and wavenumbers of the EFIE above: three current channels
 * w_q f(r_q) projected and transformed forward, their spectral cross
 * product with the three components of grad G sampled on the grid (self
 * term 0 per component: eq. gH00 gives a scalar for this vector kernel) in
 * one z pass, the field transformed back and interpolated, tested with
 * w_q f_m(r_q) x n; static entries from the
 * closed form of int (r - r')/R^3 over a triangle and the 3-point outer
 * rule, precorrection with the grid's static gradient samples.  x_dev,
 * y_dev [nrhs][n_rwg] of precision prec (caller-owned, not overlapping);
 * prec and freq_idx_host as for aim_matvec_efie.  The first call builds the EFIE's
 * tables if needed, then its own (blocking); asynchronous after that.
 * aim_mfie_export copies C_K = K_s,NR - K_s,P and G on the RWG near list
 * (order of aim_efie_export) to the host, and the build time; each pointer
 * optional; blocking.  Same plan requirements as the EFIE. */
aim_status aim_matvec_mfie(aim_plan plan, aim_precision prec, const void* x_dev, void* y_dev,
                           int32_t nrhs, const int32_t* freq_idx_host, double gram_coef,
                           void* hip_stream);
aim_status aim_mfie_export(aim_plan plan, double* ck_host, double* gram_host, double* seconds,
                           void* hip_stream);

/* The AIMx-accelerated combined-field operator of eq. CFIEAIMx (Sec. III-B;
 * the discrete CFIE, eq. CFIEdis), scaled by 1/(j k eta0):
 *   y = Z(k_f) x + (j / k_f) (K(k_f) + gram_coef G) x,
 * Z the EFIE operator of aim_matvec_efie and K, G those of aim_matvec_mfie.
 * With E_s = -j k eta0 Z J (the EFIE, tested: j k Z J = <f_m, E_inc>/eta0)
 * and the MFIE above, gram_coef = -1/2 gives their sum divided by j k:
 *   [Z + (j/k)(K - G/2)] J = (<f_m, E_inc> + eta0 <f_m, n x H_inc>) / (j k eta0)
 * (the paper writes the same combination as L - (j/k0) K with its own sign
 * convention for L and the incident-field vectors).  One projection of the four channels
 * serves both operators: the double layer takes its three current grids
 * from it.  Arguments and rules as for aim_matvec_mfie; the first call
 * builds both operators' tables and a [3 max_rhs][3N] field buffer. */
aim_status aim_matvec_cfie(aim_plan plan, aim_precision prec, const void* x_dev, void* y_dev,
                           int32_t nrhs, const int32_t* freq_idx_host, double gram_coef,
                           void* hip_stream);

/* Plane waves tested with the RWG functions (3-point rule per triangle):
 * params_host [nrhs][6] = (d, pol) with d the propagation direction
 * (normalised here) and pol the electric polarisation; vector r at
 * wavenumber k = k[freq_idx_host[r]] (NULL: all 0):
 *   field 0: b[r][m] = <f_m, pol e^{-j k d.r}>            (the EFIE's E),
 *   field 1: b[r][m] = <f_m, n x (d x pol) e^{-j k d.r}>   (eta0 <f_m, n x H_inc>,
 *            the MFIE's right-hand side, n each triangle's unit normal).
 * b_dev [nrhs][n_rwg] complex128.  Builds the EFIE tables if needed;
 * blocking.  Same plan requirements as the EFIE. */
aim_status aim_rwg_excitation(aim_plan plan, int32_t field, const double* params_host,
                              int32_t nrhs, const int32_t* freq_idx_host, void* b_dev,
                              void* hip_stream);

/* Batched restarted GMRES (the Krylov loop of aim_solve: complex128,
 * device Arnoldi, per-system stop) on an RWG operator: op 1 the EFIE Z,
 * 2 the double layer K + gram_coef G, 3 the combined field
 * Z + (j/k)(K + gram_coef G); vector r at wavenumber index freq_idx_host[r].
 * b_dev, x_dev [nrhs][n_rwg] complex128, x_dev the initial guess on entry;
 * opts as for aim_solve with pc AIM_PC_NONE and inner AIM_C128 only
 * (AIM_ERR_INVALID_ARG otherwise); info[nrhs] filled.  AIM_ERR_NOT_CONVERGED
 * if a system stops at max_iter (x holds its best iterate).  Blocking. */
aim_status aim_solve_rwg(aim_plan plan, int32_t op, double gram_coef, const void* b_dev,
                         void* x_dev, int32_t nrhs, const int32_t* freq_idx_host,
                         const aim_solve_opts* opts, aim_solve_info* info, void* hip_stream);

/* One stage of the matvec, for stage-level checks (see aim_stage for the
 * shapes).  Same rules as aim_matvec; grids are unpadded [nrhs][Nz][Ny][Nx]. */
aim_status aim_apply_stage(aim_plan plan, aim_precision prec, aim_stage stage,
                           const void* in_dev, void* out_dev, int32_t nrhs,
                           const int32_t* freq_idx_host, void* hip_stream);

/* Galerkin-tested incident field, complex128 [nrhs][N] on the device:
 * b_i = sum_p (A_i/3) u_inc(r_ip).  AIM_RHS_PLANE_WAVE: u = exp(-j k d.r) with
 * params = {dx, dy, dz} (unit direction); AIM_RHS_GAUSSIAN_PATCH:
 * u = exp(-|r - c|^2 / (2 sigma^2)) with params = {cx, cy, cz, sigma}.
 * Right-hand side r uses params + r * n_params and wavenumber
 * k[freq_idx_host[r]].  Asynchronous. */
aim_status aim_excitation(aim_plan plan, aim_rhs_kind kind, const double* params_host,
                          int32_t n_params, int32_t nrhs, const int32_t* freq_idx_host,
                          void* b_dev, void* hip_stream);

/* Solve A(k_f) x = b for nrhs right-hand sides at once (batched restarted
 * GMRES / flexible GMRES with right preconditioning, complex128 Arnoldi; with
 * inner = AIM_C64 wrapped in complex128 iterative refinement).  b_dev and
 * x_dev are complex128 [nrhs][N]; x_dev is the initial guess on entry and the
 * solution on return.  Blocking.  Returns AIM_ERR_NOT_CONVERGED if any
 * right-hand side misses rtol (x_dev still holds the best iterates and
 * info_host is filled), AIM_ERR_BREAKDOWN on non-finite values. */
aim_status aim_solve(aim_plan plan, const void* b_dev, void* x_dev, int32_t nrhs,
                     const int32_t* freq_idx_host, const aim_solve_opts* opts,
                     aim_solve_info* info_host, void* hip_stream);

/* Kernels of one matvec, in launch order (aim_profile_matvec). */
#define AIM_N_KERNELS 7
/* 0 project (P x), 1 x-forward FFT, 2 y-forward FFT, 3 z FFT * spectrum *
 * inverse z FFT, 4 y-inverse FFT, 5 x-inverse FFT, 6 interpolation + C x */

/* Returns in kernel_ms_host[AIM_N_KERNELS] the average duration in
 * milliseconds of each kernel of one matvec (the stages of eq. LAIMx:
 * projection, the zero-padded FFT convolution with the Toeplitz kernel, the
 * interpolation and the near-field correction): `reps` ordinary matvecs run
 * back to back on hip_stream with a HIP event recorded before, between and
 * after their seven kernels, and each kernel's average is taken over the
 * intervals it spans.  Same arguments and errors as aim_matvec; y_dev
 * receives the product; blocking. */
aim_status aim_profile_matvec(aim_plan plan, aim_precision prec, const void* x_dev, void* y_dev,
                              int32_t nrhs, const int32_t* freq_idx_host, int32_t reps,
                              double* kernel_ms_host, void* hip_stream);

/* Captures one aim_matvec (the seven kernels of eq. LAIMx's product: P x,
 * the five FFT passes with the spectral multiply, P^T phi + C x) on the given
 * buffers, precision, batch width and frequency indices into an
 * instantiated HIP graph.  aim_graph_launch replays it on any stream; the
 * buffers, the plan and its schedule must stay as they were at capture.
 * The graph holds no memset nodes.  Errors as aim_matvec. */
aim_status aim_matvec_capture(aim_plan plan, aim_precision prec, const void* x_dev, void* y_dev,
                              int32_t nrhs, const int32_t* freq_idx_host, void* hip_stream,
                              aim_graph* out);
aim_status aim_graph_launch(aim_graph graph, void* hip_stream);
aim_status aim_graph_destroy(aim_graph graph);  /* NULL is a no-op */

/* A schedule is AIM_SCHEDULE_LEN integers: the launch shape of each of the
 * five FFT passes (indices 0 .. AIM_FFT_SHAPES-1; not every shape exists for
 * every transform length), then the layout of the convolution workspace
 * (0 .. AIM_FFT_LAYOUTS-1: 0, 1, 4 or 12 KiB of padding after every z plane,
 * which keeps the strided z lines from falling on one memory channel), then
 * the stage modes 0..3: bit 0 the interpolation (0: the assembled P^T; 1:
 * the weights of P^T recomputed from the quadrature points' stencil
 * coordinates), bit 1 the projection (0: its own kernel writing the grid q;
 * 1: computed inside the x forward FFT pass, so q never goes to memory). */
#define AIM_FFT_SHAPES 12
#define AIM_FFT_LAYOUTS 4
#define AIM_SCHEDULE_LEN 7

/* Schedule autotuner for the convolution's five FFT passes (x forward,
 * y forward, z forward * spectrum * inverse, y inverse, x inverse) and the
 * interpolation: for every workspace layout, times every available launch
 * shape (lines per workgroup x threads per line) of each pass over `reps`
 * runs with nrhs right-hand sides on hip_stream and keeps the layout with
 * the smallest sum of per-pass best times and those shapes; then times whole
 * matvecs in the four stage modes and keeps the fastest.  The schedule is stored in the
 * plan for this precision and returned in sched_out[AIM_SCHEDULE_LEN], the
 * chosen passes' average times (ms) in pass_ms_out[5] (either may be NULL).
 * Overwrites the plan's internal grid workspace; allocates and frees two
 * vectors of scratch; blocking.  The schedule does not change results beyond
 * rounding order. */
aim_status aim_autotune(aim_plan plan, aim_precision prec, int32_t nrhs, int32_t reps,
                        int32_t* sched_out, double* pass_ms_out, void* hip_stream);


/* Installs a schedule (AIM_SCHEDULE_LEN entries) returned earlier by
 * aim_autotune (for example from a cache keyed by grid, precision and batch
 * width).  AIM_ERR_INVALID_ARG if a shape is out of range or not available
 * for that pass, or the layout or mode is out of range.  Graphs captured before keep
 * the schedule they were captured with. */
aim_status aim_set_schedule(aim_plan plan, aim_precision prec, const int32_t* sched);

/* ---------------------------------------------------------------------
 * Learned grid preconditioner (a project addition; the paper's own
 * preconditioners are the static diagonal and near-region blocks of
 * Sec. III-A).  A 3-level 3-D U-Net maps a grid field of 2 channels (the
 * real and imaginary parts of a complex64 grid [Nz][Ny][Nx], i.e. the
 * projected residual) to a grid field of 2 channels (a correction).
 * Layers, channels-last [z][y][x][c], base width C = 16:
 *   a0 = relu(conv3(in, 2->C)),  s0 = relu(conv3(a0, C->C))
 *   a1 = relu(conv3(pool(s0), C->2C)),  s1 = relu(conv3(a1, 2C->2C))
 *   a2 = relu(conv3(pool(s1), 2C->4C)), a3 = relu(conv3(a2, 4C->4C))
 *   a4 = relu(conv3([up(a3), s1], 6C->2C)), a5 = relu(conv3(a4, 2C->2C))
 *   a6 = relu(conv3([up(a5), s0], 3C->C)),  a7 = relu(conv3(a6, C->C))
 *   out = a7 W^T + b (1x1x1, C->2)
 * 3x3x3 "same" convolutions, 2x2x2 average pooling, nearest upsampling.
 * Weights and activations are bfloat16 with fp32 accumulation on MFMA;
 * master weights, gradients and Adam moments are fp32.  Parameters are one
 * flat fp32 vector: for every layer in the order above, W[co][tap][ci] with
 * tap = (dz+1)*9 + (dy+1)*3 + (dx+1), then b[co].  Grid dimensions must be
 * multiples of 4.  A network is not thread-safe.
 * --------------------------------------------------------------------- */
aim_status aim_unet_create(int32_t base_channels /* 16 */, uint64_t seed, aim_unet* out);
aim_status aim_unet_destroy(aim_unet net);
aim_status aim_unet_num_params(aim_unet net, int64_t* n);
/* host copies of the parameters and of the last accumulated gradient
 * (either pointer may be NULL); blocking */
aim_status aim_unet_get_params(aim_unet net, float* params_host, float* grads_host);
aim_status aim_unet_set_params(aim_unet net, const float* params_host);
/* out = U(in) for nbatch grids (complex64 [nbatch][Nz][Ny][Nx] in and out,
 * device); dims = {Nx, Ny, Nz}, each a multiple of 4; asynchronous.  The
 * batch is one pass (the grids stacked along z, each sample's 3x3x3
 * neighbourhoods ending at its own planes); each output equals the one its
 * grid gets alone.  The network's activation buffers grow to the largest
 * batch seen and are kept until aim_unet_destroy. */
aim_status aim_unet_forward(aim_unet net, const void* in_dev, void* out_dev, int32_t nbatch,
                            const int32_t dims[3], void* hip_stream);
/* One training step on grid pairs: gradients of the mean squared error
 * between U(in) and target over the batch (all on the device, one batched
 * pass), then, if apply != 0, one Adam step (beta 0.9/0.999, eps 1e-8) with
 * rate lr.  The loss value is returned in loss_host; blocking. */
aim_status aim_unet_train_grid(aim_unet net, const void* in_dev, const void* target_dev,
                               int32_t nbatch, const int32_t dims[3], double lr, int32_t apply,
                               double* loss_host, void* hip_stream);
aim_status aim_unet_save(aim_unet net, const char* path);
aim_status aim_unet_load(const char* path, aim_unet* out);

/* ---- Learned preconditioner on a plan ------------------------------------
 * The paper has no learned component; this is an addition on top of the
 * AIMx solve.  The network U maps the projected, normalised residual on the
 * AIM grid to a grid correction, which W = P^T (the interpolation of
 * eq. LAIMx) brings back to the mesh.  With B the base preconditioner:
 *   M(v) = B v + tau ||v|| (P^T U(g(v))) / area,
 *   g(v) = P (v/||v||) in complex64, scaled to unit RMS over the grid.
 * M is nonlinear, so aim_solve runs flexible GMRES (the stored Z basis).
 * Grid dimensions must be multiples of 4 and the plan must hold the
 * complex64 tables (precisions bit 1).  The network must have base width 16.
 *
 * Training data are pairs (r_t, e_t = x* - x_t) logged from plain GMRES on
 * training geometries.  Two losses (aim_pc_targets, aim_pc_train_step), with
 * r^ = r_t/||r_t||, c = P^T U(g(r_t)) and means over triangles:
 *   AIM_LOSS_ERROR:    mean |c/area - t/tau|^2,  t = (e_t - B r_t)/||r_t||,
 *                      the error itself;
 *   AIM_LOSS_RESIDUAL: weight mean |s - A (tau c/area)|^2,
 *                      s = r^ - A B r^, the same error measured through A
 *                      (A e_t = r_t up to the logging tolerance), which
 *                      weights the smooth components a grid can represent. */
typedef enum { AIM_LOSS_ERROR = 0, AIM_LOSS_RESIDUAL = 1 } aim_pc_loss;

/* Attach (net != NULL) or detach (net == NULL) a network.  base_pc is B
 * (AIM_PC_NONE, AIM_PC_DIAG or AIM_PC_NEARBLOCK) and tau > 0 the target scale
 * used in training.  The plan keeps the pointer, not a copy: the network
 * must outlive its use by aim_solve.  On a batch plan (aim_setup_batch) every
 * instance applies the network on its own grid, one instance after another
 * (the network's buffers are shared); every instance's grid must meet the
 * network's conditions.  Blocking. */
aim_status aim_plan_set_unet(aim_plan plan, aim_unet net, aim_pc_kind base_pc, double tau);

/* Solve A x = b with plain restarted GMRES (complex128, no preconditioner,
 * x0 = 0) and log a training pair at every restart of every unconverged
 * system: r_out[k] = r_t, e_out[k] = x* - x_t ([max_pairs][N] complex128
 * device buffers, caller-owned), rhs_out_host[k] = the system it came from
 * (may be NULL).  At most max_pairs pairs are written; *npairs is the
 * count.  Returns AIM_ERR_NOT_CONVERGED (pairs still written) if a system
 * did not reach rtol, since e_t is then inexact.  Blocking. */
aim_status aim_log_pairs(aim_plan plan, const void* b_dev, int32_t nrhs,
                         const int32_t* freq_idx_host, double rtol, int32_t restart,
                         int32_t max_iter, void* r_out_dev, void* e_out_dev,
                         int32_t* rhs_out_host, int32_t max_pairs, int32_t* npairs,
                         void* hip_stream);

/* Network inputs and targets of npairs logged pairs:
 *   grid_out[k]   = g(r_k)                           [npairs][Ng] complex64
 *   target_out[k] = (e_k - B r_k)/||r_k||   (ERROR)  [npairs][N]  complex128
 *                 = (r_k - A B r_k)/||r_k|| (RESIDUAL, frequency index 0)
 * (device buffers, caller-owned).  sums_host[0] = sum over all entries of
 * |(e_k - B r_k)/||r_k|| |^2 and sums_host[1] = the same of the RESIDUAL
 * target (0 for ERROR); over the whole training set, tau^2 = sums[0] /
 * (pairs N) makes the ERROR target unit-scale and weight = pairs N / sums[1]
 * the RESIDUAL loss.  Blocking. */
aim_status aim_pc_targets(aim_plan plan, aim_pc_kind base_pc, aim_pc_loss kind,
                          const void* r_pairs_dev, const void* e_pairs_dev, int32_t npairs,
                          void* grid_out_dev, void* target_out_dev, double* sums_host,
                          void* hip_stream);

/* One optimiser step over the samples sample_idx_host[0..nsamples) (indices
 * into grids/targets as written by aim_pc_targets on this plan with the same
 * kind, each in [0, npairs)): the loss of the given kind (ERROR: weight
 * times the ERROR loss) averaged over the samples, gradients through P^T
 * (and, for RESIDUAL, through A and its adjoint, complex64 products at
 * frequency index 0), the network's backward pass, then Adam with learning
 * rate lr if apply != 0.  *loss_host receives the loss before the step.
 * nsamples is limited by the plan's scratch (at least 128); the samples
 * run in batched passes of up to the plan's max_rhs.  Blocking. */
aim_status aim_pc_train_step(aim_plan plan, aim_unet net, aim_pc_loss kind,
                             const void* grids_dev, const void* targets_dev, int32_t npairs,
                             const int32_t* sample_idx_host, int32_t nsamples, double tau,
                             double weight, double lr, int32_t apply, double* loss_host,
                             void* hip_stream);

/* Host copies of setup tables, for validation against an independent
 * implementation.  Any pointer may be NULL to skip that table.
 *   stencil_start [3N][3] int32: first node of each quadrature point's stencil
 *   stencil_local [3N][3] double: t - s, t = (r - origin)/h per axis
 *   rowptr [N+1] int64, col [nnz] int32, val [nnz] double: C in CSR
 *   near_static [nnz] double: A_s,NR on the same pattern
 * Blocking. */
aim_status aim_export_tables(aim_plan plan, int32_t* stencil_start, double* stencil_local,
                             int64_t* rowptr, int32_t* col, double* val, double* near_static);

/* Message of the last failing call on this thread ("" if none). */
const char* aim_last_error(void);

/* Library version string. */
const char* aim_version(void);

#ifdef __cplusplus
}
#endif

#endif /* AIM_H */
