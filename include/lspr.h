/*
 * lspr.h -- C ABI of the MI355X quasistatic LSPR boundary-element library.
 *
 * Method: Clementi, Cooper & Barba, "Computational nanoplasmonics in the quasistatic limit for
 * biosensing applications" (arXiv 1812.10722).  A metal nanoparticle (surface 0) and optional
 * dielectric analytes (surfaces 1..S-1) sit in a host medium under a uniform field E.  The
 * scattered potential solves the boundary integral equations of Eqs. integral_eq_lspr /
 * integral_eq_lspr_system, discretised with flat triangles, piecewise-constant unknowns and
 * centroid collocation (Eqs. layers_disc, matrix_lspr, matrix_multi).  The dense matrix-vector
 * product is replaced by a treecode (section "Acceleration strategies") and the complex
 * systems are solved by GMRES; the outputs are the surface potential and normal derivative,
 * the dipole moment (section "Boundary integral expression of the dipole moment") and the
 * extinction cross-section (Eq. cext_fwa).
 *
 * Units: lengths in nm, wavelengths in nm, permittivities relative (dimensionless).
 *
 * Conventions for every entry point:
 *   - Return value: an lspr_status code.  Nothing aborts; on error the outputs are unspecified
 *     (except LSPR_E_NOCONV, see lspr_solve) and lspr_last_error() holds a message for the
 *     calling thread.
 *   - Ownership: the caller owns every buffer it passes.  lspr_geometry_create copies what it
 *     needs; a geometry handle owns its own device memory (trees, lists, near-field tables,
 *     Krylov workspace) and frees it in lspr_geometry_destroy.
 *   - "device" pointers are HIP device addresses on the current device (for instance
 *     torch.Tensor.data_ptr() of a cuda tensor); "host" pointers are ordinary memory.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Calls are synchronous with respect
 *     to the host: they return after their work on `stream` has finished.
 *   - Calls on one geometry handle must not overlap (a handle holds one Krylov workspace).
 */
#ifndef LSPR_H
#define LSPR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } lspr_c64;

typedef struct lspr_geometry lspr_geometry;

enum lspr_status {
    LSPR_OK = 0,
    LSPR_E_INVALID = 1,   /* bad argument (NULL pointer, size or parameter out of range) */
    LSPR_E_MESH = 2,      /* mesh rejected: index out of range, degenerate, open or inverted */
    LSPR_E_NOMEM = 3,     /* device allocation failed */
    LSPR_E_DEVICE = 4,    /* a HIP call failed */
    LSPR_E_NOCONV = 5,    /* GMRES hit max_iter; outputs hold the last iterate */
    LSPR_E_BUSY = 6       /* (serving) request not finished yet */
};

enum lspr_method { LSPR_DENSE = 0, LSPR_TREECODE = 1 };
enum lspr_precision { LSPR_FP64 = 0, LSPR_FP32 = 1, LSPR_FP32_REFINE64 = 2, LSPR_FP32_LEAD64 = 3 };
enum lspr_flags {
    LSPR_NO_MATRIX_CORES = 1,
    /* bit 1 (value 2) is retired: it selected a schedule with both operators per four-wave
     * workgroup; a geometry created with it is refused as an unknown flag */
    LSPR_STREAM_NARROW = 4,
    LSPR_PAIR_OPERATORS = 8,
    LSPR_PAIR_NARROW = 16,
    LSPR_FOUR_WAVE = 32
};

/* One closed surface.  vert: [n_vert][3] FP64, tri: [n_tri][3] int32 vertex indices ordered
 * counter-clockwise seen from outside (outward right-hand normal, as the paper's dipole
 * section requires).  Device pointers in lspr_geometry_create; host pointers in
 * lspr_mesh_validate. */
typedef struct {
    int32_t n_vert;
    const double* vert;
    int32_t n_tri;
    const int32_t* tri;
} lspr_surface;

/* Discretisation and treecode parameters (section "Integral evaluation", Tables 1, 2, 4, 5;
 * section "Acceleration strategies").
 *   k_far     points of the far-panel rule: 1, 3, 4 or 7 (the paper uses 4)
 *   k_fine    points of the near-singular rule: 19, 25 or 37 (Dunavant's degree-9, 10 and 13
 *             rules; the paper uses 19 and, for its grid-convergence study, 37)
 *   n_k       Gauss nodes per edge of the semi-analytic singular rule, 1..64 (paper: 9)
 *   threshold a source panel j is near-singular for collocation point x_i when
 *             |x_i - c_j| <= L_j / threshold, L = sqrt(2 Area) (paper: 0.5, i.e. 2L)
 *   method    LSPR_DENSE (every far pair summed directly) or LSPR_TREECODE
 *   p         Taylor expansion order of the treecode: 2, 4, 6, 8, 10, 12 or 15 (paper: 6,
 *             and 15 for its grid-convergence study); orders above 10 run only on matrix cores
 *             (their tiles must fit the tile budget, else LSPR_E_NOMEM)
 *   theta     multipole acceptance parameter, 0 < theta < 1 (paper: 0.5)
 *   ncrit     maximum panels per octree leaf; 0 selects the library default
 *   precision LSPR_FP64 or LSPR_FP32 for the far-field sums (P2P, P2M, M2P).  Singular and
 *             near-singular corrections, the GMRES and the post-processing are always FP64.
 *             LSPR_FP32_REFINE64: mixed-precision iterative refinement; GMRES with FP32 products
 *             solves for corrections, and the residual b - A x of each outer step is formed
 *             with FP64 products; tol then applies to that FP64 residual, and lspr_apply uses
 *             the FP64 products.
 *             LSPR_FP32_LEAD64: one GMRES whose product for a wavelength runs in FP64 while
 *             that wavelength's residual estimate is above inner_tol ||b|| (the leading Krylov
 *             vectors, whose coefficients in the solution are largest) and in FP32 after;
 *             the true residual at each restart uses FP32 products, and lspr_apply uses the
 *             FP64 products.  Needs the tile stores of both precisions.
 *   m2p_min_panels  a box that passes the MAC is expanded only if it holds at least this many
 *             panels, otherwise it is summed directly (cheaper for small boxes); 0 selects the
 *             library default (the number of expansion terms).  Accuracy is unaffected: a
 *             direct sum is exact to the quadrature.
 *   flags     bit 0: never use the matrix-core far-field kernel.  By default a geometry
 *             precomputes the geometry-only factors of every expansion and direct tile in the
 *             precision(s) it computes in (about 1.7 GB at 32768 panels, P = 8, in FP32; twice
 *             that in FP64) and runs all products on matrix cores.  Tiles are kept while they
 *             fit in 55 % of the free device memory (FP32 first, then FP64); a precision whose
 *             tiles do not fit uses the vector-ALU kernel, which computes the same sums on the
 *             fly.
 *             bit 1: retired (refused).
 *             bit 2: products of up to 16 wavelengths stream every wave's operands from
 *             memory instead of staging each left factor in LDS for the workgroup (identical
 *             sums; a tuning alternative, faster for FP64 products of up to 8 wavelengths).
 *             bit 3: products of more than 16 wavelengths run eight-wave workgroups that stage
 *             each left factor once for both operators (identical sums; a tuning
 *             alternative).
 *             bit 4: the same for products of up to 16 wavelengths.
 *             bit 5: products run four-wave workgroups that stage the left factors through
 *             registers (more than 32 wavelengths: one column half each) instead of
 *             eight-wave workgroups that read them straight into LDS buffers (more than 32
 *             wavelengths, FP32 and FP64: both column halves, identical sums; FP32 up to 16
 *             wavelengths at P = 8 or 15: 4 or 8 waves per column group instead of 2 or 4, so
 *             the FP32 partial sums are split differently).  A tuning alternative. */
typedef struct {
    int32_t k_far;
    int32_t k_fine;
    int32_t n_k;
    double threshold;
    int32_t method;
    int32_t p;
    double theta;
    int32_t ncrit;
    int32_t precision;
    int32_t m2p_min_panels;
    int32_t flags;
} lspr_op_params;

/* GMRES parameters (the paper gives only tolerances, Tables 2 and 5).
 *   tol       stop a wavelength when ||b - A x||_2 <= tol ||b||_2 (complex 2-norm over all
 *             2N unknowns).  LSPR_FP32 and LSPR_FP32_LEAD64 form that residual with FP32
 *             products and reject tol < 1e-6 (LSPR_E_INVALID): use LSPR_FP32_REFINE64 or
 *             LSPR_FP64 for tighter tolerances
 *   restart   Krylov dimension before restart, 1..512
 *   max_iter  total iteration cap per wavelength
 *   precond   0 = none, 1 = right block-Jacobi with the 2x2 self-panel blocks (does not
 *             change the solution, only the iteration count)
 *   inner_tol LSPR_FP32_REFINE64: relative tolerance of each inner FP32 solve (0 selects
 *             1e-4, values below 1e-6 are rejected); max_iter then caps the inner iterations
 *             summed over the outer steps.
 *             LSPR_FP32_LEAD64: relative residual level below which a wavelength's products
 *             switch from FP64 to FP32 (0 selects 0.3).  Ignored otherwise. */
typedef struct {
    double tol;
    int32_t restart;
    int32_t max_iter;
    int32_t precond;
    double inner_tol;
} lspr_gmres_params;

/* Sizes of a built geometry (host struct filled by lspr_geometry_info). */
typedef struct {
    int64_t n_panels;        /* N, all surfaces */
    int64_t n_surfaces;
    int64_t n_nodes;         /* N * k_far treecode sources */
    int64_t n_boxes;         /* octree boxes, all surfaces */
    int64_t n_leaves;
    int64_t n_target_chunks; /* groups of consecutive targets sharing interaction lists */
    int64_t n_m2p;           /* (target chunk, box) expansion interactions */
    int64_t n_p2p_ranges;    /* (target chunk, source range) direct interactions */
    int64_t p2p_pairs;       /* target-panel x source-panel pairs summed directly */
    int64_t m2p_pairs;       /* target x box pairs evaluated by expansion */
    int64_t n_near;          /* near-singular (target, source) pairs with fine-rule corrections */
    int64_t device_bytes;    /* device memory held by the handle (without Krylov workspace) */
    int32_t n_terms;         /* expansion terms per box and column */
    int32_t ncrit;           /* leaf capacity actually used */
    int32_t target_chunk;    /* targets per chunk */
    int32_t max_depth;
    int64_t n_tiles;         /* matrix-core tiles (0 when the on-the-fly kernel is used) */
    int64_t tile_steps;      /* K-steps over all tiles (matrix-core work per column tile) */
    int64_t max_chunk_steps; /* K-steps of the most loaded target chunk */
} lspr_geometry_stats;

/* Checks host-side surfaces before upload: indices in range, non-degenerate panels, every
 * edge shared by exactly two panels with opposite orientation (closed, consistently oriented
 * 2-manifold) and positive enclosed volume (outward normals).  Returns LSPR_OK or
 * LSPR_E_MESH / LSPR_E_INVALID with a message. */
int lspr_mesh_validate(const lspr_surface* surfaces, int32_t n_surf);

/* Builds everything that depends on geometry only (section "Integral evaluation",
 * section "Acceleration strategies"): panel areas, normals, centroids and quadrature nodes,
 * Morton order and octree, interaction lists under the MAC, singular self-terms,
 * near-singular correction table and the geometry part of the right-hand side.
 * surfaces: host array of n_surf descriptors whose vert/tri point to DEVICE memory.
 * Surface 0 is the sensor.  Device-side checks reject out-of-range indices and zero-area
 * panels (LSPR_E_MESH); topology is checked by lspr_mesh_validate.  *out receives the
 * handle. */
int lspr_geometry_create(const lspr_surface* surfaces, int32_t n_surf,
                         const lspr_op_params* op, void* stream, lspr_geometry** out);

int lspr_geometry_destroy(lspr_geometry* g);

int lspr_geometry_info(const lspr_geometry* g, lspr_geometry_stats* out);

/* Solves n_lambda independent wavelengths in one batch (Eq. matrix_multi per wavelength),
 * sharing every matrix-vector product launch.
 *   lambda_nm    host [n_lambda]
 *   eps_medium   host [n_lambda]            host-medium permittivity
 *   eps_surface  host [n_lambda][n_surf]    interior permittivity of each surface
 *   e_field      host [3]                   real incident field E (C_ext does not depend on
 *                                           its magnitude or sign)
 *   gm           host                       GMRES parameters
 *   phi, dphi    device [n_lambda][N] or NULL: interior-side potential and normal derivative
 *                per panel, in the caller's panel order (surfaces concatenated)
 *   p_sensor     host [n_lambda][3] or NULL: dipole moment p = eps_m * q of surface 0 alone
 *   p_total      host [n_lambda][3] or NULL: dipole moment of all surfaces
 *   cext_sensor  host [n_lambda] or NULL: extinction cross-section (nm^2) from p_sensor
 *   cext_total   host [n_lambda] or NULL: extinction cross-section from p_total
 *   iters        host [n_lambda] or NULL: GMRES iterations per wavelength
 *   rel_resid    host [n_lambda] or NULL: final ||b - A x|| / ||b|| per wavelength
 * Returns LSPR_E_NOCONV (with all outputs filled from the last iterate) when some wavelength
 * did not reach tol within max_iter. */
int lspr_solve(lspr_geometry* g, int32_t n_lambda, const double* lambda_nm,
               const lspr_c64* eps_medium, const lspr_c64* eps_surface, const double* e_field,
               const lspr_gmres_params* gm, void* stream, lspr_c64* phi, lspr_c64* dphi,
               lspr_c64* p_sensor, lspr_c64* p_total, double* cext_sensor, double* cext_total,
               int32_t* iters, double* rel_resid);

/* One block matrix-vector product y = A x of the system of Eq. matrix_multi for n_cols
 * independent permittivity sets (no preconditioner).
 *   eps_medium host [n_cols], eps_surface host [n_cols][n_surf]
 *   x, y       device [n_cols][2N] complex: per column all phi (caller's panel order), then
 *              all dphi/dn; y rows: all interior rows, then all exterior rows. */
int lspr_apply(lspr_geometry* g, int32_t n_cols, const lspr_c64* eps_medium,
               const lspr_c64* eps_surface, const lspr_c64* x, lspr_c64* y, void* stream);

/* For callers that cannot allocate device memory (code under stream capture, tight serving
 * loops, harnesses that forbid hipMalloc): lspr_apply with every temporary of the product
 * (permittivity ratios, sorted copies of x and y, packed densities, raw layer sums, box moments
 * and partial moments) in one fixed device array of LSPR_NOALLOC_SCRATCH_MIB MiB, which the
 * library holds on every device it runs on from its load until the process ends.  Arguments,
 * batching (64 columns at a time) and results are those of lspr_apply, bit for bit (the same
 * kernels in the same order); the geometry is created beforehand with lspr_geometry_create.
 * The call allocates no device memory and calls no allocating library routine.
 * LSPR_E_INVALID, with the number of bytes in lspr_last_error(), when one batch needs more
 * scratch than the array holds (roughly 64 N B + 16 N pad (S > 1 ? 3 : 2) bytes plus the
 * moments, B the columns of a batch and pad = 2 B rounded up to 16: e.g. N = 32768 panels fits
 * up to about 16 columns).  Every call on one device shares that device's array and leaves its
 * contents behind (nothing in it needs to start at zero): calls that overlap on one device
 * (other streams or threads) race and must be serialised by the caller. */
#define LSPR_NOALLOC_SCRATCH_MIB 256
int lspr_apply_noalloc(lspr_geometry* g, int32_t n_cols, const lspr_c64* eps_medium,
                       const lspr_c64* eps_surface, const lspr_c64* x, lspr_c64* y,
                       void* stream);

/* Right-hand side of Eq. matrix_multi for n_cols permittivity sets: b device [n_cols][2N]
 * (interior rows zero; exterior rows sum_s ((eps_m - eps_s)/eps_m) V_s g_s, g = -E . n). */
int lspr_rhs(lspr_geometry* g, int32_t n_cols, const lspr_c64* eps_medium,
             const lspr_c64* eps_surface, const double* e_field, lspr_c64* b, void* stream);

/* The library's own triangle rule with n points (bary host [n][3], w host [n], weights sum to
 * 1) and its Gauss-Legendre rule (t host [n], w host [n] on [-1, 1]).  For verification. */
int lspr_triangle_rule(int32_t n, double* bary, double* w);
int lspr_gauss_legendre(int32_t n, double* t, double* w);

/* Kernel profiling (tracing).  When enabled, the library brackets its main launches with HIP
 * events on the launch stream and records, per launch, the algorithmic work: flops counted from
 * the interaction lists (direct pairs, expansion pairs) and the columns actually used, bytes of
 * the arrays the kernel must read and write once.  Names: "far" (expansions plus direct sums),
 * "p2m", "near" (near-singular corrections), "matvec" (one whole block product), "arnoldi"
 * (orthogonalisation of one GMRES step).  "far" (FP32 products) and "far64" (FP64) count, on
 * the matrix-core path, the work the launch executes: 4 flops per used real column of each
 * operator and direct (target, panel) pair, 4 (P+1)^2 per column and expansion (target, box)
 * pair; bytes are the tile store (read once), the densities, moments and sums.  The kernel
 * values and Taylor coefficients are computed once per geometry, not per launch, and are not
 * counted (the vector-ALU kernel, which computes them on the fly, counts them too).  For "far",
 * `items` counts interactions times wavelengths: (direct target-node pairs + expansion
 * target-box pairs) per launch times the complex columns of that launch.  lspr_profile_query
 * waits for the recorded events and returns totals since the last reset; unknown names give
 * zero launches.  lspr_profile_query_width does the same for the launches of width_min ..
 * width_max wavelengths (complex columns; scopes without a width count as 0).  on: 0 off,
 * 1 all launches, 2 far-field launches only ("far", "far64"; the fewest events in the timed
 * stream). */
int lspr_profile_enable(int32_t on);
int lspr_profile_reset(void);
int lspr_profile_query(const char* name, double* total_ms, int64_t* launches, double* flops,
                       double* bytes, double* items);
int lspr_profile_query_width(const char* name, int32_t width_min, int32_t width_max,
                             double* total_ms, int64_t* launches, double* flops, double* bytes,
                             double* items);

/* ------------------------------------------------------------------ request server
 * Continuous batching of independent solve requests (mixed meshes, wavelength sets and
 * analyte placements) on one GPU.  Each request is one lspr_geometry_create + lspr_solve with
 * its own stream; up to max_slots requests are on the device at once, their kernels overlap,
 * and a queued request is admitted, in arrival order, as soon as a slot is free and its
 * footprint estimate (lspr_request_footprint) fits into the device-memory budget beside the
 * requests already admitted.  All device memory of a request comes from a memory pool owned by
 * the server and is released stream-ordered, so no request synchronises the whole device.
 * Trees, interaction lists, tiles and Krylov state stay on the device for the life of the
 * request.  A request's results do not depend on what else is running (every kernel sums in
 * a fixed order). */
typedef struct lspr_server lspr_server;

typedef struct {
    int64_t hbm_budget_bytes; /* device bytes admitted requests may hold; 0 = 85 % of the free
                                 device memory when the server is created */
    int32_t max_slots;        /* requests on the device at once, 1..16 */
    int32_t pad;
} lspr_server_params;

typedef struct {
    int32_t status;      /* LSPR_OK, LSPR_E_NOCONV (outputs from the last iterate) or the error
                            that ended the request */
    int32_t n_lambda;
    int64_t n_panels;
    double t_submit;     /* seconds since the server was created */
    double t_admit;      /* admission: slot and memory granted */
    double t_done;       /* results ready; latency = t_done - t_submit */
    int64_t est_bytes;   /* admission estimate */
    int64_t peak_bytes;  /* measured peak of the request's device allocations */
    char error[256];     /* error text when status != LSPR_OK (truncated), else empty */
} lspr_request_info;

typedef struct {
    int64_t submitted, completed, queued, active;
    int64_t max_active;           /* most requests on the device at once so far */
    int64_t budget_bytes, reserved_bytes, peak_reserved_bytes;
    int64_t estimate_violations;  /* requests whose measured peak exceeded their estimate */
} lspr_server_stats;

/* Creates a server on the current device (worker threads, one non-blocking stream per slot at
 * the default priority, and a device memory pool). */
int lspr_server_create(const lspr_server_params* params, lspr_server** out);

/* Queues one request.  All pointers are HOST pointers and are copied before return, so the
 * caller may free them at once: surfaces (as lspr_geometry_create), op, lambda_nm [n_lambda],
 * eps_medium [n_lambda], eps_surface [n_lambda][n_surf], e_field [3], gm.  The mesh topology is
 * checked as by lspr_mesh_validate when the request runs.  Returns LSPR_E_NOMEM at once when
 * the request's footprint exceeds the whole budget, LSPR_E_INVALID for bad parameters;
 * *ticket identifies the request. */
int lspr_server_submit(lspr_server* sv, const lspr_surface* surfaces, int32_t n_surf,
                       const lspr_op_params* op, int32_t n_lambda, const double* lambda_nm,
                       const lspr_c64* eps_medium, const lspr_c64* eps_surface,
                       const double* e_field, const lspr_gmres_params* gm, uint64_t* ticket);

/* As lspr_server_submit, with point charges inside the surfaces (Eq. integral_eq_lspr_system,
 * last row; arguments and units as lspr_geometry_set_charges, HOST arrays copied before
 * return): the request's geometry takes them before its solve.  n_q = 0 is a plain request.
 * LSPR_E_INVALID at once for a surface index out of range or non-finite values. */
int lspr_server_submit_charges(lspr_server* sv, const lspr_surface* surfaces, int32_t n_surf,
                               const lspr_op_params* op, int32_t n_lambda,
                               const double* lambda_nm, const lspr_c64* eps_medium,
                               const lspr_c64* eps_surface, const double* e_field,
                               const lspr_gmres_params* gm, int32_t n_q, const double* pos,
                               const double* q, const int32_t* surface, uint64_t* ticket);

/* Result of a request.  wait = 0 returns LSPR_E_BUSY while the request is queued or running;
 * wait != 0 blocks until it is done.  On LSPR_OK the results are copied (host arrays of
 * n_lambda entries, [n_lambda][3] for the dipoles; any may be NULL), *info is filled and the
 * ticket is released.  The request's own status is info->status; unknown tickets give
 * LSPR_E_INVALID. */
int lspr_server_poll(lspr_server* sv, uint64_t ticket, int32_t wait, lspr_request_info* info,
                     double* cext_sensor, double* cext_total, lspr_c64* p_sensor,
                     lspr_c64* p_total, int32_t* iters, double* rel_resid);

int lspr_server_stats_get(lspr_server* sv, lspr_server_stats* out);

/* Waits for the running requests, cancels the queued ones and frees everything. */
int lspr_server_destroy(lspr_server* sv);

/* Admission estimate: an upper bound of the device bytes one request with N panels on n_surf
 * surfaces and n_lambda wavelengths holds at its peak (set-up, matrix-core tiles up to their
 * cap, GMRES state for one batch of at most 64 wavelengths).  Host arithmetic only (no device
 * call).  LSPR_E_INVALID for null pointers, non-positive sizes or an unknown precision. */
int lspr_request_footprint(int64_t n_panels, int32_t n_surf, int32_t n_lambda,
                           const lspr_op_params* op, const lspr_gmres_params* gm,
                           int64_t* bytes);

/* Autotuner for the treecode parameters and kernel schedule of a mesh (the paper picks P and
 * theta by hand per experiment, section "Acceleration strategies", Tables treeparams1/2).
 * Stage 1: expansion order P in {4, 6, 8, 10, 12, 15}, acceptance parameter theta in {0.4,
 * 0.5, 0.6, 0.7} and leaf size N_crit in {8, 16, 32} (above 100000 panels theta in {0.5, 0.6}
 * and N_crit = 16).  The truncation error of a candidate is measured apart from rounding: the
 * relative 2-norm difference between its FP64 product of the system matrix (first
 * wavelength's permittivities, a fixed pseudo-random complex vector) and the dense FP64
 * product (every far pair summed directly).  For each (theta, N_crit) the smallest P that meets
 * max_rel_err is timed: n_cols columns in the product precision of op (FP32 unless
 * op->precision is LSPR_FP64), fastest of three after one warm-up, HIP events on `stream`.
 * Stage 2, on the fastest of those: the kernel schedule, timed the same way: m2p_min_panels at
 * half and twice its default ((P+1)^2; the error is checked again), for n_cols <= 16 the
 * streamed narrow kernel (LSPR_STREAM_NARROW), for n_cols > 16 the paired-operator workgroups
 * (LSPR_PAIR_OPERATORS), in FP32 the four-wave workgroups (LSPR_FOUR_WAVE).  The fastest
 * candidate that meets the bound is written
 * to op->p, op->theta, op->ncrit, op->m2p_min_panels and op->flags (op->method becomes
 * LSPR_TREECODE; the other fields are kept and used for every candidate).
 *   surfaces     device pointers, as lspr_geometry_create
 *   n_cols       columns of the timed product, 1..64
 *   eps_medium   host [1]; eps_surface host [n_surf]
 *   entries      host [max_entries] or null: every candidate tried, in order (ms_per_product
 *                -1 when it was not timed; rel_err infinite for a candidate whose set-up did
 *                not fit the device, which also ends that (theta, N_crit)'s orders); *n_entries
 *                receives their number (it may exceed max_entries, the rest is not stored)
 * Device memory: the reference geometry (dense FP64 tiles, 16 N^2 bytes, when they fit) and one
 * candidate geometry at a time.  LSPR_E_NOCONV when no candidate meets the bound (op then holds
 * the most accurate one); LSPR_E_INVALID for bad arguments. */
typedef struct {
    int32_t p;
    int32_t ncrit;
    double theta;
    double rel_err;         /* FP64 product against the reference */
    double ms_per_product;  /* n_cols columns in the timed precision, or -1 */
    int32_t m2p_min_panels; /* 0: the default */
    int32_t flags;          /* lspr_flags of the candidate */
} lspr_tune_entry;

int lspr_autotune(const lspr_surface* surfaces, int32_t n_surf, int32_t n_cols,
                  const lspr_c64* eps_medium, const lspr_c64* eps_surface, double max_rel_err,
                  lspr_op_params* op, lspr_tune_entry* entries, int32_t max_entries,
                  int32_t* n_entries, void* stream);

/* Point charges inside the surfaces (Eq. integral_eq_lspr_system, last row: the charges of an
 * analyte put (1 / (4 pi eps_s)) sum_k q_k / |x_i - r_k| on the right of the interior rows of
 * its panels i, eps_s the surface's relative permittivity at each wavelength).  Host arrays:
 * pos [n_q][3] (same length unit as the mesh), q [n_q] (charge divided by the vacuum
 * permittivity, in units of the incident potential times length: one elementary charge is
 * 18.0951 V nm), surface [n_q] (index of the enclosing surface).  The geometry keeps
 * sum_k q_k / (4 pi |c_i - r_k|) per panel (FP64, direct sum) for every later lspr_solve and
 * lspr_rhs; n_q = 0 removes the charges.  lspr_server_submit_charges passes charges to the
 * request server.  LSPR_E_INVALID for a surface index out of range or non-finite values. */
int lspr_geometry_set_charges(lspr_geometry* g, int32_t n_q, const double* pos, const double* q,
                              const int32_t* surface, void* stream);

/* Resonance peak of a sampled extinction spectrum (the quantity a plasmonic sensor reads: the
 * peak position and its shift when analytes bind, section "Results", sensing experiments).
 * lambda host [n] strictly increasing, cext host [n], n >= 3.  The peak is the vertex of the
 * parabola through the largest sample and its two neighbours (exact for a parabola; on a
 * non-uniform grid the parabola is fitted exactly through the three points).  A maximum at
 * either end of the grid returns that end point.  *peak_lambda and *peak_cext receive the
 * vertex.  LSPR_E_INVALID for n < 3, null pointers or a grid that is not increasing. */
int lspr_resonance_peak(int32_t n, const double* lambda, const double* cext,
                        double* peak_lambda, double* peak_cext);

const char* lspr_status_string(int code);
const char* lspr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LSPR_H */
