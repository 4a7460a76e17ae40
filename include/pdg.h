/*
 * pdg.h -- C-ABI of the MI355X (gfx950) library for the per-time-step solve of
 * the Crank-Nicolson / SIPG-PolyDG monodomain system with the two-level
 * non-overlapping additive Schwarz preconditioned conjugate gradient.
 *
 * Paper: "A massively parallel non-overlapping Schwarz preconditioner for
 * PolyDG methods in brain electrophysiology" (arXiv 2512.19536).
 *   - model: Section 2, eq. (1);
 *   - discretisation: Section 3, eqs. (2)-(4);
 *   - preconditioner: Section 4, eq. (5);
 *   - solver and stopping rule: Sections 4-5.
 *
 * Conventions shared by every call
 *   - Every call returns a pdg_status; no C++ exception crosses the ABI.  On
 *     error pdg_last_error(ctx) returns a message.
 *   - Call order: pdg_create -> pdg_set_mesh -> pdg_assemble -> [pdg_set_ionic]
 *     -> pdg_setup_preconditioner -> pdg_workspace_query -> pdg_bind_workspace
 *     -> compute calls.  Out-of-order calls return PDG_ESTATE.
 *   - Host arrays passed in are copied; the caller keeps ownership.
 *   - "Device" pointers are HIP device memory owned by the caller (e.g. torch
 *     tensors).  The library reads/writes them only on the stream given to
 *     pdg_create.  The library never allocates device memory itself: all of its
 *     device state lives in the single workspace bound by pdg_bind_workspace.
 *   - Coefficient vectors are element-major: entry (e, i) at e*nd + i, where i
 *     indexes the modal basis of element e (Legendre polynomials of total
 *     degree <= p on the element's bounding box, orthonormal on the box;
 *     ordering: total degree ascending, then alpha_1 descending, then
 *     alpha_2 descending).  Ionic states are [5][n_elem][nd] (state-major).
 *   - A context is not thread-safe.  Separate contexts may use separate streams.
 *   - Compute calls are asynchronous with respect to the host except where
 *     stated (pdg_solve and pdg_step synchronise the stream to report
 *     iteration counts).
 */
#ifndef PDG_H
#define PDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pdg_ctx pdg_ctx;

typedef enum {
    PDG_OK = 0,
    PDG_EINVAL = -1,      /* bad argument (size, pointer, value, label)           */
    PDG_ENOMEM = -2,      /* workspace too small / host allocation failed          */
    PDG_EHIP = -3,        /* a HIP runtime call failed                             */
    PDG_ENOTSPD = -4,     /* a Cholesky pivot <= 0 during setup                    */
    PDG_ENOCONV = -5,     /* PCG hit maxit; x holds the last iterate               */
    PDG_EBREAKDOWN = -6,  /* (p, K p) <= 0 or (r, z) <= 0 inside PCG               */
    PDG_ENONFINITE = -7,  /* NaN/Inf in PCG scalars, or a non-positive ionic
                             concentration before a logarithm                      */
    PDG_ESTATE = -8       /* call out of order / no GPU bound                      */
} pdg_status;

typedef enum { PDG_F64 = 0, PDG_F32 = 1, PDG_BF16 = 2 } pdg_precision;

typedef struct {
    int32_t iters;        /* PCG iterations performed (0 if x0 already met tol)    */
    double relres;        /* ||r_k|| / ||b|| of the recurrence residual            */
    double true_relres;   /* ||b - K x|| / ||b|| if requested, else -1             */
    double bnorm;         /* ||b||                                                 */
    int32_t guess_used;   /* pdg_step_guess: systems that started from the guess
                             (0 = all fell back to U^k); -1 = no guess offered      */
    int32_t local_fp32;   /* BF16 local store: subdomains whose rounded inverse
                             failed the positive-definiteness check at setup and
                             are applied from FP32 tiles instead (0 otherwise)      */
} pdg_solve_info;

/* Create a context on HIP device `hip_device`, launching on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  hip_device = -1 creates a
 * host-only context: setup calls work, compute calls return PDG_ESTATE. */
pdg_status pdg_create(pdg_ctx **out, int32_t hip_device, void *hip_stream);
void pdg_destroy(pdg_ctx *ctx);
const char *pdg_last_error(const pdg_ctx *ctx);
const char *pdg_status_string(int32_t status);

/* ------------------------------------------------------------------------
 * 1. Mesh and degree (Section 3: polytopal mesh T_h, broken space P^p).
 * Each element is a union of sub-cells: triangles (dim 2) or axis-aligned
 * boxes (dim 3).  Facets are the pieces of element boundaries: segments
 * (dim 2) or axis-aligned rectangles (dim 3); only interior facets
 * (plus >= 0) enter the SIPG form (homogeneous Neumann condition, eq. (1)).
 *   cell_ptr     [n_elem+1]            CSR over sub-cells
 *   cell_geom    dim 2: [n_cell][3][2] triangle vertices
 *                dim 3: [n_cell][2][3] box lo corner, hi corner
 *   facet_elem   [n_facet][2]          minus, plus (plus = -1 on the boundary)
 *   facet_geom   dim 2: [n_facet][2][2] end points; dim 3: [n_facet][2][3] lo, hi
 *   facet_normal [n_facet][dim]        unit normal from minus to plus
 *   sigma        [n_elem][dim][dim]    SPD conductivity tensor, constant per element
 * Errors: PDG_EINVAL for dim not in {2,3}, p not in 1..4, empty element,
 * out-of-range element index, non-unit normal, non-SPD sigma. */
typedef struct {
    int32_t dim;
    int64_t n_elem;
    const int64_t *cell_ptr;
    const double *cell_geom;
    int64_t n_facet;
    const int64_t *facet_elem;
    const double *facet_geom;
    const double *facet_normal;
    const double *sigma;
} pdg_mesh;

pdg_status pdg_set_mesh(pdg_ctx *ctx, const pdg_mesh *mesh, int32_t p);

/* Batch of independent systems (the batching form; not part of the paper).
 * A context may hold several independent problems of the same degree p: their
 * meshes are concatenated into the one mesh given to pdg_set_mesh, and the
 * elements of system s are the contiguous run [elem_ptr[s], elem_ptr[s+1])
 * (elem_ptr: host array of n_sys + 1 entries, from 0 to n_elem).  No facet may
 * join two systems, and no subdomain or coarse element may span two.  Each
 * system runs its own PCG (own alpha, beta, and stopping test on its own
 * ||b_s||) inside shared kernel launches; every system gets the bits it would
 * get in a context of its own.  The coarse level gets one dense K_0 per system.
 * Default: one system.  Call after pdg_set_mesh, before
 * pdg_setup_preconditioner.  Errors: PDG_EINVAL (ranges, a facet between
 * systems), PDG_ESTATE (order). */
pdg_status pdg_set_systems(pdg_ctx *ctx, int32_t n_sys, const int64_t *elem_ptr);

/* Sizes after pdg_set_mesh (any pointer may be NULL). */
pdg_status pdg_get_sizes(const pdg_ctx *ctx, int64_t *n_elem, int32_t *nd, int64_t *n_dof,
                         int64_t *nnz_blocks);

/* ------------------------------------------------------------------------
 * 2. Assembly (Section 3): K = (chi_m C_m / dt) M + 1/2 A, i.e. the paper's
 * K_h = C_m chi_m M_h + dt/2 A_h divided by dt.  A is the SIPG form of
 * eq. (3) with the penalty of eq. (2): eta = eta0 {Sigma_K}_A p^2 / {h_K}_H,
 * Sigma_K = largest eigenvalue of sigma on K, h_K = element diameter.
 * Quadrature: 2-D sub-triangles by the collapsed (Duffy) map with (p+2)^2
 * Gauss points, 3-D sub-boxes with (p+1)^3 points; facets with p+2 (2-D) or
 * (p+1)^2 (3-D) points.  Host computation; stored as block-sparse rows of
 * nd x nd element blocks (diagonal block first). */
pdg_status pdg_assemble(pdg_ctx *ctx, double chi_m, double c_m, double dt, double eta0);

/* Host copies of the assembled operators (for checking): row_ptr [n_elem+1],
 * col [nnzb], val [nnzb][nd][nd] (row = test function, col = trial), mass
 * blocks [n_elem][nd][nd].  Any pointer may be NULL. */
pdg_status pdg_get_matrix(const pdg_ctx *ctx, int64_t *row_ptr, int32_t *col, double *val,
                          double *mass);

/* ------------------------------------------------------------------------
 * Ionic model parameters (Section 2, Barreto-Cressman; the paper defers its
 * equations to the cited works).  `params` holds n_params = 24 doubles in this
 * order: g_Na, g_NaL, g_K, g_KL, g_AHP, g_ClL, g_Ca, V_Ca, phi, tau, beta,
 * rho, G_glia, eps, k_bath, Cl_i, Cl_o, nernst, gamma, ca_tau, ca_coef,
 * K_i0, Na_i0, Na_o0.  Required before pdg_step / pdg_ionic. */
pdg_status pdg_set_ionic(pdg_ctx *ctx, const double *params, int32_t n_params);

/* ------------------------------------------------------------------------
 * 3. Two-level additive Schwarz preconditioner (Section 4, eq. (5)):
 * B^{-1} = sum_i R_i^T K_i^{-1} R_i + P K_0^{-1} P^T with K_i the principal
 * submatrix of K on the dofs of subdomain i, P the exact L^2 injection of
 * P^q on each coarse agglomerate (same modal basis on the agglomerate's
 * bounding box) and K_0 = P^T K P.  Local and coarse matrices are inverted
 * densely on the host in FP64 (Cholesky); the inverses are stored as packed
 * lower-triangular 64 x 64 tiles in `local_prec` / `coarse_prec` (BF16 local
 * tiles hold the inverse scaled to unit diagonal, see PDG_OPT_BF16_MARGIN).
 *   elem_sub    [n_elem] in 0..n_sub-1 (every subdomain non-empty)
 *   elem_coarse [n_elem] in 0..n_coarse-1, or NULL = the subdomains
 *   coarse_q    0 = one-level (no coarse correction), 1..p otherwise
 * Errors: PDG_EINVAL (labels, sizes, subdomain larger than 6144 dofs, coarse
 *         system of one batch system larger than 16384 dofs),
 * PDG_ENOTSPD (a Cholesky pivot <= 0). */
typedef struct {
    int32_t n_sub;
    const int32_t *elem_sub;
    int32_t n_coarse;
    const int32_t *elem_coarse;
    int32_t coarse_q;
    int32_t local_prec;   /* pdg_precision */
    int32_t coarse_prec;  /* pdg_precision (PDG_F64 or PDG_F32) */
} pdg_precond_desc;

pdg_status pdg_setup_preconditioner(pdg_ctx *ctx, const pdg_precond_desc *desc);

/* Host copy of the FP64 inverse of subdomain `sub`'s matrix as a dense
 * [n_i][n_i] array (dofs in element-label order), and of the coarse operator:
 * P [n_elem][nd][nq0] and K_0 [N0][N0] (N0 = n_coarse * nq0, indexed by the
 * caller's coarse labels; block diagonal over the systems of a batch).  Sizes
 * via pdg_get_precond_sizes. */
pdg_status pdg_get_precond_sizes(const pdg_ctx *ctx, int32_t sub, int64_t *n_i, int64_t *n0,
                                 int32_t *nq0);
pdg_status pdg_get_local_inverse(const pdg_ctx *ctx, int32_t sub, double *out);
pdg_status pdg_get_coarse(const pdg_ctx *ctx, double *P, double *K0);

/* ------------------------------------------------------------------------
 * Device memory: the library needs one workspace of `bytes` bytes (256-byte
 * aligned) holding the matrix, the preconditioner, quadrature data and PCG
 * vectors.  pdg_bind_workspace uploads the setup data into it on the stream.
 * The caller must keep it alive and untouched until pdg_destroy. */
pdg_status pdg_workspace_query(pdg_ctx *ctx, size_t *bytes);
pdg_status pdg_bind_workspace(pdg_ctx *ctx, void *dev_ptr, size_t bytes);

/* Options (after pdg_create). */
typedef enum {
    PDG_OPT_TRUE_RESIDUAL = 1,  /* 1: pdg_solve/pdg_step compute ||b - Kx||/||b|| (one extra SpMV) */
    PDG_OPT_CHUNK = 2,          /* PCG iterations launched between host convergence polls (>= 1) */
    PDG_OPT_KERNEL_TIMING = 3,  /* k >= 1: time one in k Schwarz-apply launches of each solve
                                   with HIP events stamped by the dispatch (1: every launch;
                                   each timed launch adds a few microseconds to its PCG
                                   iteration); 0 (default): off; above 2^20: PDG_EINVAL */
    PDG_OPT_SCHWARZ_ITEM_KB = 4,/* target tile bytes (KiB) per Schwarz work item, 32..8192,
                                   default 128; items are cut further so that a workgroup's
                                   LDS stays within 64 KiB; set before pdg_setup_preconditioner */
    PDG_OPT_GRAPH = 5,          /* 1: replay each chunk of PCG iterations as a captured HIP graph
                                   (captured on first use; not while kernel timing is on);
                                   needs a non-NULL stream in pdg_create (else PDG_EINVAL) */
    PDG_OPT_SPMV_WAVES = 6,     /* wavefronts per SpMV block-row group: 1, 2, 4 (default) or 8 */
    PDG_OPT_PRECONDITIONER = 7, /* 1 (default): two-level additive Schwarz B_ad^{-1} of eq. (5);
                                   0: none (B = I, plain CG), the reference rows of the paper's
                                   Table 1.  pdg_precond_apply then copies r to z. */
    PDG_OPT_LANCZOS_CAP = 8,    /* PCG coefficients (alpha_j, beta_j) kept per system for
                                   pdg_lanczos, 1..2^20 (default 2048; 16 bytes each per
                                   system in the workspace).  Set before pdg_workspace_query /
                                   pdg_bind_workspace. */
    PDG_OPT_ION_EXTRAPOLATION = 9,/* the potential in the explicit ion term of eq. (4):
                                   1 (default): u~ = 2 u^k - u^(k-1), the second-order
                                   extrapolation to t^(k+1) that eq. (4) writes as I^(k+1);
                                   0: u~ = (3 u^k - u^(k-1)) / 2, extrapolated to the
                                   Crank-Nicolson mid-point t^(k+1/2) (stable at larger time
                                   steps, where the extrapolation to t^(k+1) can diverge) */
    PDG_OPT_PRESUM = 10,        /* 0 (default): a dedicated single-block reduction kernel
                                   pre-sums the per-workgroup partials of (p, q), (r, z) and
                                   (r, r) only where the consumers would otherwise read more
                                   than 4M partials per system; 1: always.  Both paths add in
                                   the same order (bitwise-equal results). */
    PDG_OPT_BF16_MARGIN = 11    /* k in 0..40 (default 10), set before pdg_setup_preconditioner.
                                   A BF16 local store keeps K_i^{-1} = D C D with
                                   D = diag(K_i^{-1})^{1/2} in FP32 and C (unit diagonal) in
                                   BF16, but only where the rounded C minus 2^-k I is positive
                                   definite (checked on the host by Cholesky); elsewhere the
                                   subdomain is stored in FP32 (counted in
                                   pdg_solve_info.local_fp32).  k = 0 stores every subdomain
                                   in FP32. */
} pdg_option;
pdg_status pdg_set_option(pdg_ctx *ctx, int32_t option, int64_t value);

/* Kernel timing of the Schwarz-apply kernel (local + coarse tile products)
 * accumulated while PDG_OPT_KERNEL_TIMING is on; reading resets it.
 * Synchronises the stream. */
pdg_status pdg_kernel_timing(pdg_ctx *ctx, int64_t *launches, double *total_ms,
                             double *bytes_per_launch);

/* Autotuner of the work split (the batching form's tile and wavefront
 * assignment; not part of the paper).  Every candidate is timed as whole PCG
 * iterations: the four launches of an iteration back to back, `reps` (1..1000)
 * iterations after two untimed ones, no host synchronisation between launches,
 * on a synthetic system (fixed pseudo-random right-hand side, x0 = 0, tol = 0 so
 * that no system stops while timed), with HIP events on the context's stream.
 * Knobs, one at a time in this order: the Schwarz work-item size (64, 96, 128,
 * 192, 256, 384 KiB of tiles), the split of the coarse-system items (1..4
 * pieces of that size), the wavefronts per SpMV block-row group (1, 2, 4, 8).
 * Each candidate is timed twice (two sweeps) and keeps its faster time; the
 * current value is replaced only by a candidate more than 1 % faster.  The
 * choice changes results only at rounding level: it sets the work split, and
 * with it the order in which Schwarz partials (and, for blocks of up to 32
 * rows, SpMV wavefront partials) are added; runs with the same choice stay
 * bitwise equal.  Overwrites the internal PCG vectors; synchronises.  Call
 * after pdg_bind_workspace, outside a solve.  PDG_EBREAKDOWN if the synthetic
 * solve stopped while timed. */
typedef struct {
    int32_t item_kb;        /* chosen Schwarz work-item size (KiB) */
    int32_t spmv_waves;     /* chosen wavefronts per SpMV group */
    int32_t coarse_split;   /* chosen split of the coarse-system items */
    int32_t candidates;     /* timed runs */
    double iter_us_before;  /* mean PCG iteration time with the settings on entry */
    double iter_us;         /* mean PCG iteration time at the choice */
} pdg_tune_result;
pdg_status pdg_autotune(pdg_ctx *ctx, int32_t reps, pdg_tune_result *out);

/* ------------------------------------------------------------------------
 * 4. Compute calls (device pointers, [n_elem][nd] coefficient vectors).
 */

/* coeff[c][e][:] = L^2 projection of the per-element constant vals[c][e]
 * (vals: [ncomp][n_elem], coeff: [ncomp][n_elem][nd]).  Used for initial data. */
pdg_status pdg_project_p0(pdg_ctx *ctx, const double *vals, int32_t ncomp, double *coeff);

/* y = K x (block-sparse element SpMV). */
pdg_status pdg_spmv(pdg_ctx *ctx, const double *x, double *y);

/* z = B^{-1} r (eq. (5)): all local solves plus the coarse correction. */
pdg_status pdg_precond_apply(pdg_ctx *ctx, const double *r, double *z);

/* pdg_precond_apply for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid it):
 * the same kernels and the same result, bit for bit, but the scratch of the
 * apply (device scalars, coarse restriction shares, update partials, the
 * Schwarz row and column partials) lives in a static device array of 64 MiB
 * per device, set up by pdg_create and held until the process ends; the call
 * itself allocates nothing and clears what it reads before writing it with
 * kernels (no memset).  The scratch needs 512 bytes per stored inverse tile
 * and per Schwarz work item plus small per-chunk terms; a context that needs
 * more than 64 MiB gets PDG_EINVAL and should use pdg_precond_apply.  Every
 * call on a device shares that device's array, which keeps the last call's
 * contents: calls that overlap on one device (other streams, other
 * contexts) race.  r, z: device, [n_elem][nd], caller-owned.  Call after
 * pdg_bind_workspace; enqueue only (no synchronisation). */
pdg_status pdg_precond_apply_noalloc(pdg_ctx *ctx, const double *r, double *z);

/* Ionic update (second line of eq. (4)) and ion term: ions [5][n_elem][nd]
 * Y^k -> Y^(k+1) in place; I[e][i] = int_K f(u~, y^(k+1)) phi_i with the
 * extrapolated potential u~ = 2 u^k - u^(k-1) (or (3 u^k - u^(k-1)) / 2, see
 * PDG_OPT_ION_EXTRAPOLATION).
 * Returns PDG_ENONFINITE (synchronising) if a concentration was <= 0. */
pdg_status pdg_ionic(pdg_ctx *ctx, const double *u, const double *u_prev, double *ions,
                     double *I);

/* b = 2 c M u - K u - chi_m I + f_ext (first line of eq. (4) divided by dt);
 * f_ext may be NULL (= 0). */
pdg_status pdg_rhs(pdg_ctx *ctx, const double *u, const double *I, const double *f_ext,
                   double *b);

/* Solve K x = rhs by PCG with B^{-1} (eq. (5)); x: in = initial guess, out =
 * solution.  Stops when ||r_k|| <= tol ||rhs||.  ||rhs|| = 0 gives x = 0.
 * Synchronises the stream.  PDG_ENOCONV: x holds the last iterate. */
pdg_status pdg_solve(pdg_ctx *ctx, const double *rhs, double *x, double tol, int32_t maxit,
                     pdg_solve_info *info);

/* One time step of eq. (4) in place on caller-owned device buffers:
 * ionic update, ion term, right-hand side, PCG from x0 = U^k;
 * u: U^k -> U^(k+1); u_prev: U^(k-1) -> U^k; ions: Y^k -> Y^(k+1);
 * f_ext nullable.  Synchronises the stream. */
pdg_status pdg_step(pdg_ctx *ctx, double *u, double *u_prev, double *ions, const double *f_ext,
                    double tol, int32_t maxit, pdg_solve_info *info);

/* pdg_step with an offered initial guess (the learned form; not part of the
 * paper): `guess` (device, [n_elem][nd], not aliasing u or u_prev) replaces
 * x0 = U^k for every system where ||b - K guess|| < ||b - K U^k|| (computed
 * on the device after b is built); elsewhere the step falls back to x0 = U^k.
 * The solution meets the same stopping rule either way.  info->guess_used
 * counts the systems that used the guess.  Synchronises the stream. */
pdg_status pdg_step_guess(pdg_ctx *ctx, double *u, double *u_prev, double *ions, const double *f_ext,
                          const double *guess, double tol, int32_t maxit, pdg_solve_info *info);

/* Polynomial extrapolation of the last iterates, a non-learned initial guess:
 * order 1: guess = 2 u - u1; order 2: guess = 3 u - 3 u1 + u2 (device
 * vectors, [n_elem][nd]; u2 may be NULL for order 1). */
pdg_status pdg_guess_extrapolate(pdg_ctx *ctx, const double *u, const double *u1, const double *u2,
                                 int32_t order, double *guess);

/* For a context holding a batch (pdg_set_systems) the info of pdg_solve /
 * pdg_step summarises all systems: the largest iteration count and relative
 * residuals, and bnorm over all systems; the call returns the first non-OK
 * system status.  This returns system `sys`'s own info of the last solve or
 * step, and its status (a pdg_status value) in *status (either may be NULL). */
pdg_status pdg_get_system_info(const pdg_ctx *ctx, int32_t sys, pdg_solve_info *info,
                               int32_t *status);

/* Condition-number estimate of the preconditioned operator from the last
 * solve or step of system `sys` (Section 5: the extreme eigenvalues of the
 * tridiagonal Lanczos matrix built from the PCG coefficients,
 * T_11 = 1/alpha_1, T_jj = 1/alpha_j + beta_(j-1)/alpha_(j-1),
 * T_j,j+1 = sqrt(beta_j)/alpha_j, j = 1..iters).  The coefficients are kept
 * on the device during every solve (up to PDG_OPT_LANCZOS_CAP iterations,
 * default 2048; PDG_EINVAL when the solve took more); the eigenvalues are
 * found on the device by Sturm-count bisection.  kappa = lambda_max /
 * lambda_min; any output may be NULL.  Call right after the solve (PDG_ESTATE
 * otherwise); synchronises the stream. */
pdg_status pdg_lanczos(pdg_ctx *ctx, int32_t sys, double *kappa, double *lambda_min, double *lambda_max);

/* Host copies of those PCG coefficients: alpha[j-1] = alpha_j (j = 1..m) and
 * beta[j-1] = beta_j = (r_j, z_j) / (r_(j-1), z_(j-1)), with
 * m = min(n, iterations of the last solve, PDG_OPT_LANCZOS_CAP); beta_m of the converged
 * iteration is not used by the Lanczos matrix.  Either pointer may be NULL.
 * Call right after the solve (PDG_ESTATE otherwise); synchronises. */
pdg_status pdg_get_pcg_coefficients(pdg_ctx *ctx, int32_t sys, double *alpha, double *beta, int32_t n);

/* pdg_step for n_ctx distinct contexts at once (e.g. one context per
 * polynomial degree of a batch, each on its own stream): every context's
 * chunk of PCG iterations is queued before the host waits on any of them, so
 * the contexts' launches overlap.  u, u_prev, ions: host arrays of n_ctx
 * device pointers; f_ext: NULL or n_ctx device pointers (entries may be NULL);
 * info: NULL or n_ctx entries.  Every context is completed; returns the first
 * non-OK status, with the message in pdg_last_error(ctxs[0]). */
pdg_status pdg_step_batch(pdg_ctx *const *ctxs, int32_t n_ctx, double *const *u,
                          double *const *u_prev, double *const *ions,
                          const double *const *f_ext, double tol, int32_t maxit,
                          pdg_solve_info *info);

/* ------------------------------------------------------------------------
 * 5. Learned initial guess (the learned form; not part of the paper).
 * A per-element multilayer perceptron n_in -> width -> width -> width ->
 * n_out with ReLU between layers predicts, from an element's last four
 * potentials and its ionic state, the element's update U^(k+1) - U^k; the
 * prediction is offered to pdg_step_guess, which falls back to U^k wherever it
 * does not lower the initial residual.  Parameters are FP32 masters with BF16
 * copies; every layer product runs on the matrix cores in BF16 with FP32
 * accumulation, in training (forward, backward, Adam) and in inference.
 *
 * Parameter vector (FP32, n_params entries), per layer l = 1..4 in order:
 * W_l [N_l][K_l] row-major, then b_l [N_l]; (K_l, N_l) = (n_in, width),
 * (width, width), (width, width), (width, n_out).
 *
 * Features of element e (9 nd values, then zeros up to n_in), each group of
 * nd modal coefficients: u^k, u^k - u^(k-1), u^(k-1) - u^(k-2),
 * u^(k-2) - u^(k-3), then the five ionic states y^k; normalised as
 * (value - x_shift[f]) * x_scale[f].  Targets: (U^(k+1) - U^k)[e][i] for
 * i < nd, normalised as (value - t_shift[i]) * t_scale[i]; the loss is the mean
 * of the squared normalised errors over the rows of weight 1 and the first
 * n_out_valid outputs.  Rows (samples) are elements; a batch of rows holds
 * blocks of elements (one block per time step), each padded to a multiple of
 * 32 with rows of weight 0. */
typedef struct pdg_mlp pdg_mlp;
typedef struct {
    int32_t n_in;         /* multiple of 32, >= 9 nd */
    int32_t width;        /* multiple of 32 */
    int32_t n_out;        /* multiple of 32 */
    int32_t n_out_valid;  /* outputs that carry targets (nd), 1..n_out */
    int64_t max_rows;     /* rows per batch, multiple of 32 */
} pdg_mlp_desc;

/* Create on HIP device `hip_device`, launching on `hip_stream` (NULL = default
 * stream).  Errors: PDG_EINVAL for sizes outside the stated ranges. */
pdg_status pdg_mlp_create(pdg_mlp **out, int32_t hip_device, void *hip_stream, const pdg_mlp_desc *desc);
void pdg_mlp_destroy(pdg_mlp *mlp);
const char *pdg_mlp_last_error(const pdg_mlp *mlp);
/* n_params, and the bytes of the workspace to bind (256-byte aligned, owned by
 * the caller, kept alive until pdg_mlp_destroy). */
pdg_status pdg_mlp_get_sizes(pdg_mlp *mlp, int64_t *n_params, size_t *workspace_bytes);
pdg_status pdg_mlp_bind_workspace(pdg_mlp *mlp, void *dev_ptr, size_t bytes);
/* Host parameter vector in / out (n = n_params).  Setting resets Adam. */
pdg_status pdg_mlp_set_params(pdg_mlp *mlp, const float *params, int64_t n);
pdg_status pdg_mlp_get_params(pdg_mlp *mlp, float *params, int64_t n);
/* Normalisation (host arrays: n_in feature shifts and scales, n_out target
 * shifts and scales; scales > 0). */
pdg_status pdg_mlp_set_normalisation(pdg_mlp *mlp, const float *x_shift, const float *x_scale,
                                     const float *t_shift, const float *t_scale);
/* A batch from the host: X [rows][n_in] BF16 bit patterns (already
 * normalised), T [rows][n_out] and row weights w [rows] (FP32). */
pdg_status pdg_mlp_set_batch(pdg_mlp *mlp, int64_t rows, const uint16_t *X, const float *T,
                             const float *w);
/* Features of n_elem elements (device vectors [n_elem][nd]: u0 = u^k,
 * u1 = u^(k-1), u2, u3; ions [5][n_elem][nd]) into batch rows
 * row0 .. row0 + n_rows (rows past n_elem are zero).  With raw != NULL the
 * unnormalised values go to raw (device, [n_elem][n_in] FP32) instead. */
pdg_status pdg_mlp_features(pdg_mlp *mlp, int64_t row0, int64_t n_elem, int64_t n_rows, int32_t nd,
                            const double *u0, const double *u1, const double *u2, const double *u3,
                            const double *ions, float *raw);
/* Targets from u_next = U^(k+1) and u0 = U^k into rows row0 .. row0 + n_rows
 * (weights 1 for the n_elem element rows, 0 for padding); raw: device
 * [n_elem][nd] FP32 unnormalised values instead. */
pdg_status pdg_mlp_targets(pdg_mlp *mlp, int64_t row0, int64_t n_elem, int64_t n_rows, int32_t nd,
                           const double *u_next, const double *u0, float *raw);
/* Forward pass over batch rows 0 .. rows (multiple of 32); y_out (device,
 * [rows][n_out] FP32, normalised units) may be NULL. */
pdg_status pdg_mlp_forward(pdg_mlp *mlp, int64_t rows, float *y_out);
/* guess[e][i] = u0[e][i] + de-normalised prediction of batch row row0 + e
 * (after pdg_mlp_forward). */
pdg_status pdg_mlp_guess(pdg_mlp *mlp, int64_t row0, int64_t n_elem, int32_t nd, const double *u0,
                         double *guess);
/* Forward and backward over batch rows 0 .. rows; n_valid = rows of weight 1
 * (the loss divides by n_valid * n_out_valid).  grad: host [n_params] or NULL;
 * loss: host or NULL.  Synchronises. */
pdg_status pdg_mlp_gradients(pdg_mlp *mlp, int64_t rows, int64_t n_valid, float *grad, double *loss);
/* One Adam step (bias-corrected) on those gradients.  loss: host or NULL (no
 * synchronisation when NULL). */
pdg_status pdg_mlp_train_step(pdg_mlp *mlp, int64_t rows, int64_t n_valid, float lr, float beta1,
                              float beta2, float eps, double *loss);

#ifdef __cplusplus
}
#endif

#endif /* PDG_H */
