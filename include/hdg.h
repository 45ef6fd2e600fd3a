/*
 * hdg.h - C ABI of the MI355X hot path of one implicit hybridized-DG Newton step
 * for the 2-D compressible Euler and Navier-Stokes equations
 * (Woopen, Balan, May, Schuetz, arXiv:1308.3995).
 *
 * The Newton system of Sec. 3.3 (eq. linearsystem) is split as in Sec. 3.4
 * (eq. ls, cons, hybridsystem): element-local unknowns U_K (Navier-Stokes: the
 * gradient q then w; Euler: w) and skeleton unknowns Lambda on interior faces.
 * Per element K the library assembles the Jacobian blocks
 *     A_K = dR_K/dU_K,  B_K = dR_K/dLambda,  C_K = dR_lam,K/dU_K,  D_K = dR_lam,K/dLambda
 * and right-hand sides r_K = -R_K, r_lam,K = -R_lam,K, condenses them to
 *     S_K = D_K - C_K A_K^-1 B_K,   g_K = r_lam,K - C_K A_K^-1 r_K,
 * sums S_K and g_K into the skeleton system K dLambda = E, solves it with
 * block-Jacobi preconditioned restarted GMRES, and reconstructs
 *     dU_K = A_K^-1 (r_K - B_K dLambda_K).
 * Around that step: optional shock capturing and pseudo-time terms in the element blocks
 * (hdg_params), the relaxed Newton iteration with its CFL schedule (Sec. 3.3), the
 * hybridized adjoint with element indicators and the marking decisions of Sec. 4.
 *
 * Conventions shared by every call:
 *   - Pointers named *_dev are device pointers owned by the caller; the library
 *     never frees them. Pointers named *_host are host pointers read during
 *     the call only.
 *   - Calls that take a hipStream_t are stream-ordered; their outputs are valid
 *     once that stream has synchronised. Calls that return host scalars
 *     (iterations, residuals) synchronise the stream themselves.
 *   - Inputs are never modified; outputs are overwritten, never accumulated.
 *   - No C++ exception crosses this interface. On failure a call returns a
 *     status other than HDG_OK and hdg_last_error() describes it.
 *   - Mesh: counter-clockwise triangles; local face i of a triangle is the edge
 *     (v_i, v_(i+1) mod 3); every boundary edge is a far-field boundary.
 *   - Interior faces are numbered in canonical order: sorted by (lower vertex id,
 *     higher vertex id). Face f carries 4 (p_f + 1) skeleton unknowns with
 *     p_f = max of its two neighbours' degrees (Sec. 3.1), ordered field-major
 *     (a (p_f + 1) + k, a in rho, rho u, rho v, E; k the Legendre mode), and
 *     skeleton vectors concatenate the faces in canonical order.
 *   - State arrays are padded to NP = (pmax+1)(pmax+2)/2 modes per field, pmax the
 *     largest element degree of the plan:
 *         w[e][a][i]         e < n_elements, a < 4,  i < NP   (float64)
 *         q[e][4 d + a][i]   Navier-Stokes gradient unknowns, d < 2
 *     Modes beyond an element's own degree are ignored on input and written as 0.
 */
#ifndef HDG_H
#define HDG_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HDG_OK = 0,
    HDG_ERR_INVALID_ARG = 1,     /* bad pointer, size, degree or mesh */
    HDG_ERR_OOM = 2,             /* device allocation failed */
    HDG_ERR_SINGULAR_LOCAL = 3,  /* zero pivot in a local or face-diagonal block, or a degenerate triangle */
    HDG_ERR_NONFINITE = 4,       /* a non-finite value in the state or the assembled blocks */
    HDG_ERR_NOT_CONVERGED = 5,   /* GMRES stopped at max_iter above rtol; the best iterate is returned */
    HDG_ERR_HIP = 6              /* a HIP runtime call failed */
} hdg_status;

typedef enum { HDG_EULER = 0, HDG_NS = 1 } hdg_physics;

/* HDG_FP64: every step in float64.
 * HDG_MIXED: the skeleton solve runs its inner GMRES on a float32 copy of the
 *            preconditioned skeleton matrix, wrapped in float64 iterative
 *            refinement on the float64 skeleton matrix (residuals, Krylov
 *            vectors and orthogonalisation stay float64); the condensation is float64.
 * HDG_MIXED_CONDENSE: as HDG_MIXED, and the condensation of Euler elements of degree <= 4
 *            eliminates [A_K | B_K | r_K] in float32 (the blocks are assembled in float64),
 *            refines y_K in float64 (the float64 residual r_K - A_K y_K through the recorded
 *            float32 elimination, two sweeps) and forms g_K from it; X_K and S_K keep
 *            float32 accuracy, so the skeleton matrix is that of the float32 local solves.
 *            Navier-Stokes plans refuse it (HDG_ERR_INVALID_ARG); degree-5 elements are
 *            condensed in float64. */
typedef enum { HDG_FP64 = 0, HDG_MIXED = 1, HDG_MIXED_CONDENSE = 2 } hdg_precision;

typedef struct {
    int32_t physics;      /* hdg_physics */
    int32_t precision;    /* hdg_precision */
    double gamma;         /* ratio of specific heats (Sec. 2.1) */
    double mach;          /* free-stream Mach number; rho_inf = 1, p_inf = 1/gamma */
    double aoa_rad;       /* angle of attack of the free stream */
    double reynolds;      /* Navier-Stokes: mu = rho_inf |v_inf| / Re (constant viscosity) */
    double prandtl;       /* Navier-Stokes: heat flux (mu gamma / Pr) grad e */
    double stab_alpha;    /* trace-flux constant alpha (Sec. 3.2); <= 0 selects |v_inf| + c_inf */
    double cfl;           /* pseudo-time step (Sec. 3.3): A_K gains the element mass matrix over
                             dt_K = cfl |K| / (lambda_c + 4 lambda_v) on its conserved-variable
                             block, lambda_c = sum_e (|v.n| + c)|e| and lambda_v = (mu gamma /
                             (rho Pr)) sum_e |e|^2 / |K| at the element-mean state; the right-hand
                             side is unchanged. 0 = pure Newton; must be >= 0. */
    double sc_eps0;       /* shock capturing (Sec. 3.2): the volume term
                             (grad phi, eps_K grad w_h) with eps_K = sc_eps0 (h_K / p_K)^(2 - sc_beta)
                             / |K| int_K sum_i |(div f_c(w_h))_i|, h_K the longest edge; eps_K is
                             held fixed in the Newton matrix. 0 = off (the paper: 0.2); >= 0.
                             Navier-Stokes takes the viscous form: q_h in place of grad w_h, in the
                             term and in the strong residual. */
    double sc_beta;       /* shock-capturing exponent beta (the paper: 0) */
} hdg_params;

typedef struct {
    int64_t n_elements;
    int64_t n_faces;           /* interior faces */
    int64_t n_boundary_faces;
    int64_t n_skel_dof;        /* length of skeleton vectors */
    int64_t np_max;            /* NP, modes per field in the padded state arrays */
    int64_t n_fields;          /* 4 (Euler) or 12 (Navier-Stokes: 8 gradient + 4 conserved) */
    int64_t bsr_blocks;        /* stored blocks of the skeleton matrix */
    int64_t bsr_values;        /* float64 values of the skeleton matrix */
    int64_t local_store_bytes; /* bytes of the element local-solution store (X_K, y_K) */
    int64_t workspace_bytes;   /* bytes of scratch needed by every call below */
    int64_t n_buckets;         /* (degree, face-degree) element buckets */
} hdg_sizes;

typedef struct hdg_plan hdg_plan;

/* Build the plan of a mesh (Sec. 3.1): faces, face degrees p_f = max(p_K-, p_K+),
 * skeleton offsets, the block pattern of the skeleton matrix (one diagonal and up to
 * four off-diagonal blocks per face row, Sec. 3.4), element geometry, degree buckets,
 * basis and quadrature tables, and far-field projectors. Host inputs:
 *   xy_host[nv][2] vertex coordinates, tri_host[ne][3] vertex ids (counter-clockwise),
 *   degree_host[ne] element degrees in 1..5.
 * Allocates device memory on `device`. The mesh data of a plan never change. A plan may be
 * shared by several streams and host threads: its caches (the kernel variants the first
 * assembly picks by timing, the launch graphs captured per set of buffers) are guarded by a
 * lock, and calls whose buffers (outputs and workspace) differ may run concurrently; calls
 * that share a buffer race. Plan-level settings (hdg_set_cfl, hdg_set_poly_degree,
 * hdg_set_kernel_timing) apply to every later call and are not meant to change while other
 * calls on the plan are in flight. Errors:
 * HDG_ERR_INVALID_ARG (bad sizes, ids, degrees,
 * an edge shared by more than two triangles), HDG_ERR_SINGULAR_LOCAL (a triangle of
 * non-positive area), HDG_ERR_OOM, HDG_ERR_HIP. */
hdg_status hdg_plan_create(hdg_plan** out, const double* xy_host, int32_t nv,
                           const int32_t* tri_host, int32_t ne, const int8_t* degree_host,
                           const hdg_params* prm, int device);

/* Sizes of every buffer the caller allocates. */
hdg_status hdg_plan_sizes(const hdg_plan* plan, hdg_sizes* out);

/* Face tables (host outputs, any may be NULL): face_vertices_host[n_faces][2] (sorted
 * vertex pair), face_offset_host[n_faces + 1] (skeleton offsets), face_degree_host[n_faces]. */
hdg_status hdg_plan_faces(const hdg_plan* plan, int32_t* face_vertices_host,
                          int64_t* face_offset_host, int32_t* face_degree_host);

/* Block pattern of the skeleton matrix (host outputs, any may be NULL):
 * row_ptr_host[n_faces + 1], col_host[bsr_blocks] (face index of each block),
 * val_off_host[bsr_blocks] (offset of each block in bsr_values). Block (f, f2) is
 * 4(p_f+1) x 4(p_f2+1), stored column-major; the diagonal block is first in its row. */
hdg_status hdg_plan_pattern(const hdg_plan* plan, int64_t* row_ptr_host, int32_t* col_host,
                            int64_t* val_off_host);

/* Assemble and condense (Sec. 3.2 eq. hdg_ls1..hdg_cont, Sec. 3.3 eq. linearsystem,
 * Sec. 3.4 eq. hybridsystem). For every element: quadrature assembly of r_K, A_K,
 * B_K, C_K, D_K in float64 with the trace flux f(lam).n - alpha (lam - w) and the
 * far-field boundary state, local solves X_K = A_K^-1 B_K and y_K = A_K^-1 r_K by
 * elimination with partial pivoting, S_K and g_K, then the sum into the skeleton matrix.
 * Inputs: w_dev, q_dev (Navier-Stokes only, else NULL) in the padded state layout,
 *         lam_dev[n_skel_dof] the current skeleton state.
 * Outputs: bsr_values_dev[bsr_values] the skeleton matrix K (float64, pattern above),
 *          rhs_dev[n_skel_dof] the right-hand side E,
 *          local_store_dev[local_store_bytes] X_K and y_K for hdg_back_substitute.
 * workspace_dev: workspace_bytes of scratch. elem_status_dev (optional, int32[ne]):
 * per element 0, or HDG_ERR_SINGULAR_LOCAL / HDG_ERR_NONFINITE. res_norm_host
 * (optional): if non-NULL the call synchronises and returns ||E||_2. The call itself
 * returns HDG_ERR_SINGULAR_LOCAL or HDG_ERR_NONFINITE only when res_norm_host or
 * elem_status_dev asks it to look (that needs a synchronisation).
 * Batching: one launch per (element degree, face degree) bucket; the Euler buckets run
 * concurrently on the plan's side streams, forked from `stream` and joined back into it
 * before the call's later work (the plan creates them at its first condensation). Euler
 * buckets have four kernel variants (blocked Gauss-Jordan on the matrix cores or the
 * register-resident one, each at a 128- and a 256-VGPR budget; with shock capturing on as
 * well). The first call on a plan times the variants of every
 * bucket shape the process has not met yet, keeps the fastest, runs it and synchronises the
 * stream once; the choice is kept per (physics, degree, face degree, precision, shock
 * capturing, element-count class) for every later plan of the process, so plans agree bit for
 * bit (the variants agree only up to rounding). Later calls capture the whole launch sequence
 * in a hipGraph once per set of buffer pointers and replay it; they are asynchronous unless
 * res_norm_host or elem_status_dev is given.
 * Call once outside any stream capture of the caller's own before capturing it. */
hdg_status hdg_assemble_condense(hdg_plan* plan, const double* w_dev, const double* q_dev,
                                 const double* lam_dev, double* bsr_values_dev, double* rhs_dev,
                                 void* local_store_dev, void* workspace_dev,
                                 int32_t* elem_status_dev, double* res_norm_host,
                                 hipStream_t stream);

/* Condensation of several independent cases at once (Sec. 3.4: the static condensation is
 * element by element, so the elements of different cases can share launches; for serving).
 * Equivalent to hdg_assemble_condense(plans[i], w_dev[i], q_dev ? q_dev[i] : NULL, lam_dev[i],
 * bsr_values_dev[i], rhs_dev[i], local_store_dev[i], workspace_dev[i], NULL, NULL, stream) for
 * every i < n, with bit-identical outputs. Plans whose kernel variants are already picked (any
 * earlier condensation in the process with the same bucket shapes) that are Euler, without shock
 * capturing and with float64 condensation are condensed together: one launch per (element
 * degree, face degree, kernel variant) over the elements of up to 8 plans, then each plan's face
 * sums. The other plans (Navier-Stokes, HDG_MIXED_CONDENSE, shock capturing, a first call) are
 * condensed one by one within the call. All work is ordered on `stream` (the launches run
 * concurrently on the first joined plan's side streams, forked from and joined back into
 * `stream`); nothing is captured in a graph. The plans must be distinct and live on one device; their buffers must not overlap.
 * Arrays have n entries (q_dev may be NULL for Euler plans). batched_out (optional): the number of
 * plans condensed together. Errors: HDG_ERR_INVALID_ARG for n < 0, null arrays or entries, a
 * repeated plan or plans on different devices; otherwise as hdg_assemble_condense. */
hdg_status hdg_assemble_condense_batch(int32_t n, hdg_plan* const* plans, const double* const* w_dev,
                                       const double* const* q_dev, const double* const* lam_dev,
                                       double* const* bsr_values_dev, double* const* rhs_dev,
                                       void* const* local_store_dev, void* const* workspace_dev,
                                       int32_t* batched_out, hipStream_t stream);

/* Skeleton solve K dLambda = E (Sec. 3.4 eq. hybridsystem): restarted GMRES(restart)
 * with right block-Jacobi preconditioning on the face-diagonal blocks and classical
 * Gram-Schmidt (a second pass when the first one cancels), all in float64 (HDG_MIXED: inner
 * solves on a float32 preconditioned matrix inside float64 iterative refinement).
 * With a polynomial degree d >= 2 (hdg_set_poly_degree, default 30) the first restart cycle
 * has d steps; the harmonic Ritz values of its Hessenberg matrix are the roots of a GMRES
 * residual polynomial 1 - Khat p(Khat) of degree d (Khat = K M^-1, M the block-Jacobi
 * matrix), and the later cycles run GMRES on Khat p(Khat) (a flexible update keeps
 * p(Khat) v_j), d matrix applications per Arnoldi step. If the roots are unusable (a cycle
 * converged or broke down first, a root at zero) the solve continues as plain GMRES.
 * Stops when ||E - K dLambda||_2 <= rtol ||E||_2 or after max_iter applications of the
 * preconditioned matrix. Outputs dlambda_dev[n_skel_dof]; iters_out (those applications)
 * and relres_out (true relative residual, recomputed in float64) may be NULL. Returns
 * HDG_ERR_NOT_CONVERGED with the best iterate when max_iter is reached,
 * HDG_ERR_SINGULAR_LOCAL when a face-diagonal block is singular, HDG_ERR_NONFINITE when
 * the right-hand side or the final residual is not finite. Synchronises. */
hdg_status hdg_skeleton_solve(hdg_plan* plan, const double* bsr_values_dev, const double* rhs_dev,
                              double* dlambda_dev, double rtol, int32_t restart, int32_t max_iter,
                              void* workspace_dev, hipStream_t stream, int32_t* iters_out,
                              double* relres_out);

/* Back-substitution (Sec. 3.4): dU_K = y_K - X_K dLambda_K from the stored local
 * solutions. Outputs dw_dev in the padded w layout and, for Navier-Stokes, dq_dev in
 * the padded q layout (NULL for Euler). */
hdg_status hdg_back_substitute(hdg_plan* plan, const void* local_store_dev,
                               const double* dlambda_dev, double* dw_dev, double* dq_dev,
                               void* workspace_dev, hipStream_t stream);

/* Pseudo-time CFL number used by later hdg_assemble_condense calls on this plan (the local
 * step of hdg_params.cfl, Sec. 3.3). 0 or +inf: pure Newton. A captured launch sequence
 * is re-captured on the next call. Errors: HDG_ERR_INVALID_ARG for a negative or NaN cfl. */
hdg_status hdg_set_cfl(hdg_plan* plan, double cfl);

/* ||N_h(x)||_2 at the state passed to the last hdg_assemble_condense that used workspace_dev
 * (Sec. 3.3, the norm the CFL schedule reads): over every element row (Navier-Stokes: the
 * gradient and the conserved-variable rows) and every skeleton row, the latter summed over
 * both neighbours. The condensation kernels leave the partials in the workspace; this call
 * reduces them on the device in a fixed order (repeated calls return the same bits).
 * res_norm_dev (optional, one float64 on the device) receives it stream-ordered;
 * res_norm_host (optional) makes the call synchronise and receives it. */
hdg_status hdg_residual_norm(hdg_plan* plan, void* workspace_dev, double* res_norm_dev, double* res_norm_host,
                             hipStream_t stream);

/* Newton update x <- x + dx (Sec. 3.3): w_dev += dw_dev, q_dev += dq_dev (Navier-Stokes;
 * both NULL for Euler), lam_dev += dlambda_dev, in the layouts above. The one call that
 * modifies its state arguments in place. */
hdg_status hdg_apply_update(hdg_plan* plan, double* w_dev, double* q_dev, double* lam_dev, const double* dw_dev,
                            const double* dq_dev, const double* dlambda_dev, hipStream_t stream);

/* The CFL schedule of Sec. 3.3 (eq. cfl), host arithmetic, iterations counted from n = 1:
 *   n <= n0:  c0 (3 s^2 - 2 s^3), s = n / n0   (a smooth ramp to c0)
 *   n >  n0:  cfl_prev (1 + c1 max(0, log(res_prev / res)))
 * res_prev, res: ||N_h|| at the previous and the current iterate. A zero res returns +inf
 * (the residual vanished: pure Newton). The paper's values: c0 = 1e6, c1 = 1e3, n0 = 4. */
double hdg_cfl_schedule(int32_t n, double cfl_prev, double res_prev, double res, double c0, double c1,
                        int32_t n0);

typedef struct {
    double c0;              /* eq. cfl ramp height (the paper: 1e6) */
    double c1;              /* eq. cfl growth factor (the paper: 1e3) */
    int32_t n0;             /* eq. cfl ramp length (the paper: 4) */
    int32_t max_steps;      /* Newton iterations at most */
    double rel_tol;         /* stop once ||N_h|| <= max(abs_tol, rel_tol ||N_h(x_1)||) */
    double abs_tol;
    double gmres_rtol;      /* hdg_skeleton_solve arguments of every iteration */
    int32_t restart;
    int32_t max_iter;
} hdg_newton_opts;

typedef struct {
    int32_t steps;               /* Newton iterations taken */
    int32_t converged;           /* 1 if the tolerance was met */
    int64_t gmres_iters;         /* inner GMRES iterations summed over the iterations */
    int32_t gmres_not_converged; /* iterations whose skeleton solve stopped at max_iter (their
                                    best iterate was used: an inexact Newton step) */
    double res0;                 /* ||N_h|| at the initial state */
    double res;                  /* ||N_h|| at the returned state */
} hdg_newton_report;

/* The relaxed Newton iteration of Sec. 3.3 on the device: at iterate x_n it assembles and
 * condenses with the local pseudo-time step of CFL_n (hdg_cfl_schedule, which reads
 * ||N_h(x_n)||), solves the skeleton system, back-substitutes and applies x_(n+1) = x_n + dx,
 * until ||N_h|| meets the tolerance or max_steps iterations are done. When CFL_n depends
 * on ||N_h(x_n)|| (n > n0) the state is assembled twice (the residual does not depend on
 * the CFL, the matrix does), unless the CFL is unchanged. w_dev, q_dev (Navier-Stokes, else
 * NULL) and lam_dev are updated in place; bsr_values_dev, rhs_dev, local_store_dev,
 * dlambda_dev, dw_dev, dq_dev and workspace_dev are caller-owned scratch of the sizes of
 * hdg_plan_sizes. report (optional) receives the summary; res_history_host (optional,
 * max_steps + 1 doubles) the residual norms at x_1, x_2, ..., cfl_history_host (optional,
 * max_steps doubles) CFL_1, CFL_2, ... (entries past report->steps are left alone). The
 * plan's CFL is left at the last value used. Synchronises. Errors: those of the calls it
 * makes, except HDG_ERR_NOT_CONVERGED from a skeleton solve (counted in the report). */
hdg_status hdg_pseudo_transient_solve(hdg_plan* plan, double* w_dev, double* q_dev, double* lam_dev,
                                      double* bsr_values_dev, double* rhs_dev, void* local_store_dev,
                                      double* dlambda_dev, double* dw_dev, double* dq_dev, void* workspace_dev,
                                      const hdg_newton_opts* opts, hdg_newton_report* report,
                                      double* res_history_host, double* cfl_history_host, hipStream_t stream);

/* Hybridized adjoint (Sec. 4, eq. adjoint; Sec. 4.1). For a target functional J with
 * derivative F~ = J'(x) in the element unknowns (the functional depends on w and q only, so
 * its skeleton part is zero), the adjoint system [A_K B_K; C_K D_K]^T [U~; Lambda~] = [F~; 0]
 * condenses, with the blocks of hdg_assemble_condense, to
 *     K^T Lambda~ = E~,   E~ = -sum_K X_K^T F~_K,   U~_K = A_K^-T (F~_K - C_K^T Lambda~_K).
 * The paper solves it in the space of degree p + 1; a plan built with every degree raised by
 * one, on the primal state padded with zero modes, is that space.
 *
 * K^T in the block pattern of K (the pattern is symmetric): kt_values_dev[bsr_values] from
 * bsr_values_dev. Solve K^T Lambda~ = E~ by passing kt_values_dev to hdg_skeleton_solve. */
hdg_status hdg_skeleton_transpose(hdg_plan* plan, const double* bsr_values_dev, double* kt_values_dev,
                                  hipStream_t stream);

/* E~ = -sum_K X_K^T F~_K from the local store of the last hdg_assemble_condense:
 * fw_dev (the w part of F~, padded w layout) and, for Navier-Stokes, fq_dev (the q part,
 * padded q layout; NULL for Euler) -> etilde_dev[n_skel_dof]. Uses workspace_dev as scratch
 * (the per-face slots of the condensed right-hand side). */
hdg_status hdg_adjoint_rhs(hdg_plan* plan, const void* local_store_dev, const double* fw_dev, const double* fq_dev,
                           double* etilde_dev, void* workspace_dev, hipStream_t stream);

/* Local adjoint solves U~_K = A_K^-T (F~_K - C_K^T Lambda~_K) at the state (w_dev, q_dev,
 * lam_dev) (A_K is assembled again, with the plan's CFL, and eliminated transposed with
 * partial pivoting), written to wt_dev (padded w layout) and, for Navier-Stokes, qt_dev
 * (padded q layout), and the element indicators of Sec. 4 with the skeleton adjoint dropped,
 * eta_dev[ne] = |U~_K . R_K(x)| (R_K the element's residual rows, gradient rows included).
 * q_dev, fq_dev (the q part of F~) and qt_dev are Navier-Stokes only (NULL for Euler).
 * Navier-Stokes allocates a temporary device buffer for the uncondensed blocks of a chunk of
 * elements (at most 1 GiB) and synchronises. elem_status_dev (optional, int32[ne]) as in
 * hdg_assemble_condense; when given the call synchronises and returns the first failure. */
hdg_status hdg_adjoint_local(hdg_plan* plan, const double* w_dev, const double* q_dev, const double* lam_dev,
                             const double* fw_dev, const double* fq_dev, const double* lamt_dev, double* wt_dev,
                             double* qt_dev, double* eta_dev, void* workspace_dev, int32_t* elem_status_dev,
                             hipStream_t stream);

/* Adaptation decisions of Sec. 4. Marking: the smallest set M of elements with
 * eta_M >= (1 - theta) eta_T, where eta_M^2 = sum_{K in M} eta_K^2 (Doerfler): the elements
 * in order of decreasing eta_K (ties by increasing element id) up to the first whose partial
 * sum of eta_K^2 reaches (1 - theta)^2 eta_T^2. Smoothness sensor:
 * S_K = (w - w*, w - w*)_K / (w, w)_K, w* the projection of w onto degree p_K - 1 (the inner
 * product sums the four conserved fields; with the hierarchical orthonormal basis this is
 * the energy of the degree-p_K modes over the total). Inputs: w_dev (padded w layout),
 * eta_dev[ne] (e.g. from hdg_adjoint_local), theta in [0, 1] (the paper: 0.05), eps_s >= 0
 * (the paper: 1e-6). Outputs: flag_dev[ne] int32, 0 unmarked, 1 marked for p-enrichment
 * (S_K < eps_s), 2 marked for mesh refinement; sensor_dev[ne] (optional) S_K;
 * n_marked_host (optional) the size of M, which makes the call synchronise. */
hdg_status hdg_mark_elements(hdg_plan* plan, const double* w_dev, const double* eta_dev, double theta, double eps_s,
                             int32_t* flag_dev, double* sensor_dev, int32_t* n_marked_host, void* workspace_dev,
                             hipStream_t stream);

/* hdg_mark_elements without a workspace, for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid allocation): the same
 * kernels and results, with the count, the sort buffers, the radix-sort scratch and (when
 * sensor_dev is NULL) the sensor in a static device array of 16 MiB that each GPU the library
 * runs on holds until the process ends; the call allocates nothing. That bounds the mesh:
 * 256 + 8 ne (no sensor_dev) + 24 ne + the radix sort's scratch bytes must fit, about 400k
 * elements; larger meshes get HDG_ERR_INVALID_ARG. Every call on one GPU shares the array:
 * calls that overlap on the same GPU (several streams or threads) race and must be serialised
 * by the caller. Other arguments and errors as hdg_mark_elements. */
hdg_status hdg_mark_elements_noalloc(hdg_plan* plan, const double* w_dev, const double* eta_dev, double theta,
                                     double eps_s, int32_t* flag_dev, double* sensor_dev, int32_t* n_marked_host,
                                     hipStream_t stream);

/* Inspection entry for tests: the uncondensed element blocks of one element in the
 * unknown order documented above (element: Navier-Stokes gradient fields 4d+a first,
 * then w fields, each mode-minor; faces: interior local faces in order, each
 * field-major), computed by the same device code as hdg_assemble_condense.
 * Host outputs, each column-major: A_host[n*n], B_host[n*f], C_host[f*n], D_host[f*f],
 * r_host[n], rl_host[f]; n_out and f_out receive n and f. Synchronises. */
hdg_status hdg_debug_element_blocks(hdg_plan* plan, int64_t element, const double* w_dev,
                                    const double* q_dev, const double* lam_dev,
                                    double* A_host, double* B_host, double* C_host, double* D_host,
                                    double* r_host, double* rl_host, int32_t* n_out, int32_t* f_out);

/* Inspection entry for tests: X_K (n x f, column-major) and y_K of one element read
 * back from a local store written by hdg_assemble_condense. Synchronises. */
hdg_status hdg_debug_local_solution(hdg_plan* plan, const void* local_store_dev, int64_t element,
                                    double* X_host, double* y_host, int32_t* n_out, int32_t* f_out);

/* Inspection entry for tests: the float64 Euler condensation of this plan runs kernel variant
 * `variant` on every bucket (Sec. 3.4, eq. hybridsystem, the same condensed system up to
 * rounding): 0 / 1 the register-resident elimination at a 128- / 256-VGPR budget, 2 / 3 the
 * blocked matrix-core elimination at 128 / 256; -1 returns to the timed choice (the
 * process-wide one, see hdg_assemble_condense). A plan with a forced variant is condensed on
 * its own by hdg_assemble_condense_batch. No effect on Navier-Stokes plans or on the buckets
 * the mixed-precision condensation covers. Host only; takes effect at the next condensation.
 * Errors: HDG_ERR_INVALID_ARG (null plan, variant outside -1..3). */
hdg_status hdg_debug_condense_variant(hdg_plan* plan, int32_t variant);

/* Degree d of the GMRES polynomial preconditioner of hdg_skeleton_solve on this plan
 * (0 or 1: plain block-Jacobi GMRES; at most 32; default 30) and, for HDG_MIXED, the storage
 * of the preconditioned matrix its products read: fp16_matrix = 1 (default) a float16 copy,
 * 0 the float32 copy of the inner solve. The polynomial is only a preconditioner (the outer
 * Arnoldi products and the float64 refinement residual are unchanged), so its storage changes
 * the iteration count, not the gate. HDG_FP64 always uses the float64 matrix. Errors:
 * HDG_ERR_INVALID_ARG. */
hdg_status hdg_set_poly_degree(hdg_plan* plan, int32_t degree, int32_t fp16_matrix);

/* Profiling hook for benchmarks: when enabled, hdg_skeleton_solve launches its restart cycles
 * directly (not from captured graphs) and brackets each of its SpMV launches with a pair of
 * HIP events on the caller's stream, accumulating per kernel the launch count, the summed
 * event time and the algorithmic bytes of those launches. kernel 0: the polynomial
 * preconditioner's SpMV (matrix values, the source, the previous iterate for the second
 * factor of a complex pair, the output vector and the running p(Khat) v_j); kernel 1: the
 * SpMV fused with the first Gram-Schmidt dot products (matrix values, source, output, and the
 * basis vectors the dot products read; plain GMRES also writes the new basis vector).
 * hdg_kernel_timing returns kernel `kernel`'s totals and, if reset != 0, clears them. */
hdg_status hdg_set_kernel_timing(hdg_plan* plan, int32_t enable);
hdg_status hdg_kernel_timing(hdg_plan* plan, int32_t kernel, int64_t* launches, double* total_ms,
                             double* total_bytes, int32_t reset);

/* Inspection entry for tests, host only (no device work): the eigenvalues wr + i wi of a real
 * upper Hessenberg matrix h_host[n][n] (row-major; entries below the subdiagonal are
 * ignored), by the implicit double-shift QR iteration the polynomial preconditioner uses for
 * its roots. Complex eigenvalues come in conjugate pairs, +imaginary part first. Errors:
 * HDG_ERR_INVALID_ARG (n outside 1..64, null pointer), HDG_ERR_NOT_CONVERGED. */
hdg_status hdg_debug_hessenberg_eigenvalues(int32_t n, const double* h_host, double* wr_host,
                                            double* wi_host);

/* Thread-local description of the last error of the calling thread. */
const char* hdg_last_error(void);

void hdg_plan_destroy(hdg_plan* plan);

#ifdef __cplusplus
}
#endif
#endif /* HDG_H */
