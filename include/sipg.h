/*
 * sipg.h -- C ABI of the MI355X (gfx950) library for the matrix-free SIPG
 * operators of Schussnig, Fehn, Pacheco and Kronbichler, "Higher-Order
 * Discontinuous Galerkin Splitting Schemes for Fluids with Variable Viscosity"
 * (arXiv 2506.14424).
 *
 * Operators (Sec. 4.1):
 *   viscous  a(v,u) = (alpha v, u) + v_h^e(v, u; mu): the viscous-step operator
 *            (gamma_0/dt) M - div(2 mu eps(u)), SIPG fluxes u = {{u}},
 *            tau_1 = {{mu grad u}} - tau [[u]], tau_2 = tau_1^T ("Viscous Step");
 *   poisson  the SIPG Laplacian of the pressure step ("Pressure Step"), with
 *            the coercive penalty sign and an optional mass term alpha;
 *   penalty  the operator of the penalty step (Sec. 4.3, "Consistent
 *            Stabilization", eq. penalty_step): (alpha v, u) +
 *            (div v, tau_div^e div u)_e + (v.n, tau_cont [[u]].n) on faces, with
 *            per-cell factors given by the caller, the face factor the mean of
 *            the two cells' tau_cont, and the oriented jump u - g on Dirichlet
 *            faces (no mirror doubling); alpha = 1 is the paper's form.
 * Boundary conditions are homogeneous and imposed by the mirror principle
 * (Sec. 4).  Penalty (Sec. 4.1 takes it from Hillewaert 2013 without the
 * formula): tau = P (k+1)^2 mu(x) sigma_F at every face point, with sigma_e =
 * (sum over the cell's faces of w_f |f|) / |e| the cell's surface-to-volume
 * ratio, w_f = 1/2 for faces shared with another cell and 1 on the boundary
 * (3/h for an interior cube of edge h), sigma_F = max(sigma^-, sigma^+) on an
 * interior face and the cell's own sigma on a boundary face.
 *
 * Discretisation: structured nx*ny*nz hexahedral mesh of a box, cells
 * trilinear in their vertices (straight unit box when no vertices are given),
 * tensor-product Lagrange basis of degree k on the k+1 Gauss-Legendre points,
 * the same points as quadrature rule (Sec. 4: Q_k spaces; Sec. 4.1: as many
 * integration as support points).  The viscosity is evaluated once, at
 * quadrature points (Sec. 4.1 stores it pointwise), from one of the laws below.
 *
 * Vector layout (all device vectors): cell-major,
 *   index = ((e*C + c)*n + i3)*n*n + i2*n + i1,   n = k+1,
 *   e = (ez*ny + ey)*nx + ex, C = 3 (viscous, penalty) or 1 (poisson),
 *   node (i1, i2, i3) at reference point (g[i1], g[i2], g[i3]) of cell e.
 *
 * Ownership: the caller owns every device buffer (vectors and the workspace);
 * the library never calls hipMalloc.  A plan owns host metadata and a small
 * block of pinned host memory for solver status read-back.
 *
 * Errors: every call returns a sipg_status; SIPG_OK is 0, errors are
 * negative; sipg_last_error() returns a message for the calling thread.
 * Nothing is thrown across the ABI.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = default
 * stream).  apply, diagonal, solve_begin and solve_advance only enqueue work;
 * sipg_solve blocks; sipg_solve_poll never blocks.
 */
#ifndef SIPG_H
#define SIPG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SIPG_OK = 0,
    SIPG_ERR_INVALID = -1,        /* bad argument or inconsistent plan */
    SIPG_ERR_OOM = -2,            /* workspace smaller than sipg_plan_workspace_bytes */
    SIPG_ERR_HIP = -3,            /* a HIP runtime call failed */
    SIPG_ERR_NOT_CONVERGED = -4,  /* solve hit max_iter */
    SIPG_ERR_BREAKDOWN = -5,      /* p.Ap <= 0 or non-finite value in CG */
    SIPG_ERR_UNSUPPORTED = -6,    /* valid request this build does not handle */
    SIPG_ERR_STATE = -7           /* call out of order (e.g. apply before bind) */
} sipg_status;

typedef enum { SIPG_F64 = 0, SIPG_F32 = 1 } sipg_precision;
typedef enum { SIPG_VISCOUS = 0, SIPG_POISSON = 1, SIPG_PENALTY = 2 } sipg_operator;
typedef enum { SIPG_BC_DIRICHLET = 0, SIPG_BC_NEUMANN = 1 } sipg_bc;

/* Viscosity laws, evaluated at physical quadrature points x:
 *  CONST     mu = mu
 *  SINE      mu = mu (1 + amp sin(2 pi x) sin(2 pi y) sin(2 pi z))
 *  LOGFIELD  mu = contrast^s, s = clamp((r - rmin)/(rmax - rmin), 0, 1),
 *            r(x) = sum_m a_m cos(2 pi k_m.x + phi_m)
 *  CARREAU   the generalised Newtonian law of Sec. 2,
 *            mu = mu_inf + (mu0 - mu_inf)[kappa + (lam gdot)^a]^((b-1)/a),
 *            gdot = sqrt(2 eps(w):eps(w)) of the prescribed velocity
 *            w(x) = sum_m v_m cos(2 pi k_m.x + phi_m);
 *  ARRAYS    mu given at every quadrature point (Sec. 4.1 stores it
 *            pointwise): mu_cell [ncells][n^3] in the node order of a cell,
 *            mu_face [nfaces][n^2] in the face numbering of
 *            sipg_viscosity_values, host arrays copied by sipg_plan_create,
 *            every value finite and >= 0.  No multigrid hierarchy (coarse
 *            levels have no values of their own).
 * The poisson operator ignores the law (mu = 1). */
typedef enum {
    SIPG_LAW_CONST = 0, SIPG_LAW_SINE = 1, SIPG_LAW_LOGFIELD = 2, SIPG_LAW_CARREAU = 3, SIPG_LAW_ARRAYS = 4
} sipg_law_kind;

#define SIPG_MAX_MODES 16

/* Apply-part mask (sipg_apply_parts): the three sums of the bilinear form. */
enum { SIPG_PART_CELL = 1, SIPG_PART_INTERIOR = 2, SIPG_PART_BOUNDARY = 4, SIPG_PART_ALL = 7 };

typedef struct {
    int32_t nx, ny, nz;        /* cells per direction, each >= 1 */
    const double* vertices;    /* host, [(nz+1)(ny+1)(nx+1)][3], vertex (ix,iy,iz) at
                                  row (iz*(ny+1)+iy)*(nx+1)+ix; NULL = straight unit box.
                                  Copied by sipg_plan_create. */
    int32_t bc[6];             /* sipg_bc for the sides -x,+x,-y,+y,-z,+z */
} sipg_mesh;

typedef struct {
    int32_t kind;              /* sipg_law_kind */
    double mu, amp;            /* CONST, SINE */
    double contrast, rmin, rmax;                      /* LOGFIELD */
    double mu0, mu_inf, lam, n_exp, kappa, a_exp;     /* CARREAU: b = n_exp, a = a_exp */
    int32_t n_modes;           /* <= SIPG_MAX_MODES */
    const int32_t* k;          /* host [n_modes][3] integer wave vectors */
    const double* a;           /* LOGFIELD host [n_modes] amplitudes */
    const double* v;           /* CARREAU host [n_modes][3] velocity amplitudes */
    const double* phi;         /* host [n_modes] phases */
    const double* mu_cell;     /* ARRAYS: host [ncells][n^3] */
    const double* mu_face;     /* ARRAYS: host [nfaces][n^2] */
} sipg_viscosity;

typedef struct {
    int32_t op;                /* sipg_operator */
    int32_t degree;            /* k, 1..5 */
    double alpha;              /* gamma_0/dt in front of the mass term, >= 0 */
    double penalty;            /* P > 0 (SIPG operators) */
    const double* tau_div;     /* SIPG_PENALTY: host [ncells] divergence factors >= 0, else ignored */
    const double* tau_cont;    /* SIPG_PENALTY: host [ncells] continuity factors >= 0, else ignored */
} sipg_params;

typedef struct {
    double rel_tol;            /* stop when ||b - A x|| <= rel_tol ||b|| */
    int32_t max_iter;          /* CG iterations (operator applications of A p) */
    int32_t precond_precision; /* sipg_precision of the Chebyshev-Jacobi preconditioner */
    int32_t cheb_degree;       /* >= 1; degree d uses d-1 operator applications */
    double cheb_ratio;         /* lambda_lo = lambda_hi / cheb_ratio */
    double cheb_safety;        /* lambda_hi = cheb_safety * Lanczos estimate */
    int32_t lanczos_steps;     /* 1..64 */
    int32_t check_every;       /* sipg_solve: iterations between host read-backs */
    int32_t max_restarts;      /* defect-correction restarts */
    int32_t precond_kind;      /* sipg_precond_kind; MULTIGRID needs sipg_plan_set_multigrid */
    int32_t use_graph;         /* nonzero: the iterations between read-backs are captured once into a HIP
                                  graph (per plan: chunk length, x, precision, preconditioner; two cached)
                                  and replayed, for problems small enough to be launch-bound; results are
                                  the same as without (same kernels, same order) */
    int32_t reuse_eigs;        /* nonzero: eigenvalue estimates made before a viscosity or penalty-factor
                                  update (sipg_update_viscosity, sipg_update_penalty_factors) are kept for
                                  the changed operator instead of being re-estimated (a preconditioner
                                  refreshed less often than the operator, as in time-stepping codes);
                                  zero (default): re-estimated on the next solve */
} sipg_solve_opts;

/* Preconditioner of the FP64 CG (Sec. 5.3): Chebyshev-accelerated Jacobi on
 * the operator itself, or V-cycles of the hp-multigrid hierarchy with the
 * same Chebyshev-Jacobi smoother on every level. */
typedef enum { SIPG_PRECOND_CHEBYSHEV = 0, SIPG_PRECOND_MULTIGRID = 1 } sipg_precond_kind;

/* hp-multigrid hierarchy (Sec. 5.3): the polynomial degree is lowered from
 * k to k-1 down to 1 on the plan's mesh, then the mesh is coarsened by two
 * in every direction (every other vertex) while all cell counts are even and
 * at least min_cells.  Levels stay discontinuous; transfers embed the coarse
 * polynomial of a cell in the fine space (restriction is the transpose);
 * every level evaluates the viscosity law at its own quadrature points and
 * has its own inverse diagonal and eigenvalue estimate.  Smoothing:
 * opts->cheb_degree Chebyshev-Jacobi steps before and after the coarse
 * correction.
 * continuous = 1 (default; the paper's cph-multigrid): only the finest level
 * is smoothed in the DG space; below it come continuous levels Q_k, ...,
 * Q_1 on the plan's mesh and Q_1 on the coarser meshes (nodal at the
 * Gauss-Lobatto points, embedded in the DG level of the same degree and mesh,
 * operator G^T A G of that level's cell and boundary terms, Chebyshev-Jacobi
 * smoothing on each), and the coarsest continuous level is solved by an FP64
 * dense inverse when it is of degree 1 with at most direct_max unknowns,
 * else approximated by one Chebyshev-Jacobi polynomial of degree
 * coarse_degree.  continuous = 0: the levels stay discontinuous and the
 * coarsest level gets the degree-coarse_degree polynomial (in place of the
 * paper's AMG cycles). */
typedef struct {
    int32_t coarse_degree;     /* 1..63 */
    int32_t min_cells;         /* >= 1 */
    int32_t max_levels;        /* >= 1, including the finest */
    int32_t h_coarsen;         /* 0: degree lowering only */
    int32_t continuous;        /* 1: cph hierarchy (default), 0: all levels DG */
    int32_t direct_max;        /* 0..2048: largest coarsest level solved directly (default 1024) */
} sipg_mg_opts;

typedef struct {
    int32_t iterations;
    int32_t restarts;
    double rel_residual;       /* true ||b - A x|| / ||b||, computed in FP64 */
    double lambda_max;         /* Lanczos estimate of lambda_max(D^-1 A) */
    int32_t status;            /* sipg_status of the solve */
} sipg_solve_info;

typedef struct sipg_plan sipg_plan;

/* Version of this ABI (increments on any change of a struct or signature). */
int32_t sipg_abi_version(void);

/* Thread-local message of the last error, "" if none. */
const char* sipg_last_error(void);

/* Validates and copies mesh, law and parameters into a new host-side plan
 * (Sec. 4: mesh, degree, viscosity; Sec. 4.1: penalty, alpha = gamma_0/dt).
 * Rejects degree outside 1..5, non-positive cells (det J <= 0 at a corner),
 * bad bc values, a law needing more than SIPG_MAX_MODES modes.
 * No device work. *out is NULL on error. */
sipg_status sipg_plan_create(const sipg_mesh* mesh, const sipg_viscosity* law,
                             const sipg_params* params, sipg_plan** out);

void sipg_plan_destroy(sipg_plan* plan);

/* Number of unknowns C*(k+1)^3*nx*ny*nz. */
int64_t sipg_dof_count(const sipg_plan* plan);

/* Device bytes the plan needs: operator data (geometry, viscosity at cell and
 * face quadrature points in FP64 and FP32, diagonal and inverse diagonal),
 * plus solver vectors when with_solver != 0.  Used for admission control. */
sipg_status sipg_plan_workspace_bytes(const sipg_plan* plan, int32_t with_solver, size_t* bytes);

/* Carves `workspace` (device, 256-byte aligned, at least the size above for
 * with_solver) and enqueues the setup on `stream`: geometry factors, the
 * viscosity at quadrature points (Sec. 4.1 evaluates it pointwise) and the
 * matrix diagonal with its inverse (Sec. 5.3 precomputes it).  The workspace
 * must stay valid and untouched until the plan is destroyed or re-bound. */
sipg_status sipg_plan_bind(sipg_plan* plan, void* workspace, size_t bytes, int32_t with_solver,
                           void* stream);

/* y = A x in the given precision (x, y: device, ndof elements of double or
 * float, no aliasing).  The matrix-free action of the operator above. */
sipg_status sipg_apply(sipg_plan* plan, int32_t precision, const void* x, void* y, void* stream);

/* Same, restricted to the sums selected by `parts` (SIPG_PART_*). */
sipg_status sipg_apply_parts(sipg_plan* plan, int32_t precision, int32_t parts,
                             const void* x, void* y, void* stream);

/* out = diag(A) (inverse == 0) or 1/diag(A) (inverse != 0), device, ndof
 * elements of the given precision (Sec. 5.3, Jacobi-type smoothing). */
sipg_status sipg_diagonal(sipg_plan* plan, int32_t precision, int32_t inverse, void* out,
                          void* stream);

/* Copies the viscosity the plan evaluated at quadrature points: mu_cell
 * [ncells][n^3] (node layout of a cell) and mu_face [nfaces][n^2] in FP64
 * (device; either may be NULL).  Faces are numbered x-faces first,
 * ((ez*ny + ey)*(nx+1) + fx), then y-faces ((ez*(ny+1) + fy)*nx + ex), then
 * z-faces ((fz*ny + ey)*nx + ex); face point (a, b) at index b*n + a with a
 * along the lower tangential axis. */
sipg_status sipg_viscosity_values(sipg_plan* plan, double* mu_cell, double* mu_face, void* stream);

int64_t sipg_face_count(const sipg_plan* plan);

void sipg_solve_opts_default(sipg_solve_opts* opts);

/* Solves A x = b (b, x: device FP64, ndof) with flexible CG in FP64,
 * preconditioned by Chebyshev-accelerated Jacobi in opts->precond_precision
 * (Sec. 5.3: double-precision Krylov, single-precision preconditioner,
 * Chebyshev-Jacobi on the inverse diagonal), followed by an FP64 true-residual
 * check with restarts.  Pure-Neumann Poisson with alpha = 0 is solved in the
 * mean-zero subspace (Sec. 3.2).  SIPG_ERR_UNSUPPORTED for the singular
 * cases left: pure-Neumann viscous and penalty operators with alpha = 0.
 * Needs a plan bound with_solver.  Blocks until done; info may be NULL.
 * Returns the solve's status. */
sipg_status sipg_solve(sipg_plan* plan, const double* b, double* x, const sipg_solve_opts* opts,
                       sipg_solve_info* info, void* stream);

void sipg_mg_opts_default(sipg_mg_opts* opts);   /* 12, 2, 16, 1, 1, 1024 */

/* Builds the multigrid hierarchy of a plan (host only).  Must be called
 * before sipg_plan_workspace_bytes / sipg_plan_bind: the coarse levels' data
 * (viscosity, diagonals, vectors) then live in the same caller-owned
 * workspace, and binding sets up every level.  Errors: INVALID options,
 * STATE if the plan is already bound. */
sipg_status sipg_plan_set_multigrid(sipg_plan* plan, const sipg_mg_opts* opts);

/* Number of levels (1 without a hierarchy); with non-NULL arrays of `cap`
 * entries (3*cap for cells), the degree and cells per direction of each
 * level, finest first. */
int32_t sipg_multigrid_levels(const sipg_plan* plan, int32_t* degrees, int32_t* cells, int32_t cap);

/* Transfer between multigrid level `level` and level+1 (0 = finest) in
 * precision (sipg_precision), device vectors of the two levels' sizes:
 * restrict != 0: out(level+1) = P^T in(level); else out(level) += P in(level+1).
 * Needs a bound plan with a hierarchy; stream-ordered. */
sipg_status sipg_multigrid_transfer(sipg_plan* plan, int32_t level, int32_t restrict_, int32_t precision,
                                    const void* in, void* out, void* stream);

/* One application z = M r of the preconditioner selected by opts
 * (r, z: device FP64, ndof; may alias) in opts->precond_precision, after
 * the eigenvalue estimates it needs (cached per plan).  Needs a plan bound
 * with_solver and no solve in progress; stream-ordered. */
sipg_status sipg_precondition(sipg_plan* plan, const double* r, double* z, const sipg_solve_opts* opts,
                              void* stream);

/* Asynchronous form of sipg_solve for interleaving many solves:
 * begin enqueues the eigenvalue estimate and the CG start on `stream` (the
 * solve stays bound to it); advance enqueues up to `iters` more iterations
 * (iterations after convergence are skipped on the device; nothing is
 * enqueued while poll's true-residual check is pending or after the solve
 * has finished); poll returns
 * immediately with *done = 1 once the solve has finished and `info` filled,
 * enqueueing the true-residual check and restarts itself when needed.
 * b and x must stay valid until done. */
sipg_status sipg_solve_begin(sipg_plan* plan, const double* b, double* x,
                             const sipg_solve_opts* opts, void* stream);
sipg_status sipg_solve_advance(sipg_plan* plan, int32_t iters);
sipg_status sipg_solve_poll(sipg_plan* plan, int32_t* done, sipg_solve_info* info);

/* ---------------------------------------------------------------------
 * Nonlinear viscous step (Sec. 4.1, paragraph "Viscous Step", eq.
 * viscosity_pointwise; Sec. 5.1, Alg. 1): the viscosity is updated
 * pointwise from the velocity, nu = eta(gdot(grad^S u)), and the viscous
 * step is re-solved (Picard iteration) with Aitken's adaptive relaxation
 * computed from the full nonlinear residual.  Needs a viscous plan whose
 * law is SIPG_LAW_CARREAU: its eta parameters (mu0, mu_inf, lam, n_exp,
 * kappa, a_exp) are used, its prescribed velocity modes are not.
 */

/* Re-evaluates the viscosity at every cell and face quadrature point from
 * the velocity u (device FP64, ndof of this plan): gdot = sqrt(2 eps:eps) of
 * u in the cell, of the mean of the two cells' symmetric gradients at an
 * interior face point, of the interior trace on the boundary; every
 * multigrid level evaluates the same velocity at its own quadrature points
 * (a coarse point lies in one fine cell through the nesting of the
 * reference cells).  Then recomputes every level's diagonal and inverse
 * diagonal (FP64 and FP32) and marks the cached eigenvalue estimates
 * stale, so the next solve re-estimates them (unless its opts->reuse_eigs
 * keeps them).  Needs a bound plan; stream-ordered;
 * no solve may be in progress. */
sipg_status sipg_update_viscosity(sipg_plan* plan, const double* u, void* stream);

typedef struct {
    double rel_tol;            /* stop when |R_k| <= rel_tol |R_0|, R(u) = b - A(nu(u)) u */
    double abs_tol;            /* or when |R_k| <= abs_tol (either criterion stops) */
    int32_t max_iter;          /* Picard iterations (linear solves), >= 0 */
    int32_t aitken;            /* nonzero: omega_k = -omega_{k-1} R_{k-1}.(R_k - R_{k-1}) / |R_k - R_{k-1}|^2,
                                  omega_0 = 1; zero: omega = 1 (plain Picard) */
} sipg_picard_opts;

#define SIPG_PICARD_HISTORY 64

typedef struct {
    int32_t iterations;        /* linear solves done */
    int32_t linear_iterations; /* CG iterations summed over them */
    double residual_initial;   /* |R_0| */
    double residual_final;     /* |R_k| at the returned iterate */
    int32_t status;            /* SIPG_OK, SIPG_ERR_NOT_CONVERGED, or a linear solve's error */
    int32_t recorded;          /* entries of the arrays below (<= SIPG_PICARD_HISTORY) */
    double residual_norms[SIPG_PICARD_HISTORY];  /* |R_0|, |R_1|, ... */
    double omegas[SIPG_PICARD_HISTORY];          /* omega used for step 1, 2, ... */
} sipg_picard_info;

void sipg_picard_opts_default(sipg_picard_opts* opts);

/* Device bytes of the `work` buffer of sipg_picard_solve: 3 vectors of ndof
 * FP64 values and the reduction partials. */
size_t sipg_picard_work_bytes(const sipg_plan* plan);

/* Solves the nonlinear viscous step A(nu(x)) x = b (b, x: device FP64,
 * ndof; x holds the initial iterate on entry, e.g. the extrapolated
 * velocity, and the result on return).  Each iteration updates the
 * viscosity from the current x (sipg_update_viscosity), forms
 * R = b - A x on the device, solves A delta = R with sipg_solve and
 * lin_opts (its rel_tol is relative to |R|; NULL: defaults) and sets
 * x += omega delta.  work: device buffer of sipg_picard_work_bytes, 256-byte
 * aligned, not aliasing b or x.  Needs a plan bound with_solver; blocks;
 * returns info->status (info may be NULL).  On return the plan's viscosity
 * is the one of the returned x. */
sipg_status sipg_picard_solve(sipg_plan* plan, const double* b, double* x, void* work,
                              const sipg_solve_opts* lin_opts, const sipg_picard_opts* opts,
                              sipg_picard_info* info, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * Picard iteration as sipg_picard_solve, with its work area (three vectors
 * and the reduction partials) in a static device array of the library
 * instead of a caller buffer.  The array holds SIPG_PICARD_NOALLOC_MAX_DOF
 * unknowns (48 MiB), one copy per GPU the library runs on, kept until the
 * process ends; the call allocates no device memory.  Plans with more
 * unknowns, and lin_opts->use_graph != 0 (graph instantiation allocates),
 * are refused with SIPG_ERR_INVALID before any work.  Every call on one GPU
 * uses the same array: calls that overlap in time on one GPU (other host
 * threads, other streams) race, and the caller must serialise them.
 * Arguments and results as sipg_picard_solve without `work`. */
#define SIPG_PICARD_NOALLOC_MAX_DOF 2097152
sipg_status sipg_picard_solve_noalloc(sipg_plan* plan, const double* b, double* x,
                                      const sipg_solve_opts* lin_opts, const sipg_picard_opts* opts,
                                      sipg_picard_info* info, void* stream);

/* ---------------------------------------------------------------------
 * One time step of the dual splitting scheme (Sec. 3 "Splitting Scheme";
 * the weak forms of Sec. 4.1: eqs. convective_step_weak,
 * convective_term_weak, pressure_step_weak, guhat_consistent_BC,
 * pressure_Neumann_BC, projection_step_weak; the order of Alg. 1), BDF1
 * (gamma_0 = alpha_0 = beta_0 = 1; m_p = 0, so h_p holds no extrapolated
 * convective or viscous terms) or, given u_prev = u^{n-1}, BDF2 with a
 * constant step (gamma_0 = 3/2, alpha = (2, -1/2), beta = (2, -1); m_p = 1:
 * h_p adds -n.((grad u^n) u^n) - nu n.curl(omega) + 2 n.(grad^S u^n . grad nu)
 * with the vorticity omega = curl u^n and nu = eta(gdot(u^n)) projected onto
 * DG_k element by element), on a box whose six sides are
 * walls: velocity Dirichlet data g_u constant in time (g_wall; NULL = no-slip,
 * g_u = 0), pressure Neumann.
 *
 * g_wall: device FP64, the data at the velocity's face quadrature points of
 * every boundary face: rows for the sides -x, +x, -y, +y, -z, +z in turn
 * (ny*nz, ny*nz, nx*nz, nx*nz, nx*ny, nx*ny rows), within a side the faces
 * in the order of their two cell indices along the side (slower: the higher
 * axis); each row holds the (k+1)^2 face points (b*(k+1) + a, a along the
 * lower tangential axis) times 3 components.
 *
 * Three plans on the same mesh (same cells and vertices):
 *   vel   SIPG_VISCOUS, degree k in [2, 5], all sides Dirichlet,
 *         alpha = gamma_0/dt (1/dt for BDF1, 3/(2 dt) for BDF2), law
 *         SIPG_LAW_CARREAU (its eta parameters);
 *   pres  SIPG_POISSON, degree k - 1, all sides Neumann, alpha = 0;
 *   pen   SIPG_PENALTY, degree k, all sides Dirichlet, alpha = 1 (its
 *         factors, and its multigrid levels' if any, are recomputed on the
 *         device).
 * Velocities, forces: device FP64 in vel's layout (3 components, k+1
 * Gauss points per direction); pressures: device FP64 in pres's layout
 * (k Gauss points per direction).  All integrals of the mixed forms use the
 * velocity's (k+1)-point Gauss rule.  The operators below are
 * stream-ordered and allocate nothing; b may be NULL (no body force).
 */

/* uhat = sum_i (alpha_i/gamma_0) u^{n-i} + (dt/gamma_0)(b - sum_i beta_i M^-1 c_h(u^{n-i}; u^{n-i}))
 * (u^n = u, u^{n-1} = u_prev for BDF2, NULL for BDF1) with
 * c_h(v, u; w) = (v, (w.grad) u)_e - (v, ({w}.n) u)_de + (v, ({w}.n) u_dag)_de,
 * u_dag = {u} + sign({w}.n)(u- - u+)/2 (upwind), mirror principle on the
 * walls (u+ = 2 g_u - u-, w+ = 2 g_u - w-; with g_u = 0, {w} = 0 removes the
 * face term). */
sipg_status sipg_convective_step(sipg_plan* vel, const double* u, const double* u_prev, const double* b,
                                 const double* g_wall, double dt, double* uhat, void* stream);

/* Right-hand side of the pressure Poisson equation (pres layout):
 * f_q = (gamma_0/dt)[(grad q, uhat)_e - (q, {uhat}.n)_de] + (q, h_p)_walls,
 * with {uhat} = g_uhat = (dt/gamma_0)(b - sum_i beta_i (grad u^{n-i}) u^{n-i}) +
 * sum_i (alpha_i/gamma_0) g_u on the walls and h_p = n.b (data constant in
 * time; BDF2 adds the terms above), all from interior traces of u_old = u^n,
 * u_prev = u^{n-1} (NULL: BDF1) and b.  BDF2 takes eta from vel's CARREAU law. */
sipg_status sipg_pressure_rhs(sipg_plan* vel, sipg_plan* pres, const double* uhat, const double* u_old,
                              const double* u_prev, const double* b, const double* g_wall, double dt, double* f,
                              void* stream);

/* uhh = uhat + (dt/gamma_0) M^-1 [(div v, p)_e - (v, {p} n)_de] (gamma_0 of the BDF order 1 or 2; {p} = p- on
 * the walls) and, if rhs_visc is not NULL, the viscous step's right-hand
 * side (gamma_0/dt) M uhh. */
sipg_status sipg_projection(sipg_plan* vel, sipg_plan* pres, const double* uhat, const double* p, int32_t order,
                            double dt, double* uhh, double* rhs_visc, void* stream);

/* Recomputes a penalty-step plan's per-cell factors from the velocity u:
 * tau_div = zeta |u_e| h_e dt/(k+1), tau_cont = zeta |u_e| dt (|u_e| the
 * volume mean of |u| over the cell, h_e = |cell|^(1/3)), then its face
 * factors and diagonal, and marks its cached eigenvalue estimate stale (as
 * sipg_update_viscosity does); with a multigrid hierarchy every level's
 * factors follow (degree steps share them, mesh steps take the mean of a
 * coarse cell's 8 children), with their face factors and diagonals.  Needs
 * a bound plan and no solve in progress.  A later sipg_plan_bind restores
 * the factors given at creation. */
sipg_status sipg_update_penalty_factors(sipg_plan* pen, const double* u, double dt, double zeta, void* stream);

/* y += the load of the wall data g_wall for a viscous plan (mirror
 * principle of the SIPG form, with the plan's current viscosity at the face
 * points: int -2 mu eps(v):(g (x) n) + 2 tau (v.g + (v.n)(g.n))) or a
 * penalty-step plan (oriented jump u - g: int tau_e (v.n)(g.n)), over all six
 * sides (plans with Dirichlet sides only).  Stream-ordered. */
sipg_status sipg_wall_load(sipg_plan* plan, const double* g_wall, double* y, void* stream);

/* Defaults (sipg_split_opts_default): the solve defaults with 10-step
 * Lanczos estimates for all three solves. */
typedef struct {
    sipg_solve_opts pressure;  /* pressure Poisson solve (pure Neumann: mean-zero) */
    sipg_solve_opts viscous;   /* viscous step */
    sipg_solve_opts penalty;   /* penalty step */
    double zeta;               /* penalty factor scale (1) */
    int32_t warm_start;        /* nonzero: the viscous solve starts from uhh and the penalty solve from
                                  u_visc (a correction solve for b - A x0 to the tolerance relative to
                                  |b|); zero (default): every solve starts from zero */
} sipg_split_opts;

typedef struct {
    sipg_solve_info pressure, viscous, penalty;
} sipg_split_info;

void sipg_split_opts_default(sipg_split_opts* opts);

/* Device bytes of the `work` buffer of sipg_split_step: five velocity
 * vectors, one pressure vector and reduction partials, each 256-byte aligned. */
size_t sipg_split_work_bytes(const sipg_plan* vel, const sipg_plan* pres);

/* One BDF1 step (u_prev NULL) or BDF2 step (u_prev = u^{n-1}; vel's alpha
 * = 3/(2 dt)) of Alg. 1 with linear-implicit viscosity nu(u^#), u^# =
 * sum_i beta_i u^{n-i} (the penalty factors also use u^#): uhat
 * (convective step), the pressure p (Poisson solve of sipg_pressure_rhs,
 * its mean removed, solution of zero nodal mean), uhh and the viscous
 * right-hand side (projection), the viscosity nu(u^#) on every level of
 * vel (sipg_update_viscosity), the viscous solve, the penalty factors from
 * u^# and the penalty solve with right-hand side M u_visc into u_new; with
 * g_wall, the viscous and penalty right-hand sides take sipg_wall_load.
 * Every solve starts from zero unless opts->warm_start.  u_old, u_prev, b (may be NULL): inputs;
 * u_new, p: outputs (u_new must not alias u_old or u_prev); work: device buffer of
 * sipg_split_work_bytes, 256-byte aligned.  Blocks until done; returns the
 * first failing solve's status (info, which may be NULL, holds all three). */
sipg_status sipg_split_step(sipg_plan* vel, sipg_plan* pres, sipg_plan* pen, const double* u_old,
                            const double* u_prev, const double* b, const double* g_wall, double dt, double* u_new,
                            double* p, void* work, const sipg_split_opts* opts, sipg_split_info* info, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SIPG_H */
