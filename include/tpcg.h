/*
 * tpcg: spectral two-level preconditioned conjugate gradients for the
 * SIMP-scaled linear-elastic system K(rho) u = f on one AMD MI355X (gfx950).
 *
 * The operation follows Alexandersen & Lazarov, "Robust topology optimisation
 * of microstructural details without length scale separation - using a
 * spectral coarse basis preconditioner" (arXiv:1411.3923):
 *   - K u = f from bilinear (2D, plane stress) or trilinear (3D) elements on a
 *     uniform mesh of unit elements, C(x) = E(x) C0 with unit reference
 *     modulus (Sec. 2.1);
 *   - K_e = (E_min + (E0 - E_min) rho_e^p) K0 (Sec. 2.2, element stiffness);
 *   - compliance f^T u and its self-adjoint sensitivity (Sec. 2.2, Sec. 4.2);
 *   - a coarse space from local generalised eigenproblems K_w psi =
 *     lambda diag(K_w) psi, multiplied by a partition of unity, with the
 *     Galerkin coarse matrix R_c K R_c^T (Sec. 2.4, Sec. 3.2);
 *   - that coarse space used inside a Krylov preconditioner for the SPD
 *     system (Sec. 2.4.2); here the two-level additive Schwarz form
 *     M^-1 = sum_j R_j^T A_j^-1 R_j + R_c^T K_c^-1 R_c inside PCG;
 *   - the density filter and smoothed Heaviside projection with their chain
 *     rule (Sec. 4.3), at several thresholds (Sec. 4.4).
 *
 * Index conventions (all arrays):
 *   node    n = ix + (nelx+1) * (iy + (nely+1) * iz)
 *   dof       = dim * n + c                         (c: 0 = x, 1 = y, 2 = z)
 *   element e = ex + nelx * (ey + nely * ez)
 *   Element nodes run counter-clockwise from (ex, ey); in 3D the bottom face
 *   (ez) first, then the top face.
 *
 * Conventions for every entry point:
 *   - Array arguments marked "dev" are caller-owned device pointers to
 *     contiguous float64 data laid out [nsys][...]; the library never frees,
 *     keeps or reallocates them. "host" arguments are ordinary host memory.
 *   - Work is enqueued on the stream given to tpcg_build_partition. Entry
 *     points return after enqueueing, except tpcg_pcg_solve and
 *     tpcg_build_coarse_basis, which return when their results are complete
 *     (pcg_solve fills `info` on the host).
 *   - A handle is not thread-safe; separate handles are independent.
 *   - Negative status codes mean the outputs are unspecified. TPCG_EHIP is
 *     sticky: destroy the handle. tpcg_last_error gives a message.
 */
#ifndef TPCG_H
#define TPCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tpcg_handle tpcg_handle;

typedef enum {
  TPCG_OK = 0,
  TPCG_ENOCONV = 1,      /* warning: maxit reached; outputs valid */
  TPCG_EAGAIN = 2,       /* not now: no capacity or not finished; nothing was changed, retry */
  TPCG_EINVAL = -1,      /* bad argument (size, null pointer, unsupported setting) */
  TPCG_ENOMEM = -2,      /* device allocation failed */
  TPCG_EHIP = -3,        /* HIP runtime error (sticky) */
  TPCG_ENOTSPD = -4,     /* non-positive pivot in a Cholesky factorisation */
  TPCG_EBREAKDOWN = -5,  /* PCG breakdown: p^T K p <= 0, r^T z <= 0 or NaN */
  TPCG_ESTATE = -6       /* call order: preconditioner used before it is built */
} tpcg_status;

typedef enum { TPCG_FP64 = 0, TPCG_MIXED = 1 } tpcg_precision;

/* Preconditioner of tpcg_gmres_solve. */
typedef enum {
  TPCG_PC_ADDITIVE = 0,   /* two-level additive Schwarz (the one tpcg_pcg_solve uses) */
  TPCG_PC_MSFEM_SGS = 1   /* the MsFEM coarse solve between symmetric Gauss-Seidel steps */
} tpcg_precond_kind;

/* Problem description. Sizes are in elements. */
typedef struct {
  int32_t dim;          /* 2 (Q4 plane stress) or 3 (H8) */
  int32_t nel[3];       /* elements per axis; nel[2] = 1 in 2D */
  double E0;            /* solid modulus (paper: E_max = 1) */
  double Emin;          /* void modulus (paper: 1e-9) */
  double penal;         /* SIMP exponent p */
  double nu;            /* Poisson ratio, < 0.5 */
  int32_t sub[3];       /* subdomain (unit cell) edge per axis in elements, nel[a] % sub[a] == 0;
                           the cells must be square (cubic): sub[0] == sub[1] (== sub[2] in 3D;
                           sub[2] is ignored in 2D) */
  int32_t overlap;      /* element layers of overlap; only 1 is supported */
  int32_t ncoarse;      /* k: coarse vectors per subdomain (the cap when lambda_thresh > 0) */
  int32_t nsys_max;     /* systems (realisations) solved together, 1..4 */
  int32_t precision;    /* tpcg_precision */
  int32_t eig_iters;    /* subspace iterations for the local eigenproblems (0: default 6) */
  int32_t eig_extra;    /* extra (guard) vectors in the subspace (0: default k, capped at 16 total) */
  double eig_shift;     /* shift sigma of the shift-invert eigensolver (0: default 1e-5); the
                           factorised matrix is diag(K^N)^-1/2 K^N diag(K^N)^-1/2 + sigma I, so a
                           sigma <= 0 on a floating cell (rigid-body modes at 0) is indefinite and
                           the build returns TPCG_ENOTSPD */
  double lambda_thresh; /* <= 0: exactly ncoarse vectors per subdomain; > 0: the eigenvectors with
                           eigenvalue below lambda_thresh (Sec. 2.4: one global threshold), at
                           most ncoarse per subdomain; unused columns are stored as zeros */
  int32_t coarse_dense_max; /* coarse dimensions up to this keep a dense K_c^-1 applied as a
                           product; larger ones use the block-tridiagonal coarse factor
                           (0: default 12288) */
  int32_t big_min_nb;   /* subdomain node-layer blocks of at least this many unknowns use the
                           HBM-resident factors and solves (0: only blocks the on-chip kernels
                           cannot take: more than 96 unknowns, an odd count, or layers of more
                           than 64 elements) */
  int32_t coarse_band;  /* 1: the coarse level always as the HBM-resident block-tridiagonal
                           factor (S_b^-1 and the multipliers, applied by chains of block
                           products beside the local solves); 0: only when the coarse
                           dimension exceeds coarse_dense_max and its blocks do not fit the
                           on-chip factor kernels (more than 96 or odd) */
  int32_t dedup;        /* 1: one local eigenproblem per distinct cell (Sec. 2.4: equal
                           agglomerates of a periodic microstructure): subdomains whose cell
                           densities (of the representative system) and box supports are equal
                           take the eigenpairs of the first, with their own partition of unity.
                           On-chip path only (ignored for HBM-resident blocks). 0: every cell */
} tpcg_problem;

/* Per-system result of tpcg_pcg_solve. */
typedef struct {
  int32_t iters;        /* PCG iterations taken */
  int32_t status;       /* tpcg_status of this system */
  double relres;        /* ||r_k||_2 / ||P f||_2 of the recursive residual */
  double true_relres;   /* ||P (f - K u)||_2 / ||P f||_2 recomputed at exit */
  double seconds;       /* wall time of the whole batched solve */
} tpcg_info;

/*
 * Create a handle for the structured mesh in `prob` with the supports in
 * `fixed_mask` (host, uint8 [n_dof], nonzero = displacement prescribed zero,
 * Sec. 2.1 Dirichlet parts per component). Builds the subdomain partition:
 * subdomain j is the j-th unit cell of sub^dim elements (Sec. 2.4: the coarse
 * cells are the unit cells); its unknowns are the nodes of the closed cell,
 * i.e. the cell grown by one element layer with zero displacement on the
 * grown boundary. Subdomains are numbered x fastest. `stream` is a
 * hipStream_t (NULL: the default stream). Returns TPCG_EINVAL, before any
 * device call, for nel % sub != 0, non-square (non-cubic) subdomains, dim
 * not in {2,3}, overlap != 1, ncoarse < 1 or larger than the subdomain's
 * DOFs, nsys_max not in 1..4, Emin <= 0, E0 < Emin, penal < 1, nu outside
 * (-1, 0.5), a NaN lambda_thresh or a negative coarse_dense_max. The
 * preconditioner's own size limits are checked by tpcg_build_coarse_basis.
 */
int tpcg_build_partition(const tpcg_problem* prob, const uint8_t* fixed_mask,
                         void* stream, tpcg_handle** out);

/* Device bytes a handle for `prob` with `nsys` systems allocates (admission). */
size_t tpcg_workspace_bytes(const tpcg_problem* prob, int32_t nsys);

/*
 * Build the two-level preconditioner for the physical densities rho_phys
 * (dev [nsys][n_el]). The spectral basis (Sec. 2.4, discrete eigenproblem
 * weighted by diag(K_j^N), Sec. 3.2) is computed once, from system `rep`
 * (the robust formulation uses the dilated realisation, Sec. 5.3): for every
 * subdomain the k smallest eigenpairs of the Neumann matrix of the cell's own
 * elements (physical supports kept), times the partition of unity
 * chi_j(n) = 1/(number of subdomains containing n). For every system it then
 * factors the local Dirichlet matrices A_j (principal submatrices of K) and the
 * coarse matrix K_c = Phi^T K Phi (coarse projection equation). Blocks until
 * done. With lambda_thresh > 0 a subdomain keeps only the eigenvectors whose
 * eigenvalue lies below it (at most ncoarse; Sec. 2.4 global threshold); the
 * unused coarse unknowns get a unit diagonal in K_c and stay zero.
 * Returns TPCG_EINVAL if a density is NaN or outside [0, 1], or if the
 * subdomain blocks exceed the factor kernels' limits: node-row (2D) or
 * node-layer (3D) blocks of even size at most 96 (2D s <= 47, 3D s in {1, 3}),
 * element layers of at most 64 elements, coarse blocks (k times the
 * subdomains of a cross-section along the axis with the most subdomains) of
 * even size at most 96. TPCG_ENOMEM if device memory runs out (the handle is
 * then unchanged and the build may be retried). TPCG_ENOTSPD if a
 * factorisation meets a non-positive pivot.
 */
int tpcg_build_coarse_basis(tpcg_handle* h, const double* rho_phys, int32_t nsys, int32_t rep);

/*
 * Keep the spectral basis of the last tpcg_build_coarse_basis and rebuild
 * everything else of the preconditioner for the physical densities rho_phys
 * (dev [nsys][n_el]): the local Dirichlet factors and the coarse matrix
 * K_c = Phi^T K Phi with its factor, per system. The basis re-use of Sec.
 * 5.1 and Sec. 5.2: the expensive local eigenproblems are solved again only
 * when the design has moved far enough. Blocks until done. TPCG_ESTATE
 * before a first build; other errors as tpcg_build_coarse_basis.
 */
int tpcg_refactor(tpcg_handle* h, const double* rho_phys, int32_t nsys);

/*
 * y = P K(rho) P x with K assembled from E_e = E_min + (E0 - E_min) rho_e^p
 * times the unit element matrix (Sec. 2.2), P zeroing the supported DOFs.
 * rho_phys dev [nsys][n_el], x and y dev [nsys][n_dof] (16-byte aligned).
 * Matrix-free. The densities are checked first (one synchronisation):
 * TPCG_EINVAL if one is NaN or outside [0, 1].
 */
int tpcg_apply_K(tpcg_handle* h, const double* rho_phys, const double* x, double* y, int32_t nsys);

/*
 * z = M^-1 r for the preconditioner built by tpcg_build_coarse_basis
 * (Sec. 2.4.2 with the two-level additive Schwarz form). r and z dev
 * [nsys][n_dof]; nsys must equal the nsys of the build. TPCG_ESTATE if the
 * preconditioner has not been built.
 */
int tpcg_apply_precond(tpcg_handle* h, const double* r, double* z, int32_t nsys);

/*
 * Solve K(rho_s) u_s = P f_s for all systems with PCG preconditioned by
 * M^-1 (Sec. 2.4.2). u (dev [nsys][n_dof]) holds the initial guess on entry
 * (zeros: cold start; the previous design's solution: warm start, Sec. 5.2)
 * and the solution on exit. Stops system s when ||r||_2 <= rtol ||P f_s||_2
 * or after maxit iterations. The preconditioner may be stale (built for an
 * older rho); the solution is still that of the new rho. info: host [nsys].
 * A system whose densities hold a NaN or a value outside [0, 1] does not
 * start and reports TPCG_EINVAL in its info (u then holds its initial guess
 * with the supported DOFs zeroed). Returns the worst status over the systems.
 */
int tpcg_pcg_solve(tpcg_handle* h, const double* rho_phys, const double* f, double* u,
                   int32_t nsys, double rtol, int32_t maxit, tpcg_info* info);

/*
 * The same solve enqueued on the handle's stream without any host wait (the
 * serving path's form): every iteration up to maxit is launched, each system
 * stopping at its own convergence (the launches after it return at once),
 * then the per-system results are written to info_dev (device memory, [nsys]
 * tpcg_info records; seconds = 0). Returns after enqueueing; synchronise the
 * stream before reading u or info_dev. Results are bitwise those of
 * tpcg_pcg_solve with the same arguments. Choose maxit near the expected
 * count: every iteration up to it is launched.
 */
int tpcg_pcg_solve_async(tpcg_handle* h, const double* rho_phys, const double* f, double* u,
                         int32_t nsys, double rtol, int32_t maxit, tpcg_info* info_dev);

/*
 * z = B r with the paper's multiplicative preconditioner (Sec. 2.4.2): one
 * symmetric Gauss-Seidel step S from zero, the MsFEM coarse correction, one
 * more step:  x = S(r; 0);  x += Phi K_c^-1 Phi^T (r - K x);  z = S(r; x).
 * S acts on node blocks (each node's d x d diagonal block solved exactly) in
 * multicolour order: colour = parity of x + 2 parity of y (+ 4 parity of z),
 * colours in increasing then decreasing order. K = P K(rho_phys) P with unit
 * diagonal on the supported DOFs, which stay zero in z. The coarse basis and
 * K_c^-1 are those of the last build (tpcg_build_coarse_basis); rho_phys may
 * differ from the build's. r, z dev [nsys][n_dof] (16-byte aligned, distinct);
 * nsys must equal the build's. TPCG_ESTATE before a build.
 */
int tpcg_apply_msfem(tpcg_handle* h, const double* rho_phys, const double* r, double* z,
                     int32_t nsys);

/*
 * Solve K(rho_s) u_s = P f_s for all systems with restarted GMRES, the
 * paper's solver (Sec. 2.4.2), preconditioned from the left by `precond`
 * (tpcg_precond_kind). u dev [nsys][n_dof] holds the initial guess on entry
 * and the solution on exit. System s stops when the preconditioned residual
 * ||B P (f_s - K u_s)||_2 falls to rtol ||B P f_s||_2 (the measure of Sec.
 * 3.3), or after maxit Arnoldi steps; a cycle holds `restart` steps (1..64).
 * info (host [nsys]): iters = Arnoldi steps, relres = the preconditioned
 * relative residual (GMRES's estimate), true_relres = ||P (f - K u)|| /
 * ||P f||. Allocates the Krylov basis ((restart + 1) nsys n_dof doubles) on
 * the first call, and again when a call needs a larger one (TPCG_ENOMEM if
 * that fails; the handle stays usable). Blocks until done. Densities are
 * checked first: TPCG_EINVAL if one is NaN or outside [0, 1]. Returns the
 * worst status over the systems (TPCG_ENOCONV if maxit was reached).
 */
int tpcg_gmres_solve(tpcg_handle* h, const double* rho_phys, const double* f, double* u,
                     int32_t nsys, double rtol, int32_t maxit, int32_t restart, int32_t precond,
                     tpcg_info* info);

/*
 * Compliance c_s = f_s^T u_s (dev [nsys]) and, if dc is not NULL, the element
 * sensitivities dc/drho_e = -p (E0 - E_min) rho_e^(p-1) u_e^T K0 u_e
 * (dev [nsys][n_el]) (Sec. 4.2: self-adjoint, no adjoint solve). With dc the
 * densities are checked first (one synchronisation): TPCG_EINVAL if one is
 * NaN or outside [0, 1].
 */
int tpcg_compliance_and_sensitivity(tpcg_handle* h, const double* rho_phys, const double* u,
                                    const double* f, int32_t nsys, double* c, double* dc);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * compliance c_s = f_s^T u_s and, if dc is not NULL, the element
 * sensitivities of tpcg_compliance_and_sensitivity, without a handle and
 * without any device or host allocation. prob must be a problem accepted by
 * tpcg_build_partition; fixed is the support mask as a device array (uint8
 * [n_dof], nonzero = supported); rho_phys, u, f, c and dc as in
 * tpcg_compliance_and_sensitivity; status (dev int32, may be NULL) is set to
 * 0, or to 1 if a density is NaN or outside [0, 1] (the outputs are then
 * unspecified). Work is enqueued on `stream` (a hipStream_t of the current
 * device; NULL: the default stream) and the call returns without waiting.
 * Scratch: a fixed library array of 576 + 4 * 2048 doubles per device
 * (the element matrix and the reduction partials), held until the process
 * ends; every call on a device shares it, so calls that overlap on one
 * device (concurrent streams or threads) race. Limits: nsys in 1..4
 * (TPCG_EINVAL beyond). TPCG_EHIP if the scratch address cannot be found or
 * a launch fails.
 */
int tpcg_compliance_and_sensitivity_noalloc(const tpcg_problem* prob, const uint8_t* fixed,
                                            const double* rho_phys, const double* u,
                                            const double* f, int32_t nsys, double* c, double* dc,
                                            int32_t* status, void* stream);

/*
 * Density filter and smoothed Heaviside projection (Sec. 4.3):
 * rho_tilde = W rho with hat weights max(0, rmin - distance between element
 * centres), truncated at the mesh boundary and renormalised (rmin <= 1: no
 * filtering); rho_phys[s] = H(rho_tilde; beta, eta[s]) for each threshold
 * (Sec. 4.4). rho dev [n_el], eta host [nsys], rho_tilde dev [n_el],
 * rho_phys dev [nsys][n_el]. TPCG_EINVAL if a design variable is NaN or
 * outside [0, 1] (checked first, one synchronisation).
 */
int tpcg_filter_project(tpcg_handle* h, const double* rho, double rmin, double beta,
                        const double* eta, int32_t nsys, double* rho_tilde, double* rho_phys);

/*
 * Chain rule through projection and filter (Sec. 4.3):
 * dc_drho[s][i] = sum_e dc_drho_phys[s][e] H'(rho_tilde_e; beta, eta[s]) W[e][i].
 * rho_tilde dev [n_el], dc_drho_phys and dc_drho dev [nsys][n_el], eta host [nsys].
 */
int tpcg_filter_project_adjoint(tpcg_handle* h, const double* rho_tilde, double rmin, double beta,
                                const double* eta, int32_t nsys, const double* dc_drho_phys,
                                double* dc_drho);

/*
 * Robust objective over the realisations (Sec. 4.4: mean plus kappa times the
 * standard deviation of the compliance; the paper uses kappa = 1 and three
 * equally weighted realisations): out3 (dev [3]) = {E[c] + kappa std, E[c],
 * std} with E[c] = sum_s w_s c_s and std^2 = sum_s w_s (c_s - E[c])^2 for c
 * dev [nsys]; weights host [nsys] (NULL: 1/nsys each). If dc (dev
 * [nsys][n_el], the gradients of the c_s, e.g. with respect to the design
 * variables after tpcg_filter_project_adjoint) is not NULL, df (dev [n_el])
 * receives the gradient sum_s w_s (1 + kappa (c_s - E[c]) / std) dc[s]
 * (without the variance term when std = 0). TPCG_EINVAL for nsys outside
 * 1..4, kappa < 0 or a negative weight.
 */
int tpcg_robust_objective(tpcg_handle* h, const double* c, const double* dc, int32_t nsys,
                          double kappa, const double* weights, double* out3, double* df);

/*
 * Sensitivities of periodic design variables (Sec. 4.1: one design variable
 * controls the element at the same position in every copy of the unit cell):
 * gcell[s][v] = sum of g[s][e] over the elements e at position v of the unit
 * cell of cell[0] x cell[1] (x cell[2] in 3D) elements, cells laid out from
 * the mesh origin (partial cells at the far faces count), v = vx + cell[0]
 * (vy + cell[1] vz). g dev [nsys][n_el], cell host [3], gcell dev
 * [nsys][cell volume]. TPCG_EINVAL for a cell outside the mesh.
 */
int tpcg_periodic_sum(tpcg_handle* h, const double* g, int32_t nsys, const int32_t* cell,
                      double* gcell);

/*
 * Non-discreteness measure of a density field (Sec. 5.2): out (dev [1]) =
 * sum_e 4 rho_e (1 - rho_e) / n_el for rho_phys dev [n_el].
 */
int tpcg_nondiscreteness(tpcg_handle* h, const double* rho_phys, double* out);

/*
 * Serving: many optimisation runs ("sessions") on one GPU. A session owns a
 * handle (tpcg_build_partition) on a stream of its own, so its factors and
 * coarse space stay resident in device memory across its design updates, and
 * a worker thread. tpcg_server_open admits a session when its device memory
 * (tpcg_server_session_bytes: tpcg_workspace_bytes plus the density buffers)
 * fits in the rest of the server's budget and fewer than max_active sessions
 * are open; otherwise it returns TPCG_EAGAIN and changes nothing (retry after
 * a session closes). A job (tpcg_server_submit) is one design update of a
 * session, run after the session's earlier jobs and concurrently with the
 * jobs of other sessions (their kernels overlap on the device):
 *   - physical densities of the nsys realisations from the design rho (dev
 *     [n_el]) by tpcg_filter_project (rmin > 0; rmin <= 0: rho itself);
 *   - the preconditioner rebuilt from realisation `rep` when the session has
 *     none, when rebuild > 0, or (rebuild == 0, Sec. 5.2's rule) when the
 *     previous job's PCG took more than `growth` times the lowest iteration
 *     count seen since the last rebuild (rebuild < 0: never again);
 *     otherwise the resident basis is kept and, with refactor, the local
 *     and coarse factors are rebuilt for the job's design (tpcg_refactor);
 *   - tpcg_pcg_solve of all realisations with u (dev [nsys][n_dof]) as the
 *     initial guess (warm start from the previous design's displacements,
 *     Sec. 5.2) and as the output; f dev [nsys][n_dof];
 *   - c (dev [nsys]) and, if dc (dev [nsys][n_el]) is not NULL, the
 *     sensitivities with respect to the design (chain rule through the
 *     projection and filter);
 *   - the non-discreteness of realisation `rep`.
 * The caller keeps rho, f, u, c and dc alive and unmodified until the job is
 * complete (tpcg_server_wait, or tpcg_server_test returning TPCG_OK; it
 * returns TPCG_EAGAIN while the job runs). A result is read once.
 * tpcg_server_close runs the session's remaining jobs, then frees it.
 * The server uses the device current at tpcg_server_create; its functions
 * may be called from several threads.
 */
typedef struct tpcg_server tpcg_server;

typedef struct {
  double rtol;          /* PCG relative residual */
  int32_t maxit;
  int32_t rebuild;      /* 0: iteration-count rule; > 0: every job; < 0: only the first */
  double growth;        /* rule: rebuild when iterations > growth x the reference count (>= 1) */
  double rmin, beta;    /* density filter radius (<= 0: no filter) and projection sharpness */
  double eta[4];        /* projection thresholds of the realisations */
  int32_t rep;          /* realisation the coarse basis is built from */
  int32_t refactor;     /* 1: between basis rebuilds, refactor the local and coarse factors for
                           the job's design (tpcg_refactor); 0: keep them as well */
} tpcg_job_opts;

typedef struct {
  int32_t status_all;   /* tpcg_status of the job (a failure of any step) */
  int32_t iters[4];     /* per realisation */
  int32_t status[4];
  double relres[4], true_relres[4];
  int32_t rebuilt;      /* this job rebuilt the preconditioner with a new basis */
  int32_t refactored;   /* this job refactored with the resident basis */
  int32_t rebuilds;     /* rebuilds of the session so far */
  double queue_ms;      /* from submission to the start of the job */
  double build_ms, solve_ms, total_ms;
  double m_nd;          /* non-discreteness of realisation rep */
} tpcg_job_result;

int tpcg_server_create(size_t budget_bytes, int32_t max_active, tpcg_server** out);
size_t tpcg_server_session_bytes(const tpcg_problem* prob, int32_t nsys);
int tpcg_server_open(tpcg_server* s, const tpcg_problem* prob, const uint8_t* fixed_mask,
                     int32_t nsys, int64_t* session);
int tpcg_server_submit(tpcg_server* s, int64_t session, const double* rho, const double* f,
                       double* u, double* c, double* dc, const tpcg_job_opts* opts, int64_t* job);
int tpcg_server_wait(tpcg_server* s, int64_t job, tpcg_job_result* out);
int tpcg_server_test(tpcg_server* s, int64_t job, tpcg_job_result* out);
int tpcg_server_close(tpcg_server* s, int64_t session);
size_t tpcg_server_free_bytes(const tpcg_server* s);
void tpcg_server_destroy(tpcg_server* s);

/*
 * Copy the coarse basis out (diagnostics and tests): phi dev
 * [n_sub][n_loc][k] (chi-weighted basis vectors on the subdomain's closed-cell
 * DOFs, node x fastest then component; may be NULL), lambda host [n_sub][k]
 * Ritz values and resid host [n_sub][k] residual norms ||S x - lambda x||_2
 * of the diagonally scaled problem (either may be NULL).
 */
int tpcg_export_coarse_basis(tpcg_handle* h, double* phi, double* lambda, double* resid);

/*
 * Ritz values of the local eigenproblems (Sec. 2.4 discrete eigenproblem with
 * the diag(K) weighting of Sec. 3.2) from the last build: lambda host
 * [n_sub][m], the m smallest of each subdomain in ascending order, m at most
 * tpcg_query_subspace (the eigensolver's subspace width; values beyond the
 * ncoarse-th are less accurate); kj host [n_sub] (may be NULL): coarse
 * vectors in use per subdomain (ncoarse, or fewer under lambda_thresh).
 * TPCG_ESTATE before a build, TPCG_EINVAL for m out of range.
 */
int tpcg_export_eigenvalues(tpcg_handle* h, double* lambda, int32_t m, int32_t* kj);

/*
 * Testing support: the record C_b (the inverse of the b-th Schur complement
 * of the twisted elimination of the local Dirichlet matrix of subdomain sub
 * in system sys) as a dense row-major nb x nb matrix in host memory out.
 * Only for subdomain blocks on the HBM-resident path (TPCG_EINVAL otherwise).
 */
int tpcg_export_local_record(tpcg_handle* h, int32_t sys, int32_t sub, int32_t blk, double* out);

/* Local eigenproblems solved by the last basis build: the distinct cells with
 * dedup on, else n_sub (0 before a build); TPCG_EINVAL for a null handle. */
int tpcg_query_unique_cells(const tpcg_handle* h);

/* Width of the eigensolver's subspace (ncoarse + eig_extra, at most 16 and at
 * most the subdomain's DOFs), or TPCG_EINVAL for a null handle. */
int tpcg_query_subspace(const tpcg_handle* h);

/* Sizes of the handle's structures: out[0] n_dof, out[1] n_el, out[2] n_sub,
 * out[3] n_loc, out[4] k, out[5] local block size, out[6] local block count,
 * out[7] coarse block size, out[8] coarse block count. */
int tpcg_query(const tpcg_handle* h, int64_t* out9);

/*
 * Measurement support. With profiling on, tpcg_pcg_solve records HIP events
 * around every launch of its batched block-solve kernel (the local subdomain
 * and coarse triangular solves of M^-1) on the handle's stream and
 * accumulates, over the launches in which at least one system was still
 * iterating: out3[0] the number of launches, out3[1] their summed duration
 * in milliseconds, out3[2] their summed algorithmic bytes (band Cholesky
 * factors read twice, right-hand sides read and results written once).
 * tpcg_set_profiling resets the accumulators.
 */
int tpcg_set_profiling(tpcg_handle* h, int32_t on);
int tpcg_profile_block_solves(const tpcg_handle* h, double* out3);

/*
 * Launch mode of tpcg_pcg_solve. With graphs on, the chunks of four PCG
 * iterations after the first are captured once into HIP graphs and replayed
 * (a capture is redone when the solve's arguments change). With graphs off
 * (the default: on MI355X the replay measured slightly slower than launching
 * the same kernels from the host), when profiling is on, when the coarse
 * level uses the block-tridiagonal factor, or when a capture fails (the
 * handle then stays eager), every kernel is launched from the host. Results
 * are bitwise the same in both modes. tpcg_last_solve_graph_chunks gives
 * the number of chunks the last solve replayed from graphs.
 */
int tpcg_set_graphs(tpcg_handle* h, int32_t on);

/*
 * Autotuning of the launch choices that leave results bit for bit the same
 * (off by default). PCG: graph replay on or off and the chunk length between
 * convergence polls (4 or 8 iterations), measured over the handle's first
 * solves (one warm-up, then each candidate twice; graph candidates only when
 * profiling is off and the dense coarse inverse is in use), ranked by the
 * best time per iteration; while tuning, tpcg_set_graphs is overridden.
 * GMRES: Krylov vectors per workgroup of the dot-product kernel (4, 8 or 16),
 * timed on the handle's basis at the first tpcg_gmres_solve. Choices are
 * stored in a text file keyed by device and problem ($TPCG_TUNE_CACHE, else
 * $XDG_CACHE_HOME/tpcg/tune.txt, else $HOME/.cache/tpcg/tune.txt; nothing is
 * stored if it cannot be written); a handle whose key is stored takes the
 * choice at its first solve. Not an optimisation of the numerics: every
 * candidate computes the same bits.
 */
int tpcg_set_autotune(tpcg_handle* h, int32_t on);

/*
 * State of the autotuner, out (host [8]): on, PCG choice made, taken from
 * the cache, graphs on, poll interval, GMRES choice made, GMRES vectors per
 * workgroup, solves measured so far.
 */
int tpcg_query_tune(const tpcg_handle* h, int32_t* out);
int tpcg_last_solve_graph_chunks(const tpcg_handle* h);

/*
 * Testing support for the allocation paths: the nth device allocation the
 * library makes from this call on fails as if the device were out of memory
 * (nth <= 0: none). Process-wide, not thread-safe.
 */
void tpcg_test_fail_alloc(int32_t nth);

const char* tpcg_last_error(const tpcg_handle* h);
void tpcg_destroy(tpcg_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* TPCG_H */
