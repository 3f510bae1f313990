/*
 * sem.h -- C ABI of the MI355X least-squares h-p spectral element library.
 *
 * The library minimises the discrete least-squares functional R^{N,W} of
 * Husain's thesis "h-p spectral element methods for three dimensional
 * elliptic problems on non-smooth domains using parallel computers"
 * (arXiv 1110.2316), Ch. 4, eq 4.1-4.8, for the Poisson problem
 * -Laplace(u) = f with Dirichlet data g, by PCG on its normal equations
 * X U = b (Sec. 5.3: R(U + eps V) = R(U) + 2 eps V^T (X U - b) + O(eps^2)).
 * X is applied matrix-free on the GPU in every iteration: the element
 * PDE residual collocated on the (2W+1)^3 GLL grid and its adjoint, plus the
 * interface jump and boundary terms in fractional Sobolev norms.  The
 * preconditioner is block-diagonal (Sec. 5.2), in one of two forms chosen by
 * sem_set_preconditioner: the separable element forms of Sec. 5.2 (the
 * default after sem_setup), or the exact diagonal element blocks of X, whose
 * stored inverses the element-block apply streams (the form the measured
 * solves use).
 *
 * Conventions
 *  - All floating point data is IEEE double unless a precision says otherwise.
 *  - "device pointer": memory from hipMalloc (e.g. a torch CUDA tensor's
 *    data_ptr) on the device that was current at sem_setup.  "host pointer":
 *    ordinary CPU memory.  The caller owns every pointer it passes; the
 *    library never frees them and keeps none of them after the call returns.
 *  - Unknown vector layout (length sem_ndof): the n^3 nodal values of each
 *    real element, n = W+1, in mesh order, index i + n j + n^2 k (i fastest,
 *    i/j/k along lam1/lam2/lam3, GLL nodes ascending); then the corner
 *    unknowns (vertex constants and corner polynomials) in corner-offset order.
 *  - stream: a hipStream_t passed as void*; NULL is the default stream.
 *  - Every call returns a sem_status.  On failure sem_last_error() returns
 *    a message for the calling thread.  No C++ exception crosses the ABI.
 *  - Calls on one context must not overlap in time from several host threads.
 */
#ifndef SEM_H
#define SEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SEM_OK = 0,
    SEM_EINVAL = -1,      /* bad argument or mesh */
    SEM_ENOMEM = -2,      /* device or host allocation failed */
    SEM_EHIP = -3,        /* a HIP runtime call failed */
    SEM_ENOCONV = -4,     /* PCG hit maxit before the tolerance */
    SEM_EBREAKDOWN = -5,  /* PCG breakdown: p^T X p <= 0 or r^T z <= 0 */
    SEM_ENAN = -6,        /* a NaN or Inf appeared in PCG scalars */
    SEM_ENODATA = -7      /* sem_rhs before sem_set_data */
} sem_status;

typedef enum {
    SEM_FP64 = 0,         /* every step in double precision */
    SEM_MIXED_FP32 = 1    /* inner operator contractions in float (see sem_pcg_solve_mixed) */
} sem_precision;

typedef enum {
    SEM_PRECOND_SEPARABLE = 0,     /* the separable element forms of Sec. 5.2 (default) */
    SEM_PRECOND_ELEMENT_BLOCK = 1  /* the exact diagonal element blocks of X */
} sem_precond_kind;

/* Mesh description (host pointers, read during sem_setup only).
 * Element maps from the master cube Q = (-1,1)^3 (thesis Sec. 2.3; modified
 * coordinates eq 2.3, 2.5, 2.8):
 *   chart 0 AFFINE     box in x
 *   chart 1 VTX_BOX    box in (phi, theta, chi = ln rho)
 *   chart 2 VE_BOX     box in (psi = ln tan phi, theta, zeta = ln x3)
 *   chart 3 EDGE_BOX   box in (tau = ln r, theta, x3)
 *   chart 4 VTX_PATCH  planar patch (patch row) projected to the sphere, chi in box[4:6]
 *   chart 5 COLUMN     blend between a sphere patch (radius patch[9]) and the plane
 *                      z_local = 1, t in box[4:6]
 * x = origin + frame * x_local (frame row-major 3x3).
 * region: 0 regular, 1 vertex, 2 vertex-edge, 3 edge neighbourhood.
 * kind: 0 real element (n^3 unknowns), 1 corner constant, 2 corner polynomial
 *       along lam direction cdir (n unknowns), unknowns at corner offset cdof.
 * Faces f = 2d + s are lam_d = -1 (s = 0) or +1 (s = 1); face coordinates
 * are the other two lam's in increasing order; orient bit0 swaps them,
 * bit1/bit2 negate the first/second, mapping this side's face coordinates to
 * the neighbour's.  bc: 0 interior (nbr, nbr_face, orient valid),
 * 1 Dirichlet, 2 skipped (infinite measure in modified coordinates),
 * 3 Neumann. */
typedef struct {
    int32_t W;                /* polynomial degree per direction, 1 <= W <= 12 */
    int32_t nelem;            /* elements, real and corner */
    int32_t n_corner_dof;
    const int32_t* region;    /* [nelem] */
    const int32_t* kind;      /* [nelem] */
    const int32_t* chart;     /* [nelem] */
    const double* frame;      /* [nelem][3][3] */
    const double* mframe;     /* [nelem][3][3] frame of the modified coordinates of the
                                 neighbourhood (vertex region: spherical frame whose poles
                                 lie outside the element; equals frame elsewhere) */
    const double* origin;     /* [nelem][3] */
    const double* box;        /* [nelem][6] lo1,hi1,lo2,hi2,lo3,hi3 */
    const double* patch;      /* [nelem][12] */
    const int32_t* nbr;       /* [nelem][6] */
    const int32_t* nbr_face;  /* [nelem][6] */
    const int32_t* orient;    /* [nelem][6] */
    const int32_t* bc;        /* [nelem][6] */
    const int32_t* cdof;      /* [nelem] */
    const int32_t* cdir;      /* [nelem] */
} sem_mesh;

typedef struct {
    int32_t iterations;       /* PCG iterations done (inner iterations summed for mixed) */
    int32_t outer;            /* refinement steps (mixed precision), 1 for FP64 */
    double rel_residual;      /* final ||b - X u||_2 / ||b||_2 (recursively updated for FP64) */
    int32_t status;           /* sem_status of the solve */
} sem_pcg_info;

typedef struct sem_ctx sem_ctx;

/* Builds all operator data for the mesh and copies it to the current device
 * (synchronous).  Geometry, coefficient fields of the transformed operators
 * (eq 2.22, 2.28, 2.35), face weights (eq 2.17b, 2.18, 2.25, 2.27, 2.34) and
 * the separable preconditioner bases (eq 5.15-5.20, 5.37-5.42).
 * Errors: SEM_EINVAL for an inconsistent or non-conforming mesh. */
sem_status sem_setup(const sem_mesh* mesh, void* stream, sem_ctx** out);
void sem_destroy(sem_ctx* ctx);
const char* sem_last_error(void);

int64_t sem_ndof(const sem_ctx* ctx);
int64_t sem_num_real_elements(const sem_ctx* ctx);

/* Data points.  The caller evaluates f (volume) and g, grad g (Dirichlet
 * faces) at these physical points and hands the values to sem_set_data.
 *   volume points:    [E_real][(2W+1)^3][3], GLL points of each real element
 *   Dirichlet points: [n_dirichlet_faces][(2W+1)^2][3] */
int64_t sem_num_volume_points(const sem_ctx* ctx);
int64_t sem_num_dirichlet_points(const sem_ctx* ctx);
sem_status sem_volume_points(const sem_ctx* ctx, double* xyz_host);
sem_status sem_dirichlet_points(const sem_ctx* ctx, double* xyz_host);

/* Stores the data of the functional (eq 4.2-4.7): f at the volume points
 * (host [num_volume_points]), g and grad g at the Dirichlet points (host
 * [num_dirichlet_points] and [num_dirichlet_points][3]); either Dirichlet
 * pointer may be NULL when there are no Dirichlet points. */
sem_status sem_set_data(sem_ctx* ctx, const double* f_host, const double* g_host,
                        const double* gradg_host);

/* b = A^T M d, the data side of the normal equations (Sec. 5.3).
 * b_dev: device [ndof].  SEM_ENODATA before sem_set_data. */
sem_status sem_rhs(sem_ctx* ctx, double* b_dev, void* stream);

/* r = X u (homogeneous = 1) or r = X u - b (homogeneous = 0, b from the
 * stored data), X = A^T M A applied matrix-free (Sec. 5.3).
 * u_dev, r_dev: device [ndof], must not alias. */
sem_status sem_residual(sem_ctx* ctx, const double* u_dev, double* r_dev, int homogeneous,
                        void* stream);

/* sem_residual with the compute precision of the element and face
 * contractions chosen: SEM_FP64 (identical to sem_residual) or
 * SEM_MIXED_FP32 (operator data rounded to float, products and sums of the
 * volume and face kernels in float, u, r and the corner reduction in double;
 * relative error about 1e-6 of ||X|| ||u||).  The float operator data are
 * built on the first SEM_MIXED_FP32 call (device allocation, synchronous).
 * SEM_EINVAL for another precision value. */
sem_status sem_residual_prec(sem_ctx* ctx, const double* u_dev, double* r_dev, int homogeneous,
                             int precision, void* stream);

/* z = W^{-1} r for the block-diagonal preconditioner of Sec. 5.2
 * (eq 5.19, 5.30 per element; corner unknowns by their U-form blocks).
 * r_dev, z_dev: device [ndof]; may alias. */
sem_status sem_precond(sem_ctx* ctx, const double* r_dev, double* z_dev, void* stream);

/* Selects the block-diagonal preconditioner W used by sem_precond and the
 * PCG solvers.  SEM_PRECOND_SEPARABLE: the thesis's separable forms (eq 5.19,
 * 5.30), applied by fast diagonalisation.  SEM_PRECOND_ELEMENT_BLOCK: W is the
 * exact block diagonal of X itself (one n^3 x n^3 block per real element, one
 * dense block for the corner unknowns), a stronger block-Jacobi choice of the
 * same block-diagonal family; on the first call it is assembled by applying
 * X to unit vectors on chunks of the elements of one colour (no two sharing a
 * face term) and factored X_ee = L L^T (rocSOLVER, batched).  Blocks equal to
 * an earlier one to 1e-9 relative up to reversals of lambda axes (symmetry
 * images of an element) are stored once.  The solvers apply X_ee^{-1} to all
 * elements that share a stored block at once (z = B [r_1 .. r_16] on the FP64
 * matrix cores), from the full symmetric inverse in FP64, or rounded to float
 * on the mixed path when the rounded matrix is still positive definite (else
 * G^T (G r) with G = L^{-1} rounded to float, SPD by construction).  Memory:
 * per distinct block n^3 (n^3 + 63) x 12 bytes at most for the two inverses,
 * plus n^3 (n^3 + 1) x 4 for the float factor when the rounded inverse is not
 * positive definite.  While it is built: one chunk
 * of blocks, at most 2 GiB (the environment variable SEM_BLOCK_CHUNK_KB sets
 * another limit, in KiB; at least one block), plus the distinct blocks in
 * FP64, n^6 x 8 bytes each, until they are factored.  Synchronous on the
 * first ELEMENT_BLOCK call.  Errors: SEM_ENOMEM, SEM_EINVAL if a block is not
 * positive definite. */
sem_status sem_set_preconditioner(sem_ctx* ctx, int kind, void* stream);

/* PCG on X u = b (Ch. 5 intro, Ch. 6 intro): starts from the values in u_dev,
 * stops when ||r_k||_2 / ||b||_2 <= rtol on the recursively updated residual
 * or after maxit iterations.  b_dev, u_dev: device [ndof]; u_dev is
 * overwritten with the last iterate.  info may be NULL.  Returns SEM_OK,
 * SEM_ENOCONV (u holds the last iterate), SEM_EBREAKDOWN or SEM_ENAN.
 * The iteration runs on the device; 8 iterations at a time are one HIP graph
 * launch, after which the host reads the stop flag (work buffers for one
 * right-hand side are allocated on the first call and kept).  Synchronises
 * the stream. */
sem_status sem_pcg_solve(sem_ctx* ctx, const double* b_dev, double* u_dev, double rtol,
                         int maxit, sem_pcg_info* info, void* stream);

/* Mixed-precision PCG on X u = b with FP64 accuracy (the thesis solves in
 * double; the float operator is this library's addition).  The products
 * X p of the iteration use the SEM_MIXED_FP32 operator; vectors, inner
 * products, the preconditioner and u stay in double.  Whenever the recursive
 * relative residual has fallen by a factor 10 since the last replacement, or
 * meets rtol, one iteration recomputes r = b - X u with the FP64 operator
 * (residual replacement) and keeps the search direction, so the solve stops
 * only when the TRUE FP64 relative residual ||b - X u||_2 / ||b||_2 <= rtol.
 * If a replacement shows that the float iterations have stopped lowering
 * the true residual (or they stall), the remaining iterations use the FP64
 * operator and factor.  If then two FP64 replacements in a row do not lower
 * the true residual, rtol is below the attainable accuracy in double and the
 * solve returns SEM_ENOCONV with u holding the last iterate.
 * info->outer counts the replacements, info->iterations all iterations.
 * Arguments, errors and synchronisation as sem_pcg_solve. */
sem_status sem_pcg_solve_mixed(sem_ctx* ctx, const double* b_dev, double* u_dev, double rtol,
                               int maxit, sem_pcg_info* info, void* stream);

/* Source of the adjoint workload: f(x) = sum_{a,b,c < deg} theta[a + deg (b +
 * deg c)] P_a(x1) P_b(x2) P_c(x3) (Legendre polynomials in the physical
 * coordinates) with homogeneous Dirichlet data g = 0; replaces the data of
 * sem_set_data.  theta_dev: device [deg^3]; 1 <= deg <= 12.  The right-hand
 * side is then b(theta) = A^T M d(theta), linear in theta (Sec. 5.3), with
 * d_q = s_q f(x_q) at the volume points. */
sem_status sem_set_source_legendre(sem_ctx* ctx, int deg, const double* theta_dev, void* stream);

/* Source of the batched workload: f(x) = sum_k a_k cos(pi (kappa_k . x) +
 * phi_k) with homogeneous Dirichlet data; replaces the data of sem_set_data.
 * coef_dev: device [nmodes][5] = (a, kappa_1, kappa_2, kappa_3, phi). */
sem_status sem_set_source_fourier(sem_ctx* ctx, int nmodes, const double* coef_dev, void* stream);

/* Adjoint of theta -> b(theta): grad[k] = d (lambda^T b(theta)) / d theta_k
 * = sum_q s_q z_q(lambda) P_a P_b P_c, with z_q(lambda) the weighted pointwise
 * PDE residual of lambda (homogeneous) at the volume points.  With lambda =
 * X^{-1} dL/du (X is symmetric) this is the gradient of a loss L(u(theta)),
 * u = X^{-1} b(theta).  lambda_dev: device [ndof]; grad_dev: device [deg^3].
 * Per-element partial sums, then a fixed-order sum over elements. */
sem_status sem_source_adjoint(sem_ctx* ctx, int deg, const double* lambda_dev, double* grad_dev,
                              void* stream);

/* Many independent PCG solves in one: for every context c (one mesh and
 * degree; contexts may differ in W) nrhs[c] right-hand sides b[c] (device
 * [nrhs[c]][ndof_c], one vector after the other) and initial guesses /
 * solutions u[c] (same layout).  Each right-hand side runs the FP64 PCG of
 * sem_pcg_solve with its own scalars and stopping test; every kernel of an
 * iteration covers all right-hand sides of its context (item-major, the
 * right-hand side index fastest, so neighbouring workgroups share the
 * element's coefficients and block inverse in cache).  `check` iterations of
 * all contexts are captured once into a HIP graph, which is replayed until
 * every right-hand side has stopped (the host reads the stop flags between
 * replays).  Uses each context's current preconditioner.  infos: host
 * [sum nrhs] in context order.  Work buffers of nrhs[c] right-hand sides are
 * allocated on first use and kept by the context.  Synchronises the stream.
 * precision SEM_MIXED_FP32: the iterations run the float operator and float
 * element blocks; between graph replays the residual replacement rule of
 * sem_pcg_solve_mixed is applied per context (one eager iteration for all its
 * right-hand sides whose residual is recomputed in FP64) and a stalling
 * context continues with its FP64 operator; every right-hand side stops on
 * its true FP64 residual (or at the attainable accuracy: SEM_ENOCONV).
 * infos[].outer then counts the replacements.
 * Returns the first failing status (SEM_ENOCONV, ...) when some solve did not
 * converge; infos say which. */
sem_status sem_pcg_solve_batch(int nctx, sem_ctx* const* ctxs, const int* nrhs, const double* const* b_dev,
                               double* const* u_dev, double rtol, int maxit, int check, int precision,
                               sem_pcg_info* infos, void* stream);

/* Relative broken H^1 error ||u - u_ex||_{H^1} / ||u_ex||_{H^1} (Ch. 6 intro)
 * over the real elements with the (W+6)-point Gauss rule per direction.
 * Error points: [E_real][(W+6)^3][3]; uex_host [num_error_points],
 * graduex_host [num_error_points][3].  Synchronises. */
int64_t sem_num_error_points(const sem_ctx* ctx);
sem_status sem_error_points(const sem_ctx* ctx, double* xyz_host);
sem_status sem_error(sem_ctx* ctx, const double* u_dev, const double* uex_host,
                     const double* graduex_host, double* rel_h1, void* stream);

/* The norm weights of the face terms (eq 2.17b, 2.18, 2.25, 2.27, 2.34):
 * host [num_face_terms][4][3], per quantity (value, then up to three
 * derivatives) the factors (alpha, beta, gamma) of Om x Om, K x Om, Om x K on
 * the face grid, as sem_setup derives them.  sem_set_face_weights replaces
 * them (for experiments with the functional's weighting); the operator stays
 * symmetric, and positive definite while the weights stay positive.  An
 * element-block preconditioner built before is dropped (the separable form
 * takes over until it is built again). */
int64_t sem_num_face_terms(const sem_ctx* ctx);
sem_status sem_face_weights(const sem_ctx* ctx, double* w_host);
sem_status sem_set_face_weights(sem_ctx* ctx, const double* w_host);

/* Neumann faces (mesh bc code 3; eq 2.16 / 4.2, 4.3, 4.5, 4.7): the term
 * ||w (du/dnu - h)||^2 in the face's norm (the 1/2-norm of eq 2.17b on the
 * master square, R-weighted in the vertex region; ||| . ||| of eq 2.27 / 2.34
 * in the vertex-edge and edge regions), with du/dnu the outward normal
 * derivative (the Laplacian's conormal) and w the thesis's factor of the
 * datum (1; e^chi / sin phi; e^zeta e^psi = r; e^tau = r).  Points
 * [num_neumann_points][3] and outward unit normals (host arrays, face by face
 * in face-term order); h_host [num_neumann_points] sets the data (zero until
 * set).  Neumann faces and sem_set_coefficients exclude each other (the
 * conormal of a general operator needs a at the face points). */
int64_t sem_num_neumann_points(const sem_ctx* ctx);
sem_status sem_neumann_points(const sem_ctx* ctx, double* xyz_host, double* normal_host);
sem_status sem_set_neumann_data(sem_ctx* ctx, const double* h_host);

/* General operator (eq 2.2): L u = -sum_ij a_ij u_{x_i x_j} + sum_j beta_j
 * u_{x_j} + c u, i.e. eq 2.2's divergence form with beta_j = b_j -
 * sum_i d a_ij / d x_i, not self-adjoint in general (the normal equations
 * X = A^T M A stay symmetric).  Host arrays at the volume points
 * (sem_volume_points): a [num_volume_points][6] = a11 a22 a33 a12 a13 a23
 * (symmetric, positive definite at every point, SEM_EINVAL otherwise),
 * beta [num_volume_points][3], c [num_volume_points]; NULL leaves the
 * Laplacian's value (a = I, beta = 0, c = 0).  Rebuilds the volume
 * coefficient fields (the weighted operator of eq 2.22, 2.28, 2.35 with
 * the chain rule through each element map) and uploads them (synchronous).
 * sem_set_data's f and g keep their meaning (call sem_rhs again).  An
 * element-block preconditioner built before is dropped: the context falls
 * back to the separable form until sem_set_preconditioner builds the blocks
 * of the new operator. */
sem_status sem_set_coefficients(sem_ctx* ctx, const double* a_host, const double* beta_host,
                                const double* c_host);

/* Layer-graded degrees (Sec. 2.3: W_l = [mu_1 i], W_q, V_q = [mu_2 k] per
 * geometric layer).  deg_host [E][3] (mesh element order): the polynomial
 * degree of each real element along lambda_1, lambda_2, lambda_3, each in
 * 1..W (SEM_EINVAL otherwise); entries of corner elements are ignored
 * (corner functions keep degree W); NULL restores degree W everywhere.
 * The discretisation becomes the minimiser of the same functional over the
 * graded space (the functions of those degrees, integrated with the mesh's
 * (2W+1)-point rule): vectors keep the layout of sem_ndof, a vector of the
 * graded space holding on each element the values of a polynomial of the
 * element's degrees.  From then on sem_rhs returns Q b, sem_residual Q r and
 * the PCG solvers solve Q X Q u = Q b in that space (Q: the orthogonal
 * projector onto it, per element the Kronecker product of the 1D
 * projectors onto the degree-w polynomials in the values at the GLL nodes);
 * right-hand sides given to the solvers and vectors given to sem_residual
 * must lie in the graded space (sem_project maps a vector there).  The
 * separable preconditioner becomes P (P^T C P)^-1 P^T on each element (P
 * the embedding of the element's degrees); an element-block preconditioner
 * built before is dropped (back to the separable form until
 * sem_set_preconditioner builds (Q X_ee Q + s (I - Q))^-1 per element, s =
 * tr X_ee / n^3).
 * Synchronous. */
sem_status sem_set_degrees(sem_ctx* ctx, const int* deg_host);
/* Unknowns of the graded space: sum over real elements of prod (w_d + 1),
 * plus the corner unknowns (sem_ndof when ungraded); -1 for NULL. */
int64_t sem_graded_ndof(const sem_ctx* ctx);
/* u <- Q u in place on the real elements of degree below W (device
 * [ndof]; the corner unknowns and ungraded elements unchanged).
 * Asynchronous on the stream. */
sem_status sem_project(sem_ctx* ctx, double* u_dev, void* stream);

/* Conforming correction of a solution (Appendix C.1, proof of Lemma 3.3.1;
 * the remark after Thm 4.3.2): uc = u + nu on every real element, nu the sum
 * over its interior faces of (1 -/+ lam_d)/2 times half the jump of u across
 * the face (the neighbour's value minus the element's own, at the face
 * nodes), the whole jump when the neighbour is a corner element (which the
 * correction leaves unchanged, as it does the corner unknowns).  Faces on the
 * boundary are not corrected.  u_dev, uc_dev: device [ndof], distinct.  Jumps
 * confined to the inside of faces are removed exactly; the result has the
 * layout of u.  Asynchronous on the stream. */
sem_status sem_conforming_correction(sem_ctx* ctx, const double* u_dev, double* uc_dev, void* stream);

/* sem_error for callers that cannot allocate memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * error with the exact solution already on the device, uex_dev
 * [num_error_points] and graduex_dev [num_error_points][3] (the caller's
 * device memory), and no allocation of any kind: its per-element partial sums
 * live in a fixed scratch array of the library, one copy per device, of
 * 2^19 doubles (4 MiB), which holds 2 E_real + 2 values, so contexts with
 * more than 262,143 real elements are rejected with SEM_EINVAL.  The
 * context's device must be current (SEM_EINVAL otherwise).  Calls that
 * overlap in time on one device race on that scratch.  Synchronises the
 * stream; *rel_h1 equals sem_error's result. */
sem_status sem_error_noalloc(sem_ctx* ctx, const double* u_dev, const double* uex_dev,
                             const double* graduex_dev, double* rel_h1, void* stream);

/* Autotuner of the element kernel's tile: the kernel stages its sum-factorised
 * contractions through LDS one slab of lam1-indices at a time (the slab width
 * sets its LDS per workgroup and so how many workgroups share a compute unit),
 * and its pointwise stage gives each column of a slab to 1 or 4 lanes.  Three
 * candidates are compiled per degree and precision: the whole element or the
 * widest slab under 155 KB, one lane per column; the widest slab under 78 KB,
 * one lane; that first slab capped to 128 columns with 4 lanes per column
 * (workgroups of 512).
 * This times each on the context's own mesh (reps launches, HIP events on the
 * stream, after one warm-up launch) and selects the fastest for all later
 * calls of that precision.  tile_out (host [4], may be NULL): selected index
 * and the three candidates' slab widths; ms_out (host [3], may be NULL): mean
 * ms per launch, -1 for a candidate identical to the previous one.  Results
 * agree to rounding across tiles (the forward sums are split differently) and
 * are reproducible for each.  Overwrites the context's work vectors.
 * Synchronises. */
sem_status sem_autotune(sem_ctx* ctx, int precision, int reps, int* tile_out, double* ms_out, void* stream);

/* Selects tile candidate 0, 1 or 2 of sem_autotune directly. */
sem_status sem_set_tile(sem_ctx* ctx, int precision, int tile);

/* Work counts of the operator, for roofline accounting: [0] real elements,
 * [1] all elements (with corners), [2] sum over real elements of the active
 * coefficient fields of the volume operator, [3] real elements whose
 * operator has mixed or first-derivative terms, [4] active face slots
 * (element faces that carry a face term), [5] face terms, [6] doubles of face
 * coefficient data, [7] unknowns, [8] bytes of element-block data one FP64
 * preconditioner apply reads and [9] one mixed-precision apply reads: each
 * distinct stored inverse once, n^3 x n^3 doubles or floats (the float
 * triangular-factor fallback: its packed triangle twice); both 0 with the
 * separable preconditioner.  counts: host int64 [10]. */
sem_status sem_work_counts(const sem_ctx* ctx, int64_t* counts);

/* Measurement hook: runs the kernels of one operator apply and preconditioner
 * solve in iteration order, `reps` times, on `stream` with the input vector
 * u_dev (device [ndof]), and returns in ms_out (host [4]) the mean duration
 * per launch measured with HIP events between the launches on that stream
 * (each launch sees the caches as the previous kernel of the iteration
 * leaves them): [0] element volume kernel, [1] face kernel, [2] gather
 * kernel, [3] preconditioner apply.  precision selects the kernels as the solver of
 * that precision runs them (SEM_FP64 or SEM_MIXED_FP32: float operator data,
 * and with the element-block preconditioner the float inverse; vectors are
 * FP64 in both).  Overwrites the context's work vectors.  Synchronises the
 * stream. */
sem_status sem_kernel_times(sem_ctx* ctx, const double* u_dev, int reps, int precision,
                            double* ms_out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SEM_H */
