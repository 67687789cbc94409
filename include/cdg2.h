/*
 * cdg2.h -- C ABI of the MI355X (gfx950) CDG2 operator library for the
 * six-species atherosclerotic-plaque model.
 *
 * Model (Section 2, eqs. (1)-(6) and their vector form): for
 * U = (n1, n2, n3, c1, c2, c3),  dU/dt = -div(F(U) - A grad U) + S(U), with the
 * chemotactic fluxes F_n1 = n1 w1, F_n2 = n2 w2, the tactic sensitivity
 * chi(x, y, a, b) = a x / (y + b), constant diffusivities A = diag(mu, nu) and
 * the reaction terms S; inflow boundary conditions of eqs. (7)-(9) on Gamma1
 * (low end of the wall axis) and Gamma2 (high end).
 *
 * Discretisation (Section 3.1): discontinuous Galerkin on a uniform Cartesian
 * grid of [0,1]^dim with the orthonormal tensor Legendre basis
 * phi_i(xi) = sqrt(2i+1) P_i(2 xi - 1) per direction (so M = |K| I), p+1
 * Gauss-Legendre points per direction, local Lax-Friedrichs convective flux,
 * CDG2 diffusion flux 2 chi_e (A r_e([[U]]))|_{K^-_e} with lift factor
 * chi_e = N/2 (2 for quads, 3 for hexes) and K^-_e the low-coordinate
 * neighbour of each face.  Time: f(U) = M^{-1} L_h(U) (Section 3.2), advanced by
 * SSP-RK3 in Shu-Osher form (cdg2_rk_step, the fused explicit path) or by the
 * implicit DIRK integrator of Section 3.2 (cdg2_dirk_step).
 *
 * DOF layout (all state buffers): U[s][e][m], s = species in the order above,
 * e = ix + nx (iy + ny iz), m = i + (p+1) (j + (p+1) k) (x mode fastest);
 * cdg2_num_dofs() = 6 * E * (p+1)^dim elements of float64 (CDG2_FP64) or
 * float32 (CDG2_FP32).
 *
 * Ownership: every state pointer is a DEVICE pointer to a caller-owned,
 * contiguous buffer on the handle's device; in 3D the buffers passed to the
 * operator and RK entry points must be 16-byte aligned (CDG2_EINVAL otherwise;
 * device allocations are).  The library owns its tables, two
 * stage buffers and small flag buffers; it copies the config at create.
 *
 * Asynchrony: calls that take device pointers enqueue work on the stream set by
 * cdg2_set_stream (default: the null stream) and return; launch errors are
 * returned at once, device-side conditions (non-finite values, a non-positive
 * chemotaxis denominator) are returned by cdg2_sync.  Handles are not
 * thread-safe.  No C++ exception crosses this boundary.
 *
 * Errors: 0 = CDG2_OK, negative values below; cdg2_last_error() returns a
 * thread-local message for the last failing call.
 */
#ifndef CDG2_H
#define CDG2_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CDG2_OK = 0,
  CDG2_EINVAL = -1,     /* invalid argument or configuration */
  CDG2_ENOMEM = -2,     /* device allocation failed */
  CDG2_EHIP = -3,       /* HIP runtime error (message in cdg2_last_error) */
  CDG2_ENONFINITE = -4, /* a NaN/Inf was written to a state buffer */
  CDG2_EDOMAIN = -5,    /* c + chi^th <= 0 met in a chemotactic sensitivity */
  CDG2_ENOCONV = -6     /* the implicit integrator's Newton iteration did not converge */
};

enum { CDG2_FP64 = 0, CDG2_FP32 = 1 };

/* LLF dissipation rows: all six species (default) or only n1, n2. */
enum { CDG2_LLF_ALL = 0, CDG2_LLF_CELLS = 1 };

/* Diffusion flux (Section 3.1; the others are the paper's comparison fluxes of
 * Section 4).  All share the consistency term {A grad U}:[[phi]]; they differ in
 * the stabilisation and the sign of the symmetry term {A grad phi}:[[U]]:
 *   CDG2: 2 chi_e (A r_e([[U]]))|_{K^-}, chi_e = N/2 (N = 2 dim faces per cell);
 *   BR2:  eta {A r_e([[U]])} (average of the liftings on both neighbours);
 *   IP:   eta A (p+1)^2 / h [[U]] (symmetric interior penalty);
 *   BO:   Baumann-Oden: no stabilisation, symmetry term with the opposite sign;
 *   CDG:  compact DG (the paper names it without details; read as Peraire and
 *         Persson's method with the switch selecting K^-): the flux and the
 *         symmetry term are one-sided, A (grad U^- + r~([[U]])).n^- with r~ the
 *         lifting of the whole jump onto K^- only (no average).
 * On uniform Cartesian cells the lifting has the same trace from both sides
 * (-(p+1)^2 / (2h) [[U]]), so BR2 with eta = N and IP with eta = dim coincide
 * with CDG2, and CDG is the one-sided form with penalty (p+1)^2 a / h.
 * flux_eta = 0 selects eta = 2 dim for BR2 and IP. */
enum { CDG2_FLUX_CDG2 = 0, CDG2_FLUX_BR2 = 1, CDG2_FLUX_IP = 2, CDG2_FLUX_BO = 3, CDG2_FLUX_CDG = 4 };

/* Coefficients of Section 2 (the paper gives symbols only).  The first 21 are
 * the differentiable coefficients in this order: mu1..3, nu1..3 (motilities),
 * chi0_{11,13,21,22}, chith_{11,13,21,22} (tactic sensitivities; 22 is the
 * n2-by-n1 term of eq. (2)), d1, d2 (death rates), gamma (:= F < 0, constant),
 * alpha1, alpha2 (neutralisation), f1 (production, constant), k (oxidation).
 * The last five enter only the inflow conditions of eqs. (7)-(9): beta1,
 * beta2, sigma, and the Heaviside thresholds c1*, c1**. */
typedef struct {
  double mu[3], nu[3];
  double chi0[4], chith[4];
  double d1, d2, gamma, alpha1, alpha2, f1, k;
  double beta1, beta2, sigma, c1_star, c1_sstar;
} cdg2_coeffs;

#define CDG2_NCOEFF 26
#define CDG2_NDIFF 21

typedef struct {
  int dim;              /* 2 or 3 */
  int n[3];             /* cells per axis, each >= 2 (n[2] ignored for dim 2) */
  int order;            /* p: 1..4 in 2D, 1..3 in 3D */
  int precision;        /* CDG2_FP64 | CDG2_FP32 */
  int wall_axis;        /* axis whose low end is Gamma1 and high end Gamma2
                           (dim-1 normally); -1 = fully periodic */
  int llf_mode;         /* CDG2_LLF_ALL | CDG2_LLF_CELLS */
  double gamma1_in[2];  /* Gamma_{1,in} = [g0, g1] on the first tangential axis */
  cdg2_coeffs coeffs;
  int diff_flux;        /* CDG2_FLUX_* (0: CDG2) */
  int reserved;         /* 0 */
  double flux_eta;      /* penalty parameter of BR2 / IP (>= 0; 0: default) */
} cdg2_config;

typedef struct cdg2_handle cdg2_handle;

/* Create a handle for one grid / order / coefficient set (Sections 2, 3.1).
 * Validates cfg (CDG2_EINVAL), builds the 1D tables on the host and allocates
 * the stage buffers on the current device (CDG2_ENOMEM).  No kernel launch. */
int cdg2_create(const cdg2_config* cfg, cdg2_handle** out);

/* Release everything the handle owns; NULL is accepted. */
int cdg2_destroy(cdg2_handle* h);

/* Stream for all later calls (a hipStream_t, e.g. torch's current stream). */
int cdg2_set_stream(cdg2_handle* h, void* hip_stream);

/* Replace the coefficient set (same grid and order). */
int cdg2_set_coeffs(cdg2_handle* h, const cdg2_coeffs* c);

/* Number of state entries, 6 * E * (p+1)^dim. */
size_t cdg2_num_dofs(const cdg2_handle* h);

/* dUdt = M^{-1} L_h(U) (Section 3.2: the ODE right-hand side, not the
 * pre-mass residual).  U and dUdt: device buffers of cdg2_num_dofs entries;
 * they must not overlap (CDG2_EINVAL). */
int cdg2_apply_operator(cdg2_handle* h, const void* U, void* dUdt);

/* nsteps SSP-RK3 steps of size dt, in place on U:
 *   U1 = U + dt f(U);  U2 = 3/4 U + 1/4 (U1 + dt f(U1));
 *   U <- 1/3 U + 2/3 (U2 + dt f(U2)).
 * Each stage is one fused launch (operator + stage combination); the two
 * intermediate states live in the handle's stage buffers (on 3D grids with
 * p <= 2 as values at the Gauss points of each cell, which span the same space:
 * the same discrete step up to rounding; U itself stays modes). */
int cdg2_rk_step(cdg2_handle* h, void* U, double dt, int nsteps);

/* Size of the library's static scratch memory per GPU (64 MiB), which holds the
 * two intermediate states of cdg2_rk_step_noalloc. */
#define CDG2_SCRATCH_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory during the call (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same nsteps SSP-RK3 steps as cdg2_rk_step, with the same kernels and results,
 * but the two intermediate states live in a static device array of
 * CDG2_SCRATCH_BYTES per GPU (set up at cdg2_create) instead of the handle's
 * stage buffers.  Allocates nothing (no hipMalloc / hipFree, no allocating
 * library call).  Limit: each state, rounded up to 256 bytes, must fit in half
 * of the array, i.e. cdg2_num_dofs * (8 for FP64, 4 for FP32) <= 32 MiB
 * (4,194,304 FP64 entries, e.g. 256x256 Q2 or 128x128 Q4); larger handles get
 * CDG2_EINVAL.  Every handle on a GPU shares that GPU's array, which keeps the
 * last call's intermediate states: calls that overlap in time on one GPU (other
 * streams or threads) race and must be serialised by the caller.  U: device
 * buffer on the handle's device, updated in place; asynchronous like
 * cdg2_rk_step. */
int cdg2_rk_step_noalloc(cdg2_handle* h, void* U, double dt, int nsteps);

/* CFL time step for state U (synchronous: returns after the device work):
 *   dt = cfl / (rho_hat a_max sum_a h_a^-2 / 2.51 + (2p+1) lam_max sum_a h_a^-1
 *               + r_max / 2.51),
 * with rho_hat the spectral radius of the 1D diffusion operator (a = h = 1),
 * lam_max the largest chemotactic velocity component and
 * r_max = d1 + d2 + |gamma| + k + alpha1 max n1 + alpha2 max n2, both over the
 * volume quadrature points. */
int cdg2_max_dt(cdg2_handle* h, const void* U, double cfl, double* dt);

/* Wait for the handle's stream and report device-side conditions raised since
 * the last cdg2_sync (CDG2_ENONFINITE, CDG2_EDOMAIN); clears them. */
int cdg2_sync(cdg2_handle* h);

/* Spectral constant rho_hat used by cdg2_max_dt (host-computed at create). */
double cdg2_rho_hat(const cdg2_handle* h);

/* Controls of the implicit integrator (cdg2_dirk_step). */
typedef struct {
  int order;            /* SDIRK order: 2, 3 or 4 */
  int max_newton;       /* Newton steps per stage, >= 1 */
  int krylov_dim;       /* GMRES iterations per Newton step, 1..64 */
  double newton_rtol;   /* stage solved when ||G|| <= newton_rtol (||X|| + dt a_ii ||f(X)||) */
  double krylov_rtol;   /* GMRES stops when its residual <= krylov_rtol ||G|| */
} cdg2_implicit_opts;

typedef struct {
  int newton_iters;     /* Newton steps over all stages */
  int krylov_iters;     /* GMRES iterations over all Newton steps */
  int converged;        /* 1 when every stage met newton_rtol */
  int pad;
  double max_residual;  /* largest final ||G|| / (||X|| + dt a_ii ||f(X)||) over the stages */
} cdg2_implicit_stats;

/* One implicit step of size dt (Section 3.2: a DIRK method of order 2, 3 or 4
 * whose stages are solved by a Jacobian-free Newton-Krylov method with GMRES on
 * the matrix-free operator).  The schemes are L-stable, stiffly accurate SDIRK
 * methods: order 2 Alexander's two-stage scheme (gamma = 1 - 1/sqrt(2)), order 3
 * Alexander's three-stage scheme (gamma = 0.43586652150845899942), order 4 the
 * five-stage scheme of Hairer and Wanner (gamma = 1/4).  For each stage i the
 * stage value X solves G(X) = X - dt a_ii f(X) - rhs_i = 0 with
 * rhs_i = U^n + dt sum_{j<i} a_ij K_j; each Newton step solves
 * (I - dt a_ii J(X)) d = -G by GMRES (no preconditioner, classical Gram-Schmidt
 * with a second pass when the first cancels most of the vector, Givens rotations) with the Jacobian-vector product
 * J v = (f(X + eps v) - f(X)) / eps, eps = sqrt(DBL_EPSILON) (1 + ||X||) for
 * ||v|| = 1.  K_i = (X - rhs_i) / (dt a_ii) and U^{n+1} = U^n + dt sum b_i K_i.
 * Norms are 2-norms over all entries, reduced in a fixed order (deterministic).
 * U: device buffer (FP64 handles only), updated in place on success and left
 * unchanged otherwise.  opts: NULL for defaults (order 3, max_newton 10,
 * krylov_dim 30, newton_rtol 1e-10, krylov_rtol 1e-3).  stats: NULL or filled.
 * Returns CDG2_ENOCONV when a stage misses newton_rtol within max_newton steps.
 * The call waits for the device (the Krylov scalars live on the host); the
 * library allocates its workspace ((krylov_dim + 13) state vectors) on first
 * use and keeps it until cdg2_destroy. */
int cdg2_dirk_step(cdg2_handle* h, void* U, double dt, const cdg2_implicit_opts* opts,
                   cdg2_implicit_stats* stats);

/* Adjoint of the operator (the transposed Jacobian J = d f / d U of f = M^{-1}
 * L_h, Sections 3.1-3.2): JTw = J(U)^T w.  U, w, JTw: device buffers of
 * cdg2_num_dofs entries; JTw must not overlap U or w.  If dtheta is not NULL it
 * is a HOST array of CDG2_NDIFF doubles that receives d (w . f(U)) / d theta_j
 * for the 21 differentiable coefficients (order of cdg2_coeffs); the call then
 * waits for the device.  Non-smooth points: d|x|/dx = sign(x) (0 at 0), the max
 * of the LLF speed takes the first maximiser, the inflow Heaviside has
 * derivative 0.  Parameter sums are reduced in a fixed order (deterministic).
 * Central symmetric diffusion fluxes only (CDG2, BR2, IP): CDG2_EINVAL for
 * Baumann-Oden and CDG, as for the other adjoint entry points. */
int cdg2_apply_adjoint(cdg2_handle* h, const void* U, const void* w, void* JTw, double* dtheta);

/* Discrete adjoint of one SSP-RK3 step of size dt started from U_n: given
 * lam_np1 = dL/dU^{n+1}, writes lam_n = dL/dU^n:
 *   lam2 = 2/3 lam3 + 2/3 dt J(U2)^T lam3,  lam1 = 1/4 lam2 + 1/4 dt J(U1)^T lam2,
 *   lam_n = 1/3 lam3 + 3/4 lam2 + lam1 + dt J(U_n)^T lam1,
 * with U1, U2 recomputed from U_n into the stage buffers.  lam_n may alias
 * lam_np1 (in place) but not U_n.  If dtheta_acc (a DEVICE array of CDG2_NDIFF
 * doubles) is not NULL, 2/3 dt df(U2)/dtheta^T lam3 + 1/4 dt df(U1)/dtheta^T lam2
 * + dt df(U_n)/dtheta^T lam1 is ADDED to it in stream order (no host wait). */
int cdg2_rk_step_adjoint(cdg2_handle* h, const void* U_n, const void* lam_np1, void* lam_n, double dt,
                         double* dtheta_acc);

/* Discrete adjoint of nsteps SSP-RK3 steps of size dt started from U_start (one
 * checkpoint segment of a reverse sweep, Section 3.2 time stepping): recomputes
 * the segment forward once, keeping U^n, U1 and U2 of every step in a library
 * workspace (3 nsteps states, grown on demand with hipMalloc and kept until
 * cdg2_destroy), then applies the step adjoint of cdg2_rk_step_adjoint from the
 * last step to the first.  lam (device, cdg2_num_dofs entries) holds
 * dL/dU^{start+nsteps} on entry and dL/dU^{start} on return; it must not
 * overlap U_start.  dtheta_acc: NULL or a DEVICE array of CDG2_NDIFF doubles to
 * which the parameter derivatives of the whole segment are ADDED in stream order
 * (the per-workgroup partial sums of all 3 nsteps adjoint launches are summed
 * in a fixed order, then reduced once).  Same results as nsteps calls of
 * cdg2_rk_step_adjoint up to the order of the parameter sums; all work is
 * enqueued on the handle's stream without host waits.  nsteps >= 1. */
int cdg2_rk_adjoint_segment(cdg2_handle* h, const void* U_start, int nsteps, double dt, void* lam,
                            double* dtheta_acc);

/* ---- batched instances ---------------------------------------------------------
 * Many independent 2D instances (own grid, order 1..3, coefficients; FP64) are
 * advanced together; the schedule (cdg2_batch_set_schedule, or the autotuner)
 * decides the launches of an SSP-RK3 stage: one launch over the whole work list
 * of (instance, block of cells) items, either persistent (nwg > 0 workgroups
 * walk the list) or one workgroup per item (nwg = 0), or one launch per
 * polynomial order (order 2, side by side on forked streams).  cdg2_batch_rk
 * replays the stages of nsteps steps as one HIP graph.  The packed state holds
 * instance i at element offset cdg2_batch_offset(b, i), each in the DOF layout
 * above. */
typedef struct cdg2_batch cdg2_batch;

/* Copy count configs (2D, FP64, order <= 3; else CDG2_EINVAL), allocate the
 * descriptor table, work list and two packed stage buffers (CDG2_ENOMEM). */
int cdg2_batch_create(const cdg2_config* cfgs, int count, int autotune, cdg2_batch** out);
int cdg2_batch_destroy(cdg2_batch* b);
int cdg2_batch_set_stream(cdg2_batch* b, void* hip_stream);
/* Total entries of the packed state, and the element offset of instance i
 * ((size_t)-1 if i is out of range). */
size_t cdg2_batch_num_dofs(const cdg2_batch* b);
size_t cdg2_batch_offset(const cdg2_batch* b, int i);
/* Schedule: eb = cells per work item (16, 32 or 64; 6*eb threads per
 * workgroup), nwg = persistent workgroups (0: one per item), order = 0 items
 * sorted by decreasing cost, 1 in instance order, 2 one launch per polynomial
 * order (each with its own occupancy; nwg per launch).  Rebuilds the work list. */
int cdg2_batch_set_schedule(cdg2_batch* b, int eb, int nwg, int order);
/* Autotuner: times one SSP-RK3 step of every candidate schedule (eb in
 * {16, 32, 64}, nwg in {0, 1, 2, 4} x the number of compute units, order 0, 1
 * and 2) on a zero scratch state with dt = 0 (the kernels do their full work)
 * and keeps the fastest; writes eb, nwg, order and its time in ms into
 * best[0..3] if best is not NULL.  Allocates and frees the scratch state; waits
 * for the device.  cdg2_batch_create with autotune != 0 calls it. */
int cdg2_batch_autotune(cdg2_batch* b, double* best);
/* Run the stages as one captured HIP graph per (U_packed, offsets, nsteps)
 * (on != 0, the default) or launch them one by one (on = 0). */
int cdg2_batch_set_graph(cdg2_batch* b, int on);
/* nsteps SSP-RK3 steps of every instance, in place on the packed device buffer
 * U_packed, instance i with time step dts[i] (HOST array of count doubles).
 * offsets: NULL for the library's packing (cdg2_batch_offset), else a HOST
 * array of count element offsets placing the instances anywhere inside the
 * first cdg2_batch_num_dofs entries of U_packed without overlap (CDG2_EINVAL
 * otherwise).  Asynchronous; see cdg2_batch_sync. */
int cdg2_batch_rk(cdg2_batch* b, void* U_packed, const size_t* offsets, const double* dts, int nsteps);
/* Wait for the batch's stream; report non-finite / domain conditions. */
int cdg2_batch_sync(cdg2_batch* b);

/* ---- unstructured triangle meshes (P_k, k = 1, 2, 3; FP64) ----------------------
 *
 * The same six-species operator on a conforming triangle mesh (Section 3.1 on
 * simplices, the element type of the paper's own runs): full P_k per triangle
 * with an orthonormal basis (phi_0 = 1, so mode 0 is the element mean and
 * M_K = |K| I; the reference basis is the Gram-Schmidt orthonormalisation, for
 * the mean over the reference triangle (0,0), (1,0), (0,1), of the monomials
 * xi^a eta^b by total degree, then by the power of eta: 1, xi, eta, xi^2, xi eta,
 * eta^2, xi^3, ...), collapsed Gauss rules of k + 1
 * points per direction on the triangle and k + 1 Gauss points per edge, the LLF
 * and CDG2 fluxes (lifting on K^-: the smaller triangle of an edge, ties to the
 * lower element index; chi_e = 3/2) and the inflow fluxes of eqs. (7)-(9) on the
 * edges coded Gamma1 / Gamma2.  order: k = 1, 2 or 3 (else CDG2_EINVAL; Table 1
 * of Section 4 uses the linear, quadratic and cubic spaces).  State layout:
 * U[6][E][(k+1)(k+2)/2] doubles,
 * species n1, n2, n3, c1, c2, c3.
 *
 * Mesh (HOST arrays, copied at create):
 *   xy   [E][3][2]  vertex coordinates of each element, counter-clockwise (an
 *                   element that is not gives CDG2_EINVAL); periodic images are
 *                   given unwrapped, so each element is a proper triangle;
 *   nbr  [E][3]     element across edge j (from vertex j to vertex j+1), or -1
 *                   (Gamma1) / -2 (Gamma2);
 *   nbe  [E][3]     that edge's index in the neighbour (ignored on boundaries).
 * The tables must be reciprocal (nbr[nbr[e][j]][nbe[e][j]] == e and
 * nbe[nbr[e][j]][nbe[e][j]] == j), else CDG2_EINVAL.  Gamma_{1,in} is the set of
 * Gamma1 points with x in [gamma1_in_lo, gamma1_in_hi]. */
typedef struct cdg2_tri cdg2_tri;
int cdg2_tri_create(int order, int n_elements, const double* xy, const int* nbr, const int* nbe,
                    const cdg2_coeffs* coeffs, double gamma1_in_lo, double gamma1_in_hi, cdg2_tri** out);
int cdg2_tri_destroy(cdg2_tri* t);
/* Stream of all later launches (NULL: the default stream). */
int cdg2_tri_set_stream(cdg2_tri* t, void* stream);
/* 6 E (k+1)(k+2)/2. */
size_t cdg2_tri_num_dofs(const cdg2_tri* t);
/* F = M^-1 L_h(U) (DEVICE arrays of cdg2_tri_num_dofs doubles, not overlapping).
 * Asynchronous; see cdg2_tri_sync. */
int cdg2_tri_apply_operator(cdg2_tri* t, const double* U, double* F);
/* nsteps SSP-RK3 steps of size dt on U in place (DEVICE), the stage combination
 * fused into the operator kernel as for the Cartesian grids. */
int cdg2_tri_rk_step(cdg2_tri* t, double* U, double dt, int nsteps);
/* Wait for the stream; report non-finite / domain conditions (CDG2_ENONFINITE,
 * CDG2_EDOMAIN) raised by the launches since the last call. */
int cdg2_tri_sync(cdg2_tri* t);

/* ---- unstructured tetrahedral meshes (P_k, k = 1, 2, 3; FP64) -------------------
 *
 * The same six-species operator on a conforming tetrahedral mesh (Section 3.1 on
 * tetrahedra, the element of the paper's 3D runs, whose Table 2 uses cubic
 * elements): full P_k per tetrahedron with an orthonormal basis (phi_0 = 1,
 * M_K = |K| I; Gram-Schmidt, for the mean over the reference tetrahedron (0,0,0),
 * (1,0,0), (0,1,0), (0,0,1), of the monomials xi^a eta^b zeta^c ordered by total
 * degree, then by the power of zeta, then of eta, taken about the centroid);
 * volume integrals with a fully symmetric rule on the tetrahedron of degree 2k
 * (4, 14, 24 points; the 14-point rule has degree 5, which makes it unique),
 * face integrals with a fully symmetric triangle rule of degree 2k (3, 6, 12
 * points; the orbit parameters of both solve the moment equations) so that both
 * elements of a face use the same points; LLF and CDG2 fluxes (lifting on K^-:
 * the smaller tetrahedron of a face, ties to the lower element index;
 * chi_e = 2) and the inflow fluxes of eqs. (7)-(9) on the faces coded Gamma1 /
 * Gamma2.  State
 * layout: U[6][E][(k+1)(k+2)(k+3)/6] doubles, species n1, n2, n3, c1, c2, c3.
 *
 * Mesh (HOST arrays, copied at create):
 *   xyz  [E][4][3]  vertex coordinates of each element, positively oriented
 *                   (det[v1-v0, v2-v0, v3-v0] > 0, else CDG2_EINVAL); periodic
 *                   images are given unwrapped, so each element is a proper
 *                   tetrahedron;
 *   vid  [E][4]     mesh vertex ids (the same id for the same vertex in every
 *                   element and periodic image): they fix how the two elements
 *                   of a face see its points;
 *   nbr  [E][4]     element across local face f (the face opposite local vertex
 *                   f), or -1 (Gamma1) / -2 (Gamma2);
 *   nbe  [E][4]     that face's index in the neighbour (ignored on boundaries).
 * The tables must be reciprocal and a face and its neighbour's must carry the same
 * three vertex ids, else CDG2_EINVAL.  Gamma_{1,in} is the set of Gamma1 points
 * with x in [gamma1_in_lo, gamma1_in_hi]. */
typedef struct cdg2_tet cdg2_tet;
int cdg2_tet_create(int order, int n_elements, const double* xyz, const int* vid, const int* nbr, const int* nbe,
                    const cdg2_coeffs* coeffs, double gamma1_in_lo, double gamma1_in_hi, cdg2_tet** out);
int cdg2_tet_destroy(cdg2_tet* t);
/* Stream of all later launches (NULL: the default stream). */
int cdg2_tet_set_stream(cdg2_tet* t, void* stream);
/* 6 E (k+1)(k+2)(k+3)/6. */
size_t cdg2_tet_num_dofs(const cdg2_tet* t);
/* F = M^-1 L_h(U) (DEVICE arrays of cdg2_tet_num_dofs doubles, not overlapping).
 * Asynchronous; see cdg2_tet_sync. */
int cdg2_tet_apply_operator(cdg2_tet* t, const double* U, double* F);
/* nsteps SSP-RK3 steps of size dt on U in place (DEVICE), the stage combination
 * fused into the operator kernel. */
int cdg2_tet_rk_step(cdg2_tet* t, double* U, double dt, int nsteps);
/* Wait for the stream; report non-finite / domain conditions raised since the
 * last call. */
int cdg2_tet_sync(cdg2_tet* t);

/* Thread-local message of the last error. */
const char* cdg2_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CDG2_H */
