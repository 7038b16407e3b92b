/* fr.h - C ABI of the MI355X (gfx950) flux-reconstruction library libfr.so.
 *
 * The library evaluates the FR-DG spatial residual of a system of
 * conservation laws, dU/dt = R(U) (Saez-Mischlich, Sierra-Ausin, Gressier,
 * "The Spectral Difference Raviart-Thomas method for two and three-
 * dimensional elements and its connection with the Flux Reconstruction
 * formulation", section 2: FR method, eq. "flux_fr", eq. "divergence_fr"
 * and the method-of-lines form), its right-hand-side Jacobian dR/dU over the
 * face-neighbour stencil (section 3, eq. "jacobian_rhs"; section 4 for the
 * viscous two-layer stencil), exact Jacobian-vector products, and a
 * block-Jacobi preconditioner for implicit steps.
 *
 * Conventions
 *  - Element types, vertex and face numbering:
 *      quad [-1,1]^2: v0=(-1,-1) v1=(1,-1) v2=(1,1) v3=(-1,1);
 *                     faces 0:eta=-1 1:xi=+1 2:eta=+1 3:xi=-1
 *      hex  [-1,1]^3: v0..v3 as the quad at zeta=-1, v4..v7 at zeta=+1;
 *                     faces 0:zeta=-1 1:eta=-1 2:xi=+1 3:eta=+1 4:xi=-1 5:zeta=+1
 *      tri: v0=(-1,-1) v1=(1,-1) v2=(-1,1); faces 0:v0v1 1:v1v2 2:v2v0
 *      tet: v0=(-1,-1,-1) v1=(1,-1,-1) v2=(-1,1,-1) v3=(-1,-1,1);
 *           faces 0:v0v1v2 1:v0v1v3 2:v1v2v3 3:v0v2v3
 *      pri: the triangle times [-1,1]: v0..v2 at zeta=-1, v3..v5 at zeta=+1;
 *           faces 0:v0v1v2 1:v3v4v5 2:v0v1v4v3 3:v1v2v5v4 4:v2v0v3v5
 *    (tetrahedra and prisms: FR-DG, R and the JVP for every system; Jacobian
 *    blocks for tetrahedra where one element's assembly fits a workgroup's
 *    LDS, none for prisms)
 *  - Solution points of quads/hexes are the tensor Gauss-Legendre points,
 *    index rho = i + (p+1) j (+ (p+1)^2 k), xi_i ascending (appendix A);
 *    triangles and tetrahedra use the caller's points (tri_sol_pts,
 *    tet_sol_pts); prisms the triangle points times Gauss-Legendre points
 *    along the axis, rho = i + n_tri k.  Flux points: Gauss-Legendre on
 *    edges and quadrilateral faces, tri_sol_pts on triangular faces.
 *  - State vectors are element-major U[n][rho][alpha] (alpha = conserved
 *    variable), in the context precision.  DOF index = (n*Ns + rho)*Nv + alpha
 *    (mixed meshes: element n's entries follow those of elements 0..n-1,
 *    each with its own Ns).
 *  - Jacobian blocks: for element n, 1 + n_faces blocks of b x b, b = Ns*Nv:
 *    slot 0 = dR_n/dU_n, slot 1+f = dR_n/dU_{nbr(n,f)}.  Each block is stored
 *    column-major: blocks[((n*(1+nface) + slot)*b + c)*b + r] with
 *    r = rho*Nv + alpha (row of R_n), c = sigma*Nv + beta (column of U_k).
 *    For viscous systems the exact derivative includes every path through the
 *    neighbours' corrected gradients; blocks of the second face layer (which
 *    a viscous residual also depends on) are not returned.  fr_jvp is exact.
 *    Mixed meshes: element n's blocks start at fr_block_offsets()[n]: its
 *    self block (b_n x b_n), then one block per local face f (b_n x b_m, m
 *    the neighbour across f, b_m = Ns(m)*Nv), packed, each column-major.
 *  - Pointers named U, R, v, Jv, blocks, r, z are DEVICE pointers owned by
 *    the caller, aligned to the element size.  Mesh arrays are HOST pointers,
 *    copied during fr_ctx_create.
 *  - All compute calls are asynchronous on the context stream (the HIP stream
 *    given at creation; NULL = the default stream).  They allocate nothing.
 *
 * Errors: every function returns an fr_status; argument errors return before
 * anything is launched.  fr_last_error() returns a message for the last
 * failure of a context (or of creation when ctx is NULL).  No call aborts.
 */
#ifndef FR_H
#define FR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FR_OK = 0,
  FR_E_INVALID = -1,       /* bad argument or mesh */
  FR_E_UNSUPPORTED = -2,   /* valid but not provided (element/degree/precision) */
  FR_E_NOMEM = -3,         /* device allocation failed (creation only) */
  FR_E_DEVICE = -4,        /* HIP launch or runtime error */
  FR_E_SINGULAR = -5,      /* a diagonal block has a zero pivot */
  FR_E_NOT_CONVERGED = -6, /* Newton/GMRES did not reach its tolerance */
  FR_E_NONFINITE = -7      /* a NaN or infinity was stored to R, Jv or the Jacobian blocks */
} fr_status;

typedef enum { FR_QUAD = 0, FR_TRI = 1, FR_HEX = 2, FR_TET = 3, FR_PRI = 4 } fr_elem_type;
typedef enum { FR_ADVECTION = 0, FR_EULER = 1, FR_NAVIER_STOKES = 2 } fr_system;
typedef enum { FR_F64 = 0, FR_F32 = 1, FR_BF16 = 2 } fr_precision;
/* Spatial discretisation (quadrilaterals and hexahedra; triangles FR-DG only):
 * FR-DG (correction functions that recover nodal DG), FR-SDRT (FR with the
 * Raviart-Thomas flux basis of the external flux points as correction
 * functions: on each line, the Lagrange polynomial of degree p+1 on the SD
 * flux points {-1, Gauss-Legendre points of order p, +1}; section
 * "Connections between the SDRT and FR formalisms") and SDRT (section "SDRT
 * method": the flux evaluated at interior flux points, eq.
 * "divergence_sdrt"). */
typedef enum { FR_SCHEME_FR_DG = 0, FR_SCHEME_FR_SDRT = 1, FR_SCHEME_SDRT = 2 } fr_scheme;

/* Mesh: the paper's tessellation of the domain into conforming elements
 * (section 2) with its face-neighbour stencil (section 3).  All elements of
 * a context share one polynomial degree.  A 2-D mesh may mix triangles and
 * quadrilaterals (conforming: a triangle edge and a quadrilateral edge that
 * meet carry the same p+1 Gauss-Legendre flux points; the paper's hybrid
 * meshes and its quadrilateral-to-two-triangles subdivision, section 2); its
 * elements must be listed grouped by type, all elements of one type first,
 * else FR_E_INVALID.  Mixed meshes provide fr_rhs, fr_rhs_noalloc, fr_jvp,
 * fr_rk54 and (inviscid systems) fr_jacobian_blocks in FR-DG; the block
 * preconditioners, Newton-GMRES, the Fourier analysis and batches take
 * single-type contexts (FR_E_UNSUPPORTED). */
typedef struct {
  int32_t ndim;               /* 2 or 3 */
  int64_t n_elem;
  int32_t degree;             /* p in 1..4 */
  const int8_t* elem_type;    /* [n_elem] fr_elem_type */
  const double* elem_xyz;     /* [n_elem][max_vert][ndim] vertex coordinates, unwrapped per element */
  int32_t max_vert;
  const int64_t* nbr;         /* [n_elem][max_face] element across each local face (periodic: always set) */
  const int8_t* nbr_face;     /* [n_elem][max_face] local face index of that face in the neighbour */
  int32_t max_face;
  const double* tri_sol_pts;  /* triangles: [Ns][2] reference solution points; the same set is the
                                 flux-point set of the triangular faces of tetrahedra and prisms and
                                 the cross-section of the prisms' solution points; else NULL */
  const double* tet_sol_pts;  /* tetrahedra: [Ns][3] reference solution points; else NULL */
} fr_mesh_desc;

/* Field variables and fluxes (section 2; eq. "flux_advection",
 * "fluxOperatorEuler", "fluxOperatorNavierStokes"). */
typedef struct {
  int32_t system;             /* fr_system */
  int32_t nvars;              /* 1 (advection), ndim+2 (Euler / Navier-Stokes) */
  double adv_vel[3];          /* advection velocity */
  double gamma;               /* ratio of specific heats */
  double mu;                  /* dynamic viscosity (advection: diffusivity) */
  double prandtl;
  double ldg_beta;            /* common-solution / viscous-flux weight (eq. "common_var_for_grad");
                                 must be 0 (BR1), else fr_ctx_create returns FR_E_UNSUPPORTED */
  double ldg_penalty;         /* LDG penalty eta; must be 0 (BR1), else FR_E_UNSUPPORTED */
  int32_t scheme;             /* fr_scheme.  SDRT contexts provide fr_rhs, fr_jvp and the time steppers,
                                 not Jacobian blocks, block preconditioners or fr_rhs_noalloc
                                 (FR_E_UNSUPPORTED) */
} fr_physics;

/* Mixed meshes: n_sol, n_flux, n_face and block_dim are the largest over the
 * element types, n_dof the sum over the elements. */
typedef struct {
  int32_t ndim, n_sol, n_flux, n_face, nvars, block_dim;
  int64_t n_elem, n_dof;
  int64_t blocks_per_elem;    /* 1 + n_face */
  int32_t precision;          /* fr_precision of states */
} fr_info;

typedef struct fr_ctx_s fr_ctx;
typedef struct fr_precond_s fr_precond;

/* Creates a context: builds reference operators and geometry on the host,
 * uploads them and allocates the workspaces.  precision: FR_F64 or FR_F32
 * (state vectors and arithmetic).  stream: a hipStream_t or NULL. */
fr_status fr_ctx_create(const fr_mesh_desc* mesh, const fr_physics* phys, fr_precision precision, void* stream,
                        fr_ctx** out);
fr_status fr_ctx_destroy(fr_ctx* ctx);
fr_status fr_ctx_info(const fr_ctx* ctx, fr_info* info);
const char* fr_last_error(const fr_ctx* ctx);
/* Waits for the context stream and reports any asynchronous HIP error.
 * The residual and JVP kernels record every non-finite value they store in a
 * device status word of the context, and so does the Jacobian assembly: the
 * matrix-core path (FP32 contexts, quadrilaterals and hexahedra) records the
 * non-finite entries of the per-state flux-derivative tables its blocks are
 * sums of products of (with finite geometric factors, so a non-finite block
 * entry comes from one; an overflow of a product of finite values is not
 * caught), the other paths every non-finite block value.  fr_ctx_sync
 * returns FR_E_NONFINITE if any was recorded since the previous fr_ctx_sync
 * (the message names the outputs and the smallest element index) and clears
 * the word.  The hot calls return before their kernels finish, so they
 * cannot report it themselves. */
fr_status fr_ctx_sync(fr_ctx* ctx);

/* R = R(U): the FR-DG residual, eq. "divergence_fr" and the method of
 * lines.  U, R: [n_dof] device arrays in the context precision; the
 * arithmetic is FP64 in every context (the divergence of a flux with a large
 * mean, e.g. the pressure at low Mach number, cancels). */
fr_status fr_rhs(fr_ctx* ctx, const void* U, void* R);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): fr_rhs
 * with its intermediate FP64 traces and gradients in a scratch array the
 * library holds per device (64 MiB, a static device array whose address is
 * looked up at the first fr_ctx_create on that device) instead of the
 * context's workspaces.  Same arguments, kernels and result as fr_rhs
 * (bitwise).  Allocates nothing and calls no allocating routine.  A mesh
 * whose traces and gradients exceed 64 MiB (ne * Nf * Nv * 8 bytes, plus
 * ne * Ns * ndim * Nv * 8 and ne * Nf * ndim * Nv * 8 for viscous systems,
 * each rounded up to 256 bytes; Nf = flux points per element) returns
 * FR_E_UNSUPPORTED with the sizes in the message.  Every value the kernels
 * read from the array is written earlier in the same call, so nothing is
 * cleared.  Every call on one device shares that device's array: calls that
 * may overlap on one device (other streams, other threads) race and must be
 * serialised by the caller. */
fr_status fr_rhs_noalloc(fr_ctx* ctx, const void* U, void* R);

/* Jacobian blocks dR_n/dU_k, k in {n} and the face neighbours of n (eq.
 * "jacobian_rhs").  out_prec: FR_F64 (F64 contexts) or FR_F32 / FR_BF16
 * (F32 contexts).  FR_BF16 values are stored rounded to nearest even; for
 * quadrilaterals and hexahedra of degree 3 they are also computed from
 * BF16-rounded operands (matrix cores, FP32 accumulation), elsewhere in FP32.
 * blocks: n_elem * blocks_per_elem * b * b values, layout above (mixed
 * meshes: fr_block_offsets()[n_elem] values; inviscid systems only, viscous
 * ones return FR_E_UNSUPPORTED).  On mixed meshes the blocks of an element
 * and its face blocks come from the same chain rule as on single-type meshes,
 * the face blocks through the neighbour's own interpolation to its flux
 * points (eq. "interpolate_sol_to_flux"), FP32/FP64 arithmetic. */
fr_status fr_jacobian_blocks(fr_ctx* ctx, const void* U, void* blocks, fr_precision out_prec);

/* First entry of each element's Jacobian blocks in the array of
 * fr_jacobian_blocks: off[n] for n = 0..n_elem (off[n_elem] = the array's
 * length in values).  off: host, n_elem + 1 entries.  Single-type meshes:
 * off[n] = n * blocks_per_elem * b * b. */
fr_status fr_block_offsets(const fr_ctx* ctx, int64_t* off);

/* Jv = dR/dU(U) v exactly (forward-mode tangent of every step, including the
 * viscous second layer).  R_out (may be NULL) receives R(U).  Like fr_rhs it
 * is evaluated in FP64 (dual numbers) whatever the context precision; U, v,
 * Jv and R_out are in the context precision. */
fr_status fr_jvp(fr_ctx* ctx, const void* U, const void* v, void* Jv, void* R_out);

/* ---- Fourier (von Neumann) analysis --------------------------------------
 * Linear stability of the semi-discretisation on a uniform periodic mesh
 * (section 3, temporal linear stability: eq. "semi_discrete_pattern" and the
 * Runge-Kutta amplification polynomials of eq. "rk_exponential").  There the
 * Jacobian is block-circulant and a Bloch wave of wavenumber kappa sees
 * G(kappa) = scale * sum_k B_k exp(i kappa . d_k) over the face stencil of
 * one element, B_k its blocks as fr_jacobian_blocks returns them and d_k the
 * offset of block k's element (twice the face-centroid offset: exact on a
 * uniform mesh of parallelograms or parallelepipeds). */

/* Eigenvalues of G(kappa) for nk wavenumbers.  blocks: device, the context's
 * block array (context precision, layout of fr_jacobian_blocks; only element
 * elem's blocks are read); kappa: device [nk][ndim]; eigs: device
 * [nk][b] complex values as (re, im) pairs (order unspecified).  scale
 * multiplies G (e.g. h / |c| for the CFL number of the paper).  b <= 64,
 * quadrilaterals and hexahedra (FR_E_UNSUPPORTED otherwise).  Eigenvalues
 * come from Householder reduction to Hessenberg form and the shifted QR
 * algorithm in FP64, one wavefront per wavenumber; a wavenumber whose QR
 * iteration does not converge gets NaN eigenvalues.  Asynchronous. */
fr_status fr_fourier_eigs(fr_ctx* ctx, const void* blocks, int64_t elem, const double* kappa, int64_t nk, double scale,
                          double* eigs);
/* The largest tau in [0, tau_max] with |P(tau lambda)| <= 1 + tol for all n
 * eigenvalues (device complex pairs), P(z) = sum_j coef[j] z^j (coef: host,
 * degree 1..8), by bisection: the CFL limit of an explicit Runge-Kutta scheme
 * whose amplification polynomial is P.  tol absorbs the rounding of the
 * blocks (eigenvalues of an exact, stable semi-discretisation have Re <= 0;
 * FP32 blocks move them by about 1e-7 |lambda|).  cfl: device double (NaN if
 * an eigenvalue is not finite).  Asynchronous. */
fr_status fr_cfl_max(fr_ctx* ctx, const double* eigs, int64_t n, const double* coef, int degree, double tau_max,
                     double tol, double* cfl);

/* ---- Explicit time integration ------------------------------------------
 * nsteps steps of dU/dt = R(U) with time step dt by the five-stage,
 * fourth-order, two-register Runge-Kutta scheme of Carpenter and Kennedy
 * (the RK54 of the paper's linear advection-diffusion experiments; its
 * amplification polynomial is the RK54 polynomial of eq. "rk_exponential").
 * U: device state (context precision), advanced in place.  work: device
 * array of 2 n_dof values in the context precision (the residual and the
 * second register; its contents need no initialisation), not overlapping U.
 * Each stage is one residual evaluation (FP64 arithmetic) and one update
 * kernel; asynchronous on the context stream, allocates nothing. */
fr_status fr_rk54(fr_ctx* ctx, void* U, void* work, double dt, int64_t nsteps);

/* ---- Implicit steps (backward Euler) -------------------------------------
 * The paper integrates explicitly; these calls use the same residual and
 * Jacobian for an implicit step U - U^n - dt R(U) = 0. */

typedef enum { FR_PC_BLOCK_JACOBI = 0, FR_PC_MLP = 1 } fr_pc_kind;

/* Block preconditioner over the diagonal Jacobian blocks of the face stencil
 * (eq. "jacobian_rhs", k = n).  FR_PC_BLOCK_JACOBI: A_n = shift I + scale
 * dR_n/dU_n in FP64 with partial pivoting: blocks up to 128 x 128 inverted
 * by Gauss-Jordan elimination and applied as explicit inverses, blocks from
 * 129 to 320 (hexahedra of degree 2 and 3) factorized by a blocked LU and
 * applied by substitution; larger blocks return FR_E_UNSUPPORTED.
 * FR_PC_MLP: the learned approximate inverse (network attached with
 * fr_precond_set_mlp; blocks up to 64), with block-Jacobi as the
 * per-element fallback.
 * Storage for the inverses / factors (FP64, n_elem * b * b) is allocated
 * here, not in setup/apply. */
fr_status fr_precond_create(fr_ctx* ctx, fr_pc_kind kind, fr_precond** out);
/* Assembles and inverts the diagonal blocks at state U (device, context
 * precision).  Backward Euler: shift = 1, scale = -dt.  Returns
 * FR_E_SINGULAR (message names the element) on a zero or non-finite pivot. */
fr_status fr_precond_setup(fr_precond* pc, const void* U, double shift, double scale);
/* z_n = A_n^{-1} r_n for every element (device vectors, context precision;
 * r and z must not alias). */
fr_status fr_apply_precond(fr_precond* pc, const void* r, void* z);
fr_status fr_precond_destroy(fr_precond* pc);

/* ---- Learned block preconditioner ---------------------------------------
 * A multilayer perceptron maps the normalised diagonal block A^_n = A_n / s_n
 * (s_n = max |A_n,ij|) to an approximate inverse M_n ~ A^_n^{-1}; the
 * preconditioner applies z_n = M_n r_n / s_n.  Layers b^2 -> H -> H -> b^2,
 * ReLU after each hidden layer, BF16 weights and activations with FP32
 * accumulation (matrix cores).  Blocks and outputs are vec() of the
 * column-major b x b matrix (b^2 BF16 values per sample, samples contiguous).
 * Training minimises L = (1/B) sum_n ||A^_n M_n - I||_F^2 with Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8).  The paper defines only the Jacobian
 * these blocks come from (eq. "jacobian_rhs"); the network is this library's.
 *
 * Parameters: one FP32 vector [W1 (H x b^2), b1 (H), W2 (H x H), b2 (H),
 * W3 (b^2 x H), b3 (b^2)], row o of each W holding the weights into output o;
 * n_params = 2 H b^2 + H^2 + 2 H + b^2.  All buffers are device memory owned
 * by the caller except the network's own state, allocated in fr_mlp_create. */
typedef struct fr_mlp_s fr_mlp;
/* b <= 64 with b^2 a multiple of 128, hidden a multiple of 128, max_batch =
 * samples per internal pass (activation workspace sized for it).  Weights
 * are initialised from seed (He-normal hidden layers, small output layer,
 * zero biases).  Work runs on hip_stream. */
fr_status fr_mlp_create(int b, int hidden, uint64_t seed, int max_batch, void* hip_stream, fr_mlp** out);
fr_status fr_mlp_destroy(fr_mlp* m);
const char* fr_mlp_last_error(const fr_mlp* m);
fr_status fr_mlp_info(const fr_mlp* m, int64_t* n_params, int* b, int* hidden, int* max_batch);
/* Copy the FP32 parameter vector in / out (device pointers, n_params floats). */
fr_status fr_mlp_set_params(fr_mlp* m, const float* params);
fr_status fr_mlp_get_params(fr_mlp* m, float* params);
/* Y = network(X) for nb samples (BF16, nb x b^2 each; any nb). */
fr_status fr_mlp_forward(fr_mlp* m, const void* X, int64_t nb, void* Y);
/* Loss L (device float) and its gradient (device, n_params floats,
 * overwritten) for one batch, nb <= max_batch; resid (device, nb floats, or
 * NULL) receives ||A^_n M_n - I||_F per sample. */
fr_status fr_mlp_loss_grad(fr_mlp* m, const void* X, int64_t nb, float* loss, float* grad, float* resid);
/* One Adam step at learning rate lr on the batch; loss (device float or NULL)
 * receives the batch loss before the step. */
fr_status fr_mlp_train_step(fr_mlp* m, const void* X, int64_t nb, float lr, float* loss);
/* Attach a network to an FR_PC_MLP preconditioner (m may be NULL: no
 * network, for the refinement's scaled-transpose start).  In
 * fr_precond_setup every element with ||I - A^_n M_n||_F > theta (or
 * non-finite) falls back to the FP64 block-Jacobi inverse.  The residual is
 * evaluated in FP32 against A^_n rounded from the assembled block (not the
 * network's BF16 input), after any refinement. */
fr_status fr_precond_set_mlp(fr_precond* pc, fr_mlp* m, double theta);
/* Newton-Schulz refinement of the approximate inverse in fr_precond_setup,
 * before the safeguard: E = I - A^_n M_n, M_n <- M_n + M_n E (the residual
 * squares each step), FP32 on the matrix cores, until ||E||_F <= tol, or
 * max_iters steps, or divergence (||E||_F > 1e6).  start = 0 refines the
 * network's output; start = 1 refines the scaled transpose
 * A^_n^T / (|A^_n|_1 |A^_n|_inf), which converges for every nonsingular
 * block: the same preconditioner without the network, for comparison.
 * max_iters = 0 (the default) applies the network's BF16 output as is;
 * otherwise the refined inverse is stored and applied in FP32.  max_iters in
 * 0..64, tol >= 0, start 0 or 1, else FR_E_INVALID. */
fr_status fr_precond_set_refine(fr_precond* pc, int max_iters, double tol, int start);
/* Statistics of the last fr_precond_setup of an FR_PC_MLP preconditioner
 * (zeros for block-Jacobi): elements that fell back to block-Jacobi, mean
 * refinement steps, mean and largest ||I - A^_n M_n||_F.  Any pointer may be
 * NULL. */
fr_status fr_precond_stats(const fr_precond* pc, int64_t* n_fallback, double* mean_refine_iters, double* mean_resid,
                           double* max_resid);
/* Training samples: assembles A_n = shift I + scale dR_n/dU_n at U and
 * writes X (BF16, n_elem x b^2) and s (FP32, n_elem). */
fr_status fr_precond_mlp_inputs(fr_precond* pc, const void* U, double shift, double scale, void* X, float* s);
/* Number of elements that fell back to block-Jacobi in the last setup. */
fr_status fr_precond_info(const fr_precond* pc, int64_t* n_fallback);

typedef struct fr_solver_s fr_solver;
typedef struct {
  double dt;              /* time step */
  double newton_rtol;     /* stop when |F(U_k)|_2 <= rtol |F(U^n)|_2 */
  int32_t newton_maxit;
  double gmres_rtol;      /* relative true linear residual per Newton iteration */
  int32_t gmres_maxit;    /* GMRES iterations per Newton iteration (all restarts) */
  int32_t pc_refresh;     /* 0: preconditioner set up once at U^n; 1: at every Newton iterate */
  int32_t use_graph;      /* 1: each GMRES restart cycle is a replayed hipGraph (device-resident
                             Arnoldi, one host read per cycle); 0: host-driven Arnoldi */
  int32_t gmres_augment;  /* k in 0..3.  0: plain restarted GMRES.  k > 0: loose GMRES (Baker,
                             Jessup & Manteuffel 2005), the last k of each cycle's restart
                             directions are the corrections of the k previous cycles; the
                             subspace stays restart wide.  Runs the host-driven Arnoldi (use_graph
                             is ignored).  Out of range: FR_E_INVALID. */
  int32_t gmres_stall;    /* a linear solve also stops when its true residual fell by less than
                             1% over this many restart cycles; 0 means 4.  Negative: FR_E_INVALID. */
} fr_newton_opts;
typedef struct {
  int32_t newton_iters, gmres_iters, pc_setups, converged;
  double res0, res;       /* |F(U^n)|_2 and the final |F(U)|_2 */
  double last_linear_rel; /* last GMRES true relative residual */
  double ms;              /* wall time of the step on the context stream */
  double res_hist[32];    /* |F|_2 after each Newton iteration (first 32) */
  int32_t gmres_hist[32]; /* GMRES iterations of each Newton iteration */
  int32_t cycles;         /* restart cycles replayed from the captured graph */
} fr_newton_stats;

/* Krylov workspace for GMRES(restart), restart <= 31 (FP64 contexts). */
fr_status fr_solver_create(fr_ctx* ctx, int restart, fr_solver** out);
fr_status fr_solver_destroy(fr_solver* s);
/* One backward-Euler step from Un to U (device FP64 vectors): Newton on
 * F(U) = U - Un - dt R(U), each correction from right-preconditioned
 * GMRES(restart) on (I - dt dR/dU) dU = -F with exact Jacobian-vector
 * products; the preconditioner (or NULL) is set up at Un, and again at
 * every Newton iterate when opts->pc_refresh is set.  Returns
 * FR_E_NOT_CONVERGED if newton_maxit iterations do not reach newton_rtol,
 * FR_E_NONFINITE if the residual of an iterate, or of every line-search
 * trial, is not finite (U then holds the last finite iterate).  The step
 * clears the context's non-finite status word before it returns. */
fr_status fr_newton_step(fr_solver* s, fr_precond* pc, const void* Un, void* U, const fr_newton_opts* opts,
                         fr_newton_stats* stats);

/* ---- Batches of meshes ---------------------------------------------------
 * Many independent meshes (FP32 contexts, one system: 2-D Euler or
 * Navier-Stokes; triangles and quadrilaterals of degree 1..4 mixed freely,
 * at most 64 meshes) evaluated together: each phase of fr_rhs /
 * fr_jacobian_blocks is one persistent launch over a work list of (mesh,
 * tile) items, longest first.  Every mesh's result is bitwise identical to
 * the same mesh evaluated alone.  Runs on the first context's stream; the
 * contexts' workspaces are used, so their own calls must not overlap with
 * the batch's. */
typedef struct fr_batch_s fr_batch;
fr_status fr_batch_create(fr_ctx* const* ctxs, int n_ctx, fr_batch** out);
fr_status fr_batch_destroy(fr_batch* b);
const char* fr_batch_last_error(const fr_batch* b);
/* U[i] / R[i]: device state and residual of mesh i (layouts as fr_rhs). */
fr_status fr_batch_rhs(fr_batch* b, const void* const* U, void* const* R);
/* blocks[i]: mesh i's FP32 blocks (layout as fr_jacobian_blocks). */
fr_status fr_batch_jacobian_blocks(fr_batch* b, const void* const* U, void* const* blocks);
/* Autotuner: times, per phase, the launch strategy (one mixed launch, or
 * one launch per (type, degree) group with that group's own register and
 * LDS budget, or for the Jacobian also: triangles per group, quadrilateral
 * meshes one by one on the single-mesh matrix-core path), the
 * persistent-grid size and, per (type, degree), the tiles (residual) or
 * elements (assembly) per work item, on these arrays (reps timed
 * repetitions each), and keeps the fastest. */
fr_status fr_batch_tune(fr_batch* b, const void* const* U, void* const* R, void* const* blocks, int reps);
/* The current table: modes[0] / modes[1] = residual / Jacobian launch
 * strategy (0: one mixed launch per phase, 1: one launch per (type, degree)
 * group, 2 (Jacobian only): 1 for triangles, the matrix-core single-mesh
 * path for quadrilaterals), workgroups per launch (0: one per work item, scheduled by the
 * hardware), and units per work item indexed by 8 * type + degree (32
 * entries each). */
fr_status fr_batch_tuning(const fr_batch* b, int* modes, int* grid_res, int* grid_jac, int* k_res, int* k_jac);
/* Load a table (e.g. one saved from fr_batch_tuning); modes / k_* may be NULL
 * to keep the current entries; units per work item below 1 read as 1. */
fr_status fr_batch_set_tuning(fr_batch* b, const int* modes, int grid_res, int grid_jac, const int* k_res,
                              const int* k_jac);

/* Profiling.  When enabled, the dominant kernel of fr_jacobian_blocks
 * (which = 0: block assembly) and of fr_rhs / fr_jvp (which = 1: the flux /
 * divergence pass) is bracketed by HIP events on the context stream.
 * fr_kernel_time waits for the recorded events, returns the summed kernel
 * time in milliseconds and the number of launches since the previous query,
 * and resets both.  Enabling creates the events (not a hot call). */
fr_status fr_set_kernel_timing(fr_ctx* ctx, int enable);
fr_status fr_kernel_time(fr_ctx* ctx, int which, double* ms_total, int64_t* count);

#ifdef __cplusplus
}
#endif
#endif
