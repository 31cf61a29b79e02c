/*
 * rs.h - C ABI of the reduced-Newton hot path of a Lipschitz-optimised
 * neural-subspace solver for deformable bodies (Lyu, Zhao, Xian, Cen, Cai,
 * Fang, "Accelerate Neural Subspace-Based Reduced-Order Solver of Deformable
 * Simulation by Lipschitz Optimization", ACM TOG 43(6), 2024), for AMD
 * Instinct MI355X (gfx950).
 *
 * The library minimises, for a batch of independent items, the reduced
 * quasi-static objective of Sec. 3.1 (Eq. form-reduced-space-time-integration
 * with the inertia term dropped):
 *
 *     E(z) = P~(q(z)) - sum_v m_v g.(x_v - X_v) + k_c/2 sum_{v in T} |x_v - t_v|^2
 *            - sum_{v in F} f.(x_v - X_v),      q(z) = X + m (.) f_theta(z)
 *
 * where f_theta is an MLP decoder (ELU hidden layers, linear output; Sec. 3.2),
 * m masks Dirichlet-fixed vertices, P~ = sum_{e in S} w_e P_e is the cubature
 * elastic potential (Sec. 4.3, Eq. form-cubature-gradients) of a stable
 * Neo-Hookean tetrahedral mesh, T are penalty-targeted vertices and F
 * force-loaded vertices.  It also evaluates the paper's Lipschitz loss of the
 * cubature elastic Hessian (Sec. 4.1, Eq. form-L-LS-E).
 *
 * Conventions
 *  - Every entry point returns RS_OK (0) or an RS_ERR_* code; the message of
 *    the last error is available from rs_last_error().  No C++ exception
 *    crosses the ABI.
 *  - rs_create() copies every host array it is given; the caller may free
 *    them on return.  The context owns all device memory it needs, sized for
 *    max_batch items; no hot-path call allocates device memory.
 *  - Batch arguments (z, x, J, E, g, H, iters, status, relgrad, loss, ...) are
 *    DEVICE pointers owned by the caller.  Layouts are row-major and dense.
 *  - Work is enqueued on `stream` (a hipStream_t cast to void*, NULL for the
 *    default stream) and is asynchronous, except where an entry point says it
 *    synchronises.  Argument checks are synchronous.
 *  - Latent and reduced quantities (z, E, g, H, loss) are always float64.
 *    Positions and Jacobians returned by rs_decode use the context precision
 *    (float32 for RS_PREC_BF16 contexts).
 */
#ifndef RS_H
#define RS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
enum {
    RS_OK = 0,
    RS_ERR_ARG = 1,         /* invalid argument (null pointer, size, index out of range) */
    RS_ERR_HIP = 2,         /* a HIP runtime call or kernel launch failed */
    RS_ERR_OOM = 3,         /* device allocation failed */
    RS_ERR_STATE = 4,       /* context not usable */
    RS_ERR_UNSUPPORTED = 5  /* size or mode outside what the library supports */
};

/* per-item solver outcomes: the exit conditions of the paper's solver
 * (Sec. 5 and the convergence-condition discussion of the supplement) */
enum {
    RS_CONVERGED = 0,    /* I:   |g|_inf <= rel_tol |g_0|_inf (or <= abs_tol) */
    RS_NOT_DESCENT = 1,  /* II:  no descent direction (saddle; projection off) */
    RS_LS_MAX = 2,       /* III: ls_max backtracking trials without sufficient decrease */
    RS_ITER_MAX = 3,     /* IV:  max_iter Newton steps taken without converging */
    RS_NONFINITE = 4,    /* energy, gradient or Hessian not finite */
    RS_RUNNING = -1
};

/* Context precision of the decoder and element physics.
 * RS_PREC_BF16 is the precision variant of the float32 context: the forward
 * decoder products (hidden layers and output map) run on the BF16 matrix cores
 * with float32 accumulation and float32 accuracy.  Every weight is held as three
 * BF16 parts (hi, mid, lo: round-to-nearest-even from float64), every layer input
 * is split the same way, and six of the nine part products are summed, so the
 * decoder is the same function as in the float32 context.  Pre-activations,
 * element physics, adjoint and curvature run in float32 exactly as in a float32
 * context; reduced quantities, the r x r solve and the line-search energies stay
 * float64.  It needs at least one hidden layer. */
enum { RS_PREC_F64 = 0, RS_PREC_F32 = 1, RS_PREC_BF16 = 2 };

/* rs_energy_grad_hess flags */
enum {
    RS_HESS_EXACT = 1,    /* add the decoder-curvature term sum_k g_k d2q_k/dz2 (else Gauss-Newton) */
    RS_ELASTIC_ONLY = 2,  /* cubature elastic potential only (no gravity, penalty, forces) */
    RS_ENERGY_ONLY = 4,   /* energy only; g and H may be NULL */
    RS_GRAD_REVERSE = 8,  /* g by reverse mode (a value pass, then the adjoint pass back through the
                             decoder) instead of forward-mode Jacobian columns; H must be NULL */
    RS_ELEM_PSD = 16,     /* project every cubature element Hessian H_e = V D^T (d2psi/dF2) D (12 x 12) to
                             positive semi-definite (negative eigenvalues set to zero) before it enters
                             H (supplement, projective Newton: the classic per-element projection) */
    RS_DEBUG_ELEM_HESS = 32 /* also write the 12 x 12 element Hessians H_e of the cubature tets to the
                             buffer given to rs_set_elem_hess_dump (unprojected; inspection only) */
};

/* Hessian treatment before the Newton solve */
enum {
    RS_PROJ_CLAMP = 0, /* eigenvalues below eig_floor*max|eig| raised to that floor */
    RS_PROJ_ABS = 1,   /* eigenvalues replaced by max(|eig|, eig_floor*max|eig|) */
    RS_PROJ_NONE = 2   /* no projection: a Hessian that is not positive definite ends the item (RS_NOT_DESCENT) */
};

/* Tetrahedral mesh: nv vertices X (nv x 3, metres), ne tets (ne x 4 vertex ids,
 * positively oriented), pinned[v] != 0 fixes vertex v at its rest position. */
typedef struct {
    int32_t nv, ne;
    const double* X;
    const int32_t* tets;
    const uint8_t* pinned;
} rs_mesh;

/* Stable Neo-Hookean material: Young's modulus (Pa), Poisson ratio, density
 * (kg/m^3) and the gravity vector (m/s^2). */
typedef struct {
    double young, poisson, density, gravity[3];
} rs_material;

/* Decoder f_theta: r -> n_hidden layers of `width` (ELU) -> n_out = 3 nv (linear).
 * W[l] is (out x in) row-major float64, b[l] has `out` entries, l = 0..n_hidden.
 * n_hidden = 0 gives a linear decoder (e.g. a PCA basis). */
typedef struct {
    int32_t r, n_hidden, width, n_out;
    const double* const* W;
    const double* const* b;
} rs_decoder;

/* Cubature set S: n distinct element ids with non-negative weights (Sec. 4.3). */
typedef struct {
    int32_t n;
    const int32_t* elem;
    const double* weight;
} rs_cubature;

/* Penalty-targeted vertices with stiffness k_c (N/m), force-loaded vertices,
 * and ground contact: the one-sided penalty k_ground/2 min(0, y_v - ground_y)^2
 * (N/m, m) on each contact vertex v (the y coordinate is "up"; contact treated
 * as part of the potential, Sec. 5.2's penalty collisions).  n_contact = 0: no
 * ground. */
typedef struct {
    int32_t n_target;
    const int32_t* target_vtx;
    double k_c;
    int32_t n_force;
    const int32_t* force_vtx;
    int32_t n_contact;
    const int32_t* contact_vtx;
    double k_ground;
    double ground_y;
} rs_constraints;

/* Per-batch loads (DEVICE pointers, float64, each may be NULL):
 * targets (B x n_target x 3) positions of the targeted vertices; force (B x 3)
 * the force applied to each force-loaded vertex; qbar (B x nv x 3) the
 * inertial targets of an implicit-Euler step (displacements q_bar - X, Sec.
 * 3.1, Eq. form-reduced-space-time-integration), used when dt > 0: the
 * objective gains 1/(2 dt^2) |q(z) - q_bar|_M^2 over the free rows (M the
 * lumped masses).  qbar = NULL or dt = 0: quasi-static. */
typedef struct {
    const double* targets;
    const double* force;
    const double* qbar;
    double dt;
} rs_load;

/* Newton options (host struct).  Defaults from rs_default_opts(). */
typedef struct {
    int32_t max_iter;   /* Newton steps, default 50 */
    int32_t ls_max;     /* backtracking trials per step, default 128 (Sec. 5) */
    double c1;          /* Armijo constant, default 1e-4 */
    double shrink;      /* step factor per trial, default 0.5 */
    double rel_tol;     /* |g|_inf <= rel_tol |g_0|_inf, default 1e-6 */
    double abs_tol;     /* or |g|_inf <= abs_tol, default 0 */
    int32_t hess;       /* bit 0: exact Hessian (default 1), else Gauss-Newton; bit 1: per-element
                           projection of the cubature element Hessians (RS_ELEM_PSD) */
    int32_t proj;       /* RS_PROJ_*, default RS_PROJ_ABS */
    double eig_floor;   /* relative eigenvalue floor, default 1e-8 */
    int32_t window;     /* items in flight, default 0 (all B at once).  0 < window < B: items 0 .. window-1
                           start, and item b enters as soon as fewer than `window` items run (continuous
                           batching: every super-step stays full until the last items).  Each item's
                           iterates are those of a solve with every item in flight, up to the float32
                           summation order of the launch sizes */
} rs_solve_opts;

/* L-BFGS options (host struct).  Defaults from rs_default_lbfgs_opts(). */
#define RS_MAX_HISTORY 16
typedef struct {
    int32_t max_iter;   /* accepted steps (exit IV), default 1024 (Sec. 5) */
    int32_t ls_max;     /* backtracking trials per step (exit III), default 128 (Sec. 5) */
    int32_t history;    /* (s, y) pairs kept, 0 .. RS_MAX_HISTORY, default 10 */
    double c1;          /* Armijo constant, default 1e-4 */
    double shrink;      /* step factor per trial, default 0.5 */
    double rel_tol;     /* |g|_inf <= rel_tol |g_0|_inf, default 1e-6 */
    double abs_tol;     /* or |g|_inf <= abs_tol, default 0 */
    int32_t window;     /* items in flight, default 0 (all B at once); as rs_solve_opts.window (each item's
                           history starts at its first step) */
} rs_lbfgs_opts;

/* Static description of a context (sizes used for work accounting). */
typedef struct {
    int32_t prec, r, n_hidden, width, nv, ne, n_cub, n_target, n_force;
    int32_t rows;       /* rows of the reduced output map: 9 per cubature tet, 3 per target, 1 gravity, 3 force */
    int32_t rows_pad;   /* rows padded to the GEMM tile */
    int32_t max_batch;
} rs_info;

typedef struct rs_ctx rs_ctx;

/* Fill *o with the defaults listed in rs_solve_opts. */
int rs_default_opts(rs_solve_opts* o);
/* Fill *o with the defaults listed in rs_lbfgs_opts. */
int rs_default_lbfgs_opts(rs_lbfgs_opts* o);

/* Create a context on the current HIP device.  prec is RS_PREC_F64,
 * RS_PREC_F32 or RS_PREC_BF16; max_batch bounds B of every later call (the Lipschitz loss
 * handles up to max_batch/2 pairs per internal pass).  Requires 1 <= r <= 32,
 * n_out == 3 nv, every index in range and every cubature tet of positive
 * volume; float32 and BF16 contexts also need rows_pad x (r + 1) < 4194304
 * (rows of the reduced output map, RS_ERR_UNSUPPORTED otherwise).
 * Synchronous.  On failure *out is NULL. */
int rs_create(const rs_mesh* mesh, const rs_material* mat, const rs_decoder* dec,
              const rs_cubature* cub, const rs_constraints* con, int32_t prec,
              int32_t max_batch, rs_ctx** out);

/* Release every device and host resource of the context.  NULL is accepted. */
int rs_destroy(rs_ctx* ctx);

/* Replace the decoder weights (same r, n_hidden, width, n_out).  Synchronous. */
int rs_set_decoder(rs_ctx* ctx, const rs_decoder* dec);

/* Describe the context. */
int rs_get_info(const rs_ctx* ctx, rs_info* info);

/* Decoder value and Jacobian (Sec. 3.2: q = f_theta(z)) for B <= max_batch items:
 * z (B x r) float64; x (B x nv x 3) deformed positions and J (B x 3nv x r)
 * dq/dz in the context precision (float or double).  Either output may be
 * NULL.  Pinned vertices stay at rest with zero Jacobian rows. */
int rs_decode(rs_ctx* ctx, int32_t B, const double* z, void* x, void* J, void* stream);

/* Reduced energy E (B), gradient g = J^T grad_q E (B x r) and Hessian H (B x r x r,
 * J^T H_q J plus, with RS_HESS_EXACT, the decoder-curvature term) at B latent
 * points z (B x r) (Sec. 3.1, Sec. 4.3 Eq. form-cubature-gradients and the
 * cubature Hessian of P~).  E is always evaluated in float64; g and H in the
 * context precision with float64 accumulation.  Any B >= 0 (processed in
 * chunks of max_batch).  With RS_GRAD_REVERSE (float32 and float64 contexts
 * with hidden layers) g = J^T grad_q E is formed backwards, never forming J;
 * other contexts fall back to the forward mode. */
int rs_energy_grad_hess(rs_ctx* ctx, int32_t B, const double* z, const rs_load* load,
                        uint32_t flags, double* E, double* g, double* H, void* stream);

/* Register the destination of RS_DEBUG_ELEM_HESS: He (DEVICE, float64,
 * max_items x n_cub x 12 x 12, row-major, caller-owned).  Row and column
 * 3 a + i of an element block is coordinate i of the tet's corner a (corners
 * in the mesh's tet order), as in H_e = V D^T A D of the element's stable
 * Neo-Hookean energy (Sec. 3.1 elastic energy, Sec. 5.1 material; unweighted
 * by the cubature weight).  rs_energy_grad_hess calls with the flag fill the
 * blocks of their first min(B, max_items) items, each at its batch position.
 * He = NULL or max_items = 0 unregisters.  Errors: RS_ERR_STATE (NULL ctx),
 * RS_ERR_ARG (negative max_items, or NULL He with max_items > 0). */
int rs_set_elem_hess_dump(rs_ctx* ctx, double* He, int32_t max_items);

/* Choose how a float32 or BF16 context forms the rows of J_R = W_big [h | J_h]
 * (the folded output layer, Sec. 4.3: each cubature tet's F with its r
 * Jacobian columns, and the penalty, gravity and force rows) for the element
 * physics.  on != 0: one kernel forms each chunk of rows in on-chip memory
 * just before the element physics of the same workgroup reads it, so J_R is
 * never written to device memory (products on the BF16 matrix cores in BF16
 * contexts, on the FP32 ones in float32 contexts).  on == 0: the output map
 * writes J_R to device memory and the element kernel reads it back.  Both give
 * the same function to float32 rounding.  Default: on in RS_PREC_BF16
 * contexts, off in RS_PREC_F32 ones (the faster of the two for each).  The
 * fused kernel applies when r = 16, the last hidden layer has at most 128
 * units, and the evaluation has no ground contact, inertia, RS_ELEM_PSD or
 * RS_DEBUG_ELEM_HESS (those read J_R after the element physics); elsewhere the
 * two-kernel path runs whatever `on` says.  *applies (may be NULL) receives 1
 * if the context meets the first two conditions and is not float64, else 0.
 * Errors: RS_ERR_STATE (NULL ctx). */
int rs_set_fused(rs_ctx* ctx, int32_t on, int32_t* applies);

/* Number of decoder parameters: sum over the layers (output layer last) of
 * out x in weights plus out biases, the length of rs_energy_param_grad's
 * gradient.  Errors: RS_ERR_STATE (NULL ctx), RS_ERR_ARG (NULL n). */
int rs_param_count(const rs_ctx* ctx, int64_t* n);

/* Gradient of sum_b E(z_b) over B latent points with respect to every
 * decoder parameter theta: the potential loss of the unsupervised subspace
 * construction (Sec. 3.2, Eq. form-vanilla-unsupervised-construction; its
 * expectation over z taken as the caller's sample sum), differentiated by
 * reverse mode through the cubature energy, the output layer and the hidden
 * layers, with the hidden activations recomputed from their pre-activations.
 * grad (device, float64, rs_param_count values) is overwritten, packed as
 * W_1, b_1, ..., W_L, b_L, W_out, b_out with each W row-major (out x in) as
 * in rs_decoder; rows of pinned vertices in W_out and b_out get zero.  Sums over
 * items are float64.  E (B, float64) and g = dE/dz (B x r) are per item and may
 * be NULL.  z (B x r) float64 device; any B >= 0 (chunks of max_batch; B = 0
 * gives a zero gradient).  flags: 0 or RS_ELASTIC_ONLY.  The library owns
 * its workspace; the caller owns every pointer argument.  Errors: RS_ERR_ARG
 * (NULL grad or z, other flags), RS_ERR_UNSUPPORTED (BF16 contexts, no
 * hidden layers, or hidden layers outside what the fused kernel supports). */
int rs_energy_param_grad(rs_ctx* ctx, int32_t B, const double* z, const rs_load* load, uint32_t flags,
                         double* E, double* g, double* grad, void* stream);

/* Projective Newton with backtracking line search (supplement, projective
 * Newton tests) for B <= max_batch independent items, z (B x r) in/out.
 * Per item: iters (int32) accepted steps, status (RS_CONVERGED...), relgrad
 * |g|_inf/|g_0|_inf at exit, E (float64) energy at exit.  The direction is
 * -H^-1 g with the Cholesky factor of the symmetrised Hessian when it is
 * positive definite, else with its eigen-projection (opts->proj).  Armijo
 * backtracking alpha = shrink^j, j < ls_max, on float64 energies.
 * The host enqueues one super-step (evaluate, direction, line-search round)
 * ahead and waits on one event per super-step to read how many items are
 * still running; the call returns once every item has exited, with at most
 * the last super-step's work still in flight on `stream`. */
int rs_newton_solve(rs_ctx* ctx, int32_t B, double* z, const rs_load* load,
                    const rs_solve_opts* opts, int32_t* iters, int32_t* status,
                    double* relgrad, double* E, void* stream);

/* The same solve, stream-ordered: enqueues exactly `super_steps` super-steps
 * (each: evaluate the items that need g and H, their directions, one
 * line-search round) on `stream` and returns without waiting or reading
 * anything back, so the call can be captured into a HIP graph.  Every launch
 * is sized for all B items; the kernels read the running counts on the device
 * and idle workgroups exit at once.  Items that have not exited after
 * `super_steps` keep status RS_RUNNING (-1) and their current z, iters and E;
 * an item needs one super-step per accepted Newton step plus one per extra
 * line-search round.  Outputs, workspace and errors as rs_newton_solve, plus
 * RS_ERR_ARG for super_steps < 1. */
int rs_newton_solve_async(rs_ctx* ctx, int32_t B, double* z, const rs_load* load,
                          const rs_solve_opts* opts, int32_t super_steps, int32_t* iters,
                          int32_t* status, double* relgrad, double* E, void* stream);

/* L-BFGS with backtracking line search (Sec. 5: the paper's solver for its
 * main results, with exits I converged, II saddle / not a descent direction,
 * III 128 line-search trials, IV iteration limit), for B <= max_batch
 * independent items, z (B x r) in/out, outputs as rs_newton_solve.  The
 * direction is the two-loop recursion over the last opts->history pairs
 * s = z_{k+1} - z_k, y = g_{k+1} - g_k (a pair is kept only when s.y > 0),
 * with H_0 = (s.y / y.y) I of the newest pair, and -g without pairs.  Only
 * the gradient is evaluated (no Hessian), by reverse mode where
 * RS_GRAD_REVERSE applies.  Armijo backtracking as in
 * rs_newton_solve, on float64 energies.  The history lives in the context
 * (allocated by rs_create for max_batch items), so one solve at a time per
 * context. */
int rs_lbfgs_solve(rs_ctx* ctx, int32_t B, double* z, const rs_load* load,
                   const rs_lbfgs_opts* opts, int32_t* iters, int32_t* status,
                   double* relgrad, double* E, void* stream);

/* Lipschitz loss (Sec. 4.1, Eq. form-L-LS-E) of the exact cubature elastic
 * Hessian over B pairs (z1_b, z2_b) (each B x r):
 *   per_pair[b] = |H(z1_b) - H(z2_b)|_F^2 / |z1_b - z2_b|^2   (0 where z1_b == z2_b),
 *   loss = mean over pairs with z1_b != z2_b, n_valid their count,
 *   lip_max = max_b sqrt(per_pair[b]) (the max-pair estimator, Eq. form-H-Lipschitz-estimation).
 * per_pair and lip_max may be NULL.  All outputs are device pointers. */
int rs_lipschitz_loss(rs_ctx* ctx, int32_t B, const double* z1, const double* z2,
                      double* loss, double* per_pair, int32_t* n_valid, double* lip_max,
                      void* stream);

/* Replace the decoder weights from a DEVICE buffer, stream-ordered (no host
 * round trip, no synchronisation): theta holds rs_param_count values packed as
 * rs_energy_param_grad's gradient (W_1, b_1, ..., W_L, b_L, W_out, b_out, each
 * W row-major out x in), float64 when theta_f64 != 0, else float32.  The
 * context converts them to its precision (round to nearest even for BF16
 * products) and rebuilds the output-layer fold onto the reduced rows, as
 * rs_set_decoder does from host arrays.  The learned part (Sec. 4.2, Eq.
 * form-unconstrained-lipschitz-optimization) reloads the decoder after every
 * optimiser step this way.  theta must stay valid until the work enqueued on
 * `stream` has run; later calls on other streams must be ordered after it by
 * the caller.  Errors: RS_ERR_STATE (NULL ctx), RS_ERR_ARG (NULL theta),
 * RS_ERR_HIP (launch failure). */
int rs_set_decoder_device(rs_ctx* ctx, const void* theta, int32_t theta_f64, void* stream);

/* Gradient of the Lipschitz loss (Sec. 4.1, Eq. form-L-LS-E, on the cubature
 * elastic Hessian of Sec. 4.3) with respect to every decoder parameter, the
 * latent pairs held fixed:
 *   loss = mean over pairs with z1_b != z2_b of |H(z1_b) - H(z2_b)|_F^2 / |z1_b - z2_b|^2,
 *   grad = d loss / d theta, packed as rs_energy_param_grad's gradient,
 * with H the exact reduced Hessian of the weighted cubature elastic energy
 * (RS_HESS_EXACT | RS_ELASTIC_ONLY).  The derivative is carried forward through
 * the decoder as value, Jacobian and C-contracted second-derivative columns
 * (C = 2 sym(H1 - H2) / (|dz|^2 n_valid)) and taken back by reverse mode, with
 * the hidden activations recomputed from kept pre-activations; the element
 * term needs the third derivatives of the stable Neo-Hookean energy.  z1, z2
 * (B x r) float64 device; loss (1) and grad (rs_param_count) float64 device,
 * overwritten; B = 0 or no valid pair gives zeros.  Float32 and float64
 * contexts with max_batch >= 2.  The first call allocates the pass workspace
 * (up to 128 pairs per pass) and keeps it in the context.  Errors:
 * RS_ERR_STATE, RS_ERR_ARG (B < 0, NULL pointers), RS_ERR_UNSUPPORTED (BF16
 * context, max_batch < 2), RS_ERR_OOM (workspace). */
int rs_lipschitz_param_grad(rs_ctx* ctx, int32_t B, const double* z1, const double* z2, double* loss,
                            double* grad, void* stream);

/* rs_lipschitz_param_grad for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving or training loops, harnesses
 * that forbid hipMalloc): the same arguments, results and errors, but the pass
 * workspace is carved from a static device array of RS_STATIC_SCRATCH_BYTES
 * that the library holds on every device it runs on until the process ends,
 * instead of being allocated by the first call.  It makes as many pairs per pass
 * as that array holds (at most the allocating variant's 128), so results can
 * differ from rs_lipschitz_param_grad's by the order of the float64 sums over
 * passes.  Calls that overlap on one device (any context, any stream) share the
 * array and race; the caller orders them.  Nothing has to be cleared between
 * calls: every pass overwrites what it reads.  Errors: as
 * rs_lipschitz_param_grad, and RS_ERR_UNSUPPORTED when one pair's workspace
 * exceeds the array (the message gives both sizes). */
#define RS_STATIC_SCRATCH_BYTES (64u << 20)
int rs_lipschitz_param_grad_noalloc(rs_ctx* ctx, int32_t B, const double* z1, const double* z2, double* loss,
                                    double* grad, void* stream);

/* Implicit-Euler simulation (Sec. 3.1, Eq. form-reduced-space-time-integration):
 * `steps` time steps of B independent simulations from z (B x r, DEVICE,
 * in/out: the start, then the last step's solution) with initial velocities v0
 * (B x nv x 3 displacement rates, DEVICE; NULL = at rest).  Step k minimises
 *   1/(2 dt^2) |q(z) - q_bar^(k+1)|_M^2 + P~(q(z)) + gravity, penalty targets,
 *   forces and ground contact (the load's targets and force, constant in time),
 * with q_bar^1 = q^0 + dt v0 and q_bar^(k+1) = 2 q^k - q^(k-1) (the positions of
 * the previous steps; both lie in the decoder's range, so the inertia term is
 * formed from the last hidden activations), by the projective Newton solve of
 * rs_newton_solve with `opts` (NULL = defaults).  Per item: iters (the Newton
 * iterations of all steps) and failed (the steps not ending on RS_CONVERGED),
 * int32 DEVICE; ztraj (steps x B x r, DEVICE, may be NULL) the solution of every
 * step.  Errors: as rs_newton_solve, RS_ERR_ARG (steps < 0, dt <= 0). */
int rs_simulate(rs_ctx* ctx, int32_t B, double* z, const double* v0, const rs_load* load, int32_t steps, double dt,
                const rs_solve_opts* opts, int32_t* iters, int32_t* failed, double* ztraj, void* stream);

/* ---- full-space solver ----
 * Quasi-static equilibrium over EVERY element of the mesh (Sec. 3.1, Eq.
 * form-full-space-time-integration without the inertia term): the snapshot
 * generator of the supervised construction (Sec. 3.2) and the reference for the
 * reduced solves.  Projective Newton (supplement): each element Hessian
 * V D^T (d2 psi/dF2) D with its negative eigenvalues set to zero; the Newton
 * system solved by Jacobi-preconditioned conjugate gradients with matrix-free
 * element products, stopped at |r|_2 <= eta |g|_2 with
 * eta = clamp(sqrt(|g|_inf / |g_0|_inf), eta_min, eta_max); Armijo backtracking
 * on the full energy; exits as rs_newton_solve over the free dofs.  Float64
 * throughout, whatever the context precision. */
typedef struct {
    int32_t max_iter;    /* Newton iterations (exit IV) */
    int32_t ls_max;      /* backtracking trials (exit III) */
    int32_t cg_max;      /* CG iterations per Newton step */
    double c1;           /* Armijo constant */
    double shrink;       /* step factor per trial */
    double rel_tol;      /* converged when |g|_inf <= rel_tol |g_0|_inf (free dofs) */
    double abs_tol;      /* ... or |g|_inf <= abs_tol */
    double eta_min;      /* CG forcing term bounds */
    double eta_max;
} rs_full_opts;

/* max_iter 100, ls_max 128, cg_max 4000, c1 1e-4, shrink 0.5, rel_tol 1e-6,
 * abs_tol 0, eta_min 1e-4, eta_max 0.1. */
int rs_default_full_opts(rs_full_opts* o);

/* Solve B independent load cases: u (B x nv x 3, float64 DEVICE, in/out) the
 * displacements q - X from which each solve starts (pinned vertices keep
 * theirs), load as in rs_energy_grad_hess (penalty targets and forces of the
 * context's constraint sets).  Per item: iters, status (RS_CONVERGED ...),
 * relgrad |g|_inf / |g_0|_inf and the energy E at exit (each DEVICE, may be
 * NULL); E = sum_e V_e psi_e - sum_v m_v g.u_v + k_c/2 sum_t |x_t - t_t|^2 -
 * sum_f f.u_f.  The first call builds the mesh tables, and a call with a
 * batch larger than any before grows the workspace (about 450 B per element and
 * item, float64).  Synchronises the stream once per Newton iteration, once per
 * eight CG iterations and once per line-search trial.  Errors: RS_ERR_STATE,
 * RS_ERR_ARG (B < 0, NULL u or opts, bad options), RS_ERR_OOM, RS_ERR_HIP. */
int rs_full_solve(rs_ctx* ctx, int32_t B, double* u, const rs_load* load, const rs_full_opts* opts,
                  int32_t* iters, int32_t* status, double* relgrad, double* E, void* stream);

/* ---- supervised training of the subspace (the learned part) ----
 * An autoencoder (Sec. 3.2, Eq. form-vanilla-supervised-construction): an ELU
 * encoder g: displacements (3 nv) -> r, and the context's decoder f.  One
 * gradient call on a batch of snapshot displacements d_b = q_b - X takes
 *   L_C  = mean_b |m (.) f(g(d_b)) - d_b|_M^2      (lumped masses M; m masks pinned rows)
 *   L_LS = the Lipschitz loss of the decoder (Sec. 4.1, Eq. form-L-LS-E) over the
 *          pairs (z_2p, z_2p+1), p < n_pairs, of the batch's encodings z_b = g(d_b),
 *          which are held fixed (the samples of the pull-back distribution, Sec. 4.2)
 * and the gradients of L_C + lambda_ls L_LS (Sec. 4.2, Eq.
 * form-unconstrained-lipschitz-optimization) with respect to the encoder and
 * decoder parameters, by hand-written reverse mode on the matrix cores.  Adam
 * (Kingma and Ba) then updates both networks and reloads the context's
 * decoder on the GPU (rs_set_decoder_device), so reduced solves on the context
 * use the trained subspace.  Parameters and activations are in the context
 * precision (float32 or float64); losses, bias sums and the Lipschitz
 * gradient are float64.  The trainer belongs to its context and must be
 * destroyed before it; one trainer per context at a time. */
typedef struct {
    int32_t n_in;        /* input size (3 nv for an encoder) */
    int32_t n_hidden;    /* ELU hidden layers (0..8) */
    int32_t width;       /* units per hidden layer */
    int32_t n_out;       /* output size (r for an encoder), linear */
    const double* const* W;  /* host, W[l] (out x in) row-major, l = 0..n_hidden */
    const double* const* b;
} rs_mlp;

typedef struct rs_trainer rs_trainer;

/* Create a trainer for ctx (float32 or float64, with hidden layers) from host
 * initial weights of the encoder (n_in = 3 nv, n_out = r) and of the decoder
 * (the context's shape); the context's decoder is replaced by `dec`.
 * max_batch (>= 2) bounds B of rs_trainer_grad.  Allocates its workspace here;
 * synchronous.  Errors: RS_ERR_STATE, RS_ERR_ARG (shapes, NULL pointers),
 * RS_ERR_UNSUPPORTED (BF16 context, linear decoder, encoder deeper than 8 or
 * wider than 4096), RS_ERR_OOM. */
int rs_trainer_create(rs_ctx* ctx, const rs_mlp* encoder, const rs_decoder* dec, int32_t max_batch,
                      rs_trainer** out);
int rs_trainer_destroy(rs_trainer* t);
/* Sizes of the packed encoder parameters (W_1, b_1, ..., W_out, b_out, each W
 * row-major out x in) and decoder parameters (as rs_param_count). */
int rs_trainer_param_count(const rs_trainer* t, int64_t* n_enc, int64_t* n_dec);
/* Copy the current parameters (context precision) into device buffers (either may be NULL). */
int rs_trainer_params(rs_trainer* t, void* enc, void* dec, void* stream);
/* Encodings z (B x r, float64 device) of rows idx[b] (device int32, NULL = rows
 * 0..B-1) of the snapshot store (N x 3 nv displacements, context precision,
 * device).  Any B >= 0. */
int rs_trainer_encode(rs_trainer* t, int32_t B, const void* store, const int32_t* idx, double* z, void* stream);
/* Losses and gradients of one batch: rows idx[b] of `store` (as rs_trainer_encode),
 * 1 <= B <= max_batch.  lambda_ls = 0 skips the Lipschitz term; otherwise
 * 1 <= n_pairs <= B/2.  losses (2, float64 device: L_C, L_LS), grad_enc
 * (n_enc) and grad_dec (n_dec, the gradient of L_C + lambda_ls L_LS), float64
 * device, may each be NULL; the trainer keeps its own copies for
 * rs_trainer_adam.  Errors: RS_ERR_STATE, RS_ERR_ARG. */
int rs_trainer_grad(rs_trainer* t, int32_t B, const void* store, const int32_t* idx, double lambda_ls,
                    int32_t n_pairs, double* losses, double* grad_enc, double* grad_dec, void* stream);
/* One Adam step of both networks with the gradients of the last
 * rs_trainer_grad call (bias-corrected moments, step counted by the trainer),
 * then the context's decoder is reloaded from the new parameters. */
int rs_trainer_adam(rs_trainer* t, double lr, double beta1, double beta2, double eps, void* stream);

/* PCA basis of N snapshot displacements (the linear subspace of Sec. 2's
 * related work, kept as the baseline of the learned subspace): the mean
 * displacement (n = 3 nv, float64 DEVICE) and W (n x r, row-major, float64
 * DEVICE) whose columns span the r leading principal directions of the
 * centred snapshots in the mass inner product (W^T M W = I, M the lumped
 * masses), with their captured sums of squares in evals (r, DEVICE, may be
 * NULL), largest first.  u = mean + W z is then a linear decoder (rs_decoder
 * with n_hidden = 0, W_out = W, b_out = mean), and z_rest (r, DEVICE, may be
 * NULL) = -W^T M mean the coordinates of the rest shape's projection onto
 * that affine subspace.  Subspace iteration on
 * Dc^T Dc M with r + 8 vectors (iters rounds) and a Rayleigh-Ritz step, float64
 * on the matrix cores.  store: N x 3 nv in the context precision (DEVICE).
 * Allocates its workspace for the call (about 8 N n bytes) and frees it;
 * synchronises the stream.  Errors: RS_ERR_ARG (sizes, r > min(N, 56), fewer
 * than r + 8 independent snapshots), RS_ERR_OOM, RS_ERR_HIP. */
int rs_pca(rs_ctx* ctx, int32_t N, const void* store, int32_t r, int32_t iters, double* W, double* mean,
           double* evals, double* z_rest, void* stream);

/* Message of the last error on this context ("" if none); a static message
 * when ctx is NULL. */
const char* rs_last_error(const rs_ctx* ctx);

/* Kernel timing.  rs_profile(ctx, 1, mask) clears previous records and
 * brackets every later launch of the kernel kinds in `mask` (bit k = kind k,
 * 0 = every kind) with HIP events on its stream; rs_profile(ctx, 0, 0) stops
 * recording.  rs_profile_get() synchronises the device and returns, for kernel
 * kind idx < *n_kinds, its name, launch count, summed duration and the summed
 * algorithmic HBM bytes and flops of those launches (idx < 0 only sets
 * *n_kinds). */
int rs_profile(rs_ctx* ctx, int32_t enable, uint32_t kind_mask);
int rs_profile_get(rs_ctx* ctx, int32_t idx, int32_t* n_kinds, char* name, int32_t name_len,
                   int32_t* launches, double* total_ms, double* bytes, double* flops);

#ifdef __cplusplus
}
#endif
#endif /* RS_H */
