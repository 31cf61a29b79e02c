/*
 * FP64 CPU oracle for the reduced-Newton hot path of a Lipschitz-optimised
 * neural-subspace solver (Lyu et al., ACM TOG 43(6), 2024).
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it.  It shares no
 * source, header, table or helper with the GPU library.
 *
 * Everything is float64, row-major, one item at a time (OpenMP over items).
 * Second derivatives of the decoder are taken by naive forward-over-forward
 * differentiation, never by the adjoint identity the GPU library uses.
 */
#ifndef RS_ORACLE_H
#define RS_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    /* mesh: nv vertices X (nv x 3), ne tets (ne x 4), pinned[v]=1 fixes v at rest */
    int nv, ne;
    const double* X;
    const int* tets;
    const unsigned char* pinned;
    /* material: Young's modulus, Poisson ratio, density, gravity vector */
    double young, poisson, density, gravity[3];
    /* decoder: r -> L hidden layers of `width` (ELU) -> n_out = 3 nv (linear).
     * W[l] is (out x in) row-major, b[l] has `out` entries, l = 0..L. */
    int r, L, width, n_out;
    const double* const* W;
    const double* const* b;
    /* cubature: S elements with weights */
    int S;
    const int* cub_elem;
    const double* cub_w;
    /* penalty-targeted vertices (stiffness k_c) and force-loaded vertices */
    int nt;
    const int* target_vtx;
    double k_c;
    int nf;
    const int* force_vtx;
    /* implicit Euler (Sec. 3.1): time step dt, 0 = quasi-static (no inertia term);
     * the inertial targets qbar (displacements, n per item) are call arguments */
    double dt;
    /* ground contact: one-sided penalty k_ground/2 min(0, x_v,y - ground_y)^2 on
     * the nc contact vertices */
    int nc;
    const int* contact_vtx;
    double k_ground, ground_y;
} or_problem;

typedef struct {
    int max_iter;      /* Newton iterations (accepted steps) */
    int ls_max;        /* backtracking trials per iteration */
    double c1;         /* Armijo constant */
    double shrink;     /* step factor per trial */
    double rel_tol;    /* stop when |g|_inf <= rel_tol |g_0|_inf */
    double abs_tol;    /* ... or when |g|_inf <= abs_tol */
    int hess;          /* bit 0: exact (else Gauss-Newton); bit 1: per-element PSD projection */
    int proj;          /* 0 clamp eigenvalues, 1 absolute eigenvalues, 2 none */
    double eig_floor;  /* eigenvalue floor relative to max |eig| */
} or_opts;

typedef struct {
    int max_iter;      /* accepted steps (exit IV) */
    int ls_max;        /* backtracking trials per iteration (exit III) */
    int history;       /* (s, y) pairs kept */
    double c1;         /* Armijo constant */
    double shrink;     /* step factor per trial */
    double rel_tol;    /* stop when |g|_inf <= rel_tol |g_0|_inf */
    double abs_tol;    /* ... or when |g|_inf <= abs_tol */
} or_lbfgs_opts;

enum { OR_CONVERGED = 0, OR_NOT_DESCENT = 1, OR_LS_MAX = 2, OR_ITER_MAX = 3, OR_NONFINITE = 4 };
enum { OR_EXACT = 1, OR_ELASTIC_ONLY = 2, OR_ENERGY_ONLY = 4, OR_ELEM_PSD = 8 };

/* material and stable Neo-Hookean density (F is 3x3 row-major) */
void or_lame(double young, double poisson, double* mu, double* lam);
double or_psi(const double* F, double mu, double lam);
void or_pk1(const double* F, double mu, double lam, double* P);
void or_dpdf(const double* F, double mu, double lam, double* A); /* 9x9, vec = column-major */

/* one tetrahedron: rest corners Xe (4x3), deformed corners xe (4x3) */
void or_rest(const double* Xe, double* Dminv, double* V);
double or_elem_energy(const double* Xe, const double* xe, double mu, double lam);
void or_elem_grad(const double* Xe, const double* xe, double mu, double lam, double* g12);
void or_elem_hess(const double* Xe, const double* xe, double mu, double lam, double* H144);

void or_lumped_mass(const or_problem* p, double* m);

/* decoder: x (B x nv x 3) deformed positions, J (B x n x r) nullable */
int or_decode(const or_problem* p, int B, const double* z, double* x, double* J);
/* second derivatives of the deformed positions, one item: T (n x r x r) */
int or_decode_hess(const or_problem* p, const double* z, double* T);

/* reduced energy / gradient / Hessian at B latent points.
 * targets (B x nt x 3) and force (B x 3, applied to each force vertex) nullable;
 * qbar (B x n inertial target displacements) nullable, used when p->dt > 0:
 * E += 1/(2 dt^2) sum over free rows m_row (x_row - X_row - qbar_row)^2. */
int or_reduced(const or_problem* p, int B, const double* z, const double* targets,
               const double* force, const double* qbar, int flags, double* E, double* g, double* H);

/* Newton direction of one item: dz = -H^-1 g with the Cholesky factor of the
 * symmetrised H when it is positive definite, else with its eigen-projection
 * (proj 0: eigenvalues raised to eig_floor * max|eig|; 1: replaced by
 * max(|eig|, eig_floor * max|eig|); 2: none, returns 1).  Exposed for pins. */
int or_newton_dir(int n, const double* H, const double* g, int proj, double eig_floor, double* dz);

/* reduced projective Newton with backtracking line search, z in/out */
int or_newton(const or_problem* p, int B, double* z, const double* targets,
              const double* force, const double* qbar, const or_opts* o, int* iters, int* status,
              double* relgrad, double* E);

/* L-BFGS direction d = -H g by the two-loop recursion over npair (s, y)
 * pairs stored oldest first (rows of S, Y, each r long), H_0 = gamma I with
 * gamma = s'y / y'y of the newest pair (1 without pairs).  Exposed for pins. */
void or_lbfgs_dir(int r, int npair, const double* S, const double* Y, const double* g, double* d);

/* reduced L-BFGS with the same backtracking line search and exits as
 * or_newton (gradient only), z in/out */
int or_lbfgs(const or_problem* p, int B, double* z, const double* targets,
             const double* force, const double* qbar, const or_lbfgs_opts* o, int* iters, int* status,
             double* relgrad, double* E);

/* full-space Newton on the free DOFs over every mesh element (weight 1).
 * elem_psd=1 projects each 12x12 element Hessian to PSD; else the same
 * global policy as or_newton.  x (nv x 3) in/out. */
int or_full_newton(const or_problem* p, double* x, const double* targets,
                   const double* force, const double* qbar, const or_opts* o, int elem_psd,
                   int* iters, int* status, double* relgrad, double* E);
/* full-space energy / gradient (nv x 3) at x (qbar: n inertial target displacements, nullable) */
double or_full_energy(const or_problem* p, const double* x, const double* targets,
                      const double* force, const double* qbar, double* grad);

/* Lipschitz loss of the cubature elastic Hessian over pairs (z1_b, z2_b). */
int or_lipschitz(const or_problem* p, int B, const double* z1, const double* z2,
                 double* loss, double* per_pair, int* n_valid, double* lip_max);

/* Gradient of sum_b E(z_b) with respect to every decoder parameter (the
 * potential loss of the unsupervised subspace construction, Sec. 3.2), by
 * the chain rule written out: dE/dq at q(z_b), then back through the output
 * layer and the hidden layers.  grad: packed W_1, b_1, ..., W_L, b_L, W_out,
 * b_out, each W row-major (out x in); overwritten.  E: per-item energies
 * (nullable).  flags: OR_ELASTIC_ONLY. */
int or_energy_param_grad(const or_problem* p, int B, const double* z, const double* targets,
                         const double* force, int flags, double* E, double* grad);

/* Gradient of the Lipschitz loss mean_b |H(z1_b) - H(z2_b)|_F^2 / |z1_b - z2_b|^2
 * (H the exact cubature elastic Hessian, pairs with z1 = z2 excluded) with
 * respect to every decoder parameter (packed as or_energy_param_grad), by the
 * chain rule through the value, Jacobian and contracted second derivative of
 * every layer; loss is its value.  r <= 32.  Serial over pairs. */
int or_lipschitz_param_grad(const or_problem* p, int B, const double* z1, const double* z2,
                            double* loss, double* grad);

/* an ELU MLP n_in -> L hidden layers of `width` -> n_out (linear), W[l] (out x in) row-major */
typedef struct {
    int n_in, L, width, n_out;
    const double* const* W;
    const double* const* b;
} or_mlp;

/* Supervised reconstruction loss mean_i |X + m (.) f(g(q_i - X)) - q_i|_M^2 over B
 * positions q (B x n), M the lumped masses, g the encoder (n -> r), f the
 * problem's decoder; gradients of both networks (packed like
 * or_energy_param_grad, encoder first argument) are overwritten. */
int or_recon_loss_grad(const or_problem* p, const or_mlp* enc, int B, const double* q, double* loss,
                       double* grad_enc, double* grad_dec);
/* encoder values z (B x n_out) of inputs d (B x n_in) */
int or_encode(const or_mlp* enc, int B, const double* d, double* z);

/* number of OpenMP threads of the parallel loops (timing only) */
void or_set_threads(int n);

/* symmetric eigen-decomposition by cyclic Jacobi (exposed for pins) */
void or_sym_eig(int n, const double* A, double* evals, double* evecs);

#ifdef __cplusplus
}
#endif
#endif
