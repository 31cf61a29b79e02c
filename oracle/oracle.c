/*
 * FP64 CPU oracle for the reduced-Newton hot path (Lyu et al., TOG 2024).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the library's product path.
 *
 * Every quantity is computed from its plain definition, in float64, one item
 * at a time:
 *   - the reduced objective E(z) = P(f(z)) (+ external terms) of the reduced
 *     problem (Sec. 3.1, Eq. form-reduced-space-time-integration; quasi-static,
 *     inertia dropped), with the elastic potential replaced by its cubature sum
 *     P~ = sum_{e in S} w_e P_e (Sec. 4.3, Eq. form-cubature-gradients);
 *   - its gradient by the chain rule through the decoder Jacobian J = df/dz,
 *     and its Hessian J^T H J plus the decoder-curvature term sum_k g_k d2q_k/dz2
 *     (the Hessian the paper obtains by automatic differentiation, Sec. 5),
 *     with d2q/dz2 from forward-over-forward differentiation of the MLP;
 *   - projective Newton with backtracking line search and the paper's exit
 *     conditions (Sec. 5 solver description; supplement, projective Newton
 *     tests and convergence-condition discussion);
 *   - the Lipschitz loss of the cubature elastic Hessian (Sec. 4.1,
 *     Eq. form-L-LS-E) and its max-pair estimator (Eq. form-H-Lipschitz-estimation).
 * The stable Neo-Hookean density is only cited by the paper (Sec. 5.1); the
 * polynomial form psi = mu/2 (I_C - 3) - mu (J - 1) + lam/2 (J - 1)^2 is used,
 * with lam = lam_Lame + mu so that it linearises to the given (E, nu).
 */
#include "oracle.h"

#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* material                                                                  */
/* ------------------------------------------------------------------------- */
void or_lame(double young, double poisson, double* mu, double* lam)
{
    double m = young / (2.0 * (1.0 + poisson));
    double lame = young * poisson / ((1.0 + poisson) * (1.0 - 2.0 * poisson));
    *mu = m;
    *lam = lame + m;
}

static double det3(const double* F)
{
    return F[0] * (F[4] * F[8] - F[5] * F[7])
         - F[1] * (F[3] * F[8] - F[5] * F[6])
         + F[2] * (F[3] * F[7] - F[4] * F[6]);
}

/* cof[i][j] = d det(F) / d F[i][j] */
static void cofactor(const double* F, double* C)
{
    C[0] = F[4] * F[8] - F[5] * F[7];
    C[1] = F[5] * F[6] - F[3] * F[8];
    C[2] = F[3] * F[7] - F[4] * F[6];
    C[3] = F[2] * F[7] - F[1] * F[8];
    C[4] = F[0] * F[8] - F[2] * F[6];
    C[5] = F[1] * F[6] - F[0] * F[7];
    C[6] = F[1] * F[5] - F[2] * F[4];
    C[7] = F[2] * F[3] - F[0] * F[5];
    C[8] = F[0] * F[4] - F[1] * F[3];
}

double or_psi(const double* F, double mu, double lam)
{
    double ic = 0.0;
    for (int k = 0; k < 9; ++k) ic += F[k] * F[k];
    double J = det3(F);
    return 0.5 * mu * (ic - 3.0) - mu * (J - 1.0) + 0.5 * lam * (J - 1.0) * (J - 1.0);
}

/* P = d psi / d F = mu F + (lam (J-1) - mu) cof F */
void or_pk1(const double* F, double mu, double lam, double* P)
{
    double C[9];
    cofactor(F, C);
    double s = lam * (det3(F) - 1.0) - mu;
    for (int k = 0; k < 9; ++k) P[k] = mu * F[k] + s * C[k];
}

static int levi(int i, int j, int k)
{
    if (i == j || j == k || i == k) return 0;
    return ((i == 0 && j == 1) || (i == 1 && j == 2) || (i == 2 && j == 0)) ? 1 : -1;
}

/* A[v(i,j)][v(k,l)] = d^2 psi / dF_ij dF_kl with v(i,j) = 3 j + i (column-major vec).
 * d^2 J / dF_ij dF_kl = sum_m eps(j,l,c) eps(i,k,m) F_mc, c the column left over. */
void or_dpdf(const double* F, double mu, double lam, double* A)
{
    double C[9];
    cofactor(F, C);
    double s = lam * (det3(F) - 1.0) - mu;
    for (int j = 0; j < 3; ++j)
        for (int i = 0; i < 3; ++i)
            for (int l = 0; l < 3; ++l)
                for (int k = 0; k < 3; ++k) {
                    double hj = 0.0;
                    if (j != l) {
                        int c = 3 - j - l;
                        for (int m = 0; m < 3; ++m)
                            hj += levi(j, l, c) * levi(i, k, m) * F[3 * m + c];
                    }
                    double v = lam * C[3 * i + j] * C[3 * k + l] + s * hj;
                    if (i == k && j == l) v += mu;
                    A[(3 * j + i) * 9 + (3 * l + k)] = v;
                }
}

/* ------------------------------------------------------------------------- */
/* one linear tetrahedron                                                    */
/* ------------------------------------------------------------------------- */
static void inv3(const double* M, double* Mi)
{
    double C[9];
    cofactor(M, C);
    double d = det3(M);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Mi[3 * i + j] = C[3 * j + i] / d;
}

/* Dm[i][k] = X_{k+1,i} - X_{0,i};  V = det(Dm)/6 */
void or_rest(const double* Xe, double* Dminv, double* V)
{
    double Dm[9];
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) Dm[3 * i + k] = Xe[3 * (k + 1) + i] - Xe[i];
    inv3(Dm, Dminv);
    *V = det3(Dm) / 6.0;
}

/* F = Ds Dm^{-1} */
static void deform_grad(const double* Dminv, const double* xe, double* F)
{
    double Ds[9];
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) Ds[3 * i + k] = xe[3 * (k + 1) + i] - xe[i];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += Ds[3 * i + k] * Dminv[3 * k + j];
            F[3 * i + j] = s;
        }
}

/* dF_ij / dx_{a,m} = delta_im * Dv[a][j],  Dv[a][j] = Dminv[a-1][j] (a>=1), -sum (a=0) */
static void shape_grad(const double* Dminv, double* Dv)
{
    for (int j = 0; j < 3; ++j) {
        double s = 0.0;
        for (int a = 1; a < 4; ++a) {
            Dv[3 * a + j] = Dminv[3 * (a - 1) + j];
            s += Dminv[3 * (a - 1) + j];
        }
        Dv[j] = -s;
    }
}

double or_elem_energy(const double* Xe, const double* xe, double mu, double lam)
{
    double Dminv[9], V, F[9];
    or_rest(Xe, Dminv, &V);
    deform_grad(Dminv, xe, F);
    return V * or_psi(F, mu, lam);
}

static void elem_grad_dm(const double* Dminv, double V, const double* xe, double mu,
                         double lam, double* g12)
{
    double F[9], P[9], Dv[12];
    deform_grad(Dminv, xe, F);
    or_pk1(F, mu, lam, P);
    shape_grad(Dminv, Dv);
    for (int a = 0; a < 4; ++a)
        for (int m = 0; m < 3; ++m) {
            double s = 0.0;
            for (int j = 0; j < 3; ++j) s += P[3 * m + j] * Dv[3 * a + j];
            g12[3 * a + m] = V * s;
        }
}

static void elem_hess_dm(const double* Dminv, double V, const double* xe, double mu,
                         double lam, double* H)
{
    double F[9], A[81], Dv[12];
    deform_grad(Dminv, xe, F);
    or_dpdf(F, mu, lam, A);
    shape_grad(Dminv, Dv);
    for (int a = 0; a < 4; ++a)
        for (int m = 0; m < 3; ++m)
            for (int b = 0; b < 4; ++b)
                for (int n = 0; n < 3; ++n) {
                    double s = 0.0;
                    for (int j = 0; j < 3; ++j)
                        for (int l = 0; l < 3; ++l)
                            s += Dv[3 * a + j] * Dv[3 * b + l] * A[(3 * j + m) * 9 + (3 * l + n)];
                    H[(3 * a + m) * 12 + 3 * b + n] = V * s;
                }
}

void or_elem_grad(const double* Xe, const double* xe, double mu, double lam, double* g12)
{
    double Dminv[9], V;
    or_rest(Xe, Dminv, &V);
    elem_grad_dm(Dminv, V, xe, mu, lam, g12);
}

void or_elem_hess(const double* Xe, const double* xe, double mu, double lam, double* H144)
{
    double Dminv[9], V;
    or_rest(Xe, Dminv, &V);
    elem_hess_dm(Dminv, V, xe, mu, lam, H144);
}

/* lumped mass: each tet gives rho V / 4 to each of its corners */
void or_lumped_mass(const or_problem* p, double* m)
{
    memset(m, 0, sizeof(double) * p->nv);
    for (int e = 0; e < p->ne; ++e) {
        double Xe[12], Dminv[9], V;
        for (int a = 0; a < 4; ++a)
            for (int i = 0; i < 3; ++i) Xe[3 * a + i] = p->X[3 * p->tets[4 * e + a] + i];
        or_rest(Xe, Dminv, &V);
        for (int a = 0; a < 4; ++a) m[p->tets[4 * e + a]] += p->density * V / 4.0;
    }
}

/* ------------------------------------------------------------------------- */
/* symmetric eigen-decomposition (cyclic Jacobi rotations)                    */
/* ------------------------------------------------------------------------- */
void or_sym_eig(int n, const double* A0, double* evals, double* V)
{
    double* A = (double*)malloc(sizeof(double) * n * n);
    memcpy(A, A0, sizeof(double) * n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) V[i * n + j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += A[i * n + j] * A[i * n + j];
                if (i != j) off += A[i * n + j] * A[i * n + j];
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = A[p * n + q];
                if (apq == 0.0) continue;
                /* rotation zeroing A[p][q]: tan(2t) = 2 apq / (aqq - app) */
                double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) { /* columns p, q */
                    double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) { /* rows p, q */
                    double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    double vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = c * vkp - s * vkq;
                    V[k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    for (int i = 0; i < n; ++i) evals[i] = A[i * n + i];
    free(A);
}

/* ------------------------------------------------------------------------- */
/* decoder (MLP with ELU hidden layers, linear output)                        */
/* ------------------------------------------------------------------------- */
static double elu(double a) { return a > 0.0 ? a : expm1(a); }
static double elu1(double a) { return a > 0.0 ? 1.0 : exp(a); }
static double elu2(double a) { return a > 0.0 ? 0.0 : exp(a); }

typedef struct {
    double *h, *J, *T; /* last hidden layer: h (w), J (w x r), T (w x r x r) or NULL */
    int nin;
} dec_state;

/* forward-mode value, Jacobian and (optionally) second derivative through the
 * hidden layers; on return st holds the input of the output layer. */
static void decoder_hidden(const or_problem* p, const double* z, int want_T, dec_state* st)
{
    int r = p->r, w = p->width;
    int cap = (r > w ? r : w);
    double* h = (double*)calloc(cap, sizeof(double));
    double* J = (double*)calloc((size_t)cap * r, sizeof(double));
    double* T = want_T ? (double*)calloc((size_t)cap * r * r, sizeof(double)) : NULL;
    for (int k = 0; k < r; ++k) { h[k] = z[k]; J[k * r + k] = 1.0; }
    int nin = r;
    double* h2 = (double*)calloc(cap, sizeof(double));
    double* J2 = (double*)calloc((size_t)cap * r, sizeof(double));
    double* T2 = want_T ? (double*)calloc((size_t)cap * r * r, sizeof(double)) : NULL;
    for (int l = 0; l < p->L; ++l) {
        const double* W = p->W[l];
        const double* b = p->b[l];
        for (int i = 0; i < w; ++i) {
            double a = b[i];
            for (int j = 0; j < nin; ++j) a += W[i * nin + j] * h[j];
            double s1 = elu1(a), s2 = elu2(a);
            h2[i] = elu(a);
            for (int k = 0; k < r; ++k) {
                double Ak = 0.0;
                for (int j = 0; j < nin; ++j) Ak += W[i * nin + j] * J[j * r + k];
                J2[i * r + k] = s1 * Ak;
            }
            if (want_T) {
                /* T'_i = s'' A_i (x) A_i + s' (W T)_i, A_i the pre-activation row */
                for (int k = 0; k < r; ++k)
                    for (int q = 0; q < r; ++q) {
                        double Ak = 0.0, Aq = 0.0, Tkq = 0.0;
                        for (int j = 0; j < nin; ++j) {
                            Ak += W[i * nin + j] * J[j * r + k];
                            Aq += W[i * nin + j] * J[j * r + q];
                            Tkq += W[i * nin + j] * T[(j * r + k) * r + q];
                        }
                        T2[(i * r + k) * r + q] = s2 * Ak * Aq + s1 * Tkq;
                    }
            }
        }
        double* t;
        t = h; h = h2; h2 = t;
        t = J; J = J2; J2 = t;
        t = T; T = T2; T2 = t;
        nin = w;
    }
    free(h2); free(J2); free(T2);
    st->h = h; st->J = J; st->T = T; st->nin = nin;
}

static void dec_free(dec_state* st) { free(st->h); free(st->J); free(st->T); }

/* q = X + m (.) (W_out h + b_out), J_q = m (.) W_out J (all rows) */
static void decoder_output(const or_problem* p, const dec_state* st, double* x, double* Jq)
{
    int r = p->r, nin = st->nin;
    const double* W = p->W[p->L];
    const double* b = p->b[p->L];
    for (int row = 0; row < p->n_out; ++row) {
        int v = row / 3;
        int fixed = p->pinned[v];
        double u = b[row];
        for (int j = 0; j < nin; ++j) u += W[row * nin + j] * st->h[j];
        x[row] = p->X[row] + (fixed ? 0.0 : u);
        if (Jq)
            for (int k = 0; k < r; ++k) {
                double s = 0.0;
                if (!fixed)
                    for (int j = 0; j < nin; ++j) s += W[row * nin + j] * st->J[j * r + k];
                Jq[(size_t)row * r + k] = s;
            }
    }
}

/* d2 q_row / dz2 (r x r) = m_row * sum_j W_out[row][j] T[j] */
static void decoder_row_hess(const or_problem* p, const dec_state* st, int row, double* Trow)
{
    int r = p->r, nin = st->nin;
    const double* W = p->W[p->L];
    memset(Trow, 0, sizeof(double) * r * r);
    if (p->pinned[row / 3]) return;
    for (int j = 0; j < nin; ++j) {
        double wj = W[row * nin + j];
        for (int kq = 0; kq < r * r; ++kq) Trow[kq] += wj * st->T[(size_t)j * r * r + kq];
    }
}

int or_decode(const or_problem* p, int B, const double* z, double* x, double* J)
{
    size_t n = (size_t)p->n_out, r = (size_t)p->r;
#pragma omp parallel for schedule(dynamic)
    for (int bi = 0; bi < B; ++bi) {
        dec_state st;
        decoder_hidden(p, z + bi * r, 0, &st);
        decoder_output(p, &st, x + bi * n, J ? J + bi * n * r : NULL);
        dec_free(&st);
    }
    return 0;
}

int or_decode_hess(const or_problem* p, const double* z, double* T)
{
    int r = p->r;
    dec_state st;
    decoder_hidden(p, z, 1, &st);
    for (int row = 0; row < p->n_out; ++row) decoder_row_hess(p, &st, row, T + (size_t)row * r * r);
    dec_free(&st);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* reduced objective, gradient and Hessian at one latent point               */
/* ------------------------------------------------------------------------- */
typedef struct {
    double mu, lam;
    double* Dminv; /* ne x 9 */
    double* V;     /* ne */
    double* mass;  /* nv */
} rest_data;

static void rest_build(const or_problem* p, rest_data* rd)
{
    or_lame(p->young, p->poisson, &rd->mu, &rd->lam);
    rd->Dminv = (double*)malloc(sizeof(double) * 9 * p->ne);
    rd->V = (double*)malloc(sizeof(double) * p->ne);
    rd->mass = (double*)malloc(sizeof(double) * p->nv);
    for (int e = 0; e < p->ne; ++e) {
        double Xe[12];
        for (int a = 0; a < 4; ++a)
            for (int i = 0; i < 3; ++i) Xe[3 * a + i] = p->X[3 * p->tets[4 * e + a] + i];
        or_rest(Xe, rd->Dminv + 9 * e, rd->V + e);
    }
    or_lumped_mass(p, rd->mass);
}

static void rest_free(rest_data* rd) { free(rd->Dminv); free(rd->V); free(rd->mass); }

static void gather(const or_problem* p, int e, const double* x, double* xe)
{
    for (int a = 0; a < 4; ++a)
        for (int i = 0; i < 3; ++i) xe[3 * a + i] = x[3 * p->tets[4 * e + a] + i];
}

/* energy and q-space gradient gq (n) of the reduced objective at positions x:
 * cubature elastic sum (+ gravity, penalty and nodal forces unless elastic-only) */
/* inertia and ground contact (implicit Euler, Sec. 3.1): energy, gradient
 * rows, and (H_diag, nullable) the diagonal of their q-Hessian */
static double dyn_energy(const or_problem* p, const rest_data* rd, const double* x, const double* qb,
                         double* gq, double* H_diag)
{
    double E = 0.0;
    if (p->dt > 0.0 && qb) {
        const double c = 1.0 / (p->dt * p->dt);
        for (int row = 0; row < p->n_out; ++row) {
            if (p->pinned[row / 3]) continue;
            const double m = rd->mass[row / 3];
            const double d = x[row] - p->X[row] - qb[row];
            E += 0.5 * c * m * d * d;
            if (gq) gq[row] += c * m * d;
            if (H_diag) H_diag[row] += c * m;
        }
    }
    for (int k = 0; k < p->nc; ++k) {
        const int row = 3 * p->contact_vtx[k] + 1;
        const double d = x[row] - p->ground_y;
        if (d < 0.0) {
            E += 0.5 * p->k_ground * d * d;
            if (gq) gq[row] += p->k_ground * d;
            if (H_diag) H_diag[row] += p->k_ground;
        }
    }
    return E;
}

static double q_energy(const or_problem* p, const rest_data* rd, const double* x,
                       const double* tgt, const double* f, const double* qb, int flags, double* gq)
{
    double E = 0.0;
    if (gq) memset(gq, 0, sizeof(double) * p->n_out);
    for (int s = 0; s < p->S; ++s) {
        int e = p->cub_elem[s];
        double xe[12], F[9];
        gather(p, e, x, xe);
        deform_grad(rd->Dminv + 9 * e, xe, F);
        E += p->cub_w[s] * rd->V[e] * or_psi(F, rd->mu, rd->lam);
        if (gq) {
            double g12[12];
            elem_grad_dm(rd->Dminv + 9 * e, rd->V[e], xe, rd->mu, rd->lam, g12);
            for (int a = 0; a < 4; ++a)
                for (int i = 0; i < 3; ++i) gq[3 * p->tets[4 * e + a] + i] += p->cub_w[s] * g12[3 * a + i];
        }
    }
    if (flags & OR_ELASTIC_ONLY) return E;
    /* gravity: -sum_v m_v g . (x_v - X_v) */
    for (int v = 0; v < p->nv; ++v)
        for (int i = 0; i < 3; ++i) {
            E -= rd->mass[v] * p->gravity[i] * (x[3 * v + i] - p->X[3 * v + i]);
            if (gq) gq[3 * v + i] -= rd->mass[v] * p->gravity[i];
        }
    /* penalty: k_c/2 |x_v - t_v|^2 */
    if (tgt)
        for (int c = 0; c < p->nt; ++c) {
            int v = p->target_vtx[c];
            for (int i = 0; i < 3; ++i) {
                double d = x[3 * v + i] - tgt[3 * c + i];
                E += 0.5 * p->k_c * d * d;
                if (gq) gq[3 * v + i] += p->k_c * d;
            }
        }
    /* nodal forces: -f . (x_v - X_v) on each force vertex */
    if (f)
        for (int c = 0; c < p->nf; ++c) {
            int v = p->force_vtx[c];
            for (int i = 0; i < 3; ++i) {
                E -= f[i] * (x[3 * v + i] - p->X[3 * v + i]);
                if (gq) gq[3 * v + i] -= f[i];
            }
        }
    E += dyn_energy(p, rd, x, qb, gq, NULL);
    return E;
}

static int finite_vec(const double* a, int n)
{
    for (int i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

/* per-element projection to positive semi-definite: the 12x12 element
 * Hessian's negative eigenvalues set to zero (Jacobi eigen-decomposition) */
static void psd_clamp12(double* He)
{
    double lam[12], Vv[144];
    or_sym_eig(12, He, lam, Vv);
    for (int u = 0; u < 12; ++u)
        for (int v = 0; v < 12; ++v) {
            double s = 0.0;
            for (int k = 0; k < 12; ++k) s += Vv[u * 12 + k] * fmax(lam[k], 0.0) * Vv[v * 12 + k];
            He[u * 12 + v] = s;
        }
}

/* E, g_r = J^T gq and H_r = sum_e w_e J_e^T H_e J_e + k_c sum_t J_t^T J_t
 * (+ sum_k gq_k d2q_k/dz2 when exact) at one latent point; with OR_ELEM_PSD
 * each element Hessian H_e is first projected to positive semi-definite */
static void item_eval(const or_problem* p, const rest_data* rd, const double* z,
                      const double* tgt, const double* f, const double* qb, int flags, double* E,
                      double* g, double* H)
{
    int r = p->r, n = p->n_out;
    int want_H = !(flags & OR_ENERGY_ONLY) && H;
    int want_g = !(flags & OR_ENERGY_ONLY) && g;
    int exact = want_H && (flags & OR_EXACT);
    dec_state st;
    decoder_hidden(p, z, exact, &st);
    double* x = (double*)malloc(sizeof(double) * n);
    double* Jq = (want_g || want_H) ? (double*)malloc(sizeof(double) * (size_t)n * r) : NULL;
    double* gq = (want_g || want_H) ? (double*)malloc(sizeof(double) * n) : NULL;
    decoder_output(p, &st, x, Jq);
    *E = q_energy(p, rd, x, tgt, f, qb, flags, gq);
    if (want_g)
        for (int k = 0; k < r; ++k) {
            double s = 0.0;
            for (int row = 0; row < n; ++row) s += Jq[(size_t)row * r + k] * gq[row];
            g[k] = s;
        }
    if (want_H) {
        memset(H, 0, sizeof(double) * r * r);
        double He[144];
        double* JeA = (double*)malloc(sizeof(double) * 12 * r);
        for (int s = 0; s < p->S; ++s) {
            int e = p->cub_elem[s];
            double xe[12];
            gather(p, e, x, xe);
            elem_hess_dm(rd->Dminv + 9 * e, rd->V[e], xe, rd->mu, rd->lam, He);
            if (flags & OR_ELEM_PSD) psd_clamp12(He);
            for (int a = 0; a < 4; ++a)
                for (int i = 0; i < 3; ++i)
                    for (int k = 0; k < r; ++k)
                        JeA[(3 * a + i) * r + k] = Jq[(size_t)(3 * p->tets[4 * e + a] + i) * r + k];
            for (int k = 0; k < r; ++k)
                for (int q = 0; q < r; ++q) {
                    double acc = 0.0;
                    for (int u = 0; u < 12; ++u)
                        for (int v = 0; v < 12; ++v) acc += JeA[u * r + k] * He[u * 12 + v] * JeA[v * r + q];
                    H[k * r + q] += p->cub_w[s] * acc;
                }
        }
        free(JeA);
        if (!(flags & OR_ELASTIC_ONLY) && tgt)
            for (int c = 0; c < p->nt; ++c) {
                int v = p->target_vtx[c];
                for (int i = 0; i < 3; ++i) {
                    const double* Jr = Jq + (size_t)(3 * v + i) * r;
                    for (int k = 0; k < r; ++k)
                        for (int q = 0; q < r; ++q) H[k * r + q] += p->k_c * Jr[k] * Jr[q];
                }
            }
        if (!(flags & OR_ELASTIC_ONLY) && ((p->dt > 0.0 && qb) || p->nc > 0)) {
            /* inertia and contact: J_row^T (d2E/dq_row^2) J_row */
            double* Hd = (double*)calloc(n, sizeof(double));
            dyn_energy(p, rd, x, qb, NULL, Hd);
            for (int row = 0; row < n; ++row) {
                if (Hd[row] == 0.0) continue;
                const double* Jr = Jq + (size_t)row * r;
                for (int k = 0; k < r; ++k)
                    for (int q = 0; q < r; ++q) H[k * r + q] += Hd[row] * Jr[k] * Jr[q];
            }
            free(Hd);
        }
        if (exact) {
            double* Trow = (double*)malloc(sizeof(double) * r * r);
            for (int row = 0; row < n; ++row) {
                if (gq[row] == 0.0) continue; /* zero terms contribute nothing */
                decoder_row_hess(p, &st, row, Trow);
                for (int kq = 0; kq < r * r; ++kq) H[kq] += gq[row] * Trow[kq];
            }
            free(Trow);
        }
    }
    free(x); free(Jq); free(gq);
    dec_free(&st);
}

int or_reduced(const or_problem* p, int B, const double* z, const double* targets,
               const double* force, const double* qbar, int flags, double* E, double* g, double* H)
{
    rest_data rd;
    rest_build(p, &rd);
    int r = p->r;
#pragma omp parallel for schedule(dynamic)
    for (int bi = 0; bi < B; ++bi)
        item_eval(p, &rd, z + (size_t)bi * r, targets ? targets + (size_t)bi * p->nt * 3 : NULL,
                  force ? force + (size_t)bi * 3 : NULL, qbar ? qbar + (size_t)bi * p->n_out : NULL, flags,
                  E + bi, g ? g + (size_t)bi * r : NULL,
                  H ? H + (size_t)bi * r * r : NULL);
    rest_free(&rd);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Newton direction: Cholesky of the symmetrised Hessian when it is positive  */
/* definite, else its eigen-projection (clamped or absolute eigenvalues).     */
/* Returns 0 on success, 1 when no direction is produced (no projection).     */
/* ------------------------------------------------------------------------- */
static int cholesky(int n, double* A)
{
    for (int j = 0; j < n; ++j) {
        double d = A[j * n + j];
        for (int k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
        if (!(d > 0.0) || !isfinite(d)) return 1;
        d = sqrt(d);
        A[j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double s = A[i * n + j];
            for (int k = 0; k < j; ++k) s -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = s / d;
        }
    }
    return 0;
}

static int newton_dir(int n, const double* H, const double* g, int proj, double floor_rel, double* dz)
{
    double* Hs = (double*)malloc(sizeof(double) * n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Hs[i * n + j] = 0.5 * (H[i * n + j] + H[j * n + i]);
    double* L = (double*)malloc(sizeof(double) * n * n);
    memcpy(L, Hs, sizeof(double) * n * n);
    int rc = 0;
    if (cholesky(n, L) == 0) {
        double* y = (double*)malloc(sizeof(double) * n);
        for (int i = 0; i < n; ++i) { /* L y = -g */
            double s = -g[i];
            for (int k = 0; k < i; ++k) s -= L[i * n + k] * y[k];
            y[i] = s / L[i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) { /* L^T dz = y */
            double s = y[i];
            for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * dz[k];
            dz[i] = s / L[i * n + i];
        }
        free(y);
    } else if (proj == 2) {
        rc = 1;
    } else {
        double* lam = (double*)malloc(sizeof(double) * n);
        double* V = (double*)malloc(sizeof(double) * n * n);
        or_sym_eig(n, Hs, lam, V);
        double lmax = 0.0;
        for (int i = 0; i < n; ++i) lmax = fmax(lmax, fabs(lam[i]));
        double fl = floor_rel * lmax;
        for (int i = 0; i < n; ++i) dz[i] = 0.0;
        for (int k = 0; k < n; ++k) {
            double lk = (proj == 1) ? fabs(lam[k]) : lam[k];
            if (lk < fl) lk = fl;
            if (!(lk > 0.0)) lk = 1.0; /* zero matrix: steepest descent */
            double c = 0.0;
            for (int i = 0; i < n; ++i) c += V[i * n + k] * g[i];
            for (int i = 0; i < n; ++i) dz[i] -= V[i * n + k] * c / lk;
        }
        free(lam); free(V);
    }
    free(Hs); free(L);
    return rc;
}

int or_newton_dir(int n, const double* H, const double* g, int proj, double eig_floor, double* dz)
{
    return newton_dir(n, H, g, proj, eig_floor, dz);
}

static double inf_norm(const double* a, int n)
{
    double m = 0.0;
    for (int i = 0; i < n; ++i) m = fmax(m, fabs(a[i]));
    return m;
}

static void item_newton(const or_problem* p, const rest_data* rd, double* z, const double* tgt,
                        const double* f, const double* qb, const or_opts* o, int* iters, int* status,
                        double* relgrad, double* Eout)
{
    int r = p->r;
    int flags = ((o->hess & 1) ? OR_EXACT : 0) | ((o->hess & 2) ? OR_ELEM_PSD : 0);
    double* g = (double*)malloc(sizeof(double) * r);
    double* H = (double*)malloc(sizeof(double) * r * r);
    double* dz = (double*)malloc(sizeof(double) * r);
    double* zt = (double*)malloc(sizeof(double) * r);
    double E;
    item_eval(p, rd, z, tgt, f, qb, flags, &E, g, H);
    double g0 = inf_norm(g, r), gn = g0;
    int it = 0, st;
    for (;;) {
        if (!isfinite(E) || !finite_vec(g, r) || !finite_vec(H, r * r)) { st = OR_NONFINITE; break; }
        gn = inf_norm(g, r);
        if (gn <= o->abs_tol || gn <= o->rel_tol * g0) { st = OR_CONVERGED; break; }
        if (it >= o->max_iter) { st = OR_ITER_MAX; break; }
        if (newton_dir(r, H, g, o->proj, o->eig_floor, dz)) { st = OR_NOT_DESCENT; break; }
        double slope = 0.0;
        for (int k = 0; k < r; ++k) slope += g[k] * dz[k];
        if (!(slope < 0.0)) { st = OR_NOT_DESCENT; break; }
        double alpha = 1.0, Et = 0.0;
        int ok = 0;
        for (int t = 0; t < o->ls_max; ++t) {
            for (int k = 0; k < r; ++k) zt[k] = z[k] + alpha * dz[k];
            item_eval(p, rd, zt, tgt, f, qb, OR_ENERGY_ONLY, &Et, NULL, NULL);
            if (isfinite(Et) && Et - E <= o->c1 * alpha * slope) { ok = 1; break; }
            alpha *= o->shrink;
        }
        if (!ok) { st = OR_LS_MAX; break; }
        memcpy(z, zt, sizeof(double) * r);
        ++it;
        item_eval(p, rd, z, tgt, f, qb, flags, &E, g, H);
    }
    *iters = it;
    *status = st;
    *relgrad = g0 > 0.0 ? gn / g0 : 0.0;
    *Eout = E;
    free(g); free(H); free(dz); free(zt);
}

int or_newton(const or_problem* p, int B, double* z, const double* targets, const double* force,
              const double* qbar, const or_opts* o, int* iters, int* status, double* relgrad, double* E)
{
    rest_data rd;
    rest_build(p, &rd);
#pragma omp parallel for schedule(dynamic)
    for (int bi = 0; bi < B; ++bi)
        item_newton(p, &rd, z + (size_t)bi * p->r, targets ? targets + (size_t)bi * p->nt * 3 : NULL,
                    force ? force + (size_t)bi * 3 : NULL, qbar ? qbar + (size_t)bi * p->n_out : NULL, o,
                    iters + bi, status + bi, relgrad + bi, E + bi);
    rest_free(&rd);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* reduced L-BFGS (the paper's main solver, Sec. 5): limited-memory BFGS      */
/* inverse-Hessian products by the two-loop recursion (Nocedal and Wright,   */
/* Numerical Optimization, Alg. 7.4), the Armijo backtracking of or_newton.  */
/* ------------------------------------------------------------------------- */
static double dot(const double* a, const double* b, int n)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

void or_lbfgs_dir(int r, int npair, const double* S, const double* Y, const double* g, double* d)
{
    double* q = (double*)malloc(sizeof(double) * r);
    double* alpha = (double*)malloc(sizeof(double) * (npair > 0 ? npair : 1));
    for (int k = 0; k < r; ++k) q[k] = g[k];
    /* newest pair first */
    for (int i = npair - 1; i >= 0; --i) {
        const double* si = S + (size_t)i * r;
        const double* yi = Y + (size_t)i * r;
        alpha[i] = dot(si, q, r) / dot(yi, si, r);
        for (int k = 0; k < r; ++k) q[k] -= alpha[i] * yi[k];
    }
    double gamma = 1.0;
    if (npair > 0) {
        const double* sn = S + (size_t)(npair - 1) * r;
        const double* yn = Y + (size_t)(npair - 1) * r;
        gamma = dot(sn, yn, r) / dot(yn, yn, r);
    }
    for (int k = 0; k < r; ++k) q[k] *= gamma;
    /* oldest pair first */
    for (int i = 0; i < npair; ++i) {
        const double* si = S + (size_t)i * r;
        const double* yi = Y + (size_t)i * r;
        const double beta = dot(yi, q, r) / dot(yi, si, r);
        for (int k = 0; k < r; ++k) q[k] += si[k] * (alpha[i] - beta);
    }
    for (int k = 0; k < r; ++k) d[k] = -q[k];
    free(q); free(alpha);
}

static void item_lbfgs(const or_problem* p, const rest_data* rd, double* z, const double* tgt,
                       const double* f, const double* qb, const or_lbfgs_opts* o, int* iters, int* status,
                       double* relgrad, double* Eout)
{
    int r = p->r, m = o->history;
    double* g = (double*)malloc(sizeof(double) * r);
    double* gold = (double*)malloc(sizeof(double) * r);
    double* dz = (double*)malloc(sizeof(double) * r);
    double* zt = (double*)malloc(sizeof(double) * r);
    double* S = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1) * r);
    double* Y = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1) * r);
    double* s_new = (double*)malloc(sizeof(double) * r);
    double* y_new = (double*)malloc(sizeof(double) * r);
    double E;
    int npair = 0;
    item_eval(p, rd, z, tgt, f, qb, 0, &E, g, NULL);
    double g0 = inf_norm(g, r), gn = g0;
    int it = 0, st;
    for (;;) {
        if (!isfinite(E) || !finite_vec(g, r)) { st = OR_NONFINITE; break; }
        gn = inf_norm(g, r);
        if (gn <= o->abs_tol || gn <= o->rel_tol * g0) { st = OR_CONVERGED; break; }
        if (it >= o->max_iter) { st = OR_ITER_MAX; break; }
        or_lbfgs_dir(r, npair, S, Y, g, dz);
        const double slope = dot(g, dz, r);
        if (!(slope < 0.0)) { st = OR_NOT_DESCENT; break; }
        double alpha = 1.0, Et = 0.0;
        int ok = 0;
        for (int t = 0; t < o->ls_max; ++t) {
            for (int k = 0; k < r; ++k) zt[k] = z[k] + alpha * dz[k];
            item_eval(p, rd, zt, tgt, f, qb, OR_ENERGY_ONLY, &Et, NULL, NULL);
            if (isfinite(Et) && Et - E <= o->c1 * alpha * slope) { ok = 1; break; }
            alpha *= o->shrink;
        }
        if (!ok) { st = OR_LS_MAX; break; }
        /* s = z_new - z, y = g_new - g; the pair is kept only when s'y > 0
         * (curvature condition: Armijo backtracking does not enforce it) */
        for (int k = 0; k < r; ++k) s_new[k] = zt[k] - z[k];
        memcpy(gold, g, sizeof(double) * r);
        memcpy(z, zt, sizeof(double) * r);
        ++it;
        item_eval(p, rd, z, tgt, f, qb, 0, &E, g, NULL);
        for (int k = 0; k < r; ++k) y_new[k] = g[k] - gold[k];
        if (m > 0 && dot(s_new, y_new, r) > 0.0) {
            if (npair == m) { /* drop the oldest */
                memmove(S, S + r, sizeof(double) * (size_t)(m - 1) * r);
                memmove(Y, Y + r, sizeof(double) * (size_t)(m - 1) * r);
                --npair;
            }
            memcpy(S + (size_t)npair * r, s_new, sizeof(double) * r);
            memcpy(Y + (size_t)npair * r, y_new, sizeof(double) * r);
            ++npair;
        }
    }
    *iters = it;
    *status = st;
    *relgrad = g0 > 0.0 ? gn / g0 : 0.0;
    *Eout = E;
    free(g); free(gold); free(dz); free(zt); free(S); free(Y); free(s_new); free(y_new);
}

int or_lbfgs(const or_problem* p, int B, double* z, const double* targets, const double* force,
             const double* qbar, const or_lbfgs_opts* o, int* iters, int* status, double* relgrad, double* E)
{
    if (o->history < 0) return 1;
    rest_data rd;
    rest_build(p, &rd);
#pragma omp parallel for schedule(dynamic)
    for (int bi = 0; bi < B; ++bi)
        item_lbfgs(p, &rd, z + (size_t)bi * p->r, targets ? targets + (size_t)bi * p->nt * 3 : NULL,
                   force ? force + (size_t)bi * 3 : NULL, qbar ? qbar + (size_t)bi * p->n_out : NULL, o,
                   iters + bi, status + bi, relgrad + bi, E + bi);
    rest_free(&rd);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* full-space reference: Newton on the free vertex DOFs over every mesh element */
/* ------------------------------------------------------------------------- */
static double full_energy(const or_problem* p, const rest_data* rd, const double* x,
                          const double* tgt, const double* f, const double* qb, double* grad)
{
    double E = 0.0;
    if (grad) memset(grad, 0, sizeof(double) * p->n_out);
    for (int e = 0; e < p->ne; ++e) {
        double xe[12], F[9];
        gather(p, e, x, xe);
        deform_grad(rd->Dminv + 9 * e, xe, F);
        E += rd->V[e] * or_psi(F, rd->mu, rd->lam);
        if (grad) {
            double g12[12];
            elem_grad_dm(rd->Dminv + 9 * e, rd->V[e], xe, rd->mu, rd->lam, g12);
            for (int a = 0; a < 4; ++a)
                for (int i = 0; i < 3; ++i) grad[3 * p->tets[4 * e + a] + i] += g12[3 * a + i];
        }
    }
    for (int v = 0; v < p->nv; ++v)
        for (int i = 0; i < 3; ++i) {
            E -= rd->mass[v] * p->gravity[i] * (x[3 * v + i] - p->X[3 * v + i]);
            if (grad) grad[3 * v + i] -= rd->mass[v] * p->gravity[i];
        }
    if (tgt)
        for (int c = 0; c < p->nt; ++c) {
            int v = p->target_vtx[c];
            for (int i = 0; i < 3; ++i) {
                double d = x[3 * v + i] - tgt[3 * c + i];
                E += 0.5 * p->k_c * d * d;
                if (grad) grad[3 * v + i] += p->k_c * d;
            }
        }
    if (f)
        for (int c = 0; c < p->nf; ++c) {
            int v = p->force_vtx[c];
            for (int i = 0; i < 3; ++i) {
                E -= f[i] * (x[3 * v + i] - p->X[3 * v + i]);
                if (grad) grad[3 * v + i] -= f[i];
            }
        }
    E += dyn_energy(p, rd, x, qb, grad, NULL);
    return E;
}

double or_full_energy(const or_problem* p, const double* x, const double* targets,
                      const double* force, const double* qbar, double* grad)
{
    rest_data rd;
    rest_build(p, &rd);
    double E = full_energy(p, &rd, x, targets, force, qbar, grad);
    rest_free(&rd);
    return E;
}

int or_full_newton(const or_problem* p, double* x, const double* tgt, const double* f,
                   const double* qb, const or_opts* o, int elem_psd, int* iters, int* status, double* relgrad,
                   double* Eout)
{
    rest_data rd;
    rest_build(p, &rd);
    int n = p->n_out;
    int* idx = (int*)malloc(sizeof(int) * n);
    int nf = 0;
    for (int row = 0; row < n; ++row) idx[row] = p->pinned[row / 3] ? -1 : nf++;
    double* grad = (double*)malloc(sizeof(double) * n);
    double* gf = (double*)malloc(sizeof(double) * nf);
    double* H = (double*)malloc(sizeof(double) * (size_t)nf * nf);
    double* dz = (double*)malloc(sizeof(double) * nf);
    double* xt = (double*)malloc(sizeof(double) * n);
    double He[144];
    double E = 0.0, g0 = 0.0, gn = 0.0;
    int it = 0, st;
    for (;;) {
        E = full_energy(p, &rd, x, tgt, f, qb, grad);
        for (int row = 0; row < n; ++row)
            if (idx[row] >= 0) gf[idx[row]] = grad[row];
        gn = inf_norm(gf, nf);
        if (it == 0) g0 = gn;
        if (!isfinite(E) || !finite_vec(gf, nf)) { st = OR_NONFINITE; break; }
        if (gn <= o->abs_tol || gn <= o->rel_tol * g0) { st = OR_CONVERGED; break; }
        if (it >= o->max_iter) { st = OR_ITER_MAX; break; }
        memset(H, 0, sizeof(double) * (size_t)nf * nf);
        for (int e = 0; e < p->ne; ++e) {
            double xe[12];
            gather(p, e, x, xe);
            elem_hess_dm(rd.Dminv + 9 * e, rd.V[e], xe, rd.mu, rd.lam, He);
            if (elem_psd) psd_clamp12(He);
            for (int u = 0; u < 12; ++u) {
                int ru = idx[3 * p->tets[4 * e + u / 3] + u % 3];
                if (ru < 0) continue;
                for (int v = 0; v < 12; ++v) {
                    int rv = idx[3 * p->tets[4 * e + v / 3] + v % 3];
                    if (rv >= 0) H[(size_t)ru * nf + rv] += He[u * 12 + v];
                }
            }
        }
        if (tgt)
            for (int c = 0; c < p->nt; ++c)
                for (int i = 0; i < 3; ++i) {
                    int rr = idx[3 * p->target_vtx[c] + i];
                    if (rr >= 0) H[(size_t)rr * nf + rr] += p->k_c;
                }
        {
            /* inertia and contact: diagonal in q */
            memset(xt, 0, sizeof(double) * n);
            dyn_energy(p, &rd, x, qb, NULL, xt);
            for (int row = 0; row < n; ++row)
                if (idx[row] >= 0) H[(size_t)idx[row] * nf + idx[row]] += xt[row];
        }
        if (newton_dir(nf, H, gf, o->proj, o->eig_floor, dz)) { st = OR_NOT_DESCENT; break; }
        double slope = 0.0;
        for (int k = 0; k < nf; ++k) slope += gf[k] * dz[k];
        if (!(slope < 0.0)) { st = OR_NOT_DESCENT; break; }
        double alpha = 1.0;
        int ok = 0;
        for (int t = 0; t < o->ls_max; ++t) {
            for (int row = 0; row < n; ++row) xt[row] = x[row] + (idx[row] >= 0 ? alpha * dz[idx[row]] : 0.0);
            double Et = full_energy(p, &rd, xt, tgt, f, qb, NULL);
            if (isfinite(Et) && Et - E <= o->c1 * alpha * slope) { ok = 1; break; }
            alpha *= o->shrink;
        }
        if (!ok) { st = OR_LS_MAX; break; }
        memcpy(x, xt, sizeof(double) * n);
        ++it;
    }
    *iters = it;
    *status = st;
    *relgrad = g0 > 0.0 ? gn / g0 : 0.0;
    *Eout = E;
    free(idx); free(grad); free(gf); free(H); free(dz); free(xt);
    rest_free(&rd);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Lipschitz loss of the cubature elastic Hessian                            */
/* ------------------------------------------------------------------------- */
/* ------------------------------------------------------------------------- */
/* Parameter gradient of the summed reduced energy (Sec. 3.2's potential     */
/* loss): one item at a time, serially, accumulated in item order.           */
/* ------------------------------------------------------------------------- */
int or_energy_param_grad(const or_problem* p, int B, const double* z, const double* targets,
                         const double* force, int flags, double* E, double* grad)
{
    const int r = p->r, w = p->width, L = p->L, n = p->n_out;
    const int nin_out = L > 0 ? w : r;
    /* offsets of W_l and b_l in the packed gradient */
    size_t* offW = (size_t*)malloc(sizeof(size_t) * (L + 1));
    size_t* offb = (size_t*)malloc(sizeof(size_t) * (L + 1));
    size_t off = 0;
    for (int l = 0; l <= L; ++l) {
        const int in = l == 0 ? r : w, out = l == L ? n : w;
        offW[l] = off;
        off += (size_t)out * in;
        offb[l] = off;
        off += out;
    }
    memset(grad, 0, sizeof(double) * off);
    rest_data rd;
    rest_build(p, &rd);
    const int cap = w > r ? w : r;
    /* pre-activations a_l and activations h_l of every layer (h_0 = z) */
    double* A = (double*)malloc(sizeof(double) * (size_t)(L > 0 ? L : 1) * w);
    double* Hs = (double*)malloc(sizeof(double) * (size_t)(L + 1) * cap);
    double* x = (double*)malloc(sizeof(double) * n);
    double* gq = (double*)malloc(sizeof(double) * n);
    double* gb = (double*)malloc(sizeof(double) * cap);
    double* gb2 = (double*)malloc(sizeof(double) * cap);
    for (int bi = 0; bi < B; ++bi) {
        const double* zb = z + (size_t)bi * r;
        for (int k = 0; k < r; ++k) Hs[k] = zb[k];
        for (int l = 0; l < L; ++l) {
            const int in = l == 0 ? r : w;
            const double* hin = Hs + (size_t)l * cap;
            for (int i = 0; i < w; ++i) {
                double a = p->b[l][i];
                for (int j = 0; j < in; ++j) a += p->W[l][(size_t)i * in + j] * hin[j];
                A[(size_t)l * w + i] = a;
                Hs[(size_t)(l + 1) * cap + i] = elu(a);
            }
        }
        const double* hL = Hs + (size_t)L * cap;
        for (int row = 0; row < n; ++row) {
            double u = p->b[L][row];
            for (int j = 0; j < nin_out; ++j) u += p->W[L][(size_t)row * nin_out + j] * hL[j];
            x[row] = p->X[row] + (p->pinned[row / 3] ? 0.0 : u);
        }
        const double Eb = q_energy(p, &rd, x, targets ? targets + (size_t)bi * p->nt * 3 : NULL,
                                   force ? force + (size_t)bi * 3 : NULL, NULL, flags & OR_ELASTIC_ONLY, gq);
        if (E) E[bi] = Eb;
        /* output layer: dE/du_row = gq_row on free rows (pinned rows do not move) */
        for (int j = 0; j < nin_out; ++j) gb[j] = 0.0;
        for (int row = 0; row < n; ++row) {
            if (p->pinned[row / 3]) continue;
            const double gr = gq[row];
            for (int j = 0; j < nin_out; ++j) {
                grad[offW[L] + (size_t)row * nin_out + j] += gr * hL[j];
                gb[j] += p->W[L][(size_t)row * nin_out + j] * gr;
            }
            grad[offb[L] + row] += gr;
        }
        /* hidden layers, last to first: delta_l = dE/dh_l * elu'(a_l) */
        for (int l = L - 1; l >= 0; --l) {
            const int in = l == 0 ? r : w;
            const double* hin = Hs + (size_t)l * cap;
            for (int j = 0; j < in; ++j) gb2[j] = 0.0;
            for (int i = 0; i < w; ++i) {
                const double d = gb[i] * elu1(A[(size_t)l * w + i]);
                for (int j = 0; j < in; ++j) {
                    grad[offW[l] + (size_t)i * in + j] += d * hin[j];
                    gb2[j] += p->W[l][(size_t)i * in + j] * d;
                }
                grad[offb[l] + i] += d;
            }
            for (int j = 0; j < in; ++j) gb[j] = gb2[j];
        }
    }
    free(A); free(Hs); free(x); free(gq); free(gb); free(gb2); free(offW); free(offb);
    rest_free(&rd);
    return 0;
}

int or_lipschitz(const or_problem* p, int B, const double* z1, const double* z2,
                 double* loss, double* per_pair, int* n_valid, double* lip_max)
{
    rest_data rd;
    rest_build(p, &rd);
    int r = p->r;
    double* ell = (double*)malloc(sizeof(double) * (B > 0 ? B : 1));
    int* valid = (int*)malloc(sizeof(int) * (B > 0 ? B : 1));
#pragma omp parallel for schedule(dynamic)
    for (int bi = 0; bi < B; ++bi) {
        const double* a = z1 + (size_t)bi * r;
        const double* c = z2 + (size_t)bi * r;
        double dz2 = 0.0;
        for (int k = 0; k < r; ++k) dz2 += (a[k] - c[k]) * (a[k] - c[k]);
        valid[bi] = dz2 > 0.0;
        ell[bi] = 0.0;
        if (!valid[bi]) continue;
        double E1, E2;
        double* H1 = (double*)malloc(sizeof(double) * r * r);
        double* H2 = (double*)malloc(sizeof(double) * r * r);
        item_eval(p, &rd, a, NULL, NULL, NULL, OR_EXACT | OR_ELASTIC_ONLY, &E1, NULL, H1);
        item_eval(p, &rd, c, NULL, NULL, NULL, OR_EXACT | OR_ELASTIC_ONLY, &E2, NULL, H2);
        double fro = 0.0;
        for (int k = 0; k < r * r; ++k) fro += (H1[k] - H2[k]) * (H1[k] - H2[k]);
        ell[bi] = fro / dz2;
        free(H1); free(H2);
    }
    double sum = 0.0, mx = 0.0;
    int nv = 0;
    for (int bi = 0; bi < B; ++bi) {
        if (per_pair) per_pair[bi] = ell[bi];
        if (!valid[bi]) continue;
        ++nv;
        sum += ell[bi];
        mx = fmax(mx, sqrt(ell[bi]));
    }
    *loss = nv ? sum / nv : 0.0;
    *n_valid = nv;
    if (lip_max) *lip_max = mx;
    free(ell); free(valid);
    rest_free(&rd);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Decoder-parameter gradient of the Lipschitz loss (Sec. 4.1, Eq.            */
/* form-L-LS-E; Sec. 4.2: elastic term only, cubature Hessian of Sec. 4.3).   */
/*                                                                           */
/* With D_b = H(z1_b) - H(z2_b), H the exact cubature elastic Hessian, and    */
/* l_b = |D_b|_F^2 / |z1_b - z2_b|^2, the loss mean_b l_b has the gradient    */
/*   sum_b <C_b, dH(z1_b)/dtheta> - <C_b, dH(z2_b)/dtheta>,                   */
/*   C_b = 2 D_b / (|z1_b - z2_b|^2 n_valid).                                 */
/* <C, H(z)> = sum_kq C_kq d2 P~(q(z)) / dz_k dz_q is differentiated by the   */
/* chain rule written out: forward, the value h_l, Jacobian J_l and the       */
/* C-contracted second derivative S_l = sum_kq C_kq d2 h_l / dz_k dz_q of     */
/* every layer (and of the output rows); per cubature element the contracted  */
/* Hessian tr(C K^T A(F) K) + P(F) : Fdd, K = dvecF/dz, Fdd = C-contracted    */
/* second derivative of F; backward, the adjoints of (h, J, S) down to the    */
/* first layer.  The derivative of A = d2 psi / dF2 with respect to F is      */
/* taken entry by entry from the third derivatives of det F (products of two  */
/* permutation symbols).                                                      */
/* ------------------------------------------------------------------------- */
static double elu3(double a) { return a > 0.0 ? 0.0 : exp(a); }

/* d2 det / dF_p dF_q and d3 det / dF_p dF_q dF_m at vec indices p = 3 j + i */
static double d2det(const double* F, int p, int q)
{
    int i = p % 3, j = p / 3, k = q % 3, l = q / 3;
    if (j == l) return 0.0;
    int c = 3 - j - l;
    double h = 0.0;
    for (int m = 0; m < 3; ++m) h += levi(j, l, c) * levi(i, k, m) * F[3 * m + c];
    return h;
}

static double d3det(int p, int q, int m)
{
    return (double)(levi(p % 3, q % 3, m % 3) * levi(p / 3, q / 3, m / 3));
}

static void param_offsets(const or_problem* p, size_t* offW, size_t* offb, size_t* total)
{
    size_t off = 0;
    for (int l = 0; l <= p->L; ++l) {
        int in = l == 0 ? p->r : p->width, out = l == p->L ? p->n_out : p->width;
        offW[l] = off;
        off += (size_t)out * in;
        offb[l] = off;
        off += out;
    }
    *total = off;
}

static void hess_contract_grad(const or_problem* p, const rest_data* rd, const double* z, const double* C,
                               double sign, const size_t* offW, const size_t* offb, double* grad)
{
    const int r = p->r, w = p->width, L = p->L, n = p->n_out;
    const int cap = w > r ? w : r;
    /* layer inputs (h, J, S) of every layer and of the output layer, and pre-activations */
    double* Hin = (double*)calloc((size_t)(L + 1) * cap, sizeof(double));
    double* Jin = (double*)calloc((size_t)(L + 1) * cap * r, sizeof(double));
    double* Sin = (double*)calloc((size_t)(L + 1) * cap, sizeof(double));
    double* Pa = (double*)calloc((size_t)(L > 0 ? L : 1) * w, sizeof(double));
    double* PA = (double*)calloc((size_t)(L > 0 ? L : 1) * w * r, sizeof(double));
    double* PS = (double*)calloc((size_t)(L > 0 ? L : 1) * w, sizeof(double));
    for (int k = 0; k < r; ++k) { Hin[k] = z[k]; Jin[k * r + k] = 1.0; }
    for (int l = 0; l < L; ++l) {
        const int in = l == 0 ? r : w;
        const double* h0 = Hin + (size_t)l * cap;
        const double* J0 = Jin + (size_t)l * cap * r;
        const double* S0 = Sin + (size_t)l * cap;
        double* h1 = Hin + (size_t)(l + 1) * cap;
        double* J1 = Jin + (size_t)(l + 1) * cap * r;
        double* S1 = Sin + (size_t)(l + 1) * cap;
        for (int u = 0; u < w; ++u) {
            const double* Wu = p->W[l] + (size_t)u * in;
            double a = p->b[l][u], aS = 0.0;
            double* Au = PA + ((size_t)l * w + u) * r;
            for (int j = 0; j < in; ++j) {
                a += Wu[j] * h0[j];
                aS += Wu[j] * S0[j];
                for (int k = 0; k < r; ++k) Au[k] += Wu[j] * J0[j * r + k];
            }
            double qf = 0.0;
            for (int k = 0; k < r; ++k)
                for (int k2 = 0; k2 < r; ++k2) qf += Au[k] * C[k * r + k2] * Au[k2];
            Pa[(size_t)l * w + u] = a;
            PS[(size_t)l * w + u] = aS;
            h1[u] = elu(a);
            for (int k = 0; k < r; ++k) J1[u * r + k] = elu1(a) * Au[k];
            S1[u] = elu2(a) * qf + elu1(a) * aS;
        }
    }
    const int nin = L > 0 ? w : r;
    const double* hL = Hin + (size_t)L * cap;
    const double* JL = Jin + (size_t)L * cap * r;
    const double* SL = Sin + (size_t)L * cap;
    /* output rows: u = m (W h + b), dU = m W J, uS = m W S */
    double* x = (double*)malloc(sizeof(double) * n);
    double* UJ = (double*)calloc((size_t)n * r, sizeof(double));
    double* uS = (double*)calloc(n, sizeof(double));
    const double* Wo = p->W[L];
    for (int row = 0; row < n; ++row) {
        double u = 0.0;
        if (!p->pinned[row / 3]) {
            u = p->b[L][row];
            for (int j = 0; j < nin; ++j) {
                const double wj = Wo[(size_t)row * nin + j];
                u += wj * hL[j];
                uS[row] += wj * SL[j];
                for (int k = 0; k < r; ++k) UJ[(size_t)row * r + k] += wj * JL[j * r + k];
            }
        }
        x[row] = p->X[row] + u;
    }
    /* elements: adjoints of the rows */
    double* ub = (double*)calloc(n, sizeof(double));
    double* UJb = (double*)calloc((size_t)n * r, sizeof(double));
    double* uSb = (double*)calloc(n, sizeof(double));
    double* K = (double*)malloc(sizeof(double) * 9 * r);
    double* KC = (double*)malloc(sizeof(double) * 9 * r);
    for (int s = 0; s < p->S; ++s) {
        const int e = p->cub_elem[s];
        const int* t = p->tets + 4 * e;
        const double* Dminv = rd->Dminv + 9 * e;
        double xe[12], F[9], Dv[12], A[81], P[9], cof[9];
        gather(p, e, x, xe);
        deform_grad(Dminv, xe, F);
        shape_grad(Dminv, Dv);
        or_dpdf(F, rd->mu, rd->lam, A);
        or_pk1(F, rd->mu, rd->lam, P);
        cofactor(F, cof);
        const double wV = p->cub_w[s] * rd->V[e];
        const double sfac = rd->lam * (det3(F) - 1.0) - rd->mu;
        /* K[v][k] and Fdd[v] at vec index v = 3 j + i: sum_a Dv[a][j] (row 3 t_a + i) */
        double Fdd[9], g[9], Pv[9];
        for (int j = 0; j < 3; ++j)
            for (int i = 0; i < 3; ++i) {
                const int v = 3 * j + i;
                g[v] = cof[3 * i + j];
                Pv[v] = P[3 * i + j];
                Fdd[v] = 0.0;
                for (int k = 0; k < r; ++k) K[v * r + k] = 0.0;
                for (int a = 0; a < 4; ++a) {
                    const int row = 3 * t[a] + i;
                    Fdd[v] += Dv[3 * a + j] * uS[row];
                    for (int k = 0; k < r; ++k) K[v * r + k] += Dv[3 * a + j] * UJ[(size_t)row * r + k];
                }
            }
        /* N = K C K^T, KC = K C */
        double N[81];
        for (int v = 0; v < 9; ++v)
            for (int k = 0; k < r; ++k) {
                double acc = 0.0;
                for (int k2 = 0; k2 < r; ++k2) acc += K[v * r + k2] * C[k2 * r + k];
                KC[v * r + k] = acc;
            }
        for (int v = 0; v < 9; ++v)
            for (int v2 = 0; v2 < 9; ++v2) {
                double acc = 0.0;
                for (int k = 0; k < r; ++k) acc += KC[v * r + k] * K[v2 * r + k];
                N[v * 9 + v2] = acc;
            }
        /* Fbar = wV (sum_pq N_pq dA_pq/dF + A Fdd), Kbar = 2 wV A K C, Fddbar = wV P */
        double Fb[9], Fddb[9], Kb[9 * 32];
        double HJ[81];
        for (int a = 0; a < 9; ++a)
            for (int b = 0; b < 9; ++b) HJ[a * 9 + b] = d2det(F, a, b);
        for (int m = 0; m < 9; ++m) {
            double acc = 0.0;
            for (int pp = 0; pp < 9; ++pp)
                for (int qq = 0; qq < 9; ++qq) {
                    const double dA = rd->lam * (HJ[pp * 9 + m] * g[qq] + g[pp] * HJ[qq * 9 + m]) +
                                      rd->lam * g[m] * HJ[pp * 9 + qq] + sfac * d3det(pp, qq, m);
                    acc += N[pp * 9 + qq] * dA;
                }
            double af = 0.0;
            for (int q = 0; q < 9; ++q) af += A[m * 9 + q] * Fdd[q];
            Fb[m] = wV * (acc + af);
            Fddb[m] = wV * Pv[m];
            for (int k = 0; k < r; ++k) {
                double ak = 0.0;
                for (int q = 0; q < 9; ++q) ak += A[m * 9 + q] * KC[q * r + k];
                Kb[m * r + k] = 2.0 * wV * ak;
            }
        }
        for (int a = 0; a < 4; ++a)
            for (int i = 0; i < 3; ++i) {
                const int row = 3 * t[a] + i;
                for (int j = 0; j < 3; ++j) {
                    const int v = 3 * j + i;
                    const double d = Dv[3 * a + j];
                    ub[row] += d * Fb[v];
                    uSb[row] += d * Fddb[v];
                    for (int k = 0; k < r; ++k) UJb[(size_t)row * r + k] += d * Kb[v * r + k];
                }
            }
    }
    /* output layer (free rows only) */
    double* hb = (double*)calloc(cap, sizeof(double));
    double* Jb = (double*)calloc((size_t)cap * r, sizeof(double));
    double* Sb = (double*)calloc(cap, sizeof(double));
    for (int row = 0; row < n; ++row) {
        if (p->pinned[row / 3]) continue;
        const double* Wr = Wo + (size_t)row * nin;
        for (int j = 0; j < nin; ++j) {
            double gw = ub[row] * hL[j] + uSb[row] * SL[j];
            for (int k = 0; k < r; ++k) gw += UJb[(size_t)row * r + k] * JL[j * r + k];
            grad[offW[L] + (size_t)row * nin + j] += sign * gw;
            hb[j] += Wr[j] * ub[row];
            Sb[j] += Wr[j] * uSb[row];
            for (int k = 0; k < r; ++k) Jb[j * r + k] += Wr[j] * UJb[(size_t)row * r + k];
        }
        grad[offb[L] + row] += sign * ub[row];
    }
    /* hidden layers, last to first */
    double* hb2 = (double*)calloc(cap, sizeof(double));
    double* Jb2 = (double*)calloc((size_t)cap * r, sizeof(double));
    double* Sb2 = (double*)calloc(cap, sizeof(double));
    double* Ab = (double*)malloc(sizeof(double) * r);
    double* AC = (double*)malloc(sizeof(double) * r);
    for (int l = L - 1; l >= 0; --l) {
        const int in = l == 0 ? r : w;
        const double* h0 = Hin + (size_t)l * cap;
        const double* J0 = Jin + (size_t)l * cap * r;
        const double* S0 = Sin + (size_t)l * cap;
        memset(hb2, 0, sizeof(double) * cap);
        memset(Jb2, 0, sizeof(double) * (size_t)cap * r);
        memset(Sb2, 0, sizeof(double) * cap);
        for (int u = 0; u < w; ++u) {
            const double a = Pa[(size_t)l * w + u], aS = PS[(size_t)l * w + u];
            const double* Au = PA + ((size_t)l * w + u) * r;
            const double s1 = elu1(a), s2 = elu2(a), s3 = elu3(a);
            double qf = 0.0, AJ = 0.0;
            for (int k = 0; k < r; ++k) {
                double acc = 0.0;
                for (int k2 = 0; k2 < r; ++k2) acc += Au[k2] * C[k2 * r + k];
                AC[k] = acc;
                qf += acc * Au[k];
                AJ += Au[k] * Jb[u * r + k];
            }
            const double abar = s1 * hb[u] + s2 * AJ + s3 * qf * Sb[u] + s2 * aS * Sb[u];
            for (int k = 0; k < r; ++k) Ab[k] = s1 * Jb[u * r + k] + 2.0 * s2 * Sb[u] * AC[k];
            const double aSbar = s1 * Sb[u];
            const double* Wu = p->W[l] + (size_t)u * in;
            for (int j = 0; j < in; ++j) {
                double gw = abar * h0[j] + aSbar * S0[j];
                for (int k = 0; k < r; ++k) gw += Ab[k] * J0[j * r + k];
                grad[offW[l] + (size_t)u * in + j] += sign * gw;
                hb2[j] += Wu[j] * abar;
                Sb2[j] += Wu[j] * aSbar;
                for (int k = 0; k < r; ++k) Jb2[j * r + k] += Wu[j] * Ab[k];
            }
            grad[offb[l] + u] += sign * abar;
        }
        memcpy(hb, hb2, sizeof(double) * cap);
        memcpy(Jb, Jb2, sizeof(double) * (size_t)cap * r);
        memcpy(Sb, Sb2, sizeof(double) * cap);
    }
    free(Hin); free(Jin); free(Sin); free(Pa); free(PA); free(PS);
    free(x); free(UJ); free(uS); free(ub); free(UJb); free(uSb); free(K); free(KC);
    free(hb); free(Jb); free(Sb); free(hb2); free(Jb2); free(Sb2); free(Ab); free(AC);
}

int or_lipschitz_param_grad(const or_problem* p, int B, const double* z1, const double* z2,
                            double* loss, double* grad)
{
    const int r = p->r;
    if (r > 32) return 1;
    size_t offW[16], offb[16], total;
    if (p->L + 1 > 16) return 1;
    param_offsets(p, offW, offb, &total);
    memset(grad, 0, sizeof(double) * total);
    rest_data rd;
    rest_build(p, &rd);
    int nv = 0;
    for (int b = 0; b < B; ++b) {
        double d2 = 0.0;
        for (int k = 0; k < r; ++k) d2 += (z1[b * r + k] - z2[b * r + k]) * (z1[b * r + k] - z2[b * r + k]);
        nv += d2 > 0.0;
    }
    double sum = 0.0;
    double* H1 = (double*)malloc(sizeof(double) * r * r);
    double* H2 = (double*)malloc(sizeof(double) * r * r);
    double* Cm = (double*)malloc(sizeof(double) * r * r);
    for (int b = 0; b < B; ++b) {
        const double* a = z1 + (size_t)b * r;
        const double* c = z2 + (size_t)b * r;
        double d2 = 0.0;
        for (int k = 0; k < r; ++k) d2 += (a[k] - c[k]) * (a[k] - c[k]);
        if (!(d2 > 0.0)) continue;
        double E1, E2;
        item_eval(p, &rd, a, NULL, NULL, NULL, OR_EXACT | OR_ELASTIC_ONLY, &E1, NULL, H1);
        item_eval(p, &rd, c, NULL, NULL, NULL, OR_EXACT | OR_ELASTIC_ONLY, &E2, NULL, H2);
        double fro = 0.0;
        for (int k = 0; k < r * r; ++k) fro += (H1[k] - H2[k]) * (H1[k] - H2[k]);
        sum += fro / d2;
        /* C = 2 sym(D) / (|dz|^2 n_valid) */
        for (int k = 0; k < r; ++k)
            for (int q = 0; q < r; ++q)
                Cm[k * r + q] = ((H1[k * r + q] - H2[k * r + q]) + (H1[q * r + k] - H2[q * r + k])) / (d2 * nv);
        hess_contract_grad(p, &rd, a, Cm, 1.0, offW, offb, grad);
        hess_contract_grad(p, &rd, c, Cm, -1.0, offW, offb, grad);
    }
    *loss = nv ? sum / nv : 0.0;
    free(H1); free(H2); free(Cm);
    rest_free(&rd);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Supervised construction (Sec. 3.2, Eq. form-vanilla-supervised-construction): */
/* L_C = mean_i |f(g(q_i)) - q_i|_M^2 with the positions f = X + m (.) decoder  */
/* and the encoder g fed the displacement q_i - X; gradients of both networks  */
/* by the chain rule (value passes only).                                     */
/* ------------------------------------------------------------------------- */
static void mlp_offsets(int n_in, int L, int width, int n_out, size_t* offW, size_t* offb, size_t* total)
{
    size_t off = 0;
    for (int l = 0; l <= L; ++l) {
        int in = l == 0 ? n_in : width, out = l == L ? n_out : width;
        offW[l] = off;
        off += (size_t)out * in;
        offb[l] = off;
        off += out;
    }
    *total = off;
}

/* forward of an ELU MLP keeping every layer's pre-activation (A) and input (Hs) */
static void mlp_forward(int n_in, int L, int width, int n_out, const double* const* W, const double* const* b,
                        const double* x, double* A, double* Hs, int cap, double* y)
{
    for (int j = 0; j < n_in; ++j) Hs[j] = x[j];
    for (int l = 0; l <= L; ++l) {
        const int in = l == 0 ? n_in : width, out = l == L ? n_out : width;
        const double* h = Hs + (size_t)l * cap;
        for (int u = 0; u < out; ++u) {
            double a = b[l][u];
            for (int j = 0; j < in; ++j) a += W[l][(size_t)u * in + j] * h[j];
            if (l < L) {
                A[(size_t)l * width + u] = a;
                Hs[(size_t)(l + 1) * cap + u] = elu(a);
            } else {
                y[u] = a;
            }
        }
    }
}

/* backward of the same MLP given dL/dy; accumulates parameter gradients and
 * returns dL/dx in xb (nullable) */
static void mlp_backward(int n_in, int L, int width, int n_out, const double* const* W, const double* A,
                         const double* Hs, int cap, const double* yb, const size_t* offW, const size_t* offb,
                         double* grad, double* xb)
{
    double* gb = (double*)calloc(cap, sizeof(double));
    double* gb2 = (double*)calloc(cap, sizeof(double));
    for (int l = L; l >= 0; --l) {
        const int in = l == 0 ? n_in : width, out = l == L ? n_out : width;
        const double* h = Hs + (size_t)l * cap;
        memset(gb2, 0, sizeof(double) * cap);
        for (int u = 0; u < out; ++u) {
            const double d = l == L ? yb[u] : gb[u] * elu1(A[(size_t)l * width + u]);
            if (d == 0.0) continue;
            for (int j = 0; j < in; ++j) {
                grad[offW[l] + (size_t)u * in + j] += d * h[j];
                gb2[j] += W[l][(size_t)u * in + j] * d;
            }
            grad[offb[l] + u] += d;
        }
        memcpy(gb, gb2, sizeof(double) * cap);
    }
    if (xb) memcpy(xb, gb, sizeof(double) * n_in);
    free(gb); free(gb2);
}

int or_recon_loss_grad(const or_problem* p, const or_mlp* enc, int B, const double* q, double* loss,
                       double* grad_enc, double* grad_dec)
{
    const int n = p->n_out, r = p->r, L = p->L, w = p->width;
    if (enc->n_in != n || enc->n_out != r) return 1;
    size_t eW[16], eb[16], etot, dW[16], db[16], dtot;
    if (enc->L + 1 > 16 || L + 1 > 16) return 1;
    mlp_offsets(n, enc->L, enc->width, r, eW, eb, &etot);
    param_offsets(p, dW, db, &dtot);
    memset(grad_enc, 0, sizeof(double) * etot);
    memset(grad_dec, 0, sizeof(double) * dtot);
    rest_data rd;
    rest_build(p, &rd);
    const int ecap = n > enc->width ? n : (enc->width > r ? enc->width : r);
    const int dcap = (w > r ? w : r);
    double* eA = (double*)malloc(sizeof(double) * (size_t)(enc->L > 0 ? enc->L : 1) * (enc->width > 0 ? enc->width : 1));
    double* eH = (double*)malloc(sizeof(double) * (size_t)(enc->L + 1) * ecap);
    double* dA = (double*)malloc(sizeof(double) * (size_t)(L > 0 ? L : 1) * (w > 0 ? w : 1));
    double* dH = (double*)malloc(sizeof(double) * (size_t)(L + 1) * dcap);
    double* d = (double*)malloc(sizeof(double) * n);
    double* z = (double*)malloc(sizeof(double) * r);
    double* zb = (double*)malloc(sizeof(double) * r);
    double* u = (double*)malloc(sizeof(double) * n);
    double* ub = (double*)malloc(sizeof(double) * n);
    double sum = 0.0;
    for (int i = 0; i < B; ++i) {
        const double* qi = q + (size_t)i * n;
        for (int row = 0; row < n; ++row) d[row] = qi[row] - p->X[row];
        mlp_forward(n, enc->L, enc->width, r, enc->W, enc->b, d, eA, eH, ecap, z);
        mlp_forward(r, L, w, n, p->W, p->b, z, dA, dH, dcap, u);
        /* residual on positions: X + m (.) u - q = m (.) u - d */
        for (int row = 0; row < n; ++row) {
            const int fixed = p->pinned[row / 3];
            const double res = (fixed ? 0.0 : u[row]) - d[row];
            const double mv = rd.mass[row / 3];
            sum += mv * res * res;
            ub[row] = fixed ? 0.0 : 2.0 * mv * res / B;
        }
        mlp_backward(r, L, w, n, p->W, dA, dH, dcap, ub, dW, db, grad_dec, zb);
        mlp_backward(n, enc->L, enc->width, r, enc->W, eA, eH, ecap, zb, eW, eb, grad_enc, NULL);
    }
    *loss = B ? sum / B : 0.0;
    free(eA); free(eH); free(dA); free(dH); free(d); free(z); free(zb); free(u); free(ub);
    rest_free(&rd);
    return 0;
}

int or_encode(const or_mlp* enc, int B, const double* d, double* z)
{
    const int cap = enc->n_in > enc->width ? enc->n_in : (enc->width > enc->n_out ? enc->width : enc->n_out);
    double* A = (double*)malloc(sizeof(double) * (size_t)(enc->L > 0 ? enc->L : 1) * (enc->width > 0 ? enc->width : 1));
    double* Hs = (double*)malloc(sizeof(double) * (size_t)(enc->L + 1) * cap);
    for (int i = 0; i < B; ++i)
        mlp_forward(enc->n_in, enc->L, enc->width, enc->n_out, enc->W, enc->b, d + (size_t)i * enc->n_in, A, Hs, cap,
                    z + (size_t)i * enc->n_out);
    free(A); free(Hs);
    return 0;
}

/* number of OpenMP threads of the oracle's parallel loops (for timing) */
void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

