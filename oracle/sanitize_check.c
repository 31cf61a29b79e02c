/*
 * Memory-safety driver for the FP64 oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Built by the test suite together with oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer (gcc, host code only) and run once: it calls
 * every exported oracle routine on a small beam (2x1x1 cubes, 10 tets) with a
 * small decoder, and on a linear decoder whose latent size exceeds 32, so that
 * an out-of-bounds access, a leak or undefined arithmetic anywhere in the
 * oracle ends the run with a non-zero status.  The numbers themselves are not
 * checked here (the other oracle tests do that).
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* deterministic values in [-1, 1) (64-bit linear congruential sequence) */
static unsigned long long lcg_state = 12345u;
static double uniform_pm1(void)
{
    lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg_state >> 11) / 9007199254740992.0 * 2.0 - 1.0;
}

enum { NX = 2, NY = 1, NZ = 1 };

static int vid(int i, int j, int k) { return (i * (NY + 1) + j) * (NZ + 1) + k; }

/* 5-tet cube grid with positively oriented tets */
static void build_mesh(double h, double* X, int* tets)
{
    for (int i = 0; i <= NX; ++i)
        for (int j = 0; j <= NY; ++j)
            for (int k = 0; k <= NZ; ++k) {
                int v = vid(i, j, k);
                X[3 * v] = i * h; X[3 * v + 1] = j * h; X[3 * v + 2] = k * h;
            }
    static const int ev[4][3] = {{0, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}};
    static const int od[4][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 1}};
    int t = 0;
    for (int i = 0; i < NX; ++i)
        for (int j = 0; j < NY; ++j)
            for (int k = 0; k < NZ; ++k) {
                const int (*centre)[3] = ((i + j + k) % 2 == 0) ? od : ev;
                const int (*corner)[3] = ((i + j + k) % 2 == 0) ? ev : od;
                int cl[5][4][3];
                for (int a = 0; a < 4; ++a) memcpy(cl[0][a], centre[a], sizeof(cl[0][a]));
                for (int c = 0; c < 4; ++c) {
                    memcpy(cl[c + 1][0], corner[c], sizeof(cl[0][0]));
                    for (int s = 0; s < 3; ++s) {
                        for (int d = 0; d < 3; ++d) cl[c + 1][s + 1][d] = corner[c][d] ^ (d == s);
                    }
                }
                for (int q = 0; q < 5; ++q) {
                    int ids[4];
                    for (int a = 0; a < 4; ++a) ids[a] = vid(i + cl[q][a][0], j + cl[q][a][1], k + cl[q][a][2]);
                    double e[3][3];
                    for (int a = 0; a < 3; ++a)
                        for (int d = 0; d < 3; ++d) e[a][d] = X[3 * ids[a + 1] + d] - X[3 * ids[0] + d];
                    double det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                                 e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                                 e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
                    if (det < 0) { int s = ids[1]; ids[1] = ids[2]; ids[2] = s; }
                    memcpy(&tets[4 * t], ids, sizeof(ids));
                    ++t;
                }
            }
}

int main(void)
{
    const int nv = (NX + 1) * (NY + 1) * (NZ + 1), ne = 5 * NX * NY * NZ, n = 3 * nv;
    double X[3 * (NX + 1) * (NY + 1) * (NZ + 1)];
    int tets[4 * 5 * NX * NY * NZ];
    unsigned char pinned[(NX + 1) * (NY + 1) * (NZ + 1)];
    build_mesh(0.5, X, tets);
    int tv[4], nt = 0;
    for (int v = 0; v < nv; ++v) {
        pinned[v] = X[3 * v] == 0.0;
        if (X[3 * v] == NX * 0.5) tv[nt++] = v;
    }
    /* decoder r = 4 -> 8 -> 8 -> n */
    const int r = 4, w = 8, L = 2;
    double* W[3];
    double* b[3];
    const int din[3] = {r, w, w}, dout[3] = {w, w, n};
    for (int l = 0; l <= L; ++l) {
        W[l] = (double*)malloc(sizeof(double) * din[l] * dout[l]);
        b[l] = (double*)malloc(sizeof(double) * dout[l]);
        for (int i = 0; i < din[l] * dout[l]; ++i) W[l][i] = 0.5 * uniform_pm1();
        for (int i = 0; i < dout[l]; ++i) b[l][i] = 0.2 * uniform_pm1();
    }
    int cub[8];
    double cw[8];
    for (int s = 0; s < 8; ++s) { cub[s] = s; cw[s] = 20.0 + 60.0 * (0.5 + 0.5 * uniform_pm1()); }
    or_problem p;
    memset(&p, 0, sizeof(p));
    p.nv = nv; p.ne = ne; p.X = X; p.tets = tets; p.pinned = pinned;
    p.young = 1e5; p.poisson = 0.45; p.density = 1000.0;
    p.gravity[1] = -9.81;
    p.r = r; p.L = L; p.width = w; p.n_out = n;
    p.W = (const double* const*)W; p.b = (const double* const*)b;
    p.S = 8; p.cub_elem = cub; p.cub_w = cw;
    p.nt = nt; p.target_vtx = tv; p.k_c = 1e6;
    p.nf = nt; p.force_vtx = tv;

    const int B = 3;
    double z[3 * 4], z2[3 * 4], tg[3 * 4 * 3], fo[3 * 3];
    for (int i = 0; i < B * r; ++i) { z[i] = 0.5 * uniform_pm1(); z2[i] = 0.5 * uniform_pm1(); }
    for (int bi = 0; bi < B; ++bi) {
        for (int c = 0; c < nt; ++c)
            for (int d = 0; d < 3; ++d) tg[(bi * nt + c) * 3 + d] = X[3 * tv[c] + d] + 0.05 * uniform_pm1();
        for (int d = 0; d < 3; ++d) fo[3 * bi + d] = 10.0 * uniform_pm1();
    }
    double E[3], g[3 * 4], H[3 * 16], x[3 * 36], J[3 * 36 * 4], T[36 * 16], m[12];
    or_lumped_mass(&p, m);
    or_decode(&p, B, z, x, J);
    or_decode_hess(&p, z, T);
    const int flag_sets[5] = {0, OR_EXACT, OR_EXACT | OR_ELASTIC_ONLY, OR_ENERGY_ONLY, OR_ELEM_PSD};
    for (int f = 0; f < 5; ++f) or_reduced(&p, B, z, tg, fo, NULL, flag_sets[f], E, g, H);
    double dz[4];
    for (int proj = 0; proj < 3; ++proj) or_newton_dir(r, H, g, proj, 1e-8, dz);
    or_opts o = {20, 64, 1e-4, 0.5, 1e-6, 0.0, 1, 1, 1e-8};
    int it[3], st[3];
    double rg[3];
    double zz[3 * 4];
    memcpy(zz, z, sizeof(zz));
    or_newton(&p, B, zz, tg, fo, NULL, &o, it, st, rg, E);
    or_lbfgs_opts lo = {40, 64, 5, 1e-4, 0.5, 1e-6, 0.0};
    memcpy(zz, z, sizeof(zz));
    or_lbfgs(&p, B, zz, tg, fo, NULL, &lo, it, st, rg, E);
    double loss, lmax, per[3];
    int nval;
    or_lipschitz(&p, B, z, z2, &loss, per, &nval, &lmax);
    long np = 0;
    for (int l = 0; l <= L; ++l) np += (long)din[l] * dout[l] + dout[l];
    double* grad = (double*)malloc(sizeof(double) * np);
    or_energy_param_grad(&p, B, z, tg, fo, 0, E, grad);
    double xf[36], gradf[36];
    memcpy(xf, x, sizeof(xf));
    or_full_energy(&p, xf, tg, fo, NULL, gradf);
    or_opts fo_opts = {20, 64, 1e-4, 0.5, 1e-8, 0.0, 1, 1, 1e-8};
    int fit, fst;
    double frg, fE;
    or_full_newton(&p, xf, tg, fo, NULL, &fo_opts, 1, &fit, &fst, &frg, &fE);

    /* a linear decoder selecting every free DOF: r = 24 ... and a wider one, r = 40 */
    for (int pass = 0; pass < 2; ++pass) {
        int rl = 0;
        int* free_rows = (int*)malloc(sizeof(int) * n);
        for (int row = 0; row < n; ++row)
            if (!pinned[row / 3]) free_rows[rl++] = row;
        if (pass == 1) rl = 40; /* extra latent columns map onto repeated rows */
        double* Wl = (double*)calloc((size_t)n * rl, sizeof(double));
        double* bl = (double*)calloc(n, sizeof(double));
        int nfree = 0;
        for (int row = 0; row < n; ++row) nfree += !pinned[row / 3];
        for (int k = 0; k < rl; ++k) Wl[(size_t)free_rows[k % nfree] * rl + k] = pass ? 0.5 : 1.0;
        or_problem q = p;
        q.r = rl; q.L = 0; q.width = 0;
        double* Wq[1] = {Wl};
        double* bq[1] = {bl};
        q.W = (const double* const*)Wq; q.b = (const double* const*)bq;
        double* zl = (double*)calloc(rl, sizeof(double));
        for (int k = 0; k < rl; ++k) zl[k] = 0.01 * uniform_pm1();
        double El, *gl = (double*)malloc(sizeof(double) * rl), *Hl = (double*)malloc(sizeof(double) * rl * rl);
        or_reduced(&q, 1, zl, tg, fo, NULL, OR_EXACT, &El, gl, Hl);
        int itl, stl;
        double rgl;
        or_lbfgs(&q, 1, zl, tg, fo, NULL, &lo, &itl, &stl, &rgl, &El);
        or_newton(&q, 1, zl, tg, fo, NULL, &o, &itl, &stl, &rgl, &El);
        free(free_rows); free(Wl); free(bl); free(zl); free(gl); free(Hl);
    }
    free(grad);
    for (int l = 0; l <= L; ++l) { free(W[l]); free(b[l]); }
    printf("sanitize_check ok: %d tets, loss %.6e\n", ne, loss);
    return 0;
}
