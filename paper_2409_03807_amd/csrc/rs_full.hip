// Full-space quasi-static solver (Sec. 3.1, Eq. form-full-space-time-integration
// with the inertia term dropped): projective Newton on every element of the
// mesh, batched over independent load cases.  It generates the snapshots of
// the supervised subspace construction (Sec. 3.2) and is the judge of the
// reduced solves.
//
// Per Newton iteration:
//  * element pass: F, psi, PK1 and the element Hessian H_e = V D^T A D with its
//    negative eigenvalues set to zero (the per-element projection of projective
//    Newton, supplement).  With N the Gram matrix of the shape gradients and
//    B = N^(1/2) (x) I_3 one has proj(H_e) = D^T B^-1 proj(M) B^-1 D for
//    M = V B A B (9 x 9), so each element keeps Aeff = B^-1 proj(M) B^-1
//    (45 values); M is projected only when its Cholesky factorisation fails;
//  * vertex pass: gradient g and the Jacobi preconditioner from the incident
//    elements (a fixed-order gather, no atomics), penalty, gravity and forces;
//  * preconditioned conjugate gradients on H dx = -g with matrix-free products
//    (element pass D^T Aeff D p, vertex gather), stopped per item at
//    |r|_2 <= eta |g|_2, eta = clamp(sqrt(|g|_inf / |g_0|_inf), eta_min, eta_max);
//  * Armijo backtracking on the full energy, float64 throughout.
//
// Layout: every per-item vector is dof-major with the item index fastest,
// v[(3 vertex + i) * Bp + b], Bp the batch padded to 64; a wave handles one
// element or vertex for 64 items, so every access to item data is coalesced
// and the element constants are wave-uniform.  Per-item sums are taken per
// workgroup and then over workgroups in a fixed order.
#include "rs_device.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace rs {

namespace {

constexpr int kEc = 32;      // per-element constants: Dv (12), V, Nh (9), Nhi (9), pad
constexpr int kEpw = 8;      // elements per wave in the element passes
constexpr int kVpw = 8;      // vertices (or dofs / 3) per wave in the vertex passes
constexpr int kPsdT = 64;    // threads of the projection kernel

enum { FS_RUNNING = -1, FS_CONVERGED = 0, FS_NOT_DESCENT = 1, FS_LS_MAX = 2, FS_ITER_MAX = 3, FS_NONFINITE = 4 };

struct FsArgs {
    int ne, nv, n, Bp, B;
    const int* tets;
    const double* ec;        // ne x kEc
    const int* vptr;         // nv + 1: incident (element, corner) entries per vertex
    const int* vinc;         // 4 e + corner
    const double* mass;      // nv
    const uint8_t* pinned;   // nv
    const int* tslot;        // nv: index into the targets, -1 if none
    const uint8_t* fvert;    // nv: 1 if force-loaded
    const double* X;         // 3 nv rest positions
    const double* targets;   // B x nt x 3 (item-major) or NULL
    const double* force;     // B x 3 or NULL
    int nt;
    double mu, lam, kc, grav[3];
    // state (dof-major, n x Bp)
    double* U;
    double* dx;
    double* g;
    double* dg;   // Jacobi diagonal
    double* r;
    double* z;
    double* p;
    double* q;
    // element buffers (ne x {9, 45} x Bp)
    double* Se;
    double* Ae;
    int* list;
    int* nlist;
    // partial sums (blocks x Bp)
    double* pe;   // element energies per element workgroup
    double* pv;   // vertex sums per vertex workgroup (several quantities)
    int neb, nvb; // element and vertex workgroups
    // per item (Bp)
    double* E;
    double* Et;
    double* g0;
    double* ginf;
    double* gn2;
    double* rz;
    double* tol2;
    double* acg;  // CG step length
    double* bcg;  // CG beta
    double* als;  // line-search step length
    double* slope;
    int* status;
    int* iters;
    int* act;     // Newton iteration running
    int* cgact;
    int* srch;    // searching in the line search
    int* trials;
    int* cnt;     // counters read by the host
    double eta_min, eta_max, rel_tol, abs_tol, c1, shrink;
    int max_iter, ls_max, cg_max;
};

__device__ inline int sym9(int p, int q)
{
    if (p > q) {
        const int t = p;
        p = q;
        q = t;
    }
    return p * 9 - (p * (p - 1)) / 2 + (q - p);
}

// G = F - I of element e for item b at U + alpha dx (alpha = 0: U)
__device__ inline void elem_grad_u(const FsArgs& a, const double* ec, int e, int b, double alpha, double* G)
{
#pragma unroll
    for (int m = 0; m < 9; ++m) G[m] = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int v = a.tets[4 * e + c];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const size_t o = (size_t)(3 * v + i) * a.Bp + b;
            double u = a.U[o];
            if (alpha != 0.0) u += alpha * a.dx[o];
#pragma unroll
            for (int j = 0; j < 3; ++j) G[3 * j + i] += u * ec[3 * c + j];
        }
    }
}

// Element pass.  MODE 0: energies at U + als dx of searching items; MODE 1:
// energy, V PK1 (Se) and Aeff (Ae) at U of running items, with the items whose
// M is not positive definite appended to the projection list.
template <int MODE>
__global__ __launch_bounds__(256) void k_fs_elem(FsArgs a)
{
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int b = blockIdx.y * 64 + lane;
    const bool on = b < a.B && (MODE == 0 ? a.srch[b] != 0 : a.act[b] != 0);
    double esum = 0.0;
    const double alpha = (MODE == 0 && on) ? a.als[b] : 0.0;
    for (int k = 0; k < kEpw; ++k) {
        const int e = (blockIdx.x * 4 + wave) * kEpw + k;
        if (e >= a.ne || !on) continue;
        const double* ec = a.ec + (size_t)e * kEc;
        double G[9];
        elem_grad_u(a, ec, e, b, alpha, G);
        Snh<double> sn;
        sn.set(G, a.mu, a.lam);
        const double V = ec[12];
        esum += V * sn.psi;
        if (MODE == 0) continue;
        double P[9];
        sn.pk1(a.mu, a.lam, P);
#pragma unroll
        for (int m = 0; m < 9; ++m) a.Se[((size_t)e * 9 + m) * a.Bp + b] = V * P[m];
        // M = V Bh A Bh (packed upper triangle), one column per apply of A
        const double* Nh = ec + 13;
        const double* Ni = ec + 22;
        double M[45];
#pragma unroll
        for (int qc = 0; qc < 9; ++qc) {
            const int jq = qc / 3, iq = qc % 3;
            double wv[9], y[9];
#pragma unroll
            for (int m = 0; m < 9; ++m) wv[m] = (m % 3 == iq) ? Nh[3 * (m / 3) + jq] : 0.0;
            sn.apply_hess(a.mu, a.lam, wv, y);
#pragma unroll
            for (int pr = 0; pr <= qc; ++pr) {
                const int jp = pr / 3, ip = pr % 3;
                M[sym9(pr, qc)] = V * (Nh[3 * jp + 0] * y[ip] + Nh[3 * jp + 1] * y[3 + ip] + Nh[3 * jp + 2] * y[6 + ip]);
            }
        }
        // positive definite?  Cholesky on a copy
        double Lc[45];
#pragma unroll
        for (int m = 0; m < 45; ++m) Lc[m] = M[m];
        bool pd = true;
#pragma unroll
        for (int k2 = 0; k2 < 9; ++k2) {
            double d = Lc[sym9(k2, k2)];
#pragma unroll
            for (int m = 0; m < k2; ++m) d -= Lc[sym9(m, k2)] * Lc[sym9(m, k2)];
            pd = pd && d > 0.0;
            const double inv = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
            Lc[sym9(k2, k2)] = d > 0.0 ? sqrt(d) : 0.0;
#pragma unroll
            for (int c2 = k2 + 1; c2 < 9; ++c2) {
                double t = Lc[sym9(k2, c2)];
#pragma unroll
                for (int m = 0; m < k2; ++m) t -= Lc[sym9(m, k2)] * Lc[sym9(m, c2)];
                Lc[sym9(k2, c2)] = t * inv;
            }
        }
        double* Ao = a.Ae + (size_t)e * 45 * a.Bp + b;
        if (pd) {
            // Aeff = Bhi M Bhi (= V A)
#pragma unroll
            for (int pr = 0; pr < 9; ++pr)
#pragma unroll
                for (int qc = pr; qc < 9; ++qc) {
                    const int jp = pr / 3, ip = pr % 3, jq = qc / 3, iq = qc % 3;
                    double t = 0.0;
#pragma unroll
                    for (int u = 0; u < 3; ++u)
#pragma unroll
                        for (int v = 0; v < 3; ++v) t += Ni[3 * jp + u] * M[sym9(3 * u + ip, 3 * v + iq)] * Ni[3 * v + jq];
                    Ao[(size_t)sym9(pr, qc) * a.Bp] = t;
                }
        } else {
            // M itself, projected by k_fs_psd
#pragma unroll
            for (int m = 0; m < 45; ++m) Ao[(size_t)m * a.Bp] = M[m];
            const int slot = atomicAdd(a.nlist, 1);
            a.list[slot] = e * a.Bp + b;
        }
    }
    red[wave][lane] = esum;
    __syncthreads();
    if (wave == 0) {
        const double s = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
        a.pe[(size_t)blockIdx.x * a.Bp + blockIdx.y * 64 + lane] = s;
    }
}

// Projection of the listed elements: cyclic Jacobi on M (thread-private slices of
// LDS), negative eigenvalues set to zero, Aeff = Bhi proj(M) Bhi.
__global__ __launch_bounds__(kPsdT) void k_fs_psd(FsArgs a)
{
    __shared__ double sM[81 * kPsdT];
    __shared__ double sV[81 * kPsdT];
    const int t = threadIdx.x;
    double* M = sM + t;
    double* Vv = sV + t;
    const int count = *a.nlist;
    for (int k = blockIdx.x * kPsdT + t; k < count; k += gridDim.x * kPsdT) {
        const int ent = a.list[k];
        const int e = ent / a.Bp, b = ent - e * a.Bp;
        double* Ao = a.Ae + (size_t)e * 45 * a.Bp + b;
        for (int pr = 0; pr < 9; ++pr)
            for (int qc = 0; qc < 9; ++qc) {
                M[(pr * 9 + qc) * kPsdT] = Ao[(size_t)sym9(pr, qc) * a.Bp];
                Vv[(pr * 9 + qc) * kPsdT] = pr == qc ? 1.0 : 0.0;
            }
        for (int sweep = 0; sweep < 60; ++sweep) {
            double off = 0.0, tot = 0.0;
            for (int pr = 0; pr < 9; ++pr)
                for (int qc = 0; qc < 9; ++qc) {
                    const double x = M[(pr * 9 + qc) * kPsdT];
                    tot += x * x;
                    if (pr != qc) off += x * x;
                }
            if (off <= 1e-30 * tot || off == 0.0) break;
            for (int pr = 0; pr < 8; ++pr)
                for (int qc = pr + 1; qc < 9; ++qc) {
                    const double apq = M[(pr * 9 + qc) * kPsdT];
                    if (apq == 0.0) continue;
                    const double th = (M[(qc * 9 + qc) * kPsdT] - M[(pr * 9 + pr) * kPsdT]) / (2.0 * apq);
                    const double tt = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                    const double c = 1.0 / sqrt(tt * tt + 1.0), sn = tt * c;
                    for (int m = 0; m < 9; ++m) {
                        const double mp = M[(m * 9 + pr) * kPsdT], mq = M[(m * 9 + qc) * kPsdT];
                        M[(m * 9 + pr) * kPsdT] = c * mp - sn * mq;
                        M[(m * 9 + qc) * kPsdT] = sn * mp + c * mq;
                    }
                    for (int m = 0; m < 9; ++m) {
                        const double mp = M[(pr * 9 + m) * kPsdT], mq = M[(qc * 9 + m) * kPsdT];
                        M[(pr * 9 + m) * kPsdT] = c * mp - sn * mq;
                        M[(qc * 9 + m) * kPsdT] = sn * mp + c * mq;
                    }
                    for (int m = 0; m < 9; ++m) {
                        const double vp = Vv[(m * 9 + pr) * kPsdT], vq = Vv[(m * 9 + qc) * kPsdT];
                        Vv[(m * 9 + pr) * kPsdT] = c * vp - sn * vq;
                        Vv[(m * 9 + qc) * kPsdT] = sn * vp + c * vq;
                    }
                }
        }
        // proj(M) into M's slots: sum over non-negative eigenpairs lam v v^T
        double lamk[9];
        for (int m = 0; m < 9; ++m) lamk[m] = fmax(M[(m * 9 + m) * kPsdT], 0.0);
        for (int pr = 0; pr < 9; ++pr)
            for (int qc = 0; qc < 9; ++qc) {
                double s = 0.0;
                for (int m = 0; m < 9; ++m) s += Vv[(pr * 9 + m) * kPsdT] * lamk[m] * Vv[(qc * 9 + m) * kPsdT];
                M[(pr * 9 + qc) * kPsdT] = s;
            }
        const double* Ni = a.ec + (size_t)e * kEc + 22;
        for (int pr = 0; pr < 9; ++pr)
            for (int qc = pr; qc < 9; ++qc) {
                const int jp = pr / 3, ip = pr % 3, jq = qc / 3, iq = qc % 3;
                double s = 0.0;
                for (int u = 0; u < 3; ++u)
                    for (int v = 0; v < 3; ++v)
                        s += Ni[3 * jp + u] * M[((3 * u + ip) * 9 + 3 * v + iq) * kPsdT] * Ni[3 * v + jq];
                Ao[(size_t)sym9(pr, qc) * a.Bp] = s;
            }
    }
}

// Element product: Se = Aeff (D p_e) for CG-active items
__global__ __launch_bounds__(256) void k_fs_mv_elem(FsArgs a)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int b = blockIdx.y * 64 + lane;
    if (b >= a.B || !a.cgact[b]) return;
    for (int k = 0; k < kEpw; ++k) {
        const int e = (blockIdx.x * 4 + wave) * kEpw + k;
        if (e >= a.ne) return;
        const double* ec = a.ec + (size_t)e * kEc;
        double u[9];
#pragma unroll
        for (int m = 0; m < 9; ++m) u[m] = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int v = a.tets[4 * e + c];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double pv = a.p[(size_t)(3 * v + i) * a.Bp + b];
#pragma unroll
                for (int j = 0; j < 3; ++j) u[3 * j + i] += pv * ec[3 * c + j];
            }
        }
        const double* Ao = a.Ae + (size_t)e * 45 * a.Bp + b;
        double A[45];
#pragma unroll
        for (int m = 0; m < 45; ++m) A[m] = Ao[(size_t)m * a.Bp];
#pragma unroll
        for (int pr = 0; pr < 9; ++pr) {
            double s = 0.0;
#pragma unroll
            for (int qc = 0; qc < 9; ++qc) s += A[sym9(pr, qc)] * u[qc];
            a.Se[((size_t)e * 9 + pr) * a.Bp + b] = s;
        }
    }
}

// Vertex gather: out_v = sum over incident (e, corner c) of sum_j Dv_e[c][j] Se[e][3 j + i]
__device__ inline void gather_v(const FsArgs& a, int v, int b, double* o)
{
    o[0] = o[1] = o[2] = 0.0;
    for (int k = a.vptr[v]; k < a.vptr[v + 1]; ++k) {
        const int ent = a.vinc[k], e = ent >> 2, c = ent & 3;
        const double* dv = a.ec + (size_t)e * kEc + 3 * c;
        const double* S = a.Se + (size_t)e * 9 * a.Bp + b;
#pragma unroll
        for (int i = 0; i < 3; ++i)
            o[i] += dv[0] * S[(size_t)i * a.Bp] + dv[1] * S[(size_t)(3 + i) * a.Bp] + dv[2] * S[(size_t)(6 + i) * a.Bp];
    }
}

// external energy of dof (v, i) of item b at displacement u: gravity, penalty, force
__device__ inline double ext_energy(const FsArgs& a, int v, int ts, int i, int b, double u)
{
    double e = -a.mass[v] * a.grav[i] * u;
    if (ts >= 0 && a.targets) {
        const double d = a.X[3 * v + i] + u - a.targets[((size_t)b * a.nt + ts) * 3 + i];
        e += 0.5 * a.kc * d * d;
    }
    if (a.fvert[v] && a.force) e -= a.force[(size_t)b * 3 + i] * u;
    return e;
}

// MODE 0 (gradient): g, the Jacobi diagonal, and per workgroup: external energy,
// max |g|, sum g^2 (free dofs) into pv[{0,1,2} nvb + block].
// MODE 1 (product): q = H p and per workgroup sum p.q into pv[block].
template <int MODE>
__global__ __launch_bounds__(256) void k_fs_gather(FsArgs a)
{
    __shared__ double red[3][4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int b = blockIdx.y * 64 + lane;
    const bool on = b < a.B && (MODE == 0 ? a.act[b] != 0 : a.cgact[b] != 0);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int k = 0; k < kVpw && on; ++k) {
        const int v = (blockIdx.x * 4 + wave) * kVpw + k;
        if (v >= a.nv) break;
        double o[3];
        const size_t o0 = (size_t)(3 * v) * a.Bp + b;
        const int ts = a.tslot[v];
        if (a.pinned[v]) {
            // fixed dofs: no gradient or product, but their external energy counts
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                if (MODE == 0) {
                    a.g[o0 + (size_t)i * a.Bp] = 0.0;
                    a.dg[o0 + (size_t)i * a.Bp] = 1.0;
                    s0 += ext_energy(a, v, ts, i, b, a.U[o0 + (size_t)i * a.Bp]);
                } else {
                    a.q[o0 + (size_t)i * a.Bp] = 0.0;
                }
            }
            continue;
        }
        gather_v(a, v, b, o);
        if (MODE == 0) {
            double ext = 0.0;
            double diag[3] = {0.0, 0.0, 0.0};
            for (int kk = a.vptr[v]; kk < a.vptr[v + 1]; ++kk) {
                const int ent = a.vinc[kk], e = ent >> 2, c = ent & 3;
                const double* dv = a.ec + (size_t)e * kEc + 3 * c;
                const double* Ao = a.Ae + (size_t)e * 45 * a.Bp + b;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    double d = 0.0;
#pragma unroll
                    for (int j = 0; j < 3; ++j)
#pragma unroll
                        for (int jj = 0; jj < 3; ++jj) d += dv[j] * dv[jj] * Ao[(size_t)sym9(3 * j + i, 3 * jj + i) * a.Bp];
                    diag[i] += d;
                }
            }
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double u = a.U[o0 + (size_t)i * a.Bp];
                double gi = o[i] - a.mass[v] * a.grav[i];
                ext += ext_energy(a, v, ts, i, b, u);
                double di = diag[i];
                if (ts >= 0 && a.targets) {
                    gi += a.kc * (a.X[3 * v + i] + u - a.targets[((size_t)b * a.nt + ts) * 3 + i]);
                    di += a.kc;
                }
                if (a.fvert[v] && a.force) gi -= a.force[(size_t)b * 3 + i];
                a.g[o0 + (size_t)i * a.Bp] = gi;
                a.dg[o0 + (size_t)i * a.Bp] = di > 0.0 ? di : 1.0;
                s1 = fmax(s1, fabs(gi));
                s2 += gi * gi;
            }
            s0 += ext;
        } else {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double pv = a.p[o0 + (size_t)i * a.Bp];
                double qi = o[i];
                if (ts >= 0 && a.targets) qi += a.kc * pv;
                a.q[o0 + (size_t)i * a.Bp] = qi;
                s0 += pv * qi;
            }
        }
    }
    red[0][wave][lane] = s0;
    red[1][wave][lane] = s1;
    red[2][wave][lane] = s2;
    __syncthreads();
    if (wave == 0) {
        const size_t o = (size_t)blockIdx.x * a.Bp + blockIdx.y * 64 + lane;
        a.pv[o] = ((red[0][0][lane] + red[0][1][lane]) + red[0][2][lane]) + red[0][3][lane];
        if (MODE == 0) {
            a.pv[(size_t)a.nvb * a.Bp + o] = fmax(fmax(red[1][0][lane], red[1][1][lane]), fmax(red[1][2][lane], red[1][3][lane]));
            a.pv[(size_t)2 * a.nvb * a.Bp + o] = ((red[2][0][lane] + red[2][1][lane]) + red[2][2][lane]) + red[2][3][lane];
        }
    }
}

// External energy at U + als dx of searching items, per vertex workgroup into pv
__global__ __launch_bounds__(256) void k_fs_ext_energy(FsArgs a)
{
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int b = blockIdx.y * 64 + lane;
    const bool on = b < a.B && a.srch[b] != 0;
    double s = 0.0;
    const double al = on ? a.als[b] : 0.0;
    for (int k = 0; k < kVpw && on; ++k) {
        const int v = (blockIdx.x * 4 + wave) * kVpw + k;
        if (v >= a.nv) break;
        const int ts = a.tslot[v];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const size_t o = (size_t)(3 * v + i) * a.Bp + b;
            s += ext_energy(a, v, ts, i, b, a.U[o] + al * a.dx[o]);
        }
    }
    red[wave][lane] = s;
    __syncthreads();
    if (wave == 0)
        a.pv[(size_t)blockIdx.x * a.Bp + blockIdx.y * 64 + lane] =
            ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// Newton bookkeeping after the gradient: E, |g|_inf, exits I, IV and non-finite,
// and the CG start (r = -g, z = r / diag, p = z) is left to k_fs_cg_init.
__global__ void k_fs_check(FsArgs a, int it)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.B || !a.act[b]) return;
    double E = 0.0, gi = 0.0, g2 = 0.0;
    for (int k = 0; k < a.neb; ++k) E += a.pe[(size_t)k * a.Bp + b];
    for (int k = 0; k < a.nvb; ++k) {
        E += a.pv[(size_t)k * a.Bp + b];
        gi = fmax(gi, a.pv[(size_t)(a.nvb + k) * a.Bp + b]);
        g2 += a.pv[(size_t)(2 * a.nvb + k) * a.Bp + b];
    }
    a.E[b] = E;
    a.ginf[b] = gi;
    a.gn2[b] = g2;
    if (it == 0) a.g0[b] = gi;
    int st = FS_RUNNING;
    if (!isfinite(E) || !isfinite(g2)) st = FS_NONFINITE;
    else if (gi <= a.abs_tol || gi <= a.rel_tol * a.g0[b]) st = FS_CONVERGED;
    else if (it >= a.max_iter) st = FS_ITER_MAX;
    if (st != FS_RUNNING) {
        a.status[b] = st;
        a.act[b] = 0;
    } else {
        atomicAdd(a.cnt, 1);
    }
}

// CG start per dof: dx = 0, r = -g, z = r / diag, p = z; per workgroup sum r.z into pv
__global__ __launch_bounds__(256) void k_fs_cg_init(FsArgs a)
{
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int b = blockIdx.y * 64 + lane;
    const bool on = b < a.B && a.act[b] != 0;
    double s = 0.0;
    for (int k = 0; k < 3 * kVpw && on; ++k) {
        const int d = (blockIdx.x * 4 + wave) * 3 * kVpw + k;
        if (d >= a.n) break;
        const size_t o = (size_t)d * a.Bp + b;
        const double r = -a.g[o], z = r / a.dg[o];
        a.dx[o] = 0.0;
        a.r[o] = r;
        a.z[o] = z;
        a.p[o] = z;
        s += r * z;
    }
    red[wave][lane] = s;
    __syncthreads();
    if (wave == 0)
        a.pv[(size_t)blockIdx.x * a.Bp + blockIdx.y * 64 + lane] =
            ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// rz, the stopping level (eta |g|_2)^2 and the CG-active flags
__global__ void k_fs_cg_start(FsArgs a)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.Bp) return;
    if (b >= a.B || !a.act[b]) {
        a.cgact[b] = 0;
        return;
    }
    double rz = 0.0;
    for (int k = 0; k < a.nvb; ++k) rz += a.pv[(size_t)k * a.Bp + b];
    a.rz[b] = rz;
    const double rel = a.g0[b] > 0.0 ? a.ginf[b] / a.g0[b] : 1.0;
    const double eta = fmin(a.eta_max, fmax(a.eta_min, sqrt(rel)));
    a.tol2[b] = eta * eta * a.gn2[b];
    a.cgact[b] = a.gn2[b] > 0.0 ? 1 : 0;
}

// alpha = r.z / p.q (CG-active items); a non-positive curvature ends the item's CG
__global__ void k_fs_cg_alpha(FsArgs a)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.B || !a.cgact[b]) return;
    double pq = 0.0;
    for (int k = 0; k < a.nvb; ++k) pq += a.pv[(size_t)k * a.Bp + b];
    if (pq > 0.0) {
        a.acg[b] = a.rz[b] / pq;
    } else {
        a.acg[b] = 0.0;
        a.cgact[b] = 0;
    }
}

// dx += alpha p, r -= alpha q, z = r / diag; per workgroup r.z and r.r into pv
__global__ __launch_bounds__(256) void k_fs_cg_update(FsArgs a)
{
    __shared__ double red[2][4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int b = blockIdx.y * 64 + lane;
    const bool on = b < a.B && a.cgact[b] != 0;
    double s0 = 0.0, s1 = 0.0;
    const double al = on ? a.acg[b] : 0.0;
    for (int k = 0; k < 3 * kVpw && on; ++k) {
        const int d = (blockIdx.x * 4 + wave) * 3 * kVpw + k;
        if (d >= a.n) break;
        const size_t o = (size_t)d * a.Bp + b;
        a.dx[o] += al * a.p[o];
        const double r = a.r[o] - al * a.q[o];
        const double z = r / a.dg[o];
        a.r[o] = r;
        a.z[o] = z;
        s0 += r * z;
        s1 += r * r;
    }
    red[0][wave][lane] = s0;
    red[1][wave][lane] = s1;
    __syncthreads();
    if (wave == 0) {
        const size_t o = (size_t)blockIdx.x * a.Bp + blockIdx.y * 64 + lane;
        a.pv[o] = ((red[0][0][lane] + red[0][1][lane]) + red[0][2][lane]) + red[0][3][lane];
        a.pv[(size_t)a.nvb * a.Bp + o] = ((red[1][0][lane] + red[1][1][lane]) + red[1][2][lane]) + red[1][3][lane];
    }
}

// beta = r.z (new) / r.z (old), the stopping test and the count of CG-active items
__global__ void k_fs_cg_beta(FsArgs a, int last)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.B || !a.cgact[b]) return;
    double rz = 0.0, rr = 0.0;
    for (int k = 0; k < a.nvb; ++k) {
        rz += a.pv[(size_t)k * a.Bp + b];
        rr += a.pv[(size_t)(a.nvb + k) * a.Bp + b];
    }
    a.bcg[b] = a.rz[b] > 0.0 ? rz / a.rz[b] : 0.0;
    a.rz[b] = rz;
    if (rr <= a.tol2[b] || last || !isfinite(rr)) {
        a.cgact[b] = 0;
    } else {
        atomicAdd(a.cnt + 1, 1);
    }
}

// p = z + beta p (items still in CG)
__global__ __launch_bounds__(256) void k_fs_cg_p(FsArgs a)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int b = blockIdx.y * 64 + lane;
    if (b >= a.B || !a.cgact[b]) return;
    const double be = a.bcg[b];
    for (int k = 0; k < 3 * kVpw; ++k) {
        const int d = (blockIdx.x * 4 + wave) * 3 * kVpw + k;
        if (d >= a.n) break;
        const size_t o = (size_t)d * a.Bp + b;
        a.p[o] = a.z[o] + be * a.p[o];
    }
}

// per workgroup g.dx into pv
__global__ __launch_bounds__(256) void k_fs_slope(FsArgs a)
{
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int b = blockIdx.y * 64 + lane;
    const bool on = b < a.B && a.act[b] != 0;
    double s = 0.0;
    for (int k = 0; k < 3 * kVpw && on; ++k) {
        const int d = (blockIdx.x * 4 + wave) * 3 * kVpw + k;
        if (d >= a.n) break;
        const size_t o = (size_t)d * a.Bp + b;
        s += a.g[o] * a.dx[o];
    }
    red[wave][lane] = s;
    __syncthreads();
    if (wave == 0)
        a.pv[(size_t)blockIdx.x * a.Bp + blockIdx.y * 64 + lane] =
            ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// the slope and the line-search start (alpha = 1); exit II when dx is no descent direction
__global__ void k_fs_ls_start(FsArgs a)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.Bp) return;
    if (b >= a.B || !a.act[b]) {
        a.srch[b] = 0;
        return;
    }
    double sl = 0.0;
    for (int k = 0; k < a.nvb; ++k) sl += a.pv[(size_t)k * a.Bp + b];
    a.slope[b] = sl;
    if (!(sl < 0.0)) {
        a.status[b] = FS_NOT_DESCENT;
        a.act[b] = 0;
        a.srch[b] = 0;
        return;
    }
    a.als[b] = 1.0;
    a.trials[b] = 0;
    a.srch[b] = 1;
}

// Armijo test of the trial energy; accepted items keep als, others halve it
__global__ void k_fs_armijo(FsArgs a)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.B || !a.srch[b]) return;
    double Et = 0.0;
    for (int k = 0; k < a.neb; ++k) Et += a.pe[(size_t)k * a.Bp + b];
    for (int k = 0; k < a.nvb; ++k) Et += a.pv[(size_t)k * a.Bp + b];
    const double al = a.als[b];
    if (isfinite(Et) && Et - a.E[b] <= a.c1 * al * a.slope[b]) {
        a.srch[b] = 0;   // accepted: act stays set, als is the step
        return;
    }
    const int t = a.trials[b] + 1;
    a.trials[b] = t;
    if (t >= a.ls_max) {
        a.srch[b] = 0;
        a.act[b] = 0;
        a.status[b] = FS_LS_MAX;
        return;
    }
    a.als[b] = al * a.shrink;
    atomicAdd(a.cnt + 2, 1);
}

// U += als dx for items that accepted a step; iteration count
__global__ __launch_bounds__(256) void k_fs_step(FsArgs a)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int b = blockIdx.y * 64 + lane;
    if (b >= a.B || !a.act[b]) return;
    const double al = a.als[b];
    for (int k = 0; k < 3 * kVpw; ++k) {
        const int d = (blockIdx.x * 4 + wave) * 3 * kVpw + k;
        if (d >= a.n) break;
        const size_t o = (size_t)d * a.Bp + b;
        a.U[o] += al * a.dx[o];
    }
    if (blockIdx.x == 0 && wave == 0) a.iters[b] += 1;
}

// item-major (B x n) <-> dof-major (n x Bp) through LDS
__global__ __launch_bounds__(256) void k_fs_transpose(const double* src, double* dst, int n, int B, int Bp, int to_dof)
{
    __shared__ double tile[32][33];
    const int d0 = blockIdx.x * 32, b0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    if (to_dof) {
        for (int k = ty; k < 32; k += 8) {
            const int b = b0 + k, d = d0 + tx;
            tile[k][tx] = (b < B && d < n) ? src[(size_t)b * n + d] : 0.0;
        }
        __syncthreads();
        for (int k = ty; k < 32; k += 8) {
            const int d = d0 + k, b = b0 + tx;
            if (d < n && b < Bp) dst[(size_t)d * Bp + b] = tile[tx][k];
        }
    } else {
        for (int k = ty; k < 32; k += 8) {
            const int d = d0 + k, b = b0 + tx;
            tile[k][tx] = (d < n && b < B) ? src[(size_t)d * Bp + b] : 0.0;
        }
        __syncthreads();
        for (int k = ty; k < 32; k += 8) {
            const int b = b0 + k, d = d0 + tx;
            if (b < B && d < n) dst[(size_t)b * n + d] = tile[tx][k];
        }
    }
}

__global__ void k_fs_init(FsArgs a)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.Bp) return;
    const int on = b < a.B;
    a.status[b] = on ? FS_RUNNING : FS_CONVERGED;
    a.iters[b] = 0;
    a.act[b] = on;
    a.cgact[b] = 0;
    a.srch[b] = 0;
    a.g0[b] = 0.0;
    a.E[b] = 0.0;
    a.ginf[b] = 0.0;
}

__global__ void k_fs_outputs(FsArgs a, int32_t* iters, int32_t* status, double* relgrad, double* E)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.B) return;
    if (iters) iters[b] = a.iters[b];
    if (status) status[b] = a.status[b];
    if (relgrad) relgrad[b] = a.g0[b] > 0.0 ? a.ginf[b] / a.g0[b] : 0.0;
    if (E) E[b] = a.E[b];
}

__global__ void k_fs_zero_int(int* p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct FullSolver {
    int ne = 0, nv = 0, n = 0, nt = 0;
    double mu = 0.0, lam = 0.0, kc = 0.0, grav[3] = {0, 0, 0};
    std::vector<void*> bufs;
    int* tets = nullptr;
    double* ec = nullptr;
    int* vptr = nullptr;
    int* vinc = nullptr;
    double* mass = nullptr;
    uint8_t* pinned = nullptr;
    int* tslot = nullptr;
    uint8_t* fvert = nullptr;
    double* X = nullptr;
    // batch workspace
    int Bcap = 0;
    std::vector<void*> wbufs;
    FsArgs a{};
    int* hcnt = nullptr;   // pinned host counters
};

static void* fs_alloc(std::vector<void*>& v, size_t bytes)
{
    void* p = nullptr;
    if (hipMalloc(&p, bytes ? bytes : 1) != hipSuccess) return nullptr;
    v.push_back(p);
    return p;
}

static void fs_free_list(std::vector<void*>& v)
{
    for (void* p : v) (void)hipFree(p);
    v.clear();
}

void full_solver_destroy(FullSolver* f)
{
    if (!f) return;
    (void)hipDeviceSynchronize();
    fs_free_list(f->bufs);
    fs_free_list(f->wbufs);
    if (f->hcnt) (void)hipHostFree(f->hcnt);
    delete f;
}

// principal square root of a 3x3 SPD matrix and its inverse (cyclic Jacobi)
static void sqrt3(const double* N, double* Sq, double* Si)
{
    double A[9], Q[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    std::memcpy(A, N, sizeof A);
    for (int sweep = 0; sweep < 50; ++sweep) {
        const double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
        if (off < 1e-34 * (A[0] * A[0] + A[4] * A[4] + A[8] * A[8])) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                const double apq = A[3 * p + q];
                if (apq == 0.0) continue;
                const double th = (A[3 * q + q] - A[3 * p + p]) / (2.0 * apq);
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < 3; ++k) {
                    const double akp = A[3 * k + p], akq = A[3 * k + q];
                    A[3 * k + p] = c * akp - s * akq;
                    A[3 * k + q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {
                    const double apk = A[3 * p + k], aqk = A[3 * q + k];
                    A[3 * p + k] = c * apk - s * aqk;
                    A[3 * q + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 3; ++k) {
                    const double qkp = Q[3 * k + p], qkq = Q[3 * k + q];
                    Q[3 * k + p] = c * qkp - s * qkq;
                    Q[3 * k + q] = s * qkp + c * qkq;
                }
            }
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double x = 0.0, y = 0.0;
            for (int k = 0; k < 3; ++k) {
                const double l = std::sqrt(A[4 * k]);
                x += Q[3 * i + k] * l * Q[3 * j + k];
                y += Q[3 * i + k] / l * Q[3 * j + k];
            }
            Sq[3 * i + j] = x;
            Si[3 * i + j] = y;
        }
}

int full_solver_create(const FullSolverDesc& d, FullSolver** out, const char** why)
{
    *out = nullptr;
    FullSolver* f = new (std::nothrow) FullSolver();
    if (!f) {
        *why = "host allocation failed";
        return RS_ERR_OOM;
    }
    f->ne = d.ne;
    f->nv = d.nv;
    f->n = 3 * d.nv;
    f->nt = d.nt;
    f->mu = d.mu;
    f->lam = d.lam;
    f->kc = d.kc;
    for (int i = 0; i < 3; ++i) f->grav[i] = d.grav[i];
    // per-element constants from the rest shape
    std::vector<double> ec((size_t)d.ne * kEc, 0.0);
    for (int e = 0; e < d.ne; ++e) {
        const int* t = d.tets + 4 * e;
        double Dm[9];
        for (int j = 0; j < 3; ++j)
            for (int i = 0; i < 3; ++i) Dm[3 * i + j] = d.X[3 * t[j + 1] + i] - d.X[3 * t[0] + i];
        const double det = Dm[0] * (Dm[4] * Dm[8] - Dm[5] * Dm[7]) - Dm[1] * (Dm[3] * Dm[8] - Dm[5] * Dm[6]) +
                           Dm[2] * (Dm[3] * Dm[7] - Dm[4] * Dm[6]);
        if (!(det > 0.0)) {
            delete f;
            *why = "a mesh element has non-positive volume";
            return RS_ERR_ARG;
        }
        double Di[9];
        Di[0] = (Dm[4] * Dm[8] - Dm[5] * Dm[7]) / det;
        Di[1] = (Dm[2] * Dm[7] - Dm[1] * Dm[8]) / det;
        Di[2] = (Dm[1] * Dm[5] - Dm[2] * Dm[4]) / det;
        Di[3] = (Dm[5] * Dm[6] - Dm[3] * Dm[8]) / det;
        Di[4] = (Dm[0] * Dm[8] - Dm[2] * Dm[6]) / det;
        Di[5] = (Dm[2] * Dm[3] - Dm[0] * Dm[5]) / det;
        Di[6] = (Dm[3] * Dm[7] - Dm[4] * Dm[6]) / det;
        Di[7] = (Dm[1] * Dm[6] - Dm[0] * Dm[7]) / det;
        Di[8] = (Dm[0] * Dm[4] - Dm[1] * Dm[3]) / det;
        // shape gradients: corner a >= 1 is row a-1 of Dm^-1, corner 0 minus their sum
        double Dv[4][3];
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int c = 1; c < 4; ++c) {
                Dv[c][j] = Di[3 * (c - 1) + j];
                s += Dv[c][j];
            }
            Dv[0][j] = -s;
        }
        double N[9] = {0};
        for (int c = 0; c < 4; ++c)
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) N[3 * i + j] += Dv[c][i] * Dv[c][j];
        double* o = &ec[(size_t)e * kEc];
        for (int c = 0; c < 4; ++c)
            for (int j = 0; j < 3; ++j) o[3 * c + j] = Dv[c][j];
        o[12] = det / 6.0;
        sqrt3(N, o + 13, o + 22);
    }
    // incidence lists and vertex flags
    std::vector<int> vptr(d.nv + 1, 0), vinc;
    for (int e = 0; e < d.ne; ++e)
        for (int c = 0; c < 4; ++c) vptr[d.tets[4 * e + c] + 1]++;
    for (int v = 0; v < d.nv; ++v) vptr[v + 1] += vptr[v];
    vinc.assign(vptr[d.nv], 0);
    {
        std::vector<int> fill(vptr.begin(), vptr.end() - 1);
        for (int e = 0; e < d.ne; ++e)
            for (int c = 0; c < 4; ++c) vinc[fill[d.tets[4 * e + c]]++] = 4 * e + c;
    }
    std::vector<int> tslot(d.nv, -1);
    for (int t = 0; t < d.nt; ++t) tslot[d.tvtx[t]] = t;
    std::vector<uint8_t> fvert(d.nv, 0);
    for (int t = 0; t < d.nf; ++t) fvert[d.fvtx[t]] = 1;
    bool ok = true;
    auto up = [&](const void* src, size_t bytes) {
        void* p = fs_alloc(f->bufs, bytes);
        ok = ok && p && hipMemcpy(p, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
        return p;
    };
    f->tets = (int*)up(d.tets, sizeof(int) * 4 * d.ne);
    f->ec = (double*)up(ec.data(), sizeof(double) * ec.size());
    f->vptr = (int*)up(vptr.data(), sizeof(int) * vptr.size());
    f->vinc = (int*)up(vinc.data(), sizeof(int) * vinc.size());
    f->mass = (double*)up(d.mass, sizeof(double) * d.nv);
    f->pinned = (uint8_t*)up(d.pinned, d.nv);
    f->tslot = (int*)up(tslot.data(), sizeof(int) * d.nv);
    f->fvert = (uint8_t*)up(fvert.data(), d.nv);
    f->X = (double*)up(d.X, sizeof(double) * 3 * d.nv);
    ok = ok && hipHostMalloc((void**)&f->hcnt, 4 * sizeof(int), hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        full_solver_destroy(f);
        *why = "full-space solver allocation failed";
        return RS_ERR_OOM;
    }
    *out = f;
    return RS_OK;
}

static bool fs_workspace(FullSolver* f, int Bp)
{
    if (Bp <= f->Bcap) return true;
    (void)hipDeviceSynchronize();
    fs_free_list(f->wbufs);
    f->Bcap = 0;
    FsArgs& a = f->a;
    a = FsArgs{};
    const size_t n = f->n, ne = f->ne, B = Bp;
    a.neb = (int)((ne + 4 * kEpw - 1) / (4 * kEpw));
    a.nvb = (f->nv + 4 * kVpw - 1) / (4 * kVpw);
    bool ok = true;
    auto D = [&](size_t count) {
        void* p = fs_alloc(f->wbufs, count * sizeof(double));
        ok = ok && p;
        return (double*)p;
    };
    auto I = [&](size_t count) {
        void* p = fs_alloc(f->wbufs, count * sizeof(int));
        ok = ok && p;
        return (int*)p;
    };
    a.U = D(n * B); a.dx = D(n * B); a.g = D(n * B); a.dg = D(n * B);
    a.r = D(n * B); a.z = D(n * B); a.p = D(n * B); a.q = D(n * B);
    a.Se = D(ne * 9 * B);
    a.Ae = D(ne * 45 * B);
    a.list = I(ne * B);
    a.nlist = I(1);
    a.pe = D((size_t)a.neb * B);
    a.pv = D((size_t)3 * std::max(a.nvb, (int)((n + 12 * kVpw - 1) / (12 * kVpw))) * B);
    a.E = D(B); a.Et = D(B); a.g0 = D(B); a.ginf = D(B); a.gn2 = D(B); a.rz = D(B); a.tol2 = D(B);
    a.acg = D(B); a.bcg = D(B); a.als = D(B); a.slope = D(B);
    a.status = I(B); a.iters = I(B); a.act = I(B); a.cgact = I(B); a.srch = I(B); a.trials = I(B);
    a.cnt = I(4);
    if (!ok) {
        fs_free_list(f->wbufs);
        return false;
    }
    f->Bcap = Bp;
    return true;
}

// Per-dof kernels use 3 kVpw dofs per wave; their partials use the vertex-pass
// block count, which covers n dofs as 3 kVpw per wave exactly when n = 3 nv.
int full_solve(FullSolver* f, const FullSolveCall& call, hipStream_t s, const char** why)
{
    const int B = call.B;
    if (B == 0) return RS_OK;
    const int Bp = (B + 63) / 64 * 64;
    if (!fs_workspace(f, Bp)) {
        *why = "full-space solver workspace allocation failed";
        return RS_ERR_OOM;
    }
    FsArgs a = f->a;
    a.ne = f->ne; a.nv = f->nv; a.n = f->n; a.Bp = Bp; a.B = B;
    a.tets = f->tets; a.ec = f->ec; a.vptr = f->vptr; a.vinc = f->vinc; a.mass = f->mass;
    a.pinned = f->pinned; a.tslot = f->tslot; a.fvert = f->fvert; a.X = f->X;
    a.targets = call.targets; a.force = call.force; a.nt = f->nt;
    a.mu = f->mu; a.lam = f->lam; a.kc = f->kc;
    for (int i = 0; i < 3; ++i) a.grav[i] = f->grav[i];
    a.eta_min = call.eta_min; a.eta_max = call.eta_max;
    a.rel_tol = call.rel_tol; a.abs_tol = call.abs_tol; a.c1 = call.c1; a.shrink = call.shrink;
    a.max_iter = call.max_iter; a.ls_max = call.ls_max; a.cg_max = call.cg_max;
    const dim3 eg((unsigned)a.neb, (unsigned)(Bp / 64)), vg((unsigned)a.nvb, (unsigned)(Bp / 64));
    const dim3 ib((unsigned)((Bp + 63) / 64));
    hipError_t e = hipSuccess;
#define FS_CHECK()                                                     \
    do {                                                               \
        e = hipGetLastError();                                         \
        if (e != hipSuccess) {                                         \
            *why = hipGetErrorString(e);                               \
            return RS_ERR_HIP;                                         \
        }                                                              \
    } while (0)
    auto read_counts = [&]() -> bool {
        if (hipMemcpyAsync(f->hcnt, a.cnt, 4 * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess) return false;
        return hipStreamSynchronize(s) == hipSuccess;
    };
    RS_LAUNCH(k_fs_transpose, dim3((unsigned)((f->n + 31) / 32), (unsigned)((Bp + 31) / 32)), dim3(256), 0, s, call.u,
              a.U, f->n, B, Bp, 1);
    RS_LAUNCH(k_fs_init, ib, dim3(64), 0, s, a);
    FS_CHECK();
    for (int it = 0;; ++it) {
        RS_LAUNCH(k_fs_zero_int, dim3(1), dim3(64), 0, s, a.cnt, 4);
        RS_LAUNCH(k_fs_zero_int, dim3(1), dim3(64), 0, s, a.nlist, 1);
        RS_LAUNCH(k_fs_elem<1>, eg, dim3(256), 0, s, a);
        RS_LAUNCH(k_fs_psd, dim3(2048), dim3(kPsdT), 0, s, a);
        RS_LAUNCH(k_fs_gather<0>, vg, dim3(256), 0, s, a);
        RS_LAUNCH(k_fs_check, ib, dim3(64), 0, s, a, it);
        FS_CHECK();
        if (!read_counts()) {
            *why = "stream synchronisation failed";
            return RS_ERR_HIP;
        }
        if (f->hcnt[0] == 0) break;
        // CG on H dx = -g
        RS_LAUNCH(k_fs_cg_init, vg, dim3(256), 0, s, a);
        RS_LAUNCH(k_fs_cg_start, ib, dim3(64), 0, s, a);
        FS_CHECK();
        for (int k = 0; k < a.cg_max; ++k) {
            const int last = k + 1 == a.cg_max;
            RS_LAUNCH(k_fs_zero_int, dim3(1), dim3(64), 0, s, a.cnt + 1, 1);
            RS_LAUNCH(k_fs_mv_elem, eg, dim3(256), 0, s, a);
            RS_LAUNCH(k_fs_gather<1>, vg, dim3(256), 0, s, a);
            RS_LAUNCH(k_fs_cg_alpha, ib, dim3(64), 0, s, a);
            RS_LAUNCH(k_fs_cg_update, vg, dim3(256), 0, s, a);
            RS_LAUNCH(k_fs_cg_beta, ib, dim3(64), 0, s, a, last);
            RS_LAUNCH(k_fs_cg_p, vg, dim3(256), 0, s, a);
            FS_CHECK();
            if (last) break;
            if ((k & 7) == 7) {
                if (!read_counts()) {
                    *why = "stream synchronisation failed";
                    return RS_ERR_HIP;
                }
                if (f->hcnt[1] == 0) break;
            }
        }
        // line search
        RS_LAUNCH(k_fs_slope, vg, dim3(256), 0, s, a);
        RS_LAUNCH(k_fs_ls_start, ib, dim3(64), 0, s, a);
        FS_CHECK();
        for (int t = 0; t < a.ls_max; ++t) {
            RS_LAUNCH(k_fs_zero_int, dim3(1), dim3(64), 0, s, a.cnt + 2, 1);
            RS_LAUNCH(k_fs_elem<0>, eg, dim3(256), 0, s, a);
            RS_LAUNCH(k_fs_ext_energy, vg, dim3(256), 0, s, a);
            RS_LAUNCH(k_fs_armijo, ib, dim3(64), 0, s, a);
            FS_CHECK();
            if (!read_counts()) {
                *why = "stream synchronisation failed";
                return RS_ERR_HIP;
            }
            if (f->hcnt[2] == 0) break;
        }
        RS_LAUNCH(k_fs_step, vg, dim3(256), 0, s, a);
        FS_CHECK();
    }
    RS_LAUNCH(k_fs_transpose, dim3((unsigned)((f->n + 31) / 32), (unsigned)((Bp + 31) / 32)), dim3(256), 0, s, a.U,
              call.u, f->n, B, Bp, 0);
    RS_LAUNCH(k_fs_outputs, dim3((unsigned)((B + 63) / 64)), dim3(64), 0, s, a, call.iters, call.status, call.relgrad,
              call.E);
    FS_CHECK();
#undef FS_CHECK
    return RS_OK;
}

}  // namespace rs
