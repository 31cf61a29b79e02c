// Kernels of the learned part: the decoder-parameter gradient of the
// Lipschitz loss (Sec. 4.1, Eq. form-L-LS-E, on the cubature elastic Hessian of
// Sec. 4.3), the device-side load of decoder weights (the output-layer fold
// onto the reduced rows), and the supervised training of encoder and decoder
// (Sec. 3.2, Eq. form-vanilla-supervised-construction; Sec. 4.2, Eq.
// form-unconstrained-lipschitz-optimization).
//
// Lipschitz-loss gradient.  For a symmetric r x r matrix C the contraction
// s = <C, H(z)> = sum_kq C_kq d2 P~/dz_k dz_q is carried forward through the
// decoder as three kinds of columns per latent point: the value h, the
// Jacobian columns J = dh/dz and the contracted second derivative
// S = sum_kq C_kq d2 h/dz_k dz_q.  A hidden layer maps pre-activations
// (a, A = W J, a_S = W S) to h = elu(a), J = elu'(a) A and
// S = elu''(a) (A C A^T)_uu + elu'(a) a_S.  Through the folded output map the
// element rows give F - I, K = dvecF/dz and Fdd (the contracted second
// derivative of vec F); per element s = w V [tr(C K^T A(F) K) + P(F) : Fdd].
// The backward pass takes the adjoints of the three kinds of columns back to
// the first layer; the derivative of A(F) enters through
//   d/dF tr(C K^T A(F) K) = 2 lam cofd(F, m1) + lam (sum_k M_k . cofd(F, K_k)) g
//                           + (lam (J - 1) - mu) sum_k cofd(M_k, K_k),
// with g = vec cof F, M = K C, m1 = M K^T g and cofd(X, Y) the symmetric
// bilinear form with cofd(X, X) = 2 cof X (the second derivative of det).
#include "rs_device.hpp"

#include <mutex>

namespace rs {

// ---------------------------------------------------------------------------
// Strided GEMM on the matrix cores: C(m, n) (+)= alpha sum_k A(m, k) B(k, n)
// (+ bias[m] on columns n with n % bias_every == 0), A(m, k) = A[m sAm + k sAk],
// B(k, n) = B[k sBk + n sBn], C row-major with leading dimension ldc, in T or
// float64.  64 x 64 tiles, four waves of 16 rows, 16-deep chunks through LDS.
// ---------------------------------------------------------------------------
template <typename T, typename TC>
__global__ __launch_bounds__(256) void k_gemm_s(SgemmArgs g)
{
    constexpr int TM = 64, TN = 64, TK = 16;
    __shared__ T As[TM][TK + 1];
    __shared__ T Bs[TK][TN + 1];
    const T* A = static_cast<const T*>(g.A);
    const T* B = static_cast<const T*>(g.B);
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // K slice of this workgroup (the whole K without a split); slices are multiples of TK
    int kbeg = 0, kend = g.K;
    if (g.ksplit > 1) {
        const int kc = ((g.K + g.ksplit - 1) / g.ksplit + TK - 1) / TK * TK;
        kbeg = blockIdx.z * kc;
        kend = min(g.K, kbeg + kc);
    }
    typename Mfma<T>::acc_t acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = typename Mfma<T>::acc_t{0, 0, 0, 0};
    for (int k0 = kbeg; k0 < kend; k0 += TK) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = tid + 256 * e;           // 1024 = 64 x 16 values of each tile
            const int am = idx / TK, ak = idx % TK;  // A: row-major walk
            const int gm = m0 + am, gk = k0 + ak;
            As[am][ak] = (gm < g.M && gk < kend) ? A[(long)gm * g.sAm + (long)gk * g.sAk] : T(0);
            const int bk = idx / TN, bn = idx % TN;  // B: consecutive threads, consecutive columns
            const int hk = k0 + bk, hn = n0 + bn;
            Bs[bk][bn] = (hk < kend && hn < g.N) ? B[(long)hk * g.sBk + (long)hn * g.sBn] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TK / 4; ++kk) {
            const T av = As[16 * wave + (lane & 15)][4 * kk + (lane >> 4)];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const T bv = Bs[4 * kk + (lane >> 4)][16 * t + (lane & 15)];
                acc[t] = Mfma<T>::mac(av, bv, acc[t]);
            }
        }
        __syncthreads();
    }
    TC* Cp = static_cast<TC*>(g.C);
    const T* bias = static_cast<const T*>(g.bias);
    if (g.ksplit > 1) {
        TC* part = static_cast<TC*>(g.part) + (size_t)blockIdx.z * g.M * g.N;
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int m = m0 + 16 * wave + Mfma<T>::row(lane, v), n = n0 + 16 * t + (lane & 15);
                if (m < g.M && n < g.N) part[(size_t)m * g.N + n] = (TC)acc[t][v];
            }
        return;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int m = m0 + 16 * wave + Mfma<T>::row(lane, v), n = n0 + 16 * t + (lane & 15);
            if (m >= g.M || n >= g.N) continue;
            double val = g.alpha * (double)acc[t][v];
            if (bias && g.bias_every > 0 && n % g.bias_every == 0) val += (double)bias[m];
            TC* dst = Cp + (long)m * g.ldc + n;
            *dst = g.accumulate ? (TC)((double)*dst + val) : (TC)val;
        }
}

// C = (accumulate ? C : 0) + alpha sum over the K slices (in slice order) + bias
template <typename TC, typename T>
__global__ void k_gemm_s_reduce(SgemmArgs g)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)g.M * g.N) return;
    const int m = (int)(i / g.N), n = (int)(i - (long)m * g.N);
    const TC* part = static_cast<const TC*>(g.part);
    double acc = 0.0;
    for (int z = 0; z < g.ksplit; ++z) acc += (double)part[(size_t)z * g.M * g.N + i];
    double val = g.alpha * acc;
    const T* bias = static_cast<const T*>(g.bias);
    if (bias && g.bias_every > 0 && n % g.bias_every == 0) val += (double)bias[m];
    TC* dst = static_cast<TC*>(g.C) + (long)m * g.ldc + n;
    *dst = g.accumulate ? (TC)((double)*dst + val) : (TC)val;
}

template <typename T, typename TC>
static hipError_t gemm_s_launch(const SgemmArgs& g, hipStream_t s)
{
    const dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, g.ksplit > 1 ? g.ksplit : 1);
    RS_LAUNCH((k_gemm_s<T, TC>), grid, dim3(256), 0, s, g);
    if (g.ksplit > 1)
        RS_LAUNCH((k_gemm_s_reduce<TC, T>), dim3((unsigned)(((long)g.M * g.N + 255) / 256)), dim3(256), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_gemm_s(int f32, int out_f64, const SgemmArgs& g, hipStream_t s)
{
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    if (g.ksplit > 1 && !g.part) return hipErrorInvalidValue;
    if (f32) return out_f64 ? gemm_s_launch<float, double>(g, s) : gemm_s_launch<float, float>(g, s);
    return gemm_s_launch<double, double>(g, s);
}

// ---------------------------------------------------------------------------
// Lipschitz-loss gradient: pairs, coefficients, jets, element seeds, adjoints
// ---------------------------------------------------------------------------
__global__ void k_lip_stack(const double* z1, const double* z2, double* zs, int B, int r)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * r) return;
    const int b = i / r, k = i - b * r;
    zs[(size_t)(2 * b) * r + k] = z1[i];
    zs[(size_t)(2 * b + 1) * r + k] = z2[i];
}

// One workgroup: n_valid, the loss mean_b |H1 - H2|_F^2 / |dz|^2 over this
// chunk's pairs (added to acc[0], count to acc[1]) and the signed
// coefficients Cs[2b] = 2 sym(H1 - H2) / (|dz|^2 n_total), Cs[2b+1] = -Cs[2b].
// n_total (all pairs of the call) is counted first by the caller's kernel.
__global__ __launch_bounds__(256) void k_lip_count(const double* z1, const double* z2, int B, int r, int* nvalid)
{
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    int local = 0;
    for (int b = threadIdx.x; b < B; b += blockDim.x) {
        double d2 = 0.0;
        for (int k = 0; k < r; ++k) {
            const double d = z1[(size_t)b * r + k] - z2[(size_t)b * r + k];
            d2 += d * d;
        }
        local += d2 > 0.0;
    }
    atomicAdd(&cnt, local);
    __syncthreads();
    if (threadIdx.x == 0) *nvalid = cnt;
}

__global__ __launch_bounds__(256) void k_lip_coef(const double* z1, const double* z2, const double* H, int B, int r,
                                                 const int* nvalid, double* Cs, double* ell)
{
    const int b = blockIdx.x;
    if (b >= B) return;
    const int rr = r * r;
    __shared__ double d2s;
    if (threadIdx.x == 0) {
        double d2 = 0.0;
        for (int k = 0; k < r; ++k) {
            const double d = z1[(size_t)b * r + k] - z2[(size_t)b * r + k];
            d2 += d * d;
        }
        d2s = d2;
    }
    __syncthreads();
    const double d2 = d2s;
    const double* H1 = H + (size_t)(2 * b) * rr;
    const double* H2 = H1 + rr;
    double* C1 = Cs + (size_t)(2 * b) * rr;
    double* C2 = C1 + rr;
    const int nv = *nvalid;
    for (int t = threadIdx.x; t < rr; t += blockDim.x) {
        const int k = t / r, q = t - k * r;
        double c = 0.0;
        if (d2 > 0.0)
            c = ((H1[t] - H2[t]) + (H1[q * r + k] - H2[q * r + k])) / (d2 * nv);
        C1[t] = c;
        C2[t] = -c;
    }
    if (threadIdx.x == 0) {
        double fro = 0.0;
        for (int t = 0; t < rr; ++t) fro += (H1[t] - H2[t]) * (H1[t] - H2[t]);
        ell[b] = d2 > 0.0 ? fro / d2 : 0.0;
    }
}

// loss = sum of the chunk's ell over all valid pairs / n_valid (one thread, pair order)
__global__ void k_lip_sum(const double* ell, int B, const int* nvalid, double* loss, int first)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = first ? 0.0 : *loss;
    const int nv = *nvalid;
    for (int b = 0; b < B; ++b) s += nv > 0 ? ell[b] / nv : 0.0;
    *loss = s;
}

// X_0 = [z | I | 0] (r x cols), column item * nc + c
template <typename T>
__global__ void k_jet_input(const double* zs, int items, int r, int nc, T* X, long ldx)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long cols = (long)items * nc;
    if (i >= (long)r * cols) return;
    const int k = (int)(i / cols);
    const long col = i - (long)k * cols;
    const int item = (int)(col / nc), c = (int)(col - (long)item * nc);
    T v = T(0);
    if (c == 0) v = (T)zs[(size_t)item * r + k];
    else if (c == k + 1) v = T(1);
    X[(long)k * ldx + col] = v;
}

// hidden-layer activation of the jets, one thread per (unit, item); RM >= r
template <typename T, int RM>
__global__ void k_jet_act(const T* Pre, long ldp, T* X, long ldx, int w, int items, int r, const double* Cs)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)w * items) return;
    const int u = (int)(i / items), item = (int)(i - (long)u * items);
    const int nc = r + 2;
    const T* p = Pre + (long)u * ldp + (long)item * nc;
    T* x = X + (long)u * ldx + (long)item * nc;
    const double* C = Cs + (size_t)item * r * r;
    const double a = (double)p[0], aS = (double)p[r + 1];
    double A[RM];
#pragma unroll
    for (int k = 0; k < RM; ++k) A[k] = k < r ? (double)p[1 + k] : 0.0;
    double q = 0.0;
#pragma unroll
    for (int k = 0; k < RM; ++k) {
        if (k >= r) break;
        double t = 0.0;
#pragma unroll
        for (int k2 = 0; k2 < RM; ++k2)
            if (k2 < r) t += C[k2 * r + k] * A[k2];
        q += t * A[k];
    }
    const double s1 = elu1(a), s2 = elu2(a);
    x[0] = (T)elu0(a);
#pragma unroll
    for (int k = 0; k < RM; ++k)
        if (k < r) x[1 + k] = (T)(s1 * A[k]);
    x[r + 1] = (T)(s2 * q + s1 * aS);
}

// adjoints of a hidden layer's pre-activations, one thread per (unit, item)
template <typename T, int RM>
__global__ void k_jet_back(const T* G, long ldg, const T* Pre, long ldp, T* D, long ldd, int w, int items, int r,
                           const double* Cs)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)w * items) return;
    const int u = (int)(i / items), item = (int)(i - (long)u * items);
    const int nc = r + 2;
    const T* gp = G + (long)u * ldg + (long)item * nc;
    const T* p = Pre + (long)u * ldp + (long)item * nc;
    T* d = D + (long)u * ldd + (long)item * nc;
    const double* C = Cs + (size_t)item * r * r;
    const double a = (double)p[0], aS = (double)p[r + 1];
    const double hb = (double)gp[0], Sb = (double)gp[r + 1];
    double A[RM], Jb[RM], AC[RM];
#pragma unroll
    for (int k = 0; k < RM; ++k) {
        A[k] = k < r ? (double)p[1 + k] : 0.0;
        Jb[k] = k < r ? (double)gp[1 + k] : 0.0;
    }
    double q = 0.0, AJ = 0.0;
#pragma unroll
    for (int k = 0; k < RM; ++k) {
        double t = 0.0;
#pragma unroll
        for (int k2 = 0; k2 < RM; ++k2)
            if (k < r && k2 < r) t += A[k2] * C[k2 * r + k];
        AC[k] = t;
        q += t * A[k];
        AJ += A[k] * Jb[k];
    }
    // ELU: the second and third derivatives coincide (e^a for a <= 0, zero above)
    const double s1 = elu1(a), s2 = elu2(a), s3 = s2;
    d[0] = (T)(s1 * hb + s2 * AJ + s3 * q * Sb + s2 * aS * Sb);
#pragma unroll
    for (int k = 0; k < RM; ++k)
        if (k < r) d[1 + k] = (T)(s1 * Jb[k] + 2.0 * s2 * Sb * AC[k]);
    d[r + 1] = (T)(s1 * Sb);
}

// cofd(X, Y) column j: x_{j+1} x y_{j+2} + y_{j+1} x x_{j+2} (vec column-major, 3 j + i)
__device__ inline void cofd(const double* X, const double* Y, double* out)
{
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const double* x1 = X + 3 * ((j + 1) % 3);
        const double* x2 = X + 3 * ((j + 2) % 3);
        const double* y1 = Y + 3 * ((j + 1) % 3);
        const double* y2 = Y + 3 * ((j + 2) % 3);
        out[3 * j + 0] = x1[1] * y2[2] - x1[2] * y2[1] + y1[1] * x2[2] - y1[2] * x2[1];
        out[3 * j + 1] = x1[2] * y2[0] - x1[0] * y2[2] + y1[2] * x2[0] - y1[0] * x2[2];
        out[3 * j + 2] = x1[0] * y2[1] - x1[1] * y2[0] + y1[0] * x2[1] - y1[1] * x2[0];
    }
}

// element seeds of s = <C, H> per (item, cubature tet): from the output rows
// (F - I, K, Fdd) to their adjoints (Fbar, Kbar, w V P), float64 inside.  Each
// thread stages its K (9 x r) in its own slice of LDS (kSeedThreads threads a
// workgroup) and walks the columns of M = K C one at a time.
constexpr int kSeedThreads = 64;
template <typename T>
__global__ __launch_bounds__(kSeedThreads) void k_jet_seed(const T* Out, long ldo, T* Seed, long lds, int items, int S,
                                                           int r, const double* wV, double mu, double lam,
                                                           const double* Cs)
{
    extern __shared__ double sK[]; // [v * r + k][thread]
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)items * S) return;
    const int s = (int)(i / items), item = (int)(i - (long)s * items);
    const int nc = r + 2, th = threadIdx.x;
    const double* C = Cs + (size_t)item * r * r;
    const long col = (long)item * nc;
    auto Kat = [&](int v, int k) -> double& { return sK[(size_t)(v * r + k) * kSeedThreads + th]; };
    double G[9], Fdd[9];
    for (int v = 0; v < 9; ++v) {
        const T* row = Out + (long)(9 * s + v) * ldo + col;
        G[v] = (double)row[0];
        Fdd[v] = (double)row[r + 1];
        for (int k = 0; k < r; ++k) Kat(v, k) = (double)row[1 + k];
    }
    Snh<double> sn;
    sn.set(G, mu, lam);
    double F[9], g[9];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) {
            F[3 * j + ii] = sn.f[j][ii];
            g[3 * j + ii] = sn.cof[j][ii];
        }
    const double w = wV[s];
    // T_C = 2 lam cofd(F, m1) + lam (sum_k M_k . cofd(F, K_k)) g + s_f sum_k cofd(M_k, K_k), m1 = sum_k M_k (K_k . g)
    double m1[9], sumB[9], tmp[9], Kk[9], Mk[9];
    double trm = 0.0;
#pragma unroll
    for (int v = 0; v < 9; ++v) m1[v] = sumB[v] = 0.0;
    for (int k = 0; k < r; ++k) {
        double ktg = 0.0;
#pragma unroll
        for (int v = 0; v < 9; ++v) {
            Kk[v] = Kat(v, k);
            ktg += Kk[v] * g[v];
            double t = 0.0;
            for (int k2 = 0; k2 < r; ++k2) t += Kat(v, k2) * C[k2 * r + k];
            Mk[v] = t;
        }
        cofd(F, Kk, tmp);
#pragma unroll
        for (int v = 0; v < 9; ++v) {
            trm += Mk[v] * tmp[v];
            m1[v] += Mk[v] * ktg;
        }
        cofd(Mk, Kk, tmp);
#pragma unroll
        for (int v = 0; v < 9; ++v) sumB[v] += tmp[v];
        // Kbar_k = 2 w V A(F) M_k
        sn.apply_hess(mu, lam, Mk, tmp);
#pragma unroll
        for (int v = 0; v < 9; ++v) Seed[(long)(9 * s + v) * lds + col + 1 + k] = (T)(2.0 * w * tmp[v]);
    }
    double Tc[9];
    cofd(F, m1, tmp);
#pragma unroll
    for (int v = 0; v < 9; ++v) Tc[v] = 2.0 * lam * tmp[v] + lam * trm * g[v] + sn.s * sumB[v];
    double AFdd[9], P[9];
    sn.apply_hess(mu, lam, Fdd, AFdd);
    sn.pk1(mu, lam, P);
#pragma unroll
    for (int v = 0; v < 9; ++v) {
        T* row = Seed + (long)(9 * s + v) * lds + col;
        row[0] = (T)(w * (Tc[v] + AFdd[v]));
        row[r + 1] = (T)(w * P[v]);
    }
}

// grad[u] += sum over items of D[u][item * nc] (bias gradients from the value columns)
template <typename T>
__global__ void k_value_rowsum(const T* D, long ldd, int rows, int items, int nc, double* grad)
{
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= rows) return;
    double s = 0.0;
    for (int item = 0; item < items; ++item) s += (double)D[(long)u * ldd + (long)item * nc];
    grad[u] += s;
}

hipError_t launch_lip_stack(const double* z1, const double* z2, double* zs, int B, int r, hipStream_t s)
{
    if (B <= 0) return hipSuccess;
    RS_LAUNCH(k_lip_stack, dim3((B * r + 255) / 256), dim3(256), 0, s, z1, z2, zs, B, r);
    return hipGetLastError();
}

hipError_t launch_lip_count(const double* z1, const double* z2, int B, int r, int* nvalid, hipStream_t s)
{
    RS_LAUNCH(k_lip_count, dim3(1), dim3(256), 0, s, z1, z2, B, r, nvalid);
    return hipGetLastError();
}

hipError_t launch_lip_coef(const double* z1, const double* z2, const double* H, int B, int r, const int* nvalid,
                           double* Cs, double* ell, double* loss, int first, hipStream_t s)
{
    if (B > 0) RS_LAUNCH(k_lip_coef, dim3(B), dim3(256), 0, s, z1, z2, H, B, r, nvalid, Cs, ell);
    RS_LAUNCH(k_lip_sum, dim3(1), dim3(64), 0, s, ell, B, nvalid, loss, first);
    return hipGetLastError();
}

template <typename T>
static hipError_t jet_dispatch(int kind, const JetArgs& j, hipStream_t s)
{
    const long n = kind == 0 ? (long)j.r * j.items * (j.r + 2) : kind == 3 ? (long)j.items * j.S : (long)j.w * j.items;
    if (n <= 0) return hipSuccess;
    const dim3 block(kind == 3 ? kSeedThreads : 256);
    const dim3 grid((unsigned)((n + block.x - 1) / block.x));
    const bool r16 = j.r <= 16;
    if (kind == 0) {
        RS_LAUNCH(k_jet_input<T>, grid, block, 0, s, j.zs, j.items, j.r, j.r + 2, (T*)j.X, j.ldx);
    } else if (kind == 1) {
        if (r16) RS_LAUNCH((k_jet_act<T, 16>), grid, block, 0, s, (const T*)j.Pre, j.ldp, (T*)j.X, j.ldx, j.w, j.items, j.r, j.Cs);
        else RS_LAUNCH((k_jet_act<T, kMaxR>), grid, block, 0, s, (const T*)j.Pre, j.ldp, (T*)j.X, j.ldx, j.w, j.items, j.r, j.Cs);
    } else if (kind == 2) {
        if (r16)
            RS_LAUNCH((k_jet_back<T, 16>), grid, block, 0, s, (const T*)j.G, j.ldg, (const T*)j.Pre, j.ldp, (T*)j.D, j.ldd,
                      j.w, j.items, j.r, j.Cs);
        else
            RS_LAUNCH((k_jet_back<T, kMaxR>), grid, block, 0, s, (const T*)j.G, j.ldg, (const T*)j.Pre, j.ldp, (T*)j.D,
                      j.ldd, j.w, j.items, j.r, j.Cs);
    } else {
        const size_t shm = sizeof(double) * 9 * (size_t)j.r * kSeedThreads;
        RS_LAUNCH(k_jet_seed<T>, grid, block, shm, s, (const T*)j.Pre, j.ldp, (T*)j.D, j.ldd, j.items, j.S, j.r, j.wV,
                  j.mu, j.lam, j.Cs);
    }
    return hipGetLastError();
}

// kind 0: first-layer input [z | I | 0]; 1: hidden activation; 2: hidden adjoints; 3: element seeds
hipError_t launch_jet(int f32, int kind, const JetArgs& j, hipStream_t s)
{
    if (j.r > kMaxR) return hipErrorInvalidValue;
    return f32 ? jet_dispatch<float>(kind, j, s) : jet_dispatch<double>(kind, j, s);
}

hipError_t launch_value_rowsum(int f32, const void* D, long ldd, int rows, int items, int nc, double* grad, hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    if (f32) RS_LAUNCH(k_value_rowsum<float>, dim3((rows + 255) / 256), dim3(256), 0, s, (const float*)D, ldd, rows, items, nc, grad);
    else RS_LAUNCH(k_value_rowsum<double>, dim3((rows + 255) / 256), dim3(256), 0, s, (const double*)D, ldd, rows, items, nc, grad);
    return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Static scratch of the allocation-free entry points.  Each device holds its own
// copy from module load to process end.  In host code `scratch` is a host-side
// stand-in for the symbol, never a device address: kernels and copies take the
// address hipGetSymbolAddress returns for the current device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_addr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch_address(void** ptr)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_addr[dev] = p;
    }
    *ptr = g_scratch_addr[dev];
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// Device-side decoder load: packed parameters (float32 or float64) into the
// context's padded layouts, and the output-layer fold onto the reduced rows.
// ---------------------------------------------------------------------------
// float64 -> bfloat16 with round to nearest even; a float32 midpoint is decided
// by the float64 value (the correctly rounded result)
__device__ inline uint16_t bf16_rne_dev(double x)
{
    const float f = (float)x;
    const uint32_t u = __float_as_uint(f);
    const uint32_t hi = u >> 16, lo = u & 0xFFFFu;
    if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)(hi | ((u & 0x7FFFFFu) ? 0x40u : 0u));
    bool up;
    if (lo > 0x8000u) up = true;
    else if (lo < 0x8000u) up = false;
    else {
        const double ax = fabs(x), af = fabs((double)f);
        up = ax > af ? true : ax < af ? false : (hi & 1u) != 0;
    }
    return (uint16_t)(up ? hi + 1 : hi);
}

// x as three BF16 parts hi = bf16(x), mid = bf16(x - hi), lo = bf16(x - hi - mid),
// written `plane` elements apart (the BF16 contexts' operand planes)
__device__ inline void bf16_planes_dev(double x, uint16_t* dst, size_t plane)
{
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const uint16_t h = bf16_rne_dev(x);
        dst[p * plane] = h;
        x -= (double)__uint_as_float((uint32_t)h << 16);
    }
}

template <typename TS>
__global__ void k_load_padded(const TS* src, int out, int in, int rows_pad, int ld, const uint8_t* rowmask, double* d64,
                              float* d32, uint16_t* d16)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)rows_pad * ld) return;
    const int m = (int)(i / ld), k = (int)(i - (long)m * ld);
    double v = 0.0;
    if (m < out && k < in && !(rowmask && rowmask[m])) v = (double)src[(long)m * in + k];
    if (d64) d64[i] = v;
    if (d32) d32[i] = (float)v;
    if (d16) bf16_planes_dev(v, d16 + i, (size_t)rows_pad * ld);
}

// W_big[m][k] = sum_j coef[j] W_out[src[j]][k] (+ the same for the bias, column in_last of a
// virtual [W | b]); rows past M and columns past in_last are zero
template <typename TS>
__global__ void k_fold_rows(const TS* Wout, const TS* bout, int in_last, const int* ptr, const int* src,
                            const double* coef, int M, int Mp, int ld, double* W64, float* W32, uint16_t* W16,
                            double* b64, float* b32)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)Mp * (ld + 1)) return;
    const int m = (int)(i / (ld + 1)), k = (int)(i - (long)m * (ld + 1));
    double v = 0.0;
    if (m < M && (k < in_last || k == ld)) {
        for (int j = ptr[m]; j < ptr[m + 1]; ++j)
            v += coef[j] * (k == ld ? (double)bout[src[j]] : (double)Wout[(long)src[j] * in_last + k]);
    }
    if (k == ld) {
        if (b64) b64[m] = v;
        if (b32) b32[m] = (float)v;
        return;
    }
    const long o = (long)m * ld + k;
    if (W64) W64[o] = v;
    if (W32) W32[o] = (float)v;
    if (W16) bf16_planes_dev(v, W16 + o, (size_t)Mp * ld);
}

// dst[k][m] = src[m][k] for the adjoint product's transposed W_big
template <typename T>
__global__ void k_transpose(const T* src, int rows, int cols, int ld_src, T* dst, int ld_dst, int dst_rows)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)dst_rows * ld_dst) return;
    const int k = (int)(i / ld_dst), m = (int)(i - (long)k * ld_dst);
    dst[i] = (k < cols && m < rows) ? src[(long)m * ld_src + k] : T(0);
}

template <typename TS>
__global__ void k_load_vec(const TS* src, int n, const uint8_t* rowmask, double* d64, float* d32, int n_pad)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pad) return;
    const double v = (i < n && !(rowmask && rowmask[i])) ? (double)src[i] : 0.0;
    if (d64) d64[i] = v;
    if (d32) d32[i] = (float)v;
}

static inline dim3 grid_for(long n) { return dim3((unsigned)((n + 255) / 256)); }

hipError_t launch_load_padded(int src_f64, const void* src, int out, int in, int rows_pad, int ld,
                              const uint8_t* rowmask, double* d64, float* d32, uint16_t* d16, hipStream_t s)
{
    const long n = (long)rows_pad * ld;
    if (n <= 0) return hipSuccess;
    if (src_f64) RS_LAUNCH(k_load_padded<double>, grid_for(n), dim3(256), 0, s, (const double*)src, out, in, rows_pad, ld, rowmask, d64, d32, d16);
    else RS_LAUNCH(k_load_padded<float>, grid_for(n), dim3(256), 0, s, (const float*)src, out, in, rows_pad, ld, rowmask, d64, d32, d16);
    return hipGetLastError();
}

hipError_t launch_fold_rows(int src_f64, const void* Wout, const void* bout, int in_last, const int* ptr, const int* src,
                            const double* coef, int M, int Mp, int ld, double* W64, float* W32, uint16_t* W16,
                            double* b64, float* b32, hipStream_t s)
{
    const long n = (long)Mp * (ld + 1);
    if (src_f64)
        RS_LAUNCH(k_fold_rows<double>, grid_for(n), dim3(256), 0, s, (const double*)Wout, (const double*)bout, in_last, ptr,
                  src, coef, M, Mp, ld, W64, W32, W16, b64, b32);
    else
        RS_LAUNCH(k_fold_rows<float>, grid_for(n), dim3(256), 0, s, (const float*)Wout, (const float*)bout, in_last, ptr,
                  src, coef, M, Mp, ld, W64, W32, W16, b64, b32);
    return hipGetLastError();
}

hipError_t launch_transpose(int f32, const void* src, int rows, int cols, int ld_src, void* dst, int ld_dst,
                            int dst_rows, hipStream_t s)
{
    const long n = (long)dst_rows * ld_dst;
    if (f32) RS_LAUNCH(k_transpose<float>, grid_for(n), dim3(256), 0, s, (const float*)src, rows, cols, ld_src, (float*)dst, ld_dst, dst_rows);
    else RS_LAUNCH(k_transpose<double>, grid_for(n), dim3(256), 0, s, (const double*)src, rows, cols, ld_src, (double*)dst, ld_dst, dst_rows);
    return hipGetLastError();
}

hipError_t launch_load_vec(int src_f64, const void* src, int n, const uint8_t* rowmask, double* d64, float* d32,
                           int n_pad, hipStream_t s)
{
    if (n_pad <= 0) return hipSuccess;
    if (src_f64) RS_LAUNCH(k_load_vec<double>, grid_for(n_pad), dim3(256), 0, s, (const double*)src, n, rowmask, d64, d32, n_pad);
    else RS_LAUNCH(k_load_vec<float>, grid_for(n_pad), dim3(256), 0, s, (const float*)src, n, rowmask, d64, d32, n_pad);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Supervised training (Sec. 3.2, Eq. form-vanilla-supervised-construction):
// batch gather, ELU forward/backward on (units x batch) blocks, the
// mass-weighted reconstruction residual, bias sums, Adam.  T is the context
// precision (float or double); sums run in float64.
// ---------------------------------------------------------------------------
// Dt (n x B) = rows idx[b] (or b) of the (N x n) snapshot store, transposed through LDS
template <typename T>
__global__ __launch_bounds__(256) void k_gather_batch(const T* store, int n, const int* idx, int B, T* Dt)
{
    __shared__ T tile[32][33];
    const int r0 = blockIdx.x * 32, b0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int k = ty; k < 32; k += 8) {
        const int b = b0 + k, row = r0 + tx;
        T v = T(0);
        if (b < B && row < n) {
            const long item = idx ? idx[b] : b;
            v = store[item * n + row];
        }
        tile[k][tx] = v;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int row = r0 + k, b = b0 + tx;
        if (row < n && b < B) Dt[(long)row * B + b] = tile[tx][k];
    }
}

template <typename T>
__global__ void k_elu_fwd(const T* P, T* X, long n)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) X[i] = elu0(P[i]);
}

template <typename T>
__global__ void k_elu_bwd(const T* G, const T* P, T* D, long n)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) D[i] = G[i] * (T)elu1((double)P[i]);
}

// residual of the reconstruction in the mass norm, U and Dt (n x B): on free
// rows res = U - Dt, Ubar = 2 m res / B; pinned rows are not decoded (res = -Dt,
// no adjoint).  Per-block partial sums of m res^2 into part[blockIdx.x].
template <typename T>
__global__ __launch_bounds__(256) void k_recon_residual(const T* U, const T* Dt, int n, int B, const double* rowmass,
                                                       const uint8_t* pinned_row, T* Ubar, double* part)
{
    __shared__ double sh[256];
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (i < (long)n * B) {
        const int row = (int)(i / B);
        const bool fixed = pinned_row[row] != 0;
        const double res = (fixed ? 0.0 : (double)U[i]) - (double)Dt[i];
        const double m = rowmass[row];
        acc = m * res * res;
        Ubar[i] = fixed ? T(0) : (T)(2.0 * m * res / B);
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// out = scale * sum of the partials (one thread, fixed order)
__global__ void k_sum_parts(const double* part, int n, double scale, double* out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += part[i];
    *out = s * scale;
}

// grad[u] = sum_b D[u][b] (bias gradients of a (rows x B) adjoint block)
template <typename T>
__global__ void k_rowsum(const T* D, int rows, int B, T* grad)
{
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= rows) return;
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += (double)D[(long)u * B + b];
    grad[u] = (T)s;
}

// z (B x r, float64) from the (r x B) encoder output block
template <typename T>
__global__ void k_to_items(const T* X, int rows, int B, double* z)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * B) return;
    const int b = i / rows, k = i - b * rows;
    z[i] = (double)X[(long)k * B + b];
}

// z1 (P x r) and z2 (P x r): the batch's encodings taken as pairs (z_2p, z_2p+1)
__global__ void k_split_pairs(const double* z, int P, int r, double* z1, double* z2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P * r) return;
    const int p = i / r, k = i - p * r;
    z1[i] = z[(size_t)(2 * p) * r + k];
    z2[i] = z[(size_t)(2 * p + 1) * r + k];
}

// out = g1 + scale g2 in float64 (g2 may be NULL)
template <typename T>
__global__ void k_grad_out(long n, const T* g1, const double* g2, double scale, double* out)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = (double)g1[i] + (g2 ? scale * g2[i] : 0.0);
}

// Adam (Kingma and Ba) on g = g1 + g2_scale g2 (g2 may be NULL); c1, c2 the bias corrections
template <typename T>
__global__ void k_adam(long n, T* p, const T* g1, const double* g2, double g2_scale, T* m, T* v, double lr,
                       double b1, double b2, double eps, double c1, double c2)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double g = (double)g1[i];
    if (g2) g += g2_scale * g2[i];
    const double mi = b1 * (double)m[i] + (1.0 - b1) * g;
    const double vi = b2 * (double)v[i] + (1.0 - b2) * g * g;
    m[i] = (T)mi;
    v[i] = (T)vi;
    p[i] = (T)((double)p[i] - lr * (mi / c1) / (sqrt(vi / c2) + eps));
}

template <typename T>
static hipError_t train_dispatch(const TrainOp& o, hipStream_t s)
{
    switch (o.op) {
    case TRAIN_GATHER:
        if (o.B <= 0 || o.n <= 0) return hipSuccess;
        RS_LAUNCH(k_gather_batch<T>, dim3((o.n + 31) / 32, (o.B + 31) / 32), dim3(256), 0, s, (const T*)o.a, o.n,
                  o.idx, o.B, (T*)o.out);
        break;
    case TRAIN_ELU_FWD:
        if (o.count <= 0) return hipSuccess;
        RS_LAUNCH(k_elu_fwd<T>, grid_for(o.count), dim3(256), 0, s, (const T*)o.a, (T*)o.out, o.count);
        break;
    case TRAIN_ELU_BWD:
        if (o.count <= 0) return hipSuccess;
        RS_LAUNCH(k_elu_bwd<T>, grid_for(o.count), dim3(256), 0, s, (const T*)o.a, (const T*)o.b, (T*)o.out, o.count);
        break;
    case TRAIN_RESIDUAL: {
        const long tot = (long)o.n * o.B;
        const int nb = (int)((tot + 255) / 256);
        RS_LAUNCH(k_recon_residual<T>, dim3(nb), dim3(256), 0, s, (const T*)o.a, (const T*)o.b, o.n, o.B, o.rowmass,
                  o.pinned_row, (T*)o.out, o.part);
        RS_LAUNCH(k_sum_parts, dim3(1), dim3(64), 0, s, o.part, nb, 1.0 / o.B, o.loss);
        break;
    }
    case TRAIN_ROWSUM:
        if (o.n <= 0) return hipSuccess;
        RS_LAUNCH(k_rowsum<T>, grid_for(o.n), dim3(256), 0, s, (const T*)o.a, o.n, o.B, (T*)o.out);
        break;
    case TRAIN_TO_ITEMS:
        if (o.n * o.B <= 0) return hipSuccess;
        RS_LAUNCH(k_to_items<T>, grid_for((long)o.n * o.B), dim3(256), 0, s, (const T*)o.a, o.n, o.B, o.z);
        break;
    case TRAIN_GRAD_OUT:
        if (o.count <= 0) return hipSuccess;
        RS_LAUNCH(k_grad_out<T>, grid_for(o.count), dim3(256), 0, s, o.count, (const T*)o.a, o.g2, o.scale, o.z);
        break;
    case TRAIN_ADAM: {
        if (o.count <= 0) return hipSuccess;
        const double c1 = 1.0 - pow(o.b1, (double)o.step), c2 = 1.0 - pow(o.b2, (double)o.step);
        RS_LAUNCH(k_adam<T>, grid_for(o.count), dim3(256), 0, s, o.count, (T*)o.out, (const T*)o.a, o.g2, o.scale,
                  (T*)o.m, (T*)o.v, o.lr, o.b1, o.b2, o.eps, c1, c2);
        break;
    }
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_train(int f32, const TrainOp& o, hipStream_t s)
{
    return f32 ? train_dispatch<float>(o, s) : train_dispatch<double>(o, s);
}

// ---------------------------------------------------------------------------
// PCA of snapshot displacements (the linear subspace baseline): column means,
// centring, mass scaling and the small k x k steps of a subspace iteration in
// the mass inner product, float64.
// ---------------------------------------------------------------------------
// mean[d] = (1/N) sum_i D[i][d]; Dc64 (N x n) = D - mean, float64
template <typename T>
__global__ void k_pca_center(const T* D, int N, int n, double* mean, double* Dc)
{
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= n) return;
    double s = 0.0;
    for (int i = 0; i < N; ++i) s += (double)D[(size_t)i * n + d];
    const double m = s / N;
    mean[d] = m;
    for (int i = 0; i < N; ++i) Dc[(size_t)i * n + d] = (double)D[(size_t)i * n + d] - m;
}

// deterministic start block in [-1, 1) from an integer hash of the index
__global__ void k_pca_start(double* X, long count)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    unsigned long long h = (unsigned long long)i * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
    h ^= h >> 33;
    h *= 0xFF51AFD7ED558CCDull;
    h ^= h >> 33;
    h *= 0xC4CEB9FE1A85EC53ull;
    h ^= h >> 33;
    X[i] = (double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// MX (n x k) = m_row (.) X
__global__ void k_pca_mass(const double* X, const double* rowmass, int n, int k, double* MX)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)n * k) return;
    MX[i] = rowmass[i / k] * X[i];
}

// One thread: the Cholesky factor L of the k x k Gram matrix G (row-major) and
// R = L^-T (upper triangular) into R, so that X R has orthonormal columns.
__global__ void k_pca_orth(const double* G, int k, double* R, int* fail)
{
    __shared__ double L[64 * 64];
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int i = 0; i < k * k; ++i) L[i] = 0.0;
    int bad = 0;
    for (int j = 0; j < k; ++j) {
        double d = G[j * k + j];
        for (int m = 0; m < j; ++m) d -= L[j * k + m] * L[j * k + m];
        if (!(d > 0.0)) {
            bad = 1;
            d = 1e-300;
        }
        const double ljj = sqrt(d);
        L[j * k + j] = ljj;
        for (int i = j + 1; i < k; ++i) {
            double t = G[i * k + j];
            for (int m = 0; m < j; ++m) t -= L[i * k + m] * L[j * k + m];
            L[i * k + j] = t / ljj;
        }
    }
    // R = L^-T: solve L^T R = I column by column (back substitution)
    for (int c = 0; c < k; ++c)
        for (int i = k - 1; i >= 0; --i) {
            double t = i == c ? 1.0 : 0.0;
            for (int m = i + 1; m < k; ++m) t -= L[m * k + i] * R[m * k + c];
            R[i * k + c] = t / L[i * k + i];
        }
    *fail = bad;
}

// One thread: eigenvectors of the symmetric k x k matrix T (cyclic Jacobi),
// the r of largest eigenvalue as the columns of V (k x r, row-major), in
// decreasing order; eigenvalues into ev (r)
__global__ void k_pca_ritz(const double* T, int k, int r, double* V, double* ev)
{
    __shared__ double A[64 * 64];
    __shared__ double Q[64 * 64];
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
            A[i * k + j] = 0.5 * (T[i * k + j] + T[j * k + i]);
            Q[i * k + j] = i == j ? 1.0 : 0.0;
        }
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < k * k; ++i) tot += A[i] * A[i];
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j)
                if (i != j) off += A[i * k + j] * A[i * k + j];
        if (off <= 1e-30 * tot) break;
        for (int p = 0; p < k - 1; ++p)
            for (int q = p + 1; q < k; ++q) {
                const double apq = A[p * k + q];
                if (apq == 0.0) continue;
                const double th = (A[q * k + q] - A[p * k + p]) / (2.0 * apq);
                const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int m = 0; m < k; ++m) {
                    const double mp = A[m * k + p], mq = A[m * k + q];
                    A[m * k + p] = c * mp - s * mq;
                    A[m * k + q] = s * mp + c * mq;
                }
                for (int m = 0; m < k; ++m) {
                    const double mp = A[p * k + m], mq = A[q * k + m];
                    A[p * k + m] = c * mp - s * mq;
                    A[q * k + m] = s * mp + c * mq;
                }
                for (int m = 0; m < k; ++m) {
                    const double mp = Q[m * k + p], mq = Q[m * k + q];
                    Q[m * k + p] = c * mp - s * mq;
                    Q[m * k + q] = s * mp + c * mq;
                }
            }
    }
    int used[64];
    for (int i = 0; i < k; ++i) used[i] = 0;
    for (int c = 0; c < r; ++c) {
        int best = -1;
        for (int i = 0; i < k; ++i)
            if (!used[i] && (best < 0 || A[i * k + i] > A[best * k + best])) best = i;
        used[best] = 1;
        ev[c] = A[best * k + best];
        for (int i = 0; i < k; ++i) V[i * r + c] = Q[i * k + best];
    }
}

hipError_t launch_pca_center(int f32, const void* D, int N, int n, double* mean, double* Dc, hipStream_t s)
{
    if (f32) RS_LAUNCH(k_pca_center<float>, grid_for(n), dim3(256), 0, s, (const float*)D, N, n, mean, Dc);
    else RS_LAUNCH(k_pca_center<double>, grid_for(n), dim3(256), 0, s, (const double*)D, N, n, mean, Dc);
    return hipGetLastError();
}

hipError_t launch_pca_start(double* X, long count, hipStream_t s)
{
    RS_LAUNCH(k_pca_start, grid_for(count), dim3(256), 0, s, X, count);
    return hipGetLastError();
}

hipError_t launch_pca_mass(const double* X, const double* rowmass, int n, int k, double* MX, hipStream_t s)
{
    RS_LAUNCH(k_pca_mass, grid_for((long)n * k), dim3(256), 0, s, X, rowmass, n, k, MX);
    return hipGetLastError();
}

hipError_t launch_pca_orth(const double* G, int k, double* R, int* fail, hipStream_t s)
{
    if (k > 64) return hipErrorInvalidValue;
    RS_LAUNCH(k_pca_orth, dim3(1), dim3(64), 0, s, G, k, R, fail);
    return hipGetLastError();
}

hipError_t launch_pca_ritz(const double* T, int k, int r, double* V, double* ev, hipStream_t s)
{
    if (k > 64 || r > k) return hipErrorInvalidValue;
    RS_LAUNCH(k_pca_ritz, dim3(1), dim3(64), 0, s, T, k, r, V, ev);
    return hipGetLastError();
}

hipError_t launch_split_pairs(const double* z, int P, int r, double* z1, double* z2, hipStream_t s)
{
    if (P * r <= 0) return hipSuccess;
    RS_LAUNCH(k_split_pairs, grid_for((long)P * r), dim3(256), 0, s, z, P, r, z1, z2);
    return hipGetLastError();
}

}  // namespace rs
