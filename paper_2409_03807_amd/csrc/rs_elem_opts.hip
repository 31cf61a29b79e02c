// Optional element treatments of the reduced Hessian: the per-element
// positive-semi-definite projection of the Gauss-Newton term, and a dump of
// the 12x12 element Hessians for inspection.
//
// Per-element projection (supplement, projective Newton): the element
// Hessian H_e = V D^T A D (D the 9x12 map from corner positions to vec F,
// A = d2 psi / dF2) is replaced by its projection with negative eigenvalues set
// to zero.  D has rank 9 and D D^T = N (x) I_3 with N = sum_a Dv_a Dv_a^T the
// 3x3 Gram matrix of the shape gradients.  With B = (D D^T)^(1/2) and the
// thin SVD D = U S W^T one has H_e = W (S U^T V A U S) W^T, so the nonzero
// spectrum of H_e is that of M = V B A B (the same matrix in the basis U), and
//   J_e^T proj(H_e) J_e = K^T B^-1 proj(M) B^-1 K,     K = D J_e = dvecF/dz.
// The 12x12 projection therefore needs only the 9x9 matrix M per element and
// the rows the reduced output map already provides (F - I and K).  The element
// kernel has added K^T A K = (B^-1 K)^T M (B^-1 K); this kernel adds the
// difference, sum over the negative eigenpairs (lam_k, v_k) of M of
// |lam_k| (K^T B^-1 v_k)(K^T B^-1 v_k)^T, in float64 and a fixed order.
#include "rs_device.hpp"

namespace rs {

namespace {

constexpr int kPsdLanes = 64;           // elements decomposed per pass (one wave)
constexpr int kPsdEntries = 9 * kPsdLanes;

// d2 psi / dF2 as a dense 9x9 matrix (vec F column-major: index 3 j + i is F_ij)
__device__ void snh_tangent(const double* G, double mu, double lam, double* A, int ld)
{
    Snh<double> sn;
    sn.set(G, mu, lam);
    for (int q = 0; q < 9; ++q) {
        double e[9], col[9];
#pragma unroll
        for (int m = 0; m < 9; ++m) e[m] = m == q ? 1.0 : 0.0;
        sn.apply_hess(mu, lam, e, col);
#pragma unroll
        for (int m = 0; m < 9; ++m) A[(m * 9 + q) * ld] = col[m];
    }
}

}  // namespace

template <typename T>
__global__ __launch_bounds__(256) void k_elem_psd(ElemOptArgs a)
{
    // thread-private 9x9 matrices of the decomposing wave, entry-major so
    // that consecutive lanes use consecutive banks
    __shared__ double sM[81 * kPsdLanes];
    __shared__ double sV[81 * kPsdLanes];
    __shared__ double sVec[9 * kPsdEntries];
    __shared__ int sEl[kPsdEntries];
    __shared__ int sN;
    const int item = blockIdx.x;
    if (a.count && item >= *a.count) return;
    const int tid = threadIdx.x, r = a.r, nc = a.nc;
    const T* O = static_cast<const T*>(a.out) + (size_t)item * a.rows_pad * nc;
    const int rr = r * r;
    double acc[4] = {0.0, 0.0, 0.0, 0.0}; // H entries tid, tid + 256, ... (r <= 32)
    for (int base = 0; base < a.S; base += kPsdLanes) {
        if (tid < kPsdLanes) {
            const int lane = tid, s = base + lane;
            double* M = sM + lane;
            double* V = sV + lane;
            int nneg = 0;
            double lamk[9];
            if (s < a.S) {
                const double* ec = a.ec + (size_t)s * kElemConst;
                double G[9];
#pragma unroll
                for (int m = 0; m < 9; ++m) G[m] = (double)O[(size_t)(9 * s + m) * nc];
                // V (tangent) into the M slots, then M = wV (Bh (x) I) A (Bh (x) I) through V as scratch
                snh_tangent(G, a.mu, a.lam, V, kPsdLanes);
                const double* Bh = ec;
                const double wv = ec[31] * ec[30];
                for (int p = 0; p < 9; ++p)
                    for (int j = 0; j < 3; ++j)
                        for (int i = 0; i < 3; ++i) {
                            double t = 0.0;
                            for (int jj = 0; jj < 3; ++jj) t += V[(p * 9 + 3 * jj + i) * kPsdLanes] * Bh[3 * jj + j];
                            M[(p * 9 + 3 * j + i) * kPsdLanes] = t;
                        }
                for (int q = 0; q < 9; ++q)
                    for (int j = 0; j < 3; ++j)
                        for (int i = 0; i < 3; ++i) {
                            double t = 0.0;
                            for (int jj = 0; jj < 3; ++jj) t += Bh[3 * j + jj] * M[((3 * jj + i) * 9 + q) * kPsdLanes];
                            V[((3 * j + i) * 9 + q) * kPsdLanes] = wv * t;
                        }
                for (int m = 0; m < 81; ++m) {
                    M[m * kPsdLanes] = V[m * kPsdLanes];
                    V[m * kPsdLanes] = (m / 9 == m % 9) ? 1.0 : 0.0;
                }
                // cyclic Jacobi rotations (symmetric M; V accumulates the eigenvectors)
                for (int sweep = 0; sweep < 50; ++sweep) {
                    double off = 0.0, tot = 0.0;
                    for (int p = 0; p < 9; ++p)
                        for (int q = 0; q < 9; ++q) {
                            const double x = M[(p * 9 + q) * kPsdLanes];
                            tot += x * x;
                            if (p != q) off += x * x;
                        }
                    if (off <= 1e-28 * tot || off == 0.0) break;
                    for (int p = 0; p < 8; ++p)
                        for (int q = p + 1; q < 9; ++q) {
                            const double apq = M[(p * 9 + q) * kPsdLanes];
                            if (apq == 0.0) continue;
                            const double th = (M[(q * 9 + q) * kPsdLanes] - M[(p * 9 + p) * kPsdLanes]) / (2.0 * apq);
                            const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                            const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
                            for (int k = 0; k < 9; ++k) {
                                const double mkp = M[(k * 9 + p) * kPsdLanes], mkq = M[(k * 9 + q) * kPsdLanes];
                                M[(k * 9 + p) * kPsdLanes] = c * mkp - sn * mkq;
                                M[(k * 9 + q) * kPsdLanes] = sn * mkp + c * mkq;
                            }
                            for (int k = 0; k < 9; ++k) {
                                const double mpk = M[(p * 9 + k) * kPsdLanes], mqk = M[(q * 9 + k) * kPsdLanes];
                                M[(p * 9 + k) * kPsdLanes] = c * mpk - sn * mqk;
                                M[(q * 9 + k) * kPsdLanes] = sn * mpk + c * mqk;
                            }
                            for (int k = 0; k < 9; ++k) {
                                const double vkp = V[(k * 9 + p) * kPsdLanes], vkq = V[(k * 9 + q) * kPsdLanes];
                                V[(k * 9 + p) * kPsdLanes] = c * vkp - sn * vkq;
                                V[(k * 9 + q) * kPsdLanes] = sn * vkp + c * vkq;
                            }
                        }
                }
                for (int k = 0; k < 9; ++k) {
                    lamk[k] = M[(k * 9 + k) * kPsdLanes];
                    nneg += lamk[k] < 0.0;
                }
            }
            // entries in element order, then eigenvalue order (wave prefix sum)
            int incl = nneg;
            for (int d = 1; d < 64; d <<= 1) {
                const int o = __shfl_up(incl, d, 64);
                if (lane >= d) incl += o;
            }
            const int total = __shfl(incl, 63, 64);
            int slot = incl - nneg;
            if (s < a.S && nneg) {
                const double* Bi = a.ec + (size_t)s * kElemConst + 9;
                for (int k = 0; k < 9; ++k) {
                    if (!(lamk[k] < 0.0)) continue;
                    const double sc = sqrt(-lamk[k]);
                    for (int j = 0; j < 3; ++j)
                        for (int i = 0; i < 3; ++i) {
                            double t = 0.0;
                            for (int jj = 0; jj < 3; ++jj) t += Bi[3 * j + jj] * V[((3 * jj + i) * 9 + k) * kPsdLanes];
                            sVec[slot * 9 + 3 * j + i] = sc * t;
                        }
                    sEl[slot] = s;
                    ++slot;
                }
            }
            if (lane == 0) sN = total;
        }
        __syncthreads();
        const int n = sN;
        for (int e = 0; e < n; ++e) {
            const int s = sEl[e];
            const T* Ks = O + (size_t)(9 * s) * nc + 1;
            double v[9];
#pragma unroll
            for (int m = 0; m < 9; ++m) v[m] = sVec[e * 9 + m];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = tid + 256 * u;
                if (t >= rr) break;
                const int k = t / r, q = t - k * r;
                double yk = 0.0, yq = 0.0;
#pragma unroll
                for (int m = 0; m < 9; ++m) {
                    yk += (double)Ks[(size_t)m * nc + k] * v[m];
                    yq += (double)Ks[(size_t)m * nc + q] * v[m];
                }
                acc[u] += yk * yq;
            }
        }
        __syncthreads();
    }
    double* H = a.H + (size_t)item * rr;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int t = tid + 256 * u;
        if (t < rr) H[t] += acc[u];
    }
}

// H_e = V D^T A D (12x12, corner-major rows 3 a + i) of every cubature tet of
// the first `items` items, one thread per (item, tet).
template <typename T>
__global__ __launch_bounds__(256) void k_elem_hess_dump(ElemOptArgs a, int items)
{
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (size_t)items * a.S) return;
    const int item = (int)(gid / a.S), s = (int)(gid - (size_t)item * a.S);
    const T* O = static_cast<const T*>(a.out) + (size_t)item * a.rows_pad * a.nc;
    const double* ec = a.ec + (size_t)s * kElemConst;
    double G[9], A[81];
    for (int m = 0; m < 9; ++m) G[m] = (double)O[(size_t)(9 * s + m) * a.nc];
    snh_tangent(G, a.mu, a.lam, A, 1);
    const double* Dv = ec + 18; // Dv[c][j] at 3 c + j
    const double vol = ec[30];
    double* He = a.He + gid * 144;
    for (int c = 0; c < 4; ++c)
        for (int i = 0; i < 3; ++i)
            for (int d = 0; d < 4; ++d)
                for (int i2 = 0; i2 < 3; ++i2) {
                    double t = 0.0;
                    for (int j = 0; j < 3; ++j)
                        for (int j2 = 0; j2 < 3; ++j2) t += Dv[3 * c + j] * A[(3 * j + i) * 9 + 3 * j2 + i2] * Dv[3 * d + j2];
                    He[(3 * c + i) * 12 + 3 * d + i2] = vol * t;
                }
}

hipError_t launch_elem_psd(int f32, const ElemOptArgs& a, int items, hipStream_t s)
{
    if (items <= 0) return hipSuccess;
    if (a.r > 32) return hipErrorInvalidValue;
    if (f32) RS_LAUNCH(k_elem_psd<float>, dim3(items), dim3(256), 0, s, a);
    else RS_LAUNCH(k_elem_psd<double>, dim3(items), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_elem_hess_dump(int f32, const ElemOptArgs& a, int items, hipStream_t s)
{
    if (items <= 0) return hipSuccess;
    const size_t n = (size_t)items * a.S;
    const unsigned grid = (unsigned)((n + 255) / 256);
    if (f32) RS_LAUNCH(k_elem_hess_dump<float>, dim3(grid), dim3(256), 0, s, a, items);
    else RS_LAUNCH(k_elem_hess_dump<double>, dim3(grid), dim3(256), 0, s, a, items);
    return hipGetLastError();
}

}  // namespace rs
