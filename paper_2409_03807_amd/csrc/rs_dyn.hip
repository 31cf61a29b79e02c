// Implicit-Euler dynamics with ground contact in the reduced solve (Sec. 3.1,
// Eq. form-reduced-space-time-integration): the inertia term
//   1/(2 dt^2) |f(z) - qbar|_M^2
// and a one-sided penalty k_g/2 min(0, y_v - y_g)^2 on contact vertices (contact
// treated as part of the potential, as the paper's penalty collisions).
//
// The inertia term needs every decoded row, but the output layer is linear:
// with u(z) = W h(z) + b on the free rows, h the last hidden activation, and the
// target written as qbar - b = W eta + rho,
//   |u - qbar|_M^2 = d^T G d - 2 d^T c + kappa,   d = h - eta,
//   G = W^T M W (per decoder),  c = W^T M rho,  kappa = |rho|_M^2 (per item),
// so an evaluation costs one w x w product per item instead of a decode of all
// 3 nv rows.  A simulation keeps eta = 2 h^k - h^(k-1) (rho = 0): the terms stay
// of the size of the step and the float64 energy differences of the line search
// do not cancel; a general target has eta = 0 and rho = qbar - b.  The gradient
// is J_h^T (G d - c) / dt^2, the Gauss-Newton Hessian J_h^T G J_h / dt^2, and the
// exact Hessian adds (G d - c) / dt^2 to the adjoint of h before the curvature
// pass.  Contact rows are rows of the folded output
// map (the y row of each contact vertex): value and Jacobian columns give the
// penalty's energy, gradient and Gauss-Newton Hessian, and its adjoint seed.
#include "rs_device.hpp"

namespace rs {

namespace {

// G[i][j] = sum over rows of m_row W[row][i] W[row][j] (rows of pinned vertices are zero in W)
template <typename T>
__global__ void k_dyn_gram(const T* W, int ld, int rows, const double* rowmass, int m, double* G)
{
    const int i = blockIdx.y, j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m || j < i) return;
    double s = 0.0;
    for (int row = 0; row < rows; ++row) s += rowmass[row] * (double)W[(size_t)row * ld + i] * (double)W[(size_t)row * ld + j];
    G[(size_t)i * m + j] = s;
    G[(size_t)j * m + i] = s;
}

// per item b: c[b] = W^T M (qbar_b - bias) and kappa[b] = |qbar_b - bias|_M^2 over free rows
template <typename T>
__global__ __launch_bounds__(256) void k_dyn_prep(const T* W, int ld, const T* bias, const uint8_t* pinned_row,
                                                 const double* rowmass, int rows, int m, const double* qbar,
                                                 double* cvec, double* kappa)
{
    __shared__ double red[256];
    const int b = blockIdx.x, tid = threadIdx.x;
    const double* q = qbar + (size_t)b * rows;
    for (int j = tid; j < m; j += 256) {
        double s = 0.0;
        for (int row = 0; row < rows; ++row) {
            if (pinned_row[row]) continue;
            s += rowmass[row] * (q[row] - (bias ? (double)bias[row] : 0.0)) * (double)W[(size_t)row * ld + j];
        }
        cvec[(size_t)b * m + j] = s;
    }
    double k = 0.0;
    for (int row = tid; row < rows; row += 256) {
        if (pinned_row[row]) continue;
        const double d = q[row] - (bias ? (double)bias[row] : 0.0);
        k += rowmass[row] * d * d;
    }
    red[tid] = k;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) red[tid] += red[tid + o];
        __syncthreads();
    }
    if (tid == 0) kappa[b] = red[0];
}

__device__ inline double block_sum(double v, double* red)
{
    const int tid = threadIdx.x;
    __syncthreads();
    red[tid] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) red[tid] += red[tid + o];
        __syncthreads();
    }
    const double s = red[0];
    __syncthreads();
    return s;
}

// One workgroup per item.  MODE 0: contact seeds into dseed.  MODE 1: the
// inertia adjoint (G d - c) / dt^2 added to the adjoint of h (slice 0 of gbar).
// MODE 2: inertia and contact added to E, g and the Gauss-Newton part of H.
// MODE 3: energies only (float64 value pass: act and out with one column).
// The r x r and r-vector sums run on the float64 matrix cores in 4-row steps
// (lane (c, kq) holding row 4t + kq, column c of a 16-column tile; the
// gradient as the product with a B operand that is zero outside column 0),
// waves taking every fourth step, their partials added in wave order:
// * contact: the active contact rows (penetration d < 0) of each chunk of 1024,
//   listed in index order by a wave-ballot compaction, give
//   k_g sum_k J_k^T J_k and k_g sum_k d_k J_k^T;
// * inertia: G J_h (m x r, G symmetric) on the matrix cores into LDS, then
//   J_h^T (G J_h) / dt^2 and J_h^T y / dt^2 with y = G d - c.
template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_dyn(DynArgs a)
{
    extern __shared__ double sh[];
    __shared__ double red[256];
    __shared__ int wcnt[4];
    using acc_t = typename Mfma<double>::acc_t;
    const int item = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c = lane & 15, kq = lane >> 4;
    if (a.count && item >= *a.count) return;
    if (MODE == 1 && !a.inertia) return;
    const int r = a.r, m = a.in_last, nc = a.nc;
    const int RT = (r + 15) / 16;
    const int b = a.imap ? a.imap[item] : item;
    const T* O = static_cast<const T*>(a.out) + (size_t)item * a.rows_pad * nc;
    const T* act = a.act ? static_cast<const T*>(a.act) + (size_t)item * nc * a.wrows : nullptr;
    // ---- contact seeds
    if (MODE == 0) {
        T* ds = static_cast<T*>(a.dseed) + (size_t)item * a.rows_pad;
        for (int k = tid; k < a.ncont; k += 256) {
            const double d = a.Xc[k] + (double)O[(size_t)(a.crow + k) * nc] - a.ground_y;
            ds[a.crow + k] = (T)(d < 0.0 ? a.k_ground * d : 0.0);
        }
        return;
    }
    double* dv = sh;           // m: d = h - eta
    double* y = dv + 256;      // m: G d - c
    double* wk = y + 256;      // work area: the contact list, then G J_h (m x 32), then the wave partials
    double e_acc = 0.0;
    acc_t aH[2][2], ag[2];
#pragma unroll
    for (int ti = 0; ti < 2; ++ti) {
        ag[ti] = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) aH[ti][tj] = acc_t{0, 0, 0, 0};
    }
    // ---- contact rows
    if (MODE == 2 || MODE == 3) {
        int* list = reinterpret_cast<int*>(wk); // 1024 active indices of a chunk
        double* dl = wk + 512;                  // and their penetrations
        for (int k0 = 0; k0 < a.ncont; k0 += 1024) {
            const int kn = min(1024, a.ncont - k0);
            int nact = 0;
            __syncthreads(); // the previous chunk's list is consumed
            for (int j = 0; j < kn; j += 256) {
                const int k = k0 + j + tid;
                double d = 0.0;
                bool on = false;
                if (j + tid < kn) {
                    d = a.Xc[k] + (double)O[(size_t)(a.crow + k) * nc] - a.ground_y;
                    on = d < 0.0;
                }
                if (on) e_acc += 0.5 * a.k_ground * d * d;
                if (MODE == 2) {
                    const unsigned long long bal = __ballot(on);
                    const int below = __popcll(bal & ((1ull << lane) - 1ull));
                    if (lane == 0) wcnt[wave] = __popcll(bal);
                    __syncthreads();
                    int off = nact;
                    for (int q = 0; q < wave; ++q) off += wcnt[q];
                    if (on) {
                        list[off + below] = k;
                        dl[off + below] = d;
                    }
                    nact += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
                    __syncthreads(); // wcnt is reused
                }
            }
            if (MODE == 2) {
                __syncthreads(); // the list is complete
                for (int t = wave; t < (nact + 3) / 4; t += 4) {
                    const int idx = 4 * t + kq;
                    const bool ok = idx < nact;
                    const T* row = O + (size_t)(a.crow + (ok ? list[idx] : 0)) * nc;
                    double x[2];
#pragma unroll
                    for (int ti = 0; ti < 2; ++ti) {
                        const int col = 16 * ti + c;
                        x[ti] = (ok && ti < RT && col < r) ? (double)row[1 + col] : 0.0;
                    }
                    const double bg = (ok && c == 0) ? a.k_ground * dl[idx] : 0.0;
#pragma unroll
                    for (int ti = 0; ti < 2; ++ti) {
                        if (ti >= RT) break;
                        ag[ti] = Mfma<double>::mac(x[ti], bg, ag[ti]);
#pragma unroll
                        for (int tj = 0; tj < 2; ++tj)
                            if (tj < RT) aH[ti][tj] = Mfma<double>::mac(x[ti], a.k_ground * x[tj], aH[ti][tj]);
                    }
                }
            }
        }
    }
    // ---- inertia
    if (a.inertia) {
        const double* cv = a.cvec + (size_t)b * m;
        const double* et = a.eta ? a.eta + (size_t)b * m : nullptr;
        for (int u = tid; u < m; u += 256) {
            double hv;
            if (a.L > 0) hv = (double)act[u];
            else hv = a.z[(size_t)(a.zmap ? a.zmap[item] : item) * r + u];
            dv[u] = et ? hv - et[u] : hv;
        }
        __syncthreads();
        // y = G d - c, reading G by columns (G symmetric: consecutive threads, consecutive addresses)
        for (int u = tid; u < m; u += 256) {
            double s = 0.0;
#pragma unroll 8
            for (int v = 0; v < m; ++v) s += a.G[(size_t)v * m + u] * dv[v];
            y[u] = s - cv[u];
        }
        __syncthreads();
        if (MODE == 1) {
            T* gb = static_cast<T*>(a.gbar) + (size_t)item * a.in_rows;
            for (int u = tid; u < m; u += 256) gb[u] = (T)((double)gb[u] + a.inv_dt2 * y[u]);
            return;
        }
        double e = 0.0;
        for (int u = tid; u < m; u += 256) e += dv[u] * (y[u] - cv[u]);
        e_acc += 0.5 * a.inv_dt2 * e;
        if (tid == 0) e_acc += 0.5 * a.inv_dt2 * a.kappa[b];
        if (MODE == 2) {
            // J_h (m x r): the Jacobian columns of the activation, or the identity (linear decoder)
            auto jh = [&](int u, int k) -> double {
                if (u >= m || k >= r) return 0.0;
                if (a.L > 0) return (double)act[(size_t)(1 + k) * a.wrows + u];
                return u == k ? 1.0 : 0.0;
            };
            double* GJ = wk; // m x 32
            const int ks = (m + 3) / 4, mt = (m + 15) / 16;
            __syncthreads(); // the contact list is no longer read
            for (int tile = wave; tile < mt * RT; tile += 4) {
                const int ti = tile / RT, tj = tile - ti * RT;
                acc_t acc = acc_t{0, 0, 0, 0};
                const int gi = 16 * ti + c;
#pragma unroll 4
                for (int st = 0; st < ks; ++st) {
                    const int kk = 4 * st + kq;
                    const double av = (gi < m && kk < m) ? a.G[(size_t)kk * m + gi] : 0.0; // G[gi][kk]
                    acc = Mfma<double>::mac(av, jh(kk, 16 * tj + c), acc);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 16 * ti + kq + 4 * v;
                    if (row < m) GJ[row * 32 + 16 * tj + c] = acc[v];
                }
            }
            __syncthreads();
            for (int t = wave; t < ks; t += 4) {
                const int u = 4 * t + kq;
                const bool ok = u < m;
                double x[2];
#pragma unroll
                for (int ti = 0; ti < 2; ++ti) x[ti] = (ok && ti < RT) ? jh(u, 16 * ti + c) : 0.0;
                const double bg = (ok && c == 0) ? a.inv_dt2 * y[u] : 0.0;
#pragma unroll
                for (int ti = 0; ti < 2; ++ti) {
                    if (ti >= RT) break;
                    ag[ti] = Mfma<double>::mac(x[ti], bg, ag[ti]);
#pragma unroll
                    for (int tj = 0; tj < 2; ++tj)
                        if (tj < RT) {
                            const int col = 16 * tj + c;
                            const double gv = (ok && col < r) ? a.inv_dt2 * GJ[u * 32 + col] : 0.0;
                            aH[ti][tj] = Mfma<double>::mac(x[ti], gv, aH[ti][tj]);
                        }
                }
            }
        }
    }
    const double Et = block_sum(e_acc, red);
    if (tid == 0 && a.E) a.E[item] += Et;
    if (MODE != 2) return;
    // the four waves' partials, added in wave order
    double* part = wk; // [4 waves][2][2 + 1][4][64]
    __syncthreads();   // G J_h is no longer read
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
#pragma unroll
            for (int tj = 0; tj < 2; ++tj) part[((((wave * 2 + ti) * 3 + tj) * 4) + v) * 64 + lane] = aH[ti][tj][v];
            part[((((wave * 2 + ti) * 3 + 2) * 4) + v) * 64 + lane] = ag[ti][v];
        }
    __syncthreads();
    if (wave != 0) return;
    auto sum4 = [&](int ti, int tj, int v) {
        double s = 0.0;
        for (int q = 0; q < 4; ++q) s += part[((((q * 2 + ti) * 3 + tj) * 4) + v) * 64 + lane];
        return s;
    };
    for (int ti = 0; ti < RT; ++ti)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * ti + kq + 4 * v; // float64 result layout: D[lane / 16 + 4 v][lane % 16]
            if (row >= r) continue;
            if (a.H)
                for (int tj = 0; tj < RT; ++tj) {
                    const int col = 16 * tj + c;
                    if (col < r) a.H[((size_t)item * r + row) * r + col] += sum4(ti, tj, v);
                }
            if (a.g && c == 0) a.g[(size_t)item * r + row] += sum4(ti, 2, v);
        }
}

// The inertial target of one step of a simulation, per item: eta = h0 with
// rho = dt v0 (first step: u^0 + dt v0; c = dt W^T M v0, kappa = dt^2 |v0|_M^2
// from the prepared cv0, kv0), or eta = 2 h1 - h0 with rho = 0 (later steps:
// 2 u^k - u^(k-1) lies in the decoder's range).
__global__ void k_dyn_state(int m, const double* h0, const double* h1, const double* cv0, const double* kv0,
                            double dt, int B, double* eta, double* cvec, double* kappa)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * m) return;
    const int b = i / m;
    eta[i] = h1 ? 2.0 * h1[i] - h0[i] : h0[i];
    cvec[i] = cv0 ? dt * cv0[i] : 0.0;
    if (i - b * m == 0) kappa[b] = kv0 ? dt * dt * kv0[b] : 0.0;
}

// h (B x m, float64) from the float64 value pass (act64 rows of stride wrows) or z (linear decoders)
__global__ void k_dyn_take_h(const double* act64, int wrows, const double* z, int m, int B, double* h)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * m) return;
    const int b = i / m, u = i - b * m;
    h[i] = act64 ? act64[(size_t)b * wrows + u] : z[i];
}

__global__ void k_zero_int(int* p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// per item: iters += step iterations, failed += (status != converged)
__global__ void k_sim_count(const int* it, const int* st, int B, int* iters, int* failed)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    iters[b] += it[b];
    failed[b] += st[b] != 0;
}

}  // namespace

hipError_t launch_dyn_state(int m, const double* h0, const double* h1, const double* cv0, const double* kv0,
                            double dt, int B, double* eta, double* cvec, double* kappa, hipStream_t s)
{
    if (B * m <= 0) return hipSuccess;
    RS_LAUNCH(k_dyn_state, dim3((unsigned)((B * m + 255) / 256)), dim3(256), 0, s, m, h0, h1, cv0, kv0, dt, B, eta,
              cvec, kappa);
    return hipGetLastError();
}

hipError_t launch_dyn_take_h(const double* act64, int wrows, const double* z, int m, int B, double* h, hipStream_t s)
{
    if (B * m <= 0) return hipSuccess;
    RS_LAUNCH(k_dyn_take_h, dim3((unsigned)((B * m + 255) / 256)), dim3(256), 0, s, act64, wrows, z, m, B, h);
    return hipGetLastError();
}

hipError_t launch_zero_int(int* p, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    RS_LAUNCH(k_zero_int, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_sim_count(const int* it, const int* st, int B, int* iters, int* failed, hipStream_t s)
{
    if (B <= 0) return hipSuccess;
    RS_LAUNCH(k_sim_count, dim3((unsigned)((B + 63) / 64)), dim3(64), 0, s, it, st, B, iters, failed);
    return hipGetLastError();
}

hipError_t launch_dyn_gram(int f32, const void* W, int ld, int rows, const double* rowmass, int m, double* G,
                           hipStream_t s)
{
    const dim3 grid((unsigned)((m + 127) / 128), (unsigned)m);
    if (f32) RS_LAUNCH(k_dyn_gram<float>, grid, dim3(128), 0, s, (const float*)W, ld, rows, rowmass, m, G);
    else RS_LAUNCH(k_dyn_gram<double>, grid, dim3(128), 0, s, (const double*)W, ld, rows, rowmass, m, G);
    return hipGetLastError();
}

hipError_t launch_dyn_prep(int f32, const void* W, int ld, const void* bias, const uint8_t* pinned_row,
                           const double* rowmass, int rows, int m, const double* qbar, int B, double* cvec,
                           double* kappa, hipStream_t s)
{
    if (B <= 0) return hipSuccess;
    if (f32)
        RS_LAUNCH(k_dyn_prep<float>, dim3(B), dim3(256), 0, s, (const float*)W, ld, (const float*)bias, pinned_row,
                  rowmass, rows, m, qbar, cvec, kappa);
    else
        RS_LAUNCH(k_dyn_prep<double>, dim3(B), dim3(256), 0, s, (const double*)W, ld, (const double*)bias, pinned_row,
                  rowmass, rows, m, qbar, cvec, kappa);
    return hipGetLastError();
}

// mode 0: contact seeds; 1: inertia adjoint into gbar; 2: E, g, H; 3: energies (float64 value pass)
hipError_t launch_dyn(int f32, int mode, const DynArgs& a, int cap, hipStream_t s)
{
    if (cap <= 0) return hipSuccess;
    if (a.r > 32 || a.in_last > 256) return hipErrorInvalidValue;
    // d, y and the work area (the contact list, G J_h for m <= 256, the waves' partials)
    const size_t shm = sizeof(double) * (256 + 256 + 256 * 32);
    const dim3 g(cap), blk(256);
    if (mode == 3) {
        RS_LAUNCH((k_dyn<double, 3>), g, blk, shm, s, a);
    } else if (f32) {
        if (mode == 0) RS_LAUNCH((k_dyn<float, 0>), g, blk, shm, s, a);
        else if (mode == 1) RS_LAUNCH((k_dyn<float, 1>), g, blk, shm, s, a);
        else RS_LAUNCH((k_dyn<float, 2>), g, blk, shm, s, a);
    } else {
        if (mode == 0) RS_LAUNCH((k_dyn<double, 0>), g, blk, shm, s, a);
        else if (mode == 1) RS_LAUNCH((k_dyn<double, 1>), g, blk, shm, s, a);
        else RS_LAUNCH((k_dyn<double, 2>), g, blk, shm, s, a);
    }
    return hipGetLastError();
}

}  // namespace rs
