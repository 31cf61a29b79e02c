// Device-side pieces shared by the kernel sources of librs: the launch macro
// (with the profiler's per-launch events), vector types, the matrix-core
// wrappers, ELU and its derivatives, and the stable Neo-Hookean density in
// displacement-gradient form.  Not part of the ABI.
#pragma once

#include "rs_internal.hpp"

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

namespace rs {

// Launch events armed by the profiler for the next launch only: the events
// are recorded by the dispatch itself (no marker packets between kernels).
extern thread_local hipEvent_t g_launch_ev[2];

#define RS_LAUNCH(kernel, grid, block, shm, stream, ...)                                          \
    do {                                                                                         \
        if (g_launch_ev[0]) {                                                                    \
            hipEvent_t e0_ = g_launch_ev[0], e1_ = g_launch_ev[1];                               \
            g_launch_ev[0] = g_launch_ev[1] = nullptr;                                           \
            hipExtLaunchKernelGGL(kernel, grid, block, shm, stream, e0_, e1_, 0, __VA_ARGS__);   \
        } else {                                                                                 \
            hipLaunchKernelGGL(kernel, grid, block, shm, stream, __VA_ARGS__);                   \
        }                                                                                        \
    } while (0)

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
// Both take A[i][k] from lane i + 16 k and B[k][j] from lane j + 16 k; the
// result rows differ: f32 puts D[4 (lane/16) + v][lane%16] in register v,
// f64 puts D[lane/16 + 4 v][lane%16] in register v.
template <> struct Mfma<float> {
    using acc_t = f32x4;
    __device__ static acc_t mac(float a, float b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <> struct Mfma<double> {
    using acc_t = f64x4;
    __device__ static acc_t mac(double a, double b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

// 16-byte vectors as clang native vectors (element access stays in registers)
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename T> struct Vec16;
template <> struct Vec16<float> { using type = f32x4; static constexpr int n = 4; };
template <> struct Vec16<double> { using type = f64x2; static constexpr int n = 2; };
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Workgroup barrier for LDS traffic only: this wave's LDS operations complete
// (lgkmcnt 0, vector-memory count untouched), then s_barrier.  Global stores
// may still be in flight; callers read nothing back that another wave of the
// workgroup stored to global memory.
__device__ inline void lds_barrier()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Eight float32 values as three BF16 parts: hi = bf16(x), mid = bf16(x - hi),
// lo = bf16(x - hi - mid).  Each difference is exact in float32 (the operands
// are within a factor of two of each other), so hi + mid + lo carries all 24
// significant bits of x up to the last part's rounding.
__device__ inline void split3_bf16(f32x4 x0, f32x4 x1, bf16x8& hi, bf16x8& mid, bf16x8& lo)
{
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const __bf16 h0 = (__bf16)x0[e], h1 = (__bf16)x1[e];
        const float r0 = x0[e] - (float)h0, r1 = x1[e] - (float)h1;
        const __bf16 m0 = (__bf16)r0, m1 = (__bf16)r1;
        hi[e] = h0;
        hi[4 + e] = h1;
        mid[e] = m0;
        mid[4 + e] = m1;
        lo[e] = (__bf16)(r0 - (float)m0);
        lo[4 + e] = (__bf16)(r1 - (float)m1);
    }
}

// Six BF16 products of one 32-deep chunk that give a float32-accurate product
// of two operands held as three BF16 parts each (hi, mid, lo): the terms whose
// combined weight is at least 2^-16 of hi*hi (Henry, Tang and Heinecke, "Leveraging
// the bfloat16 artificial intelligence datatype for higher-precision
// computations", ARITH 2019).  The dropped terms (mid*lo, lo*mid, lo*lo) are below
// 2^-24 relative.  The small terms go into `corr`, hi*hi into `acc`.  Lane
// (i + 16 g) supplies A[i][8g .. 8g+7] and B[8g .. 8g+7][i] of each 16x16x32
// product: the permuted-k fragment every GEMM here holds per 32-deep chunk.
__device__ inline void mfma_bf16x6_chunk(const bf16x8 (&a)[3], const bf16x8 (&b)[3], f32x4& acc, f32x4& corr)
{
    corr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[2], corr, 0, 0, 0);
    corr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[0], corr, 0, 0, 0);
    corr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[1], corr, 0, 0, 0);
    corr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[1], corr, 0, 0, 0);
    corr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[0], corr, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[0], acc, 0, 0, 0);
}

// ELU with alpha = 1 (linear branch for a > 0) and its first two derivatives.
__device__ inline float elu0(float a) { return a > 0.f ? a : expm1f(a); }
__device__ inline double elu0(double a) { return a > 0.0 ? a : expm1(a); }
__device__ inline float elu1(float a) { return a > 0.f ? 1.f : expf(a); }
__device__ inline double elu1(double a) { return a > 0.0 ? 1.0 : exp(a); }
__device__ inline double elu2(double a) { return a > 0.0 ? 0.0 : exp(a); }

template <typename T>
struct Snh {
    T g[3][3];   // g[j][i] = G_ij
    T f[3][3];   // f[j][i] = F_ij
    T cof[3][3]; // cof[j][i] = (cof F)_ij
    T cg[3][3];  // cg[j][i] = (cof G)_ij
    T jm, psi, s; // J - 1, energy density, lam (J-1) - mu

    __device__ void set(const T* gu, T mu, T lam)
    {
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                g[j][i] = gu[3 * j + i];
                f[j][i] = g[j][i] + (i == j ? T(1) : T(0));
            }
        cross(g[1], g[2], cg[0]);
        cross(g[2], g[0], cg[1]);
        cross(g[0], g[1], cg[2]);
        const T tr = g[0][0] + g[1][1] + g[2][2];
        const T detg = g[0][0] * cg[0][0] + g[0][1] * cg[0][1] + g[0][2] * cg[0][2];
        const T i2 = (g[0][0] * g[1][1] - g[1][0] * g[0][1]) + (g[0][0] * g[2][2] - g[2][0] * g[0][2])
                   + (g[1][1] * g[2][2] - g[2][1] * g[1][2]);
        T nrm = 0;
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                nrm += g[j][i] * g[j][i];
                cof[j][i] = (i == j ? T(1) + tr : T(0)) - g[i][j] + cg[j][i];
            }
        jm = tr + i2 + detg;
        psi = T(0.5) * mu * nrm - mu * (i2 + detg) + T(0.5) * lam * jm * jm;
        s = lam * jm - mu;
    }
    __device__ static void cross(const T* a, const T* b, T* c)
    {
        c[0] = a[1] * b[2] - a[2] * b[1];
        c[1] = a[2] * b[0] - a[0] * b[2];
        c[2] = a[0] * b[1] - a[1] * b[0];
    }
    // first Piola-Kirchhoff stress, vec layout
    __device__ void pk1(T mu, T lam, T* P) const
    {
        const T tr = g[0][0] + g[1][1] + g[2][2];
        const T lj = lam * jm;
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int i = 0; i < 3; ++i)
                P[3 * j + i] = mu * (g[j][i] + g[i][j] - (i == j ? tr : T(0)) - cg[j][i]) + lj * cof[j][i];
    }
    // (d2 psi / dF2) v with mu, lam and s scaled by the caller (one weight for
    // the element folded into the three scalars); the columns of d(cof F)[v]
    // as single fused chains
    __device__ void apply_hess_w(T wmu, T wlam, T ws, const T* v, T* out) const
    {
        T gv = 0;
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int i = 0; i < 3; ++i) gv = fma(cof[j][i], v[3 * j + i], gv);
        const T t = wlam * gv;
        const T* v0 = v;
        const T* v1 = v + 3;
        const T* v2 = v + 6;
        // column j of d(cof F)[v]: v_{j+1} x f_{j+2} + f_{j+1} x v_{j+2}
        auto dcol = [&](const T* va, const T* fb, const T* fa, const T* vb, int i) {
            const int i1 = (i + 1) % 3, i2 = (i + 2) % 3;
            T d = va[i1] * fb[i2];
            d = fma(-va[i2], fb[i1], d);
            d = fma(fa[i1], vb[i2], d);
            return fma(-fa[i2], vb[i1], d);
        };
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            out[i] = fma(ws, dcol(v1, f[2], f[1], v2, i), fma(t, cof[0][i], wmu * v0[i]));
            out[3 + i] = fma(ws, dcol(v2, f[0], f[2], v0, i), fma(t, cof[1][i], wmu * v1[i]));
            out[6 + i] = fma(ws, dcol(v0, f[1], f[0], v1, i), fma(t, cof[2][i], wmu * v2[i]));
        }
    }
    // (d2 psi / dF2) v = mu v + lam g (g.v) + s d(cof F)[v], g = vec cof F,
    // d(cof F)[v] = [v1 x f2 + f1 x v2, v2 x f0 + f2 x v0, v0 x f1 + f0 x v1]
    __device__ void apply_hess(T mu, T lam, const T* v, T* out) const
    {
        T gv = 0;
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int i = 0; i < 3; ++i) gv += cof[j][i] * v[3 * j + i];
        T d0[3], d1[3], d2[3], t0[3], t1[3];
        cross(v + 3, f[2], t0); cross(f[1], v + 6, t1);
#pragma unroll
        for (int i = 0; i < 3; ++i) d0[i] = t0[i] + t1[i];
        cross(v + 6, f[0], t0); cross(f[2], v, t1);
#pragma unroll
        for (int i = 0; i < 3; ++i) d1[i] = t0[i] + t1[i];
        cross(v, f[1], t0); cross(f[0], v + 3, t1);
#pragma unroll
        for (int i = 0; i < 3; ++i) d2[i] = t0[i] + t1[i];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            out[i] = mu * v[i] + lam * cof[0][i] * gv + s * d0[i];
            out[3 + i] = mu * v[3 + i] + lam * cof[1][i] * gv + s * d1[i];
            out[6 + i] = mu * v[6 + i] + lam * cof[2][i] * gv + s * d2[i];
        }
    }
};
}  // namespace rs
