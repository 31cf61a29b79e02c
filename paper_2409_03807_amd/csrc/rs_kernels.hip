// HIP kernels of the reduced-Newton hot path for gfx950 (MI355X).
//
// Data layout: every batch tensor is item-major.  For one item the decoder
// state of a layer is a (rows x nc) block, nc = 1 + r, whose column 0 is the
// value (pre-activation a, or output value) and columns 1..r its Jacobian with
// respect to z (forward mode, Sec. 3.2 decoder with its Jacobian df/dz as in
// Eq. form-cubature-gradients).  The GEMMs flatten (item, column) into one
// column index, so any r uses the same 64x64 MFMA tiles.
#include "rs_device.hpp"

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include <hip/hip_ext.h>

namespace rs {

// Launch events armed by the profiler for the next launch only: the events
// are recorded by the dispatch itself (no marker packets between kernels).
thread_local hipEvent_t g_launch_ev[2] = {nullptr, nullptr};
void set_launch_events(hipEvent_t start, hipEvent_t stop)
{
    g_launch_ev[0] = start;
    g_launch_ev[1] = stop;
}
bool launch_events_pending() { return g_launch_ev[0] != nullptr; }

// ---------------------------------------------------------------------------
// GEMM: C[item] = A * Y[item] (+ bias on column 0), MFMA 16x16x4, 64x64 tiles.
// Each of the 4 waves owns 16 rows x 64 columns (four 16x16 accumulators).
// The item count may live on the device (blocks past it exit at once), and
// the reduction may be split over blockIdx.z into partial outputs.
// ---------------------------------------------------------------------------
template <typename T, int ROLE>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs a)
{
    static_assert(kTileK == 32, "tile loads assume 32-deep chunks");
    // An MFMA sums over k, so any order of k works if A and B agree: lane
    // group g = lane/16 takes k in [8g, 8g+8) of each chunk, which lets every
    // lane read its 8 A values and 8 B values per tile with 16-byte LDS loads.
    // Rows are padded by 16 bytes so 8 consecutive rows hit distinct banks.
    using V = typename Vec16<T>::type;
    constexpr int VN = Vec16<T>::n;
    constexpr int LD = kTileK + VN;
    __shared__ __align__(16) T As[kTileM * LD];
    __shared__ __align__(16) T Ys[kTileN * LD];
    // column counts stay far below 2^31 (items * nc), so 32-bit index math
    const int items = a.count ? min(*a.count, a.items) : a.items;
    const int ncols = items * a.nc;
    const int n0 = blockIdx.y * kTileN;
    if (n0 >= ncols) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int m0 = blockIdx.x * kTileM;
    const T* A = static_cast<const T*>(a.A);
    using acc_t = typename Mfma<T>::acc_t;
    acc_t acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = acc_t{0, 0, 0, 0};
    const unsigned ncu = (unsigned)a.nc;

    int kbeg = 0, kend = a.K;
    T* Cout = static_cast<T*>(a.C);
    if (a.ksplit > 1) {
        const int kchunk = ((a.K + a.ksplit - 1) / a.ksplit + kTileK - 1) / kTileK * kTileK;
        kbeg = blockIdx.z * kchunk;
        kend = min(a.K, kbeg + kchunk);
        Cout += blockIdx.z * a.split_stride;
    }

    // global -> registers: 8 consecutive k of one A row / one Y column per thread
    const int arow = tid >> 2, akq = (tid & 3) * 8;
    const int ynn = tid & 63, ykb = (tid >> 6) * 8;
    const int yn = n0 + ynn;
    const bool ycol = yn < ncols;
    int yitem = 0, yc = 0;
    if (ycol) {
        yitem = (int)((unsigned)yn / ncu);
        yc = yn - yitem * a.nc;
    }
    long zrow = 0;
    if (a.in_mode == IN_LATENT && ycol) zrow = a.zmap ? a.zmap[yitem] : yitem;
    const T* Ycol = (a.in_mode != IN_LATENT && ycol)
                        ? static_cast<const T*>(a.Y) + (size_t)yitem * a.y_rows * a.nc : nullptr;
    const T* Ytr = (a.in_mode == IN_RAW_T && ycol)
                       ? static_cast<const T*>(a.Y) + ((size_t)yitem * a.nc + yc) * a.y_rows : nullptr;

    V ra[8 / VN];
    T ry[8];
    auto load = [&](int k0) {
        const V* src = reinterpret_cast<const V*>(A + (size_t)(m0 + arow) * a.lda + k0 + akq);
#pragma unroll
        for (int q = 0; q < 8 / VN; ++q) ra[q] = src[q];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int k = k0 + ykb + q;
            T v = T(0);
            if (ycol && k < kend) {
                if (a.in_mode == IN_LATENT) {
                    if (yc == 0) v = (T)a.z[zrow * a.r + k];
                    else v = (k == yc - 1) ? T(1) : T(0);
                } else if (a.in_mode == IN_RAW_T) {
                    v = Ytr[k];
                } else {
                    const T* Yb = Ycol + (size_t)k * a.nc;
                    if (a.in_mode == IN_ELU) {
                        const T av = Yb[0];
                        v = (yc == 0) ? elu0(av) : T(elu1(av)) * Yb[yc];
                    } else {
                        v = Yb[yc];
                    }
                }
            }
            ry[q] = v;
        }
    };

    if (kbeg < kend) load(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += kTileK) {
        {
            V* da = reinterpret_cast<V*>(As + arow * LD + akq);
#pragma unroll
            for (int q = 0; q < 8 / VN; ++q) da[q] = ra[q];
            V* dy = reinterpret_cast<V*>(Ys + ynn * LD + ykb);
#pragma unroll
            for (int q = 0; q < 8 / VN; ++q) {
                V w;
#pragma unroll
                for (int e = 0; e < VN; ++e) w[e] = ry[q * VN + e];
                dy[q] = w;
            }
        }
        __syncthreads();
        if (k0 + kTileK < kend) load(k0 + kTileK);
        T af[8], bf[4][8];
        {
            const V* sa = reinterpret_cast<const V*>(As + (wave * 16 + li) * LD + 8 * lg);
#pragma unroll
            for (int q = 0; q < 8 / VN; ++q) {
                const V w = sa[q];
#pragma unroll
                for (int e = 0; e < VN; ++e) af[q * VN + e] = w[e];
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const V* sb = reinterpret_cast<const V*>(Ys + (t * 16 + li) * LD + 8 * lg);
#pragma unroll
                for (int q = 0; q < 8 / VN; ++q) {
                    const V w = sb[q];
#pragma unroll
                    for (int e = 0; e < VN; ++e) bf[t][q * VN + e] = w[e];
                }
            }
        }
#pragma unroll
        for (int kk = 0; kk < 8; ++kk)
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[t] = Mfma<T>::mac(af[kk], bf[t][kk], acc[t]);
        __syncthreads();
    }

    const T* bias = (a.ksplit > 1 && blockIdx.z > 0) ? nullptr : static_cast<const T*>(a.bias);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int n = n0 + t * 16 + li;
        if (n >= ncols) continue;
        const int item = (int)((unsigned)n / ncu);
        const int c = n - item * a.nc;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int m = m0 + wave * 16 + Mfma<T>::row(lane, v);
            if (m >= a.rows) continue;
            T val = acc[t][v];
            if (c == 0 && bias) val += bias[m];
            if (a.out_mode == OUT_PACK) {
                Cout[((size_t)item * a.rows_pad + m) * a.nc + c] = val;
            } else if (c == 0) {
                if (a.Xo) static_cast<T*>(a.Xo)[(size_t)item * a.rows + m] = static_cast<const T*>(a.Xrest)[m] + val;
            } else if (a.Jo) {
                static_cast<T*>(a.Jo)[((size_t)item * a.rows + m) * a.r + (c - 1)] = val;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Persistent output-map GEMM (IN_RAW / IN_LATENT inputs, OUT_PACK / OUT_SPLIT):
// a workgroup keeps its 64 rows of A for the whole K in registers (loaded once
// from L2) and walks the column tiles g, g + G, g + 2G, ...; each 32-deep
// chunk of the input tile goes through a double-buffered LDS pipeline with
// the next chunk prefetched into registers behind the MFMAs (one barrier per
// chunk).  KCH = K / 32 chunks.
// ---------------------------------------------------------------------------
template <typename T, int ROLE, int KCH>
__global__ __launch_bounds__(256) void k_gemm_p(GemmArgs a, int groups)
{
    using V = typename Vec16<T>::type;
    constexpr int VN = Vec16<T>::n;
    constexpr int LD = kTileK + VN;
    __shared__ __align__(16) T Ys[2][kTileN * LD];
    const int items = a.count ? min(*a.count, a.items) : a.items;
    const int ncols = items * a.nc;
    const int ntiles = (ncols + kTileN - 1) / kTileN;
    const int g = blockIdx.y;
    if (g >= ntiles) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int m0 = blockIdx.x * kTileM;
    const unsigned ncu = (unsigned)a.nc;
    using acc_t = typename Mfma<T>::acc_t;

    // A fragments for every chunk: row m0 + 16 wave + li, k = 32 c + 8 lg .. + 7
    T af[KCH][8];
    {
        const T* A = static_cast<const T*>(a.A) + (size_t)(m0 + wave * 16 + li) * a.lda + 8 * lg;
#pragma unroll
        for (int c = 0; c < KCH; ++c) {
            const V* src = reinterpret_cast<const V*>(A + c * kTileK);
#pragma unroll
            for (int q = 0; q < 8 / VN; ++q) {
                const V w = src[q];
#pragma unroll
                for (int e = 0; e < VN; ++e) af[c][q * VN + e] = w[e];
            }
        }
    }

    // input tile loads: thread owns column ynn of the tile and 8 consecutive k
    const int ynn = tid & 63, ykb = (tid >> 6) * 8;
    T ry[8];
    auto load = [&](int ct, int c) {
        const int yn = ct * kTileN + ynn;
        const int k0 = c * kTileK + ykb;
#pragma unroll
        for (int q = 0; q < 8; ++q) ry[q] = T(0);
        if (yn < ncols) {
            const int yitem = (int)((unsigned)yn / ncu);
            const int yc = yn - yitem * a.nc;
            if (a.in_mode == IN_LATENT) {
                const long zr = a.zmap ? a.zmap[yitem] : yitem;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int k = k0 + q;
                    if (k < a.K) ry[q] = (yc == 0) ? (T)a.z[zr * a.r + k] : ((k == yc - 1) ? T(1) : T(0));
                }
            } else if (a.in_mode == IN_RAW_T) {
                const T* Yb = static_cast<const T*>(a.Y) + ((size_t)yitem * a.nc + yc) * a.y_rows + k0;
                if (k0 + 8 <= a.K) {
                    const V* v8 = reinterpret_cast<const V*>(Yb);
#pragma unroll
                    for (int q = 0; q < 8 / VN; ++q) {
                        const V w = v8[q];
#pragma unroll
                        for (int e = 0; e < VN; ++e) ry[q * VN + e] = w[e];
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        if (k0 + q < a.K) ry[q] = Yb[q];
                }
            } else {
                const T* Yb = static_cast<const T*>(a.Y) + ((size_t)yitem * a.y_rows + k0) * a.nc + yc;
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (k0 + q < a.K) ry[q] = Yb[(size_t)q * a.nc];
            }
        }
    };
    auto store = [&](int buf) {
        V* dy = reinterpret_cast<V*>(&Ys[buf][ynn * LD + ykb]);
#pragma unroll
        for (int q = 0; q < 8 / VN; ++q) {
            V w;
#pragma unroll
            for (int e = 0; e < VN; ++e) w[e] = ry[q * VN + e];
            dy[q] = w;
        }
    };

    const T* bias = static_cast<const T*>(a.bias);
    T* Cout = static_cast<T*>(a.C);
    acc_t acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = acc_t{0, 0, 0, 0};

    int ct = g, c = 0, buf = 0;
    load(ct, 0);
    store(0);
    __syncthreads();
    for (;;) {
        // next (tile, chunk) of this workgroup
        int nct = ct, nchk = c + 1;
        if (nchk == KCH) {
            nchk = 0;
            nct = ct + groups;
        }
        const bool more = nct < ntiles;
        if (more) load(nct, nchk);
        {
            T bf[4][8];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const V* sb = reinterpret_cast<const V*>(&Ys[buf][(t * 16 + li) * LD + 8 * lg]);
#pragma unroll
                for (int q = 0; q < 8 / VN; ++q) {
                    const V w = sb[q];
#pragma unroll
                    for (int e = 0; e < VN; ++e) bf[t][q * VN + e] = w[e];
                }
            }
#pragma unroll
            for (int cc = 0; cc < KCH; ++cc) {
                if (cc != c) continue;
#pragma unroll
                for (int kk = 0; kk < 8; ++kk)
#pragma unroll
                    for (int t = 0; t < 4; ++t) acc[t] = Mfma<T>::mac(af[cc][kk], bf[t][kk], acc[t]);
            }
        }
        if (c == KCH - 1) {
            // epilogue of tile ct
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int n = ct * kTileN + t * 16 + li;
                if (n < ncols) {
                    const int item = (int)((unsigned)n / ncu);
                    const int cidx = n - item * a.nc;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int m = m0 + wave * 16 + Mfma<T>::row(lane, v);
                        if (m >= a.rows) continue;
                        T val = acc[t][v];
                        if (cidx == 0 && bias) val += bias[m];
                        if (a.out_mode == OUT_PACK) {
                            Cout[((size_t)item * a.rows_pad + m) * a.nc + cidx] = val;
                        } else if (cidx == 0) {
                            if (a.Xo)
                                static_cast<T*>(a.Xo)[(size_t)item * a.rows + m] =
                                    static_cast<const T*>(a.Xrest)[m] + val;
                        } else if (a.Jo) {
                            static_cast<T*>(a.Jo)[((size_t)item * a.rows + m) * a.r + (cidx - 1)] = val;
                        }
                    }
                }
                acc[t] = acc_t{0, 0, 0, 0};
            }
        }
        if (!more) break;
        store(buf ^ 1);
        lds_barrier(); // LDS only: this tile's output stores stay in flight
        buf ^= 1;
        ct = nct;
        c = nchk;
    }
}

// Same contract with the whole K of the next column tile prefetched into
// registers (thread: one column, K/4 consecutive k) while the current tile,
// resident in LDS, feeds the MFMAs: the load latency hides behind a full
// tile of MFMAs.  Used when the tile fits 64 KB of LDS.
// The float32 output map over transposed activations (the reduced solve's
// gemm_out) is held to 128 registers: four waves per SIMD instead of three
// hide more of each tile's stores and next-tile loads (5% per launch at c2).

// Offset bias (in floats) of a dropped buffer store: the buffer spans at most
// kDropBias floats, a valid offset within a tile (at most 64 items of
// rows_pad x nc, which the launcher checks) is below it, and one or two biases
// keep the byte offset (times 4) within 32 bits.
constexpr int kDropBias = 0x10000000;

template <typename T, int ROLE, int KCH, int INM, int OUTM>
__global__ __launch_bounds__(256, (sizeof(T) == 4 && INM == IN_RAW_T && OUTM == OUT_PACK) ? 4 : 1) void k_gemm_p2(GemmArgs a, int groups)
{
    using V = typename Vec16<T>::type;
    constexpr int VN = Vec16<T>::n;
    constexpr int KT = KCH * kTileK;   // K of a tile
    constexpr int LD = KT + VN;
    constexpr int PER = KT / 4;        // k per thread (4 thread groups per column)
    __shared__ __align__(16) T Ys[kTileN * LD];
    const int items = a.count ? min(*a.count, a.items) : a.items;
    const int ncols = items * a.nc;
    const int ntiles = (ncols + kTileN - 1) / kTileN;
    const int g = blockIdx.y;
    if (g >= ntiles) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int m0 = blockIdx.x * kTileM;
    const int nc = a.nc;
    const unsigned ncu = (unsigned)nc;
    using acc_t = typename Mfma<T>::acc_t;

    T af[KCH][8];
    {
        const T* A = static_cast<const T*>(a.A) + (size_t)(m0 + wave * 16 + li) * a.lda + 8 * lg;
#pragma unroll
        for (int c = 0; c < KCH; ++c) {
            const V* src = reinterpret_cast<const V*>(A + c * kTileK);
#pragma unroll
            for (int q = 0; q < 8 / VN; ++q) {
                const V w = src[q];
#pragma unroll
                for (int e = 0; e < VN; ++e) af[c][q * VN + e] = w[e];
            }
        }
    }
    // the lane's 4 output rows do not change from tile to tile
    int mrow[4], rowoff[4];
    T brow[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        mrow[v] = m0 + wave * 16 + Mfma<T>::row(lane, v);
        rowoff[v] = mrow[v] * nc;
        brow[v] = (a.bias && mrow[v] < a.rows) ? static_cast<const T*>(a.bias)[mrow[v]] : T(0);
    }
    const int step_q = 16 / nc, step_r = 16 - step_q * nc; // 16 columns on as (items, columns)
    const size_t item_stride = (size_t)a.rows_pad * nc;

    const int ynn = tid & 63, ykb = (tid >> 6) * PER;
    T ry[PER];
    auto load = [&](int ct) {
        if constexpr (INM == IN_LATENT) {
            const int yn = ct * kTileN + ynn;
#pragma unroll
            for (int q = 0; q < PER; ++q) ry[q] = T(0);
            if (yn < ncols) {
                const int yitem = (int)((unsigned)yn / ncu);
                const int yc = yn - yitem * nc;
                const long zr = a.zmap ? a.zmap[yitem] : yitem;
#pragma unroll
                for (int q = 0; q < PER; ++q) {
                    const int k = ykb + q;
                    if (k < a.K) ry[q] = (yc == 0) ? (T)a.z[zr * a.r + k] : ((k == yc - 1) ? T(1) : T(0));
                }
            }
        } else {
            // IN_RAW_T with K a multiple of the tile depth: one contiguous run.
            // Columns past the end load the last column (their products are
            // never stored), so the loads need no predicate.
            const int yn = min(ct * kTileN + ynn, ncols - 1);
            const int yitem = (int)((unsigned)yn / ncu);
            const int yc = yn - yitem * nc;
            const V* vp = reinterpret_cast<const V*>(static_cast<const T*>(a.Y) +
                                                     ((size_t)yitem * nc + yc) * a.y_rows + ykb);
#pragma unroll
            for (int q = 0; q < PER / VN; ++q) {
                const V w = vp[q];
#pragma unroll
                for (int e = 0; e < VN; ++e) ry[q * VN + e] = w[e];
            }
        }
    };
    auto store = [&]() {
        V* dy = reinterpret_cast<V*>(&Ys[ynn * LD + ykb]);
#pragma unroll
        for (int q = 0; q < PER / VN; ++q) {
            V w;
#pragma unroll
            for (int e = 0; e < VN; ++e) w[e] = ry[q * VN + e];
            dy[q] = w;
        }
    };

    T* Cout = static_cast<T*>(a.C);
    // Float32 packed output through raw buffer stores: an output past the last
    // row or column gets an offset the hardware drops instead of a branch, so
    // every thread issues exactly 16 stores on every tile, after the next
    // tile's activation loads, and the compiler's wait for those loads leaves
    // the stores in flight.
    constexpr bool BST = std::is_same<T, float>::value && OUTM == OUT_PACK;
    if constexpr (BST) {
        // the lane group's four bias values, in the padding of activation
        // column 4 wave + lg (never written by the tile fills)
        if (li == 0) {
            f32x4 bv;
#pragma unroll
            for (int v = 0; v < 4; ++v) bv[v] = brow[v];
            *reinterpret_cast<f32x4*>(&Ys[(wave * 4 + lg) * LD + KT]) = bv;
        }
    }
    load(g);
    // the first tile's activations, waited for here: at the loop's LDS fill the
    // only loads then pending are the prefetch, with this tile's stores after it
    if constexpr (BST) __builtin_amdgcn_s_waitcnt(0x0F70); // vmcnt(0)
    for (int ct = g; ct < ntiles; ct += groups) {
        // LDS-only barriers: the previous tile's output stores stay in flight
        lds_barrier(); // the previous tile's LDS reads are done
        store();
        lds_barrier();
        if (ct + groups < ntiles) load(ct + groups);
        acc_t acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int c = 0; c < KCH; ++c) {
            if constexpr (BST) {
                // one column tile's fragments at a time (8 registers, not 32):
                // the prefetch of the next tile stays in registers
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    T bt[8];
                    const V* sb = reinterpret_cast<const V*>(&Ys[(t * 16 + li) * LD + c * kTileK + 8 * lg]);
#pragma unroll
                    for (int q = 0; q < 8 / VN; ++q) {
                        const V w = sb[q];
#pragma unroll
                        for (int e = 0; e < VN; ++e) bt[q * VN + e] = w[e];
                    }
#pragma unroll
                    for (int kk = 0; kk < 8; ++kk) acc[t] = Mfma<T>::mac(af[c][kk], bt[kk], acc[t]);
                }
            } else {
                T bf[4][8];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const V* sb = reinterpret_cast<const V*>(&Ys[(t * 16 + li) * LD + c * kTileK + 8 * lg]);
#pragma unroll
                    for (int q = 0; q < 8 / VN; ++q) {
                        const V w = sb[q];
#pragma unroll
                        for (int e = 0; e < VN; ++e) bf[t][q * VN + e] = w[e];
                    }
                }
#pragma unroll
                for (int kk = 0; kk < 8; ++kk)
#pragma unroll
                    for (int t = 0; t < 4; ++t) acc[t] = Mfma<T>::mac(af[c][kk], bf[t][kk], acc[t]);
            }
        }
        if constexpr (OUTM == OUT_PACK) {
            // the lane's column n0 + 16 t as (item, cidx), stepped from t = 0;
            // full tiles (every row below rows, every column below ncols) store
            // without predicates
            const int n0 = ct * kTileN + li;
            const bool full = m0 + kTileM <= a.rows && (ct + 1) * kTileN <= ncols;
            int item = (int)((unsigned)n0 / ncu);
            int cidx = n0 - item * nc;
            if constexpr (BST) {
                // a raw buffer over the items from the tile's first one on, at
                // most 1 GiB (a tile's outputs lie within its first 64 items):
                // offsets past its end, and the biased ones, are dropped
                const int item0 = (int)((unsigned)(ct * kTileN) / ncu);
                const size_t ext = (size_t)(items - item0) * item_stride * sizeof(float);
                const f32x4 bv = *reinterpret_cast<const f32x4*>(&Ys[(wave * 4 + lg) * LD + KT]);
                const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
                    reinterpret_cast<float*>(Cout) + (size_t)item0 * item_stride, (short)0,
                    (int)(ext < (size_t)kDropBias * 4 ? ext : (size_t)kDropBias * 4), 0x00020000);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    if (t > 0) {
                        item += step_q;
                        cidx += step_r;
                        if (cidx >= nc) {
                            cidx -= nc;
                            ++item;
                        }
                    }
                    const int cb = (n0 + 16 * t < ncols) ? (item - item0) * (int)item_stride + cidx : kDropBias;
                    // rows m0 + r4 + v of this lane, r4 from the lane id (not kept live)
                    const int r4 = __builtin_amdgcn_readfirstlane(wave) * 16 + 4 * (__lane_id() >> 4);
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int ro = (m0 + r4 + v < a.rows) ? (m0 + r4 + v) * nc : kDropBias;
                        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(acc[t][v] + (cidx == 0 ? bv[v] : 0.f)),
                                                              rsrc, (int)((unsigned)(cb + ro) * 4u), 0, 0);
                    }
                }
                continue;
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (t > 0) {
                    item += step_q;
                    cidx += step_r;
                    if (cidx >= nc) {
                        cidx -= nc;
                        ++item;
                    }
                }
                T* base = Cout + (size_t)item * item_stride + cidx;
                if (full) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) base[rowoff[v]] = acc[t][v] + (cidx == 0 ? brow[v] : T(0));
                } else if (n0 + 16 * t < ncols) {
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (mrow[v] < a.rows) base[rowoff[v]] = acc[t][v] + (cidx == 0 ? brow[v] : T(0));
                }
            }
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int n = ct * kTileN + t * 16 + li;
                if (n >= ncols) continue;
                const int item = (int)((unsigned)n / ncu);
                const int cidx = n - item * nc;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int m = mrow[v];
                    if (m >= a.rows) continue;
                    const T val = acc[t][v] + (cidx == 0 ? brow[v] : T(0));
                    if (cidx == 0) {
                        if (a.Xo)
                            static_cast<T*>(a.Xo)[(size_t)item * a.rows + m] = static_cast<const T*>(a.Xrest)[m] + val;
                    } else if (a.Jo) {
                        static_cast<T*>(a.Jo)[((size_t)item * a.rows + m) * a.r + (cidx - 1)] = val;
                    }
                }
            }
        }
    }
}

// Persistent output map on the BF16 matrix cores at float32 accuracy (FP32
// accumulation and output): A is held as three BF16 planes (hi, mid, lo) of its
// float64 values, and the workgroup's 64 x K tile of each stays in registers as
// BF16 fragments; the transposed float32 activation tile is split into three
// BF16 parts on its way into LDS, and each 32-deep chunk is six 16x16x32 BF16
// MFMAs per 16-column tile (mfma_bf16x6_chunk).  Same tiling, prefetch and
// epilogue as k_gemm_p2.
// (three waves per SIMD at K <= 128: the register budget that keeps three
// workgroups' LDS tiles resident)
template <int ROLE, int KCH, int OUTM>
__global__ __launch_bounds__(256, KCH <= 4 ? 3 : 1) void k_gemm_p2_bf16(GemmArgs a, int groups)
{
    constexpr int KT = KCH * kTileK;
    constexpr int LD = KT + 8;   // BF16 elements per LDS row (16-byte pad)
    constexpr int PER = KT / 4;  // k per thread (4 thread groups per column)
    __shared__ __align__(16) __bf16 Ys[3][kTileN * LD];
    const int items = a.count ? min(*a.count, a.items) : a.items;
    const int ncols = items * a.nc;
    const int ntiles = (ncols + kTileN - 1) / kTileN;
    const int g = blockIdx.y;
    if (g >= ntiles) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int m0 = blockIdx.x * kTileM;
    const int nc = a.nc;
    const unsigned ncu = (unsigned)nc;

    bf16x8 af[KCH][3];
    {
        const size_t plane = (size_t)a.rows_pad * a.lda;
        const __bf16* A = static_cast<const __bf16*>(a.A) + (size_t)(m0 + wave * 16 + li) * a.lda + 8 * lg;
#pragma unroll
        for (int c = 0; c < KCH; ++c)
#pragma unroll
            for (int p = 0; p < 3; ++p) af[c][p] = *reinterpret_cast<const bf16x8*>(A + p * plane + c * kTileK);
    }
    int mrow[4];
    float brow[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        mrow[v] = m0 + wave * 16 + Mfma<float>::row(lane, v);
        brow[v] = (a.bias && mrow[v] < a.rows) ? static_cast<const float*>(a.bias)[mrow[v]] : 0.f;
    }

    const int ynn = tid & 63, ykb = (tid >> 6) * PER;
    f32x4 ry[PER / 4];
    auto load = [&](int ct) {
        // columns past the end load the last column (their products are never
        // stored), so the loads need no predicate
        const int yn = min(ct * kTileN + ynn, ncols - 1);
        const int yitem = (int)((unsigned)yn / ncu);
        const int yc = yn - yitem * nc;
        const f32x4* vp = reinterpret_cast<const f32x4*>(static_cast<const float*>(a.Y) +
                                                         ((size_t)yitem * nc + yc) * a.y_rows + ykb);
#pragma unroll
        for (int q = 0; q < PER / 4; ++q) ry[q] = vp[q];
    };
    auto store = [&]() {
#pragma unroll
        for (int q = 0; q < PER / 8; ++q) {
            bf16x8 h, m, l;
            split3_bf16(ry[2 * q], ry[2 * q + 1], h, m, l);
            reinterpret_cast<bf16x8*>(&Ys[0][ynn * LD + ykb])[q] = h;
            reinterpret_cast<bf16x8*>(&Ys[1][ynn * LD + ykb])[q] = m;
            reinterpret_cast<bf16x8*>(&Ys[2][ynn * LD + ykb])[q] = l;
        }
    };

    float* Cout = static_cast<float*>(a.C);
    load(g);
    // packed output leaves through buffer stores with a fixed count per tile
    // (as in k_gemm_p2): the first tile's loads are waited for here, so the
    // wait before each later LDS fill leaves the previous tile's stores in flight
    if constexpr (OUTM == OUT_PACK) __builtin_amdgcn_s_waitcnt(0x0F70); // vmcnt(0)
    for (int ct = g; ct < ntiles; ct += groups) {
        // LDS-only barriers: the previous tile's output stores stay in flight
        lds_barrier(); // the previous tile's LDS reads are done
        store();
        lds_barrier();
        if (ct + groups < ntiles) load(ct + groups);
        f32x4 acc[4], corr[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = corr[t] = f32x4{0, 0, 0, 0};
#pragma unroll
        for (int c = 0; c < KCH; ++c)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int off = (t * 16 + li) * LD + c * kTileK + 8 * lg;
                bf16x8 b[3];
#pragma unroll
                for (int p = 0; p < 3; ++p) b[p] = *reinterpret_cast<const bf16x8*>(&Ys[p][off]);
                mfma_bf16x6_chunk(af[c], b, acc[t], corr[t]);
            }
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] += corr[t];
        if constexpr (OUTM == OUT_PACK) {
            const size_t item_stride = (size_t)a.rows_pad * nc;
            const int item0 = (int)((unsigned)(ct * kTileN) / ncu);
            const size_t ext = (size_t)(items - item0) * item_stride * sizeof(float);
            const size_t cap = (size_t)kDropBias * sizeof(float);
            const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
                Cout + (size_t)item0 * item_stride, (short)0, (int)(ext < cap ? ext : cap), 0x00020000);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int n = ct * kTileN + t * 16 + li;
                const int item = (int)((unsigned)n / ncu);
                const int cidx = n - item * nc;
                const int cb = n < ncols ? (item - item0) * (int)item_stride + cidx : kDropBias;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int ro = mrow[v] < a.rows ? mrow[v] * nc : kDropBias;
                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(acc[t][v] + (cidx == 0 ? brow[v] : 0.f)),
                                                          rsrc, (int)((unsigned)(cb + ro) * 4u), 0, 0);
                }
            }
            continue;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int n = ct * kTileN + t * 16 + li;
            if (n >= ncols) continue;
            const int item = (int)((unsigned)n / ncu);
            const int cidx = n - item * nc;
            if constexpr (OUTM == OUT_PACK) {
                float* base = Cout + (size_t)item * a.rows_pad * nc + cidx;
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (mrow[v] < a.rows) base[(size_t)mrow[v] * nc] = acc[t][v] + (cidx == 0 ? brow[v] : 0.f);
            } else {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int m = mrow[v];
                    if (m >= a.rows) continue;
                    const float val = acc[t][v] + (cidx == 0 ? brow[v] : 0.f);
                    if (cidx == 0) {
                        if (a.Xo)
                            static_cast<float*>(a.Xo)[(size_t)item * a.rows + m] = static_cast<const float*>(a.Xrest)[m] + val;
                    } else if (a.Jo) {
                        static_cast<float*>(a.Jo)[((size_t)item * a.rows + m) * a.r + (cidx - 1)] = val;
                    }
                }
            }
        }
    }
}

hipError_t launch_gemm_p_bf16(int role, const GemmArgs& a, int target_blocks, hipStream_t s)
{
    if (a.items <= 0) return hipSuccess;
    if (a.in_mode != IN_RAW_T || a.K % kTileK != 0 || a.ksplit > 1) return hipErrorInvalidValue;
    if (a.out_mode == OUT_PACK && (size_t)a.rows_pad * a.nc * kTileN >= (size_t)kDropBias) return hipErrorInvalidValue;
    const int kch = a.K / kTileK;
    const int rt = a.rows_pad / kTileM;
    const int ntiles = (a.items * a.nc + kTileN - 1) / kTileN;
    int groups = (target_blocks + rt - 1) / rt;
    if (groups > ntiles) groups = ntiles;
    if (groups < 1) groups = 1;
    dim3 grid(rt, groups);
#define RS_PB(R, KC)                                                                                     \
    do {                                                                                                 \
        if (a.out_mode == OUT_PACK) RS_LAUNCH((k_gemm_p2_bf16<R, KC, OUT_PACK>), grid, dim3(256), 0, s, a, groups); \
        else RS_LAUNCH((k_gemm_p2_bf16<R, KC, OUT_SPLIT>), grid, dim3(256), 0, s, a, groups);            \
        return hipGetLastError();                                                                        \
    } while (0)
    if (role == ROLE_DECODE) {
        switch (kch) {
        case 1: RS_PB(ROLE_DECODE, 1);
        case 2: RS_PB(ROLE_DECODE, 2);
        case 4: RS_PB(ROLE_DECODE, 4);
        case 8: RS_PB(ROLE_DECODE, 8);
        default: return hipErrorInvalidValue;
        }
    }
    switch (kch) {
    case 1: RS_PB(ROLE_OUT, 1);
    case 2: RS_PB(ROLE_OUT, 2);
    case 4: RS_PB(ROLE_OUT, 4);
    case 8: RS_PB(ROLE_OUT, 8);
    default: return hipErrorInvalidValue;
    }
#undef RS_PB
}

template <typename T, int ROLE>
static hipError_t gemm_p_dispatch(const GemmArgs& a, int groups, hipStream_t s)
{
    const int kch = (a.K + kTileK - 1) / kTileK;
    dim3 grid(a.rows_pad / kTileM, groups);
    const size_t tile = (size_t)kTileN * (kch * kTileK + Vec16<T>::n) * sizeof(T);
    // fast variant: whole-K tiles, raw transposed input (K a multiple of 32) or latent input
    const bool fast_in = (a.in_mode == IN_RAW_T && a.K % kTileK == 0) || a.in_mode == IN_LATENT;
    if (tile <= 80 * 1024 && fast_in) { // gfx950: up to 160 KB of LDS per workgroup
#define RS_P2(KC)                                                                                         \
    do {                                                                                                  \
        if (a.in_mode == IN_LATENT) {                                                                     \
            if (a.out_mode == OUT_PACK)                                                                   \
                RS_LAUNCH((k_gemm_p2<T, ROLE, KC, IN_LATENT, OUT_PACK>), grid, dim3(256), 0, s, a, groups); \
            else                                                                                          \
                RS_LAUNCH((k_gemm_p2<T, ROLE, KC, IN_LATENT, OUT_SPLIT>), grid, dim3(256), 0, s, a, groups); \
        } else {                                                                                          \
            if (a.out_mode == OUT_PACK)                                                                   \
                RS_LAUNCH((k_gemm_p2<T, ROLE, KC, IN_RAW_T, OUT_PACK>), grid, dim3(256), 0, s, a, groups); \
            else                                                                                          \
                RS_LAUNCH((k_gemm_p2<T, ROLE, KC, IN_RAW_T, OUT_SPLIT>), grid, dim3(256), 0, s, a, groups); \
        }                                                                                                 \
        return hipGetLastError();                                                                         \
    } while (0)
        switch (kch) {
        case 1: RS_P2(1);
        case 2: RS_P2(2);
        case 4: RS_P2(4);
        default: break;
        }
#undef RS_P2
    }
    switch (kch) {
    case 1: RS_LAUNCH((k_gemm_p<T, ROLE, 1>), grid, dim3(256), 0, s, a, groups); break;
    case 2: RS_LAUNCH((k_gemm_p<T, ROLE, 2>), grid, dim3(256), 0, s, a, groups); break;
    case 4: RS_LAUNCH((k_gemm_p<T, ROLE, 4>), grid, dim3(256), 0, s, a, groups); break;
    case 8: RS_LAUNCH((k_gemm_p<T, ROLE, 8>), grid, dim3(256), 0, s, a, groups); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// persistent kernel for the output maps when K is a supported chunk count
bool gemm_p_fits(int f32, int K)
{
    const int kch = (K + kTileK - 1) / kTileK;
    return (kch == 1 || kch == 2 || kch == 4 || (kch == 8 && f32));
}

hipError_t launch_gemm_p(int f32, int role, const GemmArgs& a, int target_blocks, hipStream_t s)
{
    if (a.items <= 0) return hipSuccess;
    if (a.in_mode == IN_ELU || a.ksplit > 1) return hipErrorInvalidValue;
    const int rt = a.rows_pad / kTileM;
    const int ntiles = (a.items * a.nc + kTileN - 1) / kTileN;
    int groups = (target_blocks + rt - 1) / rt;
    if (groups > ntiles) groups = ntiles;
    if (groups < 1) groups = 1;
    if (f32) {
        // packed float32 output goes through buffer stores whose valid offsets
        // (within a tile's items) must stay below the drop bias
        if (a.out_mode == OUT_PACK && (size_t)a.rows_pad * a.nc * kTileN >= (size_t)kDropBias)
            return hipErrorInvalidValue;
        if (role == ROLE_DECODE) return gemm_p_dispatch<float, ROLE_DECODE>(a, groups, s);
        return gemm_p_dispatch<float, ROLE_OUT>(a, groups, s);
    }
    if (role == ROLE_DECODE) return gemm_p_dispatch<double, ROLE_DECODE>(a, groups, s);
    return gemm_p_dispatch<double, ROLE_OUT>(a, groups, s);
}

template <typename T>
static void gemm_dispatch(int role, dim3 grid, const GemmArgs& a, hipStream_t s)
{
    switch (role) {
    case ROLE_HIDDEN: RS_LAUNCH((k_gemm<T, ROLE_HIDDEN>), grid, dim3(256), 0, s, a); break;
    case ROLE_OUT: RS_LAUNCH((k_gemm<T, ROLE_OUT>), grid, dim3(256), 0, s, a); break;
    case ROLE_ADJ: RS_LAUNCH((k_gemm<T, ROLE_ADJ>), grid, dim3(256), 0, s, a); break;
    default: RS_LAUNCH((k_gemm<T, ROLE_DECODE>), grid, dim3(256), 0, s, a); break;
    }
}

// Adjoint product C[z] = A * Y over the K slice z for one-column items
// (IN_RAW, nc = 1, OUT_PACK): every global load of the workgroup's slice (KS
// 32-deep chunks) is issued at once, so its latency is paid once rather than
// once per chunk; the chunks then pass through a double-buffered LDS tile.
template <typename T, int KS>
__global__ __launch_bounds__(256) void k_gemm_adj(GemmArgs a)
{
    using V = typename Vec16<T>::type;
    constexpr int VN = Vec16<T>::n;
    constexpr int LD = kTileK + VN;
    __shared__ __align__(16) T As[2][kTileM * LD];
    __shared__ __align__(16) T Ys[2][kTileN * LD];
    const int items = a.count ? min(*a.count, a.items) : a.items;
    const int n0 = blockIdx.y * kTileN;
    if (n0 >= items) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int m0 = blockIdx.x * kTileM;
    const int kbeg = blockIdx.z * KS * kTileK, kend = min(a.K, kbeg + KS * kTileK);
    const T* A = static_cast<const T*>(a.A);
    const T* Y = static_cast<const T*>(a.Y);
    const int arow = tid >> 2, akq = (tid & 3) * 8;
    const int ynn = tid & 63, ykb = (tid >> 6) * 8;
    const bool ycol = n0 + ynn < items;
    V ra[KS][8 / VN], ry[KS][8 / VN];
#pragma unroll
    for (int c = 0; c < KS; ++c) {
        const int k0 = kbeg + c * kTileK;
        const bool in = k0 < kend; // K is a multiple of the chunk, so a chunk is whole or absent
        const V* sa = reinterpret_cast<const V*>(A + (size_t)(m0 + arow) * a.lda + (in ? k0 : 0) + akq);
        const V* sy = reinterpret_cast<const V*>(Y + (size_t)(ycol ? n0 + ynn : 0) * a.y_rows + (in ? k0 : 0) + ykb);
#pragma unroll
        for (int q = 0; q < 8 / VN; ++q) {
            ra[c][q] = sa[q];
            ry[c][q] = sy[q];
        }
    }
    using acc_t = typename Mfma<T>::acc_t;
    acc_t acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int c = 0; c < KS; ++c) {
        if (kbeg + c * kTileK >= kend) break;
        T* as = As[c & 1];
        T* ys = Ys[c & 1];
#pragma unroll
        for (int q = 0; q < 8 / VN; ++q) {
            reinterpret_cast<V*>(as + arow * LD + akq)[q] = ra[c][q];
            V w = ry[c][q];
            if (!ycol) w = V{};
            reinterpret_cast<V*>(ys + ynn * LD + ykb)[q] = w;
        }
        __syncthreads();
        T af[8], bf[4][8];
        {
            const V* sa = reinterpret_cast<const V*>(as + (wave * 16 + li) * LD + 8 * lg);
#pragma unroll
            for (int q = 0; q < 8 / VN; ++q) {
                const V w = sa[q];
#pragma unroll
                for (int e = 0; e < VN; ++e) af[q * VN + e] = w[e];
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const V* sb = reinterpret_cast<const V*>(ys + (t * 16 + li) * LD + 8 * lg);
#pragma unroll
                for (int q = 0; q < 8 / VN; ++q) {
                    const V w = sb[q];
#pragma unroll
                    for (int e = 0; e < VN; ++e) bf[t][q * VN + e] = w[e];
                }
            }
        }
#pragma unroll
        for (int kk = 0; kk < 8; ++kk)
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[t] = Mfma<T>::mac(af[kk], bf[t][kk], acc[t]);
    }
    T* Cout = static_cast<T*>(a.C) + blockIdx.z * a.split_stride;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int item = n0 + t * 16 + li;
        if (item >= items) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int m = m0 + wave * 16 + Mfma<T>::row(lane, v);
            if (m < a.rows) Cout[(size_t)item * a.rows_pad + m] = acc[t][v];
        }
    }
}

template <typename T>
static hipError_t gemm_adj_dispatch(const GemmArgs& a, dim3 grid, int ks, hipStream_t s)
{
    switch (ks) {
    case 1: RS_LAUNCH((k_gemm_adj<T, 1>), grid, dim3(256), 0, s, a); break;
    case 2: RS_LAUNCH((k_gemm_adj<T, 2>), grid, dim3(256), 0, s, a); break;
    case 3: RS_LAUNCH((k_gemm_adj<T, 3>), grid, dim3(256), 0, s, a); break;
    case 4: RS_LAUNCH((k_gemm_adj<T, 4>), grid, dim3(256), 0, s, a); break;
    case 5: RS_LAUNCH((k_gemm_adj<T, 5>), grid, dim3(256), 0, s, a); break;
    case 6: RS_LAUNCH((k_gemm_adj<T, 6>), grid, dim3(256), 0, s, a); break;
    case 7: RS_LAUNCH((k_gemm_adj<T, 7>), grid, dim3(256), 0, s, a); break;
    case 8: RS_LAUNCH((k_gemm_adj<T, 8>), grid, dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gemm(int f32, int role, const GemmArgs& a, hipStream_t s)
{
    if (a.items <= 0) return hipSuccess;
    const long ncols = (long)a.items * a.nc;
    dim3 grid(a.rows_pad / kTileM, (unsigned)((ncols + kTileN - 1) / kTileN), a.ksplit > 1 ? a.ksplit : 1);
    if (role == ROLE_ADJ && a.nc == 1 && a.in_mode == IN_RAW && a.out_mode == OUT_PACK && a.K % kTileK == 0 &&
        a.y_rows % 8 == 0 && a.lda % 8 == 0) {
        // the slice of a K split: the same chunk count as the generic kernel's
        const int ks = a.ksplit > 1 ? a.ksplit : 1;
        const int kchunk = ((a.K + ks - 1) / ks + kTileK - 1) / kTileK;
        if (kchunk <= 8) return f32 ? gemm_adj_dispatch<float>(a, grid, kchunk, s) : gemm_adj_dispatch<double>(a, grid, kchunk, s);
    }
    if (f32) gemm_dispatch<float>(role, grid, a, s);
    else gemm_dispatch<double>(role, grid, a, s);
    return hipGetLastError();
}

// f(integral_constant<int, I>) for I = 0 .. N-1, unrolled at compile time
template <int N, int I = 0, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<N, I + 1>(f);
    }
}

// Global store of one value in inline asm (a plain vector store).  The
// compiler does not count these among its outstanding vector-memory
// operations, so its own waits for loads count exactly (vector loads complete
// in order) instead of falling back to waiting for every store as well.
// Used only for results that the kernel never reads back.
template <typename T>
__device__ inline void global_store_asm(T* p, T v)
{
    if constexpr (sizeof(T) == 4)
        asm volatile("global_store_dword %0, %1, off" : : "v"(p), "v"(v) : "memory");
    else
        asm volatile("global_store_dwordx2 %0, %1, off" : : "v"(p), "v"(v) : "memory");
}

// The same store without a memory clobber: the compiler may move other
// memory operations across it (for results nothing in the kernel reads).
template <typename T>
__device__ inline void global_store_free(T* p, T v)
{
    if constexpr (sizeof(T) == 4)
        asm volatile("global_store_dword %0, %1, off" : : "v"(p), "v"(v));
    else
        asm volatile("global_store_dwordx2 %0, %1, off" : : "v"(p), "v"(v));
}

__device__ inline void global_store_free4(float* p, f32x4 v)
{
    asm volatile("global_store_dwordx4 %0, %1, off" : : "v"(p), "v"(v));
}


// ---------------------------------------------------------------------------
// Fused hidden layers.  A workgroup owns CT*16 columns holding whole items
// (IB = CT*16 / nc of them); their layer input lives in LDS as [column][k]
// (k contiguous), each wave owns RT*16 output rows.  Weights come straight
// from L2 into registers (8 consecutive k per lane, permuted-k MFMA order as
// in k_gemm), the next 32-deep chunk prefetched behind the MFMAs.  After a
// layer the pre-activations go to global memory as (nc x wrows) blocks per
// item and, activated, replace the LDS input of the next layer.
// ---------------------------------------------------------------------------
template <typename T, int CT, int RT, int NW, typename OP = T, int PF = 1>
__global__ __launch_bounds__(64 * NW) void k_mlp(MlpArgs a)
{
    // OP: type of the weights and of the MFMA operands (T, or BF16: weights as
    // three BF16 planes (hi, mid, lo) and the FP32 layer input split into three
    // BF16 parts as its fragments are read, six MFMAs per chunk at float32
    // accuracy; mfma_bf16x6_chunk)
    constexpr bool BF = std::is_same<OP, __bf16>::value;
    static_assert(!BF || std::is_same<T, float>::value, "BF16 operands accumulate in float");
    constexpr int NTH = 64 * NW; // NW waves of RT * 16 output rows each
    using V = typename Vec16<T>::type;
    constexpr int VN = Vec16<T>::n;
    constexpr int NP = CT * 16;
    extern __shared__ __align__(16) unsigned char mlp_smem[];
    T* Ys = reinterpret_cast<T*>(mlp_smem);
    const int nc = a.nc;
    const int IB = NP / nc;
    // rows of a column: every k of the layer-0 input and every (padded) output row
    const int LDY = max((a.r + kTileK - 1) / kTileK * kTileK, a.wrows) + VN;
    T* dact = Ys + NP * LDY;        // ELU'(a) of each (item, row) of the current layer
    T* bias_s = dact + IB * a.wrows; // every layer's bias (L x wrows), staged once
    const int items = a.count ? min(*a.count, a.items) : a.items;
    const int item0 = blockIdx.x * IB;
    if (item0 >= items) return;
    const int nitems = min(IB, items - item0);
    const int ncols = nitems * nc;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    using acc_t = typename Mfma<T>::acc_t;
    // item (within the workgroup) of each of this lane's columns, and whether it is a value column
    int icol[CT];
    bool vcol[CT];
#pragma unroll
    for (int t = 0; t < CT; ++t) {
        const int n = t * 16 + li;
        icol[t] = min(n / nc, IB - 1);
        vcol[t] = n < ncols && n == icol[t] * nc;
    }

    for (int e = tid; e < a.L * a.wrows; e += NTH) {
        const int l = e / a.wrows;
        bias_s[e] = static_cast<const T*>(a.b[l])[e - l * a.wrows];
    }
    // layer-0 input [z | I]
    {
        const int kp = (a.r + kTileK - 1) / kTileK * kTileK;
        for (int e = tid; e < NP * kp; e += NTH) {
            const int n = e / kp, k = e - n * kp;
            T v = T(0);
            if (n < ncols && k < a.r) {
                const int i = n / nc, c = n - i * nc;
                const long zr = a.zmap ? a.zmap[item0 + i] : item0 + i;
                v = (c == 0) ? (T)a.z[zr * a.r + k] : ((k == c - 1) ? T(1) : T(0));
            }
            Ys[n * LDY + k] = v;
        }
    }
    // Weights stream straight into registers in k-blocks of PF 32-deep chunks:
    // chunk u of a block is consumed, then its registers take chunk u of the
    // next block (the same layer's next k-block or the next layer's first),
    // so PF chunks are in flight behind the products.
    V wa[PF][RT][8 / VN];
    bf16x8 wb[PF][RT][BF ? 3 : 1];
    auto loadw = [&](int l, int k0, auto u) {
        const int lda = l == 0 ? a.lda0 : a.lda;
#pragma unroll
        for (int i = 0; i < RT; ++i) {
            const size_t off = (size_t)(wave * RT * 16 + i * 16 + li) * lda + k0 + 8 * lg;
            if constexpr (BF) {
                const size_t plane = (size_t)a.wrows * lda;
#pragma unroll
                for (int p = 0; p < 3; ++p)
                    wb[u][i][p] = *reinterpret_cast<const bf16x8*>(static_cast<const __bf16*>(a.W[l]) + p * plane + off);
            } else {
                const V* src = reinterpret_cast<const V*>(static_cast<const T*>(a.W[l]) + off);
#pragma unroll
                for (int q = 0; q < 8 / VN; ++q) wa[u][i][q] = src[q];
            }
        }
    };
    auto kpad = [&](int l) { return ((l == 0 ? a.r : a.w) + kTileK - 1) / kTileK * kTileK; };
    // chunks past the end of the weights re-read the last one (loads stay
    // unconditional, so no register merges wait on them)
    static_for<PF>([&](auto u) { loadw(0, min((int)u * kTileK, kpad(0) - kTileK), u); });
    for (int l = 0; l < a.L; ++l) {
        const int kp = kpad(l);
        lds_barrier();
        acc_t acc[RT][CT];
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
            for (int t = 0; t < CT; ++t) acc[i][t] = acc_t{0, 0, 0, 0};
        for (int kb = 0; kb < kp; kb += PF * kTileK) {
            // the k-block whose chunks replace this one's
            const bool same = kb + PF * kTileK < kp;
            const int nl = same ? l : min(l + 1, a.L - 1), nkb = same ? kb + PF * kTileK : 0;
            const int nkp = kpad(nl);
            static_for<PF>([&](auto u) {
                const int k0 = kb + u * kTileK;
                const int nk = min(nkb + (int)u * kTileK, nkp - kTileK);
                if (k0 >= kp) { // past this layer's end: the registers only take the next chunk
                    loadw(nl, nk, u);
                    return;
                }
                if constexpr (BF) {
                    bf16x8 ab[RT][3];
#pragma unroll
                    for (int i = 0; i < RT; ++i)
#pragma unroll
                        for (int p = 0; p < 3; ++p) ab[i][p] = wb[u][i][p];
                    loadw(nl, nk, u);
#pragma unroll
                    for (int t = 0; t < CT; ++t) {
                        const V* sb = reinterpret_cast<const V*>(Ys + (t * 16 + li) * LDY + k0 + 8 * lg);
                        const V x0 = sb[0], x1 = sb[1];
                        bf16x8 b[3];
                        split3_bf16(x0, x1, b[0], b[1], b[2]);
#pragma unroll
                        for (int i = 0; i < RT; ++i) mfma_bf16x6_chunk(ab[i], b, acc[i][t], acc[i][t]);
                    }
                } else {
                    T bf[CT][8];
#pragma unroll
                    for (int t = 0; t < CT; ++t) {
                        const V* sb = reinterpret_cast<const V*>(Ys + (t * 16 + li) * LDY + k0 + 8 * lg);
#pragma unroll
                        for (int q = 0; q < 8 / VN; ++q) {
                            const V w = sb[q];
#pragma unroll
                            for (int e = 0; e < VN; ++e) bf[t][q * VN + e] = w[e];
                        }
                    }
                    // k-step outermost: RT*CT independent accumulators between dependent MFMAs;
                    // the chunk's registers are refilled once its products are issued
#pragma unroll
                    for (int kk = 0; kk < 8; ++kk)
#pragma unroll
                        for (int t = 0; t < CT; ++t)
#pragma unroll
                            for (int i = 0; i < RT; ++i)
                                acc[i][t] = Mfma<T>::mac(wa[u][i][kk / VN][kk % VN], bf[t][kk], acc[i][t]);
                    loadw(nl, nk, u);
                }
            });
        }
        lds_barrier(); // every wave is done reading this layer's input
        // Activation [ELU(a) | ELU'(a) A] of the wave's own rows, straight
        // from the accumulators: a row's value and Jacobian columns all sit in
        // this wave, so ELU'(a) reaches the Jacobian columns through the wave's
        // own LDS rows (dact) with no workgroup barrier.  The pre-activations
        // go out as (nc x wrows) blocks per item.
        const int wr = a.wrows;
        T* pre = static_cast<T*>(a.pre[l]);
        T* pre_blk = pre ? pre + (size_t)item0 * nc * wr : nullptr;
        const T* bias_l = bias_s + l * wr;
        // value columns: bias, then ELU.  With Jacobian columns only a few
        // lanes hold value columns, so their pre-activations are parked in
        // dact and ELU, ELU' taken one (item, row) per lane, all lanes busy.
#pragma unroll
        for (int t = 0; t < CT; ++t) {
            if (!vcol[t]) continue;
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int m = wave * RT * 16 + rt * 16 + Mfma<T>::row(lane, v);
                    const T av = acc[rt][t][v] + bias_l[m];
                    acc[rt][t][v] = av;
                    if (nc > 1) dact[icol[t] * wr + m] = av;
                    else Ys[(t * 16 + li) * LDY + m] = T(elu0(av));
                }
        }
        if (nc > 1) {
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); // this wave's dact rows are written
            for (int e = lane; e < nitems * RT * 16; e += 64) {
                const int i = e / (RT * 16), m = wave * RT * 16 + (e - i * RT * 16);
                const T av = dact[i * wr + m];
                dact[i * wr + m] = T(elu1(av));
                Ys[i * nc * LDY + m] = T(elu0(av));
            }
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); // ELU' of the wave's rows is in dact
        }
#pragma unroll
        for (int t = 0; t < CT; ++t) {
            const int n = t * 16 + li;
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                const int mb = wave * RT * 16 + rt * 16;
                if (!vcol[t]) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int m = mb + Mfma<T>::row(lane, v);
                        Ys[n * LDY + m] = n < ncols ? dact[icol[t] * wr + m] * acc[rt][t][v] : T(0);
                    }
                }
                if (pre_blk && n < ncols) {
                    T* pp = pre_blk + (size_t)n * wr + mb;
                    if constexpr (std::is_same<T, float>::value) {
                        // rows 4 (lane / 16) + v: four consecutive rows
                        global_store_free4(pp + 4 * lg, f32x4{acc[rt][t][0], acc[rt][t][1], acc[rt][t][2], acc[rt][t][3]});
                    } else {
#pragma unroll
                        for (int v = 0; v < 4; ++v) global_store_free(pp + Mfma<T>::row(lane, v), acc[rt][t][v]);
                    }
                }
            }
        }
        lds_barrier(); // the layer's activation is complete
    }
    // activation out as (nc x wrows) per item: consecutive threads, consecutive rows
    T* act = static_cast<T*>(a.act) + (size_t)item0 * nc * a.wrows;
    for (int e = tid; e < ncols * a.wrows; e += NTH) {
        const int n = e / a.wrows, m = e - n * a.wrows;
        act[e] = Ys[n * LDY + m];
    }
}

constexpr size_t kMlpLds = 128 * 1024; // gfx950: up to 160 KB of LDS per workgroup

template <typename T, int CT, typename OP = T>
static hipError_t mlp_dispatch(const MlpArgs& a, hipStream_t s)
{
    const int np = CT * 16;
    const int ib = np / a.nc;
    if (ib < 1) return hipErrorInvalidValue;
    const int rt = a.wrows / 64;
    const int kr = (a.r + kTileK - 1) / kTileK * kTileK;
    const int ldy = (kr > a.wrows ? kr : a.wrows) + Vec16<T>::n;
    const size_t sh = ((size_t)np * ldy + (size_t)(ib + a.L) * a.wrows) * sizeof(T);
    if (sh > kMlpLds) return hipErrorInvalidValue;
    dim3 grid((a.items + ib - 1) / ib);
    // waves of 16 output rows (two rows tiles per wave at width 256); the
    // value-only variants (few products per chunk) keep a whole 128-deep
    // k-block of weights in flight
    constexpr int PF = CT == 1 ? 4 : 1;
    switch (rt) {
    case 1: RS_LAUNCH((k_mlp<T, CT, 1, 4, OP, CT == 1 ? 2 : 1>), grid, dim3(256), sh, s, a); break;
    case 2: RS_LAUNCH((k_mlp<T, CT, 1, 8, OP, PF>), grid, dim3(512), sh, s, a); break;
    case 4:
        // (float64 with five column tiles at this width exceeds the LDS budget)
        if constexpr (std::is_same<T, double>::value && CT == 5) return hipErrorInvalidValue;
        else RS_LAUNCH((k_mlp<T, CT, 2, 8, OP>), grid, dim3(512), sh, s, a);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// LDS bytes of the fused kernel with np columns (every layer's bias staged)
static size_t mlp_lds(int f32, int np, int nc, int r, int wrows)
{
    const int kr = (r + kTileK - 1) / kTileK * kTileK;
    const size_t ldy = (size_t)(kr > wrows ? kr : wrows) + (f32 ? 4 : 2);
    return (np * ldy + (size_t)(np / nc + kMaxL) * wrows) * (f32 ? 4 : 8);
}

// whether a column tile of np columns (16 CT) holds whole items and fits
static bool mlp_tile_ok(int f32, int np, int nc, int r, int wrows)
{
    // (float64 with five column tiles at width 256 exceeds the registers)
    if (!f32 && np == 80 && wrows / 64 == 4) return false;
    return np / nc >= 1 && mlp_lds(f32, np, nc, r, wrows) <= kMlpLds;
}

bool mlp_fits(int f32, int nc, int r, int wrows)
{
    const int rt = wrows / 64;
    if (!(rt == 1 || rt == 2 || rt == 4)) return false;
    if (nc == 1) return mlp_tile_ok(f32, 16, nc, r, wrows);
    return mlp_tile_ok(f32, 80, nc, r, wrows) || mlp_tile_ok(f32, 48, nc, r, wrows) ||
           mlp_tile_ok(f32, 32, nc, r, wrows);
}

template <typename T, typename OP = T>
static hipError_t mlp_dispatch_jac(const MlpArgs& a, int n_cu, hipStream_t s)
{
    // items per workgroup: the most of 4, 2, 1 that still gives every compute
    // unit two workgroups (a workgroup runs its layers on one compute unit;
    // a second one overlaps its products with the first one's activation
    // pass, and a small batch is spread thin rather than queued on a few);
    // then the narrowest column tile that holds them, or the widest that fits
    constexpr int f32 = std::is_same<T, float>::value;
    int ib = 4;
    while (ib > 1 && (a.items + ib - 1) / ib < 2 * n_cu) ib >>= 1;
    const int cols = ib * a.nc;
    int np = cols <= 32 ? 32 : cols <= 48 ? 48 : 80;
    while (np > 32 && !mlp_tile_ok(f32, np, a.nc, a.r, a.wrows)) np = np == 80 ? 48 : 32;
    if (np == 32 && !mlp_tile_ok(f32, 32, a.nc, a.r, a.wrows)) np = 48;
    if (np == 32) return mlp_dispatch<T, 2, OP>(a, s);
    if (np == 48) return mlp_dispatch<T, 3, OP>(a, s);
    return mlp_dispatch<T, 5, OP>(a, s);
}

hipError_t launch_mlp(int f32, const MlpArgs& a, hipStream_t s, int bf16, int n_cu)
{
    if (a.items <= 0 || a.L <= 0) return hipSuccess;
    if (bf16) {
        if (!f32) return hipErrorInvalidValue;
        return a.nc > 1 ? mlp_dispatch_jac<float, __bf16>(a, n_cu, s) : mlp_dispatch<float, 1, __bf16>(a, s);
    }
    if (a.nc > 1) return f32 ? mlp_dispatch_jac<float>(a, n_cu, s) : mlp_dispatch_jac<double>(a, n_cu, s);
    return f32 ? mlp_dispatch<float, 1>(a, s) : mlp_dispatch<double, 1>(a, s);
}

// [h | J] = [ELU(a) | ELU'(a) A] for every (item, row) of a pre-activation
// block, computed once before the output map reads it from every row tile.
template <typename T>
__global__ __launch_bounds__(256) void k_activate(const T* pre, T* act, int rows, int rows_pad, int nc,
                                                  int items_cap, const int* count)
{
    const int items = count ? min(*count, items_cap) : items_cap;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x; // (item, row)
    if (idx >= items * rows) return;
    const int item = idx / rows, m = idx - item * rows;
    const T* src = pre + ((size_t)item * rows_pad + m) * nc;
    T* dst = act + (size_t)item * nc * rows_pad + m;   // (nc x rows_pad) per item
    const T av = src[0];
    const T d = T(elu1(av));
    dst[0] = elu0(av);
    for (int c = 1; c < nc; ++c) dst[(size_t)c * rows_pad] = d * src[c];
}

hipError_t launch_activate(int f32, const void* pre, void* act, int rows, int rows_pad, int nc, int items_cap,
                           const int* count, hipStream_t s)
{
    if (items_cap <= 0) return hipSuccess;
    const long n = (long)items_cap * rows;
    dim3 grid((unsigned)((n + 255) / 256));
    if (f32)
        RS_LAUNCH(k_activate<float>, grid, dim3(256), 0, s, static_cast<const float*>(pre),
                           static_cast<float*>(act), rows, rows_pad, nc, items_cap, count);
    else
        RS_LAUNCH(k_activate<double>, grid, dim3(256), 0, s, static_cast<const double*>(pre),
                           static_cast<double*>(act), rows, rows_pad, nc, items_cap, count);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Stable Neo-Hookean density psi = mu/2 (I_C - 3) - mu (J - 1) + lam/2 (J - 1)^2
// evaluated in terms of the displacement gradient G = F - I, so that no term
// is a difference of O(1) numbers (float32 keeps its relative precision at
// small strain):
//   I_C - 3 = 2 tr G + |G|^2,   J - 1 = tr G + i2(G) + det G,
//   cof F = (1 + tr G) I - G^T + cof G,
//   psi = mu/2 |G|^2 - mu (i2(G) + det G) + lam/2 (J - 1)^2,
//   P = mu (G + G^T - tr G I - cof G) + lam (J - 1) cof F.
// vec index v = 3 j + i (column-major, G_ij); columns g_j of G, f_j of F.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Element kernel: one workgroup per item (or a run of its rounds, when a small
// batch splits items), RP lanes per cubature tet: lane k owns column k of
// K_e = dvecF/dz, or with RP == 8 (r == 16) columns k and k + 8.  The item's
// rows are streamed through a
// three-slot LDS ring by direct global->LDS loads (16 bytes per lane): one
// round is EPR tets (9 rows each), then EPR penalty targets (3 rows each);
// two rounds are in flight while one is used.
// Per tet: F, psi, PK1, (d2psi/dF2) K_e[:,k], H[:,k] += w V K_e^T (A K_e[:,k]),
// g[k] += w V K_e[:,k].P; then the penalty, gravity and force rows.
// Contributions are float64-accumulated and reduced in a fixed order.
// ---------------------------------------------------------------------------

// values staged per round: (tets per round) * 9 * (1 + r) at most; the
// two-column path (RP == 8, 32 tets a round, r <= 16) needs the larger tile
constexpr int kElemTile = 2880;
constexpr int kElemTile8 = 32 * 9 * 17;
constexpr int elem_tile(int rp) { return rp == 8 ? kElemTile8 : kElemTile; }

typedef const void __attribute__((address_space(1)))* gas_ptr;
typedef void __attribute__((address_space(3)))* las_ptr;

// s_waitcnt: at most N vector-memory operations outstanding and no LDS ones
template <int N>
__device__ inline void wait_vm_lgkm()
{
    static_assert(N >= 0 && N < 64, "vmcnt field");
    __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4));
}

// LDS reads and writes of the element ring in inline asm.  The compiler
// conservatively waits for every direct global->LDS load in flight before any
// LDS access it sees; these blocks are invisible to that analysis, so reading
// one ring slot does not wait for the loads filling the other two.  Each block
// waits for its own LDS operations before it ends (its results are complete
// when it returns); the ring's explicit vmcnt wait and barrier order them
// against the direct loads.
__device__ inline unsigned lds_addr(const void* p)
{
    return static_cast<unsigned>(reinterpret_cast<uintptr_t>((las_ptr)(const_cast<void*>(p))));
}

template <typename T>
__device__ inline void lds_read9(const T* p, int stride, T (&o)[9])
{
    const unsigned st = (unsigned)(stride * (int)sizeof(T));
    const unsigned a0 = lds_addr(p), a1 = a0 + st, a2 = a1 + st, a3 = a2 + st, a4 = a3 + st, a5 = a4 + st,
                   a6 = a5 + st, a7 = a6 + st, a8 = a7 + st;
    if constexpr (sizeof(T) == 4) {
        asm volatile("ds_read_b32 %0, %9\n\tds_read_b32 %1, %10\n\tds_read_b32 %2, %11\n\t"
                     "ds_read_b32 %3, %12\n\tds_read_b32 %4, %13\n\tds_read_b32 %5, %14\n\t"
                     "ds_read_b32 %6, %15\n\tds_read_b32 %7, %16\n\tds_read_b32 %8, %17\n\t"
                     "s_waitcnt lgkmcnt(0)"
                     : "=&v"(o[0]), "=&v"(o[1]), "=&v"(o[2]), "=&v"(o[3]), "=&v"(o[4]), "=&v"(o[5]), "=&v"(o[6]),
                       "=&v"(o[7]), "=&v"(o[8])
                     : "v"(a0), "v"(a1), "v"(a2), "v"(a3), "v"(a4), "v"(a5), "v"(a6), "v"(a7), "v"(a8)
                     : "memory");
    } else {
        asm volatile("ds_read_b64 %0, %9\n\tds_read_b64 %1, %10\n\tds_read_b64 %2, %11\n\t"
                     "ds_read_b64 %3, %12\n\tds_read_b64 %4, %13\n\tds_read_b64 %5, %14\n\t"
                     "ds_read_b64 %6, %15\n\tds_read_b64 %7, %16\n\tds_read_b64 %8, %17\n\t"
                     "s_waitcnt lgkmcnt(0)"
                     : "=&v"(o[0]), "=&v"(o[1]), "=&v"(o[2]), "=&v"(o[3]), "=&v"(o[4]), "=&v"(o[5]), "=&v"(o[6]),
                       "=&v"(o[7]), "=&v"(o[8])
                     : "v"(a0), "v"(a1), "v"(a2), "v"(a3), "v"(a4), "v"(a5), "v"(a6), "v"(a7), "v"(a8)
                     : "memory");
    }
}

template <typename T>
__device__ inline void lds_read3(const T* p, int stride, T (&o)[3])
{
    const unsigned st = (unsigned)(stride * (int)sizeof(T));
    const unsigned a0 = lds_addr(p), a1 = a0 + st, a2 = a1 + st;
    if constexpr (sizeof(T) == 4)
        asm volatile("ds_read_b32 %0, %3\n\tds_read_b32 %1, %4\n\tds_read_b32 %2, %5\n\ts_waitcnt lgkmcnt(0)"
                     : "=&v"(o[0]), "=&v"(o[1]), "=&v"(o[2])
                     : "v"(a0), "v"(a1), "v"(a2)
                     : "memory");
    else
        asm volatile("ds_read_b64 %0, %3\n\tds_read_b64 %1, %4\n\tds_read_b64 %2, %5\n\ts_waitcnt lgkmcnt(0)"
                     : "=&v"(o[0]), "=&v"(o[1]), "=&v"(o[2])
                     : "v"(a0), "v"(a1), "v"(a2)
                     : "memory");
}

// nine floats 17 apart (one column of nine rows of 17), and two such columns
// eight apart, from one address register with immediate offsets
__device__ inline void lds_read9_s17(const float* p, float (&o)[9])
{
    asm volatile("ds_read_b32 %0, %9\n\tds_read_b32 %1, %9 offset:68\n\tds_read_b32 %2, %9 offset:136\n\t"
                 "ds_read_b32 %3, %9 offset:204\n\tds_read_b32 %4, %9 offset:272\n\tds_read_b32 %5, %9 offset:340\n\t"
                 "ds_read_b32 %6, %9 offset:408\n\tds_read_b32 %7, %9 offset:476\n\tds_read_b32 %8, %9 offset:544\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(o[0]), "=&v"(o[1]), "=&v"(o[2]), "=&v"(o[3]), "=&v"(o[4]), "=&v"(o[5]), "=&v"(o[6]),
                   "=&v"(o[7]), "=&v"(o[8])
                 : "v"(lds_addr(p))
                 : "memory");
}

__device__ inline void lds_read18_s17(const float* p, float (&a)[9], float (&b)[9])
{
    asm volatile("ds_read_b32 %0, %18\n\tds_read_b32 %1, %18 offset:68\n\tds_read_b32 %2, %18 offset:136\n\t"
                 "ds_read_b32 %3, %18 offset:204\n\tds_read_b32 %4, %18 offset:272\n\tds_read_b32 %5, %18 offset:340\n\t"
                 "ds_read_b32 %6, %18 offset:408\n\tds_read_b32 %7, %18 offset:476\n\tds_read_b32 %8, %18 offset:544\n\t"
                 "ds_read_b32 %9, %18 offset:32\n\tds_read_b32 %10, %18 offset:100\n\tds_read_b32 %11, %18 offset:168\n\t"
                 "ds_read_b32 %12, %18 offset:236\n\tds_read_b32 %13, %18 offset:304\n\tds_read_b32 %14, %18 offset:372\n\t"
                 "ds_read_b32 %15, %18 offset:440\n\tds_read_b32 %16, %18 offset:508\n\tds_read_b32 %17, %18 offset:576\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(a[0]), "=&v"(a[1]), "=&v"(a[2]), "=&v"(a[3]), "=&v"(a[4]), "=&v"(a[5]), "=&v"(a[6]),
                   "=&v"(a[7]), "=&v"(a[8]), "=&v"(b[0]), "=&v"(b[1]), "=&v"(b[2]), "=&v"(b[3]), "=&v"(b[4]),
                   "=&v"(b[5]), "=&v"(b[6]), "=&v"(b[7]), "=&v"(b[8])
                 : "v"(lds_addr(p))
                 : "memory");
}

__device__ inline double lds_read_f64(const double* p)
{
    double o;
    asm volatile("ds_read_b64 %0, %1\n\ts_waitcnt lgkmcnt(0)" : "=&v"(o) : "v"(lds_addr(p)) : "memory");
    return o;
}

template <typename T, int RP>
struct ElemRing {
    static constexpr int VN = 16 / (int)sizeof(T);
    // direct loads per wave per round: the slot holds a round plus the
    // misalignment of its first value
    static constexpr int NI = (elem_tile(RP) + VN + 256 * VN - 1) / (256 * VN);
    static constexpr int SLOT = 256 * NI * VN; // values per slot
};

// Two-column element lanes (8 per tet): lane 8 t + c of a wave holds columns
// c and c + 8 of tet t, so a 16-lane row holds tets 2q and 2q + 1.  The MFMA
// operand of tet 2q (column j in lane j of the row) keeps lanes j < 8 and
// takes lanes j >= 8 from the second column of lane j - 8 (row shift right
// by 8, upper two banks); the operand of tet 2q + 1 keeps lanes j >= 8 and
// takes lanes j < 8 from the first column of lane j + 8 (row shift left by 8,
// lower two banks).
template <int CTRL, int BANKS>
__device__ inline float dpp_keep(float old, float src)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src), CTRL, 0xF, BANKS, false));
}
template <int CTRL, int BANKS>
__device__ inline double dpp_keep(double old, double src)
{
    const int ohi = __double2hiint(old), olo = __double2loint(old);
    const int shi = __double2hiint(src), slo = __double2loint(src);
    return __hiloint2double(__builtin_amdgcn_update_dpp(ohi, shi, CTRL, 0xF, BANKS, false),
                            __builtin_amdgcn_update_dpp(olo, slo, CTRL, 0xF, BANKS, false));
}
template <typename T>
__device__ inline T pair_even(T first, T second) { return dpp_keep<0x118, 0xC>(first, second); }
template <typename T>
__device__ inline T pair_odd(T first, T second) { return dpp_keep<0x108, 0x3>(second, first); }

// One tet of the two-column float32 element lanes (r == 16, rows of 17
// values: value, then the 16 Jacobian columns): lane 8 t + k of a wave holds
// columns k and k + 8 of tet t, whose nine rows start at `row` in LDS, and F,
// psi and P are formed once for both.  Adds wV K^T (d2psi/dF2) K to hsum (the
// 16x16 MFMA layout, summed over the wave's 8 tets), wV K[:,k].P and
// wV K[:,k+8].P to gk and gk2, and wV psi to Ee on lane k == 0; returns P.
// A lane with wV = 0 adds nothing (lanes past the end repeat a valid tet, so
// every lane runs the same code).
__device__ inline void tet_two_col(const float* row, int k, double wV, float mu, float lam, f32x4& hsum, double& gk,
                                   double& gk2, double& Ee, float (&P)[9])
{
    float gu[9], K0[9], K1[9];
    lds_read9_s17(row, gu);
    lds_read18_s17(row + 1 + k, K0, K1);
    Snh<float> m;
    m.set(gu, mu, lam);
    m.pk1(mu, lam, P);
    const float wt = (float)wV;
    float A0[9], A1[9];
    const float wmu = wt * mu, wlam = wt * lam, ws = wt * m.s;
    m.apply_hess_w(wmu, wlam, ws, K0, A0);
    m.apply_hess_w(wmu, wlam, ws, K1, A1);
    float gp0 = 0, gp1 = 0;
#pragma unroll
    for (int v = 0; v < 9; ++v) {
        gp0 += K0[v] * P[v];
        gp1 += K1[v] * P[v];
    }
    gk += wV * (double)gp0;
    gk2 += wV * (double)gp1;
    Ee += k == 0 ? wV * (double)m.psi : 0.0;
#pragma unroll
    for (int v = 0; v < 9; ++v) {
        hsum = Mfma<float>::mac(pair_even(K0[v], K1[v]), pair_even(A0[v], A1[v]), hsum);
        hsum = Mfma<float>::mac(pair_odd(K0[v], K1[v]), pair_odd(A0[v], A1[v]), hsum);
    }
}

template <typename T, int RP>
__global__ __launch_bounds__(256) void k_elem(ElemArgs a)
{
    constexpr int EPW = 64 / RP;   // tets (or targets) per wave per round
    constexpr int EPR = 4 * EPW;   // per round
    constexpr int VN = ElemRing<T, RP>::VN;
    constexpr int NI = ElemRing<T, RP>::NI;
    constexpr int SLOT = ElemRing<T, RP>::SLOT;
    // side inputs per round: wV of its tets (2 EPR words), or the rest
    // positions and targets of its targeted vertices (12 EPR words)
    constexpr int NS = (12 * EPR + 255) / 256; // direct 4-byte loads per wave per round
    constexpr int SIDEW = 256 * NS;            // words per side slot
    __shared__ __align__(16) T ring0[SLOT];
    __shared__ __align__(16) T ring1[SLOT];
    __shared__ __align__(16) T ring2[SLOT];
    __shared__ __align__(16) double side0[SIDEW / 2], side1[SIDEW / 2], side2[SIDEW / 2];
    const int item = blockIdx.x / a.parts, part = blockIdx.x - item * a.parts;
    if (a.count && item >= *a.count) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int eg = lane / RP, k = lane % RP;
    const int r = a.r, nc = a.nc;
    const bool kact = k < r;
    const bool kact2 = RP == 8 && k + 8 < r; // second column of the two-column path
    const T* O = static_cast<const T*>(a.out) + (size_t)item * a.rows_pad * nc;
    T* dseed = a.dseed ? static_cast<T*>(a.dseed) + (size_t)item * a.rows_pad : nullptr;
    const int bidx = a.imap ? a.imap[item] : item;
    const T mu = (T)a.mu, lam = (T)a.lam;
    const bool ext = !a.elastic_only;
    const int prow = 9 * a.S;
    const double* tg = (ext && a.targets) ? a.targets + (size_t)bidx * a.nt * 3 : nullptr;
    const double kc = a.k_c;
    const int el = wave * EPW + eg;

    double Hc[RP];  // column layout: lane (tet, k) holds H[0..r)[k] (VALU path)
#pragma unroll
    for (int j = 0; j < RP; ++j) Hc[j] = 0.0;
    double Hm[4] = {0.0, 0.0, 0.0, 0.0}; // MFMA result layout (RP == 16 and 8 paths)
    // the MFMA paths accumulate H on the matrix cores across all of the
    // wave's rounds (4 tets or targets per MFMA step), in T; Hm takes it at the end
    constexpr bool MF = RP == 16 || RP == 8;
    typename Mfma<T>::acc_t hsum = {0, 0, 0, 0};
    double gk = 0.0, gk2 = 0.0, Ee = 0.0;

    const int span = 9 * nc;
    const int tet_rounds = (a.S + EPR - 1) / EPR;
    const int pen_rounds = tg ? (a.nt + EPR - 1) / EPR : 0;
    const int rounds = tet_rounds + pen_rounds;
    // this workgroup's run of the item's rounds
    const int per = (rounds + a.parts - 1) / a.parts;
    const int rbeg = min(rounds, part * per), rend = min(rounds, rbeg + per);
    // value range [v0, v1) of round rd within the item block
    auto range = [&](int rd, int& v0, int& v1) {
        if (rd < tet_rounds) {
            const int s0 = rd * EPR;
            v0 = s0 * span;
            v1 = min(a.S, s0 + EPR) * span;
        } else {
            const int t0 = (rd - tet_rounds) * EPR;
            v0 = (prow + 3 * t0) * nc;
            v1 = (prow + 3 * min(a.nt, t0 + EPR)) * nc;
        }
    };
    auto ring_of = [&](auto sl) -> T* {
        constexpr int S = decltype(sl)::value;
        if constexpr (S == 0) return ring0;
        else if constexpr (S == 1) return ring1;
        else return ring2;
    };
    auto side_of = [&](auto sl) -> double* {
        constexpr int S = decltype(sl)::value;
        if constexpr (S == 0) return side0;
        else if constexpr (S == 1) return side1;
        else return side2;
    };
    // Every wave issues exactly NI direct loads per round (lanes past the
    // range re-load its first vector into the unused tail of the slot), so the
    // vmcnt bookkeeping below holds for the ring's own loads.
    // The side inputs of the round (wV, or rest positions then targets, as
    // 4-byte words) go to the slot's side area the same way, NS loads per wave.
    auto issue = [&](auto sl, int rd) {
        int v0, v1;
        range(rd, v0, v1);
        const int a0 = v0 & ~(VN - 1);
        const int nvec = (v1 - a0 + VN - 1) / VN; // >= 1; the block has >= 4 rows past the penalty rows
        T* slot = ring_of(sl);
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int vb = (wave * NI + i) * 64;
            const int vi = min(vb + lane, nvec - 1);
            __builtin_amdgcn_global_load_lds((gas_ptr)(O + a0 + (size_t)vi * VN), (las_ptr)(slot + (size_t)vb * VN),
                                             16, 0, 0);
        }
        if (rd < tet_rounds) {
            const int s0 = rd * EPR;
            const uint32_t* w = reinterpret_cast<const uint32_t*>(a.wV);
#pragma unroll
            for (int i = 0; i < NS; ++i) {
                const int wb = (wave * NS + i) * 64;
                const int j = min(2 * s0 + wb + lane, 2 * a.S - 1);
                __builtin_amdgcn_global_load_lds((gas_ptr)(w + j), (las_ptr)(reinterpret_cast<uint32_t*>(side_of(sl)) + wb),
                                                 4, 0, 0);
            }
        } else {
            const int t0 = (rd - tet_rounds) * EPR;
            const uint32_t* xw = reinterpret_cast<const uint32_t*>(a.Xt + 3 * t0);
            const uint32_t* tw = reinterpret_cast<const uint32_t*>(tg + 3 * t0);
            const int nw = 6 * (a.nt - t0); // words left in each array
#pragma unroll
            for (int i = 0; i < NS; ++i) {
                const int wb = (wave * NS + i) * 64;
                const int j = wb + lane;
                const uint32_t* g = j < 6 * EPR ? xw + min(j, nw - 1) : tw + min(j - 6 * EPR, nw - 1);
                __builtin_amdgcn_global_load_lds((gas_ptr)g, (las_ptr)(reinterpret_cast<uint32_t*>(side_of(sl)) + wb),
                                                 4, 0, 0);
            }
        }
    };
    // one round read from slot SL; round rd + 2 is issued into slot SL + 2
    auto body = [&](auto sl, int rd) {
        constexpr int SL = decltype(sl)::value;
        using NextSlot = std::integral_constant<int, (SL + 2) % 3>;
        // Round rd has landed once at most NI + NS vector-memory operations
        // are outstanding: loads complete in order, and round rd + 1's
        // NI + NS loads were issued after round rd's (the stores in between
        // can only lower the count).  The barrier then makes every wave's part
        // visible and frees the slot of round rd - 1.
        if (rd + 1 < rend)
            wait_vm_lgkm<NI + NS>();
        else
            wait_vm_lgkm<0>();
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        if (rd + 2 < rend) issue(NextSlot{}, rd + 2);
        int v0, v1;
        range(rd, v0, v1);
        const T* tile = ring_of(sl) + (v0 - (v0 & ~(VN - 1)));
        const double* sd = side_of(sl);
        if (rd < tet_rounds) {
            const int s = rd * EPR + el;
            if constexpr (RP == 16) {
                // Gauss-Newton block on the matrix cores: lanes (tet eg, column k)
                // hold K_e[v][k] and wV (A K_e)[v][k], exactly the A / B operands of
                // a 16x16x4 MFMA whose 4-deep reduction runs over the wave's 4 tets.
                T Kc[9], AK[9];
#pragma unroll
                for (int v = 0; v < 9; ++v) {
                    Kc[v] = T(0);
                    AK[v] = T(0);
                }
                if (s < a.S) {
                    const T* row = tile + el * span;
                    T gu[9], kr[9];
                    lds_read9(row, nc, gu);
                    lds_read9(row + 1 + (kact ? k : 0), nc, kr);
#pragma unroll
                    for (int v = 0; v < 9; ++v) Kc[v] = kact ? kr[v] : T(0);
                    Snh<T> m;
                    m.set(gu, mu, lam);
                    T P[9];
                    m.pk1(mu, lam, P);
                    m.apply_hess(mu, lam, Kc, AK);
                    const double wV = lds_read_f64(sd + el);
                    T gp = 0;
#pragma unroll
                    for (int v = 0; v < 9; ++v) gp += Kc[v] * P[v];
                    gk += wV * (double)gp;
                    Ee += k == 0 ? wV * (double)m.psi : 0.0;
                    const T wt = (T)wV;
                    if (dseed) {
                        // lane k < 9 writes seed v = k (a select chain keeps P in registers)
                        T pv = P[0];
#pragma unroll
                        for (int v = 1; v < 9; ++v) pv = k == v ? P[v] : pv;
                        if (k < 9) global_store_asm(dseed + 9 * s + k, wt * pv);
                    }
#pragma unroll
                    for (int v = 0; v < 9; ++v) AK[v] *= wt;
                }
#pragma unroll
                for (int v = 0; v < 9; ++v) hsum = Mfma<T>::mac(Kc[v], AK[v], hsum);
            } else if constexpr (RP == 8) {
                // r == 16 (rows of 17 values): lane c holds columns c and c + 8,
                // and F, psi and P are formed once for both.  A lane past the
                // end of S repeats the round's last tet with weight zero, so
                // every lane runs the same code and adds nothing.
                const bool sok = s < a.S;
                const int elc = sok ? el : a.S - 1 - rd * EPR;
                const double wv = lds_read_f64(sd + el);
                const double wV = sok ? wv : 0.0;
                T P[9];
                tet_two_col(tile + elc * (9 * 17), k, wV, mu, lam, hsum, gk, gk2, Ee, P);
                const T wt = (T)wV;
                if (dseed && sok) {
                    // lane c writes seed c; lane 0 also seed 8
                    T pv = P[0];
#pragma unroll
                    for (int v = 1; v < 8; ++v) pv = k == v ? P[v] : pv;
                    global_store_asm(dseed + 9 * s + k, wt * pv);
                    if (k == 0) global_store_asm(dseed + 9 * s + 8, wt * P[8]);
                }
            } else if (s < a.S) {
                const T* row = tile + el * span;
                T gu[9], Kc[9];
#pragma unroll
                for (int v = 0; v < 9; ++v) {
                    gu[v] = row[v * nc];
                    Kc[v] = kact ? row[v * nc + 1 + k] : T(0);
                }
                Snh<T> m;
                m.set(gu, mu, lam);
                T P[9], AK[9];
                m.pk1(mu, lam, P);
                m.apply_hess(mu, lam, Kc, AK);
                const double wV = sd[el];
#pragma unroll
                for (int j = 0; j < RP; ++j) {
                    if (j < r) {
                        T h = 0;
#pragma unroll
                        for (int v = 0; v < 9; ++v) h += row[v * nc + 1 + j] * AK[v];
                        Hc[j] += wV * (double)h;
                    }
                }
                T gp = 0;
#pragma unroll
                for (int v = 0; v < 9; ++v) gp += Kc[v] * P[v];
                gk += wV * (double)gp;
                if (k == 0) Ee += wV * (double)m.psi;
                if (dseed) {
#pragma unroll
                    for (int v = 0; v < 9; ++v)
                        if (v % RP == k) dseed[9 * s + v] = (T)(wV * (double)P[v]);
                }
            }
        } else {
            // penalty k_c/2 |x_t - target_t|^2 of EPR targeted vertices
            const int t = (rd - tet_rounds) * EPR + el;
            const bool ok = t < a.nt;
            const T* row = tile + 3 * el * nc;
            T Jc[3], J2[3] = {T(0), T(0), T(0)};
            double d[3];
            if constexpr (MF) {
                T jr[3], xv[3];
                double xr[3], tr[3];
                lds_read3(row, nc, xv);
                lds_read3(row + 1 + (kact ? k : 0), nc, jr);
                if constexpr (RP == 8) {
                    T jr2[3];
                    lds_read3(row + 1 + (kact2 ? k + 8 : 0), nc, jr2);
#pragma unroll
                    for (int c = 0; c < 3; ++c) J2[c] = (ok && kact2) ? jr2[c] : T(0);
                }
                lds_read3(sd + 3 * el, 1, xr);
                lds_read3(sd + 3 * EPR + 3 * el, 1, tr);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    Jc[c] = (ok && kact) ? jr[c] : T(0);
                    d[c] = ok ? xr[c] + (double)xv[c] - tr[c] : 0.0;
                }
            } else {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    Jc[c] = (ok && kact) ? row[c * nc + 1 + k] : T(0);
                    d[c] = ok ? sd[3 * el + c] + (double)row[c * nc] - sd[3 * EPR + 3 * el + c] : 0.0;
                }
            }
            if constexpr (RP == 16) {
                const T kt = (T)kc;
#pragma unroll
                for (int c = 0; c < 3; ++c) hsum = Mfma<T>::mac(Jc[c], kt * Jc[c], hsum);
            } else if constexpr (RP == 8) {
                const T kt = (T)kc;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const T pe = pair_even(Jc[c], J2[c]), po = pair_odd(Jc[c], J2[c]);
                    hsum = Mfma<T>::mac(pe, kt * pe, hsum);
                    hsum = Mfma<T>::mac(po, kt * po, hsum);
                }
            }
            if (ok) {
                if constexpr (!MF) {
#pragma unroll
                    for (int j = 0; j < RP; ++j) {
                        if (j < r) {
                            T h = 0;
#pragma unroll
                            for (int c = 0; c < 3; ++c) h += row[c * nc + 1 + j] * Jc[c];
                            Hc[j] += kc * (double)h;
                        }
                    }
                }
                gk += kc * ((double)Jc[0] * d[0] + (double)Jc[1] * d[1] + (double)Jc[2] * d[2]);
                if constexpr (RP == 8) gk2 += kc * ((double)J2[0] * d[0] + (double)J2[1] * d[1] + (double)J2[2] * d[2]);
                Ee += k == 0 ? 0.5 * kc * (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) : 0.0;
                if (dseed && k < 3) {
                    const double dv = k == 0 ? d[0] : k == 1 ? d[1] : d[2];
                    global_store_asm(dseed + prow + 3 * t + k, (T)(kc * dv));
                }
            }
        }
    };

    if (rend > rbeg) issue(std::integral_constant<int, 0>{}, rbeg);
    if (rend > rbeg + 1) issue(std::integral_constant<int, 1>{}, rbeg + 1);
    for (int rd = rbeg; rd < rend; rd += 3) {
        body(std::integral_constant<int, 0>{}, rd);
        if (rd + 1 < rend) body(std::integral_constant<int, 1>{}, rd + 1);
        if (rd + 2 < rend) body(std::integral_constant<int, 2>{}, rd + 2);
    }

    if (ext && part == 0 && wave == 0 && eg == 0) {
        const size_t gr = (size_t)a.grav_row;
        gk -= kact ? (double)O[gr * nc + 1 + k] : 0.0;
        gk2 -= kact2 ? (double)O[gr * nc + 9 + k] : 0.0;
        if (k == 0) Ee -= (double)O[gr * nc];
        if (a.force && a.nf) {
            const double* f = a.force + (size_t)bidx * 3;
            for (int c = 0; c < 3; ++c) {
                const size_t fr = (size_t)(a.force_row + c);
                gk -= kact ? f[c] * (double)O[fr * nc + 1 + k] : 0.0;
                gk2 -= kact2 ? f[c] * (double)O[fr * nc + 9 + k] : 0.0;
                if (k == 0) Ee -= f[c] * (double)O[fr * nc];
            }
        }
    }
    if (dseed && part == 0) {
        // rows not written above: penalty rows without targets, gravity,
        // force and padding rows
        for (int row = prow + tid; row < a.rows_pad; row += 256) {
            double v = 0.0;
            if (row < a.grav_row) {
                if (tg) continue;
            } else if (row == a.grav_row) {
                v = ext ? -1.0 : 0.0;
            } else if (row < a.force_row + 3) {
                v = (ext && a.force && a.nf) ? -a.force[(size_t)bidx * 3 + (row - a.force_row)] : 0.0;
            }
            dseed[row] = (T)v;
        }
    }

    if constexpr (MF) {
#pragma unroll
        for (int q = 0; q < 4; ++q) Hm[q] = (double)hsum[q];
    }
    // reduce over the EPW tets of a wave (lanes k, k+RP, ...), then over the
    // waves in order: wave 0 keeps the running sum, waves 1..3 pass theirs
    // through the (now idle) first ring slot in turn
#pragma unroll
    for (int off = RP; off < 64; off <<= 1) {
        if constexpr (RP != 16) {
#pragma unroll
            for (int j = 0; j < RP; ++j) Hc[j] += __shfl_xor(Hc[j], off);
        }
        gk += __shfl_xor(gk, off);
        if constexpr (RP == 8) gk2 += __shfl_xor(gk2, off);
        Ee += __shfl_xor(Ee, off);
    }
    // [HN] H (MFMA layout on the MFMA paths), [GN] g, [1] E
    constexpr int HN = MF ? 256 : RP * RP, GN = RP == 8 ? 16 : RP;
    double* red = reinterpret_cast<double*>(ring0);
    static_assert((HN + GN + 1) * sizeof(double) <= SLOT * sizeof(T), "reduction fits one slot");
    for (int w = 1; w < 4; ++w) {
        __syncthreads();
        if (wave == w) {
            if constexpr (MF) {
#pragma unroll
                for (int q = 0; q < 4; ++q) red[q * 64 + lane] = Hm[q];
            } else if (eg == 0) {
#pragma unroll
                for (int j = 0; j < RP; ++j) red[j * RP + k] = Hc[j];
            }
            if (eg == 0) red[HN + k] = gk;
            if constexpr (RP == 8)
                if (eg == 0) red[HN + 8 + k] = gk2;
            if (lane == 0) red[HN + GN] = Ee;
        }
        __syncthreads();
        if (wave == 0) {
            if constexpr (MF) {
#pragma unroll
                for (int q = 0; q < 4; ++q) Hm[q] += red[q * 64 + lane];
            } else {
#pragma unroll
                for (int j = 0; j < RP; ++j) Hc[j] += red[j * RP + k];
            }
            gk += red[HN + k];
            if constexpr (RP == 8) gk2 += red[HN + 8 + k];
            Ee += red[HN + GN];
        }
    }
    if (wave == 0) {
        const size_t slot = (size_t)part * a.part_stride + item; // = item with one part
        if constexpr (MF) {
            if (a.H) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int j = Mfma<T>::row(lane, q), kk = lane & 15;
                    if (j < r && kk < r) a.H[slot * r * r + j * r + kk] = Hm[q];
                }
            }
        } else if (eg == 0 && kact && a.H) {
#pragma unroll
            for (int j = 0; j < RP; ++j)
                if (j < r) a.H[slot * r * r + j * r + k] = Hc[j];
        }
        if (eg == 0 && kact && a.g) a.g[slot * r + k] = gk;
        if (eg == 0 && kact2 && a.g) a.g[slot * r + k + 8] = gk2;
        if (lane == 0 && a.E) a.E[item] = Ee;
    }
}

hipError_t launch_elem(int f32, const ElemArgs& a, int items, hipStream_t s)
{
    if (items <= 0) return hipSuccess;
    if (a.parts > 1 && (a.E || a.part_stride < items)) return hipErrorInvalidValue;
    ElemArgs b = a;
    if (b.parts < 1) b.parts = 1;
    // r <= 16: the MFMA paths (FP32 with r == 16: 8 lanes per tet with two
    // columns each, 32 tets a round; otherwise 16 lanes per tet); r <= 32: 32
    // lanes per tet (VALU);
    // r == 0 (value rows only: energy and adjoint seeds): 4 lanes per tet, 64 tets a round
    const int rp = a.r == 0 ? 4 : (f32 && a.r == 16) ? 8 : a.r <= 16 ? 16 : 32;
    // one round's tile must fit the staging buffer and the prefetch registers
    if ((256 / rp) * 9 * a.nc > elem_tile(rp) || (rp == 8 && a.nc != 17)) return hipErrorInvalidValue;
    dim3 grid(items * b.parts), block(256);
#define RS_ELEM(T, RP) RS_LAUNCH((k_elem<T, RP>), grid, block, 0, s, b)
    if (f32) {
        switch (rp) {
        case 4: RS_ELEM(float, 4); break;
        case 8: RS_ELEM(float, 8); break;
        case 16: RS_ELEM(float, 16); break;
        default: RS_ELEM(float, 32); break;
        }
    } else {
        switch (rp) {
        case 4: RS_ELEM(double, 4); break;
        case 16: RS_ELEM(double, 16); break;
        default: RS_ELEM(double, 32); break;
        }
    }
#undef RS_ELEM
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Output map and element physics in one kernel (BF16 context, r == 16).  The
// rows of J_R = W_big [h | J_h] + [b | 0] (Sec. 4.3: the cubature tets' F and
// the penalty, gravity and force rows, each with its 16 Jacobian columns) are
// formed in LDS just before the element physics reads them, so J_R never goes
// through HBM.
// A workgroup takes a group of four items (and, when the batch is small, a
// part of their rows).  Its LDS holds the group's activation columns (64
// Jacobian columns, 4 value columns and a zero column) split once into three
// BF16 planes, for the whole run.  The rows come in chunks of 16 tets (144
// rows: nine 16-row tiles), then the rows past the tets in chunks of up to
// nine tiles.  Per chunk:
//  * wave w forms the row tiles t = w - ch (mod 4), t + 4, t + 8 (so the SIMDs
//    take the ninth tile in turn) as five 16x16 output tiles each (tile j < 4:
//    the Jacobian columns of item j; tile 4: the four value columns), by
//    six-product BF16 MFMAs over K: A, the three BF16 planes of W_big, from L2
//    straight into registers, two row tiles at a time; B from the LDS planes,
//    each fragment read once for both;
//  * the element physics runs in two passes of two items (the LDS holds the
//    rows of two items): the outputs of items 0 and 1 go to LDS, those of items
//    2 and 3 stay in registers until the first pass is done.  In a pass, waves
//    2s and 2s + 1 take item s of the pair, eight tets each, with the
//    two-column lanes of the float32 element kernel (H on the FP32 matrix
//    cores, folded into float64 per pass).
// At the end the two waves' sums of each item are added in wave order.
// Outputs as the element kernel's: E, g, H (or per-part partials), and the
// adjoint seeds dE/d(row value).
// ---------------------------------------------------------------------------
constexpr int kFuseG = 4;                           // items per workgroup
constexpr int kFuseTets = 16;                       // tets per chunk
constexpr int kFuseRows = 9 * kFuseTets;            // rows per chunk (nine 16-row tiles)
constexpr int kFuseCols = 16 * kFuseG + kFuseG + 1; // LDS columns: Jacobian, values, zeros

bool elem_fused_fits(int r, int K) { return r == 16 && K > 0 && K % kTileK == 0 && K <= 4 * kTileK; }

int elem_fused_parts(int bf16, int cap, int n_cu)
{
    // at least the workgroups that fit a compute unit at once on each (two BF16 kernels of four
    // waves, one float32 kernel of eight), at most eight parts
    const int groups = (cap + kFuseG - 1) / kFuseG;
    if (groups <= 0) return 1;
    const int want = (bf16 ? 2 : 1) * n_cu;
    return std::max(1, std::min(8, (want + groups - 1) / groups));
}

// Element physics of one item on one chunk of its rows in LDS (rows of 17
// values from Jw: the chunk's 16 tets, or for a chunk past the tets its
// penalty targets and the gravity and force rows), on the two-column lanes of
// one wave: tets (targets) r0 + rs q + eg of the chunk, q = 0, 1, ...; the
// gravity and force rows on the wave with r0 == 0.  H goes to hs (float32,
// matrix-core layout), g and E to the lanes' float64 sums, the adjoint seeds
// to memory.
__device__ inline void fused_item_chunk(const ElemArgs& e, const float* Jw, int item, bool tail, int ch, int ntc,
                                        int row0, int nrows, int r0, int rs, int eg, int k, f32x4& hs, double& gk,
                                        double& gk2, double& Ee)
{
    const float mu = (float)e.mu, lam = (float)e.lam;
    const bool ext = !e.elastic_only;
    const double kc = e.k_c;
    const int prow = 9 * e.S;
    const int bidx = e.imap ? e.imap[item] : item;
    float* dseed = e.dseed ? static_cast<float*>(e.dseed) + (size_t)item * e.rows_pad : nullptr;
    if (!tail) {
        const int s0 = kFuseTets * ch, ns = min(kFuseTets, e.S - s0);
        for (int q = 0; r0 + rs * q < ns; ++q) {
            const int sl = r0 + rs * q + eg;
            const bool sok = sl < ns;
            const int slc = sok ? sl : ns - 1;
            const double wV = sok ? e.wV[s0 + sl] : 0.0;
            float P[9];
            tet_two_col(Jw + 9 * slc * 17, k, wV, mu, lam, hs, gk, gk2, Ee, P);
            if (dseed && sok) {
                // lane k writes seed k; lane 0 also seed 8
                const float wt = (float)wV;
                float pv = P[0];
#pragma unroll
                for (int v = 1; v < 8; ++v) pv = k == v ? P[v] : pv;
                global_store_asm(dseed + 9 * (s0 + sl) + k, wt * pv);
                if (k == 0) global_store_asm(dseed + 9 * (s0 + sl) + 8, wt * P[8]);
            }
        }
        return;
    }
    // penalty k_c/2 |x_t - target_t|^2 of the chunk's targets (three rows each)
    const double* tg = (ext && e.targets) ? e.targets + (size_t)bidx * e.nt * 3 : nullptr;
    const int tb = (row0 - prow) / 3;
    const int ntg = tg ? max(0, min(kFuseRows / 3, e.nt - tb)) : 0;
    const float kt = (float)kc;
    for (int q = 0; r0 + rs * q < ntg; ++q) {
        const int tl = r0 + rs * q + eg, t = tb + tl;
        const bool ok = tl < ntg;
        const int tc = ok ? t : tb;
        double xr[3], tr[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            xr[c] = e.Xt[3 * tc + c];
            tr[c] = tg[3 * tc + c];
        }
        const float* row = Jw + 3 * (ok ? tl : 0) * 17;
        float xv[3], jr[3], jr2[3];
        lds_read3(row, 17, xv);
        lds_read3(row + 1 + k, 17, jr);
        lds_read3(row + 9 + k, 17, jr2);
        float Jc[3], J2[3];
        double d[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Jc[c] = ok ? jr[c] : 0.f;
            J2[c] = ok ? jr2[c] : 0.f;
            d[c] = ok ? xr[c] + (double)xv[c] - tr[c] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float pe = pair_even(Jc[c], J2[c]), po = pair_odd(Jc[c], J2[c]);
            hs = Mfma<float>::mac(pe, kt * pe, hs);
            hs = Mfma<float>::mac(po, kt * po, hs);
        }
        if (ok) {
            gk += kc * ((double)Jc[0] * d[0] + (double)Jc[1] * d[1] + (double)Jc[2] * d[2]);
            gk2 += kc * ((double)J2[0] * d[0] + (double)J2[1] * d[1] + (double)J2[2] * d[2]);
            Ee += k == 0 ? 0.5 * kc * (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) : 0.0;
            if (dseed && k < 3) {
                const double dv = k == 0 ? d[0] : k == 1 ? d[1] : d[2];
                global_store_asm(dseed + prow + 3 * t + k, (float)(kc * dv));
            }
        }
    }
    // gravity (-1 times the row) and force (-f_c times row c) rows of this chunk
    if (ext && r0 == 0 && eg == 0) {
        const int nrow = (e.force && e.nf) ? 4 : 1;
        for (int c = 0; c < nrow; ++c) {
            const int rg = c == 0 ? e.grav_row : e.force_row + c - 1;
            if (rg < row0 || rg >= row0 + nrows) continue;
            const double coef = c == 0 ? 1.0 : e.force[(size_t)bidx * 3 + c - 1];
            const float* rr = Jw + (rg - row0) * 17;
            gk -= coef * (double)rr[1 + k];
            gk2 -= coef * (double)rr[9 + k];
            if (k == 0) Ee -= coef * (double)rr[0];
        }
    }
}

// Seeds dE/d(row value) of the rows past the tets that no target writes:
// penalty rows without targets, gravity (-1), force (-f_c) and padding rows.
__device__ inline void fused_tail_seeds(const ElemArgs& e, int item, int lane)
{
    const bool ext = !e.elastic_only;
    const int bidx = e.imap ? e.imap[item] : item;
    const bool tgi = ext && e.targets;
    float* dseed = static_cast<float*>(e.dseed) + (size_t)item * e.rows_pad;
    for (int row = 9 * e.S + lane; row < e.rows_pad; row += 64) {
        double v = 0.0;
        if (row < e.grav_row) {
            if (tgi) continue;
        } else if (row == e.grav_row) {
            v = ext ? -1.0 : 0.0;
        } else if (row < e.force_row + 3) {
            v = (ext && e.force && e.nf) ? -e.force[(size_t)bidx * 3 + (row - e.force_row)] : 0.0;
        }
        dseed[row] = (float)v;
    }
}

template <int KCH>
__global__ __launch_bounds__(256, 2) void k_elem_fused(FusedElemArgs a)
{
    constexpr int K = KCH * kTileK;
    constexpr int LDB = K + 8; // BF16 values per LDS column (16-byte pad: staggered banks)
    __shared__ __align__(16) __bf16 Yp[3][kFuseCols * LDB];
    __shared__ __align__(16) float Jl[2 * kFuseRows * 17];
    __shared__ float Vl[2 * kFuseRows]; // value rows of items 2 and 3 (with the bias)
    constexpr int RW = 280; // final sums per (wave, pass): H (256), g (16), E
    static_assert(4 * 2 * RW * sizeof(double) <= sizeof(Jl), "the final sums fit the row buffer");
    const ElemArgs& e = a.e;
    const int grp = blockIdx.x / e.parts, part = blockIdx.x - grp * e.parts;
    const int n_items = e.count ? min(*e.count, a.cap) : a.cap;
    if (grp * kFuseG >= n_items) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & 15, lg = lane >> 4;
    const int eg = lane >> 3, k = lane & 7;
    const int nc = e.nc;

    // the group's activation columns as three BF16 planes
    {
        constexpr int Q = K / 8;
        for (int idx = tid; idx < kFuseCols * Q; idx += 256) {
            const int n = idx / Q, q = idx - n * Q;
            int it = n_items, col = 0;
            if (n < 16 * kFuseG) {
                it = grp * kFuseG + (n >> 4);
                col = 1 + (n & 15);
            } else if (n < 16 * kFuseG + kFuseG) {
                it = grp * kFuseG + n - 16 * kFuseG;
            }
            f32x4 v0 = {0.f, 0.f, 0.f, 0.f}, v1 = v0;
            if (it < n_items) {
                const float* src = a.Y + ((size_t)it * nc + col) * a.y_rows + 8 * q;
                v0 = *reinterpret_cast<const f32x4*>(src);
                v1 = *reinterpret_cast<const f32x4*>(src + 4);
            }
            bf16x8 h, m, l;
            split3_bf16(v0, v1, h, m, l);
            *reinterpret_cast<bf16x8*>(&Yp[0][n * LDB + 8 * q]) = h;
            *reinterpret_cast<bf16x8*>(&Yp[1][n * LDB + 8 * q]) = m;
            *reinterpret_cast<bf16x8*>(&Yp[2][n * LDB + 8 * q]) = l;
        }
    }

    const int S = e.S;
    const int prow = 9 * S;
    const int ntc = (S + kFuseTets - 1) / kFuseTets;
    const int ntl = (a.rows - prow + kFuseRows - 1) / kFuseRows;
    const int nch = ntc + ntl;
    const int per = (nch + e.parts - 1) / e.parts;
    const int cb = min(nch, part * per), ce = min(nch, cb + per);
    const size_t plane = (size_t)e.rows_pad * a.lda;
    const __bf16* Ab = static_cast<const __bf16*>(a.A);
    // LDS column of this lane's B fragment in output tile j
    auto bcol = [&](int j) { return j < kFuseG ? 16 * j + li : (li < kFuseG ? 16 * kFuseG + li : kFuseCols - 1); };

    // pass X of the element physics: item 2 X + (wave >> 1), tets / targets of half wave & 1
    const int slot = wave >> 1, hf = wave & 1;
    double Hm[2][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
    double gk[2] = {0.0, 0.0}, gk2[2] = {0.0, 0.0}, Ee[2] = {0.0, 0.0};

    lds_barrier(); // the activation planes
    for (int ch = cb; ch < ce; ++ch) {
        const bool tail = ch >= ntc;
        const int row0 = tail ? prow + kFuseRows * (ch - ntc) : kFuseRows * ch;
        const int ntile = tail ? min(9, (a.rows - row0 + 15) / 16) : 9;
        const int t0 = (wave - ch) & 3;
        const int nw = (t0 < ntile) + (t0 + 4 < ntile) + (t0 + 8 < ntile); // of the tiles t0, t0 + 4, t0 + 8
        // the Jacobian tiles of items 2 and 3, kept for the second pass
        f32x4 held[2][3];
        // row tiles t0 + 4 q of the wave, q = q0 .. q0 + NQ - 1: A fragments of
        // all of them in registers, loads issued at once (rows past the padded
        // end re-read the last row: their products are never used); each B
        // fragment is read from LDS once for all of them.
        auto tiles = [&](auto Q0, auto NQ) {
            constexpr int q0 = decltype(Q0)::value, nq = decltype(NQ)::value;
            auto tile_of = [&](int q) { return t0 + 4 * q; };
            bf16x8 af[nq][KCH][3];
#pragma unroll
            for (int i = 0; i < nq; ++i) {
                const int row = min(row0 + 16 * tile_of(q0 + i) + li, e.rows_pad - 1);
                const __bf16* p = Ab + (size_t)row * a.lda + 8 * lg;
#pragma unroll
                for (int c = 0; c < KCH; ++c)
#pragma unroll
                    for (int pl = 0; pl < 3; ++pl)
                        af[i][c][pl] = *reinterpret_cast<const bf16x8*>(p + pl * plane + c * kTileK);
            }
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                f32x4 acc[nq], corr[nq];
#pragma unroll
                for (int i = 0; i < nq; ++i) acc[i] = corr[i] = f32x4{0.f, 0.f, 0.f, 0.f};
                const int cofs = bcol(j) * LDB + 8 * lg;
#pragma unroll
                for (int c = 0; c < KCH; ++c) {
                    bf16x8 b[3];
#pragma unroll
                    for (int pl = 0; pl < 3; ++pl) b[pl] = *reinterpret_cast<const bf16x8*>(&Yp[pl][cofs + c * kTileK]);
#pragma unroll
                    for (int i = 0; i < nq; ++i) mfma_bf16x6_chunk(af[i][c], b, acc[i], corr[i]);
                }
#pragma unroll
                for (int i = 0; i < nq; ++i) {
                    const f32x4 o = acc[i] + corr[i];
                    if (j == 2 || j == 3) {
                        held[j - 2][q0 + i] = o;
                        continue;
                    }
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int m = 16 * tile_of(q0 + i) + 4 * lg + v; // row within the chunk
                        if (j < 2) {
                            Jl[(j * kFuseRows + m) * 17 + 1 + li] = o[v];
                        } else if (li < kFuseG) {
                            const int rg = row0 + m;
                            const float val = o[v] + (rg < a.rows ? a.bias[rg] : 0.f);
                            if (li < 2) Jl[(li * kFuseRows + m) * 17] = val;
                            else Vl[(li - 2) * kFuseRows + m] = val;
                        }
                    }
                }
            }
        };
        using I0 = std::integral_constant<int, 0>;
        using I1 = std::integral_constant<int, 1>;
        using I2 = std::integral_constant<int, 2>;
        if (nw >= 2) tiles(I0{}, I2{});
        else if (nw == 1) tiles(I0{}, I1{});
        if (nw == 3) tiles(I2{}, I1{});
        lds_barrier(); // rows of items 0 and 1

#pragma unroll
        for (int X = 0; X < 2; ++X) {
            if (X == 1) {
                lds_barrier(); // the first pass has read its rows
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    if (q >= nw) break;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int m = 16 * (t0 + 4 * q) + 4 * lg + v;
                        Jl[m * 17 + 1 + li] = held[0][q][v];
                        Jl[(kFuseRows + m) * 17 + 1 + li] = held[1][q][v];
                    }
                }
                for (int i = tid; i < 2 * kFuseRows; i += 256) Jl[i * 17] = Vl[i];
                lds_barrier(); // rows of items 2 and 3
            }
            const int item = grp * kFuseG + 2 * X + slot;
            if (item >= n_items) continue; // wave-uniform
            f32x4 hs = {0.f, 0.f, 0.f, 0.f};
            fused_item_chunk(e, Jl + slot * kFuseRows * 17, item, tail, ch, ntc, row0, 16 * ntile, 8 * hf, 16, eg, k,
                             hs, gk[X], gk2[X], Ee[X]);
#pragma unroll
            for (int q = 0; q < 4; ++q) Hm[X][q] += (double)hs[q];
        }
        lds_barrier(); // the second pass has read its rows
    }

    // each item's two waves: sums over the wave's tet lanes, then the two
    // waves' sums added in wave order through the (now idle) row buffer
    double* red = reinterpret_cast<double*>(Jl);
#pragma unroll
    for (int X = 0; X < 2; ++X) {
#pragma unroll
        for (int off = 8; off < 64; off <<= 1) {
            gk[X] += __shfl_xor(gk[X], off);
            gk2[X] += __shfl_xor(gk2[X], off);
            Ee[X] += __shfl_xor(Ee[X], off);
        }
        double* rw = red + (wave * 2 + X) * RW;
#pragma unroll
        for (int q = 0; q < 4; ++q) rw[q * 64 + lane] = Hm[X][q];
        if (eg == 0) {
            rw[256 + k] = gk[X];
            rw[264 + k] = gk2[X];
        }
        if (lane == 0) rw[272] = Ee[X];
    }
    lds_barrier();
    const int item = grp * kFuseG + wave;
    if (item >= n_items) return;
    {
        // item 2 X + s of the group: pass X of waves 2 s and 2 s + 1
        const int X = wave >> 1, s = wave & 1;
        const double* r0 = red + ((2 * s) * 2 + X) * RW;
        const double* r1 = red + ((2 * s + 1) * 2 + X) * RW;
        const size_t slot_o = (size_t)part * e.part_stride + item;
        if (e.H) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                e.H[slot_o * 256 + Mfma<float>::row(lane, q) * 16 + li] = r0[q * 64 + lane] + r1[q * 64 + lane];
        }
        if (lane < 16 && e.g) e.g[slot_o * 16 + lane] = r0[256 + lane] + r1[256 + lane];
        if (lane == 0 && e.E) e.E[item] = r0[272] + r1[272];
    }
    if (e.dseed && part == 0) fused_tail_seeds(e, item, lane);
}

// The same for float32 contexts: the output map on the FP32 matrix cores,
// with the waves specialised.  With no BF16 parts the group's activation
// columns take half the LDS, so the row buffer holds all four items' rows and
// fits twice: four producer waves form chunk ch + 1 into one buffer while four
// consumer waves run the element physics of chunk ch from the other (consumer
// w on item w, 16 tets: two rounds), one barrier per chunk.  The products no
// longer wait for the element physics (one workgroup of 8 waves per compute
// unit: a producer and a consumer wave per SIMD).  Row tiles: producer p takes
// t = p - ch (mod 4) and t + 4 with all five output tiles, and of the ninth
// row tile the output tile j = p (the value tile on producer ch mod 4), so the
// four producers' products per chunk differ by at most one output tile.  Per
// 16x16x4 product, lane (i, g) supplies W_big[row i][K/4 g + s] and the
// activation column i at the same k (step s): each lane's A and B values are
// one contiguous run of K/4.
template <int KCH>
__global__ __launch_bounds__(512, 1) void k_elem_fused_f32(FusedElemArgs a)
{
    constexpr int K = KCH * kTileK;
    constexpr int KS = K / 4;  // products per output tile (k per lane)
    constexpr int LDY = K + 4; // floats per LDS column (16-byte rows, staggered banks)
    constexpr int JL = kFuseG * kFuseRows * 17;
    __shared__ __align__(16) float Yf[kFuseCols * LDY];
    __shared__ __align__(16) float Jl[2 * JL];
    const ElemArgs& e = a.e;
    const int grp = blockIdx.x / e.parts, part = blockIdx.x - grp * e.parts;
    const int n_items = e.count ? min(*e.count, a.cap) : a.cap;
    if (grp * kFuseG >= n_items) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool producer = wave < 4;
    const int pw = wave & 3; // producer index, or the consumer's item in the group
    const int li = lane & 15, lg = lane >> 4;
    const int eg = lane >> 3, k = lane & 7;
    const int nc = e.nc;

    // the group's activation columns (Jacobian, values, zeros)
    {
        constexpr int Q = K / 4;
        for (int idx = tid; idx < kFuseCols * Q; idx += 512) {
            const int n = idx / Q, q = idx - n * Q;
            int it = n_items, col = 0;
            if (n < 16 * kFuseG) {
                it = grp * kFuseG + (n >> 4);
                col = 1 + (n & 15);
            } else if (n < 16 * kFuseG + kFuseG) {
                it = grp * kFuseG + n - 16 * kFuseG;
            }
            f32x4 v = {0.f, 0.f, 0.f, 0.f};
            if (it < n_items) v = *reinterpret_cast<const f32x4*>(a.Y + ((size_t)it * nc + col) * a.y_rows + 4 * q);
            *reinterpret_cast<f32x4*>(&Yf[n * LDY + 4 * q]) = v;
        }
    }

    const int S = e.S;
    const int prow = 9 * S;
    const int ntc = (S + kFuseTets - 1) / kFuseTets;
    const int ntl = (a.rows - prow + kFuseRows - 1) / kFuseRows;
    const int nch = ntc + ntl;
    const int per = (nch + e.parts - 1) / e.parts;
    const int cb = min(nch, part * per), ce = min(nch, cb + per);
    const float* Af = static_cast<const float*>(a.A);
    auto bcol = [&](int j) { return j < kFuseG ? 16 * j + li : (li < kFuseG ? 16 * kFuseG + li : kFuseCols - 1); };
    auto chunk_rows = [&](int ch, int& row0, int& ntile) {
        const bool tail = ch >= ntc;
        row0 = tail ? prow + kFuseRows * (ch - ntc) : kFuseRows * ch;
        ntile = tail ? min(9, (a.rows - row0 + 15) / 16) : 9;
    };

    // producer p: the rows of chunk ch into the row buffer J
    auto produce = [&](int ch, float* J) {
        int row0, ntile;
        chunk_rows(ch, row0, ntile);
        const int t0 = (pw - ch) & 3;
        // row tiles t0, t0 + 4 (all output tiles) and 8 (output tiles in m8)
        const int m8 = ntile == 9 ? (1 << pw) | (pw == (ch & 3) ? 16 : 0) : 0;
        const bool u0 = t0 < ntile, u1 = t0 + 4 < ntile;
        // A fragments of the three row tiles, all loads issued at once (rows
        // past the padded end re-read the last row: never used)
        f32x4 af[3][KS / 4];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int t = i < 2 ? t0 + 4 * i : 8;
            const int row = min(row0 + 16 * t + li, e.rows_pad - 1);
            const f32x4* p = reinterpret_cast<const f32x4*>(Af + (size_t)row * a.lda + KS * lg);
#pragma unroll
            for (int q = 0; q < KS / 4; ++q) af[i][q] = p[q];
        }
        // the products of output tiles j and j + 1 (NJ = 2) or j alone for the row tiles in M
        // (bit i: slot i): one branch per pass, none per product, up to six accumulators
        // in flight
        auto prod = [&](auto MC, auto NJC, int j) {
            constexpr int M = decltype(MC)::value, NJ = decltype(NJC)::value;
            f32x4 b[NJ][KS / 4];
#pragma unroll
            for (int jj = 0; jj < NJ; ++jj) {
                const f32x4* bp = reinterpret_cast<const f32x4*>(&Yf[bcol(j + jj) * LDY + KS * lg]);
#pragma unroll
                for (int q = 0; q < KS / 4; ++q) b[jj][q] = bp[q];
            }
            // every B read issued before the products
            __builtin_amdgcn_sched_barrier(0);
            f32x4 acc[NJ][3];
#pragma unroll
            for (int jj = 0; jj < NJ; ++jj)
#pragma unroll
                for (int i = 0; i < 3; ++i) acc[jj][i] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int q = 0; q < KS / 4; ++q)
#pragma unroll
                for (int e4 = 0; e4 < 4; ++e4)
#pragma unroll
                    for (int jj = 0; jj < NJ; ++jj)
#pragma unroll
                        for (int i = 0; i < 3; ++i)
                            if (((M >> i) & 1) != 0) acc[jj][i] = Mfma<float>::mac(af[i][q][e4], b[jj][q][e4], acc[jj][i]);
#pragma unroll
            for (int jj = 0; jj < NJ; ++jj)
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    if (((M >> i) & 1) == 0) continue; // folded: the loop is unrolled
                    const int t = i < 2 ? t0 + 4 * i : 8, jo = j + jj;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int m = 16 * t + 4 * lg + v; // row within the chunk
                        if (jo < kFuseG) {
                            J[(jo * kFuseRows + m) * 17 + 1 + li] = acc[jj][i][v];
                        } else if (li < kFuseG) {
                            const int rg = row0 + m;
                            J[(li * kFuseRows + m) * 17] = acc[jj][i][v] + (rg < a.rows ? a.bias[rg] : 0.f);
                        }
                    }
                }
        };
        using M1 = std::integral_constant<int, 1>;
        using M3 = std::integral_constant<int, 3>;
        using M4 = std::integral_constant<int, 4>;
        using M5 = std::integral_constant<int, 5>;
        using M7 = std::integral_constant<int, 7>;
        using J1 = std::integral_constant<int, 1>;
        using J2 = std::integral_constant<int, 2>;
        // output tiles (0, 1) and (2, 3) in pairs when both have the same row tiles (tile 8's
        // output tiles are split over the producers), the value tile alone
        auto mask_of = [&](int j) { return (u0 ? 1 : 0) | (u1 ? 2 : 0) | (((m8 >> j) & 1) ? 4 : 0); };
        auto one = [&](int j) {
            switch (mask_of(j)) {
            case 1: prod(M1{}, J1{}, j); break;
            case 3: prod(M3{}, J1{}, j); break;
            case 4: prod(M4{}, J1{}, j); break;
            case 5: prod(M5{}, J1{}, j); break;
            case 7: prod(M7{}, J1{}, j); break;
            default: break;
            }
        };
#pragma unroll 1
        for (int j = 0; j < 4; j += 2) {
            const int m0 = mask_of(j), m1 = mask_of(j + 1);
            if (m0 == m1 && m0 == 3) prod(M3{}, J2{}, j);
            else if (m0 == m1 && m0 == 1) prod(M1{}, J2{}, j);
            else {
                one(j);
                one(j + 1);
            }
        }
        one(4);
    };

    const int item = grp * kFuseG + pw;
    const bool cok = !producer && item < n_items; // a consumer with an item
    double Hm[4] = {0.0, 0.0, 0.0, 0.0};
    double gk = 0.0, gk2 = 0.0, Ee = 0.0;

    lds_barrier(); // the activation columns
    if (producer && cb < ce) produce(cb, Jl);
    lds_barrier(); // the first chunk's rows
    for (int ch = cb; ch < ce; ++ch) {
        float* Jc = Jl + ((ch - cb) & 1) * JL;
        if (producer) {
            // the next chunk into the other buffer (read by the consumers of chunk ch - 1,
            // which the previous barrier closed)
            if (ch + 1 < ce) produce(ch + 1, Jl + ((ch + 1 - cb) & 1) * JL);
        } else if (cok) {
            int row0, ntile;
            chunk_rows(ch, row0, ntile);
            f32x4 hs = {0.f, 0.f, 0.f, 0.f};
            fused_item_chunk(e, Jc + pw * kFuseRows * 17, item, ch >= ntc, ch, ntc, row0, 16 * ntile, 0, 8, eg, k, hs,
                             gk, gk2, Ee);
#pragma unroll
            for (int q = 0; q < 4; ++q) Hm[q] += (double)hs[q];
        }
        lds_barrier(); // chunk ch read, chunk ch + 1 formed
    }
    if (!cok) return;

    // g and E over the wave's 8 tet lanes (lanes k, k + 8, ...); H is whole per wave
#pragma unroll
    for (int off = 8; off < 64; off <<= 1) {
        gk += __shfl_xor(gk, off);
        gk2 += __shfl_xor(gk2, off);
        Ee += __shfl_xor(Ee, off);
    }
    const size_t slot = (size_t)part * e.part_stride + item;
    if (e.H) {
#pragma unroll
        for (int q = 0; q < 4; ++q) e.H[slot * 256 + Mfma<float>::row(lane, q) * 16 + li] = Hm[q];
    }
    if (eg == 0 && e.g) {
        e.g[slot * 16 + k] = gk;
        e.g[slot * 16 + 8 + k] = gk2;
    }
    if (lane == 0 && e.E) e.E[item] = Ee;
    if (e.dseed && part == 0) fused_tail_seeds(e, item, lane);
}

hipError_t launch_elem_fused(int bf16, const FusedElemArgs& a, hipStream_t s)
{
    if (a.cap <= 0) return hipSuccess;
    const ElemArgs& e = a.e;
    if (!elem_fused_fits(e.r, a.K) || e.nc != 17 || a.K > a.lda || a.K > a.y_rows || e.parts < 1 ||
        (e.parts > 1 && (e.E || e.part_stride < a.cap)) || a.rows > e.rows_pad || 9 * e.S > a.rows)
        return hipErrorInvalidValue;
    const int groups = (a.cap + kFuseG - 1) / kFuseG;
    dim3 grid(groups * e.parts);
#define RS_FUSED(KC)                                                                   \
    do {                                                                               \
        if (bf16) RS_LAUNCH((k_elem_fused<KC>), grid, dim3(256), 0, s, a);             \
        else RS_LAUNCH((k_elem_fused_f32<KC>), grid, dim3(512), 0, s, a);              \
    } while (0)
    switch (a.K / kTileK) {
    case 1: RS_FUSED(1); break;
    case 2: RS_FUSED(2); break;
    case 3: RS_FUSED(3); break;
    default: RS_FUSED(4); break;
    }
#undef RS_FUSED
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Energy-only kernel (float64): one workgroup per item, one thread per tet.
// ---------------------------------------------------------------------------
__device__ inline double block_sum256(double v, double* sh)
{
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) sh[tid] += sh[tid + w];
        __syncthreads();
    }
    const double out = sh[0];
    __syncthreads();
    return out;
}

__global__ __launch_bounds__(256) void k_energy(EnergyArgs a)
{
    __shared__ double sh[256];
    const int item = blockIdx.x, tid = threadIdx.x;
    if (a.count && item >= *a.count) return;
    const double* O = static_cast<const double*>(a.out) + (size_t)item * a.rows_pad;
    const int bidx = a.imap ? a.imap[item] : item;
    double acc = 0.0;
    for (int s = tid; s < a.S; s += 256) {
        double gu[9];
#pragma unroll
        for (int v = 0; v < 9; ++v) gu[v] = O[9 * s + v];
        Snh<double> m;
        m.set(gu, a.mu, a.lam);
        acc += a.wV[s] * m.psi;
    }
    if (!a.elastic_only) {
        if (a.targets) {
            const double* tg = a.targets + (size_t)bidx * a.nt * 3;
            for (int t = tid; t < a.nt; t += 256) {
                double e = 0.0;
                for (int c = 0; c < 3; ++c) {
                    const double d = a.Xt[3 * t + c] + O[9 * a.S + 3 * t + c] - tg[3 * t + c];
                    e += d * d;
                }
                acc += 0.5 * a.k_c * e;
            }
        }
        if (tid == 0) {
            acc -= O[a.grav_row];
            if (a.force && a.nf)
                for (int c = 0; c < 3; ++c) acc -= a.force[(size_t)bidx * 3 + c] * O[a.force_row + c];
        }
    }
    const double tot = block_sum256(acc, sh);
    if (tid == 0) a.E[item] = tot;
}

hipError_t launch_energy(const EnergyArgs& a, int items, hipStream_t s)
{
    if (items <= 0) return hipSuccess;
    RS_LAUNCH(k_energy, dim3(items), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Curvature kernel: reverse pass through the hidden layers (activations from
// the stored pre-activations) adding sum_l A_l^T diag(gbar_l s''(a_l)) A_l,
// the second-order term of the exact reduced Hessian.  dE/dh_L is the sum of
// the adjoint GEMM's K-slice partials, taken in slice order.
// ---------------------------------------------------------------------------
// Reverse pass through the hidden layers, one workgroup per item (width
// w <= 256).  Per layer l, from the last: cf = gbar_l * s''(a_l) and
// ga = gbar_l * s'(a_l); then H += A^T diag(cf) A on the matrix cores, wave q
// taking the 4-row steps t = q, q + 4, ... (lane (c, kq) holds A[u][c] for
// u = 4t + kq: the A operand of A^T and, scaled by cf[u], the B operand of
// diag(cf) A), float64 totals per layer, the four waves' sums added in order
// at the end; and gbar_{l-1} = W_l^T ga, thread (slice, vq) summing rows
// v of its slice of W_l into 4 adjacent outputs (16-byte loads), the 8
// slices added in order.
// Only gbar -> ga -> gbar is a dependent chain, so the global reads are
// issued ahead of it: the entries of layer l - 1's [a | A] block that a thread
// uses are loaded into registers while layer l runs, and the first rows of
// the thread's W_l slice at the top of layer l (before that prefetch, so that
// waiting on them leaves it in flight).  Every such load is unconditional, at
// a clamped in-bounds address, and the barriers order LDS traffic only
// (lds_barrier), so the loads stay in flight across them.
constexpr int kCurvMaxW = kMaxWidth;

// KT: 4-row steps per wave held for a layer (w <= 16 KT); WQ: rows of the
// thread's W_l slice loaded at the top of the layer (0: all in the products'
// own batches, fewer registers for batches that fill the chip several times)
template <typename T, int RT, int KT, int WQ>
__global__ __launch_bounds__(256) void k_curv(CurvArgs a)
{
    extern __shared__ double smem[];
    const int item = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (a.count && item >= *a.count) return;
    const int w = a.width, nc = a.nc, r = a.r;
    const int su = a.pre_su, sc = a.pre_sc;
    double* gh = smem;          // dE/dh_l
    double* ga = gh + w;        // dE/da_l
    double* cf = ga + w;        // dE/dh_l * s''(a_l)
    const int pw = w > r ? w : r; // outputs of W_l^T ga: w, or r for the first layer
    double* part = cf + w;        // [8 slices][pw] partial sums of W_l^T ga
    double* red = part + 8 * pw;  // [4 waves][RT][RT][4][64] per-wave H partials
    double* hpart = red + 4 * RT * RT * 4 * 64; // parts > 1: the element kernel's H summed over parts
    const int c = lane & 15, kq = lane >> 4;
    using acc_t = typename Mfma<T>::acc_t;
    using V4 = T __attribute__((ext_vector_type(4)));

    // a layer's entries used by this thread: a[tid] and A[u][16 ti + c] for
    // u = 4 (wave + 4 k) + kq (zero past the width or the latent dimension)
    T pv = T(0);
    T pj[KT][RT];
    auto fetch = [&](int l) {
        const T* P = static_cast<const T*>(a.pre[l]) + (size_t)item * a.pre_rows * nc;
        pv = P[(size_t)min(tid, w - 1) * su];
        if (!a.H) return; // value-only blocks (nc = 1) have no A
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            const int u = min(4 * (wave + 4 * k) + kq, w - 1);
#pragma unroll
            for (int ti = 0; ti < RT; ++ti)
                pj[k][ti] = P[(size_t)u * su + (size_t)(1 + min(16 * ti + c, r - 1)) * sc];
        }
    };
    fetch(a.L - 1);
    if (a.parts > 1) {
        // summed here, at the start, so that the loads overlap the layer loop;
        // every part's load is issued before the sum
        for (int e = tid; e < r * r; e += 256) {
            double v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                v[q] = q < a.parts ? a.Hp[((size_t)q * a.part_stride + item) * r * r + e] : 0.0;
            double hs = 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) hs += v[q];
            hpart[e] = hs;
        }
        if (tid < r) {
            double v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                v[q] = q < a.parts ? a.gp[((size_t)q * a.part_stride + item) * r + tid] : 0.0;
            double gs = 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) gs += v[q];
            a.g[(size_t)item * r + tid] = gs;
        }
    }
    for (int u = tid; u < w; u += 256) {
        const T* gp = static_cast<const T*>(a.gbar) + (size_t)item * a.pre_rows + u;
        T v[kMaxSplit];
#pragma unroll
        for (int z = 0; z < kMaxSplit; ++z) v[z] = gp[(size_t)min(z, a.ksplit - 1) * a.split_stride];
        double sum = 0.0;
#pragma unroll
        for (int z = 0; z < kMaxSplit; ++z)
            if (z < a.ksplit) sum += (double)v[z];
        gh[u] = sum;
    }
    double Hd[RT][RT][4];
#pragma unroll
    for (int ti = 0; ti < RT; ++ti)
#pragma unroll
        for (int tj = 0; tj < RT; ++tj)
#pragma unroll
            for (int v = 0; v < 4; ++v) Hd[ti][tj][v] = 0.0;
    const int slice = tid >> 5, vq = tid & 31;
    const int rows_per = (w + 7) / 8;
    for (int l = a.L - 1; l >= 0; --l) {
        const bool gemv = l > 0 || a.grev;
        const int in = l == 0 ? r : w;
        const int ld = l == 0 ? a.lda0 : a.lda;
        const T* Wl = static_cast<const T*>(a.W[l]);
        const int v0 = slice * rows_per, v1 = min(w, v0 + rows_per);
        const int u00 = 4 * vq;
        // the first WQ rows of the slice, first column group (clamped rows and columns)
        V4 wq[WQ > 0 ? WQ : 1];
        if (WQ > 0) {
            const T* wp = Wl + min(u00, ld - 4);
#pragma unroll
            for (int b = 0; b < WQ; ++b) wq[b] = *reinterpret_cast<const V4*>(wp + (size_t)min(v0 + b, w - 1) * ld);
        }
        // this layer's entries, then the next layer's loads behind them
        const T cv = pv;
        T cj[KT][RT];
#pragma unroll
        for (int k = 0; k < KT; ++k)
#pragma unroll
            for (int ti = 0; ti < RT; ++ti) cj[k][ti] = pj[k][ti];
        if (l > 0) fetch(l - 1);
        lds_barrier(); // gh of this layer visible; cf, ga, part free
        if (tid < w) {
            const double av = (double)cv;
            // s'(a) and s''(a) share exp(a) for a <= 0 (1 and 0 above)
            const double ex = exp(fmin(av, 0.0));
            cf[tid] = av > 0.0 ? 0.0 : gh[tid] * ex;
            ga[tid] = av > 0.0 ? gh[tid] : gh[tid] * ex;
            if (a.delta) a.delta[((size_t)item * a.L + l) * w + tid] = ga[tid];
        }
        lds_barrier();
        if (a.H) {
            acc_t acc[RT][RT];
#pragma unroll
            for (int ti = 0; ti < RT; ++ti)
#pragma unroll
                for (int tj = 0; tj < RT; ++tj) acc[ti][tj] = acc_t{0, 0, 0, 0};
#pragma unroll
            for (int k = 0; k < KT; ++k) { // steps past the width add zeros (no early exit: the loop stays unrolled)
                const int u = 4 * (wave + 4 * k) + kq;
                const bool uok = u < w;
                const T cfu = uok ? (T)cf[u] : T(0);
                T av[RT], bv[RT];
#pragma unroll
                for (int ti = 0; ti < RT; ++ti) {
                    const T x = (uok && 16 * ti + c < r) ? cj[k][ti] : T(0);
                    av[ti] = x;
                    bv[ti] = cfu * x;
                }
#pragma unroll
                for (int ti = 0; ti < RT; ++ti)
#pragma unroll
                    for (int tj = 0; tj < RT; ++tj) acc[ti][tj] = Mfma<T>::mac(av[ti], bv[tj], acc[ti][tj]);
            }
#pragma unroll
            for (int ti = 0; ti < RT; ++ti)
#pragma unroll
                for (int tj = 0; tj < RT; ++tj)
#pragma unroll
                    for (int v = 0; v < 4; ++v) Hd[ti][tj][v] += (double)acc[ti][tj][v];
        }
        if (!gemv) break;
        // gbar_{l-1}[u'] = sum_v W_l[v][u'] ga[v] over the w outputs v of layer l
#pragma unroll
        for (int cg = 0; cg < kCurvMaxW / 128; ++cg) {
            const int u0 = 128 * cg + u00; // 4 adjacent outputs; ld is a multiple of 32 and zero padded
            if (128 * cg >= in) break;
            double sacc[4] = {0.0, 0.0, 0.0, 0.0};
            if (u0 < in) {
                int vb = v0;
                if (WQ > 0 && cg == 0) {
#pragma unroll
                    for (int b = 0; b < WQ; ++b) {
                        const double g = v0 + b < v1 ? ga[v0 + b] : 0.0;
                        asm volatile("" : "+v"(wq[b])); // converted here, not at the load
#pragma unroll
                        for (int e = 0; e < 4; ++e) sacc[e] = fma((double)wq[b][e], g, sacc[e]);
                    }
                    vb = v0 + WQ;
                }
                constexpr int RB = 8; // rows in flight
                for (; vb < v1; vb += RB) {
                    V4 x[RB];
#pragma unroll
                    for (int b = 0; b < RB; ++b)
                        if (vb + b < v1) x[b] = *reinterpret_cast<const V4*>(Wl + (size_t)(vb + b) * ld + u0);
#pragma unroll
                    for (int b = 0; b < RB; ++b)
                        if (vb + b < v1) {
                            const double g = ga[vb + b];
#pragma unroll
                            for (int e = 0; e < 4; ++e) sacc[e] += (double)x[b][e] * g;
                        }
                }
            }
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (u0 + e < in) part[slice * pw + u0 + e] = sacc[e];
        }
        lds_barrier();
        for (int u = tid; u < in; u += 256) {
            double o = 0.0;
            for (int q = 0; q < 8; ++q) o += part[q * pw + u];
            if (l > 0) gh[u] = o;
            else a.grev[(size_t)item * r + u] = o;
        }
    }
    if (!a.H) return; // gradient only
    // the four waves' partial sums, added in wave order
    lds_barrier();
#pragma unroll
    for (int ti = 0; ti < RT; ++ti)
#pragma unroll
        for (int tj = 0; tj < RT; ++tj)
#pragma unroll
            for (int v = 0; v < 4; ++v) red[(((wave * RT + ti) * RT + tj) * 4 + v) * 64 + lane] = Hd[ti][tj][v];
    lds_barrier();
    if (wave == 0) {
#pragma unroll
        for (int ti = 0; ti < RT; ++ti)
#pragma unroll
            for (int tj = 0; tj < RT; ++tj)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    auto at = [&](int q) { return red[(((q * RT + ti) * RT + tj) * 4 + v) * 64 + lane]; };
                    const double h = ((at(0) + at(1)) + at(2)) + at(3);
                    const int row = 16 * ti + Mfma<T>::row(lane, v), col = 16 * tj + c;
                    if (row < r && col < r) {
                        const size_t e = (size_t)row * r + col;
                        if (a.parts > 1) {
                            // the element kernel's partials (summed in part order), then the curvature
                            a.H[(size_t)item * r * r + e] = hpart[e] + h;
                        } else {
                            a.H[(size_t)item * r * r + e] += h;
                        }
                    }
                }
    }
}

// ---------------------------------------------------------------------------
// Parameter gradients of a summed objective: batched outer products of an
// adjoint (per item, per output) with a layer input (per item, per input),
// summed over the items in float64; 64 x 64 output tiles, items staged 32 at
// a time through LDS, each thread 4 x 4 outputs.
// ---------------------------------------------------------------------------
template <typename TX, typename TY, int YM>
__global__ __launch_bounds__(256) void k_param_outer(ParamOuterArgs a, int nslice, int bper)
{
    constexpr int TB = 32;
    __shared__ double xs[TB][64 + 1];
    __shared__ double ys[TB][64 + 1];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64, sl = blockIdx.z;
    const int bbeg = sl * bper, bend = min(a.B, bbeg + bper);
    const TX* X = static_cast<const TX*>(a.X);
    const TY* Y = static_cast<const TY*>(a.Y);
    double acc[4][4], accb[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        accb[i] = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    }
    for (int b0 = bbeg; b0 < bend; b0 += TB) {
        __syncthreads();
        for (int e = tid; e < TB * 64; e += 256) {
            const int bb = e >> 6, q = e & 63, b = b0 + bb;
            double xv = 0.0, yv = 0.0;
            if (b < bend && m0 + q < a.M) xv = (double)X[(size_t)b * a.x_stride + m0 + q];
            if (b < bend && n0 + q < a.N) {
                yv = (double)Y[(size_t)b * a.y_stride + n0 + q];
                if (YM == PO_Y_ELU) yv = yv > 0.0 ? yv : expm1(yv);
            }
            xs[bb][q] = xv;
            ys[bb][q] = yv;
        }
        __syncthreads();
        const int nb = min(TB, bend - b0);
        for (int bb = 0; bb < nb; ++bb) {
            double xv[4], yv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                xv[i] = xs[bb][ty * 4 + i];
                yv[i] = ys[bb][tx * 4 + i];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                accb[i] += xv[i];
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(xv[i], yv[j], acc[i][j]);
            }
        }
    }
    // one slice: straight into the result; several: into the slice's partials
    double* po = nslice > 1 ? a.part + (size_t)sl * a.M * a.N : nullptr;
    double* pb = nslice > 1 ? a.part + (size_t)nslice * a.M * a.N + (size_t)sl * a.M : nullptr;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int m = m0 + ty * 4 + i;
        if (m >= a.M) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = n0 + tx * 4 + j;
            if (n >= a.N) continue;
            if (po) {
                po[(size_t)m * a.N + n] = acc[i][j];
            } else {
                double* o = a.out + (size_t)m * a.ldo + n;
                *o = a.accumulate ? *o + acc[i][j] : acc[i][j];
            }
        }
        if (a.outb && blockIdx.x == 0 && tx == 0) {
            if (pb) pb[m] = accb[i];
            else a.outb[m] = a.accumulate ? a.outb[m] + accb[i] : accb[i];
        }
    }
}

// the slices' partial sums added in slice order (then the bias sums)
__global__ __launch_bounds__(256) void k_param_reduce(ParamOuterArgs a, int nslice)
{
    const size_t mn = (size_t)a.M * a.N;
    const size_t tot = mn + (a.outb ? (size_t)a.M : 0);
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        double sum = 0.0;
        if (e < mn) {
            // eight loads in flight, added in slice order
            int q = 0;
            for (; q + 8 <= nslice; q += 8) {
                double v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = a.part[(size_t)(q + u) * mn + e];
#pragma unroll
                for (int u = 0; u < 8; ++u) sum += v[u];
            }
            for (; q < nslice; ++q) sum += a.part[(size_t)q * mn + e];
            const size_t m = e / a.N, n = e - m * a.N;
            double* o = a.out + m * a.ldo + n;
            *o = a.accumulate ? *o + sum : sum;
        } else {
            const size_t m = e - mn;
            for (int q = 0; q < nslice; ++q) sum += a.part[(size_t)nslice * mn + (size_t)q * a.M + m];
            a.outb[m] = a.accumulate ? a.outb[m] + sum : sum;
        }
    }
}

hipError_t launch_param_outer(int f32, const ParamOuterArgs& a, hipStream_t s)
{
    if (a.B <= 0 || a.M <= 0 || a.N <= 0) return hipSuccess;
    // item slices: about 1024 workgroups, each slice at least 8 items, within
    // the partial-sum workspace
    const int tiles = ((a.N + 63) / 64) * ((a.M + 63) / 64);
    int nslice = std::max(1, std::min({(1024 + tiles - 1) / tiles, (a.B + 7) / 8, 32}));
    nslice = std::min<size_t>(nslice, a.part_cap / ((size_t)a.M * a.N + a.M));
    nslice = std::max(nslice, 1);
    const int bper = (a.B + nslice - 1) / nslice;
    dim3 grid((a.N + 63) / 64, (a.M + 63) / 64, nslice), block(256);
#define RS_PO(TX, TY, YM) RS_LAUNCH((k_param_outer<TX, TY, YM>), grid, block, 0, s, a, nslice, bper)
    if (a.x_f64) {
        if (a.y_mode == PO_Y_F64) RS_PO(double, double, PO_Y_F64);
        else if (f32) {
            if (a.y_mode == PO_Y_ELU) RS_PO(double, float, PO_Y_ELU);
            else RS_PO(double, float, PO_Y_RAW);
        } else {
            if (a.y_mode == PO_Y_ELU) RS_PO(double, double, PO_Y_ELU);
            else RS_PO(double, double, PO_Y_RAW);
        }
    } else {
        if (!f32) return hipErrorInvalidValue; // a T adjoint is float64 only in a float64 context (x_f64)
        if (a.y_mode == PO_Y_ELU) RS_PO(float, float, PO_Y_ELU);
        else if (a.y_mode == PO_Y_RAW) RS_PO(float, float, PO_Y_RAW);
        else RS_PO(float, double, PO_Y_F64);
    }
#undef RS_PO
    if (nslice > 1) {
        const size_t tot = (size_t)a.M * a.N + (a.outb ? (size_t)a.M : 0);
        const size_t blocks = std::min<size_t>((tot + 255) / 256, 4096);
        RS_LAUNCH(k_param_reduce, dim3((unsigned)blocks), dim3(256), 0, s, a, nslice);
    }
    return hipGetLastError();
}

__global__ __launch_bounds__(128) void k_unfold(const double* src, const double* srcb, int ncols, const int* ptr,
                                                const int* row, const double* coef, int rows, double* dW, double* db)
{
    const int n = blockIdx.x;
    if (n >= rows) return;
    const int j0 = ptr[n], j1 = ptr[n + 1];
    for (int k = threadIdx.x; k < ncols; k += blockDim.x) {
        double sum = 0.0;
        for (int j = j0; j < j1; ++j) sum = fma(coef[j], src[(size_t)row[j] * ncols + k], sum);
        dW[(size_t)n * ncols + k] = sum;
    }
    if (threadIdx.x == 0) {
        double sb = 0.0;
        for (int j = j0; j < j1; ++j) sb = fma(coef[j], srcb[row[j]], sb);
        db[n] = sb;
    }
}

hipError_t launch_unfold(const double* src, const double* srcb, int ncols, const int* ptr, const int* row,
                         const double* coef, int rows, double* dW, double* db, hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    RS_LAUNCH(k_unfold, dim3(rows), dim3(128), 0, s, src, srcb, ncols, ptr, row, coef, rows, dW, db);
    return hipGetLastError();
}

__global__ void k_fill_zero(double* p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

hipError_t launch_fill_zero(double* p, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 4096);
    RS_LAUNCH(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_curv(int f32, const CurvArgs& a, int items, int n_cu, hipStream_t s)
{
    if (items <= 0 || a.L <= 0) return hipSuccess;
    if (a.r > kMaxR) return hipErrorInvalidValue;
    if (a.width > kCurvMaxW) return hipErrorInvalidValue;
    if (a.ksplit < 1 || a.ksplit > kMaxSplit || a.parts > 8) return hipErrorInvalidValue;
    const size_t pw = (size_t)(a.width > a.r ? a.width : a.r);
    const int rt = a.r <= 16 ? 1 : 2;
    const size_t sh = sizeof(double) * (3 * (size_t)a.width + 8 * pw + 4 * rt * rt * 4 * 64 + (size_t)a.r * a.r);
#define RS_CURV(RT, KT, WQ)                                                                               \
    do {                                                                                                  \
        if (f32) RS_LAUNCH((k_curv<float, RT, KT, WQ * 2>), dim3(items), dim3(256), sh, s, a);           \
        else RS_LAUNCH((k_curv<double, RT, KT, WQ>), dim3(items), dim3(256), sh, s, a);                  \
    } while (0)
    // the weight rows ahead only while a workgroup per item still fits on the chip
    // at once (their registers halve the workgroups per compute unit)
    const bool ahead = items <= 2 * n_cu;
    if (a.width <= 128) {
        if (rt == 1) { if (ahead) RS_CURV(1, 8, 8); else RS_CURV(1, 8, 0); }
        else { if (ahead) RS_CURV(2, 8, 8); else RS_CURV(2, 8, 0); }
    } else {
        if (rt == 1) { if (ahead) RS_CURV(1, 16, 8); else RS_CURV(1, 16, 0); }
        else { if (ahead) RS_CURV(2, 16, 8); else RS_CURV(2, 16, 0); }
    }
#undef RS_CURV
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Newton control (float64).  Each item is either in the evaluation phase
// (ls_j < 0: needs g and H at z) or line-searching (ls_j >= 0).  One
// super-step evaluates every item of the first kind and the next trial steps
// of every item of the second kind; the lists are rebuilt on the device.
// ---------------------------------------------------------------------------
__global__ void k_newton_init(NewtonState st, int B)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    st.status[b] = RS_RUNNING;
    st.iters[b] = 0;
    st.g0[b] = 0.0;
    st.relgrad[b] = 0.0;
    st.ls_j[b] = -1;
}

hipError_t launch_newton_init(const NewtonState& st, int B, hipStream_t s)
{
    if (B <= 0) return hipSuccess;
    RS_LAUNCH(k_newton_init, dim3((B + 255) / 256), dim3(256), 0, s, st, B);
    return hipGetLastError();
}

// Inclusive prefix sum over a 1024-thread workgroup (wave scans, then the 16
// wave totals); `total` receives the sum.  sc: 16 ints of LDS, free again
// after the next barrier.
__device__ inline int block_scan1024(int v, int* sc, int& total)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int off = 1; off < 64; off <<= 1) {
        const int x = __shfl_up(v, off, 64);
        if (lane >= off) v += x;
    }
    if (lane == 63) sc[wv] = v;
    __syncthreads();
    int before = 0, tot = 0;
    for (int q = 0; q < 16; ++q) {
        const int t = sc[q];
        before += q < wv ? t : 0;
        tot += t;
    }
    total = tot;
    return before + v;
}

// The first evaluation list: items 0 .. A - 1 are admitted (A = B, or the
// window when it is smaller); later items enter in index order as admitted
// ones finish (k_armijo).
__global__ __launch_bounds__(1024) void k_compact_eval(NewtonState st, int B, int window)
{
    __shared__ int sc[16];
    const int tid = threadIdx.x;
    const int A = (window > 0 && window < B) ? window : B;
    int base = 0;
    for (int b0 = 0; b0 < A; b0 += 1024) {
        const int b = b0 + tid;
        const int f = (b < A && st.status[b] == RS_RUNNING && st.ls_j[b] < 0) ? 1 : 0;
        int tot;
        const int inc = block_scan1024(f, sc, tot);
        if (f) st.eval_list[base + inc - 1] = b;
        __syncthreads();
        base += tot;
    }
    if (tid == 0) {
        st.counters[0] = base;
        st.counters[4] = A;
        st.counters[5] = 0;
    }
}

hipError_t launch_compact_eval(const NewtonState& st, int B, int window, hipStream_t s)
{
    RS_LAUNCH(k_compact_eval, dim3(1), dim3(1024), 0, s, st, B, window);
    return hipGetLastError();
}

// alpha_j = shrink^j by repeated multiplication
__device__ inline double step_len(double shrink, int j)
{
    double a = 1.0;
    for (int q = 0; q < j; ++q) a *= shrink;
    return a;
}

// Candidate list and candidate points: an item on its first trial evaluates
// alpha = 1 only (the Newton step is usually accepted); later rounds evaluate
// kLsCand steps.  zc[c] = z[item] + alpha_j dz[item], written per chunk of 1024
// items with consecutive threads on consecutive coordinates.  Every workgroup
// of the grid runs the same prefix sums (the state they read is not written
// here); workgroup 0 alone writes the lists, and the candidate points of a
// chunk are split over the workgroups.  A search entry's step lengths are one
// running product (alpha_{j+1} = alpha_j * shrink), the same roundings as
// backtracking from alpha = 1.
constexpr int kSearchWgs = 8;
__global__ __launch_bounds__(1024) void k_compact_search(NewtonState st, NewtonParams p, int B)
{
    constexpr int NB = 8;  // coordinates per thread and batch (loads issued before stores)
    __shared__ int sc[16];
    __shared__ int it_b[1024];                  // chunk search entry -> item
    __shared__ short cl[1024 * kLsCand];        // chunk candidate -> chunk search entry
    __shared__ double ca[1024 * kLsCand];       // chunk candidate -> step length
    const int tid = threadIdx.x, r = p.r;
    const bool lead = blockIdx.x == 0;
    // admitted items (the others wait, ls_j < 0) from the lowest one still running
    const int A = min(B, st.counters[4]), lo = min(st.counters[5], A);
    int base_s = 0, base_c = 0;
    for (int b0 = lo; b0 < A; b0 += 1024) {
        const int b = b0 + tid;
        int f = 0, nc = 0, j = 0;
        if (b < A && st.status[b] == RS_RUNNING && st.ls_j[b] >= 0) {
            j = st.ls_j[b];
            f = 1;
            nc = min(j == 0 ? 1 : kLsCand, p.ls_max - j);
        }
        int tot;
        const int inc = block_scan1024((f << 16) | nc, sc, tot);
        const int ls = (inc >> 16) - 1, lc = (inc & 0xffff) - nc;
        if (f) {
            if (lead) {
                st.search_list[base_s + ls] = b;
                st.search_start[base_s + ls] = base_c + lc;
                st.search_ncand[base_s + ls] = nc;
            }
            it_b[ls] = b;
            double a = step_len(p.shrink, j);
            for (int t = 0; t < nc; ++t) {
                if (lead) {
                    st.cand_item[base_c + lc + t] = b;
                    st.cand_j[base_c + lc + t] = j + t;
                }
                cl[lc + t] = (short)ls;
                ca[lc + t] = a;
                a *= p.shrink;
            }
        }
        __syncthreads();
        const int ne = (tot & 0xffff) * r;
        double* zc = st.zc + (size_t)base_c * r;
        for (int e0 = blockIdx.x * 1024 * NB; e0 < ne; e0 += gridDim.x * 1024 * NB) {
            double zv[NB], dv[NB], av[NB];
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const int e = e0 + q * 1024 + tid;
                zv[q] = dv[q] = av[q] = 0.0;
                if (e < ne) {
                    const int c = e / r, k = e - c * r, it = it_b[cl[c]];
                    zv[q] = st.z[(size_t)it * r + k];
                    dv[q] = st.dz[(size_t)it * r + k];
                    av[q] = ca[c];
                }
            }
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const int e = e0 + q * 1024 + tid;
                if (e < ne) zc[e] = zv[q] + av[q] * dv[q];
            }
        }
        __syncthreads(); // the chunk's LDS tables are reused
        base_s += tot >> 16;
        base_c += tot & 0xffff;
    }
    if (lead && tid == 0) {
        st.counters[1] = base_c;
        st.counters[2] = base_s;
        if (st.plog) {
            st.plog[0] = st.counters[0];
            st.plog[1] = base_c;
            st.plog[2] = base_s;
        }
    }
}

hipError_t launch_compact_search(const NewtonState& st, const NewtonParams& p, int B, hipStream_t s)
{
    RS_LAUNCH(k_compact_search, dim3(kSearchWgs), dim3(1024), 0, s, st, p, B);
    return hipGetLastError();
}

// Lane l receives lane l - 1's value (dpp_from_prev) or lane l + 1's
// (dpp_from_next) within its 16-lane row (DPP row_shr:1 / row_shl:1); the
// first / last lane of a row keeps its own value.
__device__ inline double dpp_from_prev(double x)
{
    const int lo = __double2loint(x), hi = __double2hiint(x);
    return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, 0x111, 0xF, 0xF, false),
                            __builtin_amdgcn_update_dpp(lo, lo, 0x111, 0xF, 0xF, false));
}
__device__ inline double dpp_from_next(double x)
{
    const int lo = __double2loint(x), hi = __double2hiint(x);
    return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, 0x101, 0xF, 0xF, false),
                            __builtin_amdgcn_update_dpp(lo, lo, 0x101, 0xF, 0xF, false));
}

// 1/sqrt(x) and 1/x for positive normal x: the hardware estimate refined by two
// Newton steps (y <- y (3 - x y^2) / 2 and y <- y (2 - x y)), each of which
// squares the relative error.
__device__ inline double rsq_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const double h = 0.5 * x * y;
        y = fma(y, fma(-h, y, 0.5), y);
    }
    return y;
}
__device__ inline double rcp_nr(double x)
{
    double y = __builtin_amdgcn_rcp(x);
#pragma unroll
    for (int i = 0; i < 2; ++i) y = fma(y, fma(-x, y, 1.0), y);
    return y;
}

// Jacobi sweeps stop once the squared off-diagonal norm is below this
// fraction of the squared Frobenius norm: off-diagonal entries at 1e-12 of the
// matrix leave eigenvalue errors of order 1e-24 relative (second order) and
// eigenvector errors of order 1e-12, far inside what the projected step needs.
constexpr double kJacobiTol = 1e-24;

// Parallel Jacobi eigen-decomposition of a symmetric n2 x n2 matrix (n2 even,
// n2 <= 16) held in registers of one wave (Brent-Luk layout).  The indices are
// paired by slot: slot k pairs (t_k, b_k), and one step rotates all n2/2 pairs
// at once.  Lane (I, J) = (lane / 8, lane % 8) holds the 2x2 block of rows
// {t_I, b_I} and columns {t_J, b_J} of the matrix, and of V the rows
// {2I, 2I+1} (fixed coordinates) and columns {t_J, b_J}.  After each step the
// indices move one slot along the circle t_1 -> t_2 -> ... -> t_{m-1} ->
// b_{m-1} -> ... -> b_0 -> t_1 (t_0 stays), the round-robin order in which all
// pairs meet once per n2 - 1 steps; a row moves only between lanes I +- 1 and a
// column only between lanes J +- 1.  On return Hs[k][k] holds the eigenvalue of
// slot k and column k of Vs its eigenvector (k < n2).  Rows and columns >= r
// are zero (a dummy index when r is odd: its rotations are the identity).
__device__ void jacobi_wave(double (*Hs)[kMaxR + 1], double (*Vs)[kMaxR + 1], int r, int n2, int tid)
{
    const int m = n2 / 2;
    const int I = tid >> 3, J = tid & 7;
    const bool act = I < m && J < m;
    auto hget = [&](int a, int b) { return (act && a < r && b < r) ? Hs[a][b] : 0.0; };
    double htt = hget(2 * I, 2 * J), htb = hget(2 * I, 2 * J + 1);
    double hbt = hget(2 * I + 1, 2 * J), hbb = hget(2 * I + 1, 2 * J + 1);
    double v00 = (act && I == J) ? 1.0 : 0.0, v01 = 0.0, v10 = 0.0, v11 = v00;
    const int dI = I * 9, dJ = J * 9; // lanes of the diagonal blocks (I, I) and (J, J)
    for (int sweep = 0; sweep < 40; ++sweep) {
        double tot = act ? htt * htt + htb * htb + hbt * hbt + hbb * hbb : 0.0;
        double off = (I == J) ? (act ? htb * htb + hbt * hbt : 0.0) : tot;
        for (int o = 32; o > 0; o >>= 1) {
            off += __shfl_xor(off, o);
            tot += __shfl_xor(tot, o);
        }
        off = __shfl(off, 0); // one decision for the whole wave
        tot = __shfl(tot, 0);
        if (off <= kJacobiTol * tot || off == 0.0) break;
        for (int step = 0; step < n2 - 1; ++step) {
            double c = 1.0, sn = 0.0;
            if (I == J && htb != 0.0) {
                // smaller root of t^2 + 2 theta t - 1 = 0, theta = d / (2 a_pq),
                // written as t = 2 a_pq / (d + sgn(d) sqrt(d^2 + 4 a_pq^2))
                // (reciprocal square roots and reciprocals from the hardware
                // estimates refined by two Newton steps: a short dependent chain)
                const double d = hbb - htt, two_apq = 2.0 * htb;
                const double x = d * d + two_apq * two_apq;
                const double root = x * rsq_nr(x);
                const double t = two_apq * rcp_nr(d >= 0.0 ? d + root : d - root);
                c = rsq_nr(t * t + 1.0);
                sn = t * c;
            }
            const double cI = __shfl(c, dI), sI = __shfl(sn, dI);
            const double cJ = __shfl(c, dJ), sJ = __shfl(sn, dJ);
            // rows: [t; b] <- [[c, -s], [s, c]] [t; b] with slot I's rotation
            const double rt0 = cI * htt - sI * hbt, rt1 = cI * htb - sI * hbb;
            const double rb0 = sI * htt + cI * hbt, rb1 = sI * htb + cI * hbb;
            // columns (and V's columns) with slot J's rotation
            htt = cJ * rt0 - sJ * rt1;
            htb = sJ * rt0 + cJ * rt1;
            hbt = cJ * rb0 - sJ * rb1;
            hbb = sJ * rb0 + cJ * rb1;
            if (I == J) htb = hbt = 0.0; // the annihilated pair
            {
                const double a0 = cJ * v00 - sJ * v01, a1 = sJ * v00 + cJ * v01;
                const double b0 = cJ * v10 - sJ * v11, b1 = sJ * v10 + cJ * v11;
                v00 = a0; v01 = a1; v10 = b0; v11 = b1;
            }
            if (m == 1) continue;
            // move the rows: new t_I <- old t_{I-1} (I >= 2) or old b_0 (I == 1);
            // new b_I <- old b_{I+1} (I < m-1) or old t_{m-1} (I == m-1)
            {
                const double d0 = (I == 0) ? hbt : htt, d1 = (I == 0) ? hbb : htb;
                const double up0 = __shfl(d0, tid - 8), up1 = __shfl(d1, tid - 8);
                const double dn0 = __shfl(hbt, tid + 8), dn1 = __shfl(hbb, tid + 8);
                const double nb0 = (I == m - 1) ? htt : dn0, nb1 = (I == m - 1) ? htb : dn1;
                if (I != 0) { htt = up0; htb = up1; }
                hbt = nb0; hbb = nb1;
            }
            // move the columns the same way along J (H and V): lanes J +- 1
            // share a 16-lane DPP row, so these are row shifts
            {
                const double d0 = (J == 0) ? htb : htt, d1 = (J == 0) ? hbb : hbt;
                const double e0 = (J == 0) ? v01 : v00, e1 = (J == 0) ? v11 : v10;
                const double lf0 = dpp_from_prev(d0), lf1 = dpp_from_prev(d1);
                const double lv0 = dpp_from_prev(e0), lv1 = dpp_from_prev(e1);
                const double rt_0 = dpp_from_next(htb), rt_1 = dpp_from_next(hbb);
                const double rv0 = dpp_from_next(v01), rv1 = dpp_from_next(v11);
                const bool last = (J == m - 1);
                const double nb0 = last ? htt : rt_0, nb1 = last ? hbt : rt_1;
                const double nv0 = last ? v00 : rv0, nv1 = last ? v10 : rv1;
                if (J != 0) { htt = lf0; hbt = lf1; v00 = lv0; v10 = lv1; }
                htb = nb0; hbb = nb1; v01 = nv0; v11 = nv1;
            }
        }
    }
    __syncthreads();
    if (act) {
        if (I == J) {
            Hs[2 * J][2 * J] = htt;
            Hs[2 * J + 1][2 * J + 1] = hbb;
        }
        Vs[2 * I][2 * J] = v00;
        Vs[2 * I][2 * J + 1] = v01;
        Vs[2 * I + 1][2 * J] = v10;
        Vs[2 * I + 1][2 * J + 1] = v11;
    }
    __syncthreads();
}

__device__ inline double readlane_f64(double x, int l)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l),
                            __builtin_amdgcn_readlane(__double2loint(x), l));
}

// Solve H x = -g (r <= 16) by Gauss-Jordan elimination without pivoting,
// lane a (mod 16) holding row a of [H | -g] in registers, the pivot row
// broadcast from its lane at each step; rows past r are identity rows.  For a
// symmetric H the pivots are the squares of the Cholesky diagonal, so every
// pivot is positive exactly when H is positive definite: returns 0 (x
// undefined) at the first pivot that is not, else 1 with x = x_a.
__device__ inline int gauss_jordan16(const double (*Hs)[kMaxR + 1], const double* gs, int r, int tid, double& x)
{
    const int a = tid & 15;
    double h[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) h[k] = (a < r && k < r) ? Hs[a][k] : (a == k ? 1.0 : 0.0);
    double b = a < r ? -gs[a] : 0.0, diag = 1.0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const double piv = readlane_f64(h[j], j);
        if (!(piv > 0.0) || !isfinite(piv)) return 0; // wave-uniform
        const double f = (a == j) ? 0.0 : h[j] / piv;
        if (a == j) diag = piv;
        b -= f * readlane_f64(b, j);
#pragma unroll
        for (int k = j + 1; k < 16; ++k) h[k] -= f * readlane_f64(h[k], j);
    }
    x = b / diag;
    return 1;
}

// Exit tests and the Newton direction of one item per 64-thread workgroup:
// the solve with the symmetrised Hessian if it is positive definite
// (Cholesky, or for r <= 16 the equivalent Gauss-Jordan test), else a
// Jacobi eigen-decomposition (parallel ordering: the r/2 disjoint rotations
// of one round-robin step are applied together) and the projected (clamped /
// absolute) eigenvalues.  All in float64.
__global__ __launch_bounds__(64) void k_newton_dir(NewtonState st, NewtonParams p)
{
    __shared__ double Hs[kMaxR][kMaxR + 1];
    __shared__ double Ls[kMaxR][kMaxR + 1];
    __shared__ double Vs[kMaxR][kMaxR + 1];
    __shared__ double gs[kMaxR], dzs[kMaxR], cs[kMaxR], lam[kMaxR];
    __shared__ double rc[kMaxR / 2], rs_[kMaxR / 2];
    __shared__ int rp[kMaxR / 2], rq[kMaxR / 2];
    const int i = blockIdx.x, tid = threadIdx.x, r = p.r;
    if (i >= st.counters[0]) return;
    const int item = st.eval_list[i];
    const double* gw = st.gw + (size_t)i * r;
    const double* Hw = st.Hw + (size_t)i * r * r;
    for (int q = tid; q < r; q += 64) gs[q] = gw[q];
    for (int q = tid; q < r * r; q += 64) {
        const int a = q / r, b = q - a * r;
        const double h = 0.5 * (Hw[a * r + b] + Hw[b * r + a]);
        Hs[a][b] = h;
        Ls[a][b] = h;
    }
    __syncthreads();
    {
        // exit tests, all lanes in parallel (max and min are exact, so every
        // lane ends with the same values; lane 0's are used anyway)
        double gn = 0.0;
        int fin = 1;
        for (int q = tid; q < r; q += 64) {
            gn = fmax(gn, fabs(gs[q]));
            if (!isfinite(gs[q])) fin = 0;
        }
        for (int q = tid; q < r * r; q += 64)
            if (!isfinite(Hs[q / r][q % r])) fin = 0;
        for (int o = 32; o > 0; o >>= 1) {
            gn = fmax(gn, __shfl_xor(gn, o));
            fin = min(fin, __shfl_xor(fin, o));
        }
        gn = __shfl(gn, 0);
        fin = __shfl(fin, 0) && isfinite(st.E[item]);
        const int it = st.iters[item];
        const double g0 = (it == 0) ? gn : st.g0[item];
        int status = RS_RUNNING;
        if (!fin) status = RS_NONFINITE;
        else if (gn <= p.abs_tol || gn <= p.rel_tol * g0) status = RS_CONVERGED;
        else if (it >= p.max_iter) status = RS_ITER_MAX;
        if (tid == 0) {
            if (it == 0) st.g0[item] = gn;
            st.relgrad[item] = g0 > 0.0 ? gn / g0 : 0.0;
            if (status != RS_RUNNING) st.status[item] = status;
        }
        if (status != RS_RUNNING) return;
    }

    int chol_ok = 1;
    if (r <= 16) {
        // registers and lane broadcasts (no LDS round trips, no barriers)
        double x;
        chol_ok = gauss_jordan16(Hs, gs, r, tid, x);
        if (chol_ok && tid < r) dzs[tid] = x;
        __syncthreads();
    } else {
        // right-looking Cholesky of the symmetrised Hessian (lower factor in Ls)
        for (int j = 0; j < r; ++j) {
            const double d = Ls[j][j];
            __syncthreads();
            if (!(d > 0.0) || !isfinite(d)) {
                chol_ok = 0;
                break;
            }
            const double ljj = sqrt(d);
            if (tid == 0) Ls[j][j] = ljj;
            for (int a = j + 1 + tid; a < r; a += 64) Ls[a][j] /= ljj;
            __syncthreads();
            const int m = r - j - 1;
            for (int w = tid; w < m * m; w += 64) {
                const int a = j + 1 + w / m, b = j + 1 + w % m;
                if (b <= a) Ls[a][b] -= Ls[a][j] * Ls[b][j];
            }
            __syncthreads();
        }
        if (chol_ok) {
            // L y = -g, then L^T dz = y, one column per step
            for (int q = tid; q < r; q += 64) cs[q] = -gs[q];
            __syncthreads();
            for (int j = 0; j < r; ++j) {
                const double yj = cs[j] / Ls[j][j];
                __syncthreads();
                if (tid == 0) cs[j] = yj;
                for (int a = j + 1 + tid; a < r; a += 64) cs[a] -= Ls[a][j] * yj;
                __syncthreads();
            }
            for (int j = r - 1; j >= 0; --j) {
                const double dj = cs[j] / Ls[j][j];
                __syncthreads();
                if (tid == 0) dzs[j] = dj;
                for (int a = tid; a < j; a += 64) cs[a] -= Ls[j][a] * dj;
                __syncthreads();
            }
        }
    }
    if (chol_ok) {
    } else if (p.proj == RS_PROJ_NONE) {
        if (tid == 0) st.status[item] = RS_NOT_DESCENT;
        return;
    } else {
        const int n2 = (r + 1) & ~1; // players of the round-robin (one dummy if r is odd)
        int ns = r;                  // eigen slots
        if (n2 <= 16) {
            jacobi_wave(Hs, Vs, r, n2, tid);
            ns = n2;
        } else {
            for (int q = tid; q < r * r; q += 64) {
                const int a = q / r, b = q - a * r;
                Vs[a][b] = (a == b) ? 1.0 : 0.0;
            }
            const int P = n2 / 2;
            for (int sweep = 0; sweep < 40; ++sweep) {
                __syncthreads();
                double off = 0.0, tot = 0.0;
                for (int q = tid; q < r * r; q += 64) {
                    const int a = q / r, b = q - a * r;
                    const double h2 = Hs[a][b] * Hs[a][b];
                    tot += h2;
                    if (a != b) off += h2;
                }
                for (int o = 32; o > 0; o >>= 1) {
                    off += __shfl_xor(off, o);
                    tot += __shfl_xor(tot, o);
                }
                // lane 0 decides for the whole wave (barriers follow)
                off = __shfl(off, 0);
                tot = __shfl(tot, 0);
                if (off <= kJacobiTol * tot || off == 0.0) break;
                for (int step = 0; step < n2 - 1; ++step) {
                    if (tid < P) {
                        const int m1 = tid, m2 = n2 - 1 - tid;
                        const int a = m1 == 0 ? 0 : ((m1 - 1 + step) % (n2 - 1)) + 1;
                        const int b = ((m2 - 1 + step) % (n2 - 1)) + 1;
                        const int pp = a < b ? a : b, qq = a < b ? b : a;
                        double c = 1.0, sn = 0.0;
                        if (qq < r) {
                            const double apq = Hs[pp][qq];
                            if (apq != 0.0) {
                                const double theta = (Hs[qq][qq] - Hs[pp][pp]) / (2.0 * apq);
                                const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                                c = 1.0 / sqrt(t * t + 1.0);
                                sn = t * c;
                            }
                        }
                        rp[tid] = pp;
                        rq[tid] = qq;
                        rc[tid] = c;
                        rs_[tid] = sn;
                    }
                    __syncthreads();
                    for (int w = tid; w < P * r; w += 64) { // rows p, q
                        const int pr = w / r, col = w - pr * r;
                        const int pp = rp[pr], qq = rq[pr];
                        if (qq >= r) continue;
                        const double c = rc[pr], sn = rs_[pr];
                        const double apk = Hs[pp][col], aqk = Hs[qq][col];
                        Hs[pp][col] = c * apk - sn * aqk;
                        Hs[qq][col] = sn * apk + c * aqk;
                    }
                    __syncthreads();
                    for (int w = tid; w < P * r; w += 64) { // columns p, q and eigenvectors
                        const int pr = w / r, row = w - pr * r;
                        const int pp = rp[pr], qq = rq[pr];
                        if (qq >= r) continue;
                        const double c = rc[pr], sn = rs_[pr];
                        const double akp = Hs[row][pp], akq = Hs[row][qq];
                        Hs[row][pp] = c * akp - sn * akq;
                        Hs[row][qq] = sn * akp + c * akq;
                        const double vkp = Vs[row][pp], vkq = Vs[row][qq];
                        Vs[row][pp] = c * vkp - sn * vkq;
                        Vs[row][qq] = sn * vkp + c * vkq;
                    }
                    __syncthreads();
                }
            }
        }
        __syncthreads();
        if (tid == 0) {
            double lmax = 0.0;
            for (int k = 0; k < ns; ++k) lmax = fmax(lmax, fabs(Hs[k][k]));
            const double fl = p.eig_floor * lmax;
            for (int k = 0; k < ns; ++k) {
                double lk = (p.proj == RS_PROJ_ABS) ? fabs(Hs[k][k]) : Hs[k][k];
                if (lk < fl) lk = fl;
                if (!(lk > 0.0)) lk = 1.0;
                lam[k] = lk;
            }
        }
        __syncthreads();
        if (tid < ns) {
            double c = 0.0;
            for (int a = 0; a < r; ++a) c += Vs[a][tid] * gs[a];
            cs[tid] = c / lam[tid];
        }
        __syncthreads();
        if (tid < r) {
            double d = 0.0;
            for (int k = 0; k < ns; ++k) d -= Vs[tid][k] * cs[k];
            dzs[tid] = d;
        }
        __syncthreads();
    }
    if (tid == 0) {
        double slope = 0.0;
        for (int a = 0; a < r; ++a) slope += gs[a] * dzs[a];
        if (!(slope < 0.0)) {
            st.status[item] = RS_NOT_DESCENT;
        } else if (p.ls_max <= 0) {
            st.status[item] = RS_LS_MAX;
        } else {
            st.slope[item] = slope;
            st.ls_j[item] = 0;
        }
    }
    for (int a = tid; a < r; a += 64) st.dz[(size_t)item * r + a] = dzs[a];
}

hipError_t launch_newton_dir(const NewtonState& st, const NewtonParams& p, int cap, hipStream_t s)
{
    if (cap <= 0) return hipSuccess;
    RS_LAUNCH(k_newton_dir, dim3(cap), dim3(64), 0, s, st, p);
    return hipGetLastError();
}

// Sum over the wave; every lane ends with the same value (the butterfly adds
// the same pairs in every lane, and addition is commutative).
__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// DPP move of a double within 16-lane rows (ctrl: a DPP control word)
template <int CTRL>
__device__ inline double dpp_f64(double x)
{
    const int lo = __double2loint(x), hi = __double2hiint(x);
    return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xF, 0xF, false),
                            __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xF, 0xF, false));
}

// Sum of lanes 0..15 (the other lanes' values are ignored), the same in every
// lane: within each 16-lane row, pairs (quad_perm 1,0,3,2), quads (quad_perm
// 2,3,0,1), half rows (row_half_mirror) and rows (row_mirror) are added, all
// in DPP; row 0's total is then read out of lane 0.
__device__ inline double row0_sum(double v)
{
    v += dpp_f64<0xB1>(v);
    v += dpp_f64<0x4E>(v);
    v += dpp_f64<0x141>(v);
    v += dpp_f64<0x140>(v);
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 0),
                            __builtin_amdgcn_readlane(__double2loint(v), 0));
}

// L-BFGS direction of one item per 64-thread workgroup, lane k holding
// component k: the exit tests of k_newton_dir, then the pair of the step just
// accepted (s = z - z_prev, y = g - g_prev, kept only when s.y > 0, the oldest
// dropped when the ring is full), then the two-loop recursion
//   q = g; for pairs newest first: a_i = s_i.q / s_i.y_i, q -= a_i y_i;
//   q *= s_n.y_n / y_n.y_n (newest pair; 1 without pairs);
//   for pairs oldest first: b = y_i.q / s_i.y_i, q += (a_i - b) s_i;
// and dz = -q.  All in float64.
__global__ __launch_bounds__(64) void k_lbfgs_dir(NewtonState st, NewtonParams p, LbfgsState h)
{
    constexpr int M = RS_MAX_HISTORY;
    const int i = blockIdx.x, lane = threadIdx.x, r = p.r;
    if (i >= st.counters[0]) return;
    const int item = st.eval_list[i];
    const bool kl = lane < r;
    // lanes 0..15 hold every component when r <= 16: row-local DPP sums
    auto vsum = [&](double x) { return r <= 16 ? row0_sum(x) : wave_sum(x); };
    const double g = kl ? st.gw[(size_t)i * r + lane] : 0.0;
    double gn = kl ? fabs(g) : 0.0;
    int fin = kl ? (isfinite(g) ? 1 : 0) : 1;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        gn = fmax(gn, __shfl_xor(gn, o));
        fin = min(fin, __shfl_xor(fin, o));
    }
    fin = fin && isfinite(st.E[item]);
    const int it = st.iters[item];
    const double g0 = (it == 0) ? gn : st.g0[item];
    int status = RS_RUNNING;
    if (!fin) status = RS_NONFINITE;
    else if (gn <= p.abs_tol || gn <= p.rel_tol * g0) status = RS_CONVERGED;
    else if (it >= p.max_iter) status = RS_ITER_MAX;
    if (lane == 0) {
        if (it == 0) st.g0[item] = gn;
        st.relgrad[item] = g0 > 0.0 ? gn / g0 : 0.0;
        if (status != RS_RUNNING) st.status[item] = status;
    }
    if (status != RS_RUNNING) return;

    const int m = p.hist;
    const size_t hb = (size_t)item * M;
    const double zk = kl ? st.z[(size_t)item * r + lane] : 0.0;
    int np = (it == 0) ? 0 : h.npair[item];
    int head = (it == 0) ? 0 : h.head[item];
    if (it > 0 && m > 0) {
        const double sv = kl ? zk - h.zprev[(size_t)item * r + lane] : 0.0;
        const double yv = kl ? g - h.gprev[(size_t)item * r + lane] : 0.0;
        const double sy = vsum(sv * yv);
        if (sy > 0.0) {
            int slot;
            if (np < m) {
                slot = head + np;
                if (slot >= m) slot -= m;
                ++np;
            } else {
                slot = head;
                head = head + 1 == m ? 0 : head + 1;
            }
            if (kl) {
                h.S[(hb + slot) * r + lane] = sv;
                h.Y[(hb + slot) * r + lane] = yv;
            }
            if (lane == 0) h.sy[hb + slot] = sy;
        }
    }
    // the item's pairs, oldest first, in registers
    double sj[M], yj[M], syj[M], aj[M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
        int slot = head + j;
        if (slot >= m) slot -= m;
        const bool in = j < np;
        sj[j] = (in && kl) ? h.S[(hb + slot) * r + lane] : 0.0;
        yj[j] = (in && kl) ? h.Y[(hb + slot) * r + lane] : 0.0;
        syj[j] = in ? h.sy[hb + slot] : 1.0;
        aj[j] = 0.0;
    }
    double q = g;
#pragma unroll
    for (int j = M - 1; j >= 0; --j) {
        if (j >= np) continue;
        aj[j] = vsum(sj[j] * q) / syj[j];
        q -= aj[j] * yj[j];
    }
    if (np > 0) {
        double yy = 0.0, syn = 0.0;
#pragma unroll
        for (int j = 0; j < M; ++j)
            if (j == np - 1) {
                yy = vsum(yj[j] * yj[j]);
                syn = syj[j];
            }
        q *= syn / yy;
    }
#pragma unroll
    for (int j = 0; j < M; ++j) {
        if (j >= np) continue;
        const double b = vsum(yj[j] * q) / syj[j];
        q += sj[j] * (aj[j] - b);
    }
    const double d = kl ? -q : 0.0;
    const double slope = vsum(g * d);
    if (lane == 0) {
        h.npair[item] = np;
        h.head[item] = head;
        if (!(slope < 0.0)) {
            st.status[item] = RS_NOT_DESCENT;
        } else if (p.ls_max <= 0) {
            st.status[item] = RS_LS_MAX;
        } else {
            st.slope[item] = slope;
            st.ls_j[item] = 0;
        }
    }
    if (kl) {
        st.dz[(size_t)item * r + lane] = d;
        h.zprev[(size_t)item * r + lane] = zk;
        h.gprev[(size_t)item * r + lane] = g;
    }
}

hipError_t launch_lbfgs_dir(const NewtonState& st, const NewtonParams& p, const LbfgsState& h, int cap,
                            hipStream_t s)
{
    if (cap <= 0) return hipSuccess;
    if (p.hist < 0 || p.hist > RS_MAX_HISTORY || p.r > 64) return hipErrorInvalidValue;
    RS_LAUNCH(k_lbfgs_dir, dim3(cap), dim3(64), 0, s, st, p, h);
    return hipGetLastError();
}

// Armijo test on the float64 candidate energies: accept the first (largest)
// step with E(z + a dz) - E(z) <= c1 a g.dz, as sequential backtracking would.
// End of a super-step in one workgroup: the Armijo test of every searching
// item over its candidates (first acceptable step length, in order), then
// the evaluation list of the next super-step and the count of items still
// running (also stored to `host`, coherent mapped host memory, as one 64-bit system-scope release store of
// (tag << 32) | count, so that the reader can tell this super-step's count from an older one; may be NULL).
__global__ __launch_bounds__(1024) void k_armijo(NewtonState st, NewtonParams p, int B, unsigned long long* host,
                                                 unsigned int tag)
{
    constexpr int NB = 16;
    __shared__ int sc[16];
    __shared__ int acc_item[1024], acc_cand[1024]; // accepted candidate per chunk search entry (-1: none)
    const int tid = threadIdx.x, r = p.r;
    const int ns = st.counters[2];
    const int A = min(B, st.counters[4]), lo = min(st.counters[5], A); // admitted items, lowest running
    __shared__ int lo_next;
    if (tid == 0) lo_next = A;
    for (int i0 = 0; i0 < ns; i0 += 1024) {
        const int i = i0 + tid;
        int item = -1, cand = -1;
        if (i < ns) {
            item = st.search_list[i];
            const int start = st.search_start[i], nc = st.search_ncand[i];
            const double E0 = st.E[item], slope = st.slope[item];
            const int j0 = st.ls_j[item];
            double Ev[kLsCand]; // all candidate energies in flight at once
#pragma unroll
            for (int t = 0; t < kLsCand; ++t) Ev[t] = t < nc ? st.Ec[start + t] : 0.0;
            double alpha = step_len(p.shrink, j0);
#pragma unroll
            for (int t = 0; t < kLsCand; ++t, alpha *= p.shrink) {
                if (t >= nc || cand >= 0) break;
                const double Et = Ev[t];
                if (isfinite(Et) && Et - E0 <= p.c1 * alpha * slope) {
                    cand = start + t;
                    st.E[item] = Et;
                    st.iters[item] += 1;
                    st.ls_j[item] = -1;
                }
            }
            if (cand < 0) {
                const int jn = j0 + nc;
                if (jn >= p.ls_max) st.status[item] = RS_LS_MAX;
                else st.ls_j[item] = jn;
            }
        }
        acc_item[tid] = item;
        acc_cand[tid] = cand;
        __syncthreads();
        // accepted points, consecutive threads on consecutive coordinates
        const int ne = min(1024, ns - i0) * r;
        for (int e0 = 0; e0 < ne; e0 += 1024 * NB) {
            double v[NB];
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const int e = e0 + q * 1024 + tid;
                v[q] = 0.0;
                if (e < ne) {
                    const int li = e / r, cnd = acc_cand[li];
                    if (cnd >= 0) v[q] = st.zc[(size_t)cnd * r + e - li * r];
                }
            }
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const int e = e0 + q * 1024 + tid;
                if (e < ne) {
                    const int li = e / r;
                    if (acc_cand[li] >= 0) st.z[(size_t)acc_item[li] * r + e - li * r] = v[q];
                }
            }
        }
        __syncthreads();
    }
    __syncthreads(); // statuses and trial indices of this super-step are final
    int base = 0, running = 0;
    for (int b0 = lo; b0 < A; b0 += 1024) {
        const int b = b0 + tid;
        const int run = (b < A && st.status[b] == RS_RUNNING) ? 1 : 0;
        const unsigned long long rm = __ballot(run); // one LDS atomic per wave: its lowest running item
        if (rm && (tid & 63) == 0) atomicMin(&lo_next, b + __ffsll((long long)rm) - 1);
        const int f = (run && st.ls_j[b] < 0) ? 1 : 0;
        int tot;
        const int inc = block_scan1024((f << 16) | run, sc, tot);
        if (f) st.eval_list[base + (inc >> 16) - 1] = b;
        __syncthreads();
        base += tot >> 16;
        running += tot & 0xffff;
    }
    // items waiting for the window enter in index order (their first evaluation
    // is next; newton_init set their state and the first energy pass their E)
    const int adm = (p.window > 0 && A < B) ? max(0, min(p.window - running, B - A)) : 0;
    for (int t = tid; t < adm; t += 1024) st.eval_list[base + t] = A + t;
    base += adm;
    running += adm;
    if (tid == 0) {
        st.counters[0] = base;
        st.counters[3] = running;
        st.counters[4] = A + adm;
        st.counters[5] = lo_next; // items below it have all ended (A when none of [lo, A) runs)
        if (host)
            __hip_atomic_store(host, ((unsigned long long)tag << 32) | (unsigned int)running, __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

hipError_t launch_armijo(const NewtonState& st, const NewtonParams& p, int B, unsigned long long* host,
                         unsigned int tag, hipStream_t s)
{
    RS_LAUNCH(k_armijo, dim3(1), dim3(1024), 0, s, st, p, B, host, tag);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Lipschitz loss pieces
// ---------------------------------------------------------------------------
__global__ void k_stack_pairs(const double* z1, const double* z2, double* zs, int B, int r)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * r) return;
    const int b = idx / r, k = idx - b * r;
    zs[(size_t)(2 * b) * r + k] = z1[idx];
    zs[(size_t)(2 * b + 1) * r + k] = z2[idx];
}

hipError_t launch_stack_pairs(const double* z1, const double* z2, double* zs, int B, int r, hipStream_t s)
{
    if (B <= 0) return hipSuccess;
    RS_LAUNCH(k_stack_pairs, dim3((B * r + 255) / 256), dim3(256), 0, s, z1, z2, zs, B, r);
    return hipGetLastError();
}

// per pair: |H(z1)-H(z2)|_F^2 / |z1-z2|^2 (pair b's Hessians are items 2b, 2b+1);
// one wave per pair, lanes over the entries (coalesced), a fixed butterfly sum
__global__ __launch_bounds__(256) void k_lip_pairs(const double* z1, const double* z2, const double* H, int B, int r,
                                                   double* per_pair, double* ell)
{
    const int lane = threadIdx.x & 63;
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= B) return;
    double dz2 = 0.0, f = 0.0;
    for (int k = lane; k < r; k += 64) {
        const double d = z1[(size_t)b * r + k] - z2[(size_t)b * r + k];
        dz2 += d * d;
    }
    const double* H1 = H + (size_t)(2 * b) * r * r;
    const double* H2 = H1 + (size_t)r * r;
    for (int q = lane; q < r * r; q += 64) {
        const double d = H1[q] - H2[q];
        f += d * d;
    }
    for (int o = 32; o > 0; o >>= 1) {
        dz2 += __shfl_xor(dz2, o);
        f += __shfl_xor(f, o);
    }
    if (lane == 0) {
        const double v = dz2 > 0.0 ? f / dz2 : -1.0;
        ell[b] = v;
        if (per_pair) per_pair[b] = v < 0.0 ? 0.0 : v;
    }
}

// acc = {sum, count, max sqrt}; carried over chunks, finalised on the last one
__global__ __launch_bounds__(256) void k_lip_reduce(const double* ell, int B, double* acc, int first,
                                                    int last, double* loss, int* n_valid, double* lip_max)
{
    __shared__ double ss[256], sn[256], sm[256];
    const int tid = threadIdx.x;
    double s = 0.0, n = 0.0, m = 0.0;
    for (int b = tid; b < B; b += 256) {
        const double v = ell[b];
        if (v >= 0.0) {
            s += v;
            n += 1.0;
            m = fmax(m, sqrt(v));
        }
    }
    ss[tid] = s; sn[tid] = n; sm[tid] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
            ss[tid] += ss[tid + w];
            sn[tid] += sn[tid + w];
            sm[tid] = fmax(sm[tid], sm[tid + w]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        if (first) { acc[0] = 0.0; acc[1] = 0.0; acc[2] = 0.0; }
        acc[0] += ss[0];
        acc[1] += sn[0];
        acc[2] = fmax(acc[2], sm[0]);
        if (last) {
            *loss = acc[1] > 0.0 ? acc[0] / acc[1] : 0.0;
            *n_valid = (int)acc[1];
            if (lip_max) *lip_max = acc[2];
        }
    }
}

hipError_t launch_lipschitz(const double* z1, const double* z2, const double* H, int B, int r,
                            double* per_pair, double* ell, double* acc, int first_chunk, int last_chunk,
                            double* loss, int* n_valid, double* lip_max, hipStream_t s)
{
    if (B > 0)
        RS_LAUNCH(k_lip_pairs, dim3((B + 3) / 4), dim3(256), 0, s, z1, z2, H, B, r, per_pair, ell);
    RS_LAUNCH(k_lip_reduce, dim3(1), dim3(256), 0, s, ell, B, acc, first_chunk, last_chunk, loss,
                       n_valid, lip_max);
    return hipGetLastError();
}

}  // namespace rs
