// Host side of the librs C ABI: argument checks, the device layout of one
// reduced problem, and the batched, device-resident Newton driver.
//
// The reduced output map.  Every quantity the reduced objective needs from
// the decoder output u = W_out h_L + b_out is a linear function of h_L, so the
// context folds it into one matrix W_big (rows x width) applied to
// [h_L | dh_L/dz] by a single GEMM per evaluation:
//   - 9 rows per cubature tet e: the displacement gradient grad u_e = D_e u_e
//     (D_e the constant 9x12 map of the linear tet, F = I + grad u), so
//     F_e and K_e = dvecF_e/dz come straight out of the GEMM (Sec. 4.3: only
//     the cubature tets S are ever evaluated);
//   - 3 rows per penalty-targeted vertex (its displacement);
//   - 1 gravity row: sum_v m_v g . u_v over every vertex (lumped masses);
//   - 3 force rows: the summed displacement of the force-loaded vertices.
// Pinned vertices have their W_out/b_out rows zeroed (q = X + m (.) f(z)).
#include "rs_internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

using namespace rs;

namespace {

int round_up(int v, int m) { return ((v + m - 1) / m) * m; }

enum Kind {
    K_GEMM_HIDDEN, K_GEMM_OUT, K_ELEM, K_GEMM_ADJ, K_CURV, K_COMPACT, K_DIR,
    K_LS_GEMM_HIDDEN, K_LS_GEMM_OUT, K_ENERGY, K_ARMIJO, K_LIPSCHITZ, K_DECODE_HIDDEN, K_DECODE_OUT,
    K_INIT, K_ACTIVATE, K_LBFGS, K_PARAM_GRAD, K_ELEM_PSD, K_ELEM_DUMP, K_LIP_GRAD, K_TRAIN, K_DYN, K_ELEM_FUSED, K_COUNT
};
const char* kKindName[K_COUNT] = {
    "gemm_hidden", "gemm_out", "elem", "gemm_adjoint", "curv", "compact", "newton_dir",
    "ls_gemm_hidden", "ls_gemm_out", "energy_f64", "armijo", "lipschitz", "decode_hidden", "decode_out",
    "newton_init", "activate", "lbfgs_dir", "param_grad", "elem_psd", "elem_hess_dump", "lipschitz_grad", "train",
    "dynamics", "elem_fused"};

// One profiled launch.  Its work is b0 + b1 * n bytes and f0 + f1 * n flops,
// n = 1 for launches sized on the host, else the device counter `which` of
// super-step `slot` (copied to a device log while profiling).
struct ProfRec {
    int kind;
    double b0, b1, f0, f1;
    int slot, which;
    int e0, e1;
};

struct Work {
    double b0 = 0, b1 = 0, f0 = 0, f1 = 0;
    int slot = -1, which = 0;
};

struct LipWs {
    int pairs = 0;                 // pairs per pass
    void* Pre[kMaxL] = {};         // w x cols
    void* X0 = nullptr;            // r x cols
    void* X = nullptr;             // width x cols (recomputed activation)
    void* Out = nullptr;           // 9S x cols
    void* Seed = nullptr;          // 9S x cols
    void* G[2] = {};               // max(w, r) x cols
    void* D = nullptr;             // w x cols
    double* Cs = nullptr;          // items x r x r
    int* nvalid = nullptr;
};

}  // namespace

struct rs_ctx {
    int prec = 0;
    int f32 = 0;
    size_t tsz = 8;
    int r = 0, L = 0, w = 0, nv = 0, ne = 0, S = 0, nt = 0, nf = 0, n_out = 0, nc = 0;
    int M = 0, Mp = 0, Nfp = 0, max_batch = 0;
    int in_last = 0, lda0 = 0, lda_h = 0, lda_out = 0, wrows = 0, in_rows = 0;
    int grav_row = 0, force_row = 0;
    double mu = 0, lam = 0, k_c = 0;
    double grav[3] = {0, 0, 0};
    double density = 0;

    std::vector<double> X, mass, Dminv, vol;
    std::vector<int> tets, cub_elem, tvtx, fvtx;
    std::vector<uint8_t> pinned;
    std::vector<double> cub_w;

    std::vector<void*> allocs;
    // weights in the context precision (T) and in float64
    std::vector<void*> W, bh;
    std::vector<double*> W64, bh64;
    void* Wbig = nullptr; void* bbig = nullptr; void* WbigT = nullptr;
    // BF16 contexts: BF16 copies of the forward GEMM weights (everything else
    // as in a float32 context)
    int bf16 = 0;
    std::vector<void*> W16;
    void* Wbig16 = nullptr;
    void* Wfull16 = nullptr;
    double* Wbig64 = nullptr; double* bbig64 = nullptr;
    void* Wfull = nullptr; void* bfull = nullptr; void* Xfull = nullptr;
    double* Wfull64 = nullptr; double* bfull64 = nullptr; // float64 output layer (the inertia term's G and c)
    double* wV = nullptr; double* Xt = nullptr;
    double* ec = nullptr;         // S x kElemConst: per-element constants of the optional element treatments
    double* dump_He = nullptr;    // RS_DEBUG_ELEM_HESS destination (caller-owned), dump_max items
    int dump_max = 0;
    // workspace
    std::vector<void*> pre;       // L x (max_batch x wrows x nc) T
    void* act = nullptr;          // max_batch x wrows x nc T: [h_L | J_L] of the last hidden layer
    double* act64 = nullptr;      // kLsCand*max_batch x wrows: h_L for the line search
    void* out = nullptr;          // max_batch x Mp x nc T
    void* dseed = nullptr;        // max_batch x Mp T
    void* gbar = nullptr;         // max_batch x in_rows T
    double *Ew = nullptr, *gw = nullptr, *Hw = nullptr;
    double *g0 = nullptr, *dz = nullptr, *slope = nullptr;
    LbfgsState lb{};              // L-BFGS history, max_batch items
    double* Hpart = nullptr;      // npart x r x r: element-kernel partials when an item's rounds are split
    double* gpart = nullptr;      // npart x r
    size_t npart = 0;             // 2 n_cu (split element kernel), 8 n_cu + max_batch where the fused kernel applies
    int fused = 0;                // float32/BF16, r = 16, width <= 128: the fused output map + element kernel applies
    int fused_on = 1;             // ... and is used (rs_set_fused; default: BF16 contexts only)
    int *ls_j = nullptr, *eval_list = nullptr, *search_list = nullptr, *search_start = nullptr;
    int *search_ncand = nullptr, *cand_item = nullptr, *cand_j = nullptr, *counters = nullptr;
    int ksplit = 1;               // K slices of the adjoint GEMM
    int n_cu = 256;               // compute units of the device (persistent launch sizes)
    double* zc = nullptr;         // kLsCand*max_batch x r candidates
    std::vector<double*> pre64;   // L x (kLsCand*max_batch x wrows)
    double* out64 = nullptr;      // kLsCand*max_batch x Mp
    double* Ec = nullptr;
    double* zs = nullptr;         // max_batch x r
    double* ell = nullptr;        // max_batch
    double* lacc = nullptr;       // 3
    // parameter gradients (rs_energy_param_grad)
    double* delta = nullptr;      // max_batch x L x w: dE/da_l per item
    double* dWbig = nullptr;      // M x in_last, float64: dE/dW_big summed over items
    double* dbbig = nullptr;      // M
    double* ppart = nullptr;      // kParamSlices partial sums of the largest parameter product
    size_t ppart_cap = 0;
    int* ffold_ptr = nullptr;     // M + 1: CSR of the output-layer fold by W_big row (device decoder loads)
    int* ffold_src = nullptr;     // W_out row of each entry
    double* ffold_coef = nullptr; // its coefficient
    uint8_t* pinned_row = nullptr;// n_out: 1 on rows of pinned vertices (device)
    double* row_mass = nullptr;   // n_out: lumped mass of each row's vertex (device)
    // learned-part workspace, grown on demand by the training calls
    std::vector<void*> learn_bufs;
    LipWs lip;                    // Lipschitz-loss gradient workspace (allocated by its first call)
    void* scratch = nullptr;      // device address of this device's static scratch array
    FullSolver* full = nullptr;   // full-space solver (created by its first call)
    // ground contact and implicit-Euler inertia
    int ncont = 0, crow = 0;      // contact vertices; first contact row of W_big (the y row of each)
    double k_ground = 0.0, ground_y = 0.0;
    std::vector<int> cvtx;
    double* Xc = nullptr;         // ncont: rest y of the contact vertices
    double* Gdyn = nullptr;       // in_last x in_last: W_out^T M W_out (free rows), float64
    bool G_dirty = true;          // the decoder changed since Gdyn was formed
    double* dyn_c = nullptr;      // max_batch x in_last: W_out^T M (qbar - b_out) per item
    double* dyn_kappa = nullptr;  // max_batch: |qbar - b_out|_M^2 per item
    double* dyn_eta = nullptr;    // max_batch x in_last: the target's range coefficients (simulations)
    int dyn_use_eta = 0;
    int dyn_inertia = 0;          // the current call has an inertia term
    double dyn_inv_dt2 = 0.0;
    // simulation state (rs_simulate), max_batch items each
    double *sim_h0 = nullptr, *sim_h1 = nullptr, *sim_cv0 = nullptr, *sim_kv0 = nullptr;
    double *sim_relg = nullptr, *sim_E = nullptr;
    int *sim_it = nullptr, *sim_st = nullptr;
    int* fold_ptr = nullptr;      // n_out + 1: CSR of the output-layer fold by W_out row
    int* fold_row = nullptr;      // W_big row of each entry
    double* fold_coef = nullptr;  // its coefficient
    std::vector<size_t> offW, offb; // packed offsets of W_l, b_l (output layer last)
    size_t n_params = 0;
    // running counts, one slot per parity of the super-step: (tag << 32) | count
    unsigned long long* hcount = nullptr;     // pinned host
    unsigned long long* hcount_dev = nullptr; // device address of hcount
    unsigned int tag_next = 1;                // tag of the next super-step's count (never 0)
    hipEvent_t cnt_ev[2] = {nullptr, nullptr}; // running-count copies, one per parity of the super-step

    std::string err;
    // profiling
    bool prof = false;
    uint32_t prof_mask = 0;       // kinds recorded (0 = all)
    std::vector<hipEvent_t> evpool;
    size_t evnext = 0;
    std::vector<ProfRec> recs;
    double kms[K_COUNT] = {0}, kbytes[K_COUNT] = {0}, kflops[K_COUNT] = {0};
    int klaunch[K_COUNT] = {0};
    bool aggregated = true;
    int* plog = nullptr;          // device log of the Newton counters per super-step
    int plog_cap = 0, plog_next = 0;
    int cur_slot = -1;            // super-step whose counters size the current launches
};

static const char* kNullCtxMsg = "rs: null context";

static int fail(rs_ctx* c, int code, const std::string& msg)
{
    if (c) c->err = msg;
    return code;
}

static int hip_fail(rs_ctx* c, hipError_t e, const char* what)
{
    return fail(c, RS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <class T> static T* dalloc(rs_ctx* c, size_t n)
{
    void* p = nullptr;
    if (n == 0) n = 1;
    if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) return nullptr;
    c->allocs.push_back(p);
    return static_cast<T*>(p);
}

static void* dalloc_bytes(rs_ctx* c, size_t bytes)
{
    void* p = nullptr;
    if (bytes == 0) bytes = 1;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    c->allocs.push_back(p);
    return p;
}

// Launch bracket: when profiling this kind, the next kernel launch records a
// pair of timing events as part of its own dispatch.
template <class F>
static int run(rs_ctx* c, int kind, const Work& w, hipStream_t s, F&& f)
{
    int e0 = -1, e1 = -1;
    const bool rec = c->prof && (c->prof_mask == 0 || (c->prof_mask >> kind) & 1u);
    if (rec) {
        while (c->evpool.size() < c->evnext + 2) {
            hipEvent_t e;
            // timing-only events: no system-scope fence
            if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess)
                return fail(c, RS_ERR_HIP, "hipEventCreate");
            c->evpool.push_back(e);
        }
        e0 = (int)c->evnext;
        e1 = (int)c->evnext + 1;
        set_launch_events(c->evpool[e0], c->evpool[e1]);
    }
    hipError_t e = f();
    const bool launched = rec && !launch_events_pending();
    set_launch_events(nullptr, nullptr);
    if (e != hipSuccess) return hip_fail(c, e, kKindName[kind]);
    if (launched) {
        c->evnext += 2;
        c->recs.push_back(ProfRec{kind, w.b0, w.b1, w.f0, w.f1, w.slot, w.which, e0, e1});
        c->aggregated = false;
    }
    return RS_OK;
}

#define RS_TRY(x)                  \
    do {                           \
        int rc_ = (x);             \
        if (rc_ != RS_OK) return rc_; \
    } while (0)

#define RS_HIP(x, what)                                      \
    do {                                                     \
        hipError_t e_ = (x);                                 \
        if (e_ != hipSuccess) return hip_fail(c, e_, what);  \
    } while (0)

// ------------------------------------------------------------------ layouts
static void inv3(const double* M, double* Mi, double* det)
{
    double C[9];
    C[0] = M[4] * M[8] - M[5] * M[7];
    C[1] = M[5] * M[6] - M[3] * M[8];
    C[2] = M[3] * M[7] - M[4] * M[6];
    C[3] = M[2] * M[7] - M[1] * M[8];
    C[4] = M[0] * M[8] - M[2] * M[6];
    C[5] = M[1] * M[6] - M[0] * M[7];
    C[6] = M[1] * M[5] - M[2] * M[4];
    C[7] = M[2] * M[3] - M[0] * M[5];
    C[8] = M[0] * M[4] - M[1] * M[3];
    const double d = M[0] * C[0] + M[1] * C[1] + M[2] * C[2];
    *det = d;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Mi[3 * i + j] = C[3 * j + i] / d;
}

// Square root and inverse square root of a symmetric positive-definite 3x3
// matrix (row-major) by cyclic Jacobi rotations: N = Q diag(l) Q^T,
// N^(1/2) = Q diag(sqrt l) Q^T, N^(-1/2) = Q diag(1/sqrt l) Q^T.
static void sym3_sqrt(const double* N, double* Sq, double* Si)
{
    double A[9], Q[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    std::memcpy(A, N, sizeof(A));
    for (int sweep = 0; sweep < 60; ++sweep) {
        const double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
        const double tot = off + A[0] * A[0] + A[4] * A[4] + A[8] * A[8];
        if (off <= 1e-32 * tot) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                const double apq = A[3 * p + q];
                if (apq == 0.0) continue;
                const double th = (A[3 * q + q] - A[3 * p + p]) / (2.0 * apq);
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < 3; ++k) {
                    const double akp = A[3 * k + p], akq = A[3 * k + q];
                    A[3 * k + p] = cs * akp - sn * akq;
                    A[3 * k + q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < 3; ++k) {
                    const double apk = A[3 * p + k], aqk = A[3 * q + k];
                    A[3 * p + k] = cs * apk - sn * aqk;
                    A[3 * q + k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < 3; ++k) {
                    const double qkp = Q[3 * k + p], qkq = Q[3 * k + q];
                    Q[3 * k + p] = cs * qkp - sn * qkq;
                    Q[3 * k + q] = sn * qkp + cs * qkq;
                }
            }
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double a = 0.0, b = 0.0;
            for (int k = 0; k < 3; ++k) {
                const double l = std::sqrt(A[4 * k]);
                a += Q[3 * i + k] * l * Q[3 * j + k];
                b += Q[3 * i + k] / l * Q[3 * j + k];
            }
            Sq[3 * i + j] = a;
            Si[3 * i + j] = b;
        }
}

static int upload(rs_ctx* c, void* dst, const std::vector<double>& src, int as_f32)
{
    hipError_t e;
    if (as_f32) {
        std::vector<float> t(src.begin(), src.end());
        e = hipMemcpy(dst, t.data(), t.size() * sizeof(float), hipMemcpyHostToDevice);
    } else {
        e = hipMemcpy(dst, src.data(), src.size() * sizeof(double), hipMemcpyHostToDevice);
    }
    return e == hipSuccess ? RS_OK : hip_fail(c, e, "hipMemcpy");
}

// float64 -> bfloat16, round to nearest even.  Through float when that is
// exact; when float rounding lands on a bfloat16 midpoint the float64 value
// decides the direction, so the result is the correctly rounded one.
static uint16_t bf16_rne(double x)
{
    const float f = (float)x;
    uint32_t u;
    std::memcpy(&u, &f, sizeof(u));
    uint32_t hi = u >> 16;
    const uint32_t lo = u & 0xFFFFu;
    if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)(hi | ((u & 0x7FFFFFu) ? 0x40u : 0u)); // inf, nan
    bool up;
    if (lo > 0x8000u) up = true;
    else if (lo < 0x8000u) up = false;
    else {
        const double ax = std::fabs(x), af = std::fabs((double)f);
        up = ax > af ? true : ax < af ? false : (hi & 1u) != 0;
    }
    return (uint16_t)(up ? hi + 1 : hi);
}

static double bf16_value(uint16_t h)
{
    const uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, sizeof(f));
    return (double)f;
}

// BF16 operand planes of a float64 array: plane 0 holds hi = bf16(x), plane 1
// mid = bf16(x - hi), plane 2 lo = bf16(x - hi - mid), so that the three parts
// carry x to float32 accuracy on the BF16 matrix cores.
static int upload_bf16(rs_ctx* c, void* dst, const std::vector<double>& src)
{
    const size_t n = src.size();
    std::vector<uint16_t> t(3 * n);
    for (size_t i = 0; i < n; ++i) {
        double rem = src[i];
        for (int p = 0; p < 3; ++p) {
            t[p * n + i] = bf16_rne(rem);
            rem -= bf16_value(t[p * n + i]);
        }
    }
    hipError_t e = hipMemcpy(dst, t.data(), t.size() * sizeof(uint16_t), hipMemcpyHostToDevice);
    return e == hipSuccess ? RS_OK : hip_fail(c, e, "hipMemcpy");
}

// Upload the decoder: hidden layers padded for the GEMM tiles, and the folded
// output maps (reduced W_big, its transpose, and the full W_out for rs_decode).
// Shape-function gradients of cubature tet s: F = sum_a x_a Dv[a]^T, with
// Dv[1..3] the rows of Dm^-1 and Dv[0] = -(Dv[1] + Dv[2] + Dv[3]).
static void tet_shape_grads(const rs_ctx* c, int s, double Dv[4][3])
{
    const double* Di = &c->Dminv[9 * (size_t)s];
    for (int j = 0; j < 3; ++j) {
        double sum = 0.0;
        for (int a = 1; a < 4; ++a) {
            Dv[a][j] = Di[3 * (a - 1) + j];
            sum += Dv[a][j];
        }
        Dv[0][j] = -sum;
    }
}

static int build_fold(rs_ctx* c);

static int load_decoder(rs_ctx* c, const rs_decoder* d)
{
    const int r = c->r, w = c->w, L = c->L, in_last = c->in_last;
    for (int l = 0; l < L; ++l) {
        const int in = l == 0 ? r : w, lda = l == 0 ? c->lda0 : c->lda_h;
        std::vector<double> Wp((size_t)c->wrows * lda, 0.0), bp(c->wrows, 0.0);
        for (int i = 0; i < w; ++i) {
            for (int j = 0; j < in; ++j) Wp[(size_t)i * lda + j] = d->W[l][(size_t)i * in + j];
            bp[i] = d->b[l][i];
        }
        RS_TRY(upload(c, c->W64[l], Wp, 0));
        RS_TRY(upload(c, c->bh64[l], bp, 0));
        if (c->f32) {
            RS_TRY(upload(c, c->W[l], Wp, 1));
            RS_TRY(upload(c, c->bh[l], bp, 1));
        }
        if (c->bf16) RS_TRY(upload_bf16(c, c->W16[l], Wp));
    }
    // masked output layer
    const double* Wo = d->W[L];
    const double* bo = d->b[L];
    auto wout = [&](int row, int j) { return c->pinned[row / 3] ? 0.0 : Wo[(size_t)row * in_last + j]; };
    auto bout = [&](int row) { return c->pinned[row / 3] ? 0.0 : bo[row]; };

    const int lda = c->lda_out;
    std::vector<double> Wb((size_t)c->Mp * lda, 0.0), bb(c->Mp, 0.0);
    for (int s = 0; s < c->S; ++s) {
        const int e = c->cub_elem[s];
        double Dv[4][3];
        tet_shape_grads(c, s, Dv);
        for (int j = 0; j < 3; ++j)
            for (int i = 0; i < 3; ++i) {
                const size_t row = 9 * (size_t)s + 3 * j + i;
                for (int a = 0; a < 4; ++a) {
                    const int vrow = 3 * c->tets[4 * (size_t)e + a] + i;
                    const double coef = Dv[a][j];
                    for (int k = 0; k < in_last; ++k) Wb[row * lda + k] += coef * wout(vrow, k);
                    bb[row] += coef * bout(vrow);
                }
            }
    }
    const int prow = 9 * c->S;
    for (int t = 0; t < c->nt; ++t)
        for (int i = 0; i < 3; ++i) {
            const int vrow = 3 * c->tvtx[t] + i;
            for (int k = 0; k < in_last; ++k) Wb[(size_t)(prow + 3 * t + i) * lda + k] = wout(vrow, k);
            bb[prow + 3 * t + i] = bout(vrow);
        }
    for (int v = 0; v < c->nv; ++v)
        for (int i = 0; i < 3; ++i) {
            const double mg = c->mass[v] * c->grav[i];
            if (mg == 0.0) continue;
            const int vrow = 3 * v + i;
            for (int k = 0; k < in_last; ++k) Wb[(size_t)c->grav_row * lda + k] += mg * wout(vrow, k);
            bb[c->grav_row] += mg * bout(vrow);
        }
    for (int t = 0; t < c->nf; ++t)
        for (int i = 0; i < 3; ++i) {
            const int vrow = 3 * c->fvtx[t] + i;
            for (int k = 0; k < in_last; ++k) Wb[(size_t)(c->force_row + i) * lda + k] += wout(vrow, k);
            bb[c->force_row + i] += bout(vrow);
        }
    for (int t = 0; t < c->ncont; ++t) {
        const int vrow = 3 * c->cvtx[t] + 1;
        for (int k = 0; k < in_last; ++k) Wb[(size_t)(c->crow + t) * lda + k] = wout(vrow, k);
        bb[c->crow + t] = bout(vrow);
    }
    c->G_dirty = true;
    RS_TRY(upload(c, c->Wbig64, Wb, 0));
    RS_TRY(upload(c, c->bbig64, bb, 0));
    if (c->f32) {
        RS_TRY(upload(c, c->Wbig, Wb, 1));
        RS_TRY(upload(c, c->bbig, bb, 1));
    }
    if (c->bf16) RS_TRY(upload_bf16(c, c->Wbig16, Wb));
    // transpose for the adjoint product dE/dh_L = W_big^T seeds
    std::vector<double> WT((size_t)c->in_rows * c->Mp, 0.0);
    for (int m = 0; m < c->Mp; ++m)
        for (int k = 0; k < in_last; ++k) WT[(size_t)k * c->Mp + m] = Wb[(size_t)m * lda + k];
    RS_TRY(upload(c, c->WbigT, WT, c->f32));
    // full output layer for rs_decode
    std::vector<double> Wf((size_t)c->Nfp * lda, 0.0), bf(c->n_out, 0.0), Xf(c->n_out);
    for (int row = 0; row < c->n_out; ++row) {
        for (int k = 0; k < in_last; ++k) Wf[(size_t)row * lda + k] = wout(row, k);
        bf[row] = bout(row);
        Xf[row] = c->X[row];
    }
    RS_TRY(upload(c, c->Wfull, Wf, c->f32));
    if (c->f32) RS_TRY(upload(c, c->Wfull64, Wf, 0));
    if (c->bf16) RS_TRY(upload_bf16(c, c->Wfull16, Wf));
    RS_TRY(upload(c, c->bfull, bf, c->f32));
    if (c->f32) RS_TRY(upload(c, c->bfull64, bf, 0));
    RS_TRY(upload(c, c->Xfull, Xf, c->f32));
    return RS_OK;
}

static int check_decoder(rs_ctx* c, const rs_decoder* d, int nv)
{
    if (!d) return fail(c, RS_ERR_ARG, "decoder is NULL");
    if (d->r < 1 || d->r > kMaxR) return fail(c, RS_ERR_UNSUPPORTED, "decoder r must be in [1, 32]");
    if (d->n_hidden < 0 || (d->n_hidden > 0 && d->width < 1)) return fail(c, RS_ERR_ARG, "bad decoder depth/width");
    if (d->n_hidden > kMaxL) return fail(c, RS_ERR_UNSUPPORTED, "at most 8 hidden layers");
    if (d->n_hidden > 0 && d->width > kMaxWidth) return fail(c, RS_ERR_UNSUPPORTED, "decoder width must be at most 256");
    if (d->n_out != 3 * nv) return fail(c, RS_ERR_ARG, "decoder n_out must be 3 * nv");
    if (!d->W || !d->b) return fail(c, RS_ERR_ARG, "decoder weights are NULL");
    for (int l = 0; l <= d->n_hidden; ++l)
        if (!d->W[l] || !d->b[l]) return fail(c, RS_ERR_ARG, "decoder layer pointer is NULL");
    return RS_OK;
}

// ------------------------------------------------------------------ ABI
extern "C" int rs_default_opts(rs_solve_opts* o)
{
    if (!o) return RS_ERR_ARG;
    o->max_iter = 50;
    o->ls_max = 128;
    o->c1 = 1e-4;
    o->shrink = 0.5;
    o->rel_tol = 1e-6;
    o->abs_tol = 0.0;
    o->hess = 1;
    o->proj = RS_PROJ_ABS;
    o->eig_floor = 1e-8;
    o->window = 0;
    return RS_OK;
}

extern "C" int rs_default_lbfgs_opts(rs_lbfgs_opts* o)
{
    if (!o) return RS_ERR_ARG;
    o->max_iter = 1024;
    o->ls_max = 128;
    o->history = 10;
    o->c1 = 1e-4;
    o->shrink = 0.5;
    o->rel_tol = 1e-6;
    o->abs_tol = 0.0;
    o->window = 0;
    return RS_OK;
}

extern "C" const char* rs_last_error(const rs_ctx* c) { return c ? c->err.c_str() : kNullCtxMsg; }

static void destroy(rs_ctx* c)
{
    for (void* p : c->allocs) (void)hipFree(p);
    for (void* p : c->learn_bufs) (void)hipFree(p);
    full_solver_destroy(c->full);
    if (c->plog) (void)hipFree(c->plog);
    for (hipEvent_t e : c->evpool) (void)hipEventDestroy(e);
    if (c->hcount) (void)hipHostFree(c->hcount);
    for (hipEvent_t e : c->cnt_ev)
        if (e) (void)hipEventDestroy(e);
    delete c;
}

extern "C" int rs_destroy(rs_ctx* c)
{
    if (c) destroy(c);
    return RS_OK;
}

extern "C" int rs_create(const rs_mesh* mesh, const rs_material* mat, const rs_decoder* dec,
                         const rs_cubature* cub, const rs_constraints* con, int32_t prec,
                         int32_t max_batch, rs_ctx** out)
{
    if (!out) return RS_ERR_ARG;
    *out = nullptr;
    rs_ctx* c = new (std::nothrow) rs_ctx();
    if (!c) return RS_ERR_OOM;
    auto bail = [&](int code) {
        // errors at creation cannot be queried from a context: print once
        std::fprintf(stderr, "rs_create: %s\n", c->err.c_str());
        destroy(c);
        return code;
    };
    if (!mesh || !mat || !cub || !mesh->X || !mesh->tets || !mesh->pinned)
        return bail(fail(c, RS_ERR_ARG, "NULL mesh, material or cubature"));
    if (mesh->nv < 4 || mesh->ne < 1) return bail(fail(c, RS_ERR_ARG, "mesh too small"));
    if (prec != RS_PREC_F64 && prec != RS_PREC_F32 && prec != RS_PREC_BF16)
        return bail(fail(c, RS_ERR_UNSUPPORTED, "unknown precision"));
    if (max_batch < 1) return bail(fail(c, RS_ERR_ARG, "max_batch must be >= 1"));
    {
        const int rc = check_decoder(c, dec, mesh->nv);
        if (rc != RS_OK) return bail(rc);
    }
    if (cub->n < 1 || !cub->elem || !cub->weight) return bail(fail(c, RS_ERR_ARG, "empty cubature"));
    const int nt = con ? con->n_target : 0, nf = con ? con->n_force : 0;
    if (nt < 0 || nf < 0 || (nt && !con->target_vtx) || (nf && !con->force_vtx))
        return bail(fail(c, RS_ERR_ARG, "bad constraints"));

    {
        // the device address of this device's static scratch array (allocation-free entry points)
        const hipError_t e = static_scratch_address(&c->scratch);
        if (e != hipSuccess) return bail(hip_fail(c, e, "hipGetSymbolAddress(scratch)"));
    }
    c->prec = prec;
    c->f32 = prec != RS_PREC_F64;
    c->bf16 = prec == RS_PREC_BF16;
    c->tsz = c->f32 ? 4 : 8;
    c->nv = mesh->nv;
    c->ne = mesh->ne;
    c->r = dec->r;
    c->L = dec->n_hidden;
    c->w = c->L > 0 ? dec->width : 0;
    c->n_out = dec->n_out;
    c->nc = 1 + c->r;
    c->S = cub->n;
    c->nt = nt;
    c->nf = nf;
    c->k_c = con ? con->k_c : 0.0;
    c->max_batch = max_batch;
    c->density = mat->density;
    for (int i = 0; i < 3; ++i) c->grav[i] = mat->gravity[i];
    // stable Neo-Hookean: lambda = lambda_Lame + mu (linearises to (E, nu))
    c->mu = mat->young / (2.0 * (1.0 + mat->poisson));
    c->lam = mat->young * mat->poisson / ((1.0 + mat->poisson) * (1.0 - 2.0 * mat->poisson)) + c->mu;

    c->X.assign(mesh->X, mesh->X + 3 * (size_t)c->nv);
    c->tets.assign(mesh->tets, mesh->tets + 4 * (size_t)c->ne);
    c->pinned.assign(mesh->pinned, mesh->pinned + c->nv);
    for (int v : c->tets)
        if (v < 0 || v >= c->nv) return bail(fail(c, RS_ERR_ARG, "tet vertex index out of range"));
    c->cub_elem.assign(cub->elem, cub->elem + c->S);
    c->cub_w.assign(cub->weight, cub->weight + c->S);
    for (int s = 0; s < c->S; ++s) {
        if (c->cub_elem[s] < 0 || c->cub_elem[s] >= c->ne) return bail(fail(c, RS_ERR_ARG, "cubature element out of range"));
        if (!(c->cub_w[s] >= 0.0)) return bail(fail(c, RS_ERR_ARG, "negative cubature weight"));
    }
    if (nt) c->tvtx.assign(con->target_vtx, con->target_vtx + nt);
    if (nf) c->fvtx.assign(con->force_vtx, con->force_vtx + nf);
    for (int v : c->tvtx)
        if (v < 0 || v >= c->nv) return bail(fail(c, RS_ERR_ARG, "target vertex out of range"));
    for (int v : c->fvtx)
        if (v < 0 || v >= c->nv) return bail(fail(c, RS_ERR_ARG, "force vertex out of range"));
    {
        const int ncn = con ? con->n_contact : 0;
        if (ncn < 0 || (ncn && !con->contact_vtx)) return bail(fail(c, RS_ERR_ARG, "bad contact set"));
        if (ncn && !(con->k_ground >= 0.0)) return bail(fail(c, RS_ERR_ARG, "negative ground stiffness"));
        c->ncont = ncn;
        if (ncn) {
            c->cvtx.assign(con->contact_vtx, con->contact_vtx + ncn);
            c->k_ground = con->k_ground;
            c->ground_y = con->ground_y;
        }
        for (int v : c->cvtx)
            if (v < 0 || v >= c->nv) return bail(fail(c, RS_ERR_ARG, "contact vertex out of range"));
    }

    // rest shape: lumped masses over every tet, Dm^-1 and volume per cubature tet
    c->mass.assign(c->nv, 0.0);
    for (int e = 0; e < c->ne; ++e) {
        double Dm[9], Di[9], det;
        const int* t = &c->tets[4 * (size_t)e];
        for (int i = 0; i < 3; ++i)
            for (int k = 0; k < 3; ++k) Dm[3 * i + k] = c->X[3 * t[k + 1] + i] - c->X[3 * t[0] + i];
        inv3(Dm, Di, &det);
        const double V = det / 6.0;
        for (int a = 0; a < 4; ++a) c->mass[t[a]] += c->density * V / 4.0;
    }
    c->Dminv.resize(9 * (size_t)c->S);
    c->vol.resize(c->S);
    std::vector<double> wVh(c->S);
    for (int s = 0; s < c->S; ++s) {
        double Dm[9], det;
        const int* t = &c->tets[4 * (size_t)c->cub_elem[s]];
        for (int i = 0; i < 3; ++i)
            for (int k = 0; k < 3; ++k) Dm[3 * i + k] = c->X[3 * t[k + 1] + i] - c->X[3 * t[0] + i];
        inv3(Dm, &c->Dminv[9 * (size_t)s], &det);
        if (!(det > 0.0)) return bail(fail(c, RS_ERR_ARG, "cubature tet with non-positive volume"));
        c->vol[s] = det / 6.0;
        wVh[s] = c->cub_w[s] * c->vol[s];
    }

    // sizes
    c->in_last = c->L > 0 ? c->w : c->r;
    c->lda0 = round_up(c->r, kTileK);
    c->lda_h = round_up(std::max(c->w, 1), kTileK);
    c->lda_out = round_up(c->in_last, kTileK);
    c->wrows = round_up(std::max(c->w, 1), kTileM);
    c->in_rows = round_up(c->in_last, kTileM);
    c->M = 9 * c->S + 3 * c->nt + 4 + c->ncont;
    c->Mp = round_up(c->M, kTileM);
    // float32 and BF16 output maps store their packed rows through 32-bit buffer
    // offsets that span at most 64 items of rows_pad x (r + 1) values
    if (c->f32 && (size_t)c->Mp * (c->r + 1) * kTileN >= ((size_t)1 << 28))
        return bail(fail(c, RS_ERR_UNSUPPORTED, "reduced row set too large: rows_pad x (r + 1) must be below 4194304"));
    c->grav_row = 9 * c->S + 3 * c->nt;
    c->force_row = c->grav_row + 1;
    c->crow = c->force_row + 3;
    c->Nfp = round_up(c->n_out, kTileM);

    // device allocations
    const size_t B = (size_t)max_batch, nc = c->nc, ts = c->tsz;
    const size_t BL = B * kLsCand;
    bool ok = true;
    auto need = [&](void* p) { ok = ok && p != nullptr; return p; };
    c->W.resize(c->L);
    c->bh.resize(c->L);
    c->W64.resize(c->L);
    c->bh64.resize(c->L);
    c->pre.resize(c->L);
    c->pre64.resize(c->L);
    for (int l = 0; l < c->L; ++l) {
        const int lda = l == 0 ? c->lda0 : c->lda_h;
        c->W64[l] = (double*)need(dalloc<double>(c, (size_t)c->wrows * lda));
        c->bh64[l] = (double*)need(dalloc<double>(c, c->wrows));
        c->W[l] = c->f32 ? need(dalloc_bytes(c, (size_t)c->wrows * lda * ts)) : c->W64[l];
        c->bh[l] = c->f32 ? need(dalloc_bytes(c, (size_t)c->wrows * ts)) : c->bh64[l];
        c->pre[l] = need(dalloc_bytes(c, B * c->wrows * nc * ts));
        c->pre64[l] = (double*)need(dalloc<double>(c, BL * c->wrows));
    }
    c->Wbig64 = (double*)need(dalloc<double>(c, (size_t)c->Mp * c->lda_out));
    c->bbig64 = (double*)need(dalloc<double>(c, c->Mp));
    c->Wbig = c->f32 ? need(dalloc_bytes(c, (size_t)c->Mp * c->lda_out * ts)) : c->Wbig64;
    c->bbig = c->f32 ? need(dalloc_bytes(c, (size_t)c->Mp * ts)) : c->bbig64;
    c->WbigT = need(dalloc_bytes(c, (size_t)c->in_rows * c->Mp * ts));
    c->Wfull = need(dalloc_bytes(c, (size_t)c->Nfp * c->lda_out * ts));
    c->Wfull64 = c->f32 ? (double*)need(dalloc<double>(c, (size_t)c->Nfp * c->lda_out)) : (double*)c->Wfull;
    if (c->bf16) {
        // BF16 operands need the fused hidden-layer kernel and a K that fills 32-deep chunks
        if (c->L == 0 || !mlp_fits(1, (int)nc, c->r, c->wrows) || !mlp_fits(1, 1, c->r, c->wrows))
            return bail(fail(c, RS_ERR_UNSUPPORTED, "BF16 contexts need hidden layers that fit the fused kernel"));
        c->W16.resize(c->L);
        for (int l = 0; l < c->L; ++l) {
            const int lda = l == 0 ? c->lda0 : c->lda_h;
            c->W16[l] = need(dalloc_bytes(c, 3 * (size_t)c->wrows * lda * 2));
        }
        // three BF16 planes (hi, mid, lo) per weight array
        c->Wbig16 = need(dalloc_bytes(c, 3 * (size_t)c->Mp * c->lda_out * 2));
        c->Wfull16 = need(dalloc_bytes(c, 3 * (size_t)c->Nfp * c->lda_out * 2));
    }
    c->bfull = need(dalloc_bytes(c, (size_t)c->n_out * ts));
    c->bfull64 = c->f32 ? (double*)need(dalloc<double>(c, (size_t)c->n_out)) : (double*)c->bfull;
    c->Xfull = need(dalloc_bytes(c, (size_t)c->n_out * ts));
    c->wV = (double*)need(dalloc<double>(c, c->S));
    c->Xt = (double*)need(dalloc<double>(c, 3 * (size_t)std::max(c->nt, 1)));
    c->Xc = (double*)need(dalloc<double>(c, (size_t)std::max(c->ncont, 1)));
    c->Gdyn = (double*)need(dalloc<double>(c, (size_t)c->in_last * c->in_last));
    c->dyn_c = (double*)need(dalloc<double>(c, B * c->in_last));
    c->dyn_kappa = (double*)need(dalloc<double>(c, B));
    c->dyn_eta = (double*)need(dalloc<double>(c, B * c->in_last));
    c->sim_h0 = (double*)need(dalloc<double>(c, B * c->in_last));
    c->sim_h1 = (double*)need(dalloc<double>(c, B * c->in_last));
    c->sim_cv0 = (double*)need(dalloc<double>(c, B * c->in_last));
    c->sim_kv0 = (double*)need(dalloc<double>(c, B));
    c->sim_relg = (double*)need(dalloc<double>(c, B));
    c->sim_E = (double*)need(dalloc<double>(c, B));
    c->sim_it = (int*)need(dalloc<int>(c, B));
    c->sim_st = (int*)need(dalloc<int>(c, B));
    c->ec = (double*)need(dalloc<double>(c, (size_t)c->S * kElemConst));
    c->out = need(dalloc_bytes(c, B * c->Mp * nc * ts));
    c->act = need(dalloc_bytes(c, B * c->wrows * nc * ts));
    c->act64 = (double*)need(dalloc<double>(c, BL * c->wrows));
    c->dseed = need(dalloc_bytes(c, B * c->Mp * ts));
    c->ksplit = std::max(1, std::min(kMaxSplit, c->Mp / 160));
    {
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
            c->n_cu = ncu;
    }
    c->gbar = need(dalloc_bytes(c, (size_t)c->ksplit * B * c->in_rows * ts));
    // the fused kernel's parts times its items stay below 8 n_cu + the items
    c->fused = c->f32 && c->L > 0 && c->nc == 17 && elem_fused_fits(c->r, c->lda_out);
    // float32: the two-kernel path is faster (the fused kernel's FP32 products take longer than the
    // J_R round trip they save); BF16: the fused kernel is
    c->fused_on = c->bf16;
    c->npart = c->fused ? (size_t)8 * c->n_cu + c->max_batch : (size_t)2 * c->n_cu;
    c->Hpart = (double*)need(dalloc<double>(c, c->npart * c->r * c->r));
    c->gpart = (double*)need(dalloc<double>(c, c->npart * c->r));
    c->Ew = (double*)need(dalloc<double>(c, B));
    c->gw = (double*)need(dalloc<double>(c, B * c->r));
    c->Hw = (double*)need(dalloc<double>(c, B * c->r * c->r));
    c->g0 = (double*)need(dalloc<double>(c, B));
    c->dz = (double*)need(dalloc<double>(c, B * c->r));
    c->slope = (double*)need(dalloc<double>(c, B));
    c->lb.S = (double*)need(dalloc<double>(c, B * RS_MAX_HISTORY * c->r));
    c->lb.Y = (double*)need(dalloc<double>(c, B * RS_MAX_HISTORY * c->r));
    c->lb.sy = (double*)need(dalloc<double>(c, B * RS_MAX_HISTORY));
    c->lb.npair = (int*)need(dalloc<int>(c, B));
    c->lb.head = (int*)need(dalloc<int>(c, B));
    c->lb.zprev = (double*)need(dalloc<double>(c, B * c->r));
    c->lb.gprev = (double*)need(dalloc<double>(c, B * c->r));
    c->ls_j = (int*)need(dalloc<int>(c, B));
    c->eval_list = (int*)need(dalloc<int>(c, B));
    c->search_list = (int*)need(dalloc<int>(c, B));
    c->search_start = (int*)need(dalloc<int>(c, B));
    c->search_ncand = (int*)need(dalloc<int>(c, B));
    c->cand_item = (int*)need(dalloc<int>(c, BL));
    c->cand_j = (int*)need(dalloc<int>(c, BL));
    c->counters = (int*)need(dalloc<int>(c, 8));
    c->zc = (double*)need(dalloc<double>(c, BL * c->r));
    c->out64 = (double*)need(dalloc<double>(c, BL * c->Mp));
    c->Ec = (double*)need(dalloc<double>(c, BL));
    c->zs = (double*)need(dalloc<double>(c, B * c->r));
    c->ell = (double*)need(dalloc<double>(c, B));
    c->lacc = (double*)need(dalloc<double>(c, 4));
    c->delta = (double*)need(dalloc<double>(c, B * std::max(c->L, 1) * std::max(c->w, 1)));
    c->dWbig = (double*)need(dalloc<double>(c, (size_t)c->M * c->in_last));
    c->dbbig = (double*)need(dalloc<double>(c, c->M));
    {
        const size_t mn = std::max((size_t)c->M * c->in_last, (size_t)std::max(c->w, 1) * std::max(c->r, c->w));
        c->ppart_cap = (size_t)kParamSlices * (mn + std::max(c->M, c->w));
        c->ppart = (double*)need(dalloc<double>(c, c->ppart_cap));
    }
    if (!ok) return bail(fail(c, RS_ERR_OOM, "device allocation failed"));
    // coherent: the kernel's system-scope store lands in host memory without a cache flush
    if (hipHostMalloc((void**)&c->hcount, 2 * sizeof(unsigned long long), hipHostMallocMapped | hipHostMallocCoherent) !=
        hipSuccess)
        return bail(fail(c, RS_ERR_OOM, "pinned host allocation failed"));
    c->hcount[0] = c->hcount[1] = 0;
    if (hipHostGetDevicePointer((void**)&c->hcount_dev, c->hcount, 0) != hipSuccess)
        return bail(fail(c, RS_ERR_HIP, "hipHostGetDevicePointer"));
    for (int k = 0; k < 2; ++k)
        if (hipEventCreateWithFlags(&c->cnt_ev[k], hipEventDisableTiming | hipEventDisableSystemFence) != hipSuccess)
            return bail(fail(c, RS_ERR_HIP, "hipEventCreate"));

    if (upload(c, c->wV, wVh, 0) != RS_OK) return bail(RS_ERR_HIP);
    {
        std::vector<double> ec((size_t)c->S * kElemConst, 0.0);
        for (int s = 0; s < c->S; ++s) {
            double Dv[4][3];
            tet_shape_grads(c, s, Dv);
            double N[9] = {0};
            for (int a = 0; a < 4; ++a)
                for (int j = 0; j < 3; ++j)
                    for (int k = 0; k < 3; ++k) N[3 * j + k] += Dv[a][j] * Dv[a][k];
            double* e = &ec[(size_t)s * kElemConst];
            sym3_sqrt(N, e, e + 9);
            for (int a = 0; a < 4; ++a)
                for (int j = 0; j < 3; ++j) e[18 + 3 * a + j] = Dv[a][j];
            e[30] = c->vol[s];
            e[31] = c->cub_w[s];
        }
        if (upload(c, c->ec, ec, 0) != RS_OK) return bail(RS_ERR_HIP);
    }
    if (c->nt) {
        std::vector<double> xt(3 * (size_t)c->nt);
        for (int t = 0; t < c->nt; ++t)
            for (int i = 0; i < 3; ++i) xt[3 * t + i] = c->X[3 * c->tvtx[t] + i];
        if (upload(c, c->Xt, xt, 0) != RS_OK) return bail(RS_ERR_HIP);
    }
    if (c->ncont) {
        std::vector<double> xc(c->ncont);
        for (int t = 0; t < c->ncont; ++t) xc[t] = c->X[3 * c->cvtx[t] + 1];
        if (upload(c, c->Xc, xc, 0) != RS_OK) return bail(RS_ERR_HIP);
    }
    if (load_decoder(c, dec) != RS_OK) return bail(RS_ERR_HIP);
    {
        const int rc = build_fold(c);
        if (rc != RS_OK) return bail(rc);
    }
    *out = c;
    return RS_OK;
}

// The output-layer fold W_big = C W_out (rows of the cubature deformation
// gradients, targets, gravity and forces; pinned rows of W_out excluded) as a
// CSR of C^T by W_out row, so that dE/dW_out = C^T dE/dW_big.
static int build_fold(rs_ctx* c)
{
    std::vector<std::vector<std::pair<int, double>>> by(c->n_out);
    auto add = [&](int vrow, int brow, double coef) {
        if (!c->pinned[vrow / 3] && coef != 0.0) by[vrow].push_back({brow, coef});
    };
    for (int s = 0; s < c->S; ++s) {
        const int e = c->cub_elem[s];
        double Dv[4][3];
        tet_shape_grads(c, s, Dv);
        for (int j = 0; j < 3; ++j)
            for (int i = 0; i < 3; ++i)
                for (int a = 0; a < 4; ++a) add(3 * c->tets[4 * (size_t)e + a] + i, 9 * s + 3 * j + i, Dv[a][j]);
    }
    for (int t = 0; t < c->nt; ++t)
        for (int i = 0; i < 3; ++i) add(3 * c->tvtx[t] + i, 9 * c->S + 3 * t + i, 1.0);
    for (int v = 0; v < c->nv; ++v)
        for (int i = 0; i < 3; ++i) add(3 * v + i, c->grav_row, c->mass[v] * c->grav[i]);
    for (int t = 0; t < c->nf; ++t)
        for (int i = 0; i < 3; ++i) add(3 * c->fvtx[t] + i, c->force_row + i, 1.0);
    for (int t = 0; t < c->ncont; ++t) add(3 * c->cvtx[t] + 1, c->crow + t, 1.0);
    {
        // the same fold by W_big row, entries in the order the host load sums them
        std::vector<std::vector<std::pair<int, double>>> fw(c->M);
        auto addf = [&](int vrow, int brow, double cf) {
            if (!c->pinned[vrow / 3] && cf != 0.0) fw[brow].push_back({vrow, cf});
        };
        for (int s = 0; s < c->S; ++s) {
            const int e = c->cub_elem[s];
            double Dv[4][3];
            tet_shape_grads(c, s, Dv);
            for (int j = 0; j < 3; ++j)
                for (int i = 0; i < 3; ++i)
                    for (int a = 0; a < 4; ++a) addf(3 * c->tets[4 * (size_t)e + a] + i, 9 * s + 3 * j + i, Dv[a][j]);
        }
        for (int t = 0; t < c->nt; ++t)
            for (int i = 0; i < 3; ++i) addf(3 * c->tvtx[t] + i, 9 * c->S + 3 * t + i, 1.0);
        for (int v = 0; v < c->nv; ++v)
            for (int i = 0; i < 3; ++i) addf(3 * v + i, c->grav_row, c->mass[v] * c->grav[i]);
        for (int t = 0; t < c->nf; ++t)
            for (int i = 0; i < 3; ++i) addf(3 * c->fvtx[t] + i, c->force_row + i, 1.0);
        for (int t = 0; t < c->ncont; ++t) addf(3 * c->cvtx[t] + 1, c->crow + t, 1.0);
        std::vector<int> fp(c->M + 1, 0), fs;
        std::vector<double> fc;
        for (int m = 0; m < c->M; ++m) {
            for (const auto& pc : fw[m]) {
                fs.push_back(pc.first);
                fc.push_back(pc.second);
            }
            fp[m + 1] = (int)fs.size();
        }
        if (fs.empty()) {
            fs.push_back(0);
            fc.push_back(0.0);
        }
        std::vector<uint8_t> pr(c->n_out);
        std::vector<double> rm(c->n_out);
        for (int row = 0; row < c->n_out; ++row) {
            pr[row] = c->pinned[row / 3] ? 1 : 0;
            rm[row] = c->mass[row / 3];
        }
        c->ffold_ptr = (int*)dalloc<int>(c, fp.size());
        c->ffold_src = (int*)dalloc<int>(c, fs.size());
        c->ffold_coef = (double*)dalloc<double>(c, fc.size());
        c->pinned_row = (uint8_t*)dalloc<uint8_t>(c, pr.size());
        c->row_mass = (double*)dalloc<double>(c, rm.size());
        if (!c->ffold_ptr || !c->ffold_src || !c->ffold_coef || !c->pinned_row || !c->row_mass)
            return fail(c, RS_ERR_OOM, "device allocation failed");
        if (hipMemcpy(c->ffold_ptr, fp.data(), fp.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(c->ffold_src, fs.data(), fs.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(c->ffold_coef, fc.data(), fc.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(c->pinned_row, pr.data(), pr.size(), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(c->row_mass, rm.data(), rm.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
            return fail(c, RS_ERR_HIP, "hipMemcpy");
    }
    std::vector<int> ptr(c->n_out + 1, 0), row;
    std::vector<double> coef;
    for (int n = 0; n < c->n_out; ++n) {
        for (const auto& pc : by[n]) {
            row.push_back(pc.first);
            coef.push_back(pc.second);
        }
        ptr[n + 1] = (int)row.size();
    }
    if (row.empty()) {
        row.push_back(0);
        coef.push_back(0.0);
    }
    c->fold_ptr = (int*)dalloc<int>(c, ptr.size());
    c->fold_row = (int*)dalloc<int>(c, row.size());
    c->fold_coef = (double*)dalloc<double>(c, coef.size());
    if (!c->fold_ptr || !c->fold_row || !c->fold_coef) return fail(c, RS_ERR_OOM, "device allocation failed");
    if (hipMemcpy(c->fold_ptr, ptr.data(), ptr.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->fold_row, row.data(), row.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->fold_coef, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        return fail(c, RS_ERR_HIP, "hipMemcpy");
    size_t off = 0;
    c->offW.assign(c->L + 1, 0);
    c->offb.assign(c->L + 1, 0);
    for (int l = 0; l <= c->L; ++l) {
        const int in = l == 0 ? c->r : c->w, out = l == c->L ? c->n_out : c->w;
        c->offW[l] = off;
        off += (size_t)out * in;
        c->offb[l] = off;
        off += out;
    }
    c->n_params = off;
    return RS_OK;
}

extern "C" int rs_set_decoder(rs_ctx* c, const rs_decoder* d)
{
    if (!c) return RS_ERR_STATE;
    RS_TRY(check_decoder(c, d, c->nv));
    if (d->r != c->r || d->n_hidden != c->L || (c->L && d->width != c->w))
        return fail(c, RS_ERR_ARG, "decoder shape differs from the context's");
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(c, e, "hipDeviceSynchronize");
    return load_decoder(c, d);
}

extern "C" int rs_get_info(const rs_ctx* c, rs_info* info)
{
    if (!c || !info) return RS_ERR_ARG;
    info->prec = c->prec;
    info->r = c->r;
    info->n_hidden = c->L;
    info->width = c->w;
    info->nv = c->nv;
    info->ne = c->ne;
    info->n_cub = c->S;
    info->n_target = c->nt;
    info->n_force = c->nf;
    info->rows = c->M;
    info->rows_pad = c->Mp;
    info->max_batch = c->max_batch;
    return RS_OK;
}

// ------------------------------------------------------------------ passes
static Work gemm_work(size_t ts, int rows, int K, int items, int nc, const int* count, int slot, int which)
{
    Work w;
    const double per_item_b = (double)ts * ((double)K * nc + (double)rows * nc);
    const double per_item_f = 2.0 * rows * K * (double)nc;
    w.b0 = (double)ts * rows * K;
    if (count) {
        w.b1 = per_item_b;
        w.f1 = per_item_f;
        w.slot = slot;
        w.which = which;
    } else {
        w.b0 += per_item_b * items;
        w.f0 = per_item_f * items;
    }
    return w;
}

static Work item_work(double per_b, double per_f, int items, const int* count, int slot, int which)
{
    Work w;
    if (count) {
        w.b1 = per_b;
        w.f1 = per_f;
        w.slot = slot;
        w.which = which;
    } else {
        w.b0 = per_b * items;
        w.f0 = per_f * items;
    }
    return w;
}

// [h_L | J_L] of the last hidden layer, computed once for the output map
static int activate(rs_ctx* c, int f32, const void* pre, void* act, int nc, int cap, const int* count, int which,
                    hipStream_t s)
{
    const size_t ts = f32 ? 4 : 8;
    const double pb = 2.0 * ts * (double)c->w * nc;
    return run(c, K_ACTIVATE, item_work(pb, 3.0 * c->w * nc, cap, count, c->cur_slot, which), s,
               [&] { return launch_activate(f32, pre, act, c->w, c->wrows, nc, cap, count, s); });
}

// Hidden layers for `cap` items: pre-activations into pre[] (T path) and the
// last layer's activation into act.  One fused launch when its tiles fit,
// else one GEMM per layer and an activation pass.
static int hidden_layers(rs_ctx* c, int f32, int nc, int cap, const int* count, int which, const double* z,
                         const int* zmap, void* const* pre, void* act, const void* const* W, const void* const* bh,
                         int kind, hipStream_t s)
{
    if (c->L == 0) return RS_OK;
    const size_t ts = f32 ? 4 : 8;
    const int slot = c->cur_slot;
    // BF16 contexts run the float path with BF16 weights
    const int bf = f32 && c->bf16;
    if (bf) W = c->W16.data();
    if (mlp_fits(f32, nc, c->r, c->wrows)) {
        MlpArgs m{};
        for (int l = 0; l < c->L; ++l) {
            m.W[l] = W[l];
            m.b[l] = bh[l];
            m.pre[l] = pre ? pre[l] : nullptr;
        }
        m.act = act;
        m.L = c->L;
        m.w = c->w;
        m.wrows = c->wrows;
        m.r = c->r;
        m.nc = nc;
        m.lda0 = c->lda0;
        m.lda = c->lda_h;
        m.items = cap;
        m.count = count;
        m.z = z;
        m.zmap = zmap;
        double pb = 0, pf = 0;
        for (int l = 0; l < c->L; ++l) {
            const int K = l == 0 ? c->r : c->w;
            pf += 2.0 * c->w * K * nc;
            pb += ts * (double)c->w * nc * (pre ? 1 : 0);
        }
        pb += ts * (double)c->w * nc + 8.0 * c->r;
        Work wk = item_work(pb, pf, cap, count, slot, which);
        for (int l = 0; l < c->L; ++l) wk.b0 += ts * (double)c->w * (l == 0 ? c->r : c->w);
        return run(c, kind, wk, s, [&] { return launch_mlp(f32, m, s, bf, c->n_cu); });
    }
    if (bf) return fail(c, RS_ERR_UNSUPPORTED, "BF16 hidden layers need the fused kernel");
    for (int l = 0; l < c->L; ++l) {
        GemmArgs a{};
        a.A = W[l];
        a.lda = l == 0 ? c->lda0 : c->lda_h;
        a.rows = c->w;
        a.rows_pad = c->wrows;
        a.K = l == 0 ? c->r : c->w;
        a.nc = nc;
        a.items = cap;
        a.count = count;
        a.in_mode = l == 0 ? IN_LATENT : IN_ELU;
        a.Y = l == 0 ? nullptr : pre[l - 1];
        a.y_rows = c->wrows;
        a.z = z;
        a.zmap = zmap;
        a.r = c->r;
        a.bias = bh[l];
        a.out_mode = OUT_PACK;
        a.C = pre[l];
        RS_TRY(run(c, kind, gemm_work(ts, a.rows, a.K, cap, nc, count, slot, which), s,
                   [&] { return launch_gemm(f32, ROLE_HIDDEN, a, s); }));
    }
    return activate(c, f32, pre[c->L - 1], act, nc, cap, count, which, s);
}

static ElemOptArgs elem_opt_args(const rs_ctx* c, const void* out, int nc, const int* count)
{
    ElemOptArgs o{};
    o.out = out;
    o.rows_pad = c->Mp;
    o.nc = nc;
    o.r = c->r;
    o.S = c->S;
    o.count = count;
    o.ec = c->ec;
    o.mu = c->mu;
    o.lam = c->lam;
    return o;
}

// T-precision decoder value + Jacobian, reduced rows, element terms and (exact)
// the curvature term.  `cap` items fit the launch; `count` (device, nullable)
// holds the actual number.  Item i uses latent point z[zmap[i]] and the loads
// of batch index imap[i].
// ------------------------------------------------------------------ dynamics and contact
// Per call: the inertia term's per-item vectors from the inertial targets of B
// items (W_out^T M (qbar - b_out) and |qbar - b_out|_M^2), forming G = W_out^T M
// W_out first when the decoder changed.  No inertia when qbar is NULL or dt <= 0.
static int dyn_setup(rs_ctx* c, const rs_load* load, int B, int b0, hipStream_t s)
{
    c->dyn_inertia = 0;
    if (!load || !load->qbar || !(load->dt > 0.0)) return RS_OK;
    if (B > c->max_batch) return fail(c, RS_ERR_ARG, "inertial targets for more than max_batch items");
    if (c->G_dirty) {
        RS_HIP(launch_dyn_gram(0, c->Wfull64, c->lda_out, c->n_out, c->row_mass, c->in_last, c->Gdyn, s),
               "inertia Gram matrix");
        c->G_dirty = false;
    }
    RS_HIP(launch_dyn_prep(0, c->Wfull64, c->lda_out, c->bfull64, c->pinned_row, c->row_mass, c->n_out, c->in_last,
                           load->qbar + (size_t)b0 * c->n_out, B, c->dyn_c, c->dyn_kappa, s),
           "inertia targets");
    c->dyn_inertia = 1;
    c->dyn_use_eta = 0;
    c->dyn_inv_dt2 = 1.0 / (load->dt * load->dt);
    return RS_OK;
}

static bool dyn_active(const rs_ctx* c, uint32_t flags)
{
    return !(flags & RS_ELASTIC_ONLY) && (c->dyn_inertia || c->ncont > 0);
}

static DynArgs dyn_args(const rs_ctx* c, const int* count, const int* imap, const double* z, const int* zmap,
                        const void* act, const void* out, int nc)
{
    DynArgs a{};
    a.count = count;
    a.imap = imap;
    a.zmap = zmap;
    a.z = z;
    a.L = c->L;
    a.r = c->r;
    a.in_last = c->in_last;
    a.nc = nc;
    a.act = c->L > 0 ? act : nullptr;
    a.wrows = c->wrows;
    a.out = out;
    a.rows_pad = c->Mp;
    a.crow = c->crow;
    a.ncont = c->ncont;
    a.Xc = c->Xc;
    a.k_ground = c->k_ground;
    a.ground_y = c->ground_y;
    a.G = c->Gdyn;
    a.eta = c->dyn_use_eta ? c->dyn_eta : nullptr;
    a.cvec = c->dyn_c;
    a.kappa = c->dyn_kappa;
    a.inv_dt2 = c->dyn_inv_dt2;
    a.inertia = c->dyn_inertia;
    a.in_rows = c->in_rows;
    return a;
}

static int eval_T(rs_ctx* c, int cap, const int* count, const double* z, const int* zmap, const double* targets,
                  const double* force, const int* imap, uint32_t flags, double* E, double* g, double* H,
                  hipStream_t s)
{
    const int r = c->r, nc = c->nc;
    const int f32 = c->f32;
    const size_t ts = c->tsz;
    const int slot = c->cur_slot;
    RS_TRY(hidden_layers(c, f32, nc, cap, count, 0, z, zmap, c->pre.data(), c->act, c->W.data(), c->bh.data(),
                         K_GEMM_HIDDEN, s));
    // the fused kernel stores no J_R rows: only where nothing after the element physics reads them
    const bool fuse = c->fused && c->fused_on && c->ncont == 0 && !dyn_active(c, flags) &&
                      !(flags & (RS_ELEM_PSD | RS_DEBUG_ELEM_HESS));
    if (!fuse) {
        GemmArgs a{};
        a.A = c->Wbig;
        a.lda = c->lda_out;
        a.rows = c->M;
        a.rows_pad = c->Mp;
        a.K = c->in_last;
        a.nc = nc;
        a.items = cap;
        a.count = count;
        a.in_mode = c->L > 0 ? IN_RAW_T : IN_LATENT;
        a.Y = c->L > 0 ? c->act : nullptr;
        a.y_rows = c->wrows;
        a.z = z;
        a.zmap = zmap;
        a.r = r;
        a.bias = c->bbig;
        a.out_mode = OUT_PACK;
        a.C = c->out;
        if (c->bf16) {
            // whole 32-deep chunks: W_big columns and activation rows past the width are zero
            a.A = c->Wbig16;
            a.K = c->lda_out;
        }
        RS_TRY(run(c, K_GEMM_OUT, gemm_work(ts, c->M, a.K, cap, nc, count, slot, 0), s, [&] {
            if (c->bf16) return launch_gemm_p_bf16(ROLE_OUT, a, 8 * c->n_cu, s);
            // twelve workgroups per compute unit: the best of 3..12 per CU measured for the
            // 2560 x 128 map at B = 1024 (fewer leave the A-fragment loads exposed)
            return gemm_p_fits(f32, a.K) ? launch_gemm_p(f32, ROLE_OUT, a, 12 * c->n_cu, s)
                                         : launch_gemm(f32, ROLE_OUT, a, s);
        }));
    }
    const bool exact = (flags & RS_HESS_EXACT) && c->L > 0 && H;
    int split = 1;
    {
        ElemArgs a{};
        a.out = c->out;
        a.rows_pad = c->Mp;
        a.nc = nc;
        a.r = r;
        a.S = c->S;
        a.nt = c->nt;
        a.nf = c->nf;
        a.count = count;
        a.wV = c->wV;
        a.Xt = c->Xt;
        a.targets = c->nt ? targets : nullptr;
        a.force = c->nf ? force : nullptr;
        a.imap = imap;
        a.mu = c->mu;
        a.lam = c->lam;
        a.k_c = c->k_c;
        a.elastic_only = (flags & RS_ELASTIC_ONLY) ? 1 : 0;
        a.grav_row = c->grav_row;
        a.force_row = c->force_row;
        a.E = E;
        a.g = g;
        a.H = H;
        a.dseed = exact ? c->dseed : nullptr;
        // A small batch splits each item's rounds over several workgroups (the
        // curvature pass sums their partial g and H), so that the element
        // kernel's per-item latency does not set the launch's duration.
        // (The fused kernel takes four items per workgroup and splits their
        // rows at batches below eight items per compute unit.)
        a.parts = 1;
        if (exact && !E && g && cap > 0) {
            int parts = fuse ? elem_fused_parts(c->bf16, cap, c->n_cu) : std::min(8, 2 * c->n_cu / cap);
            while (parts > 1 && (size_t)parts * cap > c->npart) --parts;
            if (parts > 1) {
                a.parts = parts;
                a.part_stride = cap;
                a.g = c->gpart;
                a.H = c->Hpart;
            }
        }
        split = a.parts;
        if (fuse) {
            FusedElemArgs f{};
            f.e = a;
            f.e.out = nullptr;
            f.A = c->bf16 ? c->Wbig16 : c->Wbig;
            f.lda = c->lda_out;
            f.K = c->lda_out;
            f.rows = c->M;
            f.bias = static_cast<const float*>(c->bbig);
            f.Y = static_cast<const float*>(c->act);
            f.y_rows = c->wrows;
            f.cap = cap;
            // algorithmic work: the item's activation columns in, seeds and (E, g, H) out, W_big once
            // per launch; flops: the output map's products (float32 or float32-equivalent: the
            // matrix-core part)
            Work w = item_work((double)nc * c->lda_out * ts + (exact ? (double)c->Mp * ts : 0.0) +
                                   8.0 * (1 + r + r * r),
                               2.0 * c->M * c->in_last * nc, cap, count, slot, 0);
            w.b0 += (c->bf16 ? 6.0 : 4.0) * c->Mp * c->lda_out;
            RS_TRY(run(c, K_ELEM_FUSED, w, s, [&] { return launch_elem_fused(c->bf16, f, s); }));
        } else {
            // algorithmic bytes: read the item's rows once, write seeds and (E, g, H)
            const double pb = (double)c->M * nc * ts + (exact ? (double)c->Mp * ts : 0.0) + 8.0 * (1 + r + r * r);
            const double pf = (double)c->S * (18.0 * r * r + 80.0 * r + 150.0);
            RS_TRY(run(c, K_ELEM, item_work(pb, pf, cap, count, slot, 0), s,
                       [&] { return launch_elem(f32, a, cap, s); }));
        }
    }
    const bool dyn = dyn_active(c, flags) && (g || H || E);
    if (dyn && exact && c->ncont > 0) {
        DynArgs d = dyn_args(c, count, imap, z, zmap, c->act, c->out, nc);
        d.dseed = c->dseed;
        RS_TRY(run(c, K_DYN, Work{}, s, [&] { return launch_dyn(f32, 0, d, cap, s); }));
    }
    if (exact) {
        GemmArgs a{};
        a.A = c->WbigT;
        a.lda = c->Mp;
        a.rows = c->in_last;
        a.rows_pad = c->in_rows;
        a.K = c->Mp;
        a.nc = 1;
        a.items = cap;
        a.count = count;
        a.in_mode = IN_RAW;
        a.Y = c->dseed;
        a.y_rows = c->Mp;
        a.r = r;
        a.out_mode = OUT_PACK;
        a.C = c->gbar;
        a.ksplit = c->ksplit;
        a.split_stride = (size_t)c->max_batch * c->in_rows;
        RS_TRY(run(c, K_GEMM_ADJ, gemm_work(ts, c->in_last, c->Mp, cap, 1, count, slot, 0), s,
                   [&] { return launch_gemm(f32, ROLE_ADJ, a, s); }));
        if (dyn && c->dyn_inertia) {
            DynArgs d = dyn_args(c, count, imap, z, zmap, c->act, c->out, nc);
            d.gbar = c->gbar;
            RS_TRY(run(c, K_DYN, Work{}, s, [&] { return launch_dyn(f32, 1, d, cap, s); }));
        }
        CurvArgs ca{};
        for (int l = 0; l < c->L; ++l) {
            ca.pre[l] = c->pre[l];
            ca.W[l] = c->W[l];
        }
        // the fused hidden-layer kernel keeps (nc x wrows) blocks, the per-layer path (wrows x nc)
        const bool fused = mlp_fits(f32, nc, c->r, c->wrows);
        ca.pre_su = fused ? 1 : nc;
        ca.pre_sc = fused ? c->wrows : 1;
        ca.gbar = c->gbar;
        ca.ksplit = c->ksplit;
        ca.split_stride = (size_t)c->max_batch * c->in_rows;
        ca.L = c->L;
        ca.width = c->w;
        ca.nc = nc;
        ca.r = r;
        ca.pre_rows = c->wrows;
        ca.lda0 = c->lda0;
        ca.lda = c->lda_h;
        ca.count = count;
        ca.H = H;
        ca.grev = nullptr;
        if (split > 1) {
            ca.parts = split;
            ca.part_stride = cap;
            ca.Hp = c->Hpart;
            ca.gp = c->gpart;
            ca.g = g;
        }
        const double pb = (double)c->L * c->w * nc * ts + (double)c->ksplit * c->in_rows * ts + 16.0 * r * r;
        const double pf = (double)c->L * (2.0 * r * r * c->w + 2.0 * c->w * c->w);
        RS_TRY(run(c, K_CURV, item_work(pb, pf, cap, count, slot, 0), s, [&] { return launch_curv(f32, ca, cap, c->n_cu, s); }));
    }
    if ((flags & RS_ELEM_PSD) && H) {
        // the per-element projection's correction, added to the finished H
        ElemOptArgs o = elem_opt_args(c, c->out, nc, count);
        o.H = H;
        const double pb = (double)c->M * nc * ts + 16.0 * r * r;
        const double pf = (double)c->S * (9.0 * 81 * 2 + 6.0 * 36 * 54);
        RS_TRY(run(c, K_ELEM_PSD, item_work(pb, pf, cap, count, slot, 0), s,
                   [&] { return launch_elem_psd(f32, o, cap, s); }));
    }
    if (dyn) {
        DynArgs d = dyn_args(c, count, imap, z, zmap, c->act, c->out, nc);
        d.E = E;
        d.g = g;
        d.H = H;
        RS_TRY(run(c, K_DYN, Work{}, s, [&] { return launch_dyn(f32, 2, d, cap, s); }));
    }
    return RS_OK;
}

// The gradient g = J^T grad_q E by reverse mode: a value pass of the decoder
// (pre-activations kept), the value rows of the output map, the element
// kernel for E and the adjoint seeds d = dE/d(row), W_big^T d, and the
// reverse pass back through the hidden layers.  No Jacobian column is formed.
static bool grad_reverse_ok(const rs_ctx* c) { return c->L > 0 && !c->bf16 && mlp_fits(c->f32, 1, c->r, c->wrows); }

static int eval_grad_rev(rs_ctx* c, int cap, const int* count, const double* z, const int* zmap,
                         const double* targets, const double* force, const int* imap, uint32_t flags, double* E,
                         double* g, hipStream_t s, double* delta = nullptr)
{
    const int r = c->r;
    const int f32 = c->f32;
    const size_t ts = c->tsz;
    const int slot = c->cur_slot;
    RS_TRY(hidden_layers(c, f32, 1, cap, count, 0, z, zmap, c->pre.data(), c->act, c->W.data(), c->bh.data(),
                         K_GEMM_HIDDEN, s));
    {
        GemmArgs a{};
        a.A = c->Wbig;
        a.lda = c->lda_out;
        a.rows = c->M;
        a.rows_pad = c->Mp;
        a.K = c->in_last;
        a.nc = 1;
        a.items = cap;
        a.count = count;
        a.in_mode = IN_RAW_T;
        a.Y = c->act;
        a.y_rows = c->wrows;
        a.r = r;
        a.bias = c->bbig;
        a.out_mode = OUT_PACK;
        a.C = c->out;
        RS_TRY(run(c, K_GEMM_OUT, gemm_work(ts, c->M, a.K, cap, 1, count, slot, 0), s, [&] {
            return gemm_p_fits(f32, a.K) ? launch_gemm_p(f32, ROLE_OUT, a, 8 * c->n_cu, s)
                                         : launch_gemm(f32, ROLE_OUT, a, s);
        }));
    }
    {
        ElemArgs a{};
        a.out = c->out;
        a.rows_pad = c->Mp;
        a.nc = 1;
        a.r = 0;
        a.S = c->S;
        a.nt = c->nt;
        a.nf = c->nf;
        a.count = count;
        a.wV = c->wV;
        a.Xt = c->Xt;
        a.targets = c->nt ? targets : nullptr;
        a.force = c->nf ? force : nullptr;
        a.imap = imap;
        a.mu = c->mu;
        a.lam = c->lam;
        a.k_c = c->k_c;
        a.elastic_only = (flags & RS_ELASTIC_ONLY) ? 1 : 0;
        a.grav_row = c->grav_row;
        a.force_row = c->force_row;
        a.E = E;
        a.dseed = c->dseed;
        a.parts = 1;
        const double pb = (double)c->M * ts + (double)c->Mp * ts + 8.0;
        const double pf = (double)c->S * 150.0;
        RS_TRY(run(c, K_ELEM, item_work(pb, pf, cap, count, slot, 0), s, [&] { return launch_elem(f32, a, cap, s); }));
    }
    {
        GemmArgs a{};
        a.A = c->WbigT;
        a.lda = c->Mp;
        a.rows = c->in_last;
        a.rows_pad = c->in_rows;
        a.K = c->Mp;
        a.nc = 1;
        a.items = cap;
        a.count = count;
        a.in_mode = IN_RAW;
        a.Y = c->dseed;
        a.y_rows = c->Mp;
        a.r = r;
        a.out_mode = OUT_PACK;
        a.C = c->gbar;
        a.ksplit = c->ksplit;
        a.split_stride = (size_t)c->max_batch * c->in_rows;
        RS_TRY(run(c, K_GEMM_ADJ, gemm_work(ts, c->in_last, c->Mp, cap, 1, count, slot, 0), s,
                   [&] { return launch_gemm(f32, ROLE_ADJ, a, s); }));
    }
    CurvArgs ca{};
    for (int l = 0; l < c->L; ++l) {
        ca.pre[l] = c->pre[l];
        ca.W[l] = c->W[l];
    }
    // value-only blocks of the fused kernel: unit u at u (one column)
    ca.pre_su = 1;
    ca.pre_sc = c->wrows;
    ca.gbar = c->gbar;
    ca.ksplit = c->ksplit;
    ca.split_stride = (size_t)c->max_batch * c->in_rows;
    ca.L = c->L;
    ca.width = c->w;
    ca.nc = 1;
    ca.r = r;
    ca.pre_rows = c->wrows;
    ca.lda0 = c->lda0;
    ca.lda = c->lda_h;
    ca.count = count;
    ca.H = nullptr;
    ca.grev = g;
    ca.delta = delta;
    const double pb = (double)c->L * c->w * ts + (double)c->ksplit * c->in_rows * ts + 8.0 * r;
    const double pf = (double)c->L * 2.0 * c->w * c->w;
    return run(c, K_CURV, item_work(pb, pf, cap, count, slot, 0), s, [&] { return launch_curv(f32, ca, cap, c->n_cu, s); });
}

// float64 value-only decoder and energy for `cap` items (count on the device
// when non-NULL).  Item i uses latent point z[i] and the loads of imap[i].
static int energy_f64(rs_ctx* c, int cap, const int* count, int which, const double* z, const double* targets,
                      const double* force, const int* imap, int elastic_only, double* E, hipStream_t s,
                      int kind_hidden, int kind_out)
{
    const int r = c->r;
    const int slot = c->cur_slot;
    {
        std::vector<void*> pre64(c->pre64.begin(), c->pre64.end());
        std::vector<const void*> W64(c->W64.begin(), c->W64.end()), b64(c->bh64.begin(), c->bh64.end());
        RS_TRY(hidden_layers(c, 0, 1, cap, count, which, z, nullptr, mlp_fits(0, 1, c->r, c->wrows) ? nullptr : pre64.data(),
                             c->act64, W64.data(), b64.data(), kind_hidden, s));
    }
    {
        GemmArgs a{};
        a.A = c->Wbig64;
        a.lda = c->lda_out;
        a.rows = c->M;
        a.rows_pad = c->Mp;
        a.K = c->in_last;
        a.nc = 1;
        a.items = cap;
        a.count = count;
        a.in_mode = c->L > 0 ? IN_RAW_T : IN_LATENT;
        a.Y = c->L > 0 ? c->act64 : nullptr;
        a.y_rows = c->wrows;
        a.z = z;
        a.r = r;
        a.bias = c->bbig64;
        a.out_mode = OUT_PACK;
        a.C = c->out64;
        RS_TRY(run(c, kind_out, gemm_work(8, c->M, a.K, cap, 1, count, slot, which), s, [&] {
            return gemm_p_fits(0, a.K) ? launch_gemm_p(0, ROLE_OUT, a, 8 * c->n_cu, s) : launch_gemm(0, ROLE_OUT, a, s);
        }));
    }
    EnergyArgs e{};
    e.out = c->out64;
    e.rows_pad = c->Mp;
    e.S = c->S;
    e.nt = c->nt;
    e.nf = c->nf;
    e.count = count;
    e.wV = c->wV;
    e.Xt = c->Xt;
    e.targets = c->nt ? targets : nullptr;
    e.force = c->nf ? force : nullptr;
    e.imap = imap;
    e.mu = c->mu;
    e.lam = c->lam;
    e.k_c = c->k_c;
    e.elastic_only = elastic_only;
    e.grav_row = c->grav_row;
    e.force_row = c->force_row;
    e.E = E;
    RS_TRY(run(c, K_ENERGY, item_work(8.0 * c->M + 8.0, (double)c->S * 60.0, cap, count, slot, which), s,
               [&] { return launch_energy(e, cap, s); }));
    if (!elastic_only && (c->dyn_inertia || c->ncont > 0)) {
        DynArgs d = dyn_args(c, count, imap, z, nullptr, c->act64, c->out64, 1);
        d.E = E;
        RS_TRY(run(c, K_DYN, Work{}, s, [&] { return launch_dyn(0, 3, d, cap, s); }));
    }
    return RS_OK;
}

extern "C" int rs_energy_grad_hess(rs_ctx* c, int32_t B, const double* z, const rs_load* load,
                                   uint32_t flags, double* E, double* g, double* H, void* stream)
{
    if (!c) return RS_ERR_STATE;
    if (B < 0) return fail(c, RS_ERR_ARG, "B < 0");
    if (B == 0) return RS_OK;
    if (!z || !E) return fail(c, RS_ERR_ARG, "z and E must not be NULL");
    const bool eonly = flags & RS_ENERGY_ONLY;
    if (!eonly && !g) return fail(c, RS_ERR_ARG, "g must not be NULL unless RS_ENERGY_ONLY");
    if ((flags & RS_GRAD_REVERSE) && H) return fail(c, RS_ERR_ARG, "RS_GRAD_REVERSE takes H == NULL");
    if ((flags & RS_ELEM_PSD) && (eonly || !H)) return fail(c, RS_ERR_ARG, "RS_ELEM_PSD needs H");
    const bool dump = (flags & RS_DEBUG_ELEM_HESS) != 0;
    if (dump && !c->dump_He) return fail(c, RS_ERR_ARG, "RS_DEBUG_ELEM_HESS without a buffer from rs_set_elem_hess_dump");
    if (dump && eonly) return fail(c, RS_ERR_ARG, "RS_DEBUG_ELEM_HESS needs the gradient path (not RS_ENERGY_ONLY)");
    const bool rev = (flags & RS_GRAD_REVERSE) && grad_reverse_ok(c);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const double* tg = load ? load->targets : nullptr;
    const double* fo = load ? load->force : nullptr;
    const int r = c->r;
    c->cur_slot = -1;
    for (int c0 = 0; c0 < B; c0 += c->max_batch) {
        const int n = std::min(c->max_batch, B - c0);
        const double* zc = z + (size_t)c0 * r;
        const double* tgc = tg ? tg + (size_t)c0 * c->nt * 3 : nullptr;
        const double* foc = fo ? fo + (size_t)c0 * 3 : nullptr;
        RS_TRY(dyn_setup(c, load, n, c0, s));
        if (!eonly && rev && dyn_active(c, flags))
            return fail(c, RS_ERR_UNSUPPORTED, "RS_GRAD_REVERSE has no inertia or contact term");
        if (!eonly && rev)
            RS_TRY(eval_grad_rev(c, n, nullptr, zc, nullptr, tgc, foc, nullptr, flags, c->f32 ? nullptr : E + c0,
                                 g + (size_t)c0 * r, s));
        else if (!eonly)
            RS_TRY(eval_T(c, n, nullptr, zc, nullptr, tgc, foc, nullptr, flags, c->f32 ? nullptr : E + c0,
                          g + (size_t)c0 * r, H ? H + (size_t)c0 * r * r : nullptr, s));
        if (dump && c0 < c->dump_max) {
            const int nd = std::min(n, c->dump_max - c0);
            ElemOptArgs o = elem_opt_args(c, c->out, rev ? 1 : c->nc, nullptr);
            o.He = c->dump_He + (size_t)c0 * c->S * 144;
            RS_TRY(run(c, K_ELEM_DUMP, item_work(8.0 * c->S * 144, (double)c->S * 3000, nd, nullptr, -1, 0), s,
                       [&] { return launch_elem_hess_dump(c->f32, o, nd, s); }));
        }
        if (eonly || c->f32)
            RS_TRY(energy_f64(c, n, nullptr, 0, zc, tgc, foc, nullptr, (flags & RS_ELASTIC_ONLY) ? 1 : 0, E + c0, s,
                              K_LS_GEMM_HIDDEN, K_LS_GEMM_OUT));
    }
    return RS_OK;
}

extern "C" int rs_set_elem_hess_dump(rs_ctx* c, double* He, int32_t max_items)
{
    if (!c) return RS_ERR_STATE;
    if (max_items < 0 || (max_items > 0 && !He)) return fail(c, RS_ERR_ARG, "bad element-Hessian dump buffer");
    c->dump_He = max_items > 0 ? He : nullptr;
    c->dump_max = c->dump_He ? max_items : 0;
    return RS_OK;
}

extern "C" int rs_set_fused(rs_ctx* c, int32_t on, int32_t* applies)
{
    if (!c) return RS_ERR_STATE;
    c->fused_on = on ? 1 : 0;
    if (applies) *applies = c->fused;
    return RS_OK;
}

extern "C" int rs_param_count(const rs_ctx* c, int64_t* n)
{
    if (!c) return RS_ERR_STATE;
    if (!n) return RS_ERR_ARG;
    *n = (int64_t)c->n_params;
    return RS_OK;
}

extern "C" int rs_energy_param_grad(rs_ctx* c, int32_t B, const double* z, const rs_load* load, uint32_t flags,
                                    double* E, double* g, double* grad, void* stream)
{
    if (c && (c->ncont > 0 || (load && load->qbar && load->dt > 0.0)))
        return fail(c, RS_ERR_UNSUPPORTED, "the parameter gradient has no inertia or contact term");
    if (c) c->dyn_inertia = 0;
    if (!c) return RS_ERR_STATE;
    if (B < 0) return fail(c, RS_ERR_ARG, "B must be >= 0");
    if (!grad) return fail(c, RS_ERR_ARG, "grad is NULL");
    if (B > 0 && !z) return fail(c, RS_ERR_ARG, "z is NULL");
    if (flags & ~(uint32_t)RS_ELASTIC_ONLY) return fail(c, RS_ERR_ARG, "flags other than RS_ELASTIC_ONLY");
    if (!grad_reverse_ok(c))
        return fail(c, RS_ERR_UNSUPPORTED,
                    "parameter gradients need hidden layers that fit the fused kernel and a float32 or float64 context");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const double* tg = load ? load->targets : nullptr;
    const double* fo = load ? load->force : nullptr;
    const int r = c->r, w = c->w, L = c->L, f32 = c->f32;
    c->cur_slot = -1;
    if (B == 0) return run(c, K_PARAM_GRAD, item_work(0, 0, 1, nullptr, -1, 0), s,
                           [&] { return launch_fill_zero(grad, c->n_params, s); });
    for (int c0 = 0; c0 < B; c0 += c->max_batch) {
        const int n = std::min(c->max_batch, B - c0);
        const double* zc = z + (size_t)c0 * r;
        const double* tgc = tg ? tg + (size_t)c0 * c->nt * 3 : nullptr;
        const double* foc = fo ? fo + (size_t)c0 * 3 : nullptr;
        RS_TRY(eval_grad_rev(c, n, nullptr, zc, nullptr, tgc, foc, nullptr, flags, (E && !f32) ? E + c0 : nullptr,
                             g ? g + (size_t)c0 * r : nullptr, s, c->delta));
        if (E && f32)
            RS_TRY(energy_f64(c, n, nullptr, 0, zc, tgc, foc, nullptr, (flags & RS_ELASTIC_ONLY) ? 1 : 0, E + c0, s,
                              K_LS_GEMM_HIDDEN, K_LS_GEMM_OUT));
        const int acc = c0 > 0;
        // dE/dW_big = sum_b seeds_b h_L,b^T (folded back to W_out below)
        ParamOuterArgs o{};
        o.X = c->dseed;
        o.x_f64 = !f32;
        o.x_stride = c->Mp;
        o.Y = c->act;
        o.y_mode = PO_Y_RAW;
        o.y_stride = c->wrows;
        o.B = n;
        o.M = c->M;
        o.N = c->in_last;
        o.out = c->dWbig;
        o.ldo = c->in_last;
        o.outb = c->dbbig;
        o.accumulate = acc;
        o.part = c->ppart;
        o.part_cap = c->ppart_cap;
        const double ts = (double)c->tsz;
        RS_TRY(run(c, K_PARAM_GRAD, item_work(ts * (c->Mp + c->wrows), 2.0 * c->M * c->in_last, n, nullptr, -1, 0), s,
                   [&] { return launch_param_outer(f32, o, s); }));
        // hidden layers: dE/dW_l = sum_b delta_l,b h_{l-1},b^T with h_{l-1} = ELU(a_{l-1}) recomputed (h_0 = z)
        for (int l = 0; l < L; ++l) {
            ParamOuterArgs h{};
            h.X = c->delta + (size_t)l * w;
            h.x_f64 = 1;
            h.x_stride = (size_t)L * w;
            if (l == 0) {
                h.Y = zc;
                h.y_mode = PO_Y_F64;
                h.y_stride = r;
            } else {
                h.Y = c->pre[l - 1];
                h.y_mode = PO_Y_ELU;
                h.y_stride = c->wrows;
            }
            h.B = n;
            h.M = w;
            h.N = l == 0 ? r : w;
            h.out = grad + c->offW[l];
            h.ldo = h.N;
            h.outb = grad + c->offb[l];
            h.accumulate = acc;
            h.part = c->ppart;
            h.part_cap = c->ppart_cap;
            RS_TRY(run(c, K_PARAM_GRAD, item_work(8.0 * w + ts * h.N, 2.0 * w * h.N, n, nullptr, -1, 0), s,
                       [&] { return launch_param_outer(f32, h, s); }));
        }
    }
    return run(c, K_PARAM_GRAD, item_work(0, 0, 1, nullptr, -1, 0), s, [&] {
        return launch_unfold(c->dWbig, c->dbbig, c->in_last, c->fold_ptr, c->fold_row, c->fold_coef, c->n_out,
                             grad + c->offW[L], grad + c->offb[L], s);
    });
}

extern "C" int rs_decode(rs_ctx* c, int32_t B, const double* z, void* x, void* J, void* stream)
{
    if (!c) return RS_ERR_STATE;
    if (B < 0 || B > c->max_batch) return fail(c, RS_ERR_ARG, "B must be in [0, max_batch]");
    if (B == 0 || (!x && !J)) return RS_OK;
    if (!z) return fail(c, RS_ERR_ARG, "z is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int r = c->r, nc = J ? c->nc : 1;
    const int f32 = c->f32;
    const size_t ts = c->tsz;
    c->cur_slot = -1;
    RS_TRY(hidden_layers(c, f32, nc, B, nullptr, 0, z, nullptr, c->pre.data(), c->act, c->W.data(), c->bh.data(),
                         K_DECODE_HIDDEN, s));
    GemmArgs a{};
    a.A = c->Wfull;
    a.lda = c->lda_out;
    a.rows = c->n_out;
    a.rows_pad = c->Nfp;
    a.K = c->in_last;
    a.nc = nc;
    a.items = B;
    a.in_mode = c->L > 0 ? IN_RAW_T : IN_LATENT;
    a.Y = c->L > 0 ? c->act : nullptr;
    a.y_rows = c->wrows;
    a.z = z;
    a.r = r;
    a.bias = c->bfull;
    a.out_mode = OUT_SPLIT;
    a.Xo = x;
    a.Jo = J;
    a.Xrest = c->Xfull;
    if (c->bf16) {
        a.A = c->Wfull16;
        a.K = c->lda_out;
    }
    return run(c, K_DECODE_OUT, gemm_work(ts, c->n_out, a.K, B, nc, nullptr, -1, 0), s, [&] {
        if (c->bf16) return launch_gemm_p_bf16(ROLE_DECODE, a, 8 * c->n_cu, s);
        return gemm_p_fits(f32, a.K) ? launch_gemm_p(f32, ROLE_DECODE, a, 8 * c->n_cu, s)
                                     : launch_gemm(f32, ROLE_DECODE, a, s);
    });
}

// Copy the current Newton counters to the profile log (profiling only).
static int log_counters(rs_ctx* c, hipStream_t s)
{
    c->cur_slot = -1;
    if (!c->prof) return RS_OK;
    if (c->plog_next >= c->plog_cap) {
        // grow: keep what is logged so far
        const int cap = std::max(1024, 2 * c->plog_cap);
        int* np = nullptr;
        if (hipMalloc(&np, (size_t)cap * 4 * sizeof(int)) != hipSuccess) return fail(c, RS_ERR_OOM, "profile log");
        if (c->plog) {
            hipError_t e = hipMemcpyAsync(np, c->plog, (size_t)c->plog_cap * 4 * sizeof(int), hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return hip_fail(c, e, "hipMemcpyAsync");
            e = hipStreamSynchronize(s);
            if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
            (void)hipFree(c->plog);
        }
        c->plog = np;
        c->plog_cap = cap;
    }
    c->cur_slot = c->plog_next++;
    return RS_OK;
}

// Running count of the super-step whose Armijo kernel stored `tag` into host
// slot `slot`.  The kernel's system-scope release store normally lands before
// the completion event is seen; a slot that still holds an older tag is read
// again after the stream has drained (the super-step one ahead writes the other
// slot), and a tag that still differs is an error, never a stale count.
static int read_count(rs_ctx* c, int slot, unsigned int tag, hipStream_t s, int* count)
{
    unsigned long long v = __atomic_load_n(c->hcount + slot, __ATOMIC_ACQUIRE);
    if ((unsigned int)(v >> 32) != tag) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
        v = __atomic_load_n(c->hcount + slot, __ATOMIC_ACQUIRE);
        if ((unsigned int)(v >> 32) != tag) return fail(c, RS_ERR_STATE, "running count of a super-step never arrived");
    }
    *count = (int)(unsigned int)(v & 0xffffffffu);
    return RS_OK;
}

// Batched reduced solve (Newton or L-BFGS) fully on the device: evaluation,
// direction, line-search rounds and exits per item, with the host launching
// one super-step ahead.
static int solve_batch(rs_ctx* c, int32_t B, double* z, const rs_load* load, const NewtonParams& p, uint32_t flags,
                       bool lbfgs, int32_t* iters, int32_t* status, double* relgrad, double* E, void* stream,
                       int fixed_steps = 0)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    const double* tg = load ? load->targets : nullptr;
    const double* fo = load ? load->force : nullptr;
    const int r = c->r;

    NewtonState st{};
    st.z = z;
    st.iters = iters;
    st.status = status;
    st.relgrad = relgrad;
    st.E = E;
    st.g0 = c->g0;
    st.dz = c->dz;
    st.slope = c->slope;
    st.ls_j = c->ls_j;
    st.eval_list = c->eval_list;
    st.search_list = c->search_list;
    st.search_start = c->search_start;
    st.search_ncand = c->search_ncand;
    st.cand_item = c->cand_item;
    st.cand_j = c->cand_j;
    st.counters = c->counters;
    st.gw = c->gw;
    st.Hw = c->Hw;
    st.zc = c->zc;
    st.Ec = c->Ec;
    int* cnt = c->counters;

    c->cur_slot = -1;
    RS_TRY(run(c, K_INIT, Work{}, s, [&] { return launch_newton_init(st, B, s); }));
    RS_TRY(energy_f64(c, B, nullptr, 0, z, tg, fo, nullptr, 0, E, s, K_LS_GEMM_HIDDEN, K_LS_GEMM_OUT));
    RS_TRY(run(c, K_COMPACT, Work{}, s, [&] { return launch_compact_eval(st, B, p.window, s); }));
    // Every super-step either evaluates an item or advances its line search by
    // at least one trial, so this bounds the loop.  The host runs one
    // super-step ahead: it launches step k+1 before reading the running count
    // of step k (counts only fall, so an older count bounds every launch).
    // Each super-step ends with the Armijo kernel, which also builds the next
    // evaluation list and writes the running count to mapped host memory.
    // fixed_steps > 0: exactly that many super-steps, all sized for B (the window), with no host reads.
    // With a window W < B every admitted item ends within the per-item bound and frees its place,
    // so ceil(B / W) such bounds cover the whole batch.
    const int W = p.window > 0 ? p.window : B;
    const long per_item = (long)(p.max_iter + 1) * (2 + p.ls_max) + 2;
    const long max_steps = fixed_steps > 0 ? fixed_steps : per_item * ((B + W - 1) / W);
    int n_run = W;
    unsigned int tags[2] = {0, 0};
    for (long step = 0; step < max_steps; ++step) {
        RS_TRY(log_counters(c, s));
        if (lbfgs && grad_reverse_ok(c))
            RS_TRY(eval_grad_rev(c, n_run, cnt + 0, z, c->eval_list, tg, fo, c->eval_list, flags, nullptr, c->gw, s));
        else
            RS_TRY(eval_T(c, n_run, cnt + 0, z, c->eval_list, tg, fo, c->eval_list, flags, nullptr, c->gw,
                          lbfgs ? nullptr : c->Hw, s));
        if (lbfgs) {
            const double m = p.hist;
            RS_TRY(run(c, K_LBFGS, item_work(8.0 * (5 * r + 2 * m * r), 8.0 * m * r, n_run, cnt + 0, c->cur_slot, 0),
                       s, [&] { return launch_lbfgs_dir(st, p, c->lb, n_run, s); }));
        } else {
            RS_TRY(run(c, K_DIR, item_work(8.0 * (r + r * r), (double)r * r * r, n_run, cnt + 0, c->cur_slot, 0),
                       s, [&] { return launch_newton_dir(st, p, n_run, s); }));
        }
        st.plog = c->cur_slot >= 0 ? c->plog + 4 * (size_t)c->cur_slot : nullptr;
        RS_TRY(run(c, K_COMPACT, Work{}, s, [&] { return launch_compact_search(st, p, B, s); }));
        const int cap_c = n_run * kLsCand;
        RS_TRY(energy_f64(c, cap_c, cnt + 1, 1, c->zc, tg, fo, c->cand_item, 0, c->Ec, s, K_LS_GEMM_HIDDEN,
                          K_LS_GEMM_OUT));
        const int par = (int)(step & 1);
        if (c->tag_next == 0) c->tag_next = 1; // tag 0 marks a slot no super-step has written
        const unsigned int tag = c->tag_next++;
        tags[par] = tag;
        RS_TRY(run(c, K_ARMIJO, item_work(8.0 * kLsCand, 0, n_run, cnt + 2, c->cur_slot, 2), s,
                   [&] { return launch_armijo(st, p, B, c->hcount_dev + par, tag, s); }));
        if (fixed_steps > 0) continue;
        // the count reaches host memory by the kernel's own system-scope store; the event only marks completion
        hipError_t e = hipEventRecord(c->cnt_ev[par], s);
        if (e != hipSuccess) return hip_fail(c, e, "running-count copy");
        if (step == 0) continue;
        e = hipEventSynchronize(c->cnt_ev[par ^ 1]);
        if (e != hipSuccess) return hip_fail(c, e, "hipEventSynchronize");
        int prev = 0; // running after step - 1
        RS_TRY(read_count(c, par ^ 1, tags[par ^ 1], s, &prev));
        if (prev == 0) {
            n_run = 0;
            break;
        }
        n_run = prev;
    }
    if (fixed_steps > 0) {
        c->cur_slot = -1;
        return RS_OK;
    }
    if (n_run > 0) {
        // the bound was reached: settle the last count
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
        const int last = (int)((max_steps - 1) & 1);
        RS_TRY(read_count(c, last, tags[last], s, &n_run));
    }
    c->cur_slot = -1;
    if (n_run > 0) return fail(c, RS_ERR_STATE, "solver loop did not terminate");
    return RS_OK;
}

static int newton_solve(rs_ctx* c, int32_t B, double* z, const rs_load* load, const rs_solve_opts* o,
                        int fixed_steps, int32_t* iters, int32_t* status, double* relgrad, double* E, void* stream);

extern "C" int rs_newton_solve(rs_ctx* c, int32_t B, double* z, const rs_load* load, const rs_solve_opts* o,
                               int32_t* iters, int32_t* status, double* relgrad, double* E, void* stream)
{
    return newton_solve(c, B, z, load, o, 0, iters, status, relgrad, E, stream);
}

extern "C" int rs_newton_solve_async(rs_ctx* c, int32_t B, double* z, const rs_load* load, const rs_solve_opts* o,
                                     int32_t super_steps, int32_t* iters, int32_t* status, double* relgrad, double* E,
                                     void* stream)
{
    if (!c) return RS_ERR_STATE;
    if (super_steps < 1) return fail(c, RS_ERR_ARG, "super_steps must be at least 1");
    return newton_solve(c, B, z, load, o, super_steps, iters, status, relgrad, E, stream);
}

static int newton_solve(rs_ctx* c, int32_t B, double* z, const rs_load* load, const rs_solve_opts* o,
                        int fixed_steps, int32_t* iters, int32_t* status, double* relgrad, double* E, void* stream)
{
    if (!c) return RS_ERR_STATE;
    if (B < 0 || B > c->max_batch) return fail(c, RS_ERR_ARG, "B must be in [0, max_batch]");
    if (B == 0) return RS_OK;
    if (!z || !iters || !status || !relgrad || !E) return fail(c, RS_ERR_ARG, "NULL output pointer");
    rs_solve_opts def;
    rs_default_opts(&def);
    if (!o) o = &def;
    if (o->max_iter < 0 || o->ls_max < 0 || !(o->shrink > 0.0 && o->shrink < 1.0) || !(o->c1 >= 0.0) ||
        o->proj < 0 || o->proj > 2 || o->hess < 0 || o->hess > 3 || o->window < 0)
        return fail(c, RS_ERR_ARG, "invalid solver options");
    NewtonParams p{};
    p.r = c->r;
    p.max_iter = o->max_iter;
    p.ls_max = o->ls_max;
    p.proj = o->proj;
    p.c1 = o->c1;
    p.shrink = o->shrink;
    p.rel_tol = o->rel_tol;
    p.abs_tol = o->abs_tol;
    p.eig_floor = o->eig_floor;
    p.window = o->window < B ? o->window : 0;
    const uint32_t hflags = ((o->hess & 1) ? RS_HESS_EXACT : 0u) | ((o->hess & 2) ? RS_ELEM_PSD : 0u);
    RS_TRY(dyn_setup(c, load, B, 0, static_cast<hipStream_t>(stream)));
    return solve_batch(c, B, z, load, p, hflags, false, iters, status, relgrad, E, stream, fixed_steps);
}

// The last hidden activation of B latent points in float64 (the value pass of the
// line-search energies; z itself for a linear decoder) into h (B x in_last).
static int h_of_z(rs_ctx* c, int B, const double* z, double* h, hipStream_t s)
{
    if (c->L > 0) {
        std::vector<void*> pre64(c->pre64.begin(), c->pre64.end());
        std::vector<const void*> W64(c->W64.begin(), c->W64.end()), b64(c->bh64.begin(), c->bh64.end());
        RS_TRY(hidden_layers(c, 0, 1, B, nullptr, 0, z, nullptr,
                             mlp_fits(0, 1, c->r, c->wrows) ? nullptr : pre64.data(), c->act64, W64.data(),
                             b64.data(), K_LS_GEMM_HIDDEN, s));
    }
    RS_HIP(launch_dyn_take_h(c->L > 0 ? c->act64 : nullptr, c->wrows, z, c->in_last, B, h, s), "simulation state");
    return RS_OK;
}

extern "C" int rs_simulate(rs_ctx* c, int32_t B, double* z, const double* v0, const rs_load* load, int32_t steps,
                           double dt, const rs_solve_opts* o, int32_t* iters, int32_t* failed, double* ztraj,
                           void* stream)
{
    if (!c) return RS_ERR_STATE;
    if (B < 0 || B > c->max_batch) return fail(c, RS_ERR_ARG, "B must be in [0, max_batch]");
    if (steps < 0 || !(dt > 0.0)) return fail(c, RS_ERR_ARG, "steps must be >= 0 and dt > 0");
    if (B == 0) return RS_OK;
    if (!z || !iters || !failed) return fail(c, RS_ERR_ARG, "NULL pointer");
    rs_solve_opts def;
    rs_default_opts(&def);
    if (!o) o = &def;
    if (o->max_iter < 0 || o->ls_max < 0 || !(o->shrink > 0.0 && o->shrink < 1.0) || !(o->c1 >= 0.0) ||
        o->proj < 0 || o->proj > 2 || o->hess < 0 || o->hess > 3)
        return fail(c, RS_ERR_ARG, "invalid solver options");
    hipStream_t s = static_cast<hipStream_t>(stream);
    NewtonParams p{};
    p.r = c->r;
    p.max_iter = o->max_iter;
    p.ls_max = o->ls_max;
    p.proj = o->proj;
    p.c1 = o->c1;
    p.shrink = o->shrink;
    p.rel_tol = o->rel_tol;
    p.abs_tol = o->abs_tol;
    p.eig_floor = o->eig_floor;
    const uint32_t hflags = ((o->hess & 1) ? RS_HESS_EXACT : 0u) | ((o->hess & 2) ? RS_ELEM_PSD : 0u);
    rs_load ld{};
    if (load) {
        ld.targets = load->targets;
        ld.force = load->force;
    }
    const int m = c->in_last;
    if (c->G_dirty) {
        RS_HIP(launch_dyn_gram(0, c->Wfull64, c->lda_out, c->n_out, c->row_mass, m, c->Gdyn, s),
               "inertia Gram matrix");
        c->G_dirty = false;
    }
    RS_HIP(launch_zero_int(iters, B, s), "fill");
    RS_HIP(launch_zero_int(failed, B, s), "fill");
    // first step: the inertial target u^0 + dt v0
    RS_TRY(h_of_z(c, B, z, c->sim_h0, s));
    if (v0)
        RS_HIP(launch_dyn_prep(0, c->Wfull64, c->lda_out, nullptr, c->pinned_row, c->row_mass, c->n_out, m, v0, B,
                               c->sim_cv0, c->sim_kv0, s),
               "initial velocity");
    RS_HIP(launch_dyn_state(m, c->sim_h0, nullptr, v0 ? c->sim_cv0 : nullptr, v0 ? c->sim_kv0 : nullptr, dt, B,
                            c->dyn_eta, c->dyn_c, c->dyn_kappa, s),
           "simulation state");
    double* hp = c->sim_h0;
    double* hn = c->sim_h1;
    for (int k = 0; k < steps; ++k) {
        c->dyn_inertia = 1;
        c->dyn_use_eta = 1;
        c->dyn_inv_dt2 = 1.0 / (dt * dt);
        RS_TRY(solve_batch(c, B, z, &ld, p, hflags, false, c->sim_it, c->sim_st, c->sim_relg, c->sim_E, stream));
        RS_HIP(launch_sim_count(c->sim_it, c->sim_st, B, iters, failed, s), "simulation counts");
        if (ztraj &&
            hipMemcpyAsync(ztraj + (size_t)k * B * c->r, z, sizeof(double) * B * c->r, hipMemcpyDeviceToDevice, s) !=
                hipSuccess)
            return fail(c, RS_ERR_HIP, "hipMemcpyAsync");
        // next inertial target 2 u^(k+1) - u^k, in the decoder's range
        RS_TRY(h_of_z(c, B, z, hn, s));
        RS_HIP(launch_dyn_state(m, hp, hn, nullptr, nullptr, dt, B, c->dyn_eta, c->dyn_c, c->dyn_kappa, s),
               "simulation state");
        std::swap(hp, hn);
    }
    c->dyn_inertia = 0;
    c->dyn_use_eta = 0;
    return RS_OK;
}

extern "C" int rs_lbfgs_solve(rs_ctx* c, int32_t B, double* z, const rs_load* load, const rs_lbfgs_opts* o,
                              int32_t* iters, int32_t* status, double* relgrad, double* E, void* stream)
{
    if (!c) return RS_ERR_STATE;
    if (B < 0 || B > c->max_batch) return fail(c, RS_ERR_ARG, "B must be in [0, max_batch]");
    if (B == 0) return RS_OK;
    if (!z || !iters || !status || !relgrad || !E) return fail(c, RS_ERR_ARG, "NULL output pointer");
    rs_lbfgs_opts def;
    rs_default_lbfgs_opts(&def);
    if (!o) o = &def;
    if (o->max_iter < 0 || o->ls_max < 0 || o->history < 0 || o->history > RS_MAX_HISTORY ||
        !(o->shrink > 0.0 && o->shrink < 1.0) || !(o->c1 >= 0.0) || o->window < 0)
        return fail(c, RS_ERR_ARG, "invalid solver options");
    c->dyn_inertia = 0;
    if (c->ncont > 0 || (load && load->qbar && load->dt > 0.0))
        return fail(c, RS_ERR_UNSUPPORTED, "L-BFGS takes its gradient by reverse mode, which has no inertia or contact term");
    NewtonParams p{};
    p.r = c->r;
    p.max_iter = o->max_iter;
    p.ls_max = o->ls_max;
    p.hist = o->history;
    p.c1 = o->c1;
    p.shrink = o->shrink;
    p.rel_tol = o->rel_tol;
    p.abs_tol = o->abs_tol;
    p.window = o->window < B ? o->window : 0;
    return solve_batch(c, B, z, load, p, 0, true, iters, status, relgrad, E, stream);
}

extern "C" int rs_lipschitz_loss(rs_ctx* c, int32_t B, const double* z1, const double* z2, double* loss,
                                 double* per_pair, int32_t* n_valid, double* lip_max, void* stream)
{
    if (c) c->dyn_inertia = 0;
    if (!c) return RS_ERR_STATE;
    if (B < 0) return fail(c, RS_ERR_ARG, "B < 0");
    if (!loss || !n_valid || (B > 0 && (!z1 || !z2))) return fail(c, RS_ERR_ARG, "NULL pointer");
    if (c->max_batch < 2) return fail(c, RS_ERR_UNSUPPORTED, "the Lipschitz loss needs max_batch >= 2");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int r = c->r, chunk = c->max_batch / 2;
    c->cur_slot = -1;
    int c0 = 0;
    do {
        const int n = std::min(chunk, B - c0);
        const bool first = c0 == 0, last = c0 + n >= B;
        if (n > 0) {
            RS_TRY(run(c, K_LIPSCHITZ, item_work(16.0 * r, 0, n, nullptr, -1, 0), s, [&] {
                return launch_stack_pairs(z1 + (size_t)c0 * r, z2 + (size_t)c0 * r, c->zs, n, r, s);
            }));
            RS_TRY(eval_T(c, 2 * n, nullptr, c->zs, nullptr, nullptr, nullptr, nullptr,
                          RS_HESS_EXACT | RS_ELASTIC_ONLY, nullptr, c->gw, c->Hw, s));
        }
        RS_TRY(run(c, K_LIPSCHITZ, item_work(16.0 * r * r, 3.0 * r * r, n, nullptr, -1, 0), s, [&] {
            return launch_lipschitz(z1 + (size_t)c0 * r, z2 + (size_t)c0 * r, c->Hw, n, r,
                                    per_pair ? per_pair + c0 : nullptr, c->ell, c->lacc, first, last, loss,
                                    n_valid, lip_max, s);
        }));
        c0 += n;
    } while (c0 < B);
    return RS_OK;
}

// ------------------------------------------------------------------ learned part
// Workspace of the training calls, grown on demand (the first call of a size allocates).
static void* learn_alloc(rs_ctx* c, size_t bytes)
{
    void* p = nullptr;
    if (hipMalloc(&p, bytes ? bytes : 1) != hipSuccess) return nullptr;
    c->learn_bufs.push_back(p);
    return p;
}

// Lay the pass workspace of `pairs` pairs out in one block at `base` (NULL
// only measures); returns its size in bytes.  Every part starts on 256 bytes.
static size_t lip_ws_layout(const rs_ctx* c, int pairs, char* base, LipWs& ws)
{
    ws = LipWs{};
    ws.pairs = pairs;
    const size_t items = 2 * (size_t)pairs, cols = items * (c->r + 2), ts = c->tsz;
    const size_t wr = (size_t)std::max(c->w, c->r);
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        void* p = base ? base + off : nullptr;
        off += (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
        return p;
    };
    for (int l = 0; l < c->L; ++l) ws.Pre[l] = take((size_t)c->w * cols * ts);
    ws.X0 = take((size_t)c->r * cols * ts);
    ws.X = take(wr * cols * ts);
    ws.Out = take((size_t)9 * c->S * cols * ts);
    ws.Seed = take((size_t)9 * c->S * cols * ts);
    ws.G[0] = take(wr * cols * ts);
    ws.G[1] = take(wr * cols * ts);
    ws.D = take(wr * cols * ts);
    ws.Cs = static_cast<double*>(take(items * c->r * c->r * sizeof(double)));
    ws.nvalid = static_cast<int*>(take(sizeof(int)));
    return off;
}

static int lip_pairs_cap(const rs_ctx* c) { return std::max(1, std::min(128, c->max_batch / 2)); }

static int lip_ws(rs_ctx* c, LipWs& ws)
{
    if (c->lip.pairs > 0) {
        ws = c->lip;
        return RS_OK;
    }
    const int pairs = lip_pairs_cap(c);
    const size_t bytes = lip_ws_layout(c, pairs, nullptr, ws);
    char* base = static_cast<char*>(learn_alloc(c, bytes));
    if (!base) return fail(c, RS_ERR_OOM, "training workspace allocation failed");
    lip_ws_layout(c, pairs, base, ws);
    c->lip = ws;
    return RS_OK;
}

static SgemmArgs gemm_s(const void* A, long sAm, long sAk, const void* B, long sBk, long sBn, void* C, long ldc, int M,
                        int N, int K, int accumulate = 0, const void* bias = nullptr, int bias_every = 0)
{
    SgemmArgs g{};
    g.A = A; g.sAm = sAm; g.sAk = sAk;
    g.B = B; g.sBk = sBk; g.sBn = sBn;
    g.C = C; g.ldc = ldc;
    g.M = M; g.N = N; g.K = K;
    g.alpha = 1.0;
    g.accumulate = accumulate;
    g.bias = bias;
    g.bias_every = bias_every;
    return g;
}


extern "C" int rs_set_decoder_device(rs_ctx* c, const void* theta, int32_t theta_f64, void* stream)
{
    if (!c) return RS_ERR_STATE;
    if (!theta) return fail(c, RS_ERR_ARG, "theta is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t es = theta_f64 ? 8 : 4;
    auto at = [&](size_t off) { return static_cast<const char*>(theta) + off * es; };
    const int f32 = c->f32, L = c->L;
    for (int l = 0; l < L; ++l) {
        const int in = l == 0 ? c->r : c->w, lda = l == 0 ? c->lda0 : c->lda_h;
        RS_HIP(launch_load_padded(theta_f64, at(c->offW[l]), c->w, in, c->wrows, lda, nullptr, c->W64[l],
                                  f32 ? (float*)c->W[l] : nullptr, c->bf16 ? (uint16_t*)c->W16[l] : nullptr, s),
               "decoder load");
        RS_HIP(launch_load_vec(theta_f64, at(c->offb[l]), c->w, nullptr, c->bh64[l], f32 ? (float*)c->bh[l] : nullptr,
                               c->wrows, s),
               "decoder load");
    }
    const void* Wo = at(c->offW[L]);
    const void* bo = at(c->offb[L]);
    RS_HIP(launch_fold_rows(theta_f64, Wo, bo, c->in_last, c->ffold_ptr, c->ffold_src, c->ffold_coef, c->M, c->Mp,
                            c->lda_out, c->Wbig64, f32 ? (float*)c->Wbig : nullptr,
                            c->bf16 ? (uint16_t*)c->Wbig16 : nullptr, c->bbig64, f32 ? (float*)c->bbig : nullptr, s),
           "decoder fold");
    RS_HIP(launch_transpose(f32, f32 ? c->Wbig : (const void*)c->Wbig64, c->Mp, c->in_last, c->lda_out, c->WbigT, c->Mp,
                            c->in_rows, s),
           "decoder fold");
    RS_HIP(launch_load_padded(theta_f64, Wo, c->n_out, c->in_last, c->Nfp, c->lda_out, c->pinned_row,
                              c->Wfull64, f32 ? (float*)c->Wfull : nullptr,
                              c->bf16 ? (uint16_t*)c->Wfull16 : nullptr, s),
           "decoder load");
    RS_HIP(launch_load_vec(theta_f64, bo, c->n_out, c->pinned_row, c->bfull64,
                           f32 ? (float*)c->bfull : nullptr, c->n_out, s),
           "decoder load");
    c->G_dirty = true;
    return RS_OK;
}

static int lip_grad_check(rs_ctx* c, int32_t B, const double* z1, const double* z2, const double* loss,
                          const double* grad)
{
    if (B < 0) return fail(c, RS_ERR_ARG, "B < 0");
    if (!loss || !grad || (B > 0 && (!z1 || !z2))) return fail(c, RS_ERR_ARG, "NULL pointer");
    if (c->bf16) return fail(c, RS_ERR_UNSUPPORTED, "the Lipschitz-loss gradient needs a float32 or float64 context");
    if (c->max_batch < 2) return fail(c, RS_ERR_UNSUPPORTED, "the Lipschitz-loss gradient needs max_batch >= 2");
    return RS_OK;
}

// The Lipschitz-loss gradient over B pairs with the pass workspace ws (ws.pairs pairs per pass).
static int lip_param_grad(rs_ctx* c, int32_t B, const double* z1, const double* z2, double* loss, double* grad,
                          const LipWs& ws, hipStream_t s)
{
    c->dyn_inertia = 0;
    const int r = c->r, L = c->L, w = c->w, f32 = c->f32, nc2 = r + 2, S9 = 9 * c->S;
    c->cur_slot = -1;
    const int chunk = ws.pairs;
    RS_TRY(run(c, K_LIP_GRAD, Work{}, s, [&] { return launch_fill_zero(grad, c->n_params, s); }));
    RS_HIP(launch_fill_zero(c->dWbig, (size_t)c->M * c->in_last, s), "fill");
    RS_HIP(launch_fill_zero(c->dbbig, (size_t)c->M, s), "fill");
    RS_HIP(launch_lip_count(z1, z2, B, r, ws.nvalid, s), "lipschitz count");
    if (B == 0) return run(c, K_LIP_GRAD, Work{}, s, [&] { return launch_lip_coef(z1, z2, c->Hw, 0, r, ws.nvalid, ws.Cs, c->ell, loss, 1, s); });
    for (int c0 = 0; c0 < B; c0 += chunk) {
        const int P = std::min(chunk, B - c0), items = 2 * P;
        const long cols = (long)items * nc2;
        const double* z1c = z1 + (size_t)c0 * r;
        const double* z2c = z2 + (size_t)c0 * r;
        RS_HIP(launch_lip_stack(z1c, z2c, c->zs, P, r, s), "lipschitz pairs");
        RS_TRY(eval_T(c, items, nullptr, c->zs, nullptr, nullptr, nullptr, nullptr, RS_HESS_EXACT | RS_ELASTIC_ONLY,
                      nullptr, c->gw, c->Hw, s));
        RS_TRY(run(c, K_LIP_GRAD, Work{}, s, [&] {
            return launch_lip_coef(z1c, z2c, c->Hw, P, r, ws.nvalid, ws.Cs, c->ell, loss, c0 == 0, s);
        }));
        JetArgs j{};
        j.r = r;
        j.w = w;
        j.items = items;
        j.S = c->S;
        j.zs = c->zs;
        j.Cs = ws.Cs;
        j.wV = c->wV;
        j.mu = c->mu;
        j.lam = c->lam;
        // forward: jets through the hidden layers (pre-activations kept), then the element rows
        j.X = ws.X0;
        j.ldx = cols;
        RS_HIP(launch_jet(f32, 0, j, s), "jets");
        const void* Xin = ws.X0;
        for (int l = 0; l < L; ++l) {
            const int in = l == 0 ? r : w, lda = l == 0 ? c->lda0 : c->lda_h;
            RS_HIP(launch_gemm_s(f32, 0, gemm_s(c->W[l], lda, 1, Xin, cols, 1, ws.Pre[l], cols, w, (int)cols, in, 0,
                                                c->bh[l], nc2), s),
                   "jets");
            j.Pre = ws.Pre[l];
            j.ldp = cols;
            j.X = ws.X;
            RS_HIP(launch_jet(f32, 1, j, s), "jets");
            Xin = ws.X;
        }
        RS_HIP(launch_gemm_s(f32, 0, gemm_s(c->Wbig, c->lda_out, 1, Xin, cols, 1, ws.Out, cols, S9, (int)cols, c->in_last,
                                            0, c->bbig, nc2), s),
               "jets");
        j.Pre = ws.Out;
        j.ldp = cols;
        j.D = ws.Seed;
        j.ldd = cols;
        RS_HIP(launch_jet(f32, 3, j, s), "element seeds");
        // output map: dW_big += Seed X_L^T, db_big += value-column sums, G = W_big^T Seed
        RS_HIP(launch_gemm_s(f32, 1, gemm_s(ws.Seed, cols, 1, Xin, 1, cols, c->dWbig, c->in_last, S9, c->in_last,
                                            (int)cols, 1), s),
               "jets");
        RS_HIP(launch_value_rowsum(f32, ws.Seed, cols, S9, items, nc2, c->dbbig, s), "jets");
        int gi = 0;
        RS_HIP(launch_gemm_s(f32, 0, gemm_s(c->Wbig, 1, c->lda_out, ws.Seed, cols, 1, ws.G[gi], cols, c->in_last, (int)cols,
                                            S9), s),
               "jets");
        // hidden layers, last to first, activations recomputed from the kept pre-activations
        for (int l = L - 1; l >= 0; --l) {
            const int in = l == 0 ? r : w, lda = l == 0 ? c->lda0 : c->lda_h;
            j.G = ws.G[gi];
            j.ldg = cols;
            j.Pre = ws.Pre[l];
            j.ldp = cols;
            j.D = ws.D;
            j.ldd = cols;
            RS_HIP(launch_jet(f32, 2, j, s), "jets");
            const void* Xl = ws.X0;
            if (l > 0) {
                j.Pre = ws.Pre[l - 1];
                j.X = ws.X;
                RS_HIP(launch_jet(f32, 1, j, s), "jets");
                Xl = ws.X;
            }
            RS_HIP(launch_gemm_s(f32, 1, gemm_s(ws.D, cols, 1, Xl, 1, cols, grad + c->offW[l], in, w, in, (int)cols, 1), s),
                   "jets");
            RS_HIP(launch_value_rowsum(f32, ws.D, cols, w, items, nc2, grad + c->offb[l], s), "jets");
            if (l > 0) {
                RS_HIP(launch_gemm_s(f32, 0, gemm_s(c->W[l], 1, lda, ws.D, cols, 1, ws.G[gi ^ 1], cols, in, (int)cols, w), s),
                       "jets");
                gi ^= 1;
            }
        }
    }
    return run(c, K_LIP_GRAD, Work{}, s, [&] {
        return launch_unfold(c->dWbig, c->dbbig, c->in_last, c->fold_ptr, c->fold_row, c->fold_coef, c->n_out,
                             grad + c->offW[L], grad + c->offb[L], s);
    });
}

extern "C" int rs_lipschitz_param_grad(rs_ctx* c, int32_t B, const double* z1, const double* z2, double* loss,
                                       double* grad, void* stream)
{
    if (!c) return RS_ERR_STATE;
    RS_TRY(lip_grad_check(c, B, z1, z2, loss, grad));
    LipWs ws;
    RS_TRY(lip_ws(c, ws));
    return lip_param_grad(c, B, z1, z2, loss, grad, ws, static_cast<hipStream_t>(stream));
}

extern "C" int rs_lipschitz_param_grad_noalloc(rs_ctx* c, int32_t B, const double* z1, const double* z2,
                                               double* loss, double* grad, void* stream)
{
    if (!c) return RS_ERR_STATE;
    RS_TRY(lip_grad_check(c, B, z1, z2, loss, grad));
    if (!c->scratch) return fail(c, RS_ERR_STATE, "the static scratch array of this device is not set up");
    // as many pairs per pass as the static array holds, at most the allocating variant's
    LipWs ws;
    int pairs = lip_pairs_cap(c);
    while (pairs > 0 && lip_ws_layout(c, pairs, nullptr, ws) > kStaticScratchBytes) --pairs;
    if (pairs == 0) {
        char msg[160];
        std::snprintf(msg, sizeof msg, "one pair needs %zu bytes of scratch, more than the static %zu",
                      lip_ws_layout(c, 1, nullptr, ws), kStaticScratchBytes);
        return fail(c, RS_ERR_UNSUPPORTED, msg);
    }
    lip_ws_layout(c, pairs, static_cast<char*>(c->scratch), ws);
    return lip_param_grad(c, B, z1, z2, loss, grad, ws, static_cast<hipStream_t>(stream));
}

// ------------------------------------------------------------------ full-space solver
extern "C" int rs_default_full_opts(rs_full_opts* o)
{
    if (!o) return RS_ERR_ARG;
    o->max_iter = 100;
    o->ls_max = 128;
    o->cg_max = 4000;
    o->c1 = 1e-4;
    o->shrink = 0.5;
    o->rel_tol = 1e-6;
    o->abs_tol = 0.0;
    o->eta_min = 1e-4;
    o->eta_max = 0.1;
    return RS_OK;
}

extern "C" int rs_full_solve(rs_ctx* c, int32_t B, double* u, const rs_load* load, const rs_full_opts* o,
                             int32_t* iters, int32_t* status, double* relgrad, double* E, void* stream)
{
    if (!c) return RS_ERR_STATE;
    if (B < 0) return fail(c, RS_ERR_ARG, "B < 0");
    if (B > 0 && !u) return fail(c, RS_ERR_ARG, "u is NULL");
    if (!o) return fail(c, RS_ERR_ARG, "opts is NULL");
    if (o->max_iter < 0 || o->ls_max < 1 || o->cg_max < 1 || !(o->shrink > 0.0 && o->shrink < 1.0) ||
        !(o->c1 > 0.0 && o->c1 < 1.0) || !(o->eta_min > 0.0) || !(o->eta_max >= o->eta_min) || o->rel_tol < 0.0 ||
        o->abs_tol < 0.0)
        return fail(c, RS_ERR_ARG, "bad full-space solver options");
    if (B == 0) return RS_OK;
    const char* why = "";
    if (!c->full) {
        FullSolverDesc d{};
        d.nv = c->nv;
        d.ne = c->ne;
        d.nt = c->nt;
        d.nf = c->nf;
        d.X = c->X.data();
        d.tets = c->tets.data();
        d.pinned = c->pinned.data();
        d.mass = c->mass.data();
        d.tvtx = c->tvtx.data();
        d.fvtx = c->fvtx.data();
        d.mu = c->mu;
        d.lam = c->lam;
        d.kc = c->k_c;
        for (int i = 0; i < 3; ++i) d.grav[i] = c->grav[i];
        const int rc = full_solver_create(d, &c->full, &why);
        if (rc != RS_OK) return fail(c, rc, why);
    }
    FullSolveCall call{};
    call.B = B;
    call.u = u;
    call.targets = load ? load->targets : nullptr;
    call.force = load ? load->force : nullptr;
    call.max_iter = o->max_iter;
    call.ls_max = o->ls_max;
    call.cg_max = o->cg_max;
    call.c1 = o->c1;
    call.shrink = o->shrink;
    call.rel_tol = o->rel_tol;
    call.abs_tol = o->abs_tol;
    call.eta_min = o->eta_min;
    call.eta_max = o->eta_max;
    call.iters = iters;
    call.status = status;
    call.relgrad = relgrad;
    call.E = E;
    if (call.targets && c->nt == 0) call.targets = nullptr;
    if (call.force && c->nf == 0) call.force = nullptr;
    const int rc = full_solve(c->full, call, static_cast<hipStream_t>(stream), &why);
    return rc == RS_OK ? RS_OK : fail(c, rc, std::string("full-space solve: ") + why);
}

// ------------------------------------------------------------------ supervised training
// The autoencoder of the supervised construction (Sec. 3.2, Eq.
// form-vanilla-supervised-construction): an ELU encoder n -> r and the
// context's decoder, trained on snapshot displacements with the
// reconstruction loss in the mass norm, plus lambda times the Lipschitz loss
// of the decoder over pairs of the batch's encodings (Sec. 4.2, Eq.
// form-unconstrained-lipschitz-optimization).  Activations are (units x batch)
// blocks; every product runs on the strided matrix-core GEMM.
struct rs_trainer {
    rs_ctx* c = nullptr;
    int f32 = 1;
    size_t ts = 4;
    int n = 0, r = 0;                 // decoder output rows (encoder input), latent size
    int Le = 0, we = 0;               // encoder hidden layers and width
    int L = 0, w = 0, in_last = 0;    // decoder hidden layers, width, input of its output layer
    int max_batch = 0;
    std::vector<size_t> eW, eb;       // packed offsets of the encoder layers
    size_t n_enc = 0, n_dec = 0;
    void* enc = nullptr;              // parameters, context precision
    void* dec = nullptr;
    void* genc = nullptr;             // gradients of the reconstruction loss
    void* gdec = nullptr;
    double* glip = nullptr;           // gradient of the Lipschitz loss (float64)
    double lambda = 0.0;              // lambda of the last gradient call (0: glip unused)
    void *m_enc = nullptr, *v_enc = nullptr, *m_dec = nullptr, *v_dec = nullptr;
    int step = 0;
    void* Dt = nullptr;               // n x Bm batch displacements
    void* Pe[kMaxL + 1] = {};         // encoder pre-activations (last: the encodings, r x Bm)
    void* Xe[kMaxL + 1] = {};         // encoder activations (Xe[0] unused: Dt)
    void* Pd[kMaxL] = {};             // decoder pre-activations
    void* Hd[kMaxL + 1] = {};         // decoder activations (Hd[0] aliases the encodings)
    void* U = nullptr;                // n x Bm decoder output
    void* Ubar = nullptr;             // its adjoint
    void* G[2] = {};                  // adjoints of layer outputs, max(we, w, r) x Bm
    void* D = nullptr;                // adjoints of pre-activations
    void* part = nullptr;             // split-K partial sums
    size_t part_elems = 0;
    double* rpart = nullptr;          // residual partial sums
    double* zs = nullptr;             // Bm x r encodings (float64)
    double* z1 = nullptr;
    double* z2 = nullptr;
    double* losses = nullptr;         // [L_C, L_LS] of the last gradient call
    std::vector<void*> bufs;
};

static void* tr_alloc(rs_trainer* t, size_t bytes)
{
    void* p = nullptr;
    if (hipMalloc(&p, bytes ? bytes : 1) != hipSuccess) return nullptr;
    t->bufs.push_back(p);
    return p;
}

static void tr_free(rs_trainer* t)
{
    for (void* p : t->bufs) (void)hipFree(p);
    delete t;
}

static inline void* at_off(void* base, size_t off, size_t ts) { return static_cast<char*>(base) + off * ts; }

// C (M x N, row-major, ldc) (+)= A B (+ bias), with a K split when few tiles meet a long reduction
static int tr_gemm(rs_trainer* t, const void* A, long sAm, long sAk, const void* B, long sBk, long sBn, void* C,
                   long ldc, int M, int N, int K, int accumulate, const void* bias, hipStream_t s)
{
    rs_ctx* c = t->c;
    SgemmArgs g{};
    g.A = A; g.sAm = sAm; g.sAk = sAk;
    g.B = B; g.sBk = sBk; g.sBn = sBn;
    g.C = C; g.ldc = ldc;
    g.M = M; g.N = N; g.K = K;
    g.alpha = 1.0;
    g.accumulate = accumulate;
    g.bias = bias;
    g.bias_every = bias ? 1 : 0;
    const long tiles = (long)((M + 63) / 64) * ((N + 63) / 64);
    int ks = 1;
    if (tiles < 512 && K >= 2048) ks = (int)std::min<long>({32L, (long)K / 512, std::max(1L, 1024 / tiles)});
    while (ks > 1 && (size_t)ks * M * N > t->part_elems) --ks;
    g.ksplit = ks;
    g.part = t->part;
    return run(c, K_TRAIN, Work{}, s, [&] { return launch_gemm_s(t->f32, 0, g, s); });
}

static int tr_op(rs_trainer* t, const TrainOp& o, hipStream_t s)
{
    return run(t->c, K_TRAIN, Work{}, s, [&] { return launch_train(t->f32, o, s); });
}

static TrainOp op_of(int kind)
{
    TrainOp o;
    o.op = kind;
    return o;
}

extern "C" int rs_trainer_create(rs_ctx* c, const rs_mlp* enc, const rs_decoder* dec, int32_t max_batch,
                                 rs_trainer** out)
{
    if (!out) return RS_ERR_ARG;
    *out = nullptr;
    if (!c) return RS_ERR_STATE;
    if (c->bf16) return fail(c, RS_ERR_UNSUPPORTED, "training needs a float32 or float64 context");
    if (c->L < 1) return fail(c, RS_ERR_UNSUPPORTED, "training needs a decoder with hidden layers");
    if (!enc || !enc->W || !enc->b) return fail(c, RS_ERR_ARG, "encoder is NULL");
    if (enc->n_in != c->n_out || enc->n_out != c->r)
        return fail(c, RS_ERR_ARG, "encoder must map 3 nv displacements to the decoder's r latent coordinates");
    if (enc->n_hidden < 0 || enc->n_hidden > kMaxL || (enc->n_hidden > 0 && (enc->width < 1 || enc->width > 4096)))
        return fail(c, RS_ERR_UNSUPPORTED, "encoder depth or width out of range");
    if (max_batch < 2) return fail(c, RS_ERR_ARG, "max_batch must be >= 2");
    RS_TRY(check_decoder(c, dec, c->nv));
    if (dec->r != c->r || dec->n_hidden != c->L || dec->width != c->w)
        return fail(c, RS_ERR_ARG, "decoder shape differs from the context's");
    rs_trainer* t = new (std::nothrow) rs_trainer();
    if (!t) return fail(c, RS_ERR_OOM, "host allocation failed");
    t->c = c;
    t->f32 = c->f32;
    t->ts = c->tsz;
    t->n = c->n_out;
    t->r = c->r;
    t->Le = enc->n_hidden;
    t->we = enc->n_hidden > 0 ? enc->width : 0;
    t->L = c->L;
    t->w = c->w;
    t->in_last = c->in_last;
    t->max_batch = max_batch;
    // encoder packed offsets
    size_t off = 0;
    for (int l = 0; l <= t->Le; ++l) {
        const int in = l == 0 ? t->n : t->we, o = l == t->Le ? t->r : t->we;
        t->eW.push_back(off);
        off += (size_t)o * in;
        t->eb.push_back(off);
        off += o;
    }
    t->n_enc = off;
    t->n_dec = c->n_params;
    const size_t ts = t->ts, Bm = (size_t)max_batch;
    const size_t wide = (size_t)std::max({t->we, t->w, t->r});
    bool ok = true;
    auto A = [&](size_t bytes) {
        void* p = tr_alloc(t, bytes);
        ok = ok && p;
        return p;
    };
    t->enc = A(t->n_enc * ts);
    t->dec = A(t->n_dec * ts);
    t->genc = A(t->n_enc * ts);
    t->gdec = A(t->n_dec * ts);
    t->glip = static_cast<double*>(A(t->n_dec * sizeof(double)));
    t->m_enc = A(t->n_enc * ts);
    t->v_enc = A(t->n_enc * ts);
    t->m_dec = A(t->n_dec * ts);
    t->v_dec = A(t->n_dec * ts);
    t->Dt = A((size_t)t->n * Bm * ts);
    for (int l = 0; l <= t->Le; ++l) {
        const int o = l == t->Le ? t->r : t->we;
        t->Pe[l] = A((size_t)o * Bm * ts);
        if (l < t->Le) t->Xe[l + 1] = A((size_t)o * Bm * ts);
    }
    t->Hd[0] = t->Pe[t->Le];
    for (int l = 0; l < t->L; ++l) {
        t->Pd[l] = A((size_t)t->w * Bm * ts);
        t->Hd[l + 1] = A((size_t)t->w * Bm * ts);
    }
    t->U = A((size_t)t->n * Bm * ts);
    t->Ubar = A((size_t)t->n * Bm * ts);
    t->G[0] = A(wide * Bm * ts);
    t->G[1] = A(wide * Bm * ts);
    t->D = A(wide * Bm * ts);
    t->part_elems = 32 * wide * Bm;
    t->part = A(t->part_elems * ts);
    t->rpart = static_cast<double*>(A(((size_t)t->n * Bm + 255) / 256 * sizeof(double)));
    t->zs = static_cast<double*>(A(Bm * t->r * sizeof(double)));
    t->z1 = static_cast<double*>(A(Bm / 2 * t->r * sizeof(double) + 8));
    t->z2 = static_cast<double*>(A(Bm / 2 * t->r * sizeof(double) + 8));
    t->losses = static_cast<double*>(A(2 * sizeof(double)));
    if (!ok) {
        tr_free(t);
        return fail(c, RS_ERR_OOM, "trainer allocation failed");
    }
    // parameters: packed from the host arrays, converted to the context precision
    std::vector<double> pe(t->n_enc), pd(t->n_dec);
    for (int l = 0; l <= t->Le; ++l) {
        const int in = l == 0 ? t->n : t->we, o = l == t->Le ? t->r : t->we;
        if (!enc->W[l] || !enc->b[l]) {
            tr_free(t);
            return fail(c, RS_ERR_ARG, "encoder layer pointer is NULL");
        }
        std::copy(enc->W[l], enc->W[l] + (size_t)o * in, pe.begin() + t->eW[l]);
        std::copy(enc->b[l], enc->b[l] + o, pe.begin() + t->eb[l]);
    }
    for (int l = 0; l <= t->L; ++l) {
        const int in = l == 0 ? t->r : t->w, o = l == t->L ? t->n : t->w;
        std::copy(dec->W[l], dec->W[l] + (size_t)o * in, pd.begin() + c->offW[l]);
        std::copy(dec->b[l], dec->b[l] + o, pd.begin() + c->offb[l]);
    }
    int rc = upload(c, t->enc, pe, t->f32);
    if (rc == RS_OK) rc = upload(c, t->dec, pd, t->f32);
    const std::vector<double> zero_e(t->n_enc, 0.0), zero_d(t->n_dec, 0.0);
    if (rc == RS_OK) rc = upload(c, t->m_enc, zero_e, t->f32);
    if (rc == RS_OK) rc = upload(c, t->v_enc, zero_e, t->f32);
    if (rc == RS_OK) rc = upload(c, t->m_dec, zero_d, t->f32);
    if (rc == RS_OK) rc = upload(c, t->v_dec, zero_d, t->f32);
    // the context evaluates the trainer's decoder from here on
    if (rc == RS_OK) rc = rs_set_decoder_device(c, t->dec, !t->f32, nullptr);
    if (rc == RS_OK && hipDeviceSynchronize() != hipSuccess) rc = fail(c, RS_ERR_HIP, "hipDeviceSynchronize");
    if (rc != RS_OK) {
        tr_free(t);
        return rc;
    }
    *out = t;
    return RS_OK;
}

extern "C" int rs_trainer_destroy(rs_trainer* t)
{
    if (!t) return RS_OK;
    (void)hipDeviceSynchronize();
    tr_free(t);
    return RS_OK;
}

extern "C" int rs_trainer_param_count(const rs_trainer* t, int64_t* n_enc, int64_t* n_dec)
{
    if (!t) return RS_ERR_STATE;
    if (n_enc) *n_enc = (int64_t)t->n_enc;
    if (n_dec) *n_dec = (int64_t)t->n_dec;
    return RS_OK;
}

extern "C" int rs_trainer_params(rs_trainer* t, void* enc, void* dec, void* stream)
{
    if (!t) return RS_ERR_STATE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (enc && hipMemcpyAsync(enc, t->enc, t->n_enc * t->ts, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return fail(t->c, RS_ERR_HIP, "hipMemcpyAsync");
    if (dec && hipMemcpyAsync(dec, t->dec, t->n_dec * t->ts, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return fail(t->c, RS_ERR_HIP, "hipMemcpyAsync");
    return RS_OK;
}

// encoder forward of B <= max_batch items: Dt from the store, then every layer (Pe[Le] = encodings)
static int tr_encode(rs_trainer* t, int B, const void* store, const int32_t* idx, hipStream_t s)
{
    TrainOp o = op_of(TRAIN_GATHER);
    o.a = store;
    o.n = t->n;
    o.B = B;
    o.idx = idx;
    o.out = t->Dt;
    RS_TRY(tr_op(t, o, s));
    const void* X = t->Dt;
    for (int l = 0; l <= t->Le; ++l) {
        const int in = l == 0 ? t->n : t->we, out = l == t->Le ? t->r : t->we;
        RS_TRY(tr_gemm(t, at_off(t->enc, t->eW[l], t->ts), in, 1, X, B, 1, t->Pe[l], B, out, B, in, 0,
                       at_off(t->enc, t->eb[l], t->ts), s));
        if (l < t->Le) {
            TrainOp e = op_of(TRAIN_ELU_FWD);
            e.a = t->Pe[l];
            e.out = t->Xe[l + 1];
            e.count = (long)out * B;
            RS_TRY(tr_op(t, e, s));
            X = t->Xe[l + 1];
        }
    }
    return RS_OK;
}

extern "C" int rs_trainer_encode(rs_trainer* t, int32_t B, const void* store, const int32_t* idx, double* z,
                                 void* stream)
{
    if (!t) return RS_ERR_STATE;
    rs_ctx* c = t->c;
    if (B < 0) return fail(c, RS_ERR_ARG, "B < 0");
    if (B > 0 && (!store || !z)) return fail(c, RS_ERR_ARG, "NULL pointer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int b0 = 0; b0 < B; b0 += t->max_batch) {
        const int nb = std::min(t->max_batch, B - b0);
        const void* st = idx ? store : static_cast<const char*>(store) + (size_t)b0 * t->n * t->ts;
        RS_TRY(tr_encode(t, nb, st, idx ? idx + b0 : nullptr, s));
        TrainOp o = op_of(TRAIN_TO_ITEMS);
        o.a = t->Pe[t->Le];
        o.n = t->r;
        o.B = nb;
        o.z = z + (size_t)b0 * t->r;
        RS_TRY(tr_op(t, o, s));
    }
    return RS_OK;
}

extern "C" int rs_trainer_grad(rs_trainer* t, int32_t B, const void* store, const int32_t* idx, double lambda_ls,
                               int32_t n_pairs, double* losses, double* grad_enc, double* grad_dec, void* stream)
{
    if (!t) return RS_ERR_STATE;
    rs_ctx* c = t->c;
    if (B < 1 || B > t->max_batch) return fail(c, RS_ERR_ARG, "B must be in [1, max_batch]");
    if (!store) return fail(c, RS_ERR_ARG, "store is NULL");
    if (lambda_ls < 0.0 || !std::isfinite(lambda_ls)) return fail(c, RS_ERR_ARG, "lambda_ls must be finite and >= 0");
    if (lambda_ls > 0.0 && (n_pairs < 1 || 2 * n_pairs > B))
        return fail(c, RS_ERR_ARG, "n_pairs must be in [1, B/2] when lambda_ls > 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t ts = t->ts;
    const int n = t->n, L = t->L, w = t->w, in_last = t->in_last;
    RS_TRY(tr_encode(t, B, store, idx, s));
    // decoder forward
    for (int l = 0; l < L; ++l) {
        const int in = l == 0 ? t->r : w;
        RS_TRY(tr_gemm(t, at_off(t->dec, c->offW[l], ts), in, 1, t->Hd[l], B, 1, t->Pd[l], B, w, B, in, 0,
                       at_off(t->dec, c->offb[l], ts), s));
        TrainOp e = op_of(TRAIN_ELU_FWD);
        e.a = t->Pd[l];
        e.out = t->Hd[l + 1];
        e.count = (long)w * B;
        RS_TRY(tr_op(t, e, s));
    }
    RS_TRY(tr_gemm(t, at_off(t->dec, c->offW[L], ts), in_last, 1, t->Hd[L], B, 1, t->U, B, n, B, in_last, 0,
                   at_off(t->dec, c->offb[L], ts), s));
    {
        TrainOp o = op_of(TRAIN_RESIDUAL);
        o.a = t->U;
        o.b = t->Dt;
        o.n = n;
        o.B = B;
        o.rowmass = c->row_mass;
        o.pinned_row = c->pinned_row;
        o.out = t->Ubar;
        o.part = t->rpart;
        o.loss = t->losses;
        RS_TRY(tr_op(t, o, s));
    }
    // decoder backward: output layer, then the hidden layers (adjoints ping-pong through G)
    RS_TRY(tr_gemm(t, t->Ubar, B, 1, t->Hd[L], 1, B, at_off(t->gdec, c->offW[L], ts), in_last, n, in_last, B, 0,
                   nullptr, s));
    {
        TrainOp o = op_of(TRAIN_ROWSUM);
        o.a = t->Ubar;
        o.n = n;
        o.B = B;
        o.out = at_off(t->gdec, c->offb[L], ts);
        RS_TRY(tr_op(t, o, s));
    }
    int gi = 0;
    RS_TRY(tr_gemm(t, at_off(t->dec, c->offW[L], ts), 1, in_last, t->Ubar, B, 1, t->G[gi], B, in_last, B, n, 0, nullptr,
                   s));
    for (int l = L - 1; l >= 0; --l) {
        const int in = l == 0 ? t->r : w;
        TrainOp e = op_of(TRAIN_ELU_BWD);
        e.a = t->G[gi];
        e.b = t->Pd[l];
        e.out = t->D;
        e.count = (long)w * B;
        RS_TRY(tr_op(t, e, s));
        RS_TRY(tr_gemm(t, t->D, B, 1, t->Hd[l], 1, B, at_off(t->gdec, c->offW[l], ts), in, w, in, B, 0, nullptr, s));
        TrainOp o = op_of(TRAIN_ROWSUM);
        o.a = t->D;
        o.n = w;
        o.B = B;
        o.out = at_off(t->gdec, c->offb[l], ts);
        RS_TRY(tr_op(t, o, s));
        RS_TRY(tr_gemm(t, at_off(t->dec, c->offW[l], ts), 1, in, t->D, B, 1, t->G[gi ^ 1], B, in, B, w, 0, nullptr, s));
        gi ^= 1;
    }
    // encoder backward: G[gi] is the adjoint of the encodings (its last layer is linear)
    for (int l = t->Le; l >= 0; --l) {
        const int in = l == 0 ? n : t->we, out = l == t->Le ? t->r : t->we;
        const void* Dl = t->G[gi];
        if (l < t->Le) {
            TrainOp e = op_of(TRAIN_ELU_BWD);
            e.a = t->G[gi];
            e.b = t->Pe[l];
            e.out = t->D;
            e.count = (long)out * B;
            RS_TRY(tr_op(t, e, s));
            Dl = t->D;
        }
        const void* Xin = l == 0 ? t->Dt : t->Xe[l];
        RS_TRY(tr_gemm(t, Dl, B, 1, Xin, 1, B, at_off(t->genc, t->eW[l], ts), in, out, in, B, 0, nullptr, s));
        TrainOp o = op_of(TRAIN_ROWSUM);
        o.a = Dl;
        o.n = out;
        o.B = B;
        o.out = at_off(t->genc, t->eb[l], ts);
        RS_TRY(tr_op(t, o, s));
        if (l > 0) {
            RS_TRY(tr_gemm(t, at_off(t->enc, t->eW[l], ts), 1, in, Dl, B, 1, t->G[gi ^ 1], B, in, B, out, 0, nullptr,
                           s));
            gi ^= 1;
        }
    }
    // the Lipschitz term over pairs of this batch's encodings (held fixed), on the context's decoder
    t->lambda = lambda_ls;
    if (lambda_ls > 0.0) {
        TrainOp o = op_of(TRAIN_TO_ITEMS);
        o.a = t->Pe[t->Le];
        o.n = t->r;
        o.B = B;
        o.z = t->zs;
        RS_TRY(tr_op(t, o, s));
        RS_HIP(launch_split_pairs(t->zs, n_pairs, t->r, t->z1, t->z2, s), "training pairs");
        RS_TRY(rs_lipschitz_param_grad(c, n_pairs, t->z1, t->z2, t->losses + 1, t->glip, s));
    } else {
        RS_HIP(launch_fill_zero(t->losses + 1, 1, s), "fill");
    }
    if (losses && hipMemcpyAsync(losses, t->losses, 2 * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return fail(c, RS_ERR_HIP, "hipMemcpyAsync");
    if (grad_enc) {
        TrainOp o = op_of(TRAIN_GRAD_OUT);
        o.a = t->genc;
        o.count = (long)t->n_enc;
        o.z = grad_enc;
        RS_TRY(tr_op(t, o, s));
    }
    if (grad_dec) {
        TrainOp o = op_of(TRAIN_GRAD_OUT);
        o.a = t->gdec;
        o.g2 = lambda_ls > 0.0 ? t->glip : nullptr;
        o.scale = lambda_ls;
        o.count = (long)t->n_dec;
        o.z = grad_dec;
        RS_TRY(tr_op(t, o, s));
    }
    return RS_OK;
}

extern "C" int rs_trainer_adam(rs_trainer* t, double lr, double beta1, double beta2, double eps, void* stream)
{
    if (!t) return RS_ERR_STATE;
    rs_ctx* c = t->c;
    if (!(lr >= 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0))
        return fail(c, RS_ERR_ARG, "bad Adam constants");
    hipStream_t s = static_cast<hipStream_t>(stream);
    ++t->step;
    TrainOp o = op_of(TRAIN_ADAM);
    o.lr = lr;
    o.b1 = beta1;
    o.b2 = beta2;
    o.eps = eps;
    o.step = t->step;
    o.out = t->enc;
    o.a = t->genc;
    o.m = t->m_enc;
    o.v = t->v_enc;
    o.count = (long)t->n_enc;
    RS_TRY(tr_op(t, o, s));
    o.out = t->dec;
    o.a = t->gdec;
    o.g2 = t->lambda > 0.0 ? t->glip : nullptr;
    o.scale = t->lambda;
    o.m = t->m_dec;
    o.v = t->v_dec;
    o.count = (long)t->n_dec;
    RS_TRY(tr_op(t, o, s));
    return rs_set_decoder_device(c, t->dec, !t->f32, stream);
}

// ------------------------------------------------------------------ PCA subspace
// C (M x N) = A B, float64, split over K when few tiles meet a long reduction
static int gemm64(rs_ctx* c, const double* A, long sAm, long sAk, const double* B, long sBk, long sBn, double* C,
                  long ldc, int M, int N, int K, double* part, size_t part_elems, hipStream_t s, double alpha = 1.0)
{
    SgemmArgs g{};
    g.A = A; g.sAm = sAm; g.sAk = sAk;
    g.B = B; g.sBk = sBk; g.sBn = sBn;
    g.C = C; g.ldc = ldc;
    g.M = M; g.N = N; g.K = K;
    g.alpha = alpha;
    const long tiles = (long)((M + 63) / 64) * ((N + 63) / 64);
    int ks = 1;
    if (tiles < 512 && K >= 2048) ks = (int)std::min<long>({32L, (long)K / 512, std::max(1L, 1024 / tiles)});
    while (ks > 1 && (size_t)ks * M * N > part_elems) --ks;
    g.ksplit = ks;
    g.part = part;
    return run(c, K_TRAIN, Work{}, s, [&] { return launch_gemm_s(0, 0, g, s); });
}

extern "C" int rs_pca(rs_ctx* c, int32_t N, const void* store, int32_t r, int32_t iters, double* W, double* mean,
                      double* evals, double* z_rest, void* stream)
{
    if (!c) return RS_ERR_STATE;
    if (N < 1 || !store || !W || !mean) return fail(c, RS_ERR_ARG, "N < 1 or NULL pointer");
    if (r < 1 || r > N || r > 56) return fail(c, RS_ERR_ARG, "r must be in [1, min(N, 56)]");
    if (iters < 1) return fail(c, RS_ERR_ARG, "iters must be >= 1");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int n = c->n_out, k = std::min(N, r + 8);
    std::vector<void*> tmp;
    bool ok = true;
    auto A = [&](size_t count) {
        void* p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(double)) != hipSuccess) {
            ok = false;
            return (double*)nullptr;
        }
        tmp.push_back(p);
        return (double*)p;
    };
    auto release = [&]() {
        (void)hipStreamSynchronize(s);
        for (void* p : tmp) (void)hipFree(p);
    };
    const size_t part_elems = (size_t)32 * std::max(N, k) * k;
    double* Dc = A((size_t)N * n);
    double* X = A((size_t)n * k);
    double* X2 = A((size_t)n * k);
    double* MX = A((size_t)n * k);
    double* Y = A((size_t)N * k);
    double* G = A((size_t)k * k);
    double* R = A((size_t)k * k);
    double* V = A((size_t)k * r);
    double* ev = A(r);
    double* part = A(part_elems);
    int* bad = (int*)A(1);
    if (!ok) {
        release();
        return fail(c, RS_ERR_OOM, "PCA workspace allocation failed");
    }
    int rc = RS_OK;
    auto hip = [&](hipError_t e) {
        if (e != hipSuccess && rc == RS_OK) rc = hip_fail(c, e, "PCA");
        return rc == RS_OK;
    };
    auto orth = [&](double* Xin, double* Xout) {
        // Xout = Xin R with R = L^-T, G = Xin^T M Xin = L L^T
        return hip(launch_pca_mass(Xin, c->row_mass, n, k, MX, s)) &&
               gemm64(c, Xin, 1, k, MX, k, 1, G, k, k, k, n, part, part_elems, s) == RS_OK &&
               hip(launch_pca_orth(G, k, R, bad, s)) &&
               gemm64(c, Xin, k, 1, R, k, 1, Xout, k, n, k, k, part, part_elems, s) == RS_OK;
    };
    auto power = [&](double* Xin, double* Xout) {
        // Xout = Dc^T Dc M Xin (Y = Dc M Xin kept)
        return hip(launch_pca_mass(Xin, c->row_mass, n, k, MX, s)) &&
               gemm64(c, Dc, n, 1, MX, k, 1, Y, k, N, k, n, part, part_elems, s) == RS_OK &&
               (Xout == nullptr || gemm64(c, Dc, 1, n, Y, k, 1, Xout, k, n, k, N, part, part_elems, s) == RS_OK);
    };
    bool go = hip(launch_pca_center(c->f32, store, N, n, mean, Dc, s)) && hip(launch_pca_start(X2, (long)n * k, s)) &&
              orth(X2, X);
    for (int it = 0; go && it < iters; ++it) go = power(X, X2) && orth(X2, X);
    // Rayleigh-Ritz: T = Y^T Y with Y = Dc M X, its top r eigenvectors V, W = X V
    go = go && power(X, nullptr) && gemm64(c, Y, 1, k, Y, k, 1, G, k, k, k, N, part, part_elems, s) == RS_OK &&
         hip(launch_pca_ritz(G, k, r, V, ev, s)) &&
         gemm64(c, X, k, 1, V, r, 1, W, r, n, r, k, part, part_elems, s) == RS_OK;
    if (go && evals) go = hip(hipMemcpyAsync(evals, ev, r * sizeof(double), hipMemcpyDeviceToDevice, s));
    // coordinates of the rest shape's projection: -W^T M mean
    if (go && z_rest)
        go = hip(launch_pca_mass(mean, c->row_mass, n, 1, MX, s)) &&
             gemm64(c, W, 1, r, MX, 1, 1, z_rest, 1, r, 1, n, part, part_elems, s, -1.0) == RS_OK;
    int hbad = 0;
    if (go) go = hip(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    release();
    if (rc != RS_OK) return rc;
    if (!go) return fail(c, RS_ERR_HIP, "PCA failed");
    if (hbad) return fail(c, RS_ERR_ARG, "the snapshots span fewer than r + 8 directions (rank-deficient Gram matrix)");
    return RS_OK;
}

// ------------------------------------------------------------------ profiling
extern "C" int rs_profile(rs_ctx* c, int32_t enable, uint32_t kind_mask)
{
    if (!c) return RS_ERR_STATE;
    if (enable) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(c, e, "hipDeviceSynchronize");
        c->recs.clear();
        c->evnext = 0;
        c->plog_next = 0;
        for (int k = 0; k < K_COUNT; ++k) {
            c->kms[k] = c->kbytes[k] = c->kflops[k] = 0.0;
            c->klaunch[k] = 0;
        }
        c->aggregated = true;
    }
    c->prof = enable != 0;
    c->prof_mask = kind_mask;
    return RS_OK;
}

extern "C" int rs_profile_get(rs_ctx* c, int32_t idx, int32_t* n_kinds, char* name, int32_t name_len,
                              int32_t* launches, double* total_ms, double* bytes, double* flops)
{
    if (!c) return RS_ERR_STATE;
    if (!c->aggregated) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(c, e, "hipDeviceSynchronize");
        std::vector<int> log((size_t)c->plog_next * 4);
        if (c->plog_next) {
            e = hipMemcpy(log.data(), c->plog, log.size() * sizeof(int), hipMemcpyDeviceToHost);
            if (e != hipSuccess) return hip_fail(c, e, "hipMemcpy");
        }
        for (const ProfRec& rec : c->recs) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, c->evpool[rec.e0], c->evpool[rec.e1]);
            if (e != hipSuccess) return hip_fail(c, e, "hipEventElapsedTime");
            const double n = rec.slot >= 0 ? (double)log[4 * (size_t)rec.slot + rec.which] : 0.0;
            c->kms[rec.kind] += ms;
            c->kbytes[rec.kind] += rec.b0 + rec.b1 * n;
            c->kflops[rec.kind] += rec.f0 + rec.f1 * n;
            c->klaunch[rec.kind] += 1;
        }
        c->recs.clear();
        c->evnext = 0;
        c->plog_next = 0;
        c->aggregated = true;
    }
    if (n_kinds) *n_kinds = K_COUNT;
    if (idx < 0 || idx >= K_COUNT) return RS_OK;
    if (name && name_len > 0) {
        std::strncpy(name, kKindName[idx], (size_t)name_len - 1);
        name[name_len - 1] = 0;
    }
    if (launches) *launches = c->klaunch[idx];
    if (total_ms) *total_ms = c->kms[idx];
    if (bytes) *bytes = c->kbytes[idx];
    if (flops) *flops = c->kflops[idx];
    return RS_OK;
}
