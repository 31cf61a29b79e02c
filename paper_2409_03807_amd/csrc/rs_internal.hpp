// Internal declarations shared by the host code (rs_api.cpp) and the kernels
// (rs_kernels.hip).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "rs.h"

#include <cstddef>
#include <cstdint>

namespace rs {

constexpr int kTileM = 64;   // GEMM rows per workgroup
constexpr int kTileN = 64;   // GEMM columns per workgroup
constexpr int kTileK = 32;   // GEMM reduction chunk (also the padding of every lda)
constexpr int kMaxR = 32;    // largest latent dimension
constexpr int kLsCand = 8;   // step lengths evaluated per line-search round after the first
constexpr int kMaxL = 8;     // largest number of hidden layers
constexpr int kMaxSplit = 16;// largest split of the adjoint GEMM's reduction
constexpr int kMaxWidth = 256;// widest hidden layer
// size of the static device scratch array of the allocation-free entry points
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;

// Device address of the current device's static scratch array (kStaticScratchBytes),
// looked up once per device with hipGetSymbolAddress and cached.
hipError_t static_scratch_address(void** ptr);

// IN_RAW: item-major (y_rows x nc) blocks; IN_RAW_T: item-major (nc x y_rows)
// blocks (k contiguous, the layout of a layer activation); IN_ELU: IN_RAW
// pre-activations activated on load; IN_LATENT: [z | I] built from z.
enum InMode { IN_RAW = 0, IN_ELU = 1, IN_LATENT = 2, IN_RAW_T = 3 };
enum OutMode { OUT_PACK = 0, OUT_SPLIT = 1 };
// kernel symbols per GEMM role (so profilers tell them apart)
enum GemmRole { ROLE_HIDDEN = 0, ROLE_OUT = 1, ROLE_ADJ = 2, ROLE_DECODE = 3 };

// C[item] (rows x nc) = A (rows x K) * Y[item] (K x nc) (+ bias on column 0)
// for `items` items stored item-major.  The column index n = item*nc + c runs
// over all items, so any nc works with the same 64-column tiles.
struct GemmArgs {
    const void* A;        // rows_pad x lda, row-major, zero padded (context precision)
    int lda;              // >= K, multiple of kTileK
    int rows;             // valid output rows
    int rows_pad;         // multiple of kTileM
    int K;                // reduction length
    int nc;               // columns per item
    int items;            // grid capacity in items
    const int* count;     // if non-NULL: the actual item count (<= items), read on the device
    int in_mode;          // InMode
    const void* Y;        // IN_RAW / IN_ELU: item-major (y_rows x nc) blocks
    int y_rows;           // rows of one Y block (padded)
    const double* z;      // IN_LATENT: (.. x r) latent points (always float64)
    const int* zmap;      // IN_LATENT: item -> row of z (NULL = identity)
    int r;
    const void* bias;     // rows, added to column 0 (NULL = none)
    int out_mode;         // OutMode
    void* C;              // OUT_PACK: item-major (rows_pad x nc)
    int ksplit;           // >1: blockIdx.z takes one K slice and writes C + z * split_stride
    size_t split_stride;  // elements between the partial outputs of two K slices
    void* Xo;             // OUT_SPLIT: column 0 -> Xo[item*rows + m] = Xrest[m] + value
    void* Jo;             // OUT_SPLIT: column c>0 -> Jo[(item*rows + m)*r + c-1]
    const void* Xrest;
};

// All hidden layers of the decoder for blocks of whole items: value and (nc > 1)
// forward-mode Jacobian, [a | A] pre-activations per layer and the final
// activation [h | J] = [ELU(a) | ELU'(a) A] of the last layer.
struct MlpArgs {
    const void* W[kMaxL];   // wrows x lda (lda0 for layer 0), zero padded
    const void* b[kMaxL];   // wrows
    void* pre[kMaxL];       // item-major (nc x wrows) pre-activations per layer (NULL = not kept)
    void* act;              // item-major (nc x wrows) activation of the last layer (k contiguous)
    int L, w, wrows, r, nc, lda0, lda;
    int items;              // grid capacity in items
    const int* count;       // actual item count (NULL = items)
    const double* z;        // latent points (float64)
    const int* zmap;        // item -> row of z (NULL = identity)
};

// Per-item cubature elastic, penalty, gravity and force terms from the rows of
// the reduced output map (energy, gradient, Gauss-Newton Hessian, adjoint seeds).
struct ElemArgs {
    const void* out;      // item-major (rows_pad x nc) [value | Jacobian] rows
    int rows_pad, nc, r;
    int S, nt, nf;        // cubature tets, targeted vertices, force vertices
    const int* count;     // actual item count (NULL = grid size)
    const double* wV;     // S: cubature weight times rest volume
    const double* Xt;     // nt x 3 rest positions of targeted vertices
    const double* targets;// (B x nt x 3) or NULL
    const double* force;  // (B x 3) or NULL
    const int* imap;      // item -> batch index for targets/force (NULL = identity)
    double mu, lam, k_c;
    int elastic_only;
    int grav_row, force_row; // first row of the gravity / force rows
    double* E;            // items (may be NULL)
    double* g;            // items x r (may be NULL)
    double* H;            // items x r x r (may be NULL)
    void* dseed;          // items x rows_pad adjoint seeds dE/d(row value) (may be NULL)
    int parts;            // workgroups per item (>= 1): each takes a run of the item's rounds
    int part_stride;      // parts > 1: g and H of part p of item i at slot p * part_stride + i (E must be NULL)
};

// Output map and element physics in one kernel (float32 and BF16 contexts,
// r == 16): the element part as ElemArgs (its `out` unused: no J_R is stored),
// plus the output map's operands.
struct FusedElemArgs {
    ElemArgs e;
    const void* A;      // W_big: float32 rows_pad x lda, or three BF16 planes (hi, mid, lo) of that
    int lda, K;         // K: a multiple of 32 (columns of W_big past the width are zero)
    int rows;           // rows of W_big (9 per tet, 3 per target, gravity, 3 force)
    const float* bias;  // rows: the value column's bias
    const float* Y;     // activations: unit k of column c (0 value, 1 + j Jacobian) of item i at
    int y_rows;         //   (i * nc + c) * y_rows + k; rows past the width are zero
    int cap;            // items of the launch (the grid's item groups)
};

// Per-element constants of the optional element treatments (kElemConst
// doubles per cubature tet): B = N^(1/2) (3x3, N the Gram matrix of the shape
// gradients), B^-1, the shape gradients Dv (4x3), the rest volume and the
// cubature weight.
constexpr int kElemConst = 32;
struct ElemOptArgs {
    const void* out;      // item-major (rows_pad x nc) [value | Jacobian] rows (context precision)
    int rows_pad, nc, r, S;
    const int* count;     // actual item count (NULL = grid size)
    const double* ec;     // S x kElemConst
    double mu, lam;
    double* H;            // items x r x r: the projection's correction is added
    double* He;           // items x S x 144 element Hessians (dump)
};

struct EnergyArgs {
    const void* out;      // item-major (rows_pad x 1) values
    int rows_pad;
    int S, nt, nf;
    const int* count;     // actual item count (NULL = grid size)
    const double* wV;
    const double* Xt;
    const double* targets;
    const double* force;
    const int* imap;      // item -> batch index for loads (NULL = identity)
    double mu, lam, k_c;
    int elastic_only;
    int grav_row, force_row;
    double* E;            // items
};

// Reverse pass through the hidden layers adding sum_l A_l^T diag(gbar_l s''(a_l)) A_l.
struct CurvArgs {
    const void* pre[kMaxL]; // item-major pre-activation blocks [a | A] per hidden layer (pre_rows * nc per item)
    int pre_su, pre_sc;     // element (unit u, column c) of a block at u * pre_su + c * pre_sc
    const void* W[kMaxL];   // hidden weights (width x in), in = r for layer 0
    const void* gbar;       // ksplit partials of items x pre_rows: dE/dh_L
    int ksplit;
    size_t split_stride;
    int L, width, nc, r;
    int pre_rows;           // padded rows of a pre-activation block
    int lda0, lda;          // leading dimensions of W[0] and of W[l>0]
    const int* count;       // actual item count (NULL = grid size)
    double* H;              // items x r x r, accumulated
    double* grev;           // items x r reverse-mode gradient (may be NULL)
    double* delta;          // items x L x width: dE/da_l of every layer (may be NULL)
    // parts > 1: H and g come as element-kernel partials (slot p * part_stride + i) that are summed
    // in part order into H (before the curvature term is added) and g
    int parts, part_stride;
    const double* Hp;
    const double* gp;
    double* g;
};

// Batched outer products for parameter gradients: out[m][n] (+)= sum over
// the B items of X_b[m] * Y_b[n] (float64 accumulation), and outb[m] (+)= sum
// of X_b[m].  X is T (x_f64 = 0) or float64; Y is T, T through ELU, or float64.
enum { PO_Y_RAW = 0, PO_Y_ELU = 1, PO_Y_F64 = 2 };
struct ParamOuterArgs {
    const void* X;
    int x_f64;
    size_t x_stride; // element m of item b at X[b * x_stride + m]
    const void* Y;
    int y_mode;
    size_t y_stride;
    int B, M, N;
    double* out;
    int ldo;
    double* outb; // may be NULL
    int accumulate;
    // item slices summed separately into part ([slice][M][N], then [slice][M]
    // for the bias sums) and added in slice order; part_cap values available
    double* part;
    size_t part_cap;
};
constexpr int kParamSlices = 8; // partial sums the workspace holds for the largest parameter product

// Per-item Newton state.  ls_j[b] < 0: the item needs its gradient and Hessian
// at z (evaluation phase); ls_j[b] >= 0: it is line-searching and the next
// trial step is shrink^ls_j[b].
struct NewtonState {
    double* z;        // B x r (caller)
    int* iters;       // B (caller)
    int* status;      // B (caller)
    double* relgrad;  // B (caller)
    double* E;        // B (caller) current float64 energy
    double* g0;       // B
    double* dz;       // B x r
    double* slope;    // B
    int* ls_j;        // B
    int* eval_list;   // items in the evaluation phase, in batch order
    int* search_list; // items line-searching, in batch order
    int* search_start;// first candidate of each searching item
    int* search_ncand;// candidates of each searching item
    int* cand_item;   // candidate -> item
    int* cand_j;      // candidate -> trial index
    int* counters;    // [0] n_eval [1] n_cand [2] n_search [3] n_running [4] n_admitted (items 0 .. n_admitted - 1)
                      // [5] lowest admitted item that may still run (every item below it has ended)
    const double* gw; // eval-list order: g (n_eval x r)
    const double* Hw; // eval-list order: H (n_eval x r x r)
    double* zc;       // candidates x r
    const double* Ec; // candidate energies
    int* plog;        // profiling only: this super-step's counters [0..2] are copied here (may be NULL)
};

struct NewtonParams {
    int r, max_iter, ls_max, proj;
    double c1, shrink, rel_tol, abs_tol, eig_floor;
    int hist;         // L-BFGS: pairs kept (<= RS_MAX_HISTORY)
    int window;       // items in flight: item b enters once fewer than `window` run (0: all at once)
};

// Per-item L-BFGS history: a ring of RS_MAX_HISTORY (s, y) pairs per item.
struct LbfgsState {
    double* S;        // B x RS_MAX_HISTORY x r
    double* Y;        // B x RS_MAX_HISTORY x r
    double* sy;       // B x RS_MAX_HISTORY: s.y of each pair
    int* npair;       // B: pairs held
    int* head;        // B: ring slot of the oldest pair
    double* zprev;    // B x r: z where the last direction was taken
    double* gprev;    // B x r: the gradient there
};

// Strided GEMM: C(m, n) (+)= alpha sum_k A(m, k) B(k, n) (+ bias[m] on columns
// n with n % bias_every == 0); A(m, k) = A[m sAm + k sAk], B(k, n) = B[k sBk + n sBn],
// C row-major (ldc), in the input precision or float64.
struct SgemmArgs {
    const void* A;
    long sAm, sAk;
    const void* B;
    long sBk, sBn;
    void* C;
    long ldc;
    int M, N, K;
    double alpha;
    int accumulate;
    const void* bias;
    int bias_every;
    int ksplit;           // > 1: blockIdx.z takes one K slice and writes raw sums to part, then a reduction
    void* part;           // ksplit x M x N partial sums (output precision)
};

// One elementwise or reduction step of supervised training (launch_train), in
// the context precision T; which fields are read depends on op.
enum TrainOpKind {
    TRAIN_GATHER = 0,   // out (n x B) = rows idx[b] (or b) of the (N x n) store a
    TRAIN_ELU_FWD,      // out = elu(a), count values
    TRAIN_ELU_BWD,      // out = a * elu'(b), count values
    TRAIN_RESIDUAL,     // out = Ubar of U = a against Dt = b (n x B), loss = mean mass-weighted squared residual
    TRAIN_ROWSUM,       // out[u] = sum_b a[u][b], u < n
    TRAIN_TO_ITEMS,     // z (B x n, float64) = a (n x B) transposed
    TRAIN_GRAD_OUT,     // z = a + scale g2 in float64, count values
    TRAIN_ADAM          // out (params) -= Adam step of a + scale g2 with moments m, v
};
struct TrainOp {
    int op = 0;
    const void* a = nullptr;
    const void* b = nullptr;
    void* out = nullptr;
    long count = 0;
    int n = 0, B = 0;
    const int* idx = nullptr;
    const double* rowmass = nullptr;
    const uint8_t* pinned_row = nullptr;
    double* part = nullptr;
    double* loss = nullptr;
    double* z = nullptr;
    const double* g2 = nullptr;
    double scale = 0.0;
    void* m = nullptr;
    void* v = nullptr;
    double lr = 0.0, b1 = 0.0, b2 = 0.0, eps = 0.0;
    int step = 1;
};

// Jets of the Lipschitz-loss gradient: (value, Jacobian, contracted second
// derivative) columns, r + 2 per item, column item * (r + 2) + c of row-major
// (units x columns) blocks.
struct JetArgs {
    int r, w, items, S;
    const double* zs;     // items x r latent points (kind 0)
    const void* Pre;      // pre-activations (kinds 1, 2) or output rows (kind 3), leading dimension ldp
    long ldp;
    void* X;              // activation out (kinds 0, 1), leading dimension ldx
    long ldx;
    const void* G;        // adjoints of the layer's output (kind 2), leading dimension ldg
    long ldg;
    void* D;              // adjoints of the pre-activations (kind 2) or element seeds (kind 3), ldd
    long ldd;
    const double* Cs;     // items x r x r signed contraction matrices
    const double* wV;     // S cubature weight times volume (kind 3)
    double mu, lam;
};

// ----------------------------------------------------------------- launchers
// arm timing events for the next kernel launch (recorded by the dispatch)
void set_launch_events(hipEvent_t start, hipEvent_t stop);
bool launch_events_pending();
hipError_t launch_gemm(int f32, int role, const GemmArgs& a, hipStream_t s);
// persistent variant for IN_RAW / IN_LATENT inputs with K a supported multiple of 32
hipError_t launch_gemm_p(int f32, int role, const GemmArgs& a, int target_blocks, hipStream_t s);
bool gemm_p_fits(int f32, int K);
// bf16: weights as three BF16 planes, the float32 layer input split into three BF16 parts, six products
// per chunk (f32 must be set; FP32 accumulation, pre-activations and activation)
// n_cu: compute units (a small batch takes fewer items per workgroup)
hipError_t launch_mlp(int f32, const MlpArgs& a, hipStream_t s, int bf16, int n_cu);
// persistent output map with A as three BF16 planes and transposed float32 input (IN_RAW_T, split into
// three BF16 parts), six products per chunk, FP32 accumulation and output
hipError_t launch_gemm_p_bf16(int role, const GemmArgs& a, int target_blocks, hipStream_t s);
bool mlp_fits(int f32, int nc, int r, int wrows); // the fused kernel's LDS and tiling limits
hipError_t launch_activate(int f32, const void* pre, void* act, int rows, int rows_pad, int nc, int items_cap,
                           const int* count, hipStream_t s);
hipError_t launch_elem(int f32, const ElemArgs& a, int items, hipStream_t s);
// the fused output map + element kernel: whether it applies (r, K), and the
// workgroups per item group it splits the rows over at a launch of cap items;
// A holds W_big as three BF16 planes (bf16 != 0) or in float32
bool elem_fused_fits(int r, int K);
int elem_fused_parts(int bf16, int cap, int n_cu);
hipError_t launch_elem_fused(int bf16, const FusedElemArgs& a, hipStream_t s);
hipError_t launch_energy(const EnergyArgs& a, int items, hipStream_t s);
// per-element positive-semi-definite projection: adds its correction to H
hipError_t launch_elem_psd(int f32, const ElemOptArgs& a, int items, hipStream_t s);
// 12x12 element Hessians of the first `items` items into a.He
hipError_t launch_elem_hess_dump(int f32, const ElemOptArgs& a, int items, hipStream_t s);
hipError_t launch_curv(int f32, const CurvArgs& a, int items, int n_cu, hipStream_t s);
hipError_t launch_param_outer(int f32, const ParamOuterArgs& a, hipStream_t s);
// dW[n][k] = sum_j coef[j] * src[row[j]][k] and db[n] = sum_j coef[j] * srcb[row[j]]
// over j in [ptr[n], ptr[n+1]): the transpose of a sparse row fold, n < rows
hipError_t launch_unfold(const double* src, const double* srcb, int ncols, const int* ptr, const int* row,
                         const double* coef, int rows, double* dW, double* db, hipStream_t s);
hipError_t launch_fill_zero(double* p, size_t n, hipStream_t s);
// the learned part
hipError_t launch_gemm_s(int f32, int out_f64, const SgemmArgs& g, hipStream_t s);
hipError_t launch_lip_stack(const double* z1, const double* z2, double* zs, int B, int r, hipStream_t s);
hipError_t launch_lip_count(const double* z1, const double* z2, int B, int r, int* nvalid, hipStream_t s);
hipError_t launch_lip_coef(const double* z1, const double* z2, const double* H, int B, int r, const int* nvalid,
                           double* Cs, double* ell, double* loss, int first, hipStream_t s);
hipError_t launch_jet(int f32, int kind, const JetArgs& j, hipStream_t s);
hipError_t launch_value_rowsum(int f32, const void* D, long ldd, int rows, int items, int nc, double* grad, hipStream_t s);
hipError_t launch_load_padded(int src_f64, const void* src, int out, int in, int rows_pad, int ld,
                              const uint8_t* rowmask, double* d64, float* d32, uint16_t* d16, hipStream_t s);
hipError_t launch_fold_rows(int src_f64, const void* Wout, const void* bout, int in_last, const int* ptr, const int* src,
                            const double* coef, int M, int Mp, int ld, double* W64, float* W32, uint16_t* W16,
                            double* b64, float* b32, hipStream_t s);
hipError_t launch_transpose(int f32, const void* src, int rows, int cols, int ld_src, void* dst, int ld_dst,
                            int dst_rows, hipStream_t s);
hipError_t launch_load_vec(int src_f64, const void* src, int n, const uint8_t* rowmask, double* d64, float* d32,
                           int n_pad, hipStream_t s);
hipError_t launch_train(int f32, const TrainOp& o, hipStream_t s);

// Implicit-Euler inertia and ground contact of one evaluation (launch_dyn)
struct DynArgs {
    const int* count;     // actual item count on the device (NULL = the launch's items)
    const int* imap;      // item -> load index (NULL = identity)
    const int* zmap;      // item -> row of z (linear decoders; NULL = identity)
    const double* z;      // latent points (linear decoders: h = z)
    int L, r, in_last, nc;
    const void* act;      // item-major (nc x wrows) last activation [h | J_h] (L > 0)
    int wrows;
    const void* out;      // item-major (rows_pad x nc) output-map rows
    int rows_pad;
    int crow, ncont;      // contact rows and their count
    const double* Xc;     // rest y of the contact vertices
    double k_ground, ground_y;
    const double* G;      // in_last x in_last
    const double* eta;    // per load index: the target's coefficients in the range (NULL = 0)
    const double* cvec;   // per load index: W^T M rho, rho the rest of the target
    const double* kappa;  // per load index: |rho|_M^2
    double inv_dt2;
    int inertia;
    double *E, *g, *H;    // added to (mode 2; E in mode 3)
    void* dseed;          // mode 0: item-major (rows_pad) seeds, context precision
    void* gbar;           // mode 1: item-major (in_rows) adjoint of h, context precision
    int in_rows;
};
hipError_t launch_dyn_gram(int f32, const void* W, int ld, int rows, const double* rowmass, int m, double* G,
                           hipStream_t s);
hipError_t launch_dyn_prep(int f32, const void* W, int ld, const void* bias, const uint8_t* pinned_row,
                           const double* rowmass, int rows, int m, const double* qbar, int B, double* cvec,
                           double* kappa, hipStream_t s);
hipError_t launch_dyn(int f32, int mode, const DynArgs& a, int cap, hipStream_t s);
hipError_t launch_dyn_state(int m, const double* h0, const double* h1, const double* cv0, const double* kv0,
                            double dt, int B, double* eta, double* cvec, double* kappa, hipStream_t s);
hipError_t launch_dyn_take_h(const double* act64, int wrows, const double* z, int m, int B, double* h, hipStream_t s);
hipError_t launch_sim_count(const int* it, const int* st, int B, int* iters, int* failed, hipStream_t s);
hipError_t launch_zero_int(int* p, int n, hipStream_t s);

// Full-space quasi-static solver over every element of the mesh (float64)
struct FullSolverDesc {
    int nv, ne, nt, nf;
    const double* X;        // 3 nv rest positions (host)
    const int* tets;        // 4 ne (host)
    const uint8_t* pinned;  // nv (host)
    const double* mass;     // nv lumped masses (host)
    const int* tvtx;        // nt penalty-targeted vertices (host)
    const int* fvtx;        // nf force-loaded vertices (host)
    double mu, lam, kc, grav[3];
};
struct FullSolveCall {
    int B;
    double* u;              // B x 3 nv displacements (device, in/out)
    const double* targets;  // B x nt x 3 or NULL
    const double* force;    // B x 3 or NULL
    int max_iter, ls_max, cg_max;
    double c1, shrink, rel_tol, abs_tol, eta_min, eta_max;
    int32_t *iters, *status;
    double *relgrad, *E;
};
struct FullSolver;
int full_solver_create(const FullSolverDesc& d, FullSolver** out, const char** why);
void full_solver_destroy(FullSolver* f);
int full_solve(FullSolver* f, const FullSolveCall& call, hipStream_t s, const char** why);
hipError_t launch_split_pairs(const double* z, int P, int r, double* z1, double* z2, hipStream_t s);
// PCA of snapshots (subspace iteration in the mass inner product)
hipError_t launch_pca_center(int f32, const void* D, int N, int n, double* mean, double* Dc, hipStream_t s);
hipError_t launch_pca_start(double* X, long count, hipStream_t s);
hipError_t launch_pca_mass(const double* X, const double* rowmass, int n, int k, double* MX, hipStream_t s);
hipError_t launch_pca_orth(const double* G, int k, double* R, int* fail, hipStream_t s);
hipError_t launch_pca_ritz(const double* T, int k, int r, double* V, double* ev, hipStream_t s);
hipError_t launch_newton_init(const NewtonState& st, int B, hipStream_t s);
hipError_t launch_compact_eval(const NewtonState& st, int B, int window, hipStream_t s);
hipError_t launch_newton_dir(const NewtonState& st, const NewtonParams& p, int cap, hipStream_t s);
// L-BFGS: exit tests, history update and the two-loop direction (same outputs as launch_newton_dir)
hipError_t launch_lbfgs_dir(const NewtonState& st, const NewtonParams& p, const LbfgsState& h, int cap,
                            hipStream_t s);
// search list, candidate list and candidate points zc
hipError_t launch_compact_search(const NewtonState& st, const NewtonParams& p, int B, hipStream_t s);
// Armijo test, then the next evaluation list and the running count, also written to `host` (device address
// of mapped pinned memory, may be NULL) as (tag << 32) | count
hipError_t launch_armijo(const NewtonState& st, const NewtonParams& p, int B, unsigned long long* host,
                         unsigned int tag, hipStream_t s);
hipError_t launch_stack_pairs(const double* z1, const double* z2, double* zs, int B, int r, hipStream_t s);
hipError_t launch_lipschitz(const double* z1, const double* z2, const double* H, int B, int r,
                            double* per_pair, double* ell, double* acc, int first_chunk, int last_chunk,
                            double* loss, int* n_valid, double* lip_max, hipStream_t s);

}  // namespace rs
