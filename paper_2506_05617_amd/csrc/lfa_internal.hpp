// Internal declarations shared by the host API (api.cpp) and the HIP kernel
// sources.  Not part of the public ABI (that is include/lfa.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lfa.h"

namespace lfa {

// Complex number in interleaved (re, im) layout, identical to
// torch.complex64 / complex128 element storage.
template <typename R>
struct alignas(2 * sizeof(R)) cplx {
    R x, y;
};

// Storage of the working matrix G (and the rotation accumulator) of a symbol
// during the Jacobi sweeps.
enum Storage : int { kLds = 0, kGlobal = 1 };

// Per-layer launch description, device-visible (passed by value).
struct LayerDesc {
    int c_out, c_in, kh, kw, n, m;
    int M, N;          // working matrix G is M x N with M = max(c), N = min(c)
    int transposed;    // 1 when c_out < c_in: G = A^H
    int tw_n, tw_m;    // offsets (in entries) of the n- and m-twiddle tables
    int L;             // lanes cooperating on one column pair (power of two)
    int threads;       // work-group size
    int storage;       // Storage
    int ldg, ldv;      // leading dimensions (elements) of G and of the accumulator
    int num_symbols;   // n*m
    int num_canon;     // frequencies with index <= that of their mirror (-k)
    int kind;          // 1: register (wave) kernel (M <= 64),
                       // 2: blocked kernel (rows in threads, column blocks in registers)
    int wave_nc;       // wave kernel: padded column count (power of two)
    int wave_ml;       // wave kernel: lanes per symbol (16, 32 or 64)
    long long sym_offset;   // first symbol of this layer in the plan's work list
    int wave_cap;      // wave kernel: work-groups resident at once on the device
                       // (0: unknown; one work-group per group of symbols)
    int wave_qcap;     // wave kernel: the same for its work-queue launch
                       // (0: work-queue launch not available)
    int wave_qgroups;  // wave kernel: groups the workspace holds queue state for
};

// ---- device helpers shared by the Jacobi kernels -------------------------

template <typename R>
struct alignas(4 * sizeof(R)) quad {
    R a, b, c, d;
};

// Numerically zero columns.  A symbol of rank below its column count keeps,
// in the columns that Jacobi drives to zero, rounding noise that every
// rotation with a nonzero column renews; its direction stays arbitrary, so
// the relative threshold below keeps rotating it until it underflows.  A
// column whose squared norm is at most (2u)^2 ||G||_F^2 (u the unit roundoff
// of R; ||G||_F is invariant under the rotations) therefore takes part in no
// rotation, and its singular value is reported as 0 (an error of at most
// 2u ||G||_F, below the normwise accuracy of the method).
template <typename R>
__host__ __device__ constexpr double negligible_sq() {
    return sizeof(R) == 4 ? 0x1p-46 : 0x1p-104;
}

// Scaled ("fast") form of the rotation for columns stored as g_j = G_j / d_j
// with per-column scale factors d_j.  gr, gi is the true gamma (of G).  The
// true rotation G_j' = c G_j - sn G_k, G_k' = c G_k + conj(sn) G_j becomes,
// with the scales multiplied by c, g_j' = g_j - tau1 g_k and
// g_k' = g_k + tau2 g_j (tau = sn / c, tau1 = tau d_k/d_j,
// tau2 = conj(tau) d_j/d_k): two complex multiply-adds per row instead of
// four real-by-complex products.  Returns (tau1, tau2) in q and updates the
// scales and the squared norms al, be that the caller tracks instead of
// recomputing: the rotation maps them to al - t |gamma| and be + t |gamma|
// (t the tangent of the angle), both clamped at 0 (tracked norms drift by
// rounding, and a negative one would pass the threshold with gamma = 0).
// Leaves everything unchanged and returns the identity (zeros) below the
// threshold or for a numerically zero column (min(al, be) <= floor).
//
// Result: 0 without a rotation, 1 for a small rotation, 2 for a larger one.
// A rotation is small when it moves each of its two columns by at most
// kappa = sqrt(tol)/4 relative to that column's own norm: the shorter
// column gains t |g_long|, so |t| sqrt(max(al, be) / min(al, be)) <= kappa
// (for columns of unequal norms -- graded symbols -- a small tangent alone
// does not bound the change of the shorter one).  A sweep whose rotations
// are all small then changes every inner product by O(kappa) times the
// products, which are themselves O(kappa), so the columns end orthogonal to
// the threshold and the rotation-free sweep that would confirm it can be
// skipped.
template <typename R>
__device__ __forceinline__ int rotation_scaled(double& al, double& be, double gr, double gi, double tol,
                                               double floor, R& dj, R& dk, quad<R>& q) {
    q = {R(0), R(0), R(0), R(0)};
    const double g2 = gr * gr + gi * gi;
    if (!(g2 > tol * tol * (al * be)) || !(fmin(al, be) > floor)) return 0;
    double rg, t, c, rjk, rkj;
    if constexpr (sizeof(R) == 4) {
        // The tangent t only selects the rotation and may be approximate.
        // What makes the applied transform orthogonal is c = 1/sqrt(1+t^2)
        // for that t and consistent 1/|gamma|, d_k/d_j and d_j/d_k: the
        // hardware reciprocal (square root) approximations are refined by one
        // Newton step each, to about 2^-46.
        rg = __builtin_amdgcn_rsq(g2);                                // 1/|gamma|
        rg = rg * fma(-0.5 * g2 * rg, rg, 1.5);
        const double z = 0.5 * (be - al) * rg;                        // zeta
        const double az = fabs(z);
        const double w = fma(az, az, 1.0);
        t = copysign(__builtin_amdgcn_rcp(az + w * __builtin_amdgcn_rsq(w)), z);
        const double w1 = fma(t, t, 1.0);
        c = __builtin_amdgcn_rsq(w1);
        c = c * fma(-0.5 * w1 * c, c, 1.5);
        double ij = __builtin_amdgcn_rcp(double(dj)), ik = __builtin_amdgcn_rcp(double(dk));
        ij = fma(ij, fma(-double(dj), ij, 1.0), ij);
        ik = fma(ik, fma(-double(dk), ik, 1.0), ik);
        rjk = double(dk) * ij;
        rkj = double(dj) * ik;
    } else {
        const double gg = sqrt(g2);
        rg = 1.0 / gg;
        const double z = (be - al) / (2.0 * gg);
        t = copysign(1.0, z) / (fabs(z) + sqrt(1.0 + z * z));
        c = 1.0 / sqrt(1.0 + t * t);
        rjk = double(dk) / double(dj);
        rkj = double(dj) / double(dk);
    }
    const double lo = fmin(al, be), hi = fmax(al, be);
    const double tg = t * g2 * rg;                                    // t |gamma|
    al = fmax(al - tg, 0.0);
    be = fmax(be + tg, 0.0);
    const double tr = t * gr * rg, ti = -t * gi * rg;                 // tau = t conj(gamma)/|gamma|
    q = {R(tr * rjk), R(ti * rjk), R(tr * rkj), R(-ti * rkj)};
    dj = R(c * double(dj));
    dk = R(c * double(dk));
    return 16.0 * t * t * hi > tol * lo ? 2 : 1;                   // t^2 hi/lo > tol/16, no division
}

// g_j' = g_j - tau1 g_k, g_k' = g_k + tau2 g_j (see rotation_scaled).
template <typename R>
__device__ __forceinline__ void rot_apply_scaled(cplx<R>& x, cplx<R>& y, R t1r, R t1i, R t2r, R t2i) {
    const cplx<R> xv = x, yv = y;
    x.x = fma(-t1r, yv.x, fma(t1i, yv.y, xv.x));
    x.y = fma(-t1r, yv.y, fma(-t1i, yv.x, xv.y));
    y.x = fma(t2r, xv.x, fma(-t2i, xv.y, yv.x));
    y.y = fma(t2r, xv.y, fma(t2i, xv.x, yv.y));
}

// Work item -> (frequency decomposed, output position, mirror output or -1).
// Real weights give A_{-k} = conj(A_k): sigma(-k) = sigma(k), U_{-k} =
// conj(U_k), V_{-k} = conj(V_k), so one symbol per conjugate pair is enough.
struct Target {
    int theta, out, mirror;
};

template <typename A>
__host__ __device__ inline int item_count(const A& a) {
    return a.theta_list ? a.theta_count : (a.canon ? a.d.num_canon : a.d.num_symbols);
}

// Canonical frequencies: flat index t = p m + q with t <= the index of its
// mirror -k = ((n-p) mod n, (m-q) mod m), in increasing order.  They are
// row p = 0 with q <= m/2, every q of the rows 0 < p < n - p, and (n even)
// row n/2 with q <= m/2.
__host__ __device__ inline int canonical_count(int n, int m) {
    const int h = m / 2 + 1, full = (n + 1) / 2 - 1;
    return h + full * m + (n % 2 == 0 && n > 1 ? h : 0);
}

__host__ __device__ inline int canonical_theta(int n, int m, int item) {
    const int h = m / 2 + 1, full = (n + 1) / 2 - 1;
    if (item < h) return item;
    const int r = item - h;
    if (r < full * m) return (1 + r / m) * m + r % m;
    return (n / 2) * m + (r - full * m);
}

// The first of one layer's (p, q, j) picks idx[0 .. s] whose symbol is that
// of pick s, or its conjugate (real weights: A_{-k} = conj(A_k), so the
// singular vectors of -k are the conjugates of those of k); `conj` tells
// which.  Picks of the same symbol need one decomposition.
__device__ inline int pick_rep(const int32_t* idx, int s, int n, int m, bool& conj) {
    const int p = idx[3 * s], q = idx[3 * s + 1];
    const int mp = p > 0 ? n - p : 0, mq = q > 0 ? m - q : 0;
    for (int t = 0; t < s; ++t) {
        const int pt = idx[3 * t], qt = idx[3 * t + 1];
        if (pt == p && qt == q) {
            conj = false;
            return t;
        }
        if (pt == mp && qt == mq) {
            conj = true;
            return t;
        }
    }
    conj = false;
    return s;
}

template <typename A>
__device__ inline Target target_of(const A& a, int item) {
    Target t;
    if (a.theta_list) {
        const int32_t* e = a.theta_list + (size_t)item * a.theta_stride;
        t.theta = a.theta_stride >= 2 ? e[0] * a.d.m + e[1] : e[0];
        t.out = item;
        t.mirror = -1;
    } else if (a.canon) {
        t.theta = canonical_theta(a.d.n, a.d.m, item);
        t.out = t.theta;
        const int p = t.theta / a.d.m, q = t.theta - (t.theta / a.d.m) * a.d.m;
        const int mi = ((a.d.n - p) % a.d.n) * a.d.m + (a.d.m - q) % a.d.m;
        t.mirror = mi != t.theta ? mi : -1;
    } else {
        t.theta = item;
        t.out = item;
        t.mirror = -1;
    }
    return t;
}

// One item of the persistent work list.
//  kind 0 ("bundle"): the work-group's waves each take SPW consecutive
//         work items of the layer, starting at `item` (register kernel, one
//         wave per symbol group);
//  kind 1 ("member"): member `member` of a team of W work-groups on work item
//         `item` of the layer (blocked kernel); `team` indexes the team's
//         barrier counters.
struct WorkItem {
    int layer, kind, item, member, W, team;
};

constexpr int kMaxLayers = 64;        // layers per plan
constexpr int kMaxLaunchLayers = 12;  // layers per multi-layer launch (kernarg <= 4 KB)
constexpr int kMaxTaps = 128;
constexpr int kMaxR = 1024;
constexpr int kRowsPerLane = 8;   // max rows of a column pair held per lane

// Arguments of one SVD launch over one layer (plain path) or over a work
// list (persistent path).
template <typename R>
struct SvdArgs {
    LayerDesc d;
    const R* W;                  // [c_out][c_in][kh*kw] weights, or null
    const cplx<R>* A;            // [n*m][c_out][c_in] symbols, or null
    R* sigma;                    // [n*m][r]
    cplx<R>* U;                  // [n*m][c_out][r] or null
    cplx<R>* V;                  // [n*m][c_in][r] or null
    int32_t* info;               // [LFA_INFO_WORDS] of this layer, or null
    const double* tw;            // twiddle table, (re, im) pairs
    char* gws;                   // global working storage, one slot per block
    long long slot_bytes;        // bytes per slot
    int canon;                   // 1: decompose the canonical frequencies (one per conjugate pair);
                                 // outputs are also written for the mirror frequency
    const int32_t* theta_list;   // optional: symbol indices to process
    int theta_stride;            // element stride in theta_list (3 for (p,q,j) triples)
    int theta_count;             // number of symbols to process
    int theta_dedup;             // theta_list holds one layer's (p, q, j) picks: a pick whose
                                 // symbol an earlier pick has (itself or its conjugate) is
                                 // skipped by the blocked kernel (see pick_rep)
    int max_sweeps;
    double tol;
    int32_t* wctr;               // register kernel: group counter (cleared) of a grid of
                                 // resident work-groups taking groups in turn, or null
    // work-queue launch of the register kernel (wq null: one work-group per
    // group of symbols, run to the end)
    int32_t* wq;                 // [kWaveQueueCtl] control words, then [wq_cap] entries
    void* wq_state;              // [groups] saved rows (see WaveSeg)
    int32_t* wq_meta;            // [groups][kWaveMeta]
    int wq_cap;                  // queue entries
    int wq_seg;                  // sweeps per run of a group
    unsigned long long* phase;   // register kernel: real-time-clock ticks per phase (load,
                                 // sweeps, finish, save), summed over the groups, or null
};

// Work queue of the register kernel: control words head (next entry to
// take), tail (next entry to fill), done (finished groups), err; the entries
// follow, 0 while empty, group + 1 once filled.
constexpr int kWaveQueueCtl = 64;
constexpr int kWaveMeta = 8;    // meta ints per group of the work queue (1 + SPW <= 5 used)

// Spectral function of one layer's operator applied to a batch of images
// (the kernels in apply.hip).  x [batch][cx][n][m] real, y [batch][cy][n][m]
// real; L [n*m][cy][r], R [n*m][cx][r] complex (U, V for identity and clip,
// V, U for pinv); sigma [n*m][r]; ws1, ws2 each batch*n*m*max(cx, cy)
// complex elements.
struct ApplyArgs {
    int batch, n, m, cx, cy, r, kind;
    double param;
    const void* sigma;
    const void* L;
    const void* R;
    const void* x;
    void* y;
    void* ws1;
    void* ws2;
    const double* tw;
    int tw_n, tw_m;
};
hipError_t launch_apply_f32(const ApplyArgs& a, hipStream_t s);
// The per-frequency map of an image chunk fits the LDS of a work-group.
bool apply_supported(int cx, int r, int elem_bytes);
hipError_t launch_apply_f64(const ApplyArgs& a, hipStream_t s);

// Global singular vectors of `count` picks idx[t] = (p, q, j) (device int32):
// u_hat[t][o][x1][x2] = e^{2 pi i (p x1 / n + q x2 / m)} U[p][q][o][j] / sqrt(n m),
// v_hat likewise from V with c_in rows; a NULL output is skipped, a pick out
// of range gives zeros.
struct LiftArgs {
    int count, n, m, c_out, c_in, r;
    const int32_t* idx;
    const void* U;
    const void* V;
    void* u_hat;
    void* v_hat;
    const double* tw;
    int tw_n, tw_m;
};
hipError_t launch_lift_f32(const LiftArgs& a, hipStream_t s);
hipError_t launch_lift_f64(const LiftArgs& a, hipStream_t s);

// A stride-`stride` layer (c_out, c_in, kh, kw) and the stride-1 layer of its
// crystal form (c_out, stride^2 c_in, kh2, kw2) on the coarse torus.
struct CrystalArgs {
    int c_out, c_in, kh, kw, stride, kh2, kw2;
};
// Forward: W -> Wc (the crystal layer's weights); adjoint: Wc -> W.
hipError_t launch_crystal_weights(const CrystalArgs& a, int elem_bytes, const void* src, void* dst, bool adjoint,
                                  hipStream_t s);

size_t lds_bytes_for(const LayerDesc& d, bool accumulate, int elem_bytes);

size_t wave_lds_bytes_for(int nc, int ml, int elem_bytes);
// LDS of one wave running a bundle in the persistent launch: the register
// kernel's arrays, plus its output staging when it writes singular vectors.
size_t wave_bundle_lds_for(int nc, int ml, int elem_bytes, bool vectors);
size_t block_lds_bytes(const LayerDesc& d, bool accumulate, int elem_bytes);
// Blocked kernel: `teams` teams of W work-groups (all resident at once when
// W > 1) over the items [item0, item_split) of the layer, and in the same
// grid, after them, teams2 teams of W2 over [item_split, item_end) (the
// short last round; teams2 = 0: none); one global slot per team; counters:
// 4*(teams + teams2) + 4 int32 of device memory, cleared by the launcher.
hipError_t launch_block_svd_f32(const SvdArgs<float>& a, int teams, int W, int item0, int item_split, int teams2,
                                int W2, int item_end, int32_t* counters, hipStream_t s);
hipError_t launch_block_svd_f64(const SvdArgs<double>& a, int teams, int W, int item0, int item_split, int teams2,
                                int W2, int item_end, int32_t* counters, hipStream_t s);
// Work-groups of the blocked kernel that fit on the device at once (0 on error).
int block_resident(const LayerDesc& d, bool accumulate, int elem_bytes);

// Launchers (each returns a hipError_t).
hipError_t launch_wave_svd_f32(const SvdArgs<float>& a, int grid, hipStream_t s);
hipError_t launch_wave_svd_f64(const SvdArgs<double>& a, int grid, hipStream_t s);
// Work-groups of the register kernel of shape (nc, ml) with `threads` per
// work-group that fit on one CU; `vectors`: U or V is written (output
// staging LDS).  0 on error or for an unsupported shape.
int wave_blocks_per_cu(int nc, int ml, int elem_bytes, int threads, bool vectors);
// Work-queue launch of the register kernel (a.wq set, control words and
// entries cleared): `grid` work-groups, all resident at once.
hipError_t launch_wave_queue_f32(const SvdArgs<float>& a, int grid, hipStream_t s);
hipError_t launch_wave_queue_f64(const SvdArgs<double>& a, int grid, hipStream_t s);
// The same for the work-queue launch.
int wave_queue_blocks_per_cu(int nc, int ml, int elem_bytes, int threads, bool vectors);

// LFA_PHASE_NORMALIZE on one layer's outputs: syms symbols of U
// [syms][rows_u][r] and V [syms][rows_v][r] (either may be null; the phase
// comes from V when it is there).
hipError_t launch_phase_normalize_f32(cplx<float>* U, cplx<float>* V, int syms, int rows_u, int rows_v, int r,
                                      hipStream_t s);
hipError_t launch_phase_normalize_f64(cplx<double>* U, cplx<double>* V, int syms, int rows_u, int rows_v, int r,
                                      hipStream_t s);

hipError_t launch_symbols_valu_f32(const LayerDesc& d, const float* W, cplx<float>* A,
                                   const double* tw, hipStream_t s);
hipError_t launch_symbols_valu_f64(const LayerDesc& d, const double* W, cplx<double>* A,
                                   const double* tw, hipStream_t s);
// mode: 0 = FP32 MFMA, 2 = split-BF16 x2 (3 products), 3 = split-BF16 x3 (6 products);
// canon_only: only the canonical symbol of each conjugate pair is written
// (at its own place in A), for the SVD of real weights
hipError_t launch_symbols_mfma(const LayerDesc& d, const float* W, cplx<float>* A,
                               const double* tw, int mode, hipStream_t s, bool canon_only = false);

hipError_t launch_fill_i32(int32_t* p, int32_t value, long long count, hipStream_t s);

// Static device scratch of lfa_svd_noalloc (noalloc.hip): 64 MiB per device.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
hipError_t noalloc_scratch(int device, void** ptr, size_t* bytes);

template <typename R>
struct TopkArgs {
    const R* sigma[kMaxLaunchLayers];
    int n[kMaxLaunchLayers], m[kMaxLaunchLayers], r[kMaxLaunchLayers];
    int num_layers;
    int k;
    R* vals;
    int32_t* idx;
};
hipError_t launch_topk_f32(const TopkArgs<float>& a, hipStream_t s);
hipError_t launch_topk_f64(const TopkArgs<double>& a, hipStream_t s);

template <typename R>
struct AdjointArgs {
    int c_out[kMaxLaunchLayers], c_in[kMaxLaunchLayers], kh[kMaxLaunchLayers],
        kw[kMaxLaunchLayers], n[kMaxLaunchLayers], m[kMaxLaunchLayers];
    int tw_n[kMaxLaunchLayers], tw_m[kMaxLaunchLayers];
    const cplx<R>* U[kMaxLaunchLayers];   // full [n*m][c_out][r] or compact [k][c_out][r]
    const cplx<R>* V[kMaxLaunchLayers];
    R* dW[kMaxLaunchLayers];
    int blocks_before[kMaxLaunchLayers + 1];
    int num_layers;
    int k;
    int compact;                    // 0: full U/V; 1: U/V hold only the k selected
                                    // symbols; 2: U/V hold one vector per pick
                                    // ([k][c_out] and [k][c_in], column j of the pick)
    const int32_t* idx;             // [num_layers][k][3]
    const R* grad;                  // [num_layers][k]
    const double* tw;
};
hipError_t launch_adjoint_f32(const AdjointArgs<float>& a, hipStream_t s);
hipError_t launch_adjoint_f64(const AdjointArgs<double>& a, hipStream_t s);

// QR preconditioning of tall symbols (qr.hip): the FP64 taps C_delta of the
// Gram convolution, then per decomposed frequency H_k and its Cholesky
// factor R (R^H R = H_k), written as the N x N symbols the SVD then takes.
template <typename R>
struct GramArgs {
    const R* W;                 // [c_out][c_in][kh*kw]
    int c_out, c_in, kh, kw, n, m;
    int M, N;                   // working matrix rows and columns (M > N)
    int transposed;             // G = A^H (c_out < c_in)
    int tw_n, tw_m;
    const double* tw;
    double* C;                  // [(2kh-1)(2kw-1)][N][N]
    void* hslots;               // [items][N][N] complex double
    cplx<R>* Rsym;              // [n*m][N][N]; canonical frequencies written
    int conj_transpose;         // write R^H instead of R
};
size_t gram_cholesky_lds_bytes(int N, int kh, int kw);

// Singular vectors of a preconditioned layer (qr.hip): Y = G_k V_R into
// per-item slots (Y column-major with leading dimension ldg, then V_R with
// ldv), then the blocked kernels' finish writing sigma, U, V.
template <typename R>
struct QrVecArgs {
    const R* W;
    int c_out, c_in, kh, kw, n, m;
    int M, N, transposed;
    int tw_n, tw_m;
    const double* tw;
    const cplx<R>* VR;          // [n*m][N][N] right singular vectors of R (left ones of R^H)
    const R* sigma;             // [n*m][N] singular values of R (same column order)
    char* slots;                // [items] slots of slot_bytes
    long long slot_bytes;
    int ldg, ldv;
};
hipError_t launch_qr_vectors_f32(const QrVecArgs<float>& q, const SvdArgs<float>& a, int items, hipStream_t s);
hipError_t launch_qr_vectors_f64(const QrVecArgs<double>& q, const SvdArgs<double>& a, int items, hipStream_t s);
hipError_t launch_gram_qr_f32(const GramArgs<float>& g, int items, hipStream_t s);
hipError_t launch_gram_qr_f64(const GramArgs<double>& g, int items, hipStream_t s);

// The singular vector a one-sided forward pass did not keep, for each pick
// (p, q, j) of each layer: with the kept side x (U when c_out >= c_in, else
// V), v = A_k^H u / sigma or u = A_k v / sigma, A_k assembled from W.
// Writes both vectors of every pick to the compact per-pick arrays of the
// adjoint (compact mode 2).
template <typename R>
struct OtherSideArgs {
    const R* W[kMaxLaunchLayers];
    const R* sigma[kMaxLaunchLayers];      // [n][m][r]
    const cplx<R>* X[kMaxLaunchLayers];    // kept side, [n][m][c_kept][r]
    cplx<R>* Uc[kMaxLaunchLayers];         // [k][c_out]
    cplx<R>* Vc[kMaxLaunchLayers];         // [k][c_in]
    int c_out[kMaxLaunchLayers], c_in[kMaxLaunchLayers], kh[kMaxLaunchLayers],
        kw[kMaxLaunchLayers], n[kMaxLaunchLayers], m[kMaxLaunchLayers];
    int tw_n[kMaxLaunchLayers], tw_m[kMaxLaunchLayers];
    int num_layers;
    int k;
    const int32_t* idx;                    // [num_layers][k][3]
    const double* tw;
};
hipError_t launch_other_side_f32(const OtherSideArgs<float>& a, hipStream_t s);
hipError_t launch_other_side_f64(const OtherSideArgs<double>& a, hipStream_t s);

// Persistent launch over a work list covering several layers.
template <typename R>
struct PersistentArgs {
    SvdArgs<R> layer[kMaxLaunchLayers];   // per-layer arguments (d, pointers; gws = slot base)
    int num_layers;
    const WorkItem* items;          // device work list, longest first
    int num_items;
    int32_t* counter;               // device dequeue counter (cleared before launch)
    int32_t* team_counters;         // 4 per team + error word (cleared before launch)
    int num_teams;
    int wave_slots;                 // waves of a work-group that run bundles
    int wave_lds;                   // LDS bytes of one wave's bundle
    int threads;                    // work-group size (256)
    long long* busy;                // optional per-work-group record [grid][4]: busy ticks
                                    // (100 MHz), items taken, XCC id, HW_ID (SE/SH/CU bits); or null
};
constexpr int kPersistentThreads = 256;

// LDS bytes of the persistent launch for the layers of `descs` (kind 1 bundles
// with `wave_slots` waves, kind 2 blocked items with 256 threads), and the
// number of work-groups of the launch that fit on the device at once.
size_t persistent_lds_bytes(const LayerDesc* descs, int n, bool accumulate, bool bundle_vectors, int elem_bytes,
                            int wave_slots);
int persistent_resident(size_t lds, int elem_bytes, bool accumulate);
hipError_t launch_persistent_f32(const PersistentArgs<float>& a, int grid, size_t lds, bool accumulate,
                                 hipStream_t s);
hipError_t launch_persistent_f64(const PersistentArgs<double>& a, int grid, size_t lds, bool accumulate,
                                 hipStream_t s);

}  // namespace lfa
