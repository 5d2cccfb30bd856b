// Host side of liblfa: plans, launch shapes, workspace layout, and the
// extern "C" entry points declared in include/lfa.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lfa.h"
#include "lfa_internal.hpp"

using namespace lfa;

namespace {

thread_local int g_last_hip = 0;

int hip_fail(hipError_t e) {
    g_last_hip = static_cast<int>(e);
    return LFA_ERR_HIP;
}

#define HIP_TRY(expr)                              \
    do {                                           \
        hipError_t _e = (expr);                    \
        if (_e != hipSuccess) return hip_fail(_e); \
    } while (0)

#define LFA_TRY(expr)                \
    do {                             \
        int _s = (expr);             \
        if (_s != LFA_OK) return _s; \
    } while (0)

constexpr size_t kAlign = 256;
constexpr size_t kLdsCap = 160 * 1024 - 1024;  // gfx950: 160 KiB of LDS per work-group
constexpr size_t kLdsSafe = 64 * 1024;         // always available without opt-in
constexpr int kGlobalGrid = 1024;              // blocks of a launch using global slots

constexpr int kMaxTopk = 64;
constexpr int kBlockCols = 16;                    // column block of the blocked kernel
constexpr size_t kCounterBytes = 256 * ((4 * (4 * 1024 + 4) + 255) / 256);   // team counters
constexpr int kMaxSweeps = 40;

size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }
int pow2ceil(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

int elem_bytes(int dtype) { return dtype == LFA_F64 ? 8 : 4; }

// Rotation threshold of a column pair: |g_j^H g_k| > tol * |g_j| |g_k| with
// tol = 2 sqrt(M) u.  The computed inner product of two orthogonal columns
// carries at most (rows per lane + log2 lanes) u |g_j| |g_k| <= 14 u of
// rounding error, below this threshold for every M >= 16, so sweeps cannot
// stall on rounding noise; the final loss of orthogonality is about tol.
double jacobi_tol(double unit_roundoff, int M) {
    return 2.0 * std::sqrt((double)std::max(M, 16)) * unit_roundoff;
}

}  // namespace

// Per-layer choices of lfa_autotune for lfa_svd (defaults: the cost
// model's automatic choices).
struct LayerTune {
    int queue_seg = -1;    // register kernel's work queue: -1 automatic, 0 off, k sweeps per turn
    int team_w = 0;        // blocked kernel: work-groups per symbol, 0 automatic
    int asm_mat = -1;      // -1 the plan's flags, 0 fused assembly, 1 materialised FP32 matrix-core assembly
};

struct lfa_plan {
    int dtype = LFA_F32;
    uint32_t flags = 0;
    std::vector<lfa_layer> layers;
    std::vector<int> tw_n, tw_m;          // twiddle offsets per layer
    std::vector<LayerDesc> desc;          // plain lfa_svd launch shape
    std::vector<LayerDesc> desc_pers;     // persistent launch shape
    std::vector<LayerDesc> desc_sel;      // SVD with vectors of selected symbols
    std::vector<double> tw_host;          // (re, im) pairs
    std::vector<WorkItem> items;          // persistent work list, LPT order per chunk
    std::vector<int> chunk_first;         // first item of each chunk of layers (+ end)
    double tol = 0;
    int max_sweeps = kMaxSweeps;          // sweep cap (lfa_plan_set_max_sweeps)
    int wq_force = -1;                    // work queue: -1 automatic, 0 off, k > 0 forced
    unsigned long long* phase_rec = nullptr;   // register kernel phase record (lfa_plan_record_phases)
    std::mutex mu;
    int device = -1;
    double* tw_dev = nullptr;
    WorkItem* items_dev = nullptr;
    std::vector<WorkItem*> old_items;     // earlier uploads (see upload_items)
    int num_cus = 0;
    // persistent launch: slots of the blocked layers, team counters, schedule
    std::vector<size_t> pers_slot_off;    // byte offset of each layer's slots (blocked layers)
    size_t pers_slots_total = 0;
    int pers_teams = 0;                   // team instances (one per blocked-layer symbol)
    int pers_wave_slots = 4;
    bool pers_acc = false;                // some layer keeps the rotation accumulator
    // cost model of the persistent work list (lfa_autotune may change it):
    // seconds per unit N^2 M of a register-kernel wave and of a 256-thread
    // blocked work-group, and the per-member overhead of a team
    double cost_wave = 7.5e-9, cost_block = 2.5e-9, team_ovh = 0.08;
    std::vector<LayerTune> tune;
    std::vector<size_t> pers_lds;         // per chunk
    std::vector<int> pers_grid;           // per chunk
    // persistent SVD-with-vectors of the selected symbols, per k
    struct GradSched {
        WorkItem* items_dev = nullptr;
        std::vector<int> chunk_first;
        std::vector<size_t> lds;
        std::vector<int> grid;
        int teams = 0;
    };
    std::map<int, GradSched> grad_sched;
    std::vector<LayerDesc> desc_gsel;     // blocked-kernel shape with vectors, 256 threads
    // QR preconditioning of tall symbols (lfa_svd, sigma only): per layer
    // whether it is used, and the launch shape of the SVD of the N x N
    // factors R
    std::vector<int> qr;
    std::vector<LayerDesc> desc_r;
};

struct lfa_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

bool accumulates(const LayerDesc& d, bool want_u, bool want_v) {
    return d.transposed ? want_u : want_v;
}

// Cost-model launch shape: enough lanes per pair that a lane holds at most
// kRowsPerLane rows, one lane group per column pair of a step (capped at
// 1024 threads), LDS storage when the working matrices fit under `lds_cap`.
LayerDesc make_desc(const lfa_layer& l, int tw_n, int tw_m, bool acc, int eb, size_t lds_cap,
                    int threads_override = 0, int L_override = 0, bool allow_wave = true) {
    LayerDesc d{};
    d.c_out = l.c_out;
    d.c_in = l.c_in;
    d.kh = l.kh;
    d.kw = l.kw;
    d.n = l.n;
    d.m = l.m;
    d.M = std::max(l.c_out, l.c_in);
    d.N = std::min(l.c_out, l.c_in);
    d.transposed = l.c_out < l.c_in ? 1 : 0;
    d.tw_n = tw_n;
    d.tw_m = tw_m;
    d.num_symbols = l.n * l.m;
    int L = pow2ceil((d.M + kRowsPerLane - 1) / kRowsPerLane);
    L = std::max(1, std::min(64, L));
    if (L_override) L = L_override;
    d.L = L;
    const int npairs = (d.N + 1) / 2;
    int threads = pow2ceil(std::max(1, npairs * L));
    threads = std::max(64, std::min(1024, threads));
    if (threads_override) threads = threads_override;
    d.threads = threads;
    d.ldg = d.M | 1;
    d.ldv = d.N | 1;
    d.storage = kLds;
    d.kind = 0;
    if (allow_wave && d.M <= 64 && !threads_override && !L_override) {
        // register-resident kernel: rows in lanes, one wave (+ one for Q)
        d.kind = 1;
        d.wave_ml = std::max(16, pow2ceil(d.M));
        d.wave_nc = std::max(4, pow2ceil(d.N));
        d.threads = acc ? 128 : 64;
    } else if (allow_wave && !threads_override && !L_override) {
        // blocked kernel: one thread per row, column blocks in registers,
        // working matrices in a global slot
        d.kind = 2;
        d.threads = (d.M + 63) / 64 * 64;
        d.storage = kGlobal;
        return d;
    }
    if (lds_bytes_for(d, acc, eb) > lds_cap) d.storage = kGlobal;
    d.sym_offset = 0;
    return d;
}

int wave_symbols_per_group(const LayerDesc& d) { return d.kind == 1 ? 64 / d.wave_ml : 1; }

// Register kernel: resident work-groups take groups from a counter when the
// groups fill the device at most this many times.
constexpr int kWaveTurnRounds = 4;

// Work-queue launch of the register kernel.  It pays off when the groups of
// symbols fill the resident work-groups more than once but only a few times:
// one work-group per group then leaves a last, partly filled round.
constexpr int kQueueMaxRounds = 4;
constexpr size_t kQueueMaxBytes = size_t(1) << 30;   // workspace for queue state, per layer

int wave_groups(const LayerDesc& d, int count) {
    const int spg = wave_symbols_per_group(d);
    return (count + spg - 1) / spg;
}

// A group runs at least one sweep per turn, so it is queued again at most
// kMaxSweeps - 1 times.
long long wave_queue_entries(int groups, int seg) {
    return (long long)groups * ((kMaxSweeps + seg - 1) / seg);
}

size_t wave_queue_state_bytes(const LayerDesc& d, bool acc, int eb) {
    return (size_t)(acc ? 2 : 1) * 64 * d.wave_nc * 2 * eb;
}

size_t wave_queue_bytes(const LayerDesc& d, bool acc, int eb, int groups) {
    return align_up(sizeof(int32_t) * (kWaveQueueCtl + wave_queue_entries(groups, 1))) +
           align_up(sizeof(int32_t) * kWaveMeta * (size_t)groups) +
           align_up((size_t)groups * wave_queue_state_bytes(d, acc, eb));
}

// Groups the workspace reserves queue state for: every symbol of the layer
// (the largest count of any entry point), or none beyond kQueueMaxBytes.
int wave_queue_reserved(const LayerDesc& d, bool acc, int eb) {
    if (d.kind != 1) return 0;
    const int g = wave_groups(d, d.num_symbols);
    return wave_queue_bytes(d, acc, eb, g) <= kQueueMaxBytes ? g : 0;
}

// Sweeps per turn of a group in the work-queue launch (0: no work queue).
// A turn costs the save and restore of the group's rows and an L2 write-back
// and invalidation; measured on the 64 x 64 layer on the 64 x 64 grid (2050
// groups, 1024 or 2048 resident; 8 to 10 sweeps per symbol): sigma only 4
// or 5 sweeps per turn were best (6: 4 % slower); with vectors 2.54, 2.51,
// 2.62 and 2.81 ms for 5, 6, 7 and 8 sweeps per turn, 2.81 ms for 10 (a
// whole symbol's sweeps: no group is saved, but the last groups start
// late), 2.90 ms without the queue.  The saved rows are about half the HBM
// bytes of the launch, which is ALU-bound: fine-grained turns pay.
constexpr int kQueueSweepsPerTurn = 5;
constexpr int kQueueSweepsPerTurnVectors = 6;
int wave_queue_seg(const LayerDesc& d, int groups, int force) {
    if (d.kind != 1 || d.wave_qcap <= 0 || groups > d.wave_qgroups || force == 0) return 0;
    if (force > 0) return force;
    if (groups <= d.wave_qcap) return 0;
    const long long rounds = ((long long)groups + d.wave_qcap - 1) / d.wave_qcap;
    if (rounds > kQueueMaxRounds) return 0;
    return d.threads > 64 ? kQueueSweepsPerTurnVectors : kQueueSweepsPerTurn;   // a Q wave: vectors
}

size_t slot_bytes(const LayerDesc& d, bool acc, int eb) {
    if (d.storage != kGlobal) return 0;
    const size_t cb = 2 * (size_t)eb;
    return align_up(cb * d.ldg * d.N + (acc ? cb * d.ldv * d.N : 0));
}

int svd_grid(const LayerDesc& d, int count) {
    return d.storage == kGlobal ? std::min(count, kGlobalGrid) : count;
}

size_t symbols_bytes(const lfa_layer& l, int eb) {
    return align_up((size_t)l.n * l.m * l.c_out * l.c_in * 2 * eb);
}

bool asm_materialized(uint32_t flags) {
    return (flags & (LFA_ASM_MFMA | LFA_ASM_BF16X2 | LFA_ASM_BF16X3)) != 0;
}

int asm_mode(uint32_t flags) {
    if (flags & LFA_ASM_BF16X3) return 3;
    if (flags & LFA_ASM_BF16X2) return 2;
    return 0;
}

// Materialised (matrix-core) assembly for layer i: the autotuner's choice,
// else the plan's flags, else by default for FP32 kernels of 25 taps or more
// (the fused assembly then costs the SVD kernel more than writing and
// reading the symbols: 7x7 kernel on the 224 x 224 grid, 18.5 ms fused
// against 0.8 ms of FP32 matrix-core assembly + 15.5 ms of SVD).
bool layer_materialized(const lfa_plan& p, size_t i) {
    const int t = p.tune[i].asm_mat;
    if (t >= 0) return t == 1;
    const lfa_layer& l = p.layers[i];
    return asm_materialized(p.flags) || (p.dtype == LFA_F32 && l.kh * l.kw >= 25);
}

size_t pers_counter_bytes(const lfa_plan& p) {
    return align_up(sizeof(int32_t) * (4 * (size_t)p.pers_teams + 4));
}

size_t sel_bytes(const lfa_layer& l, int eb) {
    const size_t r = std::min(l.c_out, l.c_in);
    return align_up((size_t)kMaxTopk * (r * eb + (size_t)(l.c_out + l.c_in) * r * 2 * eb));
}

// QR preconditioning (qr.hip) pays where the working matrix is clearly
// taller than wide and the blocked kernel would run it (M > 64): the
// sweeps then touch N rows instead of M.  FP32 plans only: the factor is
// accurate to about sqrt(N u64) sigma_max, far inside the FP32 tolerance
// but not the FP64 one.  With singular vectors the SVD of R keeps its
// right vectors and the left ones come from G V (qr_left_kernel).
// Measured on MI355X (sigma only / U / U and V): the 512 x 256 layer on the
// 32 x 32 grid (514 decomposed symbols) 112 -> 60 / 112 -> 92 / 152 -> 92 ms
// with the factors; 128 x 64 on 16 x 16 (factors run by the register
// kernel) 1.50 -> 1.15 / 1.55 -> 1.25 / 2.21 -> 1.25 ms; but with a few
// symbols of blocked-kernel factors (256 x 128 on 8 x 8, 36 symbols;
// 512 x 256 on 4 x 4, 10 symbols) the direct kernel's teams were as fast
// or faster (3.0 vs 3.4, 8.5 vs 8.3 sigma only; 3.1 vs 4.5, 8.7 vs 10.9
// with U).  So by default: factors whose SVD the register kernel runs
// (N <= 64), or at least a device's worth of symbols (one per CU of
// MI355X); lfa_autotune times both where it matters.
constexpr int kQrMinSymbols = 256;
bool qr_eligible(const lfa_layer& l, int dtype, uint32_t flags) {
    const int M = std::max(l.c_out, l.c_in), N = std::min(l.c_out, l.c_in);
    if (dtype != LFA_F32) return false;
    if (flags & (LFA_ASM_MFMA | LFA_ASM_BF16X2 | LFA_ASM_BF16X3)) return false;
    // the Cholesky kernel keeps a panel of its factor's rows in LDS
    if (gram_cholesky_lds_bytes(N, l.kh, l.kw) > kLdsCap) return false;
    return M > 64 && 4 * M >= 5 * N;
}
bool qr_applies(const lfa_layer& l, int dtype, uint32_t flags) {
    const int N = std::min(l.c_out, l.c_in);
    if (!qr_eligible(l, dtype, flags)) return false;
    // LFA_QR: "0" off, "1" on for every such layer (tests, tuning)
    if (const char* env = std::getenv("LFA_QR")) {
        if (std::strcmp(env, "0") == 0) return false;
        if (std::strcmp(env, "1") == 0) return true;
    }
    return N <= 64 || canonical_count(l.n, l.m) >= kQrMinSymbols;
}

size_t qr_taps_bytes(const lfa_layer& l) {
    const size_t N = std::min(l.c_out, l.c_in);
    return align_up((size_t)(2 * l.kh - 1) * (2 * l.kw - 1) * N * N * sizeof(double));
}
size_t qr_rsym_bytes(const lfa_layer& l, int eb) {
    const size_t N = std::min(l.c_out, l.c_in);
    return align_up((size_t)l.n * l.m * N * N * 2 * eb);
}
size_t qr_hslot_bytes(const lfa_layer& l) {
    const size_t N = std::min(l.c_out, l.c_in);
    return align_up((size_t)canonical_count(l.n, l.m) * N * N * 2 * sizeof(double));
}
// Slots of the vectors' finish: Y (ldg x N) and V_R (ldv x N) per item.
size_t qr_vec_slot_bytes(const LayerDesc& d, int eb) {
    return align_up((size_t)2 * eb * ((size_t)d.ldg * d.N + (size_t)d.ldv * d.N));
}
// The preconditioned path's region: R symbols (overwritten by the right
// singular vectors of R when vectors are wanted), then the Gram taps and
// the Cholesky slots or the R SVD's own region; the vectors' slots follow
// the R symbols once the taps and those are done.
size_t qr_region_bytes(const lfa_plan& p, int i, bool queue) {
    const int eb = elem_bytes(p.dtype);
    const bool vec = (p.flags & (LFA_WANT_U | LFA_WANT_V)) != 0;
    const lfa_layer& l = p.layers[i];
    const LayerDesc& dr = p.desc_r[i];
    LayerDesc drg = dr;
    // the SVD of the factors keeps no accumulator (see svd_layer)
    drg.storage = (lds_bytes_for(dr, false, eb) > kLdsSafe) ? kGlobal : dr.storage;
    size_t svd_r = kCounterBytes + (size_t)svd_grid(drg, dr.num_symbols) * slot_bytes(drg, false, eb);
    if (queue && dr.wave_qgroups > 0) svd_r = std::max(svd_r, wave_queue_bytes(dr, false, eb, dr.wave_qgroups));
    size_t after = qr_taps_bytes(l) + std::max(svd_r, qr_hslot_bytes(l));
    if (vec) after = std::max(after, (size_t)p.desc[i].num_canon * qr_vec_slot_bytes(p.desc[i], eb));
    return qr_rsym_bytes(l, eb) + after;
}

// Per-pick vectors of the one-sided adjoint: [k][c_out] and [k][c_in]
// complex per layer, layer after layer.
size_t pick_vector_bytes(const lfa_plan& p, int k) {
    const size_t cb = 2 * (size_t)elem_bytes(p.dtype);
    size_t b = 0;
    for (const lfa_layer& l : p.layers)
        b += align_up((size_t)k * l.c_out * cb) + align_up((size_t)k * l.c_in * cb);
    return b;
}

// Region bytes of lfa_svd for layer i with the given choices (QR factors,
// materialised assembly, the register kernel's work queue); lds_fallback
// also reserves global slots for a layer whose LDS need exceeds the
// always-available 64 KiB (a device with less LDS than the plan assumed).
size_t svd_layer_need(const lfa_plan& p, size_t i, bool qr, bool mat, bool queue, bool lds_fallback) {
    const int eb = elem_bytes(p.dtype);
    const bool wu = p.flags & LFA_WANT_U, wv = p.flags & LFA_WANT_V;
    const LayerDesc& d = p.desc[i];
    const bool acc = accumulates(d, wu, wv);
    LayerDesc dg = d;
    if (lds_fallback) dg.storage = (lds_bytes_for(d, acc, eb) > kLdsSafe) ? kGlobal : d.storage;
    const size_t sym = mat ? symbols_bytes(p.layers[i], eb) : 0;
    size_t s = sym + (size_t)svd_grid(dg, d.num_symbols) * slot_bytes(dg, acc, eb);
    if (queue && d.wave_qgroups > 0) s = std::max(s, sym + wave_queue_bytes(d, acc, eb, d.wave_qgroups));
    if (qr && !mat) s = std::max(s, qr_region_bytes(p, (int)i, queue));
    return s;
}

// Workspace layout (offsets from ws):
//   [0, 256)                   persistent dequeue counter
//   [256, 256 + big)           per-entry-point region (regions of different
//                              entry points may overlap: calls are stream-ordered)
size_t workspace_bytes(const lfa_plan& p) {
    const int eb = elem_bytes(p.dtype);
    const bool wu = p.flags & LFA_WANT_U, wv = p.flags & LFA_WANT_V;
    size_t need = 0;
    (void)wu;
    (void)wv;
    for (size_t i = 0; i < p.layers.size(); ++i) {
        // lfa_svd / lfa_svd_symbols: symbols (materialised assembly) + slots,
        // the work queue, or the QR factors' region.  A layer whose LDS need
        // exceeds the always-available 64 KiB may fall back to global slots
        // on a device with less LDS: reserve for that too.
        need = std::max(need, svd_layer_need(p, i, p.qr[i] != 0, layer_materialized(p, i), true, true));
        // lfa_sigma_grad: compact outputs of <= kMaxTopk symbols + slots
        const LayerDesc& ds = p.desc_sel[i];
        LayerDesc dsg = ds;
        dsg.storage = (lds_bytes_for(ds, true, eb) > kLdsSafe) ? kGlobal : ds.storage;
        need = std::max(need, sel_bytes(p.layers[i], eb) +
                                  (size_t)kMaxTopk * slot_bytes(dsg, true, eb));
    }
    // one-sided adjoint: both vectors of every pick of every layer
    need = std::max(need, pick_vector_bytes(p, kMaxTopk));
    // persistent: team counters, then the slots of the blocked layers
    need = std::max(need, pers_counter_bytes(p) + p.pers_slots_total);
    // persistent sigma gradient: counters, compact outputs of every layer, slots
    {
        size_t g = align_up(sizeof(int32_t) * (4 * (size_t)kMaxTopk * p.layers.size() + 4));
        for (size_t i = 0; i < p.layers.size(); ++i)
            g += sel_bytes(p.layers[i], eb) + (size_t)kMaxTopk * slot_bytes(p.desc_gsel[i], true, eb);
        need = std::max(need, g);
    }
    // team counters of the blocked kernel precede its slots
    return kAlign + kCounterBytes + align_up(need);
}

int validate_layer(const lfa_layer& l) {
    if (l.c_out <= 0 || l.c_in <= 0 || l.kh <= 0 || l.kw <= 0 || l.n <= 0 || l.m <= 0)
        return LFA_ERR_INVALID_ARG;
    if (l.kh > l.n || l.kw > l.m) return LFA_ERR_INVALID_ARG;
    if (std::max(l.c_out, l.c_in) > 64 * kRowsPerLane) return LFA_ERR_UNSUPPORTED;
    if (std::min(l.c_out, l.c_in) > kMaxR) return LFA_ERR_UNSUPPORTED;
    if (l.kh * l.kw > kMaxTaps) return LFA_ERR_UNSUPPORTED;
    const long long hw = (long long)l.n * l.m;
    if (hw > (1LL << 30) || (long long)l.c_out * l.c_in > (1LL << 24)) return LFA_ERR_UNSUPPORTED;
    return LFA_OK;
}

// Work list of the persistent launch, per chunk of layers.  Cost model (work
// units N^2 M per symbol, times 1.5 with vectors): a wave of the register
// kernel takes ~7.5 ns per unit; a 256-thread work-group of the blocked
// kernel ~2.5 ns per unit, and a team of W ~2.5 ns (1 + 0.08 W) / W per unit
// (barrier overhead, measured on MI355X).  Each blocked layer gets the
// smallest team size whose symbol time does not exceed the chunk's average
// load per work-group; units (teams, bundles) are then listed longest first
// with the members of a team consecutive.
void build_schedule(lfa_plan* p) {
    const int eb = elem_bytes(p->dtype);
    const bool wu = p->flags & LFA_WANT_U, wv = p->flags & LFA_WANT_V;
    const int nl = (int)p->layers.size();
    p->items.clear();
    p->chunk_first.clear();
    p->pers_lds.clear();
    p->pers_grid.clear();
    // waves per work-group that run bundles: as many as LDS allows (<= 4)
    size_t wmax = 0;
    for (int i = 0; i < nl; ++i)
        if (p->desc_pers[i].kind == 1)
            wmax = std::max(wmax, lfa::wave_bundle_lds_for(p->desc_pers[i].wave_nc, p->desc_pers[i].wave_ml, eb,
                                                           wu || wv));
    p->pers_wave_slots = wmax ? (int)std::max<size_t>(1, std::min<size_t>(4, kLdsCap / wmax)) : 4;
    for (int l0 = 0; l0 < nl; l0 += kMaxLaunchLayers) {
        const int l1 = std::min(nl, l0 + kMaxLaunchLayers);
        p->chunk_first.push_back((int)p->items.size());
        const bool acc_any = p->pers_acc;
        const size_t lds = persistent_lds_bytes(p->desc_pers.data() + l0, l1 - l0, acc_any, wu || wv, eb,
                                                p->pers_wave_slots);
        int grid = persistent_resident(lds, eb, acc_any);
        if (grid <= 0) grid = std::max(1, p->num_cus);
        p->pers_lds.push_back(lds);
        p->pers_grid.push_back(grid);
        struct Unit {
            double dur;
            int layer, kind, item, W;
        };
        std::vector<Unit> units;
        double total = 0;
        std::vector<double> sym_cost(l1 - l0, 0.0);
        for (int i = l0; i < l1; ++i) {
            const LayerDesc& d = p->desc_pers[i];
            const double u = double(d.N) * d.N * d.M * (accumulates(d, wu, wv) ? 1.5 : 1.0);
            if (d.kind == 1) {
                const int spw = 64 / d.wave_ml, per = spw * p->pers_wave_slots;
                const double dur = p->cost_wave * u * spw;
                for (int it = 0; it < d.num_canon; it += per) total += dur;
            } else {
                sym_cost[i - l0] = p->cost_block * u;
                total += sym_cost[i - l0] * d.num_canon;
            }
        }
        const double avg = total / grid;
        int team = 0;
        for (int i = l0; i < l1; ++i) {
            const LayerDesc& d = p->desc_pers[i];
            if (d.kind == 1) {
                const int spw = 64 / d.wave_ml, per = spw * p->pers_wave_slots;
                const double u = double(d.N) * d.N * d.M;
                for (int it = 0; it < d.num_canon; it += per)
                    units.push_back({p->cost_wave * u * spw, i - l0, 0, it, 1});
            } else {
                const int NB = (d.N + kBlockCols - 1) / kBlockCols, NBP = NB + (NB & 1);
                const double c = sym_cost[i - l0];
                int W = 1;
                while (W < NBP / 2 && W < grid && c * (1 + p->team_ovh * W) / W > avg) ++W;
                for (int it = 0; it < d.num_canon; ++it)
                    units.push_back({c * (1 + p->team_ovh * W) / W, i - l0, 1, it, W});
            }
        }
        std::stable_sort(units.begin(), units.end(),
                         [](const Unit& x, const Unit& y) { return x.dur > y.dur; });
        for (const Unit& un : units) {
            if (un.kind == 0) {
                p->items.push_back(WorkItem{un.layer, 0, un.item, 0, 1, 0});
            } else {
                for (int m = 0; m < un.W; ++m)
                    p->items.push_back(WorkItem{un.layer, 1, un.item, m, un.W, team});
                ++team;
            }
        }
    }
    p->chunk_first.push_back((int)p->items.size());
}

// The persistent work list to the device.  An earlier list stays allocated
// until the plan is destroyed: graphs captured before it was replaced (by
// lfa_autotune) still point at it.
int upload_items(lfa_plan* p) {
    if (p->items_dev) {
        p->old_items.push_back(p->items_dev);
        p->items_dev = nullptr;
    }
    HIP_TRY(hipMalloc(&p->items_dev, std::max<size_t>(1, p->items.size()) * sizeof(WorkItem)));
    if (!p->items.empty())
        HIP_TRY(hipMemcpy(p->items_dev, p->items.data(), p->items.size() * sizeof(WorkItem),
                          hipMemcpyHostToDevice));
    return LFA_OK;
}

// A stream that is capturing a graph: uploads (hipMalloc, synchronous
// copies) are not allowed there.
bool capturing(hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

// Upload device tables on the plan's first use on the current device (or
// in lfa_plan_create / lfa_plan_prepare).  A compute call whose stream is
// capturing gets LFA_ERR_NOT_PREPARED instead of an upload.
int ensure_device(lfa_plan* p, hipStream_t st = nullptr, bool check_capture = false) {
    std::lock_guard<std::mutex> lock(p->mu);
    int dev = -1;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) {
        g_last_hip = (int)e;
        return LFA_ERR_NO_DEVICE;
    }
    HIP_TRY(hipGetDevice(&dev));
    if (p->device >= 0) return p->device == dev ? LFA_OK : LFA_ERR_INVALID_ARG;
    if (check_capture && capturing(st)) return LFA_ERR_NOT_PREPARED;
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return LFA_ERR_NO_DEVICE;
    p->num_cus = prop.multiProcessorCount;
    HIP_TRY(hipMalloc(&p->tw_dev, p->tw_host.size() * sizeof(double)));
    HIP_TRY(hipMemcpy(p->tw_dev, p->tw_host.data(), p->tw_host.size() * sizeof(double),
                      hipMemcpyHostToDevice));
    // Devices reporting less LDS than the plan assumed: move layers to global slots.
    const size_t lds_dev = prop.sharedMemPerBlock;
    const int eb = elem_bytes(p->dtype);
    const bool wu = p->flags & LFA_WANT_U, wv = p->flags & LFA_WANT_V;
    for (size_t i = 0; i < p->layers.size(); ++i) {
        LayerDesc& d = p->desc[i];
        if (d.kind == 1) {
            d.wave_cap = wave_blocks_per_cu(d.wave_nc, d.wave_ml, eb, d.threads, wu || wv) * p->num_cus;
            if (d.wave_qgroups > 0)
                d.wave_qcap =
                    wave_queue_blocks_per_cu(d.wave_nc, d.wave_ml, eb, d.threads, wu || wv) * p->num_cus;
        }
        if (lds_bytes_for(p->desc[i], accumulates(p->desc[i], wu, wv), eb) > lds_dev)
            p->desc[i].storage = kGlobal;
        {
            LayerDesc& dr = p->desc_r[i];
            const bool vec = false;          // the SVD of the factors never accumulates
            if (dr.kind == 1) {
                dr.wave_cap = wave_blocks_per_cu(dr.wave_nc, dr.wave_ml, eb, dr.threads, vec) * p->num_cus;
                if (dr.wave_qgroups > 0)
                    dr.wave_qcap = wave_queue_blocks_per_cu(dr.wave_nc, dr.wave_ml, eb, dr.threads, vec) * p->num_cus;
            }
            if (lds_bytes_for(dr, vec, eb) > lds_dev) dr.storage = kGlobal;
        }
        if (lds_bytes_for(p->desc_sel[i], true, eb) > lds_dev) p->desc_sel[i].storage = kGlobal;
        if (lds_bytes_for(p->desc_pers[i], accumulates(p->desc_pers[i], wu, wv), eb) > lds_dev)
            p->desc_pers[i].storage = kGlobal;
    }
    build_schedule(p);
    LFA_TRY(upload_items(p));
    p->device = dev;
    return LFA_OK;
}

template <typename R>
int run_svd_layer(const lfa_plan* p, const LayerDesc& d, const void* W, const void* A,
                  void* sigma, void* U, void* V, int32_t* info, char* region,
                  const int32_t* theta_list, int theta_stride, int theta_count,
                  hipStream_t st, bool canon = false, bool queue_ok = true,
                  const LayerTune* tn = nullptr) {
    SvdArgs<R> a{};
    a.d = d;
    a.canon = theta_list ? 0 : (canon ? 1 : 0);
    a.W = static_cast<const R*>(W);
    a.A = static_cast<const cplx<R>*>(A);
    a.sigma = static_cast<R*>(sigma);
    a.U = static_cast<cplx<R>*>(U);
    a.V = static_cast<cplx<R>*>(V);
    a.info = info;
    a.tw = p->tw_dev;
    a.theta_list = theta_list;
    a.theta_stride = theta_stride;
    a.theta_count = theta_count;
    a.theta_dedup = theta_list != nullptr && theta_stride == 3;   // top-k picks
    a.max_sweeps = p->max_sweeps;
    a.tol = jacobi_tol(p->tol, d.M);
    a.phase = d.kind == 1 ? p->phase_rec : nullptr;
    const bool acc = (d.transposed ? U : V) != nullptr;
    const int count = item_count(a);
    if (count <= 0) return LFA_OK;
    hipError_t e;
    if (d.kind == 1) {
        if (acc != (d.threads > 64)) return LFA_ERR_INVALID_ARG;   // shape made for other outputs
        const int groups = wave_groups(d, count);
        const int force = (tn && tn->queue_seg >= 0) ? tn->queue_seg : p->wq_force;
        const int seg = queue_ok ? wave_queue_seg(d, groups, force) : 0;
        if (seg > 0) {
            // work queue in the region: control words and entries, meta, state
            const long long ents = wave_queue_entries(groups, seg);
            char* q = region;
            a.wq = reinterpret_cast<int32_t*>(q);
            q += align_up(sizeof(int32_t) * (kWaveQueueCtl + wave_queue_entries(d.wave_qgroups, 1)));
            a.wq_meta = reinterpret_cast<int32_t*>(q);
            q += align_up(sizeof(int32_t) * kWaveMeta * (size_t)d.wave_qgroups);
            a.wq_state = q;
            a.wq_cap = (int)ents;
            a.wq_seg = seg;
            HIP_TRY(launch_fill_i32(a.wq, 0, kWaveQueueCtl + ents, st));
            const int grid = std::min(groups, d.wave_qcap);
            if constexpr (sizeof(R) == 4) e = launch_wave_queue_f32(a, grid, st);
            else e = launch_wave_queue_f64(a, grid, st);
            HIP_TRY(e);
            return LFA_OK;
        }
        int grid = groups;
        if (d.wave_cap > 0 && groups <= kWaveTurnRounds * d.wave_cap) {
            // resident work-groups take the groups in turn from a counter at
            // the start of the region (a few rounds of groups: there the
            // hardware's dispatch order leaves CUs idle in the last rounds;
            // with many rounds, one work-group per group measured faster)
            a.wctr = reinterpret_cast<int32_t*>(region);
            HIP_TRY(launch_fill_i32(a.wctr, 0, 1, st));
            grid = std::min(groups, d.wave_cap);
        }
        if constexpr (sizeof(R) == 4) e = launch_wave_svd_f32(a, grid, st);
        else e = launch_wave_svd_f64(a, grid, st);
        HIP_TRY(e);
        return LFA_OK;
    }
    a.slot_bytes = (long long)slot_bytes(d, acc, sizeof(R));
    a.gws = d.storage == kGlobal ? region : nullptr;
    if (d.kind == 2) {
        // Teams of W work-groups share one symbol's block pairs when there
        // are too few symbols to fill the device; W > 1 requires every
        // work-group of the grid to be resident at once.
        // Each team barrier writes back the L2 of the arriving work-group, so
        // teams pay off only while they give work-groups CUs of their own:
        // W is about (CUs / symbols), never more than the grid can hold.
        const int resident = block_resident(d, acc, sizeof(R));
        const int NB = (d.N + kBlockCols - 1) / kBlockCols, NBP = NB + (NB & 1);
        int W = 1, teams = std::min(count, kGlobalGrid);
        const int cap = std::min(resident, p->num_cus);
        const bool forced = tn && tn->team_w > 0;
        if (forced) {
            // the autotuner's width: teams of W only as many as can be
            // resident at once (every member of a team must be)
            W = std::max(1, std::min({tn->team_w, NBP / 2, resident}));
            teams = W > 1 ? std::max(1, std::min(count, resident / W)) : teams;
        } else if (cap >= 2 && 2 * count <= cap) {
            W = std::max(1, std::min(NBP / 2, cap / count));
            teams = W > 1 ? std::min(count, cap / W) : teams;
        } else if (count < cap && 2 * count <= resident && NBP >= 4) {
            // between half a device and a device of symbols: pairs, a few
            // CUs holding two work-groups, instead of half the CUs idle
            W = 2;
            teams = count;
        }
        int32_t* counters = reinterpret_cast<int32_t*>(region);
        a.gws = region + kCounterBytes;
        // More symbols than resident work-groups: the whole rounds run one
        // work-group per symbol, and a short last round (at most half the
        // device) runs in teams instead of leaving the other CUs idle for a
        // whole symbol time.  The teams join the same grid when the slots
        // allow (they start on the CUs that the earliest finished symbols
        // free), else they follow as a launch of their own.
        int split = count;
        int W2 = 1, teams2 = 0;
        const int rem = resident > 0 ? count % resident : 0;
        if (!forced && W == 1 && cap >= 2 && count > resident && rem > 0 && 2 * rem <= cap) {
            W2 = std::max(1, std::min(NBP / 2, cap / rem));
            if (W2 > 1) {
                split = count - rem;
                teams2 = rem;
                teams = std::min(split, kGlobalGrid);
            }
        }
        auto launch = [&](int tm, int w, int i0, int i1, int tm2, int w2, int i2) {
            if constexpr (sizeof(R) == 4) return launch_block_svd_f32(a, tm, w, i0, i1, tm2, w2, i2, counters, st);
            else return launch_block_svd_f64(a, tm, w, i0, i1, tm2, w2, i2, counters, st);
        };
        if (teams2 > 0 && teams + teams2 <= svd_grid(d, d.num_symbols)) {
            HIP_TRY(launch(teams, W, 0, split, teams2, W2, count));
        } else {
            HIP_TRY(launch(teams, W, 0, split, 0, 1, split));
            if (teams2 > 0) HIP_TRY(launch(teams2, W2, split, count, 0, 1, count));
        }
        return LFA_OK;
    }
    // every layer description is of the register (M <= 64) or the blocked kind
    return LFA_ERR_UNSUPPORTED;
}

// Workspace bytes lfa_svd itself uses on the plan's device (desc as
// adjusted at upload), with or without the register kernel's work queue.
size_t svd_need(const lfa_plan& p, bool queue) {
    size_t need = 0;
    for (size_t i = 0; i < p.layers.size(); ++i)
        need = std::max(need, svd_layer_need(p, i, p.qr[i] != 0, layer_materialized(p, i), queue, false));
    return kAlign + kCounterBytes + align_up(need);
}

int check_ws(const lfa_plan* p, void* ws, size_t ws_bytes) {
    const size_t need = workspace_bytes(*p);
    if (need > kAlign && (ws == nullptr || ws_bytes < need)) return LFA_ERR_WORKSPACE;
    return LFA_OK;
}

// One layer of lfa_svd (the caller clears the info words).  `region` is the
// workspace after its first kAlign bytes.
template <typename R>
int svd_layer(const lfa_plan* p, size_t i, const void* const* W, const void* const* A, void* const* sigma,
              void* const* U, void* const* V, int32_t* info, char* region, hipStream_t st, bool queue_ok) {
    const bool wu = p->flags & LFA_WANT_U, wv = p->flags & LFA_WANT_V;
    const LayerTune* tn = &p->tune[i];
    {
        const LayerDesc& d = p->desc[i];
        const void* Wi = nullptr;
        const void* Ai = A ? A[i] : nullptr;
        char* slots = region;
        const bool mat = layer_materialized(*p, i);
        if (!A) {
            if (mat) {
                cplx<float>* sym = reinterpret_cast<cplx<float>*>(region);
                // only the canonical symbols: the SVD below takes one per
                // conjugate pair (real weights)
                HIP_TRY(launch_symbols_mfma(d, static_cast<const float*>(W[i]), sym, p->tw_dev,
                                            asm_materialized(p->flags) ? asm_mode(p->flags) : 0, st, true));
                Ai = sym;
                slots = region + symbols_bytes(p->layers[i], sizeof(R));
            } else {
                Wi = W[i];
            }
        }
        if (!A && !mat && p->qr[i]) {
            // QR preconditioning: the Cholesky factors R of the Gram
            // matrices, then the SVD of the N x N factors (one per conjugate
            // pair; the mirror's factor is the conjugate)
            const lfa_layer& l = p->layers[i];
            char* rsym = region;
            double* taps = reinterpret_cast<double*>(rsym + qr_rsym_bytes(l, sizeof(R)));
            char* rest = reinterpret_cast<char*>(taps) + qr_taps_bytes(l);
            GramArgs<R> g{};
            g.W = static_cast<const R*>(W[i]);
            g.c_out = l.c_out;
            g.c_in = l.c_in;
            g.kh = l.kh;
            g.kw = l.kw;
            g.n = l.n;
            g.m = l.m;
            g.M = d.M;
            g.N = d.N;
            g.transposed = d.transposed;
            g.tw_n = d.tw_n;
            g.tw_m = d.tw_m;
            g.tw = p->tw_dev;
            g.C = taps;
            g.hslots = rest;
            g.Rsym = reinterpret_cast<cplx<R>*>(rsym);
            g.conj_transpose = (wu || wv) ? 1 : 0;
            hipError_t e;
            if constexpr (sizeof(R) == 4) e = launch_gram_qr_f32(g, d.num_canon, st);
            else e = launch_gram_qr_f64(g, d.num_canon, st);
            HIP_TRY(e);
            const bool vec = wu || wv;
            // with vectors the factors are R^H = V_R S U_R^H: its SVD needs no
            // rotation accumulator and writes its left singular vectors, V_R,
            // over the factors (each work-group reads its own canonical factor
            // before it writes that frequency and its mirror)
            LFA_TRY(run_svd_layer<R>(p, p->desc_r[i], nullptr, rsym, sigma[i],
                                     vec ? reinterpret_cast<cplx<R>*>(rsym) : nullptr, nullptr,
                                     info ? info + i * LFA_INFO_WORDS : nullptr, rest, nullptr, 0, 0, st,
                                     true, queue_ok, tn));
            if (vec) {
                QrVecArgs<R> q{};
                q.W = static_cast<const R*>(W[i]);
                q.c_out = l.c_out;
                q.c_in = l.c_in;
                q.kh = l.kh;
                q.kw = l.kw;
                q.n = l.n;
                q.m = l.m;
                q.M = d.M;
                q.N = d.N;
                q.transposed = d.transposed;
                q.tw_n = d.tw_n;
                q.tw_m = d.tw_m;
                q.tw = p->tw_dev;
                q.VR = reinterpret_cast<const cplx<R>*>(rsym);
                q.sigma = static_cast<const R*>(sigma[i]);
                q.slots = rsym + qr_rsym_bytes(l, sizeof(R));
                q.slot_bytes = (long long)qr_vec_slot_bytes(d, sizeof(R));
                q.ldg = d.ldg;
                q.ldv = d.ldv;
                SvdArgs<R> a{};
                a.d = d;
                a.d.storage = kGlobal;
                a.canon = 1;
                a.sigma = static_cast<R*>(sigma[i]);
                a.U = wu ? static_cast<cplx<R>*>(U[i]) : nullptr;
                a.V = wv ? static_cast<cplx<R>*>(V[i]) : nullptr;
                a.tw = p->tw_dev;
                a.gws = q.slots;
                a.slot_bytes = q.slot_bytes;
                if constexpr (sizeof(R) == 4) e = launch_qr_vectors_f32(q, a, d.num_canon, st);
                else e = launch_qr_vectors_f64(q, a, d.num_canon, st);
                HIP_TRY(e);
            }
            return LFA_OK;
        }
        // weights are real: decompose one symbol per conjugate pair.  Symbols
        // handed in by the caller carry no such guarantee.
        const bool canon = A == nullptr;
        LFA_TRY(run_svd_layer<R>(p, d, Wi, Ai, sigma[i], wu ? U[i] : nullptr,
                                 wv ? V[i] : nullptr,
                                 info ? info + i * LFA_INFO_WORDS : nullptr, slots, nullptr, 0, 0,
                                 st, canon, queue_ok, tn));
    }
    return LFA_OK;
}

// LFA_PHASE_NORMALIZE: the phase pass over every layer's written vectors
// (every frequency, mirrors included).
template <typename R>
int phase_pass(const lfa_plan* p, void* const* U, void* const* V, hipStream_t st) {
    if (!(p->flags & LFA_PHASE_NORMALIZE)) return LFA_OK;
    const bool wu = p->flags & LFA_WANT_U, wv = p->flags & LFA_WANT_V;
    for (size_t i = 0; i < p->layers.size(); ++i) {
        const lfa_layer& l = p->layers[i];
        const int r = std::min(l.c_out, l.c_in);
        cplx<R>* u = wu ? static_cast<cplx<R>*>(U[i]) : nullptr;
        cplx<R>* v = wv ? static_cast<cplx<R>*>(V[i]) : nullptr;
        hipError_t e;
        if constexpr (sizeof(R) == 4) e = launch_phase_normalize_f32(u, v, l.n * l.m, l.c_out, l.c_in, r, st);
        else e = launch_phase_normalize_f64(u, v, l.n * l.m, l.c_out, l.c_in, r, st);
        HIP_TRY(e);
    }
    return LFA_OK;
}

template <typename R>
int svd_impl(const lfa_plan* p, const void* const* W, const void* const* A, void* const* sigma,
             void* const* U, void* const* V, int32_t* info, void* ws, size_t ws_bytes,
             hipStream_t st, bool queue_ok = true) {
    (void)ws_bytes;
    char* region = static_cast<char*>(ws) + kAlign;
    if (info) HIP_TRY(launch_fill_i32(info, 0, (long long)p->layers.size() * LFA_INFO_WORDS, st));
    for (size_t i = 0; i < p->layers.size(); ++i)
        LFA_TRY(svd_layer<R>(p, i, W, A, sigma, U, V, info, region, st, queue_ok));
    return phase_pass<R>(p, U, V, st);
}

int check_ptrs(const lfa_plan* p, const void* const* arr, bool required) {
    if (!required) return LFA_OK;
    if (!arr) return LFA_ERR_INVALID_ARG;
    for (size_t i = 0; i < p->layers.size(); ++i)
        if (!arr[i]) return LFA_ERR_INVALID_ARG;
    return LFA_OK;
}

template <typename R>
int persistent_impl(const lfa_plan* p, const void* const* W, void* const* sigma, void* const* U,
                    void* const* V, int32_t* info, void* ws, hipStream_t st, long long* busy = nullptr) {
    const bool wu = p->flags & LFA_WANT_U, wv = p->flags & LFA_WANT_V;
    int32_t* counter = static_cast<int32_t*>(ws);
    char* region = static_cast<char*>(ws) + kAlign;
    int32_t* team_counters = reinterpret_cast<int32_t*>(region);
    char* slots = region + pers_counter_bytes(*p);
    if (info) HIP_TRY(launch_fill_i32(info, 0, (long long)p->layers.size() * LFA_INFO_WORDS, st));
    const int nl = (int)p->layers.size();
    // one launch per chunk of kMaxLaunchLayers layers (kernel-argument limit)
    for (int l0 = 0, chunk = 0; l0 < nl; l0 += kMaxLaunchLayers, ++chunk) {
        const int l1 = std::min(nl, l0 + kMaxLaunchLayers);
        PersistentArgs<R> pa{};
        pa.num_layers = l1 - l0;
        pa.threads = kPersistentThreads;
        for (int i = l0; i < l1; ++i) {
            const LayerDesc& d = p->desc_pers[i];
            const bool acc = p->pers_acc;   // as the plan sized the slots
            SvdArgs<R>& a = pa.layer[i - l0];
            a.d = d;
            a.W = static_cast<const R*>(W[i]);
            a.sigma = static_cast<R*>(sigma[i]);
            a.U = wu ? static_cast<cplx<R>*>(U[i]) : nullptr;
            a.V = wv ? static_cast<cplx<R>*>(V[i]) : nullptr;
            a.info = info ? info + i * LFA_INFO_WORDS : nullptr;
            a.tw = p->tw_dev;
            a.max_sweeps = p->max_sweeps;
            a.tol = jacobi_tol(p->tol, d.M);
            a.canon = 1;
            if (d.kind == 2) {
                a.slot_bytes = (long long)slot_bytes(d, acc, sizeof(R));
                a.gws = slots + p->pers_slot_off[i];
            }
        }
        const int first = p->chunk_first[chunk];
        const int count = p->chunk_first[chunk + 1] - first;
        if (count == 0) continue;
        pa.items = p->items_dev + first;
        pa.num_items = count;
        pa.counter = counter;
        pa.team_counters = team_counters;
        pa.num_teams = p->pers_teams;
        pa.busy = busy;
        pa.wave_slots = p->pers_wave_slots;
        pa.wave_lds = (int)(p->pers_wave_slots ? p->pers_lds[chunk] / p->pers_wave_slots : 0);
        // per-wave LDS stride: the largest bundle region of the chunk
        size_t wl = 0;
        for (int i = l0; i < l1; ++i)
            if (p->desc_pers[i].kind == 1)
                wl = std::max(wl, wave_bundle_lds_for(p->desc_pers[i].wave_nc, p->desc_pers[i].wave_ml,
                                                     (int)sizeof(R), wu || wv));
        pa.wave_lds = (int)wl;
        HIP_TRY(launch_fill_i32(counter, 0, 1, st));
        HIP_TRY(launch_fill_i32(team_counters, 0, 4LL * p->pers_teams + 4, st));
        const int grid = std::min(p->pers_grid[chunk], count);
        hipError_t e;
        if constexpr (sizeof(R) == 4) e = launch_persistent_f32(pa, grid, p->pers_lds[chunk], p->pers_acc, st);
        else e = launch_persistent_f64(pa, grid, p->pers_lds[chunk], p->pers_acc, st);
        HIP_TRY(e);
    }
    return phase_pass<R>(p, U, V, st);
}

}  // namespace

// ---------------------------------------------------------------------------
// Selected-symbol SVD + adjoint (sigma gradient)
// ---------------------------------------------------------------------------
namespace {

template <typename R>
int adjoint_launch(const lfa_plan* p, int l0, int l1, const void* const* U, const void* const* V,
                   const int32_t* idx, const void* grad, int k, void* const* dW, int compact,
                   hipStream_t st) {
    AdjointArgs<R> a{};
    a.num_layers = l1 - l0;
    a.k = k;
    a.compact = compact;
    a.idx = idx + (size_t)l0 * k * 3;
    a.grad = static_cast<const R*>(grad) + (size_t)l0 * k;
    a.tw = p->tw_dev;
    int blocks = 0;
    for (int i = l0; i < l1; ++i) {
        const lfa_layer& l = p->layers[i];
        const int j = i - l0;
        a.c_out[j] = l.c_out;
        a.c_in[j] = l.c_in;
        a.kh[j] = l.kh;
        a.kw[j] = l.kw;
        a.n[j] = l.n;
        a.m[j] = l.m;
        a.tw_n[j] = p->tw_n[i];
        a.tw_m[j] = p->tw_m[i];
        a.U[j] = static_cast<const cplx<R>*>(U[compact ? j : i]);
        a.V[j] = static_cast<const cplx<R>*>(V[compact ? j : i]);
        a.dW[j] = static_cast<R*>(dW[i]);
        a.blocks_before[j] = blocks;
        blocks += (l.c_out * l.c_in + 255) / 256;
    }
    a.blocks_before[l1 - l0] = blocks;
    hipError_t e;
    if constexpr (sizeof(R) == 4) e = launch_adjoint_f32(a, st);
    else e = launch_adjoint_f64(a, st);
    HIP_TRY(e);
    return LFA_OK;
}

template <typename R>
int sigma_grad_impl(const lfa_plan* p, const void* const* W, const int32_t* idx, const void* grad,
                    int k, void* const* dW, void* ws, hipStream_t st) {
    char* region = static_cast<char*>(ws) + kAlign;
    const int eb = sizeof(R);
    // Layers one after the other, reusing one compact buffer: SVD with
    // vectors of the k selected symbols, then the adjoint of the layer.
    for (size_t i = 0; i < p->layers.size(); ++i) {
        const lfa_layer& l = p->layers[i];
        const LayerDesc& d = p->desc_sel[i];
        const size_t r = std::min(l.c_out, l.c_in);
        char* sig = region;
        char* Uc = sig + align_up((size_t)k * r * eb);
        char* Vc = Uc + align_up((size_t)k * l.c_out * r * 2 * eb);
        char* slots = region + sel_bytes(l, eb);
        LFA_TRY(run_svd_layer<R>(p, d, W[i], nullptr, sig, Uc, Vc, nullptr, slots,
                                 idx + (size_t)i * k * 3, 3, k, st));
        const void* Ua[1] = {Uc};
        const void* Va[1] = {Vc};
        LFA_TRY(adjoint_launch<R>(p, (int)i, (int)i + 1, Ua, Va, idx, grad, k, dW, 1, st));
    }
    return LFA_OK;
}

template <typename R>
int topk_impl(const lfa_plan* p, const void* const* sigma, int k, void* vals, int32_t* idx,
              hipStream_t st) {
    const int nl = (int)p->layers.size();
    for (int l0 = 0; l0 < nl; l0 += kMaxLaunchLayers) {
        const int l1 = std::min(nl, l0 + kMaxLaunchLayers);
        TopkArgs<R> a{};
        a.num_layers = l1 - l0;
        a.k = k;
        a.vals = static_cast<R*>(vals) + (size_t)l0 * k;
        a.idx = idx + (size_t)l0 * k * 3;
        for (int i = l0; i < l1; ++i) {
            a.sigma[i - l0] = static_cast<const R*>(sigma[i]);
            a.n[i - l0] = p->layers[i].n;
            a.m[i - l0] = p->layers[i].m;
            a.r[i - l0] = std::min(p->layers[i].c_out, p->layers[i].c_in);
        }
        hipError_t e;
        if constexpr (sizeof(R) == 4) e = launch_topk_f32(a, st);
        else e = launch_topk_f64(a, st);
        HIP_TRY(e);
    }
    return LFA_OK;
}

// Work list of the persistent SVD of the k selected symbols of every layer
// (with vectors, blocked kernel), same cost model as build_schedule.
// The schedule for k, built and uploaded on first use.  `out` points into
// the plan's map, whose nodes never move or change once inserted; the lookup
// itself runs under the plan's lock.
int ensure_grad_schedule(lfa_plan* p, int k, hipStream_t st, bool check_capture,
                         const lfa_plan::GradSched** out) {
    std::lock_guard<std::mutex> lock(p->mu);
    auto it = p->grad_sched.find(k);
    if (it != p->grad_sched.end()) {
        if (out) *out = &it->second;
        return LFA_OK;
    }
    if (check_capture && capturing(st)) return LFA_ERR_NOT_PREPARED;
    lfa_plan::GradSched gs;
    const int eb = elem_bytes(p->dtype);
    const int nl = (int)p->layers.size();
    std::vector<WorkItem> items;
    for (int l0 = 0; l0 < nl; l0 += kMaxLaunchLayers) {
        const int l1 = std::min(nl, l0 + kMaxLaunchLayers);
        gs.chunk_first.push_back((int)items.size());
        const size_t lds = persistent_lds_bytes(p->desc_gsel.data() + l0, l1 - l0, true, false, eb, 1);
        int grid = persistent_resident(lds, eb, true);
        if (grid <= 0) grid = std::max(1, p->num_cus);
        gs.lds.push_back(lds);
        gs.grid.push_back(grid);
        double total = 0;
        for (int i = l0; i < l1; ++i) {
            const LayerDesc& d = p->desc_gsel[i];
            total += p->cost_block * 1.5 * double(d.N) * d.N * d.M * k;
        }
        const double avg = total / grid;
        struct Unit {
            double dur;
            int layer, item, W;
        };
        std::vector<Unit> units;
        for (int i = l0; i < l1; ++i) {
            const LayerDesc& d = p->desc_gsel[i];
            const int NB = (d.N + kBlockCols - 1) / kBlockCols, NBP = NB + (NB & 1);
            const double c = p->cost_block * 1.5 * double(d.N) * d.N * d.M;
            int W = 1;
            while (W < NBP / 2 && W < grid && c * (1 + p->team_ovh * W) / W > avg) ++W;
            for (int s = 0; s < k; ++s) units.push_back({c * (1 + p->team_ovh * W) / W, i - l0, s, W});
        }
        std::stable_sort(units.begin(), units.end(),
                         [](const Unit& x, const Unit& y) { return x.dur > y.dur; });
        int team = 0;
        for (const Unit& un : units) {
            for (int m = 0; m < un.W; ++m) items.push_back(WorkItem{un.layer, 1, un.item, m, un.W, team});
            ++team;
        }
        gs.teams = std::max(gs.teams, team);
    }
    gs.chunk_first.push_back((int)items.size());
    HIP_TRY(hipMalloc(&gs.items_dev, std::max<size_t>(1, items.size()) * sizeof(WorkItem)));
    if (!items.empty())
        HIP_TRY(hipMemcpy(gs.items_dev, items.data(), items.size() * sizeof(WorkItem),
                          hipMemcpyHostToDevice));
    auto ins = p->grad_sched.emplace(k, gs).first;
    if (out) *out = &ins->second;
    return LFA_OK;
}

// Sigma gradient in two launches: one persistent SVD-with-vectors of the
// selected symbols of all layers (compact outputs), then one adjoint launch.
template <typename R>
int sigma_grad_persistent_impl(const lfa_plan* p, const lfa_plan::GradSched& gs, const void* const* W,
                               const int32_t* idx, const void* grad, int k, void* const* dW, void* ws,
                               hipStream_t st) {
    const int nl = (int)p->layers.size();
    const int eb = sizeof(R);
    int32_t* counter = static_cast<int32_t*>(ws);
    char* region = static_cast<char*>(ws) + kAlign;
    int32_t* team_counters = reinterpret_cast<int32_t*>(region);
    char* cur = region + align_up(sizeof(int32_t) * (4 * (size_t)kMaxTopk * nl + 4));
    std::vector<void*> sig(nl), Uc(nl), Vc(nl);
    std::vector<char*> slot(nl);
    for (int i = 0; i < nl; ++i) {
        const lfa_layer& l = p->layers[i];
        const size_t r = std::min(l.c_out, l.c_in);
        sig[i] = cur;
        Uc[i] = cur + align_up((size_t)k * r * eb);
        Vc[i] = (char*)Uc[i] + align_up((size_t)k * l.c_out * r * 2 * eb);
        cur += sel_bytes(l, eb);
    }
    for (int i = 0; i < nl; ++i) {
        slot[i] = cur;
        cur += (size_t)k * slot_bytes(p->desc_gsel[i], true, eb);
    }
    for (int l0 = 0, chunk = 0; l0 < nl; l0 += kMaxLaunchLayers, ++chunk) {
        const int l1 = std::min(nl, l0 + kMaxLaunchLayers);
        PersistentArgs<R> pa{};
        pa.num_layers = l1 - l0;
        pa.threads = kPersistentThreads;
        for (int i = l0; i < l1; ++i) {
            const LayerDesc& d = p->desc_gsel[i];
            SvdArgs<R>& a = pa.layer[i - l0];
            a.d = d;
            a.W = static_cast<const R*>(W[i]);
            a.sigma = static_cast<R*>(sig[i]);
            // vectors of A: U (c_out x r), V (c_in x r), whichever side accumulates
            a.U = static_cast<cplx<R>*>(Uc[i]);
            a.V = static_cast<cplx<R>*>(Vc[i]);
            a.tw = p->tw_dev;
            a.max_sweeps = p->max_sweeps;
            a.tol = jacobi_tol(p->tol, d.M);
            a.theta_list = idx + (size_t)i * k * 3;
            a.theta_stride = 3;
            a.theta_count = k;
            a.theta_dedup = 1;
            a.slot_bytes = (long long)slot_bytes(d, true, eb);
            a.gws = slot[i];
        }
        const int first = gs.chunk_first[chunk];
        const int count = gs.chunk_first[chunk + 1] - first;
        if (count == 0) continue;
        pa.items = gs.items_dev + first;
        pa.num_items = count;
        pa.counter = counter;
        pa.team_counters = team_counters;
        pa.num_teams = gs.teams;
        pa.wave_slots = 1;
        pa.wave_lds = 0;
        HIP_TRY(launch_fill_i32(counter, 0, 1, st));
        HIP_TRY(launch_fill_i32(team_counters, 0, 4LL * gs.teams + 4, st));
        const int grid = std::min(gs.grid[chunk], count);
        hipError_t e;
        if constexpr (sizeof(R) == 4) e = launch_persistent_f32(pa, grid, gs.lds[chunk], true, st);
        else e = launch_persistent_f64(pa, grid, gs.lds[chunk], true, st);
        HIP_TRY(e);
    }
    for (int l0 = 0; l0 < nl; l0 += kMaxLaunchLayers) {
        const int l1 = std::min(nl, l0 + kMaxLaunchLayers);
        std::vector<const void*> Uv(Uc.begin() + l0, Uc.begin() + l1), Vv(Vc.begin() + l0, Vc.begin() + l1);
        LFA_TRY(adjoint_launch<R>(p, l0, l1, Uv.data(), Vv.data(), idx, grad, k, dW, 1, st));
    }
    return LFA_OK;
}

// Gradient from one side of the picks' singular vectors: the side the
// forward pass kept (U of tall layers, V of wide ones), the other side
// recomputed from W for each pick, then the adjoint on per-pick vectors.
template <typename R>
int adjoint_onesided_impl(const lfa_plan* p, const void* const* W, const void* const* sigma,
                          const void* const* X, const int32_t* idx, const void* grad, int k,
                          void* const* dW, void* ws, hipStream_t st) {
    const int nl = (int)p->layers.size();
    const size_t cb = 2 * sizeof(R);
    char* cur = static_cast<char*>(ws) + kAlign;
    std::vector<void*> Uc(nl), Vc(nl);
    for (int i = 0; i < nl; ++i) {
        const lfa_layer& l = p->layers[i];
        Uc[i] = cur;
        cur += align_up((size_t)k * l.c_out * cb);
        Vc[i] = cur;
        cur += align_up((size_t)k * l.c_in * cb);
    }
    for (int l0 = 0; l0 < nl; l0 += kMaxLaunchLayers) {
        const int l1 = std::min(nl, l0 + kMaxLaunchLayers);
        OtherSideArgs<R> o{};
        o.num_layers = l1 - l0;
        o.k = k;
        o.idx = idx + (size_t)l0 * k * 3;
        o.tw = p->tw_dev;
        for (int i = l0; i < l1; ++i) {
            const lfa_layer& l = p->layers[i];
            const int j = i - l0;
            o.W[j] = static_cast<const R*>(W[i]);
            o.sigma[j] = static_cast<const R*>(sigma[i]);
            o.X[j] = static_cast<const cplx<R>*>(X[i]);
            o.Uc[j] = static_cast<cplx<R>*>(Uc[i]);
            o.Vc[j] = static_cast<cplx<R>*>(Vc[i]);
            o.c_out[j] = l.c_out;
            o.c_in[j] = l.c_in;
            o.kh[j] = l.kh;
            o.kw[j] = l.kw;
            o.n[j] = l.n;
            o.m[j] = l.m;
            o.tw_n[j] = p->tw_n[i];
            o.tw_m[j] = p->tw_m[i];
        }
        hipError_t e;
        if constexpr (sizeof(R) == 4) e = launch_other_side_f32(o, st);
        else e = launch_other_side_f64(o, st);
        HIP_TRY(e);
        std::vector<const void*> Uv(Uc.begin() + l0, Uc.begin() + l1), Vv(Vc.begin() + l0, Vc.begin() + l1);
        LFA_TRY(adjoint_launch<R>(p, l0, l1, Uv.data(), Vv.data(), idx, grad, k, dW, 2, st));
    }
    return LFA_OK;
}

// The side of a layer's singular vectors that its working matrix converges
// to (no accumulator): U when c_out >= c_in, V otherwise.
bool keeps_u(const lfa_layer& l) { return l.c_out >= l.c_in; }

int check_k(const lfa_plan* p, int k) {
    if (k < 1 || k > kMaxTopk) return LFA_ERR_INVALID_ARG;
    for (const lfa_layer& l : p->layers) {
        if ((long long)l.n * l.m * std::min(l.c_out, l.c_in) < k) return LFA_ERR_INVALID_ARG;
        if (k * l.kh * l.kw > 4096) return LFA_ERR_UNSUPPORTED;
    }
    return LFA_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Autotuner: choices timed on the caller's data, kept in a JSON cache
// ---------------------------------------------------------------------------
namespace {

// The cache: {"lfa_autotune": 1, "entries": {key: {field: number, ...}, ...}}.
using CacheEntries = std::map<std::string, std::map<std::string, double>>;

struct JsonIn {
    const std::string& t;
    size_t i = 0;
    explicit JsonIn(const std::string& text) : t(text) {}
    void ws() {
        while (i < t.size() && (t[i] == ' ' || t[i] == '\n' || t[i] == '\r' || t[i] == '\t')) ++i;
    }
    bool eat(char c) {
        ws();
        if (i < t.size() && t[i] == c) {
            ++i;
            return true;
        }
        return false;
    }
    bool str(std::string& out) {
        ws();
        if (i >= t.size() || t[i] != '"') return false;
        ++i;
        out.clear();
        while (i < t.size() && t[i] != '"') {
            if (t[i] == '\\' && i + 1 < t.size()) ++i;     // keys here carry no escapes but '\\' and '"'
            out.push_back(t[i++]);
        }
        return i < t.size() && t[i++] == '"';
    }
    bool num(double& v) {
        ws();
        const char* b = t.c_str() + i;
        char* e = nullptr;
        v = std::strtod(b, &e);
        if (e == b) return false;
        i += (size_t)(e - b);
        return true;
    }
    bool skip() {          // any value
        ws();
        if (i >= t.size()) return false;
        std::string tmp;
        double d;
        if (t[i] == '"') return str(tmp);
        if (t[i] == '{' || t[i] == '[') {
            const char close = t[i] == '{' ? '}' : ']';
            const bool obj = t[i] == '{';
            ++i;
            if (eat(close)) return true;
            do {
                if (obj && !(str(tmp) && eat(':'))) return false;
                if (!skip()) return false;
            } while (eat(','));
            return eat(close);
        }
        for (const char* lit : {"true", "false", "null"})
            if (t.compare(i, std::strlen(lit), lit) == 0) {
                i += std::strlen(lit);
                return true;
            }
        return num(d);
    }
};

// Entries of a cache file; an absent or unreadable file gives none.
CacheEntries read_cache(const char* path) {
    CacheEntries out;
    if (!path || !*path) return out;
    FILE* f = std::fopen(path, "rb");
    if (!f) return out;
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
    std::fclose(f);
    JsonIn in(text);
    std::string key;
    if (!in.eat('{')) return CacheEntries{};
    if (in.eat('}')) return out;
    do {
        if (!(in.str(key) && in.eat(':'))) return CacheEntries{};
        if (key != "entries") {
            if (!in.skip()) return CacheEntries{};
            continue;
        }
        if (!in.eat('{')) return CacheEntries{};
        if (in.eat('}')) continue;
        do {
            std::string ek, fk;
            if (!(in.str(ek) && in.eat(':') && in.eat('{'))) return CacheEntries{};
            std::map<std::string, double> fields;
            if (!in.eat('}')) {
                do {
                    double v;
                    if (!(in.str(fk) && in.eat(':') && in.num(v))) return CacheEntries{};
                    fields[fk] = v;
                } while (in.eat(','));
                if (!in.eat('}')) return CacheEntries{};
            }
            out[ek] = fields;
        } while (in.eat(','));
        if (!in.eat('}')) return CacheEntries{};
    } while (in.eat(','));
    return out;
}

int write_cache(const char* path, const CacheEntries& entries) {
    if (!path || !*path) return LFA_OK;
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return LFA_ERR_INVALID_ARG;
    std::fprintf(f, "{\n \"lfa_autotune\": 1,\n \"entries\": {");
    bool first = true;
    for (const auto& kv : entries) {
        std::fprintf(f, "%s\n  \"%s\": {", first ? "" : ",", kv.first.c_str());
        bool ff = true;
        for (const auto& fv : kv.second) {
            std::fprintf(f, "%s\"%s\": %.9g", ff ? "" : ", ", fv.first.c_str(), fv.second);
            ff = false;
        }
        std::fprintf(f, "}");
        first = false;
    }
    std::fprintf(f, "\n }\n}\n");
    const bool ok = std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return LFA_ERR_INVALID_ARG;
    }
    return LFA_OK;
}

std::string arch_name(int dev) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

std::string plan_prefix(const lfa_plan* p, int dev) {
    char buf[96];
    std::snprintf(buf, sizeof buf, "%s/%s/flags%u", arch_name(dev).c_str(), p->dtype == LFA_F64 ? "f64" : "f32",
                  (unsigned)p->flags);
    return buf;
}

std::string layer_key(const lfa_layer& l) {
    char buf[96];
    std::snprintf(buf, sizeof buf, "%dx%dx%dx%d@%dx%d", l.c_out, l.c_in, l.kh, l.kw, l.n, l.m);
    return buf;
}

// Minimum over `reps` of the event time of fn() on st, after one warm-up.
template <typename F>
int time_min(F&& fn, hipStream_t st, int reps, float& best_ms) {
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    int status = fn();
    best_ms = 1e30f;
    for (int r = 0; r < reps && status == LFA_OK; ++r) {
        if (hipEventRecord(e0, st) != hipSuccess) status = LFA_ERR_HIP;
        if (status == LFA_OK) status = fn();
        if (status == LFA_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
            status = LFA_ERR_HIP;
        float ms = 0;
        if (status == LFA_OK && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) best_ms = std::min(best_ms, ms);
    }
    if (status == LFA_OK && hipStreamSynchronize(st) != hipSuccess) status = LFA_ERR_HIP;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return status;
}

template <typename R>
int autotune_impl(lfa_plan* p, const void* const* W, void* const* sigma, void* const* U, void* const* V,
                  const char* cache_path, uint32_t what, hipStream_t st) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    CacheEntries cache = read_cache(cache_path);
    const std::string prefix = plan_prefix(p, dev);
    const int eb = elem_bytes(p->dtype);
    const bool wu = p->flags & LFA_WANT_U, wv = p->flags & LFA_WANT_V;
    const int nl = (int)p->layers.size();
    // a workspace of its own, large enough for every candidate
    size_t need = workspace_bytes(*p);
    for (int i = 0; i < nl; ++i) {
        const lfa_layer& l = p->layers[i];
        const bool qe = qr_eligible(l, p->dtype, p->flags);
        const bool me = p->dtype == LFA_F32 && l.kh * l.kw >= 25;
        need = std::max(need, kAlign + kCounterBytes +
                                  align_up(std::max({svd_layer_need(*p, i, qe, false, true, true),
                                                     svd_layer_need(*p, i, false, me, true, true)})));
    }
    char* ws = nullptr;
    HIP_TRY(hipMalloc(&ws, need));
    char* region = ws + kAlign;
    int status = LFA_OK;
    std::lock_guard<std::mutex> lock(p->mu);
    bool changed = false;

    if (what & LFA_TUNE_LAYERS) {
        std::map<std::string, int> done;     // shape key -> first layer tuned with it
        for (int i = 0; i < nl && status == LFA_OK; ++i) {
            const lfa_layer& l = p->layers[i];
            const std::string key = prefix + "/layer/" + layer_key(l);
            auto apply = [&](int qr, const LayerTune& t) {
                p->qr[i] = qr;
                p->tune[i] = t;
            };
            auto dn = done.find(key);
            if (dn != done.end()) {
                apply(p->qr[dn->second], p->tune[dn->second]);
                continue;
            }
            done[key] = i;
            auto hit = cache.find(key);
            if (hit != cache.end()) {
                auto& f = hit->second;
                LayerTune t;
                t.queue_seg = f.count("queue_seg") ? (int)f["queue_seg"] : -1;
                t.team_w = f.count("team_w") ? (int)f["team_w"] : 0;
                t.asm_mat = f.count("asm") ? (int)f["asm"] : -1;
                const int qr = f.count("qr") && qr_eligible(l, p->dtype, p->flags) ? (int)f["qr"] : p->qr[i];
                if (t.asm_mat == 1 && !(p->dtype == LFA_F32)) t.asm_mat = -1;
                apply(t.asm_mat == 1 ? 0 : qr, t);
                continue;
            }
            auto run = [&]() -> int {
                return svd_layer<R>(p, (size_t)i, W, nullptr, sigma, U, V, nullptr, region, st, true);
            };
            float best = 0;
            status = time_min(run, st, 2, best);
            int best_qr = p->qr[i];
            LayerTune bt = p->tune[i];
            auto trial = [&](int qr, const LayerTune& t) {
                if (status != LFA_OK) return;
                const int oq = p->qr[i];
                const LayerTune ot = p->tune[i];
                apply(qr, t);
                float ms = 0;
                status = time_min(run, st, 2, ms);
                if (status == LFA_OK && ms < best) {
                    best = ms;
                    best_qr = qr;
                    bt = t;
                } else {
                    apply(oq, ot);
                }
            };
            // materialised matrix-core assembly or fused (kernels of 25 taps
            // or more), then QR factors or not (fused assembly only)
            if (p->dtype == LFA_F32 && l.kh * l.kw >= 25 && !asm_materialized(p->flags)) {
                LayerTune t = bt;
                t.asm_mat = layer_materialized(*p, (size_t)i) ? 0 : 1;
                trial(best_qr, t);
            }
            apply(best_qr, bt);
            if (qr_eligible(l, p->dtype, p->flags) && !layer_materialized(*p, (size_t)i))
                trial(1 - best_qr, bt);
            apply(best_qr, bt);
            // the launch of the path in use: work-queue turns of the register
            // kernel, or team widths of the blocked kernel
            const LayerDesc& d = (p->qr[i] && !layer_materialized(*p, (size_t)i)) ? p->desc_r[i] : p->desc[i];
            if (d.kind == 1 && d.wave_qgroups > 0) {
                for (int seg : {0, 4, 5, 6, 8, 10, 12}) {
                    LayerTune t = bt;
                    t.queue_seg = seg;
                    trial(best_qr, t);
                }
            } else if (d.kind == 2) {
                const int NB = (d.N + kBlockCols - 1) / kBlockCols, NBP = NB + (NB & 1);
                for (int w : {1, 2, 4, 8, 16}) {
                    if (w > NBP / 2) break;
                    LayerTune t = bt;
                    t.team_w = w;
                    trial(best_qr, t);
                }
            }
            apply(best_qr, bt);
            auto& f = cache[key];
            f["qr"] = best_qr;
            f["queue_seg"] = bt.queue_seg;
            f["team_w"] = bt.team_w;
            f["asm"] = bt.asm_mat;
            f["ms"] = best;
            changed = true;
        }
    }

    if (status == LFA_OK && (what & LFA_TUNE_PERSISTENT) && !asm_materialized(p->flags)) {
        std::string key = prefix + "/persistent";
        for (const lfa_layer& l : p->layers) key += "/" + layer_key(l);
        auto hit = cache.find(key);
        if (hit != cache.end() && hit->second.count("wave_s") && hit->second.count("team_ovh")) {
            p->cost_wave = hit->second["wave_s"];
            p->team_ovh = hit->second["team_ovh"];
            build_schedule(p);
            status = upload_items(p);
        } else {
            auto run = [&]() -> int {
                if (p->dtype == LFA_F64) return persistent_impl<double>(p, W, sigma, U, V, nullptr, ws, st);
                return persistent_impl<float>(p, W, sigma, U, V, nullptr, ws, st);
            };
            const double w0 = p->cost_wave, o0 = p->team_ovh;
            double bw = w0, bo = o0;
            float best = 0;
            status = time_min(run, st, 2, best);
            for (double fw : {0.5, 1.0, 2.0}) {
                for (double ov : {0.02, 0.08, 0.25}) {
                    if (status != LFA_OK) break;
                    if (fw == 1.0 && ov == o0) continue;
                    p->cost_wave = w0 * fw;
                    p->team_ovh = ov;
                    build_schedule(p);
                    status = upload_items(p);
                    float ms = 0;
                    if (status == LFA_OK) status = time_min(run, st, 2, ms);
                    if (status == LFA_OK && ms < best) {
                        best = ms;
                        bw = p->cost_wave;
                        bo = ov;
                    }
                }
            }
            p->cost_wave = bw;
            p->team_ovh = bo;
            build_schedule(p);
            if (status == LFA_OK) status = upload_items(p);
            if (status == LFA_OK) {
                auto& f = cache[key];
                f["wave_s"] = bw;
                f["block_s"] = p->cost_block;
                f["team_ovh"] = bo;
                f["ms"] = best;
                changed = true;
            }
        }
    }
    (void)hipFree(ws);
    if (status == LFA_OK && changed) status = write_cache(cache_path, cache);
    (void)eb;
    (void)wu;
    (void)wv;
    return status;
}

}  // namespace

// ---------------------------------------------------------------------------
// extern "C"
// ---------------------------------------------------------------------------
extern "C" {

int lfa_version(void) { return LFA_VERSION; }

int lfa_last_hip_error(void) { return g_last_hip; }

const char* lfa_status_string(int status) {
    switch (status) {
        case LFA_OK: return "success";
        case LFA_ERR_INVALID_ARG: return "invalid argument";
        case LFA_ERR_UNSUPPORTED: return "unsupported size, dtype or flag combination";
        case LFA_ERR_WORKSPACE: return "workspace missing or too small";
        case LFA_ERR_HIP: return "HIP runtime error (see lfa_last_hip_error)";
        case LFA_ERR_NO_DEVICE: return "no usable gfx950 device";
        case LFA_ERR_NOT_PREPARED: return "plan not prepared on this device (needed under stream capture)";
        case LFA_WARN_NOT_CONVERGED: return "warning: some symbols hit the sweep cap";
        case LFA_WARN_NONFINITE: return "warning: non-finite singular values";
        case LFA_WARN_TEAM_TIMEOUT: return "warning: a work-group team barrier timed out";
        default: return "unknown status";
    }
}

int lfa_plan_create(lfa_plan** out, const lfa_layer* layers, int32_t num_layers, int32_t dtype,
                    uint32_t flags) {
    if (!out) return LFA_ERR_INVALID_ARG;
    *out = nullptr;
    if (!layers || num_layers < 1 || num_layers > kMaxLayers) return LFA_ERR_INVALID_ARG;
    if (dtype != LFA_F32 && dtype != LFA_F64) return LFA_ERR_INVALID_ARG;
    const uint32_t known =
        LFA_WANT_U | LFA_WANT_V | LFA_ASM_MFMA | LFA_ASM_BF16X2 | LFA_ASM_BF16X3 | LFA_PHASE_NORMALIZE;
    if (flags & ~known) return LFA_ERR_INVALID_ARG;
    if ((flags & LFA_PHASE_NORMALIZE) && !(flags & (LFA_WANT_U | LFA_WANT_V))) return LFA_ERR_INVALID_ARG;
    const uint32_t asm_flags = flags & (LFA_ASM_MFMA | LFA_ASM_BF16X2 | LFA_ASM_BF16X3);
    if (asm_flags & (asm_flags - 1)) return LFA_ERR_INVALID_ARG;   // more than one
    if (asm_flags && dtype != LFA_F32) return LFA_ERR_UNSUPPORTED;
    for (int i = 0; i < num_layers; ++i) LFA_TRY(validate_layer(layers[i]));

    lfa_plan* p = new (std::nothrow) lfa_plan();
    if (!p) return LFA_ERR_INVALID_ARG;
    p->dtype = dtype;
    p->flags = flags;
    p->layers.assign(layers, layers + num_layers);
    p->tune.assign(num_layers, LayerTune{});
    const int eb = elem_bytes(dtype);
    // unit roundoff of the working precision (see jacobi_tol)
    p->tol = dtype == LFA_F64 ? std::ldexp(1.0, -53) : std::ldexp(1.0, -24);
    // LFA_WAVE_QUEUE: "0" turns the work-queue launch off, k in 1..16 forces
    // it with k sweeps per turn (tests, tuning); unset or other values:
    // automatic
    if (const char* env = std::getenv("LFA_WAVE_QUEUE")) {
        const int v = std::atoi(env);
        if (std::strcmp(env, "0") == 0) p->wq_force = 0;
        else if (v >= 1 && v <= 16) p->wq_force = v;
    }

    // twiddles exp(2 pi i j / L) for every distinct grid length L
    std::map<int, int> off;
    for (const lfa_layer& l : p->layers) {
        for (int len : {l.n, l.m}) {
            if (off.count(len)) continue;
            off[len] = (int)(p->tw_host.size() / 2);
            for (int j = 0; j < len; ++j) {
                // reduce j/len to [-1/2, 1/2) turns before the library cos/sin
                const double turns = (2 * j < len) ? double(j) / len : double(j - len) / len;
                const double ang = 2.0 * M_PI * turns;
                p->tw_host.push_back(std::cos(ang));
                p->tw_host.push_back(std::sin(ang));
            }
        }
    }
    const bool wu = flags & LFA_WANT_U, wv = flags & LFA_WANT_V;
    // the persistent launch keeps the accumulator when some layer needs it
    // (V of a tall layer, U of a wide one); the side its working matrix
    // converges to comes without one
    for (const lfa_layer& l : p->layers) p->pers_acc |= (l.c_out < l.c_in) ? wu : wv;
    for (const lfa_layer& l : p->layers) {
        // one symbol per conjugate pair (canonical_theta enumerates them)
        const int ncanon = lfa::canonical_count(l.n, l.m);
        p->tw_n.push_back(off[l.n]);
        p->tw_m.push_back(off[l.m]);
        LayerDesc d = make_desc(l, off[l.n], off[l.m], false, eb, kLdsCap);
        d = make_desc(l, off[l.n], off[l.m], accumulates(d, wu, wv), eb, kLdsCap);
        p->desc.push_back(d);
        p->desc_sel.push_back(make_desc(l, off[l.n], off[l.m], true, eb, kLdsCap));
        // persistent launch: bundles of the register kernel for small symbols
        // without vectors, the blocked kernel (256 threads) otherwise
        // one accumulator setting for the whole persistent launch (its kernel
        // is compiled with or without the accumulator)
        const bool pacc = p->pers_acc;
        LayerDesc dp = make_desc(l, off[l.n], off[l.m], pacc, eb, kLdsCap);
        if (dp.kind != 1 || pacc) {
            dp = make_desc(l, off[l.n], off[l.m], pacc, eb, kLdsCap);
            dp.kind = 2;
            dp.threads = kPersistentThreads;
            dp.storage = kGlobal;
        }
        {
            LayerDesc dg = make_desc(l, off[l.n], off[l.m], true, eb, kLdsCap);
            dg.kind = 2;
            dg.threads = kPersistentThreads;
            dg.storage = kGlobal;
            dg.num_canon = ncanon;
            p->desc_gsel.push_back(dg);
        }
        p->desc.back().num_canon = ncanon;
        p->desc.back().wave_qgroups = wave_queue_reserved(p->desc.back(), accumulates(p->desc.back(), wu, wv), eb);
        {
            const int N = std::min(l.c_out, l.c_in);
            const bool q = qr_applies(l, dtype, flags);
            p->qr.push_back(q ? 1 : 0);
            lfa_layer lr{N, N, 1, 1, l.n, l.m};
            // the SVD of the factors never accumulates: sigma only, or the
            // left vectors of R^H (= V_R)
            LayerDesc dr = make_desc(lr, off[l.n], off[l.m], false, eb, kLdsCap);
            dr.num_canon = ncanon;
            dr.wave_qgroups = qr_eligible(l, dtype, flags) ? wave_queue_reserved(dr, false, eb) : 0;
            p->desc_r.push_back(dr);
        }
        p->desc_sel.back().num_canon = ncanon;
        dp.num_canon = ncanon;
        p->desc_pers.push_back(dp);
        if (dp.kind == 2) {
            p->pers_slot_off.push_back(p->pers_slots_total);
            p->pers_slots_total += (size_t)ncanon * slot_bytes(dp, pacc, eb);
            p->pers_teams += ncanon;
        } else {
            p->pers_slot_off.push_back(0);
        }
    }
    // device tables on the current device now, when there is a gfx950 one
    // (otherwise on first use, or in lfa_plan_prepare)
    {
        int count = 0;
        if (hipGetDeviceCount(&count) == hipSuccess && count > 0) (void)ensure_device(p);
        else (void)hipGetLastError();
    }
    *out = p;
    return LFA_OK;
}

int lfa_plan_destroy(lfa_plan* plan) {
    if (!plan) return LFA_OK;
    if (plan->tw_dev) (void)hipFree(plan->tw_dev);
    if (plan->items_dev) (void)hipFree(plan->items_dev);
    for (WorkItem* w : plan->old_items) (void)hipFree(w);
    for (auto& kv : plan->grad_sched)
        if (kv.second.items_dev) (void)hipFree(kv.second.items_dev);
    delete plan;
    return LFA_OK;
}

int lfa_plan_prepare(lfa_plan* plan, int32_t k) {
    if (!plan || k < 0) return LFA_ERR_INVALID_ARG;
    LFA_TRY(ensure_device(plan));
    if (k > 0) {
        LFA_TRY(check_k(plan, k));
        LFA_TRY(ensure_grad_schedule(plan, k, nullptr, false, nullptr));
    }
    return LFA_OK;
}

int lfa_plan_record_phases(lfa_plan* plan, unsigned long long* ticks) {
    if (!plan) return LFA_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(plan->mu);
    plan->phase_rec = ticks;
    return LFA_OK;
}

int lfa_plan_set_max_sweeps(lfa_plan* plan, int32_t max_sweeps) {
    if (!plan || max_sweeps < 1 || max_sweeps > kMaxSweeps) return LFA_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(plan->mu);
    plan->max_sweeps = max_sweeps;
    return LFA_OK;
}

int lfa_info_status(const int32_t* info, int32_t num_layers) {
    if (!info || num_layers < 1) return LFA_ERR_INVALID_ARG;
    int w = 0;
    for (int i = 0; i < num_layers; ++i) {
        const int32_t* r = info + (size_t)i * LFA_INFO_WORDS;
        if (r[LFA_INFO_NONCONVERGED] > 0) w |= LFA_WARN_NOT_CONVERGED;
        if (r[LFA_INFO_NONFINITE] & 1) w |= LFA_WARN_NONFINITE;
        if (r[LFA_INFO_NONFINITE] & 2) w |= LFA_WARN_TEAM_TIMEOUT;
    }
    return w;
}

int lfa_plan_workspace_bytes(const lfa_plan* plan, size_t* bytes) {
    if (!plan || !bytes) return LFA_ERR_INVALID_ARG;
    *bytes = workspace_bytes(*plan);
    return LFA_OK;
}

int lfa_plan_num_layers(const lfa_plan* plan, int32_t* num_layers) {
    if (!plan || !num_layers) return LFA_ERR_INVALID_ARG;
    *num_layers = (int32_t)plan->layers.size();
    return LFA_OK;
}

int lfa_plan_layer(const lfa_plan* plan, int32_t i, lfa_layer* layer) {
    if (!plan || !layer || i < 0 || i >= (int32_t)plan->layers.size()) return LFA_ERR_INVALID_ARG;
    *layer = plan->layers[i];
    return LFA_OK;
}

int lfa_plan_launch_shape(const lfa_plan* plan, int32_t layer, int32_t* lanes_per_pair,
                          int32_t* threads, int32_t* symbols_per_group, int32_t* storage) {
    if (!plan || layer < 0 || layer >= (int32_t)plan->layers.size()) return LFA_ERR_INVALID_ARG;
    const LayerDesc& d = plan->desc[layer];
    if (lanes_per_pair) *lanes_per_pair = d.L;
    if (threads) *threads = d.threads;
    if (symbols_per_group) *symbols_per_group = wave_symbols_per_group(d);
    if (storage) *storage = d.storage;
    return LFA_OK;
}

int lfa_plan_preconditioned(const lfa_plan* plan, int32_t layer, int32_t* qr) {
    if (!plan || !qr || layer < 0 || layer >= (int32_t)plan->layers.size()) return LFA_ERR_INVALID_ARG;
    *qr = plan->qr[layer];
    return LFA_OK;
}

int lfa_plan_queue_info(lfa_plan* plan, int32_t layer, int32_t* resident, int32_t* sweeps_per_turn) {
    if (!plan || layer < 0 || layer >= (int32_t)plan->layers.size()) return LFA_ERR_INVALID_ARG;
    LFA_TRY(ensure_device(plan));
    const LayerDesc& d = plan->desc[layer];
    if (resident) *resident = d.kind == 1 && d.wave_qgroups > 0 ? d.wave_qcap : 0;
    if (sweeps_per_turn) *sweeps_per_turn = wave_queue_seg(d, wave_groups(d, d.num_canon), plan->wq_force);
    return LFA_OK;
}

int lfa_apply_workspace_bytes(const lfa_plan* plan, int32_t layer, int32_t batch, size_t* bytes) {
    if (!plan || !bytes || layer < 0 || layer >= (int32_t)plan->layers.size() || batch < 0)
        return LFA_ERR_INVALID_ARG;
    const lfa_layer& l = plan->layers[layer];
    const size_t c = (size_t)std::max(l.c_out, l.c_in);
    *bytes = 2 * align_up((size_t)batch * l.n * l.m * c * 2 * elem_bytes(plan->dtype));
    return LFA_OK;
}

int lfa_apply(const lfa_plan* plan, int32_t layer, const void* sigma, const void* U, const void* V,
              int32_t kind, double param, const void* x, void* y, int32_t batch, void* ws,
              size_t ws_bytes, void* stream) {
    if (!plan || layer < 0 || layer >= (int32_t)plan->layers.size() || batch < 0) return LFA_ERR_INVALID_ARG;
    if (kind != LFA_SPECTRAL_IDENTITY && kind != LFA_SPECTRAL_CLIP && kind != LFA_SPECTRAL_PINV &&
        kind != LFA_SPECTRAL_TRUNCATE)
        return LFA_ERR_INVALID_ARG;
    if (!(param >= 0.0) || !std::isfinite(param)) return LFA_ERR_INVALID_ARG;
    if (batch == 0) return LFA_OK;
    if (!sigma || !U || !V || !x || !y) return LFA_ERR_INVALID_ARG;
    size_t need = 0;
    LFA_TRY(lfa_apply_workspace_bytes(plan, layer, batch, &need));
    if (!ws || ws_bytes < need) return LFA_ERR_WORKSPACE;
    lfa_plan* p = const_cast<lfa_plan*>(plan);
    LFA_TRY(ensure_device(p, static_cast<hipStream_t>(stream), true));
    const lfa_layer& l = p->layers[layer];
    const bool pinv = kind == LFA_SPECTRAL_PINV;
    if (!apply_supported(pinv ? l.c_out : l.c_in, std::min(l.c_out, l.c_in), elem_bytes(p->dtype)))
        return LFA_ERR_UNSUPPORTED;
    ApplyArgs a{};
    a.batch = batch;
    a.n = l.n;
    a.m = l.m;
    a.cx = pinv ? l.c_out : l.c_in;
    a.cy = pinv ? l.c_in : l.c_out;
    a.r = std::min(l.c_out, l.c_in);
    a.kind = kind;
    a.param = param;
    a.sigma = sigma;
    a.L = pinv ? V : U;
    a.R = pinv ? U : V;
    a.x = x;
    a.y = y;
    a.ws1 = ws;
    a.ws2 = static_cast<char*>(ws) + need / 2;
    a.tw = p->tw_dev;
    a.tw_n = p->tw_n[layer];
    a.tw_m = p->tw_m[layer];
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(p->dtype == LFA_F64 ? launch_apply_f64(a, st) : launch_apply_f32(a, st));
    return LFA_OK;
}

int lfa_crystal_layer(const lfa_layer* layer, int32_t stride, lfa_layer* out) {
    if (!layer || !out || stride < 1) return LFA_ERR_INVALID_ARG;
    const lfa_layer& l = *layer;
    if (l.c_out <= 0 || l.c_in <= 0 || l.kh <= 0 || l.kw <= 0 || l.n <= 0 || l.m <= 0)
        return LFA_ERR_INVALID_ARG;
    if (l.kh > l.n || l.kw > l.m || l.n % stride || l.m % stride) return LFA_ERR_INVALID_ARG;
    if ((long long)stride * stride * l.c_in > (1LL << 30)) return LFA_ERR_UNSUPPORTED;
    // coarse offsets floor(y / s) of the taps y in [-(k-1)/2, k-1-(k-1)/2]
    // span [-L, R]; the centred stride-1 window of extent max(2L+1, 2R)
    // covers them
    auto extent = [stride](int k) {
        const int c = (k - 1) / 2;
        const int L = (c + stride - 1) / stride, R = (k - 1 - c) / stride;
        return std::max(2 * L + 1, 2 * R);
    };
    lfa_layer o{};
    o.c_out = l.c_out;
    o.c_in = stride * stride * l.c_in;
    o.kh = extent(l.kh);
    o.kw = extent(l.kw);
    o.n = l.n / stride;
    o.m = l.m / stride;
    *out = o;
    return LFA_OK;
}

int lfa_crystal_weights(const lfa_layer* layer, int32_t stride, int32_t dtype, const void* src, void* dst,
                        int32_t direction, void* stream) {
    lfa_layer c{};
    LFA_TRY(lfa_crystal_layer(layer, stride, &c));
    if (dtype != LFA_F32 && dtype != LFA_F64) return LFA_ERR_INVALID_ARG;
    if (direction != LFA_CRYSTAL_FORWARD && direction != LFA_CRYSTAL_ADJOINT) return LFA_ERR_INVALID_ARG;
    if (!src || !dst) return LFA_ERR_INVALID_ARG;
    CrystalArgs a{};
    a.c_out = layer->c_out;
    a.c_in = layer->c_in;
    a.kh = layer->kh;
    a.kw = layer->kw;
    a.stride = stride;
    a.kh2 = c.kh;
    a.kw2 = c.kw;
    HIP_TRY(launch_crystal_weights(a, elem_bytes(dtype), src, dst, direction == LFA_CRYSTAL_ADJOINT,
                                   static_cast<hipStream_t>(stream)));
    return LFA_OK;
}

int lfa_lift(const lfa_plan* plan, int32_t layer, const void* U, const void* V, const int32_t* idx,
             int32_t count, void* u_hat, void* v_hat, void* stream) {
    if (!plan || layer < 0 || layer >= (int32_t)plan->layers.size() || count < 0) return LFA_ERR_INVALID_ARG;
    if ((u_hat && !U) || (v_hat && !V)) return LFA_ERR_INVALID_ARG;
    if (count == 0 || (!u_hat && !v_hat)) return LFA_OK;
    if (!idx) return LFA_ERR_INVALID_ARG;
    // one work-group per (pick, channel) row
    const lfa_layer& l0 = plan->layers[layer];
    if ((long long)count * std::max(l0.c_out, l0.c_in) > 0x7fffffffLL) return LFA_ERR_UNSUPPORTED;
    lfa_plan* p = const_cast<lfa_plan*>(plan);
    LFA_TRY(ensure_device(p, static_cast<hipStream_t>(stream), true));
    const lfa_layer& l = p->layers[layer];
    LiftArgs a{};
    a.count = count;
    a.n = l.n;
    a.m = l.m;
    a.c_out = l.c_out;
    a.c_in = l.c_in;
    a.r = std::min(l.c_out, l.c_in);
    a.idx = idx;
    a.U = U;
    a.V = V;
    a.u_hat = u_hat;
    a.v_hat = v_hat;
    a.tw = p->tw_dev;
    a.tw_n = p->tw_n[layer];
    a.tw_m = p->tw_m[layer];
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(p->dtype == LFA_F64 ? launch_lift_f64(a, st) : launch_lift_f32(a, st));
    return LFA_OK;
}

int lfa_symbols(const lfa_plan* plan, const void* const* W, void* const* A, void* stream) {
    if (!plan) return LFA_ERR_INVALID_ARG;
    LFA_TRY(check_ptrs(plan, W, true));
    LFA_TRY(check_ptrs(plan, A, true));
    lfa_plan* p = const_cast<lfa_plan*>(plan);
    hipStream_t st = static_cast<hipStream_t>(stream);
    LFA_TRY(ensure_device(p, st, true));
    for (size_t i = 0; i < p->layers.size(); ++i) {
        const LayerDesc& d = p->desc[i];
        hipError_t e;
        if (p->dtype == LFA_F64)
            e = launch_symbols_valu_f64(d, static_cast<const double*>(W[i]),
                                        static_cast<cplx<double>*>(A[i]), p->tw_dev, st);
        else if (asm_materialized(p->flags))
            e = launch_symbols_mfma(d, static_cast<const float*>(W[i]),
                                    static_cast<cplx<float>*>(A[i]), p->tw_dev,
                                    asm_mode(p->flags), st);
        else
            e = launch_symbols_valu_f32(d, static_cast<const float*>(W[i]),
                                        static_cast<cplx<float>*>(A[i]), p->tw_dev, st);
        HIP_TRY(e);
    }
    return LFA_OK;
}

static int svd_common(const lfa_plan* plan, const void* const* W, const void* const* A,
                      void* const* sigma, void* const* U, void* const* V, int32_t* info, void* ws,
                      size_t ws_bytes, void* stream, bool persistent) {
    if (!plan) return LFA_ERR_INVALID_ARG;
    LFA_TRY(check_ptrs(plan, W ? W : A, true));
    LFA_TRY(check_ptrs(plan, sigma, true));
    LFA_TRY(check_ptrs(plan, U, (plan->flags & LFA_WANT_U) != 0));
    LFA_TRY(check_ptrs(plan, V, (plan->flags & LFA_WANT_V) != 0));
    if (persistent && asm_materialized(plan->flags)) return LFA_ERR_UNSUPPORTED;
    LFA_TRY(check_ws(plan, ws, ws_bytes));
    lfa_plan* p = const_cast<lfa_plan*>(plan);
    hipStream_t st = static_cast<hipStream_t>(stream);
    LFA_TRY(ensure_device(p, st, true));
    if (persistent) {
        if (p->dtype == LFA_F64) return persistent_impl<double>(p, W, sigma, U, V, info, ws, st);
        return persistent_impl<float>(p, W, sigma, U, V, info, ws, st);
    }
    if (p->dtype == LFA_F64) return svd_impl<double>(p, W, A, sigma, U, V, info, ws, ws_bytes, st);
    return svd_impl<float>(p, W, A, sigma, U, V, info, ws, ws_bytes, st);
}

int lfa_svd(const lfa_plan* plan, const void* const* W, void* const* sigma, void* const* U,
            void* const* V, int32_t* info, void* ws, size_t ws_bytes, void* stream) {
    if (!W) return LFA_ERR_INVALID_ARG;
    return svd_common(plan, W, nullptr, sigma, U, V, info, ws, ws_bytes, stream, false);
}

int lfa_svd_noalloc(const lfa_plan* plan, const void* const* W, void* const* sigma, void* const* U,
                    void* const* V, int32_t* info, void* stream) {
    if (!plan || !W) return LFA_ERR_INVALID_ARG;
    LFA_TRY(check_ptrs(plan, W, true));
    LFA_TRY(check_ptrs(plan, sigma, true));
    LFA_TRY(check_ptrs(plan, U, (plan->flags & LFA_WANT_U) != 0));
    LFA_TRY(check_ptrs(plan, V, (plan->flags & LFA_WANT_V) != 0));
    lfa_plan* p = const_cast<lfa_plan*>(plan);
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    {
        // the device tables must be there already: no upload here
        std::lock_guard<std::mutex> lock(p->mu);
        if (p->device != dev) return LFA_ERR_NOT_PREPARED;
    }
    void* scr = nullptr;
    size_t cap = 0;
    HIP_TRY(lfa::noalloc_scratch(dev, &scr, &cap));
    // the plan's own launch when it fits; else without the work queue (the
    // same results, bit for bit); else the layer set is too large
    const bool queue = svd_need(*p, true) <= cap;
    if (!queue && svd_need(*p, false) > cap) return LFA_ERR_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (p->dtype == LFA_F64) return svd_impl<double>(p, W, nullptr, sigma, U, V, info, scr, cap, st, queue);
    return svd_impl<float>(p, W, nullptr, sigma, U, V, info, scr, cap, st, queue);
}

int lfa_svd_persistent(const lfa_plan* plan, const void* const* W, void* const* sigma,
                       void* const* U, void* const* V, int32_t* info, void* ws, size_t ws_bytes,
                       void* stream) {
    if (!W) return LFA_ERR_INVALID_ARG;
    return svd_common(plan, W, nullptr, sigma, U, V, info, ws, ws_bytes, stream, true);
}

int lfa_plan_persistent_grid(const lfa_plan* plan, int32_t* grid) {
    if (!plan || !grid) return LFA_ERR_INVALID_ARG;
    lfa_plan* p = const_cast<lfa_plan*>(plan);
    LFA_TRY(ensure_device(p));
    int g = 0;
    for (size_t c = 0; c + 1 < p->chunk_first.size(); ++c)
        g = std::max(g, std::min(p->pers_grid[c], p->chunk_first[c + 1] - p->chunk_first[c]));
    *grid = g;
    return LFA_OK;
}

int lfa_svd_persistent_busy(const lfa_plan* plan, const void* const* W, void* const* sigma, void* const* U,
                            void* const* V, int32_t* info, void* ws, size_t ws_bytes, int64_t* busy,
                            int32_t busy_len, void* stream) {
    if (!plan || !W || !busy) return LFA_ERR_INVALID_ARG;
    int32_t g = 0;
    LFA_TRY(lfa_plan_persistent_grid(plan, &g));
    if (busy_len < g) return LFA_ERR_INVALID_ARG;
    LFA_TRY(check_ptrs(plan, W, true));
    LFA_TRY(check_ptrs(plan, sigma, true));
    LFA_TRY(check_ptrs(plan, U, (plan->flags & LFA_WANT_U) != 0));
    LFA_TRY(check_ptrs(plan, V, (plan->flags & LFA_WANT_V) != 0));
    if (asm_materialized(plan->flags)) return LFA_ERR_UNSUPPORTED;
    LFA_TRY(check_ws(plan, ws, ws_bytes));
    lfa_plan* p = const_cast<lfa_plan*>(plan);
    hipStream_t st = static_cast<hipStream_t>(stream);
    LFA_TRY(ensure_device(p, st, true));
    long long* b = reinterpret_cast<long long*>(busy);
    if (p->dtype == LFA_F64) return persistent_impl<double>(p, W, sigma, U, V, info, ws, st, b);
    return persistent_impl<float>(p, W, sigma, U, V, info, ws, st, b);
}

int lfa_svd_symbols(const lfa_plan* plan, const void* const* A, void* const* sigma,
                    void* const* U, void* const* V, int32_t* info, void* ws, size_t ws_bytes,
                    void* stream) {
    if (!A) return LFA_ERR_INVALID_ARG;
    return svd_common(plan, nullptr, A, sigma, U, V, info, ws, ws_bytes, stream, false);
}

int lfa_topk(const lfa_plan* plan, const void* const* sigma, int32_t k, void* vals, int32_t* idx,
             void* stream) {
    if (!plan || !vals || !idx) return LFA_ERR_INVALID_ARG;
    LFA_TRY(check_ptrs(plan, sigma, true));
    LFA_TRY(check_k(plan, k));
    lfa_plan* p = const_cast<lfa_plan*>(plan);
    hipStream_t st = static_cast<hipStream_t>(stream);
    LFA_TRY(ensure_device(p, st, true));
    if (p->dtype == LFA_F64) return topk_impl<double>(p, sigma, k, vals, idx, st);
    return topk_impl<float>(p, sigma, k, vals, idx, st);
}

int lfa_adjoint(const lfa_plan* plan, const void* const* U, const void* const* V,
                const int32_t* idx, const void* grad, int32_t k, void* const* dW, void* stream) {
    if (!plan || !idx || !grad) return LFA_ERR_INVALID_ARG;
    LFA_TRY(check_ptrs(plan, U, true));
    LFA_TRY(check_ptrs(plan, V, true));
    LFA_TRY(check_ptrs(plan, dW, true));
    LFA_TRY(check_k(plan, k));
    lfa_plan* p = const_cast<lfa_plan*>(plan);
    hipStream_t st = static_cast<hipStream_t>(stream);
    LFA_TRY(ensure_device(p, st, true));
    const int nl = (int)p->layers.size();
    for (int l0 = 0; l0 < nl; l0 += kMaxLaunchLayers) {
        const int l1 = std::min(nl, l0 + kMaxLaunchLayers);
        if (p->dtype == LFA_F64) LFA_TRY(adjoint_launch<double>(p, l0, l1, U, V, idx, grad, k, dW, 0, st));
        else LFA_TRY(adjoint_launch<float>(p, l0, l1, U, V, idx, grad, k, dW, 0, st));
    }
    return LFA_OK;
}

int lfa_adjoint_onesided(const lfa_plan* plan, const void* const* W, const void* const* sigma,
                         const void* const* X, const int32_t* idx, const void* grad, int32_t k,
                         void* const* dW, void* ws, size_t ws_bytes, void* stream) {
    if (!plan || !idx || !grad) return LFA_ERR_INVALID_ARG;
    LFA_TRY(check_ptrs(plan, W, true));
    LFA_TRY(check_ptrs(plan, sigma, true));
    LFA_TRY(check_ptrs(plan, X, true));
    LFA_TRY(check_ptrs(plan, dW, true));
    LFA_TRY(check_k(plan, k));
    LFA_TRY(check_ws(plan, ws, ws_bytes));
    lfa_plan* p = const_cast<lfa_plan*>(plan);
    hipStream_t st = static_cast<hipStream_t>(stream);
    LFA_TRY(ensure_device(p, st, true));
    if (p->dtype == LFA_F64) return adjoint_onesided_impl<double>(p, W, sigma, X, idx, grad, k, dW, ws, st);
    return adjoint_onesided_impl<float>(p, W, sigma, X, idx, grad, k, dW, ws, st);
}

int lfa_sigma_grad(const lfa_plan* plan, const void* const* W, const int32_t* idx, const void* grad,
                   int32_t k, void* const* dW, void* ws, size_t ws_bytes, void* stream) {
    if (!plan || !idx || !grad) return LFA_ERR_INVALID_ARG;
    LFA_TRY(check_ptrs(plan, W, true));
    LFA_TRY(check_ptrs(plan, dW, true));
    LFA_TRY(check_k(plan, k));
    LFA_TRY(check_ws(plan, ws, ws_bytes));
    lfa_plan* p = const_cast<lfa_plan*>(plan);
    hipStream_t st = static_cast<hipStream_t>(stream);
    LFA_TRY(ensure_device(p, st, true));
    if (p->dtype == LFA_F64) return sigma_grad_impl<double>(p, W, idx, grad, k, dW, ws, st);
    return sigma_grad_impl<float>(p, W, idx, grad, k, dW, ws, st);
}

int lfa_sigma_grad_persistent(const lfa_plan* plan, const void* const* W, const int32_t* idx,
                              const void* grad, int32_t k, void* const* dW, void* ws,
                              size_t ws_bytes, void* stream) {
    if (!plan || !idx || !grad) return LFA_ERR_INVALID_ARG;
    LFA_TRY(check_ptrs(plan, W, true));
    LFA_TRY(check_ptrs(plan, dW, true));
    LFA_TRY(check_k(plan, k));
    LFA_TRY(check_ws(plan, ws, ws_bytes));
    lfa_plan* p = const_cast<lfa_plan*>(plan);
    hipStream_t st = static_cast<hipStream_t>(stream);
    LFA_TRY(ensure_device(p, st, true));
    const lfa_plan::GradSched* gs = nullptr;
    LFA_TRY(ensure_grad_schedule(p, k, st, true, &gs));
    if (p->dtype == LFA_F64) return sigma_grad_persistent_impl<double>(p, *gs, W, idx, grad, k, dW, ws, st);
    return sigma_grad_persistent_impl<float>(p, *gs, W, idx, grad, k, dW, ws, st);
}

namespace {

// Both graph forms: with U and V (null for the sigma-only form), the forward
// pass keeps every symbol's singular vectors and the gradient is one adjoint
// launch; without, the gradient recomputes the vectors of the picks.
// Graph forms: sigma only (U, V, X null), with U and V of every symbol, or
// one-sided (X: the kept side of every layer, U for tall layers, V for wide
// ones; the plan wants exactly that side).
int graph_create(lfa_plan* plan, const void* const* W, void* const* sigma, void* const* U, void* const* V,
                 int32_t k, void* vals, int32_t* idx, const void* grad, void* const* dW, int32_t* info,
                 void* ws, size_t ws_bytes, void* stream, lfa_graph** out, void* const* X = nullptr) {
    if (!out) return LFA_ERR_INVALID_ARG;
    *out = nullptr;
    if (!plan || !vals || !idx || !grad) return LFA_ERR_INVALID_ARG;
    const bool uv = U != nullptr || V != nullptr;
    const uint32_t want = plan->flags & (LFA_WANT_U | LFA_WANT_V);
    bool ku = false;
    if (X) {
        ku = keeps_u(plan->layers[0]);
        for (const lfa_layer& l : plan->layers)
            if (keeps_u(l) != ku) return LFA_ERR_UNSUPPORTED;
        if (want != (ku ? LFA_WANT_U : LFA_WANT_V)) return LFA_ERR_UNSUPPORTED;
        LFA_TRY(check_ptrs(plan, X, true));
    } else if (want != (uv ? (LFA_WANT_U | LFA_WANT_V) : 0u)) {
        return LFA_ERR_UNSUPPORTED;
    }
    LFA_TRY(check_ptrs(plan, W, true));
    LFA_TRY(check_ptrs(plan, sigma, true));
    LFA_TRY(check_ptrs(plan, dW, true));
    if (uv) {
        LFA_TRY(check_ptrs(plan, U, true));
        LFA_TRY(check_ptrs(plan, V, true));
    }
    LFA_TRY(check_k(plan, k));
    LFA_TRY(check_ws(plan, ws, ws_bytes));
    hipStream_t st = static_cast<hipStream_t>(stream);
    // uploads are not allowed while capturing: do them now
    LFA_TRY(ensure_device(plan, st, true));
    if (!uv && !X) LFA_TRY(ensure_grad_schedule(plan, k, st, true, nullptr));
    if (st == nullptr) return LFA_ERR_INVALID_ARG;   // cannot capture the legacy default stream
    lfa_graph* g = new (std::nothrow) lfa_graph();
    if (!g) return LFA_ERR_INVALID_ARG;
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        delete g;
        return hip_fail(e);
    }
    int s = X ? lfa_svd_persistent(plan, W, sigma, ku ? X : nullptr, ku ? nullptr : X, info, ws, ws_bytes, stream)
              : lfa_svd_persistent(plan, W, sigma, U, V, info, ws, ws_bytes, stream);
    if (s == LFA_OK) s = lfa_topk(plan, sigma, k, vals, idx, stream);
    if (s == LFA_OK) {
        if (X)
            s = lfa_adjoint_onesided(plan, W, sigma, X, idx, grad, k, dW, ws, ws_bytes, stream);
        else
            s = uv ? lfa_adjoint(plan, U, V, idx, grad, k, dW, stream)
                   : lfa_sigma_grad_persistent(plan, W, idx, grad, k, dW, ws, ws_bytes, stream);
    }
    e = hipStreamEndCapture(st, &g->graph);
    if (s != LFA_OK || e != hipSuccess) {
        if (g->graph) (void)hipGraphDestroy(g->graph);
        delete g;
        return s != LFA_OK ? s : hip_fail(e);
    }
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g->graph);
        delete g;
        return hip_fail(e);
    }
    *out = g;
    return LFA_OK;
}

}  // namespace

int lfa_graph_create(lfa_plan* plan, const void* const* W, void* const* sigma, int32_t k,
                     void* vals, int32_t* idx, const void* grad, void* const* dW, int32_t* info,
                     void* ws, size_t ws_bytes, void* stream, lfa_graph** out) {
    return graph_create(plan, W, sigma, nullptr, nullptr, k, vals, idx, grad, dW, info, ws, ws_bytes, stream,
                        out);
}

int lfa_graph_create_uv(lfa_plan* plan, const void* const* W, void* const* sigma, void* const* U,
                        void* const* V, int32_t k, void* vals, int32_t* idx, const void* grad,
                        void* const* dW, int32_t* info, void* ws, size_t ws_bytes, void* stream,
                        lfa_graph** out) {
    if (!U || !V) {
        if (out) *out = nullptr;
        return LFA_ERR_INVALID_ARG;
    }
    return graph_create(plan, W, sigma, U, V, k, vals, idx, grad, dW, info, ws, ws_bytes, stream, out);
}

int lfa_graph_create_onesided(lfa_plan* plan, const void* const* W, void* const* sigma, void* const* X,
                              int32_t k, void* vals, int32_t* idx, const void* grad, void* const* dW,
                              int32_t* info, void* ws, size_t ws_bytes, void* stream, lfa_graph** out) {
    if (!X) {
        if (out) *out = nullptr;
        return LFA_ERR_INVALID_ARG;
    }
    return graph_create(plan, W, sigma, nullptr, nullptr, k, vals, idx, grad, dW, info, ws, ws_bytes, stream,
                        out, X);
}

int lfa_graph_launch(lfa_graph* graph, void* stream) {
    if (!graph) return LFA_ERR_INVALID_ARG;
    HIP_TRY(hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream)));
    return LFA_OK;
}

int lfa_graph_destroy(lfa_graph* graph) {
    if (!graph) return LFA_OK;
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
    return LFA_OK;
}

int lfa_autotune(lfa_plan* plan, const void* const* W, void* const* sigma, void* const* U,
                 void* const* V, const char* cache_path, uint32_t what, void* stream) {
    if (!plan || (what & ~uint32_t(LFA_TUNE_LAYERS | LFA_TUNE_PERSISTENT))) return LFA_ERR_INVALID_ARG;
    LFA_TRY(check_ptrs(plan, W, true));
    LFA_TRY(check_ptrs(plan, sigma, true));
    LFA_TRY(check_ptrs(plan, U, (plan->flags & LFA_WANT_U) != 0));
    LFA_TRY(check_ptrs(plan, V, (plan->flags & LFA_WANT_V) != 0));
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (capturing(st)) return LFA_ERR_INVALID_ARG;
    LFA_TRY(ensure_device(plan));
    if (plan->dtype == LFA_F64) return autotune_impl<double>(plan, W, sigma, U, V, cache_path, what, st);
    return autotune_impl<float>(plan, W, sigma, U, V, cache_path, what, st);
}

int lfa_plan_tuning(const lfa_plan* plan, int32_t layer, int32_t* qr, int32_t* queue_seg, int32_t* team_w,
                    int32_t* asm_mat) {
    if (!plan || layer < 0 || layer >= (int32_t)plan->layers.size()) return LFA_ERR_INVALID_ARG;
    const LayerTune& t = plan->tune[layer];
    if (qr) *qr = plan->qr[layer];
    if (queue_seg) *queue_seg = t.queue_seg;
    if (team_w) *team_w = t.team_w;
    if (asm_mat) *asm_mat = t.asm_mat;
    return LFA_OK;
}

int lfa_plan_cost_model(const lfa_plan* plan, double* wave_s, double* block_s, double* team_ovh) {
    if (!plan) return LFA_ERR_INVALID_ARG;
    if (wave_s) *wave_s = plan->cost_wave;
    if (block_s) *block_s = plan->cost_block;
    if (team_ovh) *team_ovh = plan->team_ovh;
    return LFA_OK;
}

}  // extern "C"
