/*
 * lfa.h -- C ABI of liblfa: the singular value decomposition of periodic,
 * stride-1, multi-channel 2-D convolutions by local Fourier analysis (LFA),
 * on AMD Instinct MI355X (gfx950).
 *
 * The method (Sec. III of the paper, "Convolution Theorem" and Algorithm 1):
 * a convolution (A*f)(x) = sum_y M_y f(x+y) on a periodic n x m grid with
 * c_in input and c_out output channels is block diagonal in the Fourier
 * basis.  At each frequency k = (p/n, q/m) of the dual torus its block is the
 * c_out x c_in complex "symbol"
 *
 *     A_k = sum_{y in N} M_y * exp(+2 pi i <k, y>),
 *
 * and the SVD of the whole operator is the union over k of the SVDs
 * A_k = U_k S_k V_k^*.  This library computes the symbols (Algorithm 1,
 * symbol step) and their SVD (Algorithm 1, SVD step) on the GPU, plus top-k
 * selection and the adjoint that maps d(sum of selected sigma) back to the
 * weights, spectral functions of the operator through the SVD, and the
 * crystal form of strided layers.
 *
 * Conventions (all entry points)
 * ------------------------------
 *  - Weights W: real, PyTorch channel-first [c_out][c_in][kh][kw], contiguous.
 *    Tap (a, b) sits at offset y = (a - (kh-1)/2, b - (kw-1)/2) (integer
 *    division): the kernel neighbourhood is centred at x (stencil figure of
 *    Sec. III).  The first grid axis has length n, the second m.
 *  - Frequencies are enumerated row-major: theta index t = p*m + q.
 *  - Symbols A: [n][m][c_out][c_in] complex, interleaved (re, im) -- the
 *    layout of torch.complex64 / complex128 and of the paper's row-major
 *    transformed tensor (Sec. IV, "Memory Layout Effects").
 *  - r = min(c_out, c_in).  sigma: [n][m][r] real, descending per frequency.
 *    U: [n][m][c_out][r] complex; V: [n][m][c_in][r] complex (thin SVD,
 *    A_k = U_k diag(sigma_k) V_k^H).  Where sigma_j(k) == 0 the column u_j is
 *    an arbitrary unit vector orthogonal to the other columns.
 *  - dtype LFA_F32: W and sigma are float, A/U/V complex float.
 *    dtype LFA_F64: double / complex double throughout.
 *  - Every array argument that is "per layer" is a host array of num_layers
 *    device pointers.  All device buffers are allocated and owned by the
 *    caller.  The plan owns small constant tables (twiddles, work lists),
 *    uploaded to a device by lfa_plan_create when a gfx950 device is
 *    current, else by lfa_plan_prepare or on the plan's first compute call
 *    (and, for lfa_sigma_grad_persistent, on the first call with a new k);
 *    lfa_plan_destroy frees them.  Apart from those first-use uploads, which
 *    a prepared plan never makes (under stream capture a compute call
 *    returns LFA_ERR_NOT_PREPARED rather than upload), compute calls
 *    allocate no device memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).  All
 *    compute calls are asynchronous on that stream; the return value covers
 *    only the checks made at enqueue time.
 *  - Return value: LFA_OK (0) on success, a negative LFA_ERR_* on error.
 *    After an LFA_ERR_HIP, lfa_last_hip_error() returns the hipError_t of the
 *    failing HIP call (per thread).
 *  - A plan is immutable after lfa_plan_create/lfa_autotune and may be used
 *    from several threads at once, as long as concurrent calls use distinct
 *    workspaces and outputs.
 */
#ifndef LFA_H
#define LFA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LFA_VERSION 1

typedef struct lfa_plan lfa_plan;
typedef struct lfa_graph lfa_graph;

/* One stride-1, periodic convolution layer. */
typedef struct lfa_layer {
    int32_t c_out, c_in; /* channels: the symbol is c_out x c_in           */
    int32_t kh, kw;      /* kernel extent; 1 <= kh <= n, 1 <= kw <= m        */
    int32_t n, m;        /* periodic grid; n*m symbols                      */
} lfa_layer;

enum lfa_dtype { LFA_F32 = 0, LFA_F64 = 1 };

enum lfa_flags {
    LFA_WANT_U = 1u,      /* lfa_svd writes U                                   */
    LFA_WANT_V = 2u,      /* lfa_svd writes V                                   */
    LFA_ASM_MFMA = 4u,    /* lfa_svd assembles symbols with the MFMA kernel into
                             the workspace first (FP32 matrix cores) instead of
                             fusing the assembly into the SVD kernel           */
    LFA_ASM_BF16X2 = 8u,  /* as LFA_ASM_MFMA, split-BF16 with 3 products
                             (hi*hi + hi*lo + lo*hi), FP32 accumulation          */
    LFA_ASM_BF16X3 = 16u, /* as LFA_ASM_MFMA, split-BF16 with 6 products
                             (three-term split), FP32 accumulation               */
    LFA_PHASE_NORMALIZE = 32u  /* fix the phase of every singular pair: a pair
                             (u_j, v_j) is determined only up to a common factor
                             e^{i phi}; the SVD calls that write U or V multiply
                             both by the factor that makes the entry of largest
                             modulus of v_j real and positive (the lowest row
                             on ties), or of u_j when the plan writes U alone.
                             Post-processing of Algorithm 1's SVD step; needs
                             LFA_WANT_U or LFA_WANT_V (else INVALID_ARG)        */
};

enum lfa_status {
    LFA_OK = 0,
    LFA_ERR_INVALID_ARG = -1, /* null required pointer, bad sizes, kh > n ...  */
    LFA_ERR_UNSUPPORTED = -2, /* dtype/flag combination or size not supported  */
    LFA_ERR_WORKSPACE = -3,   /* workspace missing or smaller than required    */
    LFA_ERR_HIP = -4,         /* a HIP runtime call or kernel launch failed    */
    LFA_ERR_NO_DEVICE = -5,   /* no usable gfx950 device                       */
    LFA_ERR_NOT_PREPARED = -6,/* the call would have to upload device tables
                                 (first use on a device, or a new k for the
                                 persistent gradient) while its stream is
                                 capturing a graph: call lfa_plan_prepare first */
    /* Warnings (> 0, a bit set) returned by lfa_info_status once the
     * results are on the host: the outputs are written either way. */
    LFA_WARN_NOT_CONVERGED = 1, /* some symbol hit the plan's sweep cap        */
    LFA_WARN_NONFINITE = 2,     /* some singular value is NaN or infinite
                                   (non-finite weights)                        */
    LFA_WARN_TEAM_TIMEOUT = 4   /* a work-group team's barrier gave up waiting
                                   (that layer's results are not valid)        */
};

/* Per-layer convergence record written by the SVD entry points into the
 * caller's device buffer `info` (int32, LFA_INFO_WORDS per layer).  The
 * library clears it on the stream before use.  Symbols are those actually
 * decomposed (one per conjugate pair for real weights); a symbol that hit the
 * cap is counted in the bin of the cap. */
enum lfa_info_word {
    LFA_INFO_NONCONVERGED = 0, /* symbols that hit the sweep cap               */
    LFA_INFO_MAX_SWEEPS = 1,   /* largest number of sweeps used by a symbol    */
    LFA_INFO_SUM_SWEEPS = 2,   /* total sweeps over the layer's symbols        */
    LFA_INFO_NONFINITE = 3,    /* bit 1: a singular value of the layer is not
                                  finite; bit 2: a team barrier timed out      */
    LFA_INFO_HIST = 4,         /* LFA_INFO_HIST + s: symbols that used s sweeps,
                                  s = 0 .. 40 (the largest sweep cap)          */
    LFA_INFO_HIST_BINS = 41,
    LFA_INFO_WORDS = 45
};

/* Warnings of a finished call, from a host copy of its `info` record
 * ([num_layers][LFA_INFO_WORDS]): LFA_OK, or the OR of the LFA_WARN_* bits
 * that apply to any layer.  This is how a non-converged or non-finite
 * result is reported: the compute calls themselves are asynchronous, so
 * their return value cannot.  Errors: LFA_ERR_INVALID_ARG (NULL, num_layers
 * < 1).  Host only. */
int lfa_info_status(const int32_t* info, int32_t num_layers);

/* ---- plans -------------------------------------------------------------- */

/* Validate the layers and build a plan: size class and launch shape of each
 * layer, the work list of the persistent batched launch, and device twiddle
 * tables exp(2 pi i j / n) computed on the host in double precision (the grid
 * of Algorithm 1's Init step).  The device tables are uploaded to the
 * current device when it is a gfx950 device, else on first use (see
 * lfa_plan_prepare), so this call itself needs no GPU.
 *   out        : receives the plan (set to NULL on error)
 *   layers     : host array of num_layers descriptors (copied)
 *   num_layers : >= 1
 *   dtype      : LFA_F32 or LFA_F64
 *   flags      : OR of lfa_flags.  BF16/MFMA assembly requires LFA_F32.
 * Errors: INVALID_ARG for null pointers, non-positive sizes, kh > n, kw > m
 * (taps would alias); UNSUPPORTED for r > 1024, kh*kw > 128, or a flag that
 * does not fit the dtype. */
int lfa_plan_create(lfa_plan** out, const lfa_layer* layers, int32_t num_layers,
                    int32_t dtype, uint32_t flags);

/* Upload the plan's device tables (twiddles, persistent work list) to the
 * current device and, for k > 0, build and upload the work list of
 * lfa_sigma_grad_persistent for that k.  lfa_plan_create already does the
 * first when a gfx950 device is current; compute calls do both on first
 * use.  Needed before capturing calls of a plan into a graph on a device
 * where the plan has not run yet (or with a new k): under stream capture the
 * compute calls allocate nothing and return LFA_ERR_NOT_PREPARED instead.
 * Synchronous; allocates small device tables freed by lfa_plan_destroy.
 * Errors: LFA_ERR_INVALID_ARG (NULL, k < 0, k invalid as for lfa_topk, or a
 * device other than the one the plan was prepared on), LFA_ERR_NO_DEVICE,
 * LFA_ERR_HIP. */
int lfa_plan_prepare(lfa_plan* plan, int32_t k);

/* Lower the plan's cap on Jacobi sweeps per symbol (1 .. 40; the default is
 * 40).  A symbol that reaches the cap stops there, its results are written
 * from the last sweep, and it is counted in LFA_INFO_NONCONVERGED (see
 * lfa_info_status).  Call it before compute calls on the plan, not
 * concurrently with them.  Errors: LFA_ERR_INVALID_ARG. */
int lfa_plan_set_max_sweeps(lfa_plan* plan, int32_t max_sweeps);

/* Phase record of the register kernel, for measurement: the split of the
 * step into its stages that the paper's Table III reports as transformation
 * and SVD time, here for a kernel that fuses them.  With `ticks` a device
 * buffer of 4 uint64 (cleared by the caller), every later lfa_svd launch of
 * the register kernel (symbols of at most 64 rows) adds, for each group of
 * symbols it runs, the real-time-clock ticks (100 MHz) its work-group spent
 * in: [0] loading the symbols (assembly from W, or the restore of a saved
 * turn of the work queue), [1] the sweeps, [2] the finish (norms, sort,
 * normalisation, completion, writing sigma, U, V), [3] saving a turn.  The
 * sums are work-group time, not wall time: their shares apportion a
 * launch's duration.  Other kernels and entry points ignore it; NULL stops
 * recording.  The buffer must outlive the launches that use it.
 * Errors: LFA_ERR_INVALID_ARG (NULL plan).  Host only. */
int lfa_plan_record_phases(lfa_plan* plan, unsigned long long* ticks);

/* Free the plan and its device tables.  NULL is accepted. */
int lfa_plan_destroy(lfa_plan* plan);

/* Bytes of device workspace every compute call on this plan needs (the
 * maximum over entry points).  Writes 0 if none. */
int lfa_plan_workspace_bytes(const lfa_plan* plan, size_t* bytes);

/* Number of layers, and a copy of layer i's descriptor. */
int lfa_plan_num_layers(const lfa_plan* plan, int32_t* num_layers);
int lfa_plan_layer(const lfa_plan* plan, int32_t i, lfa_layer* layer);

/* ---- symbol assembly (Algorithm 1, symbol step) ----------------------- */

/* A[layer][p][q][:, :] = sum_y W[layer][:, :, y] exp(+2 pi i <k, y>)
 * (Sec. III "Convolution Theorem"; Algorithm 1 symbol step), for every
 * frequency.  W: per-layer device pointers to weights; A: per-layer device
 * pointers to [n][m][c_out][c_in] complex outputs.  The assembly kernel is
 * chosen by the plan's flags: LFA_ASM_BF16X2 / X3 use split-BF16 matrix
 * cores, LFA_ASM_MFMA FP32 matrix cores, otherwise a vector kernel
 * (FP32 or FP64 per dtype).  No workspace is used. */
int lfa_symbols(const lfa_plan* plan, const void* const* W, void* const* A, void* stream);

/* ---- SVD of every symbol (Algorithm 1, symbol and SVD steps) --------- */

/* For every layer and frequency, the SVD of the symbol (Sec. III
 * "Convolution Theorem"; Algorithm 1 SVD step) by one-sided Jacobi,
 * singular values sorted descending.
 *   W     : per-layer weights (device)
 *   sigma : per-layer [n][m][r] outputs (device), required
 *   U, V  : per-layer outputs, required iff the plan has LFA_WANT_U /
 *           LFA_WANT_V, ignored (may be NULL) otherwise
 *   info  : device int32 [num_layers][LFA_INFO_WORDS] or NULL
 *   ws    : device workspace of ws_bytes >= lfa_plan_workspace_bytes
 * The plain path: one launch per layer (plus one assembly launch per layer
 * when the plan asks for MFMA/BF16 assembly, and one phase launch per layer
 * with LFA_PHASE_NORMALIZE). */
int lfa_svd(const lfa_plan* plan, const void* const* W, void* const* sigma, void* const* U,
            void* const* V, int32_t* info, void* ws, size_t ws_bytes, void* stream);

/* lfa_svd for callers that cannot allocate device memory (code under graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and outputs, with no workspace argument.  Its scratch is a
 * static device array of the library, 64 MiB on each device that runs it,
 * held from the library's first use on that device until the process ends;
 * nothing is allocated or freed by the call (the plan must already be
 * prepared on the current device: lfa_plan_create does that when a gfx950
 * device is current, else call lfa_plan_prepare).  It runs the plan's own
 * launch when that fits the scratch, else the same kernels without the
 * register kernel's work queue (bitwise the same results).  All calls on one
 * device share that device's scratch, which keeps the last call's contents
 * (the kernels clear what must start at zero): calls that overlap in time on
 * one device race and give wrong results -- serialise them (one stream, or
 * events).
 * Errors: as lfa_svd, plus LFA_ERR_WORKSPACE when the plan's layers need
 * more than the 64 MiB scratch even without the work queue (e.g. large
 * symbols, whose blocked kernel keeps every symbol in a global slot), and
 * LFA_ERR_NOT_PREPARED when the plan's tables are not on the current device. */
int lfa_svd_noalloc(const lfa_plan* plan, const void* const* W, void* const* sigma, void* const* U,
                    void* const* V, int32_t* info, void* stream);

/* Same results as lfa_svd for all layers of the plan in ONE persistent
 * launch: work-groups take (layer, frequency) items from a device work list,
 * largest symbols first.  Fused FP32/FP64 assembly only (no MFMA/BF16 flag). */
int lfa_svd_persistent(const lfa_plan* plan, const void* const* W, void* const* sigma,
                       void* const* U, void* const* V, int32_t* info, void* ws,
                       size_t ws_bytes, void* stream);

/* Measurement form of lfa_svd_persistent: the same launch and results, and
 * a record per work-group of the launch written to `busy` (device int64
 * [busy_len][4]): ticks of the 100 MHz device clock from taking its first
 * item to finishing its last, items taken, the XCD (XCC_ID register) and the
 * shader-engine / array / compute-unit bits of its HW_ID register (bits
 * 8..15), which together name the compute unit it ran on.  busy_len must be
 * at least lfa_plan_persistent_grid's value; with more than 12 layers (more
 * than one launch) the records are those of the last launch.  Errors: as lfa_svd_persistent, plus
 * LFA_ERR_INVALID_ARG for a NULL or short `busy`. */
int lfa_svd_persistent_busy(const lfa_plan* plan, const void* const* W, void* const* sigma, void* const* U,
                            void* const* V, int32_t* info, void* ws, size_t ws_bytes, int64_t* busy,
                            int32_t busy_len, void* stream);

/* Work-groups of the plan's persistent launch on the current device (the
 * largest over its launches). */
int lfa_plan_persistent_grid(const lfa_plan* plan, int32_t* grid);

/* SVD of symbols the caller already holds (e.g. from lfa_symbols), same
 * outputs as lfa_svd.  A: per-layer [n][m][c_out][c_in] complex (device).
 * Every symbol is decomposed: caller symbols need not come in conjugate
 * pairs (lfa_svd decomposes one symbol per pair of frequencies k, -k). */
int lfa_svd_symbols(const lfa_plan* plan, const void* const* A, void* const* sigma,
                    void* const* U, void* const* V, int32_t* info, void* ws,
                    size_t ws_bytes, void* stream);

/* ---- top-k per layer ------------------------------------------------- */

/* The k largest singular values of each layer over all (p, q, j), ordered by
 * value descending, ties by flat index (p, q, j) ascending.
 *   sigma : per-layer [n][m][r] (device, dtype of the plan)
 *   k     : 1 <= k <= 64 and k <= n*m*r of every layer
 *   vals  : device [num_layers][k] (dtype of the plan)
 *   idx   : device int32 [num_layers][k][3] = (p, q, j)
 * One launch for all layers. */
int lfa_topk(const lfa_plan* plan, const void* const* sigma, int32_t k, void* vals,
             int32_t* idx, void* stream);

/* ---- adjoint: gradient of a sum of singular values -------------------- */

/* dW[layer][o][i][a][b] = sum_s g[layer][s] *
 *     Re( exp(-2 pi i <k_s, y_ab>) * U_s[o] * conj(V_s[i]) )
 * the gradient of sum_s g_s sigma_{j_s}(k_s) for simple singular values
 * (first-order perturbation d sigma = Re(u^H dA v)).  dW is overwritten.
 *   U, V  : per-layer full SVD outputs as written by lfa_svd
 *   idx   : device int32 [num_layers][k][3] (p, q, j), e.g. from lfa_topk
 *   grad  : device [num_layers][k] weights g (dtype of the plan)
 *   dW    : per-layer device outputs shaped like W
 * One launch for all layers. */
int lfa_adjoint(const lfa_plan* plan, const void* const* U, const void* const* V,
                const int32_t* idx, const void* grad, int32_t k, void* const* dW,
                void* stream);

/* As lfa_adjoint, from one side of the singular vectors: the side the
 * one-sided Jacobi working matrix converges to, which an SVD call writes
 * without a rotation accumulator -- U (c_out x r) of a layer with
 * c_out >= c_in, V (c_in x r) of one with c_out < c_in.  For each pick
 * (p, q, j) the other vector follows from the weights,
 *     v = A_k^H u / sigma_j(k)   or   u = A_k v / sigma_j(k)
 * (the SVD relations A v = sigma u, A^H u = sigma v; Sec. III "Convolution
 * Theorem" for A_k), with A_k assembled from W in the kernel; a pick with
 * sigma <= 0 adds nothing.  Accurate for the large singular values a top-k
 * picks (the relative error of the recomputed vector is about
 * u sigma_max / sigma_j).  Two launches: the other vectors (one work-group
 * per pick), then the adjoint.
 *   W     : per-layer weights (device)
 *   sigma : per-layer [n][m][r] singular values from the same SVD
 *   X     : per-layer kept side, [n][m][c_out][r] (U) or [n][m][c_in][r] (V)
 *   idx, grad, k, dW : as lfa_adjoint
 *   ws    : workspace of lfa_plan_workspace_bytes (per-pick vectors)
 * Errors: as lfa_adjoint, plus LFA_ERR_WORKSPACE. */
int lfa_adjoint_onesided(const lfa_plan* plan, const void* const* W, const void* const* sigma,
                         const void* const* X, const int32_t* idx, const void* grad, int32_t k,
                         void* const* dW, void* ws, size_t ws_bytes, void* stream);

/* As lfa_adjoint, but recomputes the singular vectors of only the selected
 * symbols (at most k per layer) from W into the workspace, so the forward
 * pass can be sigma-only.  Two launches (SVD of the selected symbols, then
 * the adjoint). */
int lfa_sigma_grad(const lfa_plan* plan, const void* const* W, const int32_t* idx,
                   const void* grad, int32_t k, void* const* dW, void* ws, size_t ws_bytes,
                   void* stream);

/* Same result as lfa_sigma_grad in two launches for all layers: one
 * persistent launch computes the singular vectors of the k selected symbols
 * of every layer (work-group teams share the large symbols), then one adjoint
 * launch.  The work list for a given k is built and uploaded by
 * lfa_plan_prepare(plan, k), or on the first call with that k
 * (synchronously; LFA_ERR_NOT_PREPARED under stream capture). */
int lfa_sigma_grad_persistent(const lfa_plan* plan, const void* const* W, const int32_t* idx,
                              const void* grad, int32_t k, void* const* dW, void* ws,
                              size_t ws_bytes, void* stream);

/* ---- batched forward + backward as one HIP graph ---------------------- */

/* Capture [lfa_svd_persistent (sigma only) -> lfa_topk -> lfa_sigma_grad_persistent]
 * for fixed buffers into a HIP graph.  Replaying it with new contents in W
 * recomputes sigma, the top-k and dW.  `grad` holds g for every selected
 * value (e.g. all ones for L = sum of the top-k).  Buffers must stay alive
 * and at the same addresses while the graph exists. */
int lfa_graph_create(lfa_plan* plan, const void* const* W, void* const* sigma, int32_t k,
                     void* vals, int32_t* idx, const void* grad, void* const* dW,
                     int32_t* info, void* ws, size_t ws_bytes, void* stream, lfa_graph** out);
/* The same step with the forward pass keeping every symbol's singular
 * vectors: [lfa_svd_persistent with U and V -> lfa_topk -> lfa_adjoint].
 * The gradient then needs no second SVD of the selected symbols (the
 * derivative of a simple singular value, Re(u^H dA v), takes only its own
 * singular vectors).  That is faster when the largest symbols dominate (for
 * instance the twelve 3x3 layers of ResNet-18 on 32x32 inputs), at the price
 * of U and V storage for every symbol.
 *   plan : must have both LFA_WANT_U and LFA_WANT_V (else UNSUPPORTED)
 *   U, V : per-layer device outputs as for lfa_svd, required (INVALID_ARG
 *          if NULL); they hold the last replay's singular vectors
 * Other arguments, ownership and errors as lfa_graph_create. */
int lfa_graph_create_uv(lfa_plan* plan, const void* const* W, void* const* sigma, void* const* U,
                        void* const* V, int32_t k, void* vals, int32_t* idx, const void* grad,
                        void* const* dW, int32_t* info, void* ws, size_t ws_bytes, void* stream,
                        lfa_graph** out);
/* The step with a one-sided forward pass: [lfa_svd_persistent keeping only
 * the side of every layer that needs no rotation accumulator -> lfa_topk ->
 * lfa_adjoint_onesided].  The forward pass costs about what a sigma-only one
 * does, and the gradient needs no second SVD.
 *   plan : every layer tall (c_out >= c_in) with exactly LFA_WANT_U, or every
 *          layer wide with exactly LFA_WANT_V (else UNSUPPORTED)
 *   X    : per-layer device outputs for that side (U or V as lfa_svd writes
 *          them), required; they hold the last replay's vectors
 * Other arguments, ownership and errors as lfa_graph_create. */
int lfa_graph_create_onesided(lfa_plan* plan, const void* const* W, void* const* sigma, void* const* X,
                              int32_t k, void* vals, int32_t* idx, const void* grad, void* const* dW,
                              int32_t* info, void* ws, size_t ws_bytes, void* stream, lfa_graph** out);
int lfa_graph_launch(lfa_graph* graph, void* stream);
int lfa_graph_destroy(lfa_graph* graph);

/* ---- spectral functions of a layer's operator ------------------------- */

/* The global SVD of the periodic operator is the lift of the symbols' SVDs
 * (Sec. III "Convolution Theorem": its singular vectors are Fourier modes
 * times the columns of U_k, V_k), so a function of its singular values acts
 * frequency by frequency:
 *   x_hat_k = sum_x x(x) e^{-2 pi i <k, x>},  y_hat_k = g_k(x_hat_k),
 *   y(x) = (1/(n m)) sum_k y_hat_k e^{+2 pi i <k, x>}   (real part). */
enum lfa_spectral_kind {
    LFA_SPECTRAL_IDENTITY = 0, /* g_k = U_k S_k V_k^*: the convolution itself     */
    LFA_SPECTRAL_CLIP = 1,     /* g_k = U_k min(S_k, param) V_k^*: singular values
                                  clipped at param (a Lipschitz bound)           */
    LFA_SPECTRAL_PINV = 2,     /* g_k = V_k S_k^+ U_k^*: pseudo-inverse, 1/sigma for
                                  sigma > param (absolute cut-off), 0 otherwise;
                                  maps c_out channels back to c_in               */
    LFA_SPECTRAL_TRUNCATE = 3  /* g_k = U_k T(S_k) V_k^*, T(sigma) = sigma for
                                  sigma > param, else 0: the low-rank truncation
                                  of the operator that keeps its singular values
                                  above param (with param = the R-th largest
                                  singular value of the layer and distinct values,
                                  the best rank-(R-1) approximation)             */
};

/* Workspace (device bytes) of lfa_apply for `batch` images of layer `layer`:
 * two complex buffers of batch * n * m * max(c_out, c_in) elements. */
int lfa_apply_workspace_bytes(const lfa_plan* plan, int32_t layer, int32_t batch, size_t* bytes);

/* Apply a spectral function of layer `layer`'s operator to a batch of
 * images, using that layer's SVD as lfa_svd writes it (with LFA_WANT_U and
 * LFA_WANT_V).  All pointers are device memory in the plan's dtype:
 *   sigma [n][m][r], U [n][m][c_out][r], V [n][m][c_in][r]  (r = min(c_out, c_in))
 *   x     [batch][c_x][n][m] real,  y [batch][c_y][n][m] real,
 *         c_x = c_in, c_y = c_out (IDENTITY, CLIP, TRUNCATE); c_x = c_out, c_y = c_in (PINV)
 *   kind  an lfa_spectral_kind; param >= 0 (CLIP level, PINV and TRUNCATE cut-off)
 *   ws    at least lfa_apply_workspace_bytes(plan, layer, batch)
 * Stream-ordered; batch == 0 does nothing.  x and y may not overlap.
 * Errors: LFA_ERR_INVALID_ARG (layer, kind, param, batch < 0, NULL pointer),
 * LFA_ERR_WORKSPACE, LFA_ERR_UNSUPPORTED (the per-frequency map of 8 images
 * does not fit one work-group's LDS: c_x + r beyond about 2200 in FP32,
 * 1000 in FP64), LFA_ERR_HIP. */
int lfa_apply(const lfa_plan* plan, int32_t layer, const void* sigma, const void* U, const void* V,
              int32_t kind, double param, const void* x, void* y, int32_t batch, void* ws,
              size_t ws_bytes, void* stream);

/* Global singular vectors of the periodic operator (Sec. III "Convolution
 * Theorem": they are the Fourier modes of a frequency k times the singular
 * vectors of the symbol A_k) for `count` picks (p, q, j) of layer `layer`,
 * as complex images:
 *   u_hat[t][o][x1][x2] = e^{2 pi i (p x1 / n + q x2 / m)} U[p][q][o][j] / sqrt(n m)
 *   v_hat[t][i][x1][x2] = e^{2 pi i (p x1 / n + q x2 / m)} V[p][q][i][j] / sqrt(n m)
 * so that the operator maps v_hat to sigma_j(k) u_hat, and both have unit
 * norm.  All pointers are device memory:
 *   U [n][m][c_out][r], V [n][m][c_in][r]  complex, as lfa_svd writes them
 *   idx   int32 [count][3] = (p, q, j), e.g. one layer's rows of lfa_topk
 *   u_hat [count][c_out][n][m], v_hat [count][c_in][n][m]  complex, plan's dtype
 * u_hat or v_hat may be NULL (not written; then U or V may be NULL too).  A
 * pick out of range (p not in [0, n), q not in [0, m) or j not in [0, r))
 * gives zero vectors.  Stream-ordered; count == 0 does nothing.
 * Errors: LFA_ERR_INVALID_ARG (layer, count < 0, idx NULL, an output without
 * its input), LFA_ERR_UNSUPPORTED (count * max(c_out, c_in) beyond 2^31 - 1),
 * LFA_ERR_HIP. */
int lfa_lift(const lfa_plan* plan, int32_t layer, const void* U, const void* V, const int32_t* idx,
             int32_t count, void* u_hat, void* v_hat, void* stream);

/* ---- strided layers as crystals ------------------------------------------ */

/* A stride-s periodic convolution y(x) = sum_y M_y f(s x + y) (f on the
 * n x m torus, y on the (n/s) x (m/s) torus, taps centred as for stride 1)
 * is, with its input read as a crystal of s*s*c_in points per cell of the
 * coarse lattice (Sec. III, "Introduction to Lattices and Crystals"), a
 * stride-1 layer on the coarse torus.  The point d = (d1, d2) in [0, s)^2 of
 * cell X, channel i, is its input channel i*s*s + d1*s + d2 (the order of
 * torch's pixel_unshuffle), and a tap at offset y reaches it through the
 * coarse offset floor(y / s), with d = y mod s.  Its symbols, SVD, top-k,
 * gradient and spectral functions are those of that stride-1 layer, with
 * the plan's limits applying to it (kh' <= n/s, channels up to 512). */
enum lfa_crystal_direction {
    LFA_CRYSTAL_FORWARD = 0,   /* W [c_out][c_in][kh][kw] -> Wc [c_out][s*s*c_in][kh'][kw']
                                  (taps of Wc that no tap of W reaches are 0) */
    LFA_CRYSTAL_ADJOINT = 1    /* Wc -> W: each tap read from its place in Wc,
                                  the transpose of FORWARD (maps a gradient with
                                  respect to Wc to one with respect to W)      */
};

/* The stride-1 layer of the crystal form of `layer` with stride `stride`:
 * {c_out, s*s*c_in, kh', kw', n/s, m/s}, kh' = max(2L+1, 2R) for the coarse
 * offsets [-L, R] of the taps (3x3, s = 2: 3x3; 7x7, s = 2: 5x5; 1x1: 1x1).
 * Host only.  Errors: LFA_ERR_INVALID_ARG (NULL, stride < 1, dims <= 0,
 * kh > n or kw > m, s not dividing n and m). */
int lfa_crystal_layer(const lfa_layer* layer, int32_t stride, lfa_layer* out);

/* Repack weights between a stride-s layer and its crystal form (device
 * pointers in `dtype`, src and dst not overlapping; dst fully written).
 * Stream-ordered.  Errors: those of lfa_crystal_layer, LFA_ERR_INVALID_ARG
 * (dtype, direction, NULL pointer), LFA_ERR_HIP. */
int lfa_crystal_weights(const lfa_layer* layer, int32_t stride, int32_t dtype, const void* src, void* dst,
                        int32_t direction, void* stream);

/* ---- tuning and diagnostics ------------------------------------------- */

/* What lfa_autotune tunes (OR of these). */
enum lfa_tune_what {
    LFA_TUNE_LAYERS = 1u,      /* per layer, for lfa_svd: QR factors or not, matrix-
                                  core assembly for kernels of 25 taps or more, the
                                  register kernel's work-queue turns, the blocked
                                  kernel's work-groups per symbol                 */
    LFA_TUNE_PERSISTENT = 2u   /* the cost model behind the persistent launch's work
                                  list (lfa_svd_persistent, the graphs): relative
                                  cost of register-kernel bundles, team overhead */
};

/* Choose the plan's launch parameters by timing candidates on the caller's
 * weights (convergence, and so time, depends on the data), one knob at a
 * time from the plan's defaults (a cost model), keeping a candidate only if
 * it is faster, and store the choices in the plan.  Layers of one shape are
 * tuned once.  Results are identical up to rounding whatever is chosen.
 *   W, sigma, U, V : as for lfa_svd; sigma/U/V are overwritten
 *   cache_path     : JSON file of earlier choices, keyed by GPU architecture,
 *                    dtype, flags and layer shape (and the whole layer list for
 *                    the persistent cost model), or NULL for no cache.  Found
 *                    entries are applied without timing; new ones are added
 *                    and the file rewritten (through a temporary file).
 *   what           : OR of lfa_tune_what
 * Synchronous; allocates (and frees) its own device workspace, and uploads a
 * new persistent work list.  Not concurrently with other calls on the plan,
 * and not while `stream` captures a graph.  Afterwards
 * lfa_plan_workspace_bytes may report a different size: query it again.
 * Errors: LFA_ERR_INVALID_ARG (NULL plan or outputs, unknown `what` bits, a
 * capturing stream, an unwritable cache file), LFA_ERR_NO_DEVICE,
 * LFA_ERR_HIP. */
int lfa_autotune(lfa_plan* plan, const void* const* W, void* const* sigma, void* const* U,
                 void* const* V, const char* cache_path, uint32_t what, void* stream);

/* The current choices for a layer (autotuned or default): QR factors (0/1),
 * work-queue sweeps per turn (-1 automatic, 0 off), work-groups per symbol
 * of the blocked kernel (0 automatic), materialised matrix-core assembly
 * (-1 as the plan's flags, 0 fused, 1 on).  Any output may be NULL. */
int lfa_plan_tuning(const lfa_plan* plan, int32_t layer, int32_t* qr, int32_t* queue_seg,
                    int32_t* team_w, int32_t* asm_mat);

/* The persistent work list's cost model: seconds per unit (N^2 M) of a
 * register-kernel wave and of a 256-thread blocked work-group, and the
 * per-member overhead factor of a team of work-groups. */
int lfa_plan_cost_model(const lfa_plan* plan, double* wave_s, double* block_s, double* team_ovh);

/* Launch shape chosen for a layer: lanes per column pair, threads per
 * work-group, symbols per work-group and storage (0 = LDS, 1 = global). */
int lfa_plan_launch_shape(const lfa_plan* plan, int32_t layer, int32_t* lanes_per_pair,
                          int32_t* threads, int32_t* symbols_per_group, int32_t* storage);

/* Whether lfa_svd runs layer `layer` through QR preconditioning (*qr = 1):
 * the N x N Cholesky factors R of the symbols' Gram matrices, formed in FP64
 * from the Gram convolution's taps, then the one-sided Jacobi SVD of R,
 * whose N rows replace the symbol's M (the singular values of R and of the
 * symbol agree to about sqrt(N u64) sigma_max); with singular vectors the
 * SVD of R keeps V and U follows from G V.  Chosen at plan creation for
 * FP32 plans (any flags but the matrix-core assembly ones) whose working
 * matrices have M > 64 rows and M >= 1.25 N, when the factors are small
 * enough for the register kernel (N <= 64) or the layer has at least 256
 * symbols to decompose (one per conjugate pair); lfa_autotune may change
 * it.  The environment variable LFA_QR, read at plan creation, turns it off
 * ("0") or on for every layer of such a shape ("1").  Host only. */
int lfa_plan_preconditioned(const lfa_plan* plan, int32_t layer, int32_t* qr);

/* Work-queue launch of a layer's register kernel (symbols of at most 64
 * rows) on the current device.  When the groups of symbols fill the resident
 * work-groups more than once (and at most 4 times), lfa_svd runs a grid of
 * resident work-groups that take groups from a device queue a few sweeps at
 * a time, saving the state of unfinished groups in the workspace, so that no
 * group starts late in a partly filled last round; the results are bitwise
 * those of the one-work-group-per-group launch.
 *   resident        : work-groups of that launch that fit on the device at
 *                     once (0: no work-queue launch for this layer)
 *   sweeps_per_turn : sweeps a group runs per turn for lfa_svd of the
 *                     layer (0: one work-group per group instead)
 * The environment variable LFA_WAVE_QUEUE, read by lfa_plan_create, turns
 * the work queue off ("0") or forces it with k sweeps per turn ("1" .. "16").
 * Needs a gfx950 device (LFA_ERR_NO_DEVICE otherwise). */
int lfa_plan_queue_info(lfa_plan* plan, int32_t layer, int32_t* resident,
                        int32_t* sweeps_per_turn);

/* Static text for a status code; never NULL. */
const char* lfa_status_string(int status);

/* hipError_t of the last failing HIP call on this thread (0 if none). */
int lfa_last_hip_error(void);

/* LFA_VERSION of the built library. */
int lfa_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LFA_H */
