// QR preconditioning of tall symbols (M > N rows of the working matrix):
// the one-sided Jacobi SVD then works on the N x N triangular factor R of
// the symbol instead of the M x N symbol, since G = Q R gives sigma(G) =
// sigma(R) and the same right singular vectors.  R comes from the Cholesky
// factor of the Gram matrix H = G^H G, formed and factored in FP64.
//
// The Gram matrix of every frequency is itself a symbol.  With
// G_k[r][c] = sum_y Wg[r][c][y] e^{2 pi i s <k, y>} (Wg the weights seen from
// the working matrix: G = A, s = +1, r = output channel, c = input channel;
// or G = A^H, s = -1, r = input, c = output channel),
//     H_k = G_k^H G_k = sum_delta C_delta e^{2 pi i s <k, delta>},
//     C_delta[c][c'] = sum over tap pairs (y, y') with y' - y = delta of
//                      sum_r Wg[r][c][y] Wg[r][c'][y'],
// the (2 kh - 1)(2 kw - 1) real N x N matrices C_delta (the taps of the
// Gram convolution A^* A or A A^*).  They are formed once per layer
// (gram_taps_kernel); each frequency's H_k is then an assembly over those
// taps, followed by a blocked right-looking Cholesky factorisation
// (gram_cholesky_kernel), both in FP64.
//
// Rounding: C and H carry FP64 rounding (about N u64 ||H||); so do the
// Cholesky factors (backward error about N u64 ||H||).  A pivot at most
// tau = 4 N u64 times the largest diagonal of H (a numerically singular
// Gram matrix: a rank-deficient symbol) gives a zero row of R.  Either way
// sigma(R)^2 = sigma(G)^2 + O(N u64 sigma_max^2), so the singular values of
// R in FP32 match those of G to about sqrt(N u64) sigma_max (3e-7 at N = 256),
// well inside the FP32 tolerance.
//
// Singular vectors: the SVD of R keeps its right singular vectors V (those
// of G), and the left ones follow as the columns of Y = G V, normalised
// (Y = U S), which are orthogonal to about u sigma_max / sigma_j (columns
// whose singular value the SVD of R found negligible are set to zero and
// completed); qr_left_kernel forms Y with G assembled from the weights, and
// the blocked kernels' finish then takes Y and V as its working matrix and
// accumulator: column norms (sigma, with the negligible-column rule), sort,
// normalisation, completion of the columns of zero singular values, and
// the writes of sigma, U and V (mirror frequencies by conjugation).
#include <hip/hip_runtime.h>

#include "jacobi_device.hpp"

namespace lfa {
namespace {
using namespace dev;

constexpr int kGramTile = 32;     // output tile of C_delta (c, c')
constexpr int kGramRows = 16;     // rows r per staged chunk
constexpr int kPanelMax = 16;     // rows of R per Cholesky panel, at most

// C_delta for delta = blockIdx.z, tiles (blockIdx.x, blockIdx.y) of (c, c').
// 256 threads: thread (tx, ty) in 32 x 8 computes c = c0 + tx, c' = c0' + ty + 8 e.
template <typename R>
__global__ void __launch_bounds__(256) gram_taps_kernel(GramArgs<R> g) {
    __shared__ double wa[kGramRows][kGramTile + 1];
    __shared__ double wb[kGramRows][kGramTile + 1];
    const int KD2 = 2 * g.kw - 1;
    const int d1 = (int)blockIdx.z / KD2 - (g.kh - 1), d2 = (int)blockIdx.z % KD2 - (g.kw - 1);
    const int c0 = blockIdx.x * kGramTile, e0 = blockIdx.y * kGramTile;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int T = g.kh * g.kw;
    double acc[4] = {0, 0, 0, 0};
    // tap pairs (y, y') with y' - y = delta: y = (a, b), y' = (a + d1, b + d2)
    for (int a = 0; a < g.kh; ++a) {
        const int a2 = a + d1;
        if (a2 < 0 || a2 >= g.kh) continue;
        for (int b = 0; b < g.kw; ++b) {
            const int b2 = b + d2;
            if (b2 < 0 || b2 >= g.kw) continue;
            const int t1 = a * g.kw + b, t2 = a2 * g.kw + b2;
            for (int r0 = 0; r0 < g.M; r0 += kGramRows) {
                __syncthreads();
                for (int x = threadIdx.x; x < kGramRows * kGramTile; x += 256) {
                    const int rr = x / kGramTile, cc = x - (x / kGramTile) * kGramTile;
                    const int r = r0 + rr;
                    double va = 0, vb = 0;
                    if (r < g.M) {
                        const int c = c0 + cc, e = e0 + cc;
                        // Wg[r][c][t] = W[o][i][t], (o, i) = (r, c) or (c, r)
                        if (c < g.N) va = double(g.W[(g.transposed ? ((size_t)c * g.c_in + r) : ((size_t)r * g.c_in + c)) * T + t1]);
                        if (e < g.N) vb = double(g.W[(g.transposed ? ((size_t)e * g.c_in + r) : ((size_t)r * g.c_in + e)) * T + t2]);
                    }
                    wa[rr][cc] = va;
                    wb[rr][cc] = vb;
                }
                __syncthreads();
#pragma unroll
                for (int rr = 0; rr < kGramRows; ++rr) {
                    const double x = wa[rr][tx];
#pragma unroll
                    for (int u = 0; u < 4; ++u) acc[u] = fma(x, wb[rr][ty + 8 * u], acc[u]);
                }
            }
        }
    }
    const int c = c0 + tx;
    if (c >= g.N) return;
    double* C = g.C + (size_t)blockIdx.z * g.N * g.N;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int e = e0 + ty + 8 * u;
        if (e < g.N) C[(size_t)c * g.N + e] = acc[u];
    }
}

// One work-group per decomposed frequency: H_k into its slot (upper
// triangle, FP64), then the Cholesky factor R (R^H R = H, upper) into the
// layer's R symbols [n*m][N][N] (FP32 or FP64, zeros below the diagonal),
// or its conjugate transpose R^H (lower) when g.conj_transpose is set.
// Right-looking in panels of PANEL rows: the panel's rows are staged in LDS
// (row stride N + 1, so that column reads of the panel spread over the
// banks), factored there with one barrier per row, written out as rows of R
// (or columns of R^H), and the trailing triangle of H in the slot takes the
// rank-PANEL update, each thread on 4 x 4 tiles of a folded triangle (rows
// I and nT - 1 - I of the tile triangle share one row of nT + 1 tiles), so
// that every thread has 16 loads of H in flight and reuses each panel value
// four times.  Taller panels pass over the trailing triangle fewer times;
// shorter ones take less LDS, so that more work-groups share a CU.
template <typename R, int PANEL>
__global__ void __launch_bounds__(256) gram_cholesky_kernel(GramArgs<R> g) {
    extern __shared__ __align__(16) char lds_raw[];
    const int item = blockIdx.x;
    const int theta = canonical_theta(g.n, g.m, item);
    const int p = theta / g.m, q = theta - (theta / g.m) * g.m;
    const int N = g.N, KD1 = 2 * g.kh - 1, KD2 = 2 * g.kw - 1, ND = KD1 * KD2;
    const int ldp = N + 1;                                             // LDS row stride of the panel
    cplx<double>* ph = reinterpret_cast<cplx<double>*>(lds_raw);     // [ND]
    cplx<double>* P = ph + ND;                                         // [PANEL][ldp]
    double* red = reinterpret_cast<double*>(P + (size_t)PANEL * ldp); // [256]
    cplx<double>* H = reinterpret_cast<cplx<double>*>(g.hslots) + (size_t)item * N * N;
    cplx<R>* Rk = g.Rsym + (size_t)theta * N * N;
    for (int x = threadIdx.x; x < ND; x += blockDim.x) {
        const int d1 = x / KD2 - (g.kh - 1), d2 = x % KD2 - (g.kw - 1);
        int i1 = (p * d1) % g.n;
        if (i1 < 0) i1 += g.n;
        int i2 = (q * d2) % g.m;
        if (i2 < 0) i2 += g.m;
        const double ar = g.tw[2 * (g.tw_n + i1)], ai = g.tw[2 * (g.tw_n + i1) + 1];
        const double br = g.tw[2 * (g.tw_m + i2)], bi = g.tw[2 * (g.tw_m + i2) + 1];
        const double im = ar * bi + ai * br;
        ph[x] = {ar * br - ai * bi, g.transposed ? -im : im};     // e^{2 pi i s <k, delta>}
    }
    __syncthreads();
    // H_k, upper triangle (c <= e); the largest diagonal entry for the
    // pivot threshold
    double dmax = 0;
    for (long long x = threadIdx.x; x < (long long)N * N; x += blockDim.x) {
        const int c = (int)(x / N), e = (int)(x - (x / N) * N);
        if (e < c) continue;
        double hr = 0, hi = 0;
        // unrolled: eight taps' loads in flight at a time
#pragma unroll 8
        for (int d = 0; d < ND; ++d) {
            const double v = g.C[((size_t)d * N + c) * N + e];
            hr = fma(v, ph[d].x, hr);
            hi = fma(v, ph[d].y, hi);
        }
        if (c == e) {
            hi = 0;                       // H is Hermitian: a real diagonal
            dmax = fmax(dmax, hr);
        }
        H[(size_t)c * N + e] = {hr, hi};
    }
    red[threadIdx.x] = dmax;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    const double floor = 4.0 * N * 0x1p-52 * red[0];
    __syncthreads();
    for (int k0 = 0; k0 < N; k0 += PANEL) {
        const int b = min(PANEL, N - k0), w = N - k0;
        // panel rows k0 .. k0+b-1, columns k0 .. N-1 (upper part)
        for (int r = 0; r < b; ++r) {
#pragma unroll 4
            for (int c = threadIdx.x; c < w; c += blockDim.x)
                P[(size_t)r * ldp + c] = c >= r ? H[(size_t)(k0 + r) * N + k0 + c] : cplx<double>{0, 0};
        }
        __syncthreads();
        // One barrier per row: step r updates rows s > r from the unscaled
        // row r (the factor 1/d2 folded into the update) and scales row r - 1,
        // which no thread reads in step r; the last row is scaled after the
        // loop.  Thread c owns column c of the panel.
        double inv_prev = 0.0, sq_prev = 0.0;
        bool zero_prev = false;
        auto scale_row = [&](int r, double inv, double sq, bool zero) {
            for (int c = r + threadIdx.x; c < w; c += blockDim.x) {
                cplx<double>& v = P[(size_t)r * ldp + c];
                v = c == r ? cplx<double>{zero ? 0.0 : sq, 0.0} : cplx<double>{v.x * inv, v.y * inv};
            }
        };
        for (int r = 0; r < b; ++r) {
            const double d2 = P[(size_t)r * ldp + r].x;
            const bool zero = !(d2 > floor) && d2 == d2;    // numerically singular pivot (not NaN)
            const double sq = sqrt(d2);
            const double inv = zero ? 0.0 : 1.0 / sq, inv2 = inv * inv;
            // rows s in (r, b): P[s][c] -= conj(P[r][s]) P[r][c] / d2, c >= s
            for (int c = r + 1 + threadIdx.x; c < w; c += blockDim.x) {
                const cplx<double> v = P[(size_t)r * ldp + c];
                const int se = min(c, b - 1);
                for (int s = r + 1; s <= se; ++s) {
                    const cplx<double> a = P[(size_t)r * ldp + s];
                    cplx<double>& t = P[(size_t)s * ldp + c];
                    // conj(a) v / d2
                    t.x -= (a.x * v.x + a.y * v.y) * inv2;
                    t.y -= (a.x * v.y - a.y * v.x) * inv2;
                }
            }
            if (r > 0) scale_row(r - 1, inv_prev, sq_prev, zero_prev);
            inv_prev = inv;
            sq_prev = sq;
            zero_prev = zero;
            __syncthreads();
        }
        scale_row(b - 1, inv_prev, sq_prev, zero_prev);
        __syncthreads();
        // rows of R (zeros left of the diagonal), or columns of R^H: thread
        // (c, r) with r fastest, so that each column's b entries of R^H go
        // out as one contiguous run
        if (g.conj_transpose) {
            for (int x = threadIdx.x; x < PANEL * N; x += blockDim.x) {
                const int c = x / PANEL, r = x - (x / PANEL) * PANEL;
                if (r >= b) continue;
                const cplx<double> v = c >= k0 + r ? P[(size_t)r * ldp + (c - k0)] : cplx<double>{0, 0};
                Rk[(size_t)c * N + k0 + r] = {R(v.x), R(-v.y)};
            }
        } else {
            for (int r = 0; r < b; ++r) {
                for (int c = threadIdx.x; c < N; c += blockDim.x) {
                    const cplx<double> v = c >= k0 + r ? P[(size_t)r * ldp + (c - k0)] : cplx<double>{0, 0};
                    Rk[(size_t)(k0 + r) * N + c] = {R(v.x), R(v.y)};
                }
            }
        }
        // trailing update of the upper triangle:
        // H[t0 + i][t0 + j] -= sum_r conj(P[r][b + i]) P[r][b + j], i <= j < tw
        const int t0 = k0 + b, tw = N - t0;
        const int nT = (tw + 3) >> 2, fold = (nT + 1) >> 1;
        for (int x = threadIdx.x; x < fold * (nT + 1); x += blockDim.x) {
            const int f = x / (nT + 1), c = x - f * (nT + 1);
            int I, J;
            if (c < nT - f) {
                I = f;
                J = f + c;
            } else {
                I = nT - 1 - f;
                J = I + (c - (nT - f));
                if (I == f) continue;      // odd nT: the middle row of tiles is covered once
            }
            const int i0 = 4 * I, j0 = 4 * J;
            cplx<double> h[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = i0 + u, j = j0 + v;
                    h[u][v] = (i < tw && j < tw && j >= i) ? H[(size_t)(t0 + i) * N + t0 + j]
                                                          : cplx<double>{0, 0};
                }
            for (int r = 0; r < b; ++r) {
                cplx<double> a[4], e[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    a[u] = P[(size_t)r * ldp + b + min(i0 + u, tw - 1)];
                    e[u] = P[(size_t)r * ldp + b + min(j0 + u, tw - 1)];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        h[u][v].x -= a[u].x * e[v].x + a[u].y * e[v].y;
                        h[u][v].y -= a[u].x * e[v].y - a[u].y * e[v].x;
                    }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = i0 + u, j = j0 + v;
                    if (i < tw && j < tw && j >= i) H[(size_t)(t0 + i) * N + t0 + j] = h[u][v];
                }
        }
        __syncthreads();
    }
}

constexpr int kQrRows = 64;      // rows of Y per work-group
constexpr int kQrChunk = 16;     // columns c of G (rows of V) per staged chunk
constexpr int kQrTaps = 16;      // taps held in registers by the matrix-core left-vector kernel

// Y = G_k V_R for the work-group (item, row tile, column tile): rows
// r0 .. r0+63 and columns j0 .. j0+16 NW-1 of Y (M x N), with G_k assembled
// from W (the symbol, or its conjugate transpose for a wide layer) in
// chunks of 16 columns, staged in LDS beside the matching rows of V_R (the
// right singular vectors of the factor R, [theta][c][j]).  Thread (rg, cg)
// accumulates rows r0 + 4 rg + u (u < 4) and columns j0 + cg + 16 w (w < NW).
// Y goes column-major into the item's slot, as the working matrix of the
// finish; the (row tile 0, column tile 0) work-group also copies V_R into
// the slot's accumulator part.  V_R comes from the SVD of R^H, whose left
// singular vectors (normalised final columns, no rotation accumulator) are
// the right ones of R.
template <typename R, int NW>
__global__ void __launch_bounds__(256) qr_left_kernel(QrVecArgs<R> q) {
    extern __shared__ __align__(16) char lds_raw[];
    constexpr int JW = 16 * NW;
    const int rtiles = (q.M + kQrRows - 1) / kQrRows, ctiles = (q.N + JW - 1) / JW;
    const int item = blockIdx.x / (rtiles * ctiles);
    const int rest = blockIdx.x - item * rtiles * ctiles;
    const int r0 = (rest / ctiles) * kQrRows, j0 = (rest - (rest / ctiles) * ctiles) * JW;
    const int theta = canonical_theta(q.n, q.m, item);
    const int p = theta / q.m, qq = theta - (theta / q.m) * q.m;
    const int N = q.N, T = q.kh * q.kw;
    cplx<R>* ph = reinterpret_cast<cplx<R>*>(lds_raw);            // [T]
    cplx<R>* gt = ph + T;                                           // [kQrRows][kQrChunk]
    cplx<R>* vt = gt + kQrRows * kQrChunk;                          // [kQrChunk][JW]
    const cplx<R>* VR = q.VR + (size_t)theta * N * N;
    cplx<R>* slot = reinterpret_cast<cplx<R>*>(q.slots + (size_t)item * q.slot_bytes);
    cplx<R>* Y = slot;                                              // [N][ldg]
    cplx<R>* Qs = slot + (size_t)q.ldg * N;                        // [N][ldv]
    for (int t = threadIdx.x; t < T; t += blockDim.x) {
        const int aa = t / q.kw, bb = t - (t / q.kw) * q.kw;
        const int y1 = aa - (q.kh - 1) / 2, y2 = bb - (q.kw - 1) / 2;
        int i1 = (p * y1) % q.n;
        if (i1 < 0) i1 += q.n;
        int i2 = (qq * y2) % q.m;
        if (i2 < 0) i2 += q.m;
        const double ar = q.tw[2 * (q.tw_n + i1)], ai = q.tw[2 * (q.tw_n + i1) + 1];
        const double br = q.tw[2 * (q.tw_m + i2)], bi = q.tw[2 * (q.tw_m + i2) + 1];
        const double im = ar * bi + ai * br;
        ph[t] = {R(ar * br - ai * bi), R(q.transposed ? -im : im)};
    }
    if (rest == 0)
        for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
            const int c = e / N, j = e - (e / N) * N;
            Qs[(size_t)j * q.ldv + c] = VR[e];
        }
    const int rg = threadIdx.x >> 4, cg = threadIdx.x & 15;
    R yr[4][NW], yi[4][NW];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int w = 0; w < NW; ++w) yr[u][w] = yi[u][w] = R(0);
    for (int c0 = 0; c0 < N; c0 += kQrChunk) {
        __syncthreads();
        // G_k[r][c] = sum_t Wg[r][c][t] e^{2 pi i s <k, y_t>}
        for (int x = threadIdx.x; x < kQrRows * kQrChunk; x += blockDim.x) {
            const int rr = x / kQrChunk, cc = x - (x / kQrChunk) * kQrChunk;
            const int r = r0 + rr, c = c0 + cc;
            cplx<R> v = {R(0), R(0)};
            if (r < q.M && c < N) {
                const R* w = q.W + (q.transposed ? ((size_t)c * q.c_in + r) : ((size_t)r * q.c_in + c)) * T;
                for (int t = 0; t < T; ++t) {
                    v.x = fma(w[t], ph[t].x, v.x);
                    v.y = fma(w[t], ph[t].y, v.y);
                }
            }
            gt[x] = v;
        }
        for (int x = threadIdx.x; x < kQrChunk * JW; x += blockDim.x) {
            const int cc = x / JW, j = j0 + (x - (x / JW) * JW);
            vt[x] = (c0 + cc < N && j < N) ? VR[(size_t)(c0 + cc) * N + j] : cplx<R>{R(0), R(0)};
        }
        __syncthreads();
#pragma unroll 2
        for (int cc = 0; cc < kQrChunk; ++cc) {
            cplx<R> g[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) g[u] = gt[(4 * rg + u) * kQrChunk + cc];
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const cplx<R> v = vt[cc * JW + cg + 16 * w];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    yr[u][w] = fma(g[u].x, v.x, fma(-g[u].y, v.y, yr[u][w]));
                    yi[u][w] = fma(g[u].x, v.y, fma(g[u].y, v.x, yi[u][w]));
                }
            }
        }
    }
    // columns of singular values the SVD of R set to zero (numerically
    // negligible) stay exactly zero: the finish then completes them
    // orthonormally instead of normalising the rounding noise of G V
    const R* sr = q.sigma + (size_t)theta * N;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int r = r0 + 4 * rg + u;
        if (r >= q.M) continue;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const int j = j0 + cg + 16 * w;
            if (j < N) {
                const bool keep = sr[j] != R(0);
                Y[(size_t)j * q.ldg + r] = {keep ? yr[u][w] : R(0), keep ? yi[u][w] : R(0)};
            }
        }
    }
}

// The same product on FP32 matrix cores.  Work-group (item, row tile of 64,
// column tile of 16 NJ): G_k assembled from W in chunks of 16 columns c into
// LDS (real and imaginary planes), the matching 16 rows of V_R beside them;
// wave w forms rows r0 + 16 w .. r0 + 16 w + 15 against the tile's columns
// as NJ tiles of 16 x 16, each complex product as four real MFMA products
// per K step of 4 (Re Re and -Im Im into the real part, Re Im and Im Re into
// the imaginary part).
typedef float qr_floatx4 __attribute__((ext_vector_type(4)));

template <int NJ>
__global__ void __launch_bounds__(256) qr_left_mfma(QrVecArgs<float> q) {
    constexpr int JW = 16 * NJ;
    __shared__ float gre[kQrRows][kQrChunk + 1], gim[kQrRows][kQrChunk + 1];   // G chunk [r][c]
    __shared__ float vre[kQrChunk][JW + 1], vim[kQrChunk][JW + 1];             // V_R chunk [c][j]
    __shared__ cplx<float> ph[kMaxTaps];
    const int rtiles = (q.M + kQrRows - 1) / kQrRows, ctiles = (q.N + JW - 1) / JW;
    const int item = blockIdx.x / (rtiles * ctiles);
    const int rest = blockIdx.x - item * rtiles * ctiles;
    const int r0 = (rest / ctiles) * kQrRows, j0 = (rest - (rest / ctiles) * ctiles) * JW;
    const int theta = canonical_theta(q.n, q.m, item);
    const int p = theta / q.m, qq = theta - (theta / q.m) * q.m;
    const int N = q.N, T = q.kh * q.kw;
    const cplx<float>* VR = q.VR + (size_t)theta * N * N;
    cplx<float>* slot = reinterpret_cast<cplx<float>*>(q.slots + (size_t)item * q.slot_bytes);
    cplx<float>* Y = slot;                                          // [N][ldg]
    cplx<float>* Qs = slot + (size_t)q.ldg * N;                    // [N][ldv]
    for (int t = threadIdx.x; t < T; t += blockDim.x) {
        const int aa = t / q.kw, bb = t - (t / q.kw) * q.kw;
        const int y1 = aa - (q.kh - 1) / 2, y2 = bb - (q.kw - 1) / 2;
        int i1 = (p * y1) % q.n;
        if (i1 < 0) i1 += q.n;
        int i2 = (qq * y2) % q.m;
        if (i2 < 0) i2 += q.m;
        const double ar = q.tw[2 * (q.tw_n + i1)], ai = q.tw[2 * (q.tw_n + i1) + 1];
        const double br = q.tw[2 * (q.tw_m + i2)], bi = q.tw[2 * (q.tw_m + i2) + 1];
        const double im = ar * bi + ai * br;
        ph[t] = {float(ar * br - ai * bi), float(q.transposed ? -im : im)};
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    qr_floatx4 yr[NJ], yi[NJ];
#pragma unroll
    for (int s = 0; s < NJ; ++s) {
        yr[s] = qr_floatx4{0.f, 0.f, 0.f, 0.f};
        yi[s] = qr_floatx4{0.f, 0.f, 0.f, 0.f};
    }
    for (int c0 = 0; c0 < N; c0 += kQrChunk) {
        __syncthreads();
        // G_k[r][c] = sum_t Wg[r][c][t] e^{2 pi i s <k, y_t>}: each thread's
        // 4 entries, their taps loaded all at once (up to kQrTaps in
        // registers) before the sums
        constexpr int PER = kQrRows * kQrChunk / 256;
        if (T <= kQrTaps) {
            float wv[PER][kQrTaps];
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int x = threadIdx.x + 256 * u;
                const int rr = x / kQrChunk, cc = x - (x / kQrChunk) * kQrChunk;
                const int r = r0 + rr, c = c0 + cc;
                const bool ok = r < q.M && c < N;
                const float* w = q.W + (q.transposed ? ((size_t)c * q.c_in + r) : ((size_t)r * q.c_in + c)) * T;
#pragma unroll
                for (int t = 0; t < kQrTaps; ++t) wv[u][t] = (ok && t < T) ? w[t] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int x = threadIdx.x + 256 * u;
                const int rr = x / kQrChunk, cc = x - (x / kQrChunk) * kQrChunk;
                float vr = 0.f, vi = 0.f;
#pragma unroll
                for (int t = 0; t < kQrTaps; ++t) {
                    if (t < T) {
                        vr = fmaf(wv[u][t], ph[t].x, vr);
                        vi = fmaf(wv[u][t], ph[t].y, vi);
                    }
                }
                gre[rr][cc] = vr;
                gim[rr][cc] = vi;
            }
        } else {
            for (int x = threadIdx.x; x < kQrRows * kQrChunk; x += blockDim.x) {
                const int rr = x / kQrChunk, cc = x - (x / kQrChunk) * kQrChunk;
                const int r = r0 + rr, c = c0 + cc;
                float vr = 0.f, vi = 0.f;
                if (r < q.M && c < N) {
                    const float* w = q.W + (q.transposed ? ((size_t)c * q.c_in + r) : ((size_t)r * q.c_in + c)) * T;
                    for (int t = 0; t < T; ++t) {
                        vr = fmaf(w[t], ph[t].x, vr);
                        vi = fmaf(w[t], ph[t].y, vi);
                    }
                }
                gre[rr][cc] = vr;
                gim[rr][cc] = vi;
            }
        }
        // (256 threads: fixed trip counts, so that the loads are unrolled
        // and four at a time in flight; full unrolling leaves one wave per SIMD)
#pragma unroll 4
        for (int x = threadIdx.x; x < kQrChunk * JW; x += 256) {
            const int cc = x / JW, jj = x - (x / JW) * JW, j = j0 + jj;
            const cplx<float> v = (c0 + cc < N && j < N) ? VR[(size_t)(c0 + cc) * N + j] : cplx<float>{0.f, 0.f};
            vre[cc][jj] = v.x;
            vim[cc][jj] = v.y;
        }
        __syncthreads();
        // the row-tile-0 work-groups also copy V_R into the slot's
        // accumulator part (Qs[j][c] = V_R[c][j]): from the staged chunk,
        // 16 consecutive c of one column j per 16 lanes
        if (r0 == 0)
#pragma unroll
            for (int x = threadIdx.x; x < kQrChunk * JW; x += 256) {
                const int jj = x / kQrChunk, cc = x - (x / kQrChunk) * kQrChunk;
                if (c0 + cc < N && j0 + jj < N)
                    Qs[(size_t)(j0 + jj) * q.ldv + c0 + cc] = {vre[cc][jj], vim[cc][jj]};
            }
#pragma unroll
        for (int kt = 0; kt < kQrChunk / 4; ++kt) {
            const float ar = gre[16 * wave + li][4 * kt + lk], ai = gim[16 * wave + li][4 * kt + lk];
#pragma unroll
            for (int s = 0; s < NJ; ++s) {
                const float br = vre[4 * kt + lk][16 * s + li], bi = vim[4 * kt + lk][16 * s + li];
                yr[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, br, yr[s], 0, 0, 0);
                yr[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai, bi, yr[s], 0, 0, 0);
                yi[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, bi, yi[s], 0, 0, 0);
                yi[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, br, yi[s], 0, 0, 0);
            }
        }
    }
    // columns of singular values the SVD of R set to zero stay exactly zero
    // (see qr_left_kernel); D[i][j]: j = lane & 15 (column), i = 4*(lane >> 4) + v (row)
    const float* sr = q.sigma + (size_t)theta * N;
#pragma unroll
    for (int s = 0; s < NJ; ++s) {
        const int j = j0 + 16 * s + li;
        if (j >= N) continue;
        const bool keep = sr[j] != 0.f;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = r0 + 16 * wave + 4 * lk + v;
            if (r < q.M) Y[(size_t)j * q.ldg + r] = {keep ? yr[s][v] : 0.f, keep ? yi[s][v] : 0.f};
        }
    }
}

// The blocked kernels' finish on Y and V_R (one work-group per decomposed
// frequency): sigma, U and V of the symbol into the layer's outputs.
//
// Columns y_j = G v_j of singular values far below the largest carry
// rounding errors of about u ||G|| in every direction, so the u_j = y_j /
// sigma_j would lose orthogonality like u sigma_max / sigma_j.  Before the
// finish, every such column (sigma_j <= sigma_0 / 64, in decreasing order)
// is orthogonalised against all earlier columns by two passes of classical
// Gram-Schmidt on the unit vectors y_i / |y_i|: U becomes orthonormal to
// working precision, and y_j changes by at most its error, about
// u sigma_max, inside the normwise tolerance.  Well-conditioned symbols skip
// the passes.
template <typename R>
__global__ void __launch_bounds__(256) qr_finish_kernel(SvdArgs<R> a, const R* sigma_r) {
    extern __shared__ __align__(16) char lds_raw[];
    const int item = blockIdx.x;
    const Target tg = target_of(a, item);
    const Shared<R> s = carve<R>(lds_raw, a.d, true, a.gws + (size_t)item * a.slot_bytes);
    const int M = a.d.M, N = a.d.N, ldg = a.d.ldg;
    const R* sr = sigma_r + (size_t)tg.theta * N;
    const int lane = threadIdx.x & 63, group = threadIdx.x >> 6, ngroups = blockDim.x >> 6;
    cplx<R>* G = s.G;
    // column norms into s.sig (the finish recomputes them afterwards)
    for (int j = group; j < N; j += ngroups) {
        R acc = 0;
#pragma unroll 8
        for (int i = lane; i < M; i += 64) {
            const cplx<R> v = G[(size_t)j * ldg + i];
            acc = fma(v.x, v.x, fma(v.y, v.y, acc));
        }
        acc = group_sum<R, 64>(acc);
        if (lane == 0) s.sig[j] = sqrt(acc);
    }
    __syncthreads();
    const R s0 = sr[0];
    for (int j = 1; j < N; ++j) {
        const R sj = sr[j];
        if (!(sj > R(0)) || !(sj * R(64) <= s0)) continue;    // uniform over the work-group
        for (int pass = 0; pass < 2; ++pass) {
            // c_i = u_i^H y_j for the earlier nonzero columns, one per group
            for (int i = group; i < j; i += ngroups) {
                cplx<R> c = {R(0), R(0)};
                const R ni = s.sig[i];
                if (ni > R(0)) {
#pragma unroll 8
                    for (int r = lane; r < M; r += 64) {
                        const cplx<R> u = G[(size_t)i * ldg + r], y = G[(size_t)j * ldg + r];
                        c.x = fma(u.x, y.x, fma(u.y, y.y, c.x));
                        c.y = fma(u.x, y.y, fma(-u.y, y.x, c.y));
                    }
                    c.x = group_sum<R, 64>(c.x) / ni;
                    c.y = group_sum<R, 64>(c.y) / ni;
                }
                if (lane == 0) s.coef[i] = c;
            }
            __syncthreads();
            // y_j -= sum_i c_i u_i
            for (int r = threadIdx.x; r < M; r += blockDim.x) {
                cplx<R> y = G[(size_t)j * ldg + r];
                for (int i = 0; i < j; ++i) {
                    const R ni = s.sig[i];
                    if (!(ni > R(0))) continue;
                    const cplx<R> c = s.coef[i], u = G[(size_t)i * ldg + r];
                    const R inv = R(1) / ni;
                    y.x -= (c.x * u.x - c.y * u.y) * inv;
                    y.y -= (c.x * u.y + c.y * u.x) * inv;
                }
                G[(size_t)j * ldg + r] = y;
            }
            __syncthreads();
        }
        if (group == 0) {
            R acc = 0;
            for (int r = lane; r < M; r += 64) {
                const cplx<R> v = G[(size_t)j * ldg + r];
                acc = fma(v.x, v.x, fma(v.y, v.y, acc));
            }
            acc = group_sum<R, 64>(acc);
            if (lane == 0) s.sig[j] = sqrt(acc);
        }
        __syncthreads();
    }
    finish<R, 64>(a, s, tg.out, tg.mirror, 0, true);
}

}  // namespace

namespace {
size_t cholesky_lds_bytes(int N, int kh, int kw, int panel) {
    return sizeof(cplx<double>) * ((size_t)(2 * kh - 1) * (2 * kw - 1) + (size_t)panel * (N + 1)) +
           sizeof(double) * 256;
}

template <typename R, int PANEL>
hipError_t launch_cholesky_p(const GramArgs<R>& g, int items, hipStream_t s) {
    const size_t lds = cholesky_lds_bytes(g.N, g.kh, g.kw, PANEL);
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(gram_cholesky_kernel<R, PANEL>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((gram_cholesky_kernel<R, PANEL>), dim3(items), dim3(256), lds, s, g);
    return hipGetLastError();
}

// Work-groups of the Cholesky kernel with PANEL rows per panel that fit on
// the device at once (0 on error).
template <typename R, int PANEL>
int cholesky_resident(const GramArgs<R>& g) {
    const size_t lds = cholesky_lds_bytes(g.N, g.kh, g.kw, PANEL);
    if (lds > 65536 && hipFuncSetAttribute(reinterpret_cast<const void*>(gram_cholesky_kernel<R, PANEL>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return 0;
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, gram_cholesky_kernel<R, PANEL>, 256, lds) !=
            hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return per_cu * cus;
}
}  // namespace

size_t gram_cholesky_lds_bytes(int N, int kh, int kw) { return cholesky_lds_bytes(N, kh, kw, kPanelMax); }

template <typename R>
hipError_t launch_gram_qr(const GramArgs<R>& g, int items, hipStream_t s) {
    const int nt = (g.N + kGramTile - 1) / kGramTile;
    const int ND = (2 * g.kh - 1) * (2 * g.kw - 1);
    hipLaunchKernelGGL(gram_taps_kernel<R>, dim3(nt, nt, ND), dim3(256), 0, s, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || items <= 0) return e;
    // the tallest panel whose work-groups all fit on the device in one
    // round (a second round of a few work-groups costs a whole factorisation)
    if (items <= cholesky_resident<R, kPanelMax>(g)) return launch_cholesky_p<R, kPanelMax>(g, items, s);
    if (items <= cholesky_resident<R, 12>(g)) return launch_cholesky_p<R, 12>(g, items, s);
    return launch_cholesky_p<R, kPanelMax>(g, items, s);
}

template <typename R, int NW>
hipError_t launch_qr_left_nw(const QrVecArgs<R>& q, int items, hipStream_t s) {
    constexpr int JW = 16 * NW;
    const int rtiles = (q.M + kQrRows - 1) / kQrRows, ctiles = (q.N + JW - 1) / JW;
    const size_t lds = sizeof(cplx<R>) * ((size_t)q.kh * q.kw + kQrRows * kQrChunk + (size_t)kQrChunk * JW);
    hipLaunchKernelGGL((qr_left_kernel<R, NW>), dim3(items * rtiles * ctiles), dim3(256), lds, s, q);
    return hipGetLastError();
}

template <int NJ>
hipError_t launch_qr_left_mfma_nj(const QrVecArgs<float>& q, int items, hipStream_t s) {
    constexpr int JW = 16 * NJ;
    const int rtiles = (q.M + kQrRows - 1) / kQrRows, ctiles = (q.N + JW - 1) / JW;
    hipLaunchKernelGGL((qr_left_mfma<NJ>), dim3(items * rtiles * ctiles), dim3(256), 0, s, q);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_qr_vectors(const QrVecArgs<R>& q, const SvdArgs<R>& a, int items, hipStream_t s) {
    if (items <= 0) return hipSuccess;
    hipError_t e;
    if constexpr (sizeof(R) == 4) {
        // FP32: matrix cores, column tiles of up to 128 (256 would hold 256
        // accumulator registers per lane: one wave per SIMD)
        if (q.N <= 16) e = launch_qr_left_mfma_nj<1>(q, items, s);
        else if (q.N <= 32) e = launch_qr_left_mfma_nj<2>(q, items, s);
        else if (q.N <= 64) e = launch_qr_left_mfma_nj<4>(q, items, s);
        else e = launch_qr_left_mfma_nj<8>(q, items, s);
    } else if (q.N <= 16) e = launch_qr_left_nw<R, 1>(q, items, s);
    else if (q.N <= 32) e = launch_qr_left_nw<R, 2>(q, items, s);
    else if (q.N <= 64) e = launch_qr_left_nw<R, 4>(q, items, s);
    else if (q.N <= 128) e = launch_qr_left_nw<R, 8>(q, items, s);
    else e = launch_qr_left_nw<R, 16>(q, items, s);
    if (e != hipSuccess) return e;
    // the finish's small arrays (carve): phases, reduction scratch, sigma,
    // sort permutations, completion coefficients and work vector, flags
    const size_t lds = sizeof(cplx<R>) * kMaxTaps + sizeof(R) * 64 + (sizeof(R) + 2 * sizeof(int)) * ((q.N + 3) & ~3) +
                       16 + sizeof(cplx<R>) * ((size_t)q.N + q.M) + sizeof(int) * 4 + 16;
    if (lds > 65536) {
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(qr_finish_kernel<R>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(qr_finish_kernel<R>, dim3(items), dim3(256), lds, s, a, q.sigma);
    return hipGetLastError();
}

hipError_t launch_qr_vectors_f32(const QrVecArgs<float>& q, const SvdArgs<float>& a, int items, hipStream_t s) {
    return launch_qr_vectors<float>(q, a, items, s);
}
hipError_t launch_qr_vectors_f64(const QrVecArgs<double>& q, const SvdArgs<double>& a, int items, hipStream_t s) {
    return launch_qr_vectors<double>(q, a, items, s);
}

hipError_t launch_gram_qr_f32(const GramArgs<float>& g, int items, hipStream_t s) {
    return launch_gram_qr<float>(g, items, s);
}
hipError_t launch_gram_qr_f64(const GramArgs<double>& g, int items, hipStream_t s) {
    return launch_gram_qr<double>(g, items, s);
}

}  // namespace lfa
