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
#include <hip/hip_runtime.h>

#include "lfa_internal.hpp"

namespace lfa {
namespace {

constexpr int kGramTile = 32;     // output tile of C_delta (c, c')
constexpr int kGramRows = 16;     // rows r per staged chunk
constexpr int kPanel = 16;        // rows of R per Cholesky panel

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
// layer's R symbols [n*m][N][N] (FP32 or FP64, zeros below the diagonal).
template <typename R>
__global__ void __launch_bounds__(256) gram_cholesky_kernel(GramArgs<R> g) {
    extern __shared__ __align__(16) char lds_raw[];
    const int item = blockIdx.x;
    const int theta = canonical_theta(g.n, g.m, item);
    const int p = theta / g.m, q = theta - (theta / g.m) * g.m;
    const int N = g.N, KD1 = 2 * g.kh - 1, KD2 = 2 * g.kw - 1, ND = KD1 * KD2;
    cplx<double>* ph = reinterpret_cast<cplx<double>*>(lds_raw);     // [ND]
    cplx<double>* P = ph + ND;                                         // [kPanel][N]
    double* red = reinterpret_cast<double*>(P + (size_t)kPanel * N);  // [256]
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
    for (int k0 = 0; k0 < N; k0 += kPanel) {
        const int b = min(kPanel, N - k0), w = N - k0;
        // panel rows k0 .. k0+b-1, columns k0 .. N-1 (upper part)
        for (int x = threadIdx.x; x < b * w; x += blockDim.x) {
            const int r = x / w, c = x - (x / w) * w;
            P[(size_t)r * N + c] = c >= r ? H[(size_t)(k0 + r) * N + k0 + c] : cplx<double>{0, 0};
        }
        __syncthreads();
        for (int r = 0; r < b; ++r) {
            const double d2 = P[(size_t)r * N + r].x;
            const bool zero = !(d2 > floor) && d2 == d2;    // numerically singular pivot (not NaN)
            const double inv = zero ? 0.0 : 1.0 / sqrt(d2);
            __syncthreads();
            for (int c = r + threadIdx.x; c < w; c += blockDim.x) {
                cplx<double>& v = P[(size_t)r * N + c];
                v = c == r ? cplx<double>{zero ? 0.0 : sqrt(d2), 0.0} : cplx<double>{v.x * inv, v.y * inv};
            }
            __syncthreads();
            // rows s in (r, b): P[s][c] -= conj(P[r][s]) P[r][c], c >= s
            const int rows = b - r - 1;
            for (int x = threadIdx.x; x < rows * w; x += blockDim.x) {
                const int s = r + 1 + x / w, c = x - (x / w) * w;
                if (c < s) continue;
                const cplx<double> a = P[(size_t)r * N + s], v = P[(size_t)r * N + c];
                cplx<double>& t = P[(size_t)s * N + c];
                // conj(a) v
                t.x -= a.x * v.x + a.y * v.y;
                t.y -= a.x * v.y - a.y * v.x;
            }
            __syncthreads();
        }
        // rows of R (zeros left of the diagonal)
        for (int x = threadIdx.x; x < b * N; x += blockDim.x) {
            const int r = x / N, c = x - (x / N) * N;
            const cplx<double> v = c >= k0 + r ? P[(size_t)r * N + (c - k0)] : cplx<double>{0, 0};
            Rk[(size_t)(k0 + r) * N + c] = {R(v.x), R(v.y)};
        }
        // trailing update of the upper triangle: H[i][j] -= sum_r conj(P[r][i]) P[r][j]
        const int t0 = k0 + b, tw = N - t0;
        for (long long x = threadIdx.x; x < (long long)tw * tw; x += blockDim.x) {
            const int i = (int)(x / tw), j = (int)(x - (x / tw) * tw);
            if (j < i) continue;
            cplx<double> h = H[(size_t)(t0 + i) * N + t0 + j];
            for (int r = 0; r < b; ++r) {
                const cplx<double> a = P[(size_t)r * N + b + i], v = P[(size_t)r * N + b + j];
                h.x -= a.x * v.x + a.y * v.y;
                h.y -= a.x * v.y - a.y * v.x;
            }
            H[(size_t)(t0 + i) * N + t0 + j] = h;
        }
        __syncthreads();
    }
}

}  // namespace

size_t gram_cholesky_lds_bytes(int N, int kh, int kw) {
    return sizeof(cplx<double>) * ((size_t)(2 * kh - 1) * (2 * kw - 1) + (size_t)kPanel * N) +
           sizeof(double) * 256;
}

template <typename R>
hipError_t launch_gram_qr(const GramArgs<R>& g, int items, hipStream_t s) {
    const int nt = (g.N + kGramTile - 1) / kGramTile;
    const int ND = (2 * g.kh - 1) * (2 * g.kw - 1);
    hipLaunchKernelGGL(gram_taps_kernel<R>, dim3(nt, nt, ND), dim3(256), 0, s, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || items <= 0) return e;
    const size_t lds = gram_cholesky_lds_bytes(g.N, g.kh, g.kw);
    if (lds > 65536) {
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(gram_cholesky_kernel<R>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(gram_cholesky_kernel<R>, dim3(items), dim3(256), lds, s, g);
    return hipGetLastError();
}

hipError_t launch_gram_qr_f32(const GramArgs<float>& g, int items, hipStream_t s) {
    return launch_gram_qr<float>(g, items, s);
}
hipError_t launch_gram_qr_f64(const GramArgs<double>& g, int items, hipStream_t s) {
    return launch_gram_qr<double>(g, items, s);
}

}  // namespace lfa
