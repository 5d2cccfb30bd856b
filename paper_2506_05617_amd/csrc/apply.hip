// Spectral functions of a layer's periodic operator applied to images
// through the per-symbol SVD (Sec. III "Convolution Theorem": the global
// singular vectors of the operator are Fourier modes times the singular
// vectors U_k, V_k of the symbols).
//
//   identity, clip, truncate:  y = U f(Sigma) V^* x   (x: c_in channels, y: c_out)
//   pinv:            y = V f(Sigma) U^* x   (x: c_out channels, y: c_in)
//
// Per image: x_hat_k = sum_x x(x) e^{-2 pi i <k, x>} (two passes of a
// one-axis DFT), y_hat_k = L_k f(S_k) R_k^H x_hat_k at every frequency
// (one work-group per frequency, L, R = U, V or V, U), and the inverse
// transform with e^{+2 pi i <k, x>} / (n m), real part (two passes).
//
// Also here: the global singular vectors themselves (the lift of chosen
// columns of U_k and V_k by the Fourier mode of k), written as images.
#include <hip/hip_runtime.h>

#include <cmath>

#include "lfa_internal.hpp"

namespace lfa {
namespace {

// Line decomposition of a DFT pass: line = (i0 * N1 + i1) * N2 + i2, element
// t of input line at in_off + t * in_st with in_off = i0 s0 + i1 s1 + i2 s2
// (same for the output, frequency f at out_off + f * out_st).
struct AxisMap {
    long long N1, N2;
    long long is0, is1, is2, ist;   // input strides (elements)
    long long os0, os1, os2, ost;   // output strides (elements)
};

// out[line][f] = scale * sum_{t < L} in[line][t] e^{sign 2 pi i f t / L}
// with e^{2 pi i j / L} = tw[j] (FP64 (re, im) table of the plan).  One
// thread per (line, f); REAL_IN reads real input, REAL_OUT writes the real
// part.  Lines x L threads in total.
template <typename R, bool REAL_IN, bool REAL_OUT>
__global__ void __launch_bounds__(256) dft_axis_kernel(const void* in_v, void* out_v, long long lines,
                                                       int L, AxisMap mp, const double* tw, int sign,
                                                       R scale) {
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= lines * L) return;
    const long long line = gid / L;
    const int f = (int)(gid - line * L);
    const long long i2 = line % mp.N2, i01 = line / mp.N2;
    const long long i1 = i01 % mp.N1, i0 = i01 / mp.N1;
    const long long ioff = i0 * mp.is0 + i1 * mp.is1 + i2 * mp.is2;
    const long long ooff = i0 * mp.os0 + i1 * mp.os1 + i2 * mp.os2 + (long long)f * mp.ost;
    R ar = 0, ai = 0;
    int j = 0;   // (f * t) mod L
    for (int t = 0; t < L; ++t) {
        const R cr = R(tw[2 * j]), ci = R(sign) * R(tw[2 * j + 1]);
        if constexpr (REAL_IN) {
            const R xr = static_cast<const R*>(in_v)[ioff + t * mp.ist];
            ar = fma(xr, cr, ar);
            ai = fma(xr, ci, ai);
        } else {
            const cplx<R> x = static_cast<const cplx<R>*>(in_v)[ioff + t * mp.ist];
            ar = fma(x.x, cr, fma(-x.y, ci, ar));
            ai = fma(x.x, ci, fma(x.y, cr, ai));
        }
        j += f;
        if (j >= L) j -= L;
    }
    if constexpr (REAL_OUT) {
        static_cast<R*>(out_v)[ooff] = ar * scale;
    } else {
        static_cast<cplx<R>*>(out_v)[ooff] = {ar * scale, ai * scale};
    }
}

// The same transform with the work-group's lines and the twiddles of L in
// LDS: LPB = max(1, 256 / L) lines per work-group, each input element read
// from memory once, every product taken from LDS.  L <= kDftLdsMaxL.
constexpr int kDftThreads = 256;
constexpr int kDftLdsMaxL = 2048;

template <typename R, bool REAL_IN, bool REAL_OUT>
__global__ void __launch_bounds__(kDftThreads) dft_axis_lds_kernel(const void* in_v, void* out_v, long long lines,
                                                                   int L, int lpb, AxisMap mp, const double* tw,
                                                                   int sign, R scale) {
    extern __shared__ __align__(16) char lds[];
    cplx<R>* w = reinterpret_cast<cplx<R>*>(lds);      // [L] e^{sign 2 pi i j / L}
    cplx<R>* xs = w + L;                               // [lpb][L]
    const int tid = threadIdx.x;
    const long long line0 = (long long)blockIdx.x * lpb;
    for (int j = tid; j < L; j += kDftThreads) w[j] = {R(tw[2 * j]), R(sign) * R(tw[2 * j + 1])};
    for (int e = tid; e < lpb * L; e += kDftThreads) {
        const int li = e / L, t = e - (e / L) * L;
        const long long line = line0 + li;
        cplx<R> v = {R(0), R(0)};
        if (line < lines) {
            const long long i2 = line % mp.N2, i01 = line / mp.N2;
            const long long i1 = i01 % mp.N1, i0 = i01 / mp.N1;
            const long long off = i0 * mp.is0 + i1 * mp.is1 + i2 * mp.is2 + (long long)t * mp.ist;
            if constexpr (REAL_IN) v.x = static_cast<const R*>(in_v)[off];
            else v = static_cast<const cplx<R>*>(in_v)[off];
        }
        xs[e] = v;
    }
    __syncthreads();
    for (int e = tid; e < lpb * L; e += kDftThreads) {
        const int li = e / L, f = e - (e / L) * L;
        const long long line = line0 + li;
        if (line >= lines) continue;
        const cplx<R>* x = xs + li * L;
        R ar = 0, ai = 0;
        int j = 0;   // (f * t) mod L
        for (int t = 0; t < L; ++t) {
            const cplx<R> c = w[j], v = x[t];
            ar = fma(v.x, c.x, fma(-v.y, c.y, ar));
            ai = fma(v.x, c.y, fma(v.y, c.x, ai));
            j += f;
            if (j >= L) j -= L;
        }
        const long long i2 = line % mp.N2, i01 = line / mp.N2;
        const long long i1 = i01 % mp.N1, i0 = i01 / mp.N1;
        const long long off = i0 * mp.os0 + i1 * mp.os1 + i2 * mp.os2 + (long long)f * mp.ost;
        if constexpr (REAL_OUT) static_cast<R*>(out_v)[off] = ar * scale;
        else static_cast<cplx<R>*>(out_v)[off] = {ar * scale, ai * scale};
    }
}

// Power-of-two L: the same transform as a radix-2 Stockham FFT in LDS (the
// self-sorting form: every stage reads one buffer and writes the other, and
// the result is in natural order).  Stage with sub-transform length n and
// stride s = L / n, butterfly i = p s + q (p < n/2, q < s):
//   Y[q + s (2p)]     = X[q + s p] + X[q + s (p + n/2)]
//   Y[q + s (2p + 1)] = (X[q + s p] - X[q + s (p + n/2)]) w^(p s),  w = e^{sign 2 pi i / L}
// LPB = max(1, 512 / L) lines per work-group, L/2 butterflies per line and
// stage shared by the 256 threads.
template <typename R, bool REAL_IN, bool REAL_OUT>
__global__ void __launch_bounds__(kDftThreads) fft_axis_lds_kernel(const void* in_v, void* out_v, long long lines,
                                                                   int L, int logL, int lpb, AxisMap mp,
                                                                   const double* tw, int sign, R scale) {
    extern __shared__ __align__(16) char lds[];
    cplx<R>* w = reinterpret_cast<cplx<R>*>(lds);      // [L] e^{sign 2 pi i j / L}
    cplx<R>* buf0 = w + L;                             // [lpb][L]
    cplx<R>* buf1 = buf0 + lpb * L;                    // [lpb][L]
    const int tid = threadIdx.x;
    const long long line0 = (long long)blockIdx.x * lpb;
    for (int j = tid; j < L; j += kDftThreads) w[j] = {R(tw[2 * j]), R(sign) * R(tw[2 * j + 1])};
    for (int e = tid; e < lpb * L; e += kDftThreads) {
        const int li = e >> logL, t = e & (L - 1);
        const long long line = line0 + li;
        cplx<R> v = {R(0), R(0)};
        if (line < lines) {
            const long long i2 = line % mp.N2, i01 = line / mp.N2;
            const long long i1 = i01 % mp.N1, i0 = i01 / mp.N1;
            const long long off = i0 * mp.is0 + i1 * mp.is1 + i2 * mp.is2 + (long long)t * mp.ist;
            if constexpr (REAL_IN) v.x = static_cast<const R*>(in_v)[off];
            else v = static_cast<const cplx<R>*>(in_v)[off];
        }
        buf0[e] = v;
    }
    __syncthreads();
    const int half_l = L >> 1;
    for (int st = 0; st < logL; ++st) {
        const int ls = st, s = 1 << ls, n = L >> ls, hn = n >> 1;   // stride, sub-transform length
        for (int e = tid; e < lpb * half_l; e += kDftThreads) {
            const int li = e >> (logL - 1), i = e & (half_l - 1);
            const int p = i >> ls, q = i & (s - 1);
            // stage st reads buffer st % 2 and writes the other
            const cplx<R>* x = ((st & 1) ? buf1 : buf0) + li * L;
            cplx<R>* y = ((st & 1) ? buf0 : buf1) + li * L;
            const cplx<R> a = x[q + s * p], b = x[q + s * (p + hn)];
            const cplx<R> wp = w[p * s];
            const R dr = a.x - b.x, di = a.y - b.y;
            y[q + s * (2 * p)] = {a.x + b.x, a.y + b.y};
            y[q + s * (2 * p + 1)] = {dr * wp.x - di * wp.y, dr * wp.y + di * wp.x};
        }
        __syncthreads();
    }
    const cplx<R>* X = (logL & 1) ? buf1 : buf0;
    for (int e = tid; e < lpb * L; e += kDftThreads) {
        const int li = e >> logL, f = e & (L - 1);
        const long long line = line0 + li;
        if (line >= lines) continue;
        const long long i2 = line % mp.N2, i01 = line / mp.N2;
        const long long i1 = i01 % mp.N1, i0 = i01 / mp.N1;
        const long long off = i0 * mp.os0 + i1 * mp.os1 + i2 * mp.os2 + (long long)f * mp.ost;
        const cplx<R> v = X[e];
        if constexpr (REAL_OUT) static_cast<R*>(out_v)[off] = v.x * scale;
        else static_cast<cplx<R>*>(out_v)[off] = {v.x * scale, v.y * scale};
    }
}

// One work-group (four waves) per frequency k, images in chunks of BC:
//   z[b][j] = fac_j * sum_c conj(Rt[k][c][j]) xh[b][k][c]   (j < r, c < cx)
//   yh[b][k][o] = sum_j Lt[k][o][j] z[b][j]                  (o < cy)
// with fac_j = f(sigma_j(k)).  The chunk's x_hat vectors and z sit in LDS.
// Both products run over blocks of 64 outputs (one per lane); each wave sums
// a contiguous quarter of the contraction index, so a lane keeps a quarter
// of its loads in flight at once (Rt: lanes read consecutive j of one row c;
// Lt: a lane reads a contiguous piece of its row o), and the four partial
// sums meet in LDS.  U and V of a frequency are read once per chunk.
constexpr int kApplyThreads = 256;
constexpr int kApplyWaves = kApplyThreads / 64;
constexpr size_t kApplyMaxLds = 160 * 1024 - 1024;   // gfx950 LDS per work-group
constexpr int kApplyBC = 8;        // images per chunk

template <typename R>
size_t apply_lds_bytes(int cx, int r) {
    return sizeof(R) * (size_t)((r + 1) & ~1) + sizeof(cplx<R>) * (size_t)kApplyBC * (cx + r) +
           sizeof(cplx<R>) * (size_t)kApplyWaves * kApplyBC * 64;
}

template <typename R>
__global__ void __launch_bounds__(kApplyThreads) spectral_apply_kernel(
    const R* sigma, const cplx<R>* Lt, const cplx<R>* Rt, const cplx<R>* xh, cplx<R>* yh, int nfreq, int batch,
    int cx, int cy, int r, int kind, R param) {
    extern __shared__ __align__(16) char lds[];
    const int k = blockIdx.x;
    if (k >= nfreq) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int NT = kApplyThreads, NW = kApplyWaves, BC = kApplyBC;
    R* fac = reinterpret_cast<R*>(lds);                                  // [r]
    cplx<R>* xs = reinterpret_cast<cplx<R>*>(fac + ((r + 1) & ~1));      // [BC][cx]
    cplx<R>* zs = xs + BC * cx;                                          // [BC][r]
    cplx<R>* part = zs + BC * r;                                         // [NW][BC][64]
    for (int j = tid; j < r; j += NT) {
        const R s = sigma[(size_t)k * r + j];
        R f = s;                                                         // identity
        if (kind == LFA_SPECTRAL_CLIP) f = s < param ? s : param;
        if (kind == LFA_SPECTRAL_PINV) f = s > param ? R(1) / s : R(0);
        if (kind == LFA_SPECTRAL_TRUNCATE) f = s > param ? s : R(0);
        fac[j] = f;
    }
    const cplx<R>* Rk = Rt + (size_t)k * cx * r;
    const cplx<R>* Lk = Lt + (size_t)k * cy * r;
    // this wave's quarter of the contraction over c (first product) and
    // over j (second product)
    const int cq = (cx + NW - 1) / NW, c_lo = wave * cq, c_hi = min(cx, c_lo + cq);
    const int jq = (r + NW - 1) / NW, j_lo = wave * jq, j_hi = min(r, j_lo + jq);
    constexpr int PF = 8;              // loads issued together
    for (int b0 = 0; b0 < batch; b0 += BC) {
        const int nb = batch - b0 < BC ? batch - b0 : BC;
        __syncthreads();
        for (int e = tid; e < nb * cx; e += NT) {
            const int b = e / cx, c = e - (e / cx) * cx;
            xs[b * cx + c] = xh[((size_t)(b0 + b) * nfreq + k) * cx + c];
        }
        __syncthreads();
        // z = fac * R^H x, 64 columns j at a time
        for (int j0 = 0; j0 < r; j0 += 64) {
            const int j = j0 + lane;
            R ar[BC], ai[BC];
#pragma unroll
            for (int b = 0; b < BC; ++b) ar[b] = ai[b] = R(0);
            if (j < r) {
                // whole batches of PF loads, then the rest one at a time
                auto acc_z = [&](const cplx<R>& a, int c) __attribute__((always_inline)) {
#pragma unroll
                    for (int b = 0; b < BC; ++b) {
                        if (b < nb) {
                            const cplx<R> v = xs[b * cx + c];
                            ar[b] = fma(a.x, v.x, fma(a.y, v.y, ar[b]));
                            ai[b] = fma(a.x, v.y, fma(-a.y, v.x, ai[b]));
                        }
                    }
                };
                int c0 = c_lo;
                for (; c0 + PF <= c_hi; c0 += PF) {
                    cplx<R> a[PF];
#pragma unroll
                    for (int u = 0; u < PF; ++u) a[u] = Rk[(size_t)(c0 + u) * r + j];
#pragma unroll
                    for (int u = 0; u < PF; ++u) acc_z(a[u], c0 + u);
                }
                for (; c0 < c_hi; ++c0) acc_z(Rk[(size_t)c0 * r + j], c0);
            }
#pragma unroll
            for (int b = 0; b < BC; ++b) part[(wave * BC + b) * 64 + lane] = {ar[b], ai[b]};
            __syncthreads();
            for (int e = tid; e < nb * 64; e += NT) {
                const int b = e >> 6, l = e & 63;
                if (j0 + l < r) {
                    R sr = 0, si = 0;
#pragma unroll
                    for (int w = 0; w < NW; ++w) {
                        const cplx<R> q = part[(w * BC + b) * 64 + l];
                        sr += q.x;
                        si += q.y;
                    }
                    const R f = fac[j0 + l];
                    zs[b * r + j0 + l] = {sr * f, si * f};
                }
            }
            __syncthreads();
        }
        // y = L z, 64 rows o at a time
        for (int o0 = 0; o0 < cy; o0 += 64) {
            const int o = o0 + lane;
            R yr[BC], yi[BC];
#pragma unroll
            for (int b = 0; b < BC; ++b) yr[b] = yi[b] = R(0);
            if (o < cy) {
                const cplx<R>* Lo = Lk + (size_t)o * r;
                auto acc_y = [&](const cplx<R>& a, int i) __attribute__((always_inline)) {
#pragma unroll
                    for (int b = 0; b < BC; ++b) {
                        if (b < nb) {
                            const cplx<R> z = zs[b * r + i];
                            yr[b] = fma(a.x, z.x, fma(-a.y, z.y, yr[b]));
                            yi[b] = fma(a.x, z.y, fma(a.y, z.x, yi[b]));
                        }
                    }
                };
                int i0 = j_lo;
                for (; i0 + PF <= j_hi; i0 += PF) {
                    cplx<R> a[PF];
#pragma unroll
                    for (int u = 0; u < PF; ++u) a[u] = Lo[i0 + u];
#pragma unroll
                    for (int u = 0; u < PF; ++u) acc_y(a[u], i0 + u);
                }
                for (; i0 < j_hi; ++i0) acc_y(Lo[i0], i0);
            }
#pragma unroll
            for (int b = 0; b < BC; ++b) part[(wave * BC + b) * 64 + lane] = {yr[b], yi[b]};
            __syncthreads();
            for (int e = tid; e < nb * 64; e += NT) {
                const int b = e >> 6, l = e & 63;
                if (o0 + l < cy) {
                    R sr = 0, si = 0;
#pragma unroll
                    for (int w = 0; w < NW; ++w) {
                        const cplx<R> q = part[(w * BC + b) * 64 + l];
                        sr += q.x;
                        si += q.y;
                    }
                    yh[((size_t)(b0 + b) * nfreq + k) * cy + o0 + l] = {sr, si};
                }
            }
            __syncthreads();
        }
    }
}

template <typename R, bool RI, bool RO>
hipError_t launch_axis(const void* in, void* out, long long lines, int L, const AxisMap& mp, const double* tw,
                       int sign, R scale, hipStream_t st) {
    const long long total = lines * L;
    if (total <= 0) return hipSuccess;
    if (L >= 2 && (L & (L - 1)) == 0 && L <= kDftLdsMaxL) {
        const int logL = __builtin_ctz((unsigned)L);
        const int lpb = L >= 2 * kDftThreads ? 1 : 2 * kDftThreads / L;
        const long long blocks = (lines + lpb - 1) / lpb;
        if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
        const size_t lds = sizeof(cplx<R>) * (size_t)L * (1 + 2 * lpb);
        if (lds > 65536) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fft_axis_lds_kernel<R, RI, RO>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL((fft_axis_lds_kernel<R, RI, RO>), dim3((unsigned)blocks), dim3(kDftThreads), lds, st, in,
                           out, lines, L, logL, lpb, mp, tw, sign, scale);
        return hipGetLastError();
    }
    if (L <= kDftLdsMaxL) {
        const int lpb = L >= kDftThreads ? 1 : kDftThreads / L;
        const long long blocks = (lines + lpb - 1) / lpb;
        if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
        const size_t lds = sizeof(cplx<R>) * (size_t)L * (1 + lpb);
        if (lds > 65536) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(dft_axis_lds_kernel<R, RI, RO>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL((dft_axis_lds_kernel<R, RI, RO>), dim3((unsigned)blocks), dim3(kDftThreads), lds, st, in,
                           out, lines, L, lpb, mp, tw, sign, scale);
        return hipGetLastError();
    }
    const int threads = 256;
    const long long blocks = (total + threads - 1) / threads;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((dft_axis_kernel<R, RI, RO>), dim3((unsigned)blocks), dim3(threads), 0, st, in, out, lines,
                       L, mp, tw, sign, scale);
    return hipGetLastError();
}

template <typename R>
hipError_t apply_t(const ApplyArgs& a, hipStream_t st) {
    const long long B = a.batch, n = a.n, m = a.m, cx = a.cx, cy = a.cy, nm = n * m;
    cplx<R>* T1 = static_cast<cplx<R>*>(a.ws1);
    cplx<R>* T2 = static_cast<cplx<R>*>(a.ws2);
    const double* twn = a.tw + 2 * (size_t)a.tw_n;
    const double* twm = a.tw + 2 * (size_t)a.tw_m;
    hipError_t e;
    // A: rows, real x [B][cx][n][m] -> T1 [B][cx][n][m]; line (b, c, x1)
    {
        AxisMap mp{1, 1, m, 0, 0, 1, m, 0, 0, 1};
        e = launch_axis<R, true, false>(a.x, T1, B * cx * n, (int)m, mp, twm, -1, R(1), st);
        if (e != hipSuccess) return e;
    }
    // B: columns, T1 [B][cx][n][m] -> T2 = x_hat [B][n][m][cx]; line (b, c, q)
    {
        AxisMap mp{cx, m, cx * nm, nm, 1, m, nm * cx, 1, cx, m * cx};
        e = launch_axis<R, false, false>(T1, T2, B * cx * m, (int)n, mp, twn, -1, R(1), st);
        if (e != hipSuccess) return e;
    }
    // C: per frequency, T2 -> T1 = y_hat [B][n][m][cy]
    {
        const size_t lds = apply_lds_bytes<R>((int)cx, a.r);
        if (lds > kApplyMaxLds) return hipErrorInvalidValue;
        if (lds > 65536) {
            e = hipFuncSetAttribute(reinterpret_cast<const void*>(spectral_apply_kernel<R>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL((spectral_apply_kernel<R>), dim3((unsigned)nm), dim3(kApplyThreads), lds, st,
                           static_cast<const R*>(a.sigma), static_cast<const cplx<R>*>(a.L),
                           static_cast<const cplx<R>*>(a.R), T2, T1, (int)nm, (int)B, (int)cx, (int)cy, a.r,
                           a.kind, R(a.param));
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // D: columns, inverse, T1 [B][n][m][cy] -> T2 [B][cy][n][m]; line (b, o, q)
    {
        AxisMap mp{cy, m, nm * cy, 1, cy, m * cy, cy * nm, nm, 1, m};
        e = launch_axis<R, false, false>(T1, T2, B * cy * m, (int)n, mp, twn, +1, R(1), st);
        if (e != hipSuccess) return e;
    }
    // E: rows, inverse, real part and 1/(n m): T2 [B][cy][n][m] -> y
    {
        AxisMap mp{1, 1, m, 0, 0, 1, m, 0, 0, 1};
        e = launch_axis<R, false, true>(T2, a.y, B * cy * n, (int)m, mp, twm, +1, R(1.0 / double(nm)), st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Global singular vector of one pick, as images: one work-group per
// (pick t, channel c) row of n*m elements, x2 fastest (coalesced writes).
// The phase index is reduced exactly in integers, (p x1) mod n and
// (q x2) mod m, and the two FP64 table entries are multiplied in FP64.
constexpr int kLiftThreads = 256;

template <typename R>
__global__ void __launch_bounds__(kLiftThreads) lift_kernel(const cplx<R>* W, const int32_t* idx,
                                                            cplx<R>* out, int n, int m, int c, int r,
                                                            const double* twn, const double* twm,
                                                            double scale) {
    const long long row = blockIdx.x;   // t * c + channel
    const long long t = row / c;
    const int ch = (int)(row - t * c);
    const int p = idx[3 * t], q = idx[3 * t + 1], j = idx[3 * t + 2];
    const int nm = n * m;
    cplx<R>* o = out + row * nm;
    if (p < 0 || p >= n || q < 0 || q >= m || j < 0 || j >= r) {
        for (int pos = threadIdx.x; pos < nm; pos += blockDim.x) o[pos] = cplx<R>{R(0), R(0)};
        return;
    }
    const cplx<R> w = W[(((long long)p * m + q) * c + ch) * r + j];
    const double wr = double(w.x) * scale, wi = double(w.y) * scale;
    for (int pos = threadIdx.x; pos < nm; pos += blockDim.x) {
        const int x1 = pos / m, x2 = pos - x1 * m;
        const int a1 = (int)(((long long)p * x1) % n), a2 = (int)(((long long)q * x2) % m);
        const double er = twn[2 * a1], ei = twn[2 * a1 + 1];
        const double fr = twm[2 * a2], fi = twm[2 * a2 + 1];
        const double cr = er * fr - ei * fi, ci = er * fi + ei * fr;
        o[pos] = cplx<R>{R(cr * wr - ci * wi), R(cr * wi + ci * wr)};
    }
}

template <typename R>
hipError_t lift_t(const LiftArgs& a, hipStream_t st) {
    const double* twn = a.tw + 2 * (size_t)a.tw_n;
    const double* twm = a.tw + 2 * (size_t)a.tw_m;
    const double scale = 1.0 / std::sqrt(double(a.n) * double(a.m));
    const void* src[2] = {a.U, a.V};
    void* dst[2] = {a.u_hat, a.v_hat};
    const int rows[2] = {a.c_out, a.c_in};
    for (int s = 0; s < 2; ++s) {
        if (!dst[s]) continue;
        const long long blocks = (long long)a.count * rows[s];
        if (blocks <= 0) continue;
        hipLaunchKernelGGL((lift_kernel<R>), dim3((unsigned)blocks), dim3(kLiftThreads), 0, st,
                           static_cast<const cplx<R>*>(src[s]), a.idx, static_cast<cplx<R>*>(dst[s]), a.n,
                           a.m, rows[s], a.r, twn, twm, scale);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

bool apply_supported(int cx, int r, int elem_bytes) {
    const size_t lds = elem_bytes == 8 ? apply_lds_bytes<double>(cx, r) : apply_lds_bytes<float>(cx, r);
    return lds <= kApplyMaxLds;
}

hipError_t launch_apply_f32(const ApplyArgs& a, hipStream_t s) { return apply_t<float>(a, s); }
hipError_t launch_apply_f64(const ApplyArgs& a, hipStream_t s) { return apply_t<double>(a, s); }
hipError_t launch_lift_f32(const LiftArgs& a, hipStream_t s) { return lift_t<float>(a, s); }
hipError_t launch_lift_f64(const LiftArgs& a, hipStream_t s) { return lift_t<double>(a, s); }

}  // namespace lfa
