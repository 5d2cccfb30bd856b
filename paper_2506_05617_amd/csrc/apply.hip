// Spectral functions of a layer's periodic operator applied to images
// through the per-symbol SVD (Sec. III "Convolution Theorem": the global
// singular vectors of the operator are Fourier modes times the singular
// vectors U_k, V_k of the symbols).
//
//   identity, clip:  y = U f(Sigma) V^* x   (x: c_in channels, y: c_out)
//   pinv:            y = V f(Sigma) U^* x   (x: c_out channels, y: c_in)
//
// Per image: x_hat_k = sum_x x(x) e^{-2 pi i <k, x>} (two passes of a
// one-axis DFT), y_hat_k = L_k f(S_k) R_k^H x_hat_k at every frequency
// (one work-group per frequency, L, R = U, V or V, U), and the inverse
// transform with e^{+2 pi i <k, x>} / (n m), real part (two passes).
#include <hip/hip_runtime.h>

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

// One work-group per frequency k: for every image b,
//   z_j = fac_j * sum_c conj(Rt[k][c][j]) xh[b][k][c]   (j < r, c < cx)
//   yh[b][k][o] = sum_j Lt[k][o][j] z_j                  (o < cy)
// with fac_j = f(sigma_j(k)).  Rt[k] is read with consecutive j across the
// threads of the work-group; row o of Lt[k] is read by thread o (each
// thread's row is contiguous, so the cache lines of a row serve that thread's
// next reads).  U and V of a frequency are read once for the whole batch.
template <typename R>
__global__ void __launch_bounds__(256) spectral_apply_kernel(const R* sigma, const cplx<R>* Lt, const cplx<R>* Rt,
                                                             const cplx<R>* xh, cplx<R>* yh, int nfreq, int batch,
                                                             int cx, int cy, int r, int kind, R param) {
    extern __shared__ __align__(16) char lds[];
    const int k = blockIdx.x;
    if (k >= nfreq) return;
    const int tid = threadIdx.x, nt = blockDim.x;
    R* fac = reinterpret_cast<R*>(lds);                            // [r]
    cplx<R>* xs = reinterpret_cast<cplx<R>*>(fac + ((r + 1) & ~1));  // [cx]
    cplx<R>* zs = xs + cx;                                         // [r]
    for (int j = tid; j < r; j += nt) {
        const R s = sigma[(size_t)k * r + j];
        R f = s;                                                   // identity
        if (kind == LFA_SPECTRAL_CLIP) f = s < param ? s : param;
        if (kind == LFA_SPECTRAL_PINV) f = s > param ? R(1) / s : R(0);
        fac[j] = f;
    }
    const cplx<R>* Rk = Rt + (size_t)k * cx * r;
    const cplx<R>* Lk = Lt + (size_t)k * cy * r;
    for (int b = 0; b < batch; ++b) {
        __syncthreads();
        for (int c = tid; c < cx; c += nt) xs[c] = xh[((size_t)b * nfreq + k) * cx + c];
        __syncthreads();
        for (int j = tid; j < r; j += nt) {
            R zr = 0, zi = 0;
            for (int c = 0; c < cx; ++c) {
                const cplx<R> a = Rk[(size_t)c * r + j], v = xs[c];
                // conj(a) * v
                zr = fma(a.x, v.x, fma(a.y, v.y, zr));
                zi = fma(a.x, v.y, fma(-a.y, v.x, zi));
            }
            zs[j] = {zr * fac[j], zi * fac[j]};
        }
        __syncthreads();
        for (int o = tid; o < cy; o += nt) {
            R yr = 0, yi = 0;
            const cplx<R>* row = Lk + (size_t)o * r;
            for (int j = 0; j < r; ++j) {
                const cplx<R> a = row[j], z = zs[j];
                yr = fma(a.x, z.x, fma(-a.y, z.y, yr));
                yi = fma(a.x, z.y, fma(a.y, z.x, yi));
            }
            yh[((size_t)b * nfreq + k) * cy + o] = {yr, yi};
        }
    }
}

template <typename R, bool RI, bool RO>
hipError_t launch_axis(const void* in, void* out, long long lines, int L, const AxisMap& mp, const double* tw,
                       int sign, R scale, hipStream_t st) {
    const long long total = lines * L;
    if (total <= 0) return hipSuccess;
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
        const int threads = 64;
        const size_t lds = sizeof(R) * ((a.r + 1) & ~1) + sizeof(cplx<R>) * (cx + a.r);
        if (lds > 65536) return hipErrorInvalidValue;
        hipLaunchKernelGGL((spectral_apply_kernel<R>), dim3((unsigned)nm), dim3(threads), lds, st,
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

}  // namespace

hipError_t launch_apply_f32(const ApplyArgs& a, hipStream_t s) { return apply_t<float>(a, s); }
hipError_t launch_apply_f64(const ApplyArgs& a, hipStream_t s) { return apply_t<double>(a, s); }

}  // namespace lfa
