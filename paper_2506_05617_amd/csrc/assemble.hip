// Symbol assembly on gfx950:
//     A[theta][o][i] = sum_t W[o][i][t] * exp(+2 pi i <k_theta, y_t>)
// (Sec. III "Convolution Theorem"; Algorithm 1 symbol step).
//
// Read as a matrix product, with Phi[theta][t] the complex phase matrix and
// W reshaped to [t][e] (e = o*c_in + i):  A = Phi * W, i.e. two real GEMMs of
// shape [n*m x T] x [T x c_out*c_in] sharing the right operand.
//
//  * symbols_valu: one thread per output element e, a tile of frequencies per
//    block; phases of the tile staged in LDS.  FP32 or FP64.
//  * symbols_mfma: 16x16 output tiles on the matrix cores, K = taps.  Modes:
//      0  FP32 MFMA (v_mfma_f32_16x16x4f32), K padded to 4;
//      2  split-BF16, 3 products  Phi1*W1 + Phi1*W2 + Phi2*W1, FP32 accumulate;
//      3  split-BF16, 6 products of a three-term split, FP32 accumulate;
//    the split terms are laid end to end along K so one accumulator chain
//    sums all products (v_mfma_f32_16x16x16bf16_1k).
// The phase of (theta, t) is the product of two double-precision twiddles
// exp(2 pi i j/n) at the integer-reduced indices (p*y1 mod n, q*y2 mod m),
// rounded once to the working precision.

#include <hip/hip_runtime.h>

#include <algorithm>

#include "lfa_internal.hpp"

namespace lfa {
namespace {

__device__ __forceinline__ void phase_d(const double* tw, const LayerDesc& d, int theta, int t,
                                        double& re, double& im) {
    const int p = theta / d.m, q = theta - (theta / d.m) * d.m;
    const int a = t / d.kw, b = t - (t / d.kw) * d.kw;
    const int y1 = a - (d.kh - 1) / 2, y2 = b - (d.kw - 1) / 2;
    int i1 = (p * y1) % d.n;
    if (i1 < 0) i1 += d.n;
    int i2 = (q * y2) % d.m;
    if (i2 < 0) i2 += d.m;
    const double ar = tw[2 * (d.tw_n + i1)], ai = tw[2 * (d.tw_n + i1) + 1];
    const double br = tw[2 * (d.tw_m + i2)], bi = tw[2 * (d.tw_m + i2) + 1];
    re = ar * br - ai * bi;
    im = ar * bi + ai * br;
}

// Symbols are written once and not read back by the kernel: streaming
// (non-temporal) stores keep them from displacing W and the twiddles in the
// caches and write at a markedly higher rate.
// One store of the whole complex value: two stores of its halves would each
// write every other word of the same lines.
template <typename R>
__device__ __forceinline__ void store_stream(cplx<R>* dst, R re, R im) {
    typedef R pair_t __attribute__((ext_vector_type(2)));
    const pair_t v = {re, im};
    __builtin_nontemporal_store(v, reinterpret_cast<pair_t*>(dst));
}

constexpr int kValuThetaTile = 16;

template <typename R>
__global__ void __launch_bounds__(256) symbols_valu(LayerDesc d, const R* __restrict__ W,
                                                   cplx<R>* __restrict__ A,
                                                   const double* __restrict__ tw) {
    __shared__ cplx<R> ph[kValuThetaTile * kMaxTaps];
    const int T = d.kh * d.kw;
    const int E = d.c_out * d.c_in;
    const int HW = d.num_symbols;
    const int theta0 = blockIdx.y * kValuThetaTile;
    const int nth = min(kValuThetaTile, HW - theta0);
    for (int x = threadIdx.x; x < nth * T; x += blockDim.x) {
        const int th = x / T, t = x - (x / T) * T;
        double re, im;
        phase_d(tw, d, theta0 + th, t, re, im);
        ph[th * kMaxTaps + t] = {R(re), R(im)};
    }
    __syncthreads();
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const R* w = W + (size_t)e * T;
    R re[kValuThetaTile], im[kValuThetaTile];
#pragma unroll
    for (int th = 0; th < kValuThetaTile; ++th) re[th] = im[th] = R(0);
    for (int t = 0; t < T; ++t) {
        const R wt = w[t];
#pragma unroll
        for (int th = 0; th < kValuThetaTile; ++th) {
            const cplx<R> p = ph[th * kMaxTaps + t];
            re[th] = fma(wt, p.x, re[th]);
            im[th] = fma(wt, p.y, im[th]);
        }
    }
#pragma unroll
    for (int th = 0; th < kValuThetaTile; ++th)
        if (th < nth) store_stream(A + (size_t)(theta0 + th) * E + e, re[th], im[th]);
}

// ---------------------------------------------------------------- MFMA ----

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short bf16x4 __attribute__((ext_vector_type(4)));

// Round-to-nearest-even float -> bfloat16 bits (finite inputs).
__device__ __forceinline__ unsigned short f2bf(float x) {
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// Split x into `terms` bfloat16 values whose sum approximates x.
__device__ __forceinline__ void split_bf16(float x, int terms, unsigned short* out) {
    float rest = x;
    for (int s = 0; s < terms; ++s) {
        const unsigned short h = f2bf(rest);
        out[s] = h;
        rest -= bf2f(h);
    }
}

// Segment tables: product s multiplies split term ta[s] of Phi with term tb[s] of W.
__constant__ int kSegA[2][6] = {{0, 0, 1, 0, 0, 0}, {0, 0, 1, 0, 1, 2}};
__constant__ int kSegB[2][6] = {{0, 1, 0, 0, 0, 0}, {0, 1, 0, 2, 1, 0}};

constexpr int kMfmaETile = 64;   // e columns per block (4 sub-tiles of 16)

// Frequency of output row r of the matrix-core kernels: every frequency in
// order, or (canon) the canonical frequency of conjugate pair r, when only
// one symbol per pair is needed (the SVD of real weights).
__device__ __forceinline__ int row_theta(const LayerDesc& d, int canon, int r) {
    return canon ? canonical_theta(d.n, d.m, r) : r;
}

// Block: 4 waves; wave w owns frequencies theta0 + 16w .. +16 and all 64
// e-columns of the block (4 output tiles of 16x16, re and im).
__global__ void __launch_bounds__(256) symbols_mfma(LayerDesc d, const float* __restrict__ W,
                                                    cplx<float>* __restrict__ A,
                                                    const double* __restrict__ tw, int mode, int canon) {
    const int T = d.kh * d.kw;
    const int E = d.c_out * d.c_in;
    const int HW = canon ? d.num_canon : d.num_symbols;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int theta0 = blockIdx.y * 64 + wave * 16;
    const int e0 = blockIdx.x * kMfmaETile;
    const int li = lane & 15, lk = lane >> 4;

    floatx4 acc_re[4], acc_im[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        acc_re[s] = floatx4{0.f, 0.f, 0.f, 0.f};
        acc_im[s] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
    const int theta_a = theta0 + li;   // row of the A operand this lane feeds
    const int freq_a = theta_a < HW ? row_theta(d, canon, theta_a) : 0;
    if (mode == 0) {
        // FP32: K-step 4; lane feeds A[i = li][k = lk], B[k = lk][j = li].
        for (int k0 = 0; k0 < T; k0 += 4) {
            const int t = k0 + lk;
            float pr = 0.f, pi = 0.f;
            if (t < T && theta_a < HW) {
                double re, im;
                phase_d(tw, d, freq_a, t, re, im);
                pr = float(re);
                pi = float(im);
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int e = e0 + s * 16 + li;
                const float b = (t < T && e < E) ? W[(size_t)e * T + t] : 0.f;
                acc_re[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(pr, b, acc_re[s], 0, 0, 0);
                acc_im[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(pi, b, acc_im[s], 0, 0, 0);
            }
        }
    } else {
        // split-BF16: K' = nseg*T, K-step 16; lane feeds k = 4*lk + v.
        const int ms = (mode == 3) ? 1 : 0;
        const int nseg = (mode == 3) ? 6 : 3;
        const int terms = (mode == 3) ? 3 : 2;
        const int Kp = nseg * T;
        for (int k0 = 0; k0 < Kp; k0 += 16) {
            bf16x4 ar, ai;
            bf16x4 bv[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int kk = k0 + 4 * lk + v;
                unsigned short hr = 0, hi = 0;
                unsigned short wb[4] = {0, 0, 0, 0};
                if (kk < Kp) {
                    const int seg = kk / T, t = kk - (kk / T) * T;
                    if (theta_a < HW) {
                        double re, im;
                        phase_d(tw, d, freq_a, t, re, im);
                        unsigned short sr[3], si[3];
                        split_bf16(float(re), terms, sr);
                        split_bf16(float(im), terms, si);
                        hr = sr[kSegA[ms][seg]];
                        hi = si[kSegA[ms][seg]];
                    }
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const int e = e0 + s * 16 + li;
                        if (e < E) {
                            unsigned short sw[3];
                            split_bf16(W[(size_t)e * T + t], terms, sw);
                            wb[s] = sw[kSegB[ms][seg]];
                        }
                    }
                }
                ar[v] = (short)hr;
                ai[v] = (short)hi;
#pragma unroll
                for (int s = 0; s < 4; ++s) bv[s][v] = (short)wb[s];
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                acc_re[s] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ar, bv[s], acc_re[s], 0, 0, 0);
                acc_im[s] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ai, bv[s], acc_im[s], 0, 0, 0);
            }
        }
    }
    // D[i][j]: j = lane & 15, i = 4*(lane >> 4) + v
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int e = e0 + s * 16 + li;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int th = theta0 + 4 * lk + v;
            if (th < HW && e < E)
                store_stream(A + (size_t)row_theta(d, canon, th) * E + e, acc_re[s][v], acc_im[s][v]);
        }
    }
}

// ---------------------------------------------- MFMA, phases held --------
// For up to kMfma2MaxTaps taps.  A block of 4 waves owns 64 kMfma2Freq
// frequencies (16 kMfma2Freq per wave, as kMfma2Freq sub-tiles of 16) and
// loops over column tiles of 64 e: the phases of its frequencies are
// evaluated once, as ready MFMA A-fragments in registers (one set per
// bfloat16 split term in the split modes), and each 64 x T tile of W is
// staged once in LDS (as its split terms) and shared by the four waves; each
// B fragment read from LDS feeds the MFMAs of every sub-tile.  The next
// tile's W values are loaded into registers while the matrix cores work on
// the current one.  The split modes run one accumulation pass over K = taps
// per product (A term, W term) of kSegA / kSegB into the same accumulators.
constexpr int kMfma2MaxTaps = 64;
constexpr int kMfma2Freq = 2;      // 16-frequency sub-tiles per wave (FP32)

// Products of split terms, (A term, W term), in the order of kSegA / kSegB.
constexpr int kProdA[2][6] = {{0, 0, 1, 0, 0, 0}, {0, 0, 1, 0, 1, 2}};
constexpr int kProdB[2][6] = {{0, 1, 0, 0, 0, 0}, {0, 1, 0, 2, 1, 0}};

template <int MODE>
struct Mfma2 {
    static constexpr int TERMS = MODE == 0 ? 1 : (MODE == 2 ? 2 : 3);
    static constexpr int NPROD = MODE == 0 ? 1 : (MODE == 2 ? 3 : 6);
    static constexpr int KSTEP = MODE == 0 ? 4 : 16;
    static constexpr int KS = kMfma2MaxTaps / KSTEP;                         // max K steps
    static constexpr int ROW = MODE == 0 ? kMfma2MaxTaps + 1 : kMfma2MaxTaps + 4;   // LDS row, padded
    static constexpr int PER = (64 * ROW + 255) / 256;                       // W values per thread per tile
};

template <int MODE, int FT>
__global__ void __launch_bounds__(256) symbols_mfma2(LayerDesc d, const float* __restrict__ W,
                                                     cplx<float>* __restrict__ A,
                                                     const double* __restrict__ tw, int echunk, int canon) {
    using C = Mfma2<MODE>;
    constexpr int ms = MODE == 3 ? 1 : 0;
    extern __shared__ __align__(16) char lds_raw[];
    const int T = d.kh * d.kw;
    const int E = d.c_out * d.c_in;
    const int HW = canon ? d.num_canon : d.num_symbols;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int theta0 = blockIdx.y * 64 * FT + wave * 16 * FT;
    const int ks = (T + C::KSTEP - 1) / C::KSTEP;     // K steps actually used

    // A-fragments (phases) of this wave's frequencies: in sub-tile f, lane
    // (li, lk) holds row theta0 + 16 f + li at taps 4 kt + lk (FP32) or
    // 16 kt + 4 lk + v (bf16)
    float pr[FT][MODE == 0 ? C::KS : 1], pi[FT][MODE == 0 ? C::KS : 1];
    bf16x4 ar[FT][C::TERMS][MODE == 0 ? 1 : C::KS], ai[FT][C::TERMS][MODE == 0 ? 1 : C::KS];
#pragma unroll
    for (int f = 0; f < FT; ++f) {
        const int theta_a = theta0 + 16 * f + li;
        const int freq_a = theta_a < HW ? row_theta(d, canon, theta_a) : 0;
#pragma unroll
        for (int kt = 0; kt < C::KS; ++kt) {
            if constexpr (MODE == 0) {
                const int t = 4 * kt + lk;
                float r = 0.f, im = 0.f;
                if (kt < ks && t < T && theta_a < HW) {
                    double re, imd;
                    phase_d(tw, d, freq_a, t, re, imd);
                    r = float(re);
                    im = float(imd);
                }
                pr[f][kt] = r;
                pi[f][kt] = im;
            } else {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int t = 16 * kt + 4 * lk + v;
                    unsigned short sr[3] = {0, 0, 0}, si[3] = {0, 0, 0};
                    if (kt < ks && t < T && theta_a < HW) {
                        double re, imd;
                        phase_d(tw, d, freq_a, t, re, imd);
                        split_bf16(float(re), C::TERMS, sr);
                        split_bf16(float(imd), C::TERMS, si);
                    }
#pragma unroll
                    for (int u = 0; u < C::TERMS; ++u) {
                        ar[f][u][kt][v] = (short)sr[u];
                        ai[f][u][kt][v] = (short)si[u];
                    }
                }
            }
        }
    }

    // W tile rows e0 .. e0+63 of T taps each (contiguous in W), zero beyond
    // T: fetched into registers, then put into LDS (split modes: one plane
    // per split term)
    const int e_begin = blockIdx.x * echunk, e_end = min(E, e_begin + echunk);
    float wreg[C::PER];
    auto fetch = [&](int e0) {
#pragma unroll
        for (int u = 0; u < C::PER; ++u) {
            const int x = threadIdx.x + 256 * u;
            const int r = x / C::ROW, t = x - r * C::ROW;
            const int e = e0 + r;
            wreg[u] = (x < 64 * C::ROW && t < T && e < E) ? W[(size_t)e * T + t] : 0.f;
        }
    };
    auto put = [&]() {
#pragma unroll
        for (int u = 0; u < C::PER; ++u) {
            const int x = threadIdx.x + 256 * u;
            if (x >= 64 * C::ROW) continue;
            if constexpr (MODE == 0) {
                reinterpret_cast<float*>(lds_raw)[x] = wreg[u];
            } else {
                unsigned short sw[3] = {0, 0, 0};
                split_bf16(wreg[u], C::TERMS, sw);
#pragma unroll
                for (int q = 0; q < C::TERMS; ++q)
                    reinterpret_cast<unsigned short*>(lds_raw)[q * 64 * C::ROW + x] = sw[q];
            }
        }
    };
    if (e_begin < e_end) fetch(e_begin);
    for (int e0 = e_begin; e0 < e_end; e0 += 64) {
        __syncthreads();          // the previous tile's readers are done
        put();
        __syncthreads();
        if (e0 + 64 < e_end) fetch(e0 + 64);       // in flight during the MFMAs
        floatx4 acc_re[FT][4], acc_im[FT][4];
#pragma unroll
        for (int f = 0; f < FT; ++f)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                acc_re[f][s] = floatx4{0.f, 0.f, 0.f, 0.f};
                acc_im[f][s] = floatx4{0.f, 0.f, 0.f, 0.f};
            }
        if constexpr (MODE == 0) {
            const float* wl = reinterpret_cast<const float*>(lds_raw);
#pragma unroll
            for (int kt = 0; kt < C::KS; ++kt) {
                if (kt < ks) {
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const float b = wl[(s * 16 + li) * C::ROW + 4 * kt + lk];
#pragma unroll
                        for (int f = 0; f < FT; ++f) {
                            acc_re[f][s] = __builtin_amdgcn_mfma_f32_16x16x4f32(pr[f][kt], b, acc_re[f][s], 0, 0, 0);
                            acc_im[f][s] = __builtin_amdgcn_mfma_f32_16x16x4f32(pi[f][kt], b, acc_im[f][s], 0, 0, 0);
                        }
                    }
                }
            }
        } else {
            const unsigned short* wl = reinterpret_cast<const unsigned short*>(lds_raw);
#pragma unroll
            for (int pp = 0; pp < C::NPROD; ++pp) {
                const int ta = kProdA[ms][pp], tb = kProdB[ms][pp];
#pragma unroll
                for (int kt = 0; kt < C::KS; ++kt) {
                    if (kt < ks) {
#pragma unroll
                        for (int s = 0; s < 4; ++s) {
                            const bf16x4 b = *reinterpret_cast<const bf16x4*>(
                                wl + tb * 64 * C::ROW + (s * 16 + li) * C::ROW + 16 * kt + 4 * lk);
#pragma unroll
                            for (int f = 0; f < FT; ++f) {
                                // split terms are selected with compile-time indices
                                bf16x4 fa_r = ar[f][0][kt], fa_i = ai[f][0][kt];
#pragma unroll
                                for (int u = 1; u < C::TERMS; ++u)
                                    if (ta == u) {
                                        fa_r = ar[f][u][kt];
                                        fa_i = ai[f][u][kt];
                                    }
                                acc_re[f][s] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fa_r, b, acc_re[f][s], 0, 0, 0);
                                acc_im[f][s] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fa_i, b, acc_im[f][s], 0, 0, 0);
                            }
                        }
                    }
                }
            }
        }
        // D[i][j]: j = lane & 15 (e), i = 4*(lane >> 4) + v (frequency)
#pragma unroll
        for (int f = 0; f < FT; ++f)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int e = e0 + s * 16 + li;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int th = theta0 + 16 * f + 4 * lk + v;
                    if (th < HW && e < E)
                        store_stream(A + (size_t)row_theta(d, canon, th) * E + e, acc_re[f][s][v], acc_im[f][s][v]);
                }
            }
    }
}

// ---------------------------------------------- MFMA, separable phases ----
// FP32 matrix cores for kernels of at most kSepMaxRows rows.  The phase of
// tap (a, b) at frequency (p, q) factors as e^{2 pi i p y1/n} e^{2 pi i q y2/m}
// (y1, y2 the tap's offsets), so
//     A_{p,q}[e] = sum_a e^{2 pi i p y1(a)/n} B_q[a][e],
//     B_q[a][e]  = sum_b W[e][a][b] e^{2 pi i q y2(b)/m}.
// A block takes one q and 64 columns e: it forms B_q for them (kh x 64
// complex, into LDS, then into registers as MFMA B fragments), and its waves
// run the contraction over a (K = kh rounded up to 4) for 16 frequencies p
// at a time, as four real products per K step (Re Re and -Im Im into the
// real part, Re Im and Im Re into the imaginary part): kh terms per output
// instead of the kh kw of the direct contraction.
constexpr int kSepMaxRows = 16;

// (p, q) is the canonical frequency of its conjugate pair: the set that
// canonical_theta enumerates (row 0 and, for even n, row n/2 up to q = m/2;
// the rows 1 .. (n+1)/2 - 1 whole).
__device__ __forceinline__ bool is_canonical(const LayerDesc& d, int p, int q) {
    const int full = (d.n + 1) / 2 - 1;
    if (p >= 1 && p <= full) return true;
    if (p == 0 || (!(d.n & 1) && p == d.n / 2)) return 2 * q <= d.m;
    return false;
}

__global__ void __launch_bounds__(256) symbols_sep(LayerDesc d, const float* __restrict__ W,
                                                   cplx<float>* __restrict__ A, const double* __restrict__ tw,
                                                   int canon) {
    __shared__ float bre[kSepMaxRows][65], bim[kSepMaxRows][65];   // B_q[a][e - e0]
    __shared__ float bq[2][kMaxTaps];                               // e^{2 pi i q y2(b)/m}
    const int T = d.kh * d.kw, E = d.c_out * d.c_in;
    const int e0 = blockIdx.x * 64, q = blockIdx.y;
    const int KA = (d.kh + 3) & ~3;
    for (int b = threadIdx.x; b < d.kw; b += blockDim.x) {
        int i2 = (q * (b - (d.kw - 1) / 2)) % d.m;
        if (i2 < 0) i2 += d.m;
        bq[0][b] = float(tw[2 * (d.tw_m + i2)]);
        bq[1][b] = float(tw[2 * (d.tw_m + i2) + 1]);
    }
    __syncthreads();
    {
        const int el = threadIdx.x & 63, e = e0 + el;
        for (int a = threadIdx.x >> 6; a < KA; a += 4) {
            float sr = 0.f, si = 0.f;
            if (a < d.kh && e < E) {
                const float* w = W + (size_t)e * T + a * d.kw;
                for (int b = 0; b < d.kw; ++b) {
                    sr = fmaf(w[b], bq[0][b], sr);
                    si = fmaf(w[b], bq[1][b], si);
                }
            }
            bre[a][el] = sr;
            bim[a][el] = si;
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    constexpr int KT = kSepMaxRows / 4;
    const int ksteps = KA / 4;
    // B fragments: lane (li, lk) holds B[k = 4 kt + lk][j = 16 s + li]
    float fr[KT][4], fi[KT][4];
#pragma unroll
    for (int kt = 0; kt < KT; ++kt)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            fr[kt][s] = kt < ksteps ? bre[4 * kt + lk][16 * s + li] : 0.f;
            fi[kt][s] = kt < ksteps ? bim[4 * kt + lk][16 * s + li] : 0.f;
        }
    const int p_end = canon ? d.n / 2 + 1 : d.n;
    const int y1off = (d.kh - 1) / 2;
    for (int p0 = wave * 16; p0 < p_end; p0 += 64) {
        floatx4 yr[4], yi[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            yr[s] = floatx4{0.f, 0.f, 0.f, 0.f};
            yi[s] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
        const int p = p0 + li;      // row of the A operand this lane feeds
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
            if (kt < ksteps) {
                const int a = 4 * kt + lk;
                float ar = 0.f, ai = 0.f;
                if (a < d.kh && p < d.n) {
                    int i1 = (p * (a - y1off)) % d.n;
                    if (i1 < 0) i1 += d.n;
                    ar = float(tw[2 * (d.tw_n + i1)]);
                    ai = float(tw[2 * (d.tw_n + i1) + 1]);
                }
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    yr[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, fr[kt][s], yr[s], 0, 0, 0);
                    yr[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai, fi[kt][s], yr[s], 0, 0, 0);
                    yi[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, fi[kt][s], yi[s], 0, 0, 0);
                    yi[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, fr[kt][s], yi[s], 0, 0, 0);
                }
            }
        }
        // D[i][j]: j = lane & 15 (e), i = 4*(lane >> 4) + v (p)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int e = e0 + s * 16 + li;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int pp = p0 + 4 * lk + v;
                if (pp < d.n && e < E && (!canon || is_canonical(d, pp, q)))
                    store_stream(A + ((size_t)pp * d.m + q) * E + e, yr[s][v], yi[s][v]);
            }
        }
    }
}

// The separable form in the split-BF16 modes (MODE 2: two terms, three
// products; MODE 3: three terms, six products).  B_q is formed in FP32 as
// above, then each value of the B fragments and of the phase fragments is
// split into bfloat16 terms; the kept products of terms accumulate in FP32
// on v_mfma_f32_16x16x16bf16_1k, the kernel rows (at most 16) in one K step.
template <int MODE>
__global__ void __launch_bounds__(256) symbols_sep_bf(LayerDesc d, const float* __restrict__ W,
                                                      cplx<float>* __restrict__ A,
                                                      const double* __restrict__ tw, int canon) {
    constexpr int TERMS = MODE == 2 ? 2 : 3, NPROD = MODE == 2 ? 3 : 6, ms = MODE == 3 ? 1 : 0;
    __shared__ float bre[kSepMaxRows][65], bim[kSepMaxRows][65];   // B_q[a][e - e0]
    __shared__ float bq[2][kMaxTaps];
    const int T = d.kh * d.kw, E = d.c_out * d.c_in;
    const int e0 = blockIdx.x * 64, q = blockIdx.y;
    for (int b = threadIdx.x; b < d.kw; b += blockDim.x) {
        int i2 = (q * (b - (d.kw - 1) / 2)) % d.m;
        if (i2 < 0) i2 += d.m;
        bq[0][b] = float(tw[2 * (d.tw_m + i2)]);
        bq[1][b] = float(tw[2 * (d.tw_m + i2) + 1]);
    }
    __syncthreads();
    {
        const int el = threadIdx.x & 63, e = e0 + el;
        for (int a = threadIdx.x >> 6; a < kSepMaxRows; a += 4) {
            float sr = 0.f, si = 0.f;
            if (a < d.kh && e < E) {
                const float* w = W + (size_t)e * T + a * d.kw;
                for (int b = 0; b < d.kw; ++b) {
                    sr = fmaf(w[b], bq[0][b], sr);
                    si = fmaf(w[b], bq[1][b], si);
                }
            }
            bre[a][el] = sr;
            bim[a][el] = si;
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    // B fragments: lane (li, lk) holds B[k = 4 lk + v][j = 16 s + li], v < 4,
    // as split terms
    bf16x4 fr[4][TERMS], fi[4][TERMS];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            unsigned short hr[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
            split_bf16(bre[4 * lk + v][16 * s + li], TERMS, hr);
            split_bf16(bim[4 * lk + v][16 * s + li], TERMS, hi);
#pragma unroll
            for (int u = 0; u < TERMS; ++u) {
                fr[s][u][v] = (short)hr[u];
                fi[s][u][v] = (short)hi[u];
            }
        }
    const int p_end = canon ? d.n / 2 + 1 : d.n;
    const int y1off = (d.kh - 1) / 2;
    for (int p0 = wave * 16; p0 < p_end; p0 += 64) {
        floatx4 yr[4], yi[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            yr[s] = floatx4{0.f, 0.f, 0.f, 0.f};
            yi[s] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
        // A fragments: row p = p0 + li, k = a = 4 lk + v; -Im kept beside Im
        const int p = p0 + li;
        bf16x4 ar[TERMS], ai[TERMS], an[TERMS];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int a = 4 * lk + v;
            float re = 0.f, im = 0.f;
            if (a < d.kh && p < d.n) {
                int i1 = (p * (a - y1off)) % d.n;
                if (i1 < 0) i1 += d.n;
                re = float(tw[2 * (d.tw_n + i1)]);
                im = float(tw[2 * (d.tw_n + i1) + 1]);
            }
            unsigned short hr[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
            split_bf16(re, TERMS, hr);
            split_bf16(im, TERMS, hi);
#pragma unroll
            for (int u = 0; u < TERMS; ++u) {
                ar[u][v] = (short)hr[u];
                ai[u][v] = (short)hi[u];
                an[u][v] = (short)(hi[u] ^ 0x8000u);     // -Im: the sign bit flipped
            }
        }
#pragma unroll
        for (int pp = 0; pp < NPROD; ++pp) {
            const int ta = kProdA[ms][pp], tb = kProdB[ms][pp];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                yr[s] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ar[ta], fr[s][tb], yr[s], 0, 0, 0);
                yr[s] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(an[ta], fi[s][tb], yr[s], 0, 0, 0);
                yi[s] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ar[ta], fi[s][tb], yi[s], 0, 0, 0);
                yi[s] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ai[ta], fr[s][tb], yi[s], 0, 0, 0);
            }
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int e = e0 + s * 16 + li;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int pp = p0 + 4 * lk + v;
                if (pp < d.n && e < E && (!canon || is_canonical(d, pp, q)))
                    store_stream(A + ((size_t)pp * d.m + q) * E + e, yr[s][v], yi[s][v]);
            }
        }
    }
}

template <int MODE>
hipError_t launch_sep_bf(const LayerDesc& d, const float* W, cplx<float>* A, const double* tw, int canon,
                         hipStream_t s) {
    const int E = d.c_out * d.c_in;
    hipLaunchKernelGGL(symbols_sep_bf<MODE>, dim3((E + 63) / 64, d.m), dim3(256), 0, s, d, W, A, tw, canon);
    return hipGetLastError();
}

hipError_t launch_sep(const LayerDesc& d, const float* W, cplx<float>* A, const double* tw, int canon,
                      hipStream_t s) {
    const int E = d.c_out * d.c_in;
    hipLaunchKernelGGL(symbols_sep, dim3((E + 63) / 64, d.m), dim3(256), 0, s, d, W, A, tw, canon);
    return hipGetLastError();
}

template <int MODE>
constexpr size_t mfma2_lds_bytes() {
    return 64 * (size_t)Mfma2<MODE>::ROW * (MODE == 0 ? sizeof(float) : Mfma2<MODE>::TERMS * sizeof(unsigned short));
}

template <int MODE, int FT>
hipError_t launch_mfma2_ft(const LayerDesc& d, const float* W, cplx<float>* A, const double* tw, int canon,
                           hipStream_t s) {
    const int E = d.c_out * d.c_in;
    const int tblocks = ((canon ? d.num_canon : d.num_symbols) + 64 * FT - 1) / (64 * FT);
    // enough blocks for the device: split the e range when there are few
    // frequency tiles (each block still covers >= 64 columns)
    const int etiles = (E + 63) / 64;
    const int split = std::max(1, std::min(etiles, (2048 + tblocks - 1) / tblocks));
    const int echunk = 64 * ((etiles + split - 1) / split);
    const dim3 grid((E + echunk - 1) / echunk, tblocks);
    const size_t lds = mfma2_lds_bytes<MODE>();
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(symbols_mfma2<MODE, FT>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((symbols_mfma2<MODE, FT>), grid, dim3(256), lds, s, d, W, A, tw, echunk, canon);
    return hipGetLastError();
}

// Two sub-tiles per wave for FP32 (0.64 -> 0.54 ms on the 7x7 224 x 224
// grid); one for the split modes, whose phase fragments for two sub-tiles
// leave one wave per SIMD (split-BF16 x3: 0.69 ms with one, 0.76 with two).
template <int MODE>
hipError_t launch_mfma2(const LayerDesc& d, const float* W, cplx<float>* A, const double* tw, int canon,
                        hipStream_t s) {
    return launch_mfma2_ft<MODE, MODE == 0 ? kMfma2Freq : 1>(d, W, A, tw, canon, s);
}

}  // namespace

hipError_t launch_symbols_valu_f32(const LayerDesc& d, const float* W, cplx<float>* A,
                                   const double* tw, hipStream_t s) {
    const int E = d.c_out * d.c_in;
    const dim3 grid((E + 255) / 256, (d.num_symbols + kValuThetaTile - 1) / kValuThetaTile);
    hipLaunchKernelGGL(symbols_valu<float>, grid, dim3(256), 0, s, d, W, A, tw);
    return hipGetLastError();
}

hipError_t launch_symbols_valu_f64(const LayerDesc& d, const double* W, cplx<double>* A,
                                   const double* tw, hipStream_t s) {
    const int E = d.c_out * d.c_in;
    const dim3 grid((E + 255) / 256, (d.num_symbols + kValuThetaTile - 1) / kValuThetaTile);
    hipLaunchKernelGGL(symbols_valu<double>, grid, dim3(256), 0, s, d, W, A, tw);
    return hipGetLastError();
}

hipError_t launch_symbols_mfma(const LayerDesc& d, const float* W, cplx<float>* A,
                               const double* tw, int mode, hipStream_t s, bool canon_only) {
    const int canon = canon_only ? 1 : 0;
    if (d.kh <= kSepMaxRows) {
        if (mode == 0) return launch_sep(d, W, A, tw, canon, s);
        if (mode == 2) return launch_sep_bf<2>(d, W, A, tw, canon, s);
        if (mode == 3) return launch_sep_bf<3>(d, W, A, tw, canon, s);
    }
    if (d.kh * d.kw <= kMfma2MaxTaps) {
        if (mode == 0) return launch_mfma2<0>(d, W, A, tw, canon, s);
        if (mode == 2) return launch_mfma2<2>(d, W, A, tw, canon, s);
        if (mode == 3) return launch_mfma2<3>(d, W, A, tw, canon, s);
    }
    const int E = d.c_out * d.c_in;
    const dim3 grid((E + kMfmaETile - 1) / kMfmaETile, ((canon ? d.num_canon : d.num_symbols) + 63) / 64);
    hipLaunchKernelGGL(symbols_mfma, grid, dim3(256), 0, s, d, W, A, tw, mode, canon);
    return hipGetLastError();
}

}  // namespace lfa
