// Top-k singular values per layer, and the adjoint of a sum of selected
// singular values with respect to the weights.
//
// Top-k: one work-group per layer.  Round r picks the first element, in the
// total order (value descending, flat index (p, q, j) ascending), that comes
// strictly after the pick of round r-1; a block-wide argmax over the layer
// per round.  NaN compares as -infinity.
//
// Adjoint: for a simple singular value, d sigma = Re(u^H dA v) and
// dA/dW[o,i,a,b] = exp(+2 pi i <k, y_ab>) E_oi, so
//     dW[o,i,a,b] = sum_s g_s Re( exp(-2 pi i <k_s, y_ab>) u_s[o] conj(v_s[i]) ).
// One thread per weight pair (o, i) and all its taps, selected values summed
// in a fixed order (deterministic, no atomics).

#include <hip/hip_runtime.h>
#include <math.h>

#include "lfa_internal.hpp"

namespace lfa {
namespace {

constexpr int kTopkThreads = 1024;

template <typename R>
__device__ __forceinline__ R key_of(R v) {
    return v == v ? v : -INFINITY;
}

// (v1, i1) comes before (v2, i2)?
template <typename R>
__device__ __forceinline__ bool before(R v1, long long i1, R v2, long long i2) {
    return v1 > v2 || (v1 == v2 && i1 < i2);
}

template <typename R>
__global__ void __launch_bounds__(kTopkThreads) topk_kernel(TopkArgs<R> a) {
    __shared__ R sv[kTopkThreads / 64];
    __shared__ long long si[kTopkThreads / 64];
    __shared__ R prev_v;
    __shared__ long long prev_i;
    const int layer = blockIdx.x;
    const R* s = a.sigma[layer];
    const int n = a.n[layer], m = a.m[layer], r = a.r[layer];
    const long long total = (long long)n * m * r;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) {
        prev_v = INFINITY;
        prev_i = -1;
    }
    __syncthreads();
    for (int round = 0; round < a.k; ++round) {
        const R pv = prev_v;
        const long long pi = prev_i;
        R bv = -INFINITY;
        long long bi = -1;
        for (long long x = tid; x < total; x += blockDim.x) {
            const R v = key_of(s[x]);
            if (before(pv, pi, v, x)) {   // strictly after the previous pick
                if (bi < 0 || before(v, x, bv, bi)) {
                    bv = v;
                    bi = x;
                }
            }
        }
        // wave argmax
        for (int off = 32; off >= 1; off >>= 1) {
            const R ov = __shfl_xor(bv, off, 64);
            const long long oi = __shfl_xor(bi, off, 64);
            if (oi >= 0 && (bi < 0 || before(ov, oi, bv, bi))) {
                bv = ov;
                bi = oi;
            }
        }
        if (lane == 0) {
            sv[wave] = bv;
            si[wave] = bi;
        }
        __syncthreads();
        if (tid == 0) {
            R v = sv[0];
            long long i = si[0];
            for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
                if (si[w] >= 0 && (i < 0 || before(sv[w], si[w], v, i))) {
                    v = sv[w];
                    i = si[w];
                }
            }
            prev_v = v;
            prev_i = i;
            const long long slot = (long long)layer * a.k + round;
            a.vals[slot] = (i >= 0) ? s[i] : R(NAN);
            long long ii = i < 0 ? 0 : i;
            const long long th = ii / r;
            a.idx[slot * 3 + 0] = (int32_t)(th / m);
            a.idx[slot * 3 + 1] = (int32_t)(th % m);
            a.idx[slot * 3 + 2] = (int32_t)(ii % r);
        }
        __syncthreads();
    }
}

template <typename R>
__global__ void __launch_bounds__(256) adjoint_kernel(AdjointArgs<R> a) {
    extern __shared__ __align__(16) char lds_raw[];
    cplx<R>* ph = reinterpret_cast<cplx<R>*>(lds_raw);   // [k][T], conjugated phases
    int layer = 0;
    while (layer + 1 < a.num_layers && (int)blockIdx.x >= a.blocks_before[layer + 1]) ++layer;
    const int blk = blockIdx.x - a.blocks_before[layer];
    const int c_out = a.c_out[layer], c_in = a.c_in[layer], kh = a.kh[layer], kw = a.kw[layer];
    const int n = a.n[layer], m = a.m[layer];
    const int T = kh * kw, r = c_out < c_in ? c_out : c_in;
    const int k = a.k;
    const int32_t* idx = a.idx + (size_t)layer * k * 3;
    const R* g = a.grad + (size_t)layer * k;
    for (int x = threadIdx.x; x < k * T; x += blockDim.x) {
        const int s = x / T, t = x - (x / T) * T;
        const int p = idx[3 * s] % n, q = idx[3 * s + 1] % m;
        const int aa = t / kw, bb = t - (t / kw) * kw;
        const int y1 = aa - (kh - 1) / 2, y2 = bb - (kw - 1) / 2;
        int i1 = (p * y1) % n;
        if (i1 < 0) i1 += n;
        int i2 = (q * y2) % m;
        if (i2 < 0) i2 += m;
        const double ar = a.tw[2 * (a.tw_n[layer] + i1)], ai = a.tw[2 * (a.tw_n[layer] + i1) + 1];
        const double br = a.tw[2 * (a.tw_m[layer] + i2)], bi = a.tw[2 * (a.tw_m[layer] + i2) + 1];
        // conj(exp(+2 pi i <k,y>)) = exp(-2 pi i <k,y>)
        ph[x] = {R(ar * br - ai * bi), R(-(ar * bi + ai * br))};
    }
    __syncthreads();
    const int e = blk * blockDim.x + threadIdx.x;
    if (e >= c_out * c_in) return;
    const int o = e / c_in, i = e - (e / c_in) * c_in;
    R* dW = a.dW[layer] + (size_t)e * T;
    // selected values in chunks of 8 held in registers; the first chunk
    // writes dW, later chunks add to it (same thread, fixed order)
    for (int s0 = 0; s0 < k; s0 += 8) {
        R zr[8], zi[8], gs[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            zr[u] = zi[u] = gs[u] = R(0);
            const int s = s0 + u;
            const bool valid = s < k && idx[3 * s] >= 0 && idx[3 * s] < n && idx[3 * s + 1] >= 0 &&
                               idx[3 * s + 1] < m && idx[3 * s + 2] >= 0 && idx[3 * s + 2] < r;
            if (valid) {   // entries outside the grid contribute nothing
                const int p = idx[3 * s], q = idx[3 * s + 1], j = idx[3 * s + 2];
                // compact slots: the pick that decomposed this symbol (the
                // conjugate symbol's vectors are the conjugates); per-pick
                // vectors: the pick's own column
                bool cj = false;
                cplx<R> uu, vv;
                if (a.compact == 2) {
                    uu = a.U[layer][(size_t)s * c_out + o];
                    vv = a.V[layer][(size_t)s * c_in + i];
                } else {
                    const long long sym = a.compact ? pick_rep(idx, s, n, m, cj) : ((long long)p * m + q);
                    uu = a.U[layer][(size_t)sym * c_out * r + (size_t)o * r + j];
                    vv = a.V[layer][(size_t)sym * c_in * r + (size_t)i * r + j];
                }
                // z = u * conj(v), conjugated with the vectors
                zr[u] = uu.x * vv.x + uu.y * vv.y;
                zi[u] = cj ? uu.x * vv.y - uu.y * vv.x : uu.y * vv.x - uu.x * vv.y;
                gs[u] = g[s];
            }
        }
        for (int t = 0; t < T; ++t) {
            R acc = (s0 == 0) ? R(0) : dW[t];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (s0 + u < k) {
                    const cplx<R> w = ph[(s0 + u) * T + t];
                    acc = fma(gs[u], w.x * zr[u] - w.y * zi[u], acc);
                }
            }
            dW[t] = acc;
        }
    }
}

constexpr int kOtherTaps = 16;   // taps of the unrolled form of other_side_kernel
constexpr int kOtherSlice = 64;  // entries of the other vector per work-group (one wave)

// One work-group per (layer, pick): the kept vector x (column j of the
// kept side at the pick's frequency) and the conjugated or plain phases of
// the taps go to LDS; each thread forms entries of the other vector,
//   v[i] = (1/sigma) sum_o sum_t W[o,i,t] e^{-2 pi i <k, y_t>} u[o]    (kept U)
//   u[o] = (1/sigma) sum_i sum_t W[o,i,t] e^{+2 pi i <k, y_t>} v[i]    (kept V),
// over the kept side's channels in a fixed order.  A pick with sigma not
// positive (or outside the grid) gets zero vectors: it adds nothing to dW.
// Each (layer, pick) is split over `parts` work-groups, each forming a slice
// of kOtherSlice entries of the other vector (the first also writes the
// kept vector).
template <typename R>
__global__ void __launch_bounds__(256) other_side_kernel(OtherSideArgs<R> a, int parts) {
    extern __shared__ __align__(16) char lds_raw[];
    const int b = blockIdx.x / parts, part = blockIdx.x - (blockIdx.x / parts) * parts;
    const int layer = b / a.k, s = b - (b / a.k) * a.k;
    const int c_out = a.c_out[layer], c_in = a.c_in[layer], kh = a.kh[layer], kw = a.kw[layer];
    const int n = a.n[layer], m = a.m[layer];
    const int T = kh * kw, r = c_out < c_in ? c_out : c_in;
    const bool keep_u = c_out >= c_in;               // the working matrix's side
    const int ck = keep_u ? c_out : c_in, co = keep_u ? c_in : c_out;
    const int e_lo = part * kOtherSlice, e_hi = min(co, e_lo + kOtherSlice);
    if (e_lo >= co) return;                       // never the first part
    cplx<R>* ph = reinterpret_cast<cplx<R>*>(lds_raw);                  // [T]
    cplx<R>* x = ph + T;                                                  // [ck]
    const int32_t* pk = a.idx + ((size_t)layer * a.k + s) * 3;
    const int p = pk[0], q = pk[1], j = pk[2];
    cplx<R>* kept_out = (keep_u ? a.Uc[layer] : a.Vc[layer]) + (size_t)s * ck;
    cplx<R>* other_out = (keep_u ? a.Vc[layer] : a.Uc[layer]) + (size_t)s * co;
    const bool valid = p >= 0 && p < n && q >= 0 && q < m && j >= 0 && j < r;
    const R sg = valid ? a.sigma[layer][((size_t)p * m + q) * r + j] : R(0);
    if (!(sg > R(0)) || !(sg < INFINITY)) {
        if (part == 0)
            for (int e = threadIdx.x; e < ck; e += blockDim.x) kept_out[e] = {R(0), R(0)};
        for (int e = e_lo + threadIdx.x; e < e_hi; e += blockDim.x) other_out[e] = {R(0), R(0)};
        return;
    }
    for (int t = threadIdx.x; t < T; t += blockDim.x) {
        const int aa = t / kw, bb = t - (t / kw) * kw;
        const int y1 = aa - (kh - 1) / 2, y2 = bb - (kw - 1) / 2;
        int i1 = (p * y1) % n;
        if (i1 < 0) i1 += n;
        int i2 = (q * y2) % m;
        if (i2 < 0) i2 += m;
        const double ar = a.tw[2 * (a.tw_n[layer] + i1)], ai = a.tw[2 * (a.tw_n[layer] + i1) + 1];
        const double br = a.tw[2 * (a.tw_m[layer] + i2)], bi = a.tw[2 * (a.tw_m[layer] + i2) + 1];
        // exp(+2 pi i <k, y>) for the kept V side, its conjugate for kept U
        const double im = ar * bi + ai * br;
        ph[t] = {R(ar * br - ai * bi), R(keep_u ? -im : im)};
    }
    const cplx<R>* xs = a.X[layer] + ((size_t)p * m + q) * ck * r;
    for (int e = threadIdx.x; e < ck; e += blockDim.x) {
        x[e] = xs[(size_t)e * r + j];
        if (part == 0) kept_out[e] = x[e];
    }
    __syncthreads();
    const R inv = R(1) / sg;
    const R* W = a.W[layer];
    for (int e = e_lo + threadIdx.x; e < e_hi; e += blockDim.x) {
        R zr = R(0), zi = R(0);
        if (T <= kOtherTaps) {
            // the same sums with the tap loop unrolled and the channel loop
            // by four, so that the weight loads are in flight together
#pragma unroll 4
            for (int c = 0; c < ck; ++c) {
                const R* w = W + (keep_u ? ((size_t)c * c_in + e) : ((size_t)e * c_in + c)) * T;
                R ar = R(0), ai = R(0);
#pragma unroll
                for (int t = 0; t < kOtherTaps; ++t) {
                    // loads without a branch (taps past T read tap 0 and
                    // add an exact zero), so that none waits on another
                    const int tt = t < T ? t : 0;
                    const R wt = w[tt];
                    const cplx<R> pt = ph[tt];
                    const R m = t < T ? wt : R(0);
                    ar = fma(m, pt.x, ar);
                    ai = fma(m, pt.y, ai);
                }
                const cplx<R> xv = x[c];
                zr = fma(ar, xv.x, fma(-ai, xv.y, zr));
                zi = fma(ar, xv.y, fma(ai, xv.x, zi));
            }
        } else {
            for (int c = 0; c < ck; ++c) {
                // weight (o, i) = (c, e) for kept U, (e, c) for kept V
                const R* w = W + (keep_u ? ((size_t)c * c_in + e) : ((size_t)e * c_in + c)) * T;
                R ar = R(0), ai = R(0);                  // sum_t w_t phase_t
                for (int t = 0; t < T; ++t) {
                    ar = fma(w[t], ph[t].x, ar);
                    ai = fma(w[t], ph[t].y, ai);
                }
                const cplx<R> xv = x[c];
                zr = fma(ar, xv.x, fma(-ai, xv.y, zr));
                zi = fma(ar, xv.y, fma(ai, xv.x, zi));
            }
        }
        other_out[e] = {zr * inv, zi * inv};
    }
}

}  // namespace

hipError_t launch_other_side_f32(const OtherSideArgs<float>& a, hipStream_t s) {
    int maxT = 0, maxC = 0;
    for (int l = 0; l < a.num_layers; ++l) {
        maxT = a.kh[l] * a.kw[l] > maxT ? a.kh[l] * a.kw[l] : maxT;
        const int ck = a.c_out[l] >= a.c_in[l] ? a.c_out[l] : a.c_in[l];
        maxC = ck > maxC ? ck : maxC;
    }
    const size_t lds = sizeof(cplx<float>) * (size_t)(maxT + maxC);
    int maxO = 1;
    for (int l = 0; l < a.num_layers; ++l) maxO = std::max(maxO, std::min(a.c_out[l], a.c_in[l]));
    const int parts = (maxO + kOtherSlice - 1) / kOtherSlice;
    hipLaunchKernelGGL(other_side_kernel<float>, dim3(a.num_layers * a.k * parts), dim3(kOtherSlice), lds, s, a,
                       parts);
    return hipGetLastError();
}
hipError_t launch_other_side_f64(const OtherSideArgs<double>& a, hipStream_t s) {
    int maxT = 0, maxC = 0;
    for (int l = 0; l < a.num_layers; ++l) {
        maxT = a.kh[l] * a.kw[l] > maxT ? a.kh[l] * a.kw[l] : maxT;
        const int ck = a.c_out[l] >= a.c_in[l] ? a.c_out[l] : a.c_in[l];
        maxC = ck > maxC ? ck : maxC;
    }
    const size_t lds = sizeof(cplx<double>) * (size_t)(maxT + maxC);
    int maxO = 1;
    for (int l = 0; l < a.num_layers; ++l) maxO = std::max(maxO, std::min(a.c_out[l], a.c_in[l]));
    const int parts = (maxO + kOtherSlice - 1) / kOtherSlice;
    hipLaunchKernelGGL(other_side_kernel<double>, dim3(a.num_layers * a.k * parts), dim3(kOtherSlice), lds, s, a,
                       parts);
    return hipGetLastError();
}

hipError_t launch_topk_f32(const TopkArgs<float>& a, hipStream_t s) {
    hipLaunchKernelGGL(topk_kernel<float>, dim3(a.num_layers), dim3(kTopkThreads), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_topk_f64(const TopkArgs<double>& a, hipStream_t s) {
    hipLaunchKernelGGL(topk_kernel<double>, dim3(a.num_layers), dim3(kTopkThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_adjoint_f32(const AdjointArgs<float>& a, hipStream_t s) {
    int maxT = 0;
    for (int l = 0; l < a.num_layers; ++l) maxT = a.kh[l] * a.kw[l] > maxT ? a.kh[l] * a.kw[l] : maxT;
    const size_t lds = sizeof(cplx<float>) * (size_t)a.k * maxT;
    hipLaunchKernelGGL(adjoint_kernel<float>, dim3(a.blocks_before[a.num_layers]), dim3(256), lds, s, a);
    return hipGetLastError();
}
hipError_t launch_adjoint_f64(const AdjointArgs<double>& a, hipStream_t s) {
    int maxT = 0;
    for (int l = 0; l < a.num_layers; ++l) maxT = a.kh[l] * a.kw[l] > maxT ? a.kh[l] * a.kw[l] : maxT;
    const size_t lds = sizeof(cplx<double>) * (size_t)a.k * maxT;
    hipLaunchKernelGGL(adjoint_kernel<double>, dim3(a.blocks_before[a.num_layers]), dim3(256), lds, s, a);
    return hipGetLastError();
}

}  // namespace lfa
