// Register-resident one-sided Jacobi SVD for symbols of at most 64 rows and
// 64 columns (rows-in-lanes layout), gfx950.
//
// A work-group is one wavefront for G (plus one for the rotation accumulator
// when singular vectors are wanted).  Lane l of the G wave owns row l of the
// M x N working matrix G of its symbol in registers, all NC (>= N, power of
// two) columns; with ML lanes per symbol (16, 32 or 64) one wave holds
// 64/ML symbols.  Lane l of the second wave owns row l of the N x N
// accumulator Q.
//
// One round-robin step pairs the columns at positions (p, NC-1-p),
// p < NC/2 -- all compile-time register indices -- and then rotates the
// positions 1..NC-1 by one (register moves).  After NC-1 steps, i.e. one
// sweep, every column is back at its starting position, so the final column
// order is the original one.
//
// Per step:
//  1. every G lane forms its row's contributions to alpha_p = |g_j|^2,
//     beta_p = |g_k|^2 and gamma_p = g_j^H g_k for all pairs and writes them
//     to LDS ([symbol][row][4 * NC/2], padded row stride: conflict-free);
//  2. lane group (p, part) of the same wave sums a slice of the rows for pair
//     p, the parts are combined with xor shuffles; the first lane of the pair
//     computes the rotation (threshold test and angle in double precision)
//     and writes (c, s e^{-i phi}, flag) to a double-buffered LDS slot;
//  3. after one work-group barrier every lane of both waves reads the
//     parameters (broadcast) and applies the pair rotations to its registers.
//     The Q wave only applies, so it runs a step behind the G wave and its
//     work overlaps the next step's inner products.  A rotation that is not
//     needed is the identity (c = 1, s = 0), applied without a branch.
// One work-group barrier per step; no LDS traffic for G or Q themselves.

#include <hip/hip_runtime.h>
#include <math.h>

#include "lfa_internal.hpp"

namespace lfa {
namespace {


template <typename R>
__device__ __forceinline__ R skey(R v) {
    return v == v ? v : R(-1);
}


template <int NC, typename T>
__device__ __forceinline__ void rotate_positions(T (&g)[NC]) {
    // new[1] = old[NC-1], new[i] = old[i-1] for i = 2..NC-1
    const T last = g[NC - 1];
#pragma unroll
    for (int i = NC - 1; i >= 2; --i) g[i] = g[i - 1];
    g[1] = last;
}

__device__ __forceinline__ void phase_of(const double* tw, const LayerDesc& d, int theta, int t,
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

template <int NC, int ML>
struct WaveShape {
    static constexpr int SPW = 64 / ML;   // symbols per wave
    static constexpr int NP = NC / 2;     // pairs per step
    static constexpr int LP = ML / NP;    // lanes summing one pair (>= 2 since NC <= ML)
    static constexpr int RPL = NP;        // rows summed by one lane
    static constexpr int PST = 2 * NC + 4;  // partial row stride (elements), padded
};

// Elements of the partial-sum region (it also holds the assembled symbols
// during the load and the staged outputs during the finish: both fit in
// SPW*ML*PST since M <= ML and N <= NC), followed by the phase table.
template <typename R, int NC, int ML>
constexpr int wave_part_elems() {
    using S = WaveShape<NC, ML>;
    return S::SPW * ML * S::PST + S::SPW * kMaxTaps * 2;
}

template <typename R, int NC, int ML>
size_t wave_lds_bytes() {
    using S = WaveShape<NC, ML>;
    const size_t part = (size_t)wave_part_elems<R, NC, ML>() * sizeof(R);
    const size_t prm = 2 * (size_t)S::SPW * S::NP * 4 * sizeof(R);   // double-buffered
    const size_t small = (size_t)S::SPW * NC * (sizeof(R) + 2 * sizeof(int)) + 64 * sizeof(int);
    return part + prm + small + 64;
}

template <typename R, int NC, int ML>
__global__ void __launch_bounds__(128) wave_svd_kernel(SvdArgs<R> a) {
    using S = WaveShape<NC, ML>;
    constexpr int SPW = S::SPW, NP = S::NP, LP = S::LP, RPL = S::RPL, PST = S::PST;
    extern __shared__ __align__(16) char lds_raw[];
    R* part = reinterpret_cast<R*>(lds_raw);                       // [SPW][ML][PST]
    quad<R>* prm = reinterpret_cast<quad<R>*>(part + wave_part_elems<R, NC, ML>());   // [2][SPW][NP]
    R* sigs = reinterpret_cast<R*>(prm + 2 * SPW * NP);             // [SPW][NC]
    int* rankof = reinterpret_cast<int*>(sigs + SPW * NC);          // [SPW][NC]
    int* nzero = rankof + SPW * NC;                                 // [SPW] zero columns
    int* flags = nzero + SPW;                                       // [SPW] rotated this sweep

    const LayerDesc& d = a.d;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;             // 0: G rows, 1: Q rows
    const bool acc = blockDim.x > 64;
    const int sym = lane / ML, row = lane - (lane / ML) * ML;
    const int M = d.M, N = d.N;
    const int count = item_count(a);
    const int T = d.kh * d.kw;
    const double tol = a.tol;

    for (int base = blockIdx.x * SPW; base < count; base += gridDim.x * SPW) {
        const int item = base + sym;
        const bool active = item < count;
        const Target tg = active ? target_of(a, item) : Target{0, 0, -1};

        // ---------------------------------------------------------- load
        // The work-group assembles (or copies) the symbols of the wave into an
        // LDS tile in G layout, [s][row][col] with ML x NC entries per symbol,
        // zero outside M x N: G = A (row o, column i), or G = A^H (row i,
        // column o) when c_out < c_in.  Every G lane then loads its row with
        // constant offsets.
        cplx<R>* tile = reinterpret_cast<cplx<R>*>(part);        // [SPW][ML][NC]
        cplx<R>* ph = reinterpret_cast<cplx<R>*>(part + SPW * ML * PST);   // [SPW][T]
        if (a.A == nullptr) {
            for (int x = threadIdx.x; x < SPW * T; x += blockDim.x) {
                const int s = x / T, t = x - (x / T) * T;
                const int it = base + s;
                double re = 1.0, im = 0.0;
                if (it < count) phase_of(a.tw, d, target_of(a, it).theta, t, re, im);
                ph[x] = {R(re), R(im)};
            }
            __syncthreads();
        }
        for (int x = threadIdx.x; x < SPW * ML * NC; x += blockDim.x) {
            const int s = x / (ML * NC), rc = x - s * (ML * NC);
            const int r = rc / NC, c = rc - (rc / NC) * NC;
            const int it = base + s;
            cplx<R> v = {R(0), R(0)};
            if (it < count && r < M && c < N) {
                const int o = d.transposed ? c : r, i = d.transposed ? r : c;
                const size_t e = (size_t)o * d.c_in + i;
                if (a.A == nullptr) {
                    const R* w = a.W + e * T;
                    for (int t = 0; t < T; ++t) {
                        const R wt = w[t];
                        const cplx<R> p = ph[s * T + t];
                        v.x = fma(wt, p.x, v.x);
                        v.y = fma(wt, p.y, v.y);
                    }
                } else {
                    v = a.A[(size_t)target_of(a, it).theta * d.c_out * d.c_in + e];
                }
                if (d.transposed) v.y = -v.y;
            }
            tile[x] = v;
        }
        __syncthreads();
        cplx<R> g[NC];
#pragma unroll
        for (int j = 0; j < NC; ++j) g[j] = tile[(sym * ML + row) * NC + j];
        if (wave != 0) {
#pragma unroll
            for (int j = 0; j < NC; ++j) g[j] = {R(0), R(0)};
        }
        __syncthreads();
        if (wave == 1) {
            // accumulator rows: Q = I (N x N), zero beyond N
#pragma unroll
            for (int j = 0; j < NC; ++j) g[j] = {R((row == j && j < N) ? 1 : 0), R(0)};
        }

        // -------------------------------------------------------- sweeps
        int sweeps = 0;
        bool my_conv = false;       // symbol of this lane converged
        int conv_at = 0;            // sweeps used by this lane's symbol
        int buf = 0;                // parameter buffer of the current step
        for (int sw = 0; sw < a.max_sweeps; ++sw) {
            if (threadIdx.x < SPW) flags[threadIdx.x] = 0;
            bool rotated = false;
            for (int step = 0; step < NC - 1; ++step) {
                quad<R>* prm_b = prm + buf * (SPW * NP);
                if (wave == 0) {
                    // 1. partial inner products of this lane's row
#pragma unroll
                    for (int p = 0; p < NP; ++p) {
                        const cplx<R> x = g[p], y = g[NC - 1 - p];
                        quad<R> q;
                        q.a = fma(x.x, x.x, x.y * x.y);
                        q.b = fma(y.x, y.x, y.y * y.y);
                        q.c = fma(x.x, y.x, x.y * y.y);
                        q.d = fma(x.x, y.y, -x.y * y.x);
                        *reinterpret_cast<quad<R>*>(part + (sym * ML + row) * PST + 4 * p) = q;
                        if ((p & 7) == 7) __builtin_amdgcn_sched_barrier(0);
                    }
                    // the partials were written by other lanes of this wave:
                    // LDS operations of one wave complete in order
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    // 2. sums over the rows, 3. rotation of pair p
                    const int p = row % NP, k = row / NP;
                    R s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll 4
                    for (int r = 0; r < RPL; ++r) {
                        const quad<R> q =
                            *reinterpret_cast<const quad<R>*>(part + (sym * ML + k * RPL + r) * PST + 4 * p);
                        s0 += q.a;
                        s1 += q.b;
                        s2 += q.c;
                        s3 += q.d;
                    }
#pragma unroll
                    for (int off = NP; off < ML; off <<= 1) {
                        s0 += __shfl_xor(s0, off, 64);
                        s1 += __shfl_xor(s1, off, 64);
                        s2 += __shfl_xor(s2, off, 64);
                        s3 += __shfl_xor(s3, off, 64);
                    }
                    if (k == 0) {
                        const quad<R> q = rotation<R>(s0, s1, s2, s3, tol);
                        rotated |= q.d != R(0);
                        prm_b[sym * NP + p] = q;
                    }
                }
                // parameters of this step visible to both waves; the Q wave
                // applies step s while the G wave already works on step s+1
                // (double-buffered parameters, one barrier per step)
                __syncthreads();
#pragma unroll
                for (int p0 = 0; p0 < NP; p0 += 8) {
#pragma unroll
                    for (int p = p0; p < p0 + 8 && p < NP; ++p) {
                        const quad<R> q = prm_b[sym * NP + p];
                        rot_apply(g[p], g[NC - 1 - p], q.a, q.b, q.c);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
                rotate_positions<NC>(g);
                buf ^= 1;
            }
            ++sweeps;
            // convergence: a sweep without rotations, per symbol
            if (rotated) flags[sym] = 1;
            __syncthreads();
            const bool conv_now = flags[sym] == 0;
            if (!my_conv && conv_now) {
                my_conv = true;
                conv_at = sweeps;
            }
            bool all = true;
#pragma unroll
            for (int s = 0; s < SPW; ++s) all = all && (flags[s] == 0);
            __syncthreads();
            if (all) break;
        }
        if (!my_conv) conv_at = sweeps;

        // -------------------------------------------------------- finish
        // column norms
        if (wave == 0) {
#pragma unroll
            for (int j = 0; j < NC; ++j)
                part[(sym * ML + row) * PST + j] = fma(g[j].x, g[j].x, g[j].y * g[j].y);
        }
        __syncthreads();
        if (wave == 0 && row < NC) {
            R s = 0;
            for (int r = 0; r < ML; ++r) s += part[(sym * ML + r) * PST + row];
            sigs[sym * NC + row] = sqrt(s);
        }
        __syncthreads();
        // rank sort of the N real columns: descending, ties by index
        if (wave == 0 && row < N) {
            const R sj = skey(sigs[sym * NC + row]);
            int rank = 0;
            for (int k = 0; k < N; ++k) {
                const R sk = skey(sigs[sym * NC + k]);
                rank += (sk > sj) || (sk == sj && k < row);
            }
            rankof[sym * NC + row] = rank;
            if (active) {
                a.sigma[(size_t)tg.out * N + rank] = sigs[sym * NC + row];
                if (tg.mirror >= 0) a.sigma[(size_t)tg.mirror * N + rank] = sigs[sym * NC + row];
            }
        }
        if (threadIdx.x < SPW) {
            int z = 0;
            for (int k = 0; k < N; ++k) z += sigs[threadIdx.x * NC + k] == R(0);
            nzero[threadIdx.x] = z;
        }
        __syncthreads();
        if (a.info && wave == 0 && row == 0 && active) {
            atomicAdd(&a.info[LFA_INFO_SUM_SWEEPS], conv_at);
            atomicMax(&a.info[LFA_INFO_MAX_SWEEPS], conv_at);
            if (!my_conv) atomicAdd(&a.info[LFA_INFO_NONCONVERGED], 1);
            bool bad = false;
            for (int k = 0; k < N; ++k) bad |= !isfinite(sigs[sym * NC + k]);
            if (bad) atomicOr(&a.info[LFA_INFO_NONFINITE], 1);
        }
        cplx<R>* left = d.transposed ? a.V : a.U;
        cplx<R>* right = d.transposed ? a.U : a.V;
        cplx<R>* stage = reinterpret_cast<cplx<R>*>(part);   // [SPW][M][N] output staging
        if (left) {
            if (wave == 0 && row < M) {
#pragma unroll
                for (int j = 0; j < NC; ++j) {
                    if (j < N) {
                        const R sj = sigs[sym * NC + j];
                        const R inv = sj > R(0) ? R(1) / sj : R(0);
                        stage[(size_t)(sym * M + row) * N + rankof[sym * NC + j]] = {g[j].x * inv, g[j].y * inv};
                    }
                    if ((j & 7) == 7) __builtin_amdgcn_sched_barrier(0);
                }
            }
            __syncthreads();
            // Columns with sigma == 0 (sorted last): orthonormal completion by
            // two passes of classical Gram-Schmidt of unit vectors against the
            // accepted columns, one symbol at a time, by the G wave alone
            // (lane = row); every loop bound below is uniform over that wave.
            if (wave == 0) {
                for (int s = 0; s < SPW; ++s) {
                    const int nz = nzero[s];
                    int cand = 0;
                    R thresh = R(0.5);
                    for (int c = N - nz; c < N; ++c) {
                        bool done = false;
                        for (int tries = 0; !done && tries < 4 * M; ++tries) {
                            if (cand == M) {
                                cand = 0;
                                thresh *= R(0.2);
                            }
                            cplx<R> x = {R(lane == cand ? 1 : 0), R(0)};
                            for (int pass = 0; pass < 2; ++pass) {
                                cplx<R> y = x;
                                for (int col = 0; col < c; ++col) {
                                    cplx<R> u = {R(0), R(0)};
                                    if (lane < M) u = stage[(size_t)(s * M + lane) * N + col];
                                    R cr = u.x * x.x + u.y * x.y;
                                    R ci = u.x * x.y - u.y * x.x;
#pragma unroll
                                    for (int off = 32; off >= 1; off >>= 1) {
                                        cr += __shfl_xor(cr, off, 64);
                                        ci += __shfl_xor(ci, off, 64);
                                    }
                                    y.x -= cr * u.x - ci * u.y;
                                    y.y -= cr * u.y + ci * u.x;
                                }
                                x = y;
                            }
                            R nrm = x.x * x.x + x.y * x.y;
#pragma unroll
                            for (int off = 32; off >= 1; off >>= 1) nrm += __shfl_xor(nrm, off, 64);
                            nrm = sqrt(nrm);
                            if (nrm > thresh) {
                                if (lane < M) stage[(size_t)(s * M + lane) * N + c] = {x.x / nrm, x.y / nrm};
                                done = true;
                            }
                            ++cand;
                            // the next candidate reads the column just written
                            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                            __builtin_amdgcn_wave_barrier();
                        }
                    }
                }
            }
            __syncthreads();
            for (int e = threadIdx.x; e < SPW * M * N; e += blockDim.x) {
                const int s = e / (M * N);
                const int it = base + s;
                if (it < count) {
                    const Target t = target_of(a, it);
                    const cplx<R> v = stage[e];
                    left[(size_t)t.out * M * N + (e - s * M * N)] = v;
                    if (t.mirror >= 0) left[(size_t)t.mirror * M * N + (e - s * M * N)] = {v.x, -v.y};
                }
            }
            __syncthreads();
        }
        if (right && acc) {
            if (wave == 1 && row < N) {
#pragma unroll
                for (int j = 0; j < NC; ++j)
                    if (j < N) stage[(size_t)(sym * N + row) * N + rankof[sym * NC + j]] = g[j];
            }
            __syncthreads();
            for (int e = threadIdx.x; e < SPW * N * N; e += blockDim.x) {
                const int s = e / (N * N);
                const int it = base + s;
                if (it < count) {
                    const Target t = target_of(a, it);
                    const cplx<R> v = stage[e];
                    right[(size_t)t.out * N * N + (e - s * N * N)] = v;
                    if (t.mirror >= 0) right[(size_t)t.mirror * N * N + (e - s * N * N)] = {v.x, -v.y};
                }
            }
            __syncthreads();
        }
    }
}

template <typename R, int NC, int ML>
hipError_t launch_wave_t(const SvdArgs<R>& a, int grid, hipStream_t st) {
    const size_t lds = wave_lds_bytes<R, NC, ML>();
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(wave_svd_kernel<R, NC, ML>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((wave_svd_kernel<R, NC, ML>), dim3(grid), dim3(a.d.threads), lds, st, a);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_wave_any(const SvdArgs<R>& a, int grid, hipStream_t st) {
    const int NC = a.d.wave_nc, ML = a.d.wave_ml;
#define LFA_CASE(nc, ml) \
    if (NC == nc && ML == ml) return launch_wave_t<R, nc, ml>(a, grid, st);
    LFA_CASE(4, 16) LFA_CASE(8, 16) LFA_CASE(16, 16)
    LFA_CASE(4, 32) LFA_CASE(8, 32) LFA_CASE(16, 32) LFA_CASE(32, 32)
    LFA_CASE(4, 64) LFA_CASE(8, 64) LFA_CASE(16, 64) LFA_CASE(32, 64) LFA_CASE(64, 64)
#undef LFA_CASE
    return hipErrorInvalidValue;
}

}  // namespace

size_t wave_lds_bytes_for(int nc, int ml, int elem_bytes) {
#define LFA_CASE(n_, m_)                                                                   \
    if (nc == n_ && ml == m_)                                                              \
        return elem_bytes == 8 ? wave_lds_bytes<double, n_, m_>() : wave_lds_bytes<float, n_, m_>();
    LFA_CASE(4, 16) LFA_CASE(8, 16) LFA_CASE(16, 16)
    LFA_CASE(4, 32) LFA_CASE(8, 32) LFA_CASE(16, 32) LFA_CASE(32, 32)
    LFA_CASE(4, 64) LFA_CASE(8, 64) LFA_CASE(16, 64) LFA_CASE(32, 64) LFA_CASE(64, 64)
#undef LFA_CASE
    return 0;
}

hipError_t launch_wave_svd_f32(const SvdArgs<float>& a, int grid, hipStream_t s) {
    return launch_wave_any<float>(a, grid, s);
}
hipError_t launch_wave_svd_f64(const SvdArgs<double>& a, int grid, hipStream_t s) {
    return launch_wave_any<double>(a, grid, s);
}

}  // namespace lfa
