// Device code of the Jacobi SVD kernels, shared by the translation units
// that define kernels (plain launches, the register kernel, the persistent
// launch).  Header-only: templates and inline functions.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "lfa_internal.hpp"

namespace lfa {
namespace dev {

// ============================ blocked kernel ================================
//  Batched one-sided Jacobi SVD of convolution symbols on gfx950.
//
// One work-group (or a team of them) owns one symbol at a time.  It
// assembles the c_out x c_in symbol A_k = sum_y M_y exp(+2 pi i <k,y>)
// (Sec. III "Convolution Theorem", Algorithm 1 symbol step) straight into
// its working matrix G (a global slot), runs complex one-sided (Hestenes)
// Jacobi sweeps on the columns of G, and writes sigma (sorted), U and V
// (Algorithm 1 SVD step).  The load and the finish below are shared with
// the QR path and the persistent kernel.
//
// G is M x N, column-major with leading dimension ldg, M = max(c_out, c_in),
// N = min(c_out, c_in).  For c_out >= c_in, G = A and the accumulated
// rotations form V; for c_out < c_in, G = A^H and the roles of U and V swap.


template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

template <typename R>
__device__ __forceinline__ R shfl_xor(R v, int mask) {
    return __shfl_xor(v, mask, 64);
}

// Sum over groups of L consecutive lanes (L a power of two <= 64).
template <typename R, int L>
__device__ __forceinline__ R group_sum(R v) {
#pragma unroll
    for (int off = L / 2; off >= 1; off >>= 1) v += shfl_xor(v, off);
    return v;
}

// Round-robin ("circle") ordering on Np (even) positions: position 0 is
// fixed, positions 1..Np-1 rotate by one each step.  Over Np-1 steps every
// unordered pair meets exactly once.
__device__ __forceinline__ void rr_pair(int pr, int step, int Np, int& j, int& k) {
    const int c = Np - 1;
    auto pos = [&](int i) { return i == 0 ? 0 : ((i - 1 + step) % c) + 1; };
    j = pos(pr);
    k = pos(Np - 1 - pr);
}

// exp(2 pi i ((p*y1 mod n)/n + (q*y2 mod m)/m)) from the double twiddle tables.
__device__ __forceinline__ void phase(const double* tw, const LayerDesc& d, int p, int q, int t,
                                      double& re, double& im) {
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

template <typename R>
struct Shared {
    cplx<R>* ph;     // [kMaxTaps] phases of the current frequency
    R* sig;          // [N] column norms
    int* perm;       // [N] sorted position -> column
    int* inv;        // [N] column -> sorted position
    cplx<R>* coef;   // [N] Gram-Schmidt coefficients (completion of zero columns)
    cplx<R>* xtmp;   // [M] Gram-Schmidt work vector
    int* flags;      // [4] rotation flags (3 rotating) + scratch
    R* red;          // [64] scratch for block reductions
    cplx<R>* G;      // working matrix (LDS or global)
    cplx<R>* Q;      // rotation accumulator (LDS or global), or null
    size_t small_end;   // LDS bytes used by the arrays above (G/Q excluded)
};

template <typename R>
__device__ __forceinline__ Shared<R> carve(char* lds, const LayerDesc& d, bool acc, char* gslot) {
    Shared<R> s;
    char* p = lds;
    s.ph = reinterpret_cast<cplx<R>*>(p);
    p += sizeof(cplx<R>) * kMaxTaps;
    s.red = reinterpret_cast<R*>(p);
    p += sizeof(R) * 64;
    s.sig = reinterpret_cast<R*>(p);
    p += sizeof(R) * ((d.N + 3) & ~3);
    s.perm = reinterpret_cast<int*>(p);
    p += sizeof(int) * ((d.N + 3) & ~3);
    s.inv = reinterpret_cast<int*>(p);
    p += sizeof(int) * ((d.N + 3) & ~3);
    p = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(p) + 15) & ~uintptr_t(15));
    s.coef = reinterpret_cast<cplx<R>*>(p);
    p += sizeof(cplx<R>) * d.N;
    s.xtmp = reinterpret_cast<cplx<R>*>(p);
    p += sizeof(cplx<R>) * d.M;
    s.flags = reinterpret_cast<int*>(p);
    p += sizeof(int) * 4;
    p = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(p) + 15) & ~uintptr_t(15));
    s.small_end = (size_t)(p - lds);
    char* base = (d.storage == kLds) ? p : gslot;
    s.G = reinterpret_cast<cplx<R>*>(base);
    base += sizeof(cplx<R>) * (size_t)d.ldg * d.N;
    s.Q = acc ? reinterpret_cast<cplx<R>*>(base) : nullptr;
    return s;
}

template <typename R>
__device__ __forceinline__ R sort_key(R v) {
    return v == v ? v : R(-1);
}

// Block-wide sum (all threads receive it).
template <typename R>
__device__ R block_sum(R v, R* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    v = group_sum<R, 64>(v);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    R t = 0;
    for (int w = 0; w < nw; ++w) t += red[w];
    return t;
}

// ---------------------------------------------------------------------------
// Load the symbol of frequency theta into G (and Q = I).
// ---------------------------------------------------------------------------
constexpr int kLoadTaps = 16;    // taps of the unrolled assembly in load_symbol

// BATCH: the assembly with its weight loads in flight together (taken by
// the kernels without an accumulator; with one, its registers spilled into
// the sweeps).
template <typename R, bool BATCH = true>
__device__ void load_symbol(const SvdArgs<R>& a, const Shared<R>& s, int theta) {
    const LayerDesc& d = a.d;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int T = d.kh * d.kw;
    const int p = theta / d.m, q = theta - (theta / d.m) * d.m;
    const int E = d.c_out * d.c_in;
    if (a.A == nullptr) {
        for (int t = tid; t < T; t += nt) {
            double re, im;
            phase(a.tw, d, p, q, t, re, im);
            s.ph[t] = {R(re), R(im)};
        }
        __syncthreads();
        if (BATCH && T <= kLoadTaps) {
            // two entries per thread at a time, their taps loaded without a
            // branch (taps past T read tap 0 and add an exact zero), so that
            // the loads are in flight together; the sums are the same
            for (int e0 = tid; e0 < E; e0 += 2 * nt) {
                R wv[2][kLoadTaps];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int e = e0 + u * nt;
                    const R* w = a.W + (size_t)(e < E ? e : 0) * T;
#pragma unroll
                    for (int t = 0; t < kLoadTaps; ++t) wv[u][t] = w[t < T ? t : 0];
                }
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int e = e0 + u * nt;
                    if (e >= E) continue;
                    R re = 0, im = 0;
#pragma unroll
                    for (int t = 0; t < kLoadTaps; ++t) {
                        const R wt = t < T ? wv[u][t] : R(0);
                        const cplx<R> ph = s.ph[t < T ? t : 0];
                        re = fma(wt, ph.x, re);
                        im = fma(wt, ph.y, im);
                    }
                    const int o = e / d.c_in, i = e - (e / d.c_in) * d.c_in;
                    if (!d.transposed) s.G[(size_t)i * d.ldg + o] = {re, im};
                    else               s.G[(size_t)o * d.ldg + i] = {re, -im};
                }
            }
        } else {
            for (int e = tid; e < E; e += nt) {
                const R* w = a.W + (size_t)e * T;
                R re = 0, im = 0;
                for (int t = 0; t < T; ++t) {
                    const R wt = w[t];
                    const cplx<R> ph = s.ph[t];
                    re = fma(wt, ph.x, re);
                    im = fma(wt, ph.y, im);
                }
                const int o = e / d.c_in, i = e - (e / d.c_in) * d.c_in;
                if (!d.transposed) s.G[(size_t)i * d.ldg + o] = {re, im};
                else               s.G[(size_t)o * d.ldg + i] = {re, -im};
            }
        }
    } else {
        // four entries per thread loaded before any is stored
        const cplx<R>* A = a.A + (size_t)theta * E;
        for (int e0 = tid; e0 < E; e0 += 4 * nt) {
            cplx<R> v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + u * nt;
                if (e < E) v[u] = A[e];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + u * nt;
                if (e >= E) continue;
                const int o = e / d.c_in, i = e - (e / d.c_in) * d.c_in;
                if (!d.transposed) s.G[(size_t)i * d.ldg + o] = v[u];
                else               s.G[(size_t)o * d.ldg + i] = {v[u].x, -v[u].y};
            }
        }
    }
    if (s.Q) {
        const int N = d.N;
        for (int e = tid; e < N * N; e += nt) {
            const int j = e / N, i = e - (e / N) * N;
            s.Q[(size_t)j * d.ldv + i] = {R(i == j ? 1 : 0), R(0)};
        }
    }
}

// ---------------------------------------------------------------------------
// Norms, sort, normalisation, completion of zero columns, outputs.
// ---------------------------------------------------------------------------
// WIDE: the completion of zero columns forms four columns' inner products at
// once (their loads and reductions overlap).  The persistent kernel and the
// blocked kernel with the rotation accumulator take the one-column loops:
// beside their other paths the wider ones spill registers into the sweeps.
template <typename R, int L, bool WIDE = true>
__device__ void finish(const SvdArgs<R>& a, const Shared<R>& s, int out_idx, int mirror,
                       int sweeps, bool converged) {
    const LayerDesc& d = a.d;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & (L - 1), group = tid / L, ngroups = nt / L;
    const int M = d.M, N = d.N, ldg = d.ldg, ldv = d.ldv;
    cplx<R>* G = s.G;
    cplx<R>* Q = s.Q;

    // column norms (unrolled: several loads in flight)
    for (int j = group; j < N; j += ngroups) {
        R acc = 0;
#pragma unroll 8
        for (int i = lane; i < M; i += L) {
            const cplx<R> v = G[(size_t)j * ldg + i];
            acc = fma(v.x, v.x, fma(v.y, v.y, acc));
        }
        acc = group_sum<R, L>(acc);
        if (lane == 0) s.sig[j] = sqrt(acc);
    }
    __syncthreads();
    {
        // numerically zero columns (see negligible_sq) are reported as 0
        R tot = 0;
        for (int j = tid; j < N; j += nt) tot = fma(s.sig[j], s.sig[j], tot);
        const double floor = negligible_sq<R>() * double(block_sum<R>(tot, s.red));
        for (int j = tid; j < N; j += nt)
            if (double(s.sig[j]) * double(s.sig[j]) <= floor) s.sig[j] = R(0);
        __syncthreads();
    }
    // rank sort: descending, ties by column index; NaN sorts as -1 so the
    // ranks always form a permutation
    for (int j = tid; j < N; j += nt) {
        const R sj = sort_key(s.sig[j]);
        int rank = 0;
        for (int k = 0; k < N; ++k) {
            const R sk = sort_key(s.sig[k]);
            rank += (sk > sj) || (sk == sj && k < j);
        }
        s.perm[rank] = j;
        s.inv[j] = rank;
    }
    __syncthreads();

    const int r = N;
    R* sig_out = a.sigma + (size_t)out_idx * r;
    R* sig_mir = mirror >= 0 ? a.sigma + (size_t)mirror * r : nullptr;
    bool bad = false;
    for (int c = tid; c < r; c += nt) {
        const R v = s.sig[s.perm[c]];
        sig_out[c] = v;
        if (sig_mir) sig_mir[c] = v;
        bad |= !isfinite(v);
    }
    const bool want_left = d.transposed ? (a.V != nullptr) : (a.U != nullptr);
    const bool want_right = d.transposed ? (a.U != nullptr) : (a.V != nullptr);

    if (want_right) {
        cplx<R>* out = (d.transposed ? a.U : a.V) + (size_t)out_idx * N * r;
        cplx<R>* mir = mirror >= 0 ? (d.transposed ? a.U : a.V) + (size_t)mirror * N * r : nullptr;
        // four entries per thread loaded before any is stored
        for (int e0 = tid; e0 < N * r; e0 += 4 * nt) {
            cplx<R> v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + u * nt;
                if (e < N * r) {
                    const int i = e / r, c = e - (e / r) * r;
                    v[u] = Q[(size_t)s.perm[c] * ldv + i];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + u * nt;
                if (e < N * r) {
                    out[e] = v[u];
                    if (mir) mir[e] = {v[u].x, -v[u].y};
                }
            }
        }
    }
    // the accumulator has been written out: its memory may serve the
    // completion below
    __syncthreads();
    if (want_left) {
        // normalise columns in place: u_j = g_j / sigma_j (zero columns stay 0)
        for (int e0 = tid; e0 < N * M; e0 += 4 * nt) {
            cplx<R> v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + u * nt;
                if (e < N * M) {
                    const int j = e / M, i = e - (e / M) * M;
                    v[u] = G[(size_t)j * ldg + i];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + u * nt;
                if (e < N * M) {
                    const int j = e / M, i = e - (e / M) * M;
                    const R sj = s.sig[j];
                    const R inv = sj > R(0) ? R(1) / sj : R(0);
                    G[(size_t)j * ldg + i] = {v[u].x * inv, v[u].y * inv};
                }
            }
        }
        __syncthreads();
        // Columns with sigma == 0 (they sort last) get an orthonormal
        // completion: unit vectors e_0, e_1, ... orthogonalised by two passes
        // of classical Gram-Schmidt against every accepted column, kept when
        // the residual norm exceeds a threshold (1/2, at most half the root
        // mean square of the residuals, lowered if no unit vector qualifies;
        // some residual has norm >= 1/sqrt(M)).
        int nz = 0;
        while (nz < N && s.sig[s.perm[N - 1 - nz]] == R(0)) ++nz;
        const int ra = N - nz;   // accepted columns, in rank order perm[0 .. ra)
        // Many zero columns (a rank-deficient symbol): the completion is the
        // trailing columns of Q = H_0 ... H_{ra-1}, the Householder
        // reflectors of the accepted columns (QR), kept in the
        // accumulator's memory: nz ra M work instead of the nz N M of
        // Gram-Schmidt, and two barriers per reflector instead of several
        // per zero column.
        // Without that memory (no accumulator) and with at least twice as
        // many zero columns as accepted ones, the reflectors go to the last
        // ra zero columns of G instead: the other zero columns are completed
        // from them, and those last ra ones by Gram-Schmidt below.
        const bool hh_q =
            nz >= 2 && ra >= 1 && want_right && Q != nullptr && (size_t)ra * M <= (size_t)N * ldv;
        const bool hh_g = !hh_q && ra >= 1 && nz >= 2 * ra && nz - ra >= 2;
        const bool householder = hh_q || hh_g;
        const int nh = hh_q ? nz : nz - ra;        // zero columns completed from the reflectors
        // reflector k: Q row block k, or zero column perm[N - ra + k] of G
        auto refl = [&](int k) -> cplx<R>* {
            return hh_q ? Q + (size_t)k * M : G + (size_t)s.perm[N - ra + k] * ldg;
        };
        if (householder) {
            for (int e = tid; e < ra * M; e += nt) {
                const int k = e / M, i = e - (e / M) * M;
                refl(k)[i] = G[(size_t)s.perm[k] * ldg + i];
            }
            __syncthreads();
            for (int k = 0; k < ra; ++k) {
                cplx<R>* v = refl(k);
                R part = 0;
                for (int i = k + tid; i < M; i += nt) part = fma(v[i].x, v[i].x, fma(v[i].y, v[i].y, part));
                const R nx = sqrt(block_sum<R>(part, s.red));
                const cplx<R> al = v[k];
                const R aa = sqrt(al.x * al.x + al.y * al.y);
                __syncthreads();
                if (tid == 0) {
                    // v_k = alpha + e^{i arg alpha} ||x||, beta = 2 / (v^H v) = 1 / (||x|| (||x|| + |alpha|))
                    const R pr = aa > R(0) ? al.x / aa : R(1), pi = aa > R(0) ? al.y / aa : R(0);
                    v[k] = {al.x + pr * nx, al.y + pi * nx};
                    s.coef[k] = {nx > R(0) ? R(1) / (nx * (nx + aa)) : R(0), R(0)};
                }
                __syncthreads();
                const R beta = s.coef[k].x;
                // H_k applied to the later accepted columns (rows >= k)
                for (int j = k + 1 + group; j < ra; j += ngroups) {
                    const cplx<R>* c = refl(j);
                    cplx<R> w = {R(0), R(0)};
                    for (int i = k + lane; i < M; i += L) {
                        w.x = fma(v[i].x, c[i].x, fma(v[i].y, c[i].y, w.x));
                        w.y = fma(v[i].x, c[i].y, fma(-v[i].y, c[i].x, w.y));
                    }
                    w.x = group_sum<R, L>(w.x);
                    w.y = group_sum<R, L>(w.y);
                    if (lane == 0) s.coef[j] = w;
                }
                __syncthreads();
                for (int e = tid; e < (ra - k - 1) * M; e += nt) {
                    const int j = k + 1 + e / M, i = e - (e / M) * M;
                    if (i < k) continue;
                    const cplx<R> w = s.coef[j], vi = v[i];
                    const R fr = beta * (w.x * vi.x - w.y * vi.y), fi = beta * (w.x * vi.y + w.y * vi.x);
                    cplx<R>* cj = refl(j);
                    cj[i] = {cj[i].x - fr, cj[i].y - fi};
                }
                __syncthreads();
            }
            // zero column z: H_0 ... H_{ra-1} e_{ra+z}
            for (int e = tid; e < nh * M; e += nt) {
                const int z = e / M, i = e - (e / M) * M;
                G[(size_t)s.perm[ra + z] * ldg + i] = {R(i == ra + z ? 1 : 0), R(0)};
            }
            __syncthreads();
            for (int k = ra - 1; k >= 0; --k) {
                const cplx<R>* v = refl(k);
                const R beta = s.coef[k].x;
                if constexpr (!WIDE) {
                    for (int z = group; z < nh; z += ngroups) {
                        const cplx<R>* x = G + (size_t)s.perm[ra + z] * ldg;
                        cplx<R> w = {R(0), R(0)};
#pragma unroll 8
                        for (int i = k + lane; i < M; i += L) {
                            w.x = fma(v[i].x, x[i].x, fma(v[i].y, x[i].y, w.x));
                            w.y = fma(v[i].x, x[i].y, fma(-v[i].y, x[i].x, w.y));
                        }
                        w.x = group_sum<R, L>(w.x);
                        w.y = group_sum<R, L>(w.y);
                        if (lane == 0) s.coef[ra + z] = w;
                    }
                } else {
                    // four columns per group at once, so that their loads and
                    // reductions overlap (each column's sum in the same order)
                    for (int z0 = 4 * group; z0 < nh; z0 += 4 * ngroups) {
                        const cplx<R>* x[4];
#pragma unroll
                        for (int c = 0; c < 4; ++c)
                            x[c] = G + (size_t)s.perm[ra + (z0 + c < nh ? z0 + c : nh - 1)] * ldg;
                        cplx<R> w[4];
#pragma unroll
                        for (int c = 0; c < 4; ++c) w[c] = {R(0), R(0)};
#pragma unroll 2
                        for (int i = k + lane; i < M; i += L) {
                            const cplx<R> vi = v[i];
                            cplx<R> xi[4];
#pragma unroll
                            for (int c = 0; c < 4; ++c) xi[c] = x[c][i];
#pragma unroll
                            for (int c = 0; c < 4; ++c) {
                                w[c].x = fma(vi.x, xi[c].x, fma(vi.y, xi[c].y, w[c].x));
                                w[c].y = fma(vi.x, xi[c].y, fma(-vi.y, xi[c].x, w[c].y));
                            }
                        }
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            w[c].x = group_sum<R, L>(w[c].x);
                            w[c].y = group_sum<R, L>(w[c].y);
                        }
                        if (lane == 0) {
#pragma unroll
                            for (int c = 0; c < 4; ++c)
                                if (z0 + c < nh) s.coef[ra + z0 + c] = w[c];
                        }
                    }
                }
                __syncthreads();
                if constexpr (!WIDE) {
                    // four entries per thread loaded before any is stored
                    for (int e0 = tid; e0 < nh * M; e0 += 4 * nt) {
                        cplx<R> xv[4], vv[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int e = e0 + u * nt;
                            const int z = e / M, i = e - (e / M) * M;
                            if (e < nh * M && i >= k) {
                                xv[u] = G[(size_t)s.perm[ra + z] * ldg + i];
                                vv[u] = v[i];
                            }
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int e = e0 + u * nt;
                            const int z = e / M, i = e - (e / M) * M;
                            if (e < nh * M && i >= k) {
                                const cplx<R> w = s.coef[ra + z];
                                G[(size_t)s.perm[ra + z] * ldg + i] = {
                                    xv[u].x - beta * (w.x * vv[u].x - w.y * vv[u].y),
                                    xv[u].y - beta * (w.x * vv[u].y + w.y * vv[u].x)};
                            }
                        }
                    }
                } else {
                    // eight entries per thread loaded, without branches (an
                    // index past the end is clamped and its value unused),
                    // before any is stored
                    const int ne = nh * M;
                    for (int e0 = tid; e0 < ne; e0 += 8 * nt) {
                        cplx<R> xv[8], vv[8];
                        int col[8], row[8];
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            const int e = e0 + u * nt < ne ? e0 + u * nt : ne - 1;
                            const int z = e / M;
                            row[u] = e - z * M;
                            col[u] = z;
                            xv[u] = G[(size_t)s.perm[ra + z] * ldg + row[u]];
                            vv[u] = v[row[u]];
                        }
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            if (e0 + u * nt < ne && row[u] >= k) {
                                const cplx<R> w = s.coef[ra + col[u]];
                                G[(size_t)s.perm[ra + col[u]] * ldg + row[u]] = {
                                    xv[u].x - beta * (w.x * vv[u].x - w.y * vv[u].y),
                                    xv[u].y - beta * (w.x * vv[u].y + w.y * vv[u].x)};
                            }
                        }
                    }
                }
                __syncthreads();
            }
        }
        // After the reflectors the directions still missing are close to the
        // unit vectors e_nz, ..., e_{M-1} (the trailing columns of Q are
        // perturbed unit vectors), so the scan starts there; otherwise at e_0.
        // The threshold is lowered after every M candidates.
        int cand = hh_g && nz < M ? nz : 0, scanned = 0;
        R thresh = R(0.5);
        for (int zc = hh_q ? N : (hh_g ? N - ra : N - nz); zc < N; ++zc) {
            const int jz = s.perm[zc];
            // zc columns are accepted: the unit vectors' residuals have mean
            // square (M - zc) / M, so some residual is at least that large
            // and half of it is accepted without a scan of every candidate
            thresh = fmin(thresh, R(0.5) * sqrt(R(M - zc > 1 ? M - zc : 1) / R(M)));
            bool done = false;
            for (int tries = 0; !done && tries < 4 * M; ++tries) {
                if (cand == M) cand = 0;
                if (scanned == M) {
                    scanned = 0;
                    thresh *= R(0.2);
                }
                for (int i = tid; i < M; i += nt) G[(size_t)jz * ldg + i] = {R(i == cand), R(0)};
                __syncthreads();
                for (int pass = 0; pass < 2; ++pass) {
                    if constexpr (!WIDE) {
                        for (int col = group; col < N; col += ngroups) {
                            // accepted: nonzero columns and zero columns completed earlier
                            const bool use = col != jz && (s.sig[col] > R(0) || s.inv[col] < zc);
                            cplx<R> acc = {0, 0};
                            if (use) {
                                for (int i = lane; i < M; i += L) {
                                    const cplx<R> u = G[(size_t)col * ldg + i];
                                    const cplx<R> x = G[(size_t)jz * ldg + i];
                                    acc.x = fma(u.x, x.x, fma(u.y, x.y, acc.x));
                                    acc.y = fma(u.x, x.y, fma(-u.y, x.x, acc.y));
                                }
                            }
                            acc.x = group_sum<R, L>(acc.x);
                            acc.y = group_sum<R, L>(acc.y);
                            if (lane == 0) s.coef[col] = acc;
                        }
                    } else {
                        // four columns per group at once (each column's sum in
                        // the same order)
                        for (int c0 = 4 * group; c0 < N; c0 += 4 * ngroups) {
                            int col[4];
                            bool use[4];
#pragma unroll
                            for (int c = 0; c < 4; ++c) {
                                const int cc = c0 + c;
                                // accepted: nonzero columns and zero columns completed earlier
                                use[c] = cc < N && cc != jz && (s.sig[cc] > R(0) || s.inv[cc] < zc);
                                col[c] = cc < N ? cc : N - 1;
                            }
                            cplx<R> acc[4];
#pragma unroll
                            for (int c = 0; c < 4; ++c) acc[c] = {R(0), R(0)};
#pragma unroll 2
                            for (int i = lane; i < M; i += L) {
                                const cplx<R> x = G[(size_t)jz * ldg + i];
                                cplx<R> u[4];
#pragma unroll
                                for (int c = 0; c < 4; ++c) u[c] = G[(size_t)col[c] * ldg + i];
#pragma unroll
                                for (int c = 0; c < 4; ++c) {
                                    acc[c].x = fma(u[c].x, x.x, fma(u[c].y, x.y, acc[c].x));
                                    acc[c].y = fma(u[c].x, x.y, fma(-u[c].y, x.x, acc[c].y));
                                }
                            }
#pragma unroll
                            for (int c = 0; c < 4; ++c) {
                                acc[c].x = group_sum<R, L>(acc[c].x);
                                acc[c].y = group_sum<R, L>(acc[c].y);
                            }
                            if (lane == 0) {
#pragma unroll
                                for (int c = 0; c < 4; ++c)
                                    if (c0 + c < N) s.coef[c0 + c] = use[c] ? acc[c] : cplx<R>{R(0), R(0)};
                            }
                        }
                    }
                    __syncthreads();
                    for (int i = tid; i < M; i += nt) {
                        cplx<R> x = G[(size_t)jz * ldg + i];
                        // eight columns' entries loaded before they are used
                        // (the same updates in the same order)
                        int col = 0;
                        for (; WIDE && col + 8 <= N; col += 8) {
                            cplx<R> u[8];
#pragma unroll
                            for (int c = 0; c < 8; ++c) u[c] = G[(size_t)(col + c) * ldg + i];
#pragma unroll
                            for (int c = 0; c < 8; ++c) {
                                const cplx<R> cf = s.coef[col + c];
                                x.x -= cf.x * u[c].x - cf.y * u[c].y;
                                x.y -= cf.x * u[c].y + cf.y * u[c].x;
                            }
                        }
                        for (; col < N; ++col) {
                            const cplx<R> cf = s.coef[col];
                            const cplx<R> u = G[(size_t)col * ldg + i];
                            x.x -= cf.x * u.x - cf.y * u.y;
                            x.y -= cf.x * u.y + cf.y * u.x;
                        }
                        s.xtmp[i] = x;
                    }
                    __syncthreads();
                    for (int i = tid; i < M; i += nt) G[(size_t)jz * ldg + i] = s.xtmp[i];
                    __syncthreads();
                }
                R nrm = 0;
                for (int i = tid; i < M; i += nt) {
                    const cplx<R> x = G[(size_t)jz * ldg + i];
                    nrm = fma(x.x, x.x, fma(x.y, x.y, nrm));
                }
                nrm = sqrt(block_sum<R>(nrm, s.red));
                if (nrm > thresh) {
                    const R inv = R(1) / nrm;
                    for (int i = tid; i < M; i += nt) {
                        const cplx<R> x = G[(size_t)jz * ldg + i];
                        G[(size_t)jz * ldg + i] = {x.x * inv, x.y * inv};
                    }
                    done = true;
                }
                ++cand;
                ++scanned;
                __syncthreads();
            }
        }
        // write: out[theta][i][c] = G[perm[c]][i]
        cplx<R>* out = (d.transposed ? a.V : a.U) + (size_t)out_idx * M * r;
        cplx<R>* mir = mirror >= 0 ? (d.transposed ? a.V : a.U) + (size_t)mirror * M * r : nullptr;
        for (int e0 = tid; e0 < M * r; e0 += 4 * nt) {
            cplx<R> v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + u * nt;
                if (e < M * r) {
                    const int i = e / r, c = e - (e / r) * r;
                    v[u] = G[(size_t)s.perm[c] * ldg + i];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + u * nt;
                if (e < M * r) {
                    out[e] = v[u];
                    if (mir) mir[e] = {v[u].x, -v[u].y};
                }
            }
        }
    }
    if (a.info) {
        if (tid == 0) {
            atomicAdd(&a.info[LFA_INFO_SUM_SWEEPS], sweeps);
            atomicMax(&a.info[LFA_INFO_MAX_SWEEPS], sweeps);
            atomicAdd(&a.info[LFA_INFO_HIST + min(sweeps, LFA_INFO_HIST_BINS - 1)], 1);
            if (!converged) atomicAdd(&a.info[LFA_INFO_NONCONVERGED], 1);
        }
        if (bad) atomicOr(&a.info[LFA_INFO_NONFINITE], 1);
    }
    __syncthreads();
}

// ---- cross-lane exchanges (gfx950 permlane swaps) ------------------------
// xadd32(a, b): lanes 0-31 receive a(l) + a(l+32), lanes 32-63 b(l-32) + b(l).
// xadd16(a, b): lanes whose bit 4 is clear receive a(l) + a(l+16), the others
// b(l-16) + b(l).  With a == b both give the sum of a lane and its partner.
__device__ __forceinline__ float xadd32(float a, float b) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float xadd16(float a, float b) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ double xadd32(double a, double b) {
    const unsigned long long ua = __double_as_longlong(a), ub = __double_as_longlong(b);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ua, (unsigned)ub, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
    return __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0])) +
           __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}
__device__ __forceinline__ double xadd16(double a, double b) {
    const unsigned long long ua = __double_as_longlong(a), ub = __double_as_longlong(b);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ua, (unsigned)ub, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
    return __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0])) +
           __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}

// v + v(lane ^ OFF)
template <int OFF, typename R>
__device__ __forceinline__ R xsum(R v) {
    if constexpr (OFF == 32) return xadd32(v, v);
    else if constexpr (OFF == 16) return xadd16(v, v);
    else return v + __shfl_xor(v, OFF, 64);
}

// Sum over the lanes l ^ OFF, l ^ 2 OFF, ..., below LIM (xor butterfly).
template <int OFF, int LIM, typename R>
__device__ __forceinline__ R xsum_range(R v) {
    if constexpr (OFF < LIM) return xsum_range<2 * OFF, LIM>(xsum<OFF>(v));
    else return v;
}

// Transpose-add stages on NV values per lane: stage 1 (S1) folds v[i] and
// v[i + NV/2] across lane^32, stage 2 (S2) folds the first half of what is
// left across lane^16.  The result is in v[0 .. NV >> (S1 + S2)).
template <int S1, int S2, typename R, int NV>
__device__ __forceinline__ void transpose_add(R (&v)[NV]) {
    if constexpr (S1 != 0) {
#pragma unroll
        for (int i = 0; i < NV / 2; ++i) v[i] = xadd32(v[i], v[i + NV / 2]);
    }
    if constexpr (S2 != 0) {
        constexpr int H = (NV >> S1) / 2;
#pragma unroll
        for (int i = 0; i < H; ++i) v[i] = xadd16(v[i], v[i + H]);
    }
}

// Column held at register position `pos` during round-robin step `step` of a
// sweep (positions 1..NC-1 rotate by one per step; position 0 is fixed).
template <int NC>
__device__ __forceinline__ int col_at(int pos, int step) {
    if (pos == 0) return 0;
    const int c = pos - 1 - step;
    return 1 + (c < 0 ? c + (NC - 1) : c);
}

// Steps between two foldings of the column scales into the stored columns:
// a column is rotated at most once per step and each rotation multiplies its
// scale by c >= 1/sqrt(2), so stored entries stay within 2^16 of the true ones.
constexpr int kWaveRenorm = 32;

// Round-robin ("circle") move of NC register positions: position 0 stays,
// positions 1..NC-1 rotate by one.
template <int NC, typename T>
__device__ __forceinline__ void rotate_positions(T (&g)[NC]) {
    // new[1] = old[NC-1], new[i] = old[i-1] for i = 2..NC-1
    const T last = g[NC - 1];
#pragma unroll
    for (int i = NC - 1; i >= 2; --i) g[i] = g[i - 1];
    g[1] = last;
}

// Register of round-robin position p, K steps after the registers were last
// moved: K moves by one would have put the value of register reg_of(p) at p.
template <int NC, int K>
__host__ __device__ constexpr int reg_of(int p) {
    return p == 0 ? 0 : 1 + (p - 1 - K % (NC - 1) + (NC - 1)) % (NC - 1);
}

// U moves by one at once: the registers permuted along the cycles of the
// rotation (about NC moves instead of U (NC - 1)).
template <int NC, int U, typename T>
__device__ __forceinline__ void rotate_positions_by(T (&g)[NC]) {
    T old[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) old[i] = g[i];
#pragma unroll
    for (int i = 1; i < NC; ++i) g[i] = old[reg_of<NC, U>(i)];
}

// Cyclic shift of B registers by U: new[k] = old[(k + U) mod B].
template <int B, int U, typename T>
__device__ __forceinline__ void shift_positions_by(T (&g)[B]) {
    T old[B];
#pragma unroll
    for (int i = 0; i < B; ++i) old[i] = g[i];
#pragma unroll
    for (int i = 0; i < B; ++i) g[i] = old[(i + U) % B];
}

// Steps of the register kernel unrolled together (a divisor of the NC - 1
// steps of a sweep): the positions of the unrolled steps are compile-time
// register names, and the registers move once per U steps.
// FP64 with 64 columns stays at one step: its registers are already full.
template <typename R, int NC>
constexpr int wave_unroll() {
    if (sizeof(R) == 8 && NC == 64) return 1;
    // measured: FP32 with 64 columns 3, 7, 9, 21 steps (9 fastest; 21
    // outgrows the instruction cache), with 16 columns 3, 5, 15 (15 fastest)
    if (NC == 64) return 9;
    if (NC == 16) return 15;
    return (NC - 1) % 3 == 0 ? 3 : ((NC - 1) <= 7 ? NC - 1 : 1);
}

// f(integral_constant<int, 0>), ..., f(integral_constant<int, U - 1>)
template <typename F, int... I>
__device__ __forceinline__ void for_steps(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}

// ---------------------------------------------------------------------------
// Blocked one-sided Jacobi for symbols with more than 64 rows.
//
// Thread t of the work-group owns row t of G (M x N, column-major in a global
// slot) and row t of the accumulator Q (N x N): it is the only thread that
// ever reads or writes those rows, so the global traffic of the sweeps needs
// no synchronisation.  Columns are taken B at a time: a block pair (2B columns
// of the thread's row, and of its Q row) sits in registers while its column
// pairs are rotated, then goes back to the slot.
//
// One sweep visits every column pair exactly once:
//  * intra pass: blocks (2i, 2i+1) are loaded together and the pairs inside
//    each block are rotated by a round-robin of B-1 steps;
//  * cross passes: a round-robin over the blocks (NB-1 outer steps); in a
//    block pair (a, b), step t rotates (a_p, b_{(p+t) mod B}) for all p.
//
// One step (B pairs):
//  1. every thread forms its rows' contributions to |g_j|^2, |g_k|^2 and
//     g_j^H g_k for the B pairs; they are folded across the lanes of the wave
//     (lane^32 and lane^16 register swaps, then an LDS transpose) into the
//     wave's sums, which go to a per-wave slot (double-buffered by step);
//  2. one work-group barrier;
//  3. every wave sums the per-wave slots and evaluates the B rotations itself
//     (identical inputs give identical results in every wave), so no second
//     barrier is needed;
//  4. the rotations are applied in scaled form: block columns are held as
//     g_j = G_j / d_j with per-column scales that the rotations multiply by
//     c (two complex multiply-adds per row and pair instead of four
//     real-by-complex products); every wave keeps its own copy of the 2B
//     scales, and they are folded into the columns before the block pair goes
//     back to the slot, so the slot always holds true columns.
// ---------------------------------------------------------------------------
constexpr int kBlk = 16;                  // columns per block
constexpr int kBlkPST = kBlk + 4;         // folded partials per lane (4B / 4) + padding
// Per-wave LDS areas hold up to two block pairs (the dual cross pass):
constexpr int kWsumW = 8 * kBlk;          // floats of sums per wave and parity
constexpr int kPrmW = 2 * kBlk;           // rotation parameters per wave
constexpr int kDscW = 4 * kBlk;           // column scales (and norms) per wave

template <typename R>
struct BlockLds {
    R* wpart;        // [waves][64][kBlkPST] folded partials of each wave
    R* wsum;         // [2][waves][kWsumW] per-wave sums of the step, by step parity
    quad<R>* wprm;   // [waves][kPrmW] rotation parameters (each wave its own)
    R* wdsc;         // [waves][kDscW] column scales of the block pair(s) (each wave its own)
    double* wnrm;    // [waves][kDscW] squared norms of those columns (each wave its own)
    int* rflag;      // rotation made in this sweep
};

template <typename R>
__device__ __forceinline__ BlockLds<R> carve_block(char* lds, size_t off) {
    const int nw = blockDim.x >> 6;
    BlockLds<R> b;
    R* p = reinterpret_cast<R*>(lds + ((off + 63) & ~size_t(63)));
    b.wpart = p;
    p += nw * 64 * kBlkPST;
    b.wsum = p;
    p += 2 * nw * kWsumW;
    b.wprm = reinterpret_cast<quad<R>*>(p);
    p = reinterpret_cast<R*>(b.wprm + nw * kPrmW);
    b.wdsc = p;
    p += nw * kDscW;
    b.wnrm = reinterpret_cast<double*>((reinterpret_cast<size_t>(p) + 7) & ~size_t(7));
    b.rflag = reinterpret_cast<int*>(b.wnrm + nw * kDscW);
    return b;
}

// Partial sums of the step -> the wave's sums in wsum[par][wave][4p .. 4p+3].
// part(p) gives pair p's four sums over the thread's rows.  Groups of four
// pairs (gi, gi+4, gi+8, gi+12) are formed and folded by two register-swap
// stages (lane^32, lane^16): lane l then holds pair gi + 4 (l / 16), summed
// over four rows; the 16 lanes of each quarter are summed through LDS.
template <typename R, typename F>
__device__ __forceinline__ void block_wave_sums(const BlockLds<R>& bl, F part, int par, int off = 0) {
    constexpr int B = kBlk;
    static_assert(B == 16, "the fold below assumes four groups of four pairs");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    R* wp = bl.wpart + wave * 64 * kBlkPST;
#pragma unroll
    for (int gi = 0; gi < 4; ++gi) {
        R v[16];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const quad<R> x = part(gi + 4 * b);
            v[4 * b + 0] = x.a;
            v[4 * b + 1] = x.b;
            v[4 * b + 2] = x.c;
            v[4 * b + 3] = x.d;
        }
        transpose_add<1, 1>(v);
        *reinterpret_cast<quad<R>*>(wp + lane * kBlkPST + 4 * gi) = quad<R>{v[0], v[1], v[2], v[3]};
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // lane l: value l = 4 p + c of pair p = l / 4, held by lanes 16 (p / 4) ..
    // +15 at slot l % 16
    const int blk = lane >> 4, slot = lane & 15;
    R s = 0;
#pragma unroll
    for (int h = 0; h < 16; ++h) s += wp[(blk * 16 + h) * kBlkPST + slot];
    bl.wsum[(par * nw + wave) * kWsumW + off + lane] = s;
}

// The same for the inner products alone (the steps after the first of a
// block pair's visit, whose column norms are carried by the rotations):
// part(p) gives pair p's g_j^H g_k over the thread's rows.  Quad i < B/2
// holds pairs i and i + B/2, so two groups of four quads are folded; the
// wave's sums go to wsum[par][wave][4i .. 4i+3].
template <typename R, typename F>
__device__ __forceinline__ void block_wave_gammas(const BlockLds<R>& bl, F part, int par) {
    constexpr int B = kBlk;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    R* wp = bl.wpart + wave * 64 * kBlkPST;
#pragma unroll
    for (int gi = 0; gi < 2; ++gi) {
        R v[16];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int qi = gi + 2 * b;
            const cplx<R> x = part(qi), y = part(qi + B / 2);
            v[4 * b + 0] = x.x;
            v[4 * b + 1] = x.y;
            v[4 * b + 2] = y.x;
            v[4 * b + 3] = y.y;
        }
        transpose_add<1, 1>(v);
        *reinterpret_cast<quad<R>*>(wp + lane * kBlkPST + 4 * gi) = quad<R>{v[0], v[1], v[2], v[3]};
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // value l = 4 i + c (l < 32) of quad i = gi + 2 b is held by lanes
    // 16 b .. 16 b + 15 at slot 4 gi + c; lanes l and l + 32 sum eight each
    const int l = lane & 31, half = lane >> 5;
    const int qi = l >> 2, gi = qi & 1, b = qi >> 1;
    R s = 0;
#pragma unroll
    for (int h = 0; h < 8; ++h) s += wp[(b * 16 + half * 8 + h) * kBlkPST + 4 * gi + (l & 3)];
    s = xsum<32>(s);
    if (half == 0) bl.wsum[(par * nw + wave) * kWsumW + l] = s;
}

// After the barrier: lanes p < B of every wave sum the per-wave slots of pair
// p, take its rotation in scaled form (scales of its columns cj, ck in the
// wave's copy) and publish it to the wave.  Returns true if this lane's pair
// rotated.  FULL: the slots hold the four sums of block_wave_sums (the first
// step of a visit, which meets every column of the block pair once and sets
// the wave's copy of the squared norms); otherwise they hold the inner
// products of block_wave_gammas and the norms come from that copy, which the
// rotations update.

template <typename R, bool TRACK>
__device__ __forceinline__ bool block_rotations(const BlockLds<R>& bl, int par, int cj, int ck, double tol,
                                                double floor, bool full) {
    constexpr int B = kBlk;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    bool rot = false;
    if (lane < B) {
        R* dsc = bl.wdsc + wave * kDscW;
        double* nrm = bl.wnrm + wave * kDscW;
        R dj = dsc[cj], dk = dsc[ck];
        const double ddj = double(dj), ddk = double(dk);
        double al, be, s2 = 0, s3 = 0;
        if (!TRACK || full) {
            double s0 = 0, s1 = 0;
            for (int w = 0; w < nw; ++w) {
                const quad<R> x =
                    *reinterpret_cast<const quad<R>*>(bl.wsum + (par * nw + w) * kWsumW + 4 * lane);
                s0 += double(x.a);
                s1 += double(x.b);
                s2 += double(x.c);
                s3 += double(x.d);
            }
            al = s0 * ddj * ddj;
            be = s1 * ddk * ddk;
        } else {
            const int off = 4 * (lane & (B / 2 - 1)) + (lane < B / 2 ? 0 : 2);
            for (int w = 0; w < nw; ++w) {
                const R* x = bl.wsum + (par * nw + w) * kWsumW + off;
                s2 += double(x[0]);
                s3 += double(x[1]);
            }
            al = nrm[cj];
            be = nrm[ck];
        }
        quad<R> q;
        // a sweep of small rotations only ends the symbol's sweeps
        rot = rotation_scaled<R>(al, be, s2 * ddj * ddk, s3 * ddj * ddk, tol, floor, dj, dk, q) > 1;
        dsc[cj] = dj;
        dsc[ck] = dk;
        if constexpr (TRACK) {
            nrm[cj] = al;
            nrm[ck] = be;
        }
        bl.wprm[wave * kPrmW + lane] = q;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    return rot;
}

// The dual cross step: two block pairs (sets 0 and 1) at once, 2B pairs.
// Lane l < 2B takes pair p = l mod B of set l / B: columns p of block a and
// (p + t) mod B of block b, at 2B (set) + p and 2B (set) + B + (p + t) mod B
// of the wave's scales and norms.  FULL: the slots hold two block_wave_sums
// results (set s at offset 4B s); otherwise one, whose quad p holds the inner
// products of pair p of set 0 and of set 1.
template <typename R>
__device__ __forceinline__ bool block_rotations_dual(const BlockLds<R>& bl, int par, int t, double tol,
                                                     double floor, bool full) {
    constexpr int B = kBlk;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    bool rot = false;
    if (lane < 2 * B) {
        const int set = lane / B, p = lane & (B - 1);
        const int cj = 2 * B * set + p, ck = 2 * B * set + B + ((p + t) & (B - 1));
        R* dsc = bl.wdsc + wave * kDscW;
        double* nrm = bl.wnrm + wave * kDscW;
        R dj = dsc[cj], dk = dsc[ck];
        const double ddj = double(dj), ddk = double(dk);
        double al, be, s2 = 0, s3 = 0;
        if (full) {
            double s0 = 0, s1 = 0;
            for (int w = 0; w < nw; ++w) {
                const quad<R> x = *reinterpret_cast<const quad<R>*>(bl.wsum + (par * nw + w) * kWsumW +
                                                                     4 * B * set + 4 * p);
                s0 += double(x.a);
                s1 += double(x.b);
                s2 += double(x.c);
                s3 += double(x.d);
            }
            al = s0 * ddj * ddj;
            be = s1 * ddk * ddk;
        } else {
            for (int w = 0; w < nw; ++w) {
                const R* x = bl.wsum + (par * nw + w) * kWsumW + 4 * p + 2 * set;
                s2 += double(x[0]);
                s3 += double(x[1]);
            }
            al = nrm[cj];
            be = nrm[ck];
        }
        quad<R> q;
        rot = rotation_scaled<R>(al, be, s2 * ddj * ddk, s3 * ddj * ddk, tol, floor, dj, dk, q) > 1;
        dsc[cj] = dj;
        dsc[ck] = dk;
        nrm[cj] = al;
        nrm[ck] = be;
        bl.wprm[wave * kPrmW + lane] = q;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    return rot;
}

template <typename R>
__device__ __forceinline__ cplx<R> pair_gamma(cplx<R> x, cplx<R> y) {
    return {fma(x.x, y.x, x.y * y.y), fma(x.x, y.y, -x.y * y.x)};
}

template <typename R>
__device__ __forceinline__ quad<R> pair_partials(cplx<R> x, cplx<R> y) {
    quad<R> q;
    q.a = fma(x.x, x.x, x.y * x.y);
    q.b = fma(y.x, y.x, y.y * y.y);
    q.c = fma(x.x, y.x, x.y * y.y);
    q.d = fma(x.x, y.y, -x.y * y.x);
    return q;
}

// Load / store block `blk` (columns blk*B ..) of this thread's row.
template <typename R>
__device__ __forceinline__ void load_block(const cplx<R>* base, int ld, int blk, int ncols, int row,
                                           bool row_ok, cplx<R> (&x)[kBlk]) {
#pragma unroll
    for (int k = 0; k < kBlk; ++k) {
        const int c = blk * kBlk + k;
        x[k] = (row_ok && c < ncols) ? base[(size_t)c * ld + row] : cplx<R>{R(0), R(0)};
    }
}
template <typename R>
__device__ __forceinline__ void store_block(cplx<R>* base, int ld, int blk, int ncols, int row,
                                            bool row_ok, const cplx<R> (&x)[kBlk]) {
#pragma unroll
    for (int k = 0; k < kBlk; ++k) {
        const int c = blk * kBlk + k;
        if (row_ok && c < ncols) base[(size_t)c * ld + row] = x[k];
    }
}

// Team of W work-groups working on one symbol.  Counters live in device
// memory, cleared before the launch; `target` counts the barriers passed.
struct Team {
    int member, W;
    int32_t* bar;        // arrivals (monotonic)
    int32_t* rot;        // work-groups that rotated, summed over the sweeps (monotonic)
    int32_t* err;        // bit 1 set when a barrier timed out
    int target;
};

// All W work-groups of the team arrive before any leaves; global writes
// before the barrier are visible to every member after it (release/acquire
// at agent scope).  The wait is bounded: on timeout the error bit is set and
// this and every later barrier return at once, so no wave ever hangs.
__device__ void team_barrier(Team& t) {
    t.target += t.W;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        __hip_atomic_fetch_add(t.bar, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        int spins = 0;
        while (__hip_atomic_load(t.bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < t.target) {
            if (__hip_atomic_load(t.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 2) break;
            __builtin_amdgcn_s_sleep(4);
            if (++spins > (1 << 24)) {
                __hip_atomic_fetch_or(t.err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
        __threadfence();
    }
    __syncthreads();
}

// RPT rows per thread: thread t owns rows t, t + nt, ..., t + (RPT-1) nt.
// ACC: the accumulator Q is present (singular vectors wanted).  TRACK: only
// the first step of a block pair's visit forms the column norms; the later
// ones form the inner products alone and take the norms the rotations carry
// (FP32 without the accumulator; see block_one).
template <typename R, int RPT, bool ACC, bool TRACK, bool DUAL = false>
__device__ __forceinline__ void block_sweeps(const LayerDesc& d, const Shared<R>& s, const BlockLds<R>& bl,
                             int max_sweeps, double tol, Team& team, int& sweeps_out,
                             bool& conv_out) {
    constexpr int B = kBlk;
    // steps unrolled together in the intra passes (B - 1 steps) and the
    // cross passes (B steps); with the accumulator, larger blocks of steps
    // spill registers (measured: 3 and 4 made the 512 x 256 layer with
    // vectors 1.7x slower, 1 and 2 made it 3 % faster); without it, 5 and 8
    // measured 2 % faster than 3 and 4 (15 and 4: no gain); FP64 keeps one
    // step
    constexpr bool F64 = sizeof(R) == 8;
    constexpr int KI = (ACC || F64) ? 1 : 5, KC = F64 ? 1 : (ACC ? 2 : 8);
    static_assert(!TRACK || (!ACC && !F64), "norm tracking: FP32 without the accumulator");
    static_assert(!DUAL || (TRACK && RPT == 1), "dual cross steps: tracked norms, one row per thread");
    static_assert((B - 1) % KI == 0 && B % KC == 0, "unrolled steps must divide a pass");
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int member = team.member, W = team.W;
    const int M = d.M, N = d.N;
    const int NB = (N + B - 1) / B, NBP = NB + (NB & 1);
    constexpr bool acc = ACC;
    int rows[RPT];
    bool grow[RPT], qrow[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        rows[r] = tid + r * nt;
        grow[r] = rows[r] < M;
        qrow[r] = acc && rows[r] < N;
    }
    cplx<R> ga[RPT][B], gb[RPT][B], va[ACC ? RPT : 1][ACC ? B : 1], vb[ACC ? RPT : 1][ACC ? B : 1];
    R* dsc = bl.wdsc + wave * kDscW;
    int par = 0;                 // step parity (per-wave sums buffer)
    // block pair in: unit scales (this wave's copy)
    auto load2 = [&](int ba, int bb) {
        if (lane < 2 * B) dsc[lane] = R(1);
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            load_block(s.G, d.ldg, ba, N, rows[r], grow[r], ga[r]);
            load_block(s.G, d.ldg, bb, N, rows[r], grow[r], gb[r]);
            if constexpr (ACC) {
                load_block(s.Q, d.ldv, ba, N, rows[r], qrow[r], va[r]);
                load_block(s.Q, d.ldv, bb, N, rows[r], qrow[r], vb[r]);
            }
        }
    };
    // block pair out: fold the scales (positions are the identity again)
    auto store2 = [&](int ba, int bb) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const R fa = dsc[k], fb = dsc[B + k];
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                ga[r][k] = {ga[r][k].x * fa, ga[r][k].y * fa};
                gb[r][k] = {gb[r][k].x * fb, gb[r][k].y * fb};
                if constexpr (ACC) {
                    va[r][k] = {va[r][k].x * fa, va[r][k].y * fa};
                    vb[r][k] = {vb[r][k].x * fb, vb[r][k].y * fb};
                }
            }
        }
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            store_block(s.G, d.ldg, ba, N, rows[r], grow[r], ga[r]);
            store_block(s.G, d.ldg, bb, N, rows[r], grow[r], gb[r]);
            if constexpr (ACC) {
                store_block(s.Q, d.ldv, ba, N, rows[r], qrow[r], va[r]);
                store_block(s.Q, d.ldv, bb, N, rows[r], qrow[r], vb[r]);
            }
        }
    };
    // numerically zero columns (see negligible_sq): ||G||_F^2 of the symbol
    // in the slot, the same value in every member of the team
    double floor;
    {
        R fro = 0;
        for (int c = 0; c < N; ++c)
#pragma unroll
            for (int r = 0; r < RPT; ++r)
                if (grow[r]) {
                    const cplx<R> v = s.G[(size_t)c * d.ldg + rows[r]];
                    fro = fma(v.x, v.x, fma(v.y, v.y, fro));
                }
        floor = negligible_sq<R>() * double(block_sum<R>(fro, s.red));
    }
    int sweeps = 0;
    bool converged = (N < 2);
    while (!converged && sweeps < max_sweeps) {
        if (tid == 0) *bl.rflag = 0;
        __syncthreads();
        // team: rotations counted before this sweep (all earlier increments
        // happened before the barrier that ended the previous sweep)
        const int rot_before =
            W > 1 ? __hip_atomic_load(team.rot, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) : 0;
        bool rotated = false;
        // ---- intra pass: pairs inside blocks 2i and 2i+1
        for (int i = member; 2 * i < NB; i += W) {
            const int ba = 2 * i, bb = 2 * i + 1;
            load2(ba, bb);
            // KI round-robin steps at a time: position x of step step0 + K is
            // register reg_of<B, K>(x); the registers move once per KI steps
            for (int step0 = 0; step0 < B - 1; step0 += KI) {
              for_steps([&](auto kc) __attribute__((always_inline)) {
                constexpr int K = decltype(kc)::value;
                const int step = step0 + K;
                // pair p < B/2: positions (p, B-1-p) of block a, else of block b;
                // the first step meets every column once and sets the norms
                const bool full = !TRACK || (K == 0 && step0 == 0);
                if (full) {
                    block_wave_sums<R>(bl, [&](int p) {
                        quad<R> q = {R(0), R(0), R(0), R(0)};
#pragma unroll
                        for (int r = 0; r < RPT; ++r) {
                            const quad<R> x =
                                p < B / 2 ? pair_partials(ga[r][reg_of<B, K>(p)], ga[r][reg_of<B, K>(B - 1 - p)])
                                          : pair_partials(gb[r][reg_of<B, K>(p - B / 2)],
                                                          gb[r][reg_of<B, K>(B - 1 - (p - B / 2))]);
                            q = {q.a + x.a, q.b + x.b, q.c + x.c, q.d + x.d};
                        }
                        return q;
                    }, par);
                } else if constexpr (TRACK) {
                    block_wave_gammas<R>(bl, [&](int p) {
                        cplx<R> q = {R(0), R(0)};
#pragma unroll
                        for (int r = 0; r < RPT; ++r) {
                            const cplx<R> x =
                                p < B / 2 ? pair_gamma(ga[r][reg_of<B, K>(p)], ga[r][reg_of<B, K>(B - 1 - p)])
                                          : pair_gamma(gb[r][reg_of<B, K>(p - B / 2)],
                                                       gb[r][reg_of<B, K>(B - 1 - (p - B / 2))]);
                            q = {q.x + x.x, q.y + x.y};
                        }
                        return q;
                    }, par);
                }
                __syncthreads();
                {
                    // columns of pair `lane` (lanes >= B compute nothing)
                    const int pp = lane < B / 2 ? lane : lane - B / 2, off = lane < B / 2 ? 0 : B;
                    const int cj = off + col_at<B>(pp, step), ck = off + col_at<B>(B - 1 - pp, step);
                    rotated |= block_rotations<R, TRACK>(bl, par, cj, ck, tol, floor, full);
                }
                par ^= 1;
                const quad<R>* prm = bl.wprm + wave * kPrmW;
#pragma unroll
                for (int p = 0; p < B / 2; ++p) {
                    const quad<R> ra = prm[p], rb = prm[B / 2 + p];
                    const int j = reg_of<B, K>(p), k = reg_of<B, K>(B - 1 - p);
#pragma unroll
                    for (int r = 0; r < RPT; ++r) {
                        rot_apply_scaled(ga[r][j], ga[r][k], ra.a, ra.b, ra.c, ra.d);
                        rot_apply_scaled(gb[r][j], gb[r][k], rb.a, rb.b, rb.c, rb.d);
                        if constexpr (ACC) {
                            rot_apply_scaled(va[r][j], va[r][k], ra.a, ra.b, ra.c, ra.d);
                            rot_apply_scaled(vb[r][j], vb[r][k], rb.a, rb.b, rb.c, rb.d);
                        }
                    }
                }
              }, std::make_integer_sequence<int, KI>{});
              // round-robin: positions 1..B-1 move by KI
#pragma unroll
              for (int r = 0; r < RPT; ++r) {
                  rotate_positions_by<B, KI>(ga[r]);
                  rotate_positions_by<B, KI>(gb[r]);
                  if constexpr (ACC) {
                      rotate_positions_by<B, KI>(va[r]);
                      rotate_positions_by<B, KI>(vb[r]);
                  }
              }
            }
            // B-1 steps bring every position back: store in place
            store2(ba, bb);
        }
        if (W > 1) team_barrier(team);
        // ---- cross passes: round-robin over block pairs
        if constexpr (DUAL) {
            // Two block pairs of the outer step at once: each step forms the
            // 2B inner products of both, folds them in one pass, takes one
            // work-group barrier and evaluates all 2B rotations, so the fixed
            // cost of a step (folds, barrier, the FP64 rotation parameters)
            // is shared by twice the work.  A missing second pair is zeros
            // (no rotation) and is not stored.
            constexpr int K2 = 8;
            for (int os = 0; os < NBP - 1; ++os) {
                for (int bp = member; bp < NBP / 2; bp += 2 * W) {
                    int ba0, bb0, ba1 = NB, bb1 = NB;
                    rr_pair(bp, os, NBP, ba0, bb0);
                    if (bp + W < NBP / 2) rr_pair(bp + W, os, NBP, ba1, bb1);
                    bool has0 = ba0 < NB && bb0 < NB, has1 = ba1 < NB && bb1 < NB;
                    if (!has0) {
                        ba0 = ba1;
                        bb0 = bb1;
                        has0 = has1;
                        has1 = false;
                    }
                    if (!has0) continue;
                    cplx<R> ga2[2][B], gb2[2][B];
                    if (lane < 2 * kBlk * 2) dsc[lane] = R(1);
                    load_block(s.G, d.ldg, ba0, N, rows[0], grow[0], ga2[0]);
                    load_block(s.G, d.ldg, bb0, N, rows[0], grow[0], gb2[0]);
                    load_block(s.G, d.ldg, ba1, N, rows[0], grow[0] && has1, ga2[1]);
                    load_block(s.G, d.ldg, bb1, N, rows[0], grow[0] && has1, gb2[1]);
                    for (int t0 = 0; t0 < B; t0 += K2) {
                      for_steps([&](auto kc) __attribute__((always_inline)) {
                        constexpr int K = decltype(kc)::value;
                        const int t = t0 + K;
                        const bool full = (K == 0 && t0 == 0);
                        if (full) {
#pragma unroll
                            for (int st = 0; st < 2; ++st)
                                block_wave_sums<R>(bl, [&](int p) {
                                    return pair_partials(ga2[st][p], gb2[st][(p + K) % B]);
                                }, par, 4 * B * st);
                        } else {
                            block_wave_sums<R>(bl, [&](int p) {
                                const cplx<R> x = pair_gamma(ga2[0][p], gb2[0][(p + K) % B]);
                                const cplx<R> y = pair_gamma(ga2[1][p], gb2[1][(p + K) % B]);
                                return quad<R>{x.x, x.y, y.x, y.y};
                            }, par);
                        }
                        __syncthreads();
                        rotated |= block_rotations_dual<R>(bl, par, t, tol, floor, full);
                        par ^= 1;
                        const quad<R>* prm = bl.wprm + wave * kPrmW;
                        // parameters read in groups of 8 pairs, so that the
                        // compiler does not hold all 2B of them at once
#pragma unroll
                        for (int st = 0; st < 2; ++st)
#pragma unroll
                            for (int p0 = 0; p0 < B; p0 += 8) {
#pragma unroll
                                for (int p = p0; p < p0 + 8; ++p) {
                                    const quad<R> rr = prm[B * st + p];
                                    rot_apply_scaled(ga2[st][p], gb2[st][(p + K) % B], rr.a, rr.b, rr.c, rr.d);
                                }
                                __builtin_amdgcn_sched_barrier(0);
                            }
                      }, std::make_integer_sequence<int, K2>{});
                      shift_positions_by<B, K2>(gb2[0]);
                      shift_positions_by<B, K2>(gb2[1]);
                    }
                    // fold the scales and store (block b is back in order)
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
#pragma unroll
                    for (int st = 0; st < 2; ++st)
#pragma unroll
                        for (int k = 0; k < B; ++k) {
                            const R fa = dsc[2 * B * st + k], fb = dsc[2 * B * st + B + k];
                            ga2[st][k] = {ga2[st][k].x * fa, ga2[st][k].y * fa};
                            gb2[st][k] = {gb2[st][k].x * fb, gb2[st][k].y * fb};
                        }
                    store_block(s.G, d.ldg, ba0, N, rows[0], grow[0], ga2[0]);
                    store_block(s.G, d.ldg, bb0, N, rows[0], grow[0], gb2[0]);
                    store_block(s.G, d.ldg, ba1, N, rows[0], grow[0] && has1, ga2[1]);
                    store_block(s.G, d.ldg, bb1, N, rows[0], grow[0] && has1, gb2[1]);
                }
                if (W > 1 && os < NBP - 2) team_barrier(team);
            }
        } else
        for (int os = 0; os < NBP - 1; ++os) {
            for (int bp = member; bp < NBP / 2; bp += W) {
                int ba, bb;
                rr_pair(bp, os, NBP, ba, bb);
                if (ba >= NB || bb >= NB) continue;
                load2(ba, bb);
                // KC steps at a time: at step t0 + K, column p of block a
                // meets register (p + K) mod B of block b; block b's
                // registers shift once per KC steps
                for (int t0 = 0; t0 < B; t0 += KC) {
                  for_steps([&](auto kc) __attribute__((always_inline)) {
                    constexpr int K = decltype(kc)::value;
                    const int t = t0 + K;
                    // the first step meets every column once and sets the norms
                    const bool full = !TRACK || (K == 0 && t0 == 0);
                    if (full) {
                        block_wave_sums<R>(bl, [&](int p) {
                            quad<R> q = {R(0), R(0), R(0), R(0)};
#pragma unroll
                            for (int r = 0; r < RPT; ++r) {
                                const quad<R> x = pair_partials(ga[r][p], gb[r][(p + K) % B]);
                                q = {q.a + x.a, q.b + x.b, q.c + x.c, q.d + x.d};
                            }
                            return q;
                        }, par);
                    } else if constexpr (TRACK) {
                        block_wave_gammas<R>(bl, [&](int p) {
                            cplx<R> q = {R(0), R(0)};
#pragma unroll
                            for (int r = 0; r < RPT; ++r) {
                                const cplx<R> x = pair_gamma(ga[r][p], gb[r][(p + K) % B]);
                                q = {q.x + x.x, q.y + x.y};
                            }
                            return q;
                        }, par);
                    }
                    __syncthreads();
                    {
                        const int cj = lane < B ? lane : 0;
                        const int ck = B + ((cj + t) & (B - 1));
                        rotated |= block_rotations<R, TRACK>(bl, par, cj, ck, tol, floor, full);
                    }
                    par ^= 1;
                    const quad<R>* prm = bl.wprm + wave * kPrmW;
#pragma unroll
                    for (int p = 0; p < B; ++p) {
                        const quad<R> rr = prm[p];
#pragma unroll
                        for (int r = 0; r < RPT; ++r) {
                            rot_apply_scaled(ga[r][p], gb[r][(p + K) % B], rr.a, rr.b, rr.c, rr.d);
                            if constexpr (ACC)
                                rot_apply_scaled(va[r][p], vb[r][(p + K) % B], rr.a, rr.b, rr.c, rr.d);
                        }
                    }
                  }, std::make_integer_sequence<int, KC>{});
                  // block b shifts by KC against block a
#pragma unroll
                  for (int r = 0; r < RPT; ++r) {
                      shift_positions_by<B, KC>(gb[r]);
                      if constexpr (ACC) shift_positions_by<B, KC>(vb[r]);
                  }
                }
                // B shifts bring block b back to its order
                store2(ba, bb);
            }
            if (W > 1 && os < NBP - 2) team_barrier(team);
        }
        // every wave computed the same rotations: wave 0 reports them
        if (wave == 0 && __any(rotated)) {
            if (lane == 0) *bl.rflag = 1;
        }
        __syncthreads();
        if (W > 1) {
            if (tid == 0 && *bl.rflag)
                __hip_atomic_fetch_add(team.rot, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            team_barrier(team);
            converged = __hip_atomic_load(team.rot, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) ==
                        rot_before;
        } else {
            converged = (*bl.rflag == 0);
        }
        ++sweeps;
        __syncthreads();
    }
    sweeps_out = sweeps;
    conv_out = converged;
}

// TRACK (block_sweeps): FP32 without the accumulator.  It makes the
// sigma-only 256 x 256 factors 10 % faster and the persistent launch of the
// ResNet-18 gradient 7 %; with the accumulator, or in FP64, the second form
// of the step in the same unrolled body spilled registers (the 512 x 256
// layer with vectors ran 1.5x slower).
// Always inlined: as a called function its arguments (the layer
// description in particular) are read through memory in the loops instead of
// from scalar registers, which measured 10 % slower in the persistent kernel.
// DUAL: two block pairs per cross step (launches without teams, W = 1).
template <typename R, int RPT, bool ACC, bool TRACK = false, bool DUAL = false, bool WIDE = true>
__device__ __forceinline__ void block_one(const SvdArgs<R>& a, char* lds, int item, char* gslot, Team& team) {
    // ACC must match the arguments: the right singular vectors (left when
    // transposed) are wanted exactly when the accumulator is kept
    bool cj;
    // a pick whose symbol an earlier pick has: every member of the team
    // skips it alike
    if (a.theta_dedup && pick_rep(a.theta_list, item, a.d.n, a.d.m, cj) != item) return;
    const Target tg = target_of(a, item);
    const Shared<R> s = carve<R>(lds, a.d, ACC, gslot);
    const BlockLds<R> bl = carve_block<R>(lds, s.small_end);
    if (team.member == 0) load_symbol<R, !ACC>(a, s, tg.theta);
    if (team.W > 1) team_barrier(team);
    else __syncthreads();
    int sweeps;
    bool converged;
    block_sweeps<R, RPT, ACC, TRACK, DUAL>(a.d, s, bl, a.max_sweeps, a.tol, team, sweeps, converged);
    if (team.member == 0) finish<R, 64, WIDE>(a, s, tg.out, tg.mirror, sweeps, converged);
    // the slot is reused for the team's next symbol: members wait for the finish
    if (team.W > 1) team_barrier(team);
    if (a.info && threadIdx.x == 0 && team.member == 0 &&
        (__hip_atomic_load(team.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 2))
        atomicOr(&a.info[LFA_INFO_NONFINITE], 2);
}


// ===================== register (rows-in-lanes) kernel =====================
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
//  1. every G lane forms its row's contributions to gamma_p = g_j^H g_k for
//     all pairs.  Groups of NB pairs are folded across lanes by transpose-add
//     stages (lane^32 and lane^16 register swaps): after them a lane holds
//     one pair's partial sum over NB rows, and the lanes of block b = row /
//     GL hold the pairs b*Q .. b*Q+Q-1.  The folded partials go to LDS,
//     [symbol][row][2Q] (padded row stride);
//  2. lane (p, k) of the same wave sums Q holder rows of pair p, the LP
//     lanes of a pair are combined with xor exchanges, and every lane of the
//     pair evaluates the rotation (threshold test and angle in double
//     precision) from gamma_p and the squared norms alpha = |g_j|^2,
//     beta = |g_k|^2.  The norms are not summed again each step: they are
//     computed exactly at the start of every sweep and updated with each
//     rotation (alpha - t|gamma|, beta + t|gamma|), so the convergence test
//     of the final, rotation-free sweep uses exact norms.  One lane of the
//     pair's set writes (c, s e^{-i phi}, flag) to a double-buffered LDS
//     slot;
//  3. after one work-group barrier every lane of both waves reads the
//     parameters (broadcast) and applies the pair rotations to its registers
//     (a pair below the threshold gets the identity, applied without a
//     branch).  The Q wave only applies, so it runs a step behind the G wave and its work
//     overlaps the next step's inner products.
// One work-group barrier per step; no LDS traffic for G or Q themselves.  The
// symbols are assembled into registers through a small LDS tile, a chunk of
// columns at a time, and the results are written from registers.


template <typename R>
__device__ __forceinline__ R skey(R v) {
    return v == v ? v : R(-1);
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

constexpr int pow2_floor(int x) {
    int p = 1;
    while (2 * p <= x) p *= 2;
    return p;
}

template <int NC, int ML>
struct WaveShape {
    static constexpr int SPW = 64 / ML;                               // symbols per wave
    static constexpr int NP = NC / 2;                                 // pairs per step
    static constexpr int S1 = (ML == 64 && NP >= 2) ? 1 : 0;          // lane^32 stage
    static constexpr int S2 = (ML >= 32 && NP >= (2 << S1)) ? 1 : 0;  // lane^16 stage
    static constexpr int NB = 1 << (S1 + S2);                         // pairs folded per group
    static constexpr int Q = NP / NB;                                 // groups = pairs per block
    static constexpr int VPL = 2 * Q;                                 // partials per lane in LDS
    static constexpr int GL = ML / NB;                                // lanes holding one block
    static constexpr int LP = ML / NP;                                // lanes summing one pair
    static constexpr int PST = VPL + 2;                               // LDS row stride, padded
    // column norms at the end: the same stages on NC values
    static constexpr int S1N = (ML == 64) ? 1 : 0;
    static constexpr int S2N = (ML >= 32 && (NC >> S1N) >= 2) ? 1 : 0;
    static constexpr int VPLN = NC >> (S1N + S2N);
    static constexpr int GLN = ML >> (S1N + S2N);
    // columns per chunk of the load tile (complex, inside the partial region)
    static constexpr int NCH = pow2_floor(PST / 2) < NC ? pow2_floor(PST / 2) : NC;
    static_assert(VPLN <= PST, "norm partials must fit a partial row");
    static_assert(LP * Q == GL, "reduction lanes must cover a block");
};

// Elements (of R) of the partial region (it also holds the load tile), then
// the phase table.
template <typename R, int NC, int ML>
constexpr int wave_part_elems() {
    using S = WaveShape<NC, ML>;
    return S::SPW * ML * S::PST + S::SPW * kMaxTaps * 2;
}

template <typename R, int NC, int ML>
__host__ __device__ constexpr size_t wave_lds_bytes() {
    using S = WaveShape<NC, ML>;
    const size_t part = (size_t)wave_part_elems<R, NC, ML>() * sizeof(R);
    const size_t prm = 2 * (size_t)S::SPW * S::NP * 4 * sizeof(R);   // double-buffered
    const size_t small = (size_t)S::SPW * NC * (sizeof(double) + 3 * sizeof(R) + 2 * sizeof(int)) +
                         (size_t)S::SPW * 2 * sizeof(int);
    return part + prm + small + 64;
}

// Output staging of launches with singular vectors, after the other LDS
// arrays: chunks of up to 32 rows (padded by one element) per symbol.
template <int ML>
__host__ __device__ constexpr int wave_stage_rows() { return ML < 32 ? ML : 32; }

template <typename R, int NC, int ML>
__host__ __device__ constexpr size_t wave_stage_bytes() {
    return (size_t)(64 / ML) * wave_stage_rows<ML>() * (NC + 1) * sizeof(cplx<R>) + 64;
}

// Synchronisation of the threads working on one group of symbols: the whole
// work-group, or a single wave ("solo": a wave of a larger work-group that
// works alone; its LDS operations complete in order).
__device__ __forceinline__ void wsync(bool solo) {
    if (solo) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    } else {
        __syncthreads();
    }
}

// Squared column norms of the G rows held by one wave: |g_j|^2 folded across
// lanes into the partial region; after the wave's LDS writes are complete,
// column_norm() sums the holder rows of column j (lanes with row < NC).
template <typename R, int NC, int ML>
__device__ __forceinline__ void fold_column_norms(const cplx<R> (&g)[NC], R* part, int sym, int row) {
    using S = WaveShape<NC, ML>;
    R nv[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j) nv[j] = fma(g[j].x, g[j].x, g[j].y * g[j].y);
    transpose_add<S::S1N, S::S2N>(nv);
#pragma unroll
    for (int i = 0; i < S::VPLN; ++i) part[(sym * ML + row) * S::PST + i] = nv[i];
}

template <typename R, int NC, int ML>
__device__ __forceinline__ R column_norm(const R* part, int sym, int j) {
    using S = WaveShape<NC, ML>;
    const int b = j / S::VPLN, slot = j - (j / S::VPLN) * S::VPLN;
    R s = 0;
#pragma unroll 4
    for (int h = 0; h < S::GLN; ++h) s += part[(sym * ML + b * S::GLN + h) * S::PST + slot];
    return s;
}

// Writes the rows of one output matrix per symbol, [rows][N] row-major (row
// r held by lane r of the symbol's ML lanes; column j of the registers goes
// to output column rank[j]), with coalesced stores: chunks of rows are copied
// into LDS in register order, and the lanes write them back in memory order,
// output column c taken from register column inv[c] (inv = rank^-1), whole
// cache lines per instruction instead of one element of each of 64 rows.
// Every lane of the wave calls it; out / mir may be null (inactive symbol,
// no mirror).
template <typename R, int NC, int ML>
__device__ void store_rows(cplx<R>* out, cplx<R>* mir, int rows, int N, const int* inv,
                           const cplx<R> (&g)[NC], cplx<R>* stage, int sym, int row) {
    constexpr int LD = NC + 1, RC = wave_stage_rows<ML>();   // padded row, rows per chunk
    cplx<R>* st = stage + sym * RC * LD;                       // this symbol's chunk [RC][LD]
    for (int c0 = 0; c0 < rows; c0 += RC) {
        const int r = row - c0;
        if (r >= 0 && r < RC) {
#pragma unroll
            for (int j = 0; j < NC; ++j) st[r * LD + j] = g[j];
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const int nrow = min(RC, rows - c0);
        for (int e = row; e < nrow * N; e += ML) {
            const int rr = e / N, cc = e - (e / N) * N;
            const cplx<R> v = st[rr * LD + inv[cc]];
            const size_t at = (size_t)(c0 + rr) * N + cc;
            if (out) out[at] = v;
            if (mir) mir[at] = {v.x, -v.y};
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// A resumable run of a wave group (work-queue launch): the group's saved
// state is its G and Q rows after a whole number of sweeps, with the column
// scales folded in, plus the sweep count and per-symbol convergence sweep.
//   state : [waves][NC/2][64 lanes] column pairs (quad = two complex values),
//           so one load or store instruction moves 64 consecutive pairs
//   meta  : [0] sweeps done, [1 + s] sweep at which symbol s converged (0: not)
//   first : no saved state yet (assemble G, Q = I)
//   budget: sweeps to run before the state is saved again
template <typename R>
struct WaveSeg {
    quad<R>* state;
    int* meta;
    int first;
    int budget;
};

// One group of SPW symbols (items base .. base+SPW-1) by `nthr` threads with
// index `tid`: 64 (G only) or 128 (G wave + Q wave, not solo).  With SEG the
// group runs at most seg.budget sweeps from its saved state; it returns true
// when the group is finished (outputs written), false when its state was
// saved for a later run.  The arithmetic is the same as one uninterrupted
// run: results are bitwise identical.
template <typename R, int NC, int ML, bool SEG = false>
__device__ bool wave_group(const SvdArgs<R>& a, char* lds_raw, int base, int tid, int nthr,
                           bool solo, const WaveSeg<R>& seg = WaveSeg<R>{nullptr, nullptr, 1, 0}) {
    using S = WaveShape<NC, ML>;
    constexpr int SPW = S::SPW, NP = S::NP, NB = S::NB, Q = S::Q, GL = S::GL, PST = S::PST;
    constexpr int NCH = S::NCH;
    R* part = reinterpret_cast<R*>(lds_raw);                       // [SPW][ML][PST]
    quad<R>* prm = reinterpret_cast<quad<R>*>(part + wave_part_elems<R, NC, ML>());   // [2][SPW][NP]
    double* nrm = reinterpret_cast<double*>(prm + 2 * SPW * NP);    // [SPW][NC] |G_j|^2 (tracked)
    R* dsc = reinterpret_cast<R*>(nrm + SPW * NC);                  // [2][SPW][NC] column scales
    R* sigs = dsc + 2 * SPW * NC;                                   // [SPW][NC]
    int* rankof = reinterpret_cast<int*>(sigs + SPW * NC);          // [SPW][NC]
    int* nzero = rankof + SPW * NC;                                 // [SPW] zero columns
    int* flags = nzero + SPW;                                       // [SPW] rotated this sweep
    int* colof = flags + SPW;                                       // [SPW][NC] rank -> column
    // output staging (launches with vectors only): after everything else
    cplx<R>* stage = reinterpret_cast<cplx<R>*>(
        reinterpret_cast<char*>(lds_raw) + ((wave_lds_bytes<R, NC, ML>() + 63) & ~size_t(63)));

    const LayerDesc& d = a.d;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // 0: G rows, 1: Q rows
    const int sym = lane / ML, row = lane - (lane / ML) * ML;
    const int M = d.M, N = d.N;
    const int count = item_count(a);
    const int T = d.kh * d.kw;
    const double tol = a.tol;

    const int item = base + sym;
    const bool active = item < count;
    const Target tg = active ? target_of(a, item) : Target{0, 0, -1};

    // ---------------------------------------------------------------- load
    // The work-group assembles (or copies) the symbols of the wave into an LDS
    // tile in G layout, [s][row][col], NCH columns at a time, zero outside
    // M x N: G = A (row o, column i), or G = A^H (row i, column o) when
    // c_out < c_in.  Every G lane then loads its row with constant offsets.
    cplx<R>* tile = reinterpret_cast<cplx<R>*>(part);        // [SPW][ML][NCH]
    cplx<R>* ph = reinterpret_cast<cplx<R>*>(part + SPW * ML * PST);   // [SPW][T]
    cplx<R> g[NC];
    const bool fresh = !SEG || seg.first;
    // optional phase record (thread 0): load, sweeps, finish, save
    unsigned long long* const phase = a.phase;
    unsigned long long t_mark = (phase && tid == 0) ? wall_clock64() : 0;
    auto phase_add = [&](int k) {
        if (phase && tid == 0) {
            const unsigned long long t = wall_clock64();
            atomicAdd(&phase[k], t - t_mark);
            t_mark = t;
        }
    };
    if (!fresh) {
        // saved rows of this wave (written by another work-group, made
        // visible by the queue's release/acquire)
        const quad<R>* src = seg.state + (size_t)wave * (NC / 2) * 64 + lane;
#pragma unroll
        for (int jp = 0; jp < NC / 2; ++jp) {
            const quad<R> v = src[jp * 64];
            g[2 * jp] = {v.a, v.b};
            g[2 * jp + 1] = {v.c, v.d};
        }
    }
    if (fresh && a.A == nullptr) {
        for (int x = tid; x < SPW * T; x += nthr) {
            const int s = x / T, t = x - (x / T) * T;
            const int it = base + s;
            double re = 1.0, im = 0.0;
            if (it < count) phase_of(a.tw, d, target_of(a, it).theta, t, re, im);
            ph[x] = {R(re), R(im)};
        }
        wsync(solo);
    }
#pragma unroll
    for (int c0 = 0; c0 < (fresh ? NC : 0); c0 += NCH) {
        for (int x = tid; x < SPW * ML * NCH; x += nthr) {
            const int s = x / (ML * NCH), rc = x - s * (ML * NCH);
            const int r = rc / NCH, c = c0 + (rc - (rc / NCH) * NCH);
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
        wsync(solo);
#pragma unroll
        for (int jj = 0; jj < NCH; ++jj) g[c0 + jj] = tile[(sym * ML + row) * NCH + jj];
        wsync(solo);
    }
    if (fresh && wave == 1) {
        // accumulator rows: Q = I (N x N), zero beyond N
#pragma unroll
        for (int j = 0; j < NC; ++j) g[j] = {R((row == j && j < N) ? 1 : 0), R(0)};
    }
    // Columns of G and of Q are stored scaled: true column = stored * d_j
    // (the same d_j for G and Q).  A sweep runs in segments of SEGL (about
    // kWaveRenorm) steps; at the start of a segment both waves fold the scales of the
    // previous segment into their stored columns and the rotations of the
    // segment update the other buffer, so the Q wave (a step behind) never
    // reads a scale the G wave is changing.  Both buffers start at 1.
    if (wave == 0 && row < NC) {
        dsc[sym * NC + row] = R(1);
        dsc[SPW * NC + sym * NC + row] = R(1);
    }
    // the Q wave reads the scales at the first segment start
    wsync(solo);
    phase_add(0);
    int cur = 0;                // scale buffer of the current segment

    // -------------------------------------------------------------- sweeps
    // (uniform over the work-group: the loop bounds below stay scalar)
    int sweeps = fresh ? 0
                       : __builtin_amdgcn_readfirstlane(
                             __hip_atomic_load(&seg.meta[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    // sweeps used by this lane's symbol
    int conv_at = fresh ? 0 : __hip_atomic_load(&seg.meta[1 + sym], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    bool my_conv = conv_at > 0;                    // symbol of this lane converged
    int buf = 0;                // parameter buffer of the current step
    // U steps at a time (compile-time register names), segments of whole
    // blocks of U steps
    constexpr int U = wave_unroll<R, NC>();
    constexpr int SEGL = U * ((kWaveRenorm + U - 1) / U);
    static_assert((NC - 1) % U == 0, "unrolled steps must divide a sweep");
    const int sw_end = SEG ? min(a.max_sweeps, sweeps + seg.budget) : a.max_sweeps;
    bool all = false;
    for (int sw = sweeps; sw < sw_end; ++sw) {
        if (tid < SPW) flags[tid] = 0;
        bool rotated = false;
        for (int seg0 = 0; seg0 < NC - 1; seg0 += SEGL) {
            // segment start: fold the previous segment's scales (positions
            // of step seg0) into G and Q, start the new scales at 1
            const R* dprev = dsc + cur * (SPW * NC);
            cur ^= 1;
            R* dcur = dsc + cur * (SPW * NC);
#pragma unroll
            for (int pos = 0; pos < NC; ++pos) {
                const R f = dprev[sym * NC + col_at<NC>(pos, seg0)];
                g[pos] = {g[pos].x * f, g[pos].y * f};
            }
            if (wave == 0) {
                if (row < NC) dcur[sym * NC + row] = R(1);
                if (seg0 == 0) {
                    // exact squared column norms at the start of every
                    // sweep; the steps update them with each rotation
                    fold_column_norms<R, NC, ML>(g, part, sym, row);
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    // numerically zero columns (see negligible_sq; the
                    // symbol's ||G||_F^2 is the sum over its lanes) start the
                    // sweep with tracked norm 0, which keeps them out of
                    // every rotation of the sweep (floor 0 below)
                    const double cn = row < NC ? double(column_norm<R, NC, ML>(part, sym, row)) : 0.0;
                    const double fl = negligible_sq<R>() * xsum_range<1, ML>(cn);
                    if (row < NC) nrm[sym * NC + row] = cn > fl ? cn : 0.0;
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
            const int seg1 = seg0 + SEGL < NC - 1 ? seg0 + SEGL : NC - 1;
            for (int step0 = seg0; step0 < seg1; step0 += U) {
              for_steps([&](auto kc) __attribute__((always_inline)) {
                // step step0 + K of the sweep; position x is in register
                // reg_of<NC, K>(x)
                constexpr int K = decltype(kc)::value;
                const int step = step0 + K;
                quad<R>* prm_b = prm + buf * (SPW * NP);
                if (wave == 0) {
                    // 1. partial inner products gamma_p = g_j^H g_k (stored
                    //    columns), folded across lanes by groups of NB pairs
                    //    (gi + b Q, b < NB)
#pragma unroll
                    for (int gi = 0; gi < Q; ++gi) {
                        R v[2 * NB];
#pragma unroll
                        for (int b = 0; b < NB; ++b) {
                            const cplx<R> x = g[reg_of<NC, K>(gi + b * Q)];
                            const cplx<R> y = g[reg_of<NC, K>(NC - 1 - gi - b * Q)];
                            v[2 * b + 0] = fma(x.x, y.x, x.y * y.y);
                            v[2 * b + 1] = fma(x.x, y.y, -x.y * y.x);
                        }
                        transpose_add<S::S1, S::S2>(v);
                        *reinterpret_cast<cplx<R>*>(part + (sym * ML + row) * PST + 2 * gi) =
                            cplx<R>{v[0], v[1]};
                        if ((gi & 3) == 3) __builtin_amdgcn_sched_barrier(0);
                    }
                    // the partials were written by other lanes of this wave:
                    // LDS operations of one wave complete in order
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    // 2. sums over the holder rows of pair p, 3. its rotation
                    //    from the tracked norms and scales of the columns at
                    //    positions p and NC-1-p
                    const int p = row % NP, k = row / NP;
                    const R* src = part + (sym * ML + (p / Q) * GL + k * Q) * PST + 2 * (p % Q);
                    R s0 = 0, s1 = 0;
#pragma unroll
                    for (int r = 0; r < Q; ++r) {
                        const cplx<R> q = *reinterpret_cast<const cplx<R>*>(src + r * PST);
                        s0 += q.x;
                        s1 += q.y;
                    }
                    s0 = xsum_range<NP, ML>(s0);
                    s1 = xsum_range<NP, ML>(s1);
                    const int cj = col_at<NC>(p, step), ck = col_at<NC>(NC - 1 - p, step);
                    double al = nrm[sym * NC + cj], be = nrm[sym * NC + ck];
                    R dj = dcur[sym * NC + cj], dk = dcur[sym * NC + ck];
                    const double gs = double(dj) * double(dk);   // true gamma = d_j d_k gamma
                    quad<R> q;
                    // only rotations larger than kappa keep the symbol
                    // sweeping (see rotation_scaled)
                    rotated |= rotation_scaled<R>(al, be, double(s0) * gs, double(s1) * gs, tol, 0.0, dj, dk, q) > 1;
                    // the LP lanes of a pair hold identical sums, parameters,
                    // norms and scales: all of them store (same value, same
                    // address)
                    prm_b[sym * NP + p] = q;
                    nrm[sym * NC + cj] = al;
                    nrm[sym * NC + ck] = be;
                    dcur[sym * NC + cj] = dj;
                    dcur[sym * NC + ck] = dk;
                }
                // parameters of this step visible to both waves; the Q wave
                // applies step s while the G wave already works on step s+1
                // (double-buffered parameters, one barrier per step)
                wsync(solo);
#pragma unroll
                for (int p0 = 0; p0 < NP; p0 += 8) {
#pragma unroll
                    for (int p = p0; p < p0 + 8 && p < NP; ++p) {
                        const quad<R> q = prm_b[sym * NP + p];
                        rot_apply_scaled(g[reg_of<NC, K>(p)], g[reg_of<NC, K>(NC - 1 - p)], q.a, q.b, q.c,
                                         q.d);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
                buf ^= 1;
              }, std::make_integer_sequence<int, U>{});
              rotate_positions_by<NC, U>(g);
            }
        }
        ++sweeps;
        // convergence: a sweep without rotations, per symbol
        if (rotated) flags[sym] = 1;
        wsync(solo);
        const bool conv_now = flags[sym] == 0;
        if (!my_conv && conv_now) {
            my_conv = true;
            conv_at = sweeps;
        }
        all = true;
#pragma unroll
        for (int s = 0; s < SPW; ++s) all = all && (flags[s] == 0);
        wsync(solo);
        if (all) break;
    }
    phase_add(1);
    if (SEG && !all && sweeps < a.max_sweeps) {
        // ------------------------------------------------------------ save
        // fold the last segment's scales (as the finish does) and save the
        // rows; the next run starts from scales 1, so the values it sees are
        // those an uninterrupted run would see
        quad<R>* dst = seg.state + (size_t)wave * (NC / 2) * 64 + lane;
#pragma unroll
        for (int jp = 0; jp < NC / 2; ++jp) {
            const R f0 = dsc[cur * (SPW * NC) + sym * NC + 2 * jp];
            const R f1 = dsc[cur * (SPW * NC) + sym * NC + 2 * jp + 1];
            dst[jp * 64] = quad<R>{g[2 * jp].x * f0, g[2 * jp].y * f0,
                                   g[2 * jp + 1].x * f1, g[2 * jp + 1].y * f1};
        }
        if (wave == 0 && row == 0) seg.meta[1 + sym] = my_conv ? conv_at : 0;
        if (wave == 0 && lane == 0) seg.meta[0] = sweeps;
        // this wave's stores complete and visible to the device before the
        // group is queued again
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        wsync(solo);
        phase_add(3);
        return false;
    }
    if (!my_conv) conv_at = sweeps;

    // -------------------------------------------------------------- finish
    // true columns of G and Q: fold the last segment's scales (positions
    // are the identity after a whole sweep; the G wave no longer changes them)
#pragma unroll
    for (int j = 0; j < NC; ++j) {
        const R f = dsc[cur * (SPW * NC) + sym * NC + j];
        g[j] = {g[j].x * f, g[j].y * f};
    }
    // column norms: |g_j|^2 folded across lanes, then summed over the holders
    if (wave == 0) fold_column_norms<R, NC, ML>(g, part, sym, row);
    wsync(solo);
    if (wave == 0) {
        // numerically zero columns (see negligible_sq) are reported as 0
        const R cn = row < NC ? column_norm<R, NC, ML>(part, sym, row) : R(0);
        const double fl = negligible_sq<R>() * xsum_range<1, ML>(double(cn));
        if (row < NC) sigs[sym * NC + row] = double(cn) <= fl ? R(0) : sqrt(cn);
    }
    wsync(solo);
    // rank sort of the N real columns: descending, ties by index
    if (wave == 0 && row < N) {
        const R sj = skey(sigs[sym * NC + row]);
        int rank = 0;
        for (int k = 0; k < N; ++k) {
            const R sk = skey(sigs[sym * NC + k]);
            rank += (sk > sj) || (sk == sj && k < row);
        }
        rankof[sym * NC + row] = rank;
        colof[sym * NC + rank] = row;
        if (active) {
            a.sigma[(size_t)tg.out * N + rank] = sigs[sym * NC + row];
            if (tg.mirror >= 0) a.sigma[(size_t)tg.mirror * N + rank] = sigs[sym * NC + row];
        }
    }
    if (tid < SPW) {
        // slots past the last item hold no symbol: nothing to complete
        int z = 0;
        if (base + tid < count)
            for (int k = 0; k < N; ++k) z += sigs[tid * NC + k] == R(0);
        nzero[tid] = z;
    }
    wsync(solo);
    if (a.info && wave == 0) {
        // the wave's symbols gathered at lane 0: one atomic per word and per
        // distinct histogram bin (with a million small symbols, per-symbol
        // atomics on the same few words serialise)
        bool bad = false;
        if (row == 0 && active)
            for (int k = 0; k < N; ++k) bad |= !isfinite(sigs[sym * NC + k]);
        int vals[SPW];
        bool act[SPW];
        int sum = 0, mx = 0, ncv = 0, anybad = 0;
#pragma unroll
        for (int s2 = 0; s2 < SPW; ++s2) {
            vals[s2] = __shfl(conv_at, s2 * ML, 64);
            act[s2] = __shfl(int(active), s2 * ML, 64) != 0;
            const int nco = __shfl(int(!my_conv), s2 * ML, 64);
            const int b = __shfl(int(bad), s2 * ML, 64);
            if (act[s2]) {
                sum += vals[s2];
                mx = max(mx, vals[s2]);
                ncv += nco;
                anybad |= b;
            }
        }
        if (lane == 0 && act[0]) {
            atomicAdd(&a.info[LFA_INFO_SUM_SWEEPS], sum);
            atomicMax(&a.info[LFA_INFO_MAX_SWEEPS], mx);
            if (ncv) atomicAdd(&a.info[LFA_INFO_NONCONVERGED], ncv);
            if (anybad) atomicOr(&a.info[LFA_INFO_NONFINITE], 1);
#pragma unroll
            for (int s2 = 0; s2 < SPW; ++s2) {
                bool first = act[s2];
                int cnt = 0;
#pragma unroll
                for (int s3 = 0; s3 < SPW; ++s3) {
                    if (s3 < s2 && act[s3] && vals[s3] == vals[s2]) first = false;
                    if (act[s3] && vals[s3] == vals[s2]) ++cnt;
                }
                if (first) atomicAdd(&a.info[LFA_INFO_HIST + min(vals[s2], LFA_INFO_HIST_BINS - 1)], cnt);
            }
        }
    }
    cplx<R>* left = d.transposed ? a.V : a.U;
    cplx<R>* right = d.transposed ? a.U : a.V;
    if (left && wave == 0) {
        // u_j = g_j / sigma_j; columns with sigma_j == 0 are zero here
        bool accd[NC];
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            const R sj = sigs[sym * NC + j];
            const R inv = (j < N && sj > R(0)) ? R(1) / sj : R(0);
            g[j] = {g[j].x * inv, g[j].y * inv};
            accd[j] = j < N && sj != R(0);
        }
        int nzmax = 0;
#pragma unroll
        for (int s = 0; s < SPW; ++s) nzmax = max(nzmax, nzero[s]);
        // Columns with sigma == 0 (sorted last, by index): orthonormal
        // completion by two passes of classical Gram-Schmidt of unit vectors
        // e_cand against the accepted columns.  Every lane keeps its own row;
        // inner products are sums over the ML lanes of its symbol, and every
        // loop bound is uniform over the wave (symbols with fewer zero
        // columns idle through the extra iterations).
        // candidates e_cand continue across the zero columns of a symbol
        // (those already used are in the span of the accepted columns)
        int cand = 0;
        R thresh = R(0.5);
        for (int c = 0; c < nzmax; ++c) {
            int jz = -1, cnt = 0;
#pragma unroll
            for (int j = 0; j < NC; ++j) {
                if (j < N && sigs[sym * NC + j] == R(0)) {
                    if (cnt == c) jz = j;
                    ++cnt;
                }
            }
            bool done = jz < 0;
            for (int tries = 0; tries < 4 * M; ++tries) {
                if (__all(done)) break;
                if (cand == M) {
                    cand = 0;
                    thresh *= R(0.2);
                }
                cplx<R> x = {R(row == cand ? 1 : 0), R(0)};
                for (int pass = 0; pass < 2; ++pass) {
                    cplx<R> y = x;
#pragma unroll
                    for (int j = 0; j < NC; ++j) {
                        R cr = g[j].x * x.x + g[j].y * x.y;
                        R ci = g[j].x * x.y - g[j].y * x.x;
                        cr = xsum_range<1, ML>(cr);
                        ci = xsum_range<1, ML>(ci);
                        if (!accd[j]) {
                            cr = R(0);
                            ci = R(0);
                        }
                        y.x -= cr * g[j].x - ci * g[j].y;
                        y.y -= cr * g[j].y + ci * g[j].x;
                    }
                    x = y;
                }
                const R nrm = sqrt(xsum_range<1, ML>(x.x * x.x + x.y * x.y));
                if (!done && nrm > thresh) {
#pragma unroll
                    for (int j = 0; j < NC; ++j) {
                        if (j == jz) {
                            g[j] = {x.x / nrm, x.y / nrm};
                            accd[j] = true;
                        }
                    }
                    done = true;
                }
                if (!done) ++cand;
            }
        }
        store_rows<R, NC, ML>(active ? left + (size_t)tg.out * M * N : nullptr,
                              active && tg.mirror >= 0 ? left + (size_t)tg.mirror * M * N : nullptr, M, N,
                              colof + sym * NC, g, stage, sym, row);
    }
    // the two waves stage through the same LDS: U first, then V
    wsync(solo);
    if (right && wave == 1) {
        store_rows<R, NC, ML>(active ? right + (size_t)tg.out * N * N : nullptr,
                              active && tg.mirror >= 0 ? right + (size_t)tg.mirror * N * N : nullptr, N, N,
                              colof + sym * NC, g, stage, sym, row);
    }
    // the LDS of this group is reused by the next one
    wsync(solo);
    phase_add(2);
    return true;
}


}  // namespace dev
}  // namespace lfa
