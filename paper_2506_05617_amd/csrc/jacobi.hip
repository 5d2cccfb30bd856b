// Batched one-sided Jacobi SVD of convolution symbols on gfx950.
//
// One work-group owns one symbol at a time.  It assembles the c_out x c_in
// symbol A_k = sum_y M_y exp(+2 pi i <k,y>) (Sec. III "Convolution Theorem",
// Algorithm 1 symbol step) straight into its working matrix G (LDS, or a
// global slot for symbols larger than LDS), runs complex one-sided (Hestenes)
// Jacobi sweeps on the columns of G with a parallel round-robin pair order,
// and writes sigma (sorted), U and V (Algorithm 1 SVD step).
//
// G is M x N, column-major with leading dimension ldg, M = max(c_out, c_in),
// N = min(c_out, c_in).  For c_out >= c_in, G = A and the accumulated
// rotations form V; for c_out < c_in, G = A^H and the roles of U and V swap.
//
// A column pair (j, k) is handled by a group of L lanes of one wavefront;
// lane l owns rows l, l+L, ... of both columns in registers.  The three inner
// products alpha = |g_j|^2, beta = |g_k|^2, gamma = g_j^H g_k are reduced with
// xor shuffles inside the lane group, the rotation is computed in double
// precision by every lane of the group (no broadcast), and applied to the
// registers, then written back.  The N/2 pairs of one round-robin step are
// disjoint, so groups never touch the same column within a step; a
// work-group barrier separates steps.

#include <hip/hip_runtime.h>
#include <math.h>

#include "lfa_internal.hpp"

namespace lfa {
namespace {

template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

template <typename R>
__device__ __forceinline__ R shfl_xor(R v, int mask) {
    return __shfl_xor(v, mask, 64);
}

// Sum over the L lanes of a lane group (L a power of two <= 64).
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
template <typename R>
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
    } else {
        const cplx<R>* A = a.A + (size_t)theta * E;
        for (int e = tid; e < E; e += nt) {
            const cplx<R> v = A[e];
            const int o = e / d.c_in, i = e - (e / d.c_in) * d.c_in;
            if (!d.transposed) s.G[(size_t)i * d.ldg + o] = v;
            else               s.G[(size_t)o * d.ldg + i] = {v.x, -v.y};
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
// One-sided Jacobi sweeps.  Returns the number of sweeps used; `converged`
// tells whether the last sweep made no rotation.
// ---------------------------------------------------------------------------
template <typename R, int L>
__device__ int jacobi(const LayerDesc& d, const Shared<R>& s, int max_sweeps, double tol,
                      bool& converged) {
    constexpr int RM = kRowsPerLane;
    const int tid = threadIdx.x;
    const int lane = tid & (L - 1), group = tid / L, ngroups = blockDim.x / L;
    const int M = d.M, N = d.N, ldg = d.ldg, ldv = d.ldv;
    const int Np = N + (N & 1);
    const int npairs = Np / 2, nsteps = Np - 1;
    cplx<R>* __restrict__ G = s.G;
    cplx<R>* __restrict__ Q = s.Q;

    if (tid == 0) s.flags[0] = s.flags[1] = s.flags[2] = 0;
    __syncthreads();
    converged = (N < 2);
    int sweep = 0;
    while (!converged && sweep < max_sweeps) {
        if (tid == 0) s.flags[(sweep + 1) % 3] = 0;
        for (int step = 0; step < nsteps; ++step) {
            for (int pb = 0; pb < npairs; pb += ngroups) {
                const int pr = pb + group;
                if (pr >= npairs) continue;
                int j, k;
                rr_pair(pr, step, Np, j, k);
                if (j >= N || k >= N) continue;
                cplx<R> x[RM], y[RM];
                R al = 0, be = 0, gr = 0, gi = 0;
#pragma unroll
                for (int t = 0; t < RM; ++t) {
                    const int i = lane + t * L;
                    if (i < M) {
                        x[t] = G[(size_t)j * ldg + i];
                        y[t] = G[(size_t)k * ldg + i];
                        al = fma(x[t].x, x[t].x, fma(x[t].y, x[t].y, al));
                        be = fma(y[t].x, y[t].x, fma(y[t].y, y[t].y, be));
                        gr = fma(x[t].x, y[t].x, fma(x[t].y, y[t].y, gr));
                        gi = fma(x[t].x, y[t].y, fma(-x[t].y, y[t].x, gi));
                    }
                }
                al = group_sum<R, L>(al);
                be = group_sum<R, L>(be);
                gr = group_sum<R, L>(gr);
                gi = group_sum<R, L>(gi);
                const double g = sqrt(double(gr) * double(gr) + double(gi) * double(gi));
                if (!(g > tol * sqrt(double(al) * double(be)))) continue;
                // Real 2x2 symmetric Schur step on [[al, g], [g, be]] after the
                // phase of gamma is moved into column k.
                const double zeta = (double(be) - double(al)) / (2.0 * g);
                const double tt = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double cs = 1.0 / sqrt(1.0 + tt * tt);
                const double sn = cs * tt;
                // x' = c x - s e^{-i phi} y ;  y' = c y + s e^{+i phi} x
                const R c = R(cs);
                const R sr = R(sn * double(gr) / g), si = R(-sn * double(gi) / g);
#pragma unroll
                for (int t = 0; t < RM; ++t) {
                    const int i = lane + t * L;
                    if (i < M) {
                        const cplx<R> xv = x[t], yv = y[t];
                        cplx<R> xn, yn;
                        xn.x = fma(c, xv.x, -fma(sr, yv.x, -si * yv.y));
                        xn.y = fma(c, xv.y, -fma(sr, yv.y, si * yv.x));
                        yn.x = fma(c, yv.x, fma(sr, xv.x, si * xv.y));
                        yn.y = fma(c, yv.y, fma(sr, xv.y, -si * xv.x));
                        G[(size_t)j * ldg + i] = xn;
                        G[(size_t)k * ldg + i] = yn;
                    }
                }
                if (Q) {
#pragma unroll
                    for (int t = 0; t < RM; ++t) {
                        const int i = lane + t * L;
                        if (i < N) {
                            const cplx<R> xv = Q[(size_t)j * ldv + i], yv = Q[(size_t)k * ldv + i];
                            cplx<R> xn, yn;
                            xn.x = fma(c, xv.x, -fma(sr, yv.x, -si * yv.y));
                            xn.y = fma(c, xv.y, -fma(sr, yv.y, si * yv.x));
                            yn.x = fma(c, yv.x, fma(sr, xv.x, si * xv.y));
                            yn.y = fma(c, yv.y, fma(sr, xv.y, -si * xv.x));
                            Q[(size_t)j * ldv + i] = xn;
                            Q[(size_t)k * ldv + i] = yn;
                        }
                    }
                }
                if (lane == 0) s.flags[sweep % 3] = 1;
            }
            __syncthreads();
        }
        converged = (s.flags[sweep % 3] == 0);
        ++sweep;
    }
    __syncthreads();
    return sweep;
}

// ---------------------------------------------------------------------------
// Norms, sort, normalisation, completion of zero columns, outputs.
// ---------------------------------------------------------------------------
template <typename R, int L>
__device__ void finish(const SvdArgs<R>& a, const Shared<R>& s, int out_idx, int mirror,
                       int sweeps, bool converged) {
    const LayerDesc& d = a.d;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & (L - 1), group = tid / L, ngroups = nt / L;
    const int M = d.M, N = d.N, ldg = d.ldg, ldv = d.ldv;
    cplx<R>* G = s.G;
    cplx<R>* Q = s.Q;

    // column norms
    for (int j = group; j < N; j += ngroups) {
        R acc = 0;
        for (int i = lane; i < M; i += L) {
            const cplx<R> v = G[(size_t)j * ldg + i];
            acc = fma(v.x, v.x, fma(v.y, v.y, acc));
        }
        acc = group_sum<R, L>(acc);
        if (lane == 0) s.sig[j] = sqrt(acc);
    }
    __syncthreads();
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

    if (want_left) {
        // normalise columns in place: u_j = g_j / sigma_j (zero columns stay 0)
        for (int e = tid; e < N * M; e += nt) {
            const int j = e / M, i = e - (e / M) * M;
            const R sj = s.sig[j];
            const cplx<R> v = G[(size_t)j * ldg + i];
            const R inv = sj > R(0) ? R(1) / sj : R(0);
            G[(size_t)j * ldg + i] = {v.x * inv, v.y * inv};
        }
        __syncthreads();
        // Columns with sigma == 0 (they sort last) get an orthonormal
        // completion: unit vectors e_0, e_1, ... orthogonalised by two passes
        // of classical Gram-Schmidt against every accepted column, kept when
        // the residual norm exceeds a threshold (1/2, lowered if no unit
        // vector qualifies; some residual has norm >= 1/sqrt(M)).
        int nz = 0;
        while (nz < N && s.sig[s.perm[N - 1 - nz]] == R(0)) ++nz;
        int cand = 0;
        R thresh = R(0.5);
        for (int zc = N - nz; zc < N; ++zc) {
            const int jz = s.perm[zc];
            bool done = false;
            for (int tries = 0; !done && tries < 4 * M; ++tries) {
                if (cand == M) {
                    cand = 0;
                    thresh *= R(0.2);
                }
                for (int i = tid; i < M; i += nt) G[(size_t)jz * ldg + i] = {R(i == cand), R(0)};
                __syncthreads();
                for (int pass = 0; pass < 2; ++pass) {
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
                    __syncthreads();
                    for (int i = tid; i < M; i += nt) {
                        cplx<R> x = G[(size_t)jz * ldg + i];
                        for (int col = 0; col < N; ++col) {
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
                __syncthreads();
            }
        }
        // write: out[theta][i][c] = G[perm[c]][i]
        cplx<R>* out = (d.transposed ? a.V : a.U) + (size_t)out_idx * M * r;
        cplx<R>* mir = mirror >= 0 ? (d.transposed ? a.V : a.U) + (size_t)mirror * M * r : nullptr;
        for (int e = tid; e < M * r; e += nt) {
            const int i = e / r, c = e - (e / r) * r;
            const cplx<R> v = G[(size_t)s.perm[c] * ldg + i];
            out[e] = v;
            if (mir) mir[e] = {v.x, -v.y};
        }
    }
    if (want_right) {
        cplx<R>* out = (d.transposed ? a.U : a.V) + (size_t)out_idx * N * r;
        cplx<R>* mir = mirror >= 0 ? (d.transposed ? a.U : a.V) + (size_t)mirror * N * r : nullptr;
        for (int e = tid; e < N * r; e += nt) {
            const int i = e / r, c = e - (e / r) * r;
            const cplx<R> v = Q[(size_t)s.perm[c] * ldv + i];
            out[e] = v;
            if (mir) mir[e] = {v.x, -v.y};
        }
    }
    if (a.info) {
        if (tid == 0) {
            atomicAdd(&a.info[LFA_INFO_SUM_SWEEPS], sweeps);
            atomicMax(&a.info[LFA_INFO_MAX_SWEEPS], sweeps);
            if (!converged) atomicAdd(&a.info[LFA_INFO_NONCONVERGED], 1);
        }
        if (bad) atomicOr(&a.info[LFA_INFO_NONFINITE], 1);
    }
    __syncthreads();
}

// Work item `item` (see target_of).
template <typename R, int L>
__device__ void svd_one(const SvdArgs<R>& a, char* lds, int item, char* gslot) {
    const Target tg = target_of(a, item);
    const int theta = tg.theta;
    const bool acc = (a.d.transposed ? a.U : a.V) != nullptr;
    const Shared<R> s = carve<R>(lds, a.d, acc, gslot);
    load_symbol<R>(a, s, theta);
    __syncthreads();
    bool converged;
    const int sweeps = jacobi<R, L>(a.d, s, a.max_sweeps, a.tol, converged);
    finish<R, L>(a, s, tg.out, tg.mirror, sweeps, converged);
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
// Inner products are reduced over rows by a per-wave LDS transpose and a sum
// over the waves; one thread per pair computes the rotation.
// ---------------------------------------------------------------------------
constexpr int kBlk = 8;   // columns per block

template <typename R>
struct BlockLds {
    R* wpart;        // [waves][64][4B+4]
    R* wsum;         // [waves][4B]
    quad<R>* prm;    // [B]
    int* rflag;      // rotation made in this sweep
};

template <typename R>
__device__ __forceinline__ BlockLds<R> carve_block(char* lds, size_t off) {
    constexpr int B = kBlk, PST = 4 * B + 4;
    const int nw = blockDim.x >> 6;
    BlockLds<R> b;
    R* p = reinterpret_cast<R*>(lds + ((off + 63) & ~size_t(63)));
    b.wpart = p;
    p += nw * 64 * PST;
    b.wsum = p;
    p += nw * 4 * B;
    b.prm = reinterpret_cast<quad<R>*>(p);
    b.rflag = reinterpret_cast<int*>(b.prm + B);
    return b;
}

// Sum the per-row contributions q[p] (p < B pairs) over all rows and compute
// the B rotations into bl.prm.  Contains two work-group barriers.
template <typename R>
__device__ __forceinline__ void block_reduce_rotate(const BlockLds<R>& bl, quad<R> (&q)[kBlk],
                                                    double tol) {
    constexpr int B = kBlk, PST = 4 * B + 4, Q = 4 * B, H = 64 / Q;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    R* wp = bl.wpart + wave * 64 * PST;
#pragma unroll
    for (int p = 0; p < B; ++p) *reinterpret_cast<quad<R>*>(wp + lane * PST + 4 * p) = q[p];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const int qi = lane % Q, h = lane / Q;
    R sum = 0;
#pragma unroll 8
    for (int r = h * (64 / H); r < (h + 1) * (64 / H); ++r) sum += wp[r * PST + qi];
#pragma unroll
    for (int off = Q; off < 64; off <<= 1) sum += __shfl_xor(sum, off, 64);
    if (lane < Q) bl.wsum[wave * Q + qi] = sum;
    __syncthreads();
    if (tid < B) {
        R s0 = 0, s1 = 0, s2 = 0, s3 = 0;
        for (int w = 0; w < nw; ++w) {
            const R* ws = bl.wsum + w * Q + 4 * tid;
            s0 += ws[0];
            s1 += ws[1];
            s2 += ws[2];
            s3 += ws[3];
        }
        const quad<R> r = rotation<R>(s0, s1, s2, s3, tol);
        bl.prm[tid] = r;
        if (r.d != R(0)) *bl.rflag = 1;
    }
    __syncthreads();
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

template <typename R>
__device__ void block_sweeps(const LayerDesc& d, const Shared<R>& s, const BlockLds<R>& bl,
                             int max_sweeps, double tol, Team& team, int& sweeps_out,
                             bool& conv_out) {
    constexpr int B = kBlk;
    const int tid = threadIdx.x;
    const int member = team.member, W = team.W;
    const int M = d.M, N = d.N;
    const int NB = (N + B - 1) / B, NBP = NB + (NB & 1);
    const bool grow = tid < M, qrow = s.Q != nullptr && tid < N;
    cplx<R> ga[B], gb[B], va[B], vb[B];
    quad<R> q[B];
    int sweeps = 0;
    bool converged = (N < 2);
    while (!converged && sweeps < max_sweeps) {
        if (tid == 0) *bl.rflag = 0;
        __syncthreads();
        // team: rotations counted before this sweep (all earlier increments
        // happened before the barrier that ended the previous sweep)
        const int rot_before =
            W > 1 ? __hip_atomic_load(team.rot, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) : 0;
        // ---- intra pass: pairs inside blocks 2i and 2i+1
        for (int i = member; 2 * i < NB; i += W) {
            const int ba = 2 * i, bb = 2 * i + 1;
            load_block(s.G, d.ldg, ba, N, tid, grow, ga);
            load_block(s.G, d.ldg, bb, N, tid, grow, gb);
            if (s.Q) {
                load_block(s.Q, d.ldv, ba, N, tid, qrow, va);
                load_block(s.Q, d.ldv, bb, N, tid, qrow, vb);
            }
            for (int step = 0; step < B - 1; ++step) {
#pragma unroll
                for (int p = 0; p < B / 2; ++p) {
                    q[p] = pair_partials(ga[p], ga[B - 1 - p]);
                    q[B / 2 + p] = pair_partials(gb[p], gb[B - 1 - p]);
                }
                block_reduce_rotate<R>(bl, q, tol);
#pragma unroll
                for (int p = 0; p < B / 2; ++p) {
                    const quad<R> ra = bl.prm[p], rb = bl.prm[B / 2 + p];
                    rot_apply(ga[p], ga[B - 1 - p], ra.a, ra.b, ra.c);
                    rot_apply(gb[p], gb[B - 1 - p], rb.a, rb.b, rb.c);
                    if (s.Q) {
                        rot_apply(va[p], va[B - 1 - p], ra.a, ra.b, ra.c);
                        rot_apply(vb[p], vb[B - 1 - p], rb.a, rb.b, rb.c);
                    }
                }
                // round-robin: positions 1..B-1 move by one
                const cplx<R> la = ga[B - 1], lb = gb[B - 1], lva = va[B - 1], lvb = vb[B - 1];
#pragma unroll
                for (int k = B - 1; k >= 2; --k) {
                    ga[k] = ga[k - 1];
                    gb[k] = gb[k - 1];
                    va[k] = va[k - 1];
                    vb[k] = vb[k - 1];
                }
                ga[1] = la;
                gb[1] = lb;
                va[1] = lva;
                vb[1] = lvb;
            }
            // B-1 steps bring every position back: store in place
            store_block(s.G, d.ldg, ba, N, tid, grow, ga);
            store_block(s.G, d.ldg, bb, N, tid, grow, gb);
            if (s.Q) {
                store_block(s.Q, d.ldv, ba, N, tid, qrow, va);
                store_block(s.Q, d.ldv, bb, N, tid, qrow, vb);
            }
        }
        if (W > 1) team_barrier(team);
        // ---- cross passes: round-robin over block pairs
        for (int os = 0; os < NBP - 1; ++os) {
            for (int bp = member; bp < NBP / 2; bp += W) {
                int ba, bb;
                rr_pair(bp, os, NBP, ba, bb);
                if (ba >= NB || bb >= NB) continue;
                load_block(s.G, d.ldg, ba, N, tid, grow, ga);
                load_block(s.G, d.ldg, bb, N, tid, grow, gb);
                if (s.Q) {
                    load_block(s.Q, d.ldv, ba, N, tid, qrow, va);
                    load_block(s.Q, d.ldv, bb, N, tid, qrow, vb);
                }
                for (int t = 0; t < B; ++t) {
#pragma unroll
                    for (int p = 0; p < B; ++p) q[p] = pair_partials(ga[p], gb[p]);
                    block_reduce_rotate<R>(bl, q, tol);
#pragma unroll
                    for (int p = 0; p < B; ++p) {
                        const quad<R> r = bl.prm[p];
                        rot_apply(ga[p], gb[p], r.a, r.b, r.c);
                        if (s.Q) rot_apply(va[p], vb[p], r.a, r.b, r.c);
                    }
                    // block b shifts by one against block a
                    const cplx<R> fb = gb[0], fv = vb[0];
#pragma unroll
                    for (int k = 0; k < B - 1; ++k) {
                        gb[k] = gb[k + 1];
                        vb[k] = vb[k + 1];
                    }
                    gb[B - 1] = fb;
                    vb[B - 1] = fv;
                }
                // B shifts bring block b back to its order
                store_block(s.G, d.ldg, ba, N, tid, grow, ga);
                store_block(s.G, d.ldg, bb, N, tid, grow, gb);
                if (s.Q) {
                    store_block(s.Q, d.ldv, ba, N, tid, qrow, va);
                    store_block(s.Q, d.ldv, bb, N, tid, qrow, vb);
                }
            }
            if (W > 1 && os < NBP - 2) team_barrier(team);
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

template <typename R>
__device__ void block_one(const SvdArgs<R>& a, char* lds, int item, char* gslot, Team& team) {
    const Target tg = target_of(a, item);
    const bool acc = (a.d.transposed ? a.U : a.V) != nullptr;
    const Shared<R> s = carve<R>(lds, a.d, acc, gslot);
    const BlockLds<R> bl = carve_block<R>(lds, s.small_end);
    if (team.member == 0) load_symbol<R>(a, s, tg.theta);
    if (team.W > 1) team_barrier(team);
    else __syncthreads();
    int sweeps;
    bool converged;
    block_sweeps<R>(a.d, s, bl, a.max_sweeps, a.tol, team, sweeps, converged);
    if (team.member == 0) finish<R, 64>(a, s, tg.out, tg.mirror, sweeps, converged);
    // the slot is reused for the team's next symbol: members wait for the finish
    if (team.W > 1) team_barrier(team);
    if (a.info && threadIdx.x == 0 && team.member == 0 &&
        (__hip_atomic_load(team.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 2))
        atomicOr(&a.info[LFA_INFO_NONFINITE], 2);
}

// Grid = teams x W work-groups, all resident at once (the host sizes the
// grid from the occupancy of this kernel).  Team t owns slot t and works on
// items t, t + teams, ...
template <typename R>
__global__ void __launch_bounds__(512) block_kernel(SvdArgs<R> a, int W, int32_t* counters) {
    extern __shared__ __align__(16) char lds[];
    const int teams = gridDim.x / W;
    const int tix = blockIdx.x / W;
    Team team;
    team.member = blockIdx.x - tix * W;
    team.W = W;
    team.bar = counters + 4 * tix;
    team.rot = counters + 4 * tix + 1;
    team.err = counters + 4 * teams;
    team.target = 0;
    char* gslot = a.gws + (size_t)tix * a.slot_bytes;
    const int count = item_count(a);
    for (int item = tix; item < count; item += teams) block_one<R>(a, lds, item, gslot, team);
}

template <typename R, int L>
__global__ void __launch_bounds__(1024) svd_kernel(SvdArgs<R> a) {
    extern __shared__ __align__(16) char lds[];
    char* gslot = a.gws ? a.gws + (size_t)blockIdx.x * a.slot_bytes : nullptr;
    // with a symbol list, outputs are compact (entry `item` of the list)
    const int count = item_count(a);
    for (int item = blockIdx.x; item < count; item += gridDim.x) svd_one<R, L>(a, lds, item, gslot);
}

// Dynamic LDS above 64 KiB needs an explicit per-kernel opt-in.
template <typename K>
hipError_t allow_lds(K kernel, size_t lds) {
    if (lds <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <typename R, int L>
hipError_t launch_svd_L(const SvdArgs<R>& a, int grid, size_t lds, hipStream_t st) {
    hipError_t e = allow_lds(svd_kernel<R, L>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((svd_kernel<R, L>), dim3(grid), dim3(a.d.threads), lds, st, a);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_svd(const SvdArgs<R>& a, int grid, size_t lds, hipStream_t st) {
    switch (a.d.L) {
        case 1: return launch_svd_L<R, 1>(a, grid, lds, st);
        case 2: return launch_svd_L<R, 2>(a, grid, lds, st);
        case 4: return launch_svd_L<R, 4>(a, grid, lds, st);
        case 8: return launch_svd_L<R, 8>(a, grid, lds, st);
        case 16: return launch_svd_L<R, 16>(a, grid, lds, st);
        case 32: return launch_svd_L<R, 32>(a, grid, lds, st);
        case 64: return launch_svd_L<R, 64>(a, grid, lds, st);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Persistent launch: work-groups dequeue (layer, theta) items.
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(256) persistent_kernel(PersistentArgs<R> pa_arg) {
    extern __shared__ __align__(16) char lds[];
    __shared__ int item_sh;
    // Index the per-layer table where it lives (the kernel-argument segment)
    // instead of letting a dynamic index copy the whole argument to scratch.
#if defined(__HIP_DEVICE_COMPILE__)
    const PersistentArgs<R>& pa = *(const PersistentArgs<R>*)__builtin_amdgcn_kernarg_segment_ptr();
    (void)pa_arg;
#else
    const PersistentArgs<R>& pa = pa_arg;
#endif
    for (;;) {
        if (threadIdx.x == 0) item_sh = atomicAdd(pa.counter, 1);
        __syncthreads();
        const int item = item_sh;
        __syncthreads();
        if (item >= pa.num_items) break;
        const WorkItem w = pa.items[item];
        const SvdArgs<R>& a = pa.layer[w.layer];
        char* gslot = a.gws ? a.gws + (size_t)blockIdx.x * a.slot_bytes : nullptr;
        switch (a.d.L) {
            case 1: svd_one<R, 1>(a, lds, w.theta, gslot); break;
            case 2: svd_one<R, 2>(a, lds, w.theta, gslot); break;
            case 4: svd_one<R, 4>(a, lds, w.theta, gslot); break;
            case 8: svd_one<R, 8>(a, lds, w.theta, gslot); break;
            case 16: svd_one<R, 16>(a, lds, w.theta, gslot); break;
            case 32: svd_one<R, 32>(a, lds, w.theta, gslot); break;
            default: svd_one<R, 64>(a, lds, w.theta, gslot); break;
        }
    }
}

__global__ void fill_i32_kernel(int32_t* p, int32_t v, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

}  // namespace

size_t lds_bytes_for(const LayerDesc& d, bool accumulate, int elem_bytes) {
    if (d.kind == 1) return wave_lds_bytes_for(d.wave_nc, d.wave_ml, elem_bytes);
    if (d.kind == 2) return block_lds_bytes(d, accumulate, elem_bytes);
    const int cb = 2 * elem_bytes;
    size_t b = (size_t)cb * kMaxTaps + (size_t)elem_bytes * 64 +
               (size_t)elem_bytes * ((d.N + 3) & ~3) + 2 * sizeof(int) * ((d.N + 3) & ~3);
    b = (b + 15) & ~size_t(15);
    b += (size_t)cb * (d.N + d.M) + sizeof(int) * 4;
    b = (b + 15) & ~size_t(15);
    if (d.storage == kLds) {
        b += (size_t)cb * d.ldg * d.N;
        if (accumulate) b += (size_t)cb * d.ldv * d.N;
    }
    return b;
}

size_t block_lds_bytes(const LayerDesc& d, bool accumulate, int elem_bytes) {
    LayerDesc dg = d;
    dg.kind = 0;
    dg.storage = kGlobal;
    const int nw = d.threads / 64;
    return lds_bytes_for(dg, accumulate, elem_bytes) +
           (size_t)elem_bytes * (nw * 64 * (4 * kBlk + 4) + nw * 4 * kBlk + 4 * kBlk) + 16 + 64;
}

template <typename R>
hipError_t launch_block(const SvdArgs<R>& a, int teams, int W, int32_t* counters, hipStream_t st) {
    const bool acc = (a.d.transposed ? a.U : a.V) != nullptr;
    const size_t lds = block_lds_bytes(a.d, acc, sizeof(R));
    hipError_t e = allow_lds(block_kernel<R>, lds);
    if (e != hipSuccess) return e;
    e = launch_fill_i32(counters, 0, 4LL * teams + 4, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(block_kernel<R>, dim3(teams * W), dim3(a.d.threads), lds, st, a, W, counters);
    return hipGetLastError();
}

template <typename R>
int block_resident_t(const LayerDesc& d, bool acc) {
    const size_t lds = block_lds_bytes(d, acc, sizeof(R));
    if (allow_lds(block_kernel<R>, lds) != hipSuccess) return 0;
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, block_kernel<R>, d.threads, lds) !=
        hipSuccess)
        return 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return per_cu * cus;
}

hipError_t launch_block_svd_f32(const SvdArgs<float>& a, int teams, int W, int32_t* counters,
                                hipStream_t s) {
    return launch_block<float>(a, teams, W, counters, s);
}
hipError_t launch_block_svd_f64(const SvdArgs<double>& a, int teams, int W, int32_t* counters,
                                hipStream_t s) {
    return launch_block<double>(a, teams, W, counters, s);
}
int block_resident(const LayerDesc& d, bool acc, int elem_bytes) {
    return elem_bytes == 8 ? block_resident_t<double>(d, acc) : block_resident_t<float>(d, acc);
}

hipError_t launch_svd_f32(const SvdArgs<float>& a, int grid, size_t lds, hipStream_t s) {
    return launch_svd<float>(a, grid, lds, s);
}
hipError_t launch_svd_f64(const SvdArgs<double>& a, int grid, size_t lds, hipStream_t s) {
    return launch_svd<double>(a, grid, lds, s);
}

hipError_t launch_persistent_f32(const PersistentArgs<float>& a, int grid, size_t lds,
                                 hipStream_t s) {
    hipError_t e = allow_lds(persistent_kernel<float>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(persistent_kernel<float>, dim3(grid), dim3(a.threads), lds, s, a);
    return hipGetLastError();
}
hipError_t launch_persistent_f64(const PersistentArgs<double>& a, int grid, size_t lds,
                                 hipStream_t s) {
    hipError_t e = allow_lds(persistent_kernel<double>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(persistent_kernel<double>, dim3(grid), dim3(a.threads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t value, long long count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int grid = (int)((count + 255) / 256 < 1024 ? (count + 255) / 256 : 1024);
    hipLaunchKernelGGL(fill_i32_kernel, dim3(grid), dim3(256), 0, s, p, value, count);
    return hipGetLastError();
}

}  // namespace lfa
