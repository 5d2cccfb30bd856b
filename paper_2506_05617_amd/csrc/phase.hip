// Phase normalisation of the singular vectors (post-processing of the SVD
// step, LFA_PHASE_NORMALIZE).  A singular pair (u_j, v_j) of a complex
// matrix is determined only up to a common factor e^{i phi}: A v = sigma u
// holds for (u e^{i phi}, v e^{i phi}) as well.  This pass fixes the factor:
// the entry of largest modulus of v_j (of u_j when only U is written)
// becomes real and positive, the lowest row winning ties.
#include <hip/hip_runtime.h>

#include "lfa_internal.hpp"

namespace lfa {
namespace {

// One work-group per symbol, one thread per column j; U [syms][rows_u][r],
// V [syms][rows_v][r] (either may be null), so the threads of a row read
// consecutive entries.
template <typename R>
__global__ void __launch_bounds__(256) phase_normalize_kernel(cplx<R>* U, cplx<R>* V, int rows_u, int rows_v,
                                                              int r) {
    const size_t th = blockIdx.x;
    cplx<R>* Ut = U ? U + th * rows_u * r : nullptr;
    cplx<R>* Vt = V ? V + th * rows_v * r : nullptr;
    cplx<R>* key = Vt ? Vt : Ut;
    const int rows_k = Vt ? rows_v : rows_u;
    for (int j = threadIdx.x; j < r; j += blockDim.x) {
        R best = R(-1);
        int bi = 0;
#pragma unroll 8
        for (int i = 0; i < rows_k; ++i) {
            const cplx<R> v = key[(size_t)i * r + j];
            const R m2 = v.x * v.x + v.y * v.y;
            if (m2 > best) {
                best = m2;
                bi = i;
            }
        }
        if (!(best > R(0))) continue;        // a zero (or non-finite) column stays as it is
        const cplx<R> vm = key[(size_t)bi * r + j];
        const double a = sqrt((double)best);
        const R c = R(vm.x / a), s = R(-vm.y / a);     // e^{-i phi} = conj(v_max) / |v_max|
        auto scale = [&](cplx<R>* X, int rows) {
#pragma unroll 8
            for (int i = 0; i < rows; ++i) {
                cplx<R>& x = X[(size_t)i * r + j];
                const cplx<R> xv = x;
                x = {xv.x * c - xv.y * s, xv.x * s + xv.y * c};
            }
        };
        if (Ut) scale(Ut, rows_u);
        if (Vt) scale(Vt, rows_v);
        key[(size_t)bi * r + j] = {R(a), R(0)};        // exactly real and positive
    }
}

template <typename R>
hipError_t launch_phase(cplx<R>* U, cplx<R>* V, int syms, int rows_u, int rows_v, int r, hipStream_t s) {
    if (syms <= 0 || r <= 0 || (!U && !V)) return hipSuccess;
    const int threads = std::min(256, (r + 63) / 64 * 64);
    hipLaunchKernelGGL(phase_normalize_kernel<R>, dim3(syms), dim3(threads), 0, s, U, V, rows_u, rows_v, r);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_phase_normalize_f32(cplx<float>* U, cplx<float>* V, int syms, int rows_u, int rows_v, int r,
                                      hipStream_t s) {
    return launch_phase<float>(U, V, syms, rows_u, rows_v, r, s);
}
hipError_t launch_phase_normalize_f64(cplx<double>* U, cplx<double>* V, int syms, int rows_u, int rows_v, int r,
                                      hipStream_t s) {
    return launch_phase<double>(U, V, syms, rows_u, rows_v, r, s);
}

}  // namespace lfa
