// Strided convolutions as crystals (Sec. III, "Introduction to Lattices and
// Crystals"): the input of a stride-s layer, read on the coarse lattice
// s Z^2, is a crystal with s*s*c_in points per unit cell, and the layer is a
// stride-1 layer on the coarse torus between that crystal and the output.
//
// The repack below writes that layer's weights.  Tap (a, b) of the strided
// layer sits at offset y = (a - (kh-1)/2, b - (kw-1)/2) (floor division,
// taps centred as for stride 1); it reaches the point d = y mod s of the
// cell at coarse offset Y = floor(y / s), i.e. input channel
// i*s*s + d1*s + d2 at the coarse tap Y + (kh'-1)/2 of the new kernel.
#include <hip/hip_runtime.h>

#include "lfa_internal.hpp"

namespace lfa {
namespace {

constexpr int kCrystalThreads = 256;

__device__ __forceinline__ int floor_div(int a, int s) { return a >= 0 ? a / s : -((-a + s - 1) / s); }

// FORWARD: one thread per element of Wc [c_out][s*s*c_in][kh2][kw2]; taps of
// Wc that no tap of W reaches are zero.  ADJOINT: one thread per element of
// W [c_out][c_in][kh][kw], read from its place in Wc (the transpose of the
// forward map, which is a one-to-one placement).
template <typename R, bool ADJOINT>
__global__ void __launch_bounds__(kCrystalThreads) crystal_weights_kernel(const R* src, R* dst, CrystalArgs a) {
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int s = a.stride, ss = s * s;
    const int ch = (a.kh - 1) / 2, cw = (a.kw - 1) / 2;
    const int ch2 = (a.kh2 - 1) / 2, cw2 = (a.kw2 - 1) / 2;
    const long long cin2 = (long long)ss * a.c_in;
    if constexpr (!ADJOINT) {
        const long long total = (long long)a.c_out * cin2 * a.kh2 * a.kw2;
        if (gid >= total) return;
        const int b2 = (int)(gid % a.kw2);
        long long rest = gid / a.kw2;
        const int a2 = (int)(rest % a.kh2);
        rest /= a.kh2;
        const int c2 = (int)(rest % cin2);
        const long long o = rest / cin2;
        const int i = c2 / ss, d = c2 - i * ss, d1 = d / s, d2 = d - d1 * s;
        const int ta = s * (a2 - ch2) + d1 + ch;   // tap row of W, if any
        const int tb = s * (b2 - cw2) + d2 + cw;
        R v = R(0);
        if (ta >= 0 && ta < a.kh && tb >= 0 && tb < a.kw)
            v = src[((o * a.c_in + i) * a.kh + ta) * a.kw + tb];
        dst[gid] = v;
    } else {
        const long long total = (long long)a.c_out * a.c_in * a.kh * a.kw;
        if (gid >= total) return;
        const int tb = (int)(gid % a.kw);
        long long rest = gid / a.kw;
        const int ta = (int)(rest % a.kh);
        rest /= a.kh;
        const int i = (int)(rest % a.c_in);
        const long long o = rest / a.c_in;
        const int y1 = ta - ch, y2 = tb - cw;
        const int Y1 = floor_div(y1, s), Y2 = floor_div(y2, s);
        const int d1 = y1 - s * Y1, d2 = y2 - s * Y2;
        const long long c2 = (long long)i * ss + d1 * s + d2;
        dst[gid] = src[((o * cin2 + c2) * a.kh2 + (Y1 + ch2)) * a.kw2 + (Y2 + cw2)];
    }
}

template <typename R>
hipError_t crystal_t(const CrystalArgs& a, const void* src, void* dst, bool adjoint, hipStream_t st) {
    const long long total = adjoint ? (long long)a.c_out * a.c_in * a.kh * a.kw
                                    : (long long)a.c_out * a.stride * a.stride * a.c_in * a.kh2 * a.kw2;
    if (total <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((total + kCrystalThreads - 1) / kCrystalThreads);
    if (adjoint)
        hipLaunchKernelGGL((crystal_weights_kernel<R, true>), dim3(blocks), dim3(kCrystalThreads), 0, st,
                           static_cast<const R*>(src), static_cast<R*>(dst), a);
    else
        hipLaunchKernelGGL((crystal_weights_kernel<R, false>), dim3(blocks), dim3(kCrystalThreads), 0, st,
                           static_cast<const R*>(src), static_cast<R*>(dst), a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_crystal_weights(const CrystalArgs& a, int elem_bytes, const void* src, void* dst, bool adjoint,
                                  hipStream_t s) {
    return elem_bytes == 8 ? crystal_t<double>(a, src, dst, adjoint, s) : crystal_t<float>(a, src, dst, adjoint, s);
}

}  // namespace lfa
