// Kernel and launchers of the register-resident (rows-in-lanes) Jacobi
// kernel for symbols of at most 64 rows; the device code is in
// jacobi_device.hpp.
#include <hip/hip_runtime.h>

#include "jacobi_device.hpp"

namespace lfa {
namespace {
using namespace dev;

// Groups of S::SPW symbols: with a group counter, a grid of resident
// work-groups takes the next group when it finishes one (no work-group waits
// for another; the hardware dispatcher, which can hold a new work-group back
// for a busy CU while another CU idles, is out of the loop); without one,
// work-group b runs groups b, b + grid, ...
template <typename R, int NC, int ML>
__device__ __forceinline__ void wave_svd_body(const SvdArgs<R>& a) {
    extern __shared__ __align__(16) char lds_raw[];
    __shared__ int next_sh;
    using S = WaveShape<NC, ML>;
    const int groups = (item_count(a) + S::SPW - 1) / S::SPW;
    int g = blockIdx.x;
    for (;;) {
        if (a.wctr) {
            if (threadIdx.x == 0) next_sh = atomicAdd(a.wctr, 1);
            __syncthreads();
            g = next_sh;
            __syncthreads();
        }
        if (g >= groups) break;
        wave_group<R, NC, ML>(a, lds_raw, g * S::SPW, threadIdx.x, blockDim.x, false);
        if (!a.wctr) g += gridDim.x;
    }
}

// FP64: the registers of a whole SIMD lane if needed (one wave per SIMD).
template <typename R, int NC, int ML>
__global__ void __launch_bounds__(128) wave_svd_kernel(SvdArgs<R> a) {
    wave_svd_body<R, NC, ML>(a);
}

// FP32: at most 256 VGPRs, so that two waves share a SIMD and hide each
// other's LDS and barrier latency.
template <int NC, int ML>
__global__ void __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(2, 2)))
wave_svd_kernel_f32(SvdArgs<float> a) {
    wave_svd_body<float, NC, ML>(a);
}

template <typename K>
hipError_t allow_wave_lds(K kernel, size_t lds) {
    if (lds <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <typename R, int NC, int ML>
hipError_t launch_wave_t(const SvdArgs<R>& a, int grid, hipStream_t st) {
    // output staging after the other arrays when singular vectors are written
    const size_t base = (wave_lds_bytes<R, NC, ML>() + 63) & ~size_t(63);
    const size_t lds = (a.U || a.V) ? base + wave_stage_bytes<R, NC, ML>() : base;
    if constexpr (sizeof(R) == 4) {
        hipError_t e = allow_wave_lds(wave_svd_kernel_f32<NC, ML>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((wave_svd_kernel_f32<NC, ML>), dim3(grid), dim3(a.d.threads), lds, st, a);
    } else {
        hipError_t e = allow_wave_lds(wave_svd_kernel<R, NC, ML>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((wave_svd_kernel<R, NC, ML>), dim3(grid), dim3(a.d.threads), lds, st, a);
    }
    return hipGetLastError();
}

template <typename R, int NC, int ML>
int wave_blocks_t(int threads, bool vectors) {
    const size_t base = (wave_lds_bytes<R, NC, ML>() + 63) & ~size_t(63);
    const size_t lds = vectors ? base + wave_stage_bytes<R, NC, ML>() : base;
    int blocks = 0;
    hipError_t e;
    if constexpr (sizeof(R) == 4) {
        if (allow_wave_lds(wave_svd_kernel_f32<NC, ML>, lds) != hipSuccess) return 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &blocks, reinterpret_cast<const void*>(wave_svd_kernel_f32<NC, ML>), threads, lds);
    } else {
        if (allow_wave_lds(wave_svd_kernel<R, NC, ML>, lds) != hipSuccess) return 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &blocks, reinterpret_cast<const void*>(wave_svd_kernel<R, NC, ML>), threads, lds);
    }
    return e == hipSuccess ? blocks : 0;
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

int wave_blocks_per_cu(int nc, int ml, int elem_bytes, int threads, bool vectors) {
#define LFA_CASE(n_, m_)                                                                \
    if (nc == n_ && ml == m_)                                                           \
        return elem_bytes == 8 ? wave_blocks_t<double, n_, m_>(threads, vectors)        \
                               : wave_blocks_t<float, n_, m_>(threads, vectors);
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
