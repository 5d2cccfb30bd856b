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

// ---------------------------------------------------------------- queue
// Work-queue launch: a grid of resident work-groups takes groups of symbols
// from a device queue and runs each for a few sweeps at a time; a group that
// is not finished saves its state and goes to the back of the queue.  Every
// group thus starts early and advances in turn, so the launch ends when the
// total work is done rather than when the last group dispatched in a final,
// partly filled round of work-groups is done.

// Next group for this work-group: 2 g + 1 for a fresh group g, 2 g for a
// saved one, -1 when there is no more work.  Thread 0 only.  The entry is
// polled with relaxed loads (an acquire load would invalidate this XCD's L2
// on every poll, slowing the work-groups that fill the queue) and acquired
// once it is seen.  The wait is bounded by the real-time clock (100 MHz).
__device__ int wave_queue_pop(int32_t* ctl, int groups, int cap, int32_t* info) {
    int32_t* ent = ctl + kWaveQueueCtl;
    const int i = __hip_atomic_fetch_add(&ctl[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (i < groups) return 2 * i + 1;
    const int j = i - groups;
    if (j >= cap) return -1;
    // entry j is filled by the work-group that runs the j-th requeued group;
    // when every group is done, no entry is filled any more
    const unsigned long long t0 = wall_clock64();
    for (;;) {
        const int v = __hip_atomic_load(&ent[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (v > 0) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            return 2 * (v - 1);
        }
        if (__hip_atomic_load(&ctl[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= groups) return -1;
        if (__hip_atomic_load(&ctl[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return -1;
        __builtin_amdgcn_s_sleep(32);
        if (wall_clock64() - t0 > 500000000ull) {
            // 5 s without an entry: report the layer as not converged, leave
            __hip_atomic_fetch_or(&ctl[3], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (info) atomicAdd(&info[LFA_INFO_NONCONVERGED], 1);
            return -1;
        }
    }
}

// Group g ran: count it as done, or queue it again (its state is saved and
// was released by every wave of the work-group).  Thread 0 only.
__device__ void wave_queue_push(int32_t* ctl, int g, bool finished, int cap, int32_t* info) {
    if (finished) {
        __hip_atomic_fetch_add(&ctl[2], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    const int j = __hip_atomic_fetch_add(&ctl[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (j < cap) {
        __hip_atomic_store(&ctl[kWaveQueueCtl + j], g + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        // cannot happen: cap bounds the requeues of every group
        __hip_atomic_fetch_or(&ctl[3], 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (info) atomicAdd(&info[LFA_INFO_NONCONVERGED], 1);
    }
}

template <typename R, int NC, int ML>
__device__ __forceinline__ void wave_queue_body(const SvdArgs<R>& a) {
    extern __shared__ __align__(16) char lds_raw[];
    using S = WaveShape<NC, ML>;
    // the next group's code, after the LDS of the wave group
    const size_t base = (wave_lds_bytes<R, NC, ML>() + 63) & ~size_t(63);
    int& item_sh = *reinterpret_cast<int*>(
        lds_raw + ((a.U || a.V) ? base + wave_stage_bytes<R, NC, ML>() : base));
    const int groups = (item_count(a) + S::SPW - 1) / S::SPW;
    const int nw = blockDim.x >> 6;
    quad<R>* state = static_cast<quad<R>*>(a.wq_state);
    // Thread 0 hands the group just run back (done or queued again) and takes
    // the next one in a single region at the top of the loop, and the loop
    // control is scalar: with a thread-0 region at the bottom of the loop
    // and a per-lane exit test, the compiler may give threads 1.. an inner
    // loop of their own that bypasses thread 0's hand-over.
    int prev = -1;              // 2 g + finished of the group just run, or -1
    for (;;) {
        if (threadIdx.x == 0) {
            if (prev >= 0) wave_queue_push(a.wq, prev >> 1, prev & 1, a.wq_cap, a.info);
            item_sh = wave_queue_pop(a.wq, groups, a.wq_cap, a.info);
        }
        __syncthreads();
        const int code = __builtin_amdgcn_readfirstlane(item_sh);
        __syncthreads();
        if (code < 0) break;
        const int g = code >> 1;
        // the saved state was acquired by thread 0 (the vector L1 and the L2
        // it invalidated are those of every wave of this work-group)
        const WaveSeg<R> sg{state + (size_t)g * nw * (NC / 2) * 64, a.wq_meta + (size_t)g * kWaveMeta,
                            code & 1, a.wq_seg};
        const bool fin = wave_group<R, NC, ML, true>(a, lds_raw, g * S::SPW, threadIdx.x, blockDim.x,
                                                     false, sg);
        prev = 2 * g + (fin ? 1 : 0);
    }
}

template <typename R, int NC, int ML>
__global__ void __launch_bounds__(128) wave_queue_kernel(SvdArgs<R> a) {
    wave_queue_body<R, NC, ML>(a);
}

template <int NC, int ML>
__global__ void __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(2, 2)))
wave_queue_kernel_f32(SvdArgs<float> a) {
    wave_queue_body<float, NC, ML>(a);
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

template <typename R, int NC, int ML>
size_t wave_launch_lds(bool vectors) {
    const size_t base = (wave_lds_bytes<R, NC, ML>() + 63) & ~size_t(63);
    return vectors ? base + wave_stage_bytes<R, NC, ML>() : base;
}

template <typename R, int NC, int ML>
const void* wave_queue_fn() {
    if constexpr (sizeof(R) == 4) return reinterpret_cast<const void*>(wave_queue_kernel_f32<NC, ML>);
    else return reinterpret_cast<const void*>(wave_queue_kernel<R, NC, ML>);
}

// LDS of the work-queue launch: the wave group's, then the next group's code
template <typename R, int NC, int ML>
size_t wave_queue_lds(bool vectors) {
    return wave_launch_lds<R, NC, ML>(vectors) + 16;
}

template <typename R, int NC, int ML>
hipError_t launch_wave_queue_t(const SvdArgs<R>& a, int grid, hipStream_t st) {
    const size_t lds = wave_queue_lds<R, NC, ML>(a.U || a.V);
    if constexpr (sizeof(R) == 4) {
        hipError_t e = allow_wave_lds(wave_queue_kernel_f32<NC, ML>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((wave_queue_kernel_f32<NC, ML>), dim3(grid), dim3(a.d.threads), lds, st, a);
    } else {
        hipError_t e = allow_wave_lds(wave_queue_kernel<R, NC, ML>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((wave_queue_kernel<R, NC, ML>), dim3(grid), dim3(a.d.threads), lds, st, a);
    }
    return hipGetLastError();
}

template <typename R, int NC, int ML>
int wave_queue_blocks_t(int threads, bool vectors) {
    const size_t lds = wave_queue_lds<R, NC, ML>(vectors);
    int blocks = 0;
    if constexpr (sizeof(R) == 4) {
        if (allow_wave_lds(wave_queue_kernel_f32<NC, ML>, lds) != hipSuccess) return 0;
    } else {
        if (allow_wave_lds(wave_queue_kernel<R, NC, ML>, lds) != hipSuccess) return 0;
    }
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, wave_queue_fn<R, NC, ML>(), threads, lds) !=
        hipSuccess)
        return 0;
    return blocks;
}

template <typename R>
hipError_t launch_wave_queue_any(const SvdArgs<R>& a, int grid, hipStream_t st) {
    const int NC = a.d.wave_nc, ML = a.d.wave_ml;
#define LFA_CASE(nc, ml) \
    if (NC == nc && ML == ml) return launch_wave_queue_t<R, nc, ml>(a, grid, st);
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

size_t wave_bundle_lds_for(int nc, int ml, int elem_bytes, bool vectors) {
    const size_t raw = wave_lds_bytes_for(nc, ml, elem_bytes);
    if (!vectors) return raw;
    size_t stage = 0;
#define LFA_CASE(n_, m_)                                                                             \
    if (nc == n_ && ml == m_)                                                                        \
        stage = elem_bytes == 8 ? wave_stage_bytes<double, n_, m_>() : wave_stage_bytes<float, n_, m_>();
    LFA_CASE(4, 16) LFA_CASE(8, 16) LFA_CASE(16, 16)
    LFA_CASE(4, 32) LFA_CASE(8, 32) LFA_CASE(16, 32) LFA_CASE(32, 32)
    LFA_CASE(4, 64) LFA_CASE(8, 64) LFA_CASE(16, 64) LFA_CASE(32, 64) LFA_CASE(64, 64)
#undef LFA_CASE
    return (((raw + 63) & ~size_t(63)) + stage + 63) & ~size_t(63);
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

int wave_queue_blocks_per_cu(int nc, int ml, int elem_bytes, int threads, bool vectors) {
#define LFA_CASE(n_, m_)                                                                      \
    if (nc == n_ && ml == m_)                                                                 \
        return elem_bytes == 8 ? wave_queue_blocks_t<double, n_, m_>(threads, vectors)        \
                               : wave_queue_blocks_t<float, n_, m_>(threads, vectors);
    LFA_CASE(4, 16) LFA_CASE(8, 16) LFA_CASE(16, 16)
    LFA_CASE(4, 32) LFA_CASE(8, 32) LFA_CASE(16, 32) LFA_CASE(32, 32)
    LFA_CASE(4, 64) LFA_CASE(8, 64) LFA_CASE(16, 64) LFA_CASE(32, 64) LFA_CASE(64, 64)
#undef LFA_CASE
    return 0;
}

hipError_t launch_wave_queue_f32(const SvdArgs<float>& a, int grid, hipStream_t s) {
    return launch_wave_queue_any<float>(a, grid, s);
}
hipError_t launch_wave_queue_f64(const SvdArgs<double>& a, int grid, hipStream_t s) {
    return launch_wave_queue_any<double>(a, grid, s);
}

hipError_t launch_wave_svd_f32(const SvdArgs<float>& a, int grid, hipStream_t s) {
    return launch_wave_any<float>(a, grid, s);
}
hipError_t launch_wave_svd_f64(const SvdArgs<double>& a, int grid, hipStream_t s) {
    return launch_wave_any<double>(a, grid, s);
}

}  // namespace lfa
