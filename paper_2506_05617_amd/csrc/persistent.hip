// Persistent launch of the SVD of every layer of a plan: 256-thread
// work-groups, about one per CU, take items from a device work list ordered
// longest first (the host builds it; see WorkItem).  Small symbols (at most
// 64 rows, no rotation accumulator) run as "bundles": each wave of the
// work-group runs the register kernel on its own symbols with wave-local
// synchronisation (writing the side of the vectors its working matrix gives,
// if wanted, through its own staging LDS).  Larger
// symbols run the blocked kernel, one row (or two) per thread, by teams of
// W work-groups whose members are consecutive in the list; a team waits only
// for members that were taken before it, and every work-group of the grid is
// resident, so the earliest unfinished team always has all its members
// running.
#include <hip/hip_runtime.h>

#include "jacobi_device.hpp"

namespace lfa {
namespace {
using namespace dev;

template <typename R>
__device__ void run_bundle(const SvdArgs<R>& a, char* lds, int base, int wave_slots, int wave_lds) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (wave >= wave_slots) return;
    char* my = lds + (size_t)wave * wave_lds;
    const int spw = 64 / a.d.wave_ml;
    const int b = base + wave * spw;
    if (b >= item_count(a)) return;
    const int NC = a.d.wave_nc, ML = a.d.wave_ml;
#define LFA_CASE(nc, ml) \
    if (NC == nc && ML == ml) {                                      \
        (void)wave_group<R, nc, ml>(a, my, b, lane, 64, true);          \
        return;                                                         \
    }
    LFA_CASE(4, 16) LFA_CASE(8, 16) LFA_CASE(16, 16)
    LFA_CASE(4, 32) LFA_CASE(8, 32) LFA_CASE(16, 32) LFA_CASE(32, 32)
    LFA_CASE(4, 64) LFA_CASE(8, 64) LFA_CASE(16, 64) LFA_CASE(32, 64) LFA_CASE(64, 64)
#undef LFA_CASE
}

// ACC: the blocked items keep the accumulator (singular vectors wanted);
// bundles of the register kernel occur only without it.
template <typename R, bool ACC>
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
    // optional record of this work-group's busy time (from taking an item
    // to finishing it) and of the compute unit it ran on
    long long busy = 0, taken = 0, t_item = 0;
    for (;;) {
        if (threadIdx.x == 0) {
            if (pa.busy && t_item) busy += (long long)(wall_clock64() - t_item);
            item_sh = atomicAdd(pa.counter, 1);
            if (pa.busy) t_item = (long long)wall_clock64();
        }
        __syncthreads();
        const int idx = item_sh;
        __syncthreads();
        if (idx >= pa.num_items) {
            if (pa.busy && threadIdx.x == 0) {
                long long* r = pa.busy + 4 * (size_t)blockIdx.x;
                r[0] = busy;
                r[1] = taken;
                r[2] = (long long)__builtin_amdgcn_s_getreg(20 | (0 << 6) | (3 << 11));    // XCC_ID
                r[3] = (long long)(__builtin_amdgcn_s_getreg(4 | (0 << 6) | (31 << 11)) & 0xff00u);   // HW_ID: CU, SH, SE
            }
            break;
        }
        ++taken;
        const WorkItem w = pa.items[idx];
        const SvdArgs<R>& a = pa.layer[w.layer];
        if (w.kind == 0) {
            if constexpr (!ACC) run_bundle<R>(a, lds, w.item, pa.wave_slots, pa.wave_lds);
            __syncthreads();
        } else {
            Team team;
            team.member = w.member;
            team.W = w.W;
            team.bar = pa.team_counters + 4 * w.team;
            team.rot = pa.team_counters + 4 * w.team + 1;
            team.err = pa.team_counters + 4 * pa.num_teams;
            team.target = 0;
            char* gslot = a.gws + (size_t)w.item * a.slot_bytes;
            constexpr bool TRACK = !ACC && sizeof(R) == 4;
            if (a.d.M > 256) {
                block_one<R, 2, ACC, TRACK, false, false>(a, lds, w.item, gslot, team);
            } else if constexpr (TRACK) {
                // a work-group of its own: two block pairs per cross step
                if (w.W == 1) block_one<R, 1, ACC, TRACK, true, false>(a, lds, w.item, gslot, team);
                else block_one<R, 1, ACC, TRACK, false, false>(a, lds, w.item, gslot, team);
            } else {
                block_one<R, 1, ACC, TRACK, false, false>(a, lds, w.item, gslot, team);
            }
        }
    }
}

template <typename K>
hipError_t allow_lds_p(K kernel, size_t lds) {
    if (lds <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <typename R, bool ACC>
hipError_t launch_p(const PersistentArgs<R>& a, int grid, size_t lds, hipStream_t s) {
    hipError_t e = allow_lds_p(persistent_kernel<R, ACC>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((persistent_kernel<R, ACC>), dim3(grid), dim3(a.threads), lds, s, a);
    return hipGetLastError();
}

template <typename R, bool ACC>
int resident_p(size_t lds) {
    if (allow_lds_p(persistent_kernel<R, ACC>, lds) != hipSuccess) return 0;
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persistent_kernel<R, ACC>,
                                                     kPersistentThreads, lds) != hipSuccess)
        return 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return per_cu * cus;
}

}  // namespace

size_t persistent_lds_bytes(const LayerDesc* descs, int n, bool accumulate, bool bundle_vectors, int elem_bytes,
                            int wave_slots) {
    size_t lds = 0;
    for (int i = 0; i < n; ++i) {
        const LayerDesc& d = descs[i];
        if (d.kind == 1) {
            lds = std::max(lds, (size_t)wave_slots *
                                    wave_bundle_lds_for(d.wave_nc, d.wave_ml, elem_bytes, bundle_vectors));
        } else {
            LayerDesc db = d;
            db.threads = kPersistentThreads;
            lds = std::max(lds, block_lds_bytes(db, accumulate, elem_bytes));
        }
    }
    return lds;
}

int persistent_resident(size_t lds, int elem_bytes, bool accumulate) {
    if (elem_bytes == 8) return accumulate ? resident_p<double, true>(lds) : resident_p<double, false>(lds);
    return accumulate ? resident_p<float, true>(lds) : resident_p<float, false>(lds);
}

hipError_t launch_persistent_f32(const PersistentArgs<float>& a, int grid, size_t lds, bool accumulate,
                                 hipStream_t s) {
    return accumulate ? launch_p<float, true>(a, grid, lds, s) : launch_p<float, false>(a, grid, lds, s);
}
hipError_t launch_persistent_f64(const PersistentArgs<double>& a, int grid, size_t lds, bool accumulate,
                                 hipStream_t s) {
    return accumulate ? launch_p<double, true>(a, grid, lds, s) : launch_p<double, false>(a, grid, lds, s);
}

}  // namespace lfa
