// Kernel and launchers of the blocked kernel (symbols of more than 64 rows);
// the device code is in jacobi_device.hpp.
#include <hip/hip_runtime.h>

#include "jacobi_device.hpp"

namespace lfa {
namespace {
using namespace dev;

// The first main_wgs work-groups form teams of W (all resident at once when
// W > 1: the host sizes the grid from the occupancy of this kernel); team t
// owns slot t and works on items item0 + t, item0 + t + teams, ... below
// item_split.  The work-groups after them form teams of W2 for the items
// item_split .. item_end - 1 (the short last round of a launch with more
// items than resident work-groups): they are dispatched as the first
// symbols of the main part finish, and each such team starts once all its
// members are resident.
// DUAL: the main part has no teams (W = 1), and each cross step of its
// sweeps takes two block pairs (FP32 without the accumulator).
template <typename R, bool ACC, bool DUAL = false>
__global__ void __launch_bounds__(512) block_kernel(SvdArgs<R> a, int W, int item0, int item_split,
                                                    int32_t* counters, int main_wgs, int W2, int item_end) {
    extern __shared__ __align__(16) char lds[];
    constexpr bool TRACK = !ACC && sizeof(R) == 4;
    const int teams1 = main_wgs / W, teams2 = ((int)gridDim.x - main_wgs) / W2;
    int tix, member, wk, first, end, stride;
    if ((int)blockIdx.x < main_wgs) {
        tix = blockIdx.x / W;
        member = blockIdx.x - tix * W;
        wk = W;
        first = item0 + tix;
        end = item_split;
        stride = teams1;
    } else {
        const int b2 = blockIdx.x - main_wgs, t2 = b2 / W2;
        tix = teams1 + t2;
        member = b2 - t2 * W2;
        wk = W2;
        first = item_split + t2;
        end = item_end;
        stride = teams2;
    }
    Team team;
    team.member = member;
    team.W = wk;
    team.bar = counters + 4 * tix;
    team.rot = counters + 4 * tix + 1;
    team.err = counters + 4 * (teams1 + teams2);
    team.target = 0;
    char* gslot = a.gws + (size_t)tix * a.slot_bytes;
    end = min(item_count(a), end);
    if constexpr (DUAL) {
        if ((int)blockIdx.x < main_wgs) {
            for (int item = first; item < end; item += stride) block_one<R, 1, ACC, TRACK, true, !ACC>(a, lds, item, gslot, team);
            return;
        }
    }
    // the wider zero-column completion of the finish only without the
    // accumulator: beside it the registers spill into the sweeps
    for (int item = first; item < end; item += stride) block_one<R, 1, ACC, TRACK, false, !ACC>(a, lds, item, gslot, team);
}

// Dynamic LDS above 64 KiB needs an explicit per-kernel opt-in.
template <typename K>
hipError_t allow_lds(K kernel, size_t lds) {
    if (lds <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
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
    // BlockLds: wpart, wsum (two buffers), wprm (quads), wdsc, wnrm (FP64), rflag
    return lds_bytes_for(dg, accumulate, elem_bytes) +
           (size_t)elem_bytes * (nw * 64 * kBlkPST + 2 * nw * kWsumW + nw * kPrmW * 4 + nw * kDscW) +
           (size_t)8 * nw * kDscW + 8 + 16 + 64;
}

// teams x W work-groups on items item0 .. item_split - 1, then teams2 x W2
// on item_split .. item_end - 1 in the same grid (teams2 = 0: none).
template <typename R, bool ACC, bool DUAL>
hipError_t launch_block_k(const SvdArgs<R>& a, int teams, int W, int item0, int item_split, int teams2, int W2,
                          int item_end, int32_t* counters, hipStream_t st) {
    const size_t lds = block_lds_bytes(a.d, ACC, sizeof(R));
    hipError_t e = allow_lds(block_kernel<R, ACC, DUAL>, lds);
    if (e != hipSuccess) return e;
    e = launch_fill_i32(counters, 0, 4LL * (teams + teams2) + 4, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((block_kernel<R, ACC, DUAL>), dim3(teams * W + teams2 * W2), dim3(a.d.threads), lds, st, a,
                       W, item0, item_split, counters, teams * W, std::max(W2, 1), item_end);
    return hipGetLastError();
}

template <typename R, bool ACC>
hipError_t launch_block_t(const SvdArgs<R>& a, int teams, int W, int item0, int item_split, int teams2, int W2,
                          int item_end, int32_t* counters, hipStream_t st) {
    if constexpr (!ACC && sizeof(R) == 4) {
        if (W == 1)
            return launch_block_k<R, ACC, true>(a, teams, W, item0, item_split, teams2, W2, item_end, counters, st);
    }
    return launch_block_k<R, ACC, false>(a, teams, W, item0, item_split, teams2, W2, item_end, counters, st);
}

template <typename R>
hipError_t launch_block(const SvdArgs<R>& a, int teams, int W, int item0, int item_split, int teams2, int W2,
                        int item_end, int32_t* counters, hipStream_t st) {
    const bool acc = (a.d.transposed ? a.U : a.V) != nullptr;
    return acc ? launch_block_t<R, true>(a, teams, W, item0, item_split, teams2, W2, item_end, counters, st)
               : launch_block_t<R, false>(a, teams, W, item0, item_split, teams2, W2, item_end, counters, st);
}

template <typename R, bool ACC>
int block_resident_t(const LayerDesc& d) {
    const size_t lds = block_lds_bytes(d, ACC, sizeof(R));
    if (allow_lds(block_kernel<R, ACC>, lds) != hipSuccess) return 0;
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, block_kernel<R, ACC>, d.threads, lds) !=
        hipSuccess)
        return 0;
    if constexpr (!ACC && sizeof(R) == 4) {
        // the launch without teams runs the dual kernel: the fewer of the two
        int per_cu2 = 0;
        if (allow_lds(block_kernel<R, ACC, true>, lds) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu2, block_kernel<R, ACC, true>, d.threads, lds) !=
                hipSuccess)
            return 0;
        per_cu = std::min(per_cu, per_cu2);
    }
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return per_cu * cus;
}

hipError_t launch_block_svd_f32(const SvdArgs<float>& a, int teams, int W, int item0, int item_split, int teams2,
                                int W2, int item_end, int32_t* counters, hipStream_t s) {
    return launch_block<float>(a, teams, W, item0, item_split, teams2, W2, item_end, counters, s);
}
hipError_t launch_block_svd_f64(const SvdArgs<double>& a, int teams, int W, int item0, int item_split, int teams2,
                                int W2, int item_end, int32_t* counters, hipStream_t s) {
    return launch_block<double>(a, teams, W, item0, item_split, teams2, W2, item_end, counters, s);
}
int block_resident(const LayerDesc& d, bool acc, int elem_bytes) {
    if (elem_bytes == 8) return acc ? block_resident_t<double, true>(d) : block_resident_t<double, false>(d);
    return acc ? block_resident_t<float, true>(d) : block_resident_t<float, false>(d);
}

hipError_t launch_fill_i32(int32_t* p, int32_t value, long long count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int grid = (int)((count + 255) / 256 < 1024 ? (count + 255) / 256 : 1024);
    hipLaunchKernelGGL(fill_i32_kernel, dim3(grid), dim3(256), 0, s, p, value, count);
    return hipGetLastError();
}

}  // namespace lfa
