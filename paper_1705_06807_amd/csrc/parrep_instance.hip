// parrep_instance.hip -- explicit instantiations of the instance kernel for
// one species count and one workgroup size (PARREP_NS species padded,
// PARREP_WAVES 64-lane waves); compiled once per pair so the variants build
// in parallel.
#include "parrep_device.h"

#include <algorithm>

#ifndef PARREP_NS
#error "PARREP_NS must be defined"
#endif
#ifndef PARREP_WAVES
#error "PARREP_WAVES must be defined"
#endif

namespace parrep {
namespace dev {
namespace {

// Dynamic LDS: the Fleming-Viot exchange buffer when it fits 32 KiB (the
// kernel applies the same rule), tab_lds doubles of propensity tables, and
// the histogram tile when the group's instances stage it.
// Zeroes the persistent launch's counter (a kernel, not a memset, so that a
// captured graph replays it reliably).
__global__ void k_set_zero(int* p) { *p = 0; }

// The persistent form of a solve launch: as many workgroups as the device
// holds at once (at most n), after the counter (the group's first
// descriptor's spare word) is zeroed.
template <int NS, int M, int RPL, int WAVES, long long SPEC>
hipError_t launch_persist(const DevInst* d, int n, int tab_lds, size_t lds, hipStream_t st) {
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void*>(&k_persist<NS, M, RPL, WAVES, SPEC>),
            64 * WAVES, lds);
    if (e != hipSuccess) return e;
    const int64_t cap = (int64_t)std::max(1, per_cu) * std::max(1, cus);
    const int grid = (int)std::min<int64_t>(n, cap);
    int* next = &const_cast<DevInst*>(d)->reserved2;
    hipLaunchKernelGGL(k_set_zero, dim3(1), dim3(1), 0, st, next);
    hipLaunchKernelGGL((k_persist<NS, M, RPL, WAVES, SPEC>), dim3(grid), dim3(64 * WAVES), lds, st,
                       d, n, next, tab_lds);
    return hipGetLastError();
}

template <int NS, int M, int RPL, int WAVES>
hipError_t launch_instance(const DevInst* d, int n, int mode, uint32_t hc, int64_t hmr,
                           int tab_lds, int stage, long long spec, int persist, hipStream_t st) {
    // the exchange buffer, the tables, and the histogram tile of instances
    // that stage it
    const size_t lead = (xbuf_lds_bytes(RPL, WAVES, NS) / 4 + 1) / 2 * 8;
    const size_t lds = lead + (size_t)tab_lds * 8 + (stage ? (size_t)kTileDoubles * 8 : 0);
    if (persist && mode == kModeSolve && !stage) {
        if constexpr (NS == 2 && M == 4)
            if (spec == kMapCross) return launch_persist<NS, M, RPL, WAVES, kMapCross>(d, n, tab_lds, lds, st);
        if constexpr (NS == 4 && M == 8 && RPL <= 4)
            if (spec == kDescSwitch) return launch_persist<NS, M, RPL, WAVES, kDescSwitch>(d, n, tab_lds, lds, st);
        if (spec >= 0) return hipErrorInvalidValue;
        return launch_persist<NS, M, RPL, WAVES, -1>(d, n, tab_lds, lds, st);
    }
    // the staging builds: narrow kernels with at most 4 replicas per lane and
    // 4 waves (the host stages no other shape)
    if (stage) {
        if constexpr (narrow_kernel(NS, M) && RPL <= 4 && WAVES <= 4) {
            if constexpr (NS == 2 && M == 4) {
                if (spec == kMapCross) {
                    hipLaunchKernelGGL((k_instance<NS, M, RPL, WAVES, kMapCross, true>), dim3(n),
                                       dim3(64 * WAVES), lds, st, d, mode, hc, hmr, tab_lds);
                    return hipGetLastError();
                }
            }
            if (spec >= 0) return hipErrorInvalidValue;
            hipLaunchKernelGGL((k_instance<NS, M, RPL, WAVES, -1, true>), dim3(n), dim3(64 * WAVES),
                               lds, st, d, mode, hc, hmr, tab_lds);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    if constexpr (NS == 2 && M == 4) {
        if (spec == kMapCross) {
            hipLaunchKernelGGL((k_instance<NS, M, RPL, WAVES, kMapCross>), dim3(n),
                               dim3(64 * WAVES), lds, st, d, mode, hc, hmr, tab_lds);
            return hipGetLastError();
        }
    }
    if constexpr (NS == 4 && M == 8 && RPL <= 4) {
        if (spec == kDescSwitch) {
            hipLaunchKernelGGL((k_instance<NS, M, RPL, WAVES, kDescSwitch>), dim3(n),
                               dim3(64 * WAVES), lds, st, d, mode, hc, hmr, tab_lds);
            return hipGetLastError();
        }
    }
    if (spec >= 0) return hipErrorInvalidValue;  // no such specialisation compiled
    hipLaunchKernelGGL((k_instance<NS, M, RPL, WAVES>), dim3(n), dim3(64 * WAVES), lds, st, d,
                       mode, hc, hmr, tab_lds);
    return hipGetLastError();
}

}  // namespace
}  // namespace dev

#define PARREP_CAT2(a, b, c, d) a##b##c##d
#define PARREP_CAT(a, b, c, d) PARREP_CAT2(a, b, c, d)
#define PARREP_FN PARREP_CAT(launch_instance_ns, PARREP_NS, _w, PARREP_WAVES)

hipError_t PARREP_FN(const DevInst* d, int n, int m, int rpl, int mode, uint32_t hc, int64_t hmr,
                     int tab_lds, int stage, long long spec, int persist, hipStream_t st) {
    constexpr int NS = PARREP_NS, WV = PARREP_WAVES;
    if (m <= 4) {
        switch (rpl) {
            case 1: return dev::launch_instance<NS, 4, 1, WV>(d, n, mode, hc, hmr, tab_lds, stage, spec, persist, st);
            case 4: return dev::launch_instance<NS, 4, 4, WV>(d, n, mode, hc, hmr, tab_lds, stage, spec, persist, st);
            case 16: return dev::launch_instance<NS, 4, 16, WV>(d, n, mode, hc, hmr, tab_lds, stage, spec, persist, st);
            case 64:
                if constexpr (WV == 16)
                    return dev::launch_instance<NS, 4, 64, WV>(d, n, mode, hc, hmr, tab_lds, stage, spec, persist, st);
                return hipErrorInvalidValue;
            default: return hipErrorInvalidValue;
        }
    }
    switch (rpl) {
        case 1: return dev::launch_instance<NS, 8, 1, WV>(d, n, mode, hc, hmr, tab_lds, stage, spec, persist, st);
        case 4: return dev::launch_instance<NS, 8, 4, WV>(d, n, mode, hc, hmr, tab_lds, stage, spec, persist, st);
        case 16: return dev::launch_instance<NS, 8, 16, WV>(d, n, mode, hc, hmr, tab_lds, stage, spec, persist, st);
        case 64:
            if constexpr (WV == 16)
                return dev::launch_instance<NS, 8, 64, WV>(d, n, mode, hc, hmr, tab_lds, stage, spec, persist, st);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

}  // namespace parrep
