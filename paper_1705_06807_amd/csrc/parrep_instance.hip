// parrep_instance.hip -- explicit instantiations of the instance kernel for
// one species count and one workgroup size (PARREP_NS species padded,
// PARREP_WAVES 64-lane waves); compiled once per pair so the variants build
// in parallel.
#include "parrep_device.h"

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
template <int NS, int M, int RPL, int WAVES>
hipError_t launch_instance(const DevInst* d, int n, int mode, uint32_t hc, int64_t hmr,
                           int tab_lds, int stage, long long spec, hipStream_t st) {
    // the exchange buffer, the tables, and the histogram tile of instances
    // that stage it
    const size_t lead = (xbuf_lds_bytes(RPL, WAVES, NS) / 4 + 1) / 2 * 8;
    const size_t lds = lead + (size_t)tab_lds * 8 + (stage ? (size_t)kTileDoubles * 8 : 0);
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
                     int tab_lds, int stage, long long spec, hipStream_t st) {
    constexpr int NS = PARREP_NS, WV = PARREP_WAVES;
    if (m <= 4) {
        switch (rpl) {
            case 1: return dev::launch_instance<NS, 4, 1, WV>(d, n, mode, hc, hmr, tab_lds, stage, spec, st);
            case 4: return dev::launch_instance<NS, 4, 4, WV>(d, n, mode, hc, hmr, tab_lds, stage, spec, st);
            case 16: return dev::launch_instance<NS, 4, 16, WV>(d, n, mode, hc, hmr, tab_lds, stage, spec, st);
            case 64:
                if constexpr (WV == 16)
                    return dev::launch_instance<NS, 4, 64, WV>(d, n, mode, hc, hmr, tab_lds, stage, spec, st);
                return hipErrorInvalidValue;
            default: return hipErrorInvalidValue;
        }
    }
    switch (rpl) {
        case 1: return dev::launch_instance<NS, 8, 1, WV>(d, n, mode, hc, hmr, tab_lds, stage, spec, st);
        case 4: return dev::launch_instance<NS, 8, 4, WV>(d, n, mode, hc, hmr, tab_lds, stage, spec, st);
        case 16: return dev::launch_instance<NS, 8, 16, WV>(d, n, mode, hc, hmr, tab_lds, stage, spec, st);
        case 64:
            if constexpr (WV == 16)
                return dev::launch_instance<NS, 8, 64, WV>(d, n, mode, hc, hmr, tab_lds, stage, spec, st);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

}  // namespace parrep
