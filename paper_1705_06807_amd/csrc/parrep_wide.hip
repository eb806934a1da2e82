// parrep_wide.hip -- launchers of the wide instance kernel (one ParRep
// instance over the workgroups of a cooperative launch) for one species
// count (PARREP_NS); compiled once per count so the variants build in
// parallel.
#include "parrep_wide.h"

#ifndef PARREP_NS
#error "PARREP_NS must be defined"
#endif

namespace parrep {
namespace dev {
namespace {

template <int NS, int M, int RPL>
hipError_t launch_wide_t(const DevInst* d, int G, int tab_lds, hipStream_t st) {
    const size_t lds = (size_t)tab_lds * 8;
    void* args[] = {(void*)&d, (void*)&tab_lds};
    return hipLaunchCooperativeKernel((const void*)&k_wide<NS, M, RPL, 4>, dim3(G), dim3(256),
                                      args, (unsigned int)lds, st);
}

}  // namespace
}  // namespace dev

#define PARREP_CAT2(a, b) a##b
#define PARREP_CAT(a, b) PARREP_CAT2(a, b)
#define PARREP_FN PARREP_CAT(launch_wide_ns, PARREP_NS)

hipError_t PARREP_FN(const DevInst* d, int G, int m, int rpl, int tab_lds, hipStream_t st) {
    constexpr int NS = PARREP_NS;
    if (m <= 4) {
        if (rpl == 1) return dev::launch_wide_t<NS, 4, 1>(d, G, tab_lds, st);
        if (rpl == 4) return dev::launch_wide_t<NS, 4, 4>(d, G, tab_lds, st);
        return hipErrorInvalidValue;
    }
    if (rpl == 1) return dev::launch_wide_t<NS, 8, 1>(d, G, tab_lds, st);
    if (rpl == 4) return dev::launch_wide_t<NS, 8, 4>(d, G, tab_lds, st);
    return hipErrorInvalidValue;
}

}  // namespace parrep
