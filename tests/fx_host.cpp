// Host build of the device's 64.64 fixed-point clock, for its test: reads
// doubles (hex floats, one per line) and prints, for each, floor(d 2^64) as
// "hi lo" (hex); then the plain and the saturating sums of all of them, in
// input order, as "plain hi lo" and "sat hi lo"; then, over the first 1024
// values only (a workgroup's lanes), the three-part sum of the device's
// reductions joined by fx_join3 and the saturating sum, as "join3 hi lo"
// and "sat1024 hi lo".
#define PARREP_HD
#include "../paper_1705_06807_amd/csrc/parrep_fx.h"

#include <cinttypes>
#include <cstdio>
#include <cstdlib>

int main() {
    using namespace parrep;
    char buf[128];
    Fx plain{0, 0}, sat{0, 0}, sat1024{0, 0};
    uint64_t a = 0, b = 0, c = 0;
    int n = 0;
    while (std::fgets(buf, sizeof buf, stdin)) {
        const double d = std::strtod(buf, nullptr);
        const Fx v = fx_from(d);
        std::printf("%" PRIx64 " %" PRIx64 "\n", v.hi, v.lo);
        plain = fx_add(plain, v);
        sat = fx_add_sat(sat, v);
        if (n++ < 1024) {
            sat1024 = fx_add_sat(sat1024, v);
            a += v.hi;
            b += v.lo >> 32;
            c += v.lo & 0xFFFFFFFFull;
        }
    }
    const Fx j = fx_join3(a, b, c);
    std::printf("plain %" PRIx64 " %" PRIx64 "\n", plain.hi, plain.lo);
    std::printf("sat %" PRIx64 " %" PRIx64 "\n", sat.hi, sat.lo);
    std::printf("join3 %" PRIx64 " %" PRIx64 "\n", j.hi, j.lo);
    std::printf("sat1024 %" PRIx64 " %" PRIx64 "\n", sat1024.hi, sat1024.lo);
    return 0;
}
