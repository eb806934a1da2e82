// Host build of the device -log(u) routine, for its accuracy test: reads
// integers m (one per line, 1 <= m <= 2^53) and prints -log(m 2^-53) as a
// hex float, then the same through the two-word entry (words hi:lo with
// (hi:lo >> 11) + 1 = m, the low 11 bits filled from m).
#define PARREP_HD
#include "../paper_1705_06807_amd/csrc/parrep_neglog.h"

#include <cinttypes>
#include <cstdio>

int main() {
    double lt[parrep::kLogTabLen];
    parrep::build_log_table(lt);
    uint64_t m;
    while (std::scanf("%" SCNu64, &m) == 1) {
        const uint64_t w = ((m - 1) << 11) | (m & 0x7FFu);
        std::printf("%a %a\n", parrep::neglog_u53(m, lt),
                    parrep::neglog_words53((uint32_t)(w >> 32), (uint32_t)w, lt));
    }
    return 0;
}
