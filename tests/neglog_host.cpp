// Host build of the device -log(u) routine, for its accuracy test: reads
// integers m (one per line, 1 <= m <= 2^53) and prints -log(m 2^-53) as a
// hex float.
#define PARREP_HD
#include "../paper_1705_06807_amd/csrc/parrep_neglog.h"

#include <cinttypes>
#include <cstdio>

int main() {
    double lt[parrep::kLogTabLen];
    parrep::build_log_table(lt);
    uint64_t m;
    while (std::scanf("%" SCNu64, &m) == 1) std::printf("%a\n", parrep::neglog_u53(m, lt));
    return 0;
}
