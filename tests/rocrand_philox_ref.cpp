// Reference Philox4x32-10 blocks from rocRAND's header-only device API,
// compiled for the host.  Used only to pin the oracle's Philox.
// Input lines on stdin: seed subsequence offset count
// Output: one line of four hex words per generated block.
#include <rocrand/rocrand_kernel.h>
#include <cstdio>

int main() {
    unsigned long long seed, subseq, offset;
    int count;
    while (std::scanf("%llu %llu %llu %d", &seed, &subseq, &offset, &count) == 4) {
        rocrand_state_philox4x32_10 s;
        rocrand_init(seed, subseq, offset, &s);
        for (int i = 0; i < count; ++i) {
            uint4 v = rocrand4(&s);
            std::printf("%08x %08x %08x %08x\n", v.x, v.y, v.z, v.w);
        }
    }
    return 0;
}
