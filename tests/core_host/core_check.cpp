// Host build of the device path's core arithmetic (hr_core.h), for CPU
// checks under AddressSanitizer and UndefinedBehaviorSanitizer: reads
// degree-1 instances from stdin, one per line "a b n lo D" (decimal), and
// prints for each
//   H <count> <k...>          every k < n with (b - lo - k a) mod 2^64 < D, in
//                             the walk's order (closest-point walk + predecessor
//                             steps, as the kernels run them)
//   L <success> <d> <iters>   Lefevre's test (swap form)
//   R <success> <d> <iters>   the regular test (unrolled)
// Built and driven by tests/test_core_host.py.
#include <cinttypes>
#include <cstdio>
#include <vector>

#include "../../paper_1211_3056_amd/csrc/hr_core.h"

int main() {
    uint64_t a, b, lo, D;
    uint32_t n;
    std::vector<uint64_t> ks;
    while (std::scanf("%" SCNu64 " %" SCNu64 " %" SCNu32 " %" SCNu64 " %" SCNu64, &a, &b, &n,
                      &lo, &D) == 5) {
        ks.clear();
        hr::search_each(a, b - lo, n, D, [&](uint64_t k) { ks.push_back(k); });
        std::printf("H %zu", ks.size());
        for (uint64_t k : ks) std::printf(" %" PRIu64, k);
        std::printf("\n");
        const hr::FilterOut l = hr::lefevre_filter(a, b - lo, n, D);
        std::printf("L %d %" PRIu64 " %u\n", l.success ? 1 : 0, l.d, l.iters);
        const hr::FilterOut r = hr::regular_filter(a, b - lo, n, D);
        std::printf("R %d %" PRIu64 " %u\n", r.success ? 1 : 0, r.d, r.iters);
    }
    return 0;
}
