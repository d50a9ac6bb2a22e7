// Host check of qf::FastDiv (Granlund-Montgomery division by an invariant
// divisor) against plain division, including divisors above 2^31.
#include <cstdio>
#include <cstdint>
#include <vector>

#include "../paper_2409_17716_amd/csrc/qf_common.h"

namespace qf {
qf_status set_error(qf_status st, const char*, ...) { return st; }
}

int main() {
    const std::vector<uint32_t> divs = {1u, 2u, 3u, 5u, 7u, 10u, 59049u, 43046721u, 1162261467u, 2147483647u,
                                        2147483648u, 2147483649u, 3486784401u, 4294967295u};
    std::vector<uint32_t> nums = {0u, 1u, 2u, 3u, 4294967295u, 4294967294u, 2147483647u, 2147483648u, 3486784400u,
                                  3486784401u, 3486784402u, 43046720u, 43046721u, 129140162u};
    uint64_t x = 88172645463325252ull;
    for (int i = 0; i < 200000; ++i) {
        x ^= x << 13;
        x ^= x >> 7;
        x ^= x << 17;
        nums.push_back(uint32_t(x));
    }
    long bad = 0;
    for (uint32_t d : divs) {
        qf::FastDiv f(d);
        std::vector<uint32_t> ns = nums;
        for (uint32_t k = 1; k < 4; ++k) {  // multiples of d and their neighbours
            const uint64_t m = uint64_t(d) * k;
            if (m <= 0xffffffffull) ns.push_back(uint32_t(m));
            if (m - 1 <= 0xffffffffull) ns.push_back(uint32_t(m - 1));
            if (m + 1 <= 0xffffffffull) ns.push_back(uint32_t(m + 1));
        }
        for (uint32_t n : ns)
            if (f.div_host(n) != n / d) {
                if (bad < 10) std::printf("FAIL d=%u n=%u got %u want %u\n", d, n, f.div_host(n), n / d);
                ++bad;
            }
    }
    std::printf("%s (%ld mismatches)\n", bad ? "FAIL" : "OK", bad);
    return bad ? 1 : 0;
}
