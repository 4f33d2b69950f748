// Host check of mgic::FastDiv against the hardware divider (built with g++ by tests/test_native.py).
#include <cstdio>
#include <cstdlib>
#include "fastdiv.h"

int main() {
    unsigned long long bad = 0, checked = 0;
    unsigned long long x = 88172645463325252ull;
    auto rnd = [&]() { x ^= x << 13; x ^= x >> 7; x ^= x << 17; return x; };
    // every divisor up to 4096, plus random large ones; n spans small, boundary and random values
    for (unsigned d = 1; d <= 4096 + 2000; ++d) {
        const unsigned dd = d <= 4096 ? d : (unsigned)(rnd() % 0x7fffffffu) + 1;
        const mgic::FastDiv f(dd);
        for (int k = 0; k < 3000; ++k) {
            unsigned n;
            if (k < 1000) n = (unsigned)k;
            else if (k < 1100) n = 0x7fffffffu - (unsigned)(k - 1000);
            else n = (unsigned)(rnd() % 0x80000000ull);
            ++checked;
            if (f.div(n) != n / dd || f.mod(n) != n % dd) {
                if (bad < 5) printf("mismatch d=%u n=%u: %u vs %u\n", dd, n, f.div(n), n / dd);
                ++bad;
            }
        }
    }
    printf("checked %llu, mismatches %llu\n", checked, bad);
    return bad ? 1 : 0;
}
