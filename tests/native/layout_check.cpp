// Host check of the storage index maps used by the kernels (built with hipcc, run on the CPU):
// for natural and colour-split layouts, lidx is a bijection onto [0, cells) and ldecode inverts
// it; the colour-split rows hold the red cells, (x+y+z) even, first.
#include <cstdio>
#include <vector>
#include "mg_internal.h"

using namespace mgic;

int main() {
    const int shapes[][3] = {{2, 2, 2}, {4, 4, 4}, {6, 6, 6}, {8, 8, 8}, {16, 16, 16}, {12, 16, 20},
                             {24, 16, 32}, {3, 3, 3}, {5, 7, 9}, {48, 48, 48}, {64, 32, 16}, {1, 1, 1}};
    long long bad = 0;
    for (auto& s : shapes) {
        for (int split = 0; split < 2; ++split) {
            if (split && (s[2] % 2)) continue;
            const Lay L = mklay(Dims{s[0], s[1], s[2]}, split);
            const size_t n = L.d.cells();
            std::vector<int> seen(n, 0);
            for (int x = 0; x < s[0]; ++x)
                for (int y = 0; y < s[1]; ++y)
                    for (int z = 0; z < s[2]; ++z) {
                        const size_t i = lidx(L, x, y, z);
                        if (i >= n) { ++bad; continue; }
                        ++seen[i];
                        int a, b, c;
                        ldecode(L, i, a, b, c);
                        if (a != x || b != y || c != z) ++bad;
                        if (split) {
                            const int red = ((x + y + z) & 1) == 0;
                            const size_t pos = i % (size_t)s[2];
                            if (red != (pos < (size_t)(s[2] / 2))) ++bad;
                        }
                    }
            for (size_t i = 0; i < n; ++i)
                if (seen[i] != 1) ++bad;
        }
    }
    printf("mismatches %lld\n", bad);
    return bad ? 1 : 0;
}
