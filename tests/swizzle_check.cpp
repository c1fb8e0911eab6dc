// Host check of the sliced bins' block-to-rows map (swizzle_block in gn_types.h):
// a bijection on [0, nb) for every block count, and blocks kSwizzle apart take
// consecutive logical blocks.  Built and run by test_swizzle_cpu.py.
#include "gn_types.h"

#include <cstdio>
#include <vector>

int main() {
    for (int nb = 0; nb <= 5000; ++nb) {
        std::vector<int> seen(nb, 0);
        for (int j = 0; j < nb; ++j) {
            const int l = swizzle_block(j, nb);
            if (l < 0 || l >= nb || seen[l]++) {
                std::printf("not a bijection: nb=%d j=%d -> %d\n", nb, j, l);
                return 1;
            }
            if (nb > kSwizzle && j + kSwizzle < nb && swizzle_block(j + kSwizzle, nb) != l + 1) {
                std::printf("not consecutive: nb=%d j=%d\n", nb, j);
                return 1;
            }
        }
    }
    std::printf("ok\n");
    return 0;
}
