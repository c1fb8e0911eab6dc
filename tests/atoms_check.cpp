// Host run of the atom census's shared code (gn_atoms.h): the per-graph
// classification and the cycle-type enumeration, summed by Burnside's lemma on
// the CPU.  Prints "n connected irregular_discrete irregular_continuous
// regular_discrete regular_continuous" for n = 1 .. argv[1].  Built and run by
// test_atoms_cpu.py; no GPU involved.
#include "gn_atoms.h"

#include <cstdio>
#include <cstdlib>

template <int N>
static int run() {
    long long nfact = 1;
    const std::vector<AtomCycleType> types = atom_cycle_types(N, nfact);
    long long sum[kAtomCounters] = {0, 0, 0, 0, 0};
    for (const AtomCycleType& t : types) {
        const int m = (int)t.orbit_rows.size();
        unsigned cnt[kAtomCounters] = {0u, 0u, 0u, 0u, 0u};
        for (uint64_t g = 0; g < (1ull << m); ++g) {
            uint64_t rows = 0;
            for (int o = 0; o < m; ++o)
                if ((g >> o) & 1u) rows |= t.orbit_rows[o];
            atom_evaluate<N>(rows, cnt);
        }
        for (int k = 0; k < kAtomCounters; ++k) sum[k] += (long long)cnt[k] * t.weight;
    }
    for (int k = 0; k < kAtomCounters; ++k)
        if (sum[k] % nfact != 0) {
            std::printf("n=%d counter %d not a multiple of n!\n", N, k);
            return 1;
        }
    std::printf("%d %lld %lld %lld %lld %lld\n", N, sum[0] / nfact, sum[1] / nfact, sum[2] / nfact, sum[3] / nfact,
                sum[4] / nfact);
    return 0;
}

int main(int argc, char** argv) {
    const int nmax = argc > 1 ? std::atoi(argv[1]) : 6;
    int rc = 0;
    if (nmax >= 1) rc |= run<1>();
    if (nmax >= 2) rc |= run<2>();
    if (nmax >= 3) rc |= run<3>();
    if (nmax >= 4) rc |= run<4>();
    if (nmax >= 5) rc |= run<5>();
    if (nmax >= 6) rc |= run<6>();
    if (nmax >= 7) rc |= run<7>();
    if (nmax >= 8) rc |= run<8>();
    return rc;
}
