// Host run of the atom census's shared code (gn_atoms.h): the per-graph
// classification and the cycle-type enumeration, summed by Burnside's lemma on
// the CPU.  Prints "n connected irregular_discrete irregular_continuous
// regular_discrete regular_continuous" for n = 1 .. argv[1].
// "classify N" (8, 9 or 10) instead reads edge masks of N-vertex graphs from stdin (bit k =
// the k-th vertex pair i < j in lexicographic order) and prints, per graph,
// "connected regular class" with class -1 (not atomic), 0 (discrete) or 1
// (continuous), or -2 for a graph that is not connected.  "linecheck" (below)
// compares the nullity-one line test with the subset search.  Built and run
// by test_atoms_cpu.py; no GPU involved.
#include "gn_atoms.h"

#include <cstdio>
#include <cstdlib>
#include <cstring>

template <int N>
static int classify() {
    constexpr int S = AtomRows<N>::S;
    unsigned long long mask;
    while (std::scanf("%llu", &mask) == 1) {
        AtomRowsT<N> rows = 0;
        int k = 0;
        for (int i = 0; i < N; ++i)
            for (int j = i + 1; j < N; ++j, ++k)
                if ((mask >> k) & 1ull) {
                    rows |= (AtomRowsT<N>)1 << (S * i + j);
                    rows |= (AtomRowsT<N>)1 << (S * j + i);
                }
        const bool conn = atom_connected<N>(rows);
        std::printf("%d %d %d\n", conn ? 1 : 0, atom_regular<N>(rows) ? 1 : 0, conn ? atom_class<N>(rows) : -2);
    }
    return 0;
}

template <int N>
static int run() {
    long long nfact = 1;
    const std::vector<AtomCycleType> types = atom_cycle_types(N, nfact);
    long long sum[kAtomCounters] = {0, 0, 0, 0, 0};
    for (const AtomCycleType& t : types) {
        const int m = (int)t.orbit_rows.size();
        unsigned long long cnt[kAtomCounters] = {0u, 0u, 0u, 0u, 0u};
        for (uint64_t g = 0; g < (1ull << m); ++g) {
            AtomRowsT<N> rows = 0;
            for (int o = 0; o < m; ++o)
                if ((g >> o) & 1u) rows |= (AtomRowsT<N>)t.orbit_rows[o];
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

// "linecheck N count seed": random graphs on N vertices whose B, or twin
// quotient's B, has nullity one; prints "tested agreeing positive" for the
// closed-form line test against the subset search.
template <int N>
static int linecheck(long long iters, unsigned long long seed) {
    unsigned long long x = seed * 0x9E3779B97F4A7C15ull + 1ull;
    auto next = [&x]() {  // xorshift64*
        x ^= x >> 12;
        x ^= x << 25;
        x ^= x >> 27;
        return x * 0x2545F4914F6CDD1Dull;
    };
    constexpr int S = AtomRows<N>::S;
    static_assert(N * (N - 1) / 2 <= 64, "one random word per graph");
    long long tested = 0, agree = 0, positive = 0;
    for (long long it = 0; it < iters; ++it) {
        const unsigned long long m = next();
        AtomRowsT<N> rows = 0;
        int k = 0;
        for (int i = 0; i < N; ++i)
            for (int j = i + 1; j < N; ++j, ++k)
                if ((m >> k) & 1ull)
                    rows |= ((AtomRowsT<N>)1 << (S * i + j)) | ((AtomRowsT<N>)1 << (S * j + i));
        if (!atom_connected<N>(rows) || atom_nested<N>(rows)) continue;
        const int f = atom_class_first<N>(rows);
        if (f <= 0) continue;
        const AtomRowsT<N> q = atom_twin_quotient<N>(rows);
        AtomRowsT<N> sys = rows;
        int r = f;
        if (q != rows) {
            const int g = atom_class_first<N>(q);
            if (g <= 0) continue;
            sys = q;
            r = g;
        }
        if (r != N - 1) continue;
        ++tested;
        const int b = atom_subset_search<N>(sys, r);
        agree += atom_line_class<N>(sys) == b ? 1 : 0;
        positive += b > 0 ? 1 : 0;
    }
    std::printf("%lld %lld %lld\n", tested, agree, positive);
    return 0;
}

int main(int argc, char** argv) {
    if (argc > 4 && std::strcmp(argv[1], "linecheck") == 0) {
        const int n = std::atoi(argv[2]);
        const long long iters = std::atoll(argv[3]);
        const unsigned long long seed = std::strtoull(argv[4], nullptr, 10);
        if (n == 8) return linecheck<8>(iters, seed);
        if (n == 9) return linecheck<9>(iters, seed);
        if (n == 10) return linecheck<10>(iters, seed);
        return 2;
    }
    if (argc > 2 && std::strcmp(argv[1], "classify") == 0) {
        const int n = std::atoi(argv[2]);
        if (n == 8) return classify<8>();
        if (n == 9) return classify<9>();
        if (n == 10) return classify<10>();
        return 2;
    }
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
