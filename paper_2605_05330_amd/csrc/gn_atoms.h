// Census of GN atoms: the per-graph classification and the enumeration of
// cycle types, shared by the census kernel and its host check (host and device).
// See gn_atoms.hip for the method.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>
#include <vector>

constexpr int kAtomMaxN = 10;

// A labelled graph as its adjacency rows packed at a fixed stride: row i (the
// neighbours of vertex i) in bits [S i, S i + S).  Up to 8 vertices the rows
// fit 8-bit fields of a 64-bit word; 9 and 10 vertices take N-bit fields of a
// 128-bit word (81 and 100 bits).
template <int N>
struct AtomRows {
    using type = std::conditional_t<(N <= 8), uint64_t, unsigned __int128>;
    static constexpr int S = N <= 8 ? 8 : N;
};
template <int N>
using AtomRowsT = typename AtomRows<N>::type;

// Neighbours of vertex i.
template <int N>
__host__ __device__ __forceinline__ unsigned atom_row(const AtomRowsT<N> rows, const int i) {
    constexpr int S = AtomRows<N>::S;
    return (unsigned)(rows >> (S * i)) & ((1u << S) - 1u);
}

// The packing stride for n vertices, for host code that takes n at run time.
inline int atom_stride(int n) { return n <= 8 ? 8 : n; }

// Per-graph counters: connected graphs, then atomic irregular discrete,
// irregular continuous, regular discrete, regular continuous.
constexpr int kAtomCounters = 5;

// Row p of M (p uniform per lane but not known at compile time: read with
// selects, so M stays in registers).
template <int N>
__host__ __device__ __forceinline__ void atom_row_of(const float (&M)[N][N + 1], const int p, float (&row)[N + 1]) {
#pragma unroll
    for (int j = 0; j <= N; ++j) {
        float v = 0.0f;
#pragma unroll
        for (int i = 0; i < N; ++i) v = i == p ? M[i][j] : v;
        row[j] = v;
    }
}

// Forward fraction-free elimination of [B_S | 1], B = A + I, S = the columns in
// `colmask` (the others read as zero).  pr[c]: pivot row of column c, or -1;
// used: the pivot rows; prev: the last pivot (the Bareiss divisor, D below).
template <int N>
__host__ __device__ __forceinline__ void atom_forward(const AtomRowsT<N> rows, const unsigned colmask,
                                                      float (&M)[N][N + 1], int (&pr)[N], unsigned& used, int& rank,
                                                      float& prev) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const unsigned ri = atom_row<N>(rows, i);
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const unsigned a = i == j ? 1u : (ri >> j) & 1u;
            M[i][j] = ((colmask >> j) & 1u) ? (float)a : 0.0f;
        }
        M[i][N] = 1.0f;
    }
    used = 0u;
    prev = 1.0f;
    rank = 0;
#pragma unroll
    for (int c = 0; c < N; ++c) {
        int p = -1;
#pragma unroll
        for (int i = 0; i < N; ++i)
            if (p < 0 && !((used >> i) & 1u) && M[i][c] != 0.0f) p = i;
        pr[c] = p;
        if (p >= 0) {
            used |= 1u << p;
            ++rank;
            float pv[N + 1];
            atom_row_of<N>(M, p, pv);
            const float pc = pv[c];
            const float inv = 1.0f / prev;
#pragma unroll
            for (int i = 0; i < N; ++i) {
                if ((used >> i) & 1u) continue;
                const float f = M[i][c];
#pragma unroll
                for (int j = c + 1; j <= N; ++j) M[i][j] = rintf((pc * M[i][j] - f * pv[j]) * inv);
                M[i][c] = 0.0f;
            }
            prev = pc;
        }
    }
}

// Fraction-free back substitution over the pivot columns: y_c = D x_c for
// the right-hand side sgn x column `rhs` of M (sgn = 1, rhs = N: B x = 1;
// sgn = 0: B x = 0) with x = 1 at column free_col (-1: none) and 0 at the
// other free columns.  Entries stay minors of [B | 1], so every step is exact
// in fp32.
template <int N>
__host__ __device__ __forceinline__ void atom_back(const float (&M)[N][N + 1], const int (&pr)[N], const float D,
                                                   const int rhs, const float sgn, const int free_col,
                                                   float (&y)[N]) {
#pragma unroll
    for (int c = N - 1; c >= 0; --c) {
        y[c] = c == free_col ? D : 0.0f;
        const int p = pr[c];
        if (p < 0) continue;
        float row[N + 1];
        atom_row_of<N>(M, p, row);
        float r = 0.0f;
#pragma unroll
        for (int j = 0; j <= N; ++j) r = j == rhs ? row[j] : r;
        float num = sgn * D * r;
#pragma unroll
        for (int j = c + 1; j < N; ++j) num -= row[j] * y[j];
        y[c] = rintf(num * (1.0f / row[c]));
    }
}

// Fraction-free elimination of [B_S | 1], B = A + I, S = the columns in
// `colmask` (the others read as zero); `rows` holds the adjacency rows.  rank:
// rank of B_S; consistent: 1 lies in the span of B_S.  When B_S has full column
// rank and the system is consistent, pos / neg receive the columns of S whose
// (unique) solution component is > 0 / < 0.
template <int N>
__host__ __device__ inline void atom_eliminate(const AtomRowsT<N> rows, const unsigned colmask, int& rank,
                                               bool& consistent, unsigned& pos, unsigned& neg) {
    float M[N][N + 1];
    int pr[N];
    unsigned used;
    float prev;
    atom_forward<N>(rows, colmask, M, pr, used, rank, prev);
    consistent = true;
#pragma unroll
    for (int i = 0; i < N; ++i)
        if (!((used >> i) & 1u) && M[i][N] != 0.0f) consistent = false;
    pos = 0u;
    neg = 0u;
    if (!consistent || rank != __builtin_popcount(colmask)) return;
    const float D = prev;
    float y[N];
    atom_back<N>(M, pr, D, N, 1.0f, -1, y);
    // accumulated in locals with selects: no store through a chosen output
    unsigned ps = 0u, ng = 0u;
#pragma unroll
    for (int c = 0; c < N; ++c) {
        const float s = pr[c] < 0 ? 0.0f : y[c] * D;
        ps |= s > 0.0f ? 1u << c : 0u;
        ng |= s < 0.0f ? 1u << c : 0u;
    }
    pos = ps;
    neg = ng;
}

// B of rank N - 1 with 1 in its span: the solutions are a line
// x(t) = (y_p + t y_z) / D (y_p: free column at 0; y_z: the kernel direction,
// free column at 1; both scaled by the last pivot D, integers below 2^9 in
// magnitude).  Some x(t) > 0 iff the components with y_z = 0 are positive and
// the lower bounds -y_p,i / y_z,i (y_z,i > 0) stay below the upper ones
// (y_z,i < 0), compared as exact fractions.  Returns 1 when it does, else -1.
template <int N>
__host__ __device__ __forceinline__ int atom_line_class(const AtomRowsT<N> rows) {
    float M[N][N + 1];
    int pr[N];
    unsigned used;
    int rank;
    float D;
    atom_forward<N>(rows, (1u << N) - 1u, M, pr, used, rank, D);
    int fc = 0;  // the free column
#pragma unroll
    for (int c = 0; c < N; ++c) fc = pr[c] < 0 ? c : fc;
    float yp[N], yz[N];
    atom_back<N>(M, pr, D, N, 1.0f, -1, yp);
    atom_back<N>(M, pr, D, N, 0.0f, fc, yz);
    const float s = D > 0.0f ? 1.0f : -1.0f;  // x(t) has the signs of s (y_p + t y_z)
    bool ok = true;
    float lo_n = -1.0f, lo_d = 0.0f;  // lower bound lo_n / lo_d, -infinity while lo_d = 0
    float hi_n = 1.0f, hi_d = 0.0f;   // upper bound, +infinity while hi_d = 0
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const float a = s * yp[i], b = s * yz[i];
        ok = ok && (b != 0.0f || a > 0.0f);
        // b > 0: t > -a / b;  b < 0: t < a / -b
        const bool up = b > 0.0f && (lo_d == 0.0f || -a * lo_d > lo_n * b);
        lo_n = up ? -a : lo_n;
        lo_d = up ? b : lo_d;
        const bool dn = b < 0.0f && (hi_d == 0.0f || a * hi_d < hi_n * -b);
        hi_n = dn ? a : hi_n;
        hi_d = dn ? -b : hi_d;
    }
    ok = ok && (lo_d == 0.0f || hi_d == 0.0f || lo_n * hi_d < hi_n * lo_d);
    return ok ? 1 : -1;
}

// Whether some closed neighbourhood strictly contains another.  Such a graph
// has no atom: with N[i] a proper subset of N[j] and x > 0, (B x)_j exceeds
// (B x)_i by the mass of N[j] \ N[i], so the two cannot both equal 1.  (Equal
// closed neighbourhoods, twins, are allowed.)
template <int N>
__host__ __device__ inline bool atom_nested(const AtomRowsT<N> rows) {
    unsigned c[N];
#pragma unroll
    for (int i = 0; i < N; ++i) c[i] = atom_row<N>(rows, i) | 1u << i;
    bool nested = false;
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j)
            if (j != i) nested = nested || ((c[i] & ~c[j]) == 0u && c[i] != c[j]);
    return nested;
}

// First part of the class of a connected graph, from the elimination of
// [B | 1]: -1 not atomic, 0 atomic and discrete, or the rank of B (>= 1) when B
// is singular and 1 lies in its span, which atom_singular_class decides.
template <int N>
__host__ __device__ __forceinline__ int atom_class_first(const AtomRowsT<N> rows) {
    constexpr unsigned full = (1u << N) - 1u;
    if (atom_nested<N>(rows)) return -1;
    int r;
    bool cons;
    unsigned pos, neg;
    atom_eliminate<N>(rows, full, r, cons, pos, neg);
    if (!cons) return -1;
    if (r == N) return pos == full ? 0 : -1;
    return r;
}

// Singular B of rank r with 1 in its span: whether the non-negative basic
// solutions of B x = 1 cover every vertex (returns 1), else -1.  The subsets of
// size r are walked in increasing order by the next-combination step (Gosper),
// so lanes of a wavefront with different ranks each eliminate their own subset
// in the same trip; a lane stops once its cover is complete.
template <int N>
__host__ __device__ __forceinline__ int atom_subset_search(const AtomRowsT<N> rows, const int r) {
    constexpr unsigned full = (1u << N) - 1u;
    unsigned cover = 0u;
    for (unsigned S = (1u << r) - 1u; S <= full;) {
        int r2;
        bool c2;
        unsigned p2, n2;
        atom_eliminate<N>(rows, S, r2, c2, p2, n2);
        if (r2 == r && c2 && n2 == 0u) cover |= p2;
        if (cover == full) break;
        const unsigned low = S & (0u - S);  // lowest set bit
        const unsigned up = S + low;
        S = up | (((up ^ S) >> 2) >> __builtin_ctz(low));
    }
    return cover == full ? 1 : -1;
}

// Twins (vertices with equal closed neighbourhoods) give B equal rows and
// equal columns, so B x = 1 depends on x only through the sums over twin
// classes, and it has a positive solution iff the system of the quotient graph
// does (one vertex per class, two classes adjacent when their vertices are;
// split each class's positive sum among its members).
// Returns the quotient's rows, its vertices numbered in the order of their
// smallest members and padded with isolated vertices up to N (an isolated
// vertex reads x = 1 and changes neither the existence of a positive solution
// nor the search over the rest); a graph without twins is its own quotient.
template <int N>
__host__ __device__ __forceinline__ AtomRowsT<N> atom_twin_quotient(const AtomRowsT<N> rows) {
    constexpr unsigned full = (1u << N) - 1u;
    constexpr int S = AtomRows<N>::S;
    unsigned c[N];
#pragma unroll
    for (int i = 0; i < N; ++i) c[i] = atom_row<N>(rows, i) | 1u << i;
    unsigned reps = 0u;  // the smallest vertex of each class
#pragma unroll
    for (int i = 0; i < N; ++i) {
        bool first = true;
#pragma unroll
        for (int j = 0; j < i; ++j) first = first && c[j] != c[i];
        reps |= first ? 1u << i : 0u;
    }
    if (reps == full) return rows;
    AtomRowsT<N> out = 0;
#pragma unroll
    for (int a = 0; a < N; ++a) {
        if (!((reps >> a) & 1u)) continue;
        const unsigned nb = c[a] & reps & ~(1u << a);  // representatives of the neighbouring classes
        unsigned row = 0u;
#pragma unroll
        for (int b = 0; b < N; ++b)
            row |= ((nb >> b) & 1u) << __builtin_popcount(reps & ((1u << b) - 1u));
        out |= (AtomRowsT<N>)row << (S * __builtin_popcount(reps & ((1u << a) - 1u)));
    }
    return out;
}

// Singular B of rank r with 1 in its span, decided where no subset search is
// needed: a graph with twins is decided on its twin quotient (smaller
// nullity; a quotient whose B is invertible answers at once), and a system of
// nullity 1 by atom_line_class.  Returns 1 (a positive solution exists), -1
// (none), or 0 with (sys, rank) the system left for atom_subset_search.
template <int N>
__host__ __device__ __forceinline__ int atom_singular_quick(const AtomRowsT<N> rows, const int r, AtomRowsT<N>& sys,
                                                            int& rank) {
    const AtomRowsT<N> q = atom_twin_quotient<N>(rows);
    sys = rows;
    rank = r;
    if (q != rows) {
        const int f = atom_class_first<N>(q);
        if (f <= 0) return f < 0 ? -1 : 1;
        sys = q;
        rank = f;
    }
    return rank == N - 1 ? atom_line_class<N>(sys) : 0;
}

// Singular B of rank r with 1 in its span: atomic (continuous, returns 1) iff
// B x = 1 has a positive solution, else -1.
template <int N>
__host__ __device__ inline int atom_singular_class(const AtomRowsT<N> rows, const int r) {
    AtomRowsT<N> sys;
    int rank;
    const int k = atom_singular_quick<N>(rows, r, sys, rank);
    return k != 0 ? k : atom_subset_search<N>(sys, rank);
}

// Class of one connected graph: -1 not atomic, else 0 discrete / 1 continuous.
template <int N>
__host__ __device__ inline int atom_class(const AtomRowsT<N> rows) {
    const int f = atom_class_first<N>(rows);
    return f <= 0 ? f : atom_singular_class<N>(rows, f);
}

// Whether the graph is connected, and whether it is regular.
template <int N>
__host__ __device__ inline bool atom_connected(const AtomRowsT<N> rows) {
    constexpr unsigned full = (1u << N) - 1u;
    unsigned reach = 1u;  // grow the set reachable from vertex 0
#pragma unroll
    for (int it = 0; it < N - 1; ++it) {
        unsigned nx = reach;
#pragma unroll
        for (int i = 0; i < N; ++i)
            if ((reach >> i) & 1u) nx |= atom_row<N>(rows, i);
        reach = nx;
    }
    return reach == full;
}

template <int N>
__host__ __device__ inline bool atom_regular(const AtomRowsT<N> rows) {
    const int d0 = __builtin_popcount(atom_row<N>(rows, 0));
    bool regular = true;
#pragma unroll
    for (int i = 1; i < N; ++i) regular = regular && __builtin_popcount(atom_row<N>(rows, i)) == d0;
    return regular;
}

// Adds an atomic class (0 discrete / 1 continuous) to the counters, with
// weight w.
__host__ __device__ inline void atom_count(const int cls, const bool regular, unsigned long long (&cnt)[kAtomCounters],
                                           const unsigned w = 1u) {
    const int idx = cls < 0 ? -1 : 1 + (regular ? 2 : 0) + cls;
#pragma unroll
    for (int k = 1; k < kAtomCounters; ++k) cnt[k] += idx == k ? w : 0u;  // fixed indices: no scratch array
}

// Weights of the marked-vertex sum: L^2 with L = lcm(1, ..., 10), so that
// L^2 / (k k') is an integer for any two counts k, k' <= 10.
constexpr unsigned kAtomLcm = 2520;
constexpr unsigned kAtomMarkW = kAtomLcm * kAtomLcm;

// Marked-vertex form of the identity's term of Burnside's sum (the number of
// labelled graphs with an invariant property P), two levels deep.  Mark a
// vertex of maximum degree d and relabel it 0 with neighbours A = {1..d};
// then mark a vertex of largest degree within A and relabel it 1 with
// neighbours {0} u {2..a+1} u {d+1..d+b}.  Counting each graph once per
// choice of marks (weight 1 / (k k')),
//     #{labelled G with P} = sum_{d,a,b} n C(n-1,d) d C(d-1,a) C(n-1-d,b)
//                            sum_G' P(G') / (k(G') k'(G')),
// G' over the graphs with those two neighbourhoods in which no vertex has
// degree above d and no vertex of A a degree above vertex 1's; k = the number
// of vertices of degree d, k' = those of A with vertex 1's degree.  For such a
// G' this returns true and w = L^2 / (k k'); false when G' is outside the sum.
template <int N>
__host__ __device__ inline bool atom_marked_weight(const AtomRowsT<N> rows, unsigned& w) {
    const unsigned A = atom_row<N>(rows, 0);  // {1..d}
    const int d0 = __builtin_popcount(A);
    const int d1 = __builtin_popcount(atom_row<N>(rows, 1));
    int k = 1, ka = 0;
    bool in = true;
#pragma unroll
    for (int v = 1; v < N; ++v) {
        const int dv = __builtin_popcount(atom_row<N>(rows, v));
        in = in && dv <= d0;
        k += dv == d0 ? 1 : 0;
        const bool ina = ((A >> v) & 1u) != 0u;
        in = in && (!ina || dv <= d1);
        ka += ina && dv == d1 ? 1 : 0;
    }
    w = kAtomMarkW / (unsigned)(k * (ka > 0 ? ka : 1));
    return in;
}

// Adds one labelled graph to the counters.
template <int N>
__host__ __device__ inline void atom_evaluate(const AtomRowsT<N> rows, unsigned long long (&cnt)[kAtomCounters]) {
    if (!atom_connected<N>(rows)) return;
    cnt[0] += 1u;
    atom_count(atom_class<N>(rows), atom_regular<N>(rows), cnt);
}

// One cycle type of the permutations of n vertices: its weight n!/z (the
// number of permutations of that type) and the orbits of a representative
// permutation on vertex pairs, each as adjacency rows packed at the stride of n
// (AtomRows; 128 bits hold every n up to 10, and for n <= 8 the low 64 are the
// packed rows themselves).
struct AtomCycleType {
    long long weight;
    std::vector<unsigned __int128> orbit_rows;
    bool identity;  // every cycle of length 1
};

inline void atom_partitions(int n, int maxp, std::vector<int>& cur, std::vector<std::vector<int>>& out) {
    if (n == 0) {
        out.push_back(cur);
        return;
    }
    for (int p = (n < maxp ? n : maxp); p >= 1; --p) {
        cur.push_back(p);
        atom_partitions(n - p, p, cur, out);
        cur.pop_back();
    }
}

// All cycle types of n vertices (1 <= n <= kAtomMaxN); nfact receives n!.
inline std::vector<AtomCycleType> atom_cycle_types(int n, long long& nfact) {
    std::vector<std::vector<int>> types;
    std::vector<int> cur;
    atom_partitions(n, n, cur, types);
    nfact = 1;
    for (int k = 2; k <= n; ++k) nfact *= k;
    std::vector<AtomCycleType> out;
    for (const auto& parts : types) {
        // representative permutation: cycles on consecutive vertices
        std::vector<int> perm(n);
        std::vector<int> mult(n + 1, 0);
        long long z = 1;
        int v = 0;
        for (int len : parts) {
            for (int k = 0; k < len; ++k) perm[v + k] = v + (k + 1) % len;
            v += len;
            z *= len;
            mult[len] += 1;
        }
        for (int len = 1; len <= n; ++len)
            for (int k = 2; k <= mult[len]; ++k) z *= k;
        AtomCycleType t;
        t.weight = nfact / z;
        t.identity = (int)parts.size() == n;
        std::vector<int> orbit(n * n, -1);
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) {
                if (orbit[i * n + j] >= 0) continue;
                const int o = (int)t.orbit_rows.size();
                const int S = atom_stride(n);
                unsigned __int128 rows = 0;
                int a = i, b = j;
                while (orbit[(a < b ? a : b) * n + (a < b ? b : a)] < 0) {
                    const int lo = a < b ? a : b, hi = a < b ? b : a;
                    orbit[lo * n + hi] = o;
                    rows |= (unsigned __int128)1 << (S * lo + hi);
                    rows |= (unsigned __int128)1 << (S * hi + lo);
                    a = perm[a];
                    b = perm[b];
                }
                t.orbit_rows.push_back(rows);
            }
        out.push_back(t);
    }
    return out;
}
