// Census of GN atoms on connected graphs of up to 10 vertices (Appendix A,
// Table atoms_10).
//
// A fixed point of GN with full support on a connected graph is an atom; with
// B = A + I the atoms are the solutions x > 0 of B x = 1.  A connected graph is
// atomic when it has one; its spectrum is discrete when det B != 0 (the single
// point B^-1 1) and continuous otherwise.  The census counts, up to
// isomorphism, the connected graphs on n vertices and the atomic ones split
// into irregular / regular x discrete / continuous.
//
// Counting up to isomorphism without an isomorphism-free generator: every
// property counted here is invariant under relabelling, so by Burnside's
// lemma the number of isomorphism classes with the property is
//     (1/n!) sum over permutations p of #{labelled graphs fixed by p with it},
// and conjugate permutations fix isomorphic families, so the sum runs over
// cycle types with weights n!/z (z = prod_k k^{m_k} m_k!).  The graphs fixed
// by p are the unions of the orbits of p on vertex pairs; one GPU thread
// evaluates one such graph.  The identity fixes every labelled graph (2^45 at
// n = 10); its term is taken in a marked-vertex form instead, which fixes the
// neighbourhoods of two marked vertices and weights each graph by the number
// of ways to mark it (atom_marked_weight): about 2.5e10 graphs at n = 10.
//
// Deciding atomicity exactly: fraction-free (Bareiss) elimination of [B | 1].
// Every entry it produces is a minor of that 0/1 matrix (Sylvester's identity),
// at most 320 in magnitude for size <= 10, so products stay below 2^24 and fp32
// arithmetic is exact; each exact division is a multiply by the reciprocal and
// a round to the nearest integer.  When B is invertible the graph is atomic iff
// every component of B^-1 1 is positive.  When B is singular, the set
// P = {x >= 0 : B x = 1} is a polytope (B x = 1 with x >= 0 bounds x by 1); some
// point of P is positive iff the supports of P's vertices cover every vertex of
// the graph (the mean of one positive-in-i vertex per i is in P and positive).
// The vertices are the non-negative basic solutions: for every set S of
// rank(B) independent columns with B_S x_S = 1 solvable, x_S >= 0.  Exact
// shortcuts before that search: nested closed neighbourhoods rule an atom out,
// twins reduce the system to the twin quotient's, and a system of nullity one
// is decided on its line of solutions (gn_atoms.h).
#include <algorithm>
#include <cstring>
#include <vector>

#include "gn_atoms.h"
#include "gn_internal.h"

namespace {

constexpr int kAtomBlock = 256;

constexpr uint64_t kAtomChunk = 1ull << 24;  // graphs per first-pass launch (queue capacity)
static_assert(kAtomChunk <= (1ull << 24), "queue entries hold a graph's index within its chunk in 24 bits");

// Bytes of a graph index (one bit per orbit on vertex pairs): at most
// n(n - 1)/2 orbits, 45 at n = 10.
constexpr int kAtomTabBytes = (kAtomMaxN * (kAtomMaxN - 1) / 2 + 7) / 8;

template <int N>
__device__ __forceinline__ AtomRowsT<N> atom_rows(const AtomRowsT<N>* s_tab, int nbytes, uint64_t g) {
    AtomRowsT<N> rows = 0;
    for (int b = 0; b < nbytes; ++b) rows |= s_tab[b * 256 + ((g >> (8 * b)) & 255u)];
    return rows;
}

template <int N>
__device__ __forceinline__ void atom_load_tab(const unsigned __int128* __restrict__ tab, int nbytes,
                                              AtomRowsT<N>* s_tab) {
    for (int k = threadIdx.x; k < nbytes * 256; k += kAtomBlock) s_tab[k] = (AtomRowsT<N>)tab[k];
    __syncthreads();
}

template <int BT>
__device__ __forceinline__ void atom_flush(unsigned long long (&cnt)[kAtomCounters], unsigned long long* acc) {
    __shared__ unsigned long long s_red[BT / 64][kAtomCounters];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kAtomCounters; ++k) {
        unsigned long long v = cnt[k];
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) s_red[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < kAtomCounters) {
        unsigned long long t = 0;
        for (int w = 0; w < BT / 64; ++w) t += s_red[w][threadIdx.x];
        if (t) atomicAdd(acc + threadIdx.x, t);
    }
}

// Appends the lanes of a wavefront that `want` to a queue: one atomic per
// wavefront, entries in lane order.
__device__ __forceinline__ void atom_push(bool want, uint32_t entry, uint32_t* __restrict__ queue,
                                          unsigned* __restrict__ qcount) {
    const int lane = threadIdx.x & 63;
    const uint64_t mask = __ballot(want);
    if (!mask) return;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    unsigned at = 0u;
    if (lane == leader) at = atomicAdd(qcount, (unsigned)__popcll(mask));
    at = __shfl(at, leader, 64);
    if (want) queue[at + __popcll(mask & ((1ull << lane) - 1ull))] = entry;
}

// First pass, one thread per labelled graph g in [base, base + count): its
// edges are the orbits whose bits are set in g; `tab` holds, for each byte of
// g, the packed adjacency rows of every combination of that byte's orbits.
// Counts the connected graphs and queues those whose closed neighbourhoods
// are not nested (the others have no atom, atom_nested), as
// (g - base) | regular << 28: most graphs stop here, and the eliminations of
// the next pass run with every lane busy.
template <int N>
__global__ __launch_bounds__(kAtomBlock) void atom_census_kernel(const unsigned __int128* __restrict__ tab, int nbytes,
                                                                 uint64_t base, uint64_t count, int marked,
                                                                 unsigned long long* __restrict__ acc,
                                                                 uint32_t* __restrict__ queue,
                                                                 unsigned* __restrict__ qcount) {
    __shared__ AtomRowsT<N> s_tab[kAtomTabBytes * 256];
    atom_load_tab<N>(tab, nbytes, s_tab);
    unsigned long long cnt[kAtomCounters] = {0u, 0u, 0u, 0u, 0u};
    const uint64_t stride = (uint64_t)gridDim.x * kAtomBlock;
    for (uint64_t k = (uint64_t)blockIdx.x * kAtomBlock + threadIdx.x; k < count; k += stride) {
        const AtomRowsT<N> rows = atom_rows<N>(s_tab, nbytes, base + k);
        unsigned w = 1u;
        const bool in = !marked || atom_marked_weight<N>(rows, w);
        bool want = false;
        if (in && atom_connected<N>(rows)) {
            cnt[0] += w;
            want = !atom_nested<N>(rows);
        }
        atom_push(want, (uint32_t)k | (atom_regular<N>(rows) ? 1u << 28 : 0u), queue, qcount);
    }
    atom_flush<kAtomBlock>(cnt, acc);
}

// Second pass over the first's queue: one elimination of [B | 1] per graph.
// Counts the discrete atoms; a graph whose B is singular with 1 in its span
// goes to the next queue as (g - base) | rank << 24 | regular << 28.
template <int N>
__global__ __launch_bounds__(kAtomBlock) void atom_first_kernel(const unsigned __int128* __restrict__ tab, int nbytes,
                                                                uint64_t base, int marked, const uint32_t* __restrict__ qin,
                                                                const unsigned* __restrict__ qin_count,
                                                                unsigned long long* __restrict__ acc,
                                                                uint32_t* __restrict__ queue,
                                                                unsigned* __restrict__ qcount) {
    __shared__ AtomRowsT<N> s_tab[kAtomTabBytes * 256];
    atom_load_tab<N>(tab, nbytes, s_tab);
    unsigned long long cnt[kAtomCounters] = {0u, 0u, 0u, 0u, 0u};
    const unsigned total = *qin_count;
    const unsigned stride = gridDim.x * kAtomBlock;
    // the bound rounded up to whole wavefronts: every lane reaches the ballot of atom_push
    const unsigned bound = (total + 63u) & ~63u;
    for (unsigned i = blockIdx.x * kAtomBlock + threadIdx.x; i < bound; i += stride) {
        bool want = false;
        uint32_t entry = 0u;
        if (i < total) {
            const uint32_t e = qin[i];
            const bool regular = ((e >> 28) & 1u) != 0u;
            const AtomRowsT<N> rows = atom_rows<N>(s_tab, nbytes, base + (e & 0x00ffffffu));
            unsigned w = 1u;
            if (marked) (void)atom_marked_weight<N>(rows, w);
            const int f = atom_class_first<N>(rows);
            if (f == 0) atom_count(0, regular, cnt, w);
            want = f > 0;
            entry = (e & 0x00ffffffu) | (uint32_t)f << 24 | (regular ? 1u << 28 : 0u);
        }
        atom_push(want, entry, queue, qcount);
    }
    atom_flush<kAtomBlock>(cnt, acc);
}

// Third pass over the second's queue: the singular graphs decided without a
// subset search (twin quotient, nullity 1); the others go to the last queue as
// (g - base) | rank << 24 | regular << 28 | quotient << 29, the rank being
// that of the system left (the twin quotient's when the bit is set).
template <int N>
__global__ __launch_bounds__(kAtomBlock) void atom_singular_kernel(const unsigned __int128* __restrict__ tab, int nbytes,
                                                                   uint64_t base, int marked,
                                                                   const uint32_t* __restrict__ qin,
                                                                   const unsigned* __restrict__ qin_count,
                                                                   unsigned long long* __restrict__ acc,
                                                                   uint32_t* __restrict__ queue,
                                                                   unsigned* __restrict__ qcount) {
    __shared__ AtomRowsT<N> s_tab[kAtomTabBytes * 256];
    atom_load_tab<N>(tab, nbytes, s_tab);
    unsigned long long cnt[kAtomCounters] = {0u, 0u, 0u, 0u, 0u};
    const unsigned total = *qin_count;
    const unsigned stride = gridDim.x * kAtomBlock;
    const unsigned bound = (total + 63u) & ~63u;  // whole wavefronts reach the ballot of atom_push
    for (unsigned i = blockIdx.x * kAtomBlock + threadIdx.x; i < bound; i += stride) {
        bool want = false;
        uint32_t entry = 0u;
        if (i < total) {
            const uint32_t e = qin[i];
            const bool regular = ((e >> 28) & 1u) != 0u;
            const AtomRowsT<N> rows = atom_rows<N>(s_tab, nbytes, base + (e & 0x00ffffffu));
            unsigned w = 1u;
            if (marked) (void)atom_marked_weight<N>(rows, w);
            AtomRowsT<N> sys;
            int rank;
            const int k = atom_singular_quick<N>(rows, (int)((e >> 24) & 15u), sys, rank);
            if (k != 0) atom_count(k, regular, cnt, w);
            want = k == 0;
            entry = (e & 0x00ffffffu) | (uint32_t)rank << 24 | (regular ? 1u << 28 : 0u) |
                    (sys != rows ? 1u << 29 : 0u);
        }
        atom_push(want, entry, queue, qcount);
    }
    atom_flush<kAtomBlock>(cnt, acc);
}

// Column sets by size for the last pass (`subsets`): every mask of N bits,
// grouped by popcount in increasing order, then increasing; start[r] is the
// first of size r (start[N + 1] = 2^N).
// Last pass: the subset search for the systems of nullity 2 or more, one
// wavefront per graph.  The lanes take the column sets of size rank in turn,
// 64 at a time, and OR their covers after each round (the same cover as the
// one-lane search: a union over the same sets), stopping once it is complete.
template <int N>
__global__ __launch_bounds__(kAtomBlock) void atom_search_kernel(const unsigned __int128* __restrict__ tab, int nbytes,
                                                                 uint64_t base, int marked,
                                                                 const uint16_t* __restrict__ subsets,
                                                                 const int32_t* __restrict__ start,
                                                                 const uint32_t* __restrict__ queue,
                                                                 const unsigned* __restrict__ qcount,
                                                                 unsigned long long* __restrict__ acc) {
    __shared__ AtomRowsT<N> s_tab[kAtomTabBytes * 256];
    __shared__ uint16_t s_sub[1 << N];
    __shared__ int32_t s_start[N + 2];
    for (int k = threadIdx.x; k < (1 << N); k += kAtomBlock) s_sub[k] = subsets[k];
    if (threadIdx.x < N + 2) s_start[threadIdx.x] = start[threadIdx.x];
    atom_load_tab<N>(tab, nbytes, s_tab);
    constexpr unsigned full = (1u << N) - 1u;
    unsigned long long cnt[kAtomCounters] = {0u, 0u, 0u, 0u, 0u};
    const int lane = threadIdx.x & 63;
    const unsigned total = *qcount;
    const unsigned waves = gridDim.x * (kAtomBlock / 64);
    for (unsigned i = blockIdx.x * (kAtomBlock / 64) + (threadIdx.x >> 6); i < total; i += waves) {
        const uint32_t e = queue[i];
        const AtomRowsT<N> rows = atom_rows<N>(s_tab, nbytes, base + (e & 0x00ffffffu));
        const AtomRowsT<N> sys = ((e >> 29) & 1u) ? atom_twin_quotient<N>(rows) : rows;
        const int r = (int)((e >> 24) & 15u);
        const int s0 = s_start[r], s1 = s_start[r + 1];
        unsigned cover = 0u;
        for (int b = s0; b < s1; b += 64) {
            if (b + lane < s1) {
                int r2;
                bool c2;
                unsigned p2, n2;
                atom_eliminate<N>(sys, s_sub[b + lane], r2, c2, p2, n2);
                if (r2 == r && c2 && n2 == 0u) cover |= p2;
            }
            for (int off = 32; off >= 1; off >>= 1) cover |= __shfl_xor(cover, off, 64);
            if (cover == full) break;
        }
        if (lane == 0) {
            unsigned w = 1u;
            if (marked) (void)atom_marked_weight<N>(rows, w);
            atom_count(cover == full ? 1 : -1, ((e >> 28) & 1u) != 0u, cnt, w);
        }
    }
    atom_flush<kAtomBlock>(cnt, acc);
}

// The four passes over the graphs of one enumeration, a chunk of 2^24 at a
// time.  queue: three arrays of qcap >= min(count, kAtomChunk) entries;
// qcount: their three counters.
template <int N>
gn_status launch_census(const unsigned __int128* tab, int nbytes, uint64_t count, int marked,
                        const uint16_t* subsets, const int32_t* start, unsigned long long* acc,
                        uint32_t* queue, uint64_t qcap, unsigned* qcount, hipStream_t s) {
    uint32_t* q1 = queue;
    uint32_t* q2 = queue + qcap;
    uint32_t* q3 = queue + 2 * qcap;
    for (uint64_t base = 0; base < count; base += kAtomChunk) {
        const uint64_t c = std::min(kAtomChunk, count - base);
        GN_HIP_TRY(hipMemsetAsync(qcount, 0, 3 * sizeof(unsigned), s));
        const uint64_t blocks = std::min<uint64_t>((c + kAtomBlock - 1) / kAtomBlock, 256 * 64);
        const unsigned later = (unsigned)std::min<uint64_t>(blocks, 256 * 16);
        hipLaunchKernelGGL(atom_census_kernel<N>, dim3((unsigned)blocks), dim3(kAtomBlock), 0, s, tab, nbytes, base,
                           c, marked, acc, q1, qcount);
        GN_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(atom_first_kernel<N>, dim3(later), dim3(kAtomBlock), 0, s, tab, nbytes, base, marked,
                           (const uint32_t*)q1, (const unsigned*)qcount, acc, q2, qcount + 1);
        GN_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(atom_singular_kernel<N>, dim3(later), dim3(kAtomBlock), 0, s, tab, nbytes, base, marked,
                           (const uint32_t*)q2, (const unsigned*)(qcount + 1), acc, q3, qcount + 2);
        GN_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(atom_search_kernel<N>, dim3(later), dim3(kAtomBlock), 0, s, tab, nbytes, base, marked,
                           subsets, start, (const uint32_t*)q3, (const unsigned*)(qcount + 2), acc);
        GN_HIP_TRY(hipGetLastError());
    }
    return GN_OK;
}

gn_status launch_census_n(int n, const unsigned __int128* tab, int nbytes, uint64_t count, int marked,
                          const uint16_t* subsets, const int32_t* start, unsigned long long* acc, uint32_t* queue,
                          uint64_t qcap, unsigned* qcount, hipStream_t s) {
#define GN_ATOM_CASE(K) \
    case K: return launch_census<K>(tab, nbytes, count, marked, subsets, start, acc, queue, qcap, qcount, s);
    switch (n) {
        GN_ATOM_CASE(1)
        GN_ATOM_CASE(2)
        GN_ATOM_CASE(3)
        GN_ATOM_CASE(4)
        GN_ATOM_CASE(5)
        GN_ATOM_CASE(6)
        GN_ATOM_CASE(7)
        GN_ATOM_CASE(8)
        GN_ATOM_CASE(9)
        default: return launch_census<10>(tab, nbytes, count, marked, subsets, start, acc, queue, qcap, qcount, s);
    }
#undef GN_ATOM_CASE
}

// One enumeration: a family of labelled graphs, each the union of the base
// rows and the orbits selected by its index bits, and the factor its counts
// take in the final sum.
struct AtomJob {
    unsigned __int128 base;
    std::vector<unsigned __int128> orbit_rows;
    long long factor;
    int marked;  // 1: the marked-vertex form (weights L^2 / (k k')), else plain counts
};

}  // namespace

extern "C" gn_status gn_atom_census(int32_t n, gn_atom_counts* out, hipStream_t stream) {
    if (!out || n < 1 || n > kAtomMaxN) return GN_E_ARG;
    std::memset(out, 0, sizeof(*out));
    long long nfact = 1;
    const std::vector<AtomCycleType> types = atom_cycle_types(n, nfact);
    // Burnside's sum: the identity's term in the two-level marked-vertex form
    // (atom_marked_weight: one job per degree d of the first marked vertex and
    // per neighbourhood sizes a, b of the second), every other cycle type as the
    // unions of its orbits (factor: the number of permutations of the type)
    const int S = atom_stride(n);
    std::vector<AtomJob> jobs;
    for (const AtomCycleType& t : types) {
        if (!t.identity || n == 1) {
            jobs.push_back(AtomJob{0, t.orbit_rows, t.weight, 0});
            continue;
        }
        std::vector<unsigned __int128> rest;  // edges among vertices 2 .. n-1
        for (int i = 2; i < n; ++i)
            for (int j = i + 1; j < n; ++j)
                rest.push_back(((unsigned __int128)1 << (S * i + j)) | ((unsigned __int128)1 << (S * j + i)));
        auto edge = [S](int i, int j) {
            return ((unsigned __int128)1 << (S * i + j)) | ((unsigned __int128)1 << (S * j + i));
        };
        auto binom = [](int p, int q) {
            long long r = 1;
            for (int t = 1; t <= q; ++t) r = r * (p - q + t) / t;
            return r;
        };
        for (int d = 1; d < n; ++d)
            for (int a = 0; a < d; ++a)
                for (int b = 0; b <= n - 1 - d && 1 + a + b <= d; ++b) {
                    unsigned __int128 base = 0;  // N(0) = {1..d}, N(1) = {0} u {2..a+1} u {d+1..d+b}
                    for (int j = 1; j <= d; ++j) base |= edge(0, j);
                    for (int j = 2; j <= a + 1; ++j) base |= edge(1, j);
                    for (int j = d + 1; j <= d + b; ++j) base |= edge(1, j);
                    const long long factor =
                        (long long)n * binom(n - 1, d) * d * binom(d - 1, a) * binom(n - 1 - d, b);
                    jobs.push_back(AtomJob{base, rest, factor, 1});
                }
    }
    const size_t J = jobs.size();
    unsigned long long* acc = nullptr;  // per job: kAtomCounters counters
    unsigned __int128* tab = nullptr;   // per job: kAtomTabBytes x 256 packed adjacency rows
    uint32_t* queue = nullptr;          // three queues of one chunk: to eliminate, singular, to search
    unsigned* qcount = nullptr;         // their counters
    uint16_t* subsets = nullptr;        // the column sets of n bits by size (last pass)
    int32_t* start = nullptr;           // first set of each size, n + 2 entries
    auto release = [&]() {
        if (acc) (void)hipFree(acc);
        if (tab) (void)hipFree(tab);
        if (queue) (void)hipFree(queue);
        if (qcount) (void)hipFree(qcount);
        if (subsets) (void)hipFree(subsets);
        if (start) (void)hipFree(start);
    };
    uint64_t most = 0;
    for (const AtomJob& jb : jobs) most = std::max<uint64_t>(most, 1ull << jb.orbit_rows.size());
    const uint64_t qcap = std::min(most, kAtomChunk);
    if (hipMalloc((void**)&acc, sizeof(unsigned long long) * kAtomCounters * J) != hipSuccess ||
        hipMalloc((void**)&tab, sizeof(unsigned __int128) * kAtomTabBytes * 256 * J) != hipSuccess ||
        hipMalloc((void**)&queue, sizeof(uint32_t) * 3 * qcap) != hipSuccess ||
        hipMalloc((void**)&qcount, 3 * sizeof(unsigned)) != hipSuccess ||
        hipMalloc((void**)&subsets, sizeof(uint16_t) << n) != hipSuccess ||
        hipMalloc((void**)&start, sizeof(int32_t) * (n + 2)) != hipSuccess) {
        (void)hipGetLastError();
        release();
        return GN_E_NOMEM;
    }
    gn_status st = GN_OK;
    // per job and byte b of the graph index: the adjacency rows of every
    // combination of orbits 8b .. 8b + 7 (the base rows folded into byte 0)
    std::vector<unsigned __int128> htab(kAtomTabBytes * 256 * J, 0);
    std::vector<int> nbytes(J);
    std::vector<uint64_t> counts(J);
    for (size_t t = 0; t < J; ++t) {
        const int m = (int)jobs[t].orbit_rows.size();
        counts[t] = 1ull << m;
        nbytes[t] = m > 8 ? (m + 7) / 8 : 1;
        for (int b = 0; b < nbytes[t]; ++b)
            for (int c = 0; c < 256; ++c) {
                unsigned __int128 rows = b == 0 ? jobs[t].base : 0;
                for (int q = 0; q < 8; ++q)
                    if (((c >> q) & 1) && 8 * b + q < m) rows |= jobs[t].orbit_rows[8 * b + q];
                htab[(t * kAtomTabBytes + b) * 256 + c] = rows;
            }
    }
    std::vector<uint16_t> hsub;
    std::vector<int32_t> hstart;
    for (int r = 0; r <= n; ++r) {
        hstart.push_back((int32_t)hsub.size());
        for (int m = 0; m < (1 << n); ++m)
            if (__builtin_popcount((unsigned)m) == r) hsub.push_back((uint16_t)m);
    }
    hstart.push_back((int32_t)hsub.size());
    if (hipMemcpyAsync(tab, htab.data(), sizeof(unsigned __int128) * htab.size(), hipMemcpyHostToDevice, stream) !=
            hipSuccess ||
        hipMemcpyAsync(subsets, hsub.data(), sizeof(uint16_t) * hsub.size(), hipMemcpyHostToDevice, stream) !=
            hipSuccess ||
        hipMemcpyAsync(start, hstart.data(), sizeof(int32_t) * hstart.size(), hipMemcpyHostToDevice, stream) !=
            hipSuccess ||
        hipMemsetAsync(acc, 0, sizeof(unsigned long long) * kAtomCounters * J, stream) != hipSuccess)
        st = GN_E_HIP;
    for (size_t t = 0; t < J && st == GN_OK; ++t)
        st = launch_census_n(n, tab + t * kAtomTabBytes * 256, nbytes[t], counts[t], jobs[t].marked, subsets, start,
                             acc + t * kAtomCounters, queue, qcap, qcount, stream);
    std::vector<unsigned long long> h(kAtomCounters * J, 0);
    if (st == GN_OK &&
        (hipMemcpyAsync(h.data(), acc, sizeof(unsigned long long) * h.size(), hipMemcpyDeviceToHost, stream) !=
             hipSuccess ||
         hipStreamSynchronize(stream) != hipSuccess))
        st = GN_E_HIP;
    release();
    if (st != GN_OK) return st;
    // Burnside: the sums are n! times the class counts; the marked-vertex jobs
    // carry the weights L^2 / (k k'), so their part is divided by L^2 first
    __int128 plain[kAtomCounters] = {0, 0, 0, 0, 0}, marked[kAtomCounters] = {0, 0, 0, 0, 0};
    for (size_t t = 0; t < J; ++t) {
        for (int k = 0; k < kAtomCounters; ++k)
            (jobs[t].marked ? marked : plain)[k] += (__int128)h[t * kAtomCounters + k] * jobs[t].factor;
        out->labelled_evaluated += (int64_t)counts[t];
    }
    long long cls[kAtomCounters];
    for (int k = 0; k < kAtomCounters; ++k) {
        // never expected to fail: the marked part counts whole labelled graphs,
        // and Burnside sums are multiples of n!
        if (marked[k] % kAtomMarkW != 0) return GN_E_NUMERIC;
        const __int128 sum = plain[k] + marked[k] / kAtomMarkW;
        if (sum % nfact != 0) return GN_E_NUMERIC;
        cls[k] = (long long)(sum / nfact);
    }
    out->connected = cls[0];
    out->irregular_discrete = cls[1];
    out->irregular_continuous = cls[2];
    out->regular_discrete = cls[3];
    out->regular_continuous = cls[4];
    out->atomic = out->irregular_discrete + out->irregular_continuous + out->regular_discrete + out->regular_continuous;
    return GN_OK;
}
