// Fractional warm start: the MWIS LP relaxation over clique constraints,
// smoothed by entropy at a temperature T and solved by exact block-coordinate
// minimisation of its dual (a Bregman-Sinkhorn scheme run alone, without
// rounding; Section 6, "Randomized start and warm start").
//
//   LP* = max c.x  s.t.  sum_{i in C} x_i <= 1 for every clique C,  x >= 0.
//
// State per start: a multiplier lam_C >= 0 per clique and Lam_i, the sum of the
// multipliers of the cliques holding i.  The smoothed primal is
// x_i = exp((c_i - Lam_i) / T).  Updating clique C sets
// lam_C' = max(0, lam_C + T log sum_{i in C} x_i) and adds lam_C' - lam_C to
// Lam_i of its members, after which the clique's x sum to at most 1.
//
// Cliques are coloured first-fit into classes of vertex-disjoint cliques at
// creation; a pass visits the classes in the start's order (the caller's
// permutation).  Disjointness makes the members' Lam updates race-free and the
// result independent of the order inside a class.  Pass p runs at
// T_p = max(t_min, t0 drop^p), computed on the host in fp64 and passed by value.
// Two ways to run the passes, with the same arithmetic and so the same bits:
//   * fused: when Lam and lam of a start fit one CU's LDS, one workgroup per
//     start runs all passes up to the next check in one launch, its multipliers
//     in LDS and the classes separated by workgroup barriers.  The cliques of a
//     class are dealt to the wavefronts as tasks laid out at creation (a clique
//     of up to 64 members per wavefront, or two of up to 32, one per half; the
//     member ids and costs in lane order), and each wavefront loads its next
//     task while it works on the current one, so a class costs LDS and
//     arithmetic latency only;
//   * per class: one launch per class for all starts together, a wavefront per
//     clique, the multipliers in global memory.
//
// The check (every check_every passes and after the last) bounds LP* from both
// sides.  D = sum lam_C + sum_i max(0, c_i - sum_{C holds i} lam_C) >= LP*, with
// the multipliers' sums rebuilt in fp64 (the incrementally kept fp32 Lam may
// drift from them, and then would not give a bound).  The feasible point
// xf_i = x_i / max(1, max_{C holds i} sum_{j in C} x_j) is raised by two rounds
// of a fair-share lift (each clique's slack split equally among its members,
// each member taking the smallest share of its cliques), giving P = c.xl.  A
// start keeps the smallest D, the largest P and that P's point over its checks,
// and stops when (D_best - P_best) / D_best <= gap_tol; its warm start is
// max(x_best, floor).
//
// Temperatures: with anneal_tol <= 0, T_p = max(t_min, t0 drop^p) per pass.
// Otherwise T is held within a check interval and drops by drop^check_every at
// a check whose smoothed primal exceeds no clique by more than anneal_tol, or
// after `stall` checks without a relative gain of 5e-5 in P_best; the check
// kernel decides and the host reads the next temperature with the stop flags.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "gn_internal.h"

namespace {

constexpr int kLpWaves = 4;                  // cliques per workgroup of the class launches
constexpr int kLpBlock = 64 * kLpWaves;
constexpr int kLpVBlock = 256;               // vertex kernel
constexpr int kLpFBlock = 256;               // finish kernel
constexpr float kExpCap = 60.0f;             // cap of the check's exponent (keeps sums finite)
constexpr int kLiftRounds = 2;               // fair-share lift rounds of the check
constexpr double kStallRel = 5e-5;           // relative gain of P_best that counts as progress

struct LpState {
    int32_t done;
    int32_t passes;
    int32_t converged;
    float temperature;     // of the last check
    double dual;           // best bound so far
    double primal;         // best feasible value so far
    double gap;
    float next_t;          // temperature of the passes after the last check
    int32_t quiet;         // checks since P_best last gained kStallRel
    int32_t improved;      // the last check raised P_best (its point is kept)
    float excess;          // worst clique excess of the smoothed primal at the last check
};

// Per launch, by value: for each start the range of cliques (in class order)
// the launch updates, empty for starts that have stopped, and the pass's
// temperature.  The kernels then need no dependent loads to find their work.
struct LpRound {
    int32_t beg[GN_MAX_STARTS];
    int32_t end[GN_MAX_STARTS];
    float T[GN_MAX_STARTS];
    float r2[GN_MAX_STARTS];  // log2(e) / T, rounded once from fp64
    float tl[GN_MAX_STARTS];  // T ln 2, rounded once from fp64
};

struct LpArgs {
    const float* cost;       // [n]
    const int32_t* cptr;     // [m + 1], cliques in class order
    const int32_t* cmem;     // members
    const int32_t* vptr;     // [n + 1] vertex -> cliques
    const int32_t* vcl;
    float* Lam;              // [S][n]
    float* lam;              // [S][m]
    float* csum;             // [S][m]
    float* share;            // [S][m] lift shares
    float* x_cand;           // [S][n] the check's feasible (then lifted) point
    double* part;            // [S][2 * nbv]
    LpState* st;             // [S]
    float* x_out;            // [S][n]
    int32_t n, m, K, nbv;
    float gap_tol, x_floor;
    float anneal_tol, t_min, drop_check;  // drop_check = drop^check_every
    int32_t stall;
};

__device__ __forceinline__ float wave_max(float v) {
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ float wave_sum(float v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_sum_d(double v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Butterfly reductions of the clique updates, over a half (32 lanes) or the
// whole wavefront, with the stages in increasing xor distance 1, 2, 4, 8, 16
// (, 32).  After the stages below 2^k every aligned block of 2^k lanes holds
// one value (max and fp32 addition commute), so at distance 4 and 8 any
// permutation that swaps the two halves of each block of 8 and 16 reads the
// same value as the xor partner: the DPP row half-mirror and row mirror do
// it without the LDS crossbar, quad permutations do distances 1 and 2, a
// swizzle 16 and a permute 32.  Every lane ends with the group's value.
//
// The clique update's log-sum-exp runs in base 2, on a_i = (c_i - Lam_i) r2
// with r2 = log2(e) / T: lam' = max(0, lam + T ln2 (max a + log2 sum 2^(a_i -
// max a))), the hardware exp2 and log2 on arguments where they are accurate
// (exponents <= 0, a sum >= 1), instead of a division, expf and logf per
// member.  r2 and T ln2 are rounded once from fp64 on the host.
// The maximum runs on order-preserving integer keys (for non-NaN floats the
// key k = b ^ ((b >> 31) & 0x7fffffff) of the bits b orders as the value), so
// that every DPP stage is one integer max; the sum's DPP stages are one add
// each.  No lane reads outside its row in these patterns, so the DPP bound
// control changes nothing.
__device__ __forceinline__ int lp_key(float v) {
    const int b = __float_as_int(v);
    return b ^ ((b >> 31) & 0x7fffffff);
}
__device__ __forceinline__ float lp_unkey(int k) { return __int_as_float(k ^ ((k >> 31) & 0x7fffffff)); }

template <bool MAX>
__device__ __forceinline__ float lp_reduce(float v, bool full);

template <>
__device__ __forceinline__ float lp_reduce<false>(float v, bool full) {
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, true));   // xor 1
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, true));   // xor 2
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, true));  // 4
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, true));  // 8
    v += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));                   // xor 16
    const float t = __shfl_xor(v, 32, 64);
    return full ? v + t : v;
}

template <>
__device__ __forceinline__ float lp_reduce<true>(float v, bool full) {
    int k = lp_key(v);
    k = max(k, __builtin_amdgcn_update_dpp(0, k, 0xB1, 0xF, 0xF, true));
    k = max(k, __builtin_amdgcn_update_dpp(0, k, 0x4E, 0xF, 0xF, true));
    k = max(k, __builtin_amdgcn_update_dpp(0, k, 0x141, 0xF, 0xF, true));
    k = max(k, __builtin_amdgcn_update_dpp(0, k, 0x140, 0xF, 0xF, true));
    k = max(k, __builtin_amdgcn_ds_swizzle(k, 0x401F));
    const int t = __shfl_xor(k, 32, 64);
    return lp_unkey(full ? max(k, t) : k);
}

// maximum of two non-NaN floats (the chunked sweeps)
__device__ __forceinline__ float lp_max2(float a, float b) { return a > b ? a : b; }

// One class of every running start: a wavefront per clique.  A clique of at
// most 64 members is held in registers (one member per lane); longer ones are
// swept in chunks of 64.
__global__ __launch_bounds__(kLpBlock) void lp_round_kernel(LpArgs a, LpRound rd) {
    const int s = blockIdx.y;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int k = rd.beg[s] + blockIdx.x * kLpWaves + wave;
    if (k >= rd.end[s]) return;
    const float r2 = rd.r2[s], tl = rd.tl[s];
    const int b = a.cptr[k], e = a.cptr[k + 1];
    float* L = a.Lam + (size_t)s * a.n;
    float* lp = a.lam + (size_t)s * a.m + k;
    const float old = *lp;
    if (e - b <= 64) {
        const bool on = b + lane < e;
        const int i = on ? a.cmem[b + lane] : 0;
        const float Li = on ? L[i] : 0.0f;
        const float ai = on ? (a.cost[i] - Li) * r2 : -INFINITY;
        const float mx = lp_reduce<true>(ai, true);
        const float sum = lp_reduce<false>(on ? __builtin_amdgcn_exp2f(ai - mx) : 0.0f, true);
        const float nw = fmaxf(0.0f, old + tl * (mx + __builtin_amdgcn_logf(sum)));
        if (on) L[i] = Li + (nw - old);
        if (lane == 0) *lp = nw;
        return;
    }
    float mx = -INFINITY;
    for (int j = b + lane; j < e; j += 64) {
        const int i = a.cmem[j];
        mx = lp_max2(mx, (a.cost[i] - L[i]) * r2);
    }
    mx = lp_reduce<true>(mx, true);
    float sum = 0.0f;
    for (int j = b + lane; j < e; j += 64) {
        const int i = a.cmem[j];
        sum += __builtin_amdgcn_exp2f((a.cost[i] - L[i]) * r2 - mx);
    }
    sum = lp_reduce<false>(sum, true);
    const float nw = fmaxf(0.0f, old + tl * (mx + __builtin_amdgcn_logf(sum)));
    const float d = nw - old;
    for (int j = b + lane; j < e; j += 64) L[a.cmem[j]] += d;
    if (lane == 0) *lp = nw;
}

// ---- fused passes --------------------------------------------------------------
constexpr int kLpPassWaves = 16;
constexpr int kLpPassBlock = 64 * kLpPassWaves;
constexpr int kLpPassMax = 16;      // passes per fused launch
constexpr int kLpTaskFull = 1;      // task flag: one clique over the whole wavefront
constexpr int kLpTaskChunked = 2;   // task flag: one clique of more than 64 members
constexpr int kLpTB = 4;            // tasks per batch of a wavefront
constexpr int kLpLdsBudget = 160 * 1024 - 2048;  // dynamic LDS of the fused passes

// Per fused launch, by value: the start of each workgroup and the temperature of
// each start's passes in this launch.
struct LpPasses {
    int32_t start[GN_MAX_STARTS];
    float r2[GN_MAX_STARTS * kLpPassMax];  // [s][pass of the launch]: log2(e) / T
    float tl[GN_MAX_STARTS * kLpPassMax];  // T ln 2
    int32_t passes;
};

struct LpTasks {
    const int4* task;      // [slots][64]: member id, cost bits, clique (class order; -1: idle lane), flags
    const int32_t* tbase;  // [K + 1]: first slot of each class
    const int32_t* order;  // [S][K]: each start's class order
};

// A clique of more than 64 members (one task): the chunked update of
// lp_round_kernel on the LDS multipliers.
__device__ __forceinline__ void lp_task_chunked(const LpArgs& a, int k, float r2, float tl, float* sL, float* sl) {
    const int lane = threadIdx.x & 63;
    const int b = a.cptr[k], e = a.cptr[k + 1];
    const float old = sl[k];
    float mx = -INFINITY;
    for (int j = b + lane; j < e; j += 64) {
        const int i = a.cmem[j];
        mx = lp_max2(mx, (a.cost[i] - sL[i]) * r2);
    }
    mx = lp_reduce<true>(mx, true);
    float sum = 0.0f;
    for (int j = b + lane; j < e; j += 64) {
        const int i = a.cmem[j];
        sum += __builtin_amdgcn_exp2f((a.cost[i] - sL[i]) * r2 - mx);
    }
    sum = lp_reduce<false>(sum, true);
    const float nw = fmaxf(0.0f, old + tl * (mx + __builtin_amdgcn_logf(sum)));
    const float dl = nw - old;
    for (int j = b + lane; j < e; j += 64) sL[a.cmem[j]] += dl;
    if (lane == 0) sl[k] = nw;
}

// A batch of NB tasks of one wavefront (idle lanes hold clique -1), their
// dependency chains interleaved: the update of lp_round_kernel for each clique.
// A clique of at most 32 members in one half gets the same bits as alone in a
// wavefront: its reduction stays inside the half, and the other half's -inf
// and 0 change neither the maximum nor the sum at distance 32.
template <int NB>
__device__ __forceinline__ void lp_batch(const LpArgs& a, const int4 (&d)[kLpTB], float r2, float tl, float* sL,
                                         float* sl) {
    const int lane = threadIdx.x & 63;
    bool chunked = false;
#pragma unroll
    for (int q = 0; q < NB; ++q) chunked |= (__builtin_amdgcn_readfirstlane(d[q].w) & kLpTaskChunked) != 0;
    if (chunked) {
        int ks[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q)
            ks[q] = (__builtin_amdgcn_readfirstlane(d[q].w) & kLpTaskChunked) ? __builtin_amdgcn_readfirstlane(d[q].z)
                                                                              : -1;
        for (int q = 0; q < NB; ++q)  // scalar indices: no register array indexed at run time
            if (ks[q] >= 0) lp_task_chunked(a, ks[q], r2, tl, sL, sl);
    }
    float Li[NB], old[NB], ai[NB], mx[NB], sm[NB];
    bool on[NB], full[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int fl = __builtin_amdgcn_readfirstlane(d[q].w);
        on[q] = d[q].z >= 0 && !(fl & kLpTaskChunked);
        full[q] = (fl & kLpTaskFull) != 0;
        Li[q] = on[q] ? sL[d[q].x] : 0.0f;
        old[q] = on[q] ? sl[d[q].z] : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) ai[q] = on[q] ? (__int_as_float(d[q].y) - Li[q]) * r2 : -INFINITY;
#pragma unroll
    for (int q = 0; q < NB; ++q) mx[q] = lp_reduce<true>(ai[q], full[q]);
#pragma unroll
    for (int q = 0; q < NB; ++q)
        sm[q] = lp_reduce<false>(on[q] ? __builtin_amdgcn_exp2f(ai[q] - mx[q]) : 0.0f, full[q]);
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const float nw = fmaxf(0.0f, old[q] + tl * (mx[q] + __builtin_amdgcn_logf(sm[q])));
        if (on[q]) sL[d[q].x] = Li[q] + (nw - old[q]);
        if (on[q] && (lane & (full[q] ? 63 : 31)) == 0) sl[d[q].z] = nw;
    }
}

// The passes of one launch for one start per workgroup (ps.start), Lam and lam
// of the start in LDS, the class order and the class task offsets too.  Wave w
// takes slots tbase[c] + w, + 16, ... of class c, kLpTB at a time, and loads
// its next batch (of this class or the next) when it starts on one: the task
// data are static, so the loads never wait on the multipliers.  A barrier ends
// each class.
__global__ __launch_bounds__(kLpPassBlock) void lp_pass_kernel(LpArgs a, LpTasks ta, LpPasses ps) {
    extern __shared__ float sm[];
    float* sL = sm;
    float* sl = sm + a.n;
    int32_t* so = reinterpret_cast<int32_t*>(sl + a.m);  // [K]
    int32_t* sb = so + a.K;                               // [K + 1]
    const int s = ps.start[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    float* gL = a.Lam + (size_t)s * a.n;
    float* gl = a.lam + (size_t)s * a.m;
    for (int q = tid; q < a.n; q += kLpPassBlock) sL[q] = gL[q];
    for (int q = tid; q < a.m; q += kLpPassBlock) sl[q] = gl[q];
    for (int q = tid; q < a.K; q += kLpPassBlock) so[q] = ta.order[(size_t)s * a.K + q];
    for (int q = tid; q <= a.K; q += kLpPassBlock) sb[q] = ta.tbase[q];
    __syncthreads();
    const int K = a.K, P = ps.passes;
    constexpr int kStride = kLpPassWaves * kLpTB;  // slots between a wave's batches
    // batch at slot t (the wave's slots t, t + 16, ... below tend); returns the
    // mask of the slots that exist (the others load slot 0 and stay unused, so
    // no register is written while its load is in flight)
    auto load = [&](int t, int tend, int4 (&d)[kLpTB]) -> unsigned {
        unsigned valid = 0u;
#pragma unroll
        for (int q = 0; q < kLpTB; ++q) {
            const int u = t + q * kLpPassWaves;
            const bool ok = u < tend;
            d[q] = ta.task[(size_t)(ok ? u : 0) * 64 + lane];
            valid |= ok ? 1u << q : 0u;
        }
        return valid;
    };
    auto cls = [&](int r, int& tb, int& te) {
        const int c = __builtin_amdgcn_readfirstlane(so[r]);
        tb = __builtin_amdgcn_readfirstlane(sb[c]) + wave;
        te = __builtin_amdgcn_readfirstlane(sb[c + 1]);
    };
    int tb, te;
    cls(0, tb, te);
    int4 cur[kLpTB];
    unsigned cv = load(tb, te, cur);
    for (int p = 0; p < P; ++p) {
        const float r2 = ps.r2[s * kLpPassMax + p], tl = ps.tl[s * kLpPassMax + p];
        for (int r = 0; r < K; ++r) {
            // cur holds the batch at tb of class position r (idle if tb >= te)
            const bool more = r + 1 < K || p + 1 < P;
            int nb, ne;
            cls(r + 1 < K ? r + 1 : 0, nb, ne);
            if (!more) ne = nb;  // nothing after the last class
            for (int t = tb;; t += kStride) {
                const bool last_batch = t + kStride >= te;
                int4 nxt[kLpTB];
                const unsigned nv = last_batch ? load(nb, ne, nxt) : load(t + kStride, te, nxt);
                // the valid slots are a prefix: a batch of their count
                switch (cv) {
                    case 0xF: lp_batch<4>(a, cur, r2, tl, sL, sl); break;
                    case 0x7: lp_batch<3>(a, cur, r2, tl, sL, sl); break;
                    case 0x3: lp_batch<2>(a, cur, r2, tl, sL, sl); break;
                    case 0x1: lp_batch<1>(a, cur, r2, tl, sL, sl); break;
                    default: break;
                }
#pragma unroll
                for (int q = 0; q < kLpTB; ++q) cur[q] = nxt[q];
                cv = nv;
                if (last_batch) break;
            }
            tb = nb;
            te = ne;
            __syncthreads();
        }
    }
    for (int q = tid; q < a.n; q += kLpPassBlock) gL[q] = sL[q];
    for (int q = tid; q < a.m; q += kLpPassBlock) gl[q] = sl[q];
}

// log2(e) / T and T ln 2 of a pass, rounded once from fp64
static float lp_r2(float T) { return (float)(1.4426950408889634074 / (double)T); }
static float lp_tl(float T) { return (float)((double)T * 0.69314718055994530942); }

// LDS bytes of the fused passes
static size_t lp_pass_lds(int32_t n, int32_t m, int32_t K) {
    return sizeof(float) * ((size_t)n + m) + sizeof(int32_t) * (2 * (size_t)K + 1);
}

// Check, part 1: the clique sums of the smoothed primal.
__global__ __launch_bounds__(kLpBlock) void lp_csum_kernel(LpArgs a, LpRound rd) {
    const int s = blockIdx.y;
    if (a.st[s].done) return;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.x * kLpWaves + wave;
    if (k >= a.m) return;
    const float T = rd.T[s];
    const float* L = a.Lam + (size_t)s * a.n;
    float sum = 0.0f;
    for (int j = a.cptr[k] + lane; j < a.cptr[k + 1]; j += 64) {
        const int i = a.cmem[j];
        sum += expf(fminf((a.cost[i] - L[i]) / T, kExpCap));
    }
    sum = wave_sum(sum);
    if (lane == 0) a.csum[(size_t)s * a.m + k] = sum;
}

// Fixed-order block sum of a per-thread fp64 value into part[s][2 b + slot].
__device__ __forceinline__ void lp_block_partial(const LpArgs& a, int s, int slot, double v, double* red) {
    v = wave_sum_d(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < kLpVBlock / 64; ++q) t += red[q];
        a.part[(size_t)s * 2 * a.nbv + 2 * blockIdx.x + slot] = t;
    }
}

// Check, part 2: the feasible point xf into x_cand, and per-block partial sums of
// max(0, c_i - sum_{C holds i} lam_C) with the multipliers' sums rebuilt in fp64.
__global__ __launch_bounds__(kLpVBlock) void lp_vertex_kernel(LpArgs a, LpRound rd) {
    const int s = blockIdx.y;
    if (a.st[s].done) return;
    __shared__ double red[kLpVBlock / 64];
    const int i = blockIdx.x * kLpVBlock + threadIdx.x;
    double dv = 0.0;
    if (i < a.n) {
        const float T = rd.T[s];
        const float c = a.cost[i];
        const float Li = a.Lam[(size_t)s * a.n + i];
        const float x = expf(fminf((c - Li) / T, kExpCap));
        float mx = 1.0f;
        double lsum = 0.0;
        const float* cs = a.csum + (size_t)s * a.m;
        const float* lm = a.lam + (size_t)s * a.m;
        for (int q = a.vptr[i]; q < a.vptr[i + 1]; ++q) {
            const int k = a.vcl[q];
            mx = fmaxf(mx, cs[k]);
            lsum += (double)lm[k];
        }
        a.x_cand[(size_t)s * a.n + i] = x / mx;
        dv = fmax(0.0, (double)c - lsum);
    }
    lp_block_partial(a, s, 1, dv, red);
}

// Lift, part 1: each clique's slack 1 - sum_{i in C} x_i, shared equally among
// its members (a wavefront per clique, the sum in fp64).
__global__ __launch_bounds__(kLpBlock) void lp_share_kernel(LpArgs a) {
    const int s = blockIdx.y;
    if (a.st[s].done) return;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.x * kLpWaves + wave;
    if (k >= a.m) return;
    const float* xc = a.x_cand + (size_t)s * a.n;
    const int b = a.cptr[k], e = a.cptr[k + 1];
    double sum = 0.0;
    for (int j = b + lane; j < e; j += 64) sum += (double)xc[a.cmem[j]];
    sum = wave_sum_d(sum);
    if (lane == 0) a.share[(size_t)s * a.m + k] = (float)(fmax(0.0, 1.0 - sum) / (double)(e - b));
}

// Lift, part 2: every vertex rises by the smallest share of its cliques (the
// shares are rounded down to fp32 from the exact quotient, and each member takes
// at most its share, so no clique exceeds 1 but by rounding of the sums); the
// last round also forms the per-block partials of c.x.
__global__ __launch_bounds__(kLpVBlock) void lp_raise_kernel(LpArgs a, int32_t last) {
    const int s = blockIdx.y;
    if (a.st[s].done) return;
    __shared__ double red[kLpVBlock / 64];
    const int i = blockIdx.x * kLpVBlock + threadIdx.x;
    double pv = 0.0;
    if (i < a.n) {
        const float* sh = a.share + (size_t)s * a.m;
        float up = INFINITY;
        for (int q = a.vptr[i]; q < a.vptr[i + 1]; ++q) up = fminf(up, sh[a.vcl[q]]);
        float* xc = a.x_cand + (size_t)s * a.n + i;
        const float xn = *xc + up;
        *xc = xn;
        pv = (double)a.cost[i] * (double)xn;
    }
    if (last) lp_block_partial(a, s, 0, pv, red);
}

// Keeps the lifted point of a check that raised P_best as the start's warm start.
__global__ __launch_bounds__(kLpVBlock) void lp_keep_kernel(LpArgs a) {
    const int s = blockIdx.y;
    if (!a.st[s].improved) return;
    const int i = blockIdx.x * kLpVBlock + threadIdx.x;
    if (i < a.n) a.x_out[(size_t)s * a.n + i] = fmaxf(a.x_cand[(size_t)s * a.n + i], a.x_floor);
}

// Check, part 3: one workgroup per start reduces the bound and the primal value
// and decides the stop.
__global__ __launch_bounds__(kLpFBlock) void lp_finish_kernel(LpArgs a, LpRound rd, int32_t p, int32_t last) {
    const int s = blockIdx.x;
    if (a.st[s].done) return;
    __shared__ double red[3][kLpFBlock / 64];
    __shared__ float redx[kLpFBlock / 64];
    double sl = 0.0, P = 0.0, D = 0.0;
    float ex = -INFINITY;
    const float* lam = a.lam + (size_t)s * a.m;
    const float* cs = a.csum + (size_t)s * a.m;
    for (int k = threadIdx.x; k < a.m; k += kLpFBlock) {
        sl += (double)lam[k];
        ex = fmaxf(ex, cs[k]);
    }
    const double* part = a.part + (size_t)s * 2 * a.nbv;
    for (int q = threadIdx.x; q < a.nbv; q += kLpFBlock) {
        P += part[2 * q];
        D += part[2 * q + 1];
    }
    sl = wave_sum_d(sl);
    P = wave_sum_d(P);
    D = wave_sum_d(D);
    ex = wave_max(ex);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = sl;
        red[1][w] = P;
        red[2][w] = D;
        redx[w] = ex;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double L = 0.0, Pt = 0.0, Dt = 0.0;
        float exc = -INFINITY;
        for (int q = 0; q < kLpFBlock / 64; ++q) {
            L += red[0][q];
            Pt += red[1][q];
            Dt += red[2][q];
            exc = fmaxf(exc, redx[q]);
        }
        Dt += L;
        LpState o = a.st[s];
        const bool first = o.passes == 0;
        const double P_prev = first ? -INFINITY : o.primal;
        o.quiet = (!first && Pt <= P_prev * (1.0 + kStallRel)) ? o.quiet + 1 : 0;
        o.improved = Pt > P_prev ? 1 : 0;
        o.primal = o.improved ? Pt : P_prev;
        o.dual = first ? Dt : fmin(o.dual, Dt);
        o.gap = (o.dual - o.primal) / o.dual;
        o.excess = exc - 1.0f;
        o.temperature = rd.T[s];
        o.passes = p + 1;
        o.next_t = rd.T[s];
        const bool conv = o.gap <= (double)a.gap_tol;
        if (conv || last) {
            o.done = 1;
            o.converged = conv ? 1 : 0;
        } else if (a.anneal_tol > 0.0f && (o.excess <= a.anneal_tol || o.quiet >= a.stall)) {
            o.next_t = fmaxf(a.t_min, (float)((double)rd.T[s] * (double)a.drop_check));
            o.quiet = 0;
        }
        a.st[s] = o;
    }
}

__global__ void lp_reset_kernel(LpArgs a, int32_t starts) {
    const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t q = tid; q < (size_t)starts * a.n; q += stride) a.Lam[q] = 0.0f;
    for (size_t q = tid; q < (size_t)starts * a.m; q += stride) a.lam[q] = 0.0f;
    if (tid < (size_t)starts) {
        LpState o{};
        a.st[tid] = o;
    }
}

}  // namespace

struct gn_lp {
    int device = 0;
    int32_t n = 0, m = 0, K = 0, max_class = 0;
    int64_t nnzc = 0;
    std::vector<int32_t> class_ptr_h;  // [K + 1]
    float* cost = nullptr;
    int32_t* cptr = nullptr;
    int32_t* cmem = nullptr;
    int32_t* vptr = nullptr;
    int32_t* vcl = nullptr;
    float* Lam = nullptr;
    float* lam = nullptr;
    float* csum = nullptr;
    float* share = nullptr;
    float* x_cand = nullptr;
    double* part = nullptr;
    LpState* st = nullptr;
    LpState* st_host = nullptr;  // pinned
    // fused passes (null when a start's multipliers do not fit one CU's LDS)
    int4* task = nullptr;
    int32_t* tbase = nullptr;
    int32_t* order_d = nullptr;
    size_t pass_lds = 0;
    bool fused_on = true;
};

static void lp_free(gn_lp* L) {
    hipFree(L->cost);
    hipFree(L->cptr);
    hipFree(L->cmem);
    hipFree(L->vptr);
    hipFree(L->vcl);
    hipFree(L->Lam);
    hipFree(L->lam);
    hipFree(L->csum);
    hipFree(L->share);
    hipFree(L->x_cand);
    hipFree(L->part);
    hipFree(L->st);
    if (L->st_host) hipHostFree(L->st_host);
    hipFree(L->task);
    hipFree(L->tbase);
    hipFree(L->order_d);
}

// The fused passes' task layout: per class, its cliques as wavefront tasks in
// class order -- a clique of more than 64 members alone (swept in chunks), one
// of 33..64 members alone, two of at most 32 in the two halves (consecutive
// ones paired, the last one alone in a half if their count is odd).  Each task
// holds per lane the member id, the member's cost bits, the clique (class-order
// index) and the flags; idle lanes hold clique -1.
static void lp_build_tasks(int32_t K, const std::vector<int32_t>& class_ptr, const std::vector<int32_t>& cptr,
                           const std::vector<int32_t>& cmem, const float* cost, std::vector<int4>& task,
                           std::vector<int32_t>& tbase) {
    tbase.assign((size_t)K + 1, 0);
    task.clear();
    auto lanes = [&](int4* t, int32_t q, int flags) {  // the members of q from lane 0 of t
        for (int32_t j = cptr[q]; j < cptr[q + 1]; ++j) {
            const int32_t i = cmem[j];
            int32_t cb;
            std::memcpy(&cb, &cost[i], sizeof(cb));
            t[j - cptr[q]] = make_int4(i, cb, q, flags);
        }
    };
    auto open = [&](int flags) -> int4* {
        const size_t at = task.size();
        task.resize(at + 64, make_int4(0, 0, -1, flags));
        return task.data() + at;
    };
    for (int32_t c = 0; c < K; ++c) {
        tbase[c] = (int32_t)(task.size() / 64);
        int32_t pend = -1;
        for (int32_t q = class_ptr[c]; q < class_ptr[c + 1]; ++q) {
            const int32_t sz = cptr[q + 1] - cptr[q];
            if (sz > 64) {
                int4* t = open(kLpTaskChunked);
                for (int l = 0; l < 64; ++l) t[l].z = q;
            } else if (sz > 32) {
                lanes(open(kLpTaskFull), q, kLpTaskFull);
            } else if (pend < 0) {
                pend = q;
            } else {
                int4* t = open(0);
                lanes(t, pend, 0);
                lanes(t + 32, q, 0);
                pend = -1;
            }
        }
        if (pend >= 0) lanes(open(0), pend, 0);
    }
    tbase[K] = (int32_t)(task.size() / 64);
}

gn_status gn_internal_check_cliques(int32_t n, int32_t m, const int32_t* ptr, const int32_t* members,
                                    const float* w, std::vector<int32_t>& cover) {
    if (n < 1 || m < 1 || !ptr || !members || !w) return GN_E_ARG;
    if (ptr[0] != 0) return GN_E_CSR;
    for (int32_t k = 0; k < m; ++k)
        if (ptr[k + 1] <= ptr[k]) return GN_E_CSR;  // empty clique or not monotone
    cover.assign(n, 0);
    for (int32_t k = 0; k < m; ++k)
        for (int32_t j = ptr[k]; j < ptr[k + 1]; ++j) {
            const int32_t i = members[j];
            if (i < 0 || i >= n) return GN_E_CSR;
            if (j > ptr[k] && i <= members[j - 1]) return GN_E_CSR;
            ++cover[i];
        }
    for (int32_t i = 0; i < n; ++i) {
        if (cover[i] == 0) return GN_E_ARG;  // a vertex outside every clique
        if (!(w[i] > 0.0f) || !std::isfinite(w[i])) return GN_E_WEIGHT;
    }
    return GN_OK;
}

static int32_t lp_nbv(int32_t n) { return (n + kLpVBlock - 1) / kLpVBlock; }

extern "C" gn_status gn_lp_create(int32_t n, int32_t m, const int32_t* clique_ptr, const int32_t* members,
                                  const float* cost, hipStream_t stream, gn_lp** out) {
    if (!out) return GN_E_ARG;
    *out = nullptr;
    if (!cost) return GN_E_ARG;
    std::vector<int32_t> cover;
    const gn_status vs = gn_internal_check_cliques(n, m, clique_ptr, members, cost, cover);
    if (vs != GN_OK) return vs;
    const int64_t nnzc = clique_ptr[m];
    // first-fit colouring in input order: the lowest class none of whose
    // cliques holds a member of clique k
    std::vector<std::vector<int32_t>> used(n);
    std::vector<int32_t> cls(m);
    std::vector<char> taken;
    int32_t K = 0;
    for (int32_t k = 0; k < m; ++k) {
        taken.assign((size_t)K + 1, 0);
        for (int32_t j = clique_ptr[k]; j < clique_ptr[k + 1]; ++j)
            for (int32_t c : used[members[j]]) taken[c] = 1;
        int32_t c = 0;
        while (taken[c]) ++c;
        cls[k] = c;
        K = std::max(K, c + 1);
        for (int32_t j = clique_ptr[k]; j < clique_ptr[k + 1]; ++j) used[members[j]].push_back(c);
    }
    // cliques grouped by class, input order inside a class
    std::vector<int32_t> class_ptr(K + 1, 0), pos(K), perm(m);
    for (int32_t k = 0; k < m; ++k) ++class_ptr[cls[k] + 1];
    for (int32_t c = 0; c < K; ++c) class_ptr[c + 1] += class_ptr[c];
    for (int32_t c = 0; c < K; ++c) pos[c] = class_ptr[c];
    for (int32_t k = 0; k < m; ++k) perm[pos[cls[k]]++] = k;
    std::vector<int32_t> cptr(m + 1, 0), cmem((size_t)nnzc);
    for (int32_t q = 0; q < m; ++q) {
        const int32_t k = perm[q];
        const int32_t sz = clique_ptr[k + 1] - clique_ptr[k];
        std::memcpy(&cmem[cptr[q]], &members[clique_ptr[k]], sizeof(int32_t) * sz);
        cptr[q + 1] = cptr[q] + sz;
    }
    std::vector<int32_t> vptr(n + 1, 0), vcl((size_t)nnzc), vpos(n);
    for (int32_t i = 0; i < n; ++i) vptr[i + 1] = vptr[i] + cover[i];
    for (int32_t i = 0; i < n; ++i) vpos[i] = vptr[i];
    for (int32_t q = 0; q < m; ++q)
        for (int32_t j = cptr[q]; j < cptr[q + 1]; ++j) vcl[vpos[cmem[j]]++] = q;

    gn_lp* L = new (std::nothrow) gn_lp();
    if (!L) return GN_E_NOMEM;
    (void)hipGetDevice(&L->device);
    L->n = n;
    L->m = m;
    L->K = K;
    L->nnzc = nnzc;
    L->class_ptr_h = class_ptr;
    for (int32_t c = 0; c < K; ++c) L->max_class = std::max(L->max_class, class_ptr[c + 1] - class_ptr[c]);
    const size_t S = GN_MAX_STARTS;
    bool ok = gn_dalloc(&L->cost, n) && gn_dalloc(&L->cptr, (size_t)m + 1) && gn_dalloc(&L->cmem, (size_t)nnzc) &&
              gn_dalloc(&L->vptr, (size_t)n + 1) &&
              gn_dalloc(&L->vcl, (size_t)nnzc) &&
              gn_dalloc(&L->Lam, S * n) && gn_dalloc(&L->lam, S * m) && gn_dalloc(&L->csum, S * m) &&
              gn_dalloc(&L->share, S * m) && gn_dalloc(&L->x_cand, S * n) &&
              gn_dalloc(&L->part, S * 2 * (size_t)lp_nbv(n)) && gn_dalloc(&L->st, S);
    if (ok && hipHostMalloc((void**)&L->st_host, sizeof(LpState) * S, hipHostMallocDefault) != hipSuccess) {
        L->st_host = nullptr;
        ok = false;
    }
    if (!ok) {
        lp_free(L);
        delete L;
        return GN_E_NOMEM;
    }
    hipError_t e = hipMemcpyAsync(L->cost, cost, sizeof(float) * n, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(L->cptr, cptr.data(), sizeof(int32_t) * (m + 1), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(L->cmem, cmem.data(), sizeof(int32_t) * nnzc, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(L->vptr, vptr.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(L->vcl, vcl.data(), sizeof(int32_t) * nnzc, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && lp_pass_lds(n, m, K) <= (size_t)kLpLdsBudget) {
        std::vector<int4> task;
        std::vector<int32_t> tbase;
        lp_build_tasks(K, class_ptr, cptr, cmem, cost, task, tbase);
        if (gn_dalloc(&L->task, task.size()) && gn_dalloc(&L->tbase, tbase.size()) &&
            gn_dalloc(&L->order_d, S * (size_t)K)) {
            e = hipMemcpyAsync(L->task, task.data(), sizeof(int4) * task.size(), hipMemcpyHostToDevice, stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(L->tbase, tbase.data(), sizeof(int32_t) * tbase.size(), hipMemcpyHostToDevice,
                                   stream);
            if (e == hipSuccess) e = hipStreamSynchronize(stream);
            L->pass_lds = lp_pass_lds(n, m, K);
            if (e == hipSuccess && L->pass_lds > 64 * 1024)
                e = hipFuncSetAttribute((const void*)lp_pass_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)L->pass_lds);
        } else {
            hipFree(L->task);
            hipFree(L->tbase);
            hipFree(L->order_d);
            L->task = nullptr;
            L->tbase = nullptr;
            L->order_d = nullptr;
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        lp_free(L);
        delete L;
        return GN_E_HIP;
    }
    *out = L;
    return GN_OK;
}

extern "C" int32_t gn_lp_set_fused(gn_lp* L, int32_t enable) {
    if (!L) return -1;
    L->fused_on = enable != 0;
    return L->fused_on && L->task ? 1 : 0;
}

extern "C" void gn_lp_destroy(gn_lp* L) {
    if (!L) return;
    (void)hipDeviceSynchronize();
    lp_free(L);
    delete L;
}

extern "C" gn_status gn_lp_info(const gn_lp* L, int32_t* n_classes, int32_t* n_cliques, int32_t* max_class) {
    if (!L) return GN_E_ARG;
    if (n_classes) *n_classes = L->K;
    if (n_cliques) *n_cliques = L->m;
    if (max_class) *max_class = L->max_class;
    return GN_OK;
}

extern "C" gn_status gn_lp_solve(gn_lp* L, int32_t starts, const float* t0, const int32_t* order, float drop,
                                 float t_min, int32_t max_passes, int32_t check_every, float gap_tol, float x_floor,
                                 float anneal_tol, int32_t stall, float* x, gn_lp_result* res, hipStream_t stream) {
    if (!L || !t0 || !order || !x || !res || starts < 1 || starts > GN_MAX_STARTS || max_passes < 1 ||
        check_every < 1 || stall < 1)
        return GN_E_ARG;
    if (!(drop > 0.0f && drop <= 1.0f) || !(t_min > 0.0f) || !std::isfinite(t_min) || !(gap_tol >= 0.0f) ||
        !std::isfinite(gap_tol) || !(x_floor >= 0.0f && x_floor < 1.0f) || !std::isfinite(anneal_tol))
        return GN_E_ARG;
    const bool anneal = anneal_tol > 0.0f;
    const int32_t K = L->K;
    std::vector<char> seen(K);
    for (int32_t s = 0; s < starts; ++s) {
        if (!(t0[s] > 0.0f) || !std::isfinite(t0[s])) return GN_E_ARG;
        std::fill(seen.begin(), seen.end(), 0);
        for (int32_t r = 0; r < K; ++r) {
            const int32_t c = order[(size_t)s * K + r];
            if (c < 0 || c >= K || seen[c]) return GN_E_ARG;  // not a permutation of the classes
            seen[c] = 1;
        }
    }
    LpArgs a;
    a.cost = L->cost;
    a.cptr = L->cptr;
    a.cmem = L->cmem;
    a.vptr = L->vptr;
    a.vcl = L->vcl;
    a.Lam = L->Lam;
    a.lam = L->lam;
    a.csum = L->csum;
    a.share = L->share;
    a.x_cand = L->x_cand;
    a.part = L->part;
    a.st = L->st;
    a.x_out = x;
    a.n = L->n;
    a.m = L->m;
    a.K = K;
    a.nbv = lp_nbv(L->n);
    a.gap_tol = gap_tol;
    a.x_floor = x_floor;
    a.anneal_tol = anneal_tol;
    a.t_min = t_min;
    a.drop_check = (float)std::pow((double)drop, (double)check_every);
    a.stall = stall;
    lp_reset_kernel<<<1024, 256, 0, stream>>>(a, starts);
    GN_HIP_TRY(hipGetLastError());
    const dim3 gcs((L->m + kLpWaves - 1) / kLpWaves, starts), gv(a.nbv, starts);
    const bool fused = L->fused_on && L->task;
    LpTasks ta{L->task, L->tbase, L->order_d};
    if (fused)
        GN_HIP_TRY(hipMemcpyAsync(L->order_d, order, sizeof(int32_t) * starts * K, hipMemcpyHostToDevice, stream));
    std::vector<char> running(starts, 1);
    std::vector<float> T_cur(t0, t0 + starts);   // annealed temperatures, set by each check
    auto temp = [&](int32_t s, int32_t q) -> float {
        return anneal ? T_cur[s] : (float)std::max((double)t_min, (double)t0[s] * std::pow((double)drop, (double)q));
    };
    LpRound rd{};
    // passes [p, pe) up to the next check, then the check after pass pe - 1
    for (int32_t p = 0; p < max_passes;) {
        const int32_t pe = (int32_t)std::min<int64_t>(max_passes, ((int64_t)p / check_every + 1) * check_every);
        if (fused) {
            for (int32_t q0 = p; q0 < pe; q0 += kLpPassMax) {
                LpPasses ps{};
                ps.passes = std::min(kLpPassMax, pe - q0);
                int32_t nb = 0;
                for (int32_t s = 0; s < starts; ++s) {
                    if (!running[s]) continue;
                    ps.start[nb++] = s;
                    for (int32_t j = 0; j < ps.passes; ++j) {
                        const float T = temp(s, q0 + j);
                        ps.r2[s * kLpPassMax + j] = lp_r2(T);
                        ps.tl[s * kLpPassMax + j] = lp_tl(T);
                    }
                }
                lp_pass_kernel<<<nb, kLpPassBlock, L->pass_lds, stream>>>(a, ta, ps);
            }
        } else {
            for (int32_t q = p; q < pe; ++q) {
                for (int32_t s = 0; s < starts; ++s) {
                    rd.T[s] = temp(s, q);
                    rd.r2[s] = lp_r2(rd.T[s]);
                    rd.tl[s] = lp_tl(rd.T[s]);
                }
                for (int32_t r = 0; r < K; ++r) {
                    int32_t gx = 0;
                    for (int32_t s = 0; s < starts; ++s) {
                        const int32_t c = order[(size_t)s * K + r];
                        rd.beg[s] = L->class_ptr_h[c];
                        rd.end[s] = running[s] ? L->class_ptr_h[c + 1] : rd.beg[s];
                        gx = std::max(gx, (rd.end[s] - rd.beg[s] + kLpWaves - 1) / kLpWaves);
                    }
                    lp_round_kernel<<<dim3(gx, starts), kLpBlock, 0, stream>>>(a, rd);
                }
            }
        }
        for (int32_t s = 0; s < starts; ++s) rd.T[s] = temp(s, pe - 1);
        const bool last = pe == max_passes;
        lp_csum_kernel<<<gcs, kLpBlock, 0, stream>>>(a, rd);
        lp_vertex_kernel<<<gv, kLpVBlock, 0, stream>>>(a, rd);
        for (int r = 0; r < kLiftRounds; ++r) {
            lp_share_kernel<<<gcs, kLpBlock, 0, stream>>>(a);
            lp_raise_kernel<<<gv, kLpVBlock, 0, stream>>>(a, r + 1 == kLiftRounds ? 1 : 0);
        }
        lp_finish_kernel<<<starts, kLpFBlock, 0, stream>>>(a, rd, pe - 1, last ? 1 : 0);
        lp_keep_kernel<<<gv, kLpVBlock, 0, stream>>>(a);
        GN_HIP_TRY(hipGetLastError());
        GN_HIP_TRY(hipMemcpyAsync(L->st_host, L->st, sizeof(LpState) * starts, hipMemcpyDeviceToHost, stream));
        GN_HIP_TRY(hipStreamSynchronize(stream));
        bool all = true;
        for (int32_t s = 0; s < starts; ++s) {
            running[s] = !L->st_host[s].done;
            T_cur[s] = L->st_host[s].next_t;
            all = all && !running[s];
        }
        p = pe;
        if (all) break;
    }
    bool conv = true;
    for (int32_t s = 0; s < starts; ++s) {
        const LpState& o = L->st_host[s];
        if (!std::isfinite(o.dual) || !std::isfinite(o.primal)) return GN_E_NUMERIC;
        res[s].passes = o.passes;
        res[s].converged = o.converged;
        res[s].temperature = o.temperature;
        res[s].pad = 0.0f;
        res[s].dual = o.dual;
        res[s].primal = o.primal;
        res[s].gap = o.gap;
        conv = conv && o.converged;
    }
    return conv ? GN_OK : GN_NOT_CONVERGED;
}
