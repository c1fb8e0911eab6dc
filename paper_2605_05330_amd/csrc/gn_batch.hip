// Batched WRGN: many independent graphs in one persistent launch.
//
// Components do not interact (Section 2, property iii), so every graph is
// iterated to its own binarisation by one workgroup: the workgroup pulls a
// graph from a device work queue (largest graphs first), keeps the graph's
// weighted state y (ping-pong) in LDS, and runs the fused WRGN
// step with a workgroup barrier between steps instead of a grid-wide one.  A
// graph whose column lines also fit in the workgroup's LDS is copied there
// once, so its steps touch no global memory; a graph too large for the state
// falls back to global ping-pong buffers.  Each graph has its own step
// counter, gamma_k and stopping test; a finished graph frees its workgroup for
// the next one.  Row sums use the library's canonical order (gn_rowsum.h), so
// every graph's states, steps and selected set are bit-identical to gn_solve
// on that graph alone.
//
// Sliced column layout (graphs of at most 65535 vertices).  Each degree class
// of rows is cut into slices: 64 light rows (one per lane), 8 mid rows (8 lanes
// each) or one heavy row (the whole wavefront).  A slice is a run of lines of
// 64 16-bit ids, an even number of them; in line q, lane l holds entry q of
// its light row, entry t + 8q of mid row l / 8 (t = l mod 8), or entry l + 64q
// of the heavy row: the entry that chain q of that thread takes in the
// canonical order.
// Positions past a row's end hold n, the id of a state slot that stays zero,
// so they add exactly 0 and mark no selection.  Rows are sorted by degree
// inside each class, which keeps the padding small.  A line is read by one
// 128-byte access, the wavefront needs no row offsets inside a step, and the
// per-position predicates of the plain CSR walk disappear.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>
#include <type_traits>
#include <vector>

#include "gn_internal.h"
#include "gn_rowsum.h"

using gnk::sign_of;

namespace {

constexpr int kLightMaxDeg = 16;  // rows up to this degree run one per thread (64 rows per slice)
constexpr int kMidMaxDeg = 64;    // rows up to this degree run 8 threads per row (8 rows per slice)
constexpr int kLdsBudget = 160 * 1024 - 2048;  // dynamic LDS per CU (static LDS of the kernel set aside)
constexpr int32_t kMaxSlicedN = 65535;          // largest graph with a sliced layout (ids and the zero slot fit 16 bits)

struct BatchDesc {
    int32_t n;        // vertices
    int32_t n_light;  // internal rows [0, n_light) have degree <= kLightMaxDeg
    int32_t n_mid;    // rows [n_light, n_mid) have degree <= kMidMaxDeg, rows [n_mid, n) more
    int32_t n_lines;  // lines of the sliced layout (0 without one)
    int64_t v_off;    // offset of the graph's vertices in the vertex arrays
    int64_t rp_off;   // offset of its row_ptr (n + 1 entries)
    int64_t e_off;    // offset of its columns
    int64_t ln_off;   // first line of its sliced layout
    int64_t so_off;   // offset of its slice table: first line of each slice (relative to ln_off), slices + 1 entries
    int32_t nnz;      // CSR entries
    int32_t pad1;
};

// Slices of a graph: light slices, then mid slices, then one per heavy row.
__host__ __device__ inline int32_t slice_count(int32_t n, int32_t nl, int32_t nm) {
    return (nl + 63) / 64 + (nm - nl + 7) / 8 + (n - nm);
}

// LDS bytes of a graph in the LDS launch: y and y' (n + 1 words each, the last
// one the zero slot) and the slice table; MODE_ALL adds the lines.  v is read
// from global memory: only its own row reads it, once per step, with a load
// that does not wait on anything else.
__host__ __device__ inline int64_t state_lds_bytes(int64_t n, int64_t slices) { return 8 * n + 8 + 4 * (slices + 1); }
__host__ __device__ inline int64_t all_lds_bytes(int64_t n, int64_t slices, int64_t lines) {
    return state_lds_bytes(n, slices) + 128 * lines;
}

// Where a graph's arrays live while its workgroup iterates it.
enum BatchMode {
    MODE_GLOBAL = 0,  // state in the global ping-pong buffers, CSR read from global memory
    MODE_STREAM = 1,  // state and slice table in LDS, column lines read from global memory
    MODE_ALL = 2      // state, slice table and column lines in LDS: the steps touch no global memory
};

struct BatchRes {
    int32_t steps, binarised;
    long long fallback;
    double relaxed, set_w;
    long long size, conflicts, uncovered;
    float stab;
    int32_t pad;
};

struct BatchArgs {
    const BatchDesc* desc;
    const int32_t* order;    // graph ids this launch processes, most entries first
    int32_t count;
    int32_t qslot;           // queue counter this launch draws from
    const int32_t* row_ptr;  // internal, per graph
    const int32_t* col;      // internal local ids
    const uint16_t* lines;   // sliced layouts, 64 ids per line
    const int32_t* slices;   // slice tables
    const float* v;          // internal order
    const float* w;          // internal order
    const int32_t* perm;     // internal row -> user local id, per graph
    const float* gamma;      // gamma table, >= max_steps + 1 entries
    int32_t max_steps, check_every;
    float tau;
    int32_t lds_vertices;    // dynamic LDS per workgroup: 12 * lds_vertices bytes
    float* x_cat;            // user order; x0 in, final x out
    uint8_t* sel_cat;
    float* yg0;              // global ping-pong state for the graphs of the global launch
    float* yg1;
    int32_t* queue;          // [0]: next slot of the LDS launch, [1]: error bits, [2]: next slot of the global launch
    BatchRes* res;
};

__device__ __forceinline__ bool step_row(float yraw, float vi, float sigma, bool nbr_sel, float g, bool do_test,
                                         bool do_write, float tau, float* y_out, int i, int& fb) {
    const float yi = fabsf(yraw);
    const float s = __fmaf_rn(g, sigma, yi);
    const bool fallback = !(s > 1e-9f);
    const float xn = fallback ? 0.5f : gnk::bounded_ratio(yi, s);
    if (do_write) {
        const float yn = vi * xn;
        y_out[i] = xn > 0.5f ? -yn : yn;
        fb += fallback ? 1 : 0;
    }
    if (!do_test) return false;
    const bool in_s = sign_of(yraw) != 0u;
    const float tv = tau * vi;
    const bool far = (yi > tv) && ((vi - yi) > tv);
    const bool uncovered = !in_s && !nbr_sel;
    const bool growing = !in_s && (yi > 0.0f) && !(s > vi);
    return far || uncovered || growing;
}

// Workgroup vote "some row failed the stopping test" with one barrier per step.
// A wavefront with a failure sets flags[f]; every thread reads it after the
// barrier; thread 0 then clears flags[(f + 2) mod 3], which was read before this
// barrier and is written again only after the next one.  The three flags must
// be zero before the first step.  The barrier also orders the step's state
// writes before the next step's reads.
__device__ __forceinline__ bool block_any_step(bool viol, int* flags, int& f) {
    if (__ballot(viol) != 0ull && (threadIdx.x & 63) == 0) flags[f] = 1;
    __syncthreads();
    const bool any = flags[f] != 0;
    const int nx = f == 2 ? 0 : f + 1;
    if (threadIdx.x == 0) flags[nx == 2 ? 0 : nx + 1] = 0;
    f = nx;
    return any;
}

template <int BT>
__device__ double block_sum_d(double x, double* sm) {
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sm[wave] = x;
    __syncthreads();
    double r = 0.0;
#pragma unroll 1
    for (int w = 0; w < BT / 64; ++w) r += sm[w];
    return r;
}

template <int BT>
__device__ long long block_sum_ll(long long x, long long* sm) {
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sm[wave] = x;
    __syncthreads();
    long long r = 0;
#pragma unroll 1
    for (int w = 0; w < BT / 64; ++w) r += sm[w];
    return r;
}

template <int BT>
__device__ float block_min_f(float x, float* sm) {
    for (int off = 32; off >= 1; off >>= 1) x = fminf(x, __shfl_xor(x, off, 64));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sm[wave] = x;
    __syncthreads();
    float r = INFINITY;
#pragma unroll 1
    for (int w = 0; w < BT / 64; ++w) r = fminf(r, sm[w]);
    return r;
}

// Rows [rb, re) of degree <= MAXD in CSR form: 8 threads per row, 8 rows per
// wavefront per round (the loop bound is uniform over the wavefront, as the
// group shuffles need).  Returns the rows' stopping-test failures.
template <int BT, int MAXD, bool GLOBAL_RP, typename CT>
__device__ __forceinline__ bool mid_rows(const int32_t* __restrict__ rp, const CT* __restrict__ col,
                                         const float* yin, const float* vv, float* yout, int rb, int re, float g,
                                         bool do_test, bool do_write, float tau, int& fb) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, t = lane & 7;
    bool viol = false;
#pragma unroll 1
    for (int base = rb + wave * 8; base < re; base += (BT / 64) * 8) {
        const int i = base + (lane >> 3);
        const bool valid = i < re;
        int s0 = 0, dd = 0;
        if (valid) {
            s0 = GLOBAL_RP ? gnk::ld_stream(rp + i) : rp[i];
            dd = (GLOBAL_RP ? gnk::ld_stream(rp + i + 1) : rp[i + 1]) - s0;
        }
        unsigned sel = 0u;
        const float sigma = gnk::row_sum<8, MAXD>(col + s0, dd, yin, t, sel);
        const bool any_sel = gnk::group_any<8>(sel != 0u);
        if (valid && t == 0) viol |= step_row(yin[i], vv[i], sigma, any_sel, g, do_test, do_write, tau, yout, i, fb);
    }
    return viol;
}

// Row sum over the first K lines of a light (G = 1, NQ = 16) or mid (G = 8,
// NQ = 8) slice in the canonical order: line q feeds chain q mod NQ of the
// thread, in increasing q (a mid row of degree up to 128 has two lines per
// chain), the chains meet in the in-thread butterfly, then the group's
// shuffles.  `ln` points at this lane's id in the slice's first line; the
// lines are 64 ids apart.  ORs the raw bits of the gathered values into `bits`
// (bit 31: some neighbour is selected).  Straight-line code: the K id loads,
// then the K gathers, each phase back to back.  Chains without a line are
// zero, and adding zero to a sum of magnitudes (never -0) changes nothing, so
// those additions of the butterfly are left out.  ABS = false sums the raw
// (signed) values, as the adjoint does: every chain starts at +0 and adds, so
// no partial sum is ever -0 (round to nearest) and the skipped additions of
// zero still change nothing.
template <int G, int NQ, int K, bool ABS = true, typename LT>
__device__ __forceinline__ float slice_sum_k(const LT* __restrict__ ln, const float* __restrict__ y,
                                             unsigned& bits) {
    int id[K > 0 ? K : 1];
    float c[NQ];
#pragma unroll
    for (int q = 0; q < K; ++q) id[q] = ln[64 * q];
#pragma unroll
    for (int q = 0; q < NQ; ++q) c[q] = 0.0f;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const float yv = y[id[q]];
        if (q < NQ) c[q] = ABS ? fabsf(yv) : 0.0f + yv;
        else c[q % NQ] += ABS ? fabsf(yv) : yv;
        if (ABS) bits |= __float_as_uint(yv);
    }
#pragma unroll
    for (int h = NQ / 2; h >= 1; h >>= 1)
#pragma unroll
        for (int j = 0; j < h; ++j)
            if (j + h < K) c[j] += c[j + h];
    float s = c[0];
#pragma unroll
    for (int off = G / 2; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    return s;
}

// The same for a slice of W lines, W even (slices are padded to an even number
// of lines), at most MAXL and uniform over the wavefront: one straight-line
// variant per W.
template <int G, int NQ, int MAXL, bool ABS = true, typename LT>
__device__ __forceinline__ float slice_sum(const LT* __restrict__ ln, int W, const float* __restrict__ y,
                                           unsigned& bits) {
    static_assert(MAXL % 2 == 0 && MAXL <= 16, "slice widths");
    switch (W) {
        case 2: return slice_sum_k<G, NQ, 2, ABS>(ln, y, bits);
        case 4: return slice_sum_k<G, NQ, 4, ABS>(ln, y, bits);
        case 6: return slice_sum_k<G, NQ, 6, ABS>(ln, y, bits);
        case 8: return slice_sum_k<G, NQ, 8, ABS>(ln, y, bits);
        case 10: if constexpr (MAXL >= 10) return slice_sum_k<G, NQ, 10, ABS>(ln, y, bits); else break;
        case 12: if constexpr (MAXL >= 12) return slice_sum_k<G, NQ, 12, ABS>(ln, y, bits); else break;
        case 14: if constexpr (MAXL >= 14) return slice_sum_k<G, NQ, 14, ABS>(ln, y, bits); else break;
        case 16: if constexpr (MAXL >= 16) return slice_sum_k<G, NQ, 16, ABS>(ln, y, bits); else break;
        default: break;
    }
    return slice_sum_k<G, NQ, 0, ABS>(ln, y, bits);
}

// K lines of a heavy slice added to the lane's chain, in line order.
template <int K, bool ABS = true, typename LT>
__device__ __forceinline__ void heavy_lines(const LT* __restrict__ ln, const float* __restrict__ y, float& acc,
                                            unsigned& bits) {
    int id[K];
    float yv[K];
#pragma unroll
    for (int q = 0; q < K; ++q) id[q] = ln[64 * q];
#pragma unroll
    for (int q = 0; q < K; ++q) yv[q] = y[id[q]];
#pragma unroll
    for (int q = 0; q < K; ++q) {
        acc += ABS ? fabsf(yv[q]) : yv[q];
        if (ABS) bits |= __float_as_uint(yv[q]);
    }
}

// Row sum over a heavy slice (one row, the whole wavefront; W even): lane l
// adds entries l + 64q in increasing q (the chain of virtual lane l), eight
// lines in flight at a time, then the 64-lane butterfly.
template <bool ABS = true, typename LT>
__device__ __forceinline__ float heavy_sum(const LT* __restrict__ ln, int W, const float* __restrict__ y,
                                           unsigned& bits) {
    float acc = 0.0f;
    int q0 = 0;
#pragma unroll 1
    for (; q0 + 8 <= W; q0 += 8) heavy_lines<8, ABS>(ln + 64 * q0, y, acc, bits);
    switch (W - q0) {
        case 2: heavy_lines<2, ABS>(ln + 64 * q0, y, acc, bits); break;
        case 4: heavy_lines<4, ABS>(ln + 64 * q0, y, acc, bits); break;
        case 6: heavy_lines<6, ABS>(ln + 64 * q0, y, acc, bits); break;
        default: break;
    }
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    return acc;
}

template <int BT, int MODE>
__device__ void solve_graph(const BatchArgs& a, const BatchDesc& d, int gi, float* lds) {
    __shared__ double sm_d[BT / 64];
    __shared__ long long sm_l[BT / 64];
    __shared__ float sm_f[BT / 64];
    __shared__ int s_flags[3];
    constexpr int NW = BT / 64;
    constexpr bool SL = MODE != MODE_GLOBAL;  // sliced layout, state in LDS
    const int n = d.n;
    // the wavefront index is uniform: stated, the slice loops compile to scalar branches
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (n == 0) return;  // result filled on the host
    const int32_t* __restrict__ rp_g = a.row_ptr + d.rp_off;
    const int32_t* __restrict__ col_g = a.col + d.e_off;
    const int32_t* __restrict__ perm = a.perm + d.v_off;
    float* ya = SL ? lds : a.yg0 + d.v_off;
    float* yb = SL ? lds + (n + 1) : a.yg1 + d.v_off;
    const float* __restrict__ vv = a.v + d.v_off;
    const int nL = (d.n_light + 63) / 64, nM = (d.n_mid - d.n_light + 7) / 8;
    const int nS = nL + nM + (n - d.n_mid);
    const int w_mid = (wave - nL % NW + NW) % NW;          // first mid slice of this wavefront
    const int w_heavy = (wave - (nL + nM) % NW + NW) % NW;  // first heavy slice
    int32_t* so = reinterpret_cast<int32_t*>(lds + 2 * n + 2);
    uint16_t* ln_l = reinterpret_cast<uint16_t*>(so + nS + 1);
    const uint16_t* __restrict__ ln_g = a.lines + d.ln_off * 64;
    const uint16_t* __restrict__ ln;
    if constexpr (MODE == MODE_ALL) ln = ln_l;
    else ln = ln_g;
    float* xg = a.x_cat + d.v_off;

    for (int i = tid; i < n; i += BT) {
        const float vi = vv[i];
        const float x = xg[perm[i]];
        const float yy = vi * x;
        ya[i] = x > 0.5f ? -yy : yy;
    }
    if constexpr (SL) {
        if (tid == 0) {
            ya[n] = 0.0f;
            yb[n] = 0.0f;
        }
        for (int s = tid; s <= nS; s += BT) so[s] = a.slices[d.so_off + s];
        if constexpr (MODE == MODE_ALL) {
            const uint32_t* __restrict__ src = reinterpret_cast<const uint32_t*>(ln_g);
            uint32_t* dst = reinterpret_cast<uint32_t*>(ln_l);
            const int nw = d.n_lines * 32;
            for (int w = tid; w < nw; w += 4 * BT) {
                uint32_t t[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) t[u] = w + u * BT < nw ? src[w + u * BT] : 0u;
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (w + u * BT < nw) dst[w + u * BT] = t[u];
            }
        }
    }
    if (tid < 3) s_flags[tid] = 0;
    __syncthreads();

    float* yin = ya;
    float* yout = yb;
    int fb = 0;
    int steps = 0;
    bool binarised = false;
    int fslot = 0, kc = 0;  // vote slot; k mod check_every
    float g_next = a.gamma[0];
    for (int k = 0;; ++k) {
        const bool do_test = k >= 1 && (kc == 0 || k == a.max_steps);
        const bool do_write = k < a.max_steps;
        // gamma of the next step is loaded one step ahead (the table covers
        // indices 0 .. max_steps): its scalar load never holds up the step's
        // LDS waits
        const float g = g_next;
        if (k + 1 <= a.max_steps) g_next = a.gamma[k + 1];
        bool viol = false;
        if constexpr (SL) {
            // slices are dealt round robin over the wavefronts across the three
            // classes in turn, so no wavefront takes more than ceil(slices / NW)
#pragma unroll 1
            for (int s = wave; s < nL; s += NW) {
                const int i = 64 * s + lane;
                const bool valid = i < d.n_light;
                const float vi = valid ? vv[i] : 1.0f;
                const int o = so[s];
                const int W = __builtin_amdgcn_readfirstlane(so[s + 1] - o);
                unsigned bits = 0u;
                const float sigma = slice_sum<1, 16, kLightMaxDeg>(ln + o * 64 + lane, W, yin, bits);
                if (valid)
                    viol |= step_row(yin[i], vi, sigma, (bits >> 31) != 0u, g, do_test, do_write, a.tau, yout, i, fb);
            }
#pragma unroll 1
            for (int s = w_mid; s < nM; s += NW) {
                const int i = d.n_light + 8 * s + (lane >> 3);
                const bool valid = i < d.n_mid && (lane & 7) == 0;
                const float vi = valid ? vv[i] : 1.0f;
                const int o = so[nL + s];
                const int W = __builtin_amdgcn_readfirstlane(so[nL + s + 1] - o);
                unsigned bits = 0u;
                const float sigma = slice_sum<8, 8, kMidMaxDeg / 8>(ln + o * 64 + lane, W, yin, bits);
                const bool any_sel = gnk::group_any<8>((bits >> 31) != 0u);
                if (valid) viol |= step_row(yin[i], vi, sigma, any_sel, g, do_test, do_write, a.tau, yout, i, fb);
            }
#pragma unroll 1
            for (int s = w_heavy; s < n - d.n_mid; s += NW) {
                const int i = d.n_mid + s;
                const float vi = lane == 0 ? vv[i] : 1.0f;
                const int o = so[nL + nM + s];
                const int W = __builtin_amdgcn_readfirstlane(so[nL + nM + s + 1] - o);
                unsigned bits = 0u;
                const float sigma = heavy_sum(ln + o * 64 + lane, W, yin, bits);
                const bool any_sel = __any((bits >> 31) != 0u);
                if (lane == 0) viol |= step_row(yin[i], vi, sigma, any_sel, g, do_test, do_write, a.tau, yout, i, fb);
            }
        } else {
#pragma unroll 1
            for (int i = tid; i < d.n_light; i += BT) {
                const int s0 = gnk::ld_stream(rp_g + i);
                const int dd = gnk::ld_stream(rp_g + i + 1) - s0;
                unsigned sel = 0u;
                const float sigma = gnk::row_sum<1, kLightMaxDeg>(col_g + s0, dd, yin, 0, sel);
                viol |= step_row(yin[i], vv[i], sigma, sel != 0u, g, do_test, do_write, a.tau, yout, i, fb);
            }
            viol |= mid_rows<BT, kMidMaxDeg, true>(rp_g, col_g, yin, vv, yout, d.n_light, d.n_mid, g, do_test,
                                                   do_write, a.tau, fb);
#pragma unroll 1
            for (int i = d.n_mid + wave; i < n; i += NW) {
                const int s0 = gnk::ld_stream(rp_g + i);
                const int dd = gnk::ld_stream(rp_g + i + 1) - s0;
                unsigned sel = 0u;
                const float sigma = gnk::row_sum_wave<8>(col_g + s0, dd, yin, lane, sel);
                const bool any_sel = __any(sel != 0u);
                if (lane == 0) viol |= step_row(yin[i], vv[i], sigma, any_sel, g, do_test, do_write, a.tau, yout, i, fb);
            }
        }
        const bool any = block_any_step(viol, s_flags, fslot);
        if (do_test && !any) {
            binarised = true;
            steps = k;
            break;
        }
        if (!do_write) {
            steps = k;
            break;
        }
        float* t = yin;
        yin = yout;
        yout = t;
        kc = kc + 1 == a.check_every ? 0 : kc + 1;
    }

    // final state, rounded set, and the statistics of the set (one more pass,
    // over the CSR in global memory)
    for (int i = tid; i < n; i += BT) {
        float x = fabsf(yin[i]) / vv[i];
        x = fminf(fmaxf(x, 0.0f), 1.0f);
        const uint8_t s = x > 0.5f ? 1 : 0;
        xg[perm[i]] = x;
        a.sel_cat[d.v_off + perm[i]] = s;
        yout[i] = s ? 1.0f : 0.0f;  // selection flags for the pass below
    }
    __syncthreads();
    double relaxed = 0.0, set_w = 0.0;
    long long size = 0, conf = 0, unc = 0;
    float stab = INFINITY;
    for (int i = tid; i < n; i += BT) {
        const bool in_s = yout[i] != 0.0f;
        float x = fabsf(yin[i]) / vv[i];
        x = fminf(fmaxf(x, 0.0f), 1.0f);
        const float wi = a.w[d.v_off + i];
        relaxed += (double)wi * (double)x;
        bool any = false;
        float vsum = 0.0f;
        for (int e = rp_g[i]; e < rp_g[i + 1]; ++e) {
            const int j = col_g[e];
            if (yout[j] != 0.0f) {
                any = true;
                if (in_s && j > i) conf += 1;
                if (!in_s) vsum += vv[j];
            }
        }
        if (in_s) {
            set_w += (double)wi;
            size += 1;
        } else {
            if (!any) unc += 1;
            stab = fminf(stab, vsum / vv[i]);
        }
    }
    long long fbl = fb;
    relaxed = block_sum_d<BT>(relaxed, sm_d);
    set_w = block_sum_d<BT>(set_w, sm_d);
    size = block_sum_ll<BT>(size, sm_l);
    conf = block_sum_ll<BT>(conf, sm_l);
    unc = block_sum_ll<BT>(unc, sm_l);
    fbl = block_sum_ll<BT>(fbl, sm_l);
    stab = block_min_f<BT>(stab, sm_f);
    if (tid == 0) {
        BatchRes r;
        r.steps = steps;
        r.binarised = binarised ? 1 : 0;
        r.fallback = fbl;
        r.relaxed = relaxed;
        r.set_w = set_w;
        r.size = size;
        r.conflicts = conf;
        r.uncovered = unc;
        r.stab = isinf(stab) ? INFINITY : a.gamma[steps] * stab;
        r.pad = 0;
        a.res[gi] = r;
    }
    __syncthreads();
}

// The persistent kernel.  BIG = false: graphs whose state fits in LDS
// (MODE_ALL or MODE_STREAM); BIG = true: the others (MODE_GLOBAL), in a launch
// of their own, because the 64-bit gathers of that path would otherwise raise
// the register count of the common one.
template <int BT, bool BIG>
__global__ __launch_bounds__(BT) void batch_solve_kernel(BatchArgs a) {
    extern __shared__ float lds[];
    __shared__ int s_g;
    if (a.queue[1] != 0) return;  // x0 rejected: leave every output untouched
    for (;;) {
        if (threadIdx.x == 0) s_g = atomicAdd(a.queue + a.qslot, 1);
        __syncthreads();
        const int q = s_g;
        __syncthreads();
        if (q >= a.count) break;
        const int gi = a.order[q];
        const BatchDesc d = a.desc[gi];
        if constexpr (BIG) {
            solve_graph<BT, MODE_GLOBAL>(a, d, gi, lds);
        } else {
            const int64_t slices = slice_count(d.n, d.n_light, d.n_mid);
            if (all_lds_bytes(d.n, slices, d.n_lines) <= 12 * (int64_t)a.lds_vertices)
                solve_graph<BT, MODE_ALL>(a, d, gi, lds);
            else
                solve_graph<BT, MODE_STREAM>(a, d, gi, lds);
        }
    }
}

// ---------------------------------------------------------------------------
// Unrolled (differentiable) steps of a whole batch: every graph's T forward
// steps, or its T adjoint steps, in one workgroup with its state in LDS.  The
// arithmetic repeats the chained unrolled path (gn_unrolled.hip) operation for
// operation -- y = v x, s = y + gamma sum |y_j|, x' = y / s with the safe
// division and support bound; t = gbar y / s^2, dL/dy = gbar / s - (t + gamma
// sum t_j), dL/dx = v dL/dy, dL/dv += x dL/dy, dL/dw = dL/dv / (2 v) -- with the
// same canonical sums, so results are bit-identical to it on the batch's
// block-diagonal union graph.
// ---------------------------------------------------------------------------
struct UnrolledArgs {
    const BatchDesc* desc;
    const int32_t* order;    // graphs, most entries first
    int32_t count;
    int32_t* queue;          // next graph to take
    const int32_t* perm;
    const uint16_t* lines;
    const int32_t* slices;
    const float* v;          // sqrt(w), internal order
    const float* gamma;      // [T]
    int32_t T;
    int32_t lds_bytes;       // dynamic LDS per workgroup
    int64_t total_n;
    const float* x0;         // forward: x0 and xT, user order
    float* xT;
    float* store;            // y of every step ([T][total_n]), then s ([T][total_n]), internal order
    const float* gxT;        // backward: dL/dx^T in, dL/dx^0 and dL/dw out, user order
    float* gx0;
    float* gw;
};

// Whether the forward step took the quotient branch at this row (the same test
// on the same fp32 values as the chained adjoint).
__device__ __forceinline__ bool unrolled_quotient(float y, float s) {
    if (!(s > 1e-9f)) return false;
    return !(y > 0.0f && y / s < gnk::kXMin);
}

// Slice loops of one step over a graph's sliced layout: for every valid row,
// `load(i)` (the row's own global values, issued before the neighbour sum so
// that their latency hides behind it), then `row(i, sigma, loaded)` with the
// neighbour sum over `src` (absolute values when ABS).
template <int BT, bool ABS, typename LT, typename Load, typename Row>
__device__ __forceinline__ void unrolled_slices(const BatchDesc& d, const int32_t* so, const LT* __restrict__ ln,
                                                const float* src, Load&& load, Row&& row) {
    using Pre = decltype(load(0));
    constexpr int NW = BT / 64;
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n = d.n;
    const int nL = (d.n_light + 63) / 64, nM = (d.n_mid - d.n_light + 7) / 8;
    const int w_mid = (wave - nL % NW + NW) % NW;
    const int w_heavy = (wave - (nL + nM) % NW + NW) % NW;
#pragma unroll 1
    for (int s = wave; s < nL; s += NW) {
        const int i = 64 * s + lane;
        const bool valid = i < d.n_light;
        Pre pre{};
        if (valid) pre = load(i);
        const int o = so[s];
        const int W = __builtin_amdgcn_readfirstlane(so[s + 1] - o);
        unsigned bits = 0u;
        const float sigma = slice_sum<1, 16, kLightMaxDeg, ABS>(ln + o * 64 + lane, W, src, bits);
        if (valid) row(i, sigma, pre);
    }
#pragma unroll 1
    for (int s = w_mid; s < nM; s += NW) {
        const int i = d.n_light + 8 * s + (lane >> 3);
        const bool valid = i < d.n_mid && (lane & 7) == 0;
        Pre pre{};
        if (valid) pre = load(i);
        const int o = so[nL + s];
        const int W = __builtin_amdgcn_readfirstlane(so[nL + s + 1] - o);
        unsigned bits = 0u;
        const float sigma = slice_sum<8, 8, kMidMaxDeg / 8, ABS>(ln + o * 64 + lane, W, src, bits);
        if (valid) row(i, sigma, pre);
    }
#pragma unroll 1
    for (int s = w_heavy; s < n - d.n_mid; s += NW) {
        const int i = d.n_mid + s;
        Pre pre{};
        if (lane == 0) pre = load(i);
        const int o = so[nL + nM + s];
        const int W = __builtin_amdgcn_readfirstlane(so[nL + nM + s + 1] - o);
        unsigned bits = 0u;
        const float sigma = heavy_sum<ABS>(ln + o * 64 + lane, W, src, bits);
        if (lane == 0) row(i, sigma, pre);
    }
}

struct FwdPre {
    float v;
};
struct BwdPre {
    float v, y, s, yp, sp;
};

// Copies a graph's slice table (and, MODE_ALL, its lines) into LDS at `so`.
template <int BT, int MODE>
__device__ __forceinline__ const uint16_t* unrolled_stage(const UnrolledArgs& a, const BatchDesc& d, int32_t* so) {
    const int tid = threadIdx.x;
    const int nS = slice_count(d.n, d.n_light, d.n_mid);
    uint16_t* ln_l = reinterpret_cast<uint16_t*>(so + nS + 1);
    const uint16_t* ln_g = a.lines + d.ln_off * 64;
    for (int s = tid; s <= nS; s += BT) so[s] = a.slices[d.so_off + s];
    if constexpr (MODE == MODE_ALL) {
        const uint32_t* __restrict__ src = reinterpret_cast<const uint32_t*>(ln_g);
        uint32_t* dst = reinterpret_cast<uint32_t*>(ln_l);
        const int nw = d.n_lines * 32;
        for (int w = tid; w < nw; w += BT) dst[w] = src[w];
        return ln_l;
    } else {
        return ln_g;
    }
}

// T forward steps of one graph; LDS: y, y' (n + 1 words each, the last the zero
// slot), slice table, lines (MODE_ALL).
template <int BT, int MODE>
__device__ void unrolled_fwd_graph(const UnrolledArgs& a, const BatchDesc& d, float* lds) {
    const int n = d.n;
    if (n == 0) return;
    const int tid = threadIdx.x;
    float* ya = lds;
    float* yb = lds + (n + 1);
    int32_t* so = reinterpret_cast<int32_t*>(lds + 2 * n + 2);
    const float* __restrict__ vv = a.v + d.v_off;
    const int32_t* __restrict__ perm = a.perm + d.v_off;
    for (int i = tid; i < n; i += BT) ya[i] = vv[i] * a.x0[d.v_off + perm[i]];
    if (tid == 0) {
        ya[n] = 0.0f;
        yb[n] = 0.0f;
    }
    const uint16_t* ln;
    if constexpr (MODE == MODE_ALL) ln = unrolled_stage<BT, MODE>(a, d, so);
    else ln = unrolled_stage<BT, MODE>(a, d, so);
    __syncthreads();
    float* yin = ya;
    float* yout = yb;
    for (int t = 0; t < a.T; ++t) {
        const float g = a.gamma[t];
        float* ys = a.store + (int64_t)t * a.total_n + d.v_off;
        float* ss = a.store + (int64_t)(a.T + t) * a.total_n + d.v_off;
        float* xT = t == a.T - 1 ? a.xT + d.v_off : nullptr;
        unrolled_slices<BT, true>(
            d, so, ln, yin, [&](int i) { return FwdPre{vv[i]}; },
            [&](int i, float sigma, const FwdPre& p) {
                const float yraw = yin[i];
                const float yi = fabsf(yraw);
                const float s = __fmaf_rn(g, sigma, yi);
                const float xn = !(s > 1e-9f) ? 0.5f : gnk::bounded_ratio(yi, s);
                ys[i] = yraw;
                ss[i] = s;
                const float yn = p.v * xn;
                yout[i] = xn > 0.5f ? -yn : yn;
                if (xT) xT[perm[i]] = xn;
            });
        __syncthreads();
        float* tmp = yin;
        yin = yout;
        yout = tmp;
    }
}

// T adjoint steps of one graph, last to first; LDS: t (ping-pong, n + 1 words
// each with the zero slot), dL/dx, dL/dv (n words each), slice table, lines.
template <int BT, int MODE>
__device__ void unrolled_bwd_graph(const UnrolledArgs& a, const BatchDesc& d, float* lds) {
    const int n = d.n;
    if (n == 0) return;
    const int tid = threadIdx.x;
    float* ta = lds;
    float* tb = lds + (n + 1);
    float* gb = lds + 2 * (n + 1);
    float* gv = gb + n;
    int32_t* so = reinterpret_cast<int32_t*>(gv + n);
    const float* __restrict__ vv = a.v + d.v_off;
    const int32_t* __restrict__ perm = a.perm + d.v_off;
    const int T = a.T;
    const float* ylast = a.store + (int64_t)(T - 1) * a.total_n + d.v_off;
    const float* slast = a.store + (int64_t)(2 * T - 1) * a.total_n + d.v_off;
    for (int i = tid; i < n; i += BT) {
        const float g = a.gxT[d.v_off + perm[i]];
        gb[i] = g;
        gv[i] = 0.0f;
        const float yy = fabsf(ylast[i]), s = slast[i];
        ta[i] = unrolled_quotient(yy, s) ? (g / s) * (yy / s) : 0.0f;
    }
    if (tid == 0) {
        ta[n] = 0.0f;
        tb[n] = 0.0f;
    }
    const uint16_t* ln;
    if constexpr (MODE == MODE_ALL) ln = unrolled_stage<BT, MODE>(a, d, so);
    else ln = unrolled_stage<BT, MODE>(a, d, so);
    __syncthreads();
    float* tin = ta;
    float* tout = tb;
    for (int t = T - 1; t >= 0; --t) {
        const float gam = a.gamma[t];
        const float* yk = a.store + (int64_t)t * a.total_n + d.v_off;
        const float* sk = a.store + (int64_t)(T + t) * a.total_n + d.v_off;
        const float* yp = t > 0 ? a.store + (int64_t)(t - 1) * a.total_n + d.v_off : nullptr;
        const float* sp = t > 0 ? a.store + (int64_t)(T + t - 1) * a.total_n + d.v_off : nullptr;
        unrolled_slices<BT, false>(
            d, so, ln, tin,
            [&](int i) {
                BwdPre p;
                p.v = vv[i];
                p.y = fabsf(yk[i]);
                p.s = sk[i];
                p.yp = yp ? fabsf(yp[i]) : 0.0f;
                p.sp = yp ? sp[i] : 0.0f;
                return p;
            },
            [&](int i, float sigma, const BwdPre& p) {
                const float g = gb[i];
                const float ai = unrolled_quotient(p.y, p.s) ? g / p.s : 0.0f;
                const float gy = ai - __fmaf_rn(gam, sigma, tin[i]);
                const float gx = p.v * gy;
                gb[i] = gx;
                gv[i] += (p.y / p.v) * gy;
                if (yp) tout[i] = unrolled_quotient(p.yp, p.sp) ? (gx / p.sp) * (p.yp / p.sp) : 0.0f;
            });
        __syncthreads();
        float* tmp = tin;
        tin = tout;
        tout = tmp;
    }
    for (int i = tid; i < n; i += BT) {
        a.gx0[d.v_off + perm[i]] = gb[i];
        a.gw[d.v_off + perm[i]] = gv[i] / (2.0f * vv[i]);
    }
    __syncthreads();
}

// LDS bytes of one graph in the unrolled kernels: the state words of the
// forward (2) or adjoint (4) pass per vertex, the zero slots, the slice table,
// and -- with lines -- the lines.
__host__ __device__ inline int64_t unrolled_state_bytes(bool bwd, int64_t n, int64_t slices) {
    return (bwd ? 16 : 8) * n + 8 + 4 * (slices + 1);
}

template <int BT, bool BWD>
__global__ __launch_bounds__(BT) void batch_unrolled_kernel(UnrolledArgs a) {
    extern __shared__ float lds[];
    __shared__ int s_g;
    for (;;) {
        if (threadIdx.x == 0) s_g = atomicAdd(a.queue, 1);
        __syncthreads();
        const int q = s_g;
        __syncthreads();
        if (q >= a.count) break;
        const BatchDesc d = a.desc[a.order[q]];
        const int64_t slices = slice_count(d.n, d.n_light, d.n_mid);
        const bool all = unrolled_state_bytes(BWD, d.n, slices) + 128 * (int64_t)d.n_lines <= a.lds_bytes;
        if constexpr (BWD) {
            if (all) unrolled_bwd_graph<BT, MODE_ALL>(a, d, lds);
            else unrolled_bwd_graph<BT, MODE_STREAM>(a, d, lds);
        } else {
            if (all) unrolled_fwd_graph<BT, MODE_ALL>(a, d, lds);
            else unrolled_fwd_graph<BT, MODE_STREAM>(a, d, lds);
        }
    }
}

// sqrt of caller weights (user order within each graph) into the batch's
// internal order: the same (float)sqrt((double)w) as the graph handles use.
__global__ void batch_sqrt_weights_kernel(int64_t total, const int32_t* __restrict__ vgraph,
                                          const BatchDesc* __restrict__ desc, const int32_t* __restrict__ perm,
                                          const float* __restrict__ w_cat, float* __restrict__ v) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const BatchDesc d = desc[vgraph[t]];
    v[t] = (float)sqrt((double)w_cat[d.v_off + perm[t]]);
}

// Reset queue / error bits and fill the gamma table (Section 6 gamma-pursuit).
__global__ void batch_init_kernel(int32_t* queue, float* gamma, int32_t max_steps, float g0, float g1, int32_t ramp) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) {
        queue[0] = 0;
        queue[1] = 0;
        queue[2] = 0;
    }
    for (int k = t; k <= max_steps; k += gridDim.x * blockDim.x) {
        double gk;
        if (ramp <= 1) {
            gk = (double)g1;
        } else {
            const int kk = k < ramp - 1 ? k : ramp - 1;
            const double p = (double)kk / (double)(ramp - 1);
            gk = p * (double)g1 + (1.0 - p) * (double)g0;
        }
        gamma[k] = (float)gk;
    }
}

// x0 checks for every graph: finite and >= 0 (error bit 1), normalizable: each
// vertex or one of its neighbours positive (error bit 2).  One thread per
// vertex of the concatenated batch.
__global__ void batch_check_x0_kernel(int64_t total, const int32_t* __restrict__ vgraph, const BatchDesc* __restrict__ desc,
                                      const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                      const int32_t* __restrict__ perm, const float* __restrict__ x_cat,
                                      int32_t* queue) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int gi = vgraph[t];
    const BatchDesc d = desc[gi];
    const int i = (int)(t - d.v_off);
    const float* xg = x_cat + d.v_off;
    const int32_t* pm = perm + d.v_off;
    const float x = xg[pm[i]];
    if (!(x >= 0.0f) || !isfinite(x)) {
        atomicOr(queue + 1, 1);
        return;
    }
    if (x > 0.0f) return;
    const int32_t* rp = row_ptr + d.rp_off;
    const int32_t* cl = col + d.e_off;
    for (int e = rp[i]; e < rp[i + 1]; ++e)
        if (xg[pm[cl[e]]] > 0.0f) return;
    atomicOr(queue + 1, 2);
}

// One small graph, one workgroup: the whole solve in a single launch, steps
// separated by workgroup barriers instead of kernel boundaries.  Works on the
// graph handle's internal order: rows [0, mid_begin) have degree > 128 (one
// wavefront each), rows [mid_begin, light_begin) degree 17 .. 128 (8 threads
// each), the rest degree <= 16 (a thread each).  The graph's LDS image -- the
// sliced layout of the head of this file, lines of up to 16 per mid slice --
// is copied into LDS with y (ping-pong, n + 1 words each with the zero slot);
// v is read from global memory by its own row.  Same arithmetic and canonical
// sums as the step kernel, so the result is bit-identical to the chained
// solve.  One compute unit does all the work, so this pays only while a step
// is small.  On entry y0 holds the signed starting state (prep_state_kernel);
// on exit the final state is in y0 or y1 by the parity of the step count, as
// after the chained solve.
struct SmallArgs {
    int32_t n, mid_begin, light_begin, n_lines;
    const int32_t* slices;   // slice table: light, mid, then heavy slices
    const uint16_t* lines;   // the slices' lines
    const float* v;
    const float* gamma;
    SolveState* st;
    int32_t* notconv;
    float* y0;
    float* y1;
};

template <int BT>
__global__ __launch_bounds__(BT) void small_solve_kernel(SmallArgs a) {
    extern __shared__ float lds[];
    __shared__ int s_fb;
    __shared__ int s_flags[3];
    constexpr int NW = BT / 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    SolveState* st = a.st;
    if (st->err) return;  // x0 rejected by the checks before this launch
    const int ms = st->max_steps, ce = st->check_every;
    const float tau = st->tau;
    const int n = a.n, mb = a.mid_begin, lb = a.light_begin;
    const int nL = (n - lb + 63) / 64, nM = (lb - mb + 7) / 8, nH = mb;
    const int nS = nL + nM + nH;
    const int w_mid = (wave - nL % NW + NW) % NW;
    const int w_heavy = (wave - (nL + nM) % NW + NW) % NW;
    float* ya = lds;
    float* yb = lds + (n + 1);
    int32_t* so = reinterpret_cast<int32_t*>(lds + 2 * n + 2);
    uint16_t* ln = reinterpret_cast<uint16_t*>(so + nS + 1);
    const float* __restrict__ vv = a.v;
    for (int i = tid; i < n; i += BT) ya[i] = a.y0[i];
    if (tid == 0) {
        ya[n] = 0.0f;
        yb[n] = 0.0f;
        s_fb = 0;
    }
    for (int s = tid; s <= nS; s += BT) so[s] = a.slices[s];
    {
        const uint32_t* __restrict__ src = reinterpret_cast<const uint32_t*>(a.lines);
        uint32_t* dst = reinterpret_cast<uint32_t*>(ln);
        const int nw = a.n_lines * 32;
        for (int w = tid; w < nw; w += 4 * BT) {
            uint32_t t[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) t[u] = w + u * BT < nw ? src[w + u * BT] : 0u;
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (w + u * BT < nw) dst[w + u * BT] = t[u];
        }
    }
    if (tid < 3) s_flags[tid] = 0;
    __syncthreads();
    float* yin = ya;
    float* yout = yb;
    int fb = 0;
    int steps = 0;
    bool binarised = false;
    float g_next = a.gamma[0];
    int fslot = 0, kc = 0;  // vote slot; k mod check_every
    for (int k = 0;; ++k) {
        const bool do_test = k >= 1 && (kc == 0 || k == ms);
        const bool do_write = k < ms;
        // gamma of the next step is loaded one step ahead (the table covers
        // indices 0 .. max_steps): no global round trip on the step's path
        const float g = g_next;
        if (k + 1 <= ms) g_next = a.gamma[k + 1];
        bool viol = false;
#pragma unroll 1
        for (int s = wave; s < nL; s += NW) {
            const int i = lb + 64 * s + lane;
            const bool valid = i < n;
            const float vi = valid ? vv[i] : 1.0f;
            const int o = so[s];
            const int W = __builtin_amdgcn_readfirstlane(so[s + 1] - o);
            unsigned bits = 0u;
            const float sigma = slice_sum<1, 16, 16>(ln + o * 64 + lane, W, yin, bits);
            if (valid) viol |= step_row(yin[i], vi, sigma, (bits >> 31) != 0u, g, do_test, do_write, tau, yout, i, fb);
        }
#pragma unroll 1
        for (int s = w_mid; s < nM; s += NW) {
            const int i = mb + 8 * s + (lane >> 3);
            const bool valid = i < lb && (lane & 7) == 0;
            const float vi = valid ? vv[i] : 1.0f;
            const int o = so[nL + s];
            const int W = __builtin_amdgcn_readfirstlane(so[nL + s + 1] - o);
            unsigned bits = 0u;
            const float sigma = slice_sum<8, 8, 16>(ln + o * 64 + lane, W, yin, bits);
            const bool any_sel = gnk::group_any<8>((bits >> 31) != 0u);
            if (valid) viol |= step_row(yin[i], vi, sigma, any_sel, g, do_test, do_write, tau, yout, i, fb);
        }
#pragma unroll 1
        for (int s = w_heavy; s < nH; s += NW) {
            const int i = s;
            const float vi = lane == 0 ? vv[i] : 1.0f;
            const int o = so[nL + nM + s];
            const int W = __builtin_amdgcn_readfirstlane(so[nL + nM + s + 1] - o);
            unsigned bits = 0u;
            const float sigma = heavy_sum(ln + o * 64 + lane, W, yin, bits);
            const bool any_sel = __any((bits >> 31) != 0u);
            if (lane == 0) viol |= step_row(yin[i], vi, sigma, any_sel, g, do_test, do_write, tau, yout, i, fb);
        }
        const bool any = block_any_step(viol, s_flags, fslot);
        if (do_test && !any) {
            binarised = true;
            steps = k;
            break;
        }
        if (!do_write) {
            steps = k;
            break;
        }
        float* t = yin;
        yin = yout;
        yout = t;
        kc = kc + 1 == ce ? 0 : kc + 1;
    }
    if (fb) atomicAdd(&s_fb, fb);
    float* dst = (steps & 1) ? a.y1 : a.y0;
    for (int i = tid; i < n; i += BT) dst[i] = yin[i];
    __syncthreads();
    if (tid == 0) {
        st->fallback = (unsigned long long)s_fb;
        if (binarised) st->done_step = steps;
        else a.notconv[ms] = 1;
    }
}

template <int BT, bool BIG>
const void* batch_kernel_ptr() {
    return (const void*)batch_solve_kernel<BT, BIG>;
}

}  // namespace

// The executable graph of the last solve and what it was built for.
struct BatchLaunch {
    hipGraphExec_t exec = nullptr;
    gn_tuning t{};
    gn_schedule sch{};
    const float* x = nullptr;
    const uint8_t* sel = nullptr;
    const float* gamma = nullptr;
};

struct gn_batch {
    int32_t count = 0;
    int64_t total_n = 0, total_nnz = 0;
    int32_t max_n = 0;
    int device = 0;
    int32_t cus = 0;
    BatchDesc* desc = nullptr;
    int32_t* order = nullptr;      // graphs that fit the LDS state size, then the others (for split_lds)
    std::vector<int32_t> h_order;  // all graphs, most entries first
    int32_t split_lds = -1;        // lds_vertices the device order was split for
    int32_t n_fit = 0;             // graphs whose LDS state fits 12 * split_lds bytes
    std::vector<int64_t> h_state;  // per graph: state_lds_bytes, or INT64_MAX without a sliced layout
    std::vector<int32_t> h_slices, h_lines;  // per graph: slices and lines of the sliced layout (-1 without)
    // unrolled (differentiable) calls: graph order, queue counter, gamma table,
    // sqrt of caller weights; allocated on first use
    int32_t* u_order = nullptr;
    int32_t* u_queue = nullptr;
    float* u_gamma = nullptr;
    int32_t u_gamma_cap = 0;
    std::vector<float> u_gamma_host;  // the table's current contents
    float* u_v = nullptr;
    int32_t* vgraph = nullptr;
    int32_t* row_ptr = nullptr;
    int32_t* col = nullptr;
    uint16_t* lines = nullptr;  // sliced layouts
    int32_t* slices = nullptr;  // slice tables
    float* v = nullptr;
    float* w = nullptr;
    int32_t* perm = nullptr;
    float* yg0 = nullptr;
    float* yg1 = nullptr;
    int32_t* queue = nullptr;
    float* gamma = nullptr;
    int32_t gamma_cap = 0;
    BatchRes* res = nullptr;
    BatchRes* res_host = nullptr;  // pinned
    bool tuned = false;
    gn_tuning tuning{};
    BatchLaunch launch;
    // host copies of the caller's CSR for the block-diagonal union graph
    std::vector<int32_t> h_n;
    std::vector<int64_t> h_nnz;
    std::vector<int32_t> h_rp, h_ci;
    std::vector<float> h_w;
    gn_graph* uni = nullptr;
};

static void batch_free(gn_batch* b) {
    auto f = [](void* p) { if (p) (void)hipFree(p); };
    f(b->desc); f(b->order); f(b->vgraph); f(b->row_ptr); f(b->col); f(b->lines); f(b->slices); f(b->v); f(b->w); f(b->perm);
    f(b->yg0); f(b->yg1); f(b->queue); f(b->gamma); f(b->res);
    f(b->u_order); f(b->u_queue); f(b->u_gamma); f(b->u_v);
    if (b->res_host) (void)hipHostFree(b->res_host);
    if (b->launch.exec) (void)hipGraphExecDestroy(b->launch.exec);
    if (b->uni) gn_graph_destroy(b->uni);
}

extern "C" void gn_batch_destroy(gn_batch* b) {
    if (!b) return;
    (void)hipDeviceSynchronize();
    batch_free(b);
    delete b;
}

template <typename T>
static bool dalloc(T** p, size_t count) {
    if (count == 0) count = 1;
    if (hipMalloc((void**)p, count * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return false;
    }
    return true;
}

// Appends the sliced layout of one graph (see the head of this file) to
// `lines` and its slice table to `slices`: light rows [lb, le) in slices of 64,
// mid rows [mb, me) in slices of 8, heavy rows [hb, he) one per slice, in this
// order; row r holds entries col[rp[r] .. rp[r+1]) of a graph of n vertices
// (n <= kMaxSlicedN).  Widths are rounded up to even; padding holds n.
// Returns the graph's line count.
static int64_t build_slices(int32_t n, const int32_t* rp, const int32_t* col, int32_t lb, int32_t le, int32_t mb,
                            int32_t me, int32_t hb, int32_t he, std::vector<uint16_t>& lines,
                            std::vector<int32_t>& slices) {
    const int32_t nL = (le - lb + 63) / 64, nM = (me - mb + 7) / 8, nH = he - hb;
    auto deg = [&](int32_t r) { return rp[r + 1] - rp[r]; };
    const size_t ln0 = lines.size() / 64, so0 = slices.size();
    int64_t acc = 0;
    slices.push_back(0);
    for (int32_t sl = 0; sl < nL; ++sl) {
        int32_t wdt = 0;
        for (int32_t r = lb + 64 * sl; r < std::min(lb + 64 * sl + 64, le); ++r) wdt = std::max(wdt, deg(r));
        acc += (wdt + 1) & ~1;
        slices.push_back((int32_t)acc);
    }
    for (int32_t sl = 0; sl < nM; ++sl) {
        int32_t wdt = 0;
        for (int32_t r = mb + 8 * sl; r < std::min(mb + 8 * sl + 8, me); ++r) wdt = std::max(wdt, (deg(r) + 7) / 8);
        acc += (wdt + 1) & ~1;
        slices.push_back((int32_t)acc);
    }
    for (int32_t sl = 0; sl < nH; ++sl) {
        acc += (((deg(hb + sl) + 63) / 64) + 1) & ~1;
        slices.push_back((int32_t)acc);
    }
    lines.resize(lines.size() + (size_t)acc * 64, (uint16_t)n);
    uint16_t* lg = lines.data() + ln0 * 64;
    const int32_t* so = slices.data() + so0;
    auto cid = [&](int32_t r, int32_t e) { return (uint16_t)col[rp[r] + e]; };
    for (int32_t sl = 0; sl < nL; ++sl)
        for (int32_t l = 0; l < 64 && lb + 64 * sl + l < le; ++l) {
            const int32_t r = lb + 64 * sl + l;
            for (int32_t e = 0; e < deg(r); ++e) lg[(size_t)(so[sl] + e) * 64 + l] = cid(r, e);
        }
    for (int32_t sl = 0; sl < nM; ++sl)
        for (int32_t l = 0; l < 64 && mb + 8 * sl + l / 8 < me; ++l) {
            const int32_t r = mb + 8 * sl + l / 8, t = l % 8;
            for (int32_t e = t; e < deg(r); e += 8) lg[(size_t)(so[nL + sl] + e / 8) * 64 + l] = cid(r, e);
        }
    for (int32_t sl = 0; sl < nH; ++sl) {
        const int32_t r = hb + sl;
        for (int32_t e = 0; e < deg(r); ++e) lg[(size_t)(so[nL + nM + sl] + e / 64) * 64 + e % 64] = cid(r, e);
    }
    return acc;
}

extern "C" gn_status gn_batch_create(int32_t count, const int32_t* n, const int64_t* nnz, const int32_t* row_ptr_cat,
                                     const int32_t* col_idx_cat, const float* w_cat, uint32_t flags, hipStream_t stream,
                                     gn_batch** out) {
    if (!out) return GN_E_ARG;
    *out = nullptr;
    if (count < 1 || !n || !nnz || !row_ptr_cat || (flags & ~3u)) return GN_E_ARG;
    int64_t tn = 0, tnnz = 0, trp = 0;
    int32_t maxn = 0;
    for (int32_t g = 0; g < count; ++g) {
        if (n[g] < 0 || nnz[g] < 0 || nnz[g] > INT32_MAX) return GN_E_ARG;
        tn += n[g];
        tnnz += nnz[g];
        trp += (int64_t)n[g] + 1;
        maxn = std::max(maxn, n[g]);
    }
    if (tn > INT32_MAX || (tn > 0 && !w_cat) || (tnnz > 0 && !col_idx_cat)) return GN_E_ARG;

    gn_batch* b = new (std::nothrow) gn_batch();
    if (!b) return GN_E_NOMEM;
    b->h_n.assign(n, n + count);
    b->h_nnz.assign(nnz, nnz + count);
    b->h_rp.resize((size_t)trp);
    b->h_ci.resize((size_t)std::max<int64_t>(tnnz, 1));
    b->h_w.resize((size_t)std::max<int64_t>(tn, 1));
    if (flags & GN_INPUT_DEVICE) {
        bool ok = hipMemcpyAsync(b->h_rp.data(), row_ptr_cat, sizeof(int32_t) * trp, hipMemcpyDeviceToHost, stream) ==
                  hipSuccess;
        if (ok && tnnz)
            ok = hipMemcpyAsync(b->h_ci.data(), col_idx_cat, sizeof(int32_t) * tnnz, hipMemcpyDeviceToHost, stream) ==
                 hipSuccess;
        if (ok && tn)
            ok = hipMemcpyAsync(b->h_w.data(), w_cat, sizeof(float) * tn, hipMemcpyDeviceToHost, stream) == hipSuccess;
        if (ok) ok = hipStreamSynchronize(stream) == hipSuccess;
        if (!ok) {
            delete b;
            return GN_E_HIP;
        }
    } else {
        std::memcpy(b->h_rp.data(), row_ptr_cat, sizeof(int32_t) * trp);
        if (tnnz) std::memcpy(b->h_ci.data(), col_idx_cat, sizeof(int32_t) * tnnz);
        if (tn) std::memcpy(b->h_w.data(), w_cat, sizeof(float) * tn);
    }

    // validate each graph (same conditions as gn_graph_create) and relabel it:
    // rows of degree <= kLightMaxDeg first, then those of degree <= kMidMaxDeg,
    // then the rest, each class by decreasing degree (ties in the original
    // order); each row keeps its entries in the caller's order
    std::vector<BatchDesc> desc((size_t)count);
    std::vector<int32_t> rp_int((size_t)trp), col_int((size_t)std::max<int64_t>(tnnz, 1)), perm((size_t)std::max<int64_t>(tn, 1));
    std::vector<int32_t> vgraph((size_t)std::max<int64_t>(tn, 1));
    std::vector<float> v_int((size_t)std::max<int64_t>(tn, 1)), w_int((size_t)std::max<int64_t>(tn, 1));
    std::vector<uint16_t> lines;
    std::vector<int32_t> slices;
    std::vector<int64_t> state_bytes((size_t)count, INT64_MAX);
    std::vector<int32_t> h_slices((size_t)count, -1), h_lines((size_t)count, -1);
    int64_t vo = 0, ro = 0, eo = 0;
    for (int32_t g = 0; g < count; ++g) {
        const int32_t ng = n[g];
        const int32_t* rp = b->h_rp.data() + ro;
        const int32_t* ci = b->h_ci.data() + eo;
        const float* wg = b->h_w.data() + vo;
        if (rp[0] != 0 || (int64_t)rp[ng] != nnz[g]) { delete b; return GN_E_CSR; }
        for (int32_t i = 0; i < ng; ++i)
            if (rp[i + 1] < rp[i]) { delete b; return GN_E_CSR; }
        for (int64_t e = 0; e < nnz[g]; ++e)
            if (ci[e] < 0 || ci[e] >= ng) { delete b; return GN_E_CSR; }
        if (!(flags & GN_NO_VALIDATE)) {
            for (int32_t i = 0; i < ng; ++i)
                for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
                    if (ci[e] == i) { delete b; return GN_E_SELF_LOOP; }
                    if (e > rp[i] && ci[e] <= ci[e - 1]) { delete b; return GN_E_CSR; }
                }
            // symmetry via a counting transpose, as in gn_graph_create
            std::vector<int32_t> tptr((size_t)ng + 1, 0);
            for (int64_t e = 0; e < nnz[g]; ++e) tptr[(size_t)ci[e] + 1]++;
            for (int32_t i = 0; i < ng; ++i) tptr[(size_t)i + 1] += tptr[i];
            for (int32_t i = 0; i <= ng; ++i)
                if (tptr[i] != rp[i]) { delete b; return GN_E_ASYMMETRIC; }
            std::vector<int32_t> fill(tptr.begin(), tptr.end() - 1), tcol((size_t)std::max<int64_t>(nnz[g], 1));
            for (int32_t i = 0; i < ng; ++i)
                for (int32_t e = rp[i]; e < rp[i + 1]; ++e) tcol[(size_t)fill[ci[e]]++] = i;
            for (int64_t e = 0; e < nnz[g]; ++e)
                if (tcol[(size_t)e] != ci[e]) { delete b; return GN_E_ASYMMETRIC; }
        }
        for (int32_t i = 0; i < ng; ++i)
            if (!(wg[i] > 0.0f) || !std::isfinite(wg[i])) { delete b; return GN_E_WEIGHT; }
        std::vector<int32_t> p((size_t)ng), q((size_t)ng);
        std::iota(p.begin(), p.end(), 0);
        auto cls = [&](int32_t i) {
            const int32_t dg = rp[i + 1] - rp[i];
            return dg <= kLightMaxDeg ? 0 : dg <= kMidMaxDeg ? 1 : 2;
        };
        std::stable_sort(p.begin(), p.end(), [&](int32_t i, int32_t j) {
            const int ci_ = cls(i), cj_ = cls(j);
            return ci_ != cj_ ? ci_ < cj_ : rp[i + 1] - rp[i] > rp[j + 1] - rp[j];
        });
        int32_t nl = 0, nm = 0;
        for (int32_t i = 0; i < ng; ++i) {
            nl += cls(i) == 0 ? 1 : 0;
            nm += cls(i) <= 1 ? 1 : 0;
        }
        for (int32_t r = 0; r < ng; ++r) q[p[r]] = r;
        int32_t* rpi = rp_int.data() + ro;
        rpi[0] = 0;
        for (int32_t r = 0; r < ng; ++r) {
            const int32_t i = p[r];
            const int32_t dg = rp[i + 1] - rp[i];
            for (int32_t e = 0; e < dg; ++e) col_int[(size_t)(eo + rpi[r] + e)] = q[ci[rp[i] + e]];
            rpi[r + 1] = rpi[r] + dg;
            perm[(size_t)(vo + r)] = i;
            v_int[(size_t)(vo + r)] = (float)std::sqrt((double)wg[i]);
            w_int[(size_t)(vo + r)] = wg[i];
            vgraph[(size_t)(vo + r)] = g;
        }
        // sliced layout (see the head of this file)
        const int64_t ln0 = (int64_t)(lines.size() / 64), so0 = (int64_t)slices.size();
        int32_t nlines = 0;
        if (ng <= kMaxSlicedN) {
            const int64_t acc = build_slices(ng, rpi, col_int.data() + eo, 0, nl, nl, nm, nm, ng, lines, slices);
            if (acc > INT32_MAX / 64) { delete b; return GN_E_ARG; }
            nlines = (int32_t)acc;
            state_bytes[g] = state_lds_bytes(ng, slice_count(ng, nl, nm));
            h_slices[g] = slice_count(ng, nl, nm);
            h_lines[g] = nlines;
        }
        desc[g] = BatchDesc{ng, nl, nm, nlines, vo, ro, eo, ln0, so0, (int32_t)nnz[g], 0};
        vo += ng;
        ro += (int64_t)ng + 1;
        eo += nnz[g];
    }
    std::vector<int32_t> order((size_t)count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) {
        return (int64_t)nnz[a] + n[a] > (int64_t)nnz[c] + n[c];
    });

    b->count = count;
    b->total_n = tn;
    b->total_nnz = tnnz;
    b->max_n = maxn;
    (void)hipGetDevice(&b->device);
    int cus = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device);
    b->cus = cus > 0 ? cus : 256;
    bool ok = dalloc(&b->desc, count) && dalloc(&b->order, count) && dalloc(&b->vgraph, tn) &&
              dalloc(&b->row_ptr, trp) && dalloc(&b->col, tnnz) && dalloc(&b->lines, std::max<size_t>(lines.size(), 64)) &&
              dalloc(&b->slices, slices.size()) && dalloc(&b->v, tn) && dalloc(&b->w, tn) &&
              dalloc(&b->perm, tn) && dalloc(&b->yg0, tn) && dalloc(&b->yg1, tn) && dalloc(&b->queue, 3) &&
              dalloc(&b->res, count);
    if (ok && hipHostMalloc((void**)&b->res_host, sizeof(BatchRes) * count, hipHostMallocDefault) != hipSuccess) {
        b->res_host = nullptr;
        ok = false;
    }
    if (!ok) {
        batch_free(b);
        delete b;
        return GN_E_NOMEM;
    }
    hipError_t e = hipSuccess;
    auto up = [&](void* dst, const void* src, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream);
    };
    up(b->desc, desc.data(), sizeof(BatchDesc) * count);
    b->h_order = order;
    up(b->vgraph, vgraph.data(), sizeof(int32_t) * tn);
    up(b->row_ptr, rp_int.data(), sizeof(int32_t) * trp);
    up(b->col, col_int.data(), sizeof(int32_t) * tnnz);
    up(b->lines, lines.data(), sizeof(uint16_t) * lines.size());
    up(b->slices, slices.data(), sizeof(int32_t) * slices.size());
    b->h_state = std::move(state_bytes);
    b->h_slices = std::move(h_slices);
    b->h_lines = std::move(h_lines);
    up(b->v, v_int.data(), sizeof(float) * tn);
    up(b->w, w_int.data(), sizeof(float) * tn);
    up(b->perm, perm.data(), sizeof(int32_t) * tn);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        batch_free(b);
        delete b;
        return GN_E_HIP;
    }
    *out = b;
    return GN_OK;
}

static bool tuning_valid(const gn_tuning& t) {
    const bool bt_ok = t.block_threads == 128 || t.block_threads == 256 || t.block_threads == 512 ||
                       (t.block_threads == 1024 && t.blocks_per_cu <= 2);
    return bt_ok && t.blocks_per_cu >= 1 && t.blocks_per_cu <= 4 && t.lds_vertices >= 0 &&
           (size_t)t.lds_vertices * 12 * t.blocks_per_cu <= kLdsBudget;
}

static gn_tuning default_tuning(const gn_batch* b) {
    gn_tuning t{};
    t.block_threads = 256;
    t.blocks_per_cu = 2;
    t.lds_vertices = kLdsBudget / (12 * 2);
    t.reserved = 0;
    return t;
}

static gn_status ensure_gamma(gn_batch* b, int32_t entries) {
    if (entries <= b->gamma_cap) return GN_OK;
    if (b->gamma) (void)hipFree(b->gamma);
    b->gamma = nullptr;
    b->gamma_cap = 0;
    if (!dalloc(&b->gamma, (size_t)entries)) return GN_E_NOMEM;
    b->gamma_cap = entries;
    return GN_OK;
}

static const void* batch_kernel(int bt, bool big = false) {
    if (big)
        return bt == 128 ? batch_kernel_ptr<128, true>() : bt == 512 ? batch_kernel_ptr<512, true>()
             : bt == 1024 ? batch_kernel_ptr<1024, true>() : batch_kernel_ptr<256, true>();
    return bt == 128 ? batch_kernel_ptr<128, false>() : bt == 512 ? batch_kernel_ptr<512, false>()
         : bt == 1024 ? batch_kernel_ptr<1024, false>() : batch_kernel_ptr<256, false>();
}

// Workgroups of the batched kernel that fit on one compute unit at this shape
// (registers and LDS).  The persistent grid never asks for more: a workgroup
// beyond it would only start once the queue is empty.
static int resident_blocks(int bt, size_t lds_bytes, bool big = false) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_kernel(bt, big), bt, lds_bytes) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return std::max(nb, 1);
}

// Host-side preparation of a solve: the gamma table's size and the device
// processing order for this LDS size (graphs whose state fits first, then the
// others, each part most entries first).  May synchronise `s`.
static gn_status prepare_batch(gn_batch* b, const gn_schedule* sch, const gn_tuning& t, hipStream_t s) {
    gn_status st = ensure_gamma(b, sch->max_steps + 1);
    if (st != GN_OK) return st;
    if (t.lds_vertices != b->split_lds) {
        std::vector<int32_t> split;
        split.reserve(b->h_order.size());
        for (int32_t g : b->h_order)
            if (b->h_state[g] <= 12 * (int64_t)t.lds_vertices) split.push_back(g);
        const int32_t nf = (int32_t)split.size();
        for (int32_t g : b->h_order)
            if (b->h_state[g] > 12 * (int64_t)t.lds_vertices) split.push_back(g);
        GN_HIP_TRY(hipMemcpyAsync(b->order, split.data(), sizeof(int32_t) * split.size(), hipMemcpyHostToDevice, s));
        GN_HIP_TRY(hipStreamSynchronize(s));  // the host vector goes out of scope
        b->split_lds = t.lds_vertices;
        b->n_fit = nf;
    }
    return GN_OK;
}

// The kernels of one solve in order (init, x0 checks, the persistent launch of
// the graphs whose state fits in LDS, then the one of the others), handed to
// `emit(func, grid, block, lds_bytes, args)`: launched directly or added to a HIP
// graph.  The argument storage lives until the function returns.
template <typename Emit>
static gn_status batch_kernels(gn_batch* b, const gn_schedule* sch, const gn_tuning& t, float* x_cat,
                               uint8_t* sel_cat, Emit&& emit) {
    {
        int32_t* queue = b->queue;
        float* gamma = b->gamma;
        int32_t ms = sch->max_steps, ramp = sch->ramp_steps;
        float g0 = sch->gamma0, g1 = sch->gamma1;
        void* args[] = {&queue, &gamma, &ms, &g0, &g1, &ramp};
        GN_HIP_TRY(emit((const void*)batch_init_kernel, dim3(std::min((sch->max_steps + 1 + 255) / 256, 1024)),
                        dim3(256), 0, args));
    }
    if (b->total_n > 0) {
        int64_t total = b->total_n;
        const int32_t* vgraph = b->vgraph;
        const BatchDesc* desc = b->desc;
        const int32_t* rp = b->row_ptr;
        const int32_t* col = b->col;
        const int32_t* perm = b->perm;
        const float* xc = x_cat;
        int32_t* queue = b->queue;
        void* args[] = {&total, &vgraph, &desc, &rp, &col, &perm, &xc, &queue};
        GN_HIP_TRY(emit((const void*)batch_check_x0_kernel, dim3((unsigned)((b->total_n + 255) / 256)), dim3(256), 0,
                        args));
    }
    BatchArgs a{};
    a.desc = b->desc;
    a.order = b->order;
    a.count = b->n_fit;
    a.qslot = 0;
    a.row_ptr = b->row_ptr;
    a.col = b->col;
    a.lines = b->lines;
    a.slices = b->slices;
    a.v = b->v;
    a.w = b->w;
    a.perm = b->perm;
    a.gamma = b->gamma;
    a.max_steps = sch->max_steps;
    a.check_every = sch->check_every;
    a.tau = sch->tau;
    a.lds_vertices = t.lds_vertices;
    a.x_cat = x_cat;
    a.sel_cat = sel_cat;
    a.yg0 = b->yg0;
    a.yg1 = b->yg1;
    a.queue = b->queue;
    a.res = b->res;
    const size_t lds = (size_t)t.lds_vertices * 3 * sizeof(float);
    if (b->n_fit > 0) {
        const int bpc = std::min(t.blocks_per_cu, resident_blocks(t.block_threads, lds, false));
        void* args[] = {&a};
        GN_HIP_TRY(emit(batch_kernel(t.block_threads, false),
                        dim3((unsigned)std::min<int64_t>((int64_t)b->cus * bpc, b->n_fit)), dim3(t.block_threads),
                        lds, args));
    }
    if (b->n_fit < b->count) {
        BatchArgs big = a;
        big.order = b->order + b->n_fit;
        big.count = b->count - b->n_fit;
        big.qslot = 2;
        const int bpc = std::min(t.blocks_per_cu, resident_blocks(t.block_threads, 0, true));
        void* args[] = {&big};
        GN_HIP_TRY(emit(batch_kernel(t.block_threads, true),
                        dim3((unsigned)std::min<int64_t>((int64_t)b->cus * bpc, big.count)), dim3(t.block_threads), 0,
                        args));
    }
    return GN_OK;
}

// Enqueue the whole batched solve with direct launches (the autotuner's timing runs).
static gn_status enqueue_batch(gn_batch* b, const gn_schedule* sch, const gn_tuning& t, float* x_cat, uint8_t* sel_cat,
                               hipStream_t s) {
    gn_status st = prepare_batch(b, sch, t, s);
    if (st != GN_OK) return st;
    return batch_kernels(b, sch, t, x_cat, sel_cat,
                         [s](const void* f, dim3 grid, dim3 block, size_t lds, void** args) {
                             return hipLaunchKernel(f, grid, block, args, lds, s);
                         });
}

// The solve as one HIP graph, kept in the handle while the tuning, the
// schedule, the buffers and the gamma table stay the same; a repeated solve is
// then a single graph launch.
static bool same_launch(const BatchLaunch& k, const gn_tuning& t, const gn_schedule* sch, const float* x,
                        const uint8_t* sel, const float* gamma) {
    return k.exec && k.t.block_threads == t.block_threads && k.t.blocks_per_cu == t.blocks_per_cu &&
           k.t.lds_vertices == t.lds_vertices && k.sch.gamma0 == sch->gamma0 && k.sch.gamma1 == sch->gamma1 &&
           k.sch.ramp_steps == sch->ramp_steps && k.sch.max_steps == sch->max_steps && k.sch.tau == sch->tau &&
           k.sch.check_every == sch->check_every && k.x == x && k.sel == sel && k.gamma == gamma;
}

static gn_status launch_batch_graph(gn_batch* b, const gn_schedule* sch, const gn_tuning& t, float* x_cat,
                                    uint8_t* sel_cat, hipStream_t s) {
    gn_status st = prepare_batch(b, sch, t, s);
    if (st != GN_OK) return st;
    BatchLaunch& k = b->launch;
    if (!same_launch(k, t, sch, x_cat, sel_cat, b->gamma)) {
        if (k.exec) (void)hipGraphExecDestroy(k.exec);
        k.exec = nullptr;
        hipGraph_t graph;
        GN_HIP_TRY(hipGraphCreate(&graph, 0));
        hipGraphNode_t prev = nullptr;
        st = batch_kernels(b, sch, t, x_cat, sel_cat,
                           [&](const void* f, dim3 grid, dim3 block, size_t lds, void** args) {
                               hipKernelNodeParams p{};
                               p.func = const_cast<void*>(f);
                               p.gridDim = grid;
                               p.blockDim = block;
                               p.sharedMemBytes = (unsigned)lds;
                               p.kernelParams = args;
                               p.extra = nullptr;
                               hipGraphNode_t node;
                               hipError_t e = hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &p);
                               if (e == hipSuccess) prev = node;
                               return e;
                           });
        hipError_t e = st == GN_OK ? hipGraphInstantiate(&k.exec, graph, nullptr, nullptr, 0) : hipSuccess;
        (void)hipGraphDestroy(graph);
        if (st != GN_OK) return st;
        if (e != hipSuccess) {
            k.exec = nullptr;
            return GN_E_HIP;
        }
        k.t = t;
        k.sch = *sch;
        k.x = x_cat;
        k.sel = sel_cat;
        k.gamma = b->gamma;
    }
    GN_HIP_TRY(hipGraphLaunch(k.exec, s));
    return GN_OK;
}

static void allow_lds(int bt, size_t bytes) {
    (void)hipFuncSetAttribute(batch_kernel(bt), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

static gn_status check_schedule(const gn_schedule* sch) {
    if (!sch || sch->max_steps < 0 || sch->check_every < 1 || !(sch->tau >= 0.0f) || !std::isfinite(sch->tau) ||
        !std::isfinite(sch->gamma0) || !std::isfinite(sch->gamma1) || sch->gamma0 < 0.0f || sch->gamma1 < 0.0f ||
        sch->max_steps > (1 << 28))
        return GN_E_ARG;
    return GN_OK;
}

extern "C" gn_status gn_batch_solve(gn_batch* b, const gn_schedule* sch, const gn_tuning* tuning, float* x_cat,
                                    uint8_t* sel_cat, gn_result* res, hipStream_t stream) {
    if (!b || !res) return GN_E_ARG;
    gn_status st = check_schedule(sch);
    if (st != GN_OK) return st;
    if (b->total_n > 0 && (!x_cat || !sel_cat)) return GN_E_ARG;
    gn_tuning t = tuning ? *tuning : (b->tuned ? b->tuning : default_tuning(b));
    if (!tuning_valid(t)) return GN_E_ARG;
    allow_lds(t.block_threads, (size_t)t.lds_vertices * 12);
    st = launch_batch_graph(b, sch, t, x_cat, sel_cat, stream);
    if (st != GN_OK) return st;
    int32_t qh[2];
    GN_HIP_TRY(hipMemcpyAsync(b->res_host, b->res, sizeof(BatchRes) * b->count, hipMemcpyDeviceToHost, stream));
    GN_HIP_TRY(hipMemcpyAsync(qh, b->queue, sizeof(qh), hipMemcpyDeviceToHost, stream));
    GN_HIP_TRY(hipStreamSynchronize(stream));
    if (qh[1] & 1) return GN_E_ARG;
    if (qh[1] & 2) return GN_E_NOT_NORMALIZABLE;
    bool all = true;
    for (int32_t g = 0; g < b->count; ++g) {
        const BatchRes& r = b->res_host[g];
        gn_result& o = res[g];
        if (b->h_n[g] == 0) {
            std::memset(&o, 0, sizeof(o));
            o.binarised = 1;
            o.stab = INFINITY;
            continue;
        }
        o.steps = r.steps;
        o.binarised = r.binarised;
        o.fallback_count = r.fallback;
        o.relaxed_objective = r.relaxed;
        o.set_objective = r.set_w;
        o.set_size = r.size;
        o.conflicts = r.conflicts;
        o.uncovered = r.uncovered;
        o.stab = r.stab;
        all = all && r.binarised;
    }
    return all ? GN_OK : GN_NOT_CONVERGED;
}

extern "C" gn_status gn_batch_autotune(gn_batch* b, const gn_schedule* sch, gn_tuning* out, hipStream_t stream) {
    if (!b || !out) return GN_E_ARG;
    gn_status st = check_schedule(sch);
    if (st != GN_OK) return st;
    // per candidate: a warm-up run of at most 64 steps, then one timed full
    // solve, from x0 = 1/2 (the largest graphs set the wall time, and only a
    // full solve shows their tail)
    gn_schedule ws = *sch;
    ws.max_steps = std::min<int32_t>(sch->max_steps, 64);
    float* x = nullptr;
    uint8_t* sel = nullptr;
    if (!dalloc(&x, (size_t)b->total_n) || !dalloc(&sel, (size_t)b->total_n)) {
        if (x) (void)hipFree(x);
        return GN_E_NOMEM;
    }
    std::vector<float> half((size_t)std::max<int64_t>(b->total_n, 1), 0.5f);
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    gn_tuning best = default_tuning(b);
    float best_ms = INFINITY;
    st = GN_OK;
    for (int bt : {128, 256, 512, 1024}) {
        for (int bpc : {1, 2, 4}) {
            gn_tuning t{};
            t.block_threads = bt;
            t.blocks_per_cu = bpc;
            t.lds_vertices = kLdsBudget / (12 * bpc);
            if (!tuning_valid(t)) continue;
            allow_lds(bt, (size_t)t.lds_vertices * 12);
            if (resident_blocks(bt, (size_t)t.lds_vertices * 12) < bpc) continue;  // same launch as a smaller bpc
            float ms_sum = 0.0f;
            for (int rep = 0; rep < 2 && st == GN_OK; ++rep) {
                if (hipMemcpyAsync(x, half.data(), sizeof(float) * b->total_n, hipMemcpyHostToDevice, stream) !=
                    hipSuccess) {
                    st = GN_E_HIP;
                    break;
                }
                (void)hipEventRecord(e0, stream);
                st = enqueue_batch(b, rep == 0 ? &ws : sch, t, x, sel, stream);
                (void)hipEventRecord(e1, stream);
                if (hipEventSynchronize(e1) != hipSuccess) st = GN_E_HIP;
                float ms = 0.0f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (rep == 1) ms_sum += ms;
            }
            if (st != GN_OK) break;
            if (ms_sum < best_ms) {
                best_ms = ms_sum;
                best = t;
            }
        }
        if (st != GN_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(x);
    (void)hipFree(sel);
    if (st != GN_OK) return st;
    b->tuning = best;
    b->tuned = true;
    *out = best;
    return GN_OK;
}

extern "C" const gn_graph* gn_batch_graph(const gn_batch* bc) {
    if (!bc) return nullptr;
    gn_batch* b = const_cast<gn_batch*>(bc);
    if (b->uni) return b->uni;
    // block-diagonal union with global vertex ids
    std::vector<int32_t> rp((size_t)b->total_n + 1), ci((size_t)std::max<int64_t>(b->total_nnz, 1));
    int64_t vo = 0, ro = 0, eo = 0;
    rp[0] = 0;
    for (int32_t g = 0; g < b->count; ++g) {
        const int32_t ng = b->h_n[g];
        for (int32_t i = 0; i < ng; ++i) rp[(size_t)(vo + i + 1)] = (int32_t)(eo + b->h_rp[(size_t)(ro + i + 1)]);
        for (int64_t e = 0; e < b->h_nnz[g]; ++e) ci[(size_t)(eo + e)] = (int32_t)(vo + b->h_ci[(size_t)(eo + e)]);
        vo += ng;
        ro += (int64_t)ng + 1;
        eo += b->h_nnz[g];
    }
    gn_graph* u = nullptr;
    if (gn_graph_create((int32_t)b->total_n, b->total_nnz, rp.data(), ci.data(), b->h_w.data(),
                        GN_INPUT_HOST | GN_NO_VALIDATE, nullptr, &u) != GN_OK)
        return nullptr;
    b->uni = u;
    return u;
}

// ---------------------------------------------------------------------------
// Unrolled (differentiable) calls on a batch.
// ---------------------------------------------------------------------------
template <int BT, bool BWD>
const void* unrolled_kernel_ptr() {
    return (const void*)batch_unrolled_kernel<BT, BWD>;
}

// Workgroup size of the unrolled kernels: 1024 threads when every graph has a
// compute unit to itself (more wavefronts share a graph's slices), else 512 so
// that two graphs share one.  Results do not depend on it.
static int unrolled_block(const gn_batch* b) { return b->count <= b->cus ? 1024 : 512; }

static const void* unrolled_kernel(int bt, bool bwd) {
    if (bt == 1024) return bwd ? unrolled_kernel_ptr<1024, true>() : unrolled_kernel_ptr<1024, false>();
    return bwd ? unrolled_kernel_ptr<512, true>() : unrolled_kernel_ptr<512, false>();
}

static gn_status unrolled_prepare(gn_batch* b, const float* w_cat, const float* gammas, int32_t T, bool bwd,
                                  hipStream_t s, UnrolledArgs& a, dim3& grid, size_t& lds) {
    // every graph needs a sliced layout whose state fits one workgroup's LDS
    int64_t maxstate = 0, maxall = 0;
    for (int32_t g = 0; g < b->count; ++g) {
        if (b->h_n[g] == 0) continue;
        if (b->h_slices[g] < 0) return GN_E_ARG;
        const int64_t st = unrolled_state_bytes(bwd, b->h_n[g], b->h_slices[g]);
        maxstate = std::max(maxstate, st);
        maxall = std::max(maxall, st + 128 * (int64_t)b->h_lines[g]);
    }
    if (maxstate > kLdsBudget) return GN_E_ARG;
    const int bt = unrolled_block(b);
    const int bpc_want = bt == 512 && maxstate <= kLdsBudget / 2 ? 2 : 1;
    lds = (size_t)((std::min<int64_t>(std::max(maxall, maxstate), kLdsBudget / bpc_want) + 15) / 16 * 16);
    if (!b->u_order) {
        if (!dalloc(&b->u_order, (size_t)b->count) || !dalloc(&b->u_queue, 1)) return GN_E_NOMEM;
        GN_HIP_TRY(hipMemcpy(b->u_order, b->h_order.data(), sizeof(int32_t) * b->count, hipMemcpyHostToDevice));
    }
    if (T > b->u_gamma_cap) {
        if (b->u_gamma) (void)hipFree(b->u_gamma);
        b->u_gamma = nullptr;
        b->u_gamma_cap = 0;
        b->u_gamma_host.clear();
        if (!dalloc(&b->u_gamma, (size_t)T)) return GN_E_NOMEM;
        b->u_gamma_cap = T;
    }
    // the table is uploaded (blocking) only when the gammas change
    if (b->u_gamma_host.size() != (size_t)T || !std::equal(gammas, gammas + T, b->u_gamma_host.begin())) {
        GN_HIP_TRY(hipStreamSynchronize(s));
        GN_HIP_TRY(hipMemcpy(b->u_gamma, gammas, sizeof(float) * T, hipMemcpyHostToDevice));
        b->u_gamma_host.assign(gammas, gammas + T);
    }
    const float* v = b->v;
    if (w_cat) {
        if (!b->u_v && !dalloc(&b->u_v, (size_t)b->total_n)) return GN_E_NOMEM;
        hipLaunchKernelGGL(batch_sqrt_weights_kernel, dim3((unsigned)((b->total_n + 255) / 256)), dim3(256), 0, s,
                           (int64_t)b->total_n, (const int32_t*)b->vgraph, (const BatchDesc*)b->desc,
                           (const int32_t*)b->perm, w_cat, b->u_v);
        GN_HIP_TRY(hipGetLastError());
        v = b->u_v;
    }
    GN_HIP_TRY(hipMemsetAsync(b->u_queue, 0, sizeof(int32_t), s));
    const void* k = unrolled_kernel(bt, bwd);
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, bt, lds) != hipSuccess) {
        (void)hipGetLastError();
        nb = 1;
    }
    const int bpc = std::max(1, std::min(bpc_want, nb));
    grid = dim3((unsigned)std::min<int64_t>((int64_t)b->cus * bpc, b->count));
    a = UnrolledArgs{};
    a.desc = b->desc;
    a.order = b->u_order;
    a.count = b->count;
    a.queue = b->u_queue;
    a.perm = b->perm;
    a.lines = b->lines;
    a.slices = b->slices;
    a.v = v;
    a.gamma = b->u_gamma;
    a.T = T;
    a.lds_bytes = (int32_t)lds;
    a.total_n = b->total_n;
    return GN_OK;
}

static gn_status check_gammas(const float* gammas, int32_t T) {
    if (T < 0 || (T > 0 && !gammas)) return GN_E_ARG;
    for (int32_t t = 0; t < T; ++t)
        if (!std::isfinite(gammas[t]) || gammas[t] < 0.0f) return GN_E_ARG;
    return GN_OK;
}

extern "C" int64_t gn_batch_unrolled_store_floats(const gn_batch* b, int32_t T) {
    if (!b || T < 0) return -1;
    return 2 * (int64_t)T * b->total_n;
}

extern "C" gn_status gn_batch_unrolled_forward(gn_batch* b, const float* w_cat, const float* gammas, int32_t T,
                                               const float* x0_cat, float* xT_cat, float* store, hipStream_t stream) {
    if (!b) return GN_E_ARG;
    gn_status st = check_gammas(gammas, T);
    if (st != GN_OK) return st;
    if (b->total_n == 0) return GN_OK;
    if (!x0_cat || !xT_cat || x0_cat == xT_cat || (T > 0 && !store)) return GN_E_ARG;
    if (T == 0) {
        GN_HIP_TRY(hipMemcpyAsync(xT_cat, x0_cat, sizeof(float) * b->total_n, hipMemcpyDeviceToDevice, stream));
        return GN_OK;
    }
    UnrolledArgs a;
    dim3 grid;
    size_t lds = 0;
    if ((st = unrolled_prepare(b, w_cat, gammas, T, false, stream, a, grid, lds)) != GN_OK) return st;
    a.x0 = x0_cat;
    a.xT = xT_cat;
    a.store = store;
    const int bt = unrolled_block(b);
    void* args[] = {&a};
    GN_HIP_TRY(hipLaunchKernel(unrolled_kernel(bt, false), grid, dim3(bt), args, lds, stream));
    GN_HIP_TRY(hipGetLastError());
    return GN_OK;
}

extern "C" gn_status gn_batch_unrolled_backward(gn_batch* b, const float* w_cat, const float* gammas, int32_t T,
                                                const float* store, const float* gxT_cat, float* gw_cat,
                                                float* gx0_cat, hipStream_t stream) {
    if (!b) return GN_E_ARG;
    gn_status st = check_gammas(gammas, T);
    if (st != GN_OK) return st;
    if (b->total_n == 0) return GN_OK;
    if (!gxT_cat || !gw_cat || !gx0_cat || (T > 0 && !store)) return GN_E_ARG;
    if (T == 0) {
        GN_HIP_TRY(hipMemcpyAsync(gx0_cat, gxT_cat, sizeof(float) * b->total_n, hipMemcpyDeviceToDevice, stream));
        GN_HIP_TRY(hipMemsetAsync(gw_cat, 0, sizeof(float) * b->total_n, stream));
        return GN_OK;
    }
    UnrolledArgs a;
    dim3 grid;
    size_t lds = 0;
    if ((st = unrolled_prepare(b, w_cat, gammas, T, true, stream, a, grid, lds)) != GN_OK) return st;
    a.store = const_cast<float*>(store);  // read only by the adjoint pass
    a.gxT = gxT_cat;
    a.gx0 = gx0_cat;
    a.gw = gw_cat;
    const int bt = unrolled_block(b);
    void* args[] = {&a};
    GN_HIP_TRY(hipLaunchKernel(unrolled_kernel(bt, true), grid, dim3(bt), args, lds, stream));
    GN_HIP_TRY(hipGetLastError());
    return GN_OK;
}

// Small-graph path of gn_solve (declared in gn_internal.h).  The graph's LDS
// image (slice table and lines over its internal order) is built at graph
// creation from the host copies of the internal CSR, and kept in the handle.
struct SmallImage {
    int32_t slices = 0, lines = 0;
    int64_t lds = INT64_MAX;  // LDS bytes of the solve; INT64_MAX: no image
    int32_t* so = nullptr;
    uint16_t* ln = nullptr;
};

void gn_internal_build_small(gn_graph* g, const int32_t* rp, const int32_t* col, hipStream_t s) {
    SmallImage* im = new (std::nothrow) SmallImage();
    if (!im) return;
    g->small = im;
    const int32_t n = g->n;
    // a cheap bound first: the lines hold at least the nnz ids
    if (n == 0 || n > kMaxSlicedN || 8 * (int64_t)n + 12 + 2 * g->nnz > kLdsBudget) return;
    const int32_t mb = g->bins.row_begin[BIN_G8], lb = g->bins.row_begin[BIN_LANE16];
    std::vector<uint16_t> lines;
    std::vector<int32_t> slices;
    const int64_t nl = build_slices(n, rp, col, lb, n, mb, lb, 0, mb, lines, slices);
    const int64_t bytes = 8 * (int64_t)n + 8 + 4 * (int64_t)slices.size() + 128 * nl;
    if (bytes > kLdsBudget) return;
    bool ok = dalloc(&im->so, slices.size()) && dalloc(&im->ln, std::max<size_t>(lines.size(), 64)) &&
              hipMemcpyAsync(im->so, slices.data(), sizeof(int32_t) * slices.size(), hipMemcpyHostToDevice, s) ==
                  hipSuccess &&
              (lines.empty() || hipMemcpyAsync(im->ln, lines.data(), sizeof(uint16_t) * lines.size(),
                                               hipMemcpyHostToDevice, s) == hipSuccess) &&
              hipStreamSynchronize(s) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        return;  // no image: the graph takes the chained path
    }
    im->slices = (int32_t)slices.size() - 1;
    im->lines = (int32_t)nl;
    im->lds = bytes;
}

void gn_internal_free_small(gn_graph* g) {
    SmallImage* im = static_cast<SmallImage*>(g->small);
    if (!im) return;
    if (im->so) (void)hipFree(im->so);
    if (im->ln) (void)hipFree(im->ln);
    delete im;
    g->small = nullptr;
}

bool gn_internal_small_fits(const gn_graph* g) {
    const SmallImage* im = static_cast<const SmallImage*>(g->small);
    return im && im->lds <= kLdsBudget;
}

gn_status gn_internal_small_solve(const gn_graph* g, hipStream_t s) {
    constexpr int BT = 1024;
    if (!gn_internal_small_fits(g)) return GN_E_ARG;
    const SmallImage* im = static_cast<const SmallImage*>(g->small);
    const size_t lds = (size_t)im->lds;
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute((const void*)small_solve_kernel<BT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
    SmallArgs a{};
    a.n = g->n;
    a.mid_begin = g->bins.row_begin[BIN_G8];
    a.light_begin = g->bins.row_begin[BIN_LANE16];
    a.n_lines = im->lines;
    a.slices = im->so;
    a.lines = im->ln;
    a.v = g->v;
    a.gamma = g->ws.gamma;
    a.st = g->ws.state;
    a.notconv = g->ws.notconv;
    a.y0 = g->ws.y[0];
    a.y1 = g->ws.y[1];
    hipLaunchKernelGGL(small_solve_kernel<BT>, dim3(1), dim3(BT), lds, s, a);
    GN_HIP_TRY(hipGetLastError());
    return GN_OK;
}
