// Sliced column layout of small graphs and the straight-line row sums over it,
// shared by the batched solve, the batched unrolled calls and the
// single-workgroup solve of gn_solve (host and device parts).
//
// The layout (graphs of at most 65535 vertices).  Each degree class
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
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "gn_rowsum.h"

namespace gnsl {

using gnk::sign_of;

// Degree classes of the sliced layout (the bin schedule): rows up to the light
// bound run one per thread (64 rows per slice), rows up to the mid bound 8
// threads per row (8 rows per slice), heavier rows a wavefront each.  The
// batched solve takes its bounds from its tuning; these are the defaults and
// the largest bounds the kernels are built for.
constexpr int kLightMaxDeg = 16;     // default light bound, and its cap (16 lines per slice)
constexpr int kMidMaxDeg = 64;       // default mid bound
constexpr int kMidMaxDegCap = 128;   // largest mid bound (16 lines per slice, two per chain)
constexpr int kLdsBudget = 160 * 1024 - 2048;  // dynamic LDS per CU (static LDS of the kernel set aside)
constexpr int32_t kMaxSlicedN = 65535;          // largest graph with a sliced layout (ids and the zero slot fit 16 bits)

// Slices of a graph: light slices, then mid slices, then one per heavy row.
__host__ __device__ inline int32_t slice_count(int32_t n, int32_t nl, int32_t nm) {
    return (nl + 63) / 64 + (nm - nl + 7) / 8 + (n - nm);
}

// LDS bytes of a graph in the LDS launch: y and y' (n + 1 words each, the last
// one the zero slot) and the slice table; with its lines in LDS too, 128 bytes
// per line more.  v is read
// from global memory: only its own row reads it, once per step, with a load
// that does not wait on anything else.
__host__ __device__ inline int64_t state_lds_bytes(int64_t n, int64_t slices) { return 8 * n + 8 + 4 * (slices + 1); }
__host__ __device__ inline int64_t all_lds_bytes(int64_t n, int64_t slices, int64_t lines) {
    return state_lds_bytes(n, slices) + 128 * lines;
}

// The WRGN update of one row (the step kernel's arithmetic) and its part of the
// stopping test: returns whether the input state fails the test at this row.
__device__ __forceinline__ bool step_row(float yraw, float vi, float sigma, bool nbr_sel, float g, bool do_test,
                                         bool do_write, float tau, float* y_out, int i, int& fb) {
    const float yi = fabsf(yraw);
    const float s = __fmaf_rn(g, sigma, yi);
    const bool fallback = !(s > 1e-9f);
    if (do_write) {
        y_out[i] = gnk::step_word(yraw, vi, s);
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
        if (q < NQ) c[q] = ABS ? gnk::nbr_term(yv) : 0.0f + yv;
        else c[q % NQ] += ABS ? gnk::nbr_term(yv) : yv;
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
        acc += ABS ? gnk::nbr_term(yv[q]) : yv[q];
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

// Appends the sliced layout of one graph (above) to
// `lines` and its slice table to `slices`: light rows [lb, le) in slices of 64,
// mid rows [mb, me) in slices of 8, heavy rows [hb, he) one per slice, in this
// order; row r holds entries col[rp[r] .. rp[r+1]) of a graph of n vertices
// (n <= kMaxSlicedN).  Widths are rounded up to even; padding holds n.
// Returns the graph's line count.
inline int64_t build_slices(int32_t n, const int32_t* rp, const int32_t* col, int32_t lb, int32_t le, int32_t mb,
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

}  // namespace gnsl
