// The fused WRGN step kernel.
//
// One step (WRGN definition; y-space form of the energy-descent appendix; safe
// division of the code appendix), for every row i:
//     s_i  = |y_i| + gamma * sum_{j in N(i)} |y_j|
//     x'_i = |y_i| / s_i  if s_i > 1e-9,  else 1/2
//     y'_i = v_i x'_i, stored with its sign bit set when x'_i > 1/2
// The sign bit carries the rounded set S to the next step, so the stopping test
// on the input state (cover of S, decay of the non-selected rows, distance to
// binary) is computed inside the same pass at no extra memory traffic.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "gn_internal.h"
#include "gn_ctl.h"
#include "gn_rowsum.h"

using gnk::sign_of;

namespace {

// Pruned lists (solve mode).  A neighbour sum adds only ordinary words, so the
// entry of a vertex that is not ordinary adds nothing whether it is read or
// not: the lists may drop it.  Invariant: every vertex whose word is ordinary
// in a step's input is listed (its entries hold its id) when the step reads
// the lists.  A row whose word becomes ordinary again in this step (input not
// ordinary, output ordinary) lists itself now if it is not listed: during
// this step its entries add nothing either way, and the next step finds it
// listed.  Dropping vertices that stopped being ordinary is left to
// prune_rebuild_kernel, run before every captured chain of steps.
__device__ __forceinline__ bool prune_revives(float yraw, float yn) {
    return gnk::mag_bits(yraw) < gnk::kLogTop && gnk::mag_bits(yn) >= gnk::kLogTop;
}

// Writes val into row i's mirror entries, thread t of nt: 16 mirror locations
// loaded back to back per round, so a row costs about two memory latencies
// (row offsets, then the locations) whatever its length per thread.
__device__ __forceinline__ void prune_write(const StepArgs& a, int i, int val, int t, int nt) {
    constexpr int U = 16;
    const int e1 = a.row_ptr[i + 1];
    for (int e = a.row_ptr[i] + t; e < e1; e += nt * U) {
        int m[U];
#pragma unroll
        for (int u = 0; u < U; ++u) m[u] = e + u * nt < e1 ? a.mloc[e + u * nt] : -1;
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (m[u] >= 0) a.pbuf[m[u]] = val;
    }
}

// Row epilogue; returns true when the input state fails the stopping test at row
// i.  act is set when the row must list itself in the pruned lists.
__device__ __forceinline__ bool row_update(const StepArgs& a, const StepCtl<StepArgs>& c, int i, float yraw,
                                           float vi, float sigma, bool nbr_sel, int& fb, int& act) {
    const float yi = fabsf(yraw);
    const float s = __fmaf_rn(c.g, sigma, yi);
    const bool fallback = !(s > 1e-9f);
    if (a.s_out) a.s_out[i] = s;
    if (c.do_write) {
        const float yn = gnk::step_word(yraw, vi, s);
        if (a.y_out) a.y_out[i] = yn;
        if (a.x_out_user) a.x_out_user[a.perm[i]] = gnk::step_x(yraw, vi, s, yn);
        fb += fallback ? 1 : 0;
        if (a.prune && prune_revives(yraw, yn) && !a.listed[i]) {
            act = 1;
            a.listed[i] = 1;
        }
    }
    if (!c.do_test) return false;
    const bool in_s = sign_of(yraw) != 0u;
    const float tv = c.tau * vi;
    const bool far = (yi > tv) && ((vi - yi) > tv);   // min(x, 1-x) > tau with x = y/v
    const bool uncovered = !in_s && !nbr_sel;
    const bool growing = !in_s && (yi > 0.0f) && !(s > vi);
    return far || uncovered || growing;
}

// Rows of a sliced bin: one wavefront per slice of 64/G rows, G threads per row,
// MAXD = the bin's degree bound.  Returns -1 when the launch does no work, else
// whether the thread's row failed the stopping test.
template <int G, int MAXD>
__device__ __forceinline__ int sliced_rows(const StepArgs& a, StepCtl<StepArgs>& c, int b, int rb, int re, int lb, int& fb) {
    constexpr int RS = 64 / G;
    lb = swizzle_block(lb, a.bins.blk_begin[b + 1] - a.bins.blk_begin[b]);
    const int lane = threadIdx.x & 63;
    const int ls = lb * kWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // slice inside the bin
    const int r0 = rb + ls * RS;
    if (r0 >= re) {  // whole wavefront past the bin
        c.fetch(a);
        return c.proceed(a) ? 0 : -1;
    }
    const int t = lane & (G - 1);
    const int i = r0 + lane / G;
    const bool valid = i < re;
    const int gs = a.bins.slice_begin[b] + ls;
    const int l0 = a.sl_off[gs];
    const int width = a.sl_off[gs + 1] - l0;
    float yraw = 0.0f, vi = 1.0f;
    if (valid) {
        yraw = a.y_in[i];
        vi = gnk::ld_stream(a.v + i);
    }
    gnk::SlicedIdx<G, MAXD> idx;
    idx.load(a.sl_col + (size_t)l0 * 64 + lane, width);
    c.fetch(a);
    if (!c.proceed(a)) return -1;
    unsigned sel = 0u;
    const float sigma = idx.template sum<true>(a.y_in, sel);
    const bool any_sel = gnk::group_any<G>(sel != 0u);
    int res = 0, act = 0;
    if (valid && t == 0) res = row_update(a, c, i, yraw, vi, sigma, any_sel, fb, act) ? 1 : 0;
    if (a.prune) {  // the row's G threads write its mirror entries
        if constexpr (G > 1) act = __shfl(act, lane & ~(G - 1), 64);
        if (act) prune_write(a, i, i, t, G);
    }
    return res;
}

}  // namespace

__global__ __launch_bounds__(kBlock) void wrgn_step_kernel(StepArgs a) {
    __shared__ float stage[kStage];
    __shared__ int s_viol[kWaves];
    __shared__ int s_fb[kWaves];
    __shared__ int s_act;

    // the gamma and flag tables cover every step index a captured chain can reach
    StepCtl<StepArgs> c;

    const int blk = blockIdx.x;
    int b = 0;
    while (b < BIN_COUNT - 1 && blk >= a.bins.blk_begin[b + 1]) ++b;
    const int lb = blk - a.bins.blk_begin[b];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int rb = a.bins.row_begin[b], re = a.bins.row_begin[b + 1];
    int r = 0;
    int fb = 0;

    if (b == BIN_BLOCK) {
        // one workgroup per row: all waves gather neighbour values into LDS,
        // wave 0 runs the 64 canonical chains over them
        const int i = rb + lb;
        const int start = gnk::ld_stream(a.row_ptr + i);
        const int d = gnk::ld_stream(a.row_ptr + i + 1) - start;
        const float yraw = a.y_in[i];
        const float vi = a.v[i];
        c.fetch(a);
        if (!c.proceed(a)) return;
        constexpr int PT = kStage / kBlock;  // entries per thread per chunk
        float acc = 0.0f;
        unsigned sel = 0u;
        for (int c0 = 0; c0 < d; c0 += kStage) {
            const int cn = min(kStage, d - c0);
            int cidx[PT];
#pragma unroll
            for (int u = 0; u < PT; ++u) {
                const int p = threadIdx.x + kBlock * u;
                cidx[u] = p < cn ? a.col[start + c0 + p] : -1;
            }
#pragma unroll
            for (int u = 0; u < PT; ++u) {
                // -1 inside the row: an entry of the pruned lists, which adds nothing
                const int p = threadIdx.x + kBlock * u;
                if (p < cn) stage[p] = cidx[u] >= 0 ? a.y_in[cidx[u]] : 0.0f;
            }
            __syncthreads();
            if (wave == 0) {
                for (int q = lane; q < cn; q += 64) {
                    const float yv = stage[q];
                    acc += gnk::nbr_term(yv);
                    sel |= sign_of(yv);
                }
            }
            __syncthreads();
        }
        if (wave == 0) {
            for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
            const bool any_sel = __any(sel != 0u);
            int act = 0;
            if (lane == 0) {
                r = row_update(a, c, i, yraw, vi, acc, any_sel, fb, act) ? 1 : 0;
                s_act = act;
            }
        }
        if (a.prune) {  // the whole workgroup writes the row's mirror entries
            __syncthreads();
            if (s_act) prune_write(a, i, i, threadIdx.x, kBlock);
        }
    } else if (b == BIN_WAVE) {
        // two rows per wavefront, all their loads in flight together
        const int ia = rb + (lb * kWaves + wave) * 2;
        const int ib = ia + 1;
        const bool act = ia < re, hb = ib < re;
        int sa = 0, ea = 0, sb = 0, eb = 0;
        float ya = 0.0f, va = 1.0f, yb = 0.0f, vb = 1.0f;
        if (act) {
            sa = gnk::ld_stream(a.row_ptr + ia);
            ea = gnk::ld_stream(a.row_ptr + ia + 1);
            ya = a.y_in[ia];
            va = a.v[ia];
            if (hb) {
                sb = ea;
                eb = gnk::ld_stream(a.row_ptr + ib + 1);
                yb = a.y_in[ib];
                vb = a.v[ib];
            }
        }
        c.fetch(a);
        if (!c.proceed(a)) return;
        if (act) {
            unsigned sela = 0u, selb = 0u;
            float acca, accb;
            gnk::row_sum_wave2<kWaveMaxDeg / 64>(a.col + sa, ea - sa, a.col + sb, eb - sb, a.y_in, lane, acca, accb,
                                                 sela, selb);
            const bool anya = __any(sela != 0u);
            const bool anyb = __any(selb != 0u);
            int pact = 0;
            if (lane == 0) r = row_update(a, c, ia, ya, va, acca, anya, fb, pact) ? 1 : 0;
            if (lane == 1 && hb) r = row_update(a, c, ib, yb, vb, accb, anyb, fb, pact) ? 1 : 0;
            if (a.prune) {  // the whole wavefront writes the rows' mirror entries
                const int act_a = __shfl(pact, 0, 64), act_b = __shfl(pact, 1, 64);
                if (act_a) prune_write(a, ia, ia, lane, 64);
                if (act_b) prune_write(a, ib, ib, lane, 64);
            }
        }
    } else {
        if (b == BIN_G8) r = sliced_rows<8, 128>(a, c, b, rb, re, lb, fb);
        else if (b == BIN_LANE32) r = sliced_rows<2, 32>(a, c, b, rb, re, lb, fb);
        else r = sliced_rows<1, 16>(a, c, b, rb, re, lb, fb);
        if (r < 0) return;  // uniform over the grid
    }

    if (a.solve) {
        // per-wavefront ballots into one slot per wavefront (no initialisation
        // needed), one barrier, one global write per block; each thread updates at
        // most one row, so fb is 0 or 1
        const bool wv = __ballot(r > 0) != 0ull;
        const int wf = __popcll(__ballot(fb != 0));
        if (lane == 0) {
            s_viol[wave] = wv ? 1 : 0;
            s_fb[wave] = wf;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int v = 0, f = 0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                v |= s_viol[w];
                f += s_fb[w];
            }
            if (v) a.notconv[a.k] = 1;
            if (f) atomicAdd(&a.st->fallback, (unsigned long long)f);
        }
    }
}

// Drops from the pruned lists every listed vertex whose word in y (the input
// of the next step) is not ordinary, and lists any ordinary one that is not
// (none while the invariant holds; at a solve's start, y_0 decides).  Eight
// lanes per row, each writing every eighth mirror entry; rows whose listing is
// already right cost one byte and one word read.
__global__ __launch_bounds__(256) void prune_rebuild_kernel(int32_t n, const int32_t* __restrict__ row_ptr,
                                                           const int32_t* __restrict__ mloc,
                                                           const float* __restrict__ y, uint8_t* __restrict__ listed,
                                                           int32_t* __restrict__ pbuf) {
    constexpr int G = 8, U = 16;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t i = (int32_t)(tid / G);
    const int t = (int)(tid % G);
    if (i >= n) return;
    const bool want = gnk::mag_bits(y[i]) >= gnk::kLogTop;
    if ((listed[i] != 0) == want) return;
    const int32_t val = want ? i : -1;
    const int32_t e1 = row_ptr[i + 1];
    for (int32_t e = row_ptr[i] + t; e < e1; e += G * U) {
        int32_t m[U];
#pragma unroll
        for (int u = 0; u < U; ++u) m[u] = e + u * G < e1 ? mloc[e + u * G] : -1;
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (m[u] >= 0) pbuf[m[u]] = val;
    }
    if (t == 0) listed[i] = want ? 1 : 0;
}

gn_status gn_internal_launch_step(const gn_graph* g, const StepArgs& a, hipStream_t s) {
    const int nblk = gn_internal_grid_blocks(g->bins);
    if (nblk == 0) return GN_OK;
    hipLaunchKernelGGL(wrgn_step_kernel, dim3(nblk), dim3(kBlock), 0, s, a);
    GN_HIP_TRY(hipGetLastError());
    return GN_OK;
}
