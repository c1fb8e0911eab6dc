// Single-workgroup solve of small graphs for gn_solve (see below).
#include <algorithm>
#include <climits>
#include <vector>

#include "gn_internal.h"
#include "gn_rowsum.h"
#include "gn_slices.h"

using namespace gnsl;

namespace {

// One small graph, one workgroup: the whole solve in a single launch, steps
// separated by workgroup barriers instead of kernel boundaries.  Works on the
// graph handle's internal order: rows [0, mid_begin) have degree > 128 (one
// wavefront each), rows [mid_begin, light_begin) degree 17 .. 128 (8 threads
// each), the rest degree <= 16 (a thread each).  The graph's LDS image -- the
// sliced layout of gn_slices.h, lines of up to 16 per mid slice --
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
            const float yr = valid ? yin[i] : 0.0f;  // issued ahead of the gathers
            const int o = so[s];
            const int W = __builtin_amdgcn_readfirstlane(so[s + 1] - o);
            unsigned bits = 0u;
            const float sigma = slice_sum<1, 16, 16>(ln + o * 64 + lane, W, yin, bits);
            if (valid) viol |= step_row(yr, vi, sigma, (bits >> 31) != 0u, g, do_test, do_write, tau, yout, i, fb);
        }
#pragma unroll 1
        for (int s = w_mid; s < nM; s += NW) {
            const int i = mb + 8 * s + (lane >> 3);
            const bool valid = i < lb && (lane & 7) == 0;
            const float vi = valid ? vv[i] : 1.0f;
            const float yr = valid ? yin[i] : 0.0f;
            const int o = so[nL + s];
            const int W = __builtin_amdgcn_readfirstlane(so[nL + s + 1] - o);
            unsigned bits = 0u;
            const float sigma = slice_sum<8, 8, 16>(ln + o * 64 + lane, W, yin, bits);
            const bool any_sel = gnk::group_any<8>((bits >> 31) != 0u);
            if (valid) viol |= step_row(yr, vi, sigma, any_sel, g, do_test, do_write, tau, yout, i, fb);
        }
#pragma unroll 1
        for (int s = w_heavy; s < nH; s += NW) {
            const int i = s;
            const float vi = lane == 0 ? vv[i] : 1.0f;
            const float yr = lane == 0 ? yin[i] : 0.0f;
            const int o = so[nL + nM + s];
            const int W = __builtin_amdgcn_readfirstlane(so[nL + nM + s + 1] - o);
            unsigned bits = 0u;
            const float sigma = heavy_sum(ln + o * 64 + lane, W, yin, bits);
            const bool any_sel = __any((bits >> 31) != 0u);
            if (lane == 0) viol |= step_row(yr, vi, sigma, any_sel, g, do_test, do_write, tau, yout, i, fb);
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

}  // namespace

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
    bool ok = gn_dalloc(&im->so, slices.size()) && gn_dalloc(&im->ln, std::max<size_t>(lines.size(), 64)) &&
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
