// Batched differentiable GN: every graph's unrolled steps and their adjoint in
// one workgroup each (see the section comment below).
#include <algorithm>
#include <cmath>
#include <vector>

#include "gn_batch_internal.h"
#include "gn_internal.h"
#include "gn_rowsum.h"
#include "gn_slices.h"

using namespace gnsl;

namespace {

// ---------------------------------------------------------------------------
// Unrolled (differentiable) steps of a whole batch: every graph's T forward
// steps, or its T adjoint steps, in one workgroup with its state in LDS.  The
// arithmetic repeats the chained unrolled path (gn_unrolled.hip) operation for
// operation -- y = v x, s = y + gamma sum |y_j|, x' = y / s with the safe
// division, in the library's state words; t = gbar y / s^2, dL/dy = gbar / s - (t + gamma
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
// on the same fp32 value as the chained adjoint).
__device__ __forceinline__ bool unrolled_quotient(float s) { return s > 1e-9f; }

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
        const float sigma = slice_sum<8, 8, kMidMaxDegCap / 8, ABS>(ln + o * 64 + lane, W, src, bits);
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
    float v, x, s, yp, sp;
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
    for (int i = tid; i < n; i += BT) ya[i] = gnk::word_from_x(a.x0[d.v_off + perm[i]], vv[i]);
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
                const float yn = gnk::step_word(yraw, p.v, s);
                ys[i] = yraw;
                ss[i] = s;
                yout[i] = yn;
                if (xT) xT[perm[i]] = gnk::step_x(yraw, p.v, s, yn);
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
        const float yy = gnk::y_of_word(ylast[i], vv[i]), s = slast[i];
        ta[i] = unrolled_quotient(s) ? (g / s) * (yy / s) : 0.0f;
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
                p.x = gnk::x_of_word(yk[i], p.v);
                p.s = sk[i];
                p.yp = yp ? gnk::y_of_word(yp[i], p.v) : 0.0f;
                p.sp = yp ? sp[i] : 0.0f;
                return p;
            },
            [&](int i, float sigma, const BwdPre& p) {
                const float g = gb[i];
                const float ai = unrolled_quotient(p.s) ? g / p.s : 0.0f;
                const float gy = ai - __fmaf_rn(gam, sigma, tin[i]);
                const float gx = p.v * gy;
                gb[i] = gx;
                gv[i] += p.x * gy;
                if (yp) tout[i] = unrolled_quotient(p.sp) ? (gx / p.sp) * (p.yp / p.sp) : 0.0f;
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

}  // namespace

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
        if (!gn_dalloc(&b->u_order, (size_t)b->count) || !gn_dalloc(&b->u_queue, 1)) return GN_E_NOMEM;
        GN_HIP_TRY(hipMemcpy(b->u_order, b->h_order.data(), sizeof(int32_t) * b->count, hipMemcpyHostToDevice));
    }
    if (T > b->u_gamma_cap) {
        if (b->u_gamma) (void)hipFree(b->u_gamma);
        b->u_gamma = nullptr;
        b->u_gamma_cap = 0;
        b->u_gamma_host.clear();
        if (!gn_dalloc(&b->u_gamma, (size_t)T)) return GN_E_NOMEM;
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
        if (!b->u_v && !gn_dalloc(&b->u_v, (size_t)b->total_n)) return GN_E_NOMEM;
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

