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

// The sliced layout and its row sums are in gn_slices.h.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <type_traits>
#include <vector>

#include "gn_batch_internal.h"
#include "gn_internal.h"
#include "gn_rowsum.h"
#include "gn_slices.h"

using namespace gnsl;

namespace {

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
        ya[i] = gnk::word_from_x(x, vi);
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
                const float yr = valid ? yin[i] : 0.0f;  // issued ahead of the gathers
                const int o = so[s];
                const int W = __builtin_amdgcn_readfirstlane(so[s + 1] - o);
                unsigned bits = 0u;
                const float sigma = slice_sum<1, 16, kLightMaxDeg>(ln + o * 64 + lane, W, yin, bits);
                if (valid)
                    viol |= step_row(yr, vi, sigma, (bits >> 31) != 0u, g, do_test, do_write, a.tau, yout, i, fb);
            }
#pragma unroll 1
            for (int s = w_mid; s < nM; s += NW) {
                const int i = d.n_light + 8 * s + (lane >> 3);
                const bool valid = i < d.n_mid && (lane & 7) == 0;
                const float vi = valid ? vv[i] : 1.0f;
                const float yr = valid ? yin[i] : 0.0f;
                const int o = so[nL + s];
                const int W = __builtin_amdgcn_readfirstlane(so[nL + s + 1] - o);
                unsigned bits = 0u;
                const float sigma = slice_sum<8, 8, kMidMaxDegCap / 8>(ln + o * 64 + lane, W, yin, bits);
                const bool any_sel = gnk::group_any<8>((bits >> 31) != 0u);
                if (valid) viol |= step_row(yr, vi, sigma, any_sel, g, do_test, do_write, a.tau, yout, i, fb);
            }
#pragma unroll 1
            for (int s = w_heavy; s < n - d.n_mid; s += NW) {
                const int i = d.n_mid + s;
                const float vi = lane == 0 ? vv[i] : 1.0f;
                const float yr = lane == 0 ? yin[i] : 0.0f;
                const int o = so[nL + nM + s];
                const int W = __builtin_amdgcn_readfirstlane(so[nL + nM + s + 1] - o);
                unsigned bits = 0u;
                const float sigma = heavy_sum(ln + o * 64 + lane, W, yin, bits);
                const bool any_sel = __any((bits >> 31) != 0u);
                if (lane == 0) viol |= step_row(yr, vi, sigma, any_sel, g, do_test, do_write, a.tau, yout, i, fb);
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
            viol |= mid_rows<BT, kMidMaxDegCap, true>(rp_g, col_g, yin, vv, yout, d.n_light, d.n_mid, g, do_test,
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
        float x = gnk::x_of_word(yin[i], vv[i]);
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
        float x = gnk::x_of_word(yin[i], vv[i]);
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

template <int BT, bool BIG>
const void* batch_kernel_ptr() {
    return (const void*)batch_solve_kernel<BT, BIG>;
}

}  // namespace

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

// Relabelling and sliced layout of every graph for the degree bounds of the
// bin schedule: rows of degree <= light first (a lane each, 64 per slice), then
// those of degree <= mid (8 lanes each, 8 per slice), then the rest (a
// wavefront each), each class by decreasing degree (ties in the original
// order); every row keeps its entries in the caller's order, so the canonical
// sums, and with them all results, do not depend on the bounds.  Uploads the
// layout; the previous one (and the solve graph built on it) is dropped.  SYNC.
static gn_status build_layout(gn_batch* b, int32_t light, int32_t mid, hipStream_t stream) {
    const int32_t count = b->count;
    const int64_t tn = b->total_n, tnnz = b->total_nnz;
    int64_t trp = 0;
    for (int32_t g = 0; g < count; ++g) trp += (int64_t)b->h_n[g] + 1;
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
        const int32_t ng = b->h_n[g];
        const int32_t* rp = b->h_rp.data() + ro;
        const int32_t* ci = b->h_ci.data() + eo;
        const float* wg = b->h_w.data() + vo;
        std::vector<int32_t> p((size_t)ng), q((size_t)ng);
        std::iota(p.begin(), p.end(), 0);
        auto cls = [&](int32_t i) {
            const int32_t dg = rp[i + 1] - rp[i];
            return dg <= light ? 0 : dg <= mid ? 1 : 2;
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
        // sliced layout (gn_slices.h)
        const int64_t ln0 = (int64_t)(lines.size() / 64), so0 = (int64_t)slices.size();
        int32_t nlines = 0;
        if (ng <= kMaxSlicedN) {
            const int64_t acc = build_slices(ng, rpi, col_int.data() + eo, 0, nl, nl, nm, nm, ng, lines, slices);
            if (acc > INT32_MAX / 64) return GN_E_ARG;
            nlines = (int32_t)acc;
            state_bytes[g] = state_lds_bytes(ng, slice_count(ng, nl, nm));
            h_slices[g] = slice_count(ng, nl, nm);
            h_lines[g] = nlines;
        }
        desc[g] = BatchDesc{ng, nl, nm, nlines, vo, ro, eo, ln0, so0, (int32_t)b->h_nnz[g], 0};
        vo += ng;
        ro += (int64_t)ng + 1;
        eo += b->h_nnz[g];
    }
    // the layout's variable-size arrays grow on demand
    const size_t nlw = std::max<size_t>(lines.size(), 64), nsl = std::max<size_t>(slices.size(), 1);
    if (nlw > b->lines_cap) {
        if (b->lines) (void)hipFree(b->lines);
        b->lines = nullptr;
        b->lines_cap = 0;
        if (!gn_dalloc(&b->lines, nlw)) return GN_E_NOMEM;
        b->lines_cap = nlw;
    }
    if (nsl > b->slices_cap) {
        if (b->slices) (void)hipFree(b->slices);
        b->slices = nullptr;
        b->slices_cap = 0;
        if (!gn_dalloc(&b->slices, nsl)) return GN_E_NOMEM;
        b->slices_cap = nsl;
    }
    hipError_t e = hipStreamSynchronize(stream);   // no earlier work may still read the old layout
    auto up = [&](void* dst, const void* src, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream);
    };
    up(b->desc, desc.data(), sizeof(BatchDesc) * count);
    up(b->vgraph, vgraph.data(), sizeof(int32_t) * tn);
    up(b->row_ptr, rp_int.data(), sizeof(int32_t) * trp);
    up(b->col, col_int.data(), sizeof(int32_t) * tnnz);
    up(b->lines, lines.data(), sizeof(uint16_t) * lines.size());
    up(b->slices, slices.data(), sizeof(int32_t) * slices.size());
    up(b->v, v_int.data(), sizeof(float) * tn);
    up(b->w, w_int.data(), sizeof(float) * tn);
    up(b->perm, perm.data(), sizeof(int32_t) * tn);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return GN_E_HIP;
    b->h_state = std::move(state_bytes);
    b->h_slices = std::move(h_slices);
    b->h_lines = std::move(h_lines);
    b->lay_light = light;
    b->lay_mid = mid;
    b->split_lds = -1;   // the processing order depends on the graphs' LDS sizes
    if (b->launch.exec) (void)hipGraphExecDestroy(b->launch.exec);
    b->launch.exec = nullptr;
    return GN_OK;
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

    // validate each graph (same conditions as gn_graph_create)
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
    b->h_order = order;
    (void)hipGetDevice(&b->device);
    int cus = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device);
    b->cus = cus > 0 ? cus : 256;
    bool ok = gn_dalloc(&b->desc, count) && gn_dalloc(&b->order, count) && gn_dalloc(&b->vgraph, tn) &&
              gn_dalloc(&b->row_ptr, trp) && gn_dalloc(&b->col, tnnz) && gn_dalloc(&b->v, tn) && gn_dalloc(&b->w, tn) &&
              gn_dalloc(&b->perm, tn) && gn_dalloc(&b->yg0, tn) && gn_dalloc(&b->yg1, tn) && gn_dalloc(&b->queue, 3) &&
              gn_dalloc(&b->res, count);
    if (ok && hipHostMalloc((void**)&b->res_host, sizeof(BatchRes) * count, hipHostMallocDefault) != hipSuccess) {
        b->res_host = nullptr;
        ok = false;
    }
    if (!ok) {
        batch_free(b);
        delete b;
        return GN_E_NOMEM;
    }
    const gn_status st = build_layout(b, kLightMaxDeg, kMidMaxDeg, stream);
    if (st != GN_OK) {
        batch_free(b);
        delete b;
        return st;
    }
    *out = b;
    return GN_OK;
}

// The bin schedule's degree bounds of a tuning (0 selects the default).
static int32_t light_bound(const gn_tuning& t) { return t.light_max_deg ? t.light_max_deg : kLightMaxDeg; }
static int32_t mid_bound(const gn_tuning& t) { return t.mid_max_deg ? t.mid_max_deg : kMidMaxDeg; }

static bool tuning_valid(const gn_tuning& t) {
    const bool bt_ok = t.block_threads == 128 || t.block_threads == 256 || t.block_threads == 512 ||
                       (t.block_threads == 1024 && t.blocks_per_cu <= 2);
    const int32_t lb = light_bound(t), mb = mid_bound(t);
    const bool bins_ok = (lb == 8 || lb == 16) && (mb == 32 || mb == 64 || mb == kMidMaxDegCap);
    return bt_ok && bins_ok && t.blocks_per_cu >= 1 && t.blocks_per_cu <= 4 && t.lds_vertices >= 0 &&
           (size_t)t.lds_vertices * 12 * t.blocks_per_cu <= kLdsBudget;
}

static gn_tuning default_tuning(const gn_batch* b) {
    gn_tuning t{};
    t.block_threads = 256;
    t.blocks_per_cu = 2;
    t.lds_vertices = kLdsBudget / (12 * 2);
    t.light_max_deg = kLightMaxDeg;
    t.mid_max_deg = kMidMaxDeg;
    return t;
}

// The layout of a tuning's bin bounds, rebuilt when they differ from the current one.
static gn_status ensure_layout(gn_batch* b, const gn_tuning& t, hipStream_t s) {
    if (b->lay_light == light_bound(t) && b->lay_mid == mid_bound(t)) return GN_OK;
    return build_layout(b, light_bound(t), mid_bound(t), s);
}

static gn_status ensure_gamma(gn_batch* b, int32_t entries) {
    if (entries <= b->gamma_cap) return GN_OK;
    if (b->gamma) (void)hipFree(b->gamma);
    b->gamma = nullptr;
    b->gamma_cap = 0;
    if (!gn_dalloc(&b->gamma, (size_t)entries)) return GN_E_NOMEM;
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
    if ((st = ensure_layout(b, t, s)) != GN_OK) return st;
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
           k.t.lds_vertices == t.lds_vertices && light_bound(k.t) == light_bound(t) &&
           mid_bound(k.t) == mid_bound(t) && k.sch.gamma0 == sch->gamma0 && k.sch.gamma1 == sch->gamma1 &&
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

// Tunings found by gn_batch_autotune, kept for the process and keyed by a
// signature of the batch: graph count, total vertices and entries (each by its
// power of two), the degree histogram (the fraction of rows of degree <= 8,
// <= 16, <= 32, <= 64, <= 128 and above, in steps of 1/32), and the schedule's
// step budget (by its power of two).
static std::mutex g_tune_mu;
static std::map<std::vector<int64_t>, gn_tuning> g_tune_cache;

static int64_t log2_bucket(int64_t v) {
    int64_t k = 0;
    while (v > 1) {
        v >>= 1;
        ++k;
    }
    return k;
}

static std::vector<int64_t> batch_signature(const gn_batch* b, const gn_schedule* sch) {
    int64_t hist[6] = {0, 0, 0, 0, 0, 0};
    int64_t ro = 0;
    for (int32_t g = 0; g < b->count; ++g) {
        const int32_t* rp = b->h_rp.data() + ro;
        for (int32_t i = 0; i < b->h_n[g]; ++i) {
            const int32_t d = rp[i + 1] - rp[i];
            hist[d <= 8 ? 0 : d <= 16 ? 1 : d <= 32 ? 2 : d <= 64 ? 3 : d <= 128 ? 4 : 5]++;
        }
        ro += (int64_t)b->h_n[g] + 1;
    }
    std::vector<int64_t> sig = {log2_bucket(b->count), log2_bucket(b->total_n), log2_bucket(b->total_nnz),
                                log2_bucket(sch->max_steps)};
    for (int64_t h : hist) sig.push_back(b->total_n ? (h * 32 + b->total_n / 2) / b->total_n : 0);
    return sig;
}

extern "C" int32_t gn_batch_tuning_cache_size(void) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    return (int32_t)g_tune_cache.size();
}

extern "C" void gn_batch_tuning_cache_clear(void) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune_cache.clear();
}

extern "C" gn_status gn_batch_autotune(gn_batch* b, const gn_schedule* sch, gn_tuning* out, hipStream_t stream) {
    if (!b || !out) return GN_E_ARG;
    gn_status st = check_schedule(sch);
    if (st != GN_OK) return st;
    const std::vector<int64_t> sig = batch_signature(b, sch);
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tune_cache.find(sig);
        if (it != g_tune_cache.end()) {
            if ((st = ensure_layout(b, it->second, stream)) != GN_OK) return st;
            b->tuning = it->second;
            b->tuned = true;
            *out = it->second;
            return GN_OK;
        }
    }
    // per candidate: a warm-up run of at most 64 steps, then one timed full
    // solve, from x0 = 1/2 (the largest graphs set the wall time, and only a
    // full solve shows their tail).  The launch shapes are searched at the
    // default bin bounds, then the bounds at the best shape, then the shapes
    // again at the best bounds.
    gn_schedule ws = *sch;
    ws.max_steps = std::min<int32_t>(sch->max_steps, 64);
    float* x = nullptr;
    uint8_t* sel = nullptr;
    if (!gn_dalloc(&x, (size_t)b->total_n) || !gn_dalloc(&sel, (size_t)b->total_n)) {
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
    auto time_one = [&](const gn_tuning& t) -> float {
        allow_lds(t.block_threads, (size_t)t.lds_vertices * 12);
        float ms_sum = 0.0f;
        for (int rep = 0; rep < 2 && st == GN_OK; ++rep) {
            if (hipMemcpyAsync(x, half.data(), sizeof(float) * b->total_n, hipMemcpyHostToDevice, stream) !=
                hipSuccess) {
                st = GN_E_HIP;
                break;
            }
            if ((st = ensure_layout(b, t, stream)) != GN_OK) break;  // rebuilds outside the timed region
            (void)hipEventRecord(e0, stream);
            st = enqueue_batch(b, rep == 0 ? &ws : sch, t, x, sel, stream);
            (void)hipEventRecord(e1, stream);
            if (hipEventSynchronize(e1) != hipSuccess) st = GN_E_HIP;
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (rep == 1) ms_sum += ms;
        }
        return st == GN_OK ? ms_sum : INFINITY;
    };
    auto search_shapes = [&](int32_t lb, int32_t mb) {
        for (int bt : {128, 256, 512, 1024}) {
            for (int bpc : {1, 2, 4}) {
                gn_tuning t{};
                t.block_threads = bt;
                t.blocks_per_cu = bpc;
                t.lds_vertices = kLdsBudget / (12 * bpc);
                t.light_max_deg = lb;
                t.mid_max_deg = mb;
                if (!tuning_valid(t)) continue;
                allow_lds(bt, (size_t)t.lds_vertices * 12);
                if (resident_blocks(bt, (size_t)t.lds_vertices * 12) < bpc) continue;  // same launch as a smaller bpc
                const float ms = time_one(t);
                if (st != GN_OK) return;
                if (ms < best_ms) {
                    best_ms = ms;
                    best = t;
                }
            }
        }
    };
    search_shapes(kLightMaxDeg, kMidMaxDeg);
    const gn_tuning shape = best;
    for (int32_t lb : {8, 16}) {
        for (int32_t mb : {32, 64, kMidMaxDegCap}) {
            if (st != GN_OK || (lb == kLightMaxDeg && mb == kMidMaxDeg)) continue;
            gn_tuning t = shape;
            t.light_max_deg = lb;
            t.mid_max_deg = mb;
            const float ms = time_one(t);
            if (st == GN_OK && ms < best_ms) {
                best_ms = ms;
                best = t;
            }
        }
    }
    if (st == GN_OK && (light_bound(best) != kLightMaxDeg || mid_bound(best) != kMidMaxDeg))
        search_shapes(light_bound(best), mid_bound(best));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(x);
    (void)hipFree(sel);
    if (st != GN_OK) return st;
    if ((st = ensure_layout(b, best, stream)) != GN_OK) return st;
    b->tuning = best;
    b->tuned = true;
    *out = best;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune_cache[sig] = best;
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

