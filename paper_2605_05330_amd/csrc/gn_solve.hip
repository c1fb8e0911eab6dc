// Solve driver of the graph solver and the pieces it shares with the assignment
// and multi-start solvers: state preparation, the normalizable check, the gamma
// table, captured chains of step launches replayed with a pipelined host check,
// the stopping outcome and the result record.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>

#include "gn_internal.h"
#include "gn_rowsum.h"

// defined in gn_step.hip
__global__ void wrgn_step_kernel(StepArgs a);
__global__ void prune_rebuild_kernel(int32_t n, const int32_t* row_ptr, const int32_t* mloc, const float* y,
                                     uint8_t* listed, int32_t* pbuf);

// x (user order) -> signed weighted state y (internal order); flags x < 0 or
// non-finite (err bit 1).
__global__ void prep_state_kernel(int32_t n, const float* __restrict__ x_user, const int32_t* __restrict__ perm,
                                  const float* __restrict__ v, float* __restrict__ y, SolveState* st) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x = x_user[perm[i]];
    if (!(x >= 0.0f) || !isfinite(x)) {
        if (st) atomicOr(&st->err, 1);
        x = 0.0f;
    }
    y[i] = gnk::word_from_x(x, v[i]);
}

// Normalizable (Section 2): (A + I) x > 0, i.e. x_i > 0 or some neighbour
// x_j > 0.  Flags err bit 2 otherwise.
__global__ void normalizable_kernel(int32_t n, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                    const float* __restrict__ x_user, const int32_t* __restrict__ perm,
                                    SolveState* st) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (x_user[perm[i]] > 0.0f) return;
    for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
        if (x_user[perm[col[e]]] > 0.0f) return;
    atomicOr(&st->err, 2);
}

// A solve's outcome after its last step, as gn_internal_solve_outcome decides
// it on the host: the stop's step when the stopping test passed, else max_steps,
// binarised when that last state passed the test; the final state words are
// y[steps & 1] and its gamma the table's entry for that step.
__global__ void pick_final_kernel(const SolveState* __restrict__ st, const int32_t* __restrict__ notconv,
                                  int32_t ms, const float* __restrict__ gamma, const float* y0, const float* y1,
                                  SolveTail* tail) {
    if (threadIdx.x != 0) return;
    const SolveState s = *st;
    FinalPick p;
    if (s.done_step >= 0) {
        p.steps = s.done_step;
        p.binarised = 1;
    } else {
        p.steps = ms;
        p.binarised = ms >= 1 && notconv[ms] == 0;
    }
    p.y = (p.steps & 1) ? y1 : y0;
    p.gamma = gamma[p.steps];
    p.skip = s.err != 0;
    tail->pick = p;
    tail->state = s;
}

// Reset the solve state and fill the gamma table (Section 6 gamma-pursuit,
// evaluated in double and rounded once to fp32).
__global__ void init_solve_kernel(SolveState* st, int32_t* notconv, float* gamma, int32_t max_steps,
                                  int32_t check_every, float tau, float g0, float g1, int32_t ramp) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) {
        st->done_step = -1;
        st->err = 0;
        st->max_steps = max_steps;
        st->check_every = check_every;
        st->tau = tau;
        st->pad = 0;
        st->fallback = 0ull;
    }
    for (int k = t; k <= max_steps; k += gridDim.x * blockDim.x) {
        notconv[k] = 0;
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

float gn_internal_host_gamma(const gn_schedule* s, int32_t k) {
    if (s->ramp_steps <= 1) return s->gamma1;
    const int32_t kk = k < s->ramp_steps - 1 ? k : s->ramp_steps - 1;
    const double p = (double)kk / (double)(s->ramp_steps - 1);
    return (float)(p * (double)s->gamma1 + (1.0 - p) * (double)s->gamma0);
}

bool gn_internal_schedule_ok(const gn_schedule* sch) {
    return sch->max_steps >= 0 && sch->check_every >= 1 && sch->tau >= 0.0f && std::isfinite(sch->tau) &&
           std::isfinite(sch->gamma0) && std::isfinite(sch->gamma1) && sch->gamma0 >= 0.0f && sch->gamma1 >= 0.0f &&
           sch->max_steps <= (1 << 28);
}

gn_status gn_internal_init_solve(GraphWorkspace& ws, const gn_schedule* sch, hipStream_t stream) {
    const int32_t ms = sch->max_steps;
    hipLaunchKernelGGL(init_solve_kernel, dim3(std::min((ms + 1 + 255) / 256, 1024)), dim3(256), 0, stream, ws.state,
                       ws.notconv, ws.gamma, ms, sch->check_every, sch->tau, sch->gamma0, sch->gamma1,
                       sch->ramp_steps);
    GN_HIP_TRY(hipGetLastError());
    return GN_OK;
}

gn_status gn_internal_solve_outcome(const GraphWorkspace& ws, int32_t ms, int32_t* steps, bool* binarised) {
    SolveState hs;
    int32_t nc_last = 1;
    GN_HIP_TRY(hipMemcpy(&hs, ws.state, sizeof(hs), hipMemcpyDeviceToHost));
    GN_HIP_TRY(hipMemcpy(&nc_last, ws.notconv + ms, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (hs.err & 1) return GN_E_ARG;
    if (hs.err & 2) return GN_E_NOT_NORMALIZABLE;
    if (hs.done_step >= 0) {
        *steps = hs.done_step;
        *binarised = true;
    } else {
        *steps = ms;
        *binarised = ms >= 1 && nc_last == 0;
    }
    return GN_OK;
}

static gn_status fill_result(const SolveState& hs, int32_t steps, bool binarised, const FinalStats& fs,
                             gn_result* res) {
    res->steps = steps;
    res->binarised = binarised ? 1 : 0;
    res->fallback_count = (int64_t)hs.fallback;
    res->relaxed_objective = fs.relaxed_objective;
    res->set_objective = fs.set_objective;
    res->set_size = fs.set_size;
    res->conflicts = fs.conflicts;
    res->uncovered = fs.uncovered;
    res->stab = fs.stab;
    return binarised ? GN_OK : GN_NOT_CONVERGED;
}

gn_status gn_internal_fill_result(const GraphWorkspace& ws, int32_t steps, bool binarised, const FinalStats& fs,
                                  gn_result* res) {
    SolveState hs;
    GN_HIP_TRY(hipMemcpy(&hs, ws.state, sizeof(hs), hipMemcpyDeviceToHost));
    return fill_result(hs, steps, binarised, fs, res);
}

static StepArgs base_args(const gn_graph* g) {
    StepArgs a{};
    a.row_ptr = g->row_ptr;
    a.col = g->col;
    a.v = g->v;
    a.perm = g->perm;
    a.sl_col = g->sl_col;
    a.sl_off = g->sl_off;
    a.bins = g->bins;
    return a;
}

gn_status gn_internal_step_with(const gn_graph* g, float gamma, const float* x_in, float* x_out, float* y_words,
                                hipStream_t stream) {
    const int n = g->n;
    hipLaunchKernelGGL(prep_state_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, n, x_in, g->perm, g->v,
                       y_words, (SolveState*)nullptr);
    GN_HIP_TRY(hipGetLastError());
    StepArgs a = base_args(g);
    a.y_in = y_words;
    a.y_out = nullptr;
    a.gamma = nullptr;
    a.gamma_scalar = gamma;
    a.solve = 0;
    a.x_out_user = x_out;
    return gn_internal_launch_step(g, a, stream);
}

gn_status gn_internal_step_args_ok(const gn_graph* g, float gamma, const float* x_in, float* x_out) {
    if (!g) return GN_E_ARG;
    if (!std::isfinite(gamma) || gamma < 0.0f) return GN_E_ARG;
    if (g->n == 0) return GN_OK;
    if (!x_in || !x_out || x_in == x_out) return GN_E_ARG;
    return GN_OK;
}

extern "C" gn_status gn_step(const gn_graph* g, float gamma, const float* x_in, float* x_out,
                             hipStream_t stream) {
    gn_status st = gn_internal_step_args_ok(g, gamma, x_in, x_out);
    if (st != GN_OK || g->n == 0) return st;
    gn_graph* gm = const_cast<gn_graph*>(g);
    st = gn_internal_ensure_ws(gm, 1);
    if (st != GN_OK) return st;
    return gn_internal_step_with(g, gamma, x_in, x_out, g->ws.y[0], stream);
}

// Progress mark of chain c for the host, a node inside the chain (one
// wavefront): words2 words from src2 to dst2 when given, the solve state's done
// step and error word, then the marker c + 1 (release), all stored to pinned
// memory with system scope.
__global__ void chain_mark_kernel(const SolveState* __restrict__ st, int32_t* slot, int32_t marker,
                                  const int32_t* __restrict__ src2, int32_t words2, int32_t* dst2) {
    for (int i = threadIdx.x; i < words2; i += blockDim.x)
        __hip_atomic_store(dst2 + i, src2[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x != 0) return;
    __hip_atomic_store(slot + 1, st->done_step, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(slot + 2, st->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(slot, marker, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Steps [c*len + j0, c*len + j1) of chain c of `len` step launches, added to
// `graph` after *prev (updated to the last node).  When the pruned lists are
// used, they are rebuilt before every step k that is a multiple of the rebuild
// interval, from k's input state (step 0's rebuild sets the lists for the
// solve's start).
static gn_status build_steps(gn_graph* g, int32_t c, int32_t len, bool prune, int32_t j0, int32_t j1,
                             hipGraph_t graph, hipGraphNode_t* last) {
    GraphWorkspace& ws = g->ws;
    if (prune && (!g->prune || !g->prune_mloc || !g->listed)) return GN_E_ARG;  // no pruned lists to read
    hipGraphNode_t prev = *last;
    const int nblk = gn_internal_grid_blocks(g->bins);
    for (int32_t j = j0; j < j1; ++j) {
        if (prune && gn_internal_rebuilds_at((int64_t)c * len + j)) {  // rebuild of the lists from step k's input
            int32_t n = g->n;
            const int32_t* rp = g->row_ptr;
            const int32_t* ml = g->prune_mloc;
            const float* y = ws.y[(c * len + j) & 1];
            uint8_t* lst = g->listed;
            int32_t* pb = g->prune;
            void* args[] = {&n, &rp, &ml, &y, &lst, &pb};
            hipKernelNodeParams p{};
            p.func = (void*)prune_rebuild_kernel;
            p.gridDim = dim3((unsigned)(((int64_t)n * 8 + 255) / 256));
            p.blockDim = dim3(256);
            p.sharedMemBytes = 0;
            p.kernelParams = args;
            p.extra = nullptr;
            hipGraphNode_t node;
            if (hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &p) != hipSuccess)
                return GN_E_HIP;
            prev = node;
        }
        StepArgs a = base_args(g);
        a.k = c * len + j;
        a.y_in = ws.y[a.k & 1];
        a.y_out = ws.y[(a.k + 1) & 1];
        a.gamma = ws.gamma;
        a.solve = 1;
        a.st = ws.state;
        a.notconv = ws.notconv;
        a.x_out_user = nullptr;
        if (prune) {
            a.prune = 1;
            a.pbuf = g->prune;
            a.mloc = g->prune_mloc;
            a.listed = g->listed;
            a.sl_col = g->prune;
            a.col = g->prune + g->prune_sl_words;
        }
        void* args[] = {&a};
        hipKernelNodeParams p{};
        p.func = (void*)wrgn_step_kernel;
        p.gridDim = dim3(nblk);
        p.blockDim = dim3(kBlock);
        p.sharedMemBytes = 0;
        p.kernelParams = args;
        p.extra = nullptr;
        hipGraphNode_t node;
        if (hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &p) != hipSuccess)
            return GN_E_HIP;
        prev = node;
    }
    *last = prev;
    return GN_OK;
}

int32_t g_chunk_len = 64;
int32_t g_prune = 1;
int32_t g_prune_every = 64;

namespace {

// Marked chains carry their progress mark this many steps before their end:
// the host launches chain c + 1 once chain c's mark is written, so the next
// chain is queued while these steps run, and a solve that has stopped by the
// mark launches no further chain.
constexpr int32_t kMarkLead = 8;
// byte offset of the two mark slots [4 words each] in a workspace's 4 KiB
// pinned block, past what the solvers stage there (gn_solve's epilogue from 0,
// the multi-start solve's staging below 3200 bytes)
constexpr size_t kMarkPin = 3584;
static_assert(sizeof(SolveTail) <= kMarkPin && kMarkPin + 32 <= 4096, "pinned block layout");

// Waits for chain c's mark (spinning on pinned memory; the stream is polled now
// and then so that a failed stream ends the wait).
gn_status wait_mark(volatile int32_t* slot, int32_t marker, hipStream_t stream) {
    for (uint32_t spin = 1;; ++spin) {
        if (__atomic_load_n(slot, __ATOMIC_ACQUIRE) == marker) return GN_OK;
        if ((spin & 1023u) == 0) {
            const hipError_t e = hipStreamQuery(stream);
            if (e == hipSuccess) return __atomic_load_n(slot, __ATOMIC_ACQUIRE) == marker ? GN_OK : GN_E_HIP;
            if (e != hipErrorNotReady) return GN_E_HIP;
        }
    }
}

}  // namespace

gn_status gn_internal_run_marked(GraphWorkspace& ws, int32_t nchunks, int32_t C, const StepRangeBuilder& build,
                                 int32_t c_begin, hipStream_t stream, bool sync_end, const ChunkHooks* hooks,
                                 int32_t* last) {
    if (ws.chunk_len != C) {
        for (auto ex : ws.chunks) if (ex) (void)hipGraphExecDestroy(ex);
        ws.chunks.clear();
        ws.chunk_len = C;
    }
    if (hooks && hooks->pin_src &&
        (hooks->pin_words < 0 || hooks->pin_offset + 8 * (size_t)hooks->pin_words > kMarkPin))
        return GN_E_ARG;  // the two copies must fit below the mark slots
    if ((int32_t)ws.chunks.size() < nchunks) ws.chunks.resize(nchunks, nullptr);
    volatile int32_t* slots = (volatile int32_t*)((char*)ws.host_pinned + kMarkPin);
    char* pin_dev = nullptr;  // the same block as the device addresses it
    GN_HIP_TRY(hipHostGetDevicePointer((void**)&pin_dev, ws.host_pinned, 0));
    const int32_t mark_at = std::max<int32_t>(0, C - kMarkLead);
    // chain c: steps before the mark, the mark, the remaining steps
    auto capture = [&](int32_t c, hipGraph_t graph) -> gn_status {
        hipGraphNode_t prev = nullptr;
        gn_status st = build(c, 0, mark_at, graph, &prev);
        if (st != GN_OK) return st;
        const SolveState* sp = ws.state;
        int32_t* slot = (int32_t*)(pin_dev + kMarkPin) + 4 * (c & 1);
        int32_t marker = c + 1;
        const bool extra = hooks && hooks->pin_src;
        const int32_t* s2 = extra ? (const int32_t*)hooks->pin_src : nullptr;
        int32_t w2 = extra ? hooks->pin_words : 0;
        int32_t* d2 = extra ? (int32_t*)(pin_dev + hooks->pin_offset) + (size_t)w2 * (c & 1) : nullptr;
        void* args[] = {&sp, &slot, &marker, &s2, &w2, &d2};
        hipKernelNodeParams p{};
        p.func = (void*)chain_mark_kernel;
        p.gridDim = dim3(1);
        p.blockDim = dim3(64);
        p.sharedMemBytes = 0;
        p.kernelParams = args;
        p.extra = nullptr;
        hipGraphNode_t node;
        if (hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &p) != hipSuccess)
            return GN_E_HIP;
        prev = node;
        return build(c, mark_at, C, graph, &prev);
    };
    auto launch = [&](int32_t c) -> gn_status {
        if (!ws.chunks[c]) {
            hipGraph_t graph;
            GN_HIP_TRY(hipGraphCreate(&graph, 0));
            gn_status st = capture(c, graph);
            if (st == GN_OK && hipGraphInstantiate(&ws.chunks[c], graph, nullptr, nullptr, 0) != hipSuccess) {
                ws.chunks[c] = nullptr;
                st = GN_E_HIP;
            }
            (void)hipGraphDestroy(graph);
            if (st != GN_OK) return st;
        }
        // slot c & 1 last held chain c - 2's mark, whose chain has ended
        __atomic_store_n(slots + 4 * (c & 1), 0, __ATOMIC_RELEASE);
        return hipGraphLaunch(ws.chunks[c], stream) == hipSuccess ? GN_OK : GN_E_HIP;
    };
    gn_status rs = launch(c_begin);
    int32_t launched = c_begin;
    for (int32_t c = c_begin; rs == GN_OK; ++c) {
        volatile int32_t* s = slots + 4 * (c & 1);
        if ((rs = wait_mark(s, c + 1, stream)) != GN_OK) break;
        if (s[1] >= 0 || s[2] != 0 || c + 1 >= nchunks) break;
        if (hooks && hooks->stop_after && hooks->stop_after(c)) break;
        if ((rs = launch(c + 1)) == GN_OK) launched = c + 1;
    }
    if (last) *last = launched;
    if (rs != GN_OK) return rs;
    if (sync_end) GN_HIP_TRY(hipStreamSynchronize(stream));
    return GN_OK;
}

gn_status gn_internal_chain_solve(gn_graph* g, int32_t nchunks, int32_t c_begin, hipStream_t stream,
                                  bool sync_end) {
    GraphWorkspace& ws = g->ws;
    const int32_t C = g_chunk_len;
    const bool prune = g->prune && (g_prune == 2 || (g_prune == 1 && g->prune_pays));
    const int32_t key = prune ? g_prune_every : 0;
    if (ws.chunk_prune != key) {  // chains captured for other lists or another rebuild interval
        for (auto ex : ws.chunks) if (ex) (void)hipGraphExecDestroy(ex);
        ws.chunks.clear();
        ws.chunk_prune = key;
    }
    if (prune && !gn_internal_rebuilds_at((int64_t)c_begin * C)) {
        // the lists may be stale (another solve's, or none yet): rebuild them
        // from this chain's input state before its first step reads them
        hipLaunchKernelGGL(prune_rebuild_kernel, dim3((unsigned)(((int64_t)g->n * 8 + 255) / 256)), dim3(256), 0,
                           stream, g->n, (const int32_t*)g->row_ptr, (const int32_t*)g->prune_mloc,
                           (const float*)ws.y[((int64_t)c_begin * C) & 1], g->listed, g->prune);
        GN_HIP_TRY(hipGetLastError());
    }
    return gn_internal_run_marked(
        ws, nchunks, C,
        [g, C, prune](int32_t c, int32_t j0, int32_t j1, hipGraph_t graph, hipGraphNode_t* last) {
            return build_steps(g, c, C, prune, j0, j1, graph, last);
        },
        c_begin, stream, sync_end);
}

extern "C" gn_status gn_set_pruning(int32_t mode) {
    if (mode < 0 || mode > 2) return GN_E_ARG;
    g_prune = mode;
    return GN_OK;
}

int32_t g_small_limit = kSmallWorkMax;

extern "C" gn_status gn_set_small_graph_limit(int32_t work_max) {
    if (work_max < 0 || work_max > kSmallWorkMax) return GN_E_ARG;
    g_small_limit = work_max;
    return GN_OK;
}

extern "C" gn_status gn_set_prune_interval(int32_t steps) {
    if (steps < 1 || steps > 4096) return GN_E_ARG;
    g_prune_every = steps;
    return GN_OK;
}

extern "C" gn_status gn_set_chunk_len(int32_t len) {
    if (len < 1 || len > 4096) return GN_E_ARG;
    g_chunk_len = len;
    return GN_OK;
}

extern "C" gn_status gn_solve(gn_graph* g, const gn_schedule* sch, float* x, uint8_t* sel, gn_result* res,
                              hipStream_t stream) {
    if (!g || !sch || !res) return GN_E_ARG;
    if (!gn_internal_schedule_ok(sch)) return GN_E_ARG;
    std::memset(res, 0, sizeof(*res));
    if (g->n == 0) {
        res->binarised = 1;
        res->stab = INFINITY;
        return GN_OK;
    }
    if (!x || !sel) return GN_E_ARG;
    const int32_t ms = sch->max_steps;
    const int32_t C = g_chunk_len;
    const int32_t nchunks = (ms + 1 + C - 1) / C;
    gn_status st = gn_internal_ensure_ws(g, nchunks * C);
    if (st != GN_OK) return st;
    GraphWorkspace& ws = g->ws;
    const int n = g->n;

    if ((st = gn_internal_init_solve(ws, sch, stream)) != GN_OK) return st;
    hipLaunchKernelGGL(prep_state_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, n, (const float*)x, g->perm,
                       g->v, ws.y[0], ws.state);
    GN_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(normalizable_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, n, g->row_ptr, g->col,
                       (const float*)x, g->perm, ws.state);
    GN_HIP_TRY(hipGetLastError());

    // one workgroup (one launch for the whole solve) while a step is small
    if (g->nnz + 2 * (int64_t)n <= g_small_limit && gn_internal_small_fits(g))
        st = gn_internal_small_solve(g, stream);
    else
        st = gn_internal_chain_solve(g, nchunks, 0, stream, false);
    if (st != GN_OK) return st;

    // Epilogue, stream-ordered after the last step: the outcome, the final state
    // and its statistics are decided on the device and come back in one copy.
    SolveTail* tail = (SolveTail*)ws.final_out;
    hipLaunchKernelGGL(pick_final_kernel, dim3(1), dim3(64), 0, stream, (const SolveState*)ws.state,
                       (const int32_t*)ws.notconv, ms, (const float*)ws.gamma, (const float*)ws.y[0],
                       (const float*)ws.y[1], tail);
    GN_HIP_TRY(hipGetLastError());
    if ((st = gn_internal_final_stats_picked(g, &tail->pick, x, sel, &tail->stats, stream)) != GN_OK) return st;
    GN_HIP_TRY(hipMemcpyAsync(ws.host_pinned, tail, sizeof(SolveTail), hipMemcpyDeviceToHost, stream));
    GN_HIP_TRY(hipStreamSynchronize(stream));
    SolveTail h;
    std::memcpy(&h, ws.host_pinned, sizeof(h));
    if (h.state.err & 1) return GN_E_ARG;
    if (h.state.err & 2) return GN_E_NOT_NORMALIZABLE;
    return fill_result(h.state, h.pick.steps, h.pick.binarised != 0, h.stats, res);
}
