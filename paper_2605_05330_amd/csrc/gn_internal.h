// Internal definitions shared by the libgn translation units (host + device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <vector>

#include "libgn.h"

#include "gn_types.h"

#define GN_HIP_TRY(expr)                                  \
    do {                                                  \
        hipError_t _e = (expr);                           \
        if (_e != hipSuccess) return GN_E_HIP;            \
    } while (0)

struct GraphWorkspace {
    int32_t cap_steps = 0;     // capacity of notconv / gamma tables (entries)
    float* y[2] = {nullptr, nullptr};
    SolveState* state = nullptr;
    int32_t* notconv = nullptr;
    float* gamma = nullptr;
    uint8_t* sel_int = nullptr;
    void* partials = nullptr;  // per-block reduction partials
    int64_t partials_cap = 0;
    void* final_out = nullptr; // reduced statistics (device)
    void* host_pinned = nullptr;  // pinned staging for SolveState / statistics
    std::vector<hipGraphExec_t> chunks;  // captured step chains, chunk c covers steps [c*C, (c+1)*C)
    int32_t chunk_len = 0;
    int32_t chunk_prune = -1;            // captured chains' lists: 0 full, else the pruned lists' rebuild interval
    hipEvent_t chain_ev[2] = {nullptr, nullptr};  // completion events of the chains in flight (created on first use)
    void destroy_chains() {
        for (auto ex : chunks) if (ex) (void)hipGraphExecDestroy(ex);
        chunks.clear();
        for (auto& e : chain_ev) {
            if (e) (void)hipEventDestroy(e);
            e = nullptr;
        }
    }
};

struct gn_graph {
    int32_t n = 0;
    int64_t nnz = 0;
    int32_t max_degree = 0;
    int device = 0;
    int32_t* row_ptr = nullptr;   // internal order
    int32_t* col = nullptr;       // internal labels, per-row order of the caller's CSR
    float* v = nullptr;           // internal order
    float* w_int = nullptr;       // internal order
    float* w_user = nullptr;      // user order
    int32_t* perm = nullptr;      // internal -> user
    int32_t* iperm = nullptr;     // user -> internal
    int32_t* sl_col = nullptr;    // sliced columns of the group bins
    int32_t* sl_off = nullptr;    // [slices + 1] line offsets
    // Pruned neighbour lists of the chained solve (gn_step.hip): the sliced
    // lines, then the CSR columns, with the id of every vertex that is not
    // listed replaced by -1.  Null when the graph has none (no symmetric,
    // sorted structure to find the mirror entries, or too many entries).
    int32_t* prune = nullptr;       // [prune_sl_words + nnz]
    int64_t prune_sl_words = 0;     // words of the sliced part
    int32_t* prune_mloc = nullptr;  // [nnz]: where entry (i -> j) of row i sits in row j's list, as i
    uint8_t* listed = nullptr;      // [n]: vertex present (not -1) in its neighbours' pruned lists
    int32_t* prune_mirror = nullptr;  // [nnz]: CSR index of each entry's mirror (the multi-start lists)
    bool prune_pays = false;        // the gathers have little locality (gn_set_pruning mode 1)
    BinLayout bins{};
    int32_t bin_count_rows[BIN_COUNT] = {0};
    mutable GraphWorkspace ws;   // work buffers; calls on one handle must not overlap
    mutable void* unrolled = nullptr;  // adjoint work buffers (gn_unrolled.hip)
    mutable void* multi = nullptr;     // multi-start work buffers (gn_multi.hip)
    void* small = nullptr;             // LDS image of the single-workgroup solve (gn_small.hip)
};

// Final statistics reduced on the device (fixed-order, deterministic).
struct FinalStats {
    double relaxed_objective;
    double set_objective;
    long long set_size;
    long long conflicts;
    long long uncovered;
    float stab;
    int32_t pad;
};

// A solve's outcome, decided on the device after its last step (gn_solve): the
// step count, whether the state binarised, the final state words and the gamma
// of the final step; `skip` is set when the solve failed its input checks, and
// then the final-state kernels write nothing.
struct FinalPick {
    const float* y;
    float gamma;
    int32_t steps;
    int32_t binarised;
    int32_t skip;
};

// The block gn_solve's epilogue fills on the device and the host reads back in
// one copy (the workspace's final_out; the statistics come first, where the
// other callers of final_out read them).
struct SolveTail {
    FinalStats stats;
    FinalPick pick;
    SolveState state;
};

// Validation of clique (hyperedge) constraints given on the host: clique k is
// members[ptr[k] .. ptr[k+1]-1], non-empty, ids strictly increasing in [0, n);
// every vertex in some clique; w finite and > 0.  cover receives each vertex's
// clique count.  GN_E_ARG / GN_E_CSR / GN_E_WEIGHT as the clique entry points
// document.  (gn_lp.hip)
gn_status gn_internal_check_cliques(int32_t n, int32_t m, const int32_t* ptr, const int32_t* members,
                                    const float* w, std::vector<int32_t>& cover);

// Device allocation of count elements (at least one); false and a cleared HIP
// error on failure.
template <typename T>
inline bool gn_dalloc(T** p, size_t count) {
    if (count == 0) count = 1;
    if (hipMalloc((void**)p, count * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return false;
    }
    return true;
}

// internal helpers implemented in gn_graph.hip / gn_step.hip / gn_check.hip
gn_status gn_internal_ensure_ws(gn_graph* g, int32_t steps_needed);
gn_status gn_internal_launch_step(const gn_graph* g, const StepArgs& a, hipStream_t s);
gn_status gn_internal_final_stats(gn_graph* g, const float* y_fin, float gamma_fin, float* x_user,
                                  uint8_t* sel_user, FinalStats* host_out, hipStream_t s);
// same, reduced into device memory without a host round trip (stream-ordered:
// consecutive calls may share the graph's work buffers)
gn_status gn_internal_final_stats_launch(gn_graph* g, const float* y_fin, float gamma_fin, float* x_user,
                                         uint8_t* sel_user, FinalStats* dev_out, hipStream_t s);
gn_status gn_internal_sel_stats(const gn_graph* g, const uint8_t* sel_user, FinalStats* host_out,
                                hipStream_t s);
// same, for the final state and gamma that `pick` (device memory) names; writes
// nothing when pick->skip is set
gn_status gn_internal_final_stats_picked(gn_graph* g, const FinalPick* pick, float* x_user, uint8_t* sel_user,
                                         FinalStats* dev_out, hipStream_t s);
int32_t gn_internal_grid_blocks(const BinLayout& b);
// gn_step's argument checks, and its work (x_in -> state words in y_words, n
// floats; one step launch writing x_out) on a caller-chosen word buffer
// (gn_solve.hip)
gn_status gn_internal_step_args_ok(const gn_graph* g, float gamma, const float* x_in, float* x_out);
gn_status gn_internal_step_with(const gn_graph* g, float gamma, const float* x_in, float* x_out, float* y_words,
                                hipStream_t stream);

// solve driver pieces shared by the graph and the assignment (rook) solvers
// (gn_step.hip): schedule check, gamma table and state reset, the pipelined
// replay of captured step chains, the stopping outcome and the result record
extern int32_t g_chunk_len;
extern int32_t g_prune;  // pruned lists in chained solves: 0 never, 1 where they pay, 2 always (gn_set_pruning)
extern int32_t g_prune_every;  // steps between rebuilds of the pruned lists (gn_set_prune_interval)
// Whether the captured chains rebuild the pruned lists before step k: at every
// multiple of the rebuild interval, step 0 included, wherever it falls in a chain.
inline bool gn_internal_rebuilds_at(int64_t k) { return k % g_prune_every == 0; }
float gn_internal_host_gamma(const gn_schedule* s, int32_t k);
bool gn_internal_schedule_ok(const gn_schedule* sch);
gn_status gn_internal_init_solve(GraphWorkspace& ws, const gn_schedule* sch, hipStream_t stream);
// Optional hooks of gn_internal_run_marked: when pin_src is set, each chain's
// progress mark also copies pin_words words from pin_src to the pinned block at
// byte offset pin_offset + 4 pin_words (c & 1) for chain c; stop_after(c) is
// asked once chain c's mark shows the solve still running, and returns true to
// launch no further chain.
struct ChunkHooks {
    const void* pin_src = nullptr;
    int32_t pin_words = 0;
    size_t pin_offset = 0;
    std::function<bool(int32_t)> stop_after;
};
// Steps [c C + j0, c C + j1) of chain c, added to `graph` after *last (null for
// none), which is updated to the last node added.
using StepRangeBuilder =
    std::function<gn_status(int32_t c, int32_t j0, int32_t j1, hipGraph_t graph, hipGraphNode_t* last)>;
// Replays chains of C steps from c_begin with a progress mark 8 steps before
// each chain's end (the solve state's done step and error word, stored to
// pinned memory): chain c + 1 is launched when chain c's mark shows the solve
// still running, none once it shows a stop or an error, so a solve that stops
// before a mark launches no further chain.  With sync_end the call returns once
// the chains have completed; *last receives the last chain launched.
gn_status gn_internal_run_marked(GraphWorkspace& ws, int32_t nchunks, int32_t C, const StepRangeBuilder& build,
                                 int32_t c_begin, hipStream_t stream, bool sync_end = true,
                                 const ChunkHooks* hooks = nullptr, int32_t* last = nullptr);
// The chained single-start solve of g from chain c_begin on: ws.y[(c_begin C) & 1]
// holds the state at step c_begin C (C = g_chunk_len), and the solve state and
// flags are set up (gn_solve.hip).
gn_status gn_internal_chain_solve(gn_graph* g, int32_t nchunks, int32_t c_begin, hipStream_t stream,
                                  bool sync_end = true);
// multi-start solves hand their last running start to the single-start chains (gn_set_multi_handoff)
extern int32_t g_multi_handoff;
gn_status gn_internal_solve_outcome(const GraphWorkspace& ws, int32_t ms, int32_t* steps, bool* binarised);
gn_status gn_internal_fill_result(const GraphWorkspace& ws, int32_t steps, bool binarised, const FinalStats& fs,
                                  gn_result* res);
gn_status gn_internal_ensure_tables(GraphWorkspace& ws, int32_t steps_needed);

// small graphs: the whole solve in one workgroup (gn_small.hip) while
// nnz + 2 n <= g_small_limit (gn_set_small_graph_limit, gn_solve.hip) and the
// graph's LDS image fits one compute unit
extern int32_t g_small_limit;
constexpr int32_t kSmallWorkMax = 1 << 20;
gn_status gn_internal_small_solve(const gn_graph* g, hipStream_t s);
bool gn_internal_small_fits(const gn_graph* g);  // the graph has an LDS image that fits one CU
// builds that image at graph creation from the host copies of the internal CSR
// (synchronises `s`); on any failure the graph has none and takes the chained path
void gn_internal_build_small(gn_graph* g, const int32_t* rp, const int32_t* col, hipStream_t s);
void gn_internal_free_small(gn_graph* g);
void gn_internal_free_unrolled(gn_graph* g);
void gn_internal_free_multi(gn_graph* g);
