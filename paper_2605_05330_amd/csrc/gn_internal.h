// Internal definitions shared by the libgn translation units (host + device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <vector>

#include "libgn.h"

// ---------------------------------------------------------------------------
// Degree bins.  Rows are relabelled at graph creation so that each bin is a
// contiguous range of internal row ids, heaviest bin first:
//   BIN_BLOCK   deg >  512   one workgroup per row, neighbour values staged in LDS
//   BIN_WAVE    deg <= 512   one wavefront per row, two rows in flight per wavefront
//   BIN_G8      deg <= 128   8 threads per row (8 rows per wavefront)
//   BIN_LANE32  deg <= 32    2 threads per row
//   BIN_LANE16  deg <= 16    one thread per row
// Launch order inside one step kernel follows the enum.  Every bin evaluates
// the same canonical neighbour-sum order (gn_rowsum.h).
//
// Sliced column layout of the group bins (G8, LANE32, LANE16).  A wavefront
// handles 64/G consecutive rows (a slice); lane l = G*r + t serves thread t of
// row r.  The slice stores its columns position-major: position q holds, in
// lane l, entry t + G*q of row r, or -1 past the row's end, so every column load
// of the wavefront reads 64 consecutive words and needs no row_ptr lookup.
// Rows inside these bins are ordered by decreasing degree within windows of
// kSortWindow rows, which keeps the padding small.
// ---------------------------------------------------------------------------
enum GnBin { BIN_BLOCK = 0, BIN_WAVE = 1, BIN_G8 = 2, BIN_LANE32 = 3, BIN_LANE16 = 4, BIN_COUNT = 5 };

constexpr int kBlock = 256;              // threads per workgroup (4 wavefronts of 64)
constexpr int kWaves = kBlock / 64;
constexpr int kWaveMaxDeg = 512;         // rows above this degree get a whole workgroup
constexpr int kStage = 4096;             // LDS staging chunk for BIN_BLOCK rows (floats)
constexpr int kSortWindow = 2048;        // degree-sort window of the sliced bins (rows)

__host__ __device__ constexpr int bin_rows_per_block(int b) {
    return b == BIN_BLOCK ? 1 : b == BIN_WAVE ? 2 * kWaves : b == BIN_G8 ? 8 * kWaves
         : b == BIN_LANE32 ? kBlock / 2 : kBlock;
}

__host__ __device__ constexpr int bin_max_degree(int b) {
    return b == BIN_BLOCK ? 0x7fffffff : b == BIN_WAVE ? kWaveMaxDeg : b == BIN_G8 ? 128 : b == BIN_LANE32 ? 32 : 16;
}

// Threads per row of a sliced bin (0: the bin keeps plain CSR access).
__host__ __device__ constexpr int bin_group(int b) {
    return b == BIN_G8 ? 8 : b == BIN_LANE32 ? 2 : b == BIN_LANE16 ? 1 : 0;
}

struct BinLayout {
    int32_t row_begin[BIN_COUNT + 1];    // internal rows of bin b: [row_begin[b], row_begin[b+1])
    int32_t blk_begin[BIN_COUNT + 1];    // blocks of bin b: [blk_begin[b], blk_begin[b+1])
    int32_t slice_begin[BIN_COUNT + 1];  // slices of bin b: [slice_begin[b], slice_begin[b+1])
};

// Device-resident state of one solve.  The step kernels read everything that
// varies between solves from here, so a captured chain of step launches only
// depends on the step indices and the buffers.
struct SolveState {
    int32_t done_step;       // -1 until some step's input state passes the stopping test
    int32_t err;             // 1: x0 negative / non-finite, 2: x0 not normalizable
    int32_t max_steps;
    int32_t check_every;
    float tau;
    int32_t pad;
    unsigned long long fallback;  // safe-division resets over all steps
};

// Arguments of the fused WRGN step kernel (passed by value).
struct StepArgs {
    const int32_t* row_ptr;  // internal CSR
    const int32_t* col;
    const float* v;          // sqrt(w), internal order
    const float* y_in;       // signed weighted state: |y| = v x, sign bit = (x > 1/2)
    float* y_out;
    const float* gamma;      // device gamma table indexed by step (solve mode)
    float gamma_scalar;      // used when gamma == nullptr
    int32_t k;               // step index (solve mode)
    int32_t solve;           // 1: solve mode (reads SolveState, may skip / test)
    SolveState* st;
    int32_t* notconv;        // [max_steps+1] per-step "state failed the test" flags
    float* x_out_user;       // optional: x' in user order (single-step mode)
    float* s_out;            // optional: closed sums s_i (internal order), for the adjoint
    const int32_t* perm;     // internal -> user vertex id
    const int32_t* sl_col;   // sliced columns of the group bins (64-word lines)
    const int32_t* sl_off;   // first line of each slice; slice s spans lines [sl_off[s], sl_off[s+1])
    BinLayout bins;
};

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
    BinLayout bins{};
    int32_t bin_count_rows[BIN_COUNT] = {0};
    mutable GraphWorkspace ws;   // work buffers; calls on one handle must not overlap
    mutable void* unrolled = nullptr;  // adjoint work buffers (gn_unrolled.hip)
    mutable void* multi = nullptr;     // multi-start work buffers (gn_multi.hip)
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

// internal helpers implemented in gn_graph.hip / gn_step.hip / gn_check.hip
gn_status gn_internal_ensure_ws(gn_graph* g, int32_t steps_needed);
gn_status gn_internal_launch_step(const gn_graph* g, const StepArgs& a, hipStream_t s);
gn_status gn_internal_final_stats(gn_graph* g, const float* y_fin, float gamma_fin, float* x_user,
                                  uint8_t* sel_user, FinalStats* host_out, hipStream_t s);
gn_status gn_internal_sel_stats(const gn_graph* g, const uint8_t* sel_user, FinalStats* host_out,
                                hipStream_t s);
int32_t gn_internal_grid_blocks(const BinLayout& b);

// solve driver pieces shared by the graph and the assignment (rook) solvers
// (gn_step.hip): schedule check, gamma table and state reset, the pipelined
// replay of captured step chains, the stopping outcome and the result record
extern int32_t g_chunk_len;
float gn_internal_host_gamma(const gn_schedule* s, int32_t k);
bool gn_internal_schedule_ok(const gn_schedule* sch);
gn_status gn_internal_init_solve(GraphWorkspace& ws, const gn_schedule* sch, hipStream_t stream);
gn_status gn_internal_run_chunks(GraphWorkspace& ws, int32_t nchunks, int32_t C,
                                 const std::function<gn_status(int32_t, hipGraphExec_t*)>& build,
                                 hipStream_t stream);
gn_status gn_internal_solve_outcome(const GraphWorkspace& ws, int32_t ms, int32_t* steps, bool* binarised);
gn_status gn_internal_fill_result(const GraphWorkspace& ws, int32_t steps, bool binarised, const FinalStats& fs,
                                  gn_result* res);
gn_status gn_internal_ensure_tables(GraphWorkspace& ws, int32_t steps_needed);
void gn_internal_free_unrolled(gn_graph* g);
void gn_internal_free_multi(gn_graph* g);
