// Internal types of the batched solve (gn_batch.hip) and the batched unrolled
// calls (gn_batch_unrolled.hip): the per-graph descriptor and the batch handle.
#pragma once

#include <vector>

#include "gn_internal.h"

struct BatchDesc {
    int32_t n;        // vertices
    int32_t n_light;  // internal rows [0, n_light) have degree <= the light bound of the layout
    int32_t n_mid;    // rows [n_light, n_mid) have degree <= its mid bound, rows [n_mid, n) more
    int32_t n_lines;  // lines of the sliced layout (0 without one)
    int64_t v_off;    // offset of the graph's vertices in the vertex arrays
    int64_t rp_off;   // offset of its row_ptr (n + 1 entries)
    int64_t e_off;    // offset of its columns
    int64_t ln_off;   // first line of its sliced layout
    int64_t so_off;   // offset of its slice table: first line of each slice (relative to ln_off), slices + 1 entries
    int32_t nnz;      // CSR entries
    int32_t pad1;
};

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
    size_t lines_cap = 0, slices_cap = 0;  // their allocated entries
    int32_t lay_light = 0, lay_mid = 0;    // degree bounds of the current layout
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

