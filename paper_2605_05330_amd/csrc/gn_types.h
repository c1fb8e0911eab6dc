// Types and constants of the step kernels' interface: degree bins, the solve
// state and the step arguments (host + device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

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
constexpr int kSwizzle = 128;            // block groups of the sliced bins' block-to-rows map

// Block-to-rows map of a sliced bin.  Workgroups are handed to the XCDs round
// robin (workgroup j to XCD j mod 8) and, inside an XCD, to its compute units in
// turn, so workgroups j and j + kSwizzle tend to share an XCD and a group of
// compute units.  Physical block j of a bin of nb blocks therefore works on
// logical block c (S - 1) + min(c, R) + s, with c = j mod kSwizzle,
// s = j / kSwizzle, S = ceil(nb / kSwizzle) and R = nb - kSwizzle (S - 1): the
// blocks of one residue class take consecutive row ranges, and with the rows in
// locality order their neighbour gathers share cache lines.  A bijection on
// [0, nb); which block computes a row never changes the row's result.
__host__ __device__ inline int swizzle_block(int j, int nb) {
    if (nb <= kSwizzle) return j;
    const int S = (nb + kSwizzle - 1) / kSwizzle;
    const int R = nb - kSwizzle * (S - 1);
    const int c = j % kSwizzle, s = j / kSwizzle;
    return c * (S - 1) + (c < R ? c : R) + s;
}

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
    // pruned lists (solve mode): col and sl_col then point into pbuf, whose
    // entries of unlisted vertices are -1; the rows that change listing rewrite
    // their mirror entries
    int32_t prune;
    int32_t* pbuf;
    const int32_t* mloc;     // [nnz] location of each entry's mirror in pbuf
    uint8_t* listed;         // [n]
};
