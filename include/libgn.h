/*
 * libgn -- Weighted Regularized Graph Normalization (WRGN) for Maximum Weight
 * Independent Set on AMD Instinct MI355X (gfx950).
 *
 * Problem (Section 2 and the WRGN definition): G = (A, w) is a simple
 * undirected graph on n vertices (A symmetric, A_ii = 0) with strictly positive
 * vertex weights w.  With v = sqrt(w) and a regularization gamma > 0, one WRGN
 * step maps a state x in [0,1]^n to
 *
 *     x'_i = x_i / (x_i + gamma * sum_{j in N(i)} (v_j / v_i) x_j),
 *
 * computed in weighted state space y = v (.) x as x'_i = y_i / s_i with
 * s = (I + gamma A) y, and with the safe division of the paper's PyTorch module
 * (code appendix): x'_i = 1/2 wherever s_i <= 1e-9.  Iterated with gamma > 1 it
 * converges to the indicator of a gamma-stable maximal independent set
 * (Theorem "Binary Regularization").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All vertex-indexed arrays passed to or returned from the library are in the
 *    caller's vertex order ("user order"), length n, contiguous.
 *  - "device" pointers are HIP device memory of the current device owned by the
 *    caller; the library never frees them.  "host" pointers are ordinary host
 *    memory.
 *  - Every call returns a gn_status.  Negative values are errors; nothing is
 *    thrown and nothing aborts.  Argument and input-validation errors are
 *    detected on the host before any work is queued.  A fault inside a kernel
 *    surfaces as GN_E_HIP at the next call that synchronises.
 *  - Calls marked ASYNC only enqueue work on `stream`; calls marked SYNC wait for
 *    `stream` before returning because they fill host outputs.
 *  - A handle's device work buffers are shared by all calls on that handle:
 *    calls on one handle must not overlap in time (on one stream they never do).
 *  - Floating-point state is fp32; reductions of objectives use fp64.
 *  - Support invariance (Section 2, property ii): a positive coordinate never
 *    becomes zero.  Internally every solver carries a coordinate whose weighted
 *    value v_i x_i falls below 2^-100 as log2 x_i in fixed point (resolution
 *    2^-17), so it keeps its own magnitude far below fp32's range, down to
 *    2^-1022 (fp64's smallest normal number), where it is held.  States handed
 *    back to the caller are fp32 x; such coordinates read as their fp32
 *    rounding (0 below 2^-149).
 */
#ifndef LIBGN_H
#define LIBGN_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gn_graph gn_graph; /* one graph: CSR, weights, degree bins, work buffers */
typedef struct gn_batch gn_batch; /* many independent graphs solved in one launch        */
typedef struct gn_rook gn_rook;   /* assignment instance: rows x cols weight matrix       */

typedef enum {
    GN_OK = 0,
    GN_NOT_CONVERGED = 1,        /* outputs written, stopping test not met by max_steps  */
    GN_E_ARG = -1,               /* bad argument (null pointer, negative size, NaN, ...)  */
    GN_E_CSR = -2,               /* row_ptr not monotone / bad bounds, column out of range,
                                    columns of a row not strictly increasing             */
    GN_E_SELF_LOOP = -3,         /* A_ii != 0                                             */
    GN_E_ASYMMETRIC = -4,        /* A != A^T                                              */
    GN_E_WEIGHT = -5,            /* some w_i not finite or not > 0                        */
    GN_E_NOT_NORMALIZABLE = -6,  /* x0 has a closed neighbourhood of zero mass            */
    GN_E_NUMERIC = -7,           /* non-finite value produced                             */
    GN_E_HIP = -8,               /* a HIP runtime call failed                             */
    GN_E_NOMEM = -9,             /* device or host allocation failed                      */
    GN_E_SIZE = -10              /* input larger than a fixed-capacity entry point allows */
} gn_status;

/* flags of gn_graph_create / gn_batch_create */
#define GN_INPUT_HOST   0u  /* row_ptr, col_idx, w are host pointers                      */
#define GN_INPUT_DEVICE 1u  /* row_ptr, col_idx, w are device pointers                    */
#define GN_NO_VALIDATE  2u  /* skip the O(nnz) symmetry / ordering checks (trusted input) */

/* Iteration schedule (Section 6, gamma-pursuit): gamma_k = p*gamma1 + (1-p)*gamma0
 * with p = min(k, ramp_steps-1)/(ramp_steps-1); ramp_steps <= 1 means constant
 * gamma1.  The paper runs 1000 steps with gamma 0.9 -> 1.5 (ramp_steps = 1000).
 * Stopping rule of this library (the paper has none): at steps k >= 1 with
 * k % check_every == 0, and at k = max_steps, the state x^k passes when
 *   (1) max_i min(x_i, 1 - x_i) <= tau,
 *   (2) every vertex with x_i <= 1/2 has a neighbour with x_j > 1/2, and
 *   (3) every vertex with 0 < x_i <= 1/2 satisfies s_i > v_i under gamma_k, i.e.
 *       the next step shrinks it (the finite-state form of stab > 1).        */
typedef struct {
    float gamma0, gamma1;
    int32_t ramp_steps;
    int32_t max_steps;
    float tau;
    int32_t check_every;
} gn_schedule;

/* Result of a solve.  The selected set is S = {i : x_i > 1/2}. */
typedef struct {
    int32_t steps;              /* WRGN steps applied                                   */
    int32_t binarised;          /* 1 when the stopping test passed                      */
    int64_t fallback_count;     /* 1/2-resets taken by the safe division, all steps     */
    double relaxed_objective;   /* sum_i w_i x_i   (fp64)                               */
    double set_objective;       /* W(S) = sum_{i in S} w_i   (fp64)                     */
    int64_t set_size;           /* |S|                                                  */
    int64_t conflicts;          /* undirected edges with both ends in S                 */
    int64_t uncovered;          /* vertices outside S with no neighbour in S            */
    float stab;                 /* gamma_k * min_{i not in S} sum_{j in N(i) cap S}
                                   sqrt(w_j / w_i)  (stability equation of Theorem
                                   "Binary Regularization"), gamma_k of the final step;
                                   +inf when S = V                                      */
} gn_result;

/* Number of degree bins a graph is split into (see gn_graph_info). */
#define GN_NUM_BINS 7

/* Create a graph from CSR + weights.  n >= 0 vertices, nnz = row_ptr[n] stored
 * entries (2|E|).  row_ptr: int32[n+1], col_idx: int32[nnz], w: float[n], all
 * host or all device per `flags`.  The CSR must be symmetric with no diagonal
 * entries and strictly increasing columns in every row; w must be finite and
 * > 0 (Section 2).  The library copies everything into memory it owns, so the
 * caller may free its arrays on return.  Precomputes v = sqrt(w) (fp32, rounded
 * from the double square root) and the degree bins.  SYNC.
 * Errors: GN_E_ARG, GN_E_CSR, GN_E_SELF_LOOP, GN_E_ASYMMETRIC, GN_E_WEIGHT,
 * GN_E_NOMEM, GN_E_HIP.  On error *out is set to NULL. */
gn_status gn_graph_create(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                          const float* w, uint32_t flags, hipStream_t stream, gn_graph** out);

/* Free a graph and everything it owns (NULL is allowed).  Waits for the device. */
void gn_graph_destroy(gn_graph* g);

/* Diagnostics: n, nnz, max degree and the number of rows in each degree bin
 * (bin_rows may be NULL; else GN_NUM_BINS entries, lightest first: one thread
 * per row (deg <= 16), 2 threads per row (deg <= 32), 8 threads per row
 * (deg <= 128), one wavefront per row (deg <= 512), one workgroup per row with
 * LDS staging (deg > 512), then unused zeros).  Host only. */
gn_status gn_graph_info(const gn_graph* g, int32_t* n, int64_t* nnz, int32_t* max_degree,
                        int32_t* bin_rows);

/* One WRGN step (definition above, with the safe division) at a given gamma:
 * x_out = N(x_in).  x_in, x_out: device float[n], user order; they must not
 * alias (GN_E_ARG).  x_in must be finite and >= 0; vertices whose closed
 * neighbourhood sum is <= 1e-9 take x = 1/2.  ASYNC. */
gn_status gn_step(const gn_graph* g, float gamma, const float* x_in, float* x_out, hipStream_t stream);

/* gn_step for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * step, bit for bit, but its work buffer (the n state words gn_step keeps in
 * the graph's workspace) is a static device array of gn_step_static_max_n()
 * words that each GPU holds until the process ends; the call allocates nothing
 * and frees nothing.  The graph must have been created on the current device
 * (GN_E_ARG otherwise); n above the capacity gives GN_E_SIZE.  All calls on one
 * GPU share its array: calls that overlap in time on one GPU (several streams
 * or threads) race on it and must be serialised by the caller.  ASYNC. */
gn_status gn_step_static(const gn_graph* g, float gamma, const float* x_in, float* x_out, hipStream_t stream);
int32_t gn_step_static_max_n(void);

/* Iterate WRGN from x to binarisation under `sch`.  x: device float[n], x^0 on
 * entry and the final state on exit (clamped to [0,1]); sel: device uint8[n],
 * sel_i = (x_i > 1/2); res: host.  x^0 must be finite, >= 0 and normalizable
 * ((A+I) x^0 > 0 componentwise, Section 2), else GN_E_ARG / GN_E_NOT_NORMALIZABLE
 * and x, sel are left unchanged.  Returns GN_OK when binarised, GN_NOT_CONVERGED
 * when max_steps ran out (outputs still valid).  SYNC. */
gn_status gn_solve(gn_graph* g, const gn_schedule* sch, float* x, uint8_t* sel, gn_result* res,
                   hipStream_t stream);

/* Relaxed MWIS objective sum_i w_i x_i (Theorem "Weighted Mass Growth"), fp64
 * accumulation in a fixed order.  x: device float[n]; out: host.  SYNC. */
gn_status gn_objective(const gn_graph* g, const float* x, double* out, hipStream_t stream);

/* Independence and maximality of a vertex set (Section 2): conflicts = number
 * of undirected edges with both ends selected (1_S^T A 1_S / 2), uncovered =
 * number of unselected vertices with no selected neighbour.  sel: device
 * uint8[n], nonzero = selected.  conflicts: host, required; uncovered: host,
 * may be NULL.  SYNC. */
gn_status gn_check_independent(const gn_graph* g, const uint8_t* sel, int64_t* conflicts,
                               int64_t* uncovered, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Batched solve: many independent graphs in one persistent launch.
 *
 * Connected components do not interact (Section 2, property iii), so a batch
 * is solved graph by graph: every graph keeps its own step counter, its own
 * gamma_k and its own stopping test, and each graph's result is bit-identical
 * to gn_solve on that graph alone (same arithmetic in the same order).
 * ------------------------------------------------------------------------- */

/* Launch shape of the batched kernel, chosen by gn_batch_autotune.  It changes
 * speed only, never results. */
typedef struct {
    int32_t block_threads;   /* threads per workgroup: 128, 256, 512 or 1024                 */
    int32_t blocks_per_cu;   /* persistent workgroups per compute unit: 1 .. 4 (1 .. 2 with 1024) */
    int32_t lds_vertices;    /* LDS per workgroup = 12 * lds_vertices bytes, and
                                lds_vertices * 12 * blocks_per_cu <= 158 KiB.  Graphs of at
                                most 65535 vertices have a sliced column layout: S slices
                                (64 rows of degree <= 16, 8 rows of degree <= 64, or one
                                heavier row each) of L lines of 64 16-bit ids in all.  With
                                8 n + 12 + 4 S + 128 L bytes <= that, a graph keeps its
                                state, slice table and lines in LDS; else, with
                                8 n + 12 + 4 S bytes, its state and slice table (the lines
                                stream from global memory); else, or above 65535 vertices,
                                it runs from global memory in a launch of its own          */
    int32_t light_max_deg;   /* bin schedule: rows of degree <= light_max_deg run a lane each,
                                64 per slice: 8 or 16 (0 = 16)                              */
    int32_t mid_max_deg;     /* rows of degree <= mid_max_deg (and above light_max_deg) run
                                8 lanes each, 8 per slice: 32, 64 or 128 (0 = 64); heavier
                                rows a wavefront each.  The bounds set how each graph's rows
                                are relabelled and sliced (rebuilt when they change, a host
                                step that synchronises the stream); every row keeps its
                                canonical sum order, so results do not depend on them      */
    int32_t reserved;
} gn_tuning;

/* Create a batch.  count >= 1 graphs; n[g], nnz[g] host arrays; row_ptr_cat:
 * the graphs' own row_ptr arrays (each starting at 0) back to back, sum(n[g]+1)
 * int32; col_idx_cat: the graphs' column arrays back to back, local vertex ids,
 * sum(nnz[g]) int32; w_cat: weights back to back, sum(n[g]) float.  The three
 * concatenated arrays are host or device per `flags`.  Each graph must satisfy
 * the conditions of gn_graph_create.  Copies everything.  SYNC.
 * Errors as gn_graph_create. */
gn_status gn_batch_create(int32_t count, const int32_t* n, const int64_t* nnz, const int32_t* row_ptr_cat,
                          const int32_t* col_idx_cat, const float* w_cat, uint32_t flags, hipStream_t stream,
                          gn_batch** out);

/* Free a batch (NULL is allowed).  Waits for the device. */
void gn_batch_destroy(gn_batch* b);

/* Solve every graph of the batch to binarisation under one schedule.  x_cat:
 * device float[sum n], x^0 on entry (user order within each graph), final
 * states on exit; sel_cat: device uint8[sum n]; res: host gn_result[count].
 * tuning may be NULL (then the cached or default shape is used).  The solve's
 * launches are kept as one HIP graph in the handle and replayed while the
 * tuning, schedule and buffers are unchanged.  If any
 * graph's x^0 is negative, non-finite or not normalizable the call returns
 * GN_E_ARG / GN_E_NOT_NORMALIZABLE and leaves x_cat, sel_cat unchanged.
 * Returns GN_OK when every graph binarised, GN_NOT_CONVERGED otherwise.  SYNC. */
gn_status gn_batch_solve(gn_batch* b, const gn_schedule* sch, const gn_tuning* tuning, float* x_cat,
                         uint8_t* sel_cat, gn_result* res, hipStream_t stream);

/* Autotuner of the batched solve: times candidate tunings on this batch (per
 * candidate a warm-up run of at most 64 steps, then one full solve under
 * `sch`, from x0 = 1/2) and returns the fastest.  It searches the launch shapes
 * (block_threads x blocks_per_cu) at the default bin bounds, then the bin
 * schedule (light_max_deg in {8, 16} x mid_max_deg in {32, 64, 128}) at the best
 * shape, then the shapes again at the best bounds.  The choice is kept in the
 * handle (used by later gn_batch_solve calls with tuning == NULL, the layout
 * left in its bounds) and in a process-wide cache keyed by the batch's bucket:
 * graph count, total vertices and entries (powers of two), the degree
 * histogram (fractions of rows of degree <= 8, 16, 32, 64, 128 and above, in
 * steps of 1/32) and max_steps (power of two).  A batch whose bucket is cached
 * takes that tuning without timing anything.  SYNC. */
gn_status gn_batch_autotune(gn_batch* b, const gn_schedule* sch, gn_tuning* out, hipStream_t stream);

/* Entries of the autotuner's process-wide cache, and clearing it (host only). */
int32_t gn_batch_tuning_cache_size(void);
void gn_batch_tuning_cache_clear(void);

/* The batch as one block-diagonal graph (vertex ids offset graph by graph),
 * owned by the batch: valid until gn_batch_destroy.  Used by the unrolled
 * (differentiable) calls and by single-graph diagnostics. */
const gn_graph* gn_batch_graph(const gn_batch* b);

/* ---------------------------------------------------------------------------
 * Differentiable GN: T unrolled WRGN steps and their adjoint (reverse mode).
 *
 * The paper presents GN as a differentiable layer (abstract, Introduction,
 * Conclusion); these calls provide its exact gradient.  For one step
 * x' = y (/) s with y = v (.) x, s = (I + gamma A) y and an incoming gradient
 * gbar = dL/dx', the chain rule gives t = gbar (.) y (/) s^2,
 * dL/dy = gbar (/) s - (I + gamma A) t, dL/dx = v (.) dL/dy,
 * dL/dv += x (.) dL/dy, and dL/dw = dL/dv (/) (2 v).  Rows that took the 1/2
 * safe-division reset pass no gradient; rows carried in log form enter y and x
 * at their fp32 value.
 * ------------------------------------------------------------------------- */

/* Floats of checkpoint storage needed for T steps checkpointed every
 * ckpt_every steps: ceil(T / ckpt_every) states of n floats (n when T = 0).
 * ckpt_every = 1 keeps instead y and the closed sums s of every step,
 * 2 T n floats, and the backward then recomputes nothing.  Returns -1 on bad
 * arguments. */
int64_t gn_unrolled_ckpt_floats(const gn_graph* g, int32_t T, int32_t ckpt_every);

/* Run T steps x^{k+1} = N_{gamma_k}(x^k) (no stopping test) from x0.
 * w: device float[n] weights to use instead of the graph's own (for learning
 * w), or NULL.  gammas: host float[T].  x0, xT: device float[n], user order, not
 * aliased.  ckpt: device float[gn_unrolled_ckpt_floats(...)], written here and
 * read by gn_unrolled_backward (layout private to the library).  x0 must be
 * finite and >= 0.  ASYNC. */
gn_status gn_unrolled_forward(const gn_graph* g, const float* w, const float* gammas, int32_t T,
                              int32_t ckpt_every, const float* x0, float* xT, float* ckpt, hipStream_t stream);

/* Gradient of <gxT, x^T> through the T steps of the matching forward call (same
 * g, w, gammas, T, ckpt_every and its ckpt): gw = dL/dw through the dynamics
 * (a direct dependence of L on w, e.g. L = w . x^T, is the caller's to add),
 * gx0 = dL/dx0.  gxT, gw, gx0: device float[n], user order.  Segments of
 * ckpt_every steps are recomputed from the checkpoints (no recompute when
 * ckpt_every = 1).  The result does not depend on ckpt_every.  ASYNC. */
gn_status gn_unrolled_backward(const gn_graph* g, const float* w, const float* gammas, int32_t T,
                               int32_t ckpt_every, const float* ckpt, const float* gxT, float* gw, float* gx0,
                               hipStream_t stream);

/* The same unrolled steps for every graph of a batch, one workgroup per graph
 * with its state in LDS: one launch per call instead of one per step.  xT,
 * gw and gx0 are bit-identical to gn_unrolled_forward / gn_unrolled_backward
 * with ckpt_every = 1 on gn_batch_graph(b) (same arithmetic, same canonical
 * sums).  w_cat (weights to use instead of the batch's own, or NULL), x0_cat,
 * xT_cat, gxT_cat, gw_cat, gx0_cat: device float[total vertices], the graphs'
 * user orders back to back (the layout of gn_batch_solve's x_cat); x0_cat and
 * xT_cat not aliased.  gammas: host float[T], finite and >= 0.  store: device
 * float[gn_batch_unrolled_store_floats(b, T)] (y and s of every step, layout
 * private to the library), written by the forward call and read by the
 * backward call with the same b, w_cat, gammas and T.  Every graph must have
 * at most 65535 vertices and an adjoint state that fits one compute unit's LDS
 * (16 n + 12 + 4 S bytes <= about 158 KB for S slices of its sliced layout,
 * see gn_tuning), else GN_E_ARG.  T = 0 copies x0 to xT (forward) and gxT to
 * gx0 with gw = 0 (backward).  ASYNC, except that a call whose gammas differ
 * from the previous call's synchronises `stream` to upload them.  Calls on one
 * batch must not overlap. */
int64_t gn_batch_unrolled_store_floats(const gn_batch* b, int32_t T);
gn_status gn_batch_unrolled_forward(gn_batch* b, const float* w_cat, const float* gammas, int32_t T,
                                    const float* x0_cat, float* xT_cat, float* store, hipStream_t stream);
gn_status gn_batch_unrolled_backward(gn_batch* b, const float* w_cat, const float* gammas, int32_t T,
                                     const float* store, const float* gxT_cat, float* gw_cat, float* gx0_cat,
                                     hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Learned warm start.
 *
 * The paper warm-starts GN from fractional solutions of an LP solver (Section 6,
 * "Randomized start and warm start"); here a small message-passing network,
 * trained on GN's own results, predicts x0 instead.  Definition (hidden width
 * 64): features h0_i = [w_i, deg_i/10, w_i / max_{N[i]} w, S_i/(w_i + S_i)] with
 * S_i = sum_{N(i)} w;  h1 = ReLU([h0 | mean_{N(i)} h0 | 0_8] W1 + b1);
 * h2 = ReLU([bf16(h1) | bf16(mean_{N(i)} bf16(h1))] W2 + b2);  z = h2 . u + c;
 * p = sigmoid(z);  x0 = clamp(p, 1e-3, 1) where |p - 1/2| > gate, else 1/2 (the
 * neutral start of GN keeps every vertex the network is not sure about; gate = 0
 * gives the plain clamped prediction).  Matrix products run on the matrix cores with
 * bfloat16 operands and fp32 accumulation.  Loss: mean binary cross-entropy of
 * sigmoid(z) against 0/1 labels.
 *
 * Parameters: one fp32 vector of GN_MPNN_NPARAMS floats (device), laid out as
 * W1 [16][64] (rows 0-3 self weights, 4-7 neighbour weights, 8-15 unused),
 * b1 [64], W2 [128][64] (rows 0-63 self, 64-127 neighbour), b2 [64], u [64], c.
 * ------------------------------------------------------------------------- */
#define GN_MPNN_NPARAMS 9409

/* Bytes of the device cache used by gn_mpnn_forward / gn_mpnn_backward for a
 * graph of n vertices (activations and reduction partials); -1 if n < 0. */
int64_t gn_mpnn_cache_bytes(int32_t n);

/* Forward pass on graph g (its own weights): x0 (device float[n], user order)
 * receives the warm start, z (device float[n] or NULL) the logits.  params:
 * device fp32[GN_MPNN_NPARAMS]; gate in [0, 1/2).  cache: device buffer of
 * gn_mpnn_cache_bytes(n) bytes, caller-owned, keeps the activations for the
 * backward pass.  ASYNC. */
gn_status gn_mpnn_forward(const gn_graph* g, const float* params, float gate, float* x0, float* z, void* cache,
                          hipStream_t stream);

/* Backward pass after gn_mpnn_forward with the same g, params and cache:
 * labels (device float[n], user order, values in [0,1]) define the loss; grad
 * (device fp32[GN_MPNN_NPARAMS]) receives dLoss/dparams, loss (device float[1])
 * the loss.  Sums over vertices are reduced in a fixed order.  n must be > 0.
 * ASYNC. */
gn_status gn_mpnn_backward(const gn_graph* g, const float* params, const float* labels, void* cache, float* grad,
                           float* loss, hipStream_t stream);

/* One Adam step (Kingma and Ba) on count parameters: m, v updated in place, t
 * counts steps from 1.  All pointers device fp32.  ASYNC. */
gn_status gn_adam_step(float* params, const float* grad, float* m, float* v, int32_t count, float lr, float beta1,
                       float beta2, float eps, int32_t t, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Multi-start: several starting points of one graph iterated together (the
 * batched starts of the paper's PyTorch module, code appendix; the experiments of
 * Section 6 run 16 random starts per instance and keep the best).
 * ------------------------------------------------------------------------- */

#define GN_MAX_STARTS 16

/* Solve `starts` (1..GN_MAX_STARTS) independent GN runs of g at once.  x: device
 * float[starts*n], start-major (start b occupies x[b*n .. b*n+n-1], user order):
 * the starting points on entry, the final states (clamped to [0,1]) on exit; sel:
 * device uint8[starts*n], same layout, (x > 1/2).  res: host gn_result[starts],
 * one per start.  *best (host): the start with the largest set objective among
 * the binarised ones (lowest index on ties; among all starts if none binarised).
 * Every start stops on its own by the stopping rule of gn_solve, and its result
 * is bit-identical to gn_solve from the same starting point (same arithmetic in
 * the same order); the call returns when every start has stopped.  Random
 * starting points are the caller's (the module draws -log U normalised by its
 * maximum and clamped to [1e-3, 1]).  Errors as gn_solve (any start's x0 invalid
 * or not normalizable fails the call).  Returns GN_OK when every start
 * binarised, else GN_NOT_CONVERGED.  SYNC. */
gn_status gn_multi_solve(gn_graph* g, const gn_schedule* sch, int32_t starts, float* x, uint8_t* sel,
                         gn_result* res, int32_t* best, hipStream_t stream);

/* Random starting points of the paper's module (code appendix): for each start,
 * x = clamp(e / max(e), 1e-3, 1) with e = -log(u), the maximum taken over that
 * start's n values (the module normalises over the whole batch; per start is
 * this library's reading).  u: device float[starts*n] start-major, every value in
 * (0, 1] (GN_E_ARG otherwise); x: device float[starts*n], ready for
 * gn_multi_solve.  e is computed with the device logf.  SYNC. */
gn_status gn_random_starts(gn_graph* g, int32_t starts, const float* u, float* x, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Assignment problem: matrix cross-normalization (Section 2).
 *
 * The graph is the line graph of the complete bipartite graph K_{rows,cols}:
 * vertex (i, j) = i*cols + j carries the weight W_ij, and two entries conflict
 * when they share a row or a column.  GN normalizes every entry by the mass of
 * its row and column, so with R_i, C_j the row and column sums of y = v (.) x
 *     s_ij = y_ij + gamma * ((R_i - y_ij) + (C_j - y_ij)),
 * which costs O(rows*cols) per step; the results are those of gn_step / gn_solve
 * on the same graph up to rounding (sums in another order, row and column sums
 * in fp64).  The MWIS of this graph is a maximum-weight matching; for
 * rows = cols the selected set is a permutation matrix.
 * All matrices are row-major, rows*cols entries, device memory unless stated.
 * ------------------------------------------------------------------------- */

/* Create an assignment instance from a weight matrix w (rows >= 1, cols >= 1,
 * rows*cols <= 2^31-1), host or device per flags (GN_INPUT_HOST /
 * GN_INPUT_DEVICE).  Every W_ij must be finite and > 0.  The library copies w.
 * SYNC.  Errors: GN_E_ARG, GN_E_WEIGHT, GN_E_NOMEM, GN_E_HIP; *out = NULL on
 * error. */
gn_status gn_rook_create(int32_t rows, int32_t cols, const float* w, uint32_t flags, hipStream_t stream,
                         gn_rook** out);

/* Free an assignment instance (NULL is allowed).  Waits for the device. */
void gn_rook_destroy(gn_rook* r);

/* One cross-normalization step at gamma: x_out = N(x_in), with the safe
 * division of gn_step.  x_in, x_out: device float[rows*cols], must not alias;
 * x_in finite and >= 0.  ASYNC. */
gn_status gn_rook_step(gn_rook* r, float gamma, const float* x_in, float* x_out, hipStream_t stream);

/* Iterate to binarisation under `sch`, with the stopping rule of gn_solve.
 * x: device float[rows*cols], x^0 on entry, final state (clamped to [0,1]) on
 * exit; sel: device uint8[rows*cols], (x > 1/2); res: host.  conflicts counts
 * pairs of selected entries sharing a row or a column, uncovered the unselected
 * entries whose row and column hold no selected entry, stab is the
 * gamma-stability of the set under gamma_k.  x^0 must be finite, >= 0 and
 * normalizable (no zero entry whose row and column are all zero), else GN_E_ARG /
 * GN_E_NOT_NORMALIZABLE.  Returns GN_OK when binarised, GN_NOT_CONVERGED when
 * max_steps ran out.  SYNC. */
gn_status gn_rook_solve(gn_rook* r, const gn_schedule* sch, float* x, uint8_t* sel, gn_result* res,
                        hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Census of GN atoms (Appendix A, Table atoms_10).
 *
 * An atom is a fixed point of GN with full support on a connected graph: with
 * B = A + I, a solution x > 0 of B x = 1.  A connected graph is atomic when it
 * has one; its atomic spectrum is discrete when det B != 0 (the single point
 * B^-1 1) and continuous otherwise; it is regular when all degrees are equal.
 * ------------------------------------------------------------------------- */

typedef struct {
    int64_t connected;             /* connected graphs on n vertices, up to isomorphism */
    int64_t irregular_discrete;    /* atomic graphs by class, up to isomorphism         */
    int64_t irregular_continuous;
    int64_t regular_discrete;
    int64_t regular_continuous;
    int64_t atomic;                /* the four classes together                         */
    int64_t labelled_evaluated;    /* labelled graphs the kernel classified             */
} gn_atom_counts;

/* Count the connected graphs on n vertices (1 <= n <= 10) and their atomic
 * classes, up to isomorphism.  By Burnside's lemma over the cycle types of the
 * vertex permutations, each labelled graph fixed by a representative
 * permutation is classified on the device, one thread each, exactly
 * (fraction-free elimination of [B | 1], whose entries stay below 2^24, after
 * an exact filter: a graph in which one closed neighbourhood strictly contains
 * another has no atom).  The identity's term is summed in a two-level
 * marked-vertex form (a vertex of maximum degree relabelled 0, then one of
 * largest degree among its neighbours relabelled 1, each with its
 * neighbourhood fixed and the graph weighted by the number of such choices):
 * about 2.5e10 graphs at n = 10 instead of 2^45.  n = 9 takes under a tenth of
 * a second, n = 10 about 11 s.  The sums are divided by n! on the host.  Allocates and
 * frees its own device buffers.  Errors: GN_E_ARG (n out of range, out NULL),
 * GN_E_NOMEM, GN_E_HIP, GN_E_NUMERIC (a weighted sum not divisible by n!: an
 * internal inconsistency, never expected).  SYNC. */
gn_status gn_atom_census(int32_t n, gn_atom_counts* out, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Fractional warm start (Section 6, "Randomized start and warm start"): the
 * MWIS LP relaxation over clique constraints,
 *     LP* = max c.x  s.t.  sum_{i in C} x_i <= 1 for every clique C,  x >= 0,
 * smoothed by entropy at a temperature T and solved by a Bregman-Sinkhorn scheme
 * alone (no rounding).  With multipliers lam_C >= 0 and Lam_i the sum of those
 * of the cliques holding i, the smoothed primal is x_i = exp((c_i - Lam_i)/T);
 * updating clique C sets lam_C' = max(0, lam_C + T log sum_{i in C} x_i) and
 * adds lam_C' - lam_C to its members' Lam (exact minimisation of the smoothed
 * dual in lam_C).  Cliques are coloured first-fit in input order into classes
 * of vertex-disjoint cliques; a pass updates the classes in the start's order,
 * the cliques of a class in parallel.  Pass p runs at
 * T_p = max(t_min, t0 * drop^p).  Diversity across starts: the class order (the
 * randomized clique order) and t0 (the jittered initial temperature) are the
 * caller's, per start.
 * ------------------------------------------------------------------------- */

typedef struct gn_lp gn_lp;   /* clique-constrained LP instance and its work buffers */

typedef struct {
    int32_t passes;       /* passes run                                                  */
    int32_t converged;    /* 1 when gap <= gap_tol at a check                            */
    float temperature;    /* temperature of the last pass                                */
    float pad;
    double dual;          /* D = sum_C lam_C + sum_i max(0, c_i - Lam_i), an upper bound  */
    double primal;        /* P = c.xf of the feasible point returned                     */
    double gap;           /* (D - P) / D                                                 */
} gn_lp_result;

/* Create an LP instance.  Host arrays: clique k is members[clique_ptr[k] ..
 * clique_ptr[k+1]-1] (m >= 1 cliques, each non-empty with strictly increasing
 * vertex ids in [0, n)); cost: float[n], finite and > 0 (the vertex weights);
 * every vertex must lie in some clique (a singleton clique is allowed), else the
 * LP is unbounded.  The library copies everything and colours the cliques.
 * Errors: GN_E_ARG (null, sizes, an uncovered vertex), GN_E_CSR (clique_ptr not
 * starting at 0 or not increasing, ids out of range or not increasing),
 * GN_E_WEIGHT, GN_E_NOMEM, GN_E_HIP; *out = NULL on error.  SYNC. */
gn_status gn_lp_create(int32_t n, int32_t m, const int32_t* clique_ptr, const int32_t* members, const float* cost,
                       hipStream_t stream, gn_lp** out);

/* Free an LP instance (NULL is allowed).  Waits for the device. */
void gn_lp_destroy(gn_lp* lp);

/* Number of clique classes (the length of each start's order), of cliques, and
 * the size of the largest class.  Any output may be NULL. */
gn_status gn_lp_info(const gn_lp* lp, int32_t* n_classes, int32_t* n_cliques, int32_t* max_class);

/* How the passes run (testing and tuning control; results are the same bits
 * either way).  Fused (enable = 1, the default): one workgroup per start keeps
 * Lam and lam in LDS and runs every pass up to the next check in one launch,
 * the classes separated by workgroup barriers; available when the instance's
 * 4 (n + m + 2 n_classes + 1) bytes fit one CU's LDS (158 KiB).  Otherwise, or
 * with enable = 0: one launch per class for all starts, the multipliers in
 * global memory.  Returns 1 when solves will run fused, 0 when not, -1 for a
 * NULL handle.  Not thread-safe against a concurrent solve on the handle. */
int32_t gn_lp_set_fused(gn_lp* lp, int32_t enable);

/* Run `starts` (1..GN_MAX_STARTS) independent solves.  t0: host float[starts],
 * finite and > 0; order: host int32[starts * n_classes], row s a permutation of
 * the classes; drop in (0, 1]; t_min > 0; max_passes >= 1; check_every >= 1;
 * gap_tol >= 0; x_floor in [0, 1); anneal_tol finite; stall >= 1.  Lam and lam
 * start at zero.
 * Checks: after pass p with (p + 1) % check_every == 0, and after the last
 * pass, each running start takes at the pass's temperature the feasible point
 * xf_i = x_i / max(1, max_{C holds i} sum_{j in C} x_j) (x's exponent capped at
 * 60), raises it by two rounds of a fair-share lift (each clique's slack split
 * equally among its members, each member taking the smallest share of its
 * cliques), and evaluates P = c.xl and the bound D = sum lam_C +
 * sum_i max(0, c_i - sum_{C holds i} lam_C) (the multipliers' sums rebuilt in
 * fp64).  It keeps D_best = min D, P_best = max P and the point of P_best, and
 * stops when (D_best - P_best) / D_best <= gap_tol.
 * Temperatures: anneal_tol <= 0 gives T_p = max(t_min, t0 drop^p) every pass;
 * anneal_tol > 0 holds T between checks and lowers it by drop^check_every (not
 * below t_min) after a check whose smoothed primal exceeds no clique by more
 * than anneal_tol, or after `stall` checks in which P_best gained less than a
 * relative 5e-5.
 * x: device float[starts * n], start-major (user vertex ids), receives
 * max(x_best, x_floor): a starting point for gn_multi_solve on the conflict graph
 * (an edge between two vertices sharing a clique).  res: host
 * gn_lp_result[starts] (dual = D_best, primal = P_best, temperature of the last
 * check).  fp32 state, fp64 sums of D and P.  Returns GN_OK when every start met
 * gap_tol, else GN_NOT_CONVERGED; GN_E_ARG on bad arguments, GN_E_NUMERIC if D or
 * P is not finite.  SYNC. */
gn_status gn_lp_solve(gn_lp* lp, int32_t starts, const float* t0, const int32_t* order, float drop, float t_min,
                      int32_t max_passes, int32_t check_every, float gap_tol, float x_floor, float anneal_tol,
                      int32_t stall, float* x, gn_lp_result* res, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * GN under hyperedge constraints (the extension to hypergraph constraints left
 * to future work in the Conclusion; no formula in the paper, so this is the
 * library's reading).  Hyperedges are clique constraints (at most one selected
 * vertex each, the form of the paper's instances) and every vertex is
 * normalised by the mass of the hyperedges holding it, as the cross-
 * normalization of the assignment problem (Section 2) does with rows and
 * columns.  With y = v (.) x and Y_e = sum_{j in e} y_j:
 *     s_i = y_i + gamma * sum_{e holds i} (Y_e - y_i),   x'_i = y_i / s_i,
 * with the safe division and log-form small states of gn_step.  This is gn_step on the
 * conflict graph whose edge (i, j) counts the hyperedges holding both; it costs
 * O(memberships) per step instead of O(conflict edges), and equals gn_step on
 * the plain conflict graph when no two vertices share two hyperedges (rows and
 * columns of an assignment instance, for instance).
 * ------------------------------------------------------------------------- */

typedef struct gn_hyper gn_hyper;  /* hyperedges, weights, work buffers */

/* Create an instance.  Host arrays: hyperedge e is members[edge_ptr[e] ..
 * edge_ptr[e+1]-1] (m >= 1, each non-empty with strictly increasing ids in
 * [0, n)); every vertex must lie in some hyperedge (a singleton is allowed);
 * w: float[n], finite and > 0.  The library copies everything.  Errors:
 * GN_E_ARG, GN_E_CSR, GN_E_WEIGHT (as gn_lp_create), GN_E_NOMEM, GN_E_HIP;
 * *out = NULL on error.  SYNC. */
gn_status gn_hyper_create(int32_t n, int32_t m, const int32_t* edge_ptr, const int32_t* members, const float* w,
                          hipStream_t stream, gn_hyper** out);

/* Free an instance (NULL is allowed).  Waits for the device. */
void gn_hyper_destroy(gn_hyper* h);

/* One step at gamma (finite, >= 0): x_out = N(x_in), device float[n] each, not
 * aliased, x_in finite and >= 0.  ASYNC. */
gn_status gn_hyper_step(gn_hyper* h, float gamma, const float* x_in, float* x_out, hipStream_t stream);

/* Iterate to binarisation under `sch` with the stopping rule of gn_solve, read
 * on the hyperedge-weighted conflict graph: a vertex is covered when one of its
 * hyperedges holds a member above 1/2.  x: device float[n], x^0 on entry (finite,
 * >= 0, every vertex with mass in its hyperedges, else GN_E_ARG /
 * GN_E_NOT_NORMALIZABLE), the final state clamped to [0,1] on exit; sel: device
 * uint8[n], (x > 1/2); res: host.  In res, conflicts counts pairs of selected
 * vertices per hyperedge holding both, uncovered the unselected vertices whose
 * hyperedges hold no selected vertex, and stab is gamma_k * min over unselected
 * i of sum_{e holds i} sum_{j in e, selected} v_j / v_i (+inf when every
 * vertex is selected).  Returns GN_OK when binarised, GN_NOT_CONVERGED when
 * max_steps ran out.  The steps replay as captured chains of launches
 * (gn_set_chunk_len), which the handle keeps for the last schedule and start
 * count it ran; calls on one handle must not overlap.  SYNC. */
gn_status gn_hyper_solve(gn_hyper* h, const gn_schedule* sch, float* x, uint8_t* sel, gn_result* res,
                         hipStream_t stream);

/* gn_hyper_solve for `starts` (1..GN_MAX_STARTS) starting points at once, one
 * launch per step pass for all of them (the batched starts of the paper's
 * experiments, Section 6).  x: device float[starts*n], start-major, the
 * starting points on entry and the final states on exit; sel: device
 * uint8[starts*n]; res: host gn_result[starts].  Every start stops on its own
 * and its result is that of gn_hyper_solve from the same point (the same
 * arithmetic in the same order).  *best (host, may be NULL): the start with the
 * largest set objective among the binarised ones (lowest index on ties; among
 * all starts if none binarised).  Errors as gn_hyper_solve; any invalid start
 * fails the call.  Returns GN_OK when every start binarised, else
 * GN_NOT_CONVERGED.  SYNC. */
gn_status gn_hyper_multi_solve(gn_hyper* h, const gn_schedule* sch, int32_t starts, float* x, uint8_t* sel,
                               gn_result* res, int32_t* best, hipStream_t stream);

/* Tuning: number of step launches captured in one replayed chain by gn_solve,
 * gn_multi_solve, gn_rook_solve and the hyperedge solves (default 64,
 * 1..4096).  The next chain is
 * launched when a progress mark 8 steps before a chain's end shows the solve
 * still running; the calling thread waits for each mark by spinning on pinned
 * host memory.  A longer chain costs fewer transitions between
 * chains; once the solve has stopped, the launches left in the chains in
 * flight return at once, so a shorter chain wastes fewer of them.  Results do
 * not change.  Process-wide; not thread-safe. */
gn_status gn_set_chunk_len(int32_t len);

/* Tuning: steps between rebuilds of the pruned neighbour lists
 * (gn_set_pruning) in gn_solve and gn_multi_solve (default 64, 1..4096).  The
 * lists are rebuilt before every step whose index is a multiple of this
 * interval (step 0 included), wherever it falls in a chain of step launches.
 * Fewer rebuilds cost less upkeep and leave more decayed vertices listed
 * (gathered, adding nothing).  Results do not change.  GN_E_ARG outside
 * 1..4096.  Process-wide; not thread-safe. */
gn_status gn_set_prune_interval(int32_t steps);

/* Tuning: gn_solve runs a graph with nnz + 2 n <= work_max (0 .. 1048576, the
 * default) in one workgroup and one launch when the graph has an LDS image that
 * fits one compute unit: at most 65535 vertices, and y (ping-pong) plus the
 * sliced 16-bit column lines of its internal order (8 n + 12 + 4 S + 128 L
 * bytes for S slices of L lines in all) within about 158 KB.  The image is
 * built at graph creation.  The steps are separated by workgroup barriers
 * instead of kernel boundaries.  Other graphs replay chains of step launches.
 * Both paths compute the same bits; 0 disables the one-workgroup path.
 * Process-wide; not thread-safe. */
gn_status gn_set_small_graph_limit(int32_t work_max);

/* Tuning: pruned neighbour lists in the chained solve of gn_solve.  A
 * neighbour sum adds only ordinary states (y >= 2^-100; the log form and exact
 * zeros add nothing), so the step launches may read a copy of the graph's
 * column lists in which the entries of vertices that are not ordinary -- most
 * of the graph once the non-selected vertices have decayed -- are marked
 * absent and not gathered.  Vertices that stopped being ordinary are dropped
 * at rebuilds every few steps (gn_set_prune_interval); a vertex
 * whose state becomes ordinary again is put back into its neighbours' lists by
 * the step that produces that state, before any step reads it.  mode 0: never;
 * 1 (the default): on graphs whose gathers have little cache-line locality in
 * the internal order (most gathers touch a line of their own), where skipping
 * them pays, and for gn_multi_solve (whose lists drop a vertex only when none
 * of its starts is ordinary) only when its 64 n bytes of states outgrow 4 MB;
 * 2: on every graph.  The lists are built at graph creation (the
 * mirror position of every entry; graphs created with GN_NO_VALIDATE whose
 * structure is not symmetric with sorted rows have none).  Results are the
 * same bits in every mode.  GN_E_ARG for another mode.  Process-wide; not
 * thread-safe. */
gn_status gn_set_pruning(int32_t mode);

/* Tuning knob of gn_multi_solve (GN multi-start above).  A 16-start step costs
 * about as much with one start still running as with sixteen.  With the
 * hand-off enabled (1, the default), once a chain's progress mark shows a
 * single start of a call with two or more still running and another chain of
 * step launches to come, its state moves at the end of that chain to the
 * chained single-start solve of
 * gn_solve (same arithmetic in the same order: the same words, tests, steps,
 * fallback count and results as without it).  0 keeps every start in the
 * 16-start steps.  GN_E_ARG for another value.  Process-wide; not thread-safe. */
gn_status gn_set_multi_handoff(int32_t enable);

/* Human-readable name of a status code (static string). */
const char* gn_status_str(gn_status s);

#ifdef __cplusplus
}
#endif

#endif /* LIBGN_H */
