// Structured GN for the assignment problem (matrix cross-normalization,
// Section 2).  The graph is the line graph of the complete bipartite graph
// K_{rows,cols}: vertex (i, j) = i*cols + j, adjacent to every other entry of row
// i and of column j.  Its closed-neighbourhood sum is
//     s_ij = |y_ij| + gamma * ((R_i - |y_ij|) + (C_j - |y_ij|)),
// R_i and C_j the row and column sums of |y|, so one step costs O(rows*cols)
// instead of the O(rows*cols*(rows+cols)) of a CSR pass over the same graph.
//
// Tiles of 32 rows x 64 columns (one block of 256 threads; wavefront w holds tile
// rows w, w+4, .., w+28, lane l column l).  Each step
//   1. reduces the row and column sums of the input state from per-tile partial
//      sums (fp64, fixed order; the sign bit of a partial carries "some entry of
//      this segment is in the rounded set") -- inside the step kernel for small
//      instances, else in a reduction kernel launched before it,
//   2. updates its tile (safe division, support bound, sign-carrying state, the
//      stopping-test flags, exactly as the CSR step),
//   3. writes the tile's partial sums of the new state for the next step.
// The subtraction R_i - |y_ij| is done in fp64 so that the dominant entry of a
// row does not lose its neighbours' mass to cancellation.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "gn_ctl.h"
#include "gn_internal.h"
#include "gn_rowsum.h"
#include "gn_stats.h"

namespace {

constexpr int kTR = 32;              // tile rows
constexpr int kTC = 64;              // tile columns (one wavefront)
constexpr int kRPW = kTR / kWaves;   // tile rows per wavefront (a power of two)
constexpr int kRowThreads = kBlock / kTR;  // fused form: threads per row of a tile's row sums
static_assert((kRPW & (kRPW - 1)) == 0 && kRPW <= 32, "rows per wavefront");

struct RookArgs {
    int32_t rows, cols, ntr, ntc;  // tiles: ntr x ntc
    const float* v;                // sqrt(w), row-major
    const float* y_in;             // signed weighted state (sign bit = x > 1/2)
    float* y_out;
    const double* rp_in;           // [rows][ntc] partial row sums of |y_in|
    const double* cp_in;           // [cols][ntr] partial column sums of |y_in|
    double* rp_out;                // partial sums of |y_out|
    double* cp_out;
    double* rsum;                  // [rows] row sums of |y_in| (split form; sign bit = a selected entry)
    double* csum;                  // [cols] column sums
    const float* x0;               // prep: the caller's x (row-major)
    float* x_out;                  // single step: x' (row-major)
    const float* gamma;            // solve: gamma table indexed by step
    float gamma_scalar;            // single step
    int32_t k;
    int32_t solve;
    SolveState* st;
    int32_t* notconv;
};

__device__ __forceinline__ double encode(double sum, bool sel) { return sel ? -sum : sum; }

// Partial sums of the new state over this tile.  Rows: the wavefront's kRPW rows
// are reduced together by a reduce-scatter butterfly over the 64 lanes.  At xor 32
// a lane keeps the upper half of its rows (lane bit 5 set) or the lower half and
// adds its partner's values of those rows; each following stage halves again,
// until one row is left per lane; the remaining xor stages finish that row over a
// group of 64 / kRPW lanes, whose first lane writes it.  The row a lane ends with
// is (lane / (64 / kRPW)) in the wavefront's row order.
// Columns: over the lane's rows in order, then the 4 wavefronts in order.
__device__ __forceinline__ void write_partials(const RookArgs& a, int tr, int tc, int lane, int wave,
                                               const int (&iw)[kRPW], const bool (&ok)[kRPW],
                                               const float (&yn)[kRPW], double (*pc)[kTC], int (*pcs)[kTC]) {
    constexpr int GRP = 64 / kRPW;  // lanes per row after the splitting stages
    double cur[kRPW];
    unsigned selbits = 0u;          // bit m: some entry of row m is selected (uniform)
#pragma unroll
    for (int m = 0; m < kRPW; ++m) {
        cur[m] = ok[m] ? (double)fabsf(yn[m]) : 0.0;
        selbits |= __ballot(ok[m] && gnk::sign_of(yn[m])) != 0ull ? 1u << m : 0u;
    }
    // both pair sums are formed and one is selected: selecting the operand
    // instead would let the compiler turn it into a lane-dependent index into
    // cur[], which it lowers to a compare-and-select per element
#pragma unroll
    for (int h = kRPW / 2, off = 32; h >= 1; h >>= 1, off >>= 1) {
        const bool up = (lane & off) != 0;
#pragma unroll
        for (int i = 0; i < h; ++i) {
            const double lo = cur[i] + __shfl_xor(cur[i], off, 64);
            const double hi = cur[h + i] + __shfl_xor(cur[h + i], off, 64);
            cur[i] = up ? hi : lo;
        }
    }
    double r = cur[0];
#pragma unroll
    for (int off = GRP / 2; off >= 1; off >>= 1) r += __shfl_xor(r, off, 64);
    if ((lane & (GRP - 1)) == 0) {
        // the lane's row, computed rather than looked up (a lane-dependent index
        // into a register array costs a compare-and-select per element)
        const int m = lane / GRP;
        const int i = tr * kTR + wave + kWaves * m;
        if (i < a.rows) a.rp_out[(size_t)i * a.ntc + tc] = encode(r, ((selbits >> m) & 1u) != 0u);
    }
    double cacc = 0.0;
    int csel = 0;
#pragma unroll
    for (int m = 0; m < kRPW; ++m)
        if (ok[m]) {
            cacc += (double)fabsf(yn[m]);
            csel |= (int)gnk::sign_of(yn[m]);
        }
    pc[wave][lane] = cacc;
    pcs[wave][lane] = csel;
    __syncthreads();
    const int j = tc * kTC + threadIdx.x;
    if (threadIdx.x < kTC && j < a.cols) {
        double t = pc[0][threadIdx.x];
        int sl = pcs[0][threadIdx.x];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) {
            t += pc[w][threadIdx.x];
            sl |= pcs[w][threadIdx.x];
        }
        a.cp_out[(size_t)j * a.ntr + tr] = encode(t, sl != 0);
    }
}

// x (caller) -> signed weighted state y and its partial sums.  Flags x < 0 or
// non-finite (err bit 1).
__global__ __launch_bounds__(kBlock) void rook_prep_kernel(RookArgs a) {
    __shared__ double pc[kWaves][kTC];
    __shared__ int pcs[kWaves][kTC];
    const int tr = blockIdx.x / a.ntc, tc = blockIdx.x - tr * a.ntc;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = tc * kTC + lane;
    int iw[kRPW];
    bool ok[kRPW];
    float yn[kRPW];
    bool bad = false;
#pragma unroll
    for (int m = 0; m < kRPW; ++m) {
        iw[m] = tr * kTR + wave + kWaves * m;
        ok[m] = j < a.cols && iw[m] < a.rows;
        yn[m] = 0.0f;
        if (ok[m]) {
            const size_t e = (size_t)iw[m] * a.cols + j;
            float x = a.x0[e];
            if (!(x >= 0.0f) || !isfinite(x)) {
                bad = true;
                x = 0.0f;
            }
            yn[m] = gnk::word_from_x(x, a.v[e]);
            a.y_out[e] = yn[m];
        }
    }
    if (bad && a.st) atomicOr(&a.st->err, 1);
    write_partials(a, tr, tc, lane, wave, iw, ok, yn, pc, pcs);
}

// Split form, first kernel of a step: row and column sums of the input state
// from the tile partials, one wavefront per row (rows first) or column; lane l
// adds partials l, l+64, ... in order, then a butterfly.
__global__ __launch_bounds__(kBlock) void rook_reduce_kernel(RookArgs a) {
    const int lane = threadIdx.x & 63;
    const int wv = blockIdx.x * kWaves + (threadIdx.x >> 6);
    const bool is_row = wv < a.rows;
    const int idx = is_row ? wv : wv - a.rows;
    if (!is_row && idx >= a.cols) return;  // whole wavefront past the end (no barrier below)
    const int cnt = is_row ? a.ntc : a.ntr;
    const double* src = is_row ? a.rp_in + (size_t)idx * a.ntc : a.cp_in + (size_t)idx * a.ntr;
    StepCtl<RookArgs> c;
    double acc = 0.0;
    int sl = 0;
    int t = lane;
    for (; t + 64 * 3 < cnt; t += 64 * 4) {
        double p[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) p[u] = src[t + 64 * u];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            acc += fabs(p[u]);
            sl |= signbit(p[u]) ? 1 : 0;
        }
    }
    for (; t < cnt; t += 64) {
        const double p = src[t];
        acc += fabs(p);
        sl |= signbit(p) ? 1 : 0;
    }
    c.fetch(a);
    if (!c.proceed(a)) return;
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    const bool any = __ballot(sl != 0) != 0ull;
    if (lane == 0) (is_row ? a.rsum : a.csum)[idx] = encode(acc, any);
}

// One step over a tile.  FUSED: the row and column sums come straight from the
// tile partials (small instances: one launch per step); otherwise from the
// sums of rook_reduce_kernel.
template <bool FUSED>
__global__ __launch_bounds__(kBlock) void rook_step_kernel(RookArgs a) {
    __shared__ double sC[kWaves][kTC];
    __shared__ int sCs[kWaves][kTC];
    __shared__ double sR[kTR][kRowThreads];
    __shared__ int sRs[kTR][kRowThreads];
    __shared__ double fC[kTC];
    __shared__ int fCs[kTC];
    __shared__ double fR[kTR];
    __shared__ int fRs[kTR];
    __shared__ double pc[kWaves][kTC];
    __shared__ int pcs[kWaves][kTC];
    __shared__ int s_viol[kWaves];
    __shared__ int s_fb[kWaves];

    const int tr = blockIdx.x / a.ntc, tc = blockIdx.x - tr * a.ntc;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = tc * kTC + lane;
    int iw[kRPW];
    bool ok[kRPW];
    float yraw[kRPW], vi[kRPW];
    // a tile inside the matrix (uniform over the block) loads and stores
    // without per-entry predicates
    const bool full = (tr + 1) * kTR <= a.rows && (tc + 1) * kTC <= a.cols;
#pragma unroll
    for (int m = 0; m < kRPW; ++m) {
        iw[m] = tr * kTR + wave + kWaves * m;
        ok[m] = j < a.cols && iw[m] < a.rows;
    }
    if (full) {
#pragma unroll
        for (int m = 0; m < kRPW; ++m) {
            const size_t e = (size_t)iw[m] * a.cols + j;
            yraw[m] = a.y_in[e];
            vi[m] = gnk::ld_stream(a.v + e);
        }
    } else {
#pragma unroll
        for (int m = 0; m < kRPW; ++m) {
            yraw[m] = 0.0f;
            vi[m] = 1.0f;
            if (ok[m]) {
                const size_t e = (size_t)iw[m] * a.cols + j;
                yraw[m] = a.y_in[e];
                vi[m] = gnk::ld_stream(a.v + e);
            }
        }
    }
    StepCtl<RookArgs> c;
    if (FUSED) {
        // column sums of this tile's 64 columns: 4 threads per column, each over a
        // contiguous quarter of the tile rows; row sums of its kTR rows:
        // kRowThreads threads per row, each over a contiguous share of the tile
        // columns
        {
            const int cc = threadIdx.x & 63, q = threadIdx.x >> 6;
            const int jj = tc * kTC + cc;
            const int per = (a.ntr + 3) >> 2;
            const int t0 = q * per, t1 = min(a.ntr, t0 + per);
            double acc = 0.0;
            int sl = 0;
            if (jj < a.cols)
                for (int t = t0; t < t1; ++t) {
                    const double p = a.cp_in[(size_t)jj * a.ntr + t];
                    acc += fabs(p);
                    sl |= signbit(p) ? 1 : 0;
                }
            sC[q][cc] = acc;
            sCs[q][cc] = sl;
        }
        {
            const int r = threadIdx.x / kRowThreads, u = threadIdx.x % kRowThreads;
            const int ii = tr * kTR + r;
            const int per = (a.ntc + kRowThreads - 1) / kRowThreads;
            const int t0 = u * per, t1 = min(a.ntc, t0 + per);
            double acc = 0.0;
            int sl = 0;
            if (ii < a.rows)
                for (int t = t0; t < t1; ++t) {
                    const double p = a.rp_in[(size_t)ii * a.ntc + t];
                    acc += fabs(p);
                    sl |= signbit(p) ? 1 : 0;
                }
            sR[r][u] = acc;
            sRs[r][u] = sl;
        }
        c.fetch(a);
        if (!c.proceed(a)) return;  // uniform over the grid
        __syncthreads();
        if (threadIdx.x < kTC) {
            double t = sC[0][threadIdx.x];
            int sl = sCs[0][threadIdx.x];
#pragma unroll
            for (int q = 1; q < kWaves; ++q) {
                t += sC[q][threadIdx.x];
                sl |= sCs[q][threadIdx.x];
            }
            fC[threadIdx.x] = t;
            fCs[threadIdx.x] = sl;
        } else if (threadIdx.x < kTC + kTR) {
            const int r = threadIdx.x - kTC;
            double t = sR[r][0];
            int sl = sRs[r][0];
            for (int u = 1; u < kRowThreads; ++u) {
                t += sR[r][u];
                sl |= sRs[r][u];
            }
            fR[r] = t;
            fRs[r] = sl;
        }
    } else {
        double p = 0.0;
        if (threadIdx.x < kTC) {
            const int jj = tc * kTC + threadIdx.x;
            if (jj < a.cols) p = a.csum[jj];
        } else if (threadIdx.x < kTC + kTR) {
            const int ii = tr * kTR + threadIdx.x - kTC;
            if (ii < a.rows) p = a.rsum[ii];
        }
        c.fetch(a);
        if (!c.proceed(a)) return;  // uniform over the grid
        if (threadIdx.x < kTC) {
            fC[threadIdx.x] = fabs(p);
            fCs[threadIdx.x] = signbit(p) ? 1 : 0;
        } else if (threadIdx.x < kTC + kTR) {
            fR[threadIdx.x - kTC] = fabs(p);
            fRs[threadIdx.x - kTC] = signbit(p) ? 1 : 0;
        }
    }
    __syncthreads();

    // every lane computes all 4 entries (entries outside the matrix hold y = 0,
    // v = 1 and are masked out of stores, flags and partials), so the loop has
    // no divergent branches
    float yn[kRPW], ynew[kRPW], sv[kRPW];
    int viol = 0, fb = 0;
    bool unnormalizable = false;
    const double C = fC[lane];
    const bool csel = fCs[lane] != 0;
#pragma unroll
    for (int m = 0; m < kRPW; ++m) {
        const double R = fR[wave + kWaves * m];
        const float yi = fabsf(yraw[m]);
        const float sigma = (float)((R - (double)yi) + (C - (double)yi));
        const float s = __fmaf_rn(c.g, sigma, yi);
        const bool fallback = !(s > 1e-9f);
        const float y_new = gnk::step_word(yraw[m], vi[m], s);
        yn[m] = ok[m] ? y_new : 0.0f;
        ynew[m] = y_new;
        sv[m] = s;
        fb += (c.do_write && ok[m] && fallback) ? 1 : 0;
        if (c.solve && c.k == 0 && ok[m] && yi == 0.0f && R == 0.0 && C == 0.0) unnormalizable = true;
        const bool in_s = gnk::sign_of(yraw[m]) != 0u;
        const bool nbr_sel = fRs[wave + kWaves * m] != 0 || csel;
        const float tv = c.tau * vi[m];
        const bool far = (yi > tv) && ((vi[m] - yi) > tv);
        const bool uncovered = !in_s && !nbr_sel;
        const bool growing = !in_s && (yi > 0.0f) && !(s > vi[m]);
        viol |= (c.do_test && ok[m] && (far || uncovered || growing)) ? 1 : 0;
    }
    if (c.do_write) {
        // outputs: one uniform test per array, then the entries
        if (a.y_out) {
#pragma unroll
            for (int m = 0; m < kRPW; ++m)
                if (full || ok[m]) a.y_out[(size_t)iw[m] * a.cols + j] = ynew[m];
        }
        if (a.x_out) {
#pragma unroll
            for (int m = 0; m < kRPW; ++m)
                if (full || ok[m]) a.x_out[(size_t)iw[m] * a.cols + j] = gnk::step_x(yraw[m], vi[m], sv[m], ynew[m]);
        }
    }
    if (unnormalizable) atomicOr(&a.st->err, 2);
    if (c.do_write && a.rp_out) write_partials(a, tr, tc, lane, wave, iw, ok, yn, pc, pcs);

    if (a.solve) {
        const bool wv = __ballot(viol != 0) != 0ull;
        // fb is 0..kRPW per lane: one ballot per bit counts it over the wavefront
        int wf = 0;
#pragma unroll
        for (int bit = 1; bit <= kRPW; bit <<= 1) wf += bit * __popcll(__ballot(fb & bit));
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

// ---- final statistics --------------------------------------------------------
// rows: one wavefront per row writes x = clamp(|y|/v, 0, 1) and S = {x > 1/2},
// and records the row's selected count and sum of v over S; the block partial
// carries the objectives, the set size and the row conflicts.
__global__ __launch_bounds__(kBlock) void rook_rows_kernel(int32_t rows, int32_t cols, const float* __restrict__ y,
                                                           const float* __restrict__ v, const float* __restrict__ w,
                                                           float* __restrict__ x_out, uint8_t* __restrict__ sel_out,
                                                           int32_t* __restrict__ rcnt, float* __restrict__ rvs,
                                                           Partial* out) {
    Partial p{0.0, 0.0, 0, 0, 0, INFINITY, 0};
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = blockIdx.x * kWaves + wave;
    if (i < rows) {
        long long cnt = 0;
        float vs = 0.0f;
        double rel = 0.0, setw = 0.0;
        for (int j = lane; j < cols; j += 64) {
            const size_t e = (size_t)i * cols + j;
            float x = gnk::x_of_word(y[e], v[e]);
            x = fminf(fmaxf(x, 0.0f), 1.0f);
            const bool s = x > 0.5f;
            x_out[e] = x;
            sel_out[e] = s ? 1 : 0;
            rel += (double)w[e] * (double)x;
            if (s) {
                cnt += 1;
                vs += v[e];
                setw += (double)w[e];
            }
        }
        rel = wave_sum_d(rel);
        setw = wave_sum_d(setw);
        cnt = wave_sum_ll(cnt);
        for (int off = 32; off >= 1; off >>= 1) vs += __shfl_xor(vs, off, 64);
        if (lane == 0) {
            rcnt[i] = (int32_t)cnt;
            rvs[i] = vs;
            p.relaxed = rel;
            p.set_w = setw;
            p.size = cnt;
            p.conflicts = cnt * (cnt - 1) / 2;
        }
    }
    block_reduce_store(p, out);
}

// columns, first pass: block b covers column group g = b mod ncg (columns 64g ..
// 64g+63, one lane each) and row block y = b / ncg (rows kColRows*y ..
// +kColRows; a 1-D grid, so neither count is bounded by the y grid limit);
// wavefront w takes a contiguous quarter of
// those rows in order, and the 4 wavefronts combine in order.  Per (row block,
// column): the selected count and the sum of v over the selected entries.
constexpr int kColRows = 64;
__global__ __launch_bounds__(kBlock) void rook_cols_part_kernel(int32_t rows, int32_t cols, int32_t ncg,
                                                                const uint8_t* __restrict__ sel,
                                                                const float* __restrict__ v, int32_t* __restrict__ pcnt,
                                                                float* __restrict__ pvs) {
    __shared__ int s_cnt[kWaves][64];
    __shared__ float s_vs[kWaves][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = (int)(blockIdx.x % (unsigned)ncg), y = (int)(blockIdx.x / (unsigned)ncg);
    const int j = g * 64 + lane;
    constexpr int per = kColRows / kWaves;
    const int i0 = y * kColRows + wave * per;
    const int i1 = min(rows, i0 + per);
    int cnt = 0;
    float vs = 0.0f;
    if (j < cols)
        for (int i = i0; i < i1; ++i) {
            const size_t e = (size_t)i * cols + j;
            if (sel[e]) {
                cnt += 1;
                vs += v[e];
            }
        }
    s_cnt[wave][lane] = cnt;
    s_vs[wave][lane] = vs;
    __syncthreads();
    if (wave == 0 && j < cols) {
#pragma unroll
        for (int w = 1; w < kWaves; ++w) {
            cnt += s_cnt[w][lane];
            vs += s_vs[w][lane];
        }
        pcnt[(size_t)y * cols + j] = cnt;
        pvs[(size_t)y * cols + j] = vs;
    }
}

// columns, second pass: one thread per column adds its row blocks in order.
__global__ __launch_bounds__(kBlock) void rook_cols_kernel(int32_t cols, int32_t nrb, const int32_t* __restrict__ pcnt,
                                                           const float* __restrict__ pvs, int32_t* __restrict__ ccnt,
                                                           float* __restrict__ cvs, Partial* out) {
    Partial p{0.0, 0.0, 0, 0, 0, INFINITY, 0};
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j < cols) {
        long long cnt = 0;
        float vs = 0.0f;
        for (int b = 0; b < nrb; ++b) {
            cnt += pcnt[(size_t)b * cols + j];
            vs += pvs[(size_t)b * cols + j];
        }
        ccnt[j] = (int32_t)cnt;
        cvs[j] = vs;
        p.conflicts = cnt * (cnt - 1) / 2;
    }
    block_reduce_store(p, out);
}

// entries outside S: maximality (some selected entry in the row or column) and
// the gamma-stability ratio (sum of v over the selected neighbours) / v.
__global__ __launch_bounds__(kBlock) void rook_cover_kernel(int32_t rows, int32_t cols, const uint8_t* __restrict__ sel,
                                                            const float* __restrict__ v,
                                                            const int32_t* __restrict__ rcnt,
                                                            const float* __restrict__ rvs,
                                                            const int32_t* __restrict__ ccnt,
                                                            const float* __restrict__ cvs, Partial* out) {
    Partial p{0.0, 0.0, 0, 0, 0, INFINITY, 0};
    const int64_t total = (int64_t)rows * cols;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < total; e += (int64_t)gridDim.x * kBlock) {
        if (sel[e]) continue;
        const int i = (int)(e / cols), j = (int)(e - (int64_t)i * cols);
        if (rcnt[i] == 0 && ccnt[j] == 0) p.uncovered += 1;
        p.stab = fminf(p.stab, (rvs[i] + cvs[j]) / v[e]);
    }
    block_reduce_store(p, out);
}

}  // namespace

struct gn_rook {
    int32_t rows = 0, cols = 0, ntr = 0, ntc = 0;
    int device = 0;
    float* w = nullptr;           // row-major weights
    float* v = nullptr;           // sqrt(w)
    double* rpart[2] = {nullptr, nullptr};
    double* cpart[2] = {nullptr, nullptr};
    double* rsum = nullptr;       // split form: row / column sums of the current state
    double* csum = nullptr;
    bool fused = true;            // one launch per step (small instances)
    int32_t* rcnt = nullptr;
    int32_t* ccnt = nullptr;
    float* rvs = nullptr;
    float* cvs = nullptr;
    int32_t* colpart_cnt = nullptr;  // [ceil(rows / kColRows)][cols] per row block
    float* colpart_vs = nullptr;
    Partial* partials = nullptr;
    int32_t npartials = 0;
    GraphWorkspace ws;
};

static void rook_free(gn_rook* r) {
    auto f = [](void* p) { if (p) (void)hipFree(p); };
    f(r->w); f(r->v); f(r->rpart[0]); f(r->rpart[1]); f(r->cpart[0]); f(r->cpart[1]); f(r->rsum); f(r->csum);
    f(r->rcnt); f(r->ccnt); f(r->rvs); f(r->cvs); f(r->colpart_cnt); f(r->colpart_vs); f(r->partials);
    GraphWorkspace& ws = r->ws;
    ws.destroy_chains();
    f(ws.y[0]); f(ws.y[1]); f(ws.state); f(ws.notconv); f(ws.gamma); f(ws.final_out);
    if (ws.host_pinned) (void)hipHostFree(ws.host_pinned);
}

template <typename T>
static bool rook_alloc(T** p, size_t count) {
    *p = nullptr;
    if (hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return false;
    }
    return true;
}

extern "C" void gn_rook_destroy(gn_rook* r) {
    if (!r) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(r->device);
    (void)hipDeviceSynchronize();
    rook_free(r);
    delete r;
    (void)hipSetDevice(cur);
}

extern "C" gn_status gn_rook_create(int32_t rows, int32_t cols, const float* w, uint32_t flags, hipStream_t stream,
                                    gn_rook** out) {
    if (!out) return GN_E_ARG;
    *out = nullptr;
    if (rows < 1 || cols < 1 || (int64_t)rows * cols > INT32_MAX || !w || (flags & ~GN_INPUT_DEVICE)) return GN_E_ARG;
    const size_t n = (size_t)rows * cols;
    std::vector<float> wh(n);
    if (flags & GN_INPUT_DEVICE) {
        GN_HIP_TRY(hipMemcpyAsync(wh.data(), w, sizeof(float) * n, hipMemcpyDeviceToHost, stream));
        GN_HIP_TRY(hipStreamSynchronize(stream));
    } else {
        std::memcpy(wh.data(), w, sizeof(float) * n);
    }
    for (size_t e = 0; e < n; ++e)
        if (!(wh[e] > 0.0f) || !std::isfinite(wh[e])) return GN_E_WEIGHT;
    std::vector<float> vh(n);
    for (size_t e = 0; e < n; ++e) vh[e] = (float)std::sqrt((double)wh[e]);

    gn_rook* r = new (std::nothrow) gn_rook();
    if (!r) return GN_E_NOMEM;
    (void)hipGetDevice(&r->device);
    r->rows = rows;
    r->cols = cols;
    r->ntr = (rows + kTR - 1) / kTR;
    r->ntc = (cols + kTC - 1) / kTC;
    // fused form while the partial sums every tile re-reads stay within 4x the
    // state's own bytes; beyond that a separate reduction per step is cheaper
    const int64_t reread = (int64_t)r->ntr * r->ntc * (kTR * (int64_t)r->ntc + kTC * (int64_t)r->ntr) * 8;
    r->fused = reread <= 16 * (int64_t)n;
    const int32_t nbr = (rows + kWaves - 1) / kWaves, nbc = (cols + kBlock - 1) / kBlock;
    const int32_t nbe = (int32_t)std::min<int64_t>(((int64_t)n + kBlock - 1) / kBlock, 2048);
    r->npartials = nbr + nbc + nbe;
    GraphWorkspace& ws = r->ws;
    bool ok = rook_alloc(&r->w, n) && rook_alloc(&r->v, n) &&
              rook_alloc(&r->rpart[0], (size_t)rows * r->ntc) && rook_alloc(&r->rpart[1], (size_t)rows * r->ntc) &&
              rook_alloc(&r->cpart[0], (size_t)cols * r->ntr) && rook_alloc(&r->cpart[1], (size_t)cols * r->ntr) &&
              rook_alloc(&r->rsum, rows) && rook_alloc(&r->csum, cols) &&
              rook_alloc(&r->rcnt, rows) && rook_alloc(&r->ccnt, cols) && rook_alloc(&r->rvs, rows) &&
              rook_alloc(&r->cvs, cols) && rook_alloc(&r->partials, (size_t)r->npartials) &&
              rook_alloc(&r->colpart_cnt, (size_t)((rows + kColRows - 1) / kColRows) * cols) &&
              rook_alloc(&r->colpart_vs, (size_t)((rows + kColRows - 1) / kColRows) * cols) &&
              rook_alloc(&ws.y[0], n) && rook_alloc(&ws.y[1], n) && rook_alloc(&ws.state, 1) &&
              rook_alloc((FinalStats**)&ws.final_out, 1);
    if (ok && hipHostMalloc(&ws.host_pinned, 4096, hipHostMallocDefault) != hipSuccess) {
        ws.host_pinned = nullptr;
        ok = false;
    }
    if (!ok) {
        rook_free(r);
        delete r;
        return GN_E_NOMEM;
    }
    hipError_t e = hipMemcpyAsync(r->w, wh.data(), sizeof(float) * n, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(r->v, vh.data(), sizeof(float) * n, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        rook_free(r);
        delete r;
        return GN_E_HIP;
    }
    *out = r;
    return GN_OK;
}

static RookArgs rook_args(const gn_rook* r) {
    RookArgs a{};
    a.rows = r->rows;
    a.cols = r->cols;
    a.ntr = r->ntr;
    a.ntc = r->ntc;
    a.v = r->v;
    a.rsum = r->rsum;
    a.csum = r->csum;
    return a;
}

static int32_t rook_blocks(const gn_rook* r) { return r->ntr * r->ntc; }
static int32_t rook_reduce_blocks(const gn_rook* r) { return (r->rows + r->cols + kWaves - 1) / kWaves; }
static void* rook_step_fn(const gn_rook* r) {
    return r->fused ? (void*)rook_step_kernel<true> : (void*)rook_step_kernel<false>;
}

static gn_status rook_prep(gn_rook* r, const float* x, SolveState* st, hipStream_t s) {
    RookArgs a = rook_args(r);
    a.x0 = x;
    a.y_out = r->ws.y[0];
    a.rp_out = r->rpart[0];
    a.cp_out = r->cpart[0];
    a.st = st;
    hipLaunchKernelGGL(rook_prep_kernel, dim3(rook_blocks(r)), dim3(kBlock), 0, s, a);
    GN_HIP_TRY(hipGetLastError());
    return GN_OK;
}

extern "C" gn_status gn_rook_step(gn_rook* r, float gamma, const float* x_in, float* x_out, hipStream_t stream) {
    if (!r || !x_in || !x_out || x_in == x_out) return GN_E_ARG;
    if (!std::isfinite(gamma) || gamma < 0.0f) return GN_E_ARG;
    gn_status st = rook_prep(r, x_in, nullptr, stream);
    if (st != GN_OK) return st;
    RookArgs a = rook_args(r);
    a.y_in = r->ws.y[0];
    a.rp_in = r->rpart[0];
    a.cp_in = r->cpart[0];
    a.x_out = x_out;
    a.gamma_scalar = gamma;
    a.solve = 0;
    if (r->fused) {
        hipLaunchKernelGGL(rook_step_kernel<true>, dim3(rook_blocks(r)), dim3(kBlock), 0, stream, a);
    } else {
        hipLaunchKernelGGL(rook_reduce_kernel, dim3(rook_reduce_blocks(r)), dim3(kBlock), 0, stream, a);
        GN_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(rook_step_kernel<false>, dim3(rook_blocks(r)), dim3(kBlock), 0, stream, a);
    }
    GN_HIP_TRY(hipGetLastError());
    return GN_OK;
}

// Steps [c len + q0, c len + q1) of a captured chain (one or two launches per
// step), added to `graph` after *last, which is updated to the last node.
static gn_status rook_build_steps(gn_rook* r, int32_t c, int32_t len, int32_t q0, int32_t q1, hipGraph_t graph,
                                 hipGraphNode_t* last) {
    GraphWorkspace& ws = r->ws;
    hipGraphNode_t prev = *last;
    for (int32_t q = q0; q < q1; ++q) {
        RookArgs a = rook_args(r);
        a.k = c * len + q;
        a.y_in = ws.y[a.k & 1];
        a.y_out = ws.y[(a.k + 1) & 1];
        a.rp_in = r->rpart[a.k & 1];
        a.cp_in = r->cpart[a.k & 1];
        a.rp_out = r->rpart[(a.k + 1) & 1];
        a.cp_out = r->cpart[(a.k + 1) & 1];
        a.gamma = ws.gamma;
        a.solve = 1;
        a.st = ws.state;
        a.notconv = ws.notconv;
        void* args[] = {&a};
        for (int part = r->fused ? 1 : 0; part < 2; ++part) {
            hipKernelNodeParams p{};
            p.func = part == 0 ? (void*)rook_reduce_kernel : rook_step_fn(r);
            p.gridDim = dim3(part == 0 ? rook_reduce_blocks(r) : rook_blocks(r));
            p.blockDim = dim3(kBlock);
            p.sharedMemBytes = 0;
            p.kernelParams = args;
            p.extra = nullptr;
            hipGraphNode_t node;
            if (hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &p) != hipSuccess) return GN_E_HIP;
            prev = node;
        }
    }
    *last = prev;
    return GN_OK;
}

static gn_status rook_final_stats(gn_rook* r, const float* y, float gamma_fin, float* x, uint8_t* sel,
                                  FinalStats* host_out, hipStream_t s) {
    const int32_t nbr = (r->rows + kWaves - 1) / kWaves, nbc = (r->cols + kBlock - 1) / kBlock;
    const int32_t nbe = r->npartials - nbr - nbc;
    hipLaunchKernelGGL(rook_rows_kernel, dim3(nbr), dim3(kBlock), 0, s, r->rows, r->cols, y, r->v, r->w, x, sel,
                       r->rcnt, r->rvs, r->partials);
    GN_HIP_TRY(hipGetLastError());
    const int32_t nrb = (r->rows + kColRows - 1) / kColRows;
    const int32_t ncg = (r->cols + 63) / 64;
    hipLaunchKernelGGL(rook_cols_part_kernel, dim3((unsigned)((int64_t)ncg * nrb)), dim3(kBlock), 0, s, r->rows,
                       r->cols, ncg, (const uint8_t*)sel, r->v, r->colpart_cnt, r->colpart_vs);
    GN_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(rook_cols_kernel, dim3(nbc), dim3(kBlock), 0, s, r->cols, nrb,
                       (const int32_t*)r->colpart_cnt, (const float*)r->colpart_vs, r->ccnt, r->cvs,
                       r->partials + nbr);
    GN_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(rook_cover_kernel, dim3(nbe), dim3(kBlock), 0, s, r->rows, r->cols, (const uint8_t*)sel, r->v,
                       (const int32_t*)r->rcnt, (const float*)r->rvs, (const int32_t*)r->ccnt, (const float*)r->cvs,
                       r->partials + nbr + nbc);
    GN_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(kBlock), 0, s, r->npartials,
                       (const Partial*)r->partials, gamma_fin, (FinalStats*)r->ws.final_out,
                       (const FinalPick*)nullptr);
    GN_HIP_TRY(hipGetLastError());
    GN_HIP_TRY(hipMemcpyAsync(r->ws.host_pinned, r->ws.final_out, sizeof(FinalStats), hipMemcpyDeviceToHost, s));
    GN_HIP_TRY(hipStreamSynchronize(s));
    std::memcpy(host_out, r->ws.host_pinned, sizeof(FinalStats));
    return GN_OK;
}

extern "C" gn_status gn_rook_solve(gn_rook* r, const gn_schedule* sch, float* x, uint8_t* sel, gn_result* res,
                                   hipStream_t stream) {
    if (!r || !sch || !res || !x || !sel) return GN_E_ARG;
    if (!gn_internal_schedule_ok(sch)) return GN_E_ARG;
    std::memset(res, 0, sizeof(*res));
    const int32_t ms = sch->max_steps;
    const int32_t C = g_chunk_len;
    const int32_t nchunks = (ms + 1 + C - 1) / C;
    GraphWorkspace& ws = r->ws;
    gn_status st = gn_internal_ensure_tables(ws, nchunks * C);
    if (st != GN_OK) return st;
    if ((st = gn_internal_init_solve(ws, sch, stream)) != GN_OK) return st;
    if ((st = rook_prep(r, x, ws.state, stream)) != GN_OK) return st;
    st = gn_internal_run_marked(
        ws, nchunks, C,
        [r, C](int32_t c, int32_t q0, int32_t q1, hipGraph_t graph, hipGraphNode_t* last) {
            return rook_build_steps(r, c, C, q0, q1, graph, last);
        },
        0, stream);
    if (st != GN_OK) return st;
    int32_t steps;
    bool binarised;
    if ((st = gn_internal_solve_outcome(ws, ms, &steps, &binarised)) != GN_OK) return st;
    FinalStats fs{};
    st = rook_final_stats(r, ws.y[steps & 1], gn_internal_host_gamma(sch, steps), x, sel, &fs, stream);
    if (st != GN_OK) return st;
    return gn_internal_fill_result(ws, steps, binarised, fs, res);
}
