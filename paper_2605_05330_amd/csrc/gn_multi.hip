// Multi-start GN: up to 16 starting points of one graph iterated together (the
// batched starts of the paper's PyTorch module, code appendix; 16 starts per
// instance in the experiments of Section 6).
//
// The 16 states are interleaved, Y[i*16 + b] for vertex i (internal order) and
// start b, so the gather of one neighbour reads 64 contiguous bytes that serve
// every start: the column stream and the gathered cache lines of one step are
// shared by all starts.  Each start's neighbour sum follows the canonical order
// of gn_rowsum.h and its update the arithmetic of the single-start step, so every
// start is bit-identical to gn_solve from the same x0.  Each start has its own
// stopping test and stops on its own: once start b passes at step k_b, its lanes
// stop writing and its final state stays in the buffer of step k_b.
//
// A lane handles a quad of starts (16-byte loads; 4 lanes cover a vertex's 64
// bytes).  Rows (internal order):
//   heavy  deg > 128 : one workgroup per row; neighbour values of all starts are
//                      staged through LDS in chunks of 256 entries, thread
//                      (t, q) = (tid / 4, tid % 4) runs chain t
//   mid    deg <= 128: one wavefront per row, 16 threads per quad (4 chains each)
//   light  deg <= 32 : rows of degree <= 16: 16 rows per wavefront, one thread per
//                      (row, quad); degree 17..32: 8 rows per wavefront, two
//                      threads per (row, quad)
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "gn_internal.h"
#include "gn_rowsum.h"

using gnk::sign_of;

namespace {

constexpr int kStarts = 16;
constexpr int kChunk = 256;  // heavy rows: entries staged per round

// Offsets in the 4 KiB pinned staging block of a multi-start solve.
constexpr size_t kPinDone = 64, kPinFb = 128, kPinNc = 256, kPinStats = 512, kPinRun = 3072;
static_assert(kPinStats + kStarts * sizeof(FinalStats) <= kPinRun && kPinRun + 2 * kStarts * 4 <= 4096,
              "pinned staging layout");
static_assert(sizeof(SolveState) <= kPinDone && kPinStats + kStarts * sizeof(FinalStats) <= 4096,
              "pinned staging layout");

struct MultiArgs {
    const int32_t* row_ptr;
    const int32_t* col;
    const float* v;
    const float* y_in;       // [n][16] signed weighted states
    float* y_out;
    const float* gamma;      // gamma table indexed by step
    int32_t k;
    SolveState* st;          // err, max_steps, check_every, tau; done_step >= 0 once every start has stopped
    int32_t* done;           // [16] per-start done step (-1 while running)
    int32_t* notconv;        // [(steps) * 16] per-step, per-start test flags
    unsigned long long* fb;  // [16] fallback counts
    int32_t n, heavy_end, mid_end;   // rows [0, heavy_end) heavy, [heavy_end, mid_end) mid, [mid_end, n) light
    int32_t l16_begin;               // light rows of degree <= 16 start here
    int32_t mid_blk, light_blk;      // first block of the mid and light parts
    int32_t l16_blk;                 // light blocks before the degree <= 16 rows
    // pruned lists: col then points at a copy of the CSR columns in which the
    // entries of vertices with no ordinary state in any start hold -1
    int32_t prune;
    int32_t* pcol;                   // the copy (written on revivals)
    const int32_t* mirror;           // [nnz] CSR index of each entry's mirror
    uint8_t* listed;                 // [n]
};

// Lanes work on quads of starts: lane l handles starts 4q .. 4q+3 with q = l % 4
// and moves them with one 16-byte load, so 4 lanes cover a vertex's 64 bytes.
struct QuadCtl {
    float g = 0.0f, tau = 0.0f;
    bool do_test = false, do_write = false;
    unsigned act = 0u;  // bit j: start 4q + j runs this step
};

// Control of this lane's quad at this launch.  Returns false when no start is
// active (the launch does no work; uniform over the grid).  Block 0 records
// newly stopped starts and, once none is left, the solve's stop.
__device__ __forceinline__ bool quad_ctl(const MultiArgs& a, int q, QuadCtl& c) {
    const SolveState* st = a.st;
    const int err = st->err, ms = st->max_steps, ce = st->check_every;
    const int k = a.k, km = k >= 1 ? k - 1 : 0;
    const int4 done = reinterpret_cast<const int4*>(a.done)[q];
    const int4 nc = reinterpret_cast<const int4*>(a.notconv + (size_t)km * kStarts)[q];
    c.tau = st->tau;
    c.g = a.gamma[k];
    const int dv[4] = {done.x, done.y, done.z, done.w};
    const int nv[4] = {nc.x, nc.y, nc.z, nc.w};
    const bool check = k >= 2 && (km % ce == 0 || km == ms);
    unsigned act = 0u;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        bool aj = !(k > ms || err) && dv[j] < 0;
        if (aj && check && nv[j] == 0) {
            aj = false;
            if (blockIdx.x == 0) a.done[4 * q + j] = km;
        }
        act |= aj ? 1u << j : 0u;
    }
    c.act = act;
    c.do_test = k >= 1 && (k % ce == 0 || k == ms);
    c.do_write = k < ms;
    if (__ballot(act != 0u) == 0ull) {
        if (blockIdx.x == 0 && threadIdx.x == 0) a.st->done_step = km;
        return false;
    }
    return true;
}

__device__ __forceinline__ float comp(const float4& v, int j) { return j == 0 ? v.x : j == 1 ? v.y : j == 2 ? v.z : v.w; }
__device__ __forceinline__ float4 abs4(const float4& v) {
    return make_float4(gnk::nbr_term(v.x), gnk::nbr_term(v.y), gnk::nbr_term(v.z), gnk::nbr_term(v.w));
}
__device__ __forceinline__ float4 add4(const float4& a, const float4& b) {
    return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
}
__device__ __forceinline__ unsigned signs4(const float4& v) {
    return sign_of(v.x) | (sign_of(v.y) << 1) | (sign_of(v.z) << 2) | (sign_of(v.w) << 3);
}
__device__ __forceinline__ float4 shfl4(const float4& v, int off) {
    return make_float4(__shfl_xor(v.x, off, 64), __shfl_xor(v.y, off, 64), __shfl_xor(v.z, off, 64),
                       __shfl_xor(v.w, off, 64));
}

// Epilogue of (row i, quad q): the arithmetic of the single-start step for each
// active start; returns the quad's violation bits.  A stopped start keeps the
// value already in y_out's slot (its final state may live there).
__device__ __forceinline__ unsigned quad_update(const MultiArgs& a, const QuadCtl& c, int i, int q,
                                                const float4& yraw, float vi, const float4& sigma, unsigned nbr_sel,
                                                unsigned (&fb)[4], bool& ord_in, bool& ord_out) {
    unsigned viol = 0u;
    float out[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float yr = comp(yraw, j);
        const float yi = fabsf(yr);
        const float s = __fmaf_rn(c.g, comp(sigma, j), yi);
        const bool fallback = !(s > 1e-9f);
        out[j] = gnk::step_word(yr, vi, s);
        const bool on = (c.act >> j) & 1u;
        ord_in |= on && gnk::mag_bits(yr) >= gnk::kLogTop;
        ord_out |= on && c.do_write && gnk::mag_bits(out[j]) >= gnk::kLogTop;
        if (on && c.do_write) fb[j] += fallback ? 1u : 0u;
        if (on && c.do_test) {
            const bool in_s = sign_of(yr) != 0u;
            const float tv = c.tau * vi;
            const bool far = (yi > tv) && ((vi - yi) > tv);
            const bool uncovered = !in_s && !((nbr_sel >> j) & 1u);
            const bool growing = !in_s && (yi > 0.0f) && !(s > vi);
            viol |= (far || uncovered || growing) ? 1u << j : 0u;
        }
    }
    if (c.do_write) {
        float* dst = a.y_out + (size_t)i * kStarts + 4 * q;
        if (c.act == 0xFu) {
            *reinterpret_cast<float4*>(dst) = make_float4(out[0], out[1], out[2], out[3]);
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if ((c.act >> j) & 1u) dst[j] = out[j];
        }
    }
    return viol;
}

// Pruned lists (as in the single-start step): a vertex is listed while some
// start's state of it may be ordinary.  Row i lists itself again when a
// running start's new word is ordinary while none of its running starts' input
// words was (then, and only then, it may have been dropped); during the step
// its entries add nothing either way.  Drops are left to multi_rebuild_kernel,
// run before every captured chain.  `rev`: the row's flags combined over its
// lanes; threads t of nt write the mirror entries.
__device__ __forceinline__ void multi_relist_rows(const MultiArgs& a, int i, int t, int nt);
__device__ __forceinline__ void multi_relist(const MultiArgs& a, int i, bool rev, int t, int nt) {
    if (!rev || a.listed[i]) return;  // every lane of the row reads before lane t = 0 writes
    multi_relist_rows(a, i, t, nt);
}
__device__ __forceinline__ void multi_relist_rows(const MultiArgs& a, int i, int t, int nt) {
    constexpr int U = 16;
    const int e1 = a.row_ptr[i + 1];
    for (int e = a.row_ptr[i] + t; e < e1; e += nt * U) {
        int m[U];
#pragma unroll
        for (int u = 0; u < U; ++u) m[u] = e + u * nt < e1 ? a.mirror[e + u * nt] : -1;
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (m[u] >= 0) a.pcol[m[u]] = i;
    }
    if (t == 0) a.listed[i] = 1;
}

// OR of a flag over the aligned group of W lanes (all lanes take part).
template <int W>
__device__ __forceinline__ bool group_or(bool f) {
    unsigned v = f ? 1u : 0u;
#pragma unroll
    for (int o = 1; o < W; o <<= 1) v |= (unsigned)__shfl_xor((int)v, o, 64);
    return v != 0u;
}

// Violation bits of the 16 starts over a wavefront: bit 4q + j from lanes
// l = q (mod 4) with bit j set.
__device__ __forceinline__ unsigned wave_start_bits(unsigned v4) {
    unsigned bits = 0u;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const unsigned long long m = __ballot((v4 >> j) & 1u);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (m & (0x1111111111111111ull << q)) bits |= 1u << (4 * q + j);
    }
    return bits;
}

// Light rows of degree <= 16: 16 rows per wavefront, lane (r, q) = (l / 4, l % 4)
// runs the whole canonical sum of its row for 4 starts (G = 1: the in-thread
// butterfly 8 .. 1 over the 16 entries).
__device__ __forceinline__ unsigned light_rows16(const MultiArgs& a, QuadCtl& c, int rb, int re, int lb, int wave,
                                               int lane, unsigned (&fb)[4], bool& quit) {
    const int q = lane & 3;
    const int i = rb + (lb * kWaves + wave) * 16 + (lane >> 2);
    const bool valid = i < re;
    const float4* __restrict__ Y4 = reinterpret_cast<const float4*>(a.y_in);
    int start = 0, d = 0;
    float4 yraw = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float vi = 1.0f;
    if (valid) {
        start = gnk::ld_stream(a.row_ptr + i);
        d = gnk::ld_stream(a.row_ptr + i + 1) - start;
        yraw = Y4[(size_t)i * 4 + q];
        vi = a.v[i];
    }
    int idx[16];
#pragma unroll
    for (int p = 0; p < 16; ++p) idx[p] = p < d ? a.col[start + p] : -1;
    if (!quad_ctl(a, q, c)) {
        quit = true;
        return 0u;
    }
    unsigned sel = 0u;
    float4 cs[16];
#pragma unroll
    for (int p = 0; p < 16; ++p) {
        float4 v = idx[p] >= 0 ? Y4[(size_t)idx[p] * 4 + q] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        sel |= signs4(v);
        cs[p] = abs4(v);
    }
#pragma unroll
    for (int off = 8; off >= 1; off >>= 1)
#pragma unroll
        for (int j = 0; j < off; ++j) cs[j] = add4(cs[j], cs[j + off]);
    unsigned viol = 0u;
    bool oi = false, oo = false;
    if (valid) viol = quad_update(a, c, i, q, yraw, vi, cs[0], sel, fb, oi, oo);
    if (a.prune) {  // the row's 4 lanes
        const bool in_any = group_or<4>(oi), out_any = group_or<4>(oo);
        if (valid) multi_relist(a, i, out_any && !in_any, q, 4);
    }
    return viol;
}

// Light rows of degree 17..32: 8 rows per wavefront, lane (r, t, q) =
// (l / 8, (l / 4) % 2, l % 4); the two threads t of a (row, quad) own chains t,
// t+2, .. t+30 (G = 2), fold them in-thread (stages 16 .. 2) and finish with the
// shuffle between t = 0 and t = 1 (stage 1, lane xor 4).
__device__ __forceinline__ unsigned light_rows_g2(const MultiArgs& a, QuadCtl& c, int rb, int re, int lb, int wave,
                                                  int lane, unsigned (&fb)[4], bool& quit) {
    const int q = lane & 3, t = (lane >> 2) & 1;
    const int i = rb + (lb * kWaves + wave) * 8 + (lane >> 3);
    const bool valid = i < re;
    const float4* __restrict__ Y4 = reinterpret_cast<const float4*>(a.y_in);
    int start = 0, d = 0;
    float4 yraw = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float vi = 1.0f;
    if (valid) {
        start = gnk::ld_stream(a.row_ptr + i);
        d = gnk::ld_stream(a.row_ptr + i + 1) - start;
        yraw = Y4[(size_t)i * 4 + q];
        vi = a.v[i];
    }
    int idx[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) idx[j] = t + 2 * j < d ? a.col[start + t + 2 * j] : -1;
    if (!quad_ctl(a, q, c)) {
        quit = true;
        return 0u;
    }
    unsigned sel = 0u;
    float4 cs[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const float4 v = idx[j] >= 0 ? Y4[(size_t)idx[j] * 4 + q] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        sel |= signs4(v);
        cs[j] = abs4(v);
    }
#pragma unroll
    for (int off = 16; off >= 2; off >>= 1)
#pragma unroll
        for (int j = 0; j < off / 2; ++j) cs[j] = add4(cs[j], cs[j + off / 2]);
    const float4 s = add4(cs[0], shfl4(cs[0], 4));
    sel |= __shfl_xor(sel, 4, 64);
    unsigned viol = 0u;
    bool oi = false, oo = false;
    if (valid && t == 0) viol = quad_update(a, c, i, q, yraw, vi, s, sel, fb, oi, oo);
    if (a.prune) {  // the row's 8 lanes
        const bool in_any = group_or<8>(oi), out_any = group_or<8>(oo);
        if (valid) multi_relist(a, i, out_any && !in_any, lane & 7, 8);
    }
    return viol;
}

__global__ __launch_bounds__(kBlock) void multi_step_kernel(MultiArgs a) {
    __shared__ float4 stage[kChunk][kStarts / 4];
    __shared__ float4 red[kBlock];
    __shared__ unsigned s_mask[kWaves];
    __shared__ unsigned s_sel[kWaves];
    __shared__ bool s_rev;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, q = tid & 3;
    const int blk = blockIdx.x;
    QuadCtl c;
    unsigned viol = 0u;
    unsigned fb[4] = {0u, 0u, 0u, 0u};

    if (blk < a.mid_blk) {
        // heavy row: thread (t, q) = (tid / 4, tid % 4) runs chain t for 4 starts
        const int i = blk;
        const int t = tid >> 2;
        const int start = gnk::ld_stream(a.row_ptr + i);
        const int d = gnk::ld_stream(a.row_ptr + i + 1) - start;
        const float4 yraw = reinterpret_cast<const float4*>(a.y_in)[(size_t)i * 4 + q];
        const float vi = a.v[i];
        if (!quad_ctl(a, q, c)) return;
        float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        unsigned sel = 0u;
        for (int c0 = 0; c0 < d; c0 += kChunk) {
            const int cn = min(kChunk, d - c0);
#pragma unroll
            for (int u = 0; u < kChunk / kBlock; ++u) {
                const int e = tid + kBlock * u;
                if (e < cn) {
                    const int j = a.col[start + c0 + e];
                    if (j >= 0) {
                        const float4* src = reinterpret_cast<const float4*>(a.y_in + (size_t)j * kStarts);
#pragma unroll
                        for (int h = 0; h < kStarts / 4; ++h) stage[e][h] = src[h];
                    } else {  // an entry of the pruned lists: adds nothing
#pragma unroll
                        for (int h = 0; h < kStarts / 4; ++h) stage[e][h] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                    }
                }
            }
            __syncthreads();
            for (int e = t; e < cn; e += 64) {
                const float4 v = stage[e][q];
                sel |= signs4(v);
                acc = add4(acc, abs4(v));
            }
            __syncthreads();
        }
        // butterfly over the 64 chains: stages 32 and 16 across wavefronts (LDS),
        // stages 8 .. 1 inside the wavefront (lane bits 5 .. 2)
        red[tid] = acc;
        __syncthreads();
        acc = add4(acc, red[tid ^ 128]);
        __syncthreads();
        red[tid] = acc;
        __syncthreads();
        acc = add4(acc, red[tid ^ 64]);
#pragma unroll
        for (int off = 8; off >= 1; off >>= 1) acc = add4(acc, shfl4(acc, off * 4));
        const unsigned ws = wave_start_bits(sel);
        if (lane == 0) s_sel[wave] = ws;
        __syncthreads();
        const unsigned all = s_sel[0] | s_sel[1] | s_sel[2] | s_sel[3];
        bool oi = false, oo = false;
        if (tid < 4) viol = quad_update(a, c, i, q, yraw, vi, acc, (all >> (4 * q)) & 0xFu, fb, oi, oo);
        if (a.prune) {  // the whole workgroup, after thread 0 has read the flag
            const bool in_any = group_or<4>(oi), out_any = group_or<4>(oo);
            if (tid == 0) s_rev = out_any && !in_any && !a.listed[i];
            __syncthreads();
            if (s_rev) multi_relist_rows(a, i, tid, kBlock);
        }
    } else if (blk < a.light_blk) {
        // mid row: one wavefront, lane (t, q) = (l / 4, l % 4) runs chains t, t+16,
        // t+32, t+48 (two entries each) for 4 starts
        const int i = a.heavy_end + (blk - a.mid_blk) * kWaves + wave;
        const int t = lane >> 2;
        const bool valid = i < a.mid_end;
        const float4* __restrict__ Y4 = reinterpret_cast<const float4*>(a.y_in);
        int start = 0, d = 0;
        float4 yraw = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        float vi = 1.0f;
        if (valid) {
            start = gnk::ld_stream(a.row_ptr + i);
            d = gnk::ld_stream(a.row_ptr + i + 1) - start;
            yraw = Y4[(size_t)i * 4 + q];
            vi = a.v[i];
        }
        int idx[2][4];
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const int p = t + 16 * jj + 64 * m;
                idx[m][jj] = p < d ? a.col[start + p] : -1;
            }
        if (!quad_ctl(a, q, c)) return;
        unsigned sel = 0u;
        float4 ch[4];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) ch[jj] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int jj = 0; jj < 4; ++jj)
                if (idx[m][jj] >= 0) {
                    const float4 v = Y4[(size_t)idx[m][jj] * 4 + q];
                    sel |= signs4(v);
                    ch[jj] = add4(ch[jj], abs4(v));
                }
        ch[0] = add4(ch[0], ch[2]);
        ch[1] = add4(ch[1], ch[3]);
        float4 s = add4(ch[0], ch[1]);
#pragma unroll
        for (int off = 8; off >= 1; off >>= 1) s = add4(s, shfl4(s, off * 4));
        // neighbour selection: OR over the 16 lanes of this quad
        unsigned any = 0u;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const unsigned long long m = __ballot((sel >> j) & 1u);
            any |= (m & (0x1111111111111111ull << q)) ? 1u << j : 0u;
        }
        bool oi = false, oo = false;
        if (valid && t == 0) viol = quad_update(a, c, i, q, yraw, vi, s, any, fb, oi, oo);
        if (a.prune) {  // the whole wavefront
            const bool in_any = __any(oi), out_any = __any(oo);
            if (valid) multi_relist(a, i, out_any && !in_any, lane, 64);
        }
    } else {
        bool quit = false;
        // the block-to-rows map of the single-start step (swizzle_block): blocks
        // that share an XCD work on neighbouring rows
        const int lb = blk - a.light_blk;
        const int nl = (int)gridDim.x - a.light_blk;
        if (lb < a.l16_blk) {
            viol = light_rows_g2(a, c, a.mid_end, a.l16_begin, swizzle_block(lb, a.l16_blk), wave, lane, fb, quit);
        } else {
            viol = light_rows16(a, c, a.l16_begin, a.n, swizzle_block(lb - a.l16_blk, nl - a.l16_blk), wave, lane, fb,
                                quit);
        }
        if (quit) return;  // uniform over the grid
    }

    // per-start test flags: one LDS slot per wavefront, one barrier, at most 16
    // global writes per block; fallbacks are rare and counted directly
    const unsigned wm = wave_start_bits(viol);
    if (lane == 0) s_mask[wave] = wm;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (fb[j]) atomicAdd(&a.fb[4 * q + j], (unsigned long long)fb[j]);
    __syncthreads();
    if (tid < kStarts) {
        const unsigned mm = s_mask[0] | s_mask[1] | s_mask[2] | s_mask[3];
        if ((mm >> tid) & 1u) a.notconv[(size_t)a.k * kStarts + tid] = 1;
    }
}

// Reset per-start state: starts >= count are stopped from the outset.
__global__ void multi_init_kernel(int32_t count, int32_t* done, unsigned long long* fb, int32_t* notconv,
                                  int32_t entries) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < kStarts) {
        done[t] = t < count ? -1 : 0;
        fb[t] = 0ull;
    }
    for (int e = t; e < entries; e += gridDim.x * blockDim.x) notconv[e] = 0;
}

// x (start-major, user order) -> interleaved signed weighted states; flags
// negative or non-finite entries (err bit 1).
__global__ void multi_prep_kernel(int32_t n, int32_t count, const float* __restrict__ x_user,
                                  const int32_t* __restrict__ perm, const float* __restrict__ v,
                                  float* __restrict__ y, SolveState* st) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * kStarts) return;
    const int i = (int)(e / kStarts), b = (int)(e % kStarts);
    float yy = 0.0f;
    if (b < count) {
        float x = x_user[(size_t)b * n + perm[i]];
        if (!(x >= 0.0f) || !isfinite(x)) {
            atomicOr(&st->err, 1);
            x = 0.0f;
        }
        yy = gnk::word_from_x(x, v[i]);
    }
    y[e] = yy;
}

// Normalizable (Section 2) for every start: some positive entry in each closed
// neighbourhood; err bit 2 otherwise.
__global__ void multi_normalizable_kernel(int32_t n, int32_t count, const int32_t* __restrict__ row_ptr,
                                          const int32_t* __restrict__ col, const float* __restrict__ y,
                                          SolveState* st) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * kStarts) return;
    const int i = (int)(e / kStarts), b = (int)(e % kStarts);
    if (b >= count || y[e] != 0.0f) return;
    for (int q = row_ptr[i]; q < row_ptr[i + 1]; ++q)
        if (y[(size_t)col[q] * kStarts + b] != 0.0f) return;
    atomicOr(&st->err, 2);
}

// Drops from the multi-start lists every listed vertex none of whose 16 words
// in y (the next step's input) is ordinary, and lists any other that is not
// (the first chain's rebuild sets the lists for the solve's start).  Eight
// lanes per row, two words each.
__global__ __launch_bounds__(256) void multi_rebuild_kernel(int32_t n, const int32_t* __restrict__ row_ptr,
                                                           const int32_t* __restrict__ mirror,
                                                           const float* __restrict__ y, uint8_t* __restrict__ listed,
                                                           int32_t* __restrict__ pcol) {
    constexpr int G = 8, U = 16;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t i = (int32_t)(tid / G);
    const int t = (int)(tid % G);
    const bool valid = i < n;
    bool o = false;
    if (valid) {
        const float2 w = reinterpret_cast<const float2*>(y + (size_t)i * kStarts)[t];
        o = gnk::mag_bits(w.x) >= gnk::kLogTop || gnk::mag_bits(w.y) >= gnk::kLogTop;
    }
    const bool want = group_or<G>(o);  // every lane takes part
    if (!valid || (listed[i] != 0) == want) return;
    const int32_t val = want ? i : -1;
    const int32_t e1 = row_ptr[i + 1];
    for (int32_t e = row_ptr[i] + t; e < e1; e += G * U) {
        int32_t m[U];
#pragma unroll
        for (int u = 0; u < U; ++u) m[u] = e + u * G < e1 ? mirror[e + u * G] : -1;
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (m[u] >= 0) pcol[m[u]] = val;
    }
    if (t == 0) listed[i] = want ? 1 : 0;
}

// start b's state out of the interleaved buffer
__global__ void multi_extract_kernel(int32_t n, int32_t b, const float* __restrict__ y, float* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = y[(size_t)i * kStarts + b];
}

// Random starting points (code appendix): x = clamp(e / max(e), 1e-3, 1) with
// e = -log(u), the maximum taken over each start's n values.  Non-negative floats
// order like their bit patterns, so the maximum is an integer max.  Grid: x runs
// over a start's values, y over the starts; each block reduces its part in
// registers and LDS and makes one atomicMax (an atomic per value would serialise
// millions of updates on 16 addresses).
__global__ __launch_bounds__(256) void random_max_kernel(int32_t n, const float* __restrict__ u,
                                                         unsigned* __restrict__ maxbits, SolveState* st) {
    __shared__ unsigned s_max[4];
    const int b = blockIdx.y;
    const float* __restrict__ ub = u + (size_t)b * n;
    unsigned m = 0u;
    bool bad = false;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float uu = ub[i];
        if (!(uu > 0.0f && uu <= 1.0f)) {
            bad = true;
            continue;
        }
        const float l = -logf(uu);
        m = max(m, __float_as_uint(l > 0.0f ? l : 0.0f));
    }
    for (int off = 32; off >= 1; off >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, off, 64));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool any_bad = __any(bad);
    if (lane == 0) {
        s_max[wave] = m;
        if (any_bad) atomicOr(&st->err, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) atomicMax(&maxbits[b], max(max(s_max[0], s_max[1]), max(s_max[2], s_max[3])));
}

__global__ void random_apply_kernel(int64_t total, int32_t n, const float* __restrict__ u,
                                    const unsigned* __restrict__ maxbits, float* __restrict__ x) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const float uu = u[e];
        const float mx = __uint_as_float(maxbits[e / n]);
        float l = (uu > 0.0f && uu <= 1.0f) ? -logf(uu) : 0.0f;
        l = l > 0.0f ? l : 0.0f;
        const float r = mx > 0.0f ? l / mx : 1.0f;
        x[e] = fminf(fmaxf(r, 1e-3f), 1.0f);
    }
}

__global__ void clear_kernel(unsigned* p, int32_t count, SolveState* st) {
    const int t = threadIdx.x;
    if (t < count) p[t] = 0u;
    if (t == 0) st->err = 0;
}

struct MultiWS {
    GraphWorkspace ws;       // state, gamma table, pinned staging, captured chains
    unsigned* maxbits = nullptr;  // [16] random starts: per-start maxima
    float* Y[2] = {nullptr, nullptr};
    float* yb = nullptr;     // one start's state, contiguous
    int32_t* done = nullptr;
    unsigned long long* fb = nullptr;
    int32_t* nc16 = nullptr;
    int32_t nc16_cap = 0;    // steps covered by nc16
    FinalStats* stats = nullptr;  // [16] final statistics per start
    int32_t heavy_end = 0, mid_end = 0, l16_begin = 0, mid_blk = 0, light_blk = 0, l16_blk = 0, nblk = 0;
    int32_t* pcol = nullptr;      // pruned lists (allocated on first use): a copy of the CSR columns
    uint8_t* listed = nullptr;    // [n]
    int32_t chunk_prune = -1;     // captured chains' lists: 0 full, else the pruned lists' rebuild interval
};

void free_ws(MultiWS* m) {
    auto f = [](void* p) { if (p) (void)hipFree(p); };
    m->ws.destroy_chains();
    f(m->Y[0]); f(m->Y[1]); f(m->yb); f(m->done); f(m->fb); f(m->nc16); f(m->maxbits); f(m->stats);
    f(m->pcol); f(m->listed);
    f(m->ws.state); f(m->ws.notconv); f(m->ws.gamma);
    if (m->ws.host_pinned) (void)hipHostFree(m->ws.host_pinned);
    delete m;
}

MultiWS* get_ws(gn_graph* g) {
    if (g->multi) return (MultiWS*)g->multi;
    MultiWS* m = new (std::nothrow) MultiWS();
    if (!m) return nullptr;
    const size_t n = (size_t)std::max(g->n, 1);
    bool ok = hipMalloc(&m->Y[0], n * kStarts * 4) == hipSuccess &&
              hipMalloc(&m->Y[1], n * kStarts * 4) == hipSuccess && hipMalloc(&m->yb, n * 4) == hipSuccess &&
              hipMalloc(&m->done, kStarts * 4) == hipSuccess && hipMalloc(&m->fb, kStarts * 8) == hipSuccess &&
              hipMalloc(&m->maxbits, kStarts * 4) == hipSuccess &&
              hipMalloc(&m->stats, kStarts * sizeof(FinalStats)) == hipSuccess &&
              hipMalloc(&m->ws.state, sizeof(SolveState)) == hipSuccess &&
              hipHostMalloc(&m->ws.host_pinned, 4096, hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        free_ws(m);
        return nullptr;
    }
    const BinLayout& bl = g->bins;
    m->heavy_end = bl.row_begin[BIN_G8];
    m->mid_end = bl.row_begin[BIN_LANE32];
    m->l16_begin = bl.row_begin[BIN_LANE16];
    m->mid_blk = m->heavy_end;
    m->light_blk = m->mid_blk + (m->mid_end - m->heavy_end + kWaves - 1) / kWaves;
    constexpr int rows32 = 8 * kWaves, rows16 = 16 * kWaves;  // rows per block of the two light classes
    m->l16_blk = (m->l16_begin - m->mid_end + rows32 - 1) / rows32;
    m->nblk = m->light_blk + m->l16_blk + (g->n - m->l16_begin + rows16 - 1) / rows16;
    g->multi = m;
    return m;
}

gn_status ensure_tables(MultiWS* m, int32_t steps) {
    gn_status st = gn_internal_ensure_tables(m->ws, steps);  // gamma (and single-start flags, unused)
    if (st != GN_OK) return st;
    if (steps > m->nc16_cap) {
        const int32_t cap = std::max(steps, 2 * m->nc16_cap);
        if (m->nc16) (void)hipFree(m->nc16);
        m->nc16 = nullptr;
        m->nc16_cap = 0;
        if (hipMalloc(&m->nc16, (size_t)cap * kStarts * 4) != hipSuccess) {
            (void)hipGetLastError();
            return GN_E_NOMEM;
        }
        m->nc16_cap = cap;
        for (auto ex : m->ws.chunks) if (ex) (void)hipGraphExecDestroy(ex);
        m->ws.chunks.clear();
    }
    return GN_OK;
}

gn_status build_steps(const gn_graph* g, MultiWS* m, int32_t c, int32_t len, bool prune, int32_t q0, int32_t q1,
                      hipGraph_t graph, hipGraphNode_t* last) {
    if (prune && (!m->pcol || !m->listed || !g->prune_mirror)) return GN_E_ARG;  // no pruned lists to read
    hipGraphNode_t prev = *last;
    for (int32_t q = q0; q < q1; ++q) {
        if (prune && gn_internal_rebuilds_at((int64_t)c * len + q)) {  // rebuild of the lists from step k's input
            int32_t n = g->n;
            const int32_t* rp = g->row_ptr;
            const int32_t* mi = g->prune_mirror;
            const float* y = m->Y[(c * len + q) & 1];
            uint8_t* lst = m->listed;
            int32_t* pc = m->pcol;
            void* args[] = {&n, &rp, &mi, &y, &lst, &pc};
            hipKernelNodeParams p{};
            p.func = (void*)multi_rebuild_kernel;
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
        MultiArgs a{};
        a.row_ptr = g->row_ptr;
        a.col = g->col;
        a.v = g->v;
        a.k = c * len + q;
        a.y_in = m->Y[a.k & 1];
        a.y_out = m->Y[(a.k + 1) & 1];
        a.gamma = m->ws.gamma;
        a.st = m->ws.state;
        a.done = m->done;
        a.notconv = m->nc16;
        a.fb = m->fb;
        a.n = g->n;
        a.heavy_end = m->heavy_end;
        a.mid_end = m->mid_end;
        a.l16_begin = m->l16_begin;
        a.mid_blk = m->mid_blk;
        a.light_blk = m->light_blk;
        a.l16_blk = m->l16_blk;
        if (prune) {
            a.prune = 1;
            a.col = m->pcol;
            a.pcol = m->pcol;
            a.mirror = g->prune_mirror;
            a.listed = m->listed;
        }
        void* args[] = {&a};
        hipKernelNodeParams p{};
        p.func = (void*)multi_step_kernel;
        p.gridDim = dim3(m->nblk);
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

}  // namespace

void gn_internal_free_multi(gn_graph* g) {
    if (g->multi) free_ws((MultiWS*)g->multi);
    g->multi = nullptr;
}

extern "C" gn_status gn_multi_solve(gn_graph* g, const gn_schedule* sch, int32_t starts, float* x, uint8_t* sel,
                                    gn_result* res, int32_t* best, hipStream_t stream) {
    if (!g || !sch || !res || !best || starts < 1 || starts > GN_MAX_STARTS) return GN_E_ARG;
    if (!gn_internal_schedule_ok(sch)) return GN_E_ARG;
    std::memset(res, 0, sizeof(gn_result) * (size_t)starts);
    *best = -1;
    if (g->n == 0) {
        for (int b = 0; b < starts; ++b) {
            res[b].binarised = 1;
            res[b].stab = INFINITY;
        }
        *best = 0;
        return GN_OK;
    }
    if (!x || !sel) return GN_E_ARG;
    const int32_t ms = sch->max_steps;
    const int32_t C = g_chunk_len;
    const int32_t nchunks = (ms + 1 + C - 1) / C;
    // the single-start buffers serve the final statistics, and the chained
    // single-start solve of a start handed over (below)
    gn_status st = gn_internal_ensure_ws(g, g_multi_handoff ? nchunks * C : 1);
    if (st != GN_OK) return st;
    MultiWS* m = get_ws(g);
    if (!m) return GN_E_NOMEM;
    if ((st = ensure_tables(m, nchunks * C)) != GN_OK) return st;
    const int n = g->n;

    if ((st = gn_internal_init_solve(m->ws, sch, stream)) != GN_OK) return st;
    const int32_t entries = nchunks * C * kStarts;
    hipLaunchKernelGGL(multi_init_kernel, dim3(std::min((entries + 255) / 256, 1024)), dim3(256), 0, stream, starts,
                       m->done, m->fb, m->nc16, entries);
    GN_HIP_TRY(hipGetLastError());
    const int64_t cells = (int64_t)n * kStarts;
    const int cblocks = (int)((cells + 255) / 256);
    hipLaunchKernelGGL(multi_prep_kernel, dim3(cblocks), dim3(256), 0, stream, n, starts, (const float*)x, g->perm,
                       g->v, m->Y[0], m->ws.state);
    GN_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(multi_normalizable_kernel, dim3(cblocks), dim3(256), 0, stream, n, starts, g->row_ptr, g->col,
                       (const float*)m->Y[0], m->ws.state);
    GN_HIP_TRY(hipGetLastError());

    // pruned lists (gn_set_pruning): allocated on first use as a copy of the
    // columns with every vertex listed.  By default only where the 64-byte state
    // rows (64 n bytes) outgrow an XCD's 4 MB L2, so that the skipped gathers
    // would have missed it: on smaller graphs they were L2 hits and the lists'
    // upkeep costs more (a 10,000-vertex conflict graph: +10%).
    const bool prune = g->prune_mirror &&
                       (g_prune == 2 || (g_prune == 1 && g->prune_pays && 64ll * g->n > (4ll << 20)));
    if (prune && !m->pcol) {
        if (hipMalloc(&m->pcol, sizeof(int32_t) * (size_t)std::max<int64_t>(g->nnz, 1)) != hipSuccess ||
            hipMalloc(&m->listed, (size_t)n) != hipSuccess) {
            (void)hipGetLastError();
            if (m->pcol) (void)hipFree(m->pcol);
            m->pcol = nullptr;
            return GN_E_NOMEM;
        }
        GN_HIP_TRY(hipMemcpyAsync(m->pcol, g->col, sizeof(int32_t) * (size_t)g->nnz, hipMemcpyDeviceToDevice, stream));
        GN_HIP_TRY(hipMemsetAsync(m->listed, 1, (size_t)n, stream));
    }
    if (m->chunk_prune != (prune ? g_prune_every : 0)) {  // chains captured for other lists or rebuild interval
        for (auto ex : m->ws.chunks) if (ex) (void)hipGraphExecDestroy(ex);
        m->ws.chunks.clear();
        m->chunk_prune = prune ? g_prune_every : 0;
    }
    // Hand-off: once a single start is left running, the 16-start step costs as
    // much as ever for it alone.  Its state moves at a chain boundary to the
    // single-start chained solve, which computes the same words, tests and
    // steps (the per-start arithmetic of the two step kernels is the same).
    char* hp = (char*)m->ws.host_pinned;
    volatile int32_t* run = (volatile int32_t*)(hp + kPinRun);  // per chain slot: done step of each start
    int32_t handoff = -1;  // the start handed over
    // Each chain's progress mark copies the starts' done steps to `run`, in
    // every call, since later calls replay the same captured chains.
    ChunkHooks hooks;
    hooks.pin_src = m->done;
    hooks.pin_words = kStarts;
    hooks.pin_offset = kPinRun;
    if (g_multi_handoff && starts > 1) {
        // asked at chain c's mark while chain c + 1 is still to come: with a
        // single start left running, no further chain is launched and that
        // start moves on at step (c + 1) C
        hooks.stop_after = [run, starts, &handoff](int32_t c) {
            int left = 0, who = -1;
            for (int b = 0; b < starts; ++b)
                if (run[kStarts * (c & 1) + b] < 0) {
                    ++left;
                    who = b;
                }
            if (left != 1) return false;
            handoff = who;
            return true;
        };
    }
    int32_t last = -1;
    st = gn_internal_run_marked(
        m->ws, nchunks, C,
        [g, m, C, prune](int32_t c, int32_t q0, int32_t q1, hipGraph_t graph, hipGraphNode_t* tl) {
            return build_steps(g, m, c, C, prune, q0, q1, graph, tl);
        },
        0, stream, true, &hooks, &last);
    if (st != GN_OK) return st;

    // solve state, per-start outcomes and the last step's flags in one round trip
    // through the pinned staging block; the per-start statistics in a second one
    SolveState* hs = (SolveState*)hp;
    int32_t* done = (int32_t*)(hp + kPinDone);
    unsigned long long* fbh = (unsigned long long*)(hp + kPinFb);
    int32_t* nc_last = (int32_t*)(hp + kPinNc);
    FinalStats* fsh = (FinalStats*)(hp + kPinStats);
    GN_HIP_TRY(hipMemcpyAsync(hs, m->ws.state, sizeof(SolveState), hipMemcpyDeviceToHost, stream));
    GN_HIP_TRY(hipMemcpyAsync(done, m->done, kStarts * 4, hipMemcpyDeviceToHost, stream));
    GN_HIP_TRY(hipMemcpyAsync(fbh, m->fb, kStarts * 8, hipMemcpyDeviceToHost, stream));
    GN_HIP_TRY(hipMemcpyAsync(nc_last, m->nc16 + (size_t)ms * kStarts, kStarts * 4, hipMemcpyDeviceToHost, stream));
    GN_HIP_TRY(hipStreamSynchronize(stream));
    if (hs->err & 1) return GN_E_ARG;
    if (hs->err & 2) return GN_E_NOT_NORMALIZABLE;

    int32_t steps_of[kStarts];
    bool bin_of[kStarts];
    for (int b = 0; b < starts; ++b) {
        bin_of[b] = done[b] >= 0 || (ms >= 1 && nc_last[b] == 0);
        steps_of[b] = done[b] >= 0 ? done[b] : ms;
    }
    // the start handed over, if it was still running after the last multi-start chain
    const float* y_handed = nullptr;
    if (handoff >= 0 && last >= 0 && last + 1 < nchunks && done[handoff] < 0) {
        const int32_t k0 = (last + 1) * C;  // its state y_k0 is in Y[k0 & 1]
        GraphWorkspace& ws = g->ws;
        if ((st = gn_internal_init_solve(ws, sch, stream)) != GN_OK) return st;
        hipLaunchKernelGGL(multi_extract_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, n, handoff,
                           (const float*)m->Y[k0 & 1], ws.y[k0 & 1]);
        GN_HIP_TRY(hipGetLastError());
        // the test of step k0 - 1, which the first single-start step reads
        GN_HIP_TRY(hipMemcpyAsync(ws.notconv + (k0 - 1), m->nc16 + (size_t)(k0 - 1) * kStarts + handoff,
                                  sizeof(int32_t), hipMemcpyDeviceToDevice, stream));
        if ((st = gn_internal_chain_solve(g, nchunks, last + 1, stream)) != GN_OK) return st;
        int32_t steps;
        bool binarised;
        if ((st = gn_internal_solve_outcome(ws, ms, &steps, &binarised)) != GN_OK) return st;
        SolveState tail;
        GN_HIP_TRY(hipMemcpy(&tail, ws.state, sizeof(tail), hipMemcpyDeviceToHost));
        steps_of[handoff] = steps;
        bin_of[handoff] = binarised;
        fbh[handoff] += tail.fallback;
        y_handed = ws.y[steps & 1];
    }
    for (int b = 0; b < starts; ++b) {
        const float* yb = m->yb;
        if (b == handoff && y_handed) {
            yb = y_handed;
        } else {
            // stream order lets consecutive starts share the extraction and statistics buffers
            hipLaunchKernelGGL(multi_extract_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, n, b,
                               (const float*)m->Y[steps_of[b] & 1], m->yb);
            GN_HIP_TRY(hipGetLastError());
        }
        st = gn_internal_final_stats_launch(g, yb, gn_internal_host_gamma(sch, steps_of[b]), x + (size_t)b * n,
                                            sel + (size_t)b * n, m->stats + b, stream);
        if (st != GN_OK) return st;
    }
    GN_HIP_TRY(hipMemcpyAsync(fsh, m->stats, sizeof(FinalStats) * (size_t)starts, hipMemcpyDeviceToHost, stream));
    GN_HIP_TRY(hipStreamSynchronize(stream));

    bool all_bin = true;
    double best_w = -INFINITY;
    int best_any = -1;
    double best_any_w = -INFINITY;
    for (int b = 0; b < starts; ++b) {
        const bool bin = bin_of[b];
        const int32_t steps = steps_of[b];
        const FinalStats fs = fsh[b];
        gn_result& r = res[b];
        r.steps = steps;
        r.binarised = bin ? 1 : 0;
        r.fallback_count = (int64_t)fbh[b];
        r.relaxed_objective = fs.relaxed_objective;
        r.set_objective = fs.set_objective;
        r.set_size = fs.set_size;
        r.conflicts = fs.conflicts;
        r.uncovered = fs.uncovered;
        r.stab = fs.stab;
        all_bin = all_bin && bin;
        if (bin && fs.set_objective > best_w) {
            best_w = fs.set_objective;
            *best = b;
        }
        if (fs.set_objective > best_any_w) {
            best_any_w = fs.set_objective;
            best_any = b;
        }
    }
    if (*best < 0) *best = best_any;
    return all_bin ? GN_OK : GN_NOT_CONVERGED;
}

int32_t g_multi_handoff = 1;

extern "C" gn_status gn_set_multi_handoff(int32_t enable) {
    if (enable != 0 && enable != 1) return GN_E_ARG;
    g_multi_handoff = enable;
    return GN_OK;
}

extern "C" gn_status gn_random_starts(gn_graph* g, int32_t starts, const float* u, float* x, hipStream_t stream) {
    if (!g || starts < 1 || starts > GN_MAX_STARTS) return GN_E_ARG;
    if (g->n == 0) return GN_OK;
    if (!u || !x) return GN_E_ARG;
    MultiWS* m = get_ws(g);
    if (!m) return GN_E_NOMEM;
    const int64_t total = (int64_t)starts * g->n;
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(clear_kernel, dim3(1), dim3(64), 0, stream, m->maxbits, kStarts, m->ws.state);
    GN_HIP_TRY(hipGetLastError());
    const int per_start = std::min((g->n + 255) / 256, 256);
    hipLaunchKernelGGL(random_max_kernel, dim3(per_start, starts), dim3(256), 0, stream, g->n, u, m->maxbits,
                       m->ws.state);
    GN_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(random_apply_kernel, dim3(blocks), dim3(256), 0, stream, total, g->n, u,
                       (const unsigned*)m->maxbits, x);
    GN_HIP_TRY(hipGetLastError());
    int32_t err = 0;
    GN_HIP_TRY(hipMemcpyAsync(m->ws.host_pinned, &m->ws.state->err, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    GN_HIP_TRY(hipStreamSynchronize(stream));
    std::memcpy(&err, m->ws.host_pinned, sizeof(err));
    return err ? GN_E_ARG : GN_OK;
}
