// Differentiable WRGN: T unrolled steps and their adjoint, with checkpoints.
//
// Forward (WRGN step, y-space): x'_i = y_i / s_i with y = v (.) x and
// s = (I + gamma A) y.  For an incoming gradient gbar = dL/dx' the chain rule
// gives, with t_i = gbar_i y_i / s_i^2 and I + gamma A symmetric,
//     dL/dy = gbar (/) s - (I + gamma A) t,
//     dL/dx = v (.) dL/dy,     dL/dv += x (.) dL/dy,
// and finally dL/dw = dL/dv (/) (2 v) because v = sqrt(w).  Rows that took the
// 1/2 safe-division reset are constant in x and pass no gradient.  States are
// the library's state words; a row carried in log form (y below 2^-100) enters
// y and x at its decoded value.  A row held at the 2^-1022 support floor would
// pass no gradient either; it is treated as a quotient row, which changes the
// gradients by less than its own value (2^-1022) times the incoming gradient.  One adjoint step is therefore one CSR pass over t in
// the library's canonical row-sum order, fused with the update of dL/dx, dL/dv
// and with the t vector of the previous step.
//
// Memory: the forward keeps y every ckpt_every steps; the backward recomputes
// one segment at a time, storing y and s of that segment, then runs the
// segment's adjoint steps last to first.
#include <algorithm>
#include <cmath>
#include <vector>

#include "gn_internal.h"
#include "gn_rowsum.h"

namespace {

struct UnrolledWS {
    int32_t n = 0, seg = 0;
    float* v = nullptr;      // sqrt(w) for an explicit w (internal order)
    float* y[2] = {nullptr, nullptr};
    float* seg_y = nullptr;  // seg * n
    float* seg_s = nullptr;  // seg * n
    float* tt[2] = {nullptr, nullptr};
    float* gb[2] = {nullptr, nullptr};
    float* gv = nullptr;
};

struct AdjArgs {
    const int32_t* row_ptr;
    const int32_t* col;
    const int32_t* sl_col;   // sliced columns of the group bins (see gn_types.h)
    const int32_t* sl_off;
    const float* v;
    BinLayout bins;
    const float* tt_in;   // t of step k (gathered)
    float* tt_out;        // t of step k-1 (own row), null when step k-1 is outside the segment
    const float* gb_in;   // dL/dx^{k+1}
    float* gb_out;        // dL/dx^k
    float* gv;            // accumulated dL/dv
    const float* y_k;
    const float* s_k;
    const float* y_p;     // step k-1 values (when tt_out != null)
    const float* s_p;
    float gamma;
};

// Whether the forward step took the quotient branch at this row (same test,
// same fp32 value as the forward kernel).
__device__ __forceinline__ bool quotient_branch(float s) { return s > 1e-9f; }

__device__ __forceinline__ void adj_row(const AdjArgs& a, int i, float sigma) {
    const float g = a.gb_in[i];
    const float s = a.s_k[i];
    const float vi = a.v[i];
    const float ai = quotient_branch(s) ? g / s : 0.0f;
    const float gy = ai - __fmaf_rn(a.gamma, sigma, a.tt_in[i]);
    const float gx = vi * gy;
    a.gb_out[i] = gx;
    a.gv[i] += gnk::x_of_word(a.y_k[i], vi) * gy;
    if (a.tt_out) {
        const float yp = gnk::y_of_word(a.y_p[i], vi);
        const float sp = a.s_p[i];
        a.tt_out[i] = quotient_branch(sp) ? (gx / sp) * (yp / sp) : 0.0f;
    }
}

// Rows of a sliced bin: one wavefront per slice of 64/G rows, columns from the
// slice's lines (the layout of the forward step).
template <int G, int MAXD>
__device__ __forceinline__ void adj_sliced_rows(const AdjArgs& a, int b, int rb, int re, int lb) {
    lb = swizzle_block(lb, a.bins.blk_begin[b + 1] - a.bins.blk_begin[b]);  // same map as the step kernel
    constexpr int RS = 64 / G;
    const int lane = threadIdx.x & 63;
    const int ls = lb * kWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r0 = rb + ls * RS;
    if (r0 >= re) return;
    const int t = lane & (G - 1);
    const int i = r0 + lane / G;
    const int gs = a.bins.slice_begin[b] + ls;
    const int l0 = a.sl_off[gs];
    const int width = a.sl_off[gs + 1] - l0;
    gnk::SlicedIdx<G, MAXD> idx;
    idx.load(a.sl_col + (size_t)l0 * 64 + lane, width);
    unsigned unused = 0u;
    const float sigma = idx.template sum<false>(a.tt_in, unused);
    if (i < re && t == 0) adj_row(a, i, sigma);
}

__global__ __launch_bounds__(kBlock) void wrgn_adjoint_kernel(AdjArgs a) {
    __shared__ float stage[kStage];
    const int blk = blockIdx.x;
    int b = 0;
    while (b < BIN_COUNT - 1 && blk >= a.bins.blk_begin[b + 1]) ++b;
    const int lb = blk - a.bins.blk_begin[b];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int rb = a.bins.row_begin[b], re = a.bins.row_begin[b + 1];
    if (b == BIN_BLOCK) {
        const int i = rb + lb;
        const int start = gnk::ld_stream(a.row_ptr + i);
        const int d = gnk::ld_stream(a.row_ptr + i + 1) - start;
        constexpr int PT = kStage / kBlock;
        float acc = 0.0f;
        for (int c0 = 0; c0 < d; c0 += kStage) {
            const int cn = min(kStage, d - c0);
            int cidx[PT];
#pragma unroll
            for (int u = 0; u < PT; ++u) {
                const int p = threadIdx.x + kBlock * u;
                cidx[u] = p < cn ? a.col[start + c0 + p] : -1;
            }
#pragma unroll
            for (int u = 0; u < PT; ++u)
                if (cidx[u] >= 0) stage[threadIdx.x + kBlock * u] = a.tt_in[cidx[u]];
            __syncthreads();
            if (wave == 0)
                for (int q = lane; q < cn; q += 64) acc += stage[q];
            __syncthreads();
        }
        if (wave == 0) {
            for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
            if (lane == 0) adj_row(a, i, acc);
        }
    } else if (b == BIN_WAVE) {
        const int ia = rb + (lb * kWaves + wave) * 2;
        const int ib = ia + 1;
        if (ia < re) {
            const bool hb = ib < re;
            const int sa = gnk::ld_stream(a.row_ptr + ia), ea = gnk::ld_stream(a.row_ptr + ia + 1);
            const int sb = hb ? ea : 0, eb = hb ? gnk::ld_stream(a.row_ptr + ib + 1) : 0;
            unsigned u0 = 0u, u1 = 0u;
            float acca, accb;
            gnk::row_sum_wave2<kWaveMaxDeg / 64, false>(a.col + sa, ea - sa, a.col + sb, eb - sb, a.tt_in, lane, acca,
                                                        accb, u0, u1);
            if (lane == 0) adj_row(a, ia, acca);
            if (lane == 1 && hb) adj_row(a, ib, accb);
        }
    } else if (b == BIN_G8) {
        adj_sliced_rows<8, 128>(a, b, rb, re, lb);
    } else if (b == BIN_LANE32) {
        adj_sliced_rows<2, 32>(a, b, rb, re, lb);
    } else {
        adj_sliced_rows<1, 16>(a, b, rb, re, lb);
    }
}

__global__ void sqrt_weights_kernel(int32_t n, const float* __restrict__ w_user, const int32_t* __restrict__ perm,
                                    float* __restrict__ v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = (float)sqrt((double)w_user[perm[i]]);
}

__global__ void weighted_state_kernel(int32_t n, const float* __restrict__ x_user, const int32_t* __restrict__ perm,
                                      const float* __restrict__ v, float* __restrict__ y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = gnk::word_from_x(x_user[perm[i]], v[i]);
}

// t of the last step of a segment from dL/dx^{k+1}: t_i = gbar_i y_i / s_i^2.
__global__ void adjoint_seed_kernel(int32_t n, const float* __restrict__ gb, const float* __restrict__ y,
                                    const float* __restrict__ s, const float* __restrict__ v,
                                    float* __restrict__ tt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float yy = gnk::y_of_word(y[i], v[i]), ss = s[i];
    tt[i] = quotient_branch(ss) ? (gb[i] / ss) * (yy / ss) : 0.0f;
}

__global__ void gather_user_kernel(int32_t n, const float* __restrict__ src_user, const int32_t* __restrict__ perm,
                                   float* __restrict__ dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src_user[perm[i]];
}

__global__ void unrolled_finish_kernel(int32_t n, const float* __restrict__ gb, const float* __restrict__ gv,
                                       const float* __restrict__ v, const int32_t* __restrict__ perm,
                                       float* __restrict__ gx0, float* __restrict__ gw) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    gx0[perm[i]] = gb[i];
    gw[perm[i]] = gv[i] / (2.0f * v[i]);
}

__global__ void fill_kernel(int64_t n, float* __restrict__ p, float value) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}

UnrolledWS* get_ws(const gn_graph* g, int32_t seg) {
    UnrolledWS* u = (UnrolledWS*)g->unrolled;
    if (u && u->seg >= seg) return u;
    if (u) {
        gn_internal_free_unrolled(const_cast<gn_graph*>(g));
        u = nullptr;
    }
    u = new (std::nothrow) UnrolledWS();
    if (!u) return nullptr;
    u->n = g->n;
    u->seg = seg;
    const size_t n = (size_t)std::max(g->n, 1);
    bool ok = hipMalloc(&u->v, n * 4) == hipSuccess && hipMalloc(&u->y[0], n * 4) == hipSuccess &&
              hipMalloc(&u->y[1], n * 4) == hipSuccess && hipMalloc(&u->seg_y, n * 4 * seg) == hipSuccess &&
              hipMalloc(&u->seg_s, n * 4 * seg) == hipSuccess && hipMalloc(&u->tt[0], n * 4) == hipSuccess &&
              hipMalloc(&u->tt[1], n * 4) == hipSuccess && hipMalloc(&u->gb[0], n * 4) == hipSuccess &&
              hipMalloc(&u->gb[1], n * 4) == hipSuccess && hipMalloc(&u->gv, n * 4) == hipSuccess;
    g->unrolled = u;
    if (!ok) {
        (void)hipGetLastError();
        gn_internal_free_unrolled(const_cast<gn_graph*>(g));
        return nullptr;
    }
    return u;
}

StepArgs fwd_args(const gn_graph* g, const float* v) {
    StepArgs a{};
    a.row_ptr = g->row_ptr;
    a.col = g->col;
    a.v = v;
    a.perm = g->perm;
    a.sl_col = g->sl_col;
    a.sl_off = g->sl_off;
    a.bins = g->bins;
    a.solve = 0;
    a.gamma = nullptr;
    return a;
}

gn_status check_common(const gn_graph* g, const float* gammas, int32_t T, int32_t K) {
    if (!g || T < 0 || K < 1 || (T > 0 && !gammas)) return GN_E_ARG;
    for (int32_t t = 0; t < T; ++t)
        if (!std::isfinite(gammas[t]) || gammas[t] < 0.0f) return GN_E_ARG;
    return GN_OK;
}

const float* weights_v(const gn_graph* g, UnrolledWS* u, const float* w, hipStream_t s) {
    if (!w) return g->v;
    hipLaunchKernelGGL(sqrt_weights_kernel, dim3((g->n + 255) / 256), dim3(256), 0, s, g->n, w, g->perm, u->v);
    return u->v;
}

}  // namespace

void gn_internal_free_unrolled(gn_graph* g) {
    UnrolledWS* u = (UnrolledWS*)g->unrolled;
    if (!u) return;
    for (float* p : {u->v, u->y[0], u->y[1], u->seg_y, u->seg_s, u->tt[0], u->tt[1], u->gb[0], u->gb[1], u->gv})
        if (p) (void)hipFree(p);
    delete u;
    g->unrolled = nullptr;
}

extern "C" int64_t gn_unrolled_ckpt_floats(const gn_graph* g, int32_t T, int32_t ckpt_every) {
    if (!g || T < 0 || ckpt_every < 1) return -1;
    const int64_t n = std::max(g->n, 1);
    if (T >= 1 && ckpt_every == 1) return 2 * (int64_t)T * n;  // y and s of every step: no recompute
    const int64_t segs = T == 0 ? 1 : (T + ckpt_every - 1) / ckpt_every;
    return segs * n;
}

extern "C" gn_status gn_unrolled_forward(const gn_graph* g, const float* w, const float* gammas, int32_t T,
                                         int32_t ckpt_every, const float* x0, float* xT, float* ckpt,
                                         hipStream_t stream) {
    gn_status st = check_common(g, gammas, T, ckpt_every);
    if (st != GN_OK) return st;
    const int n = g->n;
    if (n == 0) return GN_OK;
    if (!x0 || !xT || !ckpt || x0 == xT) return GN_E_ARG;
    UnrolledWS* u = get_ws(g, ckpt_every);
    if (!u) return GN_E_NOMEM;
    const float* v = weights_v(g, u, w, stream);
    GN_HIP_TRY(hipGetLastError());
    if (T >= 1 && ckpt_every == 1) {
        // every step's y and s go straight into ckpt ([T][n] y, then [T][n] s),
        // so the backward recomputes nothing
        hipLaunchKernelGGL(weighted_state_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, n, x0, g->perm, v,
                           ckpt);
        GN_HIP_TRY(hipGetLastError());
        for (int32_t t = 0; t < T; ++t) {
            StepArgs a = fwd_args(g, v);
            a.y_in = ckpt + (size_t)t * n;
            a.y_out = t + 1 < T ? ckpt + (size_t)(t + 1) * n : u->y[0];
            a.s_out = ckpt + (size_t)(T + t) * n;
            a.gamma_scalar = gammas[t];
            a.x_out_user = t == T - 1 ? xT : nullptr;
            st = gn_internal_launch_step(g, a, stream);
            if (st != GN_OK) return st;
        }
        return GN_OK;
    }
    hipLaunchKernelGGL(weighted_state_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, n, x0, g->perm, v, u->y[0]);
    GN_HIP_TRY(hipGetLastError());
    GN_HIP_TRY(hipMemcpyAsync(ckpt, u->y[0], sizeof(float) * n, hipMemcpyDeviceToDevice, stream));
    if (T == 0) {
        GN_HIP_TRY(hipMemcpyAsync(xT, x0, sizeof(float) * n, hipMemcpyDeviceToDevice, stream));
        return GN_OK;
    }
    for (int32_t t = 0; t < T; ++t) {
        StepArgs a = fwd_args(g, v);
        a.y_in = u->y[t & 1];
        a.y_out = u->y[(t + 1) & 1];
        a.gamma_scalar = gammas[t];
        a.x_out_user = t == T - 1 ? xT : nullptr;
        st = gn_internal_launch_step(g, a, stream);
        if (st != GN_OK) return st;
        if ((t + 1) % ckpt_every == 0 && t + 1 < T)
            GN_HIP_TRY(hipMemcpyAsync(ckpt + (size_t)((t + 1) / ckpt_every) * n, u->y[(t + 1) & 1], sizeof(float) * n,
                                      hipMemcpyDeviceToDevice, stream));
    }
    return GN_OK;
}

extern "C" gn_status gn_unrolled_backward(const gn_graph* g, const float* w, const float* gammas, int32_t T,
                                          int32_t ckpt_every, const float* ckpt, const float* gxT, float* gw,
                                          float* gx0, hipStream_t stream) {
    gn_status st = check_common(g, gammas, T, ckpt_every);
    if (st != GN_OK) return st;
    const int n = g->n;
    if (n == 0) return GN_OK;
    if (!ckpt || !gxT || !gw || !gx0) return GN_E_ARG;
    const int K = ckpt_every;
    UnrolledWS* u = get_ws(g, K);
    if (!u) return GN_E_NOMEM;
    const float* v = weights_v(g, u, w, stream);
    GN_HIP_TRY(hipGetLastError());
    const dim3 eg((n + 255) / 256), eb(256);
    int cur = 0;
    hipLaunchKernelGGL(gather_user_kernel, eg, eb, 0, stream, n, gxT, g->perm, u->gb[cur]);
    hipLaunchKernelGGL(fill_kernel, eg, eb, 0, stream, (int64_t)n, u->gv, 0.0f);
    GN_HIP_TRY(hipGetLastError());
    const int nblk = gn_internal_grid_blocks(g->bins);
    // ckpt_every = 1: the forward kept y and s of every step, and the whole run is
    // one segment that needs no recompute
    const bool stored = K == 1;
    const int32_t seglen = stored ? T : K;
    const int32_t nseg = (T + seglen - 1) / seglen;
    for (int32_t c = nseg - 1; c >= 0; --c) {
        const int32_t t0 = c * seglen, t1 = std::min(T, t0 + seglen);
        const float* sy = stored ? ckpt : u->seg_y;                 // y^t at sy + (t - t0) n
        const float* ss = stored ? ckpt + (size_t)T * n : u->seg_s;  // s^t likewise
        if (!stored) {
            // recompute the segment from its checkpoint, keeping y^t and s^t
            GN_HIP_TRY(hipMemcpyAsync(u->seg_y, ckpt + (size_t)c * n, sizeof(float) * n, hipMemcpyDeviceToDevice,
                                      stream));
            for (int32_t t = t0; t < t1; ++t) {
                StepArgs a = fwd_args(g, v);
                a.y_in = u->seg_y + (size_t)(t - t0) * n;
                a.y_out = t + 1 < t1 ? u->seg_y + (size_t)(t + 1 - t0) * n : u->y[0];
                a.s_out = u->seg_s + (size_t)(t - t0) * n;
                a.gamma_scalar = gammas[t];
                st = gn_internal_launch_step(g, a, stream);
                if (st != GN_OK) return st;
            }
        }
        int tc = 0;
        hipLaunchKernelGGL(adjoint_seed_kernel, eg, eb, 0, stream, n, u->gb[cur], sy + (size_t)(t1 - 1 - t0) * n,
                           ss + (size_t)(t1 - 1 - t0) * n, v, u->tt[tc]);
        GN_HIP_TRY(hipGetLastError());
        for (int32_t t = t1 - 1; t >= t0; --t) {
            AdjArgs a{};
            a.row_ptr = g->row_ptr;
            a.col = g->col;
            a.sl_col = g->sl_col;
            a.sl_off = g->sl_off;
            a.v = v;
            a.bins = g->bins;
            a.tt_in = u->tt[tc];
            a.tt_out = t - 1 >= t0 ? u->tt[tc ^ 1] : nullptr;
            a.gb_in = u->gb[cur];
            a.gb_out = u->gb[cur ^ 1];
            a.gv = u->gv;
            a.y_k = sy + (size_t)(t - t0) * n;
            a.s_k = ss + (size_t)(t - t0) * n;
            a.y_p = t - 1 >= t0 ? sy + (size_t)(t - 1 - t0) * n : nullptr;
            a.s_p = t - 1 >= t0 ? ss + (size_t)(t - 1 - t0) * n : nullptr;
            a.gamma = gammas[t];
            if (nblk > 0) hipLaunchKernelGGL(wrgn_adjoint_kernel, dim3(nblk), dim3(kBlock), 0, stream, a);
            GN_HIP_TRY(hipGetLastError());
            cur ^= 1;
            tc ^= 1;
        }
    }
    hipLaunchKernelGGL(unrolled_finish_kernel, eg, eb, 0, stream, n, u->gb[cur], u->gv, v, g->perm, gx0, gw);
    GN_HIP_TRY(hipGetLastError());
    return GN_OK;
}
