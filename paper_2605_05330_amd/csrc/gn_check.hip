// Final rounding, independence / maximality check, set and relaxed objectives,
// gamma-stability.  All reductions are two-level with a fixed order, so the
// results are bit-reproducible run to run.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "gn_internal.h"
#include "gn_rowsum.h"
#include "gn_stats.h"

namespace {

// Final state: x = clamp(|y| / v, 0, 1), S = {x > 1/2}; outputs in user order.
// `pick` (may be null) supplies y, or says that nothing is to be written.
__global__ void finalize_kernel(int32_t n, const float* __restrict__ y, const float* __restrict__ v,
                                const int32_t* __restrict__ perm, float* __restrict__ x_user,
                                uint8_t* __restrict__ sel_user, uint8_t* __restrict__ sel_int,
                                const FinalPick* __restrict__ pick) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (pick) {
        if (pick->skip) return;
        y = pick->y;
    }
    float x = gnk::x_of_word(y[i], v[i]);
    x = fminf(fmaxf(x, 0.0f), 1.0f);
    const uint8_t s = x > 0.5f ? 1 : 0;
    x_user[perm[i]] = x;
    sel_user[perm[i]] = s;
    sel_int[i] = s;
}

__global__ void gather_sel_kernel(int32_t n, const uint8_t* __restrict__ sel_user, const int32_t* __restrict__ perm,
                                  uint8_t* __restrict__ sel_int) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    sel_int[i] = sel_user[perm[i]] ? 1 : 0;
}

// One CSR pass over the selected set.  Heavy rows (deg > 32, internal rows
// [0, light_begin)) are handled by one wavefront each, light rows by one lane.
__global__ __launch_bounds__(kBlock) void set_stats_kernel(int32_t n, int32_t light_begin, int32_t heavy_blocks,
                                                          const int32_t* __restrict__ row_ptr,
                                                          const int32_t* __restrict__ col,
                                                          const float* __restrict__ v,
                                                          const float* __restrict__ w_int,
                                                          const float* __restrict__ y,  // may be null
                                                          const uint8_t* __restrict__ sel, Partial* out,
                                                          const FinalPick* __restrict__ pick) {  // may be null
    Partial p{0.0, 0.0, 0, 0, 0, INFINITY, 0};
    if (pick) {
        if (pick->skip) return;  // the reduction then reads stale partials, unused
        y = pick->y;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    auto row_tail = [&](int i, long long conf, bool any_sel, float vsum) {
        const bool in_s = sel[i] != 0;
        if (y) {
            float x = gnk::x_of_word(y[i], v[i]);
            x = fminf(fmaxf(x, 0.0f), 1.0f);
            p.relaxed += (double)w_int[i] * (double)x;
        }
        if (in_s) {
            p.set_w += (double)w_int[i];
            p.size += 1;
            p.conflicts += conf;
        } else {
            if (!any_sel) p.uncovered += 1;
            p.stab = fminf(p.stab, vsum / v[i]);
        }
    };
    if ((int)blockIdx.x < heavy_blocks) {
        const int i = blockIdx.x * kWaves + wave;
        if (i < light_begin) {
            const int start = __builtin_nontemporal_load(row_ptr + i), end = __builtin_nontemporal_load(row_ptr + i + 1);
            const bool in_s = sel[i] != 0;
            long long conf = 0;
            unsigned any = 0;
            float vsum = 0.0f;
            for (int e = start + lane; e < end; e += 64) {
                const int j = col[e];
                if (sel[j]) {
                    any = 1;
                    if (in_s && j > i) conf += 1;
                    if (!in_s) vsum += v[j];
                }
            }
            conf = wave_sum_ll(conf);
            for (int off = 32; off >= 1; off >>= 1) vsum += __shfl_xor(vsum, off, 64);
            const bool any_sel = __any(any != 0u);
            if (lane == 0) row_tail(i, conf, any_sel, vsum);
        }
    } else {
        const int i = light_begin + (blockIdx.x - heavy_blocks) * kBlock + threadIdx.x;
        if (i < n) {
            const bool in_s = sel[i] != 0;
            long long conf = 0;
            bool any = false;
            float vsum = 0.0f;
            const int e0 = __builtin_nontemporal_load(row_ptr + i), e1 = __builtin_nontemporal_load(row_ptr + i + 1);
            for (int e = e0; e < e1; ++e) {
                const int j = col[e];
                if (sel[j]) {
                    any = true;
                    if (in_s && j > i) conf += 1;
                    if (!in_s) vsum += v[j];
                }
            }
            row_tail(i, conf, any, vsum);
        }
    }
    block_reduce_store(p, out);
}

__global__ void objective_kernel(int32_t n, const float* __restrict__ w, const float* __restrict__ x, Partial* out) {
    Partial p{0.0, 0.0, 0, 0, 0, INFINITY, 0};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        p.relaxed += (double)w[i] * (double)x[i];
    block_reduce_store(p, out);
}

gn_status ensure_partials(const gn_graph* g, int64_t count) {
    GraphWorkspace& ws = g->ws;
    if (count <= ws.partials_cap) return GN_OK;
    if (ws.partials) (void)hipFree(ws.partials);
    ws.partials = nullptr;
    ws.partials_cap = 0;
    if (hipMalloc(&ws.partials, sizeof(Partial) * (size_t)count) != hipSuccess) {
        (void)hipGetLastError();
        ws.partials = nullptr;
        return GN_E_NOMEM;
    }
    ws.partials_cap = count;
    return GN_OK;
}

// Set statistics of sel_int (and the relaxed objective of y when given), reduced
// into dev_out on the device; no host synchronisation.
gn_status launch_set_stats(const gn_graph* g, const float* y, const uint8_t* sel_int, float gamma,
                           FinalStats* dev_out, hipStream_t s, const FinalPick* pick = nullptr) {
    const int n = g->n;
    const int light_begin = g->bins.row_begin[BIN_LANE32];
    const int heavy_blocks = (light_begin + kWaves - 1) / kWaves;
    const int light_blocks = (n - light_begin + kBlock - 1) / kBlock;
    const int nb = heavy_blocks + light_blocks;
    gn_status st = ensure_partials(g, std::max(nb, 1));
    if (st != GN_OK) return st;
    Partial* part = (Partial*)g->ws.partials;
    if (nb > 0) {
        hipLaunchKernelGGL(set_stats_kernel, dim3(nb), dim3(kBlock), 0, s, n, light_begin, heavy_blocks, g->row_ptr,
                           g->col, g->v, g->w_int, y, sel_int, part, pick);
        GN_HIP_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(kBlock), 0, s, nb, (const Partial*)part, gamma, dev_out,
                       pick);
    GN_HIP_TRY(hipGetLastError());
    return GN_OK;
}

gn_status fetch_stats(const gn_graph* g, FinalStats* host_out, hipStream_t s) {
    GN_HIP_TRY(hipMemcpyAsync(g->ws.host_pinned, g->ws.final_out, sizeof(FinalStats), hipMemcpyDeviceToHost, s));
    GN_HIP_TRY(hipStreamSynchronize(s));
    std::memcpy(host_out, g->ws.host_pinned, sizeof(FinalStats));
    return GN_OK;
}

}  // namespace

gn_status gn_internal_final_stats_launch(gn_graph* g, const float* y_fin, float gamma_fin, float* x_user,
                                         uint8_t* sel_user, FinalStats* dev_out, hipStream_t s) {
    const int n = g->n;
    hipLaunchKernelGGL(finalize_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, y_fin, g->v, g->perm, x_user,
                       sel_user, g->ws.sel_int, (const FinalPick*)nullptr);
    GN_HIP_TRY(hipGetLastError());
    return launch_set_stats(g, y_fin, g->ws.sel_int, gamma_fin, dev_out, s);
}

gn_status gn_internal_final_stats_picked(gn_graph* g, const FinalPick* pick, float* x_user, uint8_t* sel_user,
                                         FinalStats* dev_out, hipStream_t s) {
    const int n = g->n;
    hipLaunchKernelGGL(finalize_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, (const float*)nullptr, g->v,
                       g->perm, x_user, sel_user, g->ws.sel_int, pick);
    GN_HIP_TRY(hipGetLastError());
    return launch_set_stats(g, nullptr, g->ws.sel_int, 0.0f, dev_out, s, pick);
}

gn_status gn_internal_final_stats(gn_graph* g, const float* y_fin, float gamma_fin, float* x_user, uint8_t* sel_user,
                                  FinalStats* host_out, hipStream_t s) {
    gn_status st = gn_internal_final_stats_launch(g, y_fin, gamma_fin, x_user, sel_user,
                                                  (FinalStats*)g->ws.final_out, s);
    return st != GN_OK ? st : fetch_stats(g, host_out, s);
}

gn_status gn_internal_sel_stats(const gn_graph* g, const uint8_t* sel_user, FinalStats* host_out, hipStream_t s) {
    const int n = g->n;
    hipLaunchKernelGGL(gather_sel_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, sel_user, g->perm,
                       g->ws.sel_int);
    GN_HIP_TRY(hipGetLastError());
    gn_status st = launch_set_stats(g, nullptr, g->ws.sel_int, 1.0f, (FinalStats*)g->ws.final_out, s);
    return st != GN_OK ? st : fetch_stats(g, host_out, s);
}

extern "C" gn_status gn_objective(const gn_graph* g, const float* x, double* out, hipStream_t stream) {
    if (!g || !out) return GN_E_ARG;
    if (g->n == 0) {
        *out = 0.0;
        return GN_OK;
    }
    if (!x) return GN_E_ARG;
    gn_status st = gn_internal_ensure_ws(const_cast<gn_graph*>(g), 1);
    if (st != GN_OK) return st;
    const int nb = std::min((g->n + kBlock - 1) / kBlock, 1024);
    st = ensure_partials(g, nb);
    if (st != GN_OK) return st;
    Partial* part = (Partial*)g->ws.partials;
    hipLaunchKernelGGL(objective_kernel, dim3(nb), dim3(kBlock), 0, stream, g->n, (const float*)g->w_user, x, part);
    GN_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(kBlock), 0, stream, nb, (const Partial*)part, 1.0f,
                       (FinalStats*)g->ws.final_out, (const FinalPick*)nullptr);
    GN_HIP_TRY(hipGetLastError());
    GN_HIP_TRY(hipMemcpyAsync(g->ws.host_pinned, g->ws.final_out, sizeof(FinalStats), hipMemcpyDeviceToHost, stream));
    GN_HIP_TRY(hipStreamSynchronize(stream));
    FinalStats f;
    std::memcpy(&f, g->ws.host_pinned, sizeof(f));
    *out = f.relaxed_objective;
    return GN_OK;
}

extern "C" gn_status gn_check_independent(const gn_graph* g, const uint8_t* sel, int64_t* conflicts,
                                          int64_t* uncovered, hipStream_t stream) {
    if (!g || !conflicts) return GN_E_ARG;
    if (g->n == 0) {
        *conflicts = 0;
        if (uncovered) *uncovered = 0;
        return GN_OK;
    }
    if (!sel) return GN_E_ARG;
    gn_status st = gn_internal_ensure_ws(const_cast<gn_graph*>(g), 1);
    if (st != GN_OK) return st;
    FinalStats f{};
    st = gn_internal_sel_stats(g, sel, &f, stream);
    if (st != GN_OK) return st;
    *conflicts = f.conflicts;
    if (uncovered) *uncovered = f.uncovered;
    return GN_OK;
}
