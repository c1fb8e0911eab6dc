// Fixed-order reductions of the final statistics (device code), shared by the
// graph and assignment solvers.  Two levels: a butterfly inside each wavefront,
// the wavefronts of a block in order, then one block over the per-block partials
// in order, so every figure is bit-reproducible run to run.
#pragma once

#include <hip/hip_runtime.h>

#include "gn_internal.h"

namespace {

struct Partial {
    double relaxed;   // sum w_i x_i
    double set_w;     // sum_{i in S} w_i
    long long size;
    long long conflicts;
    long long uncovered;
    float stab;       // min over i not in S of (sum_{j in N(i) cap S} v_j) / v_i, before * gamma
    int32_t pad;
};

__device__ double wave_sum_d(double x) {
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}
__device__ long long wave_sum_ll(long long x) {
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}
__device__ float wave_min_f(float x) {
    for (int off = 32; off >= 1; off >>= 1) x = fminf(x, __shfl_xor(x, off, 64));
    return x;
}

// Block reduction in a fixed order (wave butterflies, then waves 0..3 in order).
__device__ void block_reduce_store(Partial p, Partial* out) {
    __shared__ Partial sp[kWaves];
    p.relaxed = wave_sum_d(p.relaxed);
    p.set_w = wave_sum_d(p.set_w);
    p.size = wave_sum_ll(p.size);
    p.conflicts = wave_sum_ll(p.conflicts);
    p.uncovered = wave_sum_ll(p.uncovered);
    p.stab = wave_min_f(p.stab);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sp[wave] = p;
    __syncthreads();
    if (threadIdx.x == 0) {
        Partial r = sp[0];
        for (int w = 1; w < kWaves; ++w) {
            r.relaxed += sp[w].relaxed;
            r.set_w += sp[w].set_w;
            r.size += sp[w].size;
            r.conflicts += sp[w].conflicts;
            r.uncovered += sp[w].uncovered;
            r.stab = fminf(r.stab, sp[w].stab);
        }
        out[blockIdx.x] = r;
    }
}

// Single-block fixed-order reduction of the per-block partials.
// gamma scales the stability; `pick` (may be null) supplies it instead.
__global__ __launch_bounds__(kBlock) void reduce_partials_kernel(int32_t count, const Partial* __restrict__ in,
                                                                 float gamma, FinalStats* out,
                                                                 const FinalPick* pick) {
    if (pick) gamma = pick->gamma;
    Partial p{0.0, 0.0, 0, 0, 0, INFINITY, 0};
    for (int b = threadIdx.x; b < count; b += kBlock) {
        const Partial q = in[b];
        p.relaxed += q.relaxed;
        p.set_w += q.set_w;
        p.size += q.size;
        p.conflicts += q.conflicts;
        p.uncovered += q.uncovered;
        p.stab = fminf(p.stab, q.stab);
    }
    __shared__ Partial tmp[1];
    block_reduce_store(p, tmp);
    __syncthreads();
    if (threadIdx.x == 0) {
        FinalStats f;
        f.relaxed_objective = tmp[0].relaxed;
        f.set_objective = tmp[0].set_w;
        f.set_size = tmp[0].size;
        f.conflicts = tmp[0].conflicts;
        f.uncovered = tmp[0].uncovered;
        f.stab = isinf(tmp[0].stab) ? INFINITY : gamma * tmp[0].stab;
        f.pad = 0;
        *out = f;
    }
}

}  // namespace
