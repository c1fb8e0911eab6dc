// Canonical-order neighbour sums for the WRGN step (device code).
//
// The canonical order of sum_{j in N(i)} |y_j| (fixed for the whole library):
// entry e of the row (CSR order) belongs to virtual lane e mod 64; each virtual
// lane adds its entries in increasing e, starting from 0; the 64 virtual lanes
// are combined by a butterfly with xor offsets 32, 16, 8, 4, 2, 1.  A group of G
// threads (G a power of two <= 64) evaluates exactly this: thread t owns virtual
// lanes t, t+G, t+2G, ...; it runs their sequential sums, folds them in-thread
// for the butterfly stages 32 .. G (the partner lane of every such stage lives
// in the same thread), and the group finishes with xor shuffles G/2 .. 1.
// Missing entries are exact zeros, so every (G, MAXD) instantiation returns the
// same bits for the same row.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gnk {

__device__ __forceinline__ unsigned sign_of(float y) { return __float_as_uint(y) >> 31; }

// Streamed (read-once-per-step) loads.  The non-temporal hint also keeps the
// compiler from fusing row_ptr[i] and row_ptr[i+1] into one 8-byte load, which
// is misaligned for odd i and costs several microseconds per step.
template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) { return __builtin_nontemporal_load(p); }

// Support invariance (Section 2, property ii) in fp32: a positive state never
// underflows to an exact zero (which would freeze it for good); it is held at
// 2^-100 or above.  Exact zeros stay zero.
constexpr float kXMin = 0x1p-100f;
__device__ __forceinline__ float bounded_ratio(float yi, float s) {
    const float r = yi / s;
    return (yi > 0.0f && r < kXMin) ? kXMin : r;
}

// Group of G threads sums one row of degree d <= MAXD.  `t` is the thread's
// index inside the group.  Returns the canonical sum (valid in every thread of
// the group) and ORs the sign bits (rounded-set membership) of the neighbours
// into `sel` (per thread; the caller reduces it over the group).
// Values entering a sum: |y| for the sign-carrying state (ABS), raw values for
// signed adjoint vectors.  Column ids are int32, or uint16 for a graph of at most
// 65536 vertices whose columns are staged in LDS.
template <bool ABS>
__device__ __forceinline__ float term(float v) { return ABS ? fabsf(v) : v; }

template <int G, int MAXD, bool ABS = true, typename IT = int32_t>
__device__ __forceinline__ float row_sum(const IT* __restrict__ cp, int d, const float* __restrict__ y, int t,
                                         unsigned& sel) {
    constexpr int NV = MAXD < 64 ? MAXD : 64;         // virtual lanes that can hold entries
    constexpr int NCH = NV / G;                       // virtual lanes (chains) per thread
    constexpr int PER = (MAXD + 63) / 64;             // entries per chain
    static_assert(NCH >= 1 && (NV % G) == 0, "bad group shape");
    float c[NCH];
    int idx[PER][NCH];
#pragma unroll
    for (int m = 0; m < PER; ++m)
#pragma unroll
        for (int j = 0; j < NCH; ++j) {
            const int p = t + G * j + 64 * m;
            idx[m][j] = p < d ? cp[p] : -1;
        }
#pragma unroll
    for (int j = 0; j < NCH; ++j) c[j] = 0.0f;
#pragma unroll
    for (int m = 0; m < PER; ++m)
#pragma unroll
        for (int j = 0; j < NCH; ++j) {
            if (idx[m][j] >= 0) {
                const float yv = y[idx[m][j]];
                c[j] += term<ABS>(yv);
                if (ABS) sel |= sign_of(yv);
            }
        }
    // butterfly stages NV/2 .. G inside the thread
#pragma unroll
    for (int off = NV / 2; off >= G; off >>= 1)
#pragma unroll
        for (int j = 0; j < off / G; ++j) c[j] += c[j + off / G];
    float s = c[0];
#pragma unroll
    for (int off = G / 2; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    return s;
}

// Same sum over the sliced layout, in two parts so that callers can issue the
// column loads early.  `cp` points at this lane's word of the slice's first line;
// `width` lines follow at a stride of 64 words, and -1 marks positions past the
// row's end.  Line q holds entry t + G*q of the row, so the chain j of block m
// (entry t + G*j + 64*m) sits in line j + m*NCH.
template <int G, int MAXD>
struct SlicedIdx {
    static constexpr int NV = MAXD < 64 ? MAXD : 64;
    static constexpr int NCH = NV / G;
    static constexpr int PER = (MAXD + 63) / 64;
    static_assert(NCH >= 1 && (NV % G) == 0, "bad group shape");
    static_assert(PER == 1 || G * NCH == 64, "blocks of 64 entries must fill whole lines");
    int idx[PER][NCH];

    __device__ __forceinline__ void load(const int32_t* __restrict__ cp, int width) {
#pragma unroll
        for (int m = 0; m < PER; ++m)
#pragma unroll
            for (int j = 0; j < NCH; ++j) {
                const int q = j + m * NCH;
                idx[m][j] = q < width ? ld_stream(cp + 64 * q) : -1;
            }
    }

    template <bool ABS>
    __device__ __forceinline__ float sum(const float* __restrict__ y, unsigned& sel) const {
        float c[NCH];
#pragma unroll
        for (int j = 0; j < NCH; ++j) c[j] = 0.0f;
#pragma unroll
        for (int m = 0; m < PER; ++m)
#pragma unroll
            for (int j = 0; j < NCH; ++j) {
                if (idx[m][j] >= 0) {
                    const float yv = y[idx[m][j]];
                    c[j] += term<ABS>(yv);
                    if (ABS) sel |= sign_of(yv);
                }
            }
#pragma unroll
        for (int off = NV / 2; off >= G; off >>= 1)
#pragma unroll
            for (int j = 0; j < off / G; ++j) c[j] += c[j + off / G];
        float s = c[0];
#pragma unroll
        for (int off = G / 2; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
        return s;
    }
};

// One wavefront (G = 64) sums a row of any degree: each lane runs its chain in
// batches of U independent loads.
template <int U, bool ABS = true, typename IT = int32_t>
__device__ __forceinline__ float row_sum_wave(const IT* __restrict__ cp, int d, const float* __restrict__ y,
                                              int lane, unsigned& sel) {
    float acc = 0.0f;
    int e = lane;
    for (; e + 64 * (U - 1) < d; e += 64 * U) {
        int c[U];
        float v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) c[u] = cp[e + 64 * u];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = y[c[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            acc += term<ABS>(v[u]);
            if (ABS) sel |= sign_of(v[u]);
        }
    }
    for (; e < d; e += 64) {
        const float yv = y[cp[e]];
        acc += term<ABS>(yv);
        if (ABS) sel |= sign_of(yv);
    }
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    return acc;
}

// One wavefront sums two rows of degree <= 64*U at once (all loads of both rows
// in flight together); same canonical order as row_sum_wave.
template <int U, bool ABS = true>
__device__ __forceinline__ void row_sum_wave2(const int32_t* __restrict__ cpa, int da, const int32_t* __restrict__ cpb,
                                              int db, const float* __restrict__ y, int lane, float& sa, float& sb,
                                              unsigned& sela, unsigned& selb) {
    int ia[U], ib[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int p = lane + 64 * u;
        ia[u] = p < da ? cpa[p] : -1;
        ib[u] = p < db ? cpb[p] : -1;
    }
    float va[U], vb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        va[u] = ia[u] >= 0 ? y[ia[u]] : 0.0f;
        vb[u] = ib[u] >= 0 ? y[ib[u]] : 0.0f;
    }
    float a = 0.0f, b = 0.0f;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        a += term<ABS>(va[u]);
        b += term<ABS>(vb[u]);
        if (ABS) {
            sela |= sign_of(va[u]);
            selb |= sign_of(vb[u]);
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
    }
    sa = a;
    sb = b;
}

// OR of a per-thread flag over an aligned group of G lanes of the wavefront.
template <int G>
__device__ __forceinline__ bool group_any(bool f) {
    if constexpr (G == 1) return f;
    const unsigned long long m = __ballot(f);
    if constexpr (G == 64) return m != 0ull;
    const int lane = threadIdx.x & 63;
    const unsigned long long gm = ((1ull << G) - 1ull) << (lane & ~(G - 1));
    return (m & gm) != 0ull;
}

}  // namespace gnk
