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

// ---------------------------------------------------------------------------
// State words.  Every solver keeps the weighted state y_i = v_i x_i in one
// 32-bit word per vertex:
//   * y_i >= 2^-100: the fp32 value, with the sign bit set when x_i > 1/2 (the
//     rounded set S that the neighbours' cover test reads);
//   * y_i = 0: +0;
//   * 0 < y_i < 2^-100: a "log word", a positive word below the bits of 2^-100
//     that holds log2 x_i in fixed point, q = (log2 x_i + 1022) 2^17, as q + 1.
// Support invariance (Section 2, property ii): a positive coordinate never
// becomes zero.  Without the log form fp32 would lose it below 2^-149, and any
// floor in the fp32 range changes when a deeply decayed vertex can regrow; with
// it x_i is carried at its own magnitude down to 2^-1022 (fp64's smallest
// normal number), where it is held.
// Read as a float, a log word is below 2^-100, like the value it stands for, so
// neighbour sums add it as is: a closed-neighbourhood sum that takes the
// quotient branch exceeds 1e-9, and deg 2^-100 is far below its last bit.
// For a row whose own word is a log word, s_i > 1e-9 makes its own term
// negligible and x'_i = x_i v_i / s_i: the update adds log2(v_i / s_i).
constexpr uint32_t kLogTop = 0x0D800000u;      // bits of 2^-100
constexpr float kYLog = 0x1p-100f;             // smallest ordinary |y|
constexpr float kLogScale = 131072.0f;         // 2^17 fixed-point steps per unit of log2
constexpr int32_t kLogFloorQ = 1022 * 131072;  // q offset: log2 x = q / 2^17 - 1022
constexpr int32_t kLogQMax = (int32_t)kLogTop - 2;

__device__ __forceinline__ uint32_t mag_bits(float w) { return __float_as_uint(w) & 0x7fffffffu; }
__device__ __forceinline__ bool is_log_mag(uint32_t mag) { return mag - 1u < kLogTop - 1u; }

// log word of fixed-point q (clamped: q < 0 is the 2^-1022 floor)
__device__ __forceinline__ float log_word(int32_t q) {
    q = q < 0 ? 0 : (q > kLogQMax ? kLogQMax : q);
    return __uint_as_float((uint32_t)q + 1u);
}
// log2 x of a log word's q, as fp32 (exact while |log2 x| < 128)
__device__ __forceinline__ float log_q_value(int32_t q) { return (float)(q - kLogFloorQ) * (1.0f / kLogScale); }
__device__ __forceinline__ int32_t log_fixed(float l) { return __float2int_rn(l * kLogScale); }

// log2 and 2^a by the hardware instructions, for arguments where they return
// what log2f and exp2f return: lg2n for positive normal numbers (every caller
// passes v_i = sqrt(w_i) >= 2^-75, s_i > 1e-9 or |y_i| >= 2^-100), ex2n for
// a >= -126 (a normal result).  log2f and exp2f add a rescaling for the
// subnormal range to every call, a dozen instructions per log-form row.
__device__ __forceinline__ float lg2n(float a) { return __builtin_amdgcn_logf(a); }
__device__ __forceinline__ float ex2n(float a) { return __builtin_amdgcn_exp2f(a); }

// Word of a state whose log2 x is q / 2^17 - 1022, in its ordinary form when
// v 2^(log2 x) >= 2^-100.  Only called for states far below 1/2.
__device__ __forceinline__ float word_from_log(int32_t q, float vi) {
    q = q < 0 ? 0 : q;
    const float ly = log_q_value(q) + lg2n(vi);
    if (ly >= -100.0f) {
        const float yn = ex2n(ly);
        if (yn >= kYLog) return yn;
    }
    return log_word(q);
}

// Word of y = v x for a user coordinate x >= 0 (finite).
__device__ __forceinline__ float word_from_x(float x, float vi) {
    const float yy = vi * x;
    if (yy >= kYLog) return x > 0.5f ? -yy : yy;
    if (!(x > 0.0f)) return 0.0f;
    const float lx = x < 0x1p-126f ? log2f(x * 0x1p64f) - 64.0f : log2f(x);
    return word_from_log(log_fixed(lx) + kLogFloorQ, vi);
}

// x of a word (fp32; a log word deeper than 2^-149 reads as 0).
__device__ __forceinline__ float x_of_word(float w, float vi) {
    const uint32_t mag = mag_bits(w);
    if (!is_log_mag(mag)) return __uint_as_float(mag) / vi;
    return exp2f(log_q_value((int32_t)mag - 1));
}

// |y| of a word (fp32; deep log words read as 0).
__device__ __forceinline__ float y_of_word(float w, float vi) {
    const uint32_t mag = mag_bits(w);
    if (!is_log_mag(mag)) return __uint_as_float(mag);
    return exp2f(log_q_value((int32_t)mag - 1) + log2f(vi));
}

// One WRGN update of a row (WRGN definition with the safe division of the code
// appendix) from its own word and s_i = |y_i| + gamma sum_j |y_j|: returns the
// new word.
__device__ __forceinline__ float step_word(float yraw, float vi, float s) {
    if (!(s > 1e-9f)) return vi * 0.5f;  // safe-division reset: x' = 1/2
    const uint32_t mag = mag_bits(yraw);
    if (!is_log_mag(mag)) {
        const float yi = __uint_as_float(mag);
        const float xn = yi / s;
        const float yn = vi * xn;
        if (yn >= kYLog || mag == 0u) return xn > 0.5f ? -yn : yn;
        // below 2^-100: log2 x' = log2 y - log2 s
        return word_from_log(log_fixed(lg2n(yi)) - log_fixed(lg2n(s)) + kLogFloorQ, vi);
    }
    return word_from_log((int32_t)mag - 1 + log_fixed(lg2n(vi) - lg2n(s)), vi);
}

// x'_i in fp32 of that update, w its new word: the quotient y_i / s_i itself
// for an ordinary word, 1/2 on the reset, the log word's value otherwise.
// Called only where x' is an output, so the solves do not pay for it.
__device__ __forceinline__ float step_x(float yraw, float vi, float s, float w) {
    if (!(s > 1e-9f)) return 0.5f;
    const uint32_t mag = mag_bits(yraw);
    if (!is_log_mag(mag)) return __uint_as_float(mag) / s;
    return x_of_word(w, vi);
}

// Group of G threads sums one row of degree d <= MAXD.  `t` is the thread's
// index inside the group.  Returns the canonical sum (valid in every thread of
// the group) and ORs the sign bits (rounded-set membership) of the neighbours
// into `sel` (per thread; the caller reduces it over the group).
// Values entering a sum: |y| for the sign-carrying state (ABS), raw values for
// signed adjoint vectors.  Column ids are int32, or uint16 for a graph of at most
// 65536 vertices whose columns are staged in LDS.
// A state word enters a neighbour sum as |y| when it is ordinary (y >= 2^-100);
// log words and zeros add nothing (their values are below 2^-100, far below
// the last bit of any sum that takes the quotient branch).
__device__ __forceinline__ float nbr_term(float w) {
    const float a = fabsf(w);
    return a >= kYLog ? a : 0.0f;
}
template <bool ABS>
__device__ __forceinline__ float term(float v) { return ABS ? nbr_term(v) : v; }

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
