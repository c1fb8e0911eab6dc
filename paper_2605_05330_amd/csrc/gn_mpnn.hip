// Learned warm start: a two-layer message-passing network that predicts x0.
//
// The paper warm-starts GN from fractional LP solutions (Section 6); here a
// small network trained on GN's own results plays that role.  Definition
// (hidden width 64, vertices in the graph's internal order):
//   features  h0_i = [w_i, deg_i/10, w_i / max_{N[i]} w, S_i / (w_i + S_i)],  S_i = sum_{N(i)} w
//   layer 1   X1 = [h0 | mean_{N(i)} h0 | 0] (16 columns, bf16),  h1 = ReLU(X1 W1 + b1)
//   layer 2   X2 = [bf16(h1) | bf16(mean_{N(i)} bf16(h1))] (128 columns),  h2 = ReLU(X2 W2 + b2)
//   head      z = h2 . bf16(u) + c,  p = sigmoid(z),
//             x0 = clamp(p, 1e-3, 1) where |p - 1/2| > gate, else 1/2 (gate = 0: plain clamp)
//   loss      mean_i softplus(z_i) - l_i z_i   (binary cross-entropy with labels l)
// The products run on the matrix cores (v_mfma_f32_16x16x16_bf16: bf16
// operands, fp32 accumulation), one wavefront per 16-row tile.  Every sum over
// vertices in the backward pass is reduced in a fixed order, so gradients are
// bit-reproducible.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "gn_internal.h"
#include "gn_rowsum.h"

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int HID = 64;
constexpr int OFF_W1 = 0, OFF_B1 = 1024, OFF_W2 = 1088, OFF_B2 = 9280, OFF_U = 9344, OFF_C = 9408;
constexpr int NPARAMS = 9409;
constexpr int RED_BLOCKS = 256;   // fixed grid of the weight-gradient reductions
constexpr int HEAD_PART = 130;    // per tile: du[64], db2[64], dc, loss

__device__ __forceinline__ unsigned short f2bf(float f) {
    const unsigned u = __float_as_uint(f);
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }

__device__ __forceinline__ floatx4 mfma(bf16x4 a, bf16x4 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x4 ld_bf4(const unsigned short* p) {
    const uint2 v = *reinterpret_cast<const uint2*>(p);
    bf16x4 r;
    r[0] = (short)(v.x & 0xFFFF);
    r[1] = (short)(v.x >> 16);
    r[2] = (short)(v.y & 0xFFFF);
    r[3] = (short)(v.y >> 16);
    return r;
}

struct Cache {
    unsigned short* X1;   // n_pad x 16
    unsigned short* X2;   // n_pad x 128
    float* H2;            // n_pad x 64
    float* Z;             // n_pad
    float* F0;            // n_pad x 4
    float* invdeg;        // n_pad
    unsigned short* W1f;  // [nb 4][lane 64][4]
    unsigned short* W2f;  // [ks 8][nb 4][lane 64][4]
    unsigned short* W2Tf; // [ks 4][nb 8][lane 64][4]
    float* ub;            // 64: bf16-rounded u as float
    unsigned short* DP2;  // n_pad x 64
    float* dX2;           // n_pad x 128
    unsigned short* DP1;  // n_pad x 64
    float* headp;         // tiles x HEAD_PART
    float* w2p;           // RED_BLOCKS x 8192
    float* w1p;           // RED_BLOCKS x 1024
    float* b1p;           // blocks(dH1) x 64
    float* red;           // kGroups x 8192: stage-1 scratch of the fixed-order sums
    float* headsum;       // 130
};

inline size_t al(size_t b) { return (b + 255) & ~(size_t)255; }
inline int64_t npad_of(int32_t n) { return ((int64_t)n + 15) / 16 * 16; }
inline int64_t dh1_blocks(int64_t npad) { return (npad * 16 + 255) / 256; }

size_t cache_layout(int32_t n, char* base, Cache* c) {
    const int64_t np = npad_of(std::max(n, 1));
    const int64_t tiles = np / 16;
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        char* p = base ? base + off : nullptr;
        off += al(bytes);
        return p;
    };
    Cache t;
    t.X1 = (unsigned short*)take(np * 16 * 2);
    t.X2 = (unsigned short*)take(np * 128 * 2);
    t.H2 = (float*)take(np * 64 * 4);
    t.Z = (float*)take(np * 4);
    t.F0 = (float*)take(np * 4 * 4);
    t.invdeg = (float*)take(np * 4);
    t.W1f = (unsigned short*)take(4 * 64 * 4 * 2);
    t.W2f = (unsigned short*)take(8 * 4 * 64 * 4 * 2);
    t.W2Tf = (unsigned short*)take(4 * 8 * 64 * 4 * 2);
    t.ub = (float*)take(64 * 4);
    t.DP2 = (unsigned short*)take(np * 64 * 2);
    t.dX2 = (float*)take(np * 128 * 4);
    t.DP1 = (unsigned short*)take(np * 64 * 2);
    t.headp = (float*)take(tiles * HEAD_PART * 4);
    t.w2p = (float*)take((size_t)RED_BLOCKS * 8192 * 4);
    t.w1p = (float*)take((size_t)RED_BLOCKS * 1024 * 4);
    t.b1p = (float*)take(dh1_blocks(np) * 64 * 4);
    t.red = (float*)take((size_t)64 * 8192 * 4);
    t.headsum = (float*)take(HEAD_PART * 4);
    if (c) *c = t;
    return off;
}

// bf16 weights in MFMA fragment order: lane l of a B fragment holds
// B[4*(l/16) + j][l % 16], j = 0..3.
__global__ void params_kernel(const float* __restrict__ p, Cache c) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 4 * 64 * 4) {  // W1: B[k][n] = W1[k][n]
        const int j = t & 3, l = (t >> 2) & 63, nb = t >> 8;
        const int k = 4 * (l / 16) + j, nn = nb * 16 + l % 16;
        c.W1f[t] = f2bf(p[OFF_W1 + k * HID + nn]);
    }
    if (t < 8 * 4 * 64 * 4) {  // W2 forward: B[k = f][n = h] = W2[f][h]
        const int j = t & 3, l = (t >> 2) & 63, nb = (t >> 8) & 3, ks = t >> 10;
        const int f = ks * 16 + 4 * (l / 16) + j, h = nb * 16 + l % 16;
        c.W2f[t] = f2bf(p[OFF_W2 + f * HID + h]);
        // W2 transposed for dX2 = DP2 W2^T: B[k = h][n = f] = W2[f][h]
        const int nb2 = (t >> 8) & 7, ks2 = t >> 11;
        const int h2 = ks2 * 16 + 4 * (l / 16) + j, f2 = nb2 * 16 + l % 16;
        c.W2Tf[t] = f2bf(p[OFF_W2 + f2 * HID + h2]);
    }
    if (t < 64) c.ub[t] = bf2f(f2bf(p[OFF_U + t]));
}

// features of every row (thread per row) and 1/deg
__global__ void features_kernel(int32_t n, int64_t npad, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                const float* __restrict__ w, Cache c) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad) return;
    if (i >= n) {
        for (int q = 0; q < 4; ++q) c.F0[i * 4 + q] = 0.0f;
        c.invdeg[i] = 0.0f;
        return;
    }
    const int s = rp[i], e = rp[i + 1];
    const float wi = w[i];
    float S = 0.0f, m = wi;
    for (int q = s; q < e; ++q) {
        const float wj = w[col[q]];
        S += wj;
        m = fmaxf(m, wj);
    }
    const int d = e - s;
    c.F0[i * 4 + 0] = wi;
    c.F0[i * 4 + 1] = (float)d / 10.0f;
    c.F0[i * 4 + 2] = wi / m;
    c.F0[i * 4 + 3] = S / (wi + S);
    c.invdeg[i] = d > 0 ? 1.0f / (float)d : 0.0f;
}

// X1 = bf16 [h0 | mean_N h0 | 0]
__global__ void x1_kernel(int32_t n, int64_t npad, const int32_t* __restrict__ rp, const int32_t* __restrict__ col, Cache c) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad) return;
    unsigned short* x = c.X1 + i * 16;
    if (i >= n) {
        for (int q = 0; q < 16; ++q) x[q] = 0;
        return;
    }
    float a[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int q = rp[i]; q < rp[i + 1]; ++q) {
        const float4 f = *reinterpret_cast<const float4*>(c.F0 + (int64_t)col[q] * 4);
        a[0] += f.x;
        a[1] += f.y;
        a[2] += f.z;
        a[3] += f.w;
    }
    const float id = c.invdeg[i];
    for (int q = 0; q < 4; ++q) {
        x[q] = f2bf(c.F0[i * 4 + q]);
        x[4 + q] = f2bf(a[q] * id);
    }
    for (int q = 8; q < 16; ++q) x[q] = 0;
}

// layer 1 on the matrix cores: one wavefront per 16-row tile
__global__ __launch_bounds__(256) void layer1_kernel(int32_t n, int64_t tiles, const float* __restrict__ p, Cache c) {
    const int lane = threadIdx.x & 63;
    const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile >= tiles) return;
    const int64_t r0 = tile * 16;
    const bf16x4 a = ld_bf4(c.X1 + (r0 + lane % 16) * 16 + 4 * (lane / 16));
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        floatx4 d = {0.0f, 0.0f, 0.0f, 0.0f};
        d = mfma(a, ld_bf4(c.W1f + (nb * 64 + lane) * 4), d);
        const int colh = nb * 16 + lane % 16;
        const float bias = p[OFF_B1 + colh];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t row = r0 + 4 * (lane / 16) + j;
            const float h = fmaxf(d[j] + bias, 0.0f);
            c.X2[row * 128 + colh] = row < n ? f2bf(h) : (unsigned short)0;
        }
    }
}

// X2[:, 64:128] = bf16(mean_N X2[:, 0:64]); 16 lanes per row, 4 columns per lane
__global__ void agg_hidden_kernel(int32_t n, int64_t npad, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                  Cache c) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = t / 16;
    const int q = (int)(t % 16);
    if (i >= npad) return;
    unsigned short* dst = c.X2 + i * 128 + 64 + 4 * q;
    if (i >= n) {
        for (int k = 0; k < 4; ++k) dst[k] = 0;
        return;
    }
    float a[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        const bf16x4 v = ld_bf4(c.X2 + (int64_t)col[e] * 128 + 4 * q);
        for (int k = 0; k < 4; ++k) a[k] += bf2f((unsigned short)v[k]);
    }
    const float id = c.invdeg[i];
    for (int k = 0; k < 4; ++k) dst[k] = f2bf(a[k] * id);
}

// layer 2 + head: h2 = ReLU(X2 W2 + b2), z = h2 . u + c, x0 = clamp(sigmoid(z))
__global__ __launch_bounds__(256) void layer2_kernel(int32_t n, int64_t tiles, const float* __restrict__ p, Cache c,
                                                     const int32_t* __restrict__ perm, float* __restrict__ x0_user,
                                                     float* __restrict__ z_user, int store_h2, float gate) {
    const int lane = threadIdx.x & 63;
    const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile >= tiles) return;
    const int64_t r0 = tile * 16;
    floatx4 d[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) d[nb] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
        const bf16x4 a = ld_bf4(c.X2 + (r0 + lane % 16) * 128 + ks * 16 + 4 * (lane / 16));
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) d[nb] = mfma(a, ld_bf4(c.W2f + ((ks * 4 + nb) * 64 + lane) * 4), d[nb]);
    }
    float zp[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        const int colh = nb * 16 + lane % 16;
        const float bias = p[OFF_B2 + colh];
        const float uu = c.ub[colh];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t row = r0 + 4 * (lane / 16) + j;
            const float h = fmaxf(d[nb][j] + bias, 0.0f);
            if (store_h2) c.H2[row * 64 + colh] = row < n ? h : 0.0f;
            zp[j] = __fmaf_rn(h, uu, zp[j]);
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
        for (int off = 8; off >= 1; off >>= 1) zp[j] += __shfl_xor(zp[j], off, 64);
    if (lane % 16 == 0) {
        const float cc = p[OFF_C];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t row = r0 + 4 * (lane / 16) + j;
            if (row < n) {
                const float z = zp[j] + cc;
                c.Z[row] = z;
                const float sg = 1.0f / (1.0f + expf(-z));
                // gated start: keep the prediction only where it is confident
                x0_user[perm[row]] = fabsf(sg - 0.5f) > gate ? fminf(fmaxf(sg, 1e-3f), 1.0f) : 0.5f;
                if (z_user) z_user[perm[row]] = z;
            } else {
                c.Z[row] = 0.0f;
            }
        }
    }
}

// head backward per 16-row tile: dz, dpre2 (-> bf16 DP2) and tile partials of
// du, db2, dc and the loss.
__global__ __launch_bounds__(256) void head_back_kernel(int32_t n, int64_t tiles, const float* __restrict__ labels_user,
                                                        const int32_t* __restrict__ perm, Cache c) {
    const int lane = threadIdx.x & 63;
    const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile >= tiles) return;
    const int64_t r0 = tile * 16;
    const float inv_n = 1.0f / (float)n;
    float dz[4], lz[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t row = r0 + 4 * (lane / 16) + j;
        dz[j] = 0.0f;
        lz[j] = 0.0f;
        if (row < n) {
            const float z = c.Z[row];
            const float l = labels_user[perm[row]];
            const float sg = 1.0f / (1.0f + expf(-z));
            dz[j] = (sg - l) * inv_n;
            lz[j] = fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z))) - l * z;
        }
    }
    float* hp = c.headp + tile * HEAD_PART;
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        const int colh = nb * 16 + lane % 16;
        const float uu = c.ub[colh];
        float du = 0.0f, db = 0.0f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t row = r0 + 4 * (lane / 16) + j;
            const float h = c.H2[row * 64 + colh];
            const float dp = h > 0.0f ? dz[j] * uu : 0.0f;
            c.DP2[row * 64 + colh] = f2bf(dp);
            du = __fmaf_rn(h, dz[j], du);
            db += dp;
        }
        du += __shfl_xor(du, 16, 64);
        du += __shfl_xor(du, 32, 64);
        db += __shfl_xor(db, 16, 64);
        db += __shfl_xor(db, 32, 64);
        if (lane < 16) {
            hp[colh] = du;
            hp[64 + colh] = db;
        }
    }
    // dc and loss: each row's value is held by the 16 lanes of its group; take lane%16 == 0
    float sdz = 0.0f, sl = 0.0f;
    if (lane % 16 == 0)
        for (int j = 0; j < 4; ++j) {
            sdz += dz[j];
            sl += lz[j];
        }
    sdz += __shfl_xor(sdz, 16, 64);
    sdz += __shfl_xor(sdz, 32, 64);
    sl += __shfl_xor(sl, 16, 64);
    sl += __shfl_xor(sl, 32, 64);
    if (lane == 0) {
        hp[128] = sdz;
        hp[129] = sl * inv_n;
    }
}

// C = A^T B summed over all row tiles, A = X (tiles x 16 rows x MA*16 columns,
// bf16, row stride lda), B = DP (row stride 64 bf16, 64 columns).  Each
// wavefront of a fixed grid of RED_BLOCKS x 4 accumulates tiles w, w + 1024,
// ...; the four wavefronts of a block are summed in LDS in order and the block
// writes its partial (MA*16 x 64 floats).
template <int MA>
__global__ __launch_bounds__(256) void wgrad_kernel(int64_t tiles, const unsigned short* __restrict__ X, int lda,
                                                    const unsigned short* __restrict__ DP, float* __restrict__ part) {
    __shared__ float red[MA * 16 * 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    floatx4 acc[MA][4];
#pragma unroll
    for (int mb = 0; mb < MA; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) acc[mb][nb] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < tiles; tile += (int64_t)RED_BLOCKS * 4) {
        const int64_t rbase = tile * 16 + 4 * (lane / 16);
        bf16x4 b[4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
#pragma unroll
            for (int j = 0; j < 4; ++j) b[nb][j] = (short)DP[(rbase + j) * 64 + nb * 16 + lane % 16];
#pragma unroll
        for (int mb = 0; mb < MA; ++mb) {
            bf16x4 a;
#pragma unroll
            for (int j = 0; j < 4; ++j) a[j] = (short)X[(rbase + j) * lda + mb * 16 + lane % 16];
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) acc[mb][nb] = mfma(a, b[nb], acc[mb][nb]);
        }
    }
    // lane holds C[mb*16 + 4*(lane/16) + j][nb*16 + lane%16]
    for (int w = 0; w < 4; ++w) {
        if (wave == w) {
#pragma unroll
            for (int mb = 0; mb < MA; ++mb)
#pragma unroll
                for (int nb = 0; nb < 4; ++nb)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int idx = (mb * 16 + 4 * (lane / 16) + j) * 64 + nb * 16 + lane % 16;
                        red[idx] = (w == 0 ? 0.0f : red[idx]) + acc[mb][nb][j];
                    }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < MA * 16 * 64; e += 256) part[(int64_t)blockIdx.x * MA * 16 * 64 + e] = red[e];
}

// dX2 = DP2 W2^T on the matrix cores (one wavefront per 16-row tile)
__global__ __launch_bounds__(256) void dx2_kernel(int64_t tiles, Cache c) {
    const int lane = threadIdx.x & 63;
    const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile >= tiles) return;
    const int64_t r0 = tile * 16;
    floatx4 d[8];
#pragma unroll
    for (int nb = 0; nb < 8; ++nb) d[nb] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        const bf16x4 a = ld_bf4(c.DP2 + (r0 + lane % 16) * 64 + ks * 16 + 4 * (lane / 16));
#pragma unroll
        for (int nb = 0; nb < 8; ++nb) d[nb] = mfma(a, ld_bf4(c.W2Tf + ((ks * 8 + nb) * 64 + lane) * 4), d[nb]);
    }
#pragma unroll
    for (int nb = 0; nb < 8; ++nb)
#pragma unroll
        for (int j = 0; j < 4; ++j) c.dX2[(r0 + 4 * (lane / 16) + j) * 128 + nb * 16 + lane % 16] = d[nb][j];
}

// dpre1 = (dX2[:, :64] + sum_{j in N(i)} dX2[j, 64:] / deg_j) * [h1 > 0] -> bf16 DP1,
// plus block partials of db1.  16 lanes per row, 4 columns per lane.
__global__ __launch_bounds__(256) void dh1_kernel(int32_t n, int64_t npad, const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ col, Cache c) {
    __shared__ float red[16][64];
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t i = t / 16;
    const int q = threadIdx.x % 16;
    float dp[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (i < npad) {
        if (i < n) {
            const float4 own = *reinterpret_cast<const float4*>(c.dX2 + i * 128 + 4 * q);
            float a[4] = {own.x, own.y, own.z, own.w};
            for (int e = rp[i]; e < rp[i + 1]; ++e) {
                const int j = col[e];
                const float s = c.invdeg[j];
                const float4 g = *reinterpret_cast<const float4*>(c.dX2 + (int64_t)j * 128 + 64 + 4 * q);
                a[0] = __fmaf_rn(g.x, s, a[0]);
                a[1] = __fmaf_rn(g.y, s, a[1]);
                a[2] = __fmaf_rn(g.z, s, a[2]);
                a[3] = __fmaf_rn(g.w, s, a[3]);
            }
            for (int k = 0; k < 4; ++k) dp[k] = bf2f(c.X2[i * 128 + 4 * q + k]) > 0.0f ? a[k] : 0.0f;
        }
        for (int k = 0; k < 4; ++k) c.DP1[i * 64 + 4 * q + k] = f2bf(dp[k]);
    }
    // db1 block partial: rows of this block in order
    const int rl = threadIdx.x / 16;
    for (int k = 0; k < 4; ++k) red[rl][4 * q + k] = dp[k];
    __syncthreads();
    if (threadIdx.x < 64) {
        float s = 0.0f;
        for (int r = 0; r < 16; ++r) s += red[r][threadIdx.x];
        c.b1p[(int64_t)blockIdx.x * 64 + threadIdx.x] = s;
    }
}

// Fixed-order sum of `parts` partial vectors: out[e] = sum_p in[p * stride + e].
// Stage 1: group g of kGroups sums its contiguous run of parts in order into
// scratch[g][e]; stage 2 sums the groups in order.  Same order on every run.
constexpr int kGroups = 64;

__global__ void sum_parts_stage1(int64_t parts, int64_t stride, int32_t len, const float* __restrict__ in,
                                 float* __restrict__ scratch) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int g = blockIdx.y;
    if (e >= len) return;
    const int64_t per = (parts + kGroups - 1) / kGroups;
    const int64_t p0 = g * per, p1 = min(parts, p0 + per);
    float s = 0.0f;
    for (int64_t p = p0; p < p1; ++p) s += in[p * stride + e];
    scratch[(int64_t)g * len + e] = s;
}

__global__ void sum_parts_stage2(int32_t len, const float* __restrict__ scratch, float* __restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= len) return;
    float s = 0.0f;
    for (int g = 0; g < kGroups; ++g) s += scratch[(int64_t)g * len + e];
    out[e] = s;
}

void sum_parts(int64_t parts, int64_t stride, int32_t len, const float* in, float* out, float* scratch, hipStream_t s) {
    const unsigned bx = (unsigned)((len + 255) / 256);
    hipLaunchKernelGGL(sum_parts_stage1, dim3(bx, kGroups), dim3(256), 0, s, parts, stride, len, in, scratch);
    hipLaunchKernelGGL(sum_parts_stage2, dim3(bx), dim3(256), 0, s, len, (const float*)scratch, out);
}

__global__ void assemble_grad_kernel(const float* __restrict__ head, float* __restrict__ grad, float* __restrict__ loss) {
    // head holds [du 64, db2 64, dc, loss] already summed over tiles
    const int t = threadIdx.x;
    if (t < 64) {
        grad[OFF_U + t] = head[t];
        grad[OFF_B2 + t] = head[64 + t];
    }
    if (t == 0) {
        grad[OFF_C] = head[128];
        *loss = head[129];
    }
}

__global__ void adam_kernel(int32_t count, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, float lr, float b1, float b2, float eps, float bc1, float bc2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / bc1;
    const float vh = vi / bc2;
    p[i] = p[i] - lr * mh / (sqrtf(vh) + eps);
}

}  // namespace

extern "C" int64_t gn_mpnn_cache_bytes(int32_t n) {
    if (n < 0) return -1;
    return (int64_t)cache_layout(n, nullptr, nullptr);
}

extern "C" gn_status gn_mpnn_forward(const gn_graph* g, const float* params, float gate, float* x0, float* z,
                                     void* cache, hipStream_t s) {
    if (!g || !params || !cache || (g->n > 0 && !x0) || !(gate >= 0.0f && gate < 0.5f)) return GN_E_ARG;
    const int32_t n = g->n;
    if (n == 0) return GN_OK;
    Cache c;
    cache_layout(n, (char*)cache, &c);
    const int64_t np = npad_of(n), tiles = np / 16;
    hipLaunchKernelGGL(params_kernel, dim3(32), dim3(256), 0, s, params, c);
    hipLaunchKernelGGL(features_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, n, np, g->row_ptr, g->col,
                       g->w_int, c);
    hipLaunchKernelGGL(x1_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, n, np, g->row_ptr, g->col, c);
    hipLaunchKernelGGL(layer1_kernel, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, s, n, tiles, params, c);
    hipLaunchKernelGGL(agg_hidden_kernel, dim3((unsigned)((np * 16 + 255) / 256)), dim3(256), 0, s, n, np, g->row_ptr,
                       g->col, c);
    hipLaunchKernelGGL(layer2_kernel, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, s, n, tiles, params, c, g->perm,
                       x0, z, 1, gate);
    GN_HIP_TRY(hipGetLastError());
    return GN_OK;
}

extern "C" gn_status gn_mpnn_backward(const gn_graph* g, const float* params, const float* labels, void* cache,
                                      float* grad, float* loss, hipStream_t s) {
    if (!g || !params || !cache || !grad || !loss || (g->n > 0 && !labels)) return GN_E_ARG;
    const int32_t n = g->n;
    if (n == 0) return GN_E_ARG;
    Cache c;
    cache_layout(n, (char*)cache, &c);
    const int64_t np = npad_of(n), tiles = np / 16;
    hipLaunchKernelGGL(head_back_kernel, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, s, n, tiles, labels, g->perm,
                       c);
    // du, db2, dc, loss: fixed-order sum of the tile partials
    sum_parts(tiles, (int64_t)HEAD_PART, HEAD_PART, c.headp, c.headsum, c.red, s);
    hipLaunchKernelGGL(assemble_grad_kernel, dim3(1), dim3(64), 0, s, (const float*)c.headsum, grad, loss);
    // dW2 = X2^T DP2
    hipLaunchKernelGGL(wgrad_kernel<8>, dim3(RED_BLOCKS), dim3(256), 0, s, tiles, c.X2, 128, c.DP2, c.w2p);
    sum_parts((int64_t)RED_BLOCKS, (int64_t)8192, 8192, c.w2p, grad + OFF_W2, c.red, s);
    // dX2, dpre1 (+ db1), dW1
    hipLaunchKernelGGL(dx2_kernel, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, s, tiles, c);
    const int64_t nb1 = dh1_blocks(np);
    hipLaunchKernelGGL(dh1_kernel, dim3((unsigned)nb1), dim3(256), 0, s, n, np, g->row_ptr, g->col, c);
    sum_parts(nb1, (int64_t)64, 64, c.b1p, grad + OFF_B1, c.red, s);
    hipLaunchKernelGGL(wgrad_kernel<1>, dim3(RED_BLOCKS), dim3(256), 0, s, tiles, c.X1, 16, c.DP1, c.w1p);
    sum_parts((int64_t)RED_BLOCKS, (int64_t)1024, 1024, c.w1p, grad + OFF_W1, c.red, s);
    GN_HIP_TRY(hipGetLastError());
    return GN_OK;
}

extern "C" gn_status gn_adam_step(float* params, const float* grad, float* m, float* v, int32_t count, float lr,
                                  float beta1, float beta2, float eps, int32_t t, hipStream_t s) {
    if (!params || !grad || !m || !v || count < 0 || t < 1 || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) ||
        !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return GN_E_ARG;
    if (count == 0) return GN_OK;
    const float bc1 = (float)(1.0 - std::pow((double)beta1, (double)t));
    const float bc2 = (float)(1.0 - std::pow((double)beta2, (double)t));
    hipLaunchKernelGGL(adam_kernel, dim3((count + 255) / 256), dim3(256), 0, s, count, params, grad, m, v, lr, beta1,
                       beta2, eps, bc1, bc2);
    GN_HIP_TRY(hipGetLastError());
    return GN_OK;
}
