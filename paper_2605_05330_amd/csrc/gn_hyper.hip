// GN under hyperedge constraints (the hypergraph extension left to future work
// in the Conclusion; no formula in the paper).  Hyperedges are clique
// constraints, at most one selected vertex each, and every vertex is
// normalised by the mass of the hyperedges holding it, as the
// cross-normalization of the assignment problem (Section 2) does with rows and
// columns:
//
//     Y_e = sum_{j in e} y_j,   s_i = y_i + gamma * sum_{e holds i} (Y_e - y_i),
//
// x'_i = y_i / s_i with the safe division of the WRGN step.  States are kept in
// x space with the library's state-word log form for x < 2^-100 (the words of
// gn_rowsum.h with v = 1), so support invariance holds at each coordinate's own
// magnitude down to 2^-1022.
// This is WRGN on the conflict graph whose edge (i, j) counts the hyperedges
// holding both, at O(memberships) per step instead of O(conflict edges).
//
// A step is two launches: a wavefront per hyperedge forms Y_e and the count of
// members above 1/2; a thread per vertex sums its hyperedges and writes x'.  In
// a solve, the vertex kernel of step k also evaluates the stopping test of
// gn_solve on x^k (tau, uncovered, growing) into a per-step violation count,
// and the hyperedge kernel of step k+1 stops the solve when step k was a check
// step with no violation: every later launch then returns at once, so the host
// enqueues the steps in chains and looks at the stop flag between chains.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "gn_internal.h"
#include "gn_rowsum.h"

namespace {

constexpr int kHWaves = 4;           // hyperedges per workgroup
constexpr int kHBlock = 64 * kHWaves;
constexpr int kHVBlock = 256;        // vertex kernels
constexpr size_t kHPinState = 1024;  // byte offset of the marks' copies of the starts' HState in the pinned block
constexpr float kSafeDiv = 1e-9f;    // safe division threshold of the WRGN step

// x-space state words: an ordinary fp32 x >= 2^-100 (or 0), never signed, else
// the log form.
__device__ __forceinline__ float hx_word_from_x(float x) { return fabsf(gnk::word_from_x(x, 1.0f)); }
__device__ __forceinline__ float hx_value(float w) { return gnk::x_of_word(w, 1.0f); }

struct HState {
    int32_t done;
    int32_t step;
    int32_t binarised;
    int32_t pad;
    unsigned long long fallback;
};

struct HPart {
    double relaxed;
    double W;
    long long size;
    long long uncovered;
    long long conflicts;
    float stab;
    int32_t pad;
};

struct HArgs {
    const float* v;
    const float* w;
    const int32_t* eptr;
    const int32_t* emem;
    const int32_t* vptr;
    const int32_t* vedge;
    float* Y;          // [S][m]
    int32_t* cnt;      // [S][m] members with x > 1/2
    float* vs;         // [S][m] sum of v over selected members (final statistics)
    int32_t* viol;     // [S][vstride], vstride = max_steps + 1
    HState* st;        // [S]
    HPart* part;       // [S][nparts]
    int32_t n, m, nbv, nbe, nparts, vstride;
    int32_t check_every;
    float tau;
};

// Per start, by value: the buffer holding its final state (0 or 1) and gamma
// of its final step.
struct HFinal {
    int32_t buf[GN_MAX_STARTS];
    float gamma[GN_MAX_STARTS];
};

__device__ __forceinline__ float hwave_sum(float v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int hwave_sum_i(int v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Hyperedge sums of y = v x and counts of members above 1/2 for start
// blockIdx.y (states start-major, n apart).  In a solve (solve = 1) the launch
// of step k first settles the start's check of step k - 1.
__global__ __launch_bounds__(kHBlock) void hyper_edge_kernel(HArgs a, const float* x, int32_t k, int32_t solve) {
    const int s = blockIdx.y;
    if (solve) {
        HState* st = a.st + s;
        if (st->done) return;
        const int kp = k - 1;
        if (kp >= 1 && kp % a.check_every == 0 && a.viol[(size_t)s * a.vstride + kp] == 0) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                st->step = kp;
                st->binarised = 1;
                st->done = 1;
            }
            return;
        }
    }
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int e = blockIdx.x * kHWaves + wave;
    if (e >= a.m) return;
    x += (size_t)s * a.n;
    float Y = 0.0f;
    int c = 0;
    for (int j = a.eptr[e] + lane; j < a.eptr[e + 1]; j += 64) {
        const int i = a.emem[j];
        const float xi = x[i];
        Y += a.v[i] * xi;
        c += xi > 0.5f ? 1 : 0;
    }
    Y = hwave_sum(Y);
    c = hwave_sum_i(c);
    if (lane == 0) {
        a.Y[(size_t)s * a.m + e] = Y;
        a.cnt[(size_t)s * a.m + e] = c;
    }
}

// x' from the hyperedge sums (write = 1), and in a solve at a check step the
// stopping test on x (check = 1), counted into the start's viol[k] once per
// workgroup.
__global__ __launch_bounds__(kHVBlock) void hyper_vertex_kernel(HArgs a, const float* x, float* xo, float gamma,
                                                               int32_t k, int32_t solve, int32_t check,
                                                               int32_t write) {
    const int s = blockIdx.y;
    if (solve && a.st[s].done) return;
    const int i = blockIdx.x * kHVBlock + threadIdx.x;
    const float* Ys = a.Y + (size_t)s * a.m;
    const int32_t* cs = a.cnt + (size_t)s * a.m;
    bool bad = false, fb = false;
    if (i < a.n) {
        const float xi = x[(size_t)s * a.n + i];
        const float vi = a.v[i];
        const float y = vi * xi;
        float nb = 0.0f;
        int cov = 0;
        for (int q = a.vptr[i]; q < a.vptr[i + 1]; ++q) {
            const int e = a.vedge[q];
            nb += Ys[e] - y;
            cov += cs[e];
        }
        const float sv = gamma * nb + y;
        if (write) {
            float xn;
            if (sv > kSafeDiv) {
                const uint32_t mag = gnk::mag_bits(xi);
                if (!gnk::is_log_mag(mag)) {
                    xn = y / sv;
                    if (xn < gnk::kYLog && mag != 0u)   // below 2^-100: log2 x' = log2 x + log2 v - log2 s
                        xn = gnk::word_from_log(gnk::log_fixed(log2f(xi) + log2f(vi) - log2f(sv)) + gnk::kLogFloorQ,
                                                1.0f);
                } else {
                    xn = gnk::word_from_log((int32_t)mag - 1 + gnk::log_fixed(log2f(vi) - log2f(sv)), 1.0f);
                }
            } else {
                xn = 0.5f;
                fb = true;
            }
            xo[(size_t)s * a.n + i] = xn;
        }
        if (check) {
            const float d = fminf(xi, 1.0f - xi);
            bad = d > a.tau;
            if (xi <= 0.5f) {
                bad = bad || cov == 0;                        // uncovered
                bad = bad || (xi > 0.0f && !(sv > vi));        // growing
            }
        }
    }
    if (solve && write) {
        const unsigned long long nf = __popcll(__ballot(fb));
        if (nf && (threadIdx.x & 63) == 0) atomicAdd(&a.st[s].fallback, nf);
    }
    if (check) {
        if (__syncthreads_or(bad ? 1 : 0) && threadIdx.x == 0) atomicAdd(&a.viol[(size_t)s * a.vstride + k], 1);
    }
}

// User states (x >= 0, checked on the host) to x-space state words.
__global__ void hyper_prep_kernel(int64_t count, const float* __restrict__ x, float* __restrict__ xw) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) xw[e] = hx_word_from_x(x[e]);
}

// x-space state words to user states.
__global__ void hyper_value_kernel(int64_t count, const float* __restrict__ xw, float* __restrict__ x) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) x[e] = hx_value(xw[e]);
}

// A start that ran to max_steps: the check of x^max_steps decides.
__global__ void hyper_resolve_kernel(HArgs a, int32_t max_steps, int32_t checked) {
    HState* st = a.st + blockIdx.x;
    if (st->done) return;
    st->step = max_steps;
    st->binarised = (checked && a.viol[(size_t)blockIdx.x * a.vstride + max_steps] == 0) ? 1 : 0;
    st->done = 1;
}

// Final statistics, part 1: per hyperedge the selected count and the sum of v
// over its selected members; per workgroup the conflicts (pairs of selected
// members, counted per hyperedge).
__global__ __launch_bounds__(kHBlock) void hyper_stats_edge_kernel(HArgs a, const float* buf0, const float* buf1,
                                                                  HFinal f) {
    __shared__ long long red[kHWaves];
    const int s = blockIdx.y;
    const float* x = (f.buf[s] ? buf1 : buf0) + (size_t)s * a.n;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int e = blockIdx.x * kHWaves + wave;
    long long conf = 0;
    if (e < a.m) {
        float vs = 0.0f;
        int c = 0;
        for (int j = a.eptr[e] + lane; j < a.eptr[e + 1]; j += 64) {
            const int i = a.emem[j];
            if (fminf(fmaxf(x[i], 0.0f), 1.0f) > 0.5f) {
                vs += a.v[i];
                ++c;
            }
        }
        vs = hwave_sum(vs);
        c = hwave_sum_i(c);
        if (lane == 0) {
            a.vs[(size_t)s * a.m + e] = vs;
            a.cnt[(size_t)s * a.m + e] = c;
        }
        conf = (long long)c * (c - 1) / 2;
    }
    if (lane == 0) red[wave] = conf;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long t = 0;
        for (int q = 0; q < kHWaves; ++q) t += red[q];
        a.part[(size_t)s * a.nparts + blockIdx.x].conflicts = t;
    }
}

// Part 2: the clamped state and the set, per-workgroup sums of the relaxed
// objective, W(S), |S|, the uncovered vertices and the minimum stability term
// gamma * sum_{e holds i} (sum of v over e's selected members) / v_i over i
// outside S.  The conflicts of part 1 are kept in the same slot.
__global__ __launch_bounds__(kHVBlock) void hyper_stats_vertex_kernel(HArgs a, const float* buf0, const float* buf1,
                                                                     HFinal f, float* x_user, uint8_t* sel) {
    __shared__ HPart red[kHVBlock / 64];
    const int s = blockIdx.y;
    const float* x = (f.buf[s] ? buf1 : buf0) + (size_t)s * a.n;
    const float gamma = f.gamma[s];
    const float* vss = a.vs + (size_t)s * a.m;
    const int32_t* cs = a.cnt + (size_t)s * a.m;
    const int i = blockIdx.x * kHVBlock + threadIdx.x;
    double rel = 0.0, W = 0.0;
    long long sz = 0, unc = 0;
    float stab = INFINITY;
    if (i < a.n) {
        const float xc = fminf(fmaxf(hx_value(x[i]), 0.0f), 1.0f);
        const bool in = xc > 0.5f;
        x_user[(size_t)s * a.n + i] = xc;
        sel[(size_t)s * a.n + i] = in ? 1 : 0;
        const float wi = a.w[i];
        rel = (double)wi * (double)xc;
        if (in) {
            W = (double)wi;
            sz = 1;
        } else {
            int cov = 0;
            float t = 0.0f;
            for (int q = a.vptr[i]; q < a.vptr[i + 1]; ++q) {
                const int e = a.vedge[q];
                cov += cs[e];
                t += vss[e];
            }
            unc = cov == 0 ? 1 : 0;
            stab = gamma * t / a.v[i];
        }
    }
    for (int o = 32; o >= 1; o >>= 1) {
        rel += __shfl_xor(rel, o, 64);
        W += __shfl_xor(W, o, 64);
        sz += __shfl_xor(sz, o, 64);
        unc += __shfl_xor(unc, o, 64);
        stab = fminf(stab, __shfl_xor(stab, o, 64));
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[w].relaxed = rel;
        red[w].W = W;
        red[w].size = sz;
        red[w].uncovered = unc;
        red[w].stab = stab;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        HPart t{};
        t.stab = INFINITY;
        for (int q = 0; q < kHVBlock / 64; ++q) {
            t.relaxed += red[q].relaxed;
            t.W += red[q].W;
            t.size += red[q].size;
            t.uncovered += red[q].uncovered;
            t.stab = fminf(t.stab, red[q].stab);
        }
        HPart& o = a.part[(size_t)s * a.nparts + blockIdx.x];
        o.relaxed = t.relaxed;
        o.W = t.W;
        o.size = t.size;
        o.uncovered = t.uncovered;
        o.stab = t.stab;
    }
}

// Part 3: one workgroup per start reduces its partials in a fixed order.
__global__ __launch_bounds__(256) void hyper_stats_finish_kernel(HArgs a, HPart* out) {
    __shared__ HPart red[256 / 64];
    const int s = blockIdx.x;
    const HPart* part = a.part + (size_t)s * a.nparts;
    HPart t{};
    t.stab = INFINITY;
    const int nb = max(a.nbv, a.nbe);
    for (int q = threadIdx.x; q < nb; q += 256) {
        const HPart& p = part[q];
        if (q < a.nbv) {
            t.relaxed += p.relaxed;
            t.W += p.W;
            t.size += p.size;
            t.uncovered += p.uncovered;
            t.stab = fminf(t.stab, p.stab);
        }
        if (q < a.nbe) t.conflicts += p.conflicts;
    }
    for (int o = 32; o >= 1; o >>= 1) {
        t.relaxed += __shfl_xor(t.relaxed, o, 64);
        t.W += __shfl_xor(t.W, o, 64);
        t.size += __shfl_xor(t.size, o, 64);
        t.uncovered += __shfl_xor(t.uncovered, o, 64);
        t.conflicts += __shfl_xor(t.conflicts, o, 64);
        t.stab = fminf(t.stab, __shfl_xor(t.stab, o, 64));
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        HPart r{};
        r.stab = INFINITY;
        for (int q = 0; q < 256 / 64; ++q) {
            r.relaxed += red[q].relaxed;
            r.W += red[q].W;
            r.size += red[q].size;
            r.uncovered += red[q].uncovered;
            r.conflicts += red[q].conflicts;
            r.stab = fminf(r.stab, red[q].stab);
        }
        out[s] = r;
    }
}

}  // namespace

struct gn_hyper {
    int device = 0;
    int32_t n = 0, m = 0;
    int64_t nnzc = 0;
    std::vector<int32_t> eptr_h, emem_h, vptr_h, vedge_h;  // host copies (normalizable check)
    std::vector<float> v_h;
    float* v = nullptr;
    float* w = nullptr;
    int32_t* eptr = nullptr;
    int32_t* emem = nullptr;
    int32_t* vptr = nullptr;
    int32_t* vedge = nullptr;
    float* Y = nullptr;      // [GN_MAX_STARTS][m]
    int32_t* cnt = nullptr;
    float* vs = nullptr;
    float* buf[2] = {nullptr, nullptr};  // [GN_MAX_STARTS][n] each
    int32_t* viol = nullptr;             // [GN_MAX_STARTS][viol_cap]
    int32_t viol_cap = 0;
    HState* st = nullptr;                // [GN_MAX_STARTS]
    HPart* part = nullptr;               // [GN_MAX_STARTS][nparts]
    HPart* out = nullptr;                // [GN_MAX_STARTS]
    void* host = nullptr;                // pinned: HState[GN_MAX_STARTS] + HPart[GN_MAX_STARTS]
    // Captured chains of steps (the steps' gamma, test steps and the start
    // count are baked in, so the chains are kept for one schedule), their
    // pinned block, and a solve state that never stops them by itself: the
    // starts' own flags do, through the marks' copies.
    GraphWorkspace ws;
    struct ChainKey {
        int32_t starts, ms, ramp, check_every, vstride;
        float g0, g1, tau;
        const int32_t* viol;
        bool operator==(const ChainKey& o) const {
            return starts == o.starts && ms == o.ms && ramp == o.ramp && check_every == o.check_every &&
                   vstride == o.vstride && g0 == o.g0 && g1 == o.g1 && tau == o.tau && viol == o.viol;
        }
    } key{};
};

static void hyper_free(gn_hyper* h) {
    hipFree(h->v);
    hipFree(h->w);
    hipFree(h->eptr);
    hipFree(h->emem);
    hipFree(h->vptr);
    hipFree(h->vedge);
    hipFree(h->Y);
    hipFree(h->cnt);
    hipFree(h->vs);
    hipFree(h->buf[0]);
    hipFree(h->buf[1]);
    hipFree(h->viol);
    hipFree(h->st);
    hipFree(h->part);
    hipFree(h->out);
    if (h->host) hipHostFree(h->host);
    h->ws.destroy_chains();
    hipFree(h->ws.state);
    if (h->ws.host_pinned) hipHostFree(h->ws.host_pinned);
}

static int32_t hyper_nbv(int32_t n) { return (n + kHVBlock - 1) / kHVBlock; }
static int32_t hyper_nbe(int32_t m) { return (m + kHWaves - 1) / kHWaves; }

static HArgs hyper_args(gn_hyper* h) {
    HArgs a;
    a.v = h->v;
    a.w = h->w;
    a.eptr = h->eptr;
    a.emem = h->emem;
    a.vptr = h->vptr;
    a.vedge = h->vedge;
    a.Y = h->Y;
    a.cnt = h->cnt;
    a.vs = h->vs;
    a.viol = h->viol;
    a.st = h->st;
    a.part = h->part;
    a.n = h->n;
    a.m = h->m;
    a.nbv = hyper_nbv(h->n);
    a.nbe = hyper_nbe(h->m);
    a.nparts = std::max(a.nbv, a.nbe);
    a.vstride = h->viol_cap;
    a.check_every = 1;
    a.tau = 0.0f;
    return a;
}

extern "C" gn_status gn_hyper_create(int32_t n, int32_t m, const int32_t* edge_ptr, const int32_t* members,
                                     const float* w, hipStream_t stream, gn_hyper** out) {
    if (!out) return GN_E_ARG;
    *out = nullptr;
    std::vector<int32_t> cover;
    const gn_status vs = gn_internal_check_cliques(n, m, edge_ptr, members, w, cover);
    if (vs != GN_OK) return vs;
    gn_hyper* h = new (std::nothrow) gn_hyper();
    if (!h) return GN_E_NOMEM;
    (void)hipGetDevice(&h->device);
    h->n = n;
    h->m = m;
    h->nnzc = edge_ptr[m];
    h->eptr_h.assign(edge_ptr, edge_ptr + m + 1);
    h->emem_h.assign(members, members + h->nnzc);
    h->vptr_h.assign(n + 1, 0);
    for (int32_t i = 0; i < n; ++i) h->vptr_h[i + 1] = h->vptr_h[i] + cover[i];
    h->vedge_h.assign((size_t)h->nnzc, 0);
    std::vector<int32_t> pos(h->vptr_h.begin(), h->vptr_h.end() - 1);
    for (int32_t e = 0; e < m; ++e)
        for (int32_t j = edge_ptr[e]; j < edge_ptr[e + 1]; ++j) h->vedge_h[pos[members[j]]++] = e;
    h->v_h.resize(n);
    for (int32_t i = 0; i < n; ++i) h->v_h[i] = (float)std::sqrt((double)w[i]);
    const size_t S = GN_MAX_STARTS;
    const size_t nparts = (size_t)std::max(hyper_nbv(n), hyper_nbe(m));
    bool ok = gn_dalloc(&h->v, n) && gn_dalloc(&h->w, n) && gn_dalloc(&h->eptr, (size_t)m + 1) &&
              gn_dalloc(&h->emem, (size_t)h->nnzc) && gn_dalloc(&h->vptr, (size_t)n + 1) &&
              gn_dalloc(&h->vedge, (size_t)h->nnzc) && gn_dalloc(&h->Y, S * m) && gn_dalloc(&h->cnt, S * m) &&
              gn_dalloc(&h->vs, S * m) && gn_dalloc(&h->buf[0], S * n) && gn_dalloc(&h->buf[1], S * n) &&
              gn_dalloc(&h->st, S) && gn_dalloc(&h->part, S * nparts) && gn_dalloc(&h->out, S);
    if (ok && hipHostMalloc(&h->host, S * (sizeof(HState) + sizeof(HPart)), hipHostMallocDefault) != hipSuccess) {
        h->host = nullptr;
        ok = false;
    }
    if (!ok) {
        hyper_free(h);
        delete h;
        return GN_E_NOMEM;
    }
    hipError_t e = hipMemcpyAsync(h->v, h->v_h.data(), sizeof(float) * n, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h->w, w, sizeof(float) * n, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->eptr, edge_ptr, sizeof(int32_t) * (m + 1), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h->emem, members, sizeof(int32_t) * h->nnzc, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->vptr, h->vptr_h.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->vedge, h->vedge_h.data(), sizeof(int32_t) * h->nnzc, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        hyper_free(h);
        delete h;
        return GN_E_HIP;
    }
    *out = h;
    return GN_OK;
}

extern "C" void gn_hyper_destroy(gn_hyper* h) {
    if (!h) return;
    (void)hipDeviceSynchronize();
    hyper_free(h);
    delete h;
}

extern "C" gn_status gn_hyper_step(gn_hyper* h, float gamma, const float* x_in, float* x_out, hipStream_t stream) {
    if (!h || !x_in || !x_out || x_in == x_out) return GN_E_ARG;
    if (!std::isfinite(gamma) || gamma < 0.0f) return GN_E_ARG;
    HArgs a = hyper_args(h);
    const unsigned nb = (unsigned)((h->n + 255) / 256);
    if (nb == 0) return GN_OK;
    // user x -> state words, one step, state words -> user x
    hyper_prep_kernel<<<nb, 256, 0, stream>>>((int64_t)h->n, x_in, h->buf[0]);
    hyper_edge_kernel<<<a.nbe, kHBlock, 0, stream>>>(a, h->buf[0], 0, 0);
    hyper_vertex_kernel<<<a.nbv, kHVBlock, 0, stream>>>(a, h->buf[0], h->buf[1], gamma, 0, 0, 0, 1);
    hyper_value_kernel<<<nb, 256, 0, stream>>>((int64_t)h->n, h->buf[1], x_out);
    GN_HIP_TRY(hipGetLastError());
    return GN_OK;
}

extern "C" gn_status gn_hyper_multi_solve(gn_hyper* h, const gn_schedule* sch, int32_t starts, float* x, uint8_t* sel,
                                          gn_result* res, int32_t* best, hipStream_t stream) {
    if (!h || !sch || !res || !x || !sel || starts < 1 || starts > GN_MAX_STARTS) return GN_E_ARG;
    if (!gn_internal_schedule_ok(sch)) return GN_E_ARG;
    std::memset(res, 0, sizeof(gn_result) * starts);
    const int32_t n = h->n, ms = sch->max_steps;
    // every x^0: finite, >= 0 and normalizable (every vertex has mass in its
    // hyperedges), checked on the host
    std::vector<float> x0((size_t)starts * n);
    GN_HIP_TRY(hipMemcpyAsync(x0.data(), x, sizeof(float) * x0.size(), hipMemcpyDeviceToHost, stream));
    GN_HIP_TRY(hipStreamSynchronize(stream));
    std::vector<double> X(h->m);
    for (int32_t s = 0; s < starts; ++s) {
        const float* xs = x0.data() + (size_t)s * n;
        for (int32_t i = 0; i < n; ++i)
            if (!(xs[i] >= 0.0f) || !std::isfinite(xs[i])) return GN_E_ARG;
        std::fill(X.begin(), X.end(), 0.0);
        for (int32_t e = 0; e < h->m; ++e)
            for (int32_t j = h->eptr_h[e]; j < h->eptr_h[e + 1]; ++j) X[e] += xs[h->emem_h[j]];
        for (int32_t i = 0; i < n; ++i) {
            double sm = xs[i];
            for (int32_t q = h->vptr_h[i]; q < h->vptr_h[i + 1]; ++q) sm += X[h->vedge_h[q]] - xs[i];
            if (!(sm > 0.0)) return GN_E_NOT_NORMALIZABLE;
        }
    }
    if (ms + 1 > h->viol_cap) {
        hipFree(h->viol);
        h->viol = nullptr;
        h->viol_cap = 0;
        if (!gn_dalloc(&h->viol, (size_t)GN_MAX_STARTS * (ms + 1))) return GN_E_NOMEM;
        h->viol_cap = ms + 1;
    }
    HArgs a = hyper_args(h);
    a.check_every = sch->check_every;
    a.tau = sch->tau;
    GN_HIP_TRY(hipMemsetAsync(h->viol, 0, sizeof(int32_t) * (size_t)starts * a.vstride, stream));
    GN_HIP_TRY(hipMemsetAsync(h->st, 0, sizeof(HState) * starts, stream));
    hyper_prep_kernel<<<dim3((unsigned)(((size_t)starts * n + 255) / 256)), 256, 0, stream>>>((int64_t)starts * n, x,
                                                                                          h->buf[0]);
    GN_HIP_TRY(hipGetLastError());
    HState* hs = (HState*)h->host;
    HPart* hp = (HPart*)((char*)h->host + GN_MAX_STARTS * sizeof(HState));
    const dim3 ge(a.nbe, starts), gv(a.nbv, starts);
    if (ms > 0) {
        // steps 0 .. ms - 1 in captured chains; no further chain once every start has stopped
        if (!h->ws.state) {
            const SolveState never{-1, 0, 0, 0, 0.0f, 0, 0ull};
            if (!gn_dalloc(&h->ws.state, 1)) return GN_E_NOMEM;
            GN_HIP_TRY(hipMemcpy(h->ws.state, &never, sizeof(never), hipMemcpyHostToDevice));
        }
        if (!h->ws.host_pinned && hipHostMalloc(&h->ws.host_pinned, 4096, hipHostMallocDefault) != hipSuccess) {
            h->ws.host_pinned = nullptr;
            return GN_E_NOMEM;
        }
        const gn_hyper::ChainKey key{starts, ms, sch->ramp_steps, sch->check_every, a.vstride,
                                     sch->gamma0, sch->gamma1, sch->tau, h->viol};
        if (!(h->key == key)) {
            h->ws.destroy_chains();
            h->key = key;
        }
        const int32_t C = g_chunk_len;
        const int32_t words = starts * (int32_t)(sizeof(HState) / sizeof(int32_t));
        const char* run = (const char*)h->ws.host_pinned + kHPinState;
        ChunkHooks hooks;
        hooks.pin_src = h->st;
        hooks.pin_words = words;
        hooks.pin_offset = kHPinState;
        hooks.stop_after = [run, words, starts](int32_t c) {
            const volatile HState* p = (const volatile HState*)(run + sizeof(int32_t) * (size_t)words * (c & 1));
            for (int32_t s = 0; s < starts; ++s)
                if (!p[s].done) return false;
            return true;
        };
        auto build = [h, a, sch, starts, ms, C](int32_t c, int32_t j0, int32_t j1, hipGraph_t graph,
                                                hipGraphNode_t* last) -> gn_status {
            hipGraphNode_t prev = *last;
            for (int32_t j = j0; j < j1 && c * C + j < ms; ++j) {
                HArgs aa = a;
                int32_t k = c * C + j, solve = 1, write = 1;
                int32_t chk = k >= 1 && k % sch->check_every == 0;
                float g = gn_internal_host_gamma(sch, k);
                const float* xin = h->buf[k & 1];
                float* xout = h->buf[(k + 1) & 1];
                void* ea[] = {&aa, &xin, &k, &solve};
                void* va[] = {&aa, &xin, &xout, &g, &k, &solve, &chk, &write};
                hipKernelNodeParams p{};
                p.func = (void*)hyper_edge_kernel;
                p.gridDim = dim3(aa.nbe, starts);
                p.blockDim = dim3(kHBlock);
                p.sharedMemBytes = 0;
                p.kernelParams = ea;
                p.extra = nullptr;
                hipGraphNode_t node;
                if (hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &p) != hipSuccess)
                    return GN_E_HIP;
                prev = node;
                p.func = (void*)hyper_vertex_kernel;
                p.gridDim = dim3(aa.nbv, starts);
                p.blockDim = dim3(kHVBlock);
                p.kernelParams = va;
                if (hipGraphAddKernelNode(&node, graph, &prev, 1, &p) != hipSuccess) return GN_E_HIP;
                prev = node;
            }
            *last = prev;
            return GN_OK;
        };
        gn_status rs = gn_internal_run_marked(h->ws, (ms + C - 1) / C, C, build, 0, stream, false, &hooks);
        if (rs != GN_OK) return rs;
    }
    // the last check: a pending check of step ms - 1, then x^ms itself
    hyper_edge_kernel<<<ge, kHBlock, 0, stream>>>(a, h->buf[ms & 1], ms, 1);
    hyper_vertex_kernel<<<gv, kHVBlock, 0, stream>>>(a, h->buf[ms & 1], nullptr, gn_internal_host_gamma(sch, ms), ms,
                                                     1, ms >= 1 ? 1 : 0, 0);
    hyper_resolve_kernel<<<starts, 1, 0, stream>>>(a, ms, ms >= 1 ? 1 : 0);
    GN_HIP_TRY(hipGetLastError());
    GN_HIP_TRY(hipMemcpyAsync(hs, h->st, sizeof(HState) * starts, hipMemcpyDeviceToHost, stream));
    GN_HIP_TRY(hipStreamSynchronize(stream));
    HFinal f{};
    for (int32_t s = 0; s < starts; ++s) {
        f.buf[s] = hs[s].step & 1;
        f.gamma[s] = gn_internal_host_gamma(sch, hs[s].step);
    }
    hyper_stats_edge_kernel<<<ge, kHBlock, 0, stream>>>(a, h->buf[0], h->buf[1], f);
    hyper_stats_vertex_kernel<<<gv, kHVBlock, 0, stream>>>(a, h->buf[0], h->buf[1], f, x, sel);
    hyper_stats_finish_kernel<<<starts, 256, 0, stream>>>(a, h->out);
    GN_HIP_TRY(hipGetLastError());
    GN_HIP_TRY(hipMemcpyAsync(hp, h->out, sizeof(HPart) * starts, hipMemcpyDeviceToHost, stream));
    GN_HIP_TRY(hipStreamSynchronize(stream));
    bool all = true;
    int32_t b = -1, b_any = 0;
    for (int32_t s = 0; s < starts; ++s) {
        gn_result& r = res[s];
        r.steps = hs[s].step;
        r.binarised = hs[s].binarised;
        r.fallback_count = (int64_t)hs[s].fallback;
        r.relaxed_objective = hp[s].relaxed;
        r.set_objective = hp[s].W;
        r.set_size = hp[s].size;
        r.conflicts = hp[s].conflicts;
        r.uncovered = hp[s].uncovered;
        r.stab = hp[s].stab;
        if (!std::isfinite(r.relaxed_objective)) return GN_E_NUMERIC;
        all = all && r.binarised;
        if (r.binarised && (b < 0 || r.set_objective > res[b].set_objective)) b = s;
        if (r.set_objective > res[b_any].set_objective) b_any = s;
    }
    if (best) *best = b >= 0 ? b : b_any;
    return all ? GN_OK : GN_NOT_CONVERGED;
}

extern "C" gn_status gn_hyper_solve(gn_hyper* h, const gn_schedule* sch, float* x, uint8_t* sel, gn_result* res,
                                    hipStream_t stream) {
    return gn_hyper_multi_solve(h, sch, 1, x, sel, res, nullptr, stream);
}
