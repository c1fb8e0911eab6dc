// Graph ingest (validation, v = sqrt(w), degree bins, relabelling) and the
// per-handle work buffers.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "gn_internal.h"

extern "C" const char* gn_status_str(gn_status s) {
    switch (s) {
        case GN_OK: return "GN_OK";
        case GN_NOT_CONVERGED: return "GN_NOT_CONVERGED";
        case GN_E_ARG: return "GN_E_ARG: invalid argument";
        case GN_E_CSR: return "GN_E_CSR: malformed CSR (row_ptr bounds/monotonicity, column range, order)";
        case GN_E_SELF_LOOP: return "GN_E_SELF_LOOP: diagonal entry in A";
        case GN_E_ASYMMETRIC: return "GN_E_ASYMMETRIC: A is not symmetric";
        case GN_E_WEIGHT: return "GN_E_WEIGHT: weight not finite or not > 0";
        case GN_E_NOT_NORMALIZABLE: return "GN_E_NOT_NORMALIZABLE: x0 has a zero closed neighbourhood";
        case GN_E_NUMERIC: return "GN_E_NUMERIC: non-finite value";
        case GN_E_HIP: return "GN_E_HIP: HIP runtime error";
        case GN_E_NOMEM: return "GN_E_NOMEM: allocation failed";
        case GN_E_SIZE: return "GN_E_SIZE: input larger than this entry point's fixed capacity";
    }
    return "unknown gn_status";
}

static int bin_of_degree(int32_t d) {
    for (int b = BIN_COUNT - 1; b > 0; --b)
        if (d <= bin_max_degree(b)) return b;
    return BIN_BLOCK;
}

int32_t gn_internal_grid_blocks(const BinLayout& b) { return b.blk_begin[BIN_COUNT]; }

// Row range and entry order: monotone row_ptr with row_ptr[0] = 0 and
// row_ptr[n] = nnz, columns in [0, n).  Always checked: the kernels index with
// these values.
static gn_status check_bounds(int32_t n, int64_t nnz, const int32_t* rp, const int32_t* ci) {
    if (rp[0] != 0 || (int64_t)rp[n] != nnz) return GN_E_CSR;
    for (int32_t i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) return GN_E_CSR;
    for (int64_t e = 0; e < nnz; ++e)
        if (ci[e] < 0 || ci[e] >= n) return GN_E_CSR;
    return GN_OK;
}

// Structure of a simple undirected graph (Section 2): no diagonal entries,
// strictly increasing columns per row, and A = A^T.  Symmetry is checked by
// building the transpose with a counting pass (rows visited in increasing
// order, so every transposed row comes out sorted) and comparing it entry by
// entry with the input.
static gn_status check_structure(int32_t n, int64_t nnz, const int32_t* rp, const int32_t* ci) {
    for (int32_t i = 0; i < n; ++i) {
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            if (ci[e] == i) return GN_E_SELF_LOOP;
            if (e > rp[i] && ci[e] <= ci[e - 1]) return GN_E_CSR;
        }
    }
    std::vector<int64_t> tptr((size_t)n + 1, 0);
    for (int64_t e = 0; e < nnz; ++e) tptr[(size_t)ci[e] + 1]++;
    for (int32_t i = 0; i < n; ++i) tptr[(size_t)i + 1] += tptr[i];
    for (int32_t i = 0; i <= n; ++i)
        if (tptr[i] != rp[i]) return GN_E_ASYMMETRIC;
    std::vector<int32_t> tcol((size_t)std::max<int64_t>(nnz, 1));
    std::vector<int64_t> fill(tptr.begin(), tptr.end() - 1);
    for (int32_t i = 0; i < n; ++i)
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) tcol[(size_t)fill[ci[e]]++] = i;
    for (int64_t e = 0; e < nnz; ++e)
        if (tcol[(size_t)e] != ci[e]) return GN_E_ASYMMETRIC;
    return GN_OK;
}

// Reverse Cuthill-McKee order (breadth-first from a minimum-degree vertex of
// every component, neighbours visited by increasing degree, then reversed): a
// bandwidth-reducing relabelling that puts neighbours at nearby ids, so one
// wavefront's gathers touch fewer cache lines.
static std::vector<int32_t> rcm_order(int32_t n, const int32_t* rp, const int32_t* ci, const std::vector<int32_t>& deg) {
    std::vector<int32_t> by_deg((size_t)n);
    std::iota(by_deg.begin(), by_deg.end(), 0);
    std::stable_sort(by_deg.begin(), by_deg.end(), [&](int32_t a, int32_t b) { return deg[a] < deg[b]; });
    std::vector<uint8_t> seen((size_t)n, 0);
    std::vector<int32_t> order;
    order.reserve((size_t)n);
    std::vector<int32_t> nb;
    for (int32_t s0 : by_deg) {
        if (seen[s0]) continue;
        seen[s0] = 1;
        size_t head = order.size();
        order.push_back(s0);
        while (head < order.size()) {
            const int32_t u = order[head++];
            nb.clear();
            for (int32_t e = rp[u]; e < rp[u + 1]; ++e)
                if (!seen[ci[e]]) {
                    seen[ci[e]] = 1;
                    nb.push_back(ci[e]);
                }
            std::stable_sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) { return deg[a] < deg[b]; });
            order.insert(order.end(), nb.begin(), nb.end());
        }
    }
    std::reverse(order.begin(), order.end());
    return order;
}

// Cache lines (32 floats) touched by the neighbour gathers of one step when the
// rows run in `perm` order, counted per group of 64 consecutive rows and entry
// position (the access pattern of the thread-per-row bins).
static int64_t gather_lines(int32_t n, const int32_t* rp, const int32_t* ci, const std::vector<int32_t>& perm,
                            const std::vector<int32_t>& iperm, const std::vector<int32_t>& deg) {
    int64_t lines = 0;
    std::vector<int32_t> buf;
    for (int32_t w0 = 0; w0 < n; w0 += 64) {
        const int32_t w1 = std::min(n, w0 + 64);
        int32_t dmax = 0;
        for (int32_t r = w0; r < w1; ++r) dmax = std::max(dmax, deg[perm[r]]);
        dmax = std::min(dmax, 64);
        for (int32_t q = 0; q < dmax; ++q) {
            buf.clear();
            for (int32_t r = w0; r < w1; ++r) {
                const int32_t i = perm[r];
                if (q < deg[i]) buf.push_back(iperm[ci[rp[i] + q]] >> 5);
            }
            std::sort(buf.begin(), buf.end());
            lines += (int64_t)(std::unique(buf.begin(), buf.end()) - buf.begin());
        }
    }
    return lines;
}

template <typename T>
static gn_status dev_alloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    if (hipMalloc((void**)p, count * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return GN_E_NOMEM;
    }
    return GN_OK;
}

static void free_graph_buffers(gn_graph* g) {
    auto f = [](void* p) { if (p) (void)hipFree(p); };
    f(g->row_ptr); f(g->col); f(g->v); f(g->w_int); f(g->w_user); f(g->perm); f(g->iperm);
    f(g->sl_col); f(g->sl_off);
    f(g->prune); f(g->prune_mloc); f(g->listed); f(g->prune_mirror);
    GraphWorkspace& ws = g->ws;
    ws.destroy_chains();
    f(ws.y[0]); f(ws.y[1]); f(ws.state); f(ws.notconv); f(ws.gamma); f(ws.sel_int);
    f(ws.partials); f(ws.final_out);
    if (ws.host_pinned) (void)hipHostFree(ws.host_pinned);
}

extern "C" void gn_graph_destroy(gn_graph* g) {
    if (!g) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(g->device);
    (void)hipDeviceSynchronize();
    gn_internal_free_unrolled(g);
    gn_internal_free_multi(g);
    gn_internal_free_small(g);
    free_graph_buffers(g);
    delete g;
    (void)hipSetDevice(cur);
}

extern "C" gn_status gn_graph_create(int32_t n, int64_t nnz, const int32_t* row_ptr,
                                     const int32_t* col_idx, const float* w, uint32_t flags,
                                     hipStream_t stream, gn_graph** out) {
    if (!out) return GN_E_ARG;
    *out = nullptr;
    if (n < 0 || nnz < 0 || nnz > INT32_MAX || (flags & ~3u)) return GN_E_ARG;
    if (!row_ptr || (n > 0 && !w) || (nnz > 0 && !col_idx)) return GN_E_ARG;

    std::vector<int32_t> rp((size_t)n + 1), ci((size_t)std::max<int64_t>(nnz, 1));
    std::vector<float> wh((size_t)std::max(n, 1));
    if (flags & GN_INPUT_DEVICE) {
        GN_HIP_TRY(hipMemcpyAsync(rp.data(), row_ptr, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToHost, stream));
        if (nnz) GN_HIP_TRY(hipMemcpyAsync(ci.data(), col_idx, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToHost, stream));
        if (n) GN_HIP_TRY(hipMemcpyAsync(wh.data(), w, sizeof(float) * (size_t)n, hipMemcpyDeviceToHost, stream));
        GN_HIP_TRY(hipStreamSynchronize(stream));
    } else {
        std::memcpy(rp.data(), row_ptr, sizeof(int32_t) * ((size_t)n + 1));
        if (nnz) std::memcpy(ci.data(), col_idx, sizeof(int32_t) * (size_t)nnz);
        if (n) std::memcpy(wh.data(), w, sizeof(float) * (size_t)n);
    }
    gn_status st = check_bounds(n, nnz, rp.data(), ci.data());
    if (st != GN_OK) return st;
    if (!(flags & GN_NO_VALIDATE)) {
        st = check_structure(n, nnz, rp.data(), ci.data());
        if (st != GN_OK) return st;
    }
    for (int32_t i = 0; i < n; ++i)
        if (!(wh[i] > 0.0f) || !std::isfinite(wh[i])) return GN_E_WEIGHT;

    gn_graph* g = new (std::nothrow) gn_graph();
    if (!g) return GN_E_NOMEM;
    (void)hipGetDevice(&g->device);
    g->n = n;
    g->nnz = nnz;

    // relabel rows into contiguous degree bins (heaviest bin first).  Inside a
    // bin rows keep either the caller's order or a Reverse Cuthill-McKee order,
    // whichever touches fewer cache lines in the neighbour gathers.
    std::vector<int32_t> deg((size_t)n);
    int32_t maxd = 0;
    for (int32_t i = 0; i < n; ++i) {
        deg[i] = rp[i + 1] - rp[i];
        maxd = std::max(maxd, deg[i]);
    }
    g->max_degree = maxd;
    auto binned = [&](const std::vector<int32_t>& base) {
        std::vector<int32_t> p(base);
        std::stable_sort(p.begin(), p.end(), [&](int32_t a, int32_t b) {
            return bin_of_degree(deg[a]) < bin_of_degree(deg[b]);
        });
        return p;
    };
    auto inverse = [&](const std::vector<int32_t>& p) {
        std::vector<int32_t> q((size_t)n);
        for (int32_t r = 0; r < n; ++r) q[p[r]] = r;
        return q;
    };
    std::vector<int32_t> natural((size_t)n);
    std::iota(natural.begin(), natural.end(), 0);
    std::vector<int32_t> perm = binned(natural);
    std::vector<int32_t> iperm = inverse(perm);
    if (n > 4096 && nnz <= 64ll * n) {
        std::vector<int32_t> p2 = binned(rcm_order(n, rp.data(), ci.data(), deg));
        std::vector<int32_t> q2 = inverse(p2);
        const int64_t l1 = gather_lines(n, rp.data(), ci.data(), perm, iperm, deg);
        const int64_t l2 = gather_lines(n, rp.data(), ci.data(), p2, q2, deg);
        if (l2 < l1 - l1 / 10) {
            perm.swap(p2);
            iperm.swap(q2);
        }
    }
    // Gather locality of the chosen order: distinct 128-byte lines per gathered
    // entry.  Rows of up to 128 neighbours (a thread or a few per row) are
    // counted over 64-row windows, one position at a time, as a wavefront
    // gathers them; heavier rows (a wavefront or a workgroup per row, every
    // 16th row sampled) over their own entries.  The pruned lists pay where most
    // gathers touch a line of their own (power-law and random graphs, the
    // column mates of assignment graphs); where neighbours share lines the
    // skipped gathers were cache hits and the lists' upkeep costs more.
    {
        int64_t lines = 0, counted = 0;
        std::vector<int32_t> buf;
        for (int32_t w0 = 0; w0 < n; w0 += 64) {
            const int32_t w1 = std::min(n, w0 + 64);
            int32_t dmax = 0;
            for (int32_t r = w0; r < w1; ++r)
                if (deg[perm[r]] <= 128) dmax = std::max(dmax, deg[perm[r]]);
            for (int32_t q = 0; q < dmax; ++q) {
                buf.clear();
                for (int32_t r = w0; r < w1; ++r) {
                    const int32_t i = perm[r];
                    if (deg[i] <= 128 && q < deg[i]) buf.push_back(iperm[ci[rp[i] + q]] >> 5);
                }
                std::sort(buf.begin(), buf.end());
                lines += (int64_t)(std::unique(buf.begin(), buf.end()) - buf.begin());
                counted += (int64_t)buf.size();
            }
        }
        int32_t heavy = 0;
        for (int32_t r = 0; r < n; ++r) {
            const int32_t i = perm[r];
            if (deg[i] <= 128 || (heavy++ & 15)) continue;
            buf.clear();
            for (int32_t e = rp[i]; e < rp[i + 1]; ++e) buf.push_back(iperm[ci[e]] >> 5);
            std::sort(buf.begin(), buf.end());
            lines += 16 * (int64_t)(std::unique(buf.begin(), buf.end()) - buf.begin());
            counted += 16 * (int64_t)buf.size();
        }
        g->prune_pays = lines * 2 > counted;
    }

    int32_t counts[BIN_COUNT] = {0};
    for (int32_t i = 0; i < n; ++i) counts[bin_of_degree(deg[i])]++;
    BinLayout bl{};
    bl.row_begin[0] = 0;
    bl.blk_begin[0] = 0;
    bl.slice_begin[0] = 0;
    for (int b = 0; b < BIN_COUNT; ++b) {
        g->bin_count_rows[b] = counts[b];
        bl.row_begin[b + 1] = bl.row_begin[b] + counts[b];
        int rpb = bin_rows_per_block(b);
        bl.blk_begin[b + 1] = bl.blk_begin[b] + (counts[b] + rpb - 1) / rpb;
        const int G = bin_group(b);
        bl.slice_begin[b + 1] = bl.slice_begin[b] + (G ? (counts[b] + 64 / G - 1) / (64 / G) : 0);
    }
    g->bins = bl;

    // inside the sliced bins: decreasing degree within windows (less padding)
    for (int b = 0; b < BIN_COUNT; ++b) {
        if (!bin_group(b)) continue;
        for (int32_t w0 = bl.row_begin[b]; w0 < bl.row_begin[b + 1]; w0 += kSortWindow) {
            const int32_t w1 = std::min(bl.row_begin[b + 1], w0 + kSortWindow);
            std::stable_sort(perm.begin() + w0, perm.begin() + w1,
                             [&](int32_t a, int32_t c) { return deg[a] > deg[c]; });
        }
    }
    iperm = inverse(perm);

    std::vector<int32_t> rp_int((size_t)n + 1), col_int((size_t)std::max<int64_t>(nnz, 1));
    std::vector<float> v_int((size_t)std::max(n, 1)), w_int((size_t)std::max(n, 1));
    rp_int[0] = 0;
    for (int32_t r = 0; r < n; ++r) {
        int32_t i = perm[r];
        int32_t base = rp_int[r];
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) col_int[(size_t)(base + e - rp[i])] = iperm[ci[e]];
        rp_int[r + 1] = base + deg[i];
        w_int[r] = wh[i];
        v_int[r] = (float)std::sqrt((double)wh[i]);
    }

    // sliced columns: slice s of a group bin covers 64/G rows; line q of the slice
    // holds, in lane G*r + t, entry t + G*q of row r (or -1)
    const int32_t nslices = bl.slice_begin[BIN_COUNT];
    std::vector<int32_t> sl_off((size_t)nslices + 1, 0);
    for (int b = 0; b < BIN_COUNT; ++b) {
        const int G = bin_group(b);
        if (!G) continue;
        const int RS = 64 / G;
        for (int32_t s = bl.slice_begin[b]; s < bl.slice_begin[b + 1]; ++s) {
            const int32_t r0 = bl.row_begin[b] + (s - bl.slice_begin[b]) * RS;
            const int32_t r1 = std::min(bl.row_begin[b + 1], r0 + RS);
            int32_t width = 0;
            for (int32_t r = r0; r < r1; ++r) width = std::max(width, (rp_int[r + 1] - rp_int[r] + G - 1) / G);
            sl_off[(size_t)s + 1] = width;
        }
    }
    int64_t lines = 0;
    for (int32_t s = 0; s < nslices; ++s) {
        lines += sl_off[(size_t)s + 1];
        if (lines > INT32_MAX / 64) {
            delete g;
            return GN_E_ARG;
        }
        sl_off[(size_t)s + 1] = (int32_t)lines;
    }
    std::vector<int32_t> sl_col((size_t)std::max<int64_t>(lines * 64, 1), -1);
    // loc_of[e]: where internal CSR entry e is read by the step kernel, in the
    // pruned lists' index space (sliced words, then CSR positions)
    const int64_t sl_words = lines * 64;
    std::vector<int32_t> loc_of((size_t)std::max<int64_t>(nnz, 1));
    bool prunable = sl_words + nnz <= INT32_MAX;
    for (int32_t r = 0; r < n && prunable; ++r)
        for (int32_t e = rp_int[r]; e < rp_int[r + 1]; ++e) loc_of[(size_t)e] = (int32_t)(sl_words + e);
    for (int b = 0; b < BIN_COUNT; ++b) {
        const int G = bin_group(b);
        if (!G) continue;
        const int RS = 64 / G;
        for (int32_t s = bl.slice_begin[b]; s < bl.slice_begin[b + 1]; ++s) {
            const int32_t r0 = bl.row_begin[b] + (s - bl.slice_begin[b]) * RS;
            const int32_t r1 = std::min(bl.row_begin[b + 1], r0 + RS);
            int32_t* base = sl_col.data() + (size_t)sl_off[s] * 64;
            for (int32_t r = r0; r < r1; ++r) {
                const int32_t d = rp_int[r + 1] - rp_int[r];
                for (int32_t p = 0; p < d; ++p) {
                    const int32_t q = p / G, lane = (r - r0) * G + p % G;
                    base[(size_t)q * 64 + lane] = col_int[(size_t)rp_int[r] + p];
                    if (prunable) loc_of[(size_t)rp_int[r] + p] = (int32_t)((int64_t)(sl_off[s] + q) * 64 + lane);
                }
            }
        }
    }

    // mirror entries: entry p of user row u points to w; u sits at position p'
    // of user row w (rows sorted: binary search).  Internal rows keep the
    // caller's per-row order, so mloc of internal entry (iperm[u], p) is the
    // location of internal entry (iperm[w], p').  A missing or repeated mirror
    // (a structure that was not validated) leaves the graph without pruned lists.
    std::vector<int32_t> mloc, mirror;
    if (prunable && nnz > 0) {
        mloc.assign((size_t)nnz, -1);
        mirror.assign((size_t)nnz, -1);
        for (int32_t u = 0; u < n && prunable; ++u) {
            const int32_t r = iperm[u];
            for (int32_t p = 0; p < rp[u + 1] - rp[u]; ++p) {
                const int32_t wv = ci[(size_t)rp[u] + p];
                const int32_t* b0 = ci.data() + rp[wv];
                const int32_t* b1 = ci.data() + rp[wv + 1];
                const int32_t* it = std::lower_bound(b0, b1, u);
                if (it == b1 || *it != u || (it + 1 < b1 && it[1] == u) || wv == u) {
                    prunable = false;
                    break;
                }
                const int32_t e_mirror = rp_int[iperm[wv]] + (int32_t)(it - b0);
                mloc[(size_t)rp_int[r] + p] = loc_of[(size_t)e_mirror];
                mirror[(size_t)rp_int[r] + p] = e_mirror;
            }
        }
    }
    prunable = prunable && nnz > 0;

    st = GN_OK;
    if (prunable && ((st = dev_alloc(&g->prune, (size_t)(sl_words + nnz))) ||
                     (st = dev_alloc(&g->prune_mloc, (size_t)nnz)) || (st = dev_alloc(&g->listed, (size_t)n)) ||
                     (st = dev_alloc(&g->prune_mirror, (size_t)nnz)))) {
        free_graph_buffers(g);
        delete g;
        return st;
    }
    g->prune_sl_words = prunable ? sl_words : 0;
    if ((st = dev_alloc(&g->sl_col, sl_col.size())) || (st = dev_alloc(&g->sl_off, sl_off.size())) ||
        (st = dev_alloc(&g->row_ptr, (size_t)n + 1)) || (st = dev_alloc(&g->col, (size_t)nnz)) ||
        (st = dev_alloc(&g->v, (size_t)n)) || (st = dev_alloc(&g->w_int, (size_t)n)) ||
        (st = dev_alloc(&g->w_user, (size_t)n)) || (st = dev_alloc(&g->perm, (size_t)n)) ||
        (st = dev_alloc(&g->iperm, (size_t)n))) {
        free_graph_buffers(g);
        delete g;
        return st;
    }
    hipError_t e = hipSuccess;
    auto up = [&](void* dst, const void* src, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream);
    };
    up(g->row_ptr, rp_int.data(), sizeof(int32_t) * ((size_t)n + 1));
    up(g->col, col_int.data(), sizeof(int32_t) * (size_t)nnz);
    up(g->v, v_int.data(), sizeof(float) * (size_t)n);
    up(g->w_int, w_int.data(), sizeof(float) * (size_t)n);
    up(g->w_user, wh.data(), sizeof(float) * (size_t)n);
    up(g->perm, perm.data(), sizeof(int32_t) * (size_t)n);
    up(g->iperm, iperm.data(), sizeof(int32_t) * (size_t)n);
    up(g->sl_col, sl_col.data(), sizeof(int32_t) * sl_col.size());
    up(g->sl_off, sl_off.data(), sizeof(int32_t) * sl_off.size());
    if (prunable) {
        // the pruned lists start as copies; positions past a row's end stay -1
        up(g->prune, sl_col.data(), sizeof(int32_t) * (size_t)sl_words);
        up(g->prune + sl_words, col_int.data(), sizeof(int32_t) * (size_t)nnz);
        up(g->prune_mloc, mloc.data(), sizeof(int32_t) * (size_t)nnz);
        up(g->prune_mirror, mirror.data(), sizeof(int32_t) * (size_t)nnz);
        if (e == hipSuccess) e = hipMemsetAsync(g->listed, 1, (size_t)n, stream);  // every vertex listed
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        free_graph_buffers(g);
        delete g;
        return GN_E_HIP;
    }
    gn_internal_build_small(g, rp_int.data(), col_int.data(), stream);
    *out = g;
    return GN_OK;
}

extern "C" gn_status gn_graph_info(const gn_graph* g, int32_t* n, int64_t* nnz, int32_t* max_degree,
                                   int32_t* bin_rows) {
    if (!g) return GN_E_ARG;
    if (n) *n = g->n;
    if (nnz) *nnz = g->nnz;
    if (max_degree) *max_degree = g->max_degree;
    if (bin_rows) {
        // public order: lightest bin first, unused entries 0
        for (int k = 0; k < GN_NUM_BINS; ++k) bin_rows[k] = 0;
        for (int b = 0; b < BIN_COUNT; ++b) bin_rows[BIN_COUNT - 1 - b] = g->bin_count_rows[b];
    }
    return GN_OK;
}

// Work buffers of a handle, grown on demand.  Growing the step tables drops the
// captured step chains, which hold the old addresses.
gn_status gn_internal_ensure_ws(gn_graph* g, int32_t steps_needed) {
    GraphWorkspace& ws = g->ws;
    const int32_t n = g->n;
    if (!ws.y[0]) {
        gn_status st;
        if ((st = dev_alloc(&ws.y[0], (size_t)n)) || (st = dev_alloc(&ws.y[1], (size_t)n)) ||
            (st = dev_alloc(&ws.state, 1)) || (st = dev_alloc(&ws.sel_int, (size_t)n)) ||
            (st = dev_alloc((SolveTail**)&ws.final_out, 1)))
            return st;
        if (hipHostMalloc(&ws.host_pinned, 4096, hipHostMallocDefault) != hipSuccess) {
            ws.host_pinned = nullptr;
            return GN_E_NOMEM;
        }
    }
    return gn_internal_ensure_tables(ws, steps_needed);
}

// Step tables (test flags, gamma) of a solve workspace, grown on demand.
gn_status gn_internal_ensure_tables(GraphWorkspace& ws, int32_t steps_needed) {
    if (steps_needed > ws.cap_steps) {
        int32_t cap = std::max(steps_needed, 2 * ws.cap_steps);
        if (ws.notconv) (void)hipFree(ws.notconv);
        if (ws.gamma) (void)hipFree(ws.gamma);
        ws.notconv = nullptr;
        ws.gamma = nullptr;
        gn_status st;
        if ((st = dev_alloc(&ws.notconv, (size_t)cap)) || (st = dev_alloc(&ws.gamma, (size_t)cap))) {
            ws.cap_steps = 0;
            return st;
        }
        ws.cap_steps = cap;
        for (auto ex : ws.chunks) if (ex) (void)hipGraphExecDestroy(ex);
        ws.chunks.clear();
    }
    return GN_OK;
}
