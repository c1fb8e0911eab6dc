// Measurement probe (not part of libgn): the rate of the random 4-byte gathers
// that bound the single-start step on the Barabasi-Albert benchmark graph.  The
// light rows (degree <= 16, 180,274 of the 200,000 rows, 1,332,030 gathers) are
// given in the step kernel's sliced layout, rows in the library's internal
// (degree-descending) order, 16 lines per 64-row slice (padding gathers a zero
// slot).  A: one slice per wavefront, column lines streamed, then the gathers (a
// step without its epilogue).  B: persistent wavefronts that hold their slices'
// column ids in registers and repeat only the gathers (L2 warm): the floor for
// the gathers alone.
//
// Build and run (repository root):
//     python paper_2605_05330_amd/probes/ba_light_lines.py /tmp
//     hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         -o /tmp/gather_rate paper_2605_05330_amd/probes/gather_rate.hip && /tmp/gather_rate /tmp/ba_lines.bin
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>
#include <vector>
#define CK(x) do { hipError_t e = (x); if (e != hipSuccess) { printf("HIP error %s line %d\n", hipGetErrorString(e), __LINE__); return 1; } } while (0)

__global__ __launch_bounds__(256) void stream_gather(const int* __restrict__ lines, int S, const float* __restrict__ y, float* __restrict__ out) {
    const int s = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (s >= S) return;
    const int* ln = lines + (size_t)s * 16 * 64 + lane;
    int id[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) id[q] = __builtin_nontemporal_load(ln + 64 * q);
    float acc = 0.f;
#pragma unroll
    for (int q = 0; q < 16; ++q) acc += y[id[q]];
    out[s * 64 + lane] = acc;
}

template <int K>
__global__ __launch_bounds__(256) void reg_gather(const int* __restrict__ lines, int S, const float* y, float* __restrict__ out, int R) {
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int W = gridDim.x * 4;
    int id[K][16];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int s = w + k * W;
#pragma unroll
        for (int q = 0; q < 16; ++q) id[k][q] = s < S ? lines[(size_t)s * 16 * 64 + 64 * q + lane] : 0;
    }
    float acc = 0.f;
    for (int r = 0; r < R; ++r) {
        asm volatile("" ::: "memory");   // the gathers below are re-issued every pass
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc += y[id[k][q]];
        acc *= 0.5f;
    }
    out[w * 64 + lane] = acc;
}

int main(int argc, char** argv) {
    const int n = 200000;
    FILE* f = fopen(argv[1], "rb");
    if (!f) { printf("no lines file\n"); return 1; }
    fseek(f, 0, SEEK_END); long bytes = ftell(f); fseek(f, 0, SEEK_SET);
    const int S = (int)(bytes / (16 * 64 * 4));
    std::vector<int> h((size_t)S * 16 * 64);
    if (fread(h.data(), 4, h.size(), f) != h.size()) { printf("short read\n"); return 1; }
    fclose(f);
    for (int v : h) if (v < 0 || v > n) { printf("bad id %d\n", v); return 1; }
    long gathers = 0; for (int v : h) gathers += v < n;
    std::vector<float> yh(n + 1);
    for (int i = 0; i < n; ++i) yh[i] = (float)((i * 2654435761u) % 1000) * 1e-3f;
    yh[n] = 0.f;
    int* dl; float *dy, *dout;
    CK(hipMalloc(&dl, h.size() * 4)); CK(hipMalloc(&dy, (n + 1) * 4)); CK(hipMalloc(&dout, (size_t)S * 64 * 4 + 4 * 1024 * 64 * 16));
    CK(hipMemcpy(dl, h.data(), h.size() * 4, hipMemcpyHostToDevice));
    CK(hipMemcpy(dy, yh.data(), (n + 1) * 4, hipMemcpyHostToDevice));
    printf("slices %d gathers %ld (padded %zu)\n", S, gathers, h.size());
    hipEvent_t a, b; CK(hipEventCreate(&a)); CK(hipEventCreate(&b));
    const int nb = (S + 3) / 4;
    for (int i = 0; i < 20; ++i) hipLaunchKernelGGL(stream_gather, dim3(nb), dim3(256), 0, 0, dl, S, dy, dout);
    CK(hipEventRecord(a));
    for (int i = 0; i < 200; ++i) hipLaunchKernelGGL(stream_gather, dim3(nb), dim3(256), 0, 0, dl, S, dy, dout);
    CK(hipEventRecord(b)); CK(hipEventSynchronize(b));
    float ms; CK(hipEventElapsedTime(&ms, a, b));
    printf("A stream+gather, one slice per wave: %.3f us per pass, %.2f G lane-gathers/s (padded)\n", ms * 1e3 / 200, h.size() / (ms * 1e-3 / 200) * 1e-9);
    fflush(stdout);
    // B: persistent waves, K slices per wave in registers
    for (int bpc : {1, 2, 4}) {
        const int G = 256 * bpc;            // blocks of 4 waves
        const int W = G * 4;
        const int K = (S + W - 1) / W;
        const int R = 100;
        if (K > 4) { printf("B bpc %d needs K=%d > 4, skipped\n", bpc, K); continue; }
        auto launch = [&](int r) {
            if (K == 1) hipLaunchKernelGGL(reg_gather<1>, dim3(G), dim3(256), 0, 0, dl, S, dy, dout, r);
            else if (K == 2) hipLaunchKernelGGL(reg_gather<2>, dim3(G), dim3(256), 0, 0, dl, S, dy, dout, r);
            else if (K == 3) hipLaunchKernelGGL(reg_gather<3>, dim3(G), dim3(256), 0, 0, dl, S, dy, dout, r);
            else hipLaunchKernelGGL(reg_gather<4>, dim3(G), dim3(256), 0, 0, dl, S, dy, dout, r);
        };
        launch(1); launch(R);
        CK(hipDeviceSynchronize());
        float t1, tR;
        CK(hipEventRecord(a)); launch(1); CK(hipEventRecord(b)); CK(hipEventSynchronize(b)); CK(hipEventElapsedTime(&t1, a, b));
        CK(hipEventRecord(a)); launch(R); CK(hipEventRecord(b)); CK(hipEventSynchronize(b)); CK(hipEventElapsedTime(&tR, a, b));
        const double per = (tR - t1) / (R - 1) * 1e3;
        printf("B regs, %d blocks/CU, K=%d slices per wave: %.3f us per gather pass (%.2f G lane-gathers/s padded)\n", bpc, K, per, (double)W * K * 16 * 64 / (per * 1e-6) * 1e-9);
        fflush(stdout);
    }
    return 0;
}
