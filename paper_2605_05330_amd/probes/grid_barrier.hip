// Measurement probe (not part of libgn): the cost of a grid-wide barrier inside
// one persistent launch, against the cost of a kernel launch, on one MI355X.  It
// decides whether a persistent solve (one launch, a grid barrier between steps)
// can beat the chained step launches.
//
// Build and run (repository root):
//     hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         -o /tmp/grid_barrier paper_2605_05330_amd/probes/grid_barrier.hip && /tmp/grid_barrier
//
// All blocks are co-resident (cooperative launch).  Every waiting loop is bounded
// (2^20 polls, then a shared timeout flag that every block checks), so the kernel
// always ends.  Each block writes its iteration number before the barrier and
// reads another block's after it: a count of stale reads checks the ordering.
// Variants: one counter with a release fetch-add per block (mode 0), a release
// fence then a relaxed add (1), the same with s_sleep in the poll (2), a
// two-level counter tree (3), and the tree with per-group release flags 4 KiB
// apart (4).  Every variant polls with relaxed agent-scope loads and issues one
// acquire fence after its wait.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>
#include <vector>

#define CK(x) do { hipError_t e = (x); if (e != hipSuccess) { printf("HIP error %s at %d\n", hipGetErrorString(e), __LINE__); return 1; } } while (0)

// Two-level barrier: groups of 16 blocks count on their own line; the group's last
// arriver counts on the top line; the last of those publishes the generation.
__global__ __launch_bounds__(256) void tree_barrier_kernel(unsigned* cnt, int iters, int* slots, int* bad, int* timeout) {
    const unsigned G = gridDim.x;
    const unsigned ng = (G + 15) / 16;
    const unsigned grp = blockIdx.x / 16;
    const unsigned gsz = min(16u, G - grp * 16);
    unsigned* top = cnt + 64 * ng;
    unsigned* gen = cnt + 64 * (ng + 1);
    int mism = 0;
    for (int it = 0; it < iters; ++it) {
        if (threadIdx.x == 0) slots[blockIdx.x * 64] = it;
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned o1 = __hip_atomic_fetch_add(cnt + 64 * grp, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            if (o1 == (unsigned)(it + 1) * gsz - 1u) {
                const unsigned o2 = __hip_atomic_fetch_add(top, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
                if (o2 == (unsigned)(it + 1) * ng - 1u)
                    __hip_atomic_store(gen, (unsigned)(it + 1), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
            unsigned spins = 0;
            while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (unsigned)(it + 1)) {
                if (++spins > (1u << 20)) { atomicOr(timeout, 1); break; }
                if ((spins & 1023u) == 0u && __hip_atomic_load(timeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const int other = (blockIdx.x + 37) % G;
            const int v = __hip_atomic_load(slots + other * 64, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (v < it) ++mism;
        }
        if (__hip_atomic_load(timeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
    }
    if (threadIdx.x == 0 && mism) atomicAdd(bad, mism);
}

// Two-level barrier with distributed release: group counters and group flags
// 4 KiB apart; each group's last arriver counts on the top line, the last of
// those publishes the generation; group leaders poll the generation and set
// their group's flag, the other blocks poll their group's flag.
constexpr int kSp = 1024;   // 4 KiB between lines
__global__ __launch_bounds__(256) void tree2_barrier_kernel(unsigned* cnt, int iters, int* slots, int* bad, int* timeout) {
    const unsigned G = gridDim.x;
    const unsigned ng = (G + 15) / 16;
    const unsigned grp = blockIdx.x / 16;
    const unsigned gsz = min(16u, G - grp * 16);
    const bool leader = (blockIdx.x % 16) == 0;
    unsigned* gc = cnt + kSp * grp;             // group counter
    unsigned* gf = cnt + kSp * (ng + grp);      // group flag
    unsigned* top = cnt + kSp * (2 * ng);
    unsigned* gen = cnt + kSp * (2 * ng + 1);
    int mism = 0;
    for (int it = 0; it < iters; ++it) {
        if (threadIdx.x == 0) slots[blockIdx.x * 64] = it;
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned want = (unsigned)(it + 1);
            const unsigned o1 = __hip_atomic_fetch_add(gc, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            if (o1 == want * gsz - 1u) {
                const unsigned o2 = __hip_atomic_fetch_add(top, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
                if (o2 == want * ng - 1u) __hip_atomic_store(gen, want, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
            unsigned* poll = leader ? gen : gf;
            unsigned spins = 0;
            while (__hip_atomic_load(poll, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < want) {
                if (++spins > (1u << 20)) { atomicOr(timeout, 1); break; }
                if ((spins & 1023u) == 0u && __hip_atomic_load(timeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
            }
            if (leader) __hip_atomic_store(gf, want, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const int other = (blockIdx.x + 37) % G;
            const int v = __hip_atomic_load(slots + other * 64, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (v < it) ++mism;
        }
        if (__hip_atomic_load(timeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
    }
    if (threadIdx.x == 0 && mism) atomicAdd(bad, mism);
}

template <int MODE>
__global__ __launch_bounds__(256) void barrier_kernel(unsigned* cnt, int iters, int* slots, int* bad, int* timeout) {
    const unsigned G = gridDim.x;
    int mism = 0;
    for (int it = 0; it < iters; ++it) {
        if (threadIdx.x == 0) slots[blockIdx.x * 64] = it;   // one slot per 256-byte line
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned target = (unsigned)(it + 1) * G;
            if (MODE == 0) {
                __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            unsigned spins = 0;
            while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                if (MODE == 2) __builtin_amdgcn_s_sleep(1);
                if (++spins > (1u << 20)) { atomicOr(timeout, 1); break; }
                if ((spins & 1023u) == 0u && __hip_atomic_load(timeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const int other = (blockIdx.x + 37) % G;
            const int v = __hip_atomic_load(slots + other * 64, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (v < it) ++mism;
        }
        if (__hip_atomic_load(timeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
    }
    if (threadIdx.x == 0 && mism) atomicAdd(bad, mism);
}

__global__ void empty_kernel(int* p) { if (p && threadIdx.x == 1023) p[0] = 0; }

template <int MODE>
int run(int bpc, int iters, int ncu) {
    const void* kfun = MODE == 4 ? (const void*)tree2_barrier_kernel
                     : MODE == 3 ? (const void*)tree_barrier_kernel : (const void*)barrier_kernel<MODE>;
    int occ = 0;
    CK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kfun, 256, 0));
    if (bpc > occ) { printf("mode %d bpc %d > occupancy %d, skipped\n", MODE, bpc, occ); return 0; }
    const int G = bpc * ncu;
    unsigned* cnt; int *slots, *bad, *timeout;
    const size_t cbytes = (size_t)4 * 1024 * (2 * (G / 16 + 1) + 4);
    CK(hipMalloc(&cnt, cbytes)); CK(hipMalloc(&slots, G * 64 * 4)); CK(hipMalloc(&bad, 4)); CK(hipMalloc(&timeout, 4));
    hipEvent_t a, b; CK(hipEventCreate(&a)); CK(hipEventCreate(&b));
    float best = 1e30f, ms0 = 0;
    for (int rep = 0; rep < 3; ++rep) {
        CK(hipMemset(cnt, 0, cbytes)); CK(hipMemset(slots, 0xff, G * 64 * 4)); CK(hipMemset(bad, 0, 4)); CK(hipMemset(timeout, 0, 4));
        CK(hipDeviceSynchronize());
        void* args[] = {&cnt, &iters, &slots, &bad, &timeout};
        CK(hipEventRecord(a));
        CK(hipLaunchCooperativeKernel(kfun, dim3(G), dim3(256), args, 0, 0));
        CK(hipEventRecord(b));
        CK(hipEventSynchronize(b));
        float ms; CK(hipEventElapsedTime(&ms, a, b));
        if (ms < best) best = ms;
    }
    int hbad, hto; CK(hipMemcpy(&hbad, bad, 4, hipMemcpyDeviceToHost)); CK(hipMemcpy(&hto, timeout, 4, hipMemcpyDeviceToHost));
    printf("mode %d blocks/CU %d grid %d iters %d: %.3f us per barrier (kernel %.3f ms) mismatches %d timeout %d\n",
           MODE, bpc, G, iters, best * 1e3 / iters, best, hbad, hto);
    CK(hipFree(cnt)); CK(hipFree(slots)); CK(hipFree(bad)); CK(hipFree(timeout));
    return 0;
}

int main() {
    hipDeviceProp_t p; CK(hipGetDeviceProperties(&p, 0));
    const int ncu = p.multiProcessorCount;
    printf("device %s CUs %d clock %d kHz\n", p.gcnArchName, ncu, p.clockRate);
    fflush(stdout);
    // launch cost of an empty full-chip kernel, back to back
    {
        hipEvent_t a, b; CK(hipEventCreate(&a)); CK(hipEventCreate(&b));
        for (int w = 0; w < 10; ++w) hipLaunchKernelGGL(empty_kernel, dim3(ncu * 4), dim3(256), 0, 0, nullptr);
        CK(hipEventRecord(a));
        for (int w = 0; w < 1000; ++w) hipLaunchKernelGGL(empty_kernel, dim3(ncu * 4), dim3(256), 0, 0, nullptr);
        CK(hipEventRecord(b)); CK(hipEventSynchronize(b));
        float ms; CK(hipEventElapsedTime(&ms, a, b));
        printf("empty kernel (%d blocks) back to back: %.3f us per launch\n", ncu * 4, ms);
        fflush(stdout);
    }
    for (int bpc : {1, 2, 4}) {
        if (bpc > 1) { if (run<4>(bpc, 2000, ncu)) return 1; continue; }
        if (run<0>(bpc, 2000, ncu)) return 1;
        if (run<1>(bpc, 2000, ncu)) return 1;
        if (run<2>(bpc, 2000, ncu)) return 1;
        if (run<3>(bpc, 2000, ncu)) return 1;
        if (run<4>(bpc, 2000, ncu)) return 1;
        fflush(stdout);
    }
    return 0;
}
