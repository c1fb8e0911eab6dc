// Per-launch control of one solve step (device code), shared by the graph and
// assignment step kernels.  `Args` provides solve, st, k, notconv, gamma and
// gamma_scalar.
#pragma once

#include <hip/hip_runtime.h>

#include "gn_types.h"

namespace {

// Per-launch control of one step.  In solve mode the kernel first reads the
// solve state (done step, error bits, the previous step's test flag, gamma);
// the decision to skip the step is taken only after each thread's first row
// loads are in flight, so the two memory round trips overlap.
template <typename Args>
struct StepCtl {
    float g = 0.0f, tau = 0.0f;
    bool do_test = false, do_write = true, solve = false;
    int k = 0, km = 0, ms = 0, ce = 1, done = -1, err = 0, nc_prev = 1;

    // Solve-mode loads.  Called after the thread has issued its column loads:
    // scalar loads complete in any order, so a wait for the row offsets would
    // otherwise also wait for these.
    __device__ __forceinline__ void fetch(const Args& a) {
        if (!a.solve) {
            g = a.gamma_scalar;
            return;
        }
        const SolveState* st = a.st;
        solve = true;
        k = a.k;
        km = a.k >= 1 ? a.k - 1 : 0;
        done = st->done_step;
        err = st->err;
        ms = st->max_steps;
        ce = st->check_every;
        tau = st->tau;
        nc_prev = a.notconv[km];
        g = a.gamma[a.k];
        do_test = k >= 1 && (k % ce == 0 || k == ms);
        do_write = k < ms;
    }

    // false: this launch does no work (the solve has stopped, or the previous
    // step's state passed the test, which block 0 records).  Uniform over the grid.
    __device__ __forceinline__ bool proceed(const Args& a) const {
        if (!solve) return true;
        if (k > ms || done >= 0 || err) return false;
        if (k >= 2 && (km % ce == 0 || km == ms) && nc_prev == 0) {
            if (blockIdx.x == 0 && threadIdx.x == 0) a.st->done_step = km;
            return false;
        }
        return true;
    }
};

}  // namespace
