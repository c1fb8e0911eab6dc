/*
 * gn_oracle.c -- plain, slow, fp64 CPU reference of Weighted Regularized Graph
 * Normalization (WRGN) for Maximum Weight Independent Set.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or load
 * this file; it exists so that tests, the smoke check and the benchmark's CPU
 * baseline can check the HIP library against an implementation written
 * directly from the paper.  It shares no code with the HIP library.
 *
 * Notation follows the paper: G = (A, w) simple undirected, w > 0, v = sqrt(w),
 * state x in [0,1]^n, weighted state y = v (.) x, closed regularized adjacency
 * B = I + gamma A.  Every loop below runs in CSR order in double precision; no
 * blocking, fusion or reordering.
 *
 * The same source also builds an all-core variant (gcc -fopenmp) used only as
 * the benchmark's second CPU baseline: the per-row loops of a step and of the
 * stopping test then run their rows on several threads.  Each row's sum keeps
 * its CSR order and the only reductions across rows are max, min and integer
 * counts, so both builds return bit-identical results (tested).
 */
#include <float.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_E_ARG (-1)
#define ORC_E_CSR (-2)
#define ORC_E_SELF_LOOP (-3)
#define ORC_E_ASYMMETRIC (-4)
#define ORC_E_WEIGHT (-5)
#define ORC_E_NOT_NORMALIZABLE (-6)

/* Safe-division constants of the paper's PyTorch module (code appendix):
 * a closed-neighbourhood sum at or below 1e-9 resets the node to 1/2. */
static const double ORC_SAFE_DIV = 1e-9;
static const double ORC_FALLBACK_X = 0.5;
/* Support invariance (Section 2, property ii): a positive coordinate stays
 * positive, since x'_i = y_i / s_i > 0 whenever y_i > 0.  fp64 breaks this only
 * by underflow: a decaying value would reach an exact 0, which is a fixed point,
 * and a vertex that later should regrow (its neighbourhood lost the set) could
 * not.  So a positive x'_i below fp64's smallest normal number 2^-1022 is held
 * at 2^-1022; above it the map is computed as written.  The level can be moved
 * (orc_set_x_floor) only so that tests can show that results do not depend on
 * it. */
static double orc_x_floor = DBL_MIN; /* 2^-1022 */

void orc_set_x_floor(double f) { orc_x_floor = f > 0.0 ? f : DBL_MIN; }
double orc_get_x_floor(void) { return orc_x_floor; }

/* Threads the row loops use: 1 in the plain build. */
int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------------------
 * Problem statement checks (Section 2): A is the adjacency matrix of a simple
 * undirected graph (symmetric, A_ii = 0), w strictly positive.
 * ------------------------------------------------------------------------- */
static int has_entry(const int32_t* rp, const int32_t* ci, int32_t row, int32_t col) {
    int64_t lo = rp[row], hi = (int64_t)rp[row + 1] - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (ci[mid] == col) return 1;
        if (ci[mid] < col) lo = mid + 1; else hi = mid - 1;
    }
    return 0;
}

int orc_validate(int32_t n, int64_t nnz, const int32_t* rp, const int32_t* ci, const double* w) {
    if (n < 0 || nnz < 0) return ORC_E_ARG;
    if (rp[0] != 0 || (int64_t)rp[n] != nnz) return ORC_E_CSR;
    for (int32_t i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) return ORC_E_CSR;
    for (int32_t i = 0; i < n; ++i) {
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            int32_t j = ci[e];
            if (j < 0 || j >= n) return ORC_E_CSR;
            if (j == i) return ORC_E_SELF_LOOP;
            if (e > rp[i] && ci[e - 1] >= j) return ORC_E_CSR;  /* sorted, no duplicates */
        }
    }
    for (int32_t i = 0; i < n; ++i)
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
            if (!has_entry(rp, ci, ci[e], i)) return ORC_E_ASYMMETRIC;
    for (int32_t i = 0; i < n; ++i)
        if (!(w[i] > 0.0) || !isfinite(w[i])) return ORC_E_WEIGHT;
    return ORC_OK;
}

/* gamma-pursuit (Section 6, "Tracking the global minimum by gamma-pursuit", and
 * the code appendix): p = k/(T-1), gamma = p*gamma1 + (1-p)*gamma0 for k < T,
 * held at gamma1 afterwards.  T <= 1 means constant gamma1. */
double orc_gamma(double gamma0, double gamma1, int32_t ramp, int64_t k) {
    if (ramp <= 1) return gamma1;
    int64_t kk = k < ramp - 1 ? k : ramp - 1;
    double p = (double)kk / (double)(ramp - 1);
    return p * gamma1 + (1.0 - p) * gamma0;
}

/* One WRGN step (Definition WRGN; y-space form of the energy-descent proof;
 * safe division of the code appendix):
 *     y_i = v_i x_i,  s_i = y_i + gamma * sum_{j in N(i)} y_j,
 *     x'_i = y_i / s_i   if s_i > 1e-9,   x'_i = 1/2 otherwise,
 * and a positive x'_i is kept >= 2^-1022 (support invariance, see orc_x_floor).
 * Returns how many nodes took the 1/2 fallback.  x and x_out may alias. */
int64_t orc_step(int32_t n, const int32_t* rp, const int32_t* ci, const double* v,
                 double gamma, const double* x, double* x_out) {
    double* y = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int32_t i = 0; i < n; ++i) y[i] = v[i] * x[i];
    int64_t fallback = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(+ : fallback)
    for (int32_t i = 0; i < n; ++i) {
        double nb = 0.0;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) nb += y[ci[e]];
        double s = gamma * nb + y[i];
        if (s > ORC_SAFE_DIV) {
            double xn = y[i] / s;
            if (y[i] > 0.0 && xn < orc_x_floor) xn = orc_x_floor;
            x_out[i] = xn;
        } else {
            x_out[i] = ORC_FALLBACK_X;
            ++fallback;
        }
    }
    free(y);
    return fallback;
}

/* Closed-neighbourhood sums (A + I) x (Section 2), used for the normalizable
 * check: x is normalizable iff every closed-neighbourhood sum is positive. */
int orc_is_normalizable(int32_t n, const int32_t* rp, const int32_t* ci, const double* x) {
    for (int32_t i = 0; i < n; ++i) {
        if (!(x[i] >= 0.0) || !isfinite(x[i])) return ORC_E_ARG;
    }
    for (int32_t i = 0; i < n; ++i) {
        double s = x[i];
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) s += x[ci[e]];
        if (!(s > 0.0)) return ORC_E_NOT_NORMALIZABLE;
    }
    return ORC_OK;
}

/* Binarisation test on a state x (this implementation's stopping rule; the
 * paper runs a fixed number of steps):
 *   r         = max_i min(x_i, 1 - x_i)                      (distance to binary)
 *   uncovered = #{i : x_i <= 1/2 and no neighbour j has x_j > 1/2}  (maximality,
 *               Section 2)
 *   growing   = #{i : 0 < x_i <= 1/2 and s_i <= v_i}, s = (I + gamma A)(v (.) x):
 *               non-selected nodes that the next step would not shrink, since
 *               x'_i / x_i = v_i / s_i.  At a binary point s_i / v_i is the
 *               per-node term of the stability equation of Theorem "Binary
 *               Regularization", so growing = 0 is stab > 1 for the current state. */
void orc_binarisation(int32_t n, const int32_t* rp, const int32_t* ci, const double* w,
                      double gamma, const double* x, double* r_out, int64_t* uncovered_out,
                      int64_t* growing_out) {
    double r = 0.0;
    int64_t unc = 0, grow = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(max : r) reduction(+ : unc, grow)
    for (int32_t i = 0; i < n; ++i) {
        double d = x[i] < 1.0 - x[i] ? x[i] : 1.0 - x[i];
        if (d > r) r = d;
        if (x[i] > 0.5) continue;
        int covered = 0;
        double nb = 0.0;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            int32_t j = ci[e];
            if (x[j] > 0.5) covered = 1;
            nb += sqrt(w[j]) * x[j];
        }
        if (!covered) ++unc;
        double vi = sqrt(w[i]);
        double s = gamma * nb + vi * x[i];
        if (x[i] > 0.0 && !(s > vi)) ++grow;
    }
    *r_out = r;
    *uncovered_out = unc;
    *growing_out = grow;
}

/* Relaxed MWIS objective sum_i w_i x_i (weighted mass, Theorem "Weighted Mass
 * Growth": M_v(y) = sum v_i y_i = sum w_i x_i). */
double orc_objective(int32_t n, const double* w, const double* x) {
    double f = 0.0;
    for (int32_t i = 0; i < n; ++i) f += w[i] * x[i];
    return f;
}

/* Independence 1_S^T A 1_S = 0 (each violating undirected edge counted once) and
 * maximality (nodes outside S with no neighbour in S), Section 2. */
void orc_check(int32_t n, const int32_t* rp, const int32_t* ci, const uint8_t* sel,
               int64_t* conflicts, int64_t* uncovered) {
    int64_t c = 0, u = 0;
    for (int32_t i = 0; i < n; ++i) {
        int any = 0;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            int32_t j = ci[e];
            if (sel[j]) any = 1;
            if (sel[i] && sel[j] && i < j) ++c;
        }
        if (!sel[i] && !any) ++u;
    }
    *conflicts = c;
    *uncovered = u;
}

/* gamma-stability of a set M (Theorem "Binary Regularization", stability
 * equation): stab = gamma * min_{i not in M} sum_{j in N(i) cap M} sqrt(w_j/w_i).
 * +inf when every node is in M. */
double orc_stab(int32_t n, const int32_t* rp, const int32_t* ci, const double* w,
                double gamma, const uint8_t* sel) {
    double best = INFINITY;
    for (int32_t i = 0; i < n; ++i) {
        if (sel[i]) continue;
        double s = 0.0;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            int32_t j = ci[e];
            if (sel[j]) s += sqrt(w[j] / w[i]);
        }
        if (gamma * s < best) best = gamma * s;
    }
    return best;
}

/* Energy in weighted state space (Section 3 and its proof appendix):
 * E(y) = 1/2 y^T (I + gamma A) y - v^T y. */
double orc_energy(int32_t n, const int32_t* rp, const int32_t* ci, const double* w,
                  double gamma, const double* y) {
    double q = 0.0, lin = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        double by = y[i];
        double nb = 0.0;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) nb += y[ci[e]];
        by += gamma * nb;
        q += y[i] * by;
        lin += sqrt(w[i]) * y[i];
    }
    return 0.5 * q - lin;
}

typedef struct {
    double gamma0, gamma1;
    int32_t ramp_steps, max_steps;
    double tau;
    int32_t check_every;
} orc_schedule;

typedef struct {
    int32_t steps, binarised;
    int64_t fallback_count;
    double relaxed_objective, set_objective;
    int64_t set_size, conflicts, uncovered;
    double stab;
    double residual;
    int64_t growing;
} orc_result;

/* Iterate WRGN from x0 to binarisation (Section 6 schedule; stopping rule of
 * this implementation: at steps k >= 1 that are multiples of check_every, or
 * at k = max_steps, stop when r <= tau, the rounded set covers V and no
 * non-selected node would grow under gamma_k; see orc_binarisation).  Output
 * x is clamped to [0,1] as in the code appendix, the selected set is
 * S = {i : x_i > 1/2}. */
int orc_solve(int32_t n, const int32_t* rp, const int32_t* ci, const double* w,
              const orc_schedule* sch, double* x, uint8_t* sel, orc_result* res) {
    if (sch->max_steps < 0 || sch->check_every < 1 || !(sch->tau >= 0.0)) return ORC_E_ARG;
    int st = orc_is_normalizable(n, rp, ci, x);
    if (st != ORC_OK) return st;
    double* v = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int32_t i = 0; i < n; ++i) v[i] = sqrt(w[i]);
    int64_t fb = 0;
    int32_t k = 0;
    int binarised = 0;
    double r = 0.0;
    int64_t unc = 0, grow = 0;
    if (n == 0) binarised = 1;   /* the empty set is the only (vacuous) MIS */
    while (!binarised) {
        if (k >= 1 && (k % sch->check_every == 0 || k == sch->max_steps)) {
            double gk = orc_gamma(sch->gamma0, sch->gamma1, sch->ramp_steps, k);
            orc_binarisation(n, rp, ci, w, gk, x, &r, &unc, &grow);
            if (r <= sch->tau && unc == 0 && grow == 0) { binarised = 1; break; }
        }
        if (k == sch->max_steps) break;
        double g = orc_gamma(sch->gamma0, sch->gamma1, sch->ramp_steps, k);
        fb += orc_step(n, rp, ci, v, g, x, x);
        ++k;
    }
    if (k == 0)
        orc_binarisation(n, rp, ci, w, orc_gamma(sch->gamma0, sch->gamma1, sch->ramp_steps, 0),
                         x, &r, &unc, &grow);
    for (int32_t i = 0; i < n; ++i) {
        if (x[i] < 0.0) x[i] = 0.0;
        if (x[i] > 1.0) x[i] = 1.0;
        sel[i] = x[i] > 0.5 ? 1 : 0;
    }
    res->steps = k;
    res->binarised = binarised;
    res->fallback_count = fb;
    res->relaxed_objective = orc_objective(n, w, x);
    double W = 0.0;
    int64_t size = 0;
    for (int32_t i = 0; i < n; ++i)
        if (sel[i]) { W += w[i]; ++size; }
    res->set_objective = W;
    res->set_size = size;
    orc_check(n, rp, ci, sel, &res->conflicts, &res->uncovered);
    /* stability is reported under gamma_k, the gamma the stopping test used */
    double g_fin = orc_gamma(sch->gamma0, sch->gamma1, sch->ramp_steps, k);
    res->stab = orc_stab(n, rp, ci, w, g_fin, sel);
    res->residual = r;
    res->growing = grow;
    free(v);
    return binarised ? ORC_OK : ORC_NOT_CONVERGED;
}

/* T unrolled WRGN steps with gammas[t] (no stopping test); xs holds x^0..x^T
 * row by row, (T+1) * n doubles.  Returns total fallback count. */
int64_t orc_unrolled_forward(int32_t n, const int32_t* rp, const int32_t* ci, const double* w,
                             const double* gammas, int32_t T, const double* x0, double* xs) {
    double* v = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int32_t i = 0; i < n; ++i) v[i] = sqrt(w[i]);
    memcpy(xs, x0, sizeof(double) * (size_t)n);
    int64_t fb = 0;
    for (int32_t t = 0; t < T; ++t)
        fb += orc_step(n, rp, ci, v, gammas[t], xs + (size_t)t * n, xs + (size_t)(t + 1) * n);
    free(v);
    return fb;
}

/* Reverse-mode derivative of T unrolled steps, by the chain rule applied to
 * the step above.  For x' = y (/) s with y = v (.) x and s = (I + gamma A) y:
 *   dL/dy = gbar (/) s - (I + gamma A) t,   t = gbar (.) y (/) s^2
 * (I + gamma A is symmetric), dL/dx = v (.) dL/dy, dL/dv += x (.) dL/dy, and
 * dL/dw = dL/dv (/) (2 v) since v = sqrt(w).  Rows that took the 1/2 fallback
 * or sit at the 2^-1022 floor are constant and pass no gradient.  gxT = dL/dx^T on input; outputs the
 * gradient through the dynamics only (gw, gx0). */
void orc_unrolled_vjp(int32_t n, const int32_t* rp, const int32_t* ci, const double* w,
                      const double* gammas, int32_t T, const double* x0, const double* gxT,
                      double* gw, double* gx0) {
    size_t N = (size_t)(n > 0 ? n : 1);
    double* xs = (double*)malloc(sizeof(double) * N * (size_t)(T + 1));
    orc_unrolled_forward(n, rp, ci, w, gammas, T, x0, xs);
    double* v = (double*)malloc(sizeof(double) * N);
    double* y = (double*)malloc(sizeof(double) * N);
    double* s = (double*)malloc(sizeof(double) * N);
    double* a = (double*)malloc(sizeof(double) * N);
    double* t = (double*)malloc(sizeof(double) * N);
    double* gbar = (double*)malloc(sizeof(double) * N);
    double* gv = (double*)calloc(N, sizeof(double));
    for (int32_t i = 0; i < n; ++i) v[i] = sqrt(w[i]);
    memcpy(gbar, gxT, sizeof(double) * (size_t)n);
    for (int32_t k = T - 1; k >= 0; --k) {
        const double* x = xs + (size_t)k * n;
        double g = gammas[k];
        for (int32_t i = 0; i < n; ++i) y[i] = v[i] * x[i];
        for (int32_t i = 0; i < n; ++i) {
            double nb = 0.0;
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e) nb += y[ci[e]];
            s[i] = g * nb + y[i];
            if (s[i] > ORC_SAFE_DIV && !(y[i] > 0.0 && y[i] / s[i] < orc_x_floor)) {
                a[i] = gbar[i] / s[i];
                t[i] = gbar[i] * y[i] / (s[i] * s[i]);
            } else {
                a[i] = 0.0;
                t[i] = 0.0;
            }
        }
        for (int32_t i = 0; i < n; ++i) {
            double nb = 0.0;
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e) nb += t[ci[e]];
            double gy = a[i] - (t[i] + g * nb);
            gv[i] += x[i] * gy;
            gbar[i] = v[i] * gy;
        }
    }
    for (int32_t i = 0; i < n; ++i) {
        gx0[i] = gbar[i];
        gw[i] = gv[i] / (2.0 * v[i]);
    }
    free(xs); free(v); free(y); free(s); free(a); free(t); free(gbar); free(gv);
}
