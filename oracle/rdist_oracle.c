/*
 * rdist_oracle.c -- plain CPU reference for the R-distance (TEST INFRASTRUCTURE).
 *
 * This file is the oracle the GPU engine is checked against.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product path never links, loads or calls it, and it shares no code, header,
 * table or helper with the GPU engine.
 *
 * It is deliberately plain: IEEE double, round-to-nearest, no fused
 * multiply-add (built with -ffp-contract=off), no blocking, no reordering.
 * OpenMP is used only across rows of one elimination step, which leaves the
 * sequence of operations applied to every single entry unchanged.
 *
 * Paper: Jing & Meister, "A fast algorithm for All-Pairs-Shortest-Paths
 * suitable for neural networks" (arXiv 2308.07403).
 *
 * Convention (Sec. 2, adjacency equation): A[i*n + j] = 1 iff there is a
 * directed edge from node j to node i; D[i*n + j] is the distance from j to i.
 *
 * Readings of points the paper leaves open (each also listed in the design
 * notes of the repository):
 *   - ceil at exact integers: D = ceil(R - eta) with a small eta (default
 *     1e-9), i.e. the smallest k with Y >= gamma^(k + eta);
 *   - Y == 0 (no walk, Eq. Y-series) maps to the sentinel 0x7FFF;
 *   - D is clamped to [-32767, 32766] (int16) with a saturation count;
 *   - gamma is explicit (0 < gamma < 1) or AUTO: gamma = c / Delta with
 *     Delta the largest out-degree (Theorem 2's Delta, a column sum here);
 *     an edgeless graph gets gamma = c;
 *   - no pivoting; the gate gamma * Delta < 1 makes I - gamma*A column-wise
 *     strictly diagonally dominant, so every pivot is positive;
 *   - next hop: among the successors j of the current node (edge cur -> j),
 *     the one with the largest Y[goal, j] (Eq. descent, read as ascent on Y as
 *     in the proof of Theorem 4); lowest index on exact ties; -1 if no
 *     successor has Y > 0.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_ARG 1
#define ORC_E_ADJ 2
#define ORC_E_NOT_DD 3
#define ORC_E_PIVOT 4
#define ORC_E_NOMEM 5

#define ORC_UNREACHABLE 0x7FFF
#define ORC_D_MAX 32766
#define ORC_D_MIN (-32767)

/* ------------------------------------------------------------------------ */
/* Degree, gain and gate.                                                    */
/* ------------------------------------------------------------------------ */

/*
 * Validates A (entries in {0,1}, no self-loops: Sec. 3.1 footnote), computes
 * the out-degree of every node (column sums, since A[i,j] = 1 means j -> i),
 * Delta = max out-degree (Theorem 2), the gain, and the diagonal-dominance
 * gate gamma * Delta < 1 (the hypothesis of Theorem 4).
 *
 * gamma_arg > 0: explicit gain, must lie in (0, 1).
 * gamma_arg < 0: AUTO, gamma = |gamma_arg| / Delta (one IEEE division),
 *                or |gamma_arg| when Delta == 0.
 */
int orc_prepare(const uint8_t *A, int n, double gamma_arg, int32_t *outdeg,
                int32_t *delta_out, double *gamma_out) {
    if (n < 1 || !(gamma_arg == gamma_arg) || gamma_arg == 0.0) return ORC_E_ARG;
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) {
            uint8_t a = A[(size_t)i * n + j];
            if (a > 1) return ORC_E_ADJ;
            if (i == j && a != 0) return ORC_E_ADJ;
        }
    }
    int32_t delta = 0;
    for (int j = 0; j < n; ++j) {
        int32_t s = 0;
        for (int i = 0; i < n; ++i) s += A[(size_t)i * n + j];
        if (outdeg) outdeg[j] = s;
        if (s > delta) delta = s;
    }
    double gamma;
    if (gamma_arg > 0.0) {
        gamma = gamma_arg;
    } else {
        double c = -gamma_arg;
        gamma = delta > 0 ? c / (double)delta : c;
    }
    if (delta_out) *delta_out = delta;
    if (gamma_out) *gamma_out = gamma;
    if (!(gamma > 0.0) || !(gamma < 1.0)) return ORC_E_ARG;
    if (!(gamma * (double)delta < 1.0)) return ORC_E_NOT_DD;
    return ORC_OK;
}

/* M = I - gamma * A (Eq. Y-defined / inverse). */
void orc_build_m(const uint8_t *A, int n, double gamma, double *M) {
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            M[(size_t)i * n + j] = (i == j ? 1.0 : 0.0) - gamma * (double)A[(size_t)i * n + j];
}

/* ------------------------------------------------------------------------ */
/* Positive integer weights (Sec. 3.2, extension to weighted graphs).        */
/* ------------------------------------------------------------------------ */

/*
 * W[i*n + j] = weight of the edge j -> i (1 .. 255), 0 = no edge (weight
 * infinity, gamma^inf = 0).  Validation: no self-loops.  The out-degree of j
 * counts its out-edges; Delta, the gain and the gate are those of
 * orc_prepare.  The gate gamma * Delta < 1 bounds every column sum of
 * X = gamma^W (each entry is at most gamma), so I - X is column-wise strictly
 * diagonally dominant as in the unweighted case.
 */
int orc_prepare_weighted(const uint8_t *W, int n, double gamma_arg, int32_t *outdeg,
                         int32_t *delta_out, double *gamma_out) {
    if (n < 1 || !(gamma_arg == gamma_arg) || gamma_arg == 0.0) return ORC_E_ARG;
    for (int i = 0; i < n; ++i)
        if (W[(size_t)i * n + i] != 0) return ORC_E_ADJ;
    int32_t delta = 0;
    for (int j = 0; j < n; ++j) {
        int32_t s = 0;
        for (int i = 0; i < n; ++i) s += W[(size_t)i * n + j] != 0;
        if (outdeg) outdeg[j] = s;
        if (s > delta) delta = s;
    }
    double gamma;
    if (gamma_arg > 0.0) {
        gamma = gamma_arg;
    } else {
        double c = -gamma_arg;
        gamma = delta > 0 ? c / (double)delta : c;
    }
    if (delta_out) *delta_out = delta;
    if (gamma_out) *gamma_out = gamma;
    if (!(gamma > 0.0) || !(gamma < 1.0)) return ORC_E_ARG;
    if (!(gamma * (double)delta < 1.0)) return ORC_E_NOT_DD;
    return ORC_OK;
}

/* M = I - X with X_ij = gamma^W_ij (Eq. Y-taylor-series-integer), 0 where W_ij = 0. */
void orc_build_m_weighted(const uint8_t *W, int n, double gamma, double *M) {
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const uint8_t w = W[(size_t)i * n + j];
            M[(size_t)i * n + j] = (i == j ? 1.0 : 0.0) - (w ? pow(gamma, (double)w) : 0.0);
        }
}

/* ------------------------------------------------------------------------ */
/* Inversion: unblocked in-place Gauss-Jordan, natural order, no pivoting.   */
/* ------------------------------------------------------------------------ */

/*
 * Runs elimination steps k0 .. k1-1 of the in-place Gauss-Jordan inverse of
 * the n x n row-major matrix M.  Steps 0 .. n-1 together turn M into M^{-1}.
 * Step k: p = M[k,k]; M[k,k] = 1; row k /= p; then for every row i != k,
 * f = M[i,k]; M[i,k] = 0; row i -= f * row k.
 *
 * would_swap (nullable) counts the steps at which partial pivoting would have
 * chosen another row (some |M[i,k]| > |M[k,k]| with i > k).  Under the gate
 * it stays 0.  Returns ORC_E_PIVOT on a zero pivot.
 */
int orc_gj_steps(double *M, int n, int k0, int k1, int64_t *would_swap) {
    if (k0 < 0) k0 = 0;
    if (k1 > n) k1 = n;
    for (int k = k0; k < k1; ++k) {
        double *rk = M + (size_t)k * n;
        double p = rk[k];
        if (would_swap) {
            double ap = fabs(p);
            for (int i = k + 1; i < n; ++i)
                if (fabs(M[(size_t)i * n + k]) > ap) { ++*would_swap; break; }
        }
        if (p == 0.0 || !(p == p)) return ORC_E_PIVOT;
        rk[k] = 1.0;
        for (int j = 0; j < n; ++j) rk[j] = rk[j] / p;
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) {
            if (i == k) continue;
            double *ri = M + (size_t)i * n;
            double f = ri[k];
            ri[k] = 0.0;
            for (int j = 0; j < n; ++j) ri[j] = ri[j] - f * rk[j];
        }
    }
    return ORC_OK;
}

int orc_gj_invert(double *M, int n, int64_t *would_swap) {
    return orc_gj_steps(M, n, 0, n, would_swap);
}

/* ------------------------------------------------------------------------ */
/* Readout: R = log_gamma Y (Eq. R-defined), D = ceil(R - eta)              */
/* (Eq. rounded-distance-function with the eta reading), Y == 0 -> 0x7FFF.  */
/* ------------------------------------------------------------------------ */

/*
 * counts (nullable, 5 entries): [0] unreachable (Y == 0), [1] subnormal
 * (0 < Y < DBL_MIN), [2] saturated (clamped to the int16 range),
 * [3] ambiguous (R - eta within beta of an integer), [4] negative Y (never
 * expected: Y >= 0 for the gated M-matrix; mapped to the sentinel).
 */
void orc_readout(const double *Y, int n, double gamma, double eta, double beta,
                 int16_t *D, int64_t *counts) {
    int64_t c_unr = 0, c_sub = 0, c_sat = 0, c_amb = 0, c_neg = 0;
    double lg = log(gamma);
    size_t nn = (size_t)n * n;
#pragma omp parallel for schedule(static) reduction(+ : c_unr, c_sub, c_sat, c_amb, c_neg)
    for (size_t idx = 0; idx < nn; ++idx) {
        double y = Y[idx];
        if (y == 0.0) { D[idx] = ORC_UNREACHABLE; ++c_unr; continue; }
        if (y < 0.0 || !(y == y)) { D[idx] = ORC_UNREACHABLE; ++c_neg; continue; }
        if (y < DBL_MIN) ++c_sub;
        double r = log(y) / lg;
        double t = r - eta;
        double d = ceil(t);
        if (fabs(t - nearbyint(t)) < beta) ++c_amb;
        if (d > ORC_D_MAX) { d = ORC_D_MAX; ++c_sat; }
        if (d < ORC_D_MIN) { d = ORC_D_MIN; ++c_sat; }
        D[idx] = (int16_t)d;
    }
    if (counts) {
        counts[0] = c_unr; counts[1] = c_sub; counts[2] = c_sat; counts[3] = c_amb; counts[4] = c_neg;
    }
}

/* ------------------------------------------------------------------------ */
/* Full pipeline.                                                            */
/* ------------------------------------------------------------------------ */

/*
 * status, Delta, gamma; D (n*n int16, required); Y (n*n double, nullable:
 * when given, the inverse is left there).  counts as in orc_readout.  On a
 * non-OK status D is filled with the sentinel.
 */
int orc_solve(const uint8_t *A, int n, double gamma_arg, double eta, double beta,
              int16_t *D, double *Y, int32_t *delta_out, double *gamma_out,
              int64_t *counts, int64_t *would_swap) {
    int32_t delta = 0;
    double gamma = 0.0;
    int st = orc_prepare(A, n, gamma_arg, NULL, &delta, &gamma);
    if (delta_out) *delta_out = delta;
    if (gamma_out) *gamma_out = gamma;
    if (st != ORC_OK) {
        if (n > 0 && D)
            for (size_t idx = 0; idx < (size_t)n * n; ++idx) D[idx] = ORC_UNREACHABLE;
        return st;
    }
    double *M = Y;
    if (!M) {
        M = (double *)malloc(sizeof(double) * (size_t)n * n);
        if (!M) return ORC_E_NOMEM;
    }
    orc_build_m(A, n, gamma, M);
    st = orc_gj_invert(M, n, would_swap);
    if (st == ORC_OK) orc_readout(M, n, gamma, eta, beta, D, counts);
    if (M != Y) free(M);
    return st;
}

/*
 * orc_solve for a weighted graph (Sec. 3.2): gate of orc_prepare_weighted,
 * Y = (I - gamma^W)^{-1}, the same readout (Eq. distance-function-integer).
 */
int orc_solve_weighted(const uint8_t *W, int n, double gamma_arg, double eta, double beta,
                       int16_t *D, double *Y, int32_t *delta_out, double *gamma_out,
                       int64_t *counts, int64_t *would_swap) {
    int32_t delta = 0;
    double gamma = 0.0;
    int st = orc_prepare_weighted(W, n, gamma_arg, NULL, &delta, &gamma);
    if (delta_out) *delta_out = delta;
    if (gamma_out) *gamma_out = gamma;
    if (st != ORC_OK) {
        if (n > 0 && D)
            for (size_t idx = 0; idx < (size_t)n * n; ++idx) D[idx] = ORC_UNREACHABLE;
        return st;
    }
    double *M = Y;
    if (!M) {
        M = (double *)malloc(sizeof(double) * (size_t)n * n);
        if (!M) return ORC_E_NOMEM;
    }
    orc_build_m_weighted(W, n, gamma, M);
    st = orc_gj_invert(M, n, would_swap);
    if (st == ORC_OK) orc_readout(M, n, gamma, eta, beta, D, counts);
    if (M != Y) free(M);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Local pursuit (Eq. descent; Theorem 4 and its corollary).                 */
/* ------------------------------------------------------------------------ */

/*
 * Next hop from cur toward goal, given yg = row goal of Y (yg[j] = Y[goal][j]):
 * the successor j of cur (edge cur -> j) with the largest yg[j] > 0, the
 * lowest j on exact ties; cur itself at the goal; -1 without such a successor
 * or for an id out of range.  Only row goal of Y is read, so a single row
 * (computed by the series below) serves large graphs.
 */
int orc_next_hop_row(const uint8_t *A, const double *yg, int n, int cur, int goal) {
    if (cur < 0 || cur >= n || goal < 0 || goal >= n) return -1;
    if (cur == goal) return cur;
    int best = -1;
    double bestv = 0.0;
    for (int j = 0; j < n; ++j) {
        if (A[(size_t)j * n + cur] == 0) continue;   /* successor j: edge cur -> j (any weight) */
        if (yg[j] > bestv) { bestv = yg[j]; best = j; }
    }
    return best;
}

int orc_next_hop(const uint8_t *A, const double *Y, int n, int cur, int goal) {
    if (goal < 0 || goal >= n) return -1;
    return orc_next_hop_row(A, Y + (size_t)goal * n, n, cur, goal);
}

/*
 * out[0] = cur; out[h] = node after h greedy hops; once the goal is reached or
 * a hop fails the remaining entries are -1.  Writes max_hops + 1 entries.
 * orc_path_row takes row goal of Y only.
 */
void orc_path_row(const uint8_t *A, const double *yg, int n, int cur, int goal, int max_hops, int32_t *out) {
    for (int h = 0; h <= max_hops; ++h) out[h] = -1;
    out[0] = cur;
    int c = cur;
    for (int h = 1; h <= max_hops; ++h) {
        if (c == goal || c < 0) break;
        int nx = orc_next_hop_row(A, yg, n, c, goal);
        out[h] = nx;
        c = nx;
    }
}

void orc_path(const uint8_t *A, const double *Y, int n, int cur, int goal, int max_hops,
              int32_t *out) {
    if (goal < 0 || goal >= n) {
        for (int h = 0; h <= max_hops; ++h) out[h] = -1;
        out[0] = cur;
        return;
    }
    orc_path_row(A, Y + (size_t)goal * n, n, cur, goal, max_hops, out);
}

/* ------------------------------------------------------------------------ */
/* Single rows / columns of Y from the series Y = sum_k gamma^k A^k           */
/* (Sec. 3.1, Eq. inverse-series).  Used to check sampled outputs of a full-   */
/* size solve one by one.  Every term is non-negative, so each entry carries   */
/* a relative rounding error of at most (number of terms) * 2^-53.            */
/* ------------------------------------------------------------------------ */

/*
 * Column j: y = sum_k (gamma A)^k e_j, i.e. y[i] = Y[i][j].  The 1-norm of
 * gamma*A is gamma*Delta < 1 (column sums), so after term t the remaining
 * tail of every entry is at most |t|_1 * gamma*Delta / (1 - gamma*Delta).
 * Stops when the support has stopped growing (every reachable node has been
 * reached) and the tail is below rel_tol times the smallest positive entry,
 * or after max_terms.  Returns the number of terms used (-1 on bad input).
 */
int orc_y_column_series(const uint8_t *A, int n, double gamma, int j, double rel_tol, int max_terms,
                        double *y) {
    if (j < 0 || j >= n) return -1;
    int32_t *deg = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    for (int c = 0; c < n; ++c)
        for (int i = 0; i < n; ++i) deg[c + 1] += A[(size_t)i * n + c] == 1;
    int32_t delta = 0;
    for (int c = 0; c < n; ++c) if (deg[c + 1] > delta) delta = deg[c + 1];
    for (int c = 0; c < n; ++c) deg[c + 1] += deg[c];
    int32_t *adj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(deg[n] > 0 ? deg[n] : 1));
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    memcpy(fill, deg, sizeof(int32_t) * (size_t)n);
    for (int i = 0; i < n; ++i)
        for (int c = 0; c < n; ++c)
            if (A[(size_t)i * n + c] == 1) adj[fill[c]++] = i;      /* successors of c */
    double *t = (double *)calloc((size_t)n, sizeof(double));
    double *t2 = (double *)calloc((size_t)n, sizeof(double));
    for (int i = 0; i < n; ++i) y[i] = 0.0;
    y[j] = 1.0; t[j] = 1.0;
    double q = gamma * (double)delta;
    long support = 1, prev_support = 0;
    int k;
    for (k = 1; k <= max_terms; ++k) {
        for (int i = 0; i < n; ++i) t2[i] = 0.0;
        for (int c = 0; c < n; ++c) {
            double v = t[c];
            if (v == 0.0) continue;
            for (int e = deg[c]; e < deg[c + 1]; ++e) t2[adj[e]] += gamma * v;
        }
        double norm1 = 0.0, ymin = 1.0e308;
        support = 0;
        for (int i = 0; i < n; ++i) {
            y[i] += t2[i];
            norm1 += t2[i];
            if (y[i] > 0.0) { ++support; if (y[i] < ymin) ymin = y[i]; }
        }
        double *sw = t; t = t2; t2 = sw;
        if (norm1 == 0.0) break;
        int settled = support == prev_support;
        prev_support = support;
        if (settled && q < 1.0 && norm1 * q / (1.0 - q) < rel_tol * ymin) break;
    }
    free(deg); free(adj); free(fill); free(t); free(t2);
    return k;
}

/*
 * Row g: y = e_g^T sum_k (gamma A)^k, i.e. y[j] = Y[g][j].  Uses the
 * infinity norm: |x^T A|_inf <= |x|_inf * Delta, so the tail after term t is
 * at most |t|_inf * gamma*Delta / (1 - gamma*Delta).
 */
int orc_y_row_series(const uint8_t *A, int n, double gamma, int g, double rel_tol, int max_terms,
                     double *y) {
    if (g < 0 || g >= n) return -1;
    int32_t *deg = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));   /* predecessors of i */
    int32_t delta = 0;
    for (int c = 0; c < n; ++c) {
        int32_t s = 0;
        for (int i = 0; i < n; ++i) s += A[(size_t)i * n + c] == 1;
        if (s > delta) delta = s;
    }
    for (int i = 0; i < n; ++i)
        for (int c = 0; c < n; ++c) deg[i + 1] += A[(size_t)i * n + c] == 1;
    for (int i = 0; i < n; ++i) deg[i + 1] += deg[i];
    int32_t *adj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(deg[n] > 0 ? deg[n] : 1));
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    memcpy(fill, deg, sizeof(int32_t) * (size_t)n);
    for (int i = 0; i < n; ++i)
        for (int c = 0; c < n; ++c)
            if (A[(size_t)i * n + c] == 1) adj[fill[i]++] = c;
    double *t = (double *)calloc((size_t)n, sizeof(double));
    double *t2 = (double *)calloc((size_t)n, sizeof(double));
    for (int i = 0; i < n; ++i) y[i] = 0.0;
    y[g] = 1.0; t[g] = 1.0;
    double q = gamma * (double)delta;
    long support = 1, prev_support = 0;
    int k;
    for (k = 1; k <= max_terms; ++k) {
        /* (t^T gamma A)[c] = gamma * sum_i t[i] A[i][c]: scatter from every i to its predecessors c */
        for (int i = 0; i < n; ++i) t2[i] = 0.0;
        for (int i = 0; i < n; ++i) {
            double v = t[i];
            if (v == 0.0) continue;
            for (int e = deg[i]; e < deg[i + 1]; ++e) t2[adj[e]] += gamma * v;
        }
        double ninf = 0.0, ymin = 1.0e308;
        support = 0;
        for (int i = 0; i < n; ++i) {
            y[i] += t2[i];
            if (t2[i] > ninf) ninf = t2[i];
            if (y[i] > 0.0) { ++support; if (y[i] < ymin) ymin = y[i]; }
        }
        double *sw = t; t = t2; t2 = sw;
        if (ninf == 0.0) break;
        int settled = support == prev_support;
        prev_support = support;
        if (settled && q < 1.0 && ninf * q / (1.0 - q) < rel_tol * ymin) break;
    }
    free(deg); free(adj); free(fill); free(t); free(t2);
    return k;
}

/*
 * Row g of Y for a graph given as successor lists (the same series as
 * orc_y_row_series, Eq. Y-series, for graphs too large for a dense A):
 * the successors of node c are idx[ptr[c] .. ptr[c+1]), w (nullable) their
 * integer weights, so the entry of X for the edge c -> i is gamma^w (Sec. 3.2;
 * gamma itself without weights).  Term k+1 of the row is
 *   t2[c] = sum over successors i of c of x(c -> i) * t[i],
 * and the terms are summed until, with the support settled, the bound
 * |tail| <= max(t) q / (1 - q) (q = gamma * largest out-degree) is below
 * rel_tol times the smallest positive entry, or a term vanishes.
 * Returns the number of terms, or -1 for a bad g.
 */
int orc_y_row_series_csr(const int64_t *ptr, const int32_t *idx, const uint8_t *w, int n, double gamma, int g,
                         double rel_tol, int max_terms, double *y) {
    if (g < 0 || g >= n) return -1;
    int64_t delta = 0;
    for (int c = 0; c < n; ++c)
        if (ptr[c + 1] - ptr[c] > delta) delta = ptr[c + 1] - ptr[c];
    double *t = (double *)calloc((size_t)n, sizeof(double));
    double *t2 = (double *)calloc((size_t)n, sizeof(double));
    for (int i = 0; i < n; ++i) y[i] = 0.0;
    y[g] = 1.0; t[g] = 1.0;
    double q = gamma * (double)delta;
    long support = 1, prev_support = 0;
    int k;
    for (k = 1; k <= max_terms; ++k) {
        for (int c = 0; c < n; ++c) {
            double acc = 0.0;
            for (int64_t e = ptr[c]; e < ptr[c + 1]; ++e) {
                double x = w ? pow(gamma, (double)w[e]) : gamma;
                acc += x * t[idx[e]];
            }
            t2[c] = acc;
        }
        double ninf = 0.0, ymin = 1.0e308;
        support = 0;
        for (int i = 0; i < n; ++i) {
            y[i] += t2[i];
            if (t2[i] > ninf) ninf = t2[i];
            if (y[i] > 0.0) { ++support; if (y[i] < ymin) ymin = y[i]; }
        }
        double *sw = t; t = t2; t2 = sw;
        if (ninf == 0.0) break;
        int settled = support == prev_support;
        prev_support = support;
        if (settled && q < 1.0 && ninf * q / (1.0 - q) < rel_tol * ymin) break;
    }
    free(t); free(t2);
    return k;
}

/* ------------------------------------------------------------------------ */
/* Brute-force companions: BFS distances and shortest-path counts, and the   */
/* Floyd-Warshall CPU baseline.                                              */
/* ------------------------------------------------------------------------ */

/*
 * dist[i*n + j] = length of a shortest path from j to i (-1: unreachable);
 * count[i*n + j] = number of distinct shortest paths S_ij (Sec. 3.1), as a
 * double (nullable).
 */
void orc_bfs(const uint8_t *A, int n, int32_t *dist, double *count) {
    int32_t *deg = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) deg[j + 1] += A[(size_t)i * n + j] == 1;
    for (int j = 0; j < n; ++j) deg[j + 1] += deg[j];
    int32_t *adj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(deg[n] > 0 ? deg[n] : 1));
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    memcpy(fill, deg, sizeof(int32_t) * (size_t)n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            if (A[(size_t)i * n + j] == 1) adj[fill[j]++] = i;
#pragma omp parallel
    {
        int32_t *dj = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        double *cj = (double *)malloc(sizeof(double) * (size_t)n);
        int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
#pragma omp for schedule(dynamic, 16)
        for (int j = 0; j < n; ++j) {
            for (int v = 0; v < n; ++v) { dj[v] = -1; cj[v] = 0.0; }
            int head = 0, tail = 0;
            dj[j] = 0; cj[j] = 1.0; queue[tail++] = j;
            while (head < tail) {
                int u = queue[head++];
                for (int e = deg[u]; e < deg[u + 1]; ++e) {
                    int v = adj[e];
                    if (dj[v] < 0) { dj[v] = dj[u] + 1; queue[tail++] = v; }
                    if (dj[v] == dj[u] + 1) cj[v] += cj[u];
                }
            }
            for (int i = 0; i < n; ++i) {
                dist[(size_t)i * n + j] = dj[i];
                if (count) count[(size_t)i * n + j] = cj[i];
            }
        }
        free(dj); free(cj); free(queue);
    }
    free(deg); free(adj); free(fill);
}

#define ORC_FW_INF 0x3FFFFFFF

/*
 * Min-plus relaxation over intermediate nodes k0 .. k1-1 (k0 == 0 initialises
 * dist from A).  dist[i*n + j]: distance from j to i, ORC_FW_INF if none.
 */
void orc_floyd_warshall(const uint8_t *A, int n, int k0, int k1, int32_t *dist) {
    if (k0 == 0) {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                dist[(size_t)i * n + j] = i == j ? 0 : (A[(size_t)i * n + j] ? 1 : ORC_FW_INF);
    }
    if (k1 > n) k1 = n;
    for (int k = k0; k < k1; ++k) {
        const int32_t *rowk = dist + (size_t)k * n;   /* dist from j to k */
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) {
            int32_t *ri = dist + (size_t)i * n;
            int32_t dik = ri[k];                          /* from k to i */
            if (dik >= ORC_FW_INF) continue;
            for (int j = 0; j < n; ++j) {
                int32_t via = dik + rowk[j];
                if (via < ri[j]) ri[j] = via;
            }
        }
    }
}

int orc_num_threads(void) {
    int t = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            t = omp_get_num_threads();
#endif
        }
    }
    return t;
}
