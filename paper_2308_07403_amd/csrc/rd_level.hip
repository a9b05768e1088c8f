// rd_level.hip -- gfx950 kernels of the batched solves (rdist_solve_batched
// and the request loop) and their launchers:
//   k_batched    persistent kernel, each workgroup solves whole graphs
//                (register-resident for n <= 128, an in-workgroup blocked
//                solver for n <= 512), longest first;
//   k_lv_*       the level-synchronous blocked plan for graphs up to 4096:
//                every graph takes blocked step K in the same launches.
// The arithmetic per tile is the single-graph blocked plan's (rd_kernels.hip).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "rd_device.h"
#include "rd_gj.h"
#include "rd_launch.h"
#include "rd_tile_kd.h"

namespace rd {

__global__ void k_counter_zero(int32_t *p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

// p[0, count) = 0 for any count (grid-stride, 64-bit offsets).
__global__ void k_zero_words(int32_t *p, size_t count) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// One graph with 128 < n <= 512 on one workgroup: blocked Gauss-Jordan with
// b = 128 on the np x np matrix M in global memory (np = n rounded up to
// 128; padded rows and columns are identity).  Per block K: the panel inverse
// in registers, the row tiles V_J = P M_KJ and the negated transposed column
// tiles on the matrix cores, then every tile updated in place; the readout
// is fused into the last update.  The phases are separated by workgroup
// barriers, which make this workgroup's global writes visible to itself.
// Each phase is its own (not inlined) function so that each gets a register
// allocation of its own; registers are saved only at the phase boundaries.

// Panel: P = M_KK^{-1}; V_K = P, Pt = P^T.  Returns false on a bad pivot.
__device__ __noinline__ bool medium_panel(double *M, int np, int K, double *V, double *Pt, double *piv) {
    RegGJ<16, 16, 8, 8> g;
    const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
    const double *base = M + (size_t)K * kTile * np + (size_t)K * kTile;
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int c = 0; c < 8; ++c) g.m[a][c] = base[(size_t)(ty + 16 * a) * np + tx + 16 * c];
    const bool ok = g.invert(kTile, piv, ty, tx);
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int i = ty + 16 * a, k = tx + 16 * c;
            V[(size_t)i * np + (size_t)K * kTile + k] = g.m[a][c];
            Pt[(size_t)k * kTile + i] = g.m[a][c];
        }
    __syncthreads();
    return ok;
}

// Row tiles V_J = P M_KJ (J != K) and column tiles Ut_I = -(M_IK)^T (+I for I = K).
__device__ __noinline__ void medium_rowcol(const double *M, int np, int K, const double *Pt, double *Ut, double *V,
                                           double *lds) {
    const int nt = np / kTile;
    for (int J = 0; J < nt; ++J) {
        if (J == K) continue;
        TileAcc acc;
        acc.zero();
        tile_mma<kTile>(Pt, kTile, M + (size_t)K * kTile * np + (size_t)J * kTile, np, lds, acc);
        double *out = V + (size_t)J * kTile;
        tile_for_each(acc, [&](int r, int c, double v) { out[(size_t)r * np + c] = v; });
    }
    for (int I = 0; I < nt; ++I) {
        double *out = Ut + (size_t)I * kTile;
        if (I == K) {
            for (int e = threadIdx.x; e < kTile * kTile; e += 256) {
                const int k = e >> 7, i = e & 127;
                out[(size_t)k * np + i] = (k == i) ? 1.0 : 0.0;
            }
        } else {
            transpose_neg(M + (size_t)I * kTile * np + (size_t)K * kTile, np, 2, out, np, lds);
        }
    }
    __syncthreads();
}

// Every tile M_IJ <- M~_IJ + Ut_I^T V_J (M~: block row and column K zeroed).
__device__ __noinline__ void medium_update(double *M, int np, int K, const double *Ut, const double *V,
                                           double *lds) {
    const int nt = np / kTile;
    for (int I = 0; I < nt; ++I)
        for (int J = 0; J < nt; ++J) {
            double *tb = M + (size_t)I * kTile * np + (size_t)J * kTile;
            TileAcc acc;
            if (I == K || J == K) acc.zero();
            else tile_load_acc(acc, tb, np);
            tile_mma<kTile>(Ut + (size_t)I * kTile, np, V + (size_t)J * kTile, np, lds, acc);
            tile_for_each(acc, [&](int r, int c, double v) { tb[(size_t)r * np + c] = v; });
        }
    __syncthreads();
}

// The last update with the readout: D (n x n) from the final tiles; M keeps Y
// only when keep is set.  Readout counters are added to red[0..4] (LDS).
__device__ __noinline__ void medium_update_last(double *M, int np, int n, int K, const double *Ut, const double *V,
                                                double *lds, int16_t *D, int keep, double lg,
                                                unsigned long long *red) {
    const int nt = np / kTile;
    Counts cnt;
    for (int I = 0; I < nt; ++I)
        for (int J = 0; J < nt; ++J) {
            double *tb = M + (size_t)I * kTile * np + (size_t)J * kTile;
            TileAcc acc;
            if (I == K || J == K) acc.zero();
            else tile_load_acc(acc, tb, np);
            tile_mma<kTile>(Ut + (size_t)I * kTile, np, V + (size_t)J * kTile, np, lds, acc);
            tile_for_each(acc, [&](int r, int c, double y) {
                if (keep) tb[(size_t)r * np + c] = y;
                const int gi = I * kTile + r, gj = J * kTile + c;
                if (gi < n && gj < n) D[(size_t)gi * n + gj] = rd_encode(y, lg, cnt);
            });
        }
    unsigned long long v[5] = {wave_sum_u64(cnt.unreachable), wave_sum_u64(cnt.subnormal),
                               wave_sum_u64(cnt.saturated), wave_sum_u64(cnt.ambiguous),
                               wave_sum_u64(cnt.negative)};
    if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < 5; ++q)
            if (v[q]) atomicAdd(&red[q], v[q]);
    __syncthreads();
}

// Column sums (out-degrees) of the n x n byte matrix A (n <= 512) added into
// colsum (LDS, zeroed by the caller), and *bad set when an entry is not 0/1
// or the diagonal is not zero.  A is scanned flat, four bytes per load and
// four loads in flight per thread; only nonzero bytes cost more (sparse
// graphs: most words are zero).
__device__ __forceinline__ void adj_colsum(const uint8_t *__restrict__ A, int n, int *colsum, int *bad_flag) {
    const unsigned total = (unsigned)n * (unsigned)n;
    const unsigned un = (unsigned)n;
    int bad = 0;
    // bytes e0 .. e0+3 of the word v; (i, j) of byte e0 advanced without a
    // division per byte
    auto add_word = [&](unsigned e0, uint32_t v) {
        unsigned i = e0 / un, j = e0 - i * un;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const unsigned byte = (v >> (8 * b)) & 0xFFu;
            if (byte) {
                bad |= (byte > 1u) | (i == j);
                atomicAdd(&colsum[j], (int)byte);
            }
            if (++j == un) { j = 0; ++i; }
        }
    };
    unsigned done = 0;
    if ((reinterpret_cast<uintptr_t>(A) & 15) == 0) {
        // 16 bytes per load, 4 loads in flight per thread
        const uint4 *W = reinterpret_cast<const uint4 *>(A);
        const unsigned nq = total >> 4;
        for (unsigned q0 = threadIdx.x; q0 < nq; q0 += 4 * 256) {
            uint4 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = q0 + u * 256 < nq ? W[q0 + u * 256] : uint4{0u, 0u, 0u, 0u};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const unsigned e0 = 16u * (q0 + u * 256);
                if (v[u].x) add_word(e0, v[u].x);
                if (v[u].y) add_word(e0 + 4, v[u].y);
                if (v[u].z) add_word(e0 + 8, v[u].z);
                if (v[u].w) add_word(e0 + 12, v[u].w);
            }
        }
        done = nq << 4;
    }
    for (unsigned e = done + threadIdx.x; e < total; e += 256) {
        const unsigned byte = A[e];
        if (byte) {
            const unsigned i = e / un, j = e - i * un;
            bad |= (byte > 1u) | (i == j);
            atomicAdd(&colsum[j], (int)byte);
        }
    }
    if (bad) atomicOr(bad_flag, 1);
}

// Column sums of the bytes [b0, b1) of the n x n byte matrix A (flat,
// row-major) added into colsum[j] (LDS, zeroed by the caller), and *bad set
// as adj_colsum.  The 16-byte words inside the range are read 4 per thread
// in flight when A is 16-byte aligned; the bytes before the first and after
// the last whole word one at a time.  One division per nonzero word.
__device__ __forceinline__ void adj_colsum_range(const uint8_t *__restrict__ A, unsigned n, unsigned b0, unsigned b1,
                                                 int *colsum, int *bad_flag) {
    int bad = 0;
    auto add_byte = [&](unsigned e, unsigned byte) {
        const unsigned i = e / n, j = e - i * n;
        bad |= (byte > 1u) | (i == j);
        atomicAdd(&colsum[j], (int)byte);
    };
    auto add_word = [&](unsigned e0, uint32_t v) {
        unsigned i = e0 / n, j = e0 - i * n;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const unsigned byte = (v >> (8 * b)) & 0xFFu;
            if (byte) {
                bad |= (byte > 1u) | (i == j);
                atomicAdd(&colsum[j], (int)byte);
            }
            if (++j == n) { j = 0; ++i; }
        }
    };
    unsigned w0 = b1, w1 = b1;   // [w0, w1): the bytes covered by whole words
    if ((reinterpret_cast<uintptr_t>(A) & 15) == 0) {
        const unsigned q0 = (b0 + 15) >> 4, q1 = b1 >> 4;
        if (q1 > q0) {
            w0 = q0 << 4;
            w1 = q1 << 4;
            const uint4 *W = reinterpret_cast<const uint4 *>(A);
            for (unsigned q = q0 + threadIdx.x; q < q1; q += 4 * 256) {
                uint4 v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) v[u] = q + u * 256 < q1 ? W[q + u * 256] : uint4{0u, 0u, 0u, 0u};
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const unsigned e0 = 16u * (q + u * 256);
                    if (v[u].x) add_word(e0, v[u].x);
                    if (v[u].y) add_word(e0 + 4, v[u].y);
                    if (v[u].z) add_word(e0 + 8, v[u].z);
                    if (v[u].w) add_word(e0 + 12, v[u].w);
                }
            }
        }
    }
    for (unsigned e = b0 + threadIdx.x; e < w0; e += 256) {
        const unsigned byte = A[e];
        if (byte) add_byte(e, byte);
    }
    for (unsigned e = w1 + threadIdx.x; e < b1; e += 256) {
        const unsigned byte = A[e];
        if (byte) add_byte(e, byte);
    }
    if (bad) atomicOr(bad_flag, 1);
}

// Ingest of one graph: out-degrees, validation, Delta, gain, gate; M = I - gamma A.
__device__ __noinline__ int medium_ingest(const uint8_t *A, int n, int np, double gamma_arg, double *M, int *ints,
                                          int *delta_out, double *gamma_out) {
    int *colsum = ints;            // np
    int *flags = ints + 512;       // [0] bad, [1] delta
    for (int j = threadIdx.x; j < np; j += 256) colsum[j] = 0;
    if (threadIdx.x == 0) { flags[0] = 0; flags[1] = 0; }
    __syncthreads();
    adj_colsum(A, n, colsum, &flags[0]);
    __syncthreads();
    int m = 0;
    for (int j = threadIdx.x; j < n; j += 256) m = max(m, colsum[j]);
    atomicMax(&flags[1], m);
    __syncthreads();
    const int delta = flags[1];
    const double gamma = gamma_arg > 0.0 ? gamma_arg : (delta > 0 ? (-gamma_arg) / (double)delta : -gamma_arg);
    int st = RDIST_OK;
    if (flags[0]) st = RDIST_E_ADJ;
    else if (!(gamma > 0.0) || !(gamma < 1.0)) st = RDIST_E_ARG;
    else if (!(gamma * (double)delta < 1.0)) st = RDIST_E_NOT_DD;
    *delta_out = delta;
    *gamma_out = gamma;
    if (st == RDIST_OK) {
        const int half = np >> 1;
        for (int e = threadIdx.x; e < np * half; e += 256) {
            const int i = e / half, j = (e - (e / half) * half) * 2;
            double v[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                double x = (i == j + q) ? 1.0 : 0.0;
                if (i < n && j + q < n) x -= gamma * (double)A[(size_t)i * n + j + q];
                v[q] = x;
            }
            *reinterpret_cast<double2 *>(M + (size_t)i * np + j) = double2{v[0], v[1]};
        }
    }
    __syncthreads();
    return st;
}

__device__ __forceinline__ void solve_medium(const BatchTask &t, double *lds, double *piv, int *ints,
                                             unsigned long long *red) {
    const int n = t.n, np = t.np, nt = np / kTile;
    int delta;
    double gamma;
    int st = medium_ingest(t.A, n, np, t.gamma_arg, t.M, ints, &delta, &gamma);
    bool ok = st == RDIST_OK;
    if (ok) {
        if (threadIdx.x < 5) red[threadIdx.x] = 0;
        __syncthreads();
        for (int K = 0; K < nt && ok; ++K) {
            ok = medium_panel(t.M, np, K, t.V, t.Pt, piv);
            medium_rowcol(t.M, np, K, t.Pt, t.Ut, t.V, lds);
            if (K + 1 < nt) medium_update(t.M, np, K, t.Ut, t.V, lds);
            else medium_update_last(t.M, np, n, K, t.Ut, t.V, lds, t.D, t.keep, rd_inv_log(gamma), red);
        }
        if (!ok) st = RDIST_E_NOT_DD;
    }
    if (st != RDIST_OK)
        for (int e = threadIdx.x; e < n * n; e += 256) t.D[e] = kUnreachable;
    if (threadIdx.x == 0) {
        rdist_info *info = t.info;
        info->status = st;
        info->delta = delta;
        info->gamma = gamma;
        info->n_unreachable = st == RDIST_OK ? (int64_t)red[0] : 0;
        info->n_subnormal = st == RDIST_OK ? (int64_t)red[1] : 0;
        info->n_saturated = st == RDIST_OK ? (int64_t)red[2] : 0;
        info->n_ambiguous = st == RDIST_OK ? (int64_t)red[3] : 0;
        info->n_negative = st == RDIST_OK ? (int64_t)red[4] : 0;
        info->n_uncertified = 0;
        info->fallback_fraction = 0.0;
    }
    __syncthreads();
}

// Persistent batched solve: each workgroup pulls task indices from *counter
// (tasks are sorted by decreasing n, longest first) and solves the graph
// alone: register-resident Gauss-Jordan for n <= 128, the in-workgroup
// blocked solver for n <= 512.  Every workgroup exits once the counter
// passes the task count.
__global__ __launch_bounds__(256, 2) void k_batched(const BatchTask *__restrict__ tasks, int count, int *counter,
                                                 double *__restrict__ scratch, int scratch_stride) {
    __shared__ double lds[kTileLdsDoubles];
    __shared__ double piv[8 * kTile];   // RegGJ<16, 16, 8, 8>::kScratch
    __shared__ int ints[512 + 2];
    __shared__ unsigned long long red[8];
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        __syncthreads();
        const int idx = next;
        __syncthreads();
        if (idx >= count) break;
        BatchTask t = tasks[idx];
        if (t.n <= 64) {
            SmallTask s{t.A, t.D, t.keep ? t.M : nullptr, t.n, t.np, t.gamma_arg, t.info};
            solve_small<16, 16, 4, 4>(s, piv, ints);
        } else if (t.n <= 128) {
            SmallTask s{t.A, t.D, t.keep ? t.M : nullptr, t.n, t.np, t.gamma_arg, t.info};
            solve_small<16, 16, 8, 8>(s, piv, ints);
        } else {
            double *sc = scratch + (size_t)blockIdx.x * scratch_stride;
            t.Ut = sc;
            t.V = sc + (size_t)kTile * t.np;
            t.Pt = sc + (size_t)2 * kTile * t.np;
            solve_medium(t, lds, piv, ints, red);
        }
    }
}

// ---------------------------------------------------------------------------
// Level-synchronous batched blocked Gauss-Jordan for 128 < n <= 4096: every
// graph of the batch takes step K in the same launches (panel, row and
// column tiles, trailing update), so one graph's tiles run on many compute
// units at once.  Each launch reads its work from a unit list built on the
// host: unit u = (graph << kLvShift) | item, or -1 for an idle slot.  The
// host keeps a small graph's units on the workgroups of one XCD (workgroup
// b runs on XCD b % 8) so that its operand slabs share one L2, and splits a
// large graph's units into contiguous runs of tile rows, one run per XCD.
// Step K uses the step buffers of parity K & 1, so step K+1's panel and
// row/column tiles (on a second stream) never overwrite what step K's update
// still reads.
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool lv_unit(const int *units, int &g, int &item) {
    const int u = units[blockIdx.x];
    if (u < 0) return false;
    g = u >> kLvShift;
    item = u & ((1 << kLvShift) - 1);
    return true;
}

// Column sums of one row chunk (item): rows [item * rows_per, + rows_per)
// of A summed per column in LDS, then added into the graph's column sums
// (zeroed before the launch) with one atomic per nonzero column; the
// validation flag is or-ed into colsum[n].
__global__ __launch_bounds__(256) void k_lv_colsum(const LevelGraph *__restrict__ gs, const int *__restrict__ units) {
    int gi, item;
    if (!lv_unit(units, gi, item)) return;
    const LevelGraph g = gs[gi];
    __shared__ int colsum[kLvMaxN];
    __shared__ int bad;
    const int n = g.n;
    for (int j = threadIdx.x; j < n; j += 256) colsum[j] = 0;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    const int r0 = item * g.rows_per, r1 = min(n, r0 + g.rows_per);
    adj_colsum_range(g.A, (unsigned)n, (unsigned)r0 * (unsigned)n, (unsigned)r1 * (unsigned)n, colsum, &bad);
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += 256) {
        const int v = colsum[j];
        if (v) atomicAdd(&g.colsum[j], v);
    }
    if (threadIdx.x == 0 && bad) atomicOr(&g.colsum[n], 1);
}

// Gate, one workgroup per graph: Delta (the largest column sum), the gain
// and the diagonal-dominance test, then info (status, delta, gamma, zeroed
// counters).
__global__ __launch_bounds__(256) void k_lv_gate(const LevelGraph *__restrict__ gs) {
    __shared__ int flags[2];
    const LevelGraph g = gs[blockIdx.x];
    if (threadIdx.x == 0) { flags[0] = 0; flags[1] = 0; }
    __syncthreads();
    const int n = g.n;
    int m = 0;
    for (int j = threadIdx.x; j < n; j += 256) m = max(m, g.colsum[j]);
    const int bad = threadIdx.x == 0 ? g.colsum[n] : 0;
    if (m) atomicMax(&flags[1], m);
    if (bad) atomicOr(&flags[0], 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        const int delta = flags[1];
        const double gamma = g.gamma_arg > 0.0 ? g.gamma_arg
                                               : (delta > 0 ? (-g.gamma_arg) / (double)delta : -g.gamma_arg);
        int st = RDIST_OK;
        if (flags[0]) st = RDIST_E_ADJ;
        else if (!(gamma > 0.0) || !(gamma < 1.0)) st = RDIST_E_ARG;
        else if (!(gamma * (double)delta < 1.0)) st = RDIST_E_NOT_DD;
        rdist_info *info = g.info;
        info->status = st;
        info->delta = delta;
        info->gamma = gamma;
        info->n_unreachable = info->n_subnormal = info->n_saturated = 0;
        info->n_ambiguous = info->n_negative = info->n_uncertified = 0;
        info->fallback_fraction = 0.0;
    }
}

// Step 0's inputs from the adjacency: items [0, nt) are the M tiles (0, J)
// of block row 0 (I - gamma A, identity on the padding), read by the panel
// and the row tiles; items [nt, 2nt-1) are the column operand blocks
// Ut_I = -(M_I0)^T for I >= 1, i.e. Ut[k][128 I + i] = gamma A[128 I + i][k]
// (these entries are off the diagonal).  Step 0's update forms its other
// starting tiles straight from A.
__global__ __launch_bounds__(256) void k_lv_build(const LevelGraph *__restrict__ gs, const int *__restrict__ units) {
    int gi, item;
    if (!lv_unit(units, gi, item)) return;
    const LevelGraph g = gs[gi];
    if (g.info->status != RDIST_OK) return;
    const double gamma = g.info->gamma;
    const int nt = g.nt, n = g.n, np = g.np;
    const uint8_t *__restrict__ A = g.A;
    double *__restrict__ M = g.M;
    if (item < nt) {
        const int J = item;
        for (int e = threadIdx.x; e < kTile * kTile / 2; e += 256) {
            const int i = e >> 6, j = J * kTile + (e & 63) * 2;
            double v[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                double x = (i == j + q) ? 1.0 : 0.0;
                if (i < n && j + q < n) x -= gamma * (double)A[(size_t)i * n + j + q];
                v[q] = x;
            }
            *reinterpret_cast<double2 *>(M + (size_t)i * np + j) = double2{v[0], v[1]};
        }
        return;
    }
    // the 128 x 128 byte block A[128 I + i][k] staged in LDS (rows read
    // coalesced, padded to 132 bytes), then written transposed
    __shared__ uint8_t blk[kTile * 132];
    const int I = item - nt + 1;
    for (int e = threadIdx.x; e < kTile * kTile; e += 256) {
        const int ii = e >> 7, k = e & 127;
        const int i = I * kTile + ii;
        blk[ii * 132 + k] = (i < n && k < n) ? A[(size_t)i * n + k] : (uint8_t)0;
    }
    __syncthreads();
    double *out = g.Ut[0] + (size_t)I * kTile;
    for (int e = threadIdx.x; e < kTile * kTile; e += 256) {
        const int k = e >> 7, ii = e & 127;
        out[(size_t)k * np + ii] = gamma * (double)blk[ii * 132 + k];
    }
}

// Panel of step K (item unused).
__global__ __launch_bounds__(256, 2) void k_lv_panel(const LevelGraph *__restrict__ gs, const int *__restrict__ units,
                                                     int K) {
    int gi, item;
    if (!lv_unit(units, gi, item)) return;
    const LevelGraph g = gs[gi];
    if (g.info->status != RDIST_OK) return;
    __builtin_amdgcn_s_setprio(3);   // lookahead chain: ahead of the update's waves on shared SIMDs
    __shared__ PanelLds lds;
    const int par = K & 1;
    // the last block holds n - 128 K pivots; its padding is an identity
    const int pivots = K == g.nt - 1 ? g.n - K * kTile : kTile;
    panel_core(g.M, g.np, K, g.Pt[par], g.V[par], g.np, g.info, lds, pivots);
}

// Row tiles of step K: items [0, nt-1) are V_J = P M_KJ for the tile
// columns J != K (the column operand Ut of step K is written by the build for
// K = 0 and by the edge update of step K-1 otherwise).  On a graph's last
// step the product runs over the block's pivot rows only.
__global__ __launch_bounds__(256, 2) void k_lv_rowcol(const LevelGraph *__restrict__ gs,
                                                      const int *__restrict__ units, int K) {
    int gi, item;
    if (!lv_unit(units, gi, item)) return;
    const LevelGraph g = gs[gi];
    if (g.info->status != RDIST_OK) return;
    __builtin_amdgcn_s_setprio(3);   // lookahead chain: ahead of the update's waves on shared SIMDs
    __shared__ double lds[kTileLdsDoubles];
    const int np = g.np, par = K & 1;
    const int J = item < K ? item : item + 1;
    const int kd = K == g.nt - 1 ? lv_last_inner(g.n, g.nt) : kTile;
    TileAcc acc;
    acc.zero();
    tile_mma_kd(kd, g.Pt[par], kTile, g.M + (size_t)K * kTile * np + (size_t)J * kTile, np, lds, acc);
    double *out = g.V[par] + (size_t)J * kTile;
    tile_for_each(acc, [&](int r, int c, double v) { out[(size_t)r * np + c] = v; });
}

// acc = tile (I, J) of I - gamma A (identity on the padding), in the
// accumulator layout: step 0's starting value for tiles outside block row
// and column 0, read from the adjacency bytes instead of a built M.
__device__ __forceinline__ void tile_acc_from_adj(TileAcc &acc, const uint8_t *__restrict__ A, int n, int I, int J,
                                                  double gamma) {
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = I * kTile + tile_row(p, r), j = J * kTile + tile_col(q);
                double x = (i == j) ? 1.0 : 0.0;
                if (i < n && j < n) x -= gamma * (double)A[(size_t)i * n + j];
                acc.v[p][q][r] = x;
            }
}

// Trailing update of step K over the tiles of `kind`, L = K + 1:
//   kLvDiag  the diagonal tile (L, L), all that step L's panel reads;
//   kLvEdge  the rest of tile row and column L (what step L's row tiles and
//            column operand read): items [0, nt-1) are (L, j), j != L, items
//            [nt-1, 2nt-2) are (i, L), i != L.  A column tile is not stored
//            to M: it is written straight into step L's column operand as
//            -(M'_iL)^T;
//   kLvRest  the other tiles: (nt-1)^2 items skipping row and column L when
//            L < nt, all nt^2 tiles (item = I nt + J) on the graph's last step.
// Block row K is V itself (U_K = -I), copied without a product.  On a
// graph's last step the product runs over the block's pivot rows only, and
// the tile's final value is read out into D (stored to M only with keep); a
// refused graph gets the sentinel there instead.
__global__ __launch_bounds__(256, 2) void k_lv_update(const LevelGraph *__restrict__ gs,
                                                      const int *__restrict__ units, int K, int kind) {
    int gi, item;
    if (!lv_unit(units, gi, item)) return;
    const LevelGraph g = gs[gi];
    const int np = g.np, nt = g.nt, n = g.n, par = K & 1;
    const int L = K + 1;
    const bool last = L == nt;
    int I, J;
    if (kind == kLvDiag) {
        I = J = L;
    } else if (kind == kLvEdge) {
        if (item < nt - 1) { I = L; J = item < L ? item : item + 1; }
        else { const int ip = item - (nt - 1); I = ip < L ? ip : ip + 1; J = L; }
    } else if (last) {
        I = item / nt;
        J = item - (item / nt) * nt;
    } else {
        const int w = nt - 1;
        const int ip = item / w, jp = item - (item / w) * w;
        I = ip < L ? ip : ip + 1;
        J = jp < L ? jp : jp + 1;
    }
    if (g.info->status != RDIST_OK) {
        if (last)
            for (int e = threadIdx.x; e < kTile * kTile; e += 256) {
                const int gi2 = I * kTile + (e >> 7), gj = J * kTile + (e & 127);
                if (gi2 < n && gj < n) g.D[(size_t)gi2 * n + gj] = kUnreachable;
            }
        return;
    }
    __shared__ double lds[kTileLdsDoubles];
    double *base = g.M + (size_t)I * kTile * np + (size_t)J * kTile;
    TileAcc acc;
    if (I == K) {
        tile_load_acc(acc, g.V[par] + (size_t)J * kTile, np);
    } else {
        const int kd = last ? lv_last_inner(n, nt) : kTile;
        const double *ut = g.Ut[par] + (size_t)I * kTile, *v = g.V[par] + (size_t)J * kTile;
        if (J == K) acc.zero();
        else if (K == 0) tile_acc_from_adj(acc, g.A, n, I, J, g.info->gamma);
        else tile_load_acc(acc, base, np);
        tile_mma_kd(kd, ut, np, v, np, lds, acc);
    }
    if (kind == kLvEdge && J == L && I != L) {
        double *out = g.Ut[par ^ 1] + (size_t)I * kTile;     // -(M'_IL)^T, k-major
        tile_for_each(acc, [&](int r, int c, double v) { out[(size_t)c * np + r] = -v; });
    } else if (!last) {
        tile_for_each(acc, [&](int r, int c, double v) { base[(size_t)r * np + c] = v; });
    } else {
        const double il = rd_inv_log(g.info->gamma);
        const int keep = g.keep;
        Counts cnt;
        tile_for_each(acc, [&](int r, int c, double y) {
            if (keep) base[(size_t)r * np + c] = y;
            const int gi2 = I * kTile + r, gj = J * kTile + c;
            if (gi2 < n && gj < n) g.D[(size_t)gi2 * n + gj] = rd_encode(y, il, cnt);
        });
        flush_counts(g.info, cnt);
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

void launch_batched(const BatchTask *tasks, int count, int *counter, int grid, double *scratch, int scratch_stride,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_counter_zero, dim3(1), dim3(64), 0, s, counter, 1);
    hipLaunchKernelGGL(k_batched, dim3(grid), dim3(256), 0, s, tasks, count, counter, scratch, scratch_stride);
}

int batched_blocks_per_cu() {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, (const void *)k_batched, 256, 0) != hipSuccess || b < 1) {
        (void)hipGetLastError();
        b = 1;
    }
    return b;
}

void launch_fill_i32(int32_t *p, size_t count, hipStream_t s) {
    if (!count) return;
    const size_t blocks = std::min<size_t>((count + 255) / 256, (size_t)1 << 16);
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)blocks), dim3(256), 0, s, p, count);
}

void launch_lv_gate(const LevelGraph *gs, int count, hipStream_t s) {
    hipLaunchKernelGGL(k_lv_gate, dim3(count), dim3(256), 0, s, gs);
}

void launch_lv(int phase, const LevelGraph *gs, const int *units, int grid, int K, hipStream_t s) {
    switch (phase) {
        case kLvColsum: hipLaunchKernelGGL(k_lv_colsum, dim3(grid), dim3(256), 0, s, gs, units); break;
        case kLvBuild: hipLaunchKernelGGL(k_lv_build, dim3(grid), dim3(256), 0, s, gs, units); break;
        case kLvPanel: hipLaunchKernelGGL(k_lv_panel, dim3(grid), dim3(256), 0, s, gs, units, K); break;
        case kLvRowcol: hipLaunchKernelGGL(k_lv_rowcol, dim3(grid), dim3(256), 0, s, gs, units, K); break;
        default: hipLaunchKernelGGL(k_lv_update, dim3(grid), dim3(256), 0, s, gs, units, K, phase); break;
    }
}

}  // namespace rd
