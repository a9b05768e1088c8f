// rd_device.h -- device building blocks of the R-distance engine (gfx950).
//
// Shared by the kernels of this library only.  Three pieces:
//   * rd_encode: the readout D = ceil(log_gamma Y - eta) with the unreachable
//     sentinel (paper Eq. R-defined and the rounded distance function of
//     Sec. 4.1.1);
//   * RegGJ: an in-place Gauss-Jordan inverse of a small matrix held in the
//     registers of one workgroup, one rank-1 step per pivot, pivot row and
//     column broadcast through LDS (the inverse of Eq. Y-defined for n <= 128
//     and for the diagonal blocks of the blocked solver);
//   * tile_mma: a 128 x 128 FP64 tile contraction on the matrix cores,
//     C -= A_k^T B_k over an inner dimension that is a multiple of 16, operands
//     staged through LDS (the trailing update of blocked Gauss-Jordan).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rdist.h"

namespace rd {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr double kEta = 1e-9;     // ceil(R - eta): exact integers stay integers
constexpr double kLn2 = 0.69314718055994530942;
constexpr double kBeta = 1e-10;   // ambiguity band reported around k + eta
constexpr int16_t kUnreachable = RDIST_UNREACHABLE;
constexpr double kDMax = 32766.0;
constexpr double kDMin = -32767.0;
constexpr double kDblMin = 2.2250738585072014e-308;

// Per-thread counters of the readout; reduced per workgroup before the atomics.
struct Counts {
    unsigned long long unreachable = 0, subnormal = 0, saturated = 0, ambiguous = 0, negative = 0;
};

__device__ __forceinline__ int16_t rd_clamp_d(double d, Counts &c) {
    if (d > kDMax) { d = kDMax; ++c.saturated; }
    if (d < kDMin) { d = kDMin; ++c.saturated; }
    return (int16_t)(int)d;
}

// D for one entry.  il = 1 / log(gamma) < 0: t = R - eta with
// R = log(Y) / log(gamma) formed as a product with the reciprocal (within an
// ulp or two of the quotient; the eta shift keeps exact integers R on the
// right side), D = ceil(t).
//
// Most entries take a short path: Y = m 2^e (m in [1, 2), e from the
// exponent bits) gives log(Y) = (e + log2 m) ln 2, with log2 m from the
// hardware FP32 logarithm of m rounded to FP32 (measured on gfx950 over
// every FP32 input in [1, 2): at most 6e-8 from log2; with the rounding of
// m, below 1.5e-7; 1e-6 is assumed).  The estimate te of t is then within
// 1e-6 |ln 2 il| + 1e-12 of t.  When no integer lies within
// band = 1e-4 + 4e-6 |ln 2 il| of te, ceil(te) = ceil(t) and t is not
// ambiguous, so D is the one the full FP64 logarithm gives.  Entries near an
// integer (exact distances, unique shortest walks with tiny corrections)
// and subnormal Y take the full FP64 logarithm.
__device__ __forceinline__ int16_t rd_encode(double y, double il, Counts &c) {
    if (y == 0.0) { ++c.unreachable; return kUnreachable; }
    if (!(y > 0.0)) { ++c.negative; return kUnreachable; }
    if (y >= kDblMin) {
        const unsigned long long bits = (unsigned long long)__double_as_longlong(y);
        const int e = (int)((bits >> 52) & 0x7FFull) - 1023;
        const double m = __longlong_as_double((long long)((bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull));
        const double l2m = (double)__builtin_amdgcn_logf((float)m);
        const double s = kLn2 * il;
        const double te = ((double)e + l2m) * s - kEta;
        const double band = 1e-4 - 4e-6 * s;   // s < 0
        if (fabs(te - rint(te)) > band) return rd_clamp_d(ceil(te), c);
    } else {
        ++c.subnormal;
    }
    const double t = log(y) * il - kEta;
    if (fabs(t - rint(t)) < kBeta) ++c.ambiguous;
    return rd_clamp_d(ceil(t), c);
}

__device__ __forceinline__ double rd_inv_log(double gamma) { return 1.0 / log(gamma); }

// 1/p from the hardware reciprocal estimate and one Newton step on the
// residual e = 1 - p*r (fused, so e is exact): |error| of order 1 ulp,
// without the long dependent sequence of the IEEE division.
__device__ __forceinline__ double recip(double p) {
    const double r0 = __builtin_amdgcn_rcp(p);
    const double e = fma(-p, r0, 1.0);
    return fma(r0, e, r0);
}

// The kernels of the lookahead chain (the next block's diagonal update, its
// inverse and its row and column tiles) run beside the big update and are
// on the critical path: their waves take the highest issue priority on the
// SIMDs they share with the update's waves.
__device__ __forceinline__ void lookahead_priority() { __builtin_amdgcn_s_setprio(3); }

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Adds a workgroup's counters to info (one atomic per counter per wave).
__device__ __forceinline__ void flush_counts(rdist_info *info, Counts c) {
    unsigned long long u = wave_sum_u64(c.unreachable);
    unsigned long long s = wave_sum_u64(c.subnormal);
    unsigned long long t = wave_sum_u64(c.saturated);
    unsigned long long a = wave_sum_u64(c.ambiguous);
    unsigned long long ng = wave_sum_u64(c.negative);
    if ((threadIdx.x & 63) == 0) {
        if (u) atomicAdd((unsigned long long *)&info->n_unreachable, u);
        if (s) atomicAdd((unsigned long long *)&info->n_subnormal, s);
        if (t) atomicAdd((unsigned long long *)&info->n_saturated, t);
        if (a) atomicAdd((unsigned long long *)&info->n_ambiguous, a);
        if (ng) atomicAdd((unsigned long long *)&info->n_negative, ng);
    }
}

// ---------------------------------------------------------------------------
// Register-resident Gauss-Jordan on an NP x NP matrix, NP = TY*RA = TX*RC.
// Thread (ty, tx) owns rows ty + TY*a and columns tx + TX*c (strided, so the
// pivot row and column reads from LDS are contiguous across lanes).
//
// One elimination step k, written uniformly for all entries (row k and column
// k of the old matrix replaced by zeros in `o`):
//     c_i = (i == k) ? -1 : M[i][k]
//     r_j = (j == k) ? 1/p : M[k][j] / p          with p = M[k][k]
//     M'[i][j] = o[i][j] - c_i * r_j
// which gives M'[k][k] = 1/p, M'[k][j] = M[k][j]/p, M'[i][k] = -M[i][k]/p and
// M'[i][j] = M[i][j] - M[i][k] M[k][j] / p: the in-place Gauss-Jordan step.
// ---------------------------------------------------------------------------
template <int TY, int TX, int RA, int RC>
struct RegGJ {
    static constexpr int NP = TY * RA;
    static_assert(TY * RA == TX * RC, "square tile");
    static constexpr int NT = TY * TX;
    double m[RA][RC];

    // LDS scratch of run / invert, in doubles: pivot rows and columns of two
    // steps, double-buffered.
    static constexpr int kScratch = 8 * NP;

    // Elimination steps k in [k_begin, k_end).  Returns false (uniformly) if
    // a pivot is not strictly positive.
    // Step k = TY*ka + kt: the pivot row is register row ka of the lanes with
    // ty == kt, the pivot column register column ka of the lanes with
    // tx == kt (square thread grid).  The loop over ka is unrolled, so the
    // register indices are compile-time and the fix-ups of the pivot row and
    // column are a few lane selects; every entry costs one FMA per step.
    // Steps are taken two per workgroup barrier: rows and columns k and k+1
    // are published together, and every lane forms row and column k+1 after
    // step k itself, with the FMAs their owners would have used, so the
    // result is bitwise that of one step per barrier.
    __device__ __forceinline__ bool run(int k_begin, int k_end, double *lds, int ty, int tx) {
        static_assert(TY == TX && RA == RC, "square thread grid and register tile");
        bool ok = true;
        int phase = 0;
        run_from<0>(k_begin, k_end, lds, ty, tx, ok, phase);
        return ok;
    }

    template <int KA>
    __device__ __forceinline__ void run_from(int k_begin, int k_end, double *lds, int ty, int tx, bool &ok,
                                             int &phase) {
        if constexpr (KA < RA) {
            steps<KA>(k_begin, k_end, lds, ty, tx, ok, phase);
            run_from<KA + 1>(k_begin, k_end, lds, ty, tx, ok, phase);
        }
    }

    // The step with pivot row ci / column rj factors already formed: zero
    // the pivot row and column (register row and column ka of the owning
    // lanes) and apply the rank-1 update.
    template <int ka>
    __device__ __forceinline__ void apply(bool rowk, bool colk, const double (&ci)[RA], const double (&rj)[RC]) {
#pragma unroll
        for (int c = 0; c < RC; ++c) m[ka][c] = rowk ? 0.0 : m[ka][c];
#pragma unroll
        for (int a = 0; a < RA; ++a) m[a][ka] = colk ? 0.0 : m[a][ka];
#pragma unroll
        for (int a = 0; a < RA; ++a)
#pragma unroll
            for (int c = 0; c < RC; ++c) m[a][c] = fma(-ci[a], rj[c], m[a][c]);
    }

    template <int ka>
    __device__ __forceinline__ void steps(int k_begin, int k_end, double *lds, int ty, int tx, bool &ok, int &phase) {
        const int kt0 = k_begin > ka * TY ? k_begin - ka * TY : 0;
        const int kt1 = k_end < (ka + 1) * TY ? k_end - ka * TY : TY;
        int kt = kt0;
        for (; kt + 1 < kt1; kt += 2) {
            const int k = ka * TY + kt, k1 = k + 1;
            double *r0 = lds + phase * (4 * NP);   // row k, row k+1, column k, column k+1
            double *r1 = r0 + NP, *c0 = r0 + 2 * NP, *c1 = r0 + 3 * NP;
            phase ^= 1;
            const bool rowk = ty == kt, colk = tx == kt, rowk1 = ty == kt + 1, colk1 = tx == kt + 1;
            if (rowk || rowk1) {
                double *rb = rowk ? r0 : r1;
#pragma unroll
                for (int c = 0; c < RC; ++c) rb[tx + TX * c] = m[ka][c];
            }
            if (colk || colk1) {
                double *cb = colk ? c0 : c1;
#pragma unroll
                for (int a = 0; a < RA; ++a) cb[ty + TY * a] = m[a][ka];
            }
            __syncthreads();
            // step k
            const double p = c0[k];
            ok = ok && (p > 0.0);
            const double rp = recip(p);
            double ci[RA], rj[RC];
#pragma unroll
            for (int a = 0; a < RA; ++a) ci[a] = c0[ty + TY * a];
#pragma unroll
            for (int c = 0; c < RC; ++c) rj[c] = r0[tx + TX * c] * rp;
            ci[ka] = rowk ? -1.0 : ci[ka];
            rj[ka] = colk ? rp : rj[ka];
            // row k+1 and column k+1 after step k (entries of row / column k
            // are zero before the update), and the pivot p' = M'[k+1][k+1]
            const double r = c0[k1], q1 = r0[k1] * rp;
            const double p1 = fma(-r, q1, r1[k1]);
            ok = ok && (p1 > 0.0);
            const double rp1 = recip(p1);
            double ci1[RA], rj1[RC];
#pragma unroll
            for (int a = 0; a < RA; ++a) {
                const double o = (rowk && a == ka) ? 0.0 : c1[ty + TY * a];
                ci1[a] = fma(-ci[a], q1, o);
            }
#pragma unroll
            for (int c = 0; c < RC; ++c) {
                const double o = (colk && c == ka) ? 0.0 : r1[tx + TX * c];
                rj1[c] = fma(-r, rj[c], o) * rp1;
            }
            ci1[ka] = rowk1 ? -1.0 : ci1[ka];
            rj1[ka] = colk1 ? rp1 : rj1[ka];
            apply<ka>(rowk, colk, ci, rj);
            apply<ka>(rowk1, colk1, ci1, rj1);
        }
        if (kt < kt1) {
            const int k = ka * TY + kt;
            double *rb = lds + phase * (4 * NP);
            double *cb = rb + 2 * NP;
            phase ^= 1;
            const bool rowk = ty == kt, colk = tx == kt;
            if (rowk) {
#pragma unroll
                for (int c = 0; c < RC; ++c) rb[tx + TX * c] = m[ka][c];
            }
            if (colk) {
#pragma unroll
                for (int a = 0; a < RA; ++a) cb[ty + TY * a] = m[a][ka];
            }
            __syncthreads();
            const double p = cb[k];
            ok = ok && (p > 0.0);
            const double rp = recip(p);
            double ci[RA], rj[RC];
#pragma unroll
            for (int a = 0; a < RA; ++a) ci[a] = cb[ty + TY * a];
#pragma unroll
            for (int c = 0; c < RC; ++c) rj[c] = rb[tx + TX * c] * rp;
            // pivot row: old entries become 0 and c_k = -1, so M'[k][j] = r_j;
            // pivot column: old entries become 0 and r_k = 1/p, so M'[i][k] = -M[i][k]/p
            ci[ka] = rowk ? -1.0 : ci[ka];
            rj[ka] = colk ? rp : rj[ka];
            apply<ka>(rowk, colk, ci, rj);
        }
    }

    // The whole inverse of the leading n x n block (steps 0 .. n-1).  LDS
    // scratch: kScratch doubles.
    __device__ __forceinline__ bool invert(int n, double *lds, int ty, int tx) { return run(0, n, lds, ty, tx); }
};

// Order of the tiles of an nr x nr grid for a big launch.  Workgroups are
// handed to the 8 XCDs round-robin (workgroup b to XCD b % 8), and each XCD
// has its own 4 MB L2.  Workgroup b = 8l + x is given position x*F + l of a
// list that walks strips of 8 tile rows column by column (F = number of
// workgroups per XCD), so the tiles an XCD holds at one time cover about 8
// tile rows x 8 tile columns and share their U and V operand slabs in L2.
// A bijection on [0, nr nc) whatever the hardware's actual assignment (nr x nc
// grids; xcd_strip_order is the square case).
__device__ __forceinline__ void xcd_strip_order_rect(int b, int nr, int nc, int &i, int &j) {
    const int total = nr * nc;
    const int full = total & ~7;
    const int idx = b < full ? (b & 7) * (full >> 3) + (b >> 3) : b;
    const int s = idx / (8 * nc);
    const int w = idx - s * 8 * nc;
    const int h = min(8, nr - 8 * s);
    j = w / h;
    i = 8 * s + (w - j * h);
}
__device__ __forceinline__ void xcd_strip_order(int b, int nr, int &i, int &j) {
    xcd_strip_order_rect(b, nr, nr, i, j);
}

// ---------------------------------------------------------------------------
// 128 x 128 FP64 tile contraction on MFMA (v_mfma_f64_16x16x4_f64).
// 256 threads = 4 waves; wave w owns the 64 x 64 quadrant (w >> 1, w & 1) as
// a 4 x 4 grid of 16 x 16 accumulators.  Operands are k-major in global
// memory: A_k[k * lda + i] (i in the tile's 128 rows), B_k[k * ldb + j].
// acc += sum_k A_k[k][i] * B_k[k][j]; the caller initialises acc (with zero
// or with the tile being updated, so that its load overlaps the first
// operand chunk instead of trailing the contraction).
//
// MFMA operand layout (lane l of the wave): A element (row l%16, k l/16),
// B element (k l/16, column l%16); accumulator element r in 0..3 of lane l is
// row l/16 + 4*r, column l%16 of the 16 x 16 block (measured on gfx950).
//
// Operand chunks of kKC k-rows are copied global -> LDS by the load unit
// (global_load_lds_dwordx4: each lane moves 16 bytes, one wave one 1 KiB row),
// double-buffered, so no VGPRs are spent on staging.
// ---------------------------------------------------------------------------
constexpr int kTile = 128;
constexpr int kKC = 16;                       // k-chunk staged per LDS buffer
constexpr int kLdsRow = kTile;                // one k-row of an operand
constexpr int kLdsChunk = kKC * kLdsRow;      // doubles per operand per buffer
constexpr int kTileLdsDoubles = 4 * kLdsChunk;  // A,B x double buffer (64 KiB)

struct TileAcc {
    d4 v[4][4];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) v[a][b] = d4{0.0, 0.0, 0.0, 0.0};
    }
};

typedef __attribute__((address_space(3))) void lds_void;
typedef const __attribute__((address_space(1))) void global_cvoid;

// Wave w copies k-rows 4w .. 4w+3 of both operands' chunk starting at k0.
__device__ __forceinline__ void tile_dma_chunk(const double *__restrict__ Ak, int lda,
                                               const double *__restrict__ Bk, int ldb, int k0,
                                               double *As, double *Bs) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < kKC / 4; ++q) {
        const int r = w * (kKC / 4) + q;
        __builtin_amdgcn_global_load_lds((global_cvoid *)(Ak + (size_t)(k0 + r) * lda + 2 * lane),
                                         (lds_void *)(As + r * kLdsRow), 16, 0, 0);
        __builtin_amdgcn_global_load_lds((global_cvoid *)(Bk + (size_t)(k0 + r) * ldb + 2 * lane),
                                         (lds_void *)(Bs + r * kLdsRow), 16, 0, 0);
    }
}

// s_waitcnt vmcnt(0) (expcnt and lgkmcnt left unconstrained): the chunk this
// wave copied has landed in LDS; the barrier after it publishes all waves' rows.
__device__ __forceinline__ void wait_vm_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }

__device__ __forceinline__ void tile_load_frags(const double *As, const double *Bs, int kk, int r0, int c0,
                                                int kr, double a[4], double b[4]) {
    const double *ar = As + (kk * 4 + kr) * kLdsRow;
    const double *br = Bs + (kk * 4 + kr) * kLdsRow;
#pragma unroll
    for (int q = 0; q < 4; ++q) { a[q] = ar[r0 + 16 * q]; b[q] = br[c0 + 16 * q]; }
}

// One k-chunk (kKC = 16, four MFMA k-steps).  Fragments are loaded one k-step
// ahead; the scheduling barriers stop the compiler from hoisting every load
// of the chunk (which would not fit next to the 128 accumulator VGPRs).
__device__ __forceinline__ void tile_mma_chunk(const double *As, const double *Bs, TileAcc &acc) {
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int r0 = (w >> 1) * 64 + (lane & 15);
    const int c0 = (w & 1) * 64 + (lane & 15);
    const int kr = lane >> 4;
    double a[2][4], b[2][4];
    tile_load_frags(As, Bs, 0, r0, c0, kr, a[0], b[0]);
#pragma unroll
    for (int kk = 0; kk < kKC / 4; ++kk) {
        const int cur = kk & 1;
        if (kk + 1 < kKC / 4) tile_load_frags(As, Bs, kk + 1, r0, c0, kr, a[cur ^ 1], b[cur ^ 1]);
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                acc.v[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[cur][p], b[cur][q], acc.v[p][q], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
    }
}

// acc += A_k^T B_k over k in [0, KDIM), KDIM a multiple of kKC (a template
// parameter: with a run-time trip count the register allocator spills).
// lds: kTileLdsDoubles doubles (a __shared__ array).  Ends with a barrier.
template <int KDIM>
__device__ __forceinline__ void tile_mma(const double *__restrict__ Ak, int lda,
                                         const double *__restrict__ Bk, int ldb,
                                         double *lds, TileAcc &acc) {
    static_assert(KDIM % kKC == 0, "inner dimension");
    // buffer q: A at lds + 2q*chunk, B right after it
    tile_dma_chunk(Ak, lda, Bk, ldb, 0, lds, lds + kLdsChunk);
    wait_vm_all();
    __syncthreads();
    constexpr int nchunks = KDIM / kKC;
#pragma unroll
    for (int ch = 0; ch < nchunks; ++ch) {
        double *cur = lds + (ch & 1) * (2 * kLdsChunk);
        double *nxt = lds + ((ch + 1) & 1) * (2 * kLdsChunk);
        if (ch + 1 < nchunks) tile_dma_chunk(Ak, lda, Bk, ldb, (ch + 1) * kKC, nxt, nxt + kLdsChunk);
        tile_mma_chunk(cur, cur + kLdsChunk, acc);
        wait_vm_all();
        __syncthreads();
    }
}

// Row and column (within the tile) of accumulator element (p, q, r) of this lane.
__device__ __forceinline__ int tile_row(int p, int r) {
    return ((threadIdx.x >> 6) >> 1) * 64 + ((threadIdx.x & 63) >> 4) + 16 * p + 4 * r;
}
__device__ __forceinline__ int tile_col(int q) {
    return ((threadIdx.x >> 6) & 1) * 64 + (threadIdx.x & 15) + 16 * q;
}

// acc = tile of C (ld), the starting value of an update C - U V.
__device__ __forceinline__ void tile_load_acc(TileAcc &acc, const double *C, int ld) {
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc.v[p][q][r] = C[(size_t)tile_row(p, r) * ld + tile_col(q)];
}

// Visits the accumulator entries: f(row_in_tile, col_in_tile, value).
template <typename F>
__device__ __forceinline__ void tile_for_each(TileAcc &acc, F &&f) {
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int rbase = (w >> 1) * 64 + (lane >> 4);
    const int cbase = (w & 1) * 64 + (lane & 15);
#pragma unroll
    for (int p = 0; p < 4; ++p) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) f(rbase + 16 * p + 4 * r, cbase + 16 * q, acc.v[p][q][r]);
        // keep at most one group of 16 entries' memory traffic in flight: the
        // accumulators already hold 128 VGPRs
        __builtin_amdgcn_sched_barrier(0);
    }
}

}  // namespace rd
