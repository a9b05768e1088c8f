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
constexpr double kBeta = 1e-10;   // ambiguity band reported around k + eta
constexpr int16_t kUnreachable = RDIST_UNREACHABLE;
constexpr double kDMax = 32766.0;
constexpr double kDMin = -32767.0;
constexpr double kDblMin = 2.2250738585072014e-308;

// Per-thread counters of the readout; reduced per workgroup before the atomics.
struct Counts {
    unsigned long long unreachable = 0, subnormal = 0, saturated = 0, ambiguous = 0, negative = 0;
};

// D for one entry.  lg = log(gamma) < 0.
__device__ __forceinline__ int16_t rd_encode(double y, double lg, Counts &c) {
    if (y == 0.0) { ++c.unreachable; return kUnreachable; }
    if (!(y > 0.0)) { ++c.negative; return kUnreachable; }
    if (y < kDblMin) ++c.subnormal;
    double t = log(y) / lg - kEta;
    double d = ceil(t);
    if (fabs(t - rint(t)) < kBeta) ++c.ambiguous;
    if (d > kDMax) { d = kDMax; ++c.saturated; }
    if (d < kDMin) { d = kDMin; ++c.saturated; }
    return (int16_t)(int)d;
}

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

    // LDS scratch: 4 * NP doubles (pivot row and column, double-buffered).
    // Returns false (uniformly) if a pivot is not strictly positive.
    __device__ __forceinline__ bool run(int nsteps, double *lds, int ty, int tx) {
        bool ok = true;
        for (int k = 0; k < nsteps; ++k) {
            double *rb = lds + (k & 1) * (2 * NP);
            double *cb = rb + NP;
            const int ka = k / TY, kty = k - ka * TY;
            const int kc = k / TX, ktx = k - kc * TX;
            if (ty == kty) {
#pragma unroll
                for (int a = 0; a < RA; ++a)
                    if (a == ka) {
#pragma unroll
                        for (int c = 0; c < RC; ++c) rb[tx + TX * c] = m[a][c];
                    }
            }
            if (tx == ktx) {
#pragma unroll
                for (int c = 0; c < RC; ++c)
                    if (c == kc) {
#pragma unroll
                        for (int a = 0; a < RA; ++a) cb[ty + TY * a] = m[a][c];
                    }
            }
            __syncthreads();
            const double p = cb[k];
            ok = ok && (p > 0.0);
            const double rp = 1.0 / p;
            double ci[RA], rj[RC];
            bool rowk[RA], colk[RC];
#pragma unroll
            for (int a = 0; a < RA; ++a) {
                rowk[a] = (a == ka) && (ty == kty);
                double v = cb[ty + TY * a];
                ci[a] = rowk[a] ? -1.0 : v;
            }
#pragma unroll
            for (int c = 0; c < RC; ++c) {
                colk[c] = (c == kc) && (tx == ktx);
                double v = rb[tx + TX * c] * rp;
                rj[c] = colk[c] ? rp : v;
            }
#pragma unroll
            for (int a = 0; a < RA; ++a)
#pragma unroll
                for (int c = 0; c < RC; ++c) {
                    double o = (rowk[a] || colk[c]) ? 0.0 : m[a][c];
                    m[a][c] = fma(-ci[a], rj[c], o);
                }
        }
        return ok;
    }
};

// ---------------------------------------------------------------------------
// 128 x 128 FP64 tile contraction on MFMA (v_mfma_f64_16x16x4_f64).
// 256 threads = 4 waves; wave w owns the 64 x 64 quadrant (w >> 1, w & 1) as
// a 4 x 4 grid of 16 x 16 accumulators.  Operands are k-major in global
// memory: A_k[k * lda + i] (i in the tile's 128 rows), B_k[k * ldb + j].
// acc += sum_k A_k[k][i] * B_k[k][j].
//
// MFMA operand layout (lane l of the wave): A element (row l%16, k l/16),
// B element (k l/16, column l%16); accumulator element r in 0..3 of lane l is
// row l/16 + 4*r, column l%16 of the 16 x 16 block (measured on gfx950).
// ---------------------------------------------------------------------------
constexpr int kTile = 128;
constexpr int kKC = 16;                       // k-chunk staged per LDS buffer
constexpr int kLdsRow = kTile + 16;           // padded row: lanes 16..31 hit the other bank half
constexpr int kLdsChunk = kKC * kLdsRow;      // doubles per operand per buffer
constexpr int kTileLdsDoubles = 4 * kLdsChunk;  // A,B x double buffer (72 KiB)

struct TileAcc {
    d4 v[4][4];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) v[a][b] = d4{0.0, 0.0, 0.0, 0.0};
    }
};

__device__ __forceinline__ void tile_load_chunk(const double *__restrict__ Ak, int lda,
                                                const double *__restrict__ Bk, int ldb, int k0,
                                                double2 ra[4], double2 rb[4]) {
    const int t = threadIdx.x;
    const int r = t >> 4;            // 0..15: k row within the chunk
    const int c = (t & 15) * 8;      // 8 consecutive doubles
    const double2 *pa = reinterpret_cast<const double2 *>(Ak + (size_t)(k0 + r) * lda + c);
    const double2 *pb = reinterpret_cast<const double2 *>(Bk + (size_t)(k0 + r) * ldb + c);
#pragma unroll
    for (int q = 0; q < 4; ++q) { ra[q] = pa[q]; rb[q] = pb[q]; }
}

__device__ __forceinline__ void tile_store_chunk(double *As, double *Bs, const double2 ra[4],
                                                 const double2 rb[4]) {
    const int t = threadIdx.x;
    const int r = t >> 4;
    const int c = (t & 15) * 8;
    double2 *pa = reinterpret_cast<double2 *>(As + r * kLdsRow + c);
    double2 *pb = reinterpret_cast<double2 *>(Bs + r * kLdsRow + c);
#pragma unroll
    for (int q = 0; q < 4; ++q) { pa[q] = ra[q]; pb[q] = rb[q]; }
}

__device__ __forceinline__ void tile_mma_chunk(const double *As, const double *Bs, TileAcc &acc) {
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int r0 = (w >> 1) * 64 + (lane & 15);
    const int c0 = (w & 1) * 64 + (lane & 15);
    const int kr = lane >> 4;
#pragma unroll
    for (int kk = 0; kk < kKC / 4; ++kk) {
        const double *ar = As + (kk * 4 + kr) * kLdsRow;
        const double *br = Bs + (kk * 4 + kr) * kLdsRow;
        double a[4], b[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) { a[q] = ar[r0 + 16 * q]; b[q] = br[c0 + 16 * q]; }
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                acc.v[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p], b[q], acc.v[p][q], 0, 0, 0);
    }
}

// acc += A_k^T B_k over k in [0, kdim), kdim a multiple of kKC.
// lds: kTileLdsDoubles doubles.  Ends with a barrier (LDS reusable afterwards).
__device__ __forceinline__ void tile_mma(const double *__restrict__ Ak, int lda,
                                         const double *__restrict__ Bk, int ldb, int kdim,
                                         double *lds, TileAcc &acc) {
    double *As[2] = {lds, lds + 2 * kLdsChunk};
    double *Bs[2] = {lds + kLdsChunk, lds + 3 * kLdsChunk};
    double2 ra[4], rb[4];
    tile_load_chunk(Ak, lda, Bk, ldb, 0, ra, rb);
    tile_store_chunk(As[0], Bs[0], ra, rb);
    __syncthreads();
    const int nchunks = kdim / kKC;
    for (int ch = 0; ch < nchunks; ++ch) {
        const int cur = ch & 1;
        const bool more = ch + 1 < nchunks;
        if (more) tile_load_chunk(Ak, lda, Bk, ldb, (ch + 1) * kKC, ra, rb);
        tile_mma_chunk(As[cur], Bs[cur], acc);
        if (more) tile_store_chunk(As[cur ^ 1], Bs[cur ^ 1], ra, rb);
        __syncthreads();
    }
}

// Visits the accumulator entries: f(row_in_tile, col_in_tile, value).
template <typename F>
__device__ __forceinline__ void tile_for_each(TileAcc &acc, F &&f) {
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int rbase = (w >> 1) * 64 + (lane >> 4);
    const int cbase = (w & 1) * 64 + (lane & 15);
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) f(rbase + 16 * p + 4 * r, cbase + 16 * q, acc.v[p][q][r]);
}

}  // namespace rd
