// rd_gj.h -- Gauss-Jordan pieces shared by the single-graph kernels
// (rd_kernels.hip) and the batched ones (rd_level.hip): the blocked panel
// inverse of a 128 x 128 block on the matrix cores, the negated transpose of
// a column block, and the single-workgroup solve of a graph with n <= 128.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rd_device.h"
#include "rd_launch.h"

namespace rd {

// ---------------------------------------------------------------------------
// Panel inverse P = M_KK^{-1} of a 128 x 128 diagonal block, blocked on the
// FP64 matrix cores.
//
// Wave w holds rows 32w .. 32w+31 of the block as 2 x 8 accumulator tiles of
// 16 x 16 (element r of lane l of tile (p, q): row 32w + 16p + l/16 + 4r,
// column 16q + l%16, the MFMA accumulator layout).  Gauss-Jordan runs in
// sub-steps of 32 pivots, ks = 0, 1, ..., with R = rows and columns
// 32ks .. 32ks+31:
//   1. wave ks inverts its 32 x 32 diagonal block in registers, pivot by
//      pivot, exchanging the pivot row and column between lanes (readlane,
//      ds_bpermute, row broadcasts), and publishes its strip with P_ks in
//      place of the diagonal block, and P_ks transposed;
//   2. the other waves form V = P_ks M_R,: (one 32-column slice each; the
//      slice R of V is P_ks itself);
//   3. every other wave updates its strip, M_w,: <- M~_w,: - M_w,R V, where M~
//      has column block R zeroed (so that block becomes -M_w,R P_ks), and wave
//      ks takes V as its rows.
// This is the blocked Gauss-Jordan step of the whole solve with width 32
// inside the panel.  Its pivots are those of the unblocked elimination
// (Schur complement diagonals), each checked positive.  The serial pivot
// loop (one wave, VALU-issue bound) touches 32 x 32 entries instead of
// 128 x 128; of the 2 * 128^3 flops, 94% run on v_mfma_f64_16x16x4f64 (per
// sub-step 2 * 32^3 in the pivot loop, 2 * 3 * 32^3 in the row block and
// 2 * 3 * 32^2 * 128 in the update).
// ---------------------------------------------------------------------------
constexpr int kPanS = 136;   // row stride (doubles) of the published strip
constexpr int kPanU = 33;    // row stride of the 32 x 32 blocks in LDS

struct PanelLds {
    double S[32 * kPanS];    // the pivot strip, then V
    double PT[32 * kPanU];   // P_ks transposed
    double U[4][32 * kPanU]; // -M_w,R of each wave (its update's A operand)
};
static_assert(sizeof(PanelLds) >= 64 * 129 * sizeof(double), "P^T staging reuses the panel's LDS");

struct PanelAcc {
    d4 v[2][8];
};

// Lane N of each row of 16 lanes, to every lane of the row (DPP row_newbcast).
template <int N>
__device__ __forceinline__ double row_bcast(double x) {
    const long long b = __builtin_bit_cast(long long, x);
    const long long r = __builtin_amdgcn_update_dpp((long long)0, b, 0x150 + N, 0xF, 0xF, false);
    return __builtin_bit_cast(double, r);
}

__device__ __forceinline__ double readlane_d(double x, int l) {
    const long long b = __builtin_bit_cast(long long, x);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// x of lane addr / 4.
__device__ __forceinline__ double bpermute_d(int addr, double x) {
    const long long b = __builtin_bit_cast(long long, x);
    const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)b);
    const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// The 32 x 32 diagonal block of a sub-step: b[p][q][r] = block row
// 16p + g + 4r, column 16q + c (g = lane / 16, c = lane % 16).
typedef double PanelBlk[2][2][4];

// Steps T and T + 1 (T even) of Gauss-Jordan on the block.  One step with
// pivot p = b[T][T] is a single fused update of every entry,
// b[i][j] -= c_i r_j with
//     c_i = b[i][T] (i != T),  c_T = p - 1,
//     r_j = b[T][j] / p (j != T),  r_T = 1 + 1/p,
// which gives b[T][j] / p in the pivot row, -b[i][T] / p in the pivot column
// and 1 / p at the pivot, with no zeroing or per-entry selects (the pivots of
// the gated M-matrix lie in (0, 1], so c_T adds no cancellation).  Row and
// column T + 1 after step T are formed by every lane with the FMAs their
// owners use, so both steps come from one exchange and the result is
// bitwise that of two single steps.
template <int T>
__device__ __forceinline__ void panel_blk_step2(PanelBlk &b, int g, int c, bool &ok) {
    constexpr int T1 = T + 1;
    constexpr int pt = T >> 4, rt = (T & 15) >> 2, qt = T >> 4;
    constexpr int g0 = T & 3, c0 = T & 15, g1 = T1 & 3, c1 = T1 & 15;
    const double p0 = readlane_d(b[pt][qt][rt], g0 * 16 + c0);
    const double b01 = readlane_d(b[pt][qt][rt], g0 * 16 + c1);
    const double b10 = readlane_d(b[pt][qt][rt], g1 * 16 + c0);
    const double b11 = readlane_d(b[pt][qt][rt], g1 * 16 + c1);
    double r0[2], r1[2];   // rows T and T+1 at this lane's columns
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        r0[q] = bpermute_d((g0 * 16 + c) * 4, b[pt][q][rt]);
        r1[q] = bpermute_d((g1 * 16 + c) * 4, b[pt][q][rt]);
    }
    double ci0[2][4], ci1[2][4];   // columns T and T+1 at this lane's rows
#pragma unroll
    for (int pp = 0; pp < 2; ++pp)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            ci0[pp][r] = row_bcast<c0>(b[pp][qt][r]);
            ci1[pp][r] = row_bcast<c1>(b[pp][qt][r]);
        }
    const double rp0 = recip(p0);
    const double s01 = b01 * rp0;             // step T's row factor at column T+1
    const double p1 = fma(-b10, s01, b11);    // pivot T+1 after step T
    ok = ok && (p0 > 0.0) && (p1 > 0.0);
    const double rp1 = recip(p1);
    double rj0[2], rj1[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) rj0[q] = r0[q] * rp0;
    rj0[qt] = c == c0 ? 1.0 + rp0 : rj0[qt];
    ci0[pt][rt] = g == g0 ? p0 - 1.0 : ci0[pt][rt];
#pragma unroll
    for (int q = 0; q < 2; ++q) rj1[q] = fma(-b10, rj0[q], r1[q]) * rp1;
#pragma unroll
    for (int pp = 0; pp < 2; ++pp)
#pragma unroll
        for (int r = 0; r < 4; ++r) ci1[pp][r] = fma(-ci0[pp][r], s01, ci1[pp][r]);
    rj1[qt] = c == c1 ? 1.0 + rp1 : rj1[qt];
    ci1[pt][rt] = g == g1 ? p1 - 1.0 : ci1[pt][rt];
#pragma unroll
    for (int pp = 0; pp < 2; ++pp)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                b[pp][q][r] = fma(-ci0[pp][r], rj0[q], b[pp][q][r]);
                b[pp][q][r] = fma(-ci1[pp][r], rj1[q], b[pp][q][r]);
            }
}

// Steps [0, rem) of the block, rem rounded up to even: a step on a pivot of
// the identity padding changes nothing.
template <int T>
__device__ __forceinline__ void panel_blk_steps(PanelBlk &b, int g, int c, bool &ok, int rem) {
    if constexpr (T < 32) {
        if (T < rem) {
            panel_blk_step2<T>(b, g, c, ok);
            panel_blk_steps<T + 2>(b, g, c, ok, rem);
        }
    }
}

// b = column block ks (tiles (p, 2ks + q)) of the strip, and back.  Selects on
// the uniform ks (not an indexed copy) keep the strip in registers, so one
// copy of the pivot loop serves every sub-step.
__device__ __forceinline__ void panel_blk_get(const PanelAcc &a, PanelBlk &b, int ks) {
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double x01 = ks == 0 ? a.v[p][q][r] : a.v[p][2 + q][r];
                const double x23 = ks == 2 ? a.v[p][4 + q][r] : a.v[p][6 + q][r];
                b[p][q][r] = ks < 2 ? x01 : x23;
            }
}
__device__ __forceinline__ void panel_blk_set(PanelAcc &a, const PanelBlk &b, int ks) {
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) a.v[p][2 * k + q][r] = ks == k ? b[p][q][r] : a.v[p][2 * k + q][r];
}

// In place: a holds the block, on return its inverse.  Only the leading
// `pivots` pivots are eliminated (sub-steps wholly in the padding are
// skipped); the trailing rows and columns must be those of an identity (the
// padding of a graph's last block), which elimination leaves unchanged, so
// the result is bitwise that of all 128 pivots.  Returns false if a pivot is
// not positive (uniform per wave).  Ends with a barrier.
__device__ __forceinline__ bool panel_blk_invert(PanelAcc &a, PanelLds &L, int pivots) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, c = lane & 15;
    bool ok = true;
    const int nsub = (pivots + 31) >> 5;
#pragma unroll 1
    for (int ks = 0; ks < nsub; ++ks) {
        PanelBlk b;
        panel_blk_get(a, b, ks);
        if (w == ks) {
            panel_blk_steps<0>(b, g, c, ok, pivots - 32 * ks);
            panel_blk_set(a, b, ks);
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int q = 0; q < 8; ++q)
#pragma unroll
                    for (int r = 0; r < 4; ++r) L.S[(16 * p + g + 4 * r) * kPanS + 16 * q + c] = a.v[p][q][r];
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int r = 0; r < 4; ++r) L.PT[(16 * q + c) * kPanU + 16 * p + g + 4 * r] = b[p][q][r];
        }
        __syncthreads();
        if (w != ks) {
            // V slice 32w .. 32w+31 = P_ks times the strip's slice, in place
            d4 o[2][2];
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int q = 0; q < 2; ++q) o[p][q] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                double A[2], B[2];
#pragma unroll
                for (int p = 0; p < 2; ++p) A[p] = L.PT[(4 * s + g) * kPanU + 16 * p + c];
#pragma unroll
                for (int q = 0; q < 2; ++q) B[q] = L.S[(4 * s + g) * kPanS + 32 * w + 16 * q + c];
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int q = 0; q < 2; ++q)
                        o[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[p], B[q], o[p][q], 0, 0, 0);
            }
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int r = 0; r < 4; ++r) L.S[(16 * p + g + 4 * r) * kPanS + 32 * w + 16 * q + c] = o[p][q][r];
        }
        __syncthreads();
        if (w != ks) {
            double *U = L.U[w];
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        U[(16 * p + g + 4 * r) * kPanU + 16 * q + c] = -b[p][q][r];
                        b[p][q][r] = 0.0;
                    }
            panel_blk_set(a, b, ks);
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                double A[2], B[8];
#pragma unroll
                for (int p = 0; p < 2; ++p) A[p] = U[(16 * p + c) * kPanU + 4 * s + g];
#pragma unroll
                for (int q = 0; q < 8; ++q) B[q] = L.S[(4 * s + g) * kPanS + 16 * q + c];
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        a.v[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[p], B[q], a.v[p][q], 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int q = 0; q < 8; ++q)
#pragma unroll
                    for (int r = 0; r < 4; ++r) a.v[p][q][r] = L.S[(16 * p + g + 4 * r) * kPanS + 16 * q + c];
        }
        __syncthreads();
    }
    return ok;
}

// P = M_KK^{-1}: writes P into V's column block K and P^T (k-major, ld 128)
// to Pt.  The block load and the P store are coalesced straight from the
// accumulators (16 lanes per 128-byte row piece); P^T is staged through the
// panel's LDS 64 rows at a time.  77 KiB of LDS and at most 256 VGPRs (the
// kernels declare two waves per SIMD), so two panels share a compute unit,
// or a panel shares one with an update workgroup.  pivots < 128: see
// panel_blk_invert.
__device__ __forceinline__ void panel_core(const double *__restrict__ M, int ld, int K, double *__restrict__ Pt,
                                           double *__restrict__ V, int ldv, rdist_info *info, PanelLds &L,
                                           int pivots = kTile) {
    const double *base = M + (size_t)K * kTile * ld + (size_t)K * kTile;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, c = lane & 15;
    PanelAcc a;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 8; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) a.v[p][q][r] = base[(size_t)(32 * w + 16 * p + g + 4 * r) * ld + 16 * q + c];
    const bool ok = panel_blk_invert(a, L, pivots);
    double *vk = V + (size_t)K * kTile;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 8; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) vk[(size_t)(32 * w + 16 * p + g + 4 * r) * ldv + 16 * q + c] = a.v[p][q][r];
    double *t = reinterpret_cast<double *>(&L);   // 64 x 129 staging
    for (int h = 0; h < 2; ++h) {
        if ((w >> 1) == h) {
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int q = 0; q < 8; ++q)
#pragma unroll
                    for (int r = 0; r < 4; ++r) t[(32 * (w & 1) + 16 * p + g + 4 * r) * 129 + 16 * q + c] = a.v[p][q][r];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < 64 * kTile; e += 256) {
            const int col = e >> 6, i = e & 63;   // Pt[col][64h + i] = P[64h + i][col]
            Pt[(size_t)col * kTile + 64 * h + i] = t[i * 129 + col];
        }
        __syncthreads();
    }
    if (!ok && lane == 0) atomicCAS(&info->status, RDIST_OK, RDIST_E_NOT_DD);
}

// out[k][i] = -src[i][k] for the 128 x (64 * kb64) block src (leading dim ld),
// 64 x 64 at a time through LDS (lds: at least 64 * 65 doubles).  Ends with a
// barrier.
__device__ __forceinline__ void transpose_neg(const double *__restrict__ src, int ld, int kb64,
                                              double *__restrict__ out, int ldv, double *lds) {
    double (*t)[65] = reinterpret_cast<double (*)[65]>(lds);
    for (int bi = 0; bi < 2; ++bi)
        for (int bk = 0; bk < kb64; ++bk) {
            for (int e = threadIdx.x; e < 64 * 64; e += 256) {
                const int r = e >> 6, c = e & 63;     // r: row i, c: column k
                t[r][c] = src[(size_t)(bi * 64 + r) * ld + bk * 64 + c];
            }
            __syncthreads();
            for (int e = threadIdx.x; e < 64 * 64; e += 256) {
                const int k = e >> 6, i = e & 63;
                out[(size_t)(bk * 64 + k) * ldv + bi * 64 + i] = -t[i][k];
            }
            __syncthreads();
        }
}

// Single-workgroup solve for n <= NP (128): ingest, register-resident
// Gauss-Jordan, readout, all in one workgroup (used by the one-graph kernel
// and by the persistent batched kernel).
template <int TY, int TX, int RA, int RC>
__device__ __forceinline__ void solve_small(const SmallTask &t, double *lds_gj, int *lds_int) {
    using G = RegGJ<TY, TX, RA, RC>;
    constexpr int NP = G::NP;
    const int n = t.n;
    const int ty = threadIdx.x / TX, tx = threadIdx.x % TX;
    int *colsum = lds_int;          // NP
    int *flags = lds_int + NP;      // [0] bad, [1] delta
    for (int j = threadIdx.x; j < NP; j += G::NT) colsum[j] = 0;
    if (threadIdx.x == 0) { flags[0] = 0; flags[1] = 0; }
    __syncthreads();
    G g;
    uint8_t a8[RA][RC];
    int bad = 0;
#pragma unroll
    for (int a = 0; a < RA; ++a)
#pragma unroll
        for (int c = 0; c < RC; ++c) {
            const int i = ty + TY * a, j = tx + TX * c;
            uint8_t v = 0;
            if (i < n && j < n) v = t.A[(size_t)i * n + j];
            a8[a][c] = v;
            bad |= (v > 1) | ((i == j) & (v != 0));
        }
#pragma unroll
    for (int c = 0; c < RC; ++c) {
        int s = 0;
#pragma unroll
        for (int a = 0; a < RA; ++a) s += a8[a][c];
        if (s) atomicAdd(&colsum[tx + TX * c], s);
    }
    if (bad) atomicOr(&flags[0], 1);
    __syncthreads();
    for (int j = threadIdx.x; j < NP; j += G::NT) atomicMax(&flags[1], colsum[j]);
    __syncthreads();
    const int delta = flags[1];
    const double gamma = t.gamma_arg > 0.0 ? t.gamma_arg
                                           : (delta > 0 ? (-t.gamma_arg) / (double)delta : -t.gamma_arg);
    int st = RDIST_OK;
    if (flags[0]) st = RDIST_E_ADJ;
    else if (!(gamma > 0.0) || !(gamma < 1.0)) st = RDIST_E_ARG;
    else if (!(gamma * (double)delta < 1.0)) st = RDIST_E_NOT_DD;
    Counts cnt;
    if (st == RDIST_OK) {
#pragma unroll
        for (int a = 0; a < RA; ++a)
#pragma unroll
            for (int c = 0; c < RC; ++c) {
                const int i = ty + TY * a, j = tx + TX * c;
                g.m[a][c] = (i == j ? 1.0 : 0.0) - gamma * (double)a8[a][c];
            }
        const bool ok = g.invert(n, lds_gj, ty, tx);
        if (!ok) st = RDIST_E_NOT_DD;
    }
    if (st == RDIST_OK) {
        const double lg = rd_inv_log(gamma);
#pragma unroll
        for (int a = 0; a < RA; ++a)
#pragma unroll
            for (int c = 0; c < RC; ++c) {
                const int i = ty + TY * a, j = tx + TX * c;
                if (i < n && j < n) {
                    const double y = g.m[a][c];
                    t.D[(size_t)i * n + j] = rd_encode(y, lg, cnt);
                    if (t.Y) t.Y[(size_t)i * t.ldy + j] = y;
                }
            }
    } else {
        for (int e = threadIdx.x; e < n * n; e += G::NT) t.D[e] = kUnreachable;
    }
    // reduce the counters across the workgroup through LDS
    __syncthreads();
    unsigned long long *red = reinterpret_cast<unsigned long long *>(lds_gj);
    if (threadIdx.x < 5) red[threadIdx.x] = 0;
    __syncthreads();
    unsigned long long v[5] = {wave_sum_u64(cnt.unreachable), wave_sum_u64(cnt.subnormal),
                               wave_sum_u64(cnt.saturated), wave_sum_u64(cnt.ambiguous),
                               wave_sum_u64(cnt.negative)};
    if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < 5; ++q)
            if (v[q]) atomicAdd(&red[q], v[q]);
    __syncthreads();
    if (threadIdx.x == 0) {
        rdist_info *info = t.info;
        info->status = st;
        info->delta = delta;
        info->gamma = gamma;
        info->n_unreachable = (int64_t)red[0];
        info->n_subnormal = (int64_t)red[1];
        info->n_saturated = (int64_t)red[2];
        info->n_ambiguous = (int64_t)red[3];
        info->n_negative = (int64_t)red[4];
        info->n_uncertified = 0;
        info->fallback_fraction = 0.0;
    }
    __syncthreads();
}

}  // namespace rd
