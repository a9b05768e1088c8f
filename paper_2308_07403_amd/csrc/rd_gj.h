// rd_gj.h -- Gauss-Jordan pieces shared by the single-graph kernels
// (rd_kernels.hip) and the batched ones (rd_level.hip): the register-resident
// panel inverse of a 128 x 128 block, the negated transpose of a column
// block, and the single-workgroup solve of a graph with n <= 128.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rd_device.h"
#include "rd_launch.h"

namespace rd {

// P = M_KK^{-1}: writes P into V's column block K and P^T (k-major) to Pt.
// Loads and the P store are coalesced straight from registers (lanes with
// consecutive tx hold consecutive columns); P^T goes through a 64 x 65 LDS
// quadrant.  About 41 KiB of LDS and under 200 VGPRs, so the kernel fits in
// the slot of one update workgroup and can run beside the update kernels.
// pivots < 128: only the leading pivots are eliminated; the block's trailing
// rows and columns must be those of an identity (the padding of the last
// block), which elimination would leave unchanged.
__device__ __forceinline__ void panel_core(const double *__restrict__ M, int ld, int K, double *__restrict__ Pt,
                                           double *__restrict__ V, int ldv, rdist_info *info, double *piv,
                                           double (*tq)[65], int pivots = kTile) {
    const double *base = M + (size_t)K * kTile * ld + (size_t)K * kTile;
    RegGJ<16, 16, 8, 8> g;
    const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int c = 0; c < 8; ++c) g.m[a][c] = base[(size_t)(ty + 16 * a) * ld + tx + 16 * c];
    const bool ok = g.invert(pivots, piv, ty, tx);
    double *vk = V + (size_t)K * kTile;
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int c = 0; c < 8; ++c) vk[(size_t)(ty + 16 * a) * ldv + tx + 16 * c] = g.m[a][c];
    // P^T one 64 x 64 quadrant at a time: rows a in [4qa, 4qa+4), columns c in [4qc, 4qc+4)
#pragma unroll
    for (int qa = 0; qa < 2; ++qa)
#pragma unroll
        for (int qc = 0; qc < 2; ++qc) {
            __syncthreads();
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c) tq[ty + 16 * a][tx + 16 * c] = g.m[4 * qa + a][4 * qc + c];
            __syncthreads();
            for (int e = threadIdx.x; e < 64 * 64; e += 256) {
                const int r = e >> 6, cc = e & 63;   // Pt[64qc + r][64qa + cc] = P[64qa + cc][64qc + r]
                Pt[(size_t)(64 * qc + r) * kTile + 64 * qa + cc] = tq[cc][r];
            }
        }
    if (!ok && threadIdx.x == 0) atomicCAS(&info->status, RDIST_OK, RDIST_E_NOT_DD);
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
