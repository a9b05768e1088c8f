// rd_kernels.hip -- gfx950 kernels of the R-distance engine and their launchers.
//
// Pipeline for one graph (paper: Jing & Meister, arXiv 2308.07403):
//   ingest   A (uint8, j -> i convention of Sec. 2) -> out-degrees, Delta,
//            gamma, the gate gamma*Delta < 1 (Theorem 4's hypothesis), and
//            M = I - gamma*A in FP64 (Eq. Y-defined), identity-padded;
//   invert   Y = M^{-1} by blocked Gauss-Jordan without pivoting;
//   readout  D = ceil(log_gamma Y - eta), Y == 0 -> unreachable
//            (Eq. R-defined, rounded distance function of Sec. 4.1.1);
//   next hop greedy ascent on Y over successors (Sec. 4.2, Eq. descent).
//
// Blocked Gauss-Jordan with block size b = 128 on an np x np matrix
// (np = n rounded up to 128), for every block index K:
//   P = M_KK^{-1}                      k_panel   (register-resident GJ)
//   V_J = P M_KJ (J != K), V_K = P     k_rowcol  (MFMA)
//   U_I = M_IK (I != K),  U_K = -I     k_rowcol  (stored transposed, k-major)
//   M <- M~ - U V                      k_update  (MFMA; M~ = M with block row
//                                                 and column K set to zero)
// which is the block form of the in-place Gauss-Jordan step: it leaves
// M_KK = P, M_KJ = P M_KJ, M_IK = -M_IK P and M_IJ - M_IK P M_KJ.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rd_device.h"
#include "rd_gj.h"
#include "rd_launch.h"

namespace rd {

// ---------------------------------------------------------------------------
// Ingest
// ---------------------------------------------------------------------------

__global__ void k_zero_i32(int32_t *p, int count) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

// Column sums of A (out-degrees) and validation, over a block of rows:
// with 16 | n and A 16-byte aligned, thread t of workgroup (x, y) reads 16
// bytes (columns 16 (256 x + t) ..) of each row of block y.
__global__ __launch_bounds__(256) void k_colsum16(const uint8_t *__restrict__ A, int n, int rows_per_block,
                                                  int32_t *outdeg, int32_t *bad, int weighted) {
    const int j0 = (blockIdx.x * 256 + threadIdx.x) * 16;
    if (j0 >= n) return;
    const int i0 = blockIdx.y * rows_per_block;
    const int i1 = min(n, i0 + rows_per_block);
    int s[16] = {};
    int b = 0;
    for (int i = i0; i < i1; ++i) {
        const uint4 v = *reinterpret_cast<const uint4 *>(A + (size_t)i * n + j0);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int a = (int)((w[q >> 2] >> (8 * (q & 3))) & 0xFFu);
            s[q] += a != 0;
            b |= (!weighted & (a > 1)) | ((i == j0 + q) & (a != 0));
        }
    }
#pragma unroll
    for (int q = 0; q < 16; ++q)
        if (s[q]) atomicAdd(&outdeg[j0 + q], s[q]);
    if (b) atomicOr(bad, 1);
}

__global__ __launch_bounds__(256) void k_colsum(const uint8_t *__restrict__ A, int n, int rows_per_block,
                                                int32_t *outdeg, int32_t *bad, int weighted) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const int i0 = blockIdx.y * rows_per_block;
    const int i1 = min(n, i0 + rows_per_block);
    int s = 0, b = 0;
    for (int i = i0; i < i1; ++i) {
        const int a = A[(size_t)i * n + j];
        s += a != 0;
        b |= (!weighted & (a > 1)) | ((i == j) & (a != 0));
    }
    if (s) atomicAdd(&outdeg[j], s);
    if (b) atomicOr(bad, 1);
}

// Delta = max out-degree, gamma (explicit or c/Delta), gate; resets info.
__global__ __launch_bounds__(1024) void k_finalize(const int32_t *outdeg, const int32_t *bad, int n,
                                                   double gamma_arg, rdist_info *info) {
    __shared__ int smax;
    if (threadIdx.x == 0) smax = 0;
    __syncthreads();
    int m = 0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) m = max(m, outdeg[j]);
    atomicMax(&smax, m);
    __syncthreads();
    if (threadIdx.x == 0) {
        const int delta = smax;
        double gamma = gamma_arg > 0.0 ? gamma_arg : (delta > 0 ? (-gamma_arg) / (double)delta : -gamma_arg);
        int st = RDIST_OK;
        if (*bad) st = RDIST_E_ADJ;
        else if (!(gamma > 0.0) || !(gamma < 1.0)) st = RDIST_E_ARG;
        else if (!(gamma * (double)delta < 1.0)) st = RDIST_E_NOT_DD;
        info->status = st;
        info->delta = delta;
        info->gamma = gamma;
        info->n_unreachable = info->n_subnormal = info->n_saturated = 0;
        info->n_ambiguous = info->n_negative = info->n_uncertified = 0;
        info->fallback_fraction = 0.0;
    }
}

// M = I - gamma*A on the n x n block, identity on the padding (np x np, ld):
// a workgroup per row (grid-stride over rows), two entries per thread and
// 16-byte stores.
__global__ __launch_bounds__(256) void k_build_m(const uint8_t *__restrict__ A, int n, int np, int ld,
                                                 double *__restrict__ M, const rdist_info *info, int weighted) {
    const double gamma = info->gamma;
    // weighted (Sec. 3.2): entry -gamma^w for an edge of weight w, from a table
    __shared__ double gpow[256];
    if (weighted) {
        gpow[threadIdx.x] = threadIdx.x ? pow(gamma, (double)threadIdx.x) : 0.0;
        __syncthreads();
    }
    for (int i = blockIdx.x; i < np; i += gridDim.x) {
        const uint8_t *__restrict__ ar = A + (size_t)i * n;
        double *__restrict__ mr = M + (size_t)i * ld;
        for (int j = 2 * threadIdx.x; j < np; j += 512) {   // even; np is even
            double v[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int jj = j + q;
                double x = (i == jj) ? 1.0 : 0.0;
                if (i < n && jj < n) x -= weighted ? gpow[ar[jj]] : gamma * (double)ar[jj];
                v[q] = x;
            }
            *reinterpret_cast<double2 *>(mr + j) = double2{v[0], v[1]};
        }
    }
}

// On a refused graph (bad adjacency or gate) D is filled with the sentinel.
__global__ __launch_bounds__(256) void k_fill_sentinel(int16_t *D, size_t count, const rdist_info *info) {
    if (info->status == RDIST_OK) return;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (size_t)gridDim.x * 256)
        D[e] = kUnreachable;
}

// ---------------------------------------------------------------------------
// Blocked Gauss-Jordan
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256, 2) void k_panel(const double *__restrict__ M, int ld, int K,
                                                  double *__restrict__ Pt, double *__restrict__ V, int ldv,
                                                  rdist_info *info) {
    if (info->status != RDIST_OK) return;
    lookahead_priority();
    __shared__ PanelLds lds;
    panel_core(M, ld, K, Pt, V, ldv, info, lds);
}

// Step with block width b = 128*m whose block starts at tile K0 (tiles are
// 128 x 128; nt tiles per side).  Pt is P^T (b x b, row-major, ld b).
// Blocks [0, m*nt): V tile (r, J) = rows 128r.. of P times M_KJ (J outside
// the block; the block's own V is P, written by the panel).
// Blocks [m*nt, m*nt + nt): the negated transposed column block,
// Ut_I = -(M_IK)^T (b x 128) for I outside the block, and +I for the
// block's own rows (U_K = -I).  The update then accumulates C + Ut^T V.
// Ut and V are b x np, row-major.
template <int MT>
__global__ __launch_bounds__(256) void k_rowcol(const double *__restrict__ M, int ld, int nt, int K0,
                                                const double *__restrict__ Pt, double *__restrict__ Ut,
                                                double *__restrict__ V, int ldv, const rdist_info *info) {
    constexpr int m = MT;
    if (info->status != RDIST_OK) return;
    lookahead_priority();
    __shared__ double lds[kTileLdsDoubles];
    const int bdim = m * kTile;
    const int blk = blockIdx.x;
    if (blk < m * nt) {
        const int r = blk / nt, J = blk - (blk / nt) * nt;
        if (J >= K0 && J < K0 + m) return;
        TileAcc acc;
        acc.zero();
        tile_mma<MT * kTile>(Pt + (size_t)r * kTile, bdim, M + (size_t)K0 * kTile * ld + (size_t)J * kTile, ld, lds,
                             acc);
        double *out = V + (size_t)r * kTile * ldv + (size_t)J * kTile;
        tile_for_each(acc, [&](int rr, int c, double v) { out[(size_t)rr * ldv + c] = v; });
        return;
    }
    const int I = blk - m * nt;
    double *out = Ut + (size_t)I * kTile;          // Ut[k][I*128 + i]
    if (I >= K0 && I < K0 + m) {
        const int off = (I - K0) * kTile;
        for (int e = threadIdx.x; e < bdim * kTile; e += 256) {
            const int k = e >> 7, i = e & 127;
            out[(size_t)k * ldv + i] = (k == off + i) ? 1.0 : 0.0;
        }
        return;
    }
    transpose_neg(M + (size_t)I * kTile * ld + (size_t)K0 * kTile, ld, 2 * m, out, ldv, lds);
}

// From P (b x b, stored with leading dimension lds): Pt = P^T (ld b) and V's
// block columns [K0, K0 + m).
__global__ __launch_bounds__(256) void k_panel_finish(const double *__restrict__ S, int lds, int b, int K0,
                                                      double *__restrict__ Pt, double *__restrict__ V, int ldv,
                                                      const rdist_info *info) {
    if (info->status != RDIST_OK) return;
    lookahead_priority();
    __shared__ double t[64][65];
    const int nb64 = b / 64;
    const int bi = blockIdx.x / nb64, bj = blockIdx.x - (blockIdx.x / nb64) * nb64;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int r = e >> 6, c = e & 63;
        const double v = S[(size_t)(bi * 64 + r) * lds + bj * 64 + c];
        t[r][c] = v;
        V[(size_t)(bi * 64 + r) * ldv + (size_t)K0 * kTile + bj * 64 + c] = v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int r = e >> 6, c = e & 63;       // Pt[bj*64 + r][bi*64 + c] = P[bi*64 + c][bj*64 + r]
        Pt[(size_t)(bj * 64 + r) * b + bi * 64 + c] = t[c][r];
    }
}

// Standalone readout over Y (ld) into D (n x n).  A workgroup takes chunks
// of 2048 columns of one row; each thread reads out two groups of four
// entries 1024 columns apart, both groups' loads issued before either is read
// out.  With VEC (Y 16-byte aligned, ld even) a group is read as two 16-byte
// loads, with DV (n a multiple of 4, D 8-byte aligned) written as one 8-byte
// store; groups that cross the row's end go entry by entry.
template <bool VEC, bool DV>
__global__ __launch_bounds__(256) void k_epilogue(const double *__restrict__ Y, int n, int ld,
                                                  int16_t *__restrict__ D, rdist_info *info) {
    if (info->status != RDIST_OK) return;
    const double lg = rd_inv_log(info->gamma);
    Counts cnt;
    const int cpr = (n + 2047) / 2048;
    const long long units = (long long)n * cpr;
    for (long long u = blockIdx.x; u < units; u += gridDim.x) {
        const int i = (int)(u / cpr), ch = (int)(u - (long long)i * cpr);
        const double *__restrict__ yr = Y + (size_t)i * ld;
        int16_t *__restrict__ dr = D + (size_t)i * n;
        int jg[2];
        double y[2][4];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            jg[h] = ch * 2048 + h * 1024 + threadIdx.x * 4;
            if (VEC && jg[h] + 3 < n) {
                const double2 a = *reinterpret_cast<const double2 *>(yr + jg[h]);
                const double2 b = *reinterpret_cast<const double2 *>(yr + jg[h] + 2);
                y[h][0] = a.x; y[h][1] = a.y; y[h][2] = b.x; y[h][3] = b.y;
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int j0 = jg[h];
            if (VEC && j0 + 3 < n) {
                int16_t d[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) d[e] = rd_encode(y[h][e], lg, cnt);
                if (DV) {
                    *reinterpret_cast<short4 *>(dr + j0) = make_short4(d[0], d[1], d[2], d[3]);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) dr[j0 + e] = d[e];
                }
            } else {
                for (int j = j0; j < min(n, j0 + 4); ++j) dr[j] = rd_encode(yr[j], lg, cnt);
            }
        }
    }
    flush_counts(info, cnt);
}

// Sets info for a caller-provided gain (standalone readout).
__global__ void k_info_set(rdist_info *info, double gamma) {
    info->status = RDIST_OK;
    info->delta = 0;
    info->gamma = gamma;
    info->n_unreachable = info->n_subnormal = info->n_saturated = 0;
    info->n_ambiguous = info->n_negative = info->n_uncertified = 0;
    info->fallback_fraction = 0.0;
}

// ---------------------------------------------------------------------------
// Single-workgroup solve for n <= NP (128): ingest, register-resident
// Gauss-Jordan, readout, all in one kernel.  One workgroup per task; the
// persistent form pulls tasks from a counter in the order of `order`.
// ---------------------------------------------------------------------------

template <int TY, int TX, int RA, int RC>
__global__ __launch_bounds__(TY *TX) void k_small_one(SmallTask t) {
    constexpr int NP = TY * RA;
    __shared__ double lds_gj[8 * NP];   // RegGJ<TY, TX, RA, RC>::kScratch
    __shared__ int lds_int[NP + 2];
    solve_small<TY, TX, RA, RC>(t, lds_gj, lds_int);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

void launch_gate(const uint8_t *A, int n, double gamma_arg, int32_t *outdeg, int32_t *bad, rdist_info *info,
                 hipStream_t s, bool weighted) {
    hipLaunchKernelGGL(k_zero_i32, dim3((n + 1 + 255) / 256), dim3(256), 0, s, outdeg, n);
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(256), 0, s, bad, 1);
    if (n % 16 == 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0) {
        const int rows = 64;
        hipLaunchKernelGGL(k_colsum16, dim3((n / 16 + 255) / 256, (n + rows - 1) / rows), dim3(256), 0, s, A, n,
                           rows, outdeg, bad, (int)weighted);
    } else {
        const int rows = 256;
        hipLaunchKernelGGL(k_colsum, dim3((n + 255) / 256, (n + rows - 1) / rows), dim3(256), 0, s, A, n, rows,
                           outdeg, bad, (int)weighted);
    }
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, s, outdeg, bad, n, gamma_arg, info);
}

void launch_ingest(const uint8_t *A, int n, int np, int ld, double gamma_arg, double *M, int32_t *outdeg,
                   int32_t *bad, rdist_info *info, hipStream_t s, bool weighted) {
    launch_gate(A, n, gamma_arg, outdeg, bad, info, s, weighted);
    hipLaunchKernelGGL(k_build_m, dim3(std::min(np, 8192)), dim3(256), 0, s, A, n, np, ld, M, info, (int)weighted);
}

void launch_fill_sentinel(int16_t *D, int n, const rdist_info *info, hipStream_t s) {
    const size_t count = (size_t)n * n;
    const int blocks = (int)std::min<size_t>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_sentinel, dim3(blocks), dim3(256), 0, s, D, count, info);
}

void launch_panel(const double *M, int ld, int K, double *Pt, double *V, int ldv, rdist_info *info, hipStream_t s) {
    hipLaunchKernelGGL(k_panel, dim3(1), dim3(256), 0, s, M, ld, K, Pt, V, ldv, info);
}

void launch_rowcol(const double *M, int ld, int nt, int K0, int m, const double *Pt, double *Ut, double *V,
                   int ldv, const rdist_info *info, hipStream_t s) {
    if (m == 1)
        hipLaunchKernelGGL(k_rowcol<1>, dim3(2 * nt), dim3(256), 0, s, M, ld, nt, K0, Pt, Ut, V, ldv, info);
    else
        hipLaunchKernelGGL(k_rowcol<2>, dim3(3 * nt), dim3(256), 0, s, M, ld, nt, K0, Pt, Ut, V, ldv, info);
}

void launch_panel_finish(const double *S, int lds, int b, int K0, double *Pt, double *V, int ldv,
                         const rdist_info *info, hipStream_t s) {
    hipLaunchKernelGGL(k_panel_finish, dim3((b / 64) * (b / 64)), dim3(256), 0, s, S, lds, b, K0, Pt, V, ldv, info);
}

void launch_epilogue(const double *Y, int n, int ld, int16_t *D, rdist_info *info, hipStream_t s) {
    const long long units = (long long)n * ((n + 2047) / 2048);
    const int blocks = (int)std::max<long long>(1, std::min<long long>(units, 8192));
    const bool vec = (reinterpret_cast<uintptr_t>(Y) & 15) == 0 && (ld & 1) == 0;
    const bool dv = (n & 3) == 0 && (reinterpret_cast<uintptr_t>(D) & 7) == 0;
    if (vec && dv)
        hipLaunchKernelGGL((k_epilogue<true, true>), dim3(blocks), dim3(256), 0, s, Y, n, ld, D, info);
    else if (vec)
        hipLaunchKernelGGL((k_epilogue<true, false>), dim3(blocks), dim3(256), 0, s, Y, n, ld, D, info);
    else
        hipLaunchKernelGGL((k_epilogue<false, false>), dim3(blocks), dim3(256), 0, s, Y, n, ld, D, info);
}

void launch_info_set(rdist_info *info, double gamma, hipStream_t s) {
    hipLaunchKernelGGL(k_info_set, dim3(1), dim3(1), 0, s, info, gamma);
}

void launch_small_one(const SmallTask &t, hipStream_t s) {
    if (t.n <= 32)
        hipLaunchKernelGGL((k_small_one<8, 8, 4, 4>), dim3(1), dim3(64), 0, s, t);
    else if (t.n <= 64)
        hipLaunchKernelGGL((k_small_one<16, 16, 4, 4>), dim3(1), dim3(256), 0, s, t);
    else
        hipLaunchKernelGGL((k_small_one<16, 16, 8, 8>), dim3(1), dim3(256), 0, s, t);
}

}  // namespace rd
