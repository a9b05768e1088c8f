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

// The kernels of the lookahead chain (the next block's diagonal update, its
// inverse and its row and column tiles) run beside the big update and are
// on the critical path: their waves take the highest issue priority on the
// SIMDs they share with the update's waves.
__device__ __forceinline__ void lookahead_priority() { __builtin_amdgcn_s_setprio(3); }

__global__ __launch_bounds__(256) void k_panel(const double *__restrict__ M, int ld, int K,
                                               double *__restrict__ Pt, double *__restrict__ V, int ldv,
                                               rdist_info *info) {
    if (info->status != RDIST_OK) return;
    lookahead_priority();
    __shared__ double piv[4 * kTile];
    __shared__ double tq[64][65];
    panel_core(M, ld, K, Pt, V, ldv, info, piv, tq);
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

// Tile sets of one update, with [L0, L0 + m) the next block's tile range and
// [L0, L0 + wt) the band of tile rows and columns the lookahead needs early
// (the next block's, or the next two blocks'):
//   ALL       every tile;
//   REST      tiles outside the band's rows and columns;
//   DIAG      the next block's m x m diagonal tiles (all its inverse needs);
//   EDGEREST  the band's tile rows and columns minus DIAG.
enum { kAll = 0, kDiag = 1, kRest = 2, kEdgeRest = 3 };

// Order of the tiles of an nr x nr grid for a big launch.  Workgroups are
// handed to the 8 XCDs round-robin (workgroup b to XCD b % 8), and each XCD
// has its own 4 MB L2.  Workgroup b = 8l + x is given position x*F + l of a
// list that walks strips of 8 tile rows column by column (F = number of
// workgroups per XCD), so the tiles an XCD holds at one time cover about 8
// tile rows x 8 tile columns and share their U and V operand slabs in L2.
// A bijection on [0, nr^2) whatever the hardware's actual assignment.
__device__ __forceinline__ void xcd_strip_order(int b, int nr, int &i, int &j) {
    const int total = nr * nr;
    const int full = total & ~7;
    const int idx = b < full ? (b & 7) * (full >> 3) + (b >> 3) : b;
    const int s = idx / (8 * nr);
    const int w = idx - s * 8 * nr;
    const int h = min(8, nr - 8 * s);
    j = w / h;
    i = 8 * s + (w - j * h);
}

template <int MODE>
__device__ __forceinline__ void update_tile_index(int b, int nt, int L0, int m, int wt, int &I, int &J) {
    if (MODE == kAll) {
        xcd_strip_order(b, nt, I, J);
    } else if (MODE == kDiag) {
        I = L0 + b / m;
        J = L0 + (b - (b / m) * m);
    } else if (MODE == kEdgeRest) {
        // tile rows [L0, L0 + wt) (minus the m x m diagonal block at L0),
        // then tile columns [L0, L0 + wt) outside those rows
        const int r1 = m * (nt - m), r2 = r1 + (wt - m) * nt;
        if (b < r1) {
            I = L0 + b / (nt - m);
            const int Jp = b - (b / (nt - m)) * (nt - m);
            J = Jp < L0 ? Jp : Jp + m;
        } else if (b < r2) {
            const int q = b - r1;
            I = L0 + m + q / nt;
            J = q - (q / nt) * nt;
        } else {
            const int q = b - r2;
            const int Ip = q / wt;
            J = L0 + (q - Ip * wt);
            I = Ip < L0 ? Ip : Ip + wt;
        }
    } else {
        int Ip, Jp;
        xcd_strip_order(b, nt - wt, Ip, Jp);
        I = Ip < L0 ? Ip : Ip + wt;
        J = Jp < L0 ? Jp : Jp + wt;
    }
}

// M_IJ <- M~_IJ - U_I V_J (inner dimension b = 128*MT) over the tiles of
// MODE, M~ = M with the current block's tile rows and columns [K0, K0 + m)
// zeroed.  The accumulators start from M~_IJ (loaded before the first operand
// chunk lands) and add (-U)^T V, Ut holding -U^T.  With FUSED the tile's
// final value is read out into D (and stored to M only if keep_y).
template <int MODE, bool FUSED, int MT>
__global__ __launch_bounds__(256, 2) void k_update(double *__restrict__ M, int ld, int nt, int K0, int L0, int wt,
                                                   const double *__restrict__ Ut, const double *__restrict__ V,
                                                   int ldv, int n, int16_t *__restrict__ D, int keep_y,
                                                   rdist_info *info) {
    constexpr int m = MT;
    if (info->status != RDIST_OK) return;
    if (MODE == kDiag || (MODE == kAll && !FUSED && MT == 1)) lookahead_priority();
    __shared__ double lds[kTileLdsDoubles];
    int I, J;
    update_tile_index<MODE>(blockIdx.x, nt, L0, m, wt, I, J);
    const bool zero_in = (I >= K0 && I < K0 + m) || (J >= K0 && J < K0 + m);
    double *base = M + (size_t)I * kTile * ld + (size_t)J * kTile;
    TileAcc acc;
    if (zero_in) acc.zero();
    else tile_load_acc(acc, base, ld);
    tile_mma<MT * kTile>(Ut + (size_t)I * kTile, ldv, V + (size_t)J * kTile, ldv, lds, acc);
    if (!FUSED) {
        tile_for_each(acc, [&](int r, int c, double v) { base[(size_t)r * ld + c] = v; });
    } else {
        const double lg = rd_inv_log(info->gamma);
        Counts cnt;
        tile_for_each(acc, [&](int r, int c, double y) {
            if (keep_y) base[(size_t)r * ld + c] = y;
            const int gi = I * kTile + r, gj = J * kTile + c;
            if (gi < n && gj < n) D[(size_t)gi * n + gj] = rd_encode(y, lg, cnt);
        });
        flush_counts(info, cnt);
    }
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
// of 1024 columns of one row, four entries per thread; with VEC (Y 16-byte
// aligned, ld even) the four are read as two 16-byte loads.
template <bool VEC>
__global__ __launch_bounds__(256) void k_epilogue(const double *__restrict__ Y, int n, int ld,
                                                  int16_t *__restrict__ D, rdist_info *info) {
    if (info->status != RDIST_OK) return;
    const double lg = rd_inv_log(info->gamma);
    Counts cnt;
    const int cpr = (n + 1023) / 1024;
    const long long units = (long long)n * cpr;
    for (long long u = blockIdx.x; u < units; u += gridDim.x) {
        const int i = (int)(u / cpr), ch = (int)(u - (long long)i * cpr);
        const int j0 = ch * 1024 + threadIdx.x * 4;
        const double *__restrict__ yr = Y + (size_t)i * ld;
        int16_t *__restrict__ dr = D + (size_t)i * n;
        if (VEC && j0 + 3 < n) {
            const double2 a = *reinterpret_cast<const double2 *>(yr + j0);
            const double2 b = *reinterpret_cast<const double2 *>(yr + j0 + 2);
            dr[j0] = rd_encode(a.x, lg, cnt);
            dr[j0 + 1] = rd_encode(a.y, lg, cnt);
            dr[j0 + 2] = rd_encode(b.x, lg, cnt);
            dr[j0 + 3] = rd_encode(b.y, lg, cnt);
        } else {
            for (int j = j0; j < min(n, j0 + 4); ++j) dr[j] = rd_encode(yr[j], lg, cnt);
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
    __shared__ double lds_gj[4 * NP];
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

int update_tiles(int mode, int nt, int m, int wt) {
    if (mode == kAll) return nt * nt;
    if (mode == kDiag) return m * m;
    if (mode == kEdgeRest) return m * (nt - m) + (wt - m) * nt + (nt - wt) * wt;
    return (nt - wt) * (nt - wt);
}

template <int MT>
static void launch_update_t(int mode, double *M, int ld, int nt, int K0, int L0, int wt, const double *Ut,
                            const double *V, int ldv, bool fused, int n, int16_t *D, int keep_y, rdist_info *info,
                            hipStream_t s) {
    const int tiles = update_tiles(mode, nt, MT, wt);
    if (tiles <= 0) return;
    const dim3 g(tiles), bl(256);
#define RD_UPD(MODE_, FUSED_) \
    hipLaunchKernelGGL((k_update<MODE_, FUSED_, MT>), g, bl, 0, s, M, ld, nt, K0, L0, wt, Ut, V, ldv, n, D, keep_y, info)
    if (fused) RD_UPD(kAll, true);
    else if (mode == kAll) RD_UPD(kAll, false);
    else if (mode == kDiag) RD_UPD(kDiag, false);
    else if (mode == kEdgeRest) RD_UPD(kEdgeRest, false);
    else RD_UPD(kRest, false);
#undef RD_UPD
}

void launch_update(int mode, double *M, int ld, int nt, int K0, int m, int L0, int wt, const double *Ut,
                   const double *V, int ldv, bool fused, int n, int16_t *D, int keep_y, rdist_info *info,
                   hipStream_t s) {
    if (m == 1)
        launch_update_t<1>(mode, M, ld, nt, K0, L0, wt, Ut, V, ldv, fused, n, D, keep_y, info, s);
    else
        launch_update_t<2>(mode, M, ld, nt, K0, L0, wt, Ut, V, ldv, fused, n, D, keep_y, info, s);
}

void launch_panel_finish(const double *S, int lds, int b, int K0, double *Pt, double *V, int ldv,
                         const rdist_info *info, hipStream_t s) {
    hipLaunchKernelGGL(k_panel_finish, dim3((b / 64) * (b / 64)), dim3(256), 0, s, S, lds, b, K0, Pt, V, ldv, info);
}

void launch_epilogue(const double *Y, int n, int ld, int16_t *D, rdist_info *info, hipStream_t s) {
    const long long units = (long long)n * ((n + 1023) / 1024);
    const int blocks = (int)std::max<long long>(1, std::min<long long>(units, 8192));
    if ((reinterpret_cast<uintptr_t>(Y) & 15) == 0 && (ld & 1) == 0)
        hipLaunchKernelGGL(k_epilogue<true>, dim3(blocks), dim3(256), 0, s, Y, n, ld, D, info);
    else
        hipLaunchKernelGGL(k_epilogue<false>, dim3(blocks), dim3(256), 0, s, Y, n, ld, D, info);
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
