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
#include "rd_launch.h"

namespace rd {

// ---------------------------------------------------------------------------
// Ingest
// ---------------------------------------------------------------------------

__global__ void k_zero_i32(int32_t *p, int count) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

// Column sums of A (out-degrees) and validation, over a block of rows.
__global__ __launch_bounds__(256) void k_colsum(const uint8_t *__restrict__ A, int n, int rows_per_block,
                                                int32_t *outdeg, int32_t *bad) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const int i0 = blockIdx.y * rows_per_block;
    const int i1 = min(n, i0 + rows_per_block);
    int s = 0, b = 0;
    for (int i = i0; i < i1; ++i) {
        const int a = A[(size_t)i * n + j];
        s += a;
        b |= (a > 1) | ((i == j) & (a != 0));
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

// M = I - gamma*A on the n x n block, identity on the padding (np x np, ld).
__global__ __launch_bounds__(256) void k_build_m(const uint8_t *__restrict__ A, int n, int np, int ld,
                                                 double *__restrict__ M, const rdist_info *info) {
    const double gamma = info->gamma;
    const size_t pairs = (size_t)np * np / 2;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < pairs; e += (size_t)gridDim.x * 256) {
        const int i = (int)((2 * e) / np);
        const int j = (int)((2 * e) % np);     // even; np is even
        double v[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int jj = j + q;
            double x = (i == jj) ? 1.0 : 0.0;
            if (i < n && jj < n) x -= gamma * (double)A[(size_t)i * n + jj];
            v[q] = x;
        }
        *reinterpret_cast<double2 *>(M + (size_t)i * ld + j) = double2{v[0], v[1]};
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

// P = M_KK^{-1}: writes P into V's column block K and P^T (k-major) to Pt.
// Loads and the P store are coalesced straight from registers (lanes with
// consecutive tx hold consecutive columns); P^T goes through a 64 x 65 LDS
// quadrant.  About 37 KiB of LDS and under 192 VGPRs, so the kernel fits in
// the slot of one update workgroup and can run beside the update kernels.
__device__ __forceinline__ void panel_core(const double *__restrict__ M, int ld, int K, double *__restrict__ Pt,
                                           double *__restrict__ V, int ldv, rdist_info *info, double *piv,
                                           double (*tq)[65]) {
    const double *base = M + (size_t)K * kTile * ld + (size_t)K * kTile;
    RegGJ<16, 16, 8, 8> g;
    const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int c = 0; c < 8; ++c) g.m[a][c] = base[(size_t)(ty + 16 * a) * ld + tx + 16 * c];
    const bool ok = g.invert(kTile, piv, ty, tx);
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

__global__ __launch_bounds__(256) void k_panel(const double *__restrict__ M, int ld, int K,
                                               double *__restrict__ Pt, double *__restrict__ V, int ldv,
                                               rdist_info *info) {
    if (info->status != RDIST_OK) return;
    __shared__ double piv[4 * kTile];
    __shared__ double tq[64][65];
    panel_core(M, ld, K, Pt, V, ldv, info, piv, tq);
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

// Standalone readout over Y (ld) into D (n x n).
__global__ __launch_bounds__(256) void k_epilogue(const double *__restrict__ Y, int n, int ld,
                                                  int16_t *__restrict__ D, rdist_info *info) {
    if (info->status != RDIST_OK) return;
    const double lg = rd_inv_log(info->gamma);
    Counts cnt;
    const size_t total = (size_t)n * n;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
        const size_t i = e / n, j = e - i * n;
        D[e] = rd_encode(Y[i * ld + j], lg, cnt);
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

template <int TY, int TX, int RA, int RC>
__global__ __launch_bounds__(TY *TX) void k_small_one(SmallTask t) {
    constexpr int NP = TY * RA;
    __shared__ double lds_gj[4 * NP];
    __shared__ int lds_int[NP + 2];
    solve_small<TY, TX, RA, RC>(t, lds_gj, lds_int);
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
    __shared__ double piv[4 * kTile];
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
// of A summed per column in LDS, written to the graph's partial sums, with
// the chunk's validation flag.
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
    int32_t *out = g.colpart + (size_t)item * n;
    for (int j = threadIdx.x; j < n; j += 256) out[j] = colsum[j];
    if (threadIdx.x == 0) g.colpart[(size_t)g.nchunk * n + item] = bad;
}

// Gate, one workgroup per graph: out-degrees (the chunks' partial sums
// added up), Delta, the gain and the diagonal-dominance test, then info
// (status, delta, gamma, zeroed counters).
__global__ __launch_bounds__(256) void k_lv_gate(const LevelGraph *__restrict__ gs) {
    __shared__ int flags[2];
    const LevelGraph g = gs[blockIdx.x];
    if (threadIdx.x == 0) { flags[0] = 0; flags[1] = 0; }
    __syncthreads();
    const int n = g.n, nc = g.nchunk;
    int m = 0, bad = 0;
    for (int j = threadIdx.x; j < n; j += 256) {
        int sum = 0;
        for (int c = 0; c < nc; ++c) sum += g.colpart[(size_t)c * n + j];
        m = max(m, sum);
    }
    for (int c = threadIdx.x; c < nc; c += 256) bad |= g.colpart[(size_t)nc * n + c];
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
__global__ __launch_bounds__(256) void k_lv_panel(const LevelGraph *__restrict__ gs, const int *__restrict__ units,
                                                  int K) {
    int gi, item;
    if (!lv_unit(units, gi, item)) return;
    const LevelGraph g = gs[gi];
    if (g.info->status != RDIST_OK) return;
    __shared__ double piv[4 * kTile];
    __shared__ double tq[64][65];
    const int par = K & 1;
    panel_core(g.M, g.np, K, g.Pt[par], g.V[par], g.np, g.info, piv, tq);
}

// Row tiles of step K: items [0, nt-1) are V_J = P M_KJ for the tile
// columns J != K (the column operand Ut of step K is written by the build for
// K = 0 and by the edge update of step K-1 otherwise).
__global__ __launch_bounds__(256) void k_lv_rowcol(const LevelGraph *__restrict__ gs, const int *__restrict__ units,
                                                   int K) {
    int gi, item;
    if (!lv_unit(units, gi, item)) return;
    const LevelGraph g = gs[gi];
    if (g.info->status != RDIST_OK) return;
    __shared__ double lds[kTileLdsDoubles];
    const int np = g.np, par = K & 1;
    const int J = item < K ? item : item + 1;
    TileAcc acc;
    acc.zero();
    tile_mma<kTile>(g.Pt[par], kTile, g.M + (size_t)K * kTile * np + (size_t)J * kTile, np, lds, acc);
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

// Trailing update of step K over the tiles of `kind`:
//   kLvEdge  tile row and column L = K + 1 (what step K+1's panel and
//            row tiles read): items [0, nt) are (L, j), items [nt, 2nt-1)
//            are (i, L), i != L.  A column tile is not stored to M: it is
//            written straight into step L's column operand as -(M'_iL)^T;
//   kLvRest  the other tiles: (nt-1)^2 items skipping row and column L when
//            L < nt, all nt^2 tiles (item = I nt + J) on the graph's last step.
// Block row K is V itself (U_K = -I), copied without a product.  On a
// graph's last step the tile's final value is read out into D (stored to M
// only with keep); a refused graph gets the sentinel there instead.
__global__ __launch_bounds__(256, 2) void k_lv_update(const LevelGraph *__restrict__ gs,
                                                      const int *__restrict__ units, int K, int kind) {
    int gi, item;
    if (!lv_unit(units, gi, item)) return;
    const LevelGraph g = gs[gi];
    const int np = g.np, nt = g.nt, n = g.n, par = K & 1;
    const int L = K + 1;
    const bool last = L == nt;
    int I, J;
    if (kind == kLvEdge) {
        if (item < nt) { I = L; J = item; }
        else { const int ip = item - nt; I = ip < L ? ip : ip + 1; J = L; }
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
        if (J == K) acc.zero();
        else if (K == 0) tile_acc_from_adj(acc, g.A, n, I, J, g.info->gamma);
        else tile_load_acc(acc, base, np);
        tile_mma<kTile>(g.Ut[par] + (size_t)I * kTile, np, g.V[par] + (size_t)J * kTile, np, lds, acc);
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
// Successor bitmaps: bit b of word w in row i is set iff there is an edge
// i -> 64w + b, i.e. A[(64w + b) * n + i] == 1.  Row i is nw = ceil(n/64)
// 64-bit words; its size is known up front, so no host synchronisation is
// needed to allocate it.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_succ_bitmap(const uint8_t *__restrict__ A, int n, int nw,
                                                     unsigned long long *__restrict__ bits) {
    const int i = blockIdx.x * 256 + threadIdx.x;   // consecutive i read consecutive bytes of row j
    const int w = blockIdx.y;
    if (i >= n) return;
    unsigned long long word = 0;
    const int j0 = w * 64;
    const int j1 = min(n, j0 + 64);
    for (int j = j0; j < j1; ++j)
        if (A[(size_t)j * n + i] == 1) word |= 1ull << (j - j0);
    bits[(size_t)i * nw + w] = word;
}

// ---------------------------------------------------------------------------
// Next hop: one wavefront per query (Sec. 4.2, Eq. descent as ascent on Y).
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_next_hop(const double *__restrict__ Y, int ld, int n,
                                                  const unsigned long long *__restrict__ bits, int nw,
                                                  const int32_t *__restrict__ cur, const int32_t *__restrict__ goal,
                                                  int q, int max_hops, int32_t *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= q) return;
    int32_t *o = out + (size_t)w * (max_hops + 1);
    for (int h = lane; h <= max_hops; h += 64) o[h] = -1;
    int c = cur[w];
    const int g = goal[w];
    if (c < 0 || c >= n || g < 0 || g >= n) return;
    if (lane == 0) o[0] = c;
    const double *yg = Y + (size_t)g * ld;
    for (int h = 1; h <= max_hops; ++h) {
        if (c == g) break;
        double bv = -1.0;
        int bj = 0x7fffffff;
        const unsigned long long *row = bits + (size_t)c * nw;
        for (int ww = lane; ww < nw; ww += 64) {
            unsigned long long word = row[ww];
            while (word) {
                const int b = __ffsll((long long)word) - 1;
                word &= word - 1;
                const int j = ww * 64 + b;
                const double v = yg[j];
                if (v > bv || (v == bv && j < bj)) { bv = v; bj = j; }
            }
        }
        for (int s = 32; s > 0; s >>= 1) {
            const double ov = __shfl_xor(bv, s, 64);
            const int oj = __shfl_xor(bj, s, 64);
            if (ov > bv || (ov == bv && oj < bj)) { bv = ov; bj = oj; }
        }
        if (!(bv > 0.0)) {
            if (lane == 0) o[h] = -1;
            break;
        }
        c = bj;
        if (lane == 0) o[h] = c;
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

void launch_gate(const uint8_t *A, int n, double gamma_arg, int32_t *outdeg, int32_t *bad, rdist_info *info,
                 hipStream_t s) {
    hipLaunchKernelGGL(k_zero_i32, dim3((n + 1 + 255) / 256), dim3(256), 0, s, outdeg, n);
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(256), 0, s, bad, 1);
    const int rows = 256;
    hipLaunchKernelGGL(k_colsum, dim3((n + 255) / 256, (n + rows - 1) / rows), dim3(256), 0, s, A, n, rows,
                       outdeg, bad);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, s, outdeg, bad, n, gamma_arg, info);
}

void launch_ingest(const uint8_t *A, int n, int np, int ld, double gamma_arg, double *M, int32_t *outdeg,
                   int32_t *bad, rdist_info *info, hipStream_t s) {
    launch_gate(A, n, gamma_arg, outdeg, bad, info, s);
    const size_t pairs = (size_t)np * np / 2;
    const int blocks = (int)std::min<size_t>((pairs + 255) / 256, 8192);
    hipLaunchKernelGGL(k_build_m, dim3(blocks), dim3(256), 0, s, A, n, np, ld, M, info);
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
    const size_t total = (size_t)n * n;
    const int blocks = (int)std::max<size_t>(1, std::min<size_t>((total + 255) / 256, 8192));
    hipLaunchKernelGGL(k_epilogue, dim3(blocks), dim3(256), 0, s, Y, n, ld, D, info);
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

void launch_batched(const BatchTask *tasks, int count, int *counter, int grid, double *scratch, int scratch_stride,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, counter, 1);
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

void launch_succ_bitmap(const uint8_t *A, int n, unsigned long long *bits, hipStream_t s) {
    const int nw = (n + 63) / 64;
    hipLaunchKernelGGL(k_succ_bitmap, dim3((n + 255) / 256, nw), dim3(256), 0, s, A, n, nw, bits);
}

void launch_next_hop(const double *Y, int ld, int n, const unsigned long long *bits, const int32_t *cur,
                     const int32_t *goal, int q, int max_hops, int32_t *out, hipStream_t s) {
    if (q <= 0) return;
    const int nw = (n + 63) / 64;
    hipLaunchKernelGGL(k_next_hop, dim3((q + 3) / 4), dim3(256), 0, s, Y, ld, n, bits, nw, cur, goal, q, max_hops,
                       out);
}

}  // namespace rd
