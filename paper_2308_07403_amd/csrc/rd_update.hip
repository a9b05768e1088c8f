// rd_update.hip -- the trailing update of blocked Gauss-Jordan (the FP64
// matrix-core kernel that carries almost all of the flops) and its launcher:
// M_IJ <- M~_IJ - U_I V_J over a tile set of one step (Sec. 3, the inverse
// of Eq. Y-defined by Gauss-Jordan elimination), optionally with the readout
// fused into the last step.  Kept in a file of its own so that its measured
// counters stay tied to exactly this code.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rd_device.h"
#include "rd_launch.h"

namespace rd {

// Tile sets of one update, with [L0, L0 + m) the next block's tile range and
// [L0, L0 + wt) the band of tile rows and columns the lookahead needs early
// (the next block's, or the next two blocks'):
//   ALL       every tile;
//   REST      tiles outside the band's rows and columns;
//   DIAG      the next block's m x m diagonal tiles (all its inverse needs);
//   EDGEREST  the band's tile rows and columns minus DIAG.
enum { kAll = 0, kDiag = 1, kRest = 2, kEdgeRest = 3 };

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

}  // namespace rd
