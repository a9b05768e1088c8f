// rd_tile_kd.h -- the 128 x 128 FP64 tile contraction of rd_device.h with its
// inner dimension chosen at run time (the batched plans' last steps, whose
// products run over the pivot rows of a graph's last block only).
#pragma once

#include <hip/hip_runtime.h>

#include "rd_device.h"

namespace rd {

// acc += A_k^T B_k over k in [0, kd), kd in {16, 32, ..., 128}.
__device__ __forceinline__ void tile_mma_kd(int kd, const double *__restrict__ Ak, int lda,
                                            const double *__restrict__ Bk, int ldb, double *lds, TileAcc &acc) {
    switch (kd) {
        case 16: tile_mma<16>(Ak, lda, Bk, ldb, lds, acc); break;
        case 32: tile_mma<32>(Ak, lda, Bk, ldb, lds, acc); break;
        case 48: tile_mma<48>(Ak, lda, Bk, ldb, lds, acc); break;
        case 64: tile_mma<64>(Ak, lda, Bk, ldb, lds, acc); break;
        case 80: tile_mma<80>(Ak, lda, Bk, ldb, lds, acc); break;
        case 96: tile_mma<96>(Ak, lda, Bk, ldb, lds, acc); break;
        case 112: tile_mma<112>(Ak, lda, Bk, ldb, lds, acc); break;
        default: tile_mma<kTile>(Ak, lda, Bk, ldb, lds, acc); break;
    }
}

}  // namespace rd
