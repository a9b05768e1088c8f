// rd_chain.hip -- the lookahead chain's small products for the blocked plan
// with 128-wide blocks (n up to 6400): between two panels the chain carries
// one diagonal-tile update (DIAG) and the row tiles V_J = P M_KJ, each a
// 128 x 128 product with inner dimension 128 (the inversion behind
// Eq. Y-defined; its cost is the one Sec. 5.2 names as dominant).  On one
// workgroup each such product takes about 21 us, waiting on its operand
// chunks; here each is four workgroups of 64 x 64, every wave one 32 x 32
// block whose operands stream straight from L2 with the k loop unrolled.
// Every output sums k = 0, 4, .. 124 on v_mfma_f64_16x16x4f64 with the lane
// mapping and starting accumulator of the tile kernels they replace, so the
// results are bit for bit theirs.
#include <hip/hip_runtime.h>

#include "rd_device.h"
#include "rd_launch.h"

namespace rd {

namespace {

// acc (this wave's 32 x 32 block of the 64 x 64 piece at (i0, j0): rows
// i0 + 32 (w >> 1) + 16 p + .., columns j0 + 32 (w & 1) + 16 q + ..) +=
// A_k^T B_k over k in [0, 128): A_k[k][i] at A[k * lda + i], B_k[k][j] at
// B[k * ldb + j].
__device__ __forceinline__ void piece_mma(d4 (&acc)[2][2], const double *__restrict__ A, int lda,
                                          const double *__restrict__ B, int ldb, int i0, int j0) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int ri = i0 + 32 * (w >> 1), cj = j0 + 32 * (w & 1);
#pragma unroll
    for (int kk = 0; kk < kTile; kk += 4) {
        double a[2], b[2];
#pragma unroll
        for (int p = 0; p < 2; ++p) a[p] = A[(size_t)(kk + lk) * lda + ri + 16 * p + li];
#pragma unroll
        for (int q = 0; q < 2; ++q) b[q] = B[(size_t)(kk + lk) * ldb + cj + 16 * q + li];
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < 2; ++q) acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p], b[q], acc[p][q], 0, 0, 0);
    }
}

// Visits this wave's elements of its block: f(row, column, value) with row
// and column inside the 64 x 64 piece.
template <typename F>
__device__ __forceinline__ void piece_for_each(const d4 (&acc)[2][2], F f) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) f(32 * (w >> 1) + 16 * p + lk + 4 * r, 32 * (w & 1) + 16 * q + li, acc[p][q][r]);
}

// DIAG of step K for one block (L0 = K + 1, outside the step's block):
// M_LL <- M_LL + Ut_L^T V_L, Ut = -U^T and V the step's operand slabs
// (128 x np, ld ldv).  Workgroup b takes the 64 x 64 quarter (b >> 1, b & 1).
__global__ __launch_bounds__(256) void k_diag64(double *__restrict__ M, int ld, int L0,
                                                const double *__restrict__ Ut, const double *__restrict__ V, int ldv,
                                                const rdist_info *info) {
    if (info->status != RDIST_OK) return;
    lookahead_priority();
    const int i0 = 64 * (blockIdx.x >> 1), j0 = 64 * (blockIdx.x & 1);
    double *base = M + (size_t)L0 * kTile * ld + (size_t)L0 * kTile + (size_t)i0 * ld + j0;
    d4 acc[2][2];
    {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        const int li = lane & 15, lk = lane >> 4;
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    acc[p][q][r] = base[(size_t)(32 * (w >> 1) + 16 * p + lk + 4 * r) * ld + 32 * (w & 1) + 16 * q + li];
    }
    piece_mma(acc, Ut + (size_t)L0 * kTile, ldv, V + (size_t)L0 * kTile, ldv, i0, j0);
    piece_for_each(acc, [&](int r, int c, double v) { base[(size_t)r * ld + c] = v; });
}

// Row and column tiles of step K (block width 128): workgroups [0, 4 nt)
// form V_J = P M_KJ for J != K, a 64 x 64 quarter each (Pt = P^T, ld 128);
// workgroups [4 nt, 8 nt) the negated transposed column block,
// Ut_I = -(M_IK)^T for I != K and +I for I = K (U_K = -I), a 64 x 64 piece
// each through LDS (one workgroup per tile, its four pieces in turn, held
// the launch at the 22 us of the single-workgroup products).
__global__ __launch_bounds__(256) void k_rowcol64(const double *__restrict__ M, int ld, int nt, int K,
                                                  const double *__restrict__ Pt, double *__restrict__ Ut,
                                                  double *__restrict__ V, int ldv, const rdist_info *info) {
    if (info->status != RDIST_OK) return;
    lookahead_priority();
    const int blk = blockIdx.x;
    if (blk < 4 * nt) {
        const int J = blk >> 2, i0 = 64 * ((blk >> 1) & 1), j0 = 64 * (blk & 1);
        if (J == K) return;
        d4 acc[2][2];
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < 2; ++q) acc[p][q] = d4{0.0, 0.0, 0.0, 0.0};
        piece_mma(acc, Pt, kTile, M + (size_t)K * kTile * ld + (size_t)J * kTile, ld, i0, j0);
        double *out = V + (size_t)J * kTile + (size_t)i0 * ldv + j0;
        piece_for_each(acc, [&](int r, int c, double v) { out[(size_t)r * ldv + c] = v; });
        return;
    }
    __shared__ double t[64][65];
    const int e0 = blk - 4 * nt, I = e0 >> 2, bi = (e0 >> 1) & 1, bk = e0 & 1;
    double *out = Ut + (size_t)I * kTile + (size_t)bk * 64 * ldv + bi * 64;   // Ut[64 bk + k][I*128 + 64 bi + i]
    if (I == K) {
        for (int e = threadIdx.x; e < 64 * 64; e += 256) {
            const int k = e >> 6, i = e & 63;
            out[(size_t)k * ldv + i] = (bk * 64 + k == bi * 64 + i) ? 1.0 : 0.0;
        }
        return;
    }
    const double *src = M + (size_t)(I * kTile + bi * 64) * ld + (size_t)K * kTile + bk * 64;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int r = e >> 6, c = e & 63;     // r: row i, c: column k
        t[r][c] = src[(size_t)r * ld + c];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int k = e >> 6, i = e & 63;
        out[(size_t)k * ldv + i] = -t[i][k];
    }
}

}  // namespace

void launch_diag64(double *M, int ld, int L0, const double *Ut, const double *V, int ldv, const rdist_info *info,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_diag64, dim3(4), dim3(256), 0, s, M, ld, L0, Ut, V, ldv, info);
}

void launch_rowcol64(const double *M, int ld, int nt, int K, const double *Pt, double *Ut, double *V, int ldv,
                     const rdist_info *info, hipStream_t s) {
    hipLaunchKernelGGL(k_rowcol64, dim3(8 * nt), dim3(256), 0, s, M, ld, nt, K, Pt, Ut, V, ldv, info);
}

}  // namespace rd
