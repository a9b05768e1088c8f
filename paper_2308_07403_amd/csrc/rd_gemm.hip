// rd_gemm.hip -- the matrix-core contractions of the mixed-precision plan
// (RDIST_MIXED_F32, the FP64 precision limit of Sec. 5.1 restated for FP32):
//
//   k_gemm32     FP32 blocked Gauss-Jordan on v_mfma_f32_32x32x2f32:
//                the row product V = P M_K,: and the trailing update
//                M <- M~ - U V of one 256-wide step, over 128 x 128 tiles;
//   k_corr_bf16  the refinement's correction C = X0 R from bf16 hi/lo parts,
//                C = Xh Rh + Xh Rl + Xl Rh on v_mfma_f32_32x32x16_bf16 with
//                FP32 accumulation, over 256 x 256 tiles;
//   k_ut32, k_split_bf16_x, k_split_bf16_t: the operand layouts these
//                read.
//
// Both contractions read k-chunks of their operands from LDS, copied there
// by the load unit (global_load_lds, 16 bytes per lane, double-buffered), so
// no VGPRs stage the copies; 256 threads = 4 waves, wave w owns a quadrant
// (w >> 1, w & 1) of the tile as blocks of 32 x 32.  (Measured and dropped
// for the FP32 update: 128 x 256 tiles with 2 x 4 blocks per wave, two
// workgroups per compute unit, 1194 against 1140 us per C4 step.)
// Accumulator element r of lane l in a 32 x 32 block is row
// 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32 (both instructions; checked
// on gfx950).
#include <hip/hip_runtime.h>
#include <algorithm>
#include <stdint.h>

#include "rd_device.h"
#include "rd_launch.h"

namespace rd {

namespace {

constexpr int kT = 128;                 // output tile
constexpr int kMB = 256;                // step width of the FP32 Gauss-Jordan (inner dimension of k_gemm32)
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

struct Acc32 {
    f32x16 v[2][2];
};

// Row / column within the tile of accumulator element (p, q, r) of this lane.
__device__ __forceinline__ int acc_row(int p, int r) {
    return ((threadIdx.x >> 6) >> 1) * 64 + 32 * p + 8 * (r >> 2) + 4 * ((threadIdx.x & 63) >> 5) + (r & 3);
}
__device__ __forceinline__ int acc_col(int q) { return ((threadIdx.x >> 6) & 1) * 64 + 32 * q + (threadIdx.x & 31); }

// ---- FP32: operands k-major, A_k[k][i], B_k[k][j] ----
// 128 x 128 output tiles, wave w owns the 64 x 64 quadrant (w >> 1, w & 1)
// as 2 x 2 blocks of 32 x 32; 16 KiB of LDS, so the registers (about 90
// VGPRs) decide how many workgroups share a compute unit (five) and hide
// each other's memory latency.  (In the C4 solve: 8-row k-chunks with
// fragments read one k-step ahead 120.5 TFLOP/s, 16-row chunks without 119.6.)
constexpr int kKC32 = 8;                      // k-rows per chunk
constexpr int kChunk32 = kKC32 * kT;          // floats per operand chunk (4 KiB)

// Wave w copies k-rows (kKC32 / 4) w .. of both operands' chunk at k0; one
// instruction moves two k-rows of 128 floats (lanes 0-31 the first).
__device__ __forceinline__ void dma32(const float *__restrict__ A, int lda, const float *__restrict__ B, int ldb,
                                      int k0, float *As, float *Bs) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int half = lane >> 5, c = (lane & 31) * 4;
#pragma unroll
    for (int q = 0; q < kKC32 / 8; ++q) {
        const int r = w * (kKC32 / 4) + 2 * q;
        __builtin_amdgcn_global_load_lds((global_cvoid *)(A + (size_t)(k0 + r + half) * lda + c),
                                         (lds_void *)(As + r * kT), 16, 0, 0);
        __builtin_amdgcn_global_load_lds((global_cvoid *)(B + (size_t)(k0 + r + half) * ldb + c),
                                         (lds_void *)(Bs + r * kT), 16, 0, 0);
    }
}

// One chunk: kKC32 / 2 k-steps of 2, four 32 x 32 blocks per step, each
// step's fragments read from LDS one step ahead.
__device__ __forceinline__ void mma32_chunk(const float *As, const float *Bs, Acc32 &acc) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m0 = (w >> 1) * 64 + (lane & 31), n0 = (w & 1) * 64 + (lane & 31), kr = lane >> 5;
    float a[2][2], b[2][2];
    auto frags = [&](int ks, float *af, float *bf) {
        const float *ar = As + (2 * ks + kr) * kT, *br = Bs + (2 * ks + kr) * kT;
        af[0] = ar[m0];
        af[1] = ar[m0 + 32];
        bf[0] = br[n0];
        bf[1] = br[n0 + 32];
    };
    frags(0, a[0], b[0]);
#pragma unroll
    for (int ks = 0; ks < kKC32 / 2; ++ks) {
        const int cur = ks & 1;
        if (ks + 1 < kKC32 / 2) frags(ks + 1, a[cur ^ 1], b[cur ^ 1]);
        acc.v[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[cur][0], b[cur][0], acc.v[0][0], 0, 0, 0);
        acc.v[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[cur][0], b[cur][1], acc.v[0][1], 0, 0, 0);
        acc.v[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[cur][1], b[cur][0], acc.v[1][0], 0, 0, 0);
        acc.v[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[cur][1], b[cur][1], acc.v[1][1], 0, 0, 0);
    }
}

// Ut (kMB x np, k-major) = -U^T for the step at column K0 of M (np x np):
// Ut[k][i] = -M[i][K0 + k] for rows i outside the block, and the identity
// (U's rows there are -I) for rows inside it.  64 x 64 pieces through LDS,
// both sides coalesced.
__global__ __launch_bounds__(256) void k_ut32(const float *__restrict__ M, int np, int K0, float *__restrict__ Ut,
                                              const rdist_info *info) {
    if (info->status != RDIST_OK) return;
    __shared__ float t[64][65];
    const int i0 = blockIdx.x * 64, k0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) t[r][tx] = M[(size_t)(i0 + r) * np + K0 + k0 + tx];
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int k = k0 + r, i = i0 + tx;
        const bool in = i >= K0 && i < K0 + kMB;
        Ut[(size_t)k * np + i] = in ? (i - K0 == k ? 1.0f : 0.0f) : -t[tx][r];
    }
}

// MODE 0 (row product): tile (I, J) = blockIdx.x as I * ntj + J, C = A_k^T B_k,
// except the tiles J in [zk0, zk0 + 2) (the step's block: its P is written
// there by the block inverse).  (The step's Ut formed by extra workgroups of
// this launch took 41 us against 26 + 13.5 us for the two launches.)
// MODE 1 (trailing update): tiles of an ntj x ntj grid in XCD strip order,
// C <- C~ + A_k^T B_k, where C~ is C with the tile rows and columns
// [zk0, zk0 + 2) (the step's block) zeroed; A_k holds -U^T.  The tiles of
// the next block's diagonal (rows and columns [zk0 + 2, zk0 + 4)) also go to
// Snext (256 x 256, FP64, exact), the input of its block inverse.
// Inner dimension kMB (256).
template <int MODE>
__global__ __launch_bounds__(256, 4) void k_gemm32(float *__restrict__ C, int ldc, int ntj, int zk0,
                                                   const float *__restrict__ Ak, int lda,
                                                   const float *__restrict__ Bk, int ldb, double *__restrict__ Snext,
                                                   const rdist_info *info) {
    if (info->status != RDIST_OK) return;
    __shared__ float lds[4 * kChunk32];   // A, B x two buffers: 16 KiB
    int I, J;
    if (MODE == 1) {
        xcd_strip_order(blockIdx.x, ntj, I, J);
    } else {
        I = blockIdx.x / ntj;
        J = blockIdx.x - I * ntj;
        if (J >= zk0 && J < zk0 + 2) return;
    }
    const float *A = Ak + (size_t)I * kT, *B = Bk + (size_t)J * kT;
    float *base = C + (size_t)I * kT * ldc + (size_t)J * kT;
    dma32(A, lda, B, ldb, 0, lds, lds + kChunk32);
    Acc32 acc;
    const bool zero = MODE == 0 || (I >= zk0 && I < zk0 + 2) || (J >= zk0 && J < zk0 + 2);
    if (zero) {
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc.v[p][q][r] = 0.0f;
    } else {
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc.v[p][q][r] = base[(size_t)acc_row(p, r) * ldc + acc_col(q)];
    }
    wait_vm_all();
    __syncthreads();
    constexpr int nch = kMB / kKC32;
#pragma unroll 1
    for (int ch = 0; ch < nch; ++ch) {
        float *cur = lds + (ch & 1) * (2 * kChunk32);
        float *nxt = lds + ((ch + 1) & 1) * (2 * kChunk32);
        if (ch + 1 < nch) dma32(A, lda, B, ldb, (ch + 1) * kKC32, nxt, nxt + kChunk32);
        mma32_chunk(cur, cur + kChunk32, acc);
        wait_vm_all();
        __syncthreads();
    }
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int r = 0; r < 16; ++r) base[(size_t)acc_row(p, r) * ldc + acc_col(q)] = acc.v[p][q][r];
    if constexpr (MODE == 1) {
        if (Snext && I >= zk0 + 2 && I < zk0 + 4 && J >= zk0 + 2 && J < zk0 + 4) {
            // read back what this thread just stored (the barrier keeps the
            // compiler from holding the accumulators live for this copy,
            // which cost the kernel 40 VGPRs and its fifth workgroup)
            asm volatile("" ::: "memory");
            double *sb = Snext + (size_t)(I - zk0 - 2) * kT * kMB + (size_t)(J - zk0 - 2) * kT;
            for (int p = 0; p < 2; ++p)
                for (int q = 0; q < 2; ++q)
                    for (int r = 0; r < 16; ++r)
                        sb[(size_t)acc_row(p, r) * kMB + acc_col(q)] =
                            (double)base[(size_t)acc_row(p, r) * ldc + acc_col(q)];
        }
    }
}

// ---- bf16: operands m-major, hi and lo parts interleaved per 32 k ----
// Row r of an operand (X, or R transposed) holds, for each block b of 32
// k-values, the 32 hi parts and then the 32 lo parts (row length 2K), so one
// 128-byte line per row and chunk carries both and the three products share
// every chunk: 64 KiB of copies per 96 MFMAs of a wave, against 64 per 64
// with the products run one after another on separate parts (the C4
// correction: 24.7 -> 21.0 ms on its own; the copies, not the matrix cores,
// bound it: without them the products run in 17.6 ms, the copies alone take
// 18.8 ms at the old layout).
// 256 x 256 output tiles; wave w owns the 128 x 128 quadrant (w >> 1, w & 1)
// as 4 x 4 blocks of 32 x 32 (accumulators in 256 AGPRs, one wave per SIMD),
// so each fragment read from LDS feeds four MFMAs per product.
// (Measured and dropped: 2 x 2 blocks per wave, LDS-bound; rings of three to
// five 32-k chunks with barriers that wait only for the oldest chunk, 27.0 -
// 27.6 ms against 25.4 for the double buffer of 64-k chunks then in use,
// whose loads were throughput- and not latency-bound; row pitches padded by
// 128 - 512 bytes, no change; this form with its chunk barrier between the
// two k-steps, so that the next chunk's copy and first fragments overlap the
// second step's products, 21.25 against 21.2 ms.)
constexpr int kTB = 256;                // output tile of the bf16 contraction
constexpr int kKCb = 32;                // k per chunk (hi and lo: 64 values per row)
constexpr int kRowB = 128;              // bytes per LDS row (eight 16-byte pieces)
constexpr int kChunkB = kTB * kRowB;    // bytes per operand chunk (32 KiB)

struct AccB {
    f32x16 v[4][4];
};

// Position of piece c of row r within the row (pieces 0-3 the hi parts of
// k0 + 8c .. k0 + 8c + 7, pieces 4-7 the lo parts): c ^ swz(r),
// swz(r) = (r & 7) ^ ((r >> 3) & 1).  A fragment load reads one piece of 32
// consecutive rows (16 bytes per lane); every 8 consecutive rows aligned to 8
// then sit in distinct 16-byte slots of a 128-byte bank window, and every 16
// aligned to 16 in distinct slots of a 256-byte one, so the load is free of
// bank conflicts whether the LDS serves 8 lanes over 32 banks or 16 lanes
// over 64 banks per cycle.  (With swz(r) = r & 7 the second case conflicts
// two ways on gfx950: SQ_LDS_BANK_CONFLICT was 4 cycles per LDS instruction,
// now 0.)
__device__ __forceinline__ int swzb(int r) { return (r & 7) ^ ((r >> 3) & 1); }

// Wave w copies rows 64w .. 64w+63 of both operands' chunk at k0 (an offset
// in the interleaved row), eight rows per instruction, each piece to its
// swizzled position.
__device__ __forceinline__ void dmab(const uint16_t *__restrict__ A, const uint16_t *__restrict__ B, int pitch,
                                     int k0, char *As, char *Bs) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int rr = lane >> 3;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int r0 = w * 64 + q * 8;
        const int c = (lane & 7) ^ swzb(r0 + rr);   // the piece that belongs at slot lane & 7
        __builtin_amdgcn_global_load_lds((global_cvoid *)(A + (size_t)(r0 + rr) * pitch + k0 + 8 * c),
                                         (lds_void *)(As + r0 * kRowB), 16, 0, 0);
        __builtin_amdgcn_global_load_lds((global_cvoid *)(B + (size_t)(r0 + rr) * pitch + k0 + 8 * c),
                                         (lds_void *)(Bs + r0 * kRowB), 16, 0, 0);
    }
}

__device__ __forceinline__ bf16x8 frag_b(const char *S, int row, int c) {
    return *reinterpret_cast<const bf16x8 *>(S + row * kRowB + ((c ^ swzb(row)) << 4));
}

// Fragments of k-step st (16 k) of the chunk: lane l holds k 8 (l / 32) ..
// +7 of the step, hi parts from piece 2 st + l / 32, lo parts four pieces on.
__device__ __forceinline__ void frags_b(const char *As, const char *Bs, int st, bf16x8 *xh, bf16x8 *xl, bf16x8 *rh,
                                        bf16x8 *rl) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int mr = (w >> 1) * 128 + (lane & 31), nr = (w & 1) * 128 + (lane & 31);
    const int c = 2 * st + (lane >> 5);
#pragma unroll
    for (int p = 0; p < 4; ++p) xh[p] = frag_b(As, mr + 32 * p, c);
#pragma unroll
    for (int q = 0; q < 4; ++q) rh[q] = frag_b(Bs, nr + 32 * q, c);
#pragma unroll
    for (int q = 0; q < 4; ++q) rl[q] = frag_b(Bs, nr + 32 * q, 4 + c);
#pragma unroll
    for (int p = 0; p < 4; ++p) xl[p] = frag_b(As, mr + 32 * p, 4 + c);
}

// One k-step: the 16 blocks' Xh Rh, then Xh Rl, then Xl Rh (each block's
// three MFMAs sixteen apart, so none waits on the one before).
__device__ __forceinline__ void mmab_step(const bf16x8 *xh, const bf16x8 *xl, const bf16x8 *rh, const bf16x8 *rl,
                                          AccB &acc) {
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            acc.v[p][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[p], rh[q], acc.v[p][q], 0, 0, 0);
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            acc.v[p][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[p], rl[q], acc.v[p][q], 0, 0, 0);
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            acc.v[p][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xl[p], rh[q], acc.v[p][q], 0, 0, 0);
}

// C (nti*256 x ntj*256, ldc) = Xh Rh + Xh Rl + Xl Rh, inner dimension K (a
// multiple of 32): X interleaved by rows (row i: row i of X), R interleaved
// transposed (row j: column j of R), both with row length 2K.
__global__ __launch_bounds__(256, 1) void k_corr_bf16(float *__restrict__ C, int ldc, int nti, int ntj, int K,
                                                      const uint16_t *__restrict__ Xi,
                                                      const uint16_t *__restrict__ Ri, const rdist_info *info) {
    if (info->status != RDIST_OK) return;
    __shared__ __attribute__((aligned(16))) char lds[4 * kChunkB];   // A, B x two buffers: 128 KiB
    int I, J;
    xcd_strip_order_rect(blockIdx.x, nti, ntj, I, J);
    const int pitch = 2 * K;
    const uint16_t *A = Xi + (size_t)I * kTB * pitch, *B = Ri + (size_t)J * kTB * pitch;
    const int nch = K / kKCb;
    dmab(A, B, pitch, 0, lds, lds + kChunkB);
    AccB acc;
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc.v[p][q][r] = 0.0f;
    wait_vm_all();
    __syncthreads();
    bf16x8 xh[4], xl[4], rh[4], rl[4];
#pragma unroll 1
    for (int ch = 0; ch < nch; ++ch) {
        char *cur = lds + (ch & 1) * (2 * kChunkB);
        char *nxt = lds + ((ch + 1) & 1) * (2 * kChunkB);
        if (ch + 1 < nch) dmab(A, B, pitch, 2 * kKCb * (ch + 1), nxt, nxt + kChunkB);
        frags_b(cur, cur + kChunkB, 0, xh, xl, rh, rl);
        mmab_step(xh, xl, rh, rl, acc);
        frags_b(cur, cur + kChunkB, 1, xh, xl, rh, rl);
        mmab_step(xh, xl, rh, rl, acc);
        wait_vm_all();
        __syncthreads();
    }
    float *base = C + (size_t)I * kTB * ldc + (size_t)J * kTB;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = (w >> 1) * 128 + 32 * p + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int col = (w & 1) * 128 + 32 * q + (lane & 31);
                base[(size_t)row * ldc + col] = acc.v[p][q][r];
            }
}

// bf16 with round to nearest even of a finite float (its 16 high bits).
__device__ __forceinline__ uint16_t bf16_bits(float x) {
    const unsigned u = __float_as_uint(x);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// Power-of-two exponent s with 2^s max|R| in [0.5, 1) (0 when R is zero).
__device__ __forceinline__ int rscale(unsigned rmax_bits) {
    if (rmax_bits == 0) return 0;
    return -((int)((rmax_bits >> 23) & 0xFF) - 127 + 1);
}

// Index of element k of interleaved row r (row length 2 cols): its hi part;
// the lo part sits 32 further on.
__device__ __forceinline__ size_t ileave(size_t r, int cols, int k) {
    return r * 2 * (size_t)cols + 2 * (size_t)(k & ~31) + (k & 31);
}

// hi / lo bf16 parts of X (rows x cols, row-major), interleaved by rows.
__global__ __launch_bounds__(256) void k_split_bf16_x(const float *__restrict__ X, int rows, int cols,
                                                      uint16_t *__restrict__ Xi) {
    const size_t count = (size_t)rows * cols;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (size_t)gridDim.x * 256) {
        const float x = X[e];
        const uint16_t h = bf16_bits(x);
        const size_t o = ileave(e / cols, cols, (int)(e % cols));
        Xi[o] = h;
        Xi[o + 32] = bf16_bits(x - __uint_as_float((unsigned)h << 16));
    }
}

// hi / lo bf16 parts of 2^s R, transposed and interleaved: R is rows x cols
// (ld cols), Ri is cols_pad x 2 rows, rows cols .. cols_pad - 1 zero; s from
// rmax as for the residual.
__global__ __launch_bounds__(256) void k_split_bf16_t(const float *__restrict__ R, int rows, int cols,
                                                      uint16_t *__restrict__ Ri, const unsigned *__restrict__ rmax) {
    __shared__ float t[64][65];
    const float sc = ldexpf(1.0f, rscale(*rmax));
    const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) t[r][tx] = c0 + tx < cols ? R[(size_t)(r0 + r) * cols + c0 + tx] * sc : 0.0f;
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const float x = t[tx][r];
        const uint16_t h = bf16_bits(x);
        const size_t o = ileave((size_t)(c0 + r), rows, r0 + tx);
        Ri[o] = h;
        Ri[o + 32] = bf16_bits(x - __uint_as_float((unsigned)h << 16));
    }
}

}  // namespace

void launch_gemm32_rows(const float *Pt, const float *M, int np, int K0, float *V, const rdist_info *info,
                        hipStream_t s) {
    const int nt = np / kT;
    hipLaunchKernelGGL(k_gemm32<0>, dim3(2 * nt), dim3(256), 0, s, V, np, nt, K0 / kT, Pt, kMB, M + (size_t)K0 * np,
                       np, nullptr, info);
}

void launch_gemm32_update(float *M, int np, int K0, const float *Ut, const float *V, double *Snext,
                          const rdist_info *info, hipStream_t s) {
    const int nt = np / kT;
    hipLaunchKernelGGL(k_gemm32<1>, dim3(nt * nt), dim3(256), 0, s, M, np, nt, K0 / kT, Ut, np, V, np, Snext, info);
}

void launch_ut32(const float *M, int np, int K0, float *Ut, const rdist_info *info, hipStream_t s) {
    hipLaunchKernelGGL(k_ut32, dim3(np / 64, kMB / 64), dim3(256), 0, s, M, np, K0, Ut, info);
}

int corr_cols(int cols) { return (cols + kTB - 1) / kTB * kTB; }

void launch_corr_bf16(float *C, int rows, int cols_pad, int K, const uint16_t *Xi, const uint16_t *Ri,
                      const rdist_info *info, hipStream_t s) {
    const int nti = rows / kTB, ntj = cols_pad / kTB;
    hipLaunchKernelGGL(k_corr_bf16, dim3(nti * ntj), dim3(256), 0, s, C, cols_pad, nti, ntj, K, Xi, Ri, info);
}

void launch_split_bf16_x(const float *X, int rows, int cols, uint16_t *Xi, hipStream_t s) {
    const int grid = (int)std::min<size_t>(((size_t)rows * cols + 255) / 256, 16384);
    hipLaunchKernelGGL(k_split_bf16_x, dim3(grid), dim3(256), 0, s, X, rows, cols, Xi);
}

void launch_split_bf16_t(const float *R, int rows, int cols, int cols_pad, uint16_t *Ri, const unsigned *rmax,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_split_bf16_t, dim3(cols_pad / 64, rows / 64), dim3(256), 0, s, R, rows, cols, Ri, rmax);
}

}  // namespace rd
