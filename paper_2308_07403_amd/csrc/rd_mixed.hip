// rd_mixed.hip -- mixed-precision solve (RDIST_MIXED_F32).
//
// Y is first formed in FP32: blocked Gauss-Jordan with b = 256, the 256 x 256
// diagonal block inverted in FP64 (the FP64 register / MFMA kernels, in
// place on a converted copy), and the row product V = P M_K,: and the
// trailing update M <- M~ - U V on the FP32 matrix cores (rd_gemm.hip).
// Every entry of the FP32 result X0 is then certified or not (Sec. 5, the
// FP64 precision limit, restated for FP32):
//   uncertified  iff  X0 < FLT_MIN (zero included: FP32 cannot tell an
//                underflowed entry from an unreachable one), or
//                |R32 - round(R32)| < margin, R32 = log(X0) / log(gamma);
// a certified entry's D = ceil(R32 - eta) is the FP64 answer, because the
// FP32 error in R is far below the margin.  Uncertified entries are
// recomputed to FP64 accuracy:
//   * no underflow: one refinement step Y = X0 + X0 (I - M X0) on the
//     128-column slabs that hold them.  The residual is formed in FP64 from
//     the sparse adjacency (it is of order eps32 * Y entrywise, M being an
//     M-matrix with Y >= 0), so the product X0 R, formed from bf16 hi/lo
//     parts on the bf16 matrix cores (rd_gemm.hip), adds an error of order
//     2^-16 eps32 * Y;
//   * some underflow: the whole graph goes through the FP64 blocked plan.
// The call synchronises the stream once (after certification), because the
// size of the recompute is data-dependent.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/rdist.h"
#include "rd_device.h"
#include "rd_engine.h"
#include "rd_launch.h"

namespace rd {

namespace {

constexpr int kMB = 256;      // block width of the FP32 Gauss-Jordan
constexpr int kSlab = 128;    // column slab of the refinement

// M32 = I - gamma A (n x n), identity on the padding (np x np).
__global__ __launch_bounds__(256) void k_m32_build(const uint8_t *__restrict__ A, int n, int np,
                                                   float *__restrict__ M, const rdist_info *info) {
    if (info->status != RDIST_OK) return;
    const double gamma = info->gamma;
    const size_t total = (size_t)np * np;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
        const int i = (int)(e / np), j = (int)(e - (size_t)i * np);
        double x = (i == j) ? 1.0 : 0.0;
        if (i < n && j < n) x -= gamma * (double)A[(size_t)i * n + j];
        M[e] = (float)x;
    }
}

// S (256 x 256 FP64) = the diagonal block at K0 of M.
__global__ __launch_bounds__(256) void k_diag_to_f64(const float *__restrict__ M, int np, int K0,
                                                     double *__restrict__ S) {
    for (int e = blockIdx.x * 256 + threadIdx.x; e < kMB * kMB; e += gridDim.x * 256) {
        const int r = e >> 8, c = e & 255;
        S[e] = (double)M[(size_t)(K0 + r) * np + K0 + c];
    }
}

__device__ __forceinline__ bool uncertified(float y, double il, double margin) {
    if (!(y >= FLT_MIN)) return true;
    const double r = log((double)y) * il;
    return fabs(r - rint(r)) < margin;
}

// Certification of X (FP32, n x n inside np x np): certified entries get D;
// uncertified ones are counted (cnt[0]; cnt[1] those below FLT_MIN) and
// their 128-column slab flagged.
__global__ __launch_bounds__(256) void k_certify(const float *__restrict__ X, int np, int n, double margin,
                                                 int16_t *__restrict__ D, int32_t *__restrict__ slab_flag,
                                                 unsigned long long *cnt, rdist_info *info) {
    if (info->status != RDIST_OK) return;
    const double il = rd_inv_log(info->gamma);
    Counts c;
    unsigned long long unc = 0, under = 0;
    const size_t total = (size_t)n * n;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
        const int i = (int)(e / n), j = (int)(e - (size_t)i * n);
        const float y = X[(size_t)i * np + j];
        if (uncertified(y, il, margin)) {
            ++unc;
            under += !(y >= FLT_MIN);
            slab_flag[j / kSlab] = 1;
        } else {
            D[e] = rd_encode((double)y, il, c);
        }
    }
    flush_counts(info, c);
    unc = wave_sum_u64(unc);
    under = wave_sum_u64(under);
    if ((threadIdx.x & 63) == 0) {
        if (unc) atomicAdd(&cnt[0], unc);
        if (under) atomicAdd(&cnt[1], under);
    }
}

// Nonzeros per row of A (row i lists the in-neighbours of i).
__global__ __launch_bounds__(256) void k_row_count(const uint8_t *__restrict__ A, int n, int32_t *cnt) {
    __shared__ int tot;
    if (threadIdx.x == 0) tot = 0;
    __syncthreads();
    const uint8_t *row = A + (size_t)blockIdx.x * n;
    int c = 0;
    for (int j = threadIdx.x; j < n; j += 256) c += row[j] != 0;
    atomicAdd(&tot, c);
    __syncthreads();
    if (threadIdx.x == 0) cnt[blockIdx.x] = tot;
}

// Column indices of row i's nonzeros, in increasing order.  The workgroup
// walks the row 256 bytes at a time (coalesced byte loads); a ballot gives
// each nonzero its rank within its wave, the four wave totals (in LDS, two
// slots used alternately, so one barrier per chunk suffices) its offset.
// (Each thread scanning its own 64-byte stretch byte by byte took 1.0 ms at
// n = 16384.)
__global__ __launch_bounds__(256) void k_row_fill(const uint8_t *__restrict__ A, int n,
                                                  const int64_t *__restrict__ off, int32_t *__restrict__ cols) {
    __shared__ int wsum[2][4];
    const uint8_t *row = A + (size_t)blockIdx.x * n;
    int32_t *out = cols + off[blockIdx.x];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int base = 0;   // nonzeros of the chunks before this one
    for (int j0 = 0, it = 0; j0 < n; j0 += 256, ++it) {
        const int j = j0 + threadIdx.x;
        const bool nz = j < n && row[j] != 0;
        const unsigned long long m = __ballot(nz);
        const int rank = __popcll(m & ((1ull << lane) - 1ull));
        int *t = wsum[it & 1];
        if (lane == 0) t[w] = __popcll(m);
        __syncthreads();
        int before = base;
        for (int v = 0; v < w; ++v) before += t[v];
        if (nz) out[before + rank] = j;
        base += t[0] + t[1] + t[2] + t[3];
    }
}

// R (np x w, w = 128 nslab) = I - M X on the slabs: for row k and column
// j of slab s, R = [k == j] - X[k][j] + gamma * sum over nonzeros l of
// A's row k of X[l][j], accumulated in FP64, stored in FP32.  A thread
// takes four columns (16-byte loads of X), 32 threads a row of the slab, a
// workgroup eight rows; the nonzero loop is unrolled by four with the index
// loads first, so that four row loads are in flight.
__global__ __launch_bounds__(256) void k_residual(const float *__restrict__ X, int np, int n,
                                                  const int64_t *__restrict__ off, const int32_t *__restrict__ cols,
                                                  const int32_t *__restrict__ slabs, int nslab, float *__restrict__ R,
                                                  unsigned *__restrict__ rmax, const rdist_info *info) {
    if (info->status != RDIST_OK) return;
    const double gamma = info->gamma;
    const int k = blockIdx.x * 8 + (threadIdx.x >> 5), c = (threadIdx.x & 31) * 4;
    const int s = blockIdx.y;
    const int j = slabs[s] * kSlab + c;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (k < n) {
        int64_t e = off[k];
        const int64_t e1 = off[k + 1];
        for (; e + 4 <= e1; e += 4) {
            const int l0 = cols[e], l1 = cols[e + 1], l2 = cols[e + 2], l3 = cols[e + 3];
            const float4 x0 = *reinterpret_cast<const float4 *>(X + (size_t)l0 * np + j);
            const float4 x1 = *reinterpret_cast<const float4 *>(X + (size_t)l1 * np + j);
            const float4 x2 = *reinterpret_cast<const float4 *>(X + (size_t)l2 * np + j);
            const float4 x3 = *reinterpret_cast<const float4 *>(X + (size_t)l3 * np + j);
            a0 += ((double)x0.x + (double)x1.x) + ((double)x2.x + (double)x3.x);
            a1 += ((double)x0.y + (double)x1.y) + ((double)x2.y + (double)x3.y);
            a2 += ((double)x0.z + (double)x1.z) + ((double)x2.z + (double)x3.z);
            a3 += ((double)x0.w + (double)x1.w) + ((double)x2.w + (double)x3.w);
        }
        for (; e < e1; ++e) {
            const float4 x = *reinterpret_cast<const float4 *>(X + (size_t)cols[e] * np + j);
            a0 += (double)x.x;
            a1 += (double)x.y;
            a2 += (double)x.z;
            a3 += (double)x.w;
        }
    }
    if (k >= np) return;
    const float4 xk = *reinterpret_cast<const float4 *>(X + (size_t)k * np + j);
    float4 r;
    r.x = (float)(((k == j) ? 1.0 : 0.0) - (double)xk.x + gamma * a0);
    r.y = (float)(((k == j + 1) ? 1.0 : 0.0) - (double)xk.y + gamma * a1);
    r.z = (float)(((k == j + 2) ? 1.0 : 0.0) - (double)xk.z + gamma * a2);
    r.w = (float)(((k == j + 3) ? 1.0 : 0.0) - (double)xk.w + gamma * a3);
    *reinterpret_cast<float4 *>(R + (size_t)k * ((size_t)nslab * kSlab) + (size_t)s * kSlab + c) = r;
    // largest |R| (the bits of a nonnegative float order like its value)
    unsigned m = max(max(__float_as_uint(fabsf(r.x)), __float_as_uint(fabsf(r.y))),
                     max(__float_as_uint(fabsf(r.z)), __float_as_uint(fabsf(r.w))));
    for (int off = 32; off > 0; off >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, off, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(rmax, m);
}

// Power-of-two exponent s with 2^s max|R| in [0.5, 1) (0 when R is zero).
__device__ __forceinline__ int residual_scale(unsigned rmax_bits) {
    if (rmax_bits == 0) return 0;
    const int e = (int)((rmax_bits >> 23) & 0xFF) - 127;   // max|R| in [2^e, 2^(e+1))
    return -(e + 1);
}

// Uncertified entries of the slabs: Y = X + (X R), the correction C = X R
// (np x w) from the GEMMs on the residual scaled by 2^s (undone here
// exactly); D from Y in FP64.  Workgroup (s, y) takes rows 32y .. 32y + 31
// of slab s, two at a time; the slabs vary fastest, so consecutive
// workgroups stream along the rows of X, C and D.
__global__ __launch_bounds__(256) void k_fix(const float *__restrict__ X, int np, int n, const float *__restrict__ C,
                                             int ldc, const int32_t *__restrict__ slabs, int nslab, double margin,
                                             const unsigned *__restrict__ rmax, int16_t *__restrict__ D,
                                             rdist_info *info) {
    if (info->status != RDIST_OK) return;
    const double il = rd_inv_log(info->gamma);
    const double unscale = rmax ? ldexp(1.0, -residual_scale(*rmax)) : 1.0;
    const int c = threadIdx.x & 127;
    const int s = blockIdx.x;
    const int j = slabs[s] * kSlab + c;
    Counts cnt;
    for (int t = 0; t < 16; ++t) {
        const int i = blockIdx.y * 32 + 2 * t + (threadIdx.x >> 7);
        if (i < n && j < n) {
            const float x = X[(size_t)i * np + j];
            if (uncertified(x, il, margin)) {
                const double y = (double)x + unscale * (double)C[(size_t)i * ldc + (size_t)s * kSlab + c];
                D[(size_t)i * n + j] = rd_encode(y, il, cnt);
            }
        }
    }
    flush_counts(info, cnt);
}

// One 128-pivot step of the 256 x 256 block inverse (2 x 2 tiles of 128):
// from S (ld 256) and P = S_kk^{-1} (ld 256, written by the panel), with
// o = 1 - k,
//     T_kk = P,  T_ko = P S_ko,  T_ok = -S_ok P,  T_oo = S_oo - S_ok (P S_ko)
// into T (ld 256): one Gauss-Jordan step of the inversion behind Eq. Y-defined
// (the cost Sec. 5.2 names as dominant) on the block's 2 x 2 tiles.  One launch in place of the row and column products
// and the tile update of the general step (two launches of one or four
// 128 x 128 products on one workgroup each, about 21 us apiece), 15.5 us:
// 64 workgroups of 32 x 32 pieces, 16 per tile; wave w forms the 16 x 16 block
// (w >> 1, w & 1) of its piece, and a piece of T_oo first forms its
// 128 x 32 strip of P S_ko in LDS.  Every product takes the operands, the
// starting accumulator (zero, or S_oo) and the k order of those kernels, so
// T is bit for bit what they give.  On the last step (Pt32 given) T is the
// block's inverse, and the FP32 roundings the next products read are written
// too: Pt32 = T^T (ld 256) and V32's columns K0 .. K0 + 255 = T (ld ldv).
// (Eight workgroups of 16 waves, one block per wave, took 27 us against 25
// for this form before its passes over k were merged and unrolled.)
__global__ __launch_bounds__(256) void k_blk2_step(const double *__restrict__ S, double *__restrict__ T,
                                                   const double *__restrict__ P, int k, float *__restrict__ Pt32,
                                                   float *__restrict__ V32, int ldv, int K0,
                                                   const rdist_info *__restrict__ info) {
    if (info->status != RDIST_OK) return;
    __shared__ double Vs[128][33];
    constexpr int ld = 2 * kTile;
    const int tile = blockIdx.x >> 4, piece = blockIdx.x & 15;
    const int pr = (piece >> 2) * 32, pc = (piece & 3) * 32;
    const int o = 1 - k;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int bi = pr + 16 * (w >> 1), bj = pc + 16 * (w & 1);
    const double *Sok = S + (size_t)o * kTile * ld + (size_t)k * kTile;   // S_ok(i, k) at Sok[i * ld + k]
    const double *Sko = S + (size_t)k * kTile * ld + (size_t)o * kTile;
    // T (i, j) = v, i and j within the block, with the FP32 copies
    auto put = [&](int i, int j, double v) {
        T[(size_t)i * ld + j] = v;
        if (Pt32) {
            Pt32[(size_t)j * ld + i] = (float)v;
            V32[(size_t)i * ldv + K0 + j] = (float)v;
        }
    };
    if (tile == 0) {   // T_kk = P
        for (int e = threadIdx.x; e < 32 * 32; e += 256) {
            const int i = pr + (e >> 5), j = pc + (e & 31);
            put(k * kTile + i, k * kTile + j, P[(size_t)i * ld + j]);
        }
        return;
    }
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    if (tile == 1) {   // T_ko = P S_ko
#pragma unroll
        for (int kk = 0; kk < kTile; kk += 4)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(P[(size_t)(bi + li) * ld + kk + lk],
                                                        Sko[(size_t)(kk + lk) * ld + bj + li], acc, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) put(k * kTile + bi + lk + 4 * r, o * kTile + bj + li, acc[r]);
        return;
    }
    if (tile == 2) {   // T_ok = (-S_ok) P
#pragma unroll
        for (int kk = 0; kk < kTile; kk += 4)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-Sok[(size_t)(bi + li) * ld + kk + lk],
                                                        P[(size_t)(kk + lk) * ld + bj + li], acc, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) put(o * kTile + bi + lk + 4 * r, k * kTile + bj + li, acc[r]);
        return;
    }
    // T_oo: the strip (P S_ko)[:, pc .. pc + 31], wave w its rows 32w .. 32w + 31
    // as 2 x 2 blocks, all four in one pass over k (four separate passes
    // waited on their operand loads four times as often); every pass over k
    // unrolled so that its loads are issued together (25 us with four passes
    // unrolled by 8, 17.5 with one, 15.5 fully unrolled)
    {
        d4 v[2][2] = {};
#pragma unroll
        for (int kk = 0; kk < kTile; kk += 4) {
            double a[2], b[2];
#pragma unroll
            for (int p = 0; p < 2; ++p) a[p] = P[(size_t)(32 * w + 16 * p + li) * ld + kk + lk];
#pragma unroll
            for (int q = 0; q < 2; ++q) b[q] = Sko[(size_t)(kk + lk) * ld + pc + 16 * q + li];
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int q = 0; q < 2; ++q) v[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p], b[q], v[p][q], 0, 0, 0);
        }
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) Vs[32 * w + 16 * p + lk + 4 * r][16 * q + li] = v[p][q][r];
    }
    __syncthreads();
    const double *Soo = S + (size_t)o * kTile * ld + (size_t)o * kTile;
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = Soo[(size_t)(bi + lk + 4 * r) * ld + bj + li];
#pragma unroll
    for (int kk = 0; kk < kTile; kk += 4)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-Sok[(size_t)(bi + li) * ld + kk + lk], Vs[kk + lk][bj - pc + li],
                                                    acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) put(o * kTile + bi + lk + 4 * r, o * kTile + bj + li, acc[r]);
}

__global__ void k_set_mixed_info(rdist_info *info, long long uncertified, double fraction) {
    info->n_uncertified = uncertified;
    info->fallback_fraction = fraction;
}

int grid_for(size_t total) { return (int)std::min<size_t>((total + 255) / 256, 16384); }

}  // namespace

void launch_m32_build(const uint8_t *A, int n, int np, float *M, const rdist_info *info, hipStream_t s) {
    hipLaunchKernelGGL(k_m32_build, dim3(grid_for((size_t)np * np)), dim3(256), 0, s, A, n, np, M, info);
}
void launch_diag_to_f64(const float *M, int np, int K0, double *S, hipStream_t s) {
    hipLaunchKernelGGL(k_diag_to_f64, dim3(256), dim3(256), 0, s, M, np, K0, S);
}
void launch_certify(const float *X, int np, int n, double margin, int16_t *D, int32_t *slab_flag,
                    unsigned long long *cnt, rdist_info *info, hipStream_t s) {
    hipLaunchKernelGGL(k_certify, dim3(grid_for((size_t)n * n)), dim3(256), 0, s, X, np, n, margin, D, slab_flag,
                       cnt, info);
}
void launch_row_count(const uint8_t *A, int n, int32_t *cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_row_count, dim3(n), dim3(256), 0, s, A, n, cnt);
}
void launch_row_fill(const uint8_t *A, int n, const int64_t *off, int32_t *cols, hipStream_t s) {
    hipLaunchKernelGGL(k_row_fill, dim3(n), dim3(256), 0, s, A, n, off, cols);
}
void launch_residual(const float *X, int np, int n, const int64_t *off, const int32_t *cols, const int32_t *slabs,
                     int nslab, float *R, unsigned *rmax, const rdist_info *info, hipStream_t s) {
    hipLaunchKernelGGL(k_residual, dim3(np / 8, nslab), dim3(256), 0, s, X, np, n, off, cols, slabs, nslab, R, rmax,
                       info);
}
void launch_fix(const float *X, int np, int n, const float *C, int ldc, const int32_t *slabs, int nslab,
                double margin, const unsigned *rmax, int16_t *D, rdist_info *info, hipStream_t s) {
    hipLaunchKernelGGL(k_fix, dim3(nslab, np / 32), dim3(256), 0, s, X, np, n, C, ldc, slabs, nslab, margin, rmax, D,
                       info);
}
void launch_blk2_step(const double *S, double *T, const double *P, int k, float *Pt32, float *V32, int ldv, int K0,
                      const rdist_info *info, hipStream_t s) {
    hipLaunchKernelGGL(k_blk2_step, dim3(64), dim3(256), 0, s, S, T, P, k, Pt32, V32, ldv, K0, info);
}
void launch_set_mixed_info(rdist_info *info, long long uncertified, double fraction, hipStream_t s) {
    hipLaunchKernelGGL(k_set_mixed_info, dim3(1), dim3(1), 0, s, info, uncertified, fraction);
}

namespace eng {

namespace {

// Certification margin on R = log_gamma Y: an FP32 entry whose R lies
// within this of an integer is recomputed.
constexpr double kCertMargin = 0.05;

}  // namespace

rdist_status solve_mixed(rdist_ctx c, const uint8_t *A, int n, double gamma, uint32_t flags, int16_t *D,
                         rdist_info *info, hipStream_t s) {
    Workspace &w = c->ws[s];
    const int np = ((n + kMB - 1) / kMB) * kMB;
    const int nb = np / kMB;
    const double margin = kCertMargin;
    rdist_status st;
    if ((st = ensure_small(c, w, n))) return st;
    if ((st = ensure(c, w.m32, (size_t)np * np * 4))) return st;
    if ((st = ensure(c, w.v32, (size_t)kMB * np * 4))) return st;
    if ((st = ensure(c, w.u32, (size_t)kMB * np * 4))) return st;
    if ((st = ensure(c, w.s64, (size_t)2 * kMB * kMB * 8))) return st;   // the block and its step copy
    if ((st = ensure(c, w.p32, (size_t)kMB * kMB * 4))) return st;
    if ((st = ensure(c, w.Ut2, (size_t)128 * 256 * 8))) return st;
    if ((st = ensure(c, w.V2, (size_t)128 * 256 * 8))) return st;
    if ((st = ensure(c, w.Pt2, (size_t)128 * 128 * 8))) return st;
    const int nslab_all = np / kSlab;
    if ((st = ensure(c, w.cert, 256 + (size_t)nslab_all * 4))) return st;
    rdist_info *dinfo = w.dinfo();
    float *M = (float *)w.m32.p, *V = (float *)w.v32.p, *Ut = (float *)w.u32.p, *Pt = (float *)w.p32.p;
    double *S = (double *)w.s64.p, *S2 = S + (size_t)kMB * kMB;
    {
        Timer t(c, s, RDIST_K_INGEST, 0.0, (double)n * n + 4.0 * np * np);
        rd::launch_gate(A, n, gamma, w.outdeg(), w.bad(), dinfo, s);
        rd::launch_m32_build(A, n, np, M, dinfo, s);
    }
    RD_HIP(hipGetLastError());
    // (Ut on a second stream beside the block inverse, 13.5 us a step, gained
    // nothing: the two cross-stream hand-offs cost about as much.)
    for (int K = 0; K < nb; ++K) {
        const int K0 = K * kMB;
        {
            Timer t(c, s, RDIST_K_PANEL, 2.0 * kMB * kMB * kMB, 16.0 * kMB * kMB);
            // the block's inverse by two 128-pivot steps, S -> S2 -> S (the
            // panel leaves P in V2's column block k2, ld 256); the second
            // also writes P^T in FP32 to Pt and P in FP32 to V's block
            // columns.  S holds the block in FP64: converted here for the
            // first, written by the previous step's update for the others.
            if (K == 0) rd::launch_diag_to_f64(M, np, K0, S, s);
            rd::launch_panel(S, kMB, 0, (double *)w.Pt2.p, (double *)w.V2.p, kMB, dinfo, s);
            rd::launch_blk2_step(S, S2, (const double *)w.V2.p, 0, nullptr, nullptr, 0, 0, dinfo, s);
            rd::launch_panel(S2, kMB, 1, (double *)w.Pt2.p, (double *)w.V2.p, kMB, dinfo, s);
            rd::launch_blk2_step(S2, S, (const double *)w.V2.p + 128, 1, Pt, V, np, K0, dinfo, s);
        }
        RD_HIP(hipGetLastError());
        {
            Timer t(c, s, RDIST_K_ROWCOL, 2.0 * kMB * (double)kMB * np, 4.0 * (4.0 * kMB * np));
            rd::launch_gemm32_rows(Pt, M, np, K0, V, dinfo, s);        // V = P M_K,: outside V_K = P
            rd::launch_ut32(M, np, K0, Ut, dinfo, s);                  // Ut = -U^T (U_K = -I)
        }
        {
            Timer t(c, s, RDIST_K_MIXED_GEMM, 2.0 * np * (double)np * kMB, 4.0 * (2.0 * np * (double)np));
            rd::launch_gemm32_update(M, np, K0, Ut, V, S, dinfo, s);   // M <- M~ - U V; next block into S
        }
        RD_HIP(hipGetLastError());
    }
    // certification
    int32_t *slab_flag = (int32_t *)((char *)w.cert.p + 256);
    unsigned long long *cnt = (unsigned long long *)w.cert.p;
    RD_HIP(hipMemsetAsync(w.cert.p, 0, 256 + (size_t)nslab_all * 4, s));
    {
        Timer t(c, s, RDIST_K_CERTIFY, 0.0, 6.0 * n * (double)n);
        rd::launch_certify(M, np, n, margin, D, slab_flag, cnt, dinfo, s);
    }
    RD_HIP(hipGetLastError());
    std::vector<int32_t> flags_h(nslab_all);
    unsigned long long cnt_h[2] = {0, 0};
    rdist_info info_h;
    RD_HIP(hipMemcpyAsync(cnt_h, cnt, sizeof(cnt_h), hipMemcpyDeviceToHost, s));
    RD_HIP(hipMemcpyAsync(flags_h.data(), slab_flag, (size_t)nslab_all * 4, hipMemcpyDeviceToHost, s));
    RD_HIP(hipMemcpyAsync(&info_h, dinfo, sizeof(info_h), hipMemcpyDeviceToHost, s));
    RD_HIP(hipStreamSynchronize(s));
    const long long unc = (long long)cnt_h[0];
    const double frac = (double)unc / ((double)n * n);
    if (info_h.status == RDIST_OK && cnt_h[1] > 0) {
        // below the FP32 range: the FP64 plan decides every entry
        st = solve_blocked(c, A, n, gamma, flags & ~RDIST_MIXED_F32, D, nullptr, nullptr, s);
        if (st) return st;
        rd::launch_set_mixed_info(dinfo, unc, 1.0, s);
        return copy_info(info, dinfo, 1, s);
    }
    if (info_h.status == RDIST_OK && unc > 0) {
        std::vector<int32_t> slabs;
        for (int q = 0; q < nslab_all; ++q)
            if (flags_h[q]) slabs.push_back(q);
        const int ns = (int)slabs.size();
        const size_t wcols = (size_t)ns * kSlab;
        Timer t(c, s, RDIST_K_REFINE, 2.0 * np * (double)np * wcols, 4.0 * np * (double)np);
        // sparse rows of A (the residual's M X0 term)
        if ((st = ensure(c, w.csr_cnt, (size_t)(n + 1) * 8))) return st;
        rd::launch_row_count(A, n, (int32_t *)w.csr_cnt.p, s);
        std::vector<int32_t> rc(n);
        RD_HIP(hipMemcpyAsync(rc.data(), w.csr_cnt.p, (size_t)n * 4, hipMemcpyDeviceToHost, s));
        RD_HIP(hipStreamSynchronize(s));
        std::vector<int64_t> off(n + 1, 0);
        for (int i = 0; i < n; ++i) off[i + 1] = off[i] + rc[i];
        if ((st = ensure(c, w.csr_off, (size_t)(n + 1) * 8 + (size_t)ns * 4))) return st;
        if ((st = ensure(c, w.csr_col, std::max<size_t>(4, (size_t)off[n] * 4)))) return st;
        if ((st = ensure(c, w.r32, (size_t)np * wcols * 4))) return st;
        int64_t *doff = (int64_t *)w.csr_off.p;
        int32_t *dslabs = (int32_t *)((char *)w.csr_off.p + (size_t)(n + 1) * 8);
        RD_HIP(hipMemcpyAsync(doff, off.data(), (size_t)(n + 1) * 8, hipMemcpyHostToDevice, s));
        RD_HIP(hipMemcpyAsync(dslabs, slabs.data(), (size_t)ns * 4, hipMemcpyHostToDevice, s));
        rd::launch_row_fill(A, n, doff, (int32_t *)w.csr_col.p, s);
        unsigned *rmax = (unsigned *)((char *)w.cert.p + 64);     // inside the 256 B header, unused by certify
        RD_HIP(hipMemsetAsync(rmax, 0, sizeof(unsigned), s));
        rd::launch_residual(M, np, n, doff, (const int32_t *)w.csr_col.p, dslabs, ns, (float *)w.r32.p, rmax, dinfo,
                            s);
        RD_HIP(hipGetLastError());
        // C = X0 R (np x w) from the bf16 hi/lo parts of X0 and of 2^s R:
        // Xh Rh + Xh Rl + Xl Rh with FP32 accumulation (the dropped parts
        // are about 2^-16 of C, and C is about eps32 Y); both operands' parts
        // interleaved per 32 k, R's transposed
        // (the correction's columns are padded to its 256-wide tiles)
        const int wpad = rd::corr_cols((int)wcols);
        const size_t nx = (size_t)np * np, nr = (size_t)np * wpad;
        if ((st = ensure(c, w.xi, nx * 4)) || (st = ensure(c, w.ri, nr * 4)) || (st = ensure(c, w.c32, nr * 4)))
            return st;
        rd::launch_split_bf16_x(M, np, np, (uint16_t *)w.xi.p, s);
        rd::launch_split_bf16_t((const float *)w.r32.p, np, (int)wcols, wpad, (uint16_t *)w.ri.p, rmax, s);
        rd::launch_corr_bf16((float *)w.c32.p, np, wpad, np, (const uint16_t *)w.xi.p, (const uint16_t *)w.ri.p,
                             dinfo, s);
        RD_HIP(hipGetLastError());
        rd::launch_fix(M, np, n, (const float *)w.c32.p, wpad, dslabs, ns, margin, rmax, D, dinfo, s);
        RD_HIP(hipGetLastError());
        // keep the host vectors alive until the copies above have run
        RD_HIP(hipStreamSynchronize(s));
    }
    rd::launch_set_mixed_info(dinfo, unc, frac, s);
    rd::launch_fill_sentinel(D, n, dinfo, s);
    RD_HIP(hipGetLastError());
    return copy_info(info, dinfo, 1, s);
}

}  // namespace eng
}  // namespace rd
