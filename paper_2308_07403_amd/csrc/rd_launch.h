// rd_launch.h -- host-side launchers of the gfx950 kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/rdist.h"

namespace rd {

// One graph for the single-workgroup solver (n <= 128).
struct SmallTask {
    const uint8_t *A;      // n x n adjacency
    int16_t *D;            // n x n distances
    double *Y;             // nullable: n x ldy inverse
    int32_t n;
    int32_t ldy;
    double gamma_arg;      // explicit (> 0) or AUTO (< 0)
    rdist_info *info;      // device
};

// One graph of a batched solve (n <= 512).  M: np x np workspace (np = n
// rounded up to 128; for n <= 128 it receives Y with ld np when keep is set).
// Ut, V, Pt: the solving workgroup's scratch, filled in by the kernel.
struct BatchTask {
    const uint8_t *A;
    int16_t *D;
    double *M;
    double *Ut, *V, *Pt;
    int32_t n;
    int32_t np;
    int32_t keep;
    int32_t pad;
    double gamma_arg;
    rdist_info *info;
};

// One graph of the level-synchronous batched solver (n <= kLvMaxN).
// M: np x np (np = n rounded up to 128, nt = np / 128 tiles per side).
// Step buffers by step parity: Ut, V 128 x np; Pt 128 x 128.
// colsum: int32 [n + 1], zeroed before the plan: the column sums of A
// (out-degrees), then the validation flag (an entry not 0/1, or a
// self-loop); the column sums are taken over nchunk row chunks of rows_per.
// gamma_arg explicit (> 0) or AUTO (< 0).
struct LevelGraph {
    const uint8_t *A;
    int16_t *D;
    double *M;
    double *Ut[2], *V[2], *Pt[2];
    rdist_info *info;
    int32_t *colsum;
    int32_t n, np, nt, keep;
    int32_t rows_per, nchunk;
    double gamma_arg;
};
constexpr int kLvMaxN = 4096;  // largest graph of the level plan
constexpr int kLvShift = 10;   // unit = (graph << 10) | item, item < 1024 (nt^2 <= 1024)
// Launch phases of the level plan (Diag, Edge and Rest are update tile sets).
enum LevelPhase { kLvBuild = 0, kLvPanel = 1, kLvRowcol = 2, kLvEdge = 3, kLvRest = 4, kLvColsum = 5, kLvDiag = 6 };
// Rows of the last block of a graph that hold pivots (n - 128 (nt - 1)),
// rounded up to the contraction's k-chunk of 16: the inner dimension of the
// last step's products (the block's padding rows and columns are an
// identity, which contributes nothing to any other tile).
__host__ __device__ inline int lv_last_inner(int n, int nt) { return ((n - 128 * (nt - 1) + 15) / 16) * 16; }

// Out-degrees, validation and the gate: info (status, delta, gamma, zeroed counters).
// weighted: A holds integer weights (0 = no edge); out-degrees count edges and
// only self-loops are invalid.
void launch_gate(const uint8_t *A, int n, double gamma_arg, int32_t *outdeg, int32_t *bad, rdist_info *info,
                 hipStream_t s, bool weighted = false);
// ... then M = I - gamma A (weighted: I - gamma^W elementwise).
void launch_ingest(const uint8_t *A, int n, int np, int ld, double gamma_arg, double *M, int32_t *outdeg,
                   int32_t *bad, rdist_info *info, hipStream_t s, bool weighted = false);
void launch_fill_sentinel(int16_t *D, int n, const rdist_info *info, hipStream_t s);
void launch_panel(const double *M, int ld, int K, double *Pt, double *V, int ldv, rdist_info *info, hipStream_t s);
// Blocked Gauss-Jordan pieces (tiles are 128 x 128; a block is m tiles wide,
// starting at tile K0; nt tiles per side).
enum UpdateMode { kUpdateAll = 0, kUpdateDiag = 1, kUpdateRest = 2, kUpdateEdgeRest = 3 };
int update_tiles(int mode, int nt, int m, int wt);
void launch_rowcol(const double *M, int ld, int nt, int K0, int m, const double *Pt, double *Ut, double *V,
                   int ldv, const rdist_info *info, hipStream_t s);
// wt: width in tiles of the band [L0, L0 + wt) of EDGEREST / REST (>= m).
void launch_update(int mode, double *M, int ld, int nt, int K0, int m, int L0, int wt, const double *Ut,
                   const double *V, int ldv, bool fused, int n, int16_t *D, int keep_y, rdist_info *info,
                   hipStream_t s);
void launch_panel_finish(const double *S, int lds, int b, int K0, double *Pt, double *V, int ldv,
                         const rdist_info *info, hipStream_t s);
void launch_epilogue(const double *Y, int n, int ld, int16_t *D, rdist_info *info, hipStream_t s);
void launch_info_set(rdist_info *info, double gamma, hipStream_t s);
void launch_small_one(const SmallTask &t, hipStream_t s);
void launch_batched(const BatchTask *tasks, int count, int *counter, int grid, double *scratch, int scratch_stride,
                    hipStream_t s);
int batched_blocks_per_cu();
void launch_fill_i32(int32_t *p, size_t count, hipStream_t s);   // p[0, count) = 0
void launch_lv_gate(const LevelGraph *gs, int count, hipStream_t s);
void launch_lv(int phase, const LevelGraph *gs, const int *units, int grid, int K, hipStream_t s);
// Mixed precision (rd_mixed.hip).
void launch_m32_build(const uint8_t *A, int n, int np, float *M, const rdist_info *info, hipStream_t s);
void launch_diag_to_f64(const float *M, int np, int K0, double *S, hipStream_t s);
void launch_certify(const float *X, int np, int n, double margin, int16_t *D, int32_t *slab_flag,
                    unsigned long long *cnt, rdist_info *info, hipStream_t s);
void launch_row_count(const uint8_t *A, int n, int32_t *cnt, hipStream_t s);
void launch_row_fill(const uint8_t *A, int n, const int64_t *off, int32_t *cols, hipStream_t s);
// rmax: device unsigned, zeroed by the caller; receives the bits of max |R|.
void launch_residual(const float *X, int np, int n, const int64_t *off, const int32_t *cols, const int32_t *slabs,
                     int nslab, float *R, unsigned *rmax, const rdist_info *info, hipStream_t s);
// C: the correction X0 R of the slabs (np x ldc, column 128 s + c of slab s);
// rmax as written by launch_residual (C formed from the residual scaled by
// 2^s, undone here).
void launch_fix(const float *X, int np, int n, const float *C, int ldc, const int32_t *slabs, int nslab,
                double margin, const unsigned *rmax, int16_t *D, rdist_info *info, hipStream_t s);
// FP32 matrix-core steps of the mixed plan (rd_gemm.hip), step width 256:
// Ut = -U^T; V = P M_K,: (Pt = P^T in FP32, 256 x 256) outside V's block
// columns at K0 (written with P by the block inverse); M <- M~ - U V over
// every tile, with the next block's diagonal (when there is one) also
// written to Snext in FP64 (256 x 256).
void launch_ut32(const float *M, int np, int K0, float *Ut, const rdist_info *info, hipStream_t s);
void launch_gemm32_rows(const float *Pt, const float *M, int np, int K0, float *V, const rdist_info *info,
                        hipStream_t s);
void launch_gemm32_update(float *M, int np, int K0, const float *Ut, const float *V, double *Snext,
                          const rdist_info *info, hipStream_t s);
// The bf16 operands of the correction: row r of an interleaved operand holds,
// per block of 32 k-values, their 32 hi parts and then their 32 lo parts
// (16-bit patterns, row length 2K).
// C (rows x cols_pad, ld cols_pad) = Xh Rh + Xh Rl + Xl Rh: Xi rows x 2K
// (rows of X), Ri cols_pad x 2K (columns of R, zero rows past its columns);
// rows a multiple of 256, cols_pad = corr_cols(cols), K a multiple of 32.
int corr_cols(int cols);
void launch_corr_bf16(float *C, int rows, int cols_pad, int K, const uint16_t *Xi, const uint16_t *Ri,
                      const rdist_info *info, hipStream_t s);
// Xi = the interleaved hi / lo parts of X (rows x cols, row-major; cols a
// multiple of 32).
void launch_split_bf16_x(const float *X, int rows, int cols, uint16_t *Xi, hipStream_t s);
// Ri = the interleaved hi / lo parts of 2^s R (rows x cols, s from rmax),
// transposed (cols_pad x 2 rows, the rows past cols zero); rows a multiple of
// 64, cols_pad a multiple of 64 not below cols.
void launch_split_bf16_t(const float *R, int rows, int cols, int cols_pad, uint16_t *Ri, const unsigned *rmax,
                         hipStream_t s);
// One 128-pivot step of a 256 x 256 block inverse (ld 256): T from S and
// P = S_kk^{-1} (ld 256), pivot tile k of the 2 x 2 tiles; with Pt32 given,
// also Pt32 = T^T (FP32, ld 256) and V32's columns K0 .. K0 + 255 = T (FP32,
// ld ldv).
void launch_blk2_step(const double *S, double *T, const double *P, int k, float *Pt32, float *V32, int ldv, int K0,
                      const rdist_info *info, hipStream_t s);
void launch_set_mixed_info(rdist_info *info, long long uncertified, double fraction, hipStream_t s);
// The lookahead chain's products for 128-wide blocks (rd_chain.hip), as four
// 64 x 64 workgroups each: the DIAG update of tile (L0, L0), and the row and
// column tiles of step K (as launch_rowcol with m = 1).
void launch_diag64(double *M, int ld, int L0, const double *Ut, const double *V, int ldv, const rdist_info *info,
                   hipStream_t s);
void launch_rowcol64(const double *M, int ld, int nt, int K, const double *Pt, double *Ut, double *V, int ldv,
                     const rdist_info *info, hipStream_t s);
// Entries per query of a path output: the next node alone for max_hops = 1,
// else the start and max_hops hops.
__host__ __device__ inline int path_row_len(int max_hops) { return max_hops == 1 ? 1 : max_hops + 1; }
// Path requests of a batch (the request loop), one task per graph with q > 0
// queries; blk0 and q0 are the prefix sums of path_task_blocks(n) and of q
// over the tasks before it.
struct PathTask {
    const uint8_t *A;            // n x n adjacency (device)
    const double *Y;             // Y with leading dimension ld (device)
    unsigned long long *bits;    // n x ceil(n/64) successor bitmap, written by launch_paths_multi
    const int32_t *cur, *goal;   // q start and goal nodes (device)
    int32_t *out;                // q x path_row_len(max_hops), as rdist_next_hop's out
    int32_t n, ld, q, max_hops;
    int32_t blk0, q0;
};
int path_task_blocks(int n);
// Bitmaps then paths of every task (tasks: device copy of the table).
void launch_paths_multi(const PathTask *tasks, int ntasks, int total_blocks, int total_q, hipStream_t s);
void launch_succ_bitmap(const uint8_t *A, int n, unsigned long long *bits, hipStream_t s);
// Edge changes of a kept graph (rd_dynamic.hip).
void launch_outdeg_from_bits(const unsigned long long *bits, int n, int32_t *outdeg, hipStream_t s);
// Up to kMaxBatch edge changes applied in one pass (rd_dynamic.hip).
constexpr int kMaxBatch = 8;
// The largest relative error bound an entry of a changed Y keeps: an entry
// whose bound grows beyond it counts as lost and the graph is re-inverted.
constexpr double kBetaCap = 0x1p-20;
struct EdgeBatch {
    int k;
    int src[kMaxBatch], dst[kMaxBatch], w[kMaxBatch];
};
size_t batch_scratch_doubles(int n);
void launch_edge_batch_prep(const double *Y, int ld, int n, const uint16_t *Q, double *sm, double *bs,
                            const uint8_t *A, const int32_t *outdeg, const rdist_info *ginfo, const EdgeBatch &B,
                            hipStream_t s);
void launch_edge_batch_apply(double *Y, int ld, int n, uint16_t *Q, double *sm, const double *bs, int16_t *D,
                             uint8_t *A, int32_t *outdeg, int32_t *hist, unsigned long long *bits, rdist_info *ginfo,
                             const EdgeBatch &B, hipStream_t s);
// Q: per-entry error bounds (n x n, 16-bit -log2 in 1/256 steps); sm: the
// update's scratch (16 + 3n doubles) holding the call's info at sm + 2.
// hist: n + 1 counts of nodes per out-degree.
void launch_beta_fill(uint16_t *Q, int n, const rdist_info *ginfo, hipStream_t s);
void launch_deg_hist(const int32_t *outdeg, int n, int32_t *hist, hipStream_t s);
void launch_edge_prep(const double *Y, int ld, int n, const uint8_t *A, const int32_t *outdeg, const int32_t *hist,
                      const uint16_t *Q, const rdist_info *ginfo, double *sm, int src, int dst, int weight,
                      hipStream_t s);
void launch_edge_apply(double *Y, int ld, int n, uint16_t *Q, double *sm, int16_t *D, uint8_t *A, int32_t *outdeg,
                       int32_t *hist, unsigned long long *bits, rdist_info *ginfo, int src, int dst, int weight,
                       hipStream_t s);
// Goal rows without an inversion (rd_rows.hip): successor lists in CSR,
// optional per-edge weights, q goals.
struct RowsLaunch {
    const int64_t *ptr;
    const int32_t *idx;
    const uint8_t *wts;      // nullable: unit weights
    const double *gpow;      // gamma^w table (256 entries)
    int n;
    int64_t nnz;
    const int32_t *goals;
    int q;
    const rdist_info *info;
};
int rows_group(int q);   // goals per chunk: the power of two >= q, at most 64
void launch_rows_check(const int64_t *ptr, const int32_t *idx, const uint8_t *wts, int n, int64_t nnz,
                       double gamma, rdist_info *info, int32_t *bad, double *gpow, hipStream_t s);
void launch_rows_step(const RowsLaunch &L, const double *Vo, double *Vn, int32_t *flag, hipStream_t s);
void launch_rows_out(const double *V, int n, int q, double *Y, int16_t *D, rdist_info *info, hipStream_t s);
void launch_rows_paths(const int64_t *ptr, const int32_t *idx, int n, int64_t nnz, const double *Y,
                       const int32_t *goals, const int32_t *starts, int q, int max_hops, int32_t *out, hipStream_t s);
// Gain bounds and the per-entry certificate (rd_gamma.hip).
size_t power_scratch_bytes();
void launch_power_init(void *scratch, hipStream_t s);
void launch_power_step(const uint8_t *A, int n, const double *x, double *y, void *scratch, int step, hipStream_t s);
void launch_power_fold(void *scratch, int last_step, hipStream_t s);
void power_read(const void *host_copy, double *lo_ratio, double *hi_ratio);
void launch_certify(const double *Y, int ld, int n, const rdist_info *ginfo, bool weighted, double err_floor,
                    uint8_t *mask, unsigned long long *count, hipStream_t s);
void launch_next_hop(const double *Y, int ld, int n, const unsigned long long *bits, const int32_t *cur,
                     const int32_t *goal, int q, int max_hops, int32_t *out, hipStream_t s);

}  // namespace rd
