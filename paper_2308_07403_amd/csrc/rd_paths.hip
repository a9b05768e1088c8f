// rd_paths.hip -- the greedy next hop (Sec. 4.2, Eq. descent read as ascent
// on Y, Theorem 4): successor bitmaps of a graph and the path walks, one
// wavefront per (start, goal) query; single-graph launches for
// rdist_next_hop and task-table launches that serve every path request of a
// batch at once (the request loop).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rd_launch.h"

namespace rd {

// Successor bitmaps: bit b of word w in row i is set iff there is an edge
// i -> 64w + b, i.e. A[(64w + b) * n + i] != 0 (any weight).  Row i is nw = ceil(n/64)
// 64-bit words; its size is known up front, so no host synchronisation is
// needed to allocate it.  Thread i of the word-w pass reads column i of 64
// rows (consecutive i read consecutive bytes of a row).
__device__ __forceinline__ void succ_word(const uint8_t *__restrict__ A, int n, int nw, int i, int w,
                                          unsigned long long *__restrict__ bits) {
    unsigned long long word = 0;
    const int j0 = w * 64;
    const int j1 = min(n, j0 + 64);
    for (int j = j0; j < j1; ++j)
        if (A[(size_t)j * n + i] != 0) word |= 1ull << (j - j0);
    bits[(size_t)i * nw + w] = word;
}

// One query on one wavefront: from c0, repeatedly move to the successor j
// with the largest Y[goal][j] (lowest j among exact ties) until the goal,
// a node without a successor of positive Y, or max_hops.  Path form
// (max_hops > 1): o holds max_hops + 1 entries, the start first and -1 past
// the end of the path; an out-of-range start or goal leaves the row -1.
// Single-hop form (max_hops == 1): o[0] is the next node, the start itself
// when it is the goal, -1 when no successor has positive Y or an id is out
// of range.
__device__ __forceinline__ void next_hop_wave(const double *__restrict__ Y, int ld, int n,
                                              const unsigned long long *__restrict__ bits, int nw, int c, int g,
                                              int max_hops, int32_t *__restrict__ o) {
    const int lane = threadIdx.x & 63;
    const int sh = max_hops == 1 ? 1 : 0;   // hop h goes to o[h - sh]
    for (int h = lane; h < path_row_len(max_hops); h += 64) o[h] = -1;
    if (c < 0 || c >= n || g < 0 || g >= n) return;
    if (lane == 0) o[0] = c;   // the start; in the single-hop form replaced by hop 1 unless c is the goal
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
            if (lane == 0) o[h - sh] = -1;
            break;
        }
        c = bj;
        if (lane == 0) o[h - sh] = c;
    }
}

__global__ __launch_bounds__(256) void k_succ_bitmap(const uint8_t *__restrict__ A, int n, int nw,
                                                     unsigned long long *__restrict__ bits) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) succ_word(A, n, nw, i, blockIdx.y, bits);
}

__global__ __launch_bounds__(256) void k_next_hop(const double *__restrict__ Y, int ld, int n,
                                                  const unsigned long long *__restrict__ bits, int nw,
                                                  const int32_t *__restrict__ cur, const int32_t *__restrict__ goal,
                                                  int q, int max_hops, int32_t *__restrict__ out) {
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= q) return;
    next_hop_wave(Y, ld, n, bits, nw, cur[w], goal[w], max_hops, out + (size_t)w * path_row_len(max_hops));
}

// The task whose range [key_of(t), key_of(t + 1)) holds key: the last task
// with key_of <= key (tasks in increasing key order, ntasks >= 1).
template <bool BY_QUERY>
__device__ __forceinline__ int find_task(const PathTask *__restrict__ t, int ntasks, int key) {
    int lo = 0, hi = ntasks - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int k = BY_QUERY ? t[mid].q0 : t[mid].blk0;
        if (k <= key) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Bitmaps of every task: workgroup b belongs to the task whose blk0 range
// holds it; within the task it is pass (w, i-block) as k_succ_bitmap.
__global__ __launch_bounds__(256) void k_succ_bitmap_multi(const PathTask *__restrict__ tasks, int ntasks) {
    const int k = find_task<false>(tasks, ntasks, blockIdx.x);
    const PathTask t = tasks[k];
    const int local = blockIdx.x - t.blk0;
    const int nb = (t.n + 255) / 256, nw = (t.n + 63) / 64;
    const int w = local / nb, ib = local - (local / nb) * nb;
    const int i = ib * 256 + threadIdx.x;
    if (w < nw && i < t.n) succ_word(t.A, t.n, nw, i, w, t.bits);
}

// Queries of every task: wavefront gw is query gw - q0 of the task whose
// range holds it.
__global__ __launch_bounds__(256) void k_next_hop_multi(const PathTask *__restrict__ tasks, int ntasks, int total_q) {
    const int gw = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (gw >= total_q) return;
    const PathTask t = tasks[find_task<true>(tasks, ntasks, gw)];
    const int w = gw - t.q0;
    next_hop_wave(t.Y, t.ld, t.n, t.bits, (t.n + 63) / 64, t.cur[w], t.goal[w], t.max_hops,
                  t.out + (size_t)w * path_row_len(t.max_hops));
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

int path_task_blocks(int n) { return ((n + 255) / 256) * ((n + 63) / 64); }

void launch_paths_multi(const PathTask *tasks, int ntasks, int total_blocks, int total_q, hipStream_t s) {
    if (ntasks <= 0 || total_q <= 0) return;
    hipLaunchKernelGGL(k_succ_bitmap_multi, dim3(total_blocks), dim3(256), 0, s, tasks, ntasks);
    hipLaunchKernelGGL(k_next_hop_multi, dim3((total_q + 3) / 4), dim3(256), 0, s, tasks, ntasks, total_q);
}

}  // namespace rd
