// rd_rows.hip -- goal rows of Y without an inversion.
//
// Row g of Y = (I - X)^{-1} is the fixed point of
//   y_j = [j == g] + sum_{i in succ(j)} x_ij y_i        (x_ij = gamma^w of edge j -> i)
// i.e. y^T (I - X) = e_g^T: the recurrent network of Sec. 2 run on the
// reversed edges with the drive at the goal (each node adds its successors'
// outputs).  The walk series (Eq. Y-series) is its Jacobi iteration from
// y = 0: after k steps y holds every walk of length < k.  The gate
// gamma Delta < 1 makes the step a contraction in the max norm.
//
// Every coefficient is non-negative and rounding is monotone, so the
// iterates never decrease, also in floating point, and reach a floating-point
// fixed point after finitely many steps; the iteration stops at the first
// checked step that changes no entry.
//
// Layout: q goals in chunks of G (one chunk per grid row); the state of a
// chunk is node-major, V[j][g] (G doubles per node), so a successor's values
// for all G goals are one contiguous read.  Three step kernels: 64 goals
// with a batch of nodes per wavefront (lane = goal); 2 .. 32 goals on sparse
// graphs with one node per lane; otherwise a wavefront's 64 lanes as
// (N nodes) x (S successor slots) x (G goals), N = 64 / (G S), the S partial
// sums of a node combined by lane shuffles.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rd_device.h"
#include "rd_launch.h"

namespace rd {

namespace {

// One block per 256 nodes: successor lists checked (ids in range, no
// self-loop, strictly increasing, weights non-zero), out-degree maxima into
// info->delta, bad input into *bad.
__global__ __launch_bounds__(256) void k_rows_check(const int64_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                                                    const uint8_t *__restrict__ wts, int n, int64_t nnz,
                                                    rdist_info *__restrict__ info, int32_t *__restrict__ bad) {
    __shared__ int smax;
    if (threadIdx.x == 0) smax = 0;
    __syncthreads();
    const int j = blockIdx.x * 256 + threadIdx.x;
    int deg = 0;
    bool ok = true;
    if (j < n) {
        const int64_t e0 = ptr[j], e1 = ptr[j + 1];
        ok = e0 >= 0 && e1 >= e0 && e1 <= nnz && (j > 0 || e0 == 0) && (j < n - 1 || e1 == nnz);
        if (ok) {
            deg = (int)min<int64_t>(e1 - e0, 0x7FFFFFFF);
            int prev = -1;
            for (int64_t e = e0; e < e1; ++e) {
                const int i = idx[e];
                ok = ok && i >= 0 && i < n && i != j && i > prev && (!wts || wts[e] != 0);
                prev = i;
            }
        }
        atomicMax(&smax, deg);
    }
    if (!ok) atomicOr(bad, 1);
    __syncthreads();
    if (threadIdx.x == 0) atomicMax(&info->delta, smax);
}

// Gain, gate and the table of gamma^w (weighted graphs).
__global__ void k_rows_gate(double gamma_arg, const int32_t *__restrict__ bad, rdist_info *__restrict__ info,
                            double *__restrict__ gpow) {
    const int d = info->delta;
    const double gamma = gamma_arg > 0.0 ? gamma_arg : (d > 0 ? -gamma_arg / (double)d : -gamma_arg);
    if (threadIdx.x == 0) {
        info->gamma = gamma;
        info->status = *bad ? RDIST_E_ADJ : (gamma * (double)d < 1.0 ? RDIST_OK : RDIST_E_NOT_DD);
    }
    gpow[threadIdx.x] = threadIdx.x ? pow(gamma, (double)threadIdx.x) : 0.0;
}

// One Jacobi step for every node and goal.  flag (nullable): set when any
// entry changed.
template <int G, int S>
__global__ __launch_bounds__(256) void k_rows_step(const int64_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                                                   const uint8_t *__restrict__ wts, const double *__restrict__ gpow,
                                                   int n, const int32_t *__restrict__ goals, int q,
                                                   const double *__restrict__ Vold, double *__restrict__ Vnew,
                                                   const rdist_info *__restrict__ info, int32_t *__restrict__ flag) {
    constexpr int N = 64 / (G * S);
    if (info->status != RDIST_OK) return;
    const double gamma = info->gamma;
    const int lane = threadIdx.x & 63;
    const int g = lane % G;
    const int s = (lane / G) % S;
    const int nd = lane / (G * S);
    // workgroup b runs on XCD b % 8: each XCD takes a contiguous range of
    // nodes, so neighbouring nodes' states stay in that XCD's L2
    const int per = gridDim.x / 8;
    const int blk = (blockIdx.x % 8) * per + blockIdx.x / 8;
    const int j = (blk * 4 + (int)(threadIdx.x >> 6)) * N + nd;
    const size_t base = (size_t)blockIdx.y * n * G;
    const double *__restrict__ Vo = Vold + base;
    double acc = 0.0;
    if (j < n) {
        const int64_t e1 = ptr[j + 1];
        if (wts) {
            for (int64_t e = ptr[j] + s; e < e1; e += S) acc = fma(gpow[wts[e]], Vo[(size_t)idx[e] * G + g], acc);
        } else {
#pragma unroll 4
            for (int64_t e = ptr[j] + s; e < e1; e += S) acc += Vo[(size_t)idx[e] * G + g];
        }
    }
#pragma unroll
    for (int m = 1; m < S; m <<= 1) acc += __shfl_xor(acc, G * m);
    bool changed = false;
    if (j < n && s == 0) {
        const int k = blockIdx.y * G + g;
        const double seed = (k < q && goals[k] == j) ? 1.0 : 0.0;
        const double v = wts ? seed + acc : fma(gamma, acc, seed);
        Vnew[base + (size_t)j * G + g] = v;
        changed = v != Vo[(size_t)j * G + g];
    }
    if (flag && __any(changed) && lane == 0) *flag = 1;
}

// The step for chunks of 64 goals, NB consecutive nodes per wavefront
// (lane = goal): one load brings the batch's successor offsets, one the
// successor ids of up to 64 of its edges, and the gathers of 16 edges (8
// for batches under 8 nodes, which keep more wavefronts resident) are in
// flight together, so the wavefront waits for three memory latencies per
// batch rather than per node.  Sums run in edge order, as in k_rows_step.
template <int NB>
__global__ __launch_bounds__(256) void k_rows_step64(const int64_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                                                     const uint8_t *__restrict__ wts, const double *__restrict__ gpow,
                                                     int n, const int32_t *__restrict__ goals, int q,
                                                     const double *__restrict__ Vold, double *__restrict__ Vnew,
                                                     const rdist_info *__restrict__ info, int32_t *__restrict__ flag) {
    constexpr int kInFlight = NB >= 8 ? 16 : 8;
    if (info->status != RDIST_OK) return;
    const double gamma = info->gamma;
    const int lane = threadIdx.x & 63;
    const int per = gridDim.x / 8;
    const int blk = (blockIdx.x % 8) * per + blockIdx.x / 8;   // contiguous node ranges per XCD
    const int j0 = (blk * 4 + (int)(threadIdx.x >> 6)) * NB;
    if (j0 >= n) return;                                       // whole wavefront
    const int nb = min(NB, n - j0);
    const size_t base = (size_t)blockIdx.y * n * 64;
    const double *__restrict__ Vo = Vold + base;
    double *__restrict__ Vn = Vnew + base;
    const int k = blockIdx.y * 64 + lane;
    const int goal = k < q ? goals[k] : -1;
    const long long pl = lane <= nb ? (long long)ptr[j0 + lane] : 0;
    const long long E0 = __shfl(pl, 0), E1 = __shfl(pl, nb);
    int node = 0;
    long long bound = __shfl(pl, 1);
    double acc = 0.0;
    bool changed = false;
    auto finish = [&]() {
        const int j = j0 + node;
        const double seed = goal == j ? 1.0 : 0.0;
        const double v = wts ? seed + acc : fma(gamma, acc, seed);
        Vn[(size_t)j * 64 + lane] = v;
        if (flag) changed |= v != Vo[(size_t)j * 64 + lane];
        ++node;
        acc = 0.0;
        bound = __shfl(pl, min(node + 1, nb));
    };
    for (long long c0 = E0; c0 < E1; c0 += 64) {
        const int cnt = (int)min<long long>(64, E1 - c0);
        const int myi = lane < cnt ? idx[c0 + lane] : 0;
        const double myx = (wts && lane < cnt) ? gpow[wts[c0 + lane]] : 1.0;
        for (int k0 = 0; k0 < cnt; k0 += kInFlight) {
            double v[kInFlight];
#pragma unroll
            for (int u = 0; u < kInFlight; ++u) {
                const int i = __shfl(myi, min(k0 + u, 63));
                v[u] = k0 + u < cnt ? Vo[(size_t)i * 64 + lane] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kInFlight; ++u) {
                if (k0 + u >= cnt) break;
                while (c0 + k0 + u >= bound) finish();
                if (wts) acc = fma(__shfl(myx, k0 + u), v[u], acc);
                else acc += v[u];
            }
        }
    }
    while (node < nb) finish();
    if (flag && __any(changed) && lane == 0) *flag = 1;
}

// The step for chunks of 2 .. 32 goals, one node per lane: the lane keeps its
// node's G sums in registers and reads each successor's G values as one
// contiguous G x 8 bytes (whole cache lines from G = 16 on); 64 consecutive
// nodes per wavefront, contiguous node ranges per XCD.  Sums run in edge
// order.
template <int G>
__global__ __launch_bounds__(256) void k_rows_step_lane(const int64_t *__restrict__ ptr,
                                                        const int32_t *__restrict__ idx,
                                                        const uint8_t *__restrict__ wts,
                                                        const double *__restrict__ gpow, int n,
                                                        const int32_t *__restrict__ goals, int q,
                                                        const double *__restrict__ Vold, double *__restrict__ Vnew,
                                                        const rdist_info *__restrict__ info,
                                                        int32_t *__restrict__ flag) {
    if (info->status != RDIST_OK) return;
    const double gamma = info->gamma;
    const int per = gridDim.x / 8;
    const int blk = (blockIdx.x % 8) * per + blockIdx.x / 8;
    const int j = blk * 256 + (int)threadIdx.x;
    const size_t base = (size_t)blockIdx.y * n * G;
    const double *__restrict__ Vo = Vold + base;
    bool changed = false;
    if (j < n) {
        double acc[G];
#pragma unroll
        for (int g = 0; g < G; ++g) acc[g] = 0.0;
        const int64_t e1 = ptr[j + 1];
        for (int64_t e = ptr[j]; e < e1; ++e) {
            const double *__restrict__ src = Vo + (size_t)idx[e] * G;
            const double x = wts ? gpow[wts[e]] : 1.0;
#pragma unroll
            for (int g = 0; g < G; g += 2) {
                const double2 v = *reinterpret_cast<const double2 *>(src + g);
                if (wts) {
                    acc[g] = fma(x, v.x, acc[g]);
                    acc[g + 1] = fma(x, v.y, acc[g + 1]);
                } else {
                    acc[g] += v.x;
                    acc[g + 1] += v.y;
                }
            }
        }
        const double *__restrict__ own = Vo + (size_t)j * G;
        double *__restrict__ out = Vnew + base + (size_t)j * G;
#pragma unroll
        for (int g = 0; g < G; g += 2) {
            double v2[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int k = blockIdx.y * G + g + h;
                const double seed = (k < q && goals[k] == j) ? 1.0 : 0.0;
                v2[h] = wts ? seed + acc[g + h] : fma(gamma, acc[g + h], seed);
            }
            if (flag) {
                const double2 o = *reinterpret_cast<const double2 *>(own + g);
                changed = changed || v2[0] != o.x || v2[1] != o.y;
            }
            *reinterpret_cast<double2 *>(out + g) = make_double2(v2[0], v2[1]);
        }
    }
    if (flag && __any(changed) && (threadIdx.x & 63) == 0) *flag = 1;
}

// Rows out: Y[k * n + j] and the readout D[k * n + j] (either nullable);
// status not OK: Y = 0 and D = the sentinel.
template <int G>
__global__ __launch_bounds__(256) void k_rows_out(const double *__restrict__ V, int n, int q, double *__restrict__ Y,
                                                  int16_t *__restrict__ D, rdist_info *__restrict__ info) {
    const bool ok = info->status == RDIST_OK;
    const double il = ok ? rd_inv_log(info->gamma) : 0.0;
    Counts cnt;
    const int k = blockIdx.y;
    const int c = k / G, g = k % G;
    for (int j = blockIdx.x * 256 + threadIdx.x; j < n; j += gridDim.x * 256) {
        const double v = ok ? V[((size_t)c * n + j) * G + g] : 0.0;
        if (Y) Y[(size_t)k * n + j] = v;
        if (D) D[(size_t)k * n + j] = ok ? rd_encode(v, il, cnt) : kUnreachable;
    }
    if (ok && D) flush_counts(info, cnt);
}

// Greedy paths over the rows: query k walks from start[k] toward goals[k]
// on row k, each hop to the successor with the largest row value (lowest
// id on ties); layout and ending as rdist_next_hop.  One wavefront per query;
// offsets are clamped to [0, nnz) and ids outside [0, n) skipped.
__global__ __launch_bounds__(256) void k_rows_paths(const int64_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                                                    int n, int64_t nnz, const double *__restrict__ Y,
                                                    const int32_t *__restrict__ goals,
                                                    const int32_t *__restrict__ starts, int q, int max_hops,
                                                    int32_t *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int k = (blockIdx.x * 256 + threadIdx.x) >> 6;
    if (k >= q) return;
    const int sh = max_hops == 1 ? 1 : 0;   // hop h goes to o[h - sh]
    int32_t *o = out + (size_t)k * path_row_len(max_hops);
    const int goal = goals[k];
    int cur = starts[k];
    const bool valid = cur >= 0 && cur < n && goal >= 0 && goal < n;
    if (lane == 0) o[0] = valid ? cur : -1;   // single-hop form: replaced by hop 1 unless cur is the goal
    const double *__restrict__ row = Y + (size_t)k * n;
    for (int h = 1; h <= max_hops; ++h) {
        if (!valid || cur < 0 || cur == goal) {
            for (int t = h + lane; t <= max_hops && !sh; t += 64) o[t] = -1;
            break;
        }
        double best = 0.0;
        int bj = 0x7FFFFFFF;
        const int64_t e0 = max<int64_t>(ptr[cur], 0), e1 = min<int64_t>(ptr[cur + 1], nnz);
        for (int64_t e = e0 + lane; e < e1; e += 64) {
            const int i = idx[e];
            if (i < 0 || i >= n) continue;
            const double v = row[i];
            if (v > best || (v == best && v > 0.0 && i < bj)) { best = v; bj = i; }
        }
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            const double ob = __shfl_xor(best, m);
            const int oj = __shfl_xor(bj, m);
            if (ob > best || (ob == best && oj < bj)) { best = ob; bj = oj; }
        }
        cur = best > 0.0 ? bj : -1;
        if (lane == 0) o[h - sh] = cur;
    }
}

template <int G, int S>
void step_gs(const RowsLaunch &L, const double *Vo, double *Vn, int32_t *flag, hipStream_t s) {
    constexpr int N = 64 / (G * S);
    const int waves = (L.n + N - 1) / N;
    const int blocks = (waves + 3) / 4;
    const dim3 grid(((blocks + 7) / 8) * 8, (L.q + G - 1) / G);   // a multiple of the 8 XCDs
    hipLaunchKernelGGL((k_rows_step<G, S>), grid, dim3(256), 0, s, L.ptr, L.idx, L.wts, L.wts ? L.gpow : nullptr,
                       L.n, L.goals, L.q, Vo, Vn, L.info, flag);
}

template <int G>
void step_g(int log_s, const RowsLaunch &L, const double *Vo, double *Vn, int32_t *flag, hipStream_t s) {
    switch (log_s) {
        case 0: step_gs<G, 1>(L, Vo, Vn, flag, s); break;
        case 1: if constexpr (G <= 32) step_gs<G, 2>(L, Vo, Vn, flag, s); break;
        case 2: if constexpr (G <= 16) step_gs<G, 4>(L, Vo, Vn, flag, s); break;
        case 3: if constexpr (G <= 8) step_gs<G, 8>(L, Vo, Vn, flag, s); break;
        case 4: if constexpr (G <= 4) step_gs<G, 16>(L, Vo, Vn, flag, s); break;
        case 5: if constexpr (G <= 2) step_gs<G, 32>(L, Vo, Vn, flag, s); break;
        default: if constexpr (G <= 1) step_gs<G, 64>(L, Vo, Vn, flag, s); break;
    }
}

int ilog2(int x) {
    int l = 0;
    while ((1 << (l + 1)) <= x) ++l;
    return l;
}

}  // namespace

int rows_group(int q) {
    int g = 1;
    while (g < q && g < 64) g <<= 1;
    return g;
}

void launch_rows_check(const int64_t *ptr, const int32_t *idx, const uint8_t *wts, int n, int64_t nnz,
                       double gamma, rdist_info *info, int32_t *bad, double *gpow, hipStream_t s) {
    hipLaunchKernelGGL(k_rows_check, dim3((n + 255) / 256), dim3(256), 0, s, ptr, idx, wts, n, nnz, info, bad);
    hipLaunchKernelGGL(k_rows_gate, dim3(1), dim3(256), 0, s, gamma, bad, info, gpow);
}

template <int NB>
void step64(const RowsLaunch &L, const double *Vo, double *Vn, int32_t *flag, hipStream_t s) {
    const int waves = (L.n + NB - 1) / NB;
    const int blocks = (waves + 3) / 4;
    const dim3 grid(((blocks + 7) / 8) * 8, (L.q + 63) / 64);
    hipLaunchKernelGGL((k_rows_step64<NB>), grid, dim3(256), 0, s, L.ptr, L.idx, L.wts, L.wts ? L.gpow : nullptr,
                       L.n, L.goals, L.q, Vo, Vn, L.info, flag);
}

void launch_rows_step(const RowsLaunch &L, const double *Vo, double *Vn, int32_t *flag, hipStream_t s) {
    const int G = rows_group(L.q);
    const int deg = (int)std::max<int64_t>(1, (L.nnz + L.n - 1) / std::max(L.n, 1));
    if (G >= 2 && G <= 32 && deg <= 16) {   // sparse graphs: a lane walks its node's few successors
        const int blocks = (L.n + 255) / 256;
        const dim3 grid(((blocks + 7) / 8) * 8, (L.q + G - 1) / G);
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, L.ptr, L.idx, L.wts, L.wts ? L.gpow : nullptr, L.n,
                               L.goals, L.q, Vo, Vn, L.info, flag);
        };
        switch (ilog2(G)) {
            case 1: go(k_rows_step_lane<2>); break;
            case 2: go(k_rows_step_lane<4>); break;
            case 3: go(k_rows_step_lane<8>); break;
            case 4: go(k_rows_step_lane<16>); break;
            default: go(k_rows_step_lane<32>); break;
        }
        return;
    }
    if (G == 64) {
        // nodes per wavefront: about 64 edges' worth, at most 16
        const int nb = std::max(1, std::min(16, 64 / deg));
        if (nb >= 16) step64<16>(L, Vo, Vn, flag, s);
        else if (nb >= 8) step64<8>(L, Vo, Vn, flag, s);
        else if (nb >= 4) step64<4>(L, Vo, Vn, flag, s);
        else if (nb >= 2) step64<2>(L, Vo, Vn, flag, s);
        else step64<1>(L, Vo, Vn, flag, s);
        return;
    }
    // successor slots per node: a quarter of the mean degree (each lane then
    // walks a few successors, four loads in flight), so more nodes share a
    // wavefront
    int S = 1;
    while (S < deg / 4 && G * S < 64) S <<= 1;
    const int ls = ilog2(S);
    switch (ilog2(G)) {
        case 0: step_g<1>(ls, L, Vo, Vn, flag, s); break;
        case 1: step_g<2>(ls, L, Vo, Vn, flag, s); break;
        case 2: step_g<4>(ls, L, Vo, Vn, flag, s); break;
        case 3: step_g<8>(ls, L, Vo, Vn, flag, s); break;
        case 4: step_g<16>(ls, L, Vo, Vn, flag, s); break;
        case 5: step_g<32>(ls, L, Vo, Vn, flag, s); break;
        default: step_g<64>(ls, L, Vo, Vn, flag, s); break;
    }
}

void launch_rows_out(const double *V, int n, int q, double *Y, int16_t *D, rdist_info *info, hipStream_t s) {
    const int G = rows_group(q);
    const dim3 grid((unsigned)std::min((n + 255) / 256, 64), (unsigned)q);
    switch (ilog2(G)) {
        case 0: hipLaunchKernelGGL(k_rows_out<1>, grid, dim3(256), 0, s, V, n, q, Y, D, info); break;
        case 1: hipLaunchKernelGGL(k_rows_out<2>, grid, dim3(256), 0, s, V, n, q, Y, D, info); break;
        case 2: hipLaunchKernelGGL(k_rows_out<4>, grid, dim3(256), 0, s, V, n, q, Y, D, info); break;
        case 3: hipLaunchKernelGGL(k_rows_out<8>, grid, dim3(256), 0, s, V, n, q, Y, D, info); break;
        case 4: hipLaunchKernelGGL(k_rows_out<16>, grid, dim3(256), 0, s, V, n, q, Y, D, info); break;
        case 5: hipLaunchKernelGGL(k_rows_out<32>, grid, dim3(256), 0, s, V, n, q, Y, D, info); break;
        default: hipLaunchKernelGGL(k_rows_out<64>, grid, dim3(256), 0, s, V, n, q, Y, D, info); break;
    }
}

void launch_rows_paths(const int64_t *ptr, const int32_t *idx, int n, int64_t nnz, const double *Y,
                       const int32_t *goals, const int32_t *starts, int q, int max_hops, int32_t *out, hipStream_t s) {
    hipLaunchKernelGGL(k_rows_paths, dim3((q + 3) / 4), dim3(256), 0, s, ptr, idx, n, nnz, Y, goals, starts, q,
                       max_hops, out);
}

}  // namespace rd
