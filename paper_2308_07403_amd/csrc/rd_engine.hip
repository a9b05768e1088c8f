// rd_engine.hip -- host side of the C ABI declared in include/rdist.h.
//
// Owns: per-stream workspaces (so solves on different streams never share
// scratch), HBM budget accounting, graph handles that keep Y resident, the
// per-kernel event timing, and plan selection:
//   n <= 128                 single-workgroup register-resident solve
//   otherwise / PLAN_BLOCKED blocked Gauss-Jordan, b = 128, MFMA updates
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "../../include/rdist.h"
#include "rd_engine.h"
#include "rd_launch.h"

// Static scratch of rdist_solve_noalloc (one copy per GPU the library runs
// on, held until the process ends): the blocked plan's buffers for order up
// to RDIST_NOALLOC_MAX_N -- M, Ut[2], V[2], Pt[2], the 256-block inverse's
// Ut2, V2, Pt2 -- and the small buffer (out-degrees, input flag, device
// info), at the 256-byte aligned offsets below.  Host code never passes
// this name to a kernel: rdist_create takes the device address with
// hipGetSymbolAddress once per device, and the launches receive that.
namespace rd {
namespace eng {
constexpr size_t na_al(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t kNaMax = RDIST_NOALLOC_MAX_N;
constexpr size_t kNaM = 0;
constexpr size_t kNaUt = kNaM + na_al(kNaMax * kNaMax * 8);
constexpr size_t kNaStep = na_al(256 * kNaMax * 8);   // one Ut or V buffer
constexpr size_t kNaV = kNaUt + 2 * kNaStep;
constexpr size_t kNaPt = kNaV + 2 * kNaStep;
constexpr size_t kNaUt2 = kNaPt + 2 * na_al(256 * 256 * 8);
constexpr size_t kNaV2 = kNaUt2 + na_al(128 * 256 * 8);
constexpr size_t kNaPt2 = kNaV2 + na_al(128 * 256 * 8);
constexpr size_t kNaSmall = kNaPt2 + na_al(128 * 128 * 8);
constexpr size_t kNaSmallBytes = 256 * ((4 * (kNaMax + 2) + 255) / 256) + sizeof(rdist_info);
constexpr size_t kNaBytes = kNaSmall + na_al(kNaSmallBytes);
}  // namespace eng
}  // namespace rd

static __device__ __align__(256) unsigned char scratch[rd::eng::kNaBytes];

namespace rd {
namespace eng {

rdist_status ensure_small(rdist_ctx c, Workspace &w, int n) {
    if (w.small.p && w.n_cap >= n) return RDIST_OK;
    const int cap = std::max(n, 1024);
    const size_t ints = 256 * ((sizeof(int32_t) * (size_t)(cap + 2) + 255) / 256);
    release(c, w.small);
    rdist_status st = ensure(c, w.small, ints + sizeof(rdist_info));
    if (st == RDIST_OK) w.n_cap = cap;
    return st;
}

// Blocked-plan buffers for order np.  A graph kept with RDIST_KEEP_Y takes
// M over; it is then reallocated here on the next blocked solve.
rdist_status ensure_big(rdist_ctx c, Workspace &w, int np) {
    if (w.np_cap < np) {
        release(c, w.M);
        for (int q = 0; q < 2; ++q) { release(c, w.Ut[q]); release(c, w.V[q]); }
        w.np_cap = np;
    }
    const int cap = w.np_cap;
    rdist_status st;
    if ((st = ensure(c, w.M, (size_t)cap * cap * 8))) return st;
    for (int q = 0; q < 2; ++q) {
        if ((st = ensure(c, w.Ut[q], (size_t)256 * cap * 8))) return st;
        if ((st = ensure(c, w.V[q], (size_t)256 * cap * 8))) return st;
        if ((st = ensure(c, w.Pt[q], (size_t)256 * 256 * 8))) return st;
    }
    if ((st = ensure(c, w.Ut2, (size_t)128 * 256 * 8))) return st;
    if ((st = ensure(c, w.V2, (size_t)128 * 256 * 8))) return st;
    if ((st = ensure(c, w.Pt2, (size_t)128 * 128 * 8))) return st;
    if ((st = ensure_aux(w))) return st;
    return ensure_aux2(w);   // the band update beside the second panel (b = 256)
}

void drain_timing(rdist_ctx c) {
    for (auto &t : c->pending) {
        (void)hipEventSynchronize(t.b);
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
            rdist_kernel_stats &s = c->stats[t.which];
            s.launches += 1;
            s.total_ms += ms;
            s.flops += t.flops;
            s.bytes += t.bytes;
        }
        c->event_pool.push_back(t.a);
        c->event_pool.push_back(t.b);
    }
    c->pending.clear();
}

rdist_status copy_info(rdist_info *host, const rdist_info *dev, int count, hipStream_t s) {
    if (!host || count <= 0) return RDIST_OK;
    RD_HIP(hipMemcpyAsync(host, dev, sizeof(rdist_info) * (size_t)count, hipMemcpyDeviceToHost, s));
    return RDIST_OK;
}

rdist_status make_graph(rdist_ctx c, int n, double *Y, int ld, size_t ybytes, const uint8_t *A, hipStream_t s,
                        rdist_graph *out, const rdist_info *dinfo, bool weighted) {
    const int nw = (n + 63) / 64;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t b_succ = al((size_t)n * nw * 8), b_a = al((size_t)n * n), b_deg = al((size_t)n * 4),
                 b_info = al(sizeof(rdist_info)), b_sm = al(((size_t)3 * n + 16) * 8);
    const size_t bytes = b_succ + b_a + b_deg + b_info + b_sm;
    void *aux = nullptr;
    rdist_status st = dalloc(c, &aux, bytes);
    if (st) return st;
    char *p = (char *)aux;
    auto *g = new rdist_graph_s();
    g->ctx = c;
    g->Y = Y;
    g->n = n;
    g->ld = ld;
    g->succ = (unsigned long long *)p;
    g->A = (uint8_t *)(p + b_succ);
    g->outdeg = (int32_t *)(p + b_succ + b_a);
    g->ginfo = (rdist_info *)(p + b_succ + b_a + b_deg);
    g->sm = (double *)(p + b_succ + b_a + b_deg + b_info);
    g->weighted = weighted ? 1 : 0;
    g->aux = aux;
    g->ybytes = ybytes;
    g->aux_bytes = bytes;
    g->bytes = ybytes + bytes;
    rd::launch_succ_bitmap(A, n, g->succ, s);
    rd::launch_outdeg_from_bits(g->succ, n, g->outdeg, s);
    hipError_t e = hipMemcpyAsync(g->A, A, (size_t)n * n, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(g->ginfo, dinfo, sizeof(rdist_info), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) {
        dfree(c, aux, bytes);
        delete g;
        return fail(RDIST_E_HIP, std::string("graph handle: ") + hipGetErrorString(e));
    }
    c->graphs.insert(g);
    *out = g;
    return RDIST_OK;
}

void release_graph_locked(rdist_graph g) {
    rdist_ctx c = g->ctx;
    (void)hipFree(g->Y);
    (void)hipFree(g->aux);
    if (g->beta) (void)hipFree(g->beta);
    if (g->hinfo) (void)hipHostFree(g->hinfo);
    if (g->bs) (void)hipFree(g->bs);
    c->in_use -= std::min(g->bytes, c->in_use);
    c->graphs.erase(g);
    delete g;
}

// Block width of the blocked plan, in 128-tiles (1: b = 128, 2: b = 256);
// the RDIST_BLOCK_* flags override the default: 128 up to n = 6400, 256
// above.  Measured on one graph per n (ER, single-graph plan), time at
// b = 128 over time at b = 256: 0.88 (n = 2048), 0.85 (3072), 0.86 (4096),
// 0.89 (5120), 0.98 (6144), 1.07 (7168), 1.12 (8192), 1.14 (12288 and
// 16384): above about 6400 the 256 block's rank-256 updates (half the
// passes over M) outweigh its longer lookahead chain.
constexpr int kBlock256MinN = 6401;
int block_tiles(int n, uint32_t flags) {
    if (flags & RDIST_BLOCK_128) return 1;
    if (flags & RDIST_BLOCK_256) return 2;
    return n >= kBlock256MinN ? 2 : 1;
}

// P = M_KK^{-1} for the block at tile K0 (m tiles wide) into Pt (P^T) and
// V's block columns, on stream st.  For m = 2 the 256 x 256 block is
// inverted in place inside M by two Gauss-Jordan steps of 128 (the step
// update of this block overwrites the diagonal block with P anyway).
void enqueue_inverse(rdist_ctx c, Workspace &w, int ld, int K0, int m, int par, rdist_info *dinfo,
                     hipStream_t st) {
    double *M = w.m();
    double *Pt = (double *)w.Pt[par].p, *V = (double *)w.V[par].p;
    const double b = 128.0 * m;
    Timer t(c, st, RDIST_K_PANEL, 2.0 * b * b * b, 16.0 * b * b);
    if (m == 1) {
        rd::launch_panel(M, ld, K0, Pt, V, ld, dinfo, st);
        return;
    }
    double *S = M + (size_t)K0 * kB * ld + (size_t)K0 * kB;     // the diagonal block, leading dim ld
    double *Ut2 = (double *)w.Ut2.p, *V2 = (double *)w.V2.p, *Pt2 = (double *)w.Pt2.p;
    for (int k2 = 0; k2 < 2; ++k2) {
        rd::launch_panel(S, ld, k2, Pt2, V2, 256, dinfo, st);
        rd::launch_rowcol(S, ld, 2, k2, 1, Pt2, Ut2, V2, 256, dinfo, st);
        rd::launch_update(rd::kUpdateAll, S, ld, 2, k2, 1, 0, 1, Ut2, V2, 256, false, 0, nullptr, 0, dinfo, st);
    }
    rd::launch_panel_finish(S, ld, 256, K0, Pt, V, ld, dinfo, st);
}

// Zeroes the 128 x 128 blocks at column block J of rows [0, 128) of the
// k-major slabs V and Ut (leading dimension ld).
__global__ __launch_bounds__(128) void k_zero_pair_blocks(double *__restrict__ V, double *__restrict__ Ut, int ld,
                                                          int J) {
    double *slab = blockIdx.x < 128 ? V : Ut;
    const int row = blockIdx.x & 127;
    slab[(size_t)row * ld + (size_t)J * kB + threadIdx.x] = 0.0;
}

// The factors of the 256-wide block at tiles j, j+1 (b = 256) from two
// 128-pivot steps over the whole band instead of inverting the 256 x 256
// diagonal block first:
//   step j    P^j = M_jj^{-1}; V rows [0, 128) = P^j M_j,: (P^j at block j),
//             Ut rows [0, 128) = -(M_:,j)^T (identity at block j);
//             then tile row and column j+1 take step j (a 128-wide update);
//   step j+1  P^{j+1} = M'_{j+1,j+1}^{-1}; V rows [128, 256) = P^{j+1} M'_{j+1,:},
//             Ut rows [128, 256) = -(M'_:,j+1)^T (identity at block j+1).
// With V^j's block j+1 and Ut^j's block j+1 set to zero afterwards (their
// contribution to row and column j+1 is inside step j+1's factors), the
// rank-256 update M~ + Ut^T V over the concatenated slabs is the two steps
// together: row j gets V^j + (Ut^{j+1}_j)^T V^{j+1}, row j+1 gets V^{j+1},
// column j+1 gets (Ut^{j+1})^T P^{j+1}, every other tile both products.  The
// DIAG, EDGEREST and REST updates of the 256 block run on these slabs
// unchanged.  wait_ev (nullable): recorded on the main stream once tile rows
// and columns j, j+1 are final (EDGEREST of the previous step); waited for
// on st before the first launch that reads them in full.  The panel of step
// j reads only the diagonal tile, which the previous step's DIAG updated.
// side (nullable): a second stream for step j's update of the rest of tile
// row and column j+1, which only the row and column tiles of step j+1 read,
// so that it runs beside the second panel (forked after the first row and
// column tiles, joined before the second).
rdist_status enqueue_pair256(rdist_ctx c, Workspace &w, int ld, int nt, int j, int par, rdist_info *dinfo,
                             hipStream_t st, hipEvent_t wait_ev, hipStream_t side) {
    double *M = w.m();
    double *Ut = (double *)w.Ut[par].p, *V = (double *)w.V[par].p, *Pt = (double *)w.Pt2.p;
    double *Ut1 = Ut + (size_t)kB * ld, *V1 = V + (size_t)kB * ld;   // rows [128, 256): step j+1
    const double b = 128.0;
    const double p_flops = 2.0 * b * b * b, p_bytes = 16.0 * b * b;
    const double rc_flops = 2.0 * b * b * (nt * 128.0 - b), rc_bytes = 8.0 * 4 * b * nt * 128.0;
    const int te = rd::update_tiles(rd::kUpdateEdgeRest, nt, 1, 1);
    // step j
    {
        Timer t(c, st, RDIST_K_PANEL, p_flops, p_bytes);
        rd::launch_panel(M, ld, j, Pt, V, ld, dinfo, st);
    }
    if (wait_ev) RD_HIP(hipStreamWaitEvent(st, wait_ev, 0));
    {
        Timer t(c, st, RDIST_K_ROWCOL, rc_flops, rc_bytes);
        rd::launch_rowcol(M, ld, nt, j, 1, Pt, Ut, V, ld, dinfo, st);
    }
    // step j on tile row and column j+1: the rest of the band (on side if
    // given) and the diagonal tile, which is all the second panel reads
    hipStream_t es = side ? side : st;
    if (side) {
        RD_HIP(hipEventRecord(w.ev_fork, st));
        RD_HIP(hipStreamWaitEvent(side, w.ev_fork, 0));
    }
    {
        Timer t(c, es, RDIST_K_UPDATE_EDGE, p_flops * te, p_bytes * te);
        rd::launch_update(rd::kUpdateEdgeRest, M, ld, nt, j, 1, j + 1, 1, Ut, V, ld, false, 0, nullptr, 0, dinfo,
                          es);
    }
    if (side) RD_HIP(hipEventRecord(w.ev_join, side));
    {
        Timer t(c, st, RDIST_K_UPDATE_EDGE, p_flops, p_bytes);
        rd::launch_update(rd::kUpdateDiag, M, ld, nt, j, 1, j + 1, 1, Ut, V, ld, false, 0, nullptr, 0, dinfo, st);
    }
    // step j+1
    {
        Timer t(c, st, RDIST_K_PANEL, p_flops, p_bytes);
        rd::launch_panel(M, ld, j + 1, Pt, V1, ld, dinfo, st);
    }
    if (side) RD_HIP(hipStreamWaitEvent(st, w.ev_join, 0));
    {
        Timer t(c, st, RDIST_K_ROWCOL, rc_flops, rc_bytes);
        rd::launch_rowcol(M, ld, nt, j + 1, 1, Pt, Ut1, V1, ld, dinfo, st);
    }
    // V^j's block j+1 and Ut^j's block j+1: read by step j's band and
    // diagonal updates, both finished here
    hipLaunchKernelGGL(k_zero_pair_blocks, dim3(256), dim3(128), 0, st, V, Ut, ld, j + 1);
    RD_HIP(hipGetLastError());
    return RDIST_OK;
}

void enqueue_rowcol(rdist_ctx c, Workspace &w, int ld, int nt, int K0, int m, int par, rdist_info *dinfo,
                    hipStream_t st) {
    const double b = 128.0 * m;
    Timer t(c, st, RDIST_K_ROWCOL, 2.0 * b * b * (nt * 128.0 - b), 8.0 * 4 * b * nt * 128.0);
    if (m == 1)
        rd::launch_rowcol64(w.m(), ld, nt, K0, (double *)w.Pt[par].p, (double *)w.Ut[par].p, (double *)w.V[par].p, ld,
                            dinfo, st);
    else
        rd::launch_rowcol(w.m(), ld, nt, K0, m, (double *)w.Pt[par].p, (double *)w.Ut[par].p, (double *)w.V[par].p,
                          ld, dinfo, st);
}

// Blocked solve of one graph on stream s: blocks of b = 128*m columns.
// Step K's update is split by what the lookahead needs (lookahead depth 2):
//   DIAG      the next block's diagonal tiles (its inverse needs only these),
//   EDGEREST  the rest of the next two blocks' tile rows and columns,
//   REST      everything else.
// Schedule of step K (s = caller's stream, aux = lookahead stream):
//   s  : wait ev_panel (step K's row/column tiles); EDGEREST(K);
//        record ev_er; REST(K)
//   aux: DIAG(K); inverse(K+1); wait ev_er; row/column tiles (K+1);
//        record ev_panel
// (for b = 256 the inverse and the row/column tiles of block K+1 are the two
// 128-pivot steps of enqueue_pair256, which waits for ev_er after its first
// panel)
// DIAG(K) reads the next-next block's tiles as EDGEREST(K-1) left them, so the
// lookahead chain never waits for a REST update: the next block's inverse
// runs beside the big update.  U, V and P^T are double-buffered by step
// parity; a step's buffers are rewritten only after the main stream has
// passed the EDGEREST that follows the REST reading them.
// The launch sequence of a blocked solve in workspace w (M, Ut, V, Pt and
// the 256-block buffers sized for order ld, small for n), ending with D and
// dinfo written.  as: the lookahead stream; as == s runs every step on s in
// order (no events), which is correct for the same reason the two-stream
// schedule is: each step's launches only read what earlier launches wrote.
rdist_status enqueue_blocked(rdist_ctx c, Workspace &w, int ld, const uint8_t *A, int n, double gamma,
                             uint32_t flags, int16_t *D, rdist_info *dinfo, hipStream_t s, hipStream_t as) {
    const int m = block_tiles(n, flags);
    const int bw = 128 * m;
    const int np = ((n + bw - 1) / bw) * bw;
    const int nt = np / kB, nbk = np / bw;
    const bool two = as != s;
    double *M = w.m();
    const bool keep_y = (flags & RDIST_KEEP_Y) != 0;
    const bool fused = !(flags & RDIST_UNFUSED_EPILOGUE);
    {
        Timer t(c, s, RDIST_K_INGEST, 0.0, (double)n * n + 8.0 * np * np);
        rd::launch_ingest(A, n, np, ld, gamma, M, w.outdeg(), w.bad(), dinfo, s, (flags & RDIST_WEIGHTED) != 0);
    }
    RD_HIP(hipGetLastError());
    // a third stream for the band update only while this context drives one
    // stream: the process has four hardware queues, and the streams of
    // several concurrent solves already share them (three solves on three
    // streams: 43 graphs/s with it against 52 without, at n = 8192)
    hipStream_t side = two && c->ws.size() == 1 ? w.aux2 : nullptr;
    if (m == 2) {
        rdist_status st0 = enqueue_pair256(c, w, ld, nt, 0, 0, dinfo, s, nullptr, side);
        if (st0) return st0;
    } else {
        enqueue_inverse(c, w, ld, 0, m, 0, dinfo, s);
        enqueue_rowcol(c, w, ld, nt, 0, m, 0, dinfo, s);
    }
    // streams of the step loop: the caller's stream and the lookahead stream
    hipStream_t ms = s;
    if (nbk > 1 && two) {
        RD_HIP(hipEventRecord(w.ev_panel, ms));          // block 0's row/column tiles are ready
        RD_HIP(hipStreamWaitEvent(as, w.ev_panel, 0));
    }
    const double tile_flops = 2.0 * kB * kB * bw;
    for (int K = 0; K < nbk; ++K) {
        const int par = K & 1;
        const int K0 = K * m;
        const double *Ut = (const double *)w.Ut[par].p, *V = (const double *)w.V[par].p;
        if (K + 1 < nbk) {
            const int L0 = K0 + m;
            const int wt = std::min(2 * m, nt - L0);      // the next two blocks' tile rows and columns
            const int td = rd::update_tiles(rd::kUpdateDiag, nt, m, wt);
            const int te = rd::update_tiles(rd::kUpdateEdgeRest, nt, m, wt);
            const int tr = rd::update_tiles(rd::kUpdateRest, nt, m, wt);
            if (K > 0 && two) RD_HIP(hipStreamWaitEvent(ms, w.ev_panel, 0));
            {
                Timer t(c, ms, RDIST_K_UPDATE_EDGE, tile_flops * te, 16.0 * kB * kB * te);
                rd::launch_update(rd::kUpdateEdgeRest, M, ld, nt, K0, m, L0, wt, Ut, V, ld, false, n, D, 0, dinfo,
                                  ms);
            }
            if (two) RD_HIP(hipEventRecord(w.ev_er, ms));
            {
                Timer t(c, ms, RDIST_K_UPDATE, tile_flops * tr, 16.0 * kB * kB * tr);
                rd::launch_update(rd::kUpdateRest, M, ld, nt, K0, m, L0, wt, Ut, V, ld, false, n, D, 0, dinfo, ms);
            }
            {
                Timer t(c, as, RDIST_K_UPDATE_EDGE, tile_flops * td, 16.0 * kB * kB * td);
                if (m == 1)
                    rd::launch_diag64(M, ld, L0, Ut, V, ld, dinfo, as);
                else
                    rd::launch_update(rd::kUpdateDiag, M, ld, nt, K0, m, L0, wt, Ut, V, ld, false, n, D, 0, dinfo,
                                      as);
            }
            if (m == 2) {
                rdist_status sp = enqueue_pair256(c, w, ld, nt, L0, par ^ 1, dinfo, as, two ? w.ev_er : nullptr,
                                                  side);
                if (sp) return sp;
            } else {
                enqueue_inverse(c, w, ld, L0, m, par ^ 1, dinfo, as);
                if (two) RD_HIP(hipStreamWaitEvent(as, w.ev_er, 0));
                enqueue_rowcol(c, w, ld, nt, L0, m, par ^ 1, dinfo, as);
            }
            if (two) RD_HIP(hipEventRecord(w.ev_panel, as));
        } else {
            if (K > 0 && two) RD_HIP(hipStreamWaitEvent(ms, w.ev_panel, 0));
            Timer t(c, ms, RDIST_K_UPDATE_EDGE, tile_flops * nt * nt, 16.0 * kB * kB * nt * nt);
            rd::launch_update(rd::kUpdateAll, M, ld, nt, K0, m, 0, m, Ut, V, ld, fused, n, D, keep_y ? 1 : 0, dinfo,
                              ms);
        }
        RD_HIP(hipGetLastError());
    }
    if (!fused) {
        Timer t(c, s, RDIST_K_EPILOGUE, 0.0, 10.0 * n * n);
        rd::launch_epilogue(M, n, ld, D, dinfo, s);
    }
    rd::launch_fill_sentinel(D, n, dinfo, s);
    RD_HIP(hipGetLastError());
    return RDIST_OK;
}

rdist_status solve_blocked(rdist_ctx c, const uint8_t *A, int n, double gamma, uint32_t flags, int16_t *D,
                           rdist_graph *keep, rdist_info *info, hipStream_t s) {
    Workspace &w = c->ws[s];
    const int bw = 128 * block_tiles(n, flags);
    const int np = ((n + bw - 1) / bw) * bw;
    rdist_status st = ensure_small(c, w, n);
    if (st) return st;
    if ((st = ensure_big(c, w, np))) return st;
    const int ld = w.np_cap;                     // M, Ut, V leading dimension
    rdist_info *dinfo = w.dinfo();
    if ((st = enqueue_blocked(c, w, ld, A, n, gamma, flags, D, dinfo, s, w.aux))) return st;
    if ((flags & RDIST_KEEP_Y) && keep) {
        Buf y = w.M;          // the graph takes M over (its bytes stay counted)
        w.M = Buf{};
        st = make_graph(c, n, (double *)y.p, ld, y.bytes, A, s, keep, dinfo, (flags & RDIST_WEIGHTED) != 0);
        if (st) {
            release(c, y);
            return st;
        }
    }
    return copy_info(info, dinfo, 1, s);
}

// Workspace view of the static scratch at its device address base, for a
// blocked solve of padded order np <= RDIST_NOALLOC_MAX_N (leading
// dimension np) or a small solve: nothing is allocated.
Workspace noalloc_view(void *base, int np) {
    char *b = (char *)base;
    Workspace v;
    v.np_cap = np;
    v.M = Buf{b + kNaM, (size_t)np * np * 8};
    for (int q = 0; q < 2; ++q) {
        v.Ut[q] = Buf{b + kNaUt + q * kNaStep, (size_t)256 * np * 8};
        v.V[q] = Buf{b + kNaV + q * kNaStep, (size_t)256 * np * 8};
        v.Pt[q] = Buf{b + kNaPt + q * na_al(256 * 256 * 8), (size_t)256 * 256 * 8};
    }
    v.Ut2 = Buf{b + kNaUt2, (size_t)128 * 256 * 8};
    v.V2 = Buf{b + kNaV2, (size_t)128 * 256 * 8};
    v.Pt2 = Buf{b + kNaPt2, (size_t)128 * 128 * 8};
    v.small = Buf{b + kNaSmall, kNaSmallBytes};
    v.n_cap = (int)kNaMax;
    return v;
}

rdist_status solve_small(rdist_ctx c, const uint8_t *A, int n, double gamma, uint32_t flags, int16_t *D,
                         rdist_graph *keep, rdist_info *info, hipStream_t s) {
    Workspace &w = c->ws[s];
    rdist_status st = ensure_small(c, w, n);
    if (st) return st;
    double *Y = nullptr;
    const size_t yb = (size_t)n * n * 8;
    const bool keep_y = (flags & RDIST_KEEP_Y) && keep;
    if (keep_y && (st = dalloc(c, (void **)&Y, yb))) return st;
    rd::SmallTask t{A, D, Y, n, n, gamma, w.dinfo()};
    {
        Timer tm(c, s, RDIST_K_SMALL, 2.0 * n * n * n, (double)n * n * (keep_y ? 11.0 : 3.0));
        rd::launch_small_one(t, s);
    }
    RD_HIP(hipGetLastError());
    if (keep_y) {
        st = make_graph(c, n, Y, n, yb, A, s, keep, w.dinfo(), false);
        if (st) { dfree(c, Y, yb); return st; }
    }
    return copy_info(info, w.dinfo(), 1, s);
}

// Frees everything a workspace holds (its buffers, lookahead streams and
// events, its transient batched plan).
void free_workspace(rdist_ctx c, Workspace &w) {
    free_transient_plan(c, w);
    for (Buf *b : {&w.M, &w.Ut[0], &w.Ut[1], &w.V[0], &w.V[1], &w.Pt[0], &w.Pt[1], &w.Ut2, &w.V2, &w.Pt2, &w.small,
                   &w.m32, &w.v32, &w.u32, &w.s64, &w.p32, &w.cert, &w.csr_cnt, &w.csr_off, &w.csr_col, &w.r32,
                   &w.c32, &w.xi, &w.ri, &w.rv, &w.rmisc, &w.rgoals, &w.gb})
        release(c, *b);
    if (w.rows_exec) (void)hipGraphExecDestroy(w.rows_exec);
    if (w.rows_graph) (void)hipGraphDestroy(w.rows_graph);
    if (w.rflag_h) (void)hipHostFree(w.rflag_h);
    for (hipEvent_t e : {w.ev_er, w.ev_panel, w.ev_fork, w.ev_join})
        if (e) (void)hipEventDestroy(e);
    if (w.aux) (void)hipStreamDestroy(w.aux);
    if (w.aux2) (void)hipStreamDestroy(w.aux2);
    w = Workspace{};
}

// Drops the workspace of a stream that is about to be destroyed (its work
// must have finished), so that a later stream with the same handle starts
// afresh and the memory returns to the budget.
void release_stream_workspace(rdist_ctx c, hipStream_t s) {
    auto it = c->ws.find(s);
    if (it == c->ws.end()) return;
    free_workspace(c, it->second);
    c->ws.erase(it);
}

}  // namespace eng
}  // namespace rd

using namespace rd::eng;

extern "C" {

const char *rdist_last_error(void) { return g_last_error.c_str(); }

const char *rdist_status_string(rdist_status s) {
    switch (s) {
        case RDIST_OK: return "RDIST_OK";
        case RDIST_E_ARG: return "RDIST_E_ARG";
        case RDIST_E_ADJ: return "RDIST_E_ADJ";
        case RDIST_E_NOT_DD: return "RDIST_E_NOT_DD";
        case RDIST_E_NOMEM: return "RDIST_E_NOMEM";
        case RDIST_E_AGAIN: return "RDIST_E_AGAIN";
        case RDIST_E_HIP: return "RDIST_E_HIP";
        case RDIST_E_STATE: return "RDIST_E_STATE";
    }
    return "RDIST_E_UNKNOWN";
}

rdist_status rdist_create(rdist_ctx *out, int device, size_t hbm_budget_bytes, const char *tile_cache_path,
                          uint32_t flags) {
    if (!out) return fail(RDIST_E_ARG, "out is NULL");
    *out = nullptr;
    if (flags & ~RDIST_THREADSAFE) return fail(RDIST_E_ARG, "unknown create flags");
    int count = 0;
    RD_HIP(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(RDIST_E_ARG, "no such device");
    RD_HIP(hipSetDevice(device));
    // device address of this device's copy of the static scratch, taken
    // once per device with the device current
    static std::mutex na_mu;
    static std::map<int, std::pair<void *, std::string>> na_addr;
    void *na_ptr = nullptr;
    std::string na_err;
    {
        std::lock_guard<std::mutex> lk(na_mu);
        auto it = na_addr.find(device);
        if (it == na_addr.end()) {
            void *ptr = nullptr;
            const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess) (void)hipGetLastError();
            it = na_addr.emplace(device, std::make_pair(e == hipSuccess ? ptr : nullptr,
                                                        e == hipSuccess ? std::string()
                                                                        : std::string("hipGetSymbolAddress(scratch): ") +
                                                                              hipGetErrorString(e))).first;
        }
        na_ptr = it->second.first;
        na_err = it->second.second;
    }
    auto *c = new rdist_ctx_s();
    c->device = device;
    c->noalloc_scratch = na_ptr;
    c->noalloc_error = na_err;
    c->budget = hbm_budget_bytes;
    c->threadsafe = (flags & RDIST_THREADSAFE) != 0;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->num_cu = prop.multiProcessorCount;
    std::memset(c->stats, 0, sizeof(c->stats));
    if (tile_cache_path && *tile_cache_path) {
        c->tile_cache_path = tile_cache_path;
        load_tile_cache(c);
    }
    *out = c;
    g_last_error.clear();
    return RDIST_OK;
}

void rdist_destroy(rdist_ctx c) {
    if (!c) return;
    {
        Guard g(c);
        (void)hipSetDevice(c->device);
        drain_timing(c);
        destroy_plans(c);
        if (c->tuned_dirty) save_tile_cache(c);
        for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
        std::vector<rdist_graph_s *> gs(c->graphs.begin(), c->graphs.end());
        for (auto *gr : gs) release_graph_locked(gr);
        for (auto &kv : c->ws) free_workspace(c, kv.second);
        c->ws.clear();
    }
    delete c;
}

rdist_status rdist_solve(rdist_ctx c, const uint8_t *A_dev, int32_t n, double gamma, uint32_t flags,
                         int16_t *D_dev, rdist_graph *keep, rdist_info *info, void *stream) {
    if (!c) return fail(RDIST_E_ARG, "ctx is NULL");
    if (!A_dev || !D_dev) return fail(RDIST_E_ARG, "A_dev and D_dev are required");
    if (n < 1 || n > 65536) return fail(RDIST_E_ARG, "n must lie in [1, 65536]");
    rdist_status st;
    if ((st = check_flags(flags))) return st;
    if ((st = check_gamma(gamma))) return st;
    if ((flags & RDIST_PLAN_SMALL) && n > 128) return fail(RDIST_E_ARG, "RDIST_PLAN_SMALL needs n <= 128");
    if (keep) *keep = nullptr;
    Guard g(c);
    RD_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    if (flags & RDIST_MIXED_F32) return solve_mixed(c, A_dev, n, gamma, flags, D_dev, info, s);
    const bool small = !(flags & (RDIST_PLAN_BLOCKED | RDIST_WEIGHTED)) && n <= 128;
    if (small) return solve_small(c, A_dev, n, gamma, flags, D_dev, keep, info, s);
    return solve_blocked(c, A_dev, n, gamma, flags, D_dev, keep, info, s);
}

rdist_status rdist_solve_noalloc(rdist_ctx c, const uint8_t *A_dev, int32_t n, double gamma, uint32_t flags,
                                 int16_t *D_dev, rdist_info *info, void *stream) {
    if (!c) return fail(RDIST_E_ARG, "ctx is NULL");
    if (!A_dev || !D_dev) return fail(RDIST_E_ARG, "A_dev and D_dev are required");
    if (n < 1 || n > RDIST_NOALLOC_MAX_N)
        return fail(RDIST_E_ARG, "rdist_solve_noalloc: n must lie in [1, " + std::to_string(RDIST_NOALLOC_MAX_N) +
                                     "], the largest order its static scratch holds");
    rdist_status st;
    if ((st = check_flags(flags))) return st;
    if ((st = check_gamma(gamma))) return st;
    if (flags & (RDIST_MIXED_F32 | RDIST_KEEP_Y | RDIST_NO_GRAPH))
        return fail(RDIST_E_ARG, "rdist_solve_noalloc takes no RDIST_MIXED_F32, RDIST_KEEP_Y or RDIST_NO_GRAPH");
    if ((flags & RDIST_PLAN_SMALL) && n > 128) return fail(RDIST_E_ARG, "RDIST_PLAN_SMALL needs n <= 128");
    Guard g(c);
    if (!c->noalloc_scratch) return fail(RDIST_E_HIP, "rdist_solve_noalloc: " + c->noalloc_error);
    RD_HIP(hipSetDevice(c->device));
    struct Untimed {
        Untimed() { g_untimed = true; }
        ~Untimed() { g_untimed = false; }
    } untimed;
    hipStream_t s = (hipStream_t)stream;
    const int bw = 128 * block_tiles(n, flags);
    const int np = ((n + bw - 1) / bw) * bw;
    Workspace v = noalloc_view(c->noalloc_scratch, np);
    const bool small = !(flags & (RDIST_PLAN_BLOCKED | RDIST_WEIGHTED)) && n <= 128;
    if (small) {
        rd::SmallTask t{A_dev, D_dev, nullptr, n, n, gamma, v.dinfo()};
        rd::launch_small_one(t, s);
        RD_HIP(hipGetLastError());
    } else if ((st = enqueue_blocked(c, v, np, A_dev, n, gamma, flags, D_dev, v.dinfo(), s, s))) {
        return st;
    }
    return copy_info(info, v.dinfo(), 1, s);
}

rdist_status rdist_next_hop(rdist_ctx c, rdist_graph gr, const int32_t *cur_dev, const int32_t *goal_dev, int32_t q,
                            int32_t max_hops, int32_t *out_dev, void *stream) {
    if (!c || !gr) return fail(RDIST_E_ARG, "NULL handle");
    if (gr->ctx != c) return fail(RDIST_E_STATE, "graph belongs to another context");
    if (q < 0 || max_hops < 1 || max_hops > 65535) return fail(RDIST_E_ARG, "bad q or max_hops");
    if (q == 0) return RDIST_OK;
    if (!cur_dev || !goal_dev || !out_dev) return fail(RDIST_E_ARG, "NULL query array");
    Guard g(c);
    RD_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    {
        Timer tm(c, s, RDIST_K_NEXTHOP, 0.0, 0.0);
        rd::launch_next_hop(gr->Y, gr->ld, gr->n, gr->succ, cur_dev, goal_dev, q, max_hops, out_dev, s);
    }
    RD_HIP(hipGetLastError());
    return RDIST_OK;
}

void rdist_graph_release(rdist_graph g) {
    if (!g) return;
    rdist_ctx c = g->ctx;
    Guard gd(c);
    (void)hipSetDevice(c->device);
    release_graph_locked(g);
}

rdist_status rdist_graph_y(rdist_graph g, const double **Y_dev, int32_t *n, int32_t *ld) {
    if (!g) return fail(RDIST_E_ARG, "NULL graph");
    if (Y_dev) *Y_dev = g->Y;
    if (n) *n = g->n;
    if (ld) *ld = g->ld;
    return RDIST_OK;
}

// Re-inverts a kept graph from its own (already changed) adjacency at its
// gain and takes the new Y over; the error bounds restart.  D gets the new
// graph's D (a temporary when the caller passed none); *out the solve's info.
static rdist_status refresh_graph(rdist_ctx c, rdist_graph g, double gamma, int16_t *D, rdist_info *out,
                                  hipStream_t s) {
    void *tmp = nullptr;
    const size_t db = (size_t)g->n * g->n * 2;
    rdist_status st;
    if (!D) {
        if ((st = dalloc(c, &tmp, db))) return st;
        D = (int16_t *)tmp;
    }
    const uint32_t flags = RDIST_KEEP_Y | (g->weighted ? RDIST_WEIGHTED : 0u);
    rdist_graph fresh = nullptr;
    st = (!g->weighted && g->n <= 128) ? solve_small(c, g->A, g->n, gamma, flags, D, &fresh, nullptr, s)
                                       : solve_blocked(c, g->A, g->n, gamma, flags, D, &fresh, nullptr, s);
    if (!st && !fresh) st = fail(RDIST_E_STATE, "re-inversion kept no graph");
    if (!st) {
        std::swap(g->Y, fresh->Y);
        std::swap(g->ld, fresh->ld);
        std::swap(g->ybytes, fresh->ybytes);
        g->changed = false;
        g->bytes = g->ybytes + g->aux_bytes + g->beta_bytes + g->bs_bytes;
        fresh->bytes = fresh->ybytes + fresh->aux_bytes + fresh->beta_bytes + fresh->bs_bytes;
        hipError_t e = hipMemcpyAsync(g->ginfo, fresh->ginfo, sizeof(rdist_info), hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(out, fresh->ginfo, sizeof(rdist_info), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) {
            rd::launch_beta_fill(g->beta, g->n, g->ginfo, s);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = fail(RDIST_E_HIP, std::string("re-inversion: ") + hipGetErrorString(e));
        release_graph_locked(fresh);   // frees the old Y
    }
    if (tmp) dfree(c, tmp, db);
    return st;
}

// What edge changes keep beside Y, made by the first change: the pinned
// info copy, the per-entry error bounds and the out-degree histogram.
static rdist_status ensure_change_state(rdist_ctx c, rdist_graph g, hipStream_t s) {
    const int n = g->n;
    rdist_status st;
    if (!g->hinfo) RD_HIP(hipHostMalloc((void **)&g->hinfo, sizeof(rdist_info), hipHostMallocDefault));
    if (!g->beta) {
        const size_t qb = ((size_t)n * n * 2 + 255) & ~(size_t)255;
        const size_t bb = qb + (size_t)(n + 1) * 4;
        if ((st = dalloc(c, (void **)&g->beta, bb))) return st;
        g->hist = (int32_t *)((char *)g->beta + qb);
        g->beta_bytes = bb;
        g->bytes += bb;
        rd::launch_beta_fill(g->beta, n, g->ginfo, s);
        rd::launch_deg_hist(g->outdeg, n, g->hist, s);
    }
    return RDIST_OK;
}

static rdist_status check_change(rdist_graph g, int32_t src, int32_t dst, int32_t weight) {
    if (src < 0 || src >= g->n || dst < 0 || dst >= g->n || src == dst)
        return fail(RDIST_E_ARG, "src and dst must be distinct nodes of the graph");
    if (weight < 0 || weight > (g->weighted ? 255 : 1))
        return fail(RDIST_E_ARG, g->weighted ? "weight must lie in [0, 255]" : "weight must be 0 or 1");
    return RDIST_OK;
}

rdist_status rdist_graph_update_edges(rdist_ctx c, rdist_graph g, int32_t count, const int32_t *src,
                                      const int32_t *dst, const int32_t *weight, int16_t *D_dev, rdist_info *info,
                                      void *stream) {
    if (!c || !g) return fail(RDIST_E_ARG, "NULL handle");
    if (g->ctx != c) return fail(RDIST_E_STATE, "graph belongs to another context");
    if (count < 0 || (count > 0 && (!src || !dst || !weight))) return fail(RDIST_E_ARG, "bad count or NULL arrays");
    rdist_status st;
    for (int32_t e = 0; e < count; ++e)
        if ((st = check_change(g, src[e], dst[e], weight[e]))) return st;
    Guard gd(c);
    RD_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    if (count == 0) {   // nothing to change: the graph's status, Delta and gain
        if (info) {
            rdist_info cur{};
            RD_HIP(hipMemcpyAsync(&cur, g->ginfo, sizeof(rdist_info), hipMemcpyDeviceToHost, s));
            RD_HIP(hipStreamSynchronize(s));
            *info = rdist_info{};
            info->status = cur.status;
            info->delta = cur.delta;
            info->gamma = cur.gamma;
        }
        return RDIST_OK;
    }
    const int n = g->n;
    if ((st = ensure_change_state(c, g, s))) return st;
    if (!g->bs) {
        const size_t b = rd::batch_scratch_doubles(n) * 8;
        if ((st = dalloc(c, (void **)&g->bs, b))) return st;
        g->bs_bytes = b;
        g->bytes += b;
    }
    rdist_info *ci = reinterpret_cast<rdist_info *>(g->sm + 2);
    rdist_info hi{};
    hi.status = RDIST_OK;
    int64_t lost_total = 0;
    bool reinverted = false;
    for (int32_t off = 0; off < count; off += rd::kMaxBatch) {
        rd::EdgeBatch B{};
        B.k = std::min(rd::kMaxBatch, count - off);
        for (int a = 0; a < B.k; ++a) {
            B.src[a] = src[off + a];
            B.dst[a] = dst[off + a];
            B.w[a] = weight[off + a];
        }
        const bool last = off + B.k >= count;
        int16_t *D = last ? D_dev : nullptr;
        rd::launch_edge_batch_prep(g->Y, g->ld, n, g->beta, g->sm, g->bs, g->A, g->outdeg, g->ginfo, B, s);
        {
            const double n2 = (double)n * n;
            Timer t(c, s, RDIST_K_EDGE_UPDATE, 2.0 * B.k * n2, (D ? 22.0 : 20.0) * n2);
            rd::launch_edge_batch_apply(g->Y, g->ld, n, g->beta, g->sm, g->bs, D, g->A, g->outdeg, g->hist, g->succ,
                                        g->ginfo, B, s);
        }
        RD_HIP(hipGetLastError());
        RD_HIP(hipMemcpyAsync(g->hinfo, ci, sizeof(rdist_info), hipMemcpyDeviceToHost, s));
        RD_HIP(hipStreamSynchronize(s));
        hi = *g->hinfo;
        if (hi.status != RDIST_OK) break;
        g->changed = true;
        if (hi.n_uncertified > 0) {
            lost_total += hi.n_uncertified;
            if ((st = refresh_graph(c, g, hi.gamma, D, &hi, s))) return st;
            reinverted = true;
        }
    }
    hi.n_uncertified = lost_total;
    hi.fallback_fraction = reinverted ? 1.0 : 0.0;
    if (info) *info = hi;
    return RDIST_OK;
}

rdist_status rdist_graph_update_edge(rdist_ctx c, rdist_graph g, int32_t src, int32_t dst, int32_t weight,
                                     int16_t *D_dev, rdist_info *info, void *stream) {
    if (!c || !g) return fail(RDIST_E_ARG, "NULL handle");
    if (g->ctx != c) return fail(RDIST_E_STATE, "graph belongs to another context");
    rdist_status st;
    if ((st = check_change(g, src, dst, weight))) return st;
    Guard gd(c);
    RD_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    const int n = g->n;
    if ((st = ensure_change_state(c, g, s))) return st;
    rdist_info *ci = reinterpret_cast<rdist_info *>(g->sm + 2);
    rd::launch_edge_prep(g->Y, g->ld, n, g->A, g->outdeg, g->hist, g->beta, g->ginfo, g->sm, src, dst, weight, s);
    {
        const double n2 = (double)n * n;
        Timer t(c, s, RDIST_K_EDGE_UPDATE, 2.0 * n2, (D_dev ? 22.0 : 20.0) * n2);
        rd::launch_edge_apply(g->Y, g->ld, n, g->beta, g->sm, D_dev, g->A, g->outdeg, g->hist, g->succ, g->ginfo,
                              src, dst, weight, s);
    }
    RD_HIP(hipGetLastError());
    RD_HIP(hipMemcpyAsync(g->hinfo, ci, sizeof(rdist_info), hipMemcpyDeviceToHost, s));
    RD_HIP(hipStreamSynchronize(s));
    rdist_info hi = *g->hinfo;
    if (hi.status == RDIST_OK) g->changed = true;
    if (hi.status == RDIST_OK && hi.n_uncertified > 0) {
        const int64_t lost = hi.n_uncertified;
        if ((st = refresh_graph(c, g, hi.gamma, D_dev, &hi, s))) return st;
        hi.n_uncertified = lost;
        hi.fallback_fraction = 1.0;
    }
    if (info) *info = hi;
    return RDIST_OK;
}

// Layout of the goal-rows scratch: info, bad-input flag, change flag, then
// the 256-entry table of gamma^w.
static constexpr size_t kRowsInfo = 0, kRowsBad = 256, kRowsFlag = 512, kRowsPow = 768;
static constexpr size_t kRowsMisc = kRowsPow + 256 * 8;
static constexpr int kRowsCheckEvery = 16;
static constexpr int64_t kRowsMaxSteps = 1 << 22;

rdist_status rdist_goal_rows(rdist_ctx c, int32_t n, const int64_t *succ_ptr, const int32_t *succ_idx, int64_t nnz,
                             const uint8_t *weights, double gamma, const int32_t *goals, int32_t q, double *Y_dev,
                             int16_t *D_dev, int32_t *steps, rdist_info *info, void *stream) {
    if (!c) return fail(RDIST_E_ARG, "ctx is NULL");
    if (n < 1 || q < 1 || q > 65535 || nnz < 0) return fail(RDIST_E_ARG, "need n >= 1, 1 <= q <= 65535, nnz >= 0");
    if (!succ_ptr || !goals || (nnz > 0 && !succ_idx)) return fail(RDIST_E_ARG, "NULL graph or goal array");
    rdist_status st;
    if ((st = check_gamma(gamma))) return st;
    Guard gd(c);
    RD_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    Workspace &w = c->ws[s];
    const size_t G = (size_t)rd::rows_group(q);
    const size_t vbytes = (size_t)n * G * (size_t)((q + G - 1) / G) * 8;
    if ((st = ensure_grow(c, w.rv, 2 * vbytes))) return st;
    if ((st = ensure_grow(c, w.rmisc, kRowsMisc))) return st;
    if (!w.rflag_h) RD_HIP(hipHostMalloc((void **)&w.rflag_h, sizeof(int32_t), hipHostMallocDefault));
    char *misc = (char *)w.rmisc.p;
    rdist_info *dinfo = (rdist_info *)(misc + kRowsInfo);
    int32_t *bad = (int32_t *)(misc + kRowsBad), *flag = (int32_t *)(misc + kRowsFlag);
    double *gpow = (double *)(misc + kRowsPow);
    double *V[2] = {(double *)w.rv.p, (double *)((char *)w.rv.p + vbytes)};
    // the goals in workspace memory, so that a captured chunk serves any goal set
    if ((st = ensure_grow(c, w.rgoals, (size_t)q * 4))) return st;
    int32_t *wgoals = (int32_t *)w.rgoals.p;
    RD_HIP(hipMemcpyAsync(wgoals, goals, (size_t)q * 4, hipMemcpyDeviceToDevice, s));
    rd::launch_info_set(dinfo, gamma, s);
    rd::launch_fill_i32(bad, 1, s);
    rd::launch_rows_check(succ_ptr, succ_idx, weights, n, nnz, gamma, dinfo, bad, gpow, s);
    rd::launch_fill_i32((int32_t *)V[0], vbytes / 4, s);
    rd::RowsLaunch L{succ_ptr, succ_idx, weights, gpow, n, nnz, wgoals, q, dinfo};
    const double step_bytes = 16.0 * (double)vbytes / 8.0 + 8.0 * n + (weights ? 5.0 : 4.0) * (double)nnz;
    // One chunk: kRowsCheckEvery steps (an even count, so the state ends in
    // V[0] again), the last of which reports whether any entry changed, and
    // the report's copy to the host.
    auto enqueue_chunk = [&](hipStream_t cs, bool timed) {
        int cur = 0;
        for (int t = 0; t < kRowsCheckEvery; ++t) {
            const bool check = t == kRowsCheckEvery - 1;
            if (check) rd::launch_fill_i32(flag, 1, cs);
            if (timed) {
                Timer tm(c, cs, RDIST_K_ROWS_STEP, 0.0, step_bytes);
                rd::launch_rows_step(L, V[cur], V[cur ^ 1], check ? flag : nullptr, cs);
            } else {
                rd::launch_rows_step(L, V[cur], V[cur ^ 1], check ? flag : nullptr, cs);
            }
            cur ^= 1;
        }
        return hipMemcpyAsync(w.rflag_h, flag, sizeof(int32_t), hipMemcpyDeviceToHost, cs);
    };
    // per-step timing (not held) asks for the eager launches; otherwise the
    // chunk is a HIP graph, captured once per (lists, weights, sizes, buffers)
    const bool eager = (c->timing_mask & (1u << RDIST_K_ROWS_STEP)) != 0 && !c->timing_hold;
    if (!eager) {
        const void *key[6] = {succ_ptr, succ_idx, weights, w.rv.p, w.rmisc.p, wgoals};
        const int64_t key_n[3] = {n, nnz, q};
        bool same = w.rows_exec != nullptr;
        for (int t = 0; t < 6 && same; ++t) same = key[t] == w.rows_key[t];
        for (int t = 0; t < 3 && same; ++t) same = key_n[t] == w.rows_key_n[t];
        if (!same) {
            if (w.rows_exec) (void)hipGraphExecDestroy(w.rows_exec);
            if (w.rows_graph) (void)hipGraphDestroy(w.rows_graph);
            w.rows_exec = nullptr;
            w.rows_graph = nullptr;
            if ((st = ensure_capture_streams(c))) return st;
            // the capture stream must see the set-up above
            hipEvent_t ev = nullptr;
            RD_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
            RD_HIP(hipEventRecord(ev, s));
            RD_HIP(hipStreamWaitEvent(c->capture, ev, 0));
            (void)hipEventDestroy(ev);
            RD_HIP(hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal));
            const hipError_t ce = enqueue_chunk(c->capture, false);
            hipGraph_t gr = nullptr;
            const hipError_t ee = hipStreamEndCapture(c->capture, &gr);
            if (ce != hipSuccess || ee != hipSuccess) {
                if (gr) (void)hipGraphDestroy(gr);
                return fail(RDIST_E_HIP, std::string("goal rows capture: ") +
                                             hipGetErrorString(ce != hipSuccess ? ce : ee));
            }
            w.rows_graph = gr;
            RD_HIP(hipGraphInstantiate(&w.rows_exec, w.rows_graph, nullptr, nullptr, 0));
            for (int t = 0; t < 6; ++t) w.rows_key[t] = key[t];
            for (int t = 0; t < 3; ++t) w.rows_key_n[t] = key_n[t];
        }
    }
    int64_t k = 0;
    for (;;) {
        if (eager) RD_HIP(enqueue_chunk(s, true));
        else RD_HIP(hipGraphLaunch(w.rows_exec, s));
        k += kRowsCheckEvery;
        RD_HIP(hipGetLastError());
        RD_HIP(hipStreamSynchronize(s));
        if (*w.rflag_h == 0) break;
        if (k >= kRowsMaxSteps) return fail(RDIST_E_STATE, "goal rows did not settle");
    }
    const int cur = 0;
    rd::launch_rows_out(V[cur], n, q, Y_dev, D_dev, dinfo, s);
    RD_HIP(hipGetLastError());
    if (steps) *steps = (int32_t)std::min<int64_t>(k, 0x7FFFFFFF);
    return copy_info(info, dinfo, 1, s);
}

rdist_status rdist_goal_paths(rdist_ctx c, int32_t n, const int64_t *succ_ptr, const int32_t *succ_idx, int64_t nnz,
                              const double *Y_rows, const int32_t *goals, const int32_t *starts, int32_t q,
                              int32_t max_hops, int32_t *out_dev, void *stream) {
    if (!c) return fail(RDIST_E_ARG, "ctx is NULL");
    if (n < 1 || q < 0 || nnz < 0 || max_hops < 1 || max_hops > 65535) return fail(RDIST_E_ARG, "bad n, nnz, q or max_hops");
    if (q == 0) return RDIST_OK;
    if (!succ_ptr || (nnz > 0 && !succ_idx) || !Y_rows || !goals || !starts || !out_dev) return fail(RDIST_E_ARG, "NULL argument");
    Guard gd(c);
    RD_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    {
        Timer tm(c, s, RDIST_K_NEXTHOP, 0.0, 0.0);
        rd::launch_rows_paths(succ_ptr, succ_idx, n, nnz, Y_rows, goals, starts, q, max_hops, out_dev, s);
    }
    RD_HIP(hipGetLastError());
    return RDIST_OK;
}

rdist_status rdist_gain_bounds(rdist_ctx c, const uint8_t *A_dev, int32_t n, int32_t diameter, int32_t max_steps,
                               double rel_tol, rdist_gain_report *out, void *stream) {
    if (!c || !A_dev || !out) return fail(RDIST_E_ARG, "NULL argument");
    if (n < 1 || n > 65536 || diameter < 0 || diameter >= n || max_steps < 1 || !(rel_tol >= 0.0))
        return fail(RDIST_E_ARG, "need 1 <= n <= 65536, 0 <= diameter < n, max_steps >= 1, rel_tol >= 0");
    Guard gd(c);
    RD_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    Workspace &w = c->ws[s];
    const size_t vb = (((size_t)n * 8 + 255) / 256) * 256, sb = (rd::power_scratch_bytes() + 255) & ~(size_t)255;
    const size_t db = (((size_t)n + 2) * 4 + 255) & ~(size_t)255;
    rdist_status st;
    if ((st = ensure_grow(c, w.gb, 2 * vb + sb + db + 256))) return st;
    char *base = (char *)w.gb.p;
    double *x[2] = {(double *)base, (double *)(base + vb)};
    void *pw = base + 2 * vb;
    int32_t *outdeg = (int32_t *)(base + 2 * vb + sb), *badp = outdeg + n + 1;
    rdist_info *ginf = (rdist_info *)(base + 2 * vb + sb + db);
    std::vector<char> host(rd::power_scratch_bytes());
    // Delta and the input check (0/1 entries, no self-loop): the solve's gate
    rd::launch_gate(A_dev, n, -0.5, outdeg, badp, ginf, s);
    rd::launch_power_init(pw, s);
    rdist_info gi{};
    RD_HIP(hipMemcpyAsync(&gi, ginf, sizeof(rdist_info), hipMemcpyDeviceToHost, s));
    RD_HIP(hipStreamSynchronize(s));
    const int delta = gi.delta, bad = gi.status == RDIST_E_ADJ;
    const double u = 0x1p-53;
    double lo = 1.0, hi = HUGE_VAL;
    int k = 0;
    while (!bad && k < max_steps) {
        const int chunk = std::min(16, max_steps - k);
        for (int t = 0; t < chunk; ++t, ++k) rd::launch_power_step(A_dev, n, x[k & 1], x[(k & 1) ^ 1], pw, k, s);
        rd::launch_power_fold(pw, k - 1, s);
        RD_HIP(hipGetLastError());
        RD_HIP(hipMemcpyAsync(host.data(), pw, host.size(), hipMemcpyDeviceToHost, s));
        RD_HIP(hipStreamSynchronize(s));
        double lr, hr;
        rd::power_read(host.data(), &lr, &hr);
        // each ratio carries the rounding of a sum of at most Delta + 1 terms and a quotient
        const double m = (delta + 3) * u;
        lo = std::max(0.0, lr * (1.0 - m) - 1.0);
        hi = std::min((double)delta, hr * (1.0 + m) - 1.0);
        if (hi - lo <= rel_tol * hi) break;
    }
    rdist_gain_report r{};
    r.status = bad ? RDIST_E_ADJ : RDIST_OK;
    r.delta = delta;
    r.steps = k;
    const int d = diameter > 0 ? diameter : std::max(n - 1, 1);
    r.diameter = d;
    r.rho_lo = lo;
    r.rho_hi = std::max(lo, hi);
    r.gamma_c_lo = r.rho_hi > 0.0 ? 1.0 / r.rho_hi : HUGE_VAL;
    r.gamma_c_hi = r.rho_lo > 0.0 ? 1.0 / r.rho_lo : HUGE_VAL;
    r.gamma_gate = delta > 0 ? 1.0 / delta : HUGE_VAL;
    const double dd = (double)delta;
    r.gamma_global = delta > 0 ? 1.0 / (dd + std::pow(dd, (double)(d - 1))) : HUGE_VAL;
    r.gamma_tree = delta > 0 ? (-1.0 + std::sqrt(1.0 + 4.0 * dd * (d + 2))) / (2.0 * dd * (d + 2)) : HUGE_VAL;
    r.gamma_precision = std::exp(std::log(4.9406564584124654e-324) / (double)d);
    *out = r;
    return RDIST_OK;
}

rdist_status rdist_certify(rdist_ctx c, rdist_graph g, uint8_t *mask_dev, int64_t *n_certified, void *stream) {
    if (!c || !g || !n_certified) return fail(RDIST_E_ARG, "NULL argument");
    if (g->ctx != c) return fail(RDIST_E_STATE, "graph belongs to another context");
    Guard gd(c);
    RD_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    Workspace &w = c->ws[s];
    rdist_status st;
    if ((st = ensure_grow(c, w.rmisc, kRowsMisc))) return st;
    unsigned long long *cnt = (unsigned long long *)((char *)w.rmisc.p + kRowsFlag);
    rd::launch_fill_i32((int32_t *)cnt, 2, s);
    {
        Timer tm(c, s, RDIST_K_CERTIFY, 0.0, (8.0 + (mask_dev ? 1.0 : 0.0)) * (double)g->n * g->n);
        rd::launch_certify(g->Y, g->ld, g->n, g->ginfo, g->weighted != 0, g->changed ? rd::kBetaCap : 0.0, mask_dev,
                           cnt, s);
    }
    RD_HIP(hipGetLastError());
    unsigned long long h = 0;
    RD_HIP(hipMemcpyAsync(&h, cnt, 8, hipMemcpyDeviceToHost, s));
    RD_HIP(hipStreamSynchronize(s));
    *n_certified = (int64_t)h;
    return RDIST_OK;
}

rdist_status rdist_epilogue(rdist_ctx c, const double *Y_dev, int32_t n, int32_t ld, double gamma, int16_t *D_dev,
                            rdist_info *info, void *stream) {
    if (!c || !Y_dev || !D_dev) return fail(RDIST_E_ARG, "NULL argument");
    if (n < 1 || ld < n) return fail(RDIST_E_ARG, "bad n or ld");
    if (!(gamma > 0.0 && gamma < 1.0)) return fail(RDIST_E_ARG, "gamma must lie in (0, 1)");
    Guard g(c);
    RD_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    Workspace &w = c->ws[s];
    rdist_status st = ensure_small(c, w, 1);
    if (st) return st;
    rd::launch_info_set(w.dinfo(), gamma, s);
    {
        Timer t(c, s, RDIST_K_EPILOGUE, 0.0, 10.0 * n * (double)n);
        rd::launch_epilogue(Y_dev, n, ld, D_dev, w.dinfo(), s);
    }
    RD_HIP(hipGetLastError());
    return copy_info(info, w.dinfo(), 1, s);
}

rdist_status rdist_set_timing(rdist_ctx c, int enable) {
    if (!c) return fail(RDIST_E_ARG, "ctx is NULL");
    Guard g(c);
    if (enable < 0) return fail(RDIST_E_ARG, "negative timing mask");
    drain_timing(c);
    c->timing_mask = enable == 1 ? (1u << RDIST_K_COUNT) - 1 : ((uint32_t)enable >> 1) & ((1u << RDIST_K_COUNT) - 1);
    if (enable) std::memset(c->stats, 0, sizeof(c->stats));
    return RDIST_OK;
}

rdist_status rdist_timing_hold(rdist_ctx c, int hold) {
    if (!c) return fail(RDIST_E_ARG, "ctx is NULL");
    Guard g(c);
    c->timing_hold = hold != 0;
    return RDIST_OK;
}

rdist_status rdist_kernel_stats_get(rdist_ctx c, int which, rdist_kernel_stats *out) {
    if (!c || !out || which < 0 || which >= RDIST_K_COUNT) return fail(RDIST_E_ARG, "bad argument");
    Guard g(c);
    (void)hipSetDevice(c->device);
    drain_timing(c);
    *out = c->stats[which];
    return RDIST_OK;
}

size_t rdist_hbm_in_use(rdist_ctx c) { return c ? c->in_use : 0; }

}  // extern "C"
