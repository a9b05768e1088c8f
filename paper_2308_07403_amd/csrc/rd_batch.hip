// rd_batch.hip -- rdist_solve_batched: many independent graphs per call.
//
// A batch is split by size:
//   n <= T            the persistent kernel: each workgroup pulls whole graphs
//                     from a counter, longest first (register-resident
//                     Gauss-Jordan for n <= 128, an in-workgroup blocked solver
//                     up to 512);
//   T < n <= 4096     the level-synchronous plan: every such graph takes
//                     blocked step K in the same panel / row-column / update
//                     launches, so one graph's tiles spread over many compute
//                     units;
//   n > 4096          the single-graph blocked plan, one graph after another.
// The first two run concurrently (the persistent kernel on a forked stream).
// Their launch sequence is built once per distinct batch (sizes, pointers,
// gains, flags, stream), captured into a HIP graph and replayed on identical
// later calls.  T and the persistent kernel's grid are the tuned parameters:
// with a tile cache file the autotuner times the candidates on the first
// batch of each size class and records the fastest.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/rdist.h"
#include "rd_engine.h"
#include "rd_launch.h"

namespace rd {
namespace eng {

namespace {

constexpr int kMaxCachedPlans = 4;
constexpr int kXcds = 8;   // workgroup b of a launch runs on XCD b % 8

int np_of(int n) { return ((n + kB - 1) / kB) * kB; }

}  // namespace

struct BatchPlan {
    // what the plan was built for
    hipStream_t stream = nullptr;
    uint32_t flags = 0;
    std::vector<int32_t> n;
    std::vector<const uint8_t *> A;
    std::vector<double> gamma;
    std::vector<int16_t *> D;
    BatchTuning tune;
    // partition (original graph indices)
    std::vector<int> persist_ids, level_ids, big_ids;
    // device side
    Buf infos;      // rdist_info per graph, original order (entries of big graphs unused)
    Buf table;      // BatchTask[n_persist] | LevelGraph[n_level] | unit lists | counter
    Buf pool;       // matrices and step buffers (when Y is not kept)
    Buf scratch;    // per-workgroup scratch of the persistent kernel's blocked solver
    size_t off_level = 0, off_units = 0, off_counter = 0;
    size_t colsum_ints = 0;   // the level graphs' column sums at the start of the pool (zeroed by kFill)
    int persist_grid = 0;
    int persist_stride = 0;
    // launch program: kernel launches, event records and waits on three
    // streams (0: the caller's, 1: lookahead, 2: persistent kernel)
    // kMark (eager launches with marks only): records marks[K] on the op's
    // stream once the graphs of completion group K are final (group 0: the
    // persistent kernel's graphs; group t >= 1: the level graphs with nt = t)
    enum OpKind { kLaunch = 0, kIngest = 1, kPersist = 2, kRecord = 3, kWait = 4, kFill = 5, kMark = 6 };
    struct Op {
        int kind, stream, phase, K, offset, grid, event;
        double flops = 0.0, bytes = 0.0;   // update launches: algorithmic work, for per-kernel timing
    };
    std::vector<Op> ops;
    double flops = 0.0, bytes = 0.0;
    // host staging of the table (pinned), reused when the plan is rebuilt
    void *staging = nullptr;
    size_t staging_bytes = 0;
    hipEvent_t ev_upload = nullptr;
    // recorded after every launch of the captured graph: eviction waits for
    // it, not for the caller's stream, which may be gone by then
    hipEvent_t ev_done = nullptr;
    bool launched = false;
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};   // fork, join, edge done, row tiles done, diagonal done
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;

    bool matches(hipStream_t s, uint32_t f, int count, const int32_t *n_, const uint8_t *const *A_, const double *g_,
                 int16_t *const *D_, const BatchTuning &t) const {
        if (s != stream || f != flags || (int)n.size() != count) return false;
        if (t.persist_max_n != tune.persist_max_n || t.persist_grid != tune.persist_grid) return false;
        for (int i = 0; i < count; ++i)
            if (n[i] != n_[i] || A[i] != A_[i] || gamma[i] != g_[i] || D[i] != D_[i]) return false;
        return true;
    }
};

rdist_status ensure_capture_streams(rdist_ctx c) {
    if (!c->capture) RD_HIP(hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking));
    if (!c->capture_aux) RD_HIP(hipStreamCreateWithFlags(&c->capture_aux, hipStreamNonBlocking));
    if (!c->capture_aux2) RD_HIP(hipStreamCreateWithFlags(&c->capture_aux2, hipStreamNonBlocking));
    return RDIST_OK;
}

namespace {

// Frees a plan once its last graph launch and its table upload have
// finished (a transient plan's eager launches are the caller's to wait for).
void free_plan(rdist_ctx c, BatchPlan *p) {
    if (!p) return;
    if (p->ev_done) {
        if (p->launched) (void)hipEventSynchronize(p->ev_done);
        (void)hipEventDestroy(p->ev_done);
    }
    if (p->ev_upload) {
        (void)hipEventSynchronize(p->ev_upload);
        (void)hipEventDestroy(p->ev_upload);
    }
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    for (Buf *b : {&p->infos, &p->table, &p->pool, &p->scratch}) release(c, *b);
    if (p->staging) (void)hipHostFree(p->staging);
    for (hipEvent_t e : p->ev)
        if (e) (void)hipEventDestroy(e);
    delete p;
}

// Assigns the items of one launch to workgroups.  A graph's items are cut
// into contiguous runs of at most kRunItems (items are numbered tile-row
// major, so a run shares its rows' operand slab); runs are placed longest
// first on the least loaded XCD, and the XCD lists are interleaved so that
// workgroup b takes an item of XCD b % 8.  A small graph is one run on one
// XCD; a large one spreads over all of them.
constexpr int kRunItems = 64;
int build_units(const std::vector<std::pair<int, int>> &graph_items, std::vector<int> &units) {
    struct Run { int g, first, count; };
    std::vector<Run> runs;
    for (const auto &gi : graph_items) {
        const int items = gi.second, parts = (items + kRunItems - 1) / kRunItems;
        const int per = (items + parts - 1) / parts;
        for (int f = 0; f < items; f += per) runs.push_back(Run{gi.first, f, std::min(per, items - f)});
    }
    std::stable_sort(runs.begin(), runs.end(), [](const Run &a, const Run &b) { return a.count > b.count; });
    std::vector<std::vector<int>> lists(kXcds);
    std::vector<size_t> load(kXcds, 0);
    for (const Run &r : runs) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        for (int it = r.first; it < r.first + r.count; ++it) lists[x].push_back((r.g << rd::kLvShift) | it);
        load[x] += r.count;
    }
    size_t slots = 0;
    for (auto &l : lists) slots = std::max(slots, l.size());
    for (size_t sl = 0; sl < slots; ++sl)
        for (int x = 0; x < kXcds; ++x) units.push_back(sl < lists[x].size() ? lists[x][sl] : -1);
    return (int)(slots * kXcds);
}

// Row-chunk height of the level plan's column sums: about 64 KB of A per
// workgroup.
int colsum_rows(int n) { return std::max(1, (65536 + n - 1) / n); }

// Builds the plan's tables and buffers for the batch.  ys (keep_y only):
// per-graph Y buffers, allocated here and handed to the graph handles after
// the launch; the persistent graphs' Y has leading dimension np.  ext_y
// (nullable): caller-owned Y buffers (np x np, ld np) instead, for the
// graphs whose entry is non-null; nothing is allocated for them.
rdist_status build_plan(rdist_ctx c, BatchPlan &p, hipStream_t s, uint32_t flags, int count, const int32_t *n,
                        const uint8_t *const *A, const double *gamma, int16_t *const *D, const BatchTuning &tune,
                        bool keep_y, std::vector<Buf> &ys, double *const *ext_y = nullptr) {
    rdist_status st;
    p.stream = s;
    p.flags = flags;
    p.n.assign(n, n + count);
    p.A.assign(A, A + count);
    p.gamma.assign(gamma, gamma + count);
    p.D.assign(D, D + count);
    p.tune = tune;
    p.persist_ids.clear();
    p.level_ids.clear();
    p.big_ids.clear();
    p.ops.clear();
    for (int g = 0; g < count; ++g) {
        if (n[g] > kBatchMaxN) p.big_ids.push_back(g);
        else if (n[g] <= tune.persist_max_n) p.persist_ids.push_back(g);
        else p.level_ids.push_back(g);
    }
    auto by_n = [&](int a, int b) { return n[a] > n[b]; };
    std::stable_sort(p.persist_ids.begin(), p.persist_ids.end(), by_n);
    std::stable_sort(p.level_ids.begin(), p.level_ids.end(), by_n);
    const int np_ = (int)p.persist_ids.size(), nl = (int)p.level_ids.size();

    if ((st = ensure_grow(c, p.infos, sizeof(rdist_info) * (size_t)count))) return st;
    rdist_info *dinfo = (rdist_info *)p.infos.p;

    // device memory: matrices (unless kept), level step buffers and column
    // sums, scratch
    auto kept = [&](int g) { return keep_y || (ext_y && ext_y[g]); };
    p.colsum_ints = 0;
    for (int g : p.level_ids) p.colsum_ints += (size_t)n[g] + 1;
    if (p.colsum_ints > (size_t)INT32_MAX) return fail(RDIST_E_NOMEM, "batch too large for one plan");
    const size_t colsum_doubles = ((p.colsum_ints + 1) / 2 + 31) / 32 * 32;
    size_t pool = colsum_doubles;
    for (int g : p.persist_ids)
        if (!kept(g) && n[g] > 128) pool += (size_t)np_of(n[g]) * np_of(n[g]);
    for (int g : p.level_ids) {
        const size_t q = np_of(n[g]);
        pool += (kept(g) ? 0 : q * q) + 2 * (2 * (size_t)kB * q + (size_t)kB * kB);
    }
    if (pool && (st = ensure_grow(c, p.pool, pool * 8))) return st;
    bool persist_medium = false;
    for (int g : p.persist_ids) persist_medium |= n[g] > 128;
    // default grid: half the compute units, so that the level plan's
    // launches keep most of the device while it runs
    const int grid_default = std::max(1, c->num_cu / 2);
    p.persist_grid = std::max(1, std::min(np_, tune.persist_grid > 0 ? tune.persist_grid : grid_default));
    p.persist_stride = 2 * kB * kPersistMaxN + kB * kB;
    if (np_ && persist_medium &&
        (st = ensure_grow(c, p.scratch, (size_t)p.persist_grid * p.persist_stride * 8)))
        return st;
    if (keep_y) {
        ys.assign(count, Buf{});
        for (int g : p.persist_ids) ys[g].bytes = (size_t)np_of(n[g]) * np_of(n[g]) * 8;
        for (int g : p.level_ids) ys[g].bytes = (size_t)np_of(n[g]) * np_of(n[g]) * 8;
        for (int g = 0; g < count; ++g) {
            if (!ys[g].bytes) continue;
            const size_t b = ys[g].bytes;
            ys[g].bytes = 0;
            if ((st = dalloc(c, &ys[g].p, b))) {
                for (Buf &y : ys) release(c, y);
                return st;
            }
            ys[g].bytes = b;
        }
    }

    // host tables
    std::vector<rd::BatchTask> tasks(np_);
    std::vector<rd::LevelGraph> lgs(nl);
    int32_t *cs = (int32_t *)p.pool.p;
    double *cur = (double *)p.pool.p + colsum_doubles;
    p.flops = p.bytes = 0.0;
    for (int q = 0; q < np_; ++q) {
        const int g = p.persist_ids[q], npg = np_of(n[g]);
        double *M = nullptr;
        if (ext_y && ext_y[g]) M = ext_y[g];
        else if (keep_y) M = (double *)ys[g].p;
        else if (n[g] > 128) { M = cur; cur += (size_t)npg * npg; }
        tasks[q] = rd::BatchTask{A[g], D[g], M, nullptr, nullptr, nullptr, n[g], npg, kept(g) ? 1 : 0, 0, gamma[g],
                                 dinfo + g};
    }
    for (int q = 0; q < nl; ++q) {
        const int g = p.level_ids[q], npg = np_of(n[g]);
        rd::LevelGraph &L = lgs[q];
        if (ext_y && ext_y[g]) L.M = ext_y[g];
        else if (keep_y) L.M = (double *)ys[g].p;
        else { L.M = cur; cur += (size_t)npg * npg; }
        for (int par = 0; par < 2; ++par) {
            L.Ut[par] = cur;
            L.V[par] = cur + (size_t)kB * npg;
            L.Pt[par] = cur + 2 * (size_t)kB * npg;
            cur += 2 * (size_t)kB * npg + (size_t)kB * kB;
        }
        L.colsum = cs;
        cs += n[g] + 1;
        L.rows_per = colsum_rows(n[g]);
        L.nchunk = (n[g] + L.rows_per - 1) / L.rows_per;
        L.A = A[g];
        L.D = D[g];
        L.info = dinfo + g;
        L.n = n[g];
        L.np = npg;
        L.nt = npg / kB;
        L.keep = kept(g) ? 1 : 0;
        L.gamma_arg = gamma[g];
    }
    for (int g : p.persist_ids) {
        p.flops += 2.0 * n[g] * (double)n[g] * n[g];
        p.bytes += 3.0 * n[g] * (double)n[g];
    }
    for (int g : p.level_ids) {
        p.flops += 2.0 * n[g] * (double)n[g] * n[g];
        p.bytes += 3.0 * n[g] * (double)n[g];
    }

    // launch program
    using Op = BatchPlan::Op;
    std::vector<int> units;
    // update launches: per graph, the tiles that take a product (block row K
    // is a copy) at 2 * 128^2 * kd flops, and the tile's 256 KiB of old and
    // new value
    auto update_work = [](const rd::LevelGraph &L, int phase, int K, double &fl, double &by) {
        const int nt = L.nt;
        const bool last = K + 1 == nt;
        const double kd = last ? rd::lv_last_inner(L.n, nt) : kB;
        int prod = 0, all = 0;
        if (phase == rd::kLvDiag) { prod = 1; all = 1; }
        else if (phase == rd::kLvEdge) { all = 2 * nt - 2; prod = all - 1; }
        else if (!last) { all = (nt - 1) * (nt - 1); prod = all - (nt - 1); }
        else { all = nt * nt; prod = all - nt; }
        fl += prod * 2.0 * kB * kB * kd;
        by += all * 2.0 * kB * kB * 8.0;
    };
    auto launch = [&](int stream, int phase, int K, auto items_of) {
        std::vector<std::pair<int, int>> gi;
        double fl = 0.0, by = 0.0;
        const bool upd = phase == rd::kLvDiag || phase == rd::kLvEdge || phase == rd::kLvRest;
        for (int q = 0; q < nl; ++q) {
            const int it = items_of(lgs[q]);
            if (it > 0) {
                gi.emplace_back(q, it);
                if (upd) update_work(lgs[q], phase, K, fl, by);
            }
        }
        const int off = (int)units.size();
        const int grid = build_units(gi, units);
        if (grid) {
            Op o{BatchPlan::kLaunch, stream, phase, K, off, grid, 0};
            o.flops = fl;
            o.bytes = by;
            p.ops.push_back(o);
        }
    };
    auto record = [&](int stream, int ev) { p.ops.push_back(Op{BatchPlan::kRecord, stream, 0, 0, 0, 0, ev}); };
    auto wait = [&](int stream, int ev) { p.ops.push_back(Op{BatchPlan::kWait, stream, 0, 0, 0, 0, ev}); };
    // the persistent kernel forks off first: its graphs run beside the
    // level plan's ingest and build, which are bound by HBM and atomics
    using LG = rd::LevelGraph;
    if (np_ && nl) {
        record(0, 0);
        wait(2, 0);
    }
    if (np_) p.ops.push_back(Op{BatchPlan::kPersist, nl ? 2 : 0, 0, 0, 0, p.persist_grid, 0});
    if (nl) {
        p.ops.push_back(Op{BatchPlan::kFill, 0, 0, 0, 0, 0, 0});       // zero the column sums
        launch(0, rd::kLvColsum, 0, [](const LG &L) { return L.nchunk; });
        p.ops.push_back(Op{BatchPlan::kIngest, 0, 0, 0, 0, nl, 0});   // the gate
        launch(0, rd::kLvBuild, 0, [](const LG &L) { return 2 * L.nt - 1; });
    }
    if (np_) p.ops.push_back(Op{BatchPlan::kMark, nl ? 2 : 0, 0, 0, 0, 0, 0});
    if (np_ && nl) record(2, 1);
    if (nl) {
        launch(0, rd::kLvPanel, 0, [](const LG &) { return 1; });
        launch(0, rd::kLvRowcol, 0, [](const LG &L) { return L.nt - 1; });
        const int max_nt = lgs[0].nt;
        for (int K = 0; K < max_nt; ++K) {
            if (K > 0) wait(0, 3);                       // step K's row/column tiles are ready
            const bool next = max_nt > K + 1;
            if (next) {
                // the next diagonal tiles first, so that the next panels
                // start while the rest of the band is updated
                launch(0, rd::kLvDiag, K, [K](const LG &L) { return L.nt > K + 1 ? 1 : 0; });
                record(0, 4);
                launch(0, rd::kLvEdge, K, [K](const LG &L) { return L.nt > K + 1 ? 2 * L.nt - 2 : 0; });
                record(0, 2);
            }
            launch(0, rd::kLvRest, K, [K](const LG &L) {
                return L.nt > K + 1 ? (L.nt - 1) * (L.nt - 1) : L.nt == K + 1 ? L.nt * L.nt : 0;
            });
            p.ops.push_back(Op{BatchPlan::kMark, 0, 0, K + 1, 0, 0, 0});   // graphs with nt = K + 1 are final
            if (next) {
                wait(1, 4);
                launch(1, rd::kLvPanel, K + 1, [K](const LG &L) { return L.nt > K + 1 ? 1 : 0; });
                wait(1, 2);
                launch(1, rd::kLvRowcol, K + 1, [K](const LG &L) { return L.nt > K + 1 ? L.nt - 1 : 0; });
                record(1, 3);
            }
        }
    }
    if (np_ && nl) wait(0, 1);

    // one table: tasks | level graphs | units | counter
    auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
    p.off_level = align(sizeof(rd::BatchTask) * tasks.size());
    p.off_units = p.off_level + align(sizeof(rd::LevelGraph) * lgs.size());
    p.off_counter = p.off_units + align(sizeof(int) * units.size());
    const size_t tbytes = p.off_counter + 256;
    if ((st = ensure_grow(c, p.table, tbytes))) return st;
    if (!p.ev_upload) RD_HIP(hipEventCreateWithFlags(&p.ev_upload, hipEventDisableTiming));
    else RD_HIP(hipEventSynchronize(p.ev_upload));   // the previous upload has left the staging buffer
    if (p.staging_bytes < tbytes) {
        if (p.staging) (void)hipHostFree(p.staging);
        p.staging = nullptr;
        p.staging_bytes = 0;
        RD_HIP(hipHostMalloc(&p.staging, tbytes, hipHostMallocDefault));
        p.staging_bytes = tbytes;
    }
    char *h = (char *)p.staging;
    std::memset(h, 0, tbytes);
    if (!tasks.empty()) std::memcpy(h, tasks.data(), sizeof(rd::BatchTask) * tasks.size());
    if (!lgs.empty()) std::memcpy(h + p.off_level, lgs.data(), sizeof(rd::LevelGraph) * lgs.size());
    if (!units.empty()) std::memcpy(h + p.off_units, units.data(), sizeof(int) * units.size());
    RD_HIP(hipMemcpyAsync(p.table.p, h, tbytes, hipMemcpyHostToDevice, s));
    RD_HIP(hipEventRecord(p.ev_upload, s));
    for (hipEvent_t &e : p.ev)
        if (!e) RD_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return RDIST_OK;
}

// Runs the plan's launch program on the streams st[0] (the caller's),
// st[1] (lookahead) and st[2] (persistent kernel).  timed (eager launches
// only): the context whose per-kernel timing records the update launches
// (RDIST_K_UPDATE_EDGE for the diagonal and edge tiles, RDIST_K_UPDATE for
// the rest).
rdist_status enqueue_plan(BatchPlan &p, const hipStream_t st[3], hipEvent_t *marks = nullptr,
                          rdist_ctx timed = nullptr) {
    char *t = (char *)p.table.p;
    const rd::LevelGraph *lgs = (const rd::LevelGraph *)(t + p.off_level);
    const int *units = (const int *)(t + p.off_units);
    for (const BatchPlan::Op &o : p.ops) {
        hipStream_t s = st[o.stream];
        switch (o.kind) {
            case BatchPlan::kLaunch:
                if (timed && (o.phase == rd::kLvDiag || o.phase == rd::kLvEdge || o.phase == rd::kLvRest)) {
                    Timer tm(timed, s, o.phase == rd::kLvRest ? RDIST_K_UPDATE : RDIST_K_UPDATE_EDGE, o.flops,
                             o.bytes);
                    rd::launch_lv(o.phase, lgs, units + o.offset, o.grid, o.K, s);
                } else {
                    rd::launch_lv(o.phase, lgs, units + o.offset, o.grid, o.K, s);
                }
                break;
            case BatchPlan::kIngest: rd::launch_lv_gate(lgs, o.grid, s); break;
            case BatchPlan::kFill: rd::launch_fill_i32((int32_t *)p.pool.p, p.colsum_ints, s); break;
            case BatchPlan::kPersist:
                rd::launch_batched((const rd::BatchTask *)t, (int)p.persist_ids.size(), (int *)(t + p.off_counter),
                                   o.grid, (double *)p.scratch.p, p.persist_stride, s);
                break;
            case BatchPlan::kRecord: RD_HIP(hipEventRecord(p.ev[o.event], s)); break;
            case BatchPlan::kMark:
                if (marks) RD_HIP(hipEventRecord(marks[o.K], s));
                break;
            case BatchPlan::kWait: RD_HIP(hipStreamWaitEvent(s, p.ev[o.event], 0)); break;
        }
    }
    RD_HIP(hipGetLastError());
    return RDIST_OK;
}

// Records the plan's launches into a HIP graph (captured on the context's
// own streams, so the caller's stream may be the null stream).
rdist_status capture_plan(rdist_ctx c, BatchPlan &p) {
    rdist_status st;
    if ((st = ensure_capture_streams(c))) return st;
    RD_HIP(hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal));
    const hipStream_t sts[3] = {c->capture, c->capture_aux, c->capture_aux2};
    st = enqueue_plan(p, sts);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->capture, &g);
    if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(RDIST_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    p.graph = g;
    RD_HIP(hipGraphInstantiate(&p.exec, p.graph, nullptr, nullptr, 0));
    return RDIST_OK;
}

// ---- autotuner ----

// Size class of a batch: count rounded up to a power of two, and the share
// of graphs in each size bucket in sixteenths.
std::string batch_class(int count, const int32_t *n) {
    int cnt[5] = {0, 0, 0, 0, 0};
    for (int g = 0; g < count; ++g) {
        const int v = n[g];
        cnt[v <= 64 ? 0 : v <= 128 ? 1 : v <= 256 ? 2 : v <= 512 ? 3 : 4]++;
    }
    int c2 = 1;
    while (c2 < count) c2 <<= 1;
    std::ostringstream os;
    os << "count" << c2;
    for (int b = 0; b < 5; ++b) os << ":" << (cnt[b] * 16 + count / 2) / count;
    return os.str();
}

const BatchTuning *find_tuning(rdist_ctx c, const std::string &cls) {
    for (auto &kv : c->tuned)
        if (kv.first == cls) return &kv.second;
    return nullptr;
}

// Times every candidate (persistent/level threshold x persistent grid) on
// this batch with eager launches on s and keeps the fastest.  Blocks the
// host until the trial runs finish.
rdist_status autotune(rdist_ctx c, hipStream_t s, uint32_t flags, int count, const int32_t *n,
                      const uint8_t *const *A, const double *gamma, int16_t *const *D, BatchTuning &best) {
    Workspace &w = c->ws[s];
    rdist_status st;
    if ((st = ensure_aux(w))) return st;
    if ((st = ensure_aux2(w))) return st;
    if (!w.transient) w.transient = new BatchPlan();
    BatchPlan &p = *w.transient;
    hipEvent_t e0 = take_event(c), e1 = take_event(c);
    if (!e0 || !e1) return fail(RDIST_E_HIP, "hipEventCreate failed");
    float best_ms = 1e30f;
    std::vector<Buf> none;
    const int base = c->num_cu;
    for (int T : {128, 256, 512})
        for (int grid : {base / 8, base / 4, base / 2, base}) {   // base: one workgroup per compute unit
            BatchTuning cand{T, grid};
            if ((st = build_plan(c, p, s, flags, count, n, A, gamma, D, cand, false, none))) break;
            const hipStream_t sts[3] = {s, w.aux, w.aux2};
            if ((st = enqueue_plan(p, sts))) break;   // warm-up
            RD_HIP(hipEventRecord(e0, s));
            for (int r = 0; r < 3 && !st; ++r) st = enqueue_plan(p, sts);
            if (st) break;
            RD_HIP(hipEventRecord(e1, s));
            RD_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            RD_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best_ms) {
                best_ms = ms;
                best = cand;
            }
        }
    c->event_pool.push_back(e0);
    c->event_pool.push_back(e1);
    return st;
}

BatchPlan *lookup_plan(rdist_ctx c, hipStream_t s, uint32_t flags, int count, const int32_t *n,
                       const uint8_t *const *A, const double *gamma, int16_t *const *D, const BatchTuning &tune) {
    for (BatchPlan *p : c->plans)
        if (p->matches(s, flags, count, n, A, gamma, D, tune)) return p;
    return nullptr;
}

}  // namespace

void free_transient_plan(rdist_ctx c, Workspace &w) {
    free_plan(c, w.transient);
    w.transient = nullptr;
}

void destroy_plans(rdist_ctx c) {
    for (BatchPlan *p : c->plans) free_plan(c, p);
    c->plans.clear();
    for (auto &kv : c->ws) free_transient_plan(c, kv.second);
    if (c->capture) (void)hipStreamDestroy(c->capture);
    if (c->capture_aux) (void)hipStreamDestroy(c->capture_aux);
    if (c->capture_aux2) (void)hipStreamDestroy(c->capture_aux2);
    c->capture = c->capture_aux = c->capture_aux2 = nullptr;
}

// Tile cache file: {"batched": [{"class": "...", "persist_max_n": T,
// "persist_grid": G}, ...]}, written by save_tile_cache.
void load_tile_cache(rdist_ctx c) {
    std::ifstream f(c->tile_cache_path);
    if (!f) return;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string t = ss.str();
    size_t pos = 0;
    while ((pos = t.find("\"class\"", pos)) != std::string::npos) {
        const size_t q0 = t.find('"', t.find(':', pos) + 1);
        const size_t q1 = q0 == std::string::npos ? q0 : t.find('"', q0 + 1);
        if (q1 == std::string::npos) break;
        const std::string cls = t.substr(q0 + 1, q1 - q0 - 1);
        const size_t end = t.find('}', q1);
        auto num = [&](const char *key, int &out) {
            const size_t k = t.find(key, q1);
            if (k == std::string::npos || k > end) return false;
            out = std::atoi(t.c_str() + t.find(':', k) + 1);
            return true;
        };
        BatchTuning bt;
        if (num("\"persist_max_n\"", bt.persist_max_n) && num("\"persist_grid\"", bt.persist_grid) &&
            (bt.persist_max_n == 128 || bt.persist_max_n == 256 || bt.persist_max_n == 512) && bt.persist_grid >= 0 &&
            !find_tuning(c, cls))
            c->tuned.emplace_back(cls, bt);
        pos = q1;
    }
}

void save_tile_cache(rdist_ctx c) {
    if (c->tile_cache_path.empty()) return;
    std::ofstream f(c->tile_cache_path, std::ios::trunc);
    if (!f) return;
    f << "{\"batched\": [";
    for (size_t i = 0; i < c->tuned.size(); ++i) {
        const auto &kv = c->tuned[i];
        f << (i ? ",\n  " : "\n  ") << "{\"class\": \"" << kv.first << "\", \"persist_max_n\": "
          << kv.second.persist_max_n << ", \"persist_grid\": " << kv.second.persist_grid << "}";
    }
    f << "\n]}\n";
    c->tuned_dirty = false;
}

rdist_status solve_batch_into(rdist_ctx c, hipStream_t s, int count, const int32_t *n, const uint8_t *const *A,
                              const double *gamma, int16_t *const *D, double *const *ext_y, rdist_info *info_host,
                              hipEvent_t *marks, hipStream_t *tail, const rdist_info **info_dev) {
    for (int g = 0; g < count; ++g)
        if (n[g] < 1 || n[g] > kBatchMaxN) return fail(RDIST_E_ARG, "n out of the batched range");
    Workspace &w = c->ws[s];
    rdist_status st;
    if ((st = ensure_aux(w))) return st;
    if ((st = ensure_aux2(w))) return st;
    // the default threshold T = 128 whatever the batch, so that a graph's
    // arithmetic never depends on what it is batched with
    const BatchTuning tune;
    if (!w.transient) w.transient = new BatchPlan();
    BatchPlan &p = *w.transient;
    std::vector<Buf> none;
    if ((st = build_plan(c, p, s, RDIST_F64, count, n, A, gamma, D, tune, false, none, ext_y))) return st;
    {
        Timer tm(c, s, RDIST_K_BATCHED, p.flops, p.bytes);
        const hipStream_t sts[3] = {s, w.aux, w.aux2};
        if ((st = enqueue_plan(p, sts, marks))) return st;
    }
    if (tail) *tail = w.aux2;
    if (info_dev) *info_dev = (const rdist_info *)p.infos.p;
    if (info_host)
        RD_HIP(hipMemcpyAsync(info_host, p.infos.p, sizeof(rdist_info) * (size_t)count, hipMemcpyDeviceToHost, s));
    return RDIST_OK;
}

}  // namespace eng
}  // namespace rd

using namespace rd::eng;

extern "C" rdist_status rdist_solve_batched(rdist_ctx c, int32_t count, const int32_t *n,
                                            const uint8_t *const *A_dev, const double *gamma, uint32_t flags,
                                            int16_t *const *D_dev, rdist_graph *keep, rdist_info *info,
                                            void *stream) {
    if (!c) return fail(RDIST_E_ARG, "ctx is NULL");
    if (count < 0) return fail(RDIST_E_ARG, "count < 0");
    if (count == 0) return RDIST_OK;
    if (!n || !A_dev || !gamma || !D_dev) return fail(RDIST_E_ARG, "NULL array");
    rdist_status st;
    if ((st = check_flags(flags))) return st;
    if (flags & (RDIST_PLAN_SMALL | RDIST_PLAN_BLOCKED)) return fail(RDIST_E_ARG, "plan flags are per solve");
    if (flags & RDIST_MIXED_F32) return fail(RDIST_E_ARG, "RDIST_MIXED_F32 is a single-graph plan");
    if (flags & RDIST_WEIGHTED) return fail(RDIST_E_ARG, "RDIST_WEIGHTED is a single-graph plan");
    if (count > (1 << 20)) return fail(RDIST_E_ARG, "count too large (at most 2^20 graphs per call)");
    for (int g = 0; g < count; ++g) {
        if (n[g] < 1 || n[g] > 65536) return fail(RDIST_E_ARG, "n out of range");
        if (!A_dev[g] || !D_dev[g]) return fail(RDIST_E_ARG, "NULL graph pointer");
        if ((st = check_gamma(gamma[g]))) return st;
    }
    const bool keep_y = (flags & RDIST_KEEP_Y) && keep;
    if (keep) for (int g = 0; g < count; ++g) keep[g] = nullptr;
    Guard gd(c);
    RD_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    Workspace &w = c->ws[s];
    if ((st = ensure_aux(w))) return st;
    if ((st = ensure_aux2(w))) return st;

    BatchTuning tune;
    {
        const std::string cls = batch_class(count, n);
        const BatchTuning *t = find_tuning(c, cls);
        if (t) {
            tune = *t;
        } else if (!c->tile_cache_path.empty() && !keep_y) {
            if ((st = autotune(c, s, flags, count, n, A_dev, gamma, D_dev, tune))) return st;
            c->tuned.emplace_back(cls, tune);
            c->tuned_dirty = true;
            save_tile_cache(c);
        }
    }

    // cached plan with its graph, or a transient plan launched eagerly
    BatchPlan *p = nullptr;
    std::vector<Buf> ys;
    const bool use_graph = !keep_y && !(flags & RDIST_NO_GRAPH);
    if (use_graph) {
        // the tuning is part of the key: a plan built under another tuning
        // never matches and ages out of the cache
        p = lookup_plan(c, s, flags, count, n, A_dev, gamma, D_dev, tune);
        if (!p) {
            if ((int)c->plans.size() >= kMaxCachedPlans) {
                auto it = std::min_element(c->plans.begin(), c->plans.end(),
                                           [](BatchPlan *a, BatchPlan *b) { return a->last_use < b->last_use; });
                free_plan(c, *it);   // waits on the plan's own events, never on its stream
                c->plans.erase(it);
            }
            p = new BatchPlan();
            st = build_plan(c, *p, s, flags, count, n, A_dev, gamma, D_dev, tune, false, ys);
            if (!st && !p->ev_done) {
                const hipError_t e = hipEventCreateWithFlags(&p->ev_done, hipEventDisableTiming);
                if (e != hipSuccess) {
                    p->ev_done = nullptr;
                    st = fail(RDIST_E_HIP, std::string("hipEventCreateWithFlags: ") + hipGetErrorString(e));
                }
            }
            if (!st) st = capture_plan(c, *p);
            if (st) {
                free_plan(c, p);
                return st;
            }
            c->plans.push_back(p);
        }
        p->last_use = ++c->plan_clock;
    } else {
        if (!w.transient) w.transient = new BatchPlan();
        p = w.transient;
        if ((st = build_plan(c, *p, s, flags, count, n, A_dev, gamma, D_dev, tune, keep_y, ys))) return st;
    }

    if (!p->persist_ids.empty() || !p->level_ids.empty()) {
        Timer tm(c, s, RDIST_K_BATCHED, p->flops, p->bytes);
        if (p->exec) {
            RD_HIP(hipGraphLaunch(p->exec, s));
            RD_HIP(hipEventRecord(p->ev_done, s));
            p->launched = true;
        } else {
            const hipStream_t sts[3] = {s, w.aux, w.aux2};
            if ((st = enqueue_plan(*p, sts, nullptr, c))) return st;
        }
    }
    if (info && (!p->persist_ids.empty() || !p->level_ids.empty()))
        RD_HIP(hipMemcpyAsync(info, p->infos.p, sizeof(rdist_info) * (size_t)count, hipMemcpyDeviceToHost, s));
    if (keep_y) {
        for (int g = 0; g < count; ++g) {
            if (!ys[g].p) continue;
            Buf y = ys[g];
            ys[g] = Buf{};
            if ((st = make_graph(c, n[g], (double *)y.p, np_of(n[g]), y.bytes, A_dev[g], s, &keep[g],
                                 (const rdist_info *)p->infos.p + g, false))) {
                release(c, y);
                for (Buf &b : ys) release(c, b);
                return st;
            }
        }
    }
    // graphs above the batched range, one after another (their info entries
    // are copied after the batch's, so they are the ones that stay)
    for (int g : p->big_ids) {
        st = solve_blocked(c, A_dev[g], n[g], gamma[g], flags & ~RDIST_NO_GRAPH, D_dev[g], keep ? &keep[g] : nullptr,
                           info ? info + g : nullptr, s);
        if (st) return st;
    }
    return RDIST_OK;
}
