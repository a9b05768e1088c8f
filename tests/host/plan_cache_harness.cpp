// Host harness of the batched plans' host logic (rd_batch.hip with
// rd_host.cpp), built with g++ against the HIP stand-in in this folder and
// run under AddressSanitizer by tests/test_host_plan_cache.py.
//
// Stand-ins of the kernel launchers check, when the work runs (eagerly or in
// a graph replay), that every table, workspace and caller buffer a launch
// names is live and large enough, and touch them, so that a plan replayed
// after its memory was freed, or a table pointing at freed memory, is caught.
// Caller buffers come from a pool that re-issues freed addresses for the same
// size, as a caching allocator does, so pointer-keyed plan lookups see
// recurring pointers.
//
// Scenarios: captured plans matched, replayed and evicted across more
// batches than the cache holds; eager and kept-Y transient plans growing and
// shrinking; a tuning change between calls (the new plan must be captured
// once, then replayed); the autotuner; a caller stream destroyed while a plan
// built on it is still cached; and at the end every device byte returned.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <random>
#include <set>
#include <string>
#include <vector>

#include "../../include/rdist.h"
#include "../../paper_2308_07403_amd/csrc/rd_engine.h"
#include "../../paper_2308_07403_amd/csrc/rd_launch.h"

namespace {

[[noreturn]] void die(const std::string &msg) {
    std::fprintf(stderr, "harness: %s\n", msg.c_str());
    std::fflush(stderr);
    std::abort();
}

// Caller memory with a caching allocator's address reuse.
struct UserPool {
    std::map<size_t, std::vector<void *>> free_lists;
    std::map<const void *, size_t> live;
    std::vector<void *> all;
    void *get(size_t bytes) {
        auto &fl = free_lists[bytes];
        void *p;
        if (!fl.empty()) {
            p = fl.back();
            fl.pop_back();
        } else {
            p = std::malloc(bytes);
            all.push_back(p);
        }
        live[p] = bytes;
        return p;
    }
    void put(void *p) {
        auto it = live.find(p);
        if (it == live.end()) die("user pool: double free");
        free_lists[it->second].push_back(p);
        live.erase(it);
    }
    bool ok(const void *p, size_t bytes) const {
        auto it = live.find(p);
        return it != live.end() && it->second >= bytes;
    }
    ~UserPool() {
        for (void *p : all) std::free(p);
    }
} g_user;

long g_kernel_items = 0;

int np_of(int n) { return (n + 127) / 128 * 128; }

void need_dev(const void *p, size_t bytes, const char *what) {
    if (!hipstub::device_range_live(p, bytes)) die(std::string(what) + ": not inside a live device allocation");
}

void need_user(const void *p, size_t bytes, const char *what) {
    if (!g_user.ok(p, bytes)) die(std::string(what) + ": caller buffer is not live");
}

void touch_user(const uint8_t *A, int16_t *D, int n) {
    volatile uint8_t a = A[(size_t)n * n - 1];
    (void)a;
    D[0] = (int16_t)7;
    D[(size_t)n * n - 1] = (int16_t)7;
}

void check_level_graph(const rd::LevelGraph &L) {
    const int n = L.n, np = L.np;
    if (n < 1 || n > rd::kLvMaxN || np != np_of(n) || L.nt != np / 128) die("level graph: inconsistent sizes");
    if (L.rows_per < 1 || (size_t)L.rows_per * L.nchunk < (size_t)n) die("level graph: row chunks do not cover A");
    need_user(L.A, (size_t)n * n, "level graph A");
    need_user(L.D, (size_t)n * n * 2, "level graph D");
    need_dev(L.M, (size_t)np * np * 8, "level graph M");
    for (int par = 0; par < 2; ++par) {
        need_dev(L.Ut[par], (size_t)128 * np * 8, "level graph Ut");
        need_dev(L.V[par], (size_t)128 * np * 8, "level graph V");
        need_dev(L.Pt[par], (size_t)128 * 128 * 8, "level graph Pt");
    }
    need_dev(L.colsum, (size_t)(n + 1) * 4, "level graph column sums");
    need_dev(L.info, sizeof(rdist_info), "level graph info");
    touch_user(L.A, L.D, n);
    L.M[0] = 1.0;
    L.M[(size_t)np * np - 1] = 1.0;
}

// Graphs handed out as kept handles (Y only; released by the harness).
void release_kept(rdist_ctx c, rdist_graph g) {
    if (!c->graphs.count(g)) die("kept graph: unknown handle");
    (void)hipFree(g->Y);
    c->in_use -= std::min(g->bytes, c->in_use);
    c->graphs.erase(g);
    delete g;
}

}  // namespace

// ---- stand-ins of the kernel launchers and of the single-graph plan ----
namespace rd {

void launch_fill_i32(int32_t *p, size_t count, hipStream_t s) {
    hipstub::enqueue(s, "fill", [=]() {
        need_dev(p, count * 4, "fill");
        std::memset(p, 0, count * 4);
    });
}

void launch_lv_gate(const LevelGraph *gs, int count, hipStream_t s) {
    hipstub::enqueue(s, "lv_gate", [=]() {
        need_dev(gs, sizeof(LevelGraph) * (size_t)count, "level table");
        for (int g = 0; g < count; ++g) check_level_graph(gs[g]);
    });
}

void launch_lv(int phase, const LevelGraph *gs, const int *units, int grid, int K, hipStream_t s) {
    hipstub::enqueue(s, "lv", [=]() {
        need_dev(units, sizeof(int) * (size_t)grid, "unit list");
        for (int b = 0; b < grid; ++b) {
            const int u = units[b];
            if (u < 0) continue;
            const int g = u >> kLvShift, item = u & ((1 << kLvShift) - 1);
            need_dev(gs + g, sizeof(LevelGraph), "level table entry");
            const LevelGraph &L = gs[g];
            check_level_graph(L);
            int limit = 0;
            switch (phase) {
                case kLvColsum: limit = L.nchunk; break;
                case kLvBuild: limit = 2 * L.nt - 1; break;
                case kLvPanel: limit = K < L.nt ? 1 : 0; break;
                case kLvRowcol: limit = K < L.nt ? L.nt - 1 : 0; break;
                case kLvDiag: limit = K + 1 < L.nt ? 1 : 0; break;
                case kLvEdge: limit = K + 1 < L.nt ? 2 * L.nt - 2 : 0; break;
                case kLvRest: limit = L.nt * L.nt; break;
                default: die("unknown level phase");
            }
            if (item >= limit) die("unit item beyond its graph's items");
            g_kernel_items += 1;
        }
    });
}

void launch_batched(const BatchTask *tasks, int count, int *counter, int grid, double *scratch, int stride,
                    hipStream_t s) {
    hipstub::enqueue(s, "batched", [=]() {
        need_dev(tasks, sizeof(BatchTask) * (size_t)count, "task table");
        need_dev(counter, sizeof(int), "task counter");
        bool medium = false;
        for (int q = 0; q < count; ++q) {
            const BatchTask &t = tasks[q];
            if (t.n < 1 || t.n > 512 || t.np != np_of(t.n)) die("task: inconsistent sizes");
            need_user(t.A, (size_t)t.n * t.n, "task A");
            need_user(t.D, (size_t)t.n * t.n * 2, "task D");
            need_dev(t.info, sizeof(rdist_info), "task info");
            if (t.M) need_dev(t.M, (size_t)t.np * t.np * 8, "task M");
            else if (t.n > 128) die("task: n > 128 without a matrix");
            medium |= t.n > 128;
            touch_user(t.A, t.D, t.n);
            g_kernel_items += 1;
        }
        if (medium) need_dev(scratch, (size_t)grid * stride * 8, "persistent scratch");
        *counter = 0;
    });
}

namespace eng {

rdist_status make_graph(rdist_ctx c, int n, double *Y, int ld, size_t ybytes, const uint8_t *A, hipStream_t s,
                        rdist_graph *out, const rdist_info *dinfo, bool) {
    need_dev(Y, ybytes, "kept Y");
    if (ybytes < (size_t)n * ld * 8) die("kept Y smaller than n x ld");
    hipstub::enqueue(s, "make_graph", [=]() {
        need_user(A, (size_t)n * n, "kept graph A");
        need_dev(dinfo, sizeof(rdist_info), "kept graph info");
    });
    auto *g = new rdist_graph_s();
    g->ctx = c;
    g->Y = Y;
    g->n = n;
    g->ld = ld;
    g->ybytes = ybytes;
    g->bytes = ybytes;
    c->graphs.insert(g);
    *out = g;
    return RDIST_OK;
}

rdist_status solve_blocked(rdist_ctx, const uint8_t *A, int n, double, uint32_t, int16_t *D, rdist_graph *keep,
                           rdist_info *info, hipStream_t s) {
    hipstub::enqueue(s, "solve_blocked", [=]() {
        need_user(A, (size_t)n * n, "big graph A");
        need_user(D, (size_t)n * n * 2, "big graph D");
        touch_user(A, D, n);
    });
    if (keep) *keep = nullptr;
    if (info) info->status = RDIST_OK;
    return RDIST_OK;
}

}  // namespace eng
}  // namespace rd

// ---- driver ----
namespace {

struct Batch {
    std::vector<int32_t> n;
    std::vector<const uint8_t *> A;
    std::vector<int16_t *> D;
    std::vector<double> gamma;
};

Batch take(const std::vector<int> &sizes, double gamma) {
    Batch b;
    for (int n : sizes) {
        b.n.push_back(n);
        b.A.push_back((const uint8_t *)g_user.get((size_t)n * n));
        b.D.push_back((int16_t *)g_user.get((size_t)n * n * 2));
        b.gamma.push_back(gamma);
    }
    return b;
}

void give_back(Batch &b) {   // reverse order, so that the pool re-issues the same addresses
    for (size_t i = b.n.size(); i-- > 0;) {
        g_user.put(b.D[i]);
        g_user.put((void *)b.A[i]);
    }
    b = Batch{};
}

void solve(rdist_ctx c, Batch &b, uint32_t flags, hipStream_t s) {
    const int count = (int)b.n.size();
    std::vector<rdist_info> info(count);
    std::vector<rdist_graph> keep(count, nullptr);
    const bool k = flags & RDIST_KEEP_Y;
    rdist_status st = rdist_solve_batched(c, count, b.n.data(), b.A.data(), b.gamma.data(), flags, b.D.data(),
                                          k ? keep.data() : nullptr, info.data(), s);
    if (st != RDIST_OK) die("rdist_solve_batched: " + rd::eng::g_last_error);
    if ((int)c->plans.size() > 4) die("more cached plans than the cache holds");
    for (rdist_graph g : keep)
        if (g) release_kept(c, g);
}

std::vector<int> log_uniform_sizes(std::mt19937 &rng, int count, int lo, int hi) {
    std::uniform_real_distribution<double> u(std::log((double)lo), std::log((double)hi));
    std::vector<int> v;
    for (int i = 0; i < count; ++i) v.push_back((int)std::lround(std::exp(u(rng))));
    return v;
}

rdist_ctx new_ctx() {
    auto *c = new rdist_ctx_s();
    c->device = 0;
    c->num_cu = 256;
    return c;
}

void end_ctx(rdist_ctx c) {
    rd::eng::destroy_plans(c);
    for (auto &kv : c->ws) rd::eng::free_workspace(c, kv.second);
    c->ws.clear();
    if (c->in_use != 0) die("budget not returned: " + std::to_string(c->in_use) + " bytes in use");
    for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
    delete c;
}

}  // namespace

// free_workspace lives in rd_engine.hip with the kernels; the harness frees
// the parts a batched call creates.
namespace rd {
namespace eng {
void free_workspace(rdist_ctx c, Workspace &w) {
    free_transient_plan(c, w);
    if (w.aux) (void)hipStreamDestroy(w.aux);
    if (w.aux2) (void)hipStreamDestroy(w.aux2);
    for (hipEvent_t e : {w.ev_er, w.ev_panel, w.ev_fork, w.ev_join})
        if (e) (void)hipEventDestroy(e);
    w = Workspace{};
}
}  // namespace eng
}  // namespace rd

int main(int argc, char **argv) {
    const std::string only = argc > 1 ? argv[1] : "all";
    auto run = [&](const char *k) { return only == "all" || only == k; };
    std::mt19937 rng(20260);
    const std::vector<std::vector<int>> templates = {
        log_uniform_sizes(rng, 96, 32, 512),
        {600, 40, 300, 1030, 128},
        {257},
        log_uniform_sizes(rng, 64, 32, 512),
        {4096, 2000, 64},
        {5000, 100},
        {40},
        log_uniform_sizes(rng, 200, 32, 1500),
    };

    // 1. captured, eager and kept-Y batches in random order, buffers reused
    if (run("1")) {
        rdist_ctx c = new_ctx();
        std::vector<Batch> held;
        for (int it = 0; it < 240; ++it) {
            const auto &t = templates[rng() % templates.size()];
            Batch b = take(t, (rng() % 4) ? -0.5 : 0.01);
            const int f = rng() % 4;
            const uint32_t flags = f == 0 ? RDIST_NO_GRAPH : f == 1 ? RDIST_KEEP_Y : 0u;
            solve(c, b, flags, nullptr);
            if (f == 3) solve(c, b, 0u, nullptr);   // immediate replay of the same batch
            if (rng() % 5 == 0) held.push_back(b);  // keep its buffers: the next one gets other pointers
            else give_back(b);
            if (held.size() > 3) {
                give_back(held.front());
                held.erase(held.begin());
            }
        }
        for (Batch &b : held) give_back(b);
        end_ctx(c);
        std::printf("[harness] random sequence: %ld captures, %ld replays, %ld kernel items\n",
                    hipstub::counters().captures, hipstub::counters().graph_launches, g_kernel_items);
    }

    // 2. a tuning change between calls: one new capture, then replays
    if (run("2")) {
        rdist_ctx c = new_ctx();
        c->tile_cache_path = "/dev/null";   // the autotuner runs; the file write goes nowhere
        Batch b = take(templates[0], -0.5);
        solve(c, b, 0u, nullptr);           // autotune + capture
        if (c->tuned.size() != 1) die("autotuner recorded no tuning");
        const long cap0 = hipstub::counters().captures;
        for (int r = 0; r < 3; ++r) solve(c, b, 0u, nullptr);
        if (hipstub::counters().captures != cap0) die("identical calls re-captured the plan");
        rd::eng::BatchTuning &t = c->tuned[0].second;
        t.persist_max_n = t.persist_max_n == 256 ? 512 : 256;
        t.persist_grid = 32;
        for (int r = 0; r < 3; ++r) solve(c, b, 0u, nullptr);
        const long extra = hipstub::counters().captures - cap0;
        if (extra != 1) die("after a tuning change the plan was captured " + std::to_string(extra) + " times, not once");
        give_back(b);
        end_ctx(c);
        std::printf("[harness] tuning change: captured once, then replayed\n");
    }

    // 3. the caller destroys a stream whose plan is still cached; later
    //    batches evict that plan
    if (run("3")) {
        rdist_ctx c = new_ctx();
        hipStream_t s1 = nullptr;
        (void)hipStreamCreateWithFlags(&s1, hipStreamNonBlocking);
        Batch b = take(templates[1], -0.5);
        solve(c, b, 0u, s1);
        (void)hipStreamDestroy(s1);
        give_back(b);
        for (int k = 0; k < 6; ++k) {   // six distinct batches: the cache of four evicts the first plan
            Batch o = take(templates[k + 2 < (int)templates.size() ? k + 2 : 0], -0.5);
            solve(c, o, 0u, nullptr);
            give_back(o);
        }
        end_ctx(c);
        std::printf("[harness] plan of a destroyed stream evicted\n");
    }

    if (hipstub::live_device_allocations() != 0)
        die("device allocations leaked: " + std::to_string(hipstub::live_device_allocations()));
    std::printf("[harness] OK\n");
    return 0;
}
