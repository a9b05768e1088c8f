// rd_server.hip -- the request loop (rdist_server_*): a queue, slots (HIP
// streams with their own workspaces), admission by HBM footprint and
// continuous batching: every request with n <= 4096, full D or paths, joins
// the next batch of a free slot (one level-synchronous batched solve; a path
// request keeps Y in the slot's own buffer), except that one with n > 1024
// runs alone on the single-graph plan while at most 8 requests wait.  A batch completes in groups:
// the graphs with n <= 128 when the persistent kernel ends, those with
// ceil(n / 128) = t after blocked step t - 1; each group's results (D, infos,
// and the greedy paths of its path requests) are copied out as soon as the
// group is final and its requests are reported then, while the batch's
// larger graphs still run.  Slot buffers grow with headroom and are kept, so
// a warmed-up server allocates nothing per request.  Driven by the caller's
// polls; no thread of its own, and the device is never waited on except in
// rdist_server_destroy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <deque>
#include <string>
#include <vector>

#include "../../include/rdist.h"
#include "rd_engine.h"

namespace rd {
namespace eng {
namespace {

constexpr int kMaxPairs = 4096;

struct Pending {
    rdist_request r;
    size_t footprint;
};

// Requests of a slot that complete together, and the event after their copies.
struct Group {
    int index = 0;             // completion group (its info block in info_h and its events)
    std::vector<int> reqs;     // indices into Slot::reqs
    bool done = false;
};

struct Slot {
    hipStream_t stream = nullptr;
    bool busy = false;
    std::vector<Pending> reqs;           // in flight on this slot
    std::vector<Group> groups;           // their completion groups
    int groups_left = 0;
    Buf D, Y, bits, paths, pairs, tasks; // device buffers, grown with headroom and kept
    rdist_info *info_h = nullptr;        // pinned, kBatchMarks blocks of max_batch infos
    int32_t *pairs_h = nullptr;          // pinned staging of (cur, goal), max_batch * kMaxPairs pairs
    rd::PathTask *tasks_h = nullptr;     // pinned staging of a batch's path tasks, max_batch entries
    hipEvent_t marks[kBatchMarks] = {};  // group t's results are final (recorded by the plan)
    hipEvent_t gdone[kBatchMarks] = {};  // group t's results are in host memory
    size_t footprint = 0;
    bool single = false;                 // the slot's request runs on the single-graph plan
};

size_t footprint_of(const rdist_request &r) {
    const size_t np = ((size_t)r.n + 127) / 128 * 128;
    const size_t f = 8 * np * np + 4096 * np;
    return r.kind == RDIST_QUERY_PATHS ? 2 * f : f;
}

bool batchable(const rdist_request &r) { return r.n <= kBatchMaxN; }
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
// Completion group of a batched graph (the batched plan's threshold T = 128).
int group_of(int n) { return n <= kB ? 0 : (n + kB - 1) / kB; }

}  // namespace
}  // namespace eng
}  // namespace rd

using namespace rd::eng;

struct rdist_server_s {
    rdist_ctx ctx = nullptr;
    size_t budget = 0;
    int max_batch = 1;
    std::vector<Slot> slots;
    std::deque<Pending> queue;
    std::vector<int64_t> finished;       // reported by the next poll
    rdist_server_stats st{};
};

namespace {

rdist_status grow(rdist_ctx c, Buf &b, size_t bytes) { return ensure_grow(c, b, std::max<size_t>(bytes, 256)); }

void fail_request(rdist_server s, const Pending &p, rdist_status why) {
    if (p.r.info_host) {
        std::memset(p.r.info_host, 0, sizeof(rdist_info));
        p.r.info_host->status = why;
    }
    s->finished.push_back(p.r.id);
    s->st.failed += 1;
}

// A request above the batched range, alone on the slot's stream: the
// single-graph plan, its D, or its paths on Y left in the stream's workspace;
// one group.
rdist_status dispatch_single(rdist_server s, Slot &sl, const rdist_request &r0) {
    rdist_ctx c = s->ctx;
    hipStream_t st = sl.stream;
    rdist_status e;
    const size_t n2 = (size_t)r0.n * r0.n;
    if ((e = grow(c, sl.D, n2 * 2))) return e;
    if (r0.kind == RDIST_QUERY_D) {
        e = rdist_solve(c, r0.A_dev, r0.n, r0.gamma, RDIST_F64, (int16_t *)sl.D.p, nullptr, sl.info_h, st);
        if (e) return e;
        RD_HIP(hipMemcpyAsync(r0.D_host, sl.D.p, n2 * 2, hipMemcpyDeviceToHost, st));
    } else {
        // Y stays in the workspace of the slot's stream (M, leading dimension
        // its np_cap) until the next solve on that stream, which starts only
        // after this request is reported: no graph handle, so nothing is
        // allocated for the request and nothing freed when it completes (a
        // free synchronises the whole device and would stall the caller's
        // poll loop behind the other slots' work).  The paths come from the
        // batched plan's path kernel (successor bitmap, then greedy hops).
        const size_t pb = (size_t)r0.q * rd::path_row_len(r0.max_hops) * 4;
        const size_t nw = ((size_t)r0.n + 63) / 64;
        if ((e = grow(c, sl.paths, pb))) return e;
        if ((e = grow(c, sl.pairs, (size_t)2 * kMaxPairs * 4))) return e;
        if ((e = grow(c, sl.bits, (size_t)r0.n * nw * 8))) return e;
        if ((e = grow(c, sl.tasks, sizeof(rd::PathTask)))) return e;
        e = rdist_solve(c, r0.A_dev, r0.n, r0.gamma, RDIST_F64 | RDIST_KEEP_Y, (int16_t *)sl.D.p, nullptr, sl.info_h,
                        st);
        if (e) return e;
        if (r0.q > 0) {
            const Workspace &w = c->ws[st];
            std::memcpy(sl.pairs_h, r0.cur_host, (size_t)r0.q * 4);
            std::memcpy(sl.pairs_h + kMaxPairs, r0.goal_host, (size_t)r0.q * 4);
            int32_t *cur = (int32_t *)sl.pairs.p, *goal = cur + kMaxPairs;
            RD_HIP(hipMemcpyAsync(cur, sl.pairs_h, (size_t)2 * kMaxPairs * 4, hipMemcpyHostToDevice, st));
            rd::PathTask &t = sl.tasks_h[0];
            t.A = r0.A_dev;
            t.Y = (const double *)w.M.p;
            t.bits = (unsigned long long *)sl.bits.p;
            t.cur = cur;
            t.goal = goal;
            t.out = (int32_t *)sl.paths.p;
            t.n = r0.n;
            t.ld = w.np_cap;
            t.q = r0.q;
            t.max_hops = r0.max_hops;
            t.blk0 = 0;
            t.q0 = 0;
            RD_HIP(hipMemcpyAsync(sl.tasks.p, sl.tasks_h, sizeof(rd::PathTask), hipMemcpyHostToDevice, st));
            {
                Timer tm(c, st, RDIST_K_NEXTHOP, 0.0, 0.0);
                rd::launch_paths_multi((const rd::PathTask *)sl.tasks.p, 1, rd::path_task_blocks(r0.n), r0.q, st);
            }
            RD_HIP(hipGetLastError());
            RD_HIP(hipMemcpyAsync(r0.paths_host, sl.paths.p, pb, hipMemcpyDeviceToHost, st));
        }
    }
    RD_HIP(hipEventRecord(sl.gdone[0], st));
    sl.groups.assign(1, Group{0, {0}, false});
    return RDIST_OK;
}

// Requests with n <= kBatchMaxN: one batched solve on the slot's stream,
// then per completion group (on the plan's tail stream, after the group's
// mark): the infos, the group's greedy paths (one bitmap and one path launch
// for all its path requests), the copies to host memory, and its event.
rdist_status dispatch_batch(rdist_server s, Slot &sl, const std::vector<Pending> &batch) {
    rdist_ctx c = s->ctx;
    hipStream_t st = sl.stream;
    rdist_status e;
    const int cnt = (int)batch.size();
    std::vector<size_t> offD(cnt), offY(cnt), offB(cnt), offQ(cnt), offP(cnt);
    std::vector<int> grp(cnt);
    size_t tD = 0, tY = 0, tB = 0, tQ = 0, tP = 0;
    for (int i = 0; i < cnt; ++i) {
        const rdist_request &r = batch[i].r;
        grp[i] = group_of(r.n);
        offD[i] = tD;
        tD += align256((size_t)r.n * r.n * 2);
        if (r.kind != RDIST_QUERY_PATHS) continue;
        const size_t np = ((size_t)r.n + kB - 1) / kB * kB, nw = ((size_t)r.n + 63) / 64;
        offY[i] = tY;
        tY += np * np * 8;
        offB[i] = tB;
        tB += align256((size_t)r.n * nw * 8);
        offQ[i] = tQ;
        tQ += (size_t)r.q;
        offP[i] = tP;
        tP += align256((size_t)r.q * rd::path_row_len(r.max_hops) * 4);
    }
    if ((e = grow(c, sl.D, tD))) return e;
    if (tY && ((e = grow(c, sl.Y, tY)) || (e = grow(c, sl.bits, tB)))) return e;
    if (tQ && ((e = grow(c, sl.pairs, 2 * tQ * 4)) || (e = grow(c, sl.paths, tP)))) return e;
    std::vector<int32_t> ns(cnt);
    std::vector<const uint8_t *> As(cnt);
    std::vector<double> gs(cnt);
    std::vector<int16_t *> Ds(cnt);
    std::vector<double *> Ys(cnt, nullptr);
    for (int i = 0; i < cnt; ++i) {
        const rdist_request &r = batch[i].r;
        ns[i] = r.n;
        As[i] = r.A_dev;
        gs[i] = r.gamma;
        Ds[i] = (int16_t *)((char *)sl.D.p + offD[i]);
        if (r.kind == RDIST_QUERY_PATHS) Ys[i] = (double *)((char *)sl.Y.p + offY[i]);
    }
    // groups present, in completion order, with their requests
    std::vector<Group> groups;
    for (int g = 0; g < kBatchMarks; ++g) {
        Group G;
        G.index = g;
        for (int i = 0; i < cnt; ++i)
            if (grp[i] == g) G.reqs.push_back(i);
        if (!G.reqs.empty()) groups.push_back(std::move(G));
    }
    // path tasks group by group (each group's tasks contiguous, prefix sums
    // within the group) and the (cur, goal) pairs, uploaded on st before the
    // plan, so that every group's work (which waits for a mark of the plan)
    // sees them
    const size_t ng = groups.size();
    int32_t *cur_d = (int32_t *)sl.pairs.p, *goal_d = cur_d + tQ;
    std::vector<int> task0(ng + 1, 0), tblk(ng, 0), tq(ng, 0);
    int ntask = 0;
    for (size_t gi = 0; gi < ng; ++gi) {
        task0[gi] = ntask;
        for (int i : groups[gi].reqs) {
            const rdist_request &r = batch[i].r;
            if (r.kind != RDIST_QUERY_PATHS || r.q == 0) continue;
            rd::PathTask &t = sl.tasks_h[ntask++];
            t.A = r.A_dev;
            t.Y = Ys[i];
            t.bits = (unsigned long long *)((char *)sl.bits.p + offB[i]);
            t.cur = cur_d + offQ[i];
            t.goal = goal_d + offQ[i];
            t.out = (int32_t *)((char *)sl.paths.p + offP[i]);
            t.n = r.n;
            t.ld = (r.n + kB - 1) / kB * kB;
            t.q = r.q;
            t.max_hops = r.max_hops;
            t.blk0 = tblk[gi];
            t.q0 = tq[gi];
            tblk[gi] += rd::path_task_blocks(r.n);
            tq[gi] += r.q;
            std::memcpy(sl.pairs_h + offQ[i], r.cur_host, (size_t)r.q * 4);
            std::memcpy(sl.pairs_h + tQ + offQ[i], r.goal_host, (size_t)r.q * 4);
        }
    }
    task0[ng] = ntask;
    if (ntask) {
        if ((e = grow(c, sl.tasks, sizeof(rd::PathTask) * (size_t)ntask))) return e;
        RD_HIP(hipMemcpyAsync(cur_d, sl.pairs_h, 2 * tQ * 4, hipMemcpyHostToDevice, st));
        RD_HIP(hipMemcpyAsync(sl.tasks.p, sl.tasks_h, sizeof(rd::PathTask) * (size_t)ntask, hipMemcpyHostToDevice,
                              st));
    }
    hipStream_t tail = nullptr;
    const rdist_info *info_dev = nullptr;
    e = solve_batch_into(c, st, cnt, ns.data(), As.data(), gs.data(), Ds.data(), Ys.data(), nullptr, sl.marks, &tail,
                         &info_dev);
    if (e) return e;
    const rd::PathTask *tasks_d = (const rd::PathTask *)sl.tasks.p;
    for (size_t gi = 0; gi < ng; ++gi) {
        const Group &G = groups[gi];
        RD_HIP(hipStreamWaitEvent(tail, sl.marks[G.index], 0));
        RD_HIP(hipMemcpyAsync(sl.info_h + (size_t)G.index * s->max_batch, info_dev, sizeof(rdist_info) * (size_t)cnt,
                              hipMemcpyDeviceToHost, tail));
        const int nt = task0[gi + 1] - task0[gi];
        if (nt) {
            Timer tm(c, tail, RDIST_K_NEXTHOP, 0.0, 0.0);
            rd::launch_paths_multi(tasks_d + task0[gi], nt, tblk[gi], tq[gi], tail);
        }
        RD_HIP(hipGetLastError());
        for (int i : G.reqs) {
            const rdist_request &r = batch[i].r;
            if (r.kind == RDIST_QUERY_D)
                RD_HIP(hipMemcpyAsync(r.D_host, Ds[i], (size_t)r.n * r.n * 2, hipMemcpyDeviceToHost, tail));
            else if (r.q > 0)
                RD_HIP(hipMemcpyAsync(r.paths_host, (char *)sl.paths.p + offP[i], (size_t)r.q * rd::path_row_len(r.max_hops) * 4,
                                      hipMemcpyDeviceToHost, tail));
        }
        RD_HIP(hipEventRecord(sl.gdone[G.index], tail));
    }
    sl.groups = std::move(groups);
    s->st.batches += 1;
    s->st.batched_requests += cnt;
    return RDIST_OK;
}

// A request from this order on runs alone on the single-graph plan (width
// 128 up to n = 6400) when few requests wait: faster than the level plan for
// one graph (n = 4096: 4.16 against 6.19 ms; n = 2048: 1.53 against 2.26)
// and the same results bit for bit (both take the same 128-pivot steps with
// the same products in the same order).  Behind a backlog it joins the batch
// instead, whose level plan keeps many large graphs in flight at once.  At
// the C5 request mix (two slots, 0.1x of saturation) this moved p99 from
// 11.9 to 8.0 ms with the saturated rate unchanged (6.3 ms once the lone
// plan's chain products were split into 64 x 64 pieces); taking such requests out
// of batches always cost a third of the saturated rate.
constexpr int kLoneSingleMinN = 1025;
bool lone(const rdist_request &r) { return r.n >= kLoneSingleMinN; }
// Queue length up to which such requests are taken out of batches.
constexpr size_t kLoneMaxQueue = 8;

// Launches the requests of `batch` on slot k.  Returns RDIST_E_AGAIN when the
// context's own budget is in use (the caller puts them back in the queue).
rdist_status dispatch(rdist_server s, int k, std::vector<Pending> &batch) {
    Slot &sl = s->slots[k];
    const bool single = batch.size() == 1 && (!batchable(batch[0].r) || lone(batch[0].r));
    const rdist_status e = single ? dispatch_single(s, sl, batch[0].r) : dispatch_batch(s, sl, batch);
    if (e) return e;
    sl.busy = true;
    sl.single = single;
    sl.reqs = batch;
    sl.groups_left = (int)sl.groups.size();
    sl.footprint = 0;
    for (auto &p : batch) sl.footprint += p.footprint;
    s->st.footprint_in_flight += sl.footprint;
    s->st.in_flight += (int64_t)batch.size();
    s->st.max_in_flight = std::max(s->st.max_in_flight, s->st.in_flight);
    s->st.max_footprint_in_flight = std::max(s->st.max_footprint_in_flight, s->st.footprint_in_flight);
    return RDIST_OK;
}

bool fits(rdist_server s, size_t f) { return !s->budget || s->st.footprint_in_flight + f <= s->budget; }

// Dispatches queued requests, oldest first, while a slot is free and the
// footprint fits.  A waiting request at the head that does not fit blocks
// the ones behind it (no overtaking, so nothing starves).
void pump(rdist_server s) {
    for (;;) {
        if (s->queue.empty()) return;
        int k = -1;
        for (int i = 0; i < (int)s->slots.size(); ++i)
            if (!s->slots[i].busy) { k = i; break; }
        if (k < 0) return;
        std::vector<Pending> batch;
        size_t f = 0;
        // With few requests waiting, one with n > 1024 runs alone on the
        // single-graph plan (latency); with a backlog it joins the batch,
        // whose level plan runs many large graphs at once (throughput).
        const bool split = s->queue.size() <= kLoneMaxQueue;
        auto batches = [&](const rdist_request &r) { return batchable(r) && !(split && lone(r)); };
        if (batches(s->queue.front().r)) {
            // every waiting request that batches, in order, while it fits;
            // the ones that run alone stay queued for the next free slot
            for (auto it = s->queue.begin(); it != s->queue.end() && (int)batch.size() < s->max_batch;) {
                if (batches(it->r) && fits(s, f + it->footprint)) {
                    f += it->footprint;
                    batch.push_back(*it);
                    it = s->queue.erase(it);
                } else if (batches(it->r)) {
                    break;
                } else {
                    ++it;
                }
            }
            if (batch.empty()) return;
        } else {
            if (!fits(s, s->queue.front().footprint)) return;
            batch.push_back(s->queue.front());
            s->queue.pop_front();
        }
        s->st.queued = (int64_t)s->queue.size();
        const rdist_status e = dispatch(s, k, batch);
        if (e == RDIST_E_AGAIN && s->st.in_flight > 0) {
            // the context's budget is in use: retry after something finishes
            (void)hipDeviceSynchronize();   // whatever the failed dispatch enqueued
            for (auto it = batch.rbegin(); it != batch.rend(); ++it) s->queue.push_front(*it);
            s->st.queued = (int64_t)s->queue.size();
            s->slots[k].groups.clear();
            return;
        }
        if (e) {
            Slot &sl = s->slots[k];
            (void)hipDeviceSynchronize();   // the slot's stream and the plan's other streams
            sl.groups.clear();
            for (auto &p : batch) fail_request(s, p, e);
        }
    }
}

// Reports the requests of a finished group of slot sl.
void complete_group(rdist_server s, Slot &sl, Group &G, bool single) {
    for (int i : G.reqs) {
        const rdist_request &r = sl.reqs[i].r;
        if (r.info_host) *r.info_host = single ? sl.info_h[0] : sl.info_h[(size_t)G.index * s->max_batch + i];
        s->finished.push_back(r.id);
        s->st.completed += 1;
        s->st.in_flight -= 1;
    }
    G.done = true;
    sl.groups_left -= 1;
}

void release_slot(rdist_server s, Slot &sl) {
    s->st.footprint_in_flight -= sl.footprint;
    sl.reqs.clear();
    sl.groups.clear();
    sl.groups_left = 0;
    sl.footprint = 0;
    sl.busy = false;
}

}  // namespace

extern "C" {

rdist_status rdist_server_create(rdist_ctx ctx, int32_t slots, size_t hbm_budget_bytes, int32_t max_batch,
                                 rdist_server *out) {
    if (!out) return fail(RDIST_E_ARG, "out is NULL");
    *out = nullptr;
    if (!ctx) return fail(RDIST_E_ARG, "ctx is NULL");
    if (slots < 1 || slots > 64) return fail(RDIST_E_ARG, "slots must lie in [1, 64]");
    if (max_batch < 1 || max_batch > 1024) return fail(RDIST_E_ARG, "max_batch must lie in [1, 1024]");
    RD_HIP(hipSetDevice(ctx->device));
    auto *s = new rdist_server_s();
    s->ctx = ctx;
    s->budget = hbm_budget_bytes;
    s->max_batch = max_batch;
    s->slots.resize(slots);
    for (Slot &sl : s->slots) {
        bool ok = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess &&
                  hipHostMalloc((void **)&sl.info_h, sizeof(rdist_info) * (size_t)max_batch * kBatchMarks,
                                hipHostMallocDefault) == hipSuccess &&
                  hipHostMalloc((void **)&sl.pairs_h, (size_t)2 * kMaxPairs * 4 * max_batch, hipHostMallocDefault) ==
                      hipSuccess &&
                  hipHostMalloc((void **)&sl.tasks_h, sizeof(rd::PathTask) * (size_t)max_batch,
                                hipHostMallocDefault) == hipSuccess;
        for (int g = 0; ok && g < kBatchMarks; ++g)
            ok = hipEventCreateWithFlags(&sl.marks[g], hipEventDisableTiming) == hipSuccess &&
                 hipEventCreateWithFlags(&sl.gdone[g], hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            rdist_server_destroy(s);
            return fail(RDIST_E_HIP, "server stream, event or pinned buffer creation failed");
        }
    }
    *out = s;
    return RDIST_OK;
}

rdist_status rdist_server_submit(rdist_server s, const rdist_request *req) {
    if (!s || !req) return fail(RDIST_E_ARG, "NULL argument");
    const rdist_request &r = *req;
    if (!r.A_dev || r.n < 1 || r.n > 65536) return fail(RDIST_E_ARG, "bad A_dev or n");
    rdist_status e;
    if ((e = check_gamma(r.gamma))) return e;
    if (r.kind == RDIST_QUERY_D) {
        if (!r.D_host) return fail(RDIST_E_ARG, "D_host is required");
    } else if (r.kind == RDIST_QUERY_PATHS) {
        if (r.q < 0 || r.q > kMaxPairs || r.max_hops < 1 || r.max_hops > 65535)
            return fail(RDIST_E_ARG, "bad q or max_hops");
        if (r.q > 0 && (!r.cur_host || !r.goal_host || !r.paths_host)) return fail(RDIST_E_ARG, "NULL path array");
    } else {
        return fail(RDIST_E_ARG, "unknown query kind");
    }
    const size_t f = footprint_of(r);
    if (s->budget && f > s->budget) return fail(RDIST_E_NOMEM, "request footprint exceeds the server budget");
    Guard g(s->ctx);
    s->queue.push_back(Pending{r, f});
    s->st.submitted += 1;
    s->st.queued = (int64_t)s->queue.size();
    return RDIST_OK;
}

rdist_status rdist_server_poll(rdist_server s, int64_t *done_ids, int32_t max, int32_t *n_done) {
    if (!s || !n_done || max < 0 || (max > 0 && !done_ids)) return fail(RDIST_E_ARG, "bad argument");
    Guard g(s->ctx);
    RD_HIP(hipSetDevice(s->ctx->device));
    for (Slot &sl : s->slots) {
        if (!sl.busy) continue;
        const bool single = sl.single;
        bool failed = false;
        for (Group &G : sl.groups) {
            if (G.done) continue;
            const hipError_t q = hipEventQuery(sl.gdone[G.index]);
            if (q == hipSuccess) {
                complete_group(s, sl, G, single);
            } else if (q != hipErrorNotReady) {
                failed = true;
                break;
            }
        }
        if (failed) {
            (void)hipGetLastError();
            for (Group &G : sl.groups) {
                if (G.done) continue;
                for (int i : G.reqs) fail_request(s, sl.reqs[i], RDIST_E_HIP);
                s->st.in_flight -= (int64_t)G.reqs.size();
                G.done = true;
            }
            sl.groups_left = 0;
        }
        if (sl.groups_left == 0) release_slot(s, sl);
    }
    pump(s);
    const int32_t k = (int32_t)std::min<size_t>((size_t)max, s->finished.size());
    for (int32_t i = 0; i < k; ++i) done_ids[i] = s->finished[i];
    s->finished.erase(s->finished.begin(), s->finished.begin() + k);
    *n_done = k;
    return RDIST_OK;
}

rdist_status rdist_server_stats_get(rdist_server s, rdist_server_stats *out) {
    if (!s || !out) return fail(RDIST_E_ARG, "bad argument");
    *out = s->st;
    return RDIST_OK;
}

void rdist_server_destroy(rdist_server s) {
    if (!s) return;
    {
        Guard g(s->ctx);
        (void)hipSetDevice(s->ctx->device);
        (void)hipDeviceSynchronize();   // every slot's streams, the plans' tail streams included
        for (Slot &sl : s->slots) {
            for (Buf *b : {&sl.D, &sl.Y, &sl.bits, &sl.paths, &sl.pairs, &sl.tasks}) release(s->ctx, *b);
            if (sl.info_h) (void)hipHostFree(sl.info_h);
            if (sl.pairs_h) (void)hipHostFree(sl.pairs_h);
            if (sl.tasks_h) (void)hipHostFree(sl.tasks_h);
            for (int g = 0; g < kBatchMarks; ++g) {
                if (sl.marks[g]) (void)hipEventDestroy(sl.marks[g]);
                if (sl.gdone[g]) (void)hipEventDestroy(sl.gdone[g]);
            }
            if (sl.stream) {
                release_stream_workspace(s->ctx, sl.stream);
                (void)hipStreamDestroy(sl.stream);
            }
        }
    }
    delete s;
}

}  // extern "C"
