// rd_server.hip -- the request loop (rdist_server_*): a queue, slots (HIP
// streams with their own workspaces), admission by HBM footprint and
// continuous batching: every request with n <= 4096, full D or paths, joins
// the next batch of a free slot (one level-synchronous batched solve; a path
// request keeps Y in the slot's own buffer and its next hops run right after
// the batch).  Slot buffers grow with headroom and are kept, so a warmed-up
// server allocates nothing per request.  Driven by the caller's polls; no
// thread of its own, and the device is never waited on except in
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

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<Pending> reqs;           // in flight on this slot
    rdist_graph graph = nullptr;         // a path request above the batched range: its kept Y
    Buf D, Y, bits, paths, pairs, tasks; // device buffers, grown with headroom and kept
    rdist_info *info_h = nullptr;        // pinned, one per batched request
    int32_t *pairs_h = nullptr;          // pinned staging of (cur, goal), max_batch * kMaxPairs pairs
    rd::PathTask *tasks_h = nullptr;     // pinned staging of a batch's path tasks, max_batch entries
    size_t footprint = 0;
};

size_t footprint_of(const rdist_request &r) {
    const size_t np = ((size_t)r.n + 127) / 128 * 128;
    const size_t f = 8 * np * np + 4096 * np;
    return r.kind == RDIST_QUERY_PATHS ? 2 * f : f;
}

bool batchable(const rdist_request &r) { return r.n <= kBatchMaxN; }
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

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

// Launches the requests of `batch` on slot k.  Returns RDIST_E_AGAIN when the
// context's own budget is in use (the caller puts them back in the queue).
rdist_status dispatch(rdist_server s, int k, std::vector<Pending> &batch) {
    rdist_ctx c = s->ctx;
    Slot &sl = s->slots[k];
    hipStream_t st = sl.stream;
    rdist_status e = RDIST_OK;
    const rdist_request &r0 = batch[0].r;
    if (batch.size() == 1 && !batchable(r0)) {
        const size_t n2 = (size_t)r0.n * r0.n;
        if ((e = grow(c, sl.D, n2 * 2))) return e;
        if (r0.kind == RDIST_QUERY_D) {
            e = rdist_solve(c, r0.A_dev, r0.n, r0.gamma, RDIST_F64, (int16_t *)sl.D.p, nullptr, sl.info_h, st);
            if (e) return e;
            RD_HIP(hipMemcpyAsync(r0.D_host, sl.D.p, n2 * 2, hipMemcpyDeviceToHost, st));
        } else {
            const size_t pb = (size_t)r0.q * (r0.max_hops + 1) * 4;
            if ((e = grow(c, sl.paths, pb))) return e;
            if ((e = grow(c, sl.pairs, (size_t)2 * kMaxPairs * 4))) return e;
            rdist_graph g = nullptr;
            e = rdist_solve(c, r0.A_dev, r0.n, r0.gamma, RDIST_F64 | RDIST_KEEP_Y, (int16_t *)sl.D.p, &g, sl.info_h,
                            st);
            if (e) return e;
            sl.graph = g;
            if (r0.q > 0) {
                std::memcpy(sl.pairs_h, r0.cur_host, (size_t)r0.q * 4);
                std::memcpy(sl.pairs_h + kMaxPairs, r0.goal_host, (size_t)r0.q * 4);
                int32_t *cur = (int32_t *)sl.pairs.p, *goal = cur + kMaxPairs;
                RD_HIP(hipMemcpyAsync(cur, sl.pairs_h, (size_t)2 * kMaxPairs * 4, hipMemcpyHostToDevice, st));
                e = rdist_next_hop(c, g, cur, goal, r0.q, r0.max_hops, (int32_t *)sl.paths.p, st);
                if (e) return e;
                RD_HIP(hipMemcpyAsync(r0.paths_host, sl.paths.p, pb, hipMemcpyDeviceToHost, st));
            }
        }
    } else {
        // one batched solve; path requests keep Y in the slot's buffer
        const int cnt = (int)batch.size();
        std::vector<size_t> offD(cnt), offY(cnt), offB(cnt), offQ(cnt), offP(cnt);
        size_t tD = 0, tY = 0, tB = 0, tQ = 0, tP = 0;
        for (int i = 0; i < cnt; ++i) {
            const rdist_request &r = batch[i].r;
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
            tP += align256((size_t)r.q * (r.max_hops + 1) * 4);
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
        e = solve_batch_into(c, st, cnt, ns.data(), As.data(), gs.data(), Ds.data(), Ys.data(), sl.info_h);
        if (e) return e;
        int32_t *cur_d = (int32_t *)sl.pairs.p, *goal_d = cur_d + tQ;
        if (tQ) {
            for (int i = 0; i < cnt; ++i) {
                const rdist_request &r = batch[i].r;
                if (r.kind != RDIST_QUERY_PATHS || r.q == 0) continue;
                std::memcpy(sl.pairs_h + offQ[i], r.cur_host, (size_t)r.q * 4);
                std::memcpy(sl.pairs_h + tQ + offQ[i], r.goal_host, (size_t)r.q * 4);
            }
            RD_HIP(hipMemcpyAsync(cur_d, sl.pairs_h, 2 * tQ * 4, hipMemcpyHostToDevice, st));
        }
        // every path request of the batch: one task table, one bitmap launch
        // and one path launch
        int ntask = 0, tblk = 0, tq = 0;
        for (int i = 0; i < cnt; ++i) {
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
            t.blk0 = tblk;
            t.q0 = tq;
            tblk += rd::path_task_blocks(r.n);
            tq += r.q;
        }
        if (ntask) {
            if ((e = grow(c, sl.tasks, sizeof(rd::PathTask) * (size_t)ntask))) return e;
            RD_HIP(hipMemcpyAsync(sl.tasks.p, sl.tasks_h, sizeof(rd::PathTask) * (size_t)ntask,
                                  hipMemcpyHostToDevice, st));
            {
                Timer tm(c, st, RDIST_K_NEXTHOP, 0.0, 0.0);
                rd::launch_paths_multi((const rd::PathTask *)sl.tasks.p, ntask, tblk, tq, st);
            }
            RD_HIP(hipGetLastError());
        }
        for (int i = 0; i < cnt; ++i) {
            const rdist_request &r = batch[i].r;
            if (r.kind == RDIST_QUERY_D)
                RD_HIP(hipMemcpyAsync(r.D_host, Ds[i], (size_t)r.n * r.n * 2, hipMemcpyDeviceToHost, st));
            else if (r.q > 0)
                RD_HIP(hipMemcpyAsync(r.paths_host, (char *)sl.paths.p + offP[i], (size_t)r.q * (r.max_hops + 1) * 4,
                                      hipMemcpyDeviceToHost, st));
        }
        s->st.batches += 1;
        s->st.batched_requests += cnt;
    }
    RD_HIP(hipEventRecord(sl.done, st));
    sl.busy = true;
    sl.reqs = batch;
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
        if (batchable(s->queue.front().r)) {
            // every batchable request in the queue, in order, while it fits
            for (auto it = s->queue.begin(); it != s->queue.end() && (int)batch.size() < s->max_batch;) {
                if (batchable(it->r) && fits(s, f + it->footprint)) {
                    f += it->footprint;
                    batch.push_back(*it);
                    it = s->queue.erase(it);
                } else if (batchable(it->r)) {
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
            for (auto it = batch.rbegin(); it != batch.rend(); ++it) s->queue.push_front(*it);
            s->st.queued = (int64_t)s->queue.size();
            Slot &sl = s->slots[k];
            if (sl.graph) { rdist_graph_release(sl.graph); sl.graph = nullptr; }
            return;
        }
        if (e) {
            Slot &sl = s->slots[k];
            (void)hipStreamSynchronize(sl.stream);
            if (sl.graph) { rdist_graph_release(sl.graph); sl.graph = nullptr; }
            for (auto &p : batch) fail_request(s, p, e);
        }
    }
}

void complete(rdist_server s, Slot &sl) {
    for (size_t i = 0; i < sl.reqs.size(); ++i) {
        const rdist_request &r = sl.reqs[i].r;
        if (r.info_host) *r.info_host = sl.info_h[i];
        s->finished.push_back(r.id);
        s->st.completed += 1;
    }
    if (sl.graph) {
        rdist_graph_release(sl.graph);
        sl.graph = nullptr;
    }
    s->st.in_flight -= (int64_t)sl.reqs.size();
    s->st.footprint_in_flight -= sl.footprint;
    sl.reqs.clear();
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
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc((void **)&sl.info_h, sizeof(rdist_info) * (size_t)max_batch, hipHostMallocDefault) !=
                hipSuccess ||
            hipHostMalloc((void **)&sl.pairs_h, (size_t)2 * kMaxPairs * 4 * max_batch, hipHostMallocDefault) !=
                hipSuccess ||
            hipHostMalloc((void **)&sl.tasks_h, sizeof(rd::PathTask) * (size_t)max_batch, hipHostMallocDefault) !=
                hipSuccess) {
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
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipSuccess) {
            complete(s, sl);
        } else if (q != hipErrorNotReady) {
            (void)hipGetLastError();
            for (auto &p : sl.reqs) fail_request(s, p, RDIST_E_HIP);
            s->st.in_flight -= (int64_t)sl.reqs.size();
            s->st.footprint_in_flight -= sl.footprint;
            sl.reqs.clear();
            sl.busy = false;
        }
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
        for (Slot &sl : s->slots) {
            if (sl.stream) (void)hipStreamSynchronize(sl.stream);
            if (sl.graph) rdist_graph_release(sl.graph);
            for (Buf *b : {&sl.D, &sl.Y, &sl.bits, &sl.paths, &sl.pairs, &sl.tasks}) release(s->ctx, *b);
            if (sl.info_h) (void)hipHostFree(sl.info_h);
            if (sl.pairs_h) (void)hipHostFree(sl.pairs_h);
            if (sl.tasks_h) (void)hipHostFree(sl.tasks_h);
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.stream) {
                release_stream_workspace(s->ctx, sl.stream);
                (void)hipStreamDestroy(sl.stream);
            }
        }
    }
    delete s;
}

}  // extern "C"
