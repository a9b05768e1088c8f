// Host-only stand-in of the HIP runtime calls declared in hip/hip_runtime.h
// (see there).  Single-threaded; every check failure aborts the process with
// a message on stderr, so a harness run under AddressSanitizer either ends
// cleanly or names the first misuse.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <set>
#include <string>
#include <vector>

struct ihipGraph_t;

struct ihipStream_t {
    ihipGraph_t *capturing = nullptr;   // graph this stream records into
    long cap_seq = 0;                   // operations recorded on it in that capture
};

struct ihipEvent_t {
    ihipGraph_t *cap_graph = nullptr;   // capture the record happened in (nullptr: eager)
    hipStream_t cap_stream = nullptr;
    long cap_seq = 0;
};

struct Op {
    std::string what;
    std::function<void()> work;
};

struct ihipGraph_t {
    hipStream_t origin = nullptr;
    std::set<hipStream_t> members;
    std::map<hipStream_t, long> joined;   // member -> ops of it the origin has waited for
    bool open = true;
    std::shared_ptr<std::vector<Op>> ops = std::make_shared<std::vector<Op>>();
};

struct ihipGraphExec_t {
    std::shared_ptr<std::vector<Op>> ops;
};

namespace {

[[noreturn]] void die(const std::string &msg) {
    std::fprintf(stderr, "hip stand-in: %s\n", msg.c_str());
    std::fflush(stderr);
    std::abort();
}

std::map<uintptr_t, size_t> g_dev;          // live device allocations
std::map<uintptr_t, size_t> g_host;         // live pinned host allocations
std::set<hipStream_t> g_streams;            // live streams (the null stream is always live)
std::set<hipEvent_t> g_events;
std::set<hipGraph_t> g_graphs;
std::set<hipGraphExec_t> g_execs;
ihipStream_t g_null_stream;                 // state of the null stream
hipstub::Counters g_cnt{};
float g_next_ms = 1.0f;

ihipStream_t *state(hipStream_t s, const char *call) {
    if (!s) return &g_null_stream;
    if (!g_streams.count(s)) die(std::string(call) + ": stream is not live (destroyed or never created)");
    return s;
}

void check_event(hipEvent_t e, const char *call) {
    if (!e || !g_events.count(e)) die(std::string(call) + ": event is not live");
}

bool in_map(const std::map<uintptr_t, size_t> &m, const void *p, size_t bytes) {
    const uintptr_t a = (uintptr_t)p;
    auto it = m.upper_bound(a);
    if (it == m.begin()) return false;
    --it;
    return a >= it->first && a + bytes <= it->first + it->second;
}

}  // namespace

namespace hipstub {

void enqueue(hipStream_t s, const char *what, std::function<void()> work) {
    ihipStream_t *st = state(s, what);
    if (st->capturing) {
        st->cap_seq += 1;
        st->capturing->ops->push_back(Op{what, std::move(work)});
        return;
    }
    g_cnt.eager_ops += 1;
    work();
}

bool device_range_live(const void *p, size_t bytes) { return in_map(g_dev, p, bytes); }
Counters counters() { return g_cnt; }
size_t live_device_allocations() { return g_dev.size(); }
size_t live_device_bytes() {
    size_t b = 0;
    for (auto &kv : g_dev) b += kv.second;
    return b;
}
void set_next_elapsed(float ms) { g_next_ms = ms; }

}  // namespace hipstub

const char *hipGetErrorString(hipError_t e) {
    switch (e) {
        case hipSuccess: return "hipSuccess";
        case hipErrorInvalidValue: return "hipErrorInvalidValue";
        case hipErrorOutOfMemory: return "hipErrorOutOfMemory";
        case hipErrorStreamCaptureUnjoined: return "hipErrorStreamCaptureUnjoined";
        default: return "hipError(stand-in)";
    }
}
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipSetDevice(int) { return hipSuccess; }

hipError_t hipMalloc(void **p, size_t bytes) {
    if (!p) die("hipMalloc: NULL out pointer");
    *p = std::malloc(bytes ? bytes : 1);
    if (!*p) return hipErrorOutOfMemory;
    g_dev[(uintptr_t)*p] = bytes;
    g_cnt.mallocs += 1;
    return hipSuccess;
}

hipError_t hipFree(void *p) {
    if (!p) return hipSuccess;
    auto it = g_dev.find((uintptr_t)p);
    if (it == g_dev.end()) die("hipFree: pointer is not a live device allocation");
    g_dev.erase(it);
    g_cnt.frees += 1;
    std::free(p);
    return hipSuccess;
}

hipError_t hipHostMalloc(void **p, size_t bytes, unsigned) {
    *p = std::malloc(bytes ? bytes : 1);
    g_host[(uintptr_t)*p] = bytes;
    return hipSuccess;
}

hipError_t hipHostFree(void *p) {
    if (!p) return hipSuccess;
    auto it = g_host.find((uintptr_t)p);
    if (it == g_host.end()) die("hipHostFree: pointer is not a live pinned allocation");
    g_host.erase(it);
    std::free(p);
    return hipSuccess;
}

hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind kind, hipStream_t s) {
    const bool dst_dev = kind == hipMemcpyHostToDevice || kind == hipMemcpyDeviceToDevice;
    const bool src_dev = kind == hipMemcpyDeviceToHost || kind == hipMemcpyDeviceToDevice;
    hipstub::enqueue(s, "hipMemcpyAsync", [=]() {
        if (dst_dev && !in_map(g_dev, dst, bytes)) die("hipMemcpyAsync: destination outside a live device allocation");
        if (src_dev && !in_map(g_dev, src, bytes)) die("hipMemcpyAsync: source outside a live device allocation");
        if (!src_dev && kind == hipMemcpyHostToDevice && !in_map(g_host, src, bytes))
            die("hipMemcpyAsync: host source is not live pinned memory");
        std::memmove(dst, src, bytes);
    });
    return hipSuccess;
}

hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
    *s = new ihipStream_t();
    g_streams.insert(*s);
    return hipSuccess;
}

hipError_t hipStreamDestroy(hipStream_t s) {
    ihipStream_t *st = state(s, "hipStreamDestroy");
    if (st->capturing) die("hipStreamDestroy: stream is capturing");
    g_streams.erase(s);
    delete s;
    return hipSuccess;
}

hipError_t hipStreamSynchronize(hipStream_t s) {
    ihipStream_t *st = state(s, "hipStreamSynchronize");
    if (st->capturing) die("hipStreamSynchronize: stream is capturing");
    return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t *e) {
    *e = new ihipEvent_t();
    g_events.insert(*e);
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }

hipError_t hipEventDestroy(hipEvent_t e) {
    check_event(e, "hipEventDestroy");
    g_events.erase(e);
    delete e;
    return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
    check_event(e, "hipEventRecord");
    ihipStream_t *st = state(s, "hipEventRecord");
    if (st->capturing) {
        e->cap_graph = st->capturing;
        e->cap_stream = s;
        e->cap_seq = st->cap_seq;
    } else {
        e->cap_graph = nullptr;
    }
    return hipSuccess;
}

hipError_t hipEventSynchronize(hipEvent_t e) {
    check_event(e, "hipEventSynchronize");
    if (e->cap_graph) die("hipEventSynchronize: event was recorded during a capture");
    return hipSuccess;
}

hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b) {
    check_event(a, "hipEventElapsedTime");
    check_event(b, "hipEventElapsedTime");
    *ms = g_next_ms;
    g_next_ms = 1.0f;
    return hipSuccess;
}

hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
    check_event(e, "hipStreamWaitEvent");
    ihipStream_t *st = state(s, "hipStreamWaitEvent");
    ihipGraph_t *g = e->cap_graph;
    if (g && !g_graphs.count(g)) die("hipStreamWaitEvent: event of a finished capture");
    if (g && g->open) {
        if (st->capturing && st->capturing != g) die("hipStreamWaitEvent: stream captures another graph");
        if (!st->capturing) {   // the stream joins the capture
            st->capturing = g;
            st->cap_seq = 0;
            g->members.insert(s);
        }
        if (s == g->origin && e->cap_stream != g->origin) {
            long &j = g->joined[e->cap_stream];
            j = std::max(j, e->cap_seq);
        }
        return hipSuccess;
    }
    if (st->capturing) die("hipStreamWaitEvent: capturing stream waits on an event from outside the capture");
    return hipSuccess;
}

hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
    ihipStream_t *st = state(s, "hipStreamBeginCapture");
    if (!s) die("hipStreamBeginCapture: the null stream cannot be captured");
    if (st->capturing) die("hipStreamBeginCapture: stream already capturing");
    auto *g = new ihipGraph_t();
    g->origin = s;
    g->members.insert(s);
    g_graphs.insert(g);
    st->capturing = g;
    st->cap_seq = 0;
    g_cnt.captures += 1;
    return hipSuccess;
}

hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *out) {
    ihipStream_t *st = state(s, "hipStreamEndCapture");
    ihipGraph_t *g = st->capturing;
    if (!g || g->origin != s) die("hipStreamEndCapture: stream is not the origin of a capture");
    hipError_t rc = hipSuccess;
    for (hipStream_t m : g->members) {
        if (m == s) continue;
        ihipStream_t *ms = state(m, "hipStreamEndCapture");
        auto it = g->joined.find(m);
        if (ms->cap_seq > 0 && (it == g->joined.end() || it->second < ms->cap_seq)) rc = hipErrorStreamCaptureUnjoined;
        ms->capturing = nullptr;
    }
    st->capturing = nullptr;
    g->open = false;
    if (rc != hipSuccess) {
        g_graphs.erase(g);
        delete g;
        *out = nullptr;
        return rc;
    }
    *out = g;
    return hipSuccess;
}

hipError_t hipGraphInstantiate(hipGraphExec_t *exec, hipGraph_t g, hipGraphNode_t *, char *, size_t) {
    if (!g || !g_graphs.count(g)) die("hipGraphInstantiate: graph is not live");
    *exec = new ihipGraphExec_t{std::make_shared<std::vector<Op>>(*g->ops)};
    g_execs.insert(*exec);
    return hipSuccess;
}

hipError_t hipGraphLaunch(hipGraphExec_t exec, hipStream_t s) {
    if (!exec || !g_execs.count(exec)) die("hipGraphLaunch: executable graph is not live");
    ihipStream_t *st = state(s, "hipGraphLaunch");
    if (st->capturing) die("hipGraphLaunch: stand-in does not nest graphs");
    g_cnt.graph_launches += 1;
    for (const Op &o : *exec->ops) {
        g_cnt.graph_ops += 1;
        o.work();
    }
    return hipSuccess;
}

hipError_t hipGraphExecDestroy(hipGraphExec_t exec) {
    if (!exec || !g_execs.count(exec)) die("hipGraphExecDestroy: executable graph is not live");
    g_execs.erase(exec);
    delete exec;
    return hipSuccess;
}

hipError_t hipGraphDestroy(hipGraph_t g) {
    if (!g || !g_graphs.count(g)) die("hipGraphDestroy: graph is not live");
    g_graphs.erase(g);
    delete g;
    return hipSuccess;
}
