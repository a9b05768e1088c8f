// rd_host.cpp -- host-only helpers of the engine (no device code): device
// allocation against the HBM budget, per-stream auxiliary streams, the event
// pool of the timing, argument checks and the thread-local error message.
// Kept apart from the kernels' sources so that the batched plans' host logic
// (rd_batch.hip, also free of device code) can be built and exercised on a
// CPU against a stand-in of the HIP runtime.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "../../include/rdist.h"
#include "rd_engine.h"

namespace rd {
namespace eng {

thread_local std::string g_last_error;
thread_local bool g_untimed = false;

rdist_status dalloc(rdist_ctx c, void **p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) return RDIST_OK;
    if (c->budget) {
        if (bytes > c->budget) return fail(RDIST_E_NOMEM, "request exceeds the HBM budget");
        if (c->in_use + bytes > c->budget) return fail(RDIST_E_AGAIN, "HBM budget in use");
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(RDIST_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    c->in_use += bytes;
    return RDIST_OK;
}

void dfree(rdist_ctx c, void *p, size_t bytes) {
    if (!p) return;
    (void)hipFree(p);
    c->in_use -= std::min(bytes, c->in_use);
}

rdist_status ensure(rdist_ctx c, Buf &b, size_t bytes) {
    if (b.p && b.bytes >= bytes) return RDIST_OK;
    dfree(c, b.p, b.bytes);
    b.p = nullptr;
    b.bytes = 0;
    rdist_status st = dalloc(c, &b.p, bytes);
    if (st == RDIST_OK) b.bytes = bytes;
    return st;
}

rdist_status ensure_grow(rdist_ctx c, Buf &b, size_t bytes) {
    if (b.p && b.bytes >= bytes) return RDIST_OK;
    const size_t want = std::max(bytes, b.bytes + b.bytes / 2);
    if (want > bytes && ensure(c, b, want) == RDIST_OK) return RDIST_OK;
    return ensure(c, b, bytes);
}

void release(rdist_ctx c, Buf &b) {
    dfree(c, b.p, b.bytes);
    b.p = nullptr;
    b.bytes = 0;
}

// The workspace's second auxiliary stream (the batched plans' persistent
// kernel), created on first use.
rdist_status ensure_aux2(Workspace &w) {
    if (!w.aux2 && hipStreamCreateWithFlags(&w.aux2, hipStreamNonBlocking) != hipSuccess) {
        w.aux2 = nullptr;
        return fail(RDIST_E_HIP, "hipStreamCreateWithFlags failed");
    }
    if (!w.ev_fork && hipEventCreateWithFlags(&w.ev_fork, hipEventDisableTiming) != hipSuccess) {
        w.ev_fork = nullptr;
        return fail(RDIST_E_HIP, "hipEventCreateWithFlags failed");
    }
    if (!w.ev_join && hipEventCreateWithFlags(&w.ev_join, hipEventDisableTiming) != hipSuccess) {
        w.ev_join = nullptr;
        return fail(RDIST_E_HIP, "hipEventCreateWithFlags failed");
    }
    return RDIST_OK;
}

// The workspace's auxiliary stream (default priority) and its events.
rdist_status ensure_aux(Workspace &w) {
    if (!w.aux) {
        if (hipStreamCreateWithFlags(&w.aux, hipStreamNonBlocking) != hipSuccess) {
            w.aux = nullptr;
            return fail(RDIST_E_HIP, "hipStreamCreateWithFlags failed");
        }
        if (hipEventCreateWithFlags(&w.ev_er, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&w.ev_panel, hipEventDisableTiming) != hipSuccess)
            return fail(RDIST_E_HIP, "hipEventCreateWithFlags failed");
    }
    return RDIST_OK;
}

// ---- timing ----
hipEvent_t take_event(rdist_ctx c) {
    if (!c->event_pool.empty()) {
        hipEvent_t e = c->event_pool.back();
        c->event_pool.pop_back();
        return e;
    }
    // timing only: no system-scope fence at the record (nothing on the host
    // reads device memory through these events), so timed launches run as
    // they would untimed
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

rdist_status check_flags(uint32_t flags) {
    const uint32_t known = RDIST_MIXED_F32 | RDIST_KEEP_Y | RDIST_PLAN_SMALL | RDIST_PLAN_BLOCKED |
                           RDIST_UNFUSED_EPILOGUE | RDIST_BLOCK_128 | RDIST_BLOCK_256 | RDIST_NO_GRAPH |
                           RDIST_WEIGHTED;
    if (flags & ~known) return fail(RDIST_E_ARG, "unknown flag bits");
    if ((flags & RDIST_BLOCK_128) && (flags & RDIST_BLOCK_256)) return fail(RDIST_E_ARG, "two block widths");
    if ((flags & RDIST_PLAN_SMALL) && (flags & RDIST_PLAN_BLOCKED)) return fail(RDIST_E_ARG, "two plan flags");
    if ((flags & RDIST_MIXED_F32) && (flags & (RDIST_KEEP_Y | RDIST_PLAN_SMALL | RDIST_PLAN_BLOCKED)))
        return fail(RDIST_E_ARG, "RDIST_MIXED_F32 takes no KEEP_Y or plan flag");
    if ((flags & RDIST_WEIGHTED) && (flags & (RDIST_MIXED_F32 | RDIST_PLAN_SMALL)))
        return fail(RDIST_E_ARG, "RDIST_WEIGHTED runs on the FP64 blocked plan only");
    return RDIST_OK;
}

rdist_status check_gamma(double gamma) {
    if (!std::isfinite(gamma) || gamma == 0.0) return fail(RDIST_E_ARG, "gamma must be finite and non-zero");
    if (gamma > 0.0 && !(gamma < 1.0)) return fail(RDIST_E_ARG, "explicit gamma must lie in (0, 1)");
    if (gamma < 0.0 && !(-gamma < 1.0)) return fail(RDIST_E_ARG, "AUTO factor |gamma| must lie in (0, 1)");
    return RDIST_OK;
}

}  // namespace eng
}  // namespace rd
