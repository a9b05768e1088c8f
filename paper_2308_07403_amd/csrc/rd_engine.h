// rd_engine.h -- host-side state shared by the engine's translation units
// (internal to the library): the context, per-stream workspaces, device
// allocation against the HBM budget, per-kernel event timing, graph handles.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "../../include/rdist.h"
#include "rd_launch.h"

namespace rd {
namespace eng {

extern thread_local std::string g_last_error;

inline rdist_status fail(rdist_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

#define RD_HIP(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return ::rd::eng::fail(RDIST_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr int kB = 128;           // block size of the blocked solver = tile size
constexpr int kBatchMaxN = rd::kLvMaxN;   // largest graph the batched plans solve (larger: blocked plan)
constexpr int kPersistMaxN = 512;        // largest graph of the persistent kernel's in-workgroup solver

struct BatchPlan;   // rd_batch.hip

// A device allocation with its size, so the budget can be returned exactly.
struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct Workspace {
    int np_cap = 0;      // blocked plan: padded order the buffers below hold
    Buf M;               // np x np
    Buf Ut[2], V[2];     // 256 x np each (double-buffered by step parity)
    Buf Pt[2];           // 256 x 256
    Buf Ut2, V2, Pt2;    // scratch of the 256-block inverse (128x256, 128x256, 128^2)
    Buf small;           // out-degrees (n_cap + 1), flag, device info
    int n_cap = 0;
    hipStream_t aux = nullptr;    // lookahead stream (default priority)
    hipStream_t aux2 = nullptr;   // batched plans: the persistent kernel's stream
    hipEvent_t ev_er = nullptr, ev_panel = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;   // blocked plan (b = 256): the band update beside the second panel
    BatchPlan *transient = nullptr;   // batched plan rebuilt per call (not captured)
    // mixed precision: FP32 matrix, row product, column copy, FP64 diagonal
    // block, FP32 P, certification counters + slab flags, sparse rows of A,
    // residual and correction slabs
    Buf m32, v32, u32, s64, p32, cert, csr_cnt, csr_off, csr_col, r32, c32;
    Buf xi, ri;   // bf16 hi/lo parts of the FP32 inverse and of the scaled residual (interleaved)
    // goal rows: the two iteration states, and [info | bad flag | change flag | gamma^w table]
    Buf rv, rmisc, rgoals;
    Buf gb;               // gain bounds: two vectors of n doubles and the iteration's scratch
    int32_t *rflag_h = nullptr;   // pinned host copy of the change flag
    // a captured chunk of goal-row steps, replayed while its inputs stay the same
    hipGraph_t rows_graph = nullptr;
    hipGraphExec_t rows_exec = nullptr;
    const void *rows_key[6] = {};
    int64_t rows_key_n[3] = {};
    double *m() const { return (double *)M.p; }
    int32_t *outdeg() const { return (int32_t *)small.p; }
    int32_t *bad() const { return outdeg() + n_cap + 1; }
    rdist_info *dinfo() const {
        return (rdist_info *)((char *)small.p + 256 * ((sizeof(int32_t) * (n_cap + 2) + 255) / 256));
    }
};

struct TimedLaunch {
    hipEvent_t a, b;
    int which;
    double flops, bytes;
};

// Tuned parameters of the batched plans (rd_batch.hip).
struct BatchTuning {
    int persist_max_n = 128;   // graphs with n <= this go to the persistent kernel
    int persist_grid = 0;      // workgroups of the persistent kernel (0: half the compute units)
};

}  // namespace eng
}  // namespace rd

struct rdist_graph_s {
    rdist_ctx ctx = nullptr;
    double *Y = nullptr;
    int n = 0, ld = 0;
    unsigned long long *succ = nullptr;   // successor bitmaps (n x ceil(n/64))
    // for edge changes: the graph's own adjacency or weights (n x n), its
    // out-degrees, its info (gain, status), scratch of an update
    uint8_t *A = nullptr;
    int32_t *outdeg = nullptr;
    rdist_info *ginfo = nullptr;
    double *sm = nullptr;
    uint16_t *beta = nullptr;             // per-entry error bounds, made by the first change,
    int32_t *hist = nullptr;              // and in the same allocation the out-degree histogram
    rdist_info *hinfo = nullptr;          // pinned host copy of a change's info
    double *bs = nullptr;                 // scratch of batched changes, made by the first batch
    int weighted = 0;
    bool changed = false;                 // Y carries edge changes made since its inversion
    void *aux = nullptr;                  // one allocation holding succ .. sm
    size_t ybytes = 0, aux_bytes = 0, beta_bytes = 0, bs_bytes = 0;
    size_t bytes = 0;                     // their sum, counted in the context's budget
};

struct rdist_ctx_s {
    int device = 0;
    size_t budget = 0;
    size_t in_use = 0;
    bool threadsafe = false;
    std::recursive_mutex mu;
    std::map<hipStream_t, rd::eng::Workspace> ws;
    std::set<rdist_graph_s *> graphs;
    uint32_t timing_mask = 0;   // bit k: kernel class k is timed
    bool timing_hold = false;   // no launch is timed while set (rdist_timing_hold)
    std::vector<rd::eng::TimedLaunch> pending;
    std::vector<hipEvent_t> event_pool;
    rdist_kernel_stats stats[RDIST_K_COUNT];
    int num_cu = 256;
    // batched plans cached with their instantiated HIP graphs
    std::vector<rd::eng::BatchPlan *> plans;
    uint64_t plan_clock = 0;
    hipStream_t capture = nullptr, capture_aux = nullptr, capture_aux2 = nullptr;   // batch graph capture
    std::string tile_cache_path;
    std::vector<std::pair<std::string, rd::eng::BatchTuning>> tuned;   // batch class -> tuning
    bool tuned_dirty = false;
    void *noalloc_scratch = nullptr;   // device address of this device's static scratch (rdist_solve_noalloc)
    std::string noalloc_error;         // why that address is unavailable, if it is
};

namespace rd {
namespace eng {

struct Guard {
    rdist_ctx c;
    explicit Guard(rdist_ctx c_) : c(c_) { if (c->threadsafe) c->mu.lock(); }
    ~Guard() { if (c->threadsafe) c->mu.unlock(); }
};

rdist_status dalloc(rdist_ctx c, void **p, size_t bytes);
void dfree(rdist_ctx c, void *p, size_t bytes);
rdist_status ensure(rdist_ctx c, Buf &b, size_t bytes);
// ensure with headroom: a buffer that has to grow takes 1.5x its old size
// (or the request, if larger), falling back to the exact size.
rdist_status ensure_grow(rdist_ctx c, Buf &b, size_t bytes);
void release(rdist_ctx c, Buf &b);
rdist_status ensure_small(rdist_ctx c, Workspace &w, int n);
rdist_status ensure_capture_streams(rdist_ctx c);   // the context's streams for graph capture (rd_batch.hip)
rdist_status ensure_aux(Workspace &w);
rdist_status ensure_aux2(Workspace &w);

hipEvent_t take_event(rdist_ctx c);

// Set while this thread runs a call that may not create events (the
// allocation-free solve): its launches are never timed.
extern thread_local bool g_untimed;

// Records an event pair around the launches made during its lifetime when
// timing is on; drain_timing folds finished pairs into the per-kernel stats.
struct Timer {
    rdist_ctx c;
    hipStream_t s;
    int which;
    double flops, bytes;
    hipEvent_t a = nullptr;
    Timer(rdist_ctx c_, hipStream_t s_, int w, double f, double b) : c(c_), s(s_), which(w), flops(f), bytes(b) {
        if ((c->timing_mask & (1u << w)) && !c->timing_hold && !g_untimed) {
            a = take_event(c);
            if (a) (void)hipEventRecord(a, s);
        }
    }
    ~Timer() {
        if (!a) return;
        hipEvent_t b2 = take_event(c);
        if (!b2) return;
        (void)hipEventRecord(b2, s);
        c->pending.push_back(TimedLaunch{a, b2, which, flops, bytes});
    }
};

void drain_timing(rdist_ctx c);
rdist_status copy_info(rdist_info *host, const rdist_info *dev, int count, hipStream_t s);
// A graph handle owning Y (ld) and ybytes of it; copies A, builds the
// successor bitmaps and out-degrees and keeps a copy of the solve's info
// (dinfo, device), all on stream s.
rdist_status make_graph(rdist_ctx c, int n, double *Y, int ld, size_t ybytes, const uint8_t *A, hipStream_t s,
                        rdist_graph *out, const rdist_info *dinfo, bool weighted);
void release_graph_locked(rdist_graph g);
rdist_status check_flags(uint32_t flags);
rdist_status check_gamma(double gamma);
rdist_status solve_blocked(rdist_ctx c, const uint8_t *A, int n, double gamma, uint32_t flags, int16_t *D,
                           rdist_graph *keep, rdist_info *info, hipStream_t s);

// rd_mixed.hip
rdist_status solve_mixed(rdist_ctx c, const uint8_t *A, int n, double gamma, uint32_t flags, int16_t *D,
                         rdist_info *info, hipStream_t s);

void free_workspace(rdist_ctx c, Workspace &w);
void release_stream_workspace(rdist_ctx c, hipStream_t s);

// rd_batch.hip
void destroy_plans(rdist_ctx c);
void free_transient_plan(rdist_ctx c, Workspace &w);
// Eager batched solve on stream s for the request loop: every n <= kBatchMaxN,
// threshold T = 128 whatever the batch.  ext_y[g] (nullable array, nullable
// entries): caller-owned Y of graph g (np x np, ld np = n rounded up to 128);
// info_host (nullable, pinned, count entries) receives the infos at the end of
// stream s.  marks (nullable, kBatchMarks events): marks[0] is recorded once
// the graphs with n <= 128 are final, marks[t] once those with
// ceil(n / 128) = t are (each only if such graphs exist); *tail (nullable)
// receives the stream the graphs with n <= 128 finish on (work queued there
// after the call runs after them), *info_dev the device infos (valid until
// the next batched call on s).
constexpr int kBatchMarks = kBatchMaxN / kB + 1;
rdist_status solve_batch_into(rdist_ctx c, hipStream_t s, int count, const int32_t *n, const uint8_t *const *A,
                              const double *gamma, int16_t *const *D, double *const *ext_y, rdist_info *info_host,
                              hipEvent_t *marks, hipStream_t *tail, const rdist_info **info_dev);
void load_tile_cache(rdist_ctx c);
void save_tile_cache(rdist_ctx c);

}  // namespace eng
}  // namespace rd
