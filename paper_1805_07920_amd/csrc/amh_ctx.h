// Private to the library: the context object and the host-side helpers
// shared by the translation units of the C-ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "amh_internal.h"
#include "amhmvs.h"

namespace amh {

struct View {
    int W = 0, H = 0;
    float *img = nullptr;   // float32 copy (reference use)
    void *quads = nullptr;  // gather layout (source use)
    int half = 0;
    double K[9], R[9], t[3];
};

struct NetState;  // proposal network (amh_nn_api.hip)

struct JobResult {
    int W = 0, H = 0;
    RefDev ref{};
    float4 *planes = nullptr;
    float *cost = nullptr;
    uint32_t *S = nullptr;
    int32_t *v = nullptr;
    // learned-proposal batches: network input, depth base and prediction of the job
    void *feats = nullptr;
    float *qref = nullptr;
    float *pred = nullptr;
    size_t cells = 0;
};

}  // namespace amh

using namespace amh;  // private header: the library's own translation units only

struct amh_ctx {
    amh_params p;
    int alloc_count = 0;      // device allocations made by this context
    int fail_alloc_at = 0;    // AMH_FAIL_ALLOC_AT at creation: that allocation reports out-of-memory (test hook)
    hipStream_t stream = nullptr;
    int device = 0;
    std::string err;
    int half = 0;
    std::vector<View> views;
    // current reference
    int ref = -1;
    std::vector<int> srcs;
    std::vector<ViewDev> h_viewc;
    ViewDev *d_viewc = nullptr;
    size_t viewc_cap = 0;
    RefDev refdev{};
    float4 *planes = nullptr;
    float *cost = nullptr;
    uint32_t *S = nullptr;
    int32_t *v = nullptr;
    size_t state_cap = 0;
    bool have_state = false;
    unsigned long long *counters = nullptr;
    // timing
    std::vector<hipEvent_t> ev;  // pairs: [2i] start, [2i+1] stop
    int n_timed = 0;
    hipEvent_t ev_init[2] = {nullptr, nullptr};
    bool init_timed = false;
    // launch configuration (autotuned): tile order of a launch, job order of a batch
    int cfg_order = 0;
    int cfg_job_order = 1;
    int cfg_waves = kDefaultTileRows;  // tile rows of the half-pass (2 or 4)
    int cfg_persist = 0;               // batches: every half-pass in one persistent launch (1) or one launch each
    // batch: per-job state, device tables and the captured graph of the last job list
    std::vector<JobResult> jobs;
    std::vector<int> batch_key;       // serialized job list of the captured graph
    hipStream_t cap_stream = nullptr;  // private stream for graph capture
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    BatchJobDev *d_jobs = nullptr;
    ViewDev *d_bviews = nullptr;
    int *d_tables = nullptr;
    unsigned long long *d_bcount = nullptr;  // [kCounterKinds * kCounterSlots] counts, [n_jobs] tiles done, [n_jobs + 1] clocks
    void *d_persist = nullptr;  // persistent launch: PersistArgs, PersistPhase table, work / barrier / fault counters
    unsigned *d_pfault = nullptr;  // ... its fault flag (inside d_persist)
    // workgroups of the persistent kernel measured resident at once, per (half, tile rows, largest view count)
    std::vector<std::vector<int>> persist_resident;
    int batch_jobs = 0;
    bool batch_ran = false;
    bool batch_stats = false;
    unsigned long long batch_counts[kCounterKinds] = {};
    // proposal network (weights, optimiser state, activations), created by amh_nn_init
    amh::NetState *net = nullptr;
    void *prop_feats = nullptr;   // amh_run_proposal: network input and prediction of the reference
    float *prop_pred = nullptr;
    float *prop_qref = nullptr;
    float *hyp = nullptr;         // amh_set_initial_hypotheses: packed per-pixel hypotheses (+ host staging)
    size_t hyp_cap = 0;           // floats
    size_t prop_cap = 0;          // cells
    // fusion workspace (amh_fuse): used marks, one view's dense outputs, tables
    void *fuse_ws = nullptr;
    size_t fuse_ws_cap = 0;
    std::vector<hipEvent_t> fuse_ev;  // timing = 1: a start/stop pair per fusion kernel launch
    float fuse_ms = 0.f;               // their total device time in the last amh_fuse
    int fuse_n = 0;
};

namespace amh {

void free_net(amh_ctx *c);
void free_fusion(amh_ctx *c);

amh_status fail(amh_ctx *c, amh_status s, const char *fmt, ...) __attribute__((format(printf, 3, 4)));

#define HIPCHK(c, expr)                                                                          \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) return fail((c), AMH_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// device allocation with an optional injected failure (AMH_FAIL_ALLOC_AT=n at amh_create: the context's
// n-th allocation fails, 1-based)
amh_status dalloc(amh_ctx *c, void **ptr, size_t bytes);

// proposal network (amh_nn_api.hip): reserve activations for `cells` level-0 cells, and a forward pass
// on an explicit stream that neither allocates nor synchronises (capturable)
amh_status nn_reserve(amh_ctx *c, size_t cells);
amh_status nn_forward_stream(amh_ctx *c, const void *feats, const float *q_ref, int n, int h, int w, float *out,
                             hipStream_t s);

}  // namespace amh
