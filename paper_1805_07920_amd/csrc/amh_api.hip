// Host runtime and C-ABI of the checkerboard PatchMatch library (include/amhmvs.h).
// Validates every argument before touching HIP, owns all device buffers of a
// context, and orders all work on the context's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "amh_ctx.h"

using namespace amh;

// ---------------------------------------------------------------------------
// Storage of the allocation-free run (amh_run_checkerboard_static): the warp
// constants of the reference's sources and the per-pixel state (planes, cost,
// view masks, best views) live in this file-scope device array, one copy per
// GPU, held until the process ends.  On the host the array's name only stands
// for the symbol: kernels receive its device address, looked up once per
// device with hipGetSymbolAddress when a context is first created there.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kStaticAlign = 256;
constexpr size_t static_align(size_t b) { return (b + kStaticAlign - 1) & ~(kStaticAlign - 1); }
constexpr size_t kStaticMaxPixels = AMH_STATIC_MAX_PIXELS;
constexpr size_t kStaticViewcOff = 0;
constexpr size_t kStaticPlanesOff = kStaticViewcOff + static_align(sizeof(ViewDev) * kMaxSrc);
constexpr size_t kStaticCostOff = kStaticPlanesOff + static_align(kStaticMaxPixels * sizeof(float4));
constexpr size_t kStaticSOff = kStaticCostOff + static_align(kStaticMaxPixels * sizeof(float));
constexpr size_t kStaticVOff = kStaticSOff + static_align(kStaticMaxPixels * sizeof(uint32_t));
constexpr size_t kStaticBytes = kStaticVOff + static_align(kStaticMaxPixels * sizeof(int32_t));

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

constexpr int kStaticMaxDevices = 64;
std::mutex g_static_mu;
unsigned char *g_static_ptr[kStaticMaxDevices] = {};
hipError_t g_static_err[kStaticMaxDevices] = {};
bool g_static_done[kStaticMaxDevices] = {};

// Called with `device` current: looks up that device's copy of the array once, and returns the result of
// that lookup (the address, or the error that left it unknown).
hipError_t static_scratch(int device, unsigned char **ptr) {
    *ptr = nullptr;
    if (device < 0 || device >= kStaticMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_done[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_static_err[device] = e;
        g_static_ptr[device] = e == hipSuccess ? static_cast<unsigned char *>(p) : nullptr;
        g_static_done[device] = true;
    }
    *ptr = g_static_ptr[device];
    return g_static_err[device];
}

}  // namespace

namespace amh {

amh_status fail(amh_ctx *c, amh_status s, const char *fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return s;
}

amh_status dalloc(amh_ctx *c, void **ptr, size_t bytes) {
    if (++c->alloc_count == c->fail_alloc_at)
        return fail(c, AMH_E_OOM, "injected allocation failure (%zu bytes)", bytes);
    hipError_t e = hipMalloc(ptr, bytes ? bytes : 16);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(c, AMH_E_OOM, "hipMalloc(%zu) failed: out of memory", bytes);
    if (e != hipSuccess) return fail(c, AMH_E_HIP, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    return AMH_OK;
}

}  // namespace amh

namespace {

bool finite_all(const double *a, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

amh_status check_params(amh_ctx *c, const amh_params *p) {
    if (!p) return fail(c, AMH_E_INVALID_ARG, "params is NULL");
    if (!(p->depth_min > 0.f) || !(p->depth_max > p->depth_min) || !std::isfinite(p->depth_max))
        return fail(c, AMH_E_INVALID_ARG, "need 0 < depth_min < depth_max < inf");
    if (!(p->sigma_color > 0.f) || !(p->sigma_spatial > 0.f) || !std::isfinite(p->sigma_color) ||
        !std::isfinite(p->sigma_spatial))
        return fail(c, AMH_E_INVALID_ARG, "sigma_color and sigma_spatial must be positive and finite");
    if (!(p->alpha > 0.f) || !(p->beta > 0.f) || !std::isfinite(p->tau_mc_init) || !std::isfinite(p->tau_up))
        return fail(c, AMH_E_INVALID_ARG, "alpha and beta must be positive; thresholds finite");
    if (p->n1 < 0 || p->n1 > 8 || p->n2 < 0 || p->n2 > 9 || p->k < 1 || p->k > kMaxSrc)
        return fail(c, AMH_E_INVALID_ARG, "need 0 <= n1 <= 8, 0 <= n2 <= 9, 1 <= k <= 32");
    if ((p->refine != 0 && p->refine != 1) || (p->include_self != 0 && p->include_self != 1) ||
        (p->timing != 0 && p->timing != 1))
        return fail(c, AMH_E_INVALID_ARG, "refine, include_self and timing are 0 or 1");
    if ((p->sym_prop < 0 || p->sym_prop > 2) || (p->heuristic_views != 0 && p->heuristic_views != 1) ||
        (p->bilateral_squared != 0 && p->bilateral_squared != 1))
        return fail(c, AMH_E_INVALID_ARG, "sym_prop is 0, 1 or 2; heuristic_views and bilateral_squared 0 or 1");
    if (p->sweep_sources < 0 || p->sweep_sources > kMaxSrc)
        return fail(c, AMH_E_INVALID_ARG, "sweep_sources %d outside [0, %d]", p->sweep_sources, kMaxSrc);
    if (!(p->conf_min >= 0.f && p->conf_min <= 1.f)) return fail(c, AMH_E_INVALID_ARG, "conf_min must be in [0, 1]");
    return AMH_OK;
}

amh_status check_camera(amh_ctx *c, const amh_camera &cam, int i) {
    if (!finite_all(cam.K, 9) || !finite_all(cam.R, 9) || !finite_all(cam.t, 3))
        return fail(c, AMH_E_INVALID_ARG, "camera %d has non-finite entries", i);
    if (cam.K[3] != 0.0 || cam.K[6] != 0.0 || cam.K[7] != 0.0 || cam.K[8] == 0.0)
        return fail(c, AMH_E_UNSUPPORTED, "camera %d: K must be upper triangular with K[8] != 0", i);
    const double fx = cam.K[0] / cam.K[8], fy = cam.K[4] / cam.K[8];
    if (fx == 0.0 || fy == 0.0) return fail(c, AMH_E_INVALID_ARG, "camera %d: singular K", i);
    return AMH_OK;
}

MethodDev method_dev(const amh_params &p, int t) {
    MethodDev m;
    m.d_min = p.depth_min;
    m.d_max = p.depth_max;
    m.inv_2sc2 = (float)(1.0 / (2.0 * (double)p.sigma_color * p.sigma_color));
    m.inv_2sx2 = (float)(1.0 / (2.0 * (double)p.sigma_spatial * p.sigma_spatial));
    m.tau = (float)((double)p.tau_mc_init * std::exp(-(double)t * t / (double)p.alpha));
    m.tau_up = p.tau_up;
    m.inv_2b2 = (float)(1.0 / (2.0 * (double)p.beta * p.beta));
    m.n1 = p.n1;
    m.n2 = p.n2;
    m.k = p.k;
    m.include_self = p.include_self;
    m.refine = p.refine;
    m.seed = p.seed;
    m.sym_prop = p.sym_prop;
    m.heuristic = p.heuristic_views;
    m.bil_sq = p.bilateral_squared;
    m.q_lo = 1.0 / ((double)p.depth_max * (1.0 + 1e-5));
    m.q_hi = 1.0 / ((double)p.depth_min * (1.0 - 1e-5));
    return m;
}

void kinv_upper(const double Kin[9], double &a, double &b, double &cc, double &e, double &f) {
    const double s = Kin[8];
    const double fx = Kin[0] / s, sk = Kin[1] / s, cx = Kin[2] / s, fy = Kin[4] / s, cy = Kin[5] / s;
    a = 1.0 / fx;
    b = -sk / (fx * fy);
    cc = (sk * cy - cx * fy) / (fx * fy);
    e = 1.0 / fy;
    f = -cy / fy;
}

void mat3_mul(const double *A, const double *B, double *C) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

// warp constants of source view j relative to reference view r
ViewDev view_dev(const View &r, const View &s) {
    double Rrel[9], RrT[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) RrT[3 * i + j] = r.R[3 * j + i];
    mat3_mul(s.R, RrT, Rrel);
    double trel[3];
    for (int i = 0; i < 3; ++i)
        trel[i] = s.t[i] - (Rrel[3 * i] * r.t[0] + Rrel[3 * i + 1] * r.t[1] + Rrel[3 * i + 2] * r.t[2]);
    double a, b, cc, e, f;
    kinv_upper(r.K, a, b, cc, e, f);
    const double Kinv[9] = {a, b, cc, 0, e, f, 0, 0, 1};
    double Ks[9];
    for (int i = 0; i < 9; ++i) Ks[i] = s.K[i] / s.K[8];
    double KR[9];
    mat3_mul(Ks, Rrel, KR);
    ViewDev v;
    mat3_mul(KR, Kinv, v.A);
    for (int i = 0; i < 3; ++i) v.b[i] = Ks[3 * i] * trel[0] + Ks[3 * i + 1] * trel[1] + Ks[3 * i + 2] * trel[2];
    v.quads = s.quads;
    v.W = s.W;
    v.H = s.H;
    return v;
}

void free_view(View &v) {
    if (v.img) (void)hipFree(v.img);
    if (v.quads) (void)hipFree(v.quads);
    v.img = nullptr;
    v.quads = nullptr;
}

void free_job(JobResult &j) {
    for (void *p : {(void *)j.planes, (void *)j.cost, (void *)j.S, (void *)j.v, j.feats, (void *)j.qref, (void *)j.pred})
        if (p) (void)hipFree(p);
    j = JobResult{};
}

PassArgs pass_args(amh_ctx *c, int t, int colour) {
    PassArgs a;
    a.ref = c->refdev;
    a.views = c->d_viewc;
    a.n_src = (int)c->srcs.size();
    a.m = method_dev(c->p, t);
    a.st = StateDev{c->planes, c->cost, c->S, c->v};
    a.t = t;
    a.colour = colour;
    const int W = c->refdev.W, H = c->refdev.H;
    const int per_row = (W + 1) / 2;  // same-colour pixels per row (upper bound)
    a.tiles_x = (per_row + kTilePix - 1) / kTilePix;
    const int tiles_y = (H + c->cfg_waves - 1) / c->cfg_waves;
    a.n_tiles = a.tiles_x * tiles_y;
    a.counters = c->counters;
    a.order = c->cfg_order;
    a.waves = c->cfg_waves;
    return a;
}

// cells of the proposal grid along a side of n pixels: 1/4 resolution rounded up to a multiple of 8
int cell_rows(int n) { return 8 * ((n + 31) / 32); }

// plane-sweep arguments of a reference (proposal input)
SweepArgs sweep_args(amh_ctx *c, const RefDev &ref, const ViewDev *views, int n_src, void *feats, float *q_ref,
                     unsigned long long *counters) {
    SweepArgs a;
    a.ref = ref;
    a.views = views;
    a.n_net = std::min(c->p.sweep_sources > 0 ? c->p.sweep_sources : kNetSrc, n_src);
    a.m = method_dev(c->p, 0);
    a.h4 = cell_rows(ref.H);
    a.w4 = cell_rows(ref.W);
    a.sub = std::max(1, (ref.W + 80) / 160);  // one sweep step moves a near source's warp by ~2 px
    const double qf = 1.0 / (double)c->p.depth_max, qn = 1.0 / (double)c->p.depth_min;
    a.q_far = (float)qf;
    a.q_step = (float)((qn - qf) / (kSweepCoarse * a.sub));
    a.feats = static_cast<unsigned short *>(feats);
    a.q_ref = q_ref;
    a.counters = counters;
    return a;
}

// initialisation of both colours: random planes, or per-cell predictions where usable
amh_status init_state(amh_ctx *c, const float *pred, int pred_w, int cell) {
    const int half = c->half;
    if (c->p.timing) {
        for (int i = 0; i < 2; ++i)
            if (!c->ev_init[i]) HIPCHK(c, hipEventCreate(&c->ev_init[i]));
        HIPCHK(c, hipEventRecord(c->ev_init[0], c->stream));
    }
    for (int colour = 0; colour < 2; ++colour) {
        PassArgs a = pass_args(c, 0, colour);
        a.prop = pred;
        a.prop_w = pred_w;
        a.prop_s = cell;
        a.conf_min = c->p.conf_min;
        HIPCHK(c, launch_init(a, half, c->stream));
    }
    if (c->p.timing) {
        HIPCHK(c, hipEventRecord(c->ev_init[1], c->stream));
        c->init_timed = true;
    }
    c->have_state = true;
    return AMH_OK;
}

amh_status ensure_events(amh_ctx *c, int n) {
    while ((int)c->ev.size() < 2 * n) {
        hipEvent_t e;
        HIPCHK(c, hipEventCreate(&e));
        c->ev.push_back(e);
    }
    return AMH_OK;
}


// launch configurations: tile order {XCD bands, hardware} x job order {given, largest first} x tile rows {4, 2}
// x batch launch {one per phase, persistent}; configuration = tile_order + 2 job_order + 4 (tile rows == 2)
// + 8 persistent
constexpr int kTuneConfigs = 16;

void apply_config(amh_ctx *c, int cfg) {
    c->cfg_order = cfg & 1;
    c->cfg_job_order = (cfg >> 1) & 1;
    c->cfg_waves = (cfg & 4) ? 2 : kDefaultTileRows;
    c->cfg_persist = (cfg >> 3) & 1;
}

amh_status check_jobs(amh_ctx *c, int n_jobs, const amh_job *jobs) {
    if (!jobs || n_jobs < 1 || n_jobs > 4096) return fail(c, AMH_E_INVALID_ARG, "need 1 <= n_jobs <= 4096 jobs");
    if (c->views.empty()) return fail(c, AMH_E_STATE, "no views registered (amh_init_views)");
    const int nv = (int)c->views.size();
    for (int j = 0; j < n_jobs; ++j) {
        const amh_job &jb = jobs[j];
        if (jb.ref < 0 || jb.ref >= nv) return fail(c, AMH_E_INVALID_ARG, "job %d: ref %d out of range", j, jb.ref);
        if (!jb.srcs || jb.n_src < 1 || jb.n_src > kMaxSrc)
            return fail(c, AMH_E_INVALID_ARG, "job %d: need 1 <= n_src <= 32 sources", j);
        if (jb.iters < 0 || jb.iters > 1000) return fail(c, AMH_E_INVALID_ARG, "job %d: iters outside 0..1000", j);
        for (int i = 0; i < jb.n_src; ++i) {
            const int v = jb.srcs[i];
            if (v < 0 || v >= nv || v == jb.ref) return fail(c, AMH_E_INVALID_ARG, "job %d: bad source %d", j, v);
            for (int k = 0; k < i; ++k)
                if (jb.srcs[k] == v) return fail(c, AMH_E_INVALID_ARG, "job %d: source %d listed twice", j, v);
        }
    }
    return AMH_OK;
}

void free_batch(amh_ctx *c) {
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
    c->batch_key.clear();
    if (c->d_jobs) (void)hipFree(c->d_jobs);
    if (c->d_bviews) (void)hipFree(c->d_bviews);
    if (c->d_tables) (void)hipFree(c->d_tables);
    if (c->d_bcount) (void)hipFree(c->d_bcount);
    if (c->d_persist) (void)hipFree(c->d_persist);
    c->d_jobs = nullptr;
    c->d_bviews = nullptr;
    c->d_tables = nullptr;
    c->d_bcount = nullptr;
    c->d_persist = nullptr;
    c->d_pfault = nullptr;
}

// A persistent batch whose grid barrier ran out of time (its workgroups were not all resident) leaves a
// flag; the calls that read a batch's results report it.
amh_status check_persist_fault(amh_ctx *c) {
    if (!c->d_pfault) return AMH_OK;
    unsigned f = 0;
    HIPCHK(c, hipMemcpyAsync(&f, c->d_pfault, sizeof f, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (f) return fail(c, AMH_E_HIP, "persistent batch: a grid barrier timed out (workgroups not all resident)");
    return AMH_OK;
}

// Builds the device tables of a batch and captures its phases into a graph:
// zero counters, stamp the start clock, init (2 colours), then per iteration
// the red and the black half-pass over the jobs that still iterate.
amh_status build_batch(amh_ctx *c, int n_jobs, const amh_job *jobs, bool proposal) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    free_batch(c);
    c->batch_ran = false;
    // per-job state (kept across batches when the size matches)
    for (size_t j = (size_t)n_jobs; j < c->jobs.size(); ++j) free_job(c->jobs[j]);
    c->jobs.resize(n_jobs);
    int total_src = 0, max_src = 0, max_iters = 0;
    for (int j = 0; j < n_jobs; ++j) {
        const View &r = c->views[jobs[j].ref];
        JobResult &jr = c->jobs[j];
        if (jr.W != r.W || jr.H != r.H || !jr.planes) {
            free_job(jr);
            const size_t P = (size_t)r.W * r.H;
            amh_status st;
            if ((st = dalloc(c, (void **)&jr.planes, P * sizeof(float4))) != AMH_OK) return st;
            if ((st = dalloc(c, (void **)&jr.cost, P * sizeof(float))) != AMH_OK) return st;
            if ((st = dalloc(c, (void **)&jr.S, P * sizeof(uint32_t))) != AMH_OK) return st;
            if ((st = dalloc(c, (void **)&jr.v, P * sizeof(int32_t))) != AMH_OK) return st;
            jr.W = r.W;
            jr.H = r.H;
        }
        if (proposal) {
            const size_t cells = (size_t)cell_rows(r.H) * cell_rows(r.W);
            if (cells > jr.cells) {
                for (void *p : {jr.feats, (void *)jr.qref, (void *)jr.pred})
                    if (p) (void)hipFree(p);
                jr.feats = nullptr;
                jr.qref = jr.pred = nullptr;
                jr.cells = 0;
                amh_status st;
                if ((st = dalloc(c, &jr.feats, cells * 16 * sizeof(uint16_t))) != AMH_OK) return st;
                if ((st = dalloc(c, (void **)&jr.qref, cells * sizeof(float))) != AMH_OK) return st;
                if ((st = dalloc(c, (void **)&jr.pred, cells * 5 * sizeof(float))) != AMH_OK) return st;
                jr.cells = cells;
            }
        }
        jr.ref.img = r.img;
        jr.ref.W = r.W;
        jr.ref.H = r.H;
        kinv_upper(r.K, jr.ref.kinv_a, jr.ref.kinv_b, jr.ref.kinv_c, jr.ref.kinv_e, jr.ref.kinv_f);
        total_src += jobs[j].n_src;
        max_src = std::max(max_src, jobs[j].n_src);
        max_iters = std::max(max_iters, jobs[j].iters);
    }
    amh_status st;
    if ((st = dalloc(c, (void **)&c->d_bviews, sizeof(ViewDev) * total_src)) != AMH_OK) return st;
    if ((st = dalloc(c, (void **)&c->d_jobs, sizeof(BatchJobDev) * n_jobs)) != AMH_OK) return st;
    const size_t ncount = kCounterKinds * (size_t)kCounterSlots + (size_t)n_jobs + (size_t)n_jobs + 1;
    if ((st = dalloc(c, (void **)&c->d_bcount, sizeof(unsigned long long) * ncount)) != AMH_OK) return st;
    std::vector<ViewDev> hv(total_src);
    std::vector<BatchJobDev> hj(n_jobs);
    int so = 0;
    for (int j = 0; j < n_jobs; ++j) {
        const View &r = c->views[jobs[j].ref];
        for (int i = 0; i < jobs[j].n_src; ++i) hv[so + i] = view_dev(r, c->views[jobs[j].srcs[i]]);
        BatchJobDev &b = hj[j];
        b.ref = c->jobs[j].ref;
        b.views = c->d_bviews + so;
        b.view_off = so;
        b.n_src = jobs[j].n_src;
        b.st = StateDev{c->jobs[j].planes, c->jobs[j].cost, c->jobs[j].S, c->jobs[j].v};
        b.tiles_x = ((r.W + 1) / 2 + kTilePix - 1) / kTilePix;
        b.n_tiles = b.tiles_x * ((r.H + c->cfg_waves - 1) / c->cfg_waves);
        b.n_iblocks = (int)init_blocks(r.W, r.H);
        b.prop = proposal ? c->jobs[j].pred : nullptr;
        b.prop_w = proposal ? cell_rows(r.W) : 0;
        so += jobs[j].n_src;
    }
    // job order within a phase: as given, or the largest first (shorter tail)
    std::vector<int> order(n_jobs);
    for (int j = 0; j < n_jobs; ++j) order[j] = j;
    if (c->cfg_job_order == 1)
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return hj[a].n_tiles > hj[b].n_tiles; });
    // phases and their tables
    struct Phase {
        int kind, colour, t, n_active, total, off, grid, max_src;
    };
    std::vector<Phase> phases;
    std::vector<int> tab;
    // A half-pass is launched once per LDS class: workgroups whose sources need less LDS fit more of them on
    // a CU (160 KB), so the jobs of a phase are grouped by how many workgroups per CU their view count
    // allows (capped at 4 waves per SIMD); one launch per group, largest occupancy first.
    const int wg_cap = 16 / c->cfg_waves;
    auto wg_per_cu = [&](int n) { return std::min(wg_cap, (int)((size_t)160 * 1024 / pass_lds_bytes(n, c->cfg_waves))); };
    auto add_group = [&](int kind, int colour, int t, const std::vector<int> &act) {
        Phase ph{kind, colour, t, 0, 0, (int)tab.size(), 0, 0};
        ph.n_active = (int)act.size();
        if (ph.n_active == 0) return;
        for (int j : act) ph.max_src = std::max(ph.max_src, jobs[j].n_src);
        // work items per job: initialisation blocks or pass tiles
        auto items = [&](int j) { return kind == 0 ? hj[j].n_iblocks : hj[j].n_tiles; };
        int acc = 0;
        for (int j : act) {
            tab.push_back(acc);
            acc += items(j);
        }
        tab.push_back(acc);
        ph.total = acc;
        for (int j : act) tab.push_back(j);
        for (int j : act) {
            const bool last = colour == 1 && ((kind == 0 && jobs[j].iters == 0) || (kind == 1 && t == jobs[j].iters - 1));
            tab.push_back(last ? 1 : 0);
        }
        // tile order 0: each job's tiles in 8 contiguous bands [n b / 8, n (b + 1) / 8); XCD x takes band
        // (x + slot) mod 8 of the job at active slot `slot`; per XCD the prefix sums of its band sizes
        int longest = 1;
        for (int x = 0; x < 8; ++x) {
            int acc_x = 0;
            tab.push_back(0);
            for (int k = 0; k < (int)act.size(); ++k) {
                const long long n = items(act[k]);
                const int bi = (x + k) & 7;
                acc_x += (int)((n * (bi + 1)) >> 3) - (int)((n * bi) >> 3);
                tab.push_back(acc_x);
            }
            longest = std::max(longest, acc_x);
        }
        ph.grid = c->cfg_order == 0 ? 8 * longest : acc;
        phases.push_back(ph);
    };
    auto add_phase = [&](int kind, int colour, int t) {
        std::vector<int> act;
        for (int j : order)
            if (kind == 0 || jobs[j].iters > t) act.push_back(j);
        if (kind == 0) {  // the initialisation's LDS (costs of 256 pixels) is small for every view count
            add_group(kind, colour, t, act);
            return;
        }
        for (int w = wg_cap; w >= 1; --w) {
            std::vector<int> grp;
            for (int j : act)
                if (std::max(1, wg_per_cu(jobs[j].n_src)) == w) grp.push_back(j);
            add_group(kind, colour, t, grp);
        }
    };
    add_phase(0, 0, 0);
    add_phase(0, 1, 0);
    // persistent launch: the half-passes of all jobs as phases of one kernel, all jobs in one LDS class
    // (the largest view count), tiles in per-XCD bands
    std::vector<Phase> pphases;
    for (int t = 0; t < max_iters; ++t)
        for (int colour = 0; colour < 2; ++colour) {
            if (!c->cfg_persist) {
                add_phase(1, colour, t);
                continue;
            }
            std::vector<int> act;
            for (int j : order)
                if (jobs[j].iters > t) act.push_back(j);
            const size_t before = phases.size();
            add_group(1, colour, t, act);
            if (phases.size() > before) {
                pphases.push_back(phases.back());
                phases.pop_back();
            }
        }
    if ((st = dalloc(c, (void **)&c->d_tables, sizeof(int) * tab.size())) != AMH_OK) return st;
    HIPCHK(c, hipMemcpyAsync(c->d_bviews, hv.data(), sizeof(ViewDev) * total_src, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_jobs, hj.data(), sizeof(BatchJobDev) * n_jobs, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_tables, tab.data(), sizeof(int) * tab.size(), hipMemcpyHostToDevice, c->stream));
    if (proposal) {
        size_t most = 0;
        for (int j = 0; j < n_jobs; ++j) most = std::max(most, c->jobs[j].cells);
        if ((st = nn_reserve(c, most)) != AMH_OK) return st;  // before capture: may allocate
    }
    unsigned long long *tiles_done = c->d_bcount + kCounterKinds * kCounterSlots;
    unsigned long long *clocks = tiles_done + n_jobs;  // [n_jobs] completion, [n_jobs] start
    // persistent launch: its arguments and phase table in device memory, then the counters it clears
    // (next tile of each XCD's queue per phase, barrier arrivals, fault flag) as 64-bit words
    const int n_pp = (int)pphases.size();
    int p_grid = 0;
    PersistArgs *d_pargs = nullptr;
    unsigned long long *d_psync = nullptr;
    size_t n_psync = 0;
    if (n_pp > 0) {
        int cus = 0, khz = 0;
        HIPCHK(c, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
        HIPCHK(c, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device));
        const int per_cu = persist_blocks_per_cu(c->half, c->cfg_waves, max_src);
        if (per_cu < 1 || cus < 1 || khz <= 0)
            return fail(c, AMH_E_UNSUPPORTED, "persistent batch: no resident workgroup fits (%d per CU)", per_cu);
        int most_tiles = 0;
        for (const Phase &ph : pphases) most_tiles = std::max(most_tiles, ph.total);
        // every workgroup must be resident at once (grid barrier): at most one per free slot, a multiple of 8
        p_grid = std::max(8, (std::min(per_cu * cus, most_tiles + 7) / 8) * 8);
        const size_t o_args = 0, o_ph = 256, o_sync = o_ph + ((sizeof(PersistPhase) * n_pp + 255) & ~(size_t)255);
        n_psync = ((size_t)n_pp * 8 + 2 + 1) / 2;
        if ((st = dalloc(c, &c->d_persist, o_sync + n_psync * 8)) != AMH_OK) return st;
        unsigned char *base = static_cast<unsigned char *>(c->d_persist);
        d_pargs = reinterpret_cast<PersistArgs *>(base + o_args);
        PersistPhase *d_ph = reinterpret_cast<PersistPhase *>(base + o_ph);
        d_psync = reinterpret_cast<unsigned long long *>(base + o_sync);
        unsigned *sync32 = reinterpret_cast<unsigned *>(d_psync);
        std::vector<PersistPhase> hp(n_pp);
        for (int i = 0; i < n_pp; ++i) {
            const Phase &ph = pphases[i];
            PersistPhase &q = hp[i];
            q.tile_start = c->d_tables + ph.off;
            q.job_of = c->d_tables + ph.off + ph.n_active + 1;
            q.is_last = c->d_tables + ph.off + 2 * ph.n_active + 1;
            q.xcd_pre = c->d_tables + ph.off + 3 * ph.n_active + 1;
            q.n_active = ph.n_active;
            q.total_tiles = ph.total;
            q.t = ph.t;
            q.colour = ph.colour;
            q.m = method_dev(c->p, ph.t);
        }
        PersistArgs pa;
        pa.jobs = c->d_jobs;
        pa.views = c->d_bviews;
        pa.phases = d_ph;
        pa.n_phases = n_pp;
        pa.conf_min = c->p.conf_min;
        pa.counters = c->d_bcount;
        pa.tiles_done = tiles_done;
        pa.job_end = clocks;
        pa.next = sync32;
        pa.arrived = sync32 + (size_t)n_pp * 8;
        pa.fault = sync32 + (size_t)n_pp * 8 + 1;
        pa.spin_limit = (unsigned long long)khz * 1000ull * 4ull;  // 4 s of device clock per wait
        if (const char *sl = getenv("AMH_PERSIST_SPIN_TICKS"))     // test hook: a wait this short fails
            pa.spin_limit = strtoull(sl, nullptr, 10);
        pa.probe = 0;
        pa.probe_ticks = (unsigned long long)khz * 20ull;  // 20 ms
        c->d_pfault = pa.fault;
        HIPCHK(c, hipMemcpyAsync(d_ph, hp.data(), sizeof(PersistPhase) * n_pp, hipMemcpyHostToDevice, c->stream));
        // the grid barrier needs every workgroup resident at once: the occupancy figure is checked once per
        // shape by a probe launch of the same kernel (residency can also be limited by scratch or reserved CUs)
        int resident = -1;
        for (const auto &r : c->persist_resident)
            if (r[0] == c->half && r[1] == c->cfg_waves && r[2] == max_src && r[3] == p_grid) resident = r[4];
        if (resident < 0) {
            PersistArgs probe = pa;
            probe.probe = 1;
            HIPCHK(c, launch_zero_u64(d_psync, (int)n_psync, c->stream));
            HIPCHK(c, hipMemcpyAsync(d_pargs, &probe, sizeof probe, hipMemcpyHostToDevice, c->stream));
            HIPCHK(c, launch_persist(d_pargs, c->half, c->cfg_waves, max_src, p_grid, c->stream));
            unsigned peak = 0;
            HIPCHK(c, hipMemcpyAsync(&peak, reinterpret_cast<unsigned *>(d_psync) + 2, sizeof peak,
                                     hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            resident = (int)peak;
            c->persist_resident.push_back({c->half, c->cfg_waves, max_src, p_grid, resident});
        }
        if (resident < p_grid) p_grid = (resident / 8) * 8;
        if (p_grid < 8)
            return fail(c, AMH_E_UNSUPPORTED, "persistent batch: only %d workgroups resident at once", resident);
        HIPCHK(c, hipMemcpyAsync(d_pargs, &pa, sizeof pa, hipMemcpyHostToDevice, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // capture (kernels only: counters are cleared by a kernel, not a memset)
    if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = launch_zero_u64(c->d_bcount, kCounterKinds * kCounterSlots + n_jobs, c->cap_stream);
    if (e == hipSuccess && n_psync) e = launch_zero_u64(d_psync, (int)n_psync, c->cap_stream);
    if (e == hipSuccess) e = launch_stamp(clocks + n_jobs, c->cap_stream);
    // learned proposal: sweep and network forward of every job before its initialisation
    for (int j = 0; proposal && j < n_jobs && e == hipSuccess; ++j) {
        const JobResult &jr = c->jobs[j];
        SweepArgs sa = sweep_args(c, jr.ref, hj[j].views, jobs[j].n_src, jr.feats, jr.qref, c->d_bcount);
        e = launch_sweep(sa, c->half, c->cap_stream);
        if (e == hipSuccess &&
            nn_forward_stream(c, jr.feats, jr.qref, 1, sa.h4, sa.w4, jr.pred, c->cap_stream) != AMH_OK)
            e = hipErrorLaunchFailure;
    }
    for (const Phase &ph : phases) {
        if (e != hipSuccess) break;
        BatchPhaseArgs b;
        b.jobs = c->d_jobs;
        b.views = c->d_bviews;
        b.tile_start = c->d_tables + ph.off;
        b.job_of = c->d_tables + ph.off + ph.n_active + 1;
        b.is_last = c->d_tables + ph.off + 2 * ph.n_active + 1;
        b.xcd_pre = c->d_tables + ph.off + 3 * ph.n_active + 1;
        b.n_active = ph.n_active;
        b.total_tiles = ph.total;
        b.grid = ph.grid;
        b.m = method_dev(c->p, ph.t);
        b.t = ph.t;
        b.colour = ph.colour;
        b.kind = ph.kind;
        b.order = c->cfg_order;
        b.waves = c->cfg_waves;
        b.conf_min = c->p.conf_min;
        b.counters = c->d_bcount;
        b.tiles_done = tiles_done;
        b.job_end = clocks;
        e = launch_batch(b, c->half, ph.max_src, c->cap_stream);
    }
    if (e == hipSuccess && n_pp > 0) e = launch_persist(d_pargs, c->half, c->cfg_waves, max_src, p_grid, c->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(c, AMH_E_HIP, "batch capture: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    }
    c->graph = g;
    HIPCHK(c, hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
    return AMH_OK;
}

}  // namespace

extern "C" {

const char *amh_status_str(amh_status s) {
    switch (s) {
        case AMH_OK: return "ok";
        case AMH_E_INVALID_ARG: return "invalid argument";
        case AMH_E_OOM: return "out of device memory";
        case AMH_E_HIP: return "HIP runtime error";
        case AMH_E_STATE: return "call out of order";
        case AMH_E_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *amh_last_error(const amh_ctx *ctx) { return ctx ? ctx->err.c_str() : "NULL context"; }

amh_status amh_params_default(amh_params *out) {
    if (!out) return AMH_E_INVALID_ARG;
    memset(out, 0, sizeof *out);
    out->refine = 1;
    out->include_self = 1;
    out->depth_min = 2.f;
    out->depth_max = 6.f;
    out->sigma_color = 3.f;
    out->sigma_spatial = 30.f;
    out->tau_mc_init = 0.8f;
    out->alpha = 90.f;
    out->beta = 0.3f;
    out->tau_up = 1.2f;
    out->n1 = 2;
    out->n2 = 3;
    out->k = 4;
    out->seed = 0;
    out->timing = 0;
    out->conf_min = 0.0f;  // measured best after one iteration (see amhmvs.h)
    out->sym_prop = 0;
    out->heuristic_views = 0;
    out->bilateral_squared = 0;
    out->sweep_sources = 0;
    return AMH_OK;
}

amh_status amh_create(amh_ctx **out, const amh_params *p, void *hip_stream) {
    if (!out) return AMH_E_INVALID_ARG;
    *out = nullptr;
    amh_status st = check_params(nullptr, p);
    if (st != AMH_OK) return st;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return AMH_E_HIP;
    amh_ctx *c = new (std::nothrow) amh_ctx();
    if (!c) return AMH_E_OOM;
    c->p = *p;
    c->stream = (hipStream_t)hip_stream;
    const char *inj = getenv("AMH_FAIL_ALLOC_AT");  // test hook: fail this context's n-th device allocation
    c->fail_alloc_at = inj ? atoi(inj) : 0;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return AMH_E_HIP;
    }
    st = dalloc(c, (void **)&c->counters, sizeof(unsigned long long) * kCounterKinds * kCounterSlots);
    if (st != AMH_OK) {
        delete c;
        return st;
    }
    // device address of this GPU's copy of the allocation-free run's array (once per device); a failed
    // lookup is kept and reported by amh_run_checkerboard_static, the rest of the library does not need it
    unsigned char *sp = nullptr;
    (void)static_scratch(c->device, &sp);
    *out = c;
    return AMH_OK;
}

amh_status amh_set_params(amh_ctx *c, const amh_params *p) {
    if (!c) return AMH_E_INVALID_ARG;
    amh_status st = check_params(c, p);
    if (st != AMH_OK) return st;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    free_batch(c);  // the captured batch holds the old parameters
    c->p = *p;
    return AMH_OK;
}

amh_status amh_init_views(amh_ctx *c, int n_views, const amh_image *views, const amh_camera *cams,
                          amh_dtype store_as) {
    if (!c) return AMH_E_INVALID_ARG;
    if (n_views < 1 || n_views > 4096 || !views || !cams)
        return fail(c, AMH_E_INVALID_ARG, "need 1 <= n_views <= 4096 and non-NULL views and cams");
    if (store_as != AMH_F32 && store_as != AMH_F16) return fail(c, AMH_E_INVALID_ARG, "store_as must be F32 or F16");
    for (int i = 0; i < n_views; ++i) {
        const amh_image &im = views[i];
        if (!im.data) return fail(c, AMH_E_INVALID_ARG, "view %d: data is NULL", i);
        if (im.width < 1 || im.height < 1 || im.width > kMaxImageSide || im.height > kMaxImageSide)
            return fail(c, AMH_E_INVALID_ARG, "view %d: size %dx%d outside 1..%d", i, im.width, im.height,
                        kMaxImageSide);
        if (im.pitch_elems < im.width) return fail(c, AMH_E_INVALID_ARG, "view %d: pitch < width", i);
        if (im.dtype != AMH_F32 && im.dtype != AMH_F16) return fail(c, AMH_E_INVALID_ARG, "view %d: bad dtype", i);
        if (im.on_device != 0 && im.on_device != 1) return fail(c, AMH_E_INVALID_ARG, "view %d: on_device is 0/1", i);
        if (cams[i].width != im.width || cams[i].height != im.height)
            return fail(c, AMH_E_INVALID_ARG, "view %d: camera size differs from image size", i);
        amh_status st = check_camera(c, cams[i], i);
        if (st != AMH_OK) return st;
    }
    // replace the registered views; buffers of a view with the same size and storage type are reused
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::vector<View> old = std::move(c->views);
    c->views.clear();
    c->have_state = false;
    c->ref = -1;
    c->half = store_as == AMH_F16;
    free_batch(c);  // a captured batch refers to the old view buffers
    c->batch_ran = false;
    c->batch_stats = false;
    void *staging = nullptr;
    size_t staging_cap = 0;
    amh_status result = AMH_OK;
    for (int i = 0; i < n_views && result == AMH_OK; ++i) {
        const amh_image &im = views[i];
        View v;
        v.W = im.width;
        v.H = im.height;
        v.half = c->half;
        memcpy(v.K, cams[i].K, sizeof v.K);
        memcpy(v.R, cams[i].R, sizeof v.R);
        memcpy(v.t, cams[i].t, sizeof v.t);
        const size_t px = (size_t)v.W * v.H;
        const size_t qbytes = (size_t)(v.W + 2 + 2 * kQuadPad) * (v.H + 1 + 2 * kQuadPad) * (c->half ? 4 : 8);
        if (i < (int)old.size() && old[i].W == v.W && old[i].H == v.H && old[i].half == v.half && old[i].img) {
            v.img = old[i].img;
            v.quads = old[i].quads;
            old[i].img = nullptr;
            old[i].quads = nullptr;
        } else {
            if ((result = dalloc(c, (void **)&v.img, px * sizeof(float))) != AMH_OK) break;
            if ((result = dalloc(c, &v.quads, qbytes)) != AMH_OK) {
                free_view(v);
                break;
            }
        }
        const size_t esz = im.dtype == AMH_F16 ? 2 : 4;
        const void *src = im.data;
        int64_t pitch = im.pitch_elems;
        if (!im.on_device) {
            const size_t need = px * esz;
            if (need > staging_cap) {
                if (staging) (void)hipFree(staging);
                staging = nullptr;
                staging_cap = 0;
                if ((result = dalloc(c, &staging, need)) != AMH_OK) {
                    free_view(v);
                    break;
                }
                staging_cap = need;
            }
            hipError_t e = hipMemcpy2DAsync(staging, v.W * esz, im.data, (size_t)im.pitch_elems * esz, v.W * esz, v.H,
                                            hipMemcpyHostToDevice, c->stream);
            if (e != hipSuccess) {
                free_view(v);
                result = fail(c, AMH_E_HIP, "upload of view %d: %s", i, hipGetErrorString(e));
                break;
            }
            src = staging;
            pitch = v.W;
        }
        hipError_t e = launch_convert_to_f32(src, im.dtype == AMH_F16 ? 1 : 0, pitch, v.W, v.H, v.img, c->stream);
        if (e == hipSuccess) e = launch_pack_quads(v.img, v.W, v.H, v.quads, c->half, c->stream);
        if (e != hipSuccess) {
            free_view(v);
            result = fail(c, AMH_E_HIP, "layout kernels of view %d: %s", i, hipGetErrorString(e));
            break;
        }
        if (!im.on_device) {
            // the staging buffer is reused by the next host view: wait for this one
            e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) {
                free_view(v);
                result = fail(c, AMH_E_HIP, "view %d: %s", i, hipGetErrorString(e));
                break;
            }
        }
        c->views.push_back(v);
    }
    if (staging) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(staging);
    }
    for (auto &v : old) free_view(v);
    if (result != AMH_OK) {
        for (auto &v : c->views) free_view(v);
        c->views.clear();
    }
    return result;
}

// reference and source list of a depth map: registered views, no repeats, the reference not a source
static amh_status check_sources(amh_ctx *c, int ref, const int *srcs, int n_src) {
    if (c->views.empty()) return fail(c, AMH_E_STATE, "no views registered (amh_init_views)");
    const int nv = (int)c->views.size();
    if (ref < 0 || ref >= nv) return fail(c, AMH_E_INVALID_ARG, "ref %d outside 0..%d", ref, nv - 1);
    if (!srcs || n_src < 1 || n_src > kMaxSrc) return fail(c, AMH_E_INVALID_ARG, "need 1 <= n_src <= 32 sources");
    for (int i = 0; i < n_src; ++i) {
        if (srcs[i] < 0 || srcs[i] >= nv) return fail(c, AMH_E_INVALID_ARG, "source %d: view %d out of range", i, srcs[i]);
        if (srcs[i] == ref) return fail(c, AMH_E_INVALID_ARG, "source %d is the reference", i);
        for (int k = 0; k < i; ++k)
            if (srcs[k] == srcs[i]) return fail(c, AMH_E_INVALID_ARG, "source view %d listed twice", srcs[i]);
    }
    return AMH_OK;
}

amh_status amh_begin(amh_ctx *c, int ref, const int *srcs, int n_src) {
    if (!c) return AMH_E_INVALID_ARG;
    amh_status chk = check_sources(c, ref, srcs, n_src);
    if (chk != AMH_OK) return chk;
    HIPCHK(c, hipStreamSynchronize(c->stream));  // the previous constants may still be in flight
    const View &r = c->views[ref];
    c->ref = ref;
    c->srcs.assign(srcs, srcs + n_src);
    c->h_viewc.resize(n_src);
    for (int i = 0; i < n_src; ++i) c->h_viewc[i] = view_dev(r, c->views[srcs[i]]);
    if ((size_t)n_src > c->viewc_cap) {
        if (c->d_viewc) (void)hipFree(c->d_viewc);
        c->d_viewc = nullptr;
        c->viewc_cap = 0;
        amh_status st = dalloc(c, (void **)&c->d_viewc, sizeof(ViewDev) * kMaxSrc);
        if (st != AMH_OK) return st;
        c->viewc_cap = kMaxSrc;
    }
    HIPCHK(c, hipMemcpyAsync(c->d_viewc, c->h_viewc.data(), sizeof(ViewDev) * n_src, hipMemcpyHostToDevice, c->stream));
    c->refdev.img = r.img;
    c->refdev.W = r.W;
    c->refdev.H = r.H;
    kinv_upper(r.K, c->refdev.kinv_a, c->refdev.kinv_b, c->refdev.kinv_c, c->refdev.kinv_e, c->refdev.kinv_f);
    const size_t P = (size_t)r.W * r.H;
    if (P > c->state_cap) {
        if (c->planes) (void)hipFree(c->planes);
        if (c->cost) (void)hipFree(c->cost);
        if (c->S) (void)hipFree(c->S);
        if (c->v) (void)hipFree(c->v);
        c->planes = nullptr;
        c->cost = nullptr;
        c->S = nullptr;
        c->v = nullptr;
        c->state_cap = 0;
        amh_status st;
        if ((st = dalloc(c, (void **)&c->planes, P * sizeof(float4))) != AMH_OK) return st;
        if ((st = dalloc(c, (void **)&c->cost, P * sizeof(float))) != AMH_OK) return st;
        if ((st = dalloc(c, (void **)&c->S, P * sizeof(uint32_t))) != AMH_OK) return st;
        if ((st = dalloc(c, (void **)&c->v, P * sizeof(int32_t))) != AMH_OK) return st;
        c->state_cap = P;
    }
    c->have_state = false;
    c->n_timed = 0;
    c->init_timed = false;
    c->batch_stats = false;
    HIPCHK(c, launch_zero_u64(c->counters, kCounterKinds * kCounterSlots, c->stream));
    return AMH_OK;
}

amh_status amh_init_hypotheses(amh_ctx *c) {
    if (!c) return AMH_E_INVALID_ARG;
    if (c->ref < 0) return fail(c, AMH_E_STATE, "no reference selected (amh_begin)");
    return init_state(c, nullptr, 0, 0);
}

amh_status amh_pass(amh_ctx *c, int t, int colour) {
    if (!c) return AMH_E_INVALID_ARG;
    if (t < 0 || t > 1000000 || (colour != 0 && colour != 1))
        return fail(c, AMH_E_INVALID_ARG, "need t >= 0 and colour 0 or 1");
    if (c->ref < 0 || !c->have_state) return fail(c, AMH_E_STATE, "no initialised state (amh_init_hypotheses)");
    PassArgs a = pass_args(c, t, colour);
    const bool timed = c->p.timing && c->n_timed < 64;
    if (timed) {
        amh_status st = ensure_events(c, c->n_timed + 1);
        if (st != AMH_OK) return st;
        HIPCHK(c, hipEventRecord(c->ev[2 * c->n_timed], c->stream));
    }
    HIPCHK(c, launch_pass(a, c->half, c->stream));
    if (timed) {
        HIPCHK(c, hipEventRecord(c->ev[2 * c->n_timed + 1], c->stream));
        ++c->n_timed;
    }
    return AMH_OK;
}

amh_status amh_run_checkerboard(amh_ctx *c, int ref, const int *srcs, int n_src, int iters) {
    if (!c) return AMH_E_INVALID_ARG;
    if (iters < 0 || iters > 1000) return fail(c, AMH_E_INVALID_ARG, "iters must be in 0..1000");
    amh_status st = amh_begin(c, ref, srcs, n_src);
    if (st != AMH_OK) return st;
    if ((st = amh_init_hypotheses(c)) != AMH_OK) return st;
    for (int t = 0; t < iters; ++t)
        for (int colour = 0; colour < 2; ++colour)
            if ((st = amh_pass(c, t, colour)) != AMH_OK) return st;
    return AMH_OK;
}

amh_status amh_run_checkerboard_static(amh_ctx *c, int ref, const int *srcs, int n_src, int iters, float *depth,
                                       float *normal, float *cost) {
    if (!c) return AMH_E_INVALID_ARG;
    if (iters < 0 || iters > 1000) return fail(c, AMH_E_INVALID_ARG, "iters must be in 0..1000");
    amh_status st = check_sources(c, ref, srcs, n_src);
    if (st != AMH_OK) return st;
    const View &r = c->views[ref];
    const size_t P = (size_t)r.W * r.H;
    if (P > kStaticMaxPixels)
        return fail(c, AMH_E_INVALID_ARG, "reference of %dx%d = %zu pixels: the allocation-free run holds at most %zu",
                    r.W, r.H, P, kStaticMaxPixels);
    unsigned char *base = nullptr;
    const hipError_t se = static_scratch(c->device, &base);
    if (se != hipSuccess || !base)
        return fail(c, AMH_E_HIP, "no device address for the allocation-free run's array: %s", hipGetErrorString(se));
    ViewDev *viewc = reinterpret_cast<ViewDev *>(base + kStaticViewcOff);
    const StateDev sd{reinterpret_cast<float4 *>(base + kStaticPlanesOff), reinterpret_cast<float *>(base + kStaticCostOff),
                      reinterpret_cast<uint32_t *>(base + kStaticSOff), reinterpret_cast<int32_t *>(base + kStaticVOff)};
    // the context's current reference is released: its own state is not this run's, and its warp-constant
    // table no longer matches the source list (the host copy below is reused for this run)
    HIPCHK(c, hipStreamSynchronize(c->stream));  // an earlier copy from the host table may still be in flight
    c->ref = -1;
    c->have_state = false;
    c->srcs.assign(srcs, srcs + n_src);
    c->h_viewc.resize(n_src);
    for (int i = 0; i < n_src; ++i) c->h_viewc[i] = view_dev(r, c->views[srcs[i]]);
    HIPCHK(c, hipMemcpyAsync(viewc, c->h_viewc.data(), sizeof(ViewDev) * n_src, hipMemcpyHostToDevice, c->stream));
    c->refdev.img = r.img;
    c->refdev.W = r.W;
    c->refdev.H = r.H;
    kinv_upper(r.K, c->refdev.kinv_a, c->refdev.kinv_b, c->refdev.kinv_c, c->refdev.kinv_e, c->refdev.kinv_f);
    // statistics count this run's evaluations (no per-pass times)
    c->n_timed = 0;
    c->init_timed = false;
    c->batch_stats = false;
    HIPCHK(c, launch_zero_u64(c->counters, kCounterKinds * kCounterSlots, c->stream));
    for (int colour = 0; colour < 2; ++colour) {  // random initialisation writes every pixel of the state
        PassArgs a = pass_args(c, 0, colour);
        a.views = viewc;
        a.st = sd;
        HIPCHK(c, launch_init(a, c->half, c->stream));
    }
    for (int t = 0; t < iters; ++t)
        for (int colour = 0; colour < 2; ++colour) {
            PassArgs a = pass_args(c, t, colour);
            a.views = viewc;
            a.st = sd;
            HIPCHK(c, launch_pass(a, c->half, c->stream));
        }
    if (depth || normal || cost) HIPCHK(c, launch_outputs(c->refdev, sd, depth, normal, cost, c->stream));
    return AMH_OK;
}

amh_status amh_get_depth_normal_cost(amh_ctx *c, float *depth, float *normal, float *cost, int dst_on_device) {
    if (!c) return AMH_E_INVALID_ARG;
    if (dst_on_device != 0 && dst_on_device != 1) return fail(c, AMH_E_INVALID_ARG, "dst_on_device is 0 or 1");
    if (c->ref < 0 || !c->have_state) return fail(c, AMH_E_STATE, "no result yet");
    const size_t P = (size_t)c->refdev.W * c->refdev.H;
    StateDev st{c->planes, c->cost, c->S, c->v};
    if (dst_on_device) {
        HIPCHK(c, launch_outputs(c->refdev, st, depth, normal, cost, c->stream));
        return AMH_OK;
    }
    float *tmp = nullptr;
    amh_status s = dalloc(c, (void **)&tmp, P * 5 * sizeof(float));
    if (s != AMH_OK) return s;
    hipError_t e = launch_outputs(c->refdev, st, depth ? tmp : nullptr, normal ? tmp + P : nullptr,
                                  cost ? tmp + 4 * P : nullptr, c->stream);
    if (e == hipSuccess && depth) e = hipMemcpyAsync(depth, tmp, P * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && normal) e = hipMemcpyAsync(normal, tmp + P, P * 12, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && cost) e = hipMemcpyAsync(cost, tmp + 4 * P, P * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(tmp);
    if (e != hipSuccess) return fail(c, AMH_E_HIP, "get_depth_normal_cost: %s", hipGetErrorString(e));
    return AMH_OK;
}

amh_status amh_get_state(amh_ctx *c, float *planes, float *cost, uint32_t *S, int32_t *v, int dst_on_device) {
    if (!c) return AMH_E_INVALID_ARG;
    if (dst_on_device != 0 && dst_on_device != 1) return fail(c, AMH_E_INVALID_ARG, "dst_on_device is 0 or 1");
    if (c->ref < 0 || !c->have_state) return fail(c, AMH_E_STATE, "no state yet");
    const size_t P = (size_t)c->refdev.W * c->refdev.H;
    const hipMemcpyKind k = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (planes) HIPCHK(c, hipMemcpyAsync(planes, c->planes, P * 16, k, c->stream));
    if (cost) HIPCHK(c, hipMemcpyAsync(cost, c->cost, P * 4, k, c->stream));
    if (S) HIPCHK(c, hipMemcpyAsync(S, c->S, P * 4, k, c->stream));
    if (v) HIPCHK(c, hipMemcpyAsync(v, c->v, P * 4, k, c->stream));
    if (!dst_on_device) HIPCHK(c, hipStreamSynchronize(c->stream));
    return AMH_OK;
}

amh_status amh_set_state(amh_ctx *c, const float *planes, const float *cost, const uint32_t *S, const int32_t *v,
                         int src_on_device) {
    if (!c) return AMH_E_INVALID_ARG;
    if (!planes || !cost || !S || !v) return fail(c, AMH_E_INVALID_ARG, "all four state arrays are required");
    if (src_on_device != 0 && src_on_device != 1) return fail(c, AMH_E_INVALID_ARG, "src_on_device is 0 or 1");
    if (c->ref < 0) return fail(c, AMH_E_STATE, "no reference selected (amh_begin)");
    const size_t P = (size_t)c->refdev.W * c->refdev.H;
    const hipMemcpyKind k = src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIPCHK(c, hipMemcpyAsync(c->planes, planes, P * 16, k, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->cost, cost, P * 4, k, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->S, S, P * 4, k, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->v, v, P * 4, k, c->stream));
    if (!src_on_device) HIPCHK(c, hipStreamSynchronize(c->stream));
    c->have_state = true;
    return AMH_OK;
}

amh_status amh_score_fixed(amh_ctx *c, const float *planes, const int *pix, int Q, float *costs, int on_device) {
    if (!c) return AMH_E_INVALID_ARG;
    if (Q < 0 || Q > (1 << 24)) return fail(c, AMH_E_INVALID_ARG, "need 0 <= Q <= 2^24");
    if (on_device != 0 && on_device != 1) return fail(c, AMH_E_INVALID_ARG, "on_device is 0 or 1");
    if (Q > 0 && (!planes || !pix || !costs)) return fail(c, AMH_E_INVALID_ARG, "NULL buffer");
    if (c->ref < 0) return fail(c, AMH_E_STATE, "no reference selected (amh_begin)");
    const int N = (int)c->srcs.size();
    if (!on_device)
        for (int i = 0; i < Q; ++i)
            if (pix[2 * i] < 0 || pix[2 * i] >= c->refdev.W || pix[2 * i + 1] < 0 || pix[2 * i + 1] >= c->refdev.H)
                return fail(c, AMH_E_INVALID_ARG, "query %d: pixel outside the reference image", i);
    if (Q == 0) return AMH_OK;
    ScoreArgs a;
    a.ref = c->refdev;
    a.views = c->d_viewc;
    a.n_src = N;
    a.m = method_dev(c->p, 0);
    a.Q = Q;
    if (on_device) {
        a.planes = reinterpret_cast<const float4 *>(planes);
        a.pix = reinterpret_cast<const int2 *>(pix);
        a.costs = costs;
        HIPCHK(c, launch_score(a, c->half, c->stream));
        return AMH_OK;
    }
    unsigned char *buf = nullptr;
    const size_t bp = (size_t)Q * 16, bq = (size_t)Q * 8, bc = (size_t)Q * N * 4;
    amh_status s = dalloc(c, (void **)&buf, bp + bq + bc);
    if (s != AMH_OK) return s;
    hipError_t e = hipMemcpyAsync(buf, planes, bp, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(buf + bp, pix, bq, hipMemcpyHostToDevice, c->stream);
    a.planes = reinterpret_cast<const float4 *>(buf);
    a.pix = reinterpret_cast<const int2 *>(buf + bp);
    a.costs = reinterpret_cast<float *>(buf + bp + bq);
    if (e == hipSuccess) e = launch_score(a, c->half, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(costs, a.costs, bc, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(buf);
    if (e != hipSuccess) return fail(c, AMH_E_HIP, "score_fixed: %s", hipGetErrorString(e));
    return AMH_OK;
}

static amh_status run_batch_impl(amh_ctx *c, int n_jobs, const amh_job *jobs, bool proposal) {
    amh_status st = check_jobs(c, n_jobs, jobs);
    if (st != AMH_OK) return st;
    if (proposal && !c->net) return fail(c, AMH_E_STATE, "no proposal network (amh_nn_init or amh_nn_load)");
    if (c->p.sym_prop || c->p.heuristic_views)
        return fail(c, AMH_E_UNSUPPORTED, "the ablation modes run on the single-image path only");
    std::vector<int> key = {n_jobs, c->cfg_order, c->cfg_job_order, c->cfg_waves, c->cfg_persist, proposal ? 1 : 0};
    for (int j = 0; j < n_jobs; ++j) {
        key.push_back(jobs[j].ref);
        key.push_back(jobs[j].n_src);
        key.push_back(jobs[j].iters);
        key.insert(key.end(), jobs[j].srcs, jobs[j].srcs + jobs[j].n_src);
    }
    if (!(c->graph_exec && key == c->batch_key)) {
        st = build_batch(c, n_jobs, jobs, proposal);
        if (st != AMH_OK) return st;
        c->batch_key = key;
    }
    HIPCHK(c, hipGraphLaunch(c->graph_exec, c->stream));
    c->batch_ran = true;
    c->batch_stats = true;
    c->batch_jobs = n_jobs;
    return AMH_OK;
}

amh_status amh_run_batch(amh_ctx *c, int n_jobs, const amh_job *jobs) {
    if (!c) return AMH_E_INVALID_ARG;
    return run_batch_impl(c, n_jobs, jobs, false);
}

amh_status amh_run_batch_proposal(amh_ctx *c, int n_jobs, const amh_job *jobs) {
    if (!c) return AMH_E_INVALID_ARG;
    return run_batch_impl(c, n_jobs, jobs, true);
}

amh_status amh_get_job_result(amh_ctx *c, int job, float *depth, float *normal, float *cost, int dst_on_device) {
    if (!c) return AMH_E_INVALID_ARG;
    if (dst_on_device != 0 && dst_on_device != 1) return fail(c, AMH_E_INVALID_ARG, "dst_on_device is 0 or 1");
    if (!c->batch_ran) return fail(c, AMH_E_STATE, "no batch has run");
    if (job < 0 || job >= c->batch_jobs) return fail(c, AMH_E_INVALID_ARG, "job %d outside 0..%d", job, c->batch_jobs - 1);
    const JobResult &r = c->jobs[job];
    const size_t P = (size_t)r.W * r.H;
    StateDev sd{r.planes, r.cost, r.S, r.v};
    if (dst_on_device) {
        HIPCHK(c, launch_outputs(r.ref, sd, depth, normal, cost, c->stream));
        return AMH_OK;
    }
    float *tmp = nullptr;
    amh_status s = dalloc(c, (void **)&tmp, P * 5 * sizeof(float));
    if (s != AMH_OK) return s;
    hipError_t e = launch_outputs(r.ref, sd, depth ? tmp : nullptr, normal ? tmp + P : nullptr, cost ? tmp + 4 * P : nullptr,
                                  c->stream);
    if (e == hipSuccess && depth) e = hipMemcpyAsync(depth, tmp, P * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && normal) e = hipMemcpyAsync(normal, tmp + P, P * 12, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && cost) e = hipMemcpyAsync(cost, tmp + 4 * P, P * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(tmp);
    if (e != hipSuccess) return fail(c, AMH_E_HIP, "get_job_result: %s", hipGetErrorString(e));
    return check_persist_fault(c);
}

amh_status amh_get_job_times(amh_ctx *c, int n, float *job_ms) {
    if (!c) return AMH_E_INVALID_ARG;
    if (!c->batch_ran) return fail(c, AMH_E_STATE, "no batch has run");
    if (!job_ms || n != c->batch_jobs) return fail(c, AMH_E_INVALID_ARG, "need n == the batch's job count");
    if (!c->d_bcount) return fail(c, AMH_E_STATE, "the batch's clocks were released (parameters changed)");
    amh_status fs = check_persist_fault(c);
    if (fs != AMH_OK) return fs;
    // clocks: [n] job completions then the batch start, after the evaluation counters and tiles-done
    std::vector<unsigned long long> h((size_t)n + 1);
    const size_t off = kCounterKinds * (size_t)kCounterSlots + (size_t)n;
    HIPCHK(c, hipMemcpyAsync(h.data(), c->d_bcount + off, h.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int khz = 0;
    HIPCHK(c, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device));
    if (khz <= 0) return fail(c, AMH_E_HIP, "device wall clock rate unavailable");
    const unsigned long long t0 = h[n];
    for (int j = 0; j < n; ++j) job_ms[j] = (float)((double)(h[j] - t0) / (double)khz);
    return AMH_OK;
}

amh_status amh_set_launch_config(amh_ctx *c, int config) {
    if (!c) return AMH_E_INVALID_ARG;
    if (config < 0 || config >= kTuneConfigs)
        return fail(c, AMH_E_INVALID_ARG, "launch configuration %d outside 0..%d", config, kTuneConfigs - 1);
    apply_config(c, config);
    return AMH_OK;
}

amh_status amh_tune(amh_ctx *c, int n_jobs, const amh_job *jobs, int *best_config, float *ms_per_config) {
    if (!c) return AMH_E_INVALID_ARG;
    amh_status st = check_jobs(c, n_jobs, jobs);
    if (st != AMH_OK) return st;
    // the bucket: job count, largest view count, pixel count (powers of two)
    int max_src = 0;
    double px = 0;
    for (int j = 0; j < n_jobs; ++j) {
        max_src = std::max(max_src, jobs[j].n_src);
        px += (double)c->views[jobs[j].ref].W * c->views[jobs[j].ref].H;
    }
    char bucket[128];
    snprintf(bucket, sizeof bucket, "gfx950/cfg16/jobs%d/src%d/px2^%d/half%d", n_jobs, max_src,
             (int)std::ceil(std::log2(px + 1)), c->half);
    const char *path = getenv("AMH_TUNE_CACHE");
    int cached = -1;
    if (path) {
        FILE *f = fopen(path, "r");
        if (f) {
            char k[256];
            int v;
            while (fscanf(f, "%255s %d", k, &v) == 2)
                if (strcmp(k, bucket) == 0) cached = v;
            fclose(f);
        }
    }
    float ms[kTuneConfigs];
    for (int i = 0; i < kTuneConfigs; ++i) ms[i] = -1.f;
    int best = cached;
    if (best < 0 || best >= kTuneConfigs) {
        hipEvent_t e0, e1;
        HIPCHK(c, hipEventCreate(&e0));
        HIPCHK(c, hipEventCreate(&e1));
        float best_ms = 0.f;
        for (int cfg = 0; cfg < kTuneConfigs; ++cfg) {
            apply_config(c, cfg);
            st = amh_run_batch(c, n_jobs, jobs);  // build + warm
            if (st == AMH_E_UNSUPPORTED && c->cfg_persist) continue;  // the persistent grid does not fit
            if (st != AMH_OK) return st;
            HIPCHK(c, hipEventRecord(e0, c->stream));
            if ((st = amh_run_batch(c, n_jobs, jobs)) != AMH_OK) return st;  // replay, timed
            HIPCHK(c, hipEventRecord(e1, c->stream));
            HIPCHK(c, hipEventSynchronize(e1));
            HIPCHK(c, hipEventElapsedTime(&ms[cfg], e0, e1));
            if (best < 0 || ms[cfg] < best_ms) {
                best = cfg;
                best_ms = ms[cfg];
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (path) {
            FILE *f = fopen(path, "a");
            if (f) {
                fprintf(f, "%s %d\n", bucket, best);
                fclose(f);
            }
        }
    }
    apply_config(c, best);
    if (best_config) *best_config = best;
    if (ms_per_config)
        for (int i = 0; i < kTuneConfigs; ++i) ms_per_config[i] = ms[i];
    return AMH_OK;
}

amh_status amh_sweep_features(amh_ctx *c, void *feats, float *q_ref) {
    if (!c) return AMH_E_INVALID_ARG;
    if (!feats) return fail(c, AMH_E_INVALID_ARG, "feats is NULL");
    if (c->ref < 0) return fail(c, AMH_E_STATE, "no reference selected (amh_begin)");
    const SweepArgs a = sweep_args(c, c->refdev, c->d_viewc, (int)c->srcs.size(), feats, q_ref, c->counters);
    HIPCHK(c, launch_sweep(a, c->half, c->stream));
    return AMH_OK;
}

amh_status amh_init_from_proposal(amh_ctx *c, const float *pred, int h, int w) {
    if (!c) return AMH_E_INVALID_ARG;
    if (!pred || h < 1 || w < 1) return fail(c, AMH_E_INVALID_ARG, "need pred and a positive cell grid");
    if (c->ref < 0) return fail(c, AMH_E_STATE, "no reference selected (amh_begin)");
    const int W = c->refdev.W, H = c->refdev.H;
    if ((int64_t)w * kCell < W || (int64_t)h * kCell < H)
        return fail(c, AMH_E_INVALID_ARG, "a %dx%d grid of 4x4 cells does not cover a %dx%d image", w, h, W, H);
    return init_state(c, pred, w, kCell);
}

amh_status amh_set_initial_hypotheses(amh_ctx *c, const float *depth, const float *normal, const float *conf,
                                      int on_device) {
    if (!c) return AMH_E_INVALID_ARG;
    if (on_device != 0 && on_device != 1) return fail(c, AMH_E_INVALID_ARG, "on_device is 0 or 1");
    if (!depth || !normal) return fail(c, AMH_E_INVALID_ARG, "depth and normal are required (conf may be NULL)");
    if (c->ref < 0) return fail(c, AMH_E_STATE, "no reference selected (amh_begin)");
    const size_t P = (size_t)c->refdev.W * c->refdev.H;
    // packed [H][W][5] (depth, normal, confidence), followed by a staging copy of host inputs
    const size_t need = P * (on_device ? 5 : 10);
    if (need > c->hyp_cap) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (c->hyp) (void)hipFree(c->hyp);
        c->hyp = nullptr;
        c->hyp_cap = 0;
        amh_status st = dalloc(c, (void **)&c->hyp, need * sizeof(float));
        if (st != AMH_OK) return st;
        c->hyp_cap = need;
    }
    float *packed = c->hyp;
    const float *d = depth, *n = normal, *w = conf;
    if (!on_device) {
        float *stage = c->hyp + 5 * P;
        HIPCHK(c, hipMemcpyAsync(stage, depth, P * 4, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(stage + P, normal, P * 12, hipMemcpyHostToDevice, c->stream));
        if (conf) HIPCHK(c, hipMemcpyAsync(stage + 4 * P, conf, P * 4, hipMemcpyHostToDevice, c->stream));
        d = stage;
        n = stage + P;
        w = conf ? stage + 4 * P : nullptr;
    }
    HIPCHK(c, launch_pack_hypotheses(d, n, w, (int64_t)P, packed, c->stream));
    amh_status st = init_state(c, packed, c->refdev.W, 1);
    // host inputs: the caller may reuse its buffers once this returns
    if (st == AMH_OK && !on_device) HIPCHK(c, hipStreamSynchronize(c->stream));
    return st;
}

amh_status amh_run_proposal(amh_ctx *c, int ref, const int *srcs, int n_src, int iters) {
    if (!c) return AMH_E_INVALID_ARG;
    if (iters < 0 || iters > 1000) return fail(c, AMH_E_INVALID_ARG, "iters must be in 0..1000");
    if (!c->net) return fail(c, AMH_E_STATE, "no proposal network (amh_nn_init or amh_nn_load)");
    amh_status st = amh_begin(c, ref, srcs, n_src);
    if (st != AMH_OK) return st;
    const int h4 = cell_rows(c->refdev.H), w4 = cell_rows(c->refdev.W);
    const size_t cells = (size_t)h4 * w4;
    if (cells > c->prop_cap) {
        if (c->prop_feats) (void)hipFree(c->prop_feats);
        if (c->prop_pred) (void)hipFree(c->prop_pred);
        if (c->prop_qref) (void)hipFree(c->prop_qref);
        c->prop_feats = nullptr;
        c->prop_pred = nullptr;
        c->prop_qref = nullptr;
        c->prop_cap = 0;
        if ((st = dalloc(c, &c->prop_feats, cells * 16 * 2)) != AMH_OK) return st;
        if ((st = dalloc(c, (void **)&c->prop_pred, cells * 5 * sizeof(float))) != AMH_OK) return st;
        if ((st = dalloc(c, (void **)&c->prop_qref, cells * sizeof(float))) != AMH_OK) return st;
        c->prop_cap = cells;
    }
    if ((st = amh_sweep_features(c, c->prop_feats, c->prop_qref)) != AMH_OK) return st;
    if ((st = amh_nn_forward(c, c->prop_feats, c->prop_qref, 1, h4, w4, c->prop_pred)) != AMH_OK) return st;
    if ((st = amh_init_from_proposal(c, c->prop_pred, h4, w4)) != AMH_OK) return st;
    for (int t = 0; t < iters; ++t)
        for (int colour = 0; colour < 2; ++colour)
            if ((st = amh_pass(c, t, colour)) != AMH_OK) return st;
    return AMH_OK;
}

amh_status amh_get_stats(const amh_ctx *cc, amh_stats *out) {
    amh_ctx *c = const_cast<amh_ctx *>(cc);
    if (!c || !out) return AMH_E_INVALID_ARG;
    memset(out, 0, sizeof *out);
    if (c->batch_stats && c->d_bcount) {
        std::vector<unsigned long long> h(kCounterKinds * kCounterSlots);
        HIPCHK(c, hipMemcpyAsync(h.data(), c->d_bcount, h.size() * 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        amh_status fs = check_persist_fault(c);
        if (fs != AMH_OK) return fs;
        for (int k = 0; k < kCounterKinds; ++k) {
            c->batch_counts[k] = 0;
            for (int i = 0; i < kCounterSlots; ++i) c->batch_counts[k] += h[k * kCounterSlots + i];
        }
        out->evals_init = c->batch_counts[0];
        out->evals_propagation = c->batch_counts[1];
        out->evals_refine = c->batch_counts[2];
        out->fallback_pixels = c->batch_counts[3];
        out->evals_short = c->batch_counts[4];
        out->evals_init_short = c->batch_counts[5];
    } else if (!c->batch_stats && c->counters) {
        std::vector<unsigned long long> h(kCounterKinds * kCounterSlots);
        HIPCHK(c, hipMemcpyAsync(h.data(), c->counters, h.size() * 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        unsigned long long s[kCounterKinds] = {};
        for (int k = 0; k < kCounterKinds; ++k)
            for (int i = 0; i < kCounterSlots; ++i) s[k] += h[k * kCounterSlots + i];
        out->evals_init = s[0];
        out->evals_propagation = s[1];
        out->evals_refine = s[2];
        out->fallback_pixels = s[3];
        out->evals_short = s[4];
        out->evals_init_short = s[5];
    }
    out->evals_total = out->evals_init + out->evals_propagation + out->evals_refine;
    out->n_passes = c->n_timed;
    for (int i = 0; i < c->n_timed && i < 64; ++i) {
        float ms = 0.f;
        HIPCHK(c, hipEventSynchronize(c->ev[2 * i + 1]));
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]));
        out->ms_per_pass[i] = ms;
    }
    if (c->init_timed) {
        HIPCHK(c, hipEventSynchronize(c->ev_init[1]));
        HIPCHK(c, hipEventElapsedTime(&out->ms_init, c->ev_init[0], c->ev_init[1]));
    }
    out->ms_fuse_kernels = c->fuse_ms;
    out->n_fuse_kernels = c->fuse_n;
    return AMH_OK;
}

void amh_destroy(amh_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    free_net(c);
    free_fusion(c);
    for (auto &v : c->views) free_view(v);
    for (auto &j : c->jobs) free_job(j);
    free_batch(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->d_viewc) (void)hipFree(c->d_viewc);
    if (c->planes) (void)hipFree(c->planes);
    if (c->cost) (void)hipFree(c->cost);
    if (c->S) (void)hipFree(c->S);
    if (c->v) (void)hipFree(c->v);
    if (c->counters) (void)hipFree(c->counters);
    if (c->prop_feats) (void)hipFree(c->prop_feats);
    if (c->prop_pred) (void)hipFree(c->prop_pred);
    if (c->prop_qref) (void)hipFree(c->prop_qref);
    if (c->hyp) (void)hipFree(c->hyp);
    for (auto e : c->ev) (void)hipEventDestroy(e);
    for (auto e : c->ev_init)
        if (e) (void)hipEventDestroy(e);
    delete c;
}

}  // extern "C"
