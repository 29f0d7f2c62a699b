// Internal interface between the host runtime (amh_api.hip) and the gfx950
// kernels (amh_kernels.hip).  Plain-old-data structs passed by value to kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace amh {

constexpr int kMaxSrc = 32;
// Border of the sources' gather layout: kQuadPad extra texel columns on every side, holding the clamped footprint
// (a window that crosses the image edge by up to kQuadPad texels reads the values clamping would give, without
// clamping).  Images are limited to kMaxImageSide so that the layout's byte offsets stay below 2^32.
constexpr int kQuadPad = 16;
constexpr int kMaxImageSide = 16383 - 2 * kQuadPad;
constexpr int kCounterSlots = 256;    // eval counters are spread over slots to avoid one hot atomic
constexpr int kCounterKinds = 6;      // init, propagation, refinement evaluations; proposal fallbacks;
                                       // short evaluations (no samples taken) of the half-pass and of init
constexpr int kGroups = 7;            // pixels per wave (7 groups x 9 lanes = 63 lanes)
constexpr int kRows = 9;              // 8 propagated hypotheses + the pixel's own
constexpr int kTilePix = kGroups;     // same-colour pixels per tile row
// image rows per workgroup tile of the half-pass (one wave per row): 4 by default, 2 as the
// autotuner's alternative tile shape
constexpr int kDefaultTileRows = 4;

// One source view relative to the current reference (Sec. 3.3: plane-induced warp).
// Homogeneous source pixel of reference pixel (x, y) on the plane with inverse
// depth q(x, y):  A (x, y, 1)^T + b q.
struct ViewDev {
    double A[9];            // K_j R_rel K_ref^-1 (row-major)
    double b[3];            // K_j t_rel
    const void *quads;      // (H+1+2P) x (W+2+2P) texel columns, 2 x float or 2 x half
    int W, H;
};

struct RefDev {
    const float *img;       // H x W float32 reference intensities
    int W, H;
    double kinv_a, kinv_b, kinv_c, kinv_e, kinv_f;  // K_ref^-1 = [[a, b, c], [0, e, f], [0, 0, 1]]
};

struct MethodDev {
    float d_min, d_max;
    float inv_2sc2, inv_2sx2;    // 1 / (2 sigma_color^2), 1 / (2 sigma_spatial^2)
    float tau, tau_up;           // tau_mc(t) of the pass, upper threshold
    float inv_2b2;               // 1 / (2 beta^2)
    int n1, n2, k;
    int include_self, refine;
    uint64_t seed;
    int sym_prop, heuristic;     // ablation switches (symmetric propagation, heuristic views)
    int bil_sq;                  // squared colour difference and distance in the bilateral weight
    double q_lo, q_hi;           // inverse depths of d_max (1 + 1e-5) and d_min (1 - 1e-5): the range test
};

struct StateDev {
    float4 *planes;              // H x W (n_x, n_y, n_z, d)
    float *cost;
    uint32_t *S;
    int32_t *v;
};

struct PassArgs {
    RefDev ref;
    const ViewDev *views;        // device array [n_src]
    int n_src;
    MethodDev m;
    StateDev st;
    int t, colour;
    int tiles_x, n_tiles;        // tile grid of this colour
    unsigned long long *counters;  // [kCounterKinds][kCounterSlots], kinds as listed at kCounterKinds
    int order;                   // tile order: 0 XCD bands, 1 hardware order
    int waves = kDefaultTileRows;  // tile rows = waves per workgroup (2 or 4)
    // initialisation from per-cell predictions (NULL: random initialisation)
    const float *prop = nullptr;  // [prop_h][prop_w][5]: depth, normal (3), confidence
    int prop_w = 0, prop_s = 0;   // cell grid width, cell size in reference pixels
    float conf_min = 0.f;
};

// Pixels of one colour per initialisation workgroup (one per pair of lanes), and the workgroups of one colour.
constexpr int kInitBlock = 128;
__host__ __device__ inline long long init_blocks(int W, int H) {
    return ((long long)H * ((W + 1) / 2) + kInitBlock - 1) / kInitBlock;
}

// one reference image of a batch
struct BatchJobDev {
    RefDev ref;
    const ViewDev *views;        // n_src warp constants
    int view_off;                // ... at BatchPhaseArgs::views + view_off
    int n_src;
    StateDev st;
    int tiles_x, n_tiles;        // tile grid of one colour
    int n_iblocks;               // initialisation blocks of one colour (init_blocks)
    const float *prop;           // per-cell predictions for the initialisation, or NULL (random)
    int prop_w;                  // cell grid width
};

// one phase (init of a colour, or a half-pass) over the active jobs of a batch
struct BatchPhaseArgs {
    const BatchJobDev *jobs;
    const ViewDev *views;        // the warp constants of every job's sources
    const int *tile_start;       // [n_active + 1] prefix sums of the active jobs' tile counts
    const int *job_of;           // [n_active] job index of each active entry
    const int *is_last;          // [n_active] 1 if this phase is the job's last one
    const int *xcd_pre;          // [8][n_active + 1] per-XCD prefix sums of the band sizes (tile order 0)
    int n_active, total_tiles;
    int grid;                    // workgroups of the launch
    MethodDev m;
    int t, colour, kind;         // kind 0: init, 1: half-pass
    int order;
    int waves;                   // tile rows = waves per workgroup (2 or 4)
    float conf_min;              // proposal initialisation threshold
    unsigned long long *counters;
    unsigned long long *tiles_done;  // [n_jobs] tiles finished in the job's last phase
    unsigned long long *job_end; // [n_jobs] device clock at the job's completion
};

// One phase of the persistent batched launch: the tables of BatchPhaseArgs, with every job of the phase
// in one LDS class (the launch's).
struct PersistPhase {
    const int *tile_start, *job_of, *is_last, *xcd_pre;
    int n_active, total_tiles;
    int t, colour;
    MethodDev m;
};

// The persistent batched launch: every half-pass of every job in one kernel.  Workgroup b serves the queue of
// XCD b mod 8 (that XCD's bands of every job, as tile order 0 of the per-phase launches), taking tiles with
// a device-scope counter; the phases are separated by a grid barrier (device-scope release, arrival count,
// acquire).  Every wait is bounded by spin_limit device-clock ticks; a wait that runs out sets *fault and
// every workgroup leaves (reported by the host as an error).
struct PersistArgs {
    const BatchJobDev *jobs;
    const ViewDev *views;
    const PersistPhase *phases;  // [n_phases]
    int n_phases;
    float conf_min;
    unsigned long long *counters, *tiles_done, *job_end;
    unsigned *next;              // [n_phases][8] tiles taken from each XCD's queue
    unsigned *arrived;           // grid-barrier arrivals (monotonic over the phases)
    unsigned *fault;
    unsigned long long spin_limit;
    // residency probe (probe = 1): every workgroup counts in (next[0]), waits up to probe_ticks for the
    // whole grid to be in at once, records the most it saw resident together (next[2]), counts out (next[1])
    int probe;
    unsigned long long probe_ticks;
};

constexpr int kSweepCoarse = 12;  // coarse inverse-depth bins of the proposal's input sweep
constexpr int kNetSrc = 4;        // sources the sweep reads unless amh_params::sweep_sources says otherwise
constexpr int kSweepK = 2;        // aggregate: mean of the kSweepK lowest costs
constexpr int kCell = 4;          // reference pixels per feature cell side

// plane-sweep input of the proposal network: one 16-channel bf16 vector per 4x4 cell
struct SweepArgs {
    RefDev ref;
    const ViewDev *views;
    int n_net;                   // sources used (the first min(sweep_sources or 4, n_src))
    MethodDev m;
    int h4, w4;                  // cell grid
    int sub;                     // sweep planes per coarse bin (12 * sub planes)
    float q_far, q_step;         // inverse depth of plane i: q_far + (i + 1/2) q_step
    unsigned short *feats;       // [h4 * w4][16] bf16
    float *q_ref;                // [h4 * w4] inverse depth of the winning plane, or NULL
    unsigned long long *counters;
};

struct ScoreArgs {
    RefDev ref;
    const ViewDev *views;
    int n_src;
    MethodDev m;
    const float4 *planes;        // Q
    const int2 *pix;             // Q
    int Q;
    float *costs;                // Q x n_src
};

// launchers (amh_kernels.hip); all return the launch status
hipError_t launch_convert_to_f32(const void *src, int src_dtype, int64_t pitch, int W, int H, float *dst,
                                 hipStream_t s);
hipError_t launch_pack_quads(const float *img, int W, int H, void *quads, int half, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long *p, int n, hipStream_t s);
hipError_t launch_init(const PassArgs &a, int half, hipStream_t s);
hipError_t launch_pass(const PassArgs &a, int half, hipStream_t s);
hipError_t launch_persist(const PersistArgs *a, int half, int waves, int max_src, int grid, hipStream_t s);
int persist_blocks_per_cu(int half, int waves, int max_src);
hipError_t launch_pack_hypotheses(const float *depth, const float *normal, const float *conf, int64_t n, float *out,
                                  hipStream_t s);
hipError_t launch_score(const ScoreArgs &a, int half, hipStream_t s);
hipError_t launch_outputs(const RefDev &ref, const StateDev &st, float *depth, float *normal, float *cost,
                          hipStream_t s);
hipError_t launch_batch(const BatchPhaseArgs &b, int half, int max_src, hipStream_t s);
hipError_t launch_stamp(unsigned long long *p, hipStream_t s);
hipError_t launch_sweep(const SweepArgs &a, int half, hipStream_t s);
size_t pass_lds_bytes(int n_src, int waves, int rb = 1);

}  // namespace amh
