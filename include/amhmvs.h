/*
 * amhmvs.h -- C-ABI of the MI355X (gfx950) checkerboard PatchMatch library.
 *
 * The library computes the depth and normal map of one reference image from N
 * calibrated source images with the method of Xu & Tao, "Multi-View Stereo with
 * Asymmetric Checkerboard Propagation and Multi-Hypothesis Joint View
 * Selection" (arXiv 1805.07920):
 *   - random scene-plane hypotheses per pixel (Sec. 2 / 3, PatchMatch init),
 *   - red/black checkerboard half-passes (Sec. 3.1, Fig. 2(a)) in which every
 *     pixel takes the lowest-cost neighbour of each of 8 asymmetric regions
 *     (Sec. 3.1, Fig. 2(d)), scores the 8 planes (plus its own) on every source
 *     with the bilaterally weighted NCC over an 11x11 window sampled every
 *     other row and column (Sec. 3.3, Eq. 8), infers per-pixel view weights
 *     from the 8 x N cost matrix (Sec. 3.2, Eq. 1-6), keeps the plane with the
 *     lowest aggregated cost (Eq. 7) and refines it (Sec. 3.3).
 *
 * Conventions
 *   - Every call returns amh_status; AMH_OK is 0, errors are negative.  No C++
 *     exception crosses the ABI.  amh_last_error() returns a message for the
 *     last failing call on a context.
 *   - Arguments are validated on the host before any HIP call, so invalid
 *     arguments are reported even on a machine without a GPU.
 *   - Cameras map world points to camera coordinates by X_cam = R X + t (R, K
 *     row-major).  K must be upper triangular with K[8] != 0.  Pixel (x, y) has
 *     its centre at integer coordinates, y points down; depth is camera z.
 *   - Images are row-major grayscale intensities on the [0, 255] scale.
 *   - Ownership: the caller owns every buffer it passes in; the context owns
 *     every buffer it allocates and frees them in amh_destroy.
 *   - Streams: all device work of a context runs in order on the HIP stream
 *     given to amh_create (NULL = the null stream).  Calls that return data to
 *     host memory synchronise that stream; calls with device destinations are
 *     stream-ordered and return without waiting.
 *   - A context is used by one host thread at a time.
 *   - Limits: 1..32 sources per reference (the view-selection set is a 32-bit
 *     mask); images up to 16351 x 16351 (the gather layout of one image, with its
 *     border of 16 texels, stays within 4 GiB).
 */
#ifndef AMHMVS_H
#define AMHMVS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct amh_ctx amh_ctx;

typedef enum {
    AMH_OK = 0,
    AMH_E_INVALID_ARG = -1, /* a pointer, size or parameter is out of its documented range */
    AMH_E_OOM = -2,         /* a device allocation failed */
    AMH_E_HIP = -3,         /* the HIP runtime reported an error (no device, launch failure, ...) */
    AMH_E_STATE = -4,       /* the call needs an earlier call that has not happened (e.g. views, a run) */
    AMH_E_UNSUPPORTED = -5  /* a valid request outside what the library supports */
} amh_status;

typedef enum { AMH_F32 = 0, AMH_F16 = 1 } amh_dtype;

/* Calibrated pinhole camera: x ~ K (R X + t). */
typedef struct {
    double K[9], R[9], t[3];
    int width, height;
} amh_camera;

/* An image handed to amh_init_views.  data points to height rows of
 * pitch_elems elements (pitch_elems >= width) of type dtype, in host memory
 * (on_device = 0) or device memory of the context's GPU (on_device = 1). */
typedef struct {
    const void *data;
    int width, height;
    int64_t pitch_elems;
    amh_dtype dtype;
    int on_device;
} amh_image;

/* Method parameters.  amh_params_default() fills the paper's values
 * (Sec. 4: tau_mc_init 0.8, alpha 90, beta 0.3, n1 2, n2 3, tau_up 1.2, k 4,
 * sigma_color 3, sigma_spatial 30). */
typedef struct {
    int refine;          /* 1: perturbation refinement after each pixel update (Sec. 3.3) */
    int include_self;    /* 1: the pixel's current plane competes in the final argmin */
    float depth_min, depth_max;
    float sigma_color, sigma_spatial;   /* bilateral NCC weights (Eq. 8) */
    float tau_mc_init, alpha;           /* threshold schedule (Eq. 2) */
    float beta;                         /* confidence width (Eq. 3) */
    float tau_up;                       /* good-view upper threshold (Sec. 3.2) */
    int n1, n2, k;                      /* good-view counts and top-k (Sec. 3.2) */
    uint64_t seed;                      /* key of the counter-based random generator */
    int timing;                         /* 1: record per-pass device times (amh_get_stats) */
    float conf_min;                     /* learned proposal: lowest confidence that replaces a random plane
                                         * (default 0: on held-out 1920x1280 scenes every in-range predicted
                                         * plane beat a random one after one iteration) */
    int sym_prop;        /* ablation of Sec. 4 (default 0): 1 replaces the asymmetric propagation by the
                          * symmetric checkerboard of the fast version (Fig. 2(c)): row r of the cost
                          * matrix takes the one neighbour at distance 1 (r < 4) or 5 (r >= 4) up, down,
                          * left, right; 2 by the standard version (Fig. 2(b)): 20 rows, one per
                          * other-colour neighbour within L1 distance 3 and the four axial ones at
                          * distance 5 (row-major order), the view selection's counts n1, n2 compared as
                          * the same fractions of the 20 rows (n 20 / 8) */
    int heuristic_views; /* ablation of Sec. 4 (default 0): 1 replaces the joint view selection by the
                          * heuristic one (Sec. 3.2): each hypothesis and each refinement candidate costs
                          * the mean of its own k lowest per-view costs; S = 0 and v = -1 are kept.
                          * Either ablation runs on the single-image path only (amh_pass and the calls
                          * built on it); the batched calls return UNSUPPORTED. */
    int bilateral_squared; /* 1: the bilateral weight of Eq. 8 with squared colour difference and squared
                            * distance, exp(-dI^2 / (2 sigma_color^2) - |dx|^2 / (2 sigma_spatial^2));
                            * default 0: unsquared, as the equation is printed */
    int sweep_sources;   /* learned proposal: the plane sweep reads the first min(sweep_sources, n_src)
                          * sources (list the nearest first); 0 (default) = 4; at most 32 */
} amh_params;

/* Counters of the work performed since the last amh_begin / amh_run_checkerboard. */
typedef struct {
    uint64_t evals_total;       /* hypothesis x view NCC evaluations (36 samples each) */
    uint64_t evals_init;        /* ... in the random initialisation */
    uint64_t evals_propagation; /* ... of the 8 propagated planes and the pixel's own */
    uint64_t evals_refine;      /* ... of refinement candidates */
    int n_passes;
    float ms_per_pass[64];      /* device time of each half-pass (timing = 1), else 0 */
    float ms_init;
    float ms_fuse_kernels;      /* timing = 1: device time of the per-view fusion kernels of the last amh_fuse */
    int n_fuse_kernels;         /* ... and their number (one per view) */
    uint64_t fallback_pixels;   /* initialisation from a proposal: pixels that kept the random plane (confidence
                                 * below conf_min, no normal, or the predicted plane out of range there) */
    uint64_t evals_short;       /* of evals_propagation + evals_refine: evaluations whose cost 2 was decided
                                 * before any sample was taken (plane depth outside [depth_min, depth_max] at the
                                 * pixel, window centre behind the source camera or outside its image, a window
                                 * corner not in front of it) */
    uint64_t evals_init_short;  /* the same among evals_init */
} amh_stats;

/* Batched job (see amh_run_batch). */
typedef struct {
    int ref;             /* view index (amh_init_views order) of the reference image */
    const int *srcs;     /* n_src view indices of its sources (host memory) */
    int n_src;
    int iters;
} amh_job;

/* Fills *out with the paper's parameters, depth range [2, 6], refine 1,
 * include_self 1, seed 0, timing 0, conf_min 0, no ablation.  INVALID_ARG if out is NULL. */
amh_status amh_params_default(amh_params *out);

/* Creates a context on the current HIP device.  p: parameters (copied).
 * hip_stream: a hipStream_t or NULL.  INVALID_ARG on bad parameters (checked
 * first), HIP if no device is usable. */
amh_status amh_create(amh_ctx **out, const amh_params *p, void *hip_stream);

/* Replaces the parameters of a context (INVALID_ARG if out of range). */
amh_status amh_set_params(amh_ctx *ctx, const amh_params *p);

/* Registers n_views images with their cameras (index = view id).  The library
 * copies them into its own device buffers: a float32 copy for use as a
 * reference, and a gather layout of the same values for use as a source, in
 * float32 or float16 (store_sources_as; float32 input is rounded to nearest
 * even).  The caller's buffers may be freed on return.  Replaces any views
 * registered before. */
amh_status amh_init_views(amh_ctx *ctx, int n_views, const amh_image *views, const amh_camera *cams,
                          amh_dtype store_sources_as);

/* Selects the reference view and its n_src sources for the following calls,
 * builds the per-view plane-induced warp constants (Sec. 3.3) and allocates
 * the per-pixel state.  Resets the statistics. */
amh_status amh_begin(amh_ctx *ctx, int ref, const int *srcs, int n_src);

/* Random initialisation of every pixel's plane (Philox keyed by the seed,
 * counter = pixel, iteration 0); initial cost = mean of the k lowest per-view
 * costs; empty view-selection memory. */
amh_status amh_init_hypotheses(amh_ctx *ctx);

/* One checkerboard half-pass of iteration t (0-based) on the pixels of one
 * colour (0 = red, (x + y) even; 1 = black): asymmetric propagation, cost
 * matrix, joint view selection, best plane, refinement (Sec. 3.1-3.3). */
amh_status amh_pass(amh_ctx *ctx, int t, int colour);

/* amh_begin + amh_init_hypotheses + iters x (red pass, black pass). */
amh_status amh_run_checkerboard(amh_ctx *ctx, int ref, const int *srcs, int n_src, int iters);

/* Copies the result of the current reference: depth (H*W, camera z), normal
 * (H*W*3, unit, facing the camera) and cost (H*W, aggregated NCC cost).  Any
 * of the three may be NULL.  dst_on_device: destinations are device pointers. */
amh_status amh_get_depth_normal_cost(amh_ctx *ctx, float *depth, float *normal, float *cost, int dst_on_device);

/* Largest reference (pixels) of amh_run_checkerboard_static, e.g. 2048 x 1280. */
#define AMH_STATIC_MAX_PIXELS 2621440

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): amh_run_checkerboard
 * followed by amh_get_depth_normal_cost into device buffers, allocating
 * nothing.  The per-pixel state and the sources' warp constants live in one
 * library-wide static device array (about 70 MiB per GPU the library runs on,
 * held until the process ends) instead of context buffers.
 *   ref, srcs, n_src, iters: as amh_run_checkerboard (views registered with
 *     amh_init_views); the reference may have at most AMH_STATIC_MAX_PIXELS
 *     pixels, larger ones give AMH_E_INVALID_ARG before any work.
 *   depth (H*W), normal (H*W*3), cost (H*W): device pointers owned by the
 *     caller, any may be NULL; written in stream order on the context's stream.
 * Results equal amh_run_checkerboard's bit for bit.  The context's current
 * reference is released (amh_get_state / amh_score_fixed need a new amh_begin);
 * amh_get_stats counts this run's evaluations, without per-pass times.
 * Every call on a GPU shares that GPU's array and leaves its state there: calls
 * that overlap on one GPU (other streams or contexts, not yet complete) race.
 * Synchronises the context's stream once, before writing the constants. */
amh_status amh_run_checkerboard_static(amh_ctx *ctx, int ref, const int *srcs, int n_src, int iters, float *depth,
                                       float *normal, float *cost);

/* Per-pixel state of the current reference: planes (H*W*4: n_x, n_y, n_z, d
 * with n.X + d = 0 in the reference camera frame), cost (H*W), S (H*W view
 * masks, bit j = j-th source of amh_begin), v (H*W, most important view or -1).
 * get: any pointer may be NULL; set: all four are required.  on_device as above. */
amh_status amh_get_state(amh_ctx *ctx, float *planes, float *cost, uint32_t *S, int32_t *v, int dst_on_device);
amh_status amh_set_state(amh_ctx *ctx, const float *planes, const float *cost, const uint32_t *S,
                         const int32_t *v, int src_on_device);

/* Matching cost (Eq. 8) of Q fixed hypotheses on every source of amh_begin:
 * planes (Q*4), pix (Q*2 ints: x, y) -> costs (Q*n_src, row-major by query).
 * All three in host memory (on_device = 0) or device memory (1). */
amh_status amh_score_fixed(amh_ctx *ctx, const float *planes, const int *pix, int Q, float *costs, int on_device);

/* Runs n_jobs reference images (views registered by amh_init_views; sizes and
 * view counts may differ) as one batch: one launch per phase (init of a
 * colour, or a half-pass) covering the tiles of every job that is still
 * iterating, all phases captured in one HIP graph.  The graph is kept and
 * replayed while the job list, the views and the parameters stay the same.
 * Stream-ordered; results are read with amh_get_job_result, work counters
 * with amh_get_stats and per-job completion times with amh_get_job_times.
 * INVALID_ARG on bad jobs (checked before any HIP call), STATE without views. */
amh_status amh_run_batch(amh_ctx *ctx, int n_jobs, const amh_job *jobs);

/* amh_run_batch with every job initialised from the learned proposal instead of
 * random planes: the plane sweep and the network's forward pass of each job
 * (amh_sweep_features, amh_nn_forward; sweep on the job's first min(s, n_src), s = sweep_sources or 4,
 * sources) and the proposal initialisation (amh_init_from_proposal) are
 * captured in the same graph ahead of the iterations.  STATE if the network
 * does not exist. */
amh_status amh_run_batch_proposal(amh_ctx *ctx, int n_jobs, const amh_job *jobs);

/* Depth / normal / cost of job `job` of the last batch (as amh_get_depth_normal_cost). */
amh_status amh_get_job_result(amh_ctx *ctx, int job, float *depth, float *normal, float *cost, int dst_on_device);

/* Completion time of every job of the last batch, in ms after the batch started
 * (device clock, stamped by the workgroup that finished the job's last tile).
 * n must equal the batch's job count.  Synchronises the stream. */
amh_status amh_get_job_times(amh_ctx *ctx, int n, float *job_ms);

/* Autotuner: times the batch under each launch configuration -- tile order (XCD
 * bands or hardware order) x job order (as given or largest first) x tile shape
 * of the half-pass (4 or 2 image rows per workgroup) x the batch's half-passes
 * launched one per phase or all in one persistent launch; configuration =
 * tile_order + 2 * job_order + 4 * (two-row tiles) + 8 * persistent -- keeps the
 * fastest for the following launches of this context (single images included)
 * and returns it in *best_config (may be NULL) with the measured ms in
 * ms_per_config[16] (may be NULL; -1 where not measured).  The persistent
 * launch runs every half-pass of every job in one kernel: each XCD's workgroups
 * take tiles from that XCD's bands of every job through a device-scope
 * counter, and the half-passes are separated by a grid barrier (device-scope
 * release, arrival count, acquire), so its grid is sized to the workgroups
 * that are resident at once; every wait is bounded, and a barrier that runs out
 * (workgroups not all resident, e.g. other work on the GPU) is reported as
 * AMH_E_HIP by amh_get_job_result, amh_get_job_times and amh_get_stats (the
 * bound is 4 s of device clock; the environment variable AMH_PERSIST_SPIN_TICKS,
 * read when a batch is built, replaces it by that many device-clock ticks -- a
 * test hook).  If the environment variable AMH_TUNE_CACHE
 * names a file, the choice is looked up there by shape bucket (job count,
 * largest view count, pixel count) and appended after tuning. */
amh_status amh_tune(amh_ctx *ctx, int n_jobs, const amh_job *jobs, int *best_config, float *ms_per_config);

/* Sets the launch configuration (0..15, numbered as for amh_tune) for the
 * following launches of this context; results do not depend on it.
 * INVALID_ARG outside 0..15. */
amh_status amh_set_launch_config(amh_ctx *ctx, int config);

/* Work counters and timings of the current reference (or of the last batch). */
amh_status amh_get_stats(const amh_ctx *ctx, amh_stats *out);

/* ------------------------------------------------------------------------
 * Learned proposal.  Not part of the paper: a small convolutional network
 * predicts a plane and a confidence per 4 x 4 cell of the reference image, so
 * that the iterations of Sec. 3 start from it instead of random planes
 * (random planes stay where the confidence is low).  The confidence target is
 * C(m) of Eq. 3 applied to the final cost of the plain method.
 * Network: 4-level encoder-decoder (channels 16/32/48/64, two 3x3
 * convolutions + ReLU per encoder level, 2x2 average pooling, nearest 2x
 * upsampling concatenated with the skip, one 3x3 convolution + ReLU per
 * decoder level, 1x1 head with 5 outputs); bf16 weights and activations, fp32
 * accumulation on the matrix cores; trained on the device (forward, loss and
 * gradient, Adam on fp32 master weights).  Parameters in canonical order, layer
 * by layer (enc0a, enc0b, enc1a, enc1b, enc2a, enc2b, enc3a, enc3b, dec2, dec1,
 * dec0, head), each the weight [c_out][ky][kx][c_in] then the bias [c_out].
 * ------------------------------------------------------------------------ */

/* Number of network parameters (196341).  INVALID_ARG if n is NULL. */
amh_status amh_nn_param_count(int64_t *n);

/* Creates (or re-creates) the network on the context: He-normal weights drawn
 * from the seed, biases 0 except the head's normal-z bias -1 (the initial
 * prediction faces the camera), cleared optimiser state. */
amh_status amh_nn_init(amh_ctx *ctx, uint64_t seed);

/* Host copies of the fp32 master parameters and of the last gradient (n floats,
 * canonical order; n must equal the parameter count).  set also clears the
 * optimiser state.  STATE if the network does not exist. */
amh_status amh_nn_get_params(amh_ctx *ctx, float *out, int64_t n);
amh_status amh_nn_set_params(amh_ctx *ctx, const float *in, int64_t n);
amh_status amh_nn_get_grads(amh_ctx *ctx, float *out, int64_t n);

/* Forward pass over n inputs of h x w cells (h, w positive multiples of 8):
 * feats (device, bf16 bit patterns, [n][h][w][16]) and q_ref (device, float,
 * [n][h][w], the sweep's winning inverse depth, amh_sweep_features) -> out
 * (device, float, [n][h][w][5]: depth, unit normal, confidence in (0, 1));
 * out may be NULL.  The depth head corrects q_ref by at most a twelfth of the
 * inverse-depth range: depth = 1 / clamp(q_ref + R tanh(z0), 1/depth_max,
 * 1/depth_min), R = (1/depth_min - 1/depth_max) / 12.  The inputs are copied
 * and the activations kept for amh_nn_backward. */
amh_status amh_nn_forward(amh_ctx *ctx, const void *feats, const float *q_ref, int n, int h, int w, float *out);

/* Loss of the last forward pass against target (device, float, [n][h][w][6]:
 * depth, normal (3), confidence target, weight of the depth and normal terms):
 * the mean over cells of weight * (|s - t| + 1 - n_hat . n_target) plus the
 * binary cross-entropy of the confidence, with s and t the predicted and target
 * depth mapped linearly from [depth_min, depth_max] to [0, 1].  Computes the
 * gradient of every parameter; *loss (host, may be NULL) receives the loss,
 * which synchronises the stream.  STATE without a forward pass. */
amh_status amh_nn_backward(amh_ctx *ctx, const float *target, float *loss);

/* Training targets of the proposal network from a depth map of the plain method:
 * depth (H*W), normal (H*W*3) and cost (H*W, the final aggregated matching
 * cost) of a width x height reference, device pointers -> target (device,
 * [h][w][6], h = 8 ceil(H / 32), w = 8 ceil(W / 32)), for cell (i, j) the
 * values at pixel (min(4j + 2, W - 1), min(4i + 2, H - 1)): depth, normal (3),
 * and the confidence C(m) = exp(-m^2 / (2 beta^2)) of Eq. 3 twice (the
 * confidence target and the weight of the depth and normal terms).  Stream-ordered. */
amh_status amh_nn_targets(amh_ctx *ctx, const float *depth, const float *normal, const float *cost, int width,
                          int height, float *target);

/* One Adam step (Kingma & Ba, bias-corrected) with the last gradient. */
amh_status amh_nn_adam_step(amh_ctx *ctx, float lr, float beta1, float beta2, float eps);

/* Saves / loads the parameters: 8-byte magic "AMHNN001", int64 count, count
 * little-endian floats in canonical order.  load creates the network if needed. */
amh_status amh_nn_save(amh_ctx *ctx, const char *path);
amh_status amh_nn_load(amh_ctx *ctx, const char *path);

/* Network input of the current reference (amh_begin), one 16-channel vector per
 * cell of 4 x 4 pixels on a grid of h4 = 8 ceil(H/32) rows x w4 = 8 ceil(W/32)
 * columns (cells past the image repeat its edge: coordinates are clamped).  A
 * plane sweep at the cell's pixel (min(4j + 2, W - 1), min(4i + 2, H - 1)) scores
 * D = 12 m fronto-parallel planes, m = max(1, (W + 80) / 160) (integer
 * division), at inverse depths 1/depth_max + (i + 1/2) (1/depth_min -
 * 1/depth_max) / D; a plane's aggregate is the mean of the min(2, n) lowest
 * matching costs (Eq. 8) over the first n = min(s, n_src) sources, s = amh_params.sweep_sources (4 when 0).  Channels:
 * (mean of the cell's 16 reference intensities - 127.5) / 64, their standard
 * deviation / 32, 2 (i* + 1/2) / D - 1 for the lowest aggregate i* (first on
 * ties), 1 - that aggregate, and 1 - the lowest aggregate of each of the 12
 * coarse bins of m consecutive planes.  feats: device, bf16 bit patterns,
 * [h4][w4][16]; q_ref (device, float, [h4][w4], may be NULL): the winning
 * plane's inverse depth. */
amh_status amh_sweep_features(amh_ctx *ctx, void *feats, float *q_ref);

/* Initialisation from per-cell predictions pred (device, float, [h][w][5] as
 * amh_nn_forward writes them) on a grid of 4 x 4 cells covering the image
 * (4 w >= W, 4 h >= H): pixel (x, y) takes the plane through the point at the
 * predicted depth on the ray of its cell's pixel (min(4j + 2, W - 1),
 * min(4i + 2, H - 1)), (i, j) = (y / 4, x / 4), with the predicted normal, when
 * the confidence is at least conf_min and that plane's depth along the pixel's
 * ray lies in [depth_min, depth_max]; otherwise the random plane of
 * amh_init_hypotheses.  Initial cost, S and v as there.  Replaces
 * amh_init_hypotheses after amh_begin. */
amh_status amh_init_from_proposal(amh_ctx *ctx, const float *pred, int h, int w);

/* Initial hypotheses from per-pixel estimates (for instance an earlier depth
 * map, another reference's result warped here, or a learned predictor at full
 * resolution), in place of the random initialisation (Sec. 3, the PatchMatch
 * random start):  depth (H*W, camera z), normal (H*W*3, camera frame, any
 * length and orientation) and conf (H*W, or NULL for all 1) of the current
 * reference, in host (on_device = 0) or device memory (1).  Pixel (x, y) takes
 * the plane through the point at its depth on its ray with its normal turned
 * to face the camera when conf >= conf_min, the normal is non-zero and finite
 * and the depth is finite and within [depth_min, depth_max]; otherwise the
 * random plane of amh_init_hypotheses.  Initial cost (mean of the k lowest
 * per-view costs), S and v as there.  Replaces amh_init_hypotheses after
 * amh_begin; amh_pass continues from it.  Host inputs may be reused on return;
 * device inputs must stay unchanged until the stream reaches this work. */
amh_status amh_set_initial_hypotheses(amh_ctx *ctx, const float *depth, const float *normal, const float *conf,
                                      int on_device);

/* amh_begin + amh_sweep_features + amh_nn_forward + amh_init_from_proposal +
 * iters x (red pass, black pass).  The sweep reads the first min(s, n_src), s = sweep_sources or 4,
 * sources (list the nearest first); the iterations use all of them.  STATE if
 * the network does not exist. */
amh_status amh_run_proposal(amh_ctx *ctx, int ref, const int *srcs, int n_src, int iters);

/* ------------------------------------------------------------------------ */
/* After the depth maps (Sec. 3.3, last two paragraphs): the 4 x 4 median     */
/* filter and the consistency-check fusion into a point cloud.                */
/* ------------------------------------------------------------------------ */

/* Thresholds of the fusion's consistency check (the check of Gipuma the paper
 * adopts, with its values): f_eps disparity difference in pixels (0.3), f_ang
 * normal angle in degrees (30), f_con consistent views needed (2). */
typedef struct {
    float f_eps;
    float f_ang_deg;
    int f_con;
} amh_fusion_params;

/* Fills *out with f_eps 0.3, f_ang_deg 30, f_con 2.  INVALID_ARG if out is NULL. */
amh_status amh_fusion_params_default(amh_fusion_params *out);

/* 4 x 4 median filter of a depth map (Sec. 3.3).  src, dst: device pointers to
 * width * height floats, row-major, not overlapping (INVALID_ARG if src == dst).
 * dst(x, y) is the median of src over columns x-1..x+2 and rows y-1..y+2 clipped
 * to the image; NaN values are skipped (all NaN: NaN); an even count takes the
 * mean of the two middle values.  Enqueued on the context's stream (no wait). */
amh_status amh_median_filter4(amh_ctx *ctx, const float *src, float *dst, int width, int height);

/* Consistency-check fusion (Sec. 3.3, fusion paragraph) of n_views (1..128)
 * depth maps into one point cloud.  views[k]: a view registered with
 * amh_init_views (its camera and size); depth[k] (H*W floats, camera z; a value
 * that is not finite or not positive means no depth) and normal[k] (H*W*3
 * floats, unit, camera frame): device pointers.  Views are taken as references
 * in the order given.  A pixel p of view k not consumed by an earlier view
 * back-projects to a world point X; another view j is consistent when X lies in
 * front of j, projects to a pixel q (nearest, floor(u + 0.5)) inside j where j
 * has a depth, the disparity difference f_j |C_k - C_j| |1/z_j(X) - 1/d_j(q)|
 * is below f_eps (f_j = K_j[0][0] / K_j[2][2]) and the angle between the two
 * world normals is below f_ang.  With at least f_con consistent views p yields
 * a point (mean of X and the consistent back-projections, normalised sum of the
 * normals) and its witnesses q are consumed.  Points come in view order, then
 * raster order: points (capacity * 3 floats, world frame), point_normals
 * (capacity * 3 floats, or NULL), origin (capacity * 3 int32: view slot k,
 * pixel index y W + x, number of consistent views; or NULL) -- device pointers;
 * the first min(total, capacity) points are written and *n_points (host)
 * receives the total.  Waits for the result.  The context keeps a workspace of
 * the views' pixel count + 36 bytes per pixel of the largest view. */
amh_status amh_fuse(amh_ctx *ctx, int n_views, const int *views, const float *const *depth,
                    const float *const *normal, const amh_fusion_params *fp, float *points, float *point_normals,
                    int32_t *origin, int64_t capacity, int64_t *n_points);

/* Instruction-throughput probe of the current device: a measurement utility for
 * the roofline (the issue rate of one vector-ALU instruction kind), no part of
 * the method.  Launches `blocks` workgroups of 256 threads on the null stream;
 * every lane runs 16 independent chains of `iters` instructions of one kind,
 * so the launch issues 16 * iters * blocks * 4 wave instructions of it.  kind:
 * 0 v_fma_f32 (vector-register operands), 1 v_fma_f32 reading a scalar
 * register, 2 v_rcp_f32, 3 v_fract_f32, 4 v_cvt_flr_i32_f32, 5 v_med3_i32,
 * 6 v_mad_u32_u24, 7 v_add_f32 with a literal.  *ms (host) receives the
 * launch's device time (a first one-block launch loads the code untimed).
 * INVALID_ARG for another kind, blocks or iters outside 1..65536 or ms NULL;
 * OOM if its output (blocks KiB, freed on return) cannot be allocated; HIP_ERROR
 * without a device.  Synchronous. */
amh_status amh_probe_valu(int kind, int blocks, int iters, float *ms);

const char *amh_status_str(amh_status s);
const char *amh_last_error(const amh_ctx *ctx);

/* Frees the context and everything it owns.  NULL is ignored. */
void amh_destroy(amh_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
