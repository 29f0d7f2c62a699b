/*
 * CPU oracle for the checkerboard PatchMatch pass of AMHMVS
 * (Xu & Tao, "Multi-View Stereo with Asymmetric Checkerboard Propagation and
 * Multi-Hypothesis Joint View Selection", arXiv 1805.07920).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, double-precision
 * restatement of the method, used to check the GPU library.  Only the tests,
 * the smoke check and the benchmark's CPU-baseline leg may call it; the
 * library never does.  It shares no code, header, table or constant with the
 * GPU path.
 *
 * Parity status per function (pins live in tests/):
 *   orc_philox4x64_10      pinned (bit-exact vs numpy.random.Philox)
 *   orc_project            pinned (closed-form homography, renderer geometry)
 *   orc_matching_cost      pinned (numpy.cov / corrcoef reductions, invariances,
 *                          exact integer-disparity case)
 *   orc_view_selection     pinned (hand-computed matrices, closed forms of Eq. 2-4)
 *   orc_acp_offsets        pinned (invariants of the region table)
 *   orc_scp_offsets        pinned (symmetry, colour and subset invariants)
 *   orc_sscp_offsets       pinned (the same invariants; one half-pass reaches exactly
 *                          its 20 neighbours)
 *   orc_view_selection_rows  pinned (20-row matrices against a brute-force count
 *                          with the thresholds scaled; 8 rows equal orc_view_selection)
 *   heuristic view mode    pinned (mean of the k lowest against numpy sorts; k >= N
 *                          equals the plain mean, k = 1 the minimum)
 *   orc_random_plane       pinned (uniform depth on the range; direction uniform on
 *                          the hemisphere facing the ray: Kolmogorov-Smirnov tests)
 *   orc_init               pinned (mean of the min(k, N) lowest costs against a numpy
 *                          sort; empty selection memory)
 *   orc_pass / orc_run     pinned by recovery of rendered ground truth, brute-force
 *                          plane sweep and order independence; the empty-selection
 *                          fallback by a hand-built matrix; refinement by the
 *                          invariants of its candidates (counts, perturbation
 *                          ranges reached and never exceeded, shared and fresh
 *                          draws, clamping), Eq. 7 scoring on the weighted views
 *                          and strict in-order acceptance (an exact-tie case).
 *                          The refinement schedule itself is a reading (R13) of a
 *                          step the paper defers to an earlier system.
 */
#ifndef AMH_ORACLE_H
#define AMH_ORACLE_H
#include <stdint.h>

#define ORC_MAX_SRC 32
#define ORC_N_OFFSETS 72
#define ORC_MAX_ROWS 21   /* propagated rows (8, or 20 in the standard symmetric pattern) + the pixel's own */

/* decisions of a pixel update that clear a given margin (orc_diag.robust) */
#define ORC_ROBUST_S 1       /* good-view tests (S_t) */
#define ORC_ROBUST_V 2       /* most important view v_t */
#define ORC_ROBUST_TOPK 4    /* top-k cut of the weights */
#define ORC_ROBUST_ARGMIN 8  /* best hypothesis */
#define ORC_ROBUST_REFINE 16 /* refinement acceptances */

typedef struct {
    int W, H, n_src;
    const float *ref;                 /* H*W row-major intensities in [0,255] */
    const float *src[ORC_MAX_SRC];    /* source j: srcH[j]*srcW[j] row-major */
    int srcW[ORC_MAX_SRC], srcH[ORC_MAX_SRC];
    double Kref[9], Rref[9], tref[3]; /* X_cam = R X_world + t, row-major 3x3 */
    double Ksrc[ORC_MAX_SRC][9], Rsrc[ORC_MAX_SRC][9], tsrc[ORC_MAX_SRC][3];
} orc_views;

typedef struct {
    int refine, include_self;
    double d_min, d_max, sigma_color, sigma_spatial;
    double tau_mc_init, alpha, beta, tau_up;
    int n1, n2, k;
    uint64_t seed;
    int view_mode;   /* 0: joint view selection (the method); 1: plain mean over all views
                        (a static objective, used only by the brute-force sweep pin);
                        2: heuristic selection, mean of each hypothesis' k lowest costs */
    int prop_mode;   /* 0: asymmetric checkerboard propagation (the method);
                        1: symmetric checkerboard propagation, fast version (ablation, Fig. 2(c));
                        2: symmetric checkerboard propagation, standard version (ablation, Fig. 2(b)):
                           20 rows, the view selection's counts n1, n2 scaled by 20/8 */
    int bilateral_sq; /* 1: squared colour difference and distance in the bilateral weight */
    int sample_f32;   /* conditioning probe, not the method: 1 rounds every sample's source position
                         (relative to the texel under the window centre) and its interpolated value to
                         float32, to measure how far the method's result moves when those carry single
                         precision; 2 also forms the weights' sums and the NCC's moments in float32;
                         3 instead moves every sample value by the first-order bound of rounding its
                         position and value to float32, in the direction that moves the cost towards
                         1 (the worst case of that rounding), in double otherwise; 0 (the method):
                         every step in double */
    double cost_noise; /* conditioning probe, not the method: > 0 adds to every scored cost a deterministic
                          offset uniform in [-cost_noise/2, cost_noise/2) (a hash of pixel, view and
                          plane), to measure what cost errors of that size do to the result; 0: none */
} orc_params;

typedef struct {
    double *plane;   /* P*4: n_x, n_y, n_z, d_p with n.X + d_p = 0 in the reference camera frame */
    double *cost;    /* P */
    uint32_t *S;     /* P: view-selection set of the pixel's last update (bit j = source j) */
    int32_t *v;      /* P: most important view of the last update, -1 if none */
} orc_state;

typedef struct {
    /* rows 0..n_prop-1 are the propagated hypotheses (regions), row n_prop the pixel's own plane;
       n_prop = 8, or 20 in the standard symmetric pattern */
    double mfinal[ORC_MAX_ROWS];   /* aggregated cost of every row; +inf if absent */
    double M[ORC_MAX_ROWS][ORC_MAX_SRC];
    int row_valid[ORC_MAX_ROWS];
    int cand_index[ORC_MAX_ROWS - 1];  /* index into the offset table of the picked neighbour, -1 if none */
    double w[ORC_MAX_SRC];
    uint32_t S;
    int v;
    int chosen;         /* 0..n_prop-1 region row, n_prop self, n_prop+1+c refinement candidate c */
    double cand_cost[6];
    double cand_plane[6][4];
    int n_cand;
    int robust;         /* ORC_ROBUST_* bits of the decisions that clear the margin delta */
    int n_prop;
} orc_diag;

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
double orc_u24(uint64_t w);
int orc_acp_offsets(int *dx, int *dy, int *region);
int orc_scp_offsets(int *dx, int *dy, int *region);
int orc_sscp_offsets(int *dx, int *dy, int *region);
void orc_project(const orc_views *V, double sx, double sy, const double plane[4], int j, double out[3]);
double orc_matching_cost(const orc_views *V, const orc_params *p, int x, int y, const double plane[4], int j);
double orc_tau(const orc_params *p, int t);
void orc_view_selection(const orc_params *p, int t, const double *M, const int *row_valid, int N,
                        uint32_t S_prev, int v_prev, uint32_t *S_out, int *v_out, double *w_out);
void orc_view_selection_rows(const orc_params *p, int t, const double *M, const int *row_valid, int R, int N,
                             uint32_t S_prev, int v_prev, uint32_t *S_out, int *v_out, double *w_out);
void orc_random_plane(const orc_views *V, const orc_params *p, int x, int y, uint64_t t, uint64_t purpose,
                      double plane[4]);
void orc_init(const orc_views *V, const orc_params *p, orc_state *s);
void orc_pass(const orc_views *V, const orc_params *p, orc_state *s, int t, int colour,
              const int *order, int n_order, double delta, orc_diag *diag);
void orc_run(const orc_views *V, const orc_params *p, orc_state *s, int iters);
void orc_depth_normal(const orc_views *V, const orc_state *s, double *depth, double *normal);
int orc_num_threads(void);
void orc_set_num_threads(int n);

#endif
