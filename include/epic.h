/*
 * epic.h -- C ABI of the MI355X (gfx950) sparse-to-dense, edge-preserving
 * interpolation library (EpicFlow, Revaud et al. 2015, Sec. 3).
 *
 * Given an edge cost map C and a sparse set of matches M = {(p_m, p'_m)},
 * the library computes a dense displacement field:
 *   1. geodesic distance D(p) from every pixel to its nearest match and the
 *      geodesic Voronoi label L(p) (Eq. 3; Sec. 3.4, "Geodesic Voronoi
 *      diagram");
 *   2. the match graph: cells adjacent in L are joined, weighted by the
 *      geodesic distance restricted to the two cells (Sec. 3.4,
 *      "Approximated geodesic distance", Eq. 4);
 *   3. the K nearest matches of every match by Dijkstra on that graph
 *      (Algorithm 1, steps 4-5);
 *   4. one Nadaraya-Watson (Eq. 1) or locally-weighted affine (Eq. 2) model
 *      per match with weights exp(-a d) (Algorithm 1, step 6);
 *   5. every pixel takes the model of its cell (Algorithm 1, steps 7-8;
 *      Sec. 3.4, "Piecewise field").
 *
 * Conventions (all entry points):
 *   - C linkage; no exception crosses the ABI; every entry point returns an
 *     epic_status (0 = success) unless stated otherwise.
 *   - Device pointers are plain HIP device addresses (e.g. torch tensors'
 *     data pointers) on the context's device; host pointers are marked.
 *   - The caller owns every input and output buffer and keeps it alive until
 *     the work queued on `stream` has completed.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls are asynchronous: they enqueue kernels and return without
 *     synchronising, except where stated.
 *   - A context is used by one host thread at a time.  Its workspace is
 *     allocated once, in epic_create; no call allocates device memory.
 *   - Coordinates: pixel (x = column, y = row), integer pixel centres,
 *     origin at the top-left pixel.  Row-major images.
 *   - cost: H*W float32, every value finite and > 0 (checked on the device
 *     only with the debug_validate option; without it other values give
 *     undefined results).
 *   - matches: N*4 float32 rows (x, y, x', y').  A match is placed on the
 *     pixel floor(x+0.5), floor(y+0.5) (matches are pixels, Sec. 3.1);
 *     matches outside the image are dropped, and when several matches fall
 *     on one pixel the lowest index keeps it.  Dropped matches are counted.
 *   - flow: H*W*2 float32, interleaved displacement (u, v) = F(p) - p.
 */
#ifndef EPIC_H_
#define EPIC_H_

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    EPIC_NW = 0,   /* Nadaraya-Watson: kernel-weighted mean displacement, Eq. (1) */
    EPIC_LA = 1    /* locally-weighted affine least squares, Eq. (2)              */
} epic_mode;

typedef enum {
    EPIC_OK = 0,
    EPIC_ERR_ARG = -1,         /* invalid argument (checked on the host)            */
    EPIC_ERR_WORKSPACE = -2,   /* workspace of the context too small for the call   */
    EPIC_ERR_NO_MATCHES = -3,  /* no match lies in the image (flow is filled with NaN) */
    EPIC_ERR_HIP = -4,         /* a HIP runtime call failed                          */
    EPIC_ERR_BUDGET = -5,      /* request exceeds the memory budget it was given     */
    EPIC_ERR_CAPACITY = -6,    /* a fixed-capacity device structure overflowed: the
                                  match-graph hash; on the FP32 path, a match
                                  whose cell touches more than 65535 others; or a
                                  match whose graph search visited more nodes than
                                  the largest K-NN table holds (2048 entries for
                                  K <= 256; that match's model is then zero)      */
    EPIC_ERR_CONVERGENCE = -7, /* the geodesic transform hit its iteration bound     */
    EPIC_ERR_COST = -8,        /* debug_validate found a cost value that is not
                                  finite and > 0 (the flow is filled with NaN)     */
    EPIC_ERR_INVARIANT = -9    /* debug_validate found a violated invariant of the
                                  transform or the match graph (n_invariant)       */
} epic_status;

/* Options; NULL selects the defaults shown. */
typedef struct epic_options {
    int   connectivity;     /* 8 (default) or 4: pixel neighbourhood of the
                               discretised geodesic (Eq. 3)                    */
    int   la_weight_power;  /* 2 (default): each equation of Eq. (2) scaled by
                               k, i.e. weights k^2 in the normal equations;
                               1: weights k                                    */
    int   precision;        /* 0 (default): FP32 distances and fits, FP64 only
                               for ill-conditioned affine fits;
                               1: FP64 graph distances and fits everywhere     */
    float fp64_route;       /* FP32 conditioning (eigenvalue ratio of the
                               weighted neighbour covariance) below which an
                               affine fit is redone in FP64; default 1e-3      */
    double degenerate_tau;  /* eigenvalue ratio at or below which the
                               neighbourhood is near-collinear and LA falls
                               back to NW (decided in FP64); default 1e-9      */
    int   tile_w, tile_h;   /* geodesic-transform tile (0 = default 32 x 16;
                               supported: 32x16, 32x32, 32x64; tile_w is 32)   */
    int   geo_passes;       /* bulk-synchronous passes of the geodesic
                               transform launched per call, at most 255;
                               0 (default) = automatic: the most passes
                               the last 8 finished calls needed, plus 1
                               when those needs differed (16 before the
                               first; the FP64 path keeps this per phase of
                               its transform and launches at least 16 when
                               the needs differed).  A
                               single-workgroup finisher completes the
                               transform if they do not reach the fixpoint,
                               so this only affects speed, never results     */
    int   geo_threads;      /* threads per tile in the transform's passes after
                               the first: 0 (default: 256 for 32x16 tiles,
                               128 for 32x32, 256 for 32x64); 128 or 256 are
                               accepted with 32x16 tiles (runs of 4 or 2
                               pixels), other values give the default.  Only
                               speed depends on it                          */
    int   debug_validate;   /* 0 (default); 1: every call first checks on the
                               device that each cost value is finite and > 0
                               (one extra read of the cost map).  A pair whose
                               map fails is not interpolated: it reports
                               EPIC_ERR_COST and n_bad_cost in epic_stats and
                               its flow is filled with NaN; the other pairs of
                               a batch are unaffected.  It also checks the
                               intermediate state on the device: after the
                               transform, that every pixel has a defined label,
                               that seeds hold D = 0 and their own (lowest)
                               index, and that no neighbour offers a pixel a
                               better (D, label) than it holds in the
                               transform's arithmetic (the fixpoint of Eq. (3)
                               on the pixel graph); after the graph build, that
                               the adjacency is symmetric with equal weights
                               and consistent row pointers.  Violations are
                               counted in n_invariant and reported as
                               EPIC_ERR_INVARIANT; results are unchanged.
                               2: as 1, after first raising pixel 0's distance
                               of every pair by one (a planted violation that
                               tests the checks; results are then not
                               meaningful)                                     */
    float prune_px;         /* consistency check of the matches (Sec. 5.1,
                               "Pruning of matches"): 0 (default) = off; > 0:
                               every call first interpolates with NW (same K
                               and a), removes the matches whose displacement
                               differs from that estimate at their own pixel
                               by more than prune_px pixels (the paper uses
                               5), then interpolates the kept matches with the
                               requested estimator.  Twice the work of a call
                               without it; stats report n_pruned           */
} epic_options;

typedef struct epic_ctx epic_ctx;

/* Creates a context on HIP device `device` that owns `workspace_bytes` of
 * device memory (allocated here, once).  Returns NULL on failure (bad
 * device, allocation failure); epic_last_error() then tells why. */
epic_ctx* epic_create(int device, size_t workspace_bytes, const epic_options* opts);

/* Frees the context and its workspace.  The caller must have synchronised
 * every stream used with it.  NULL is ignored. */
void epic_destroy(epic_ctx* ctx);

/* Workspace bytes one call with these sizes needs (host only; no device
 * access).  Returns 0 for invalid sizes. */
size_t epic_workspace_bytes(int H, int W, int N, int K, int mode, int precision);

/* Dense interpolation of one image pair (Algorithm 1).
 *   cost    device, H*W float32 (edge cost map C)
 *   matches device, N*4 float32 (x, y, x', y')
 *   K       neighbours per match (>= 1; clamped to the number of usable
 *           matches); supported up to 256
 *   a       kernel parameter of exp(-a d) (finite, >= 0)
 *   mode    EPIC_NW or EPIC_LA
 *   flow    device, H*W*2 float32 output (u, v)
 * Host-side validation returns EPIC_ERR_ARG (null pointers, cost not
 * 4-byte, matches not 16-byte or flow not 8-byte aligned, H, W, N or K
 * < 1, H*W >= 2^31, K > 256, non-finite or negative a, bad mode) and
 * EPIC_ERR_WORKSPACE, before anything is enqueued.  Conditions found on the
 * device (no usable match, capacity overflow) are reported by
 * epic_get_stats after the stream has been synchronised. */
int epic_interp(epic_ctx* ctx, const float* cost, int H, int W,
                const float* matches, int N, int K, float a, int mode,
                float* flow, void* stream);

/* One request of a batch: same meaning as the arguments of epic_interp. */
typedef struct epic_request {
    const float* cost;
    int H, W;
    const float* matches;
    int N, K;
    float a;
    int mode;
    float* flow;
} epic_request;

/* Interpolates n independent pairs in one fused sequence of launches: each
 * stage runs once for all pairs (tiles, pixels and matches of every pair
 * are the work items of one launch).  Each pair's result equals what
 * epic_interp gives for it alone.  `reqs` is a host array.  The sum of the
 * pairs' workspace needs must fit the context workspace. */
int epic_interp_batch(epic_ctx* ctx, const epic_request* reqs, int n, void* stream);

/* Captured launch sequence of one batch (a HIP graph).  The graph is bound
 * to the buffers of `reqs` (their contents may change between launches) and
 * to the context's workspace; replaying it runs exactly the work that
 * epic_interp_batch(ctx, reqs, n, ...) enqueues, with one graph launch.
 * Capture happens on a private stream and does not run any work.  The
 * context must outlive the graph, and launches of graphs and other calls
 * on one context must be ordered by the caller (same stream, or events). */
typedef struct epic_graph epic_graph;
epic_graph* epic_graph_capture(epic_ctx* ctx, const epic_request* reqs, int n);
int epic_graph_launch(epic_graph* g, void* stream);
void epic_graph_destroy(epic_graph* g);

/* Per-call device-side counters, valid once the stream of the last call
 * has been synchronised (this call synchronises that stream itself). */
typedef struct epic_stats {
    int status;            /* EPIC_OK or a device-detected epic_status     */
    int n_used;            /* matches placed on a pixel                     */
    int n_outside;         /* matches dropped: outside the image            */
    int n_duplicate;       /* matches dropped: pixel held by a lower index  */
    int n_edges;           /* edges of the match graph                      */
    int n_degenerate;      /* LA fits that fell back to NW                  */
    int n_fp64_fits;       /* affine fits solved in FP64                    */
    int tile_visits;       /* tiles processed by the geodesic transform     */
    int n_bad_cost;        /* cost values not finite and > 0 (counted only
                              with debug_validate)                          */
    int n_pruned;          /* placed matches removed by the consistency check
                              (prune_px > 0); the other counts then refer to
                              the kept matches, except n_outside and
                              n_duplicate, which count the original ones    */
    int n_invariant;       /* violated device invariants (debug_validate)  */
} epic_stats;
int epic_get_stats(epic_ctx* ctx, int pair, epic_stats* out);

/* Stage outputs of one epic_interp call for testing; every output pointer
 * is a device pointer and may be NULL.
 *   D        H*W geodesic distance to the nearest match: float32, or
 *            float64 for a context created with precision 1
 *   L        H*W int32 nearest-match label
 *   edge_m, edge_n, edge_w   graph edges (m < n), up to max_edges of them,
 *            in no particular order; n_edges (device int) receives the
 *            number of edges
 *   knn_idx, knn_d  N*K neighbour ids (-1 = none) and graph distances, in
 *            (distance, index) order
 *   params   N*6 float32 model b00 b01 b10 b11 c0 c1 of
 *            flow(p) = B (p - p_m) + c
 *   flow     as in epic_interp (may be NULL here) */
int epic_debug_stages(epic_ctx* ctx, const float* cost, int H, int W,
                      const float* matches, int N, int K, float a, int mode,
                      float* D, int* L, int* edge_m, int* edge_n,
                      float* edge_w, int max_edges, int* n_edges,
                      int* knn_idx, float* knn_d, float* params, float* flow,
                      void* stream);

/* The consistency check of the matches alone (Sec. 5.1, "Pruning of
 * matches"): one NW interpolation (K, a as given) and the test
 * |u_m - F_NW(p_m)| <= prune_px at every placed match, where u_m is the
 * match's displacement and F_NW(p_m) the NW field at its pixel.
 *   kept     device, N int32: the original indices of the kept matches in
 *            increasing order (entries beyond the count are unspecified)
 *   n_kept   device int32: their count
 * Matches outside the image or on a pixel held by a lower index are never
 * kept.  prune_px must be finite and > 0 (EPIC_ERR_ARG otherwise); other
 * arguments as in epic_interp.  Asynchronous on `stream`. */
int epic_prune(epic_ctx* ctx, const float* cost, int H, int W,
               const float* matches, int N, int K, float a, float prune_px,
               int* kept, int* n_kept, void* stream);

/* Cost maps from images (Table 2, the norm-of-gradient contour row: the
 * cost is the norm of the image gradient; Sec. 4 uses the same norm):
 *   C(p) = sqrt(sum over channels of gx^2 + gy^2) + eps
 * with central differences gx = (I(x+1) - I(x-1)) / 2, gy = (I(y+1) -
 * I(y-1)) / 2 and the border pixel repeated outside the image; FP32, each
 * operation rounded on its own.  eps (finite, > 0) keeps C > 0 on flat
 * regions, as the transform requires.
 *   image    device, H*W*channels float32, channels (1 to 4) interleaved
 *   cost     device, H*W float32 output (caller-owned; may be passed to
 *            epic_interp as its cost map)
 * `imgs` is a host array of n descriptors; images with equal channel
 * counts share launches (up to 64 per launch).  Needs no context and no
 * workspace.  Host-side validation returns EPIC_ERR_ARG (null or
 * misaligned pointers, sizes, channels, eps); asynchronous on `stream`. */
typedef struct epic_image {
    const float* image;
    int H, W, channels;
    float* cost;
} epic_image;
int epic_image_cost(const epic_image* imgs, int n, float eps, void* stream);

/* epic_interp with an image in place of the cost map: the cost of
 * epic_image_cost (image H*W*channels float32 on the device) is computed
 * into the context's workspace, then the pair is interpolated as by
 * epic_interp.  The workspace must hold epic_workspace_bytes(...) plus
 * 4*H*W + 512 bytes (EPIC_ERR_WORKSPACE otherwise). */
int epic_interp_image(epic_ctx* ctx, const float* image, int H, int W, int channels, float eps,
                      const float* matches, int N, int K, float a, int mode, float* flow,
                      void* stream);

/* The exact per-pixel geodesic interpolation (Table 2, "Geodesic (exact)";
 * the quality reference for the approximation of Sec. 3.4): every pixel p
 * gets its own K nearest matches under the geodesic distance of Eq. (3)
 * itself, D_G(p, p_m), ordered by (distance, index), with weights
 * exp(-a D_G), and its own NW (Eq. 1) or LA (Eq. 2) estimate evaluated at
 * p.  The approximated interpolation runs first: its distances (each the
 * length of a path of the pixel graph) bound, at every pixel, the distance
 * of the K-th nearest match; then one single-source transform per match (in
 * chunks of up to 1024 that fit the workspace) keeps only distances within
 * those bounds, a per-pixel selection folds each chunk into the pixels' K
 * nearest, and a per-pixel fit ends it; the near-collinear LA rule and FP64
 * routing are those of epic_interp.  The bound only skips work: the result
 * is the same as with full-image transforms.
 * Arguments as in epic_interp, with K <= 128 and a context created with
 * precision 0 (EPIC_ERR_ARG otherwise).  The workspace must hold
 * 8*K*H*W + 4*H*W + N + 8*N*K bytes plus 34 KB at its end for the
 * pixels' lists, the bounds, the approximated lists, the boxes of tiles a
 * chunk's transforms reached and alignment, besides
 * epic_workspace_bytes(H, W, N, K, mode, 0) for the approximated pass and,
 * per match of a chunk, epic_workspace_bytes(H, W, 1, 1, mode, 0)
 * (EPIC_ERR_WORKSPACE when not even one fits); a chunk of 1024 at
 * 1024 x 436 needs about 3.7 GB.  No per-call statistics (epic_get_stats
 * refers to no pair afterwards).  Asynchronous on `stream`. */
int epic_interp_exact(epic_ctx* ctx, const float* cost, int H, int W, const float* matches, int N,
                      int K, float a, int mode, float* flow, void* stream);

/* One-level variational refinement of a dense flow field (Sec. 4: the
 * interpolated field initialises an energy minimisation run at the full
 * resolution only, without coarse-to-fine).  The energy (the data term is
 * cited by the paper, not written out; this is the library's reading of
 * it): with I2w = I2 warped by the input field u0 (bilinear, coordinates
 * clamped), derivatives by central differences with the border pixel
 * repeated, and per channel Iz = I2w - I1, Ixz/Iyz the gradient of I2w
 * minus that of I1,
 *   E(du) = sum_x  delta psi(sum_c (Iz + Ix du + Iy dv)^2 / (Ix^2 + Iy^2 + zeta^2))
 *               + gamma psi(sum_c (Ixz + Ixx du + Ixy dv)^2 / (Ixx^2 + Ixy^2 + zeta^2)
 *                                + (Iyz + Ixy du + Iyy dv)^2 / (Ixy^2 + Iyy^2 + zeta^2))
 *         + sum over 4-neighbour edges (i, j)
 *               lam (alpha_i + alpha_j) / 2 psi(|U_j - U_i|^2 + |V_j - V_i|^2)
 * where psi(s^2) = sqrt(s^2 + eps^2), U = u0 + du, V = v0 + dv and the
 * local smoothness weight alpha = exp(-kappa ||grad I1||) (kappa = 5 in the
 * paper).  The data term is linearised once about u0; `fixed_point` times
 * (5 in the paper) the weights psi' are evaluated at the current update and
 * the linear Euler-Lagrange system is relaxed by `sor` red-black
 * successive-over-relaxation sweeps (30 in the paper) with factor omega.
 * The output is u0 + du.  FP32 throughout.
 *   I1, I2     device, H*W*channels float32 (channels 1 to 4, interleaved)
 *   flow_in    device, H*W*2 float32, the field to refine (e.g. the output
 *              of epic_interp)
 *   flow_out   device, H*W*2 float32 output; may be flow_in itself, must not
 *              overlap it otherwise
 *   params     host; NULL takes epic_refine_defaults
 * Scratch: epic_refine_bytes(H, W, channels) bytes at the end of the
 * context's workspace (104 + 4*channels bytes per pixel plus alignment),
 * after the workspace's fixed 4096 + descriptor-ring head; EPIC_ERR_WORKSPACE
 * when it does not fit.  The statistics of the last interpolation remain
 * readable when the workspace also holds that call's part.  Host-side
 * validation returns EPIC_ERR_ARG (null or misaligned pointers, sizes,
 * non-finite or negative parameters, eps or zeta not > 0, omega outside
 * (0, 2), fixed_point outside [0, 100], sor outside [0, 10000]).
 * Asynchronous on `stream`; calls on one context must be ordered (one
 * stream), as for epic_interp. */
typedef struct epic_refine_params {
    float lam;          /* smoothness weight, default 0.1 */
    float delta;        /* colour-constancy weight, default 0.1 */
    float gamma;        /* gradient-constancy weight, default 0.7 */
    float kappa;        /* alpha = exp(-kappa ||grad I1||), default 5 */
    float eps;          /* psi's regulariser, default 1e-3 */
    float zeta;         /* normalisation floor, default 0.1 */
    float omega;        /* over-relaxation factor, default 1.6 */
    int fixed_point;    /* outer iterations, default 5 */
    int sor;            /* sweeps per outer iteration, default 30 */
} epic_refine_params;
void epic_refine_defaults(epic_refine_params* p);
size_t epic_refine_bytes(int H, int W, int channels);
int epic_refine(epic_ctx* ctx, const float* I1, const float* I2, int H, int W, int channels,
                const float* flow_in, float* flow_out, const epic_refine_params* params,
                void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): epic_interp without a
 * context.  Its workspace is a 64 MiB device array inside the library, one
 * copy per GPU, held until the process ends; the call allocates nothing (no
 * hipMalloc, no pinned memory, no events) and runs on the current HIP
 * device with the default options (FP32, 8-connected, LA weights k^2) and a
 * fixed pass budget (results equal epic_interp's).  Arguments as in
 * epic_interp.  Sizes whose workspace (epic_workspace_bytes with precision
 * 0) exceeds 64 MiB -- e.g. beyond 2048 x 1080 pixels with 40000 matches --
 * return EPIC_ERR_WORKSPACE before anything runs.  Every call on one GPU
 * shares that GPU's array and leaves its contents behind (each call clears
 * what it needs first): calls that overlap on one GPU race, so order them
 * on one stream (or with events), from one host thread at a time.  There
 * are no per-call statistics; a pair without a usable match gets NaN flow. */
int epic_interp_noalloc(const float* cost, int H, int W, const float* matches, int N, int K,
                        float a, int mode, float* flow, void* stream);

/* Stage timing (instrumentation).  While enabled, every call records HIP
 * events between its stages on the call's stream (a ring of the last 64
 * calls).  epic_stage_times synchronises those calls and writes, for each
 * stage in launch order, the mean elapsed milliseconds over the last
 * `calls` profiled calls (at most 64) into ms[0..n_stages): 0 clear,
 * 1 seed, 2 geodesic transform, 3 graph emit, 4 CSR scan, 5 CSR scatter,
 * 6 K-NN + fit, 7 assignment.  Returns the number of stages written, or a
 * negative epic_status. */
int epic_profile(epic_ctx* ctx, int enable);
int epic_stage_times(epic_ctx* ctx, float* ms, int n_stages, int calls);

/* Name of stage i of epic_stage_times ("" when out of range). */
const char* epic_stage_name(int i);

/* Tile visits per pass of the last call's geodesic transform (pass 0 the
 * first pass over every tile, then the dirty-tile passes, the finisher's
 * passes after them), summed over the call's pairs.  Counted only for FP32
 * calls made while profiling is enabled (epic_profile); otherwise all zero.
 * Synchronises the last call's stream, writes min(n, 256) counts and
 * returns the number of passes that visited a tile (or a negative
 * epic_status). */
int epic_pass_visits(epic_ctx* ctx, int* visits, int n);

/* Human-readable text of an epic_status. */
const char* epic_strerror(int status);

/* Text of the last error of epic_create on this thread ("" if none). */
const char* epic_last_error(void);

/* Host-only validation of one request's arguments (what epic_interp checks
 * before enqueueing).  Returns EPIC_OK or EPIC_ERR_ARG. */
int epic_validate(const float* cost, int H, int W, const float* matches,
                  int N, int K, float a, int mode, const float* flow);

#ifdef __cplusplus
}
#endif

#endif /* EPIC_H_ */
